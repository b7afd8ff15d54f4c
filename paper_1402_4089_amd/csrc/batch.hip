// Batched sampler kernels around the split-precision pass: every chain of every problem
// of a batch per launch. Work items are numbered problem table entry by entry (item i
// belongs to entry b with first[b] <= i < first[b + 1]; an entry carries its problem's
// global chain index); within a problem, chain c's items follow chain c - 1's. The arithmetic per chain is that of the single-problem kernels
// (trajectory start, gradient epilogue, Metropolis test); reductions run in float64 in a
// fixed order. The iteration index is read from device memory, so a captured graph of one
// iteration can be replayed.
#include <math.h>

#include "device_common.h"

namespace hmcx {
namespace {

using namespace dev;

__device__ __forceinline__ int find_problem(const int32_t* first, int nprob, int64_t item) {
  int lo = 0, hi = nprob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ double block_sum256(double v, double* sh4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh4[w] = v;
  __syncthreads();
  return ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
}

// Fixed-order float64 sum of v[0], v[s], v[2 s], ... (n terms) by one wave: lane l adds terms
// l, l + 64, ... in turn (loads issued eight at a time before their adds, so their latencies
// overlap), then the lanes are combined by wave_sum.
__device__ double wave_sum_strided(const double* v, int64_t n, int64_t s) {
  double t = 0.0;
  int64_t i = threadIdx.x & 63;
  for (; i + 7 * 64 < n; i += 8 * 64) {
    double q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = v[(i + 64 * u) * s];
#pragma unroll
    for (int u = 0; u < 8; ++u) t += q[u];
  }
  for (; i < n; i += 64) t += v[i * s];
  return wave_sum(t);
}

// Trajectory start: eta = M xi (Philox), KE0 partials, opening half kick, drift into Bp.
__global__ __launch_bounds__(256) void batch_start(BatchArgs a) {
  __shared__ double sh4[4];
  const int64_t it = blockIdx.x;
  const int b = find_problem(a.first_upd, a.nprob, it);
  const BatchProb& P = a.probs[b];
  const int64_t k = it - a.first_upd[b];
  const int c = (int)(k / P.nu), q = (int)(k % P.nu);
  const int64_t pk = (int64_t)P.p * P.K;
  const int64_t e = (int64_t)q * 256 + threadIdx.x;
  const int64_t iter = a.ctr[0];
  const int64_t t = iter - a.ctr[1];
  const bool replay = P.normals && t >= 0 && t < a.n_rec;
  const double h = 0.5 * P.eps;
  double ke = 0.0;
  if (e < pk) {
    const int64_t o = c * pk + e;
    const bool pinned = P.pin && (int)(e % P.K) == P.K - 1;
    const double xi = replay ? P.normals[(t * a.chains + c) * pk + e]
                             : philox_normal(a.seed, P.chain0 + c, iter, e);
    float ev = pinned ? 0.0f : (float)xi;
    ke = 0.5 * (double)ev * (double)ev;
    ev = ev + (float)h * P.G[o];                      // opening half kick, equation (hmc1)
    P.Bp[o] = pinned ? 0.0f : P.B[o] + (float)P.eps * ev;
    P.eta[o] = ev;
  }
  ke = block_sum256(ke, sh4);
  if (threadIdx.x == 0) {
    P.k0part[(int64_t)c * P.nu + q] = ke;
    if (q == 0) P.scal[c] = P.logpost[c];
  }
}

// Gradient epilogue for 256 elements of one chain, one thread per element: fixed-order sum of
// the row-slice partials, prior term, mask, then the leapfrog kicks / drift of `mode`. The
// partials are summed in four interleaved slices (w = s, s + 4, ... in turn), combined as
// ((s0 + s1) + s2) + s3; wave w's 64 elements fill partial-sum slot 4 q4 + w of the chain.
__global__ __launch_bounds__(256) void batch_epilogue(BatchArgs a) {
  const int64_t it = blockIdx.x;
  const int b = find_problem(a.first_epi, a.nprob, it);
  const BatchProb& P = a.probs[b];
  const int64_t k = it - a.first_epi[b];
  const int c = (int)(k / P.ne4), q4 = (int)(k % P.ne4);
  const int64_t pk = (int64_t)P.p * P.K;
  const int el = threadIdx.x & 63;
  const int q = 4 * q4 + (threadIdx.x >> 6);
  const int64_t e = (int64_t)q4 * 256 + threadIdx.x;
  double gsum = 0.0;
  if (e < pk) {
    const float* gp = P.gpart + c * P.cstride + e;
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    const int ns = P.nsplit;
    int w = 0;
    for (; w + 8 <= ns; w += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = gp[(int64_t)(w + u) * P.gstride];
#pragma unroll
      for (int u = 0; u < 8; ++u) s4[u & 3] += v[u];
    }
    for (; w < ns; ++w) s4[w & 3] += gp[(int64_t)w * P.gstride];
    gsum = ((s4[0] + s4[1]) + s4[2]) + s4[3];
  }
  double pr = 0.0, ke = 0.0;
  float* Bv = a.at_current ? P.B : P.Bp;
  float* Gv = a.at_current ? P.G : P.Gp;
  if (e < pk) {
    const int64_t o = c * pk + e;
    const bool pinned = P.pin && (int)(e % P.K) == P.K - 1;
    const float bt = Bv[o];
    const double bd = (double)bt;
    const float gt = pinned ? 0.0f : (float)(gsum + prior_grad(bd, P.prior, P.scale));
    Gv[o] = gt;
    pr = pinned ? 0.0 : prior_logd(bd, P.prior, P.scale);
    if (a.mode != 0) {
      const float hh = (float)(0.5 * P.eps);
      float ev = P.eta[o] + hh * gt;                  // closing half kick, equation (hmc3)
      if (a.mode == 1) {
        ev = ev + hh * gt;                            // opening half kick of the next update
        const float bn = pinned ? 0.0f : bt + (float)P.eps * ev;
        Bv[o] = bn;
        // the next pass's packed B operand (class k of chain c is lane k % 16 of block
        // c group + k / 16), written here instead of by a pass of its own
        const int k = (int)(e % P.K);
        store_packed_b(P.Bpk, a.chains * a.group, c * a.group + k / 16, e / P.K, k % 16, bn);
      } else {
        ke = 0.5 * (double)ev * (double)ev;
      }
      P.eta[o] = ev;
    }
  }
  pr = wave_sum(pr);
  ke = wave_sum(ke);
  if (el == 0 && q < P.ne) {
    P.ppart[(int64_t)c * P.ne + q] = pr;
    if (a.mode == 2) P.k1part[(int64_t)c * P.ne + q] = ke;
  }
}

// Metropolis test for one chain (recomputed by each of its workgroups from the partials),
// then selection and recording for 256 of its elements.
__global__ __launch_bounds__(256) void batch_accept(BatchArgs a) {
  __shared__ int sh_acc;
  const int64_t it = blockIdx.x;
  const int b = find_problem(a.first_upd, a.nprob, it);
  const BatchProb& P = a.probs[b];
  const int64_t k = it - a.first_upd[b];
  const int c = (int)(k / P.nu), q = (int)(k % P.nu);
  const int64_t pk = (int64_t)P.p * P.K;
  const int64_t iter = a.ctr[0];
  const int64_t t = iter - a.ctr[1];
  if (threadIdx.x < 64) {
    const double logk1 = wave_sum_strided(P.lpart + c, P.nrb, a.chains) +
                         wave_sum_strided(P.ppart + (int64_t)c * P.ne, P.ne, 1);
    const double ke0 = wave_sum_strided(P.k0part + (int64_t)c * P.nu, P.nu, 1);
    const double ke1 = wave_sum_strided(P.k1part + (int64_t)c * P.ne, P.ne, 1);
    if (threadIdx.x == 0) {
      const double logk0 = P.scal[c];
      const double H0 = -logk0 + ke0;
      const double H1 = -logk1 + ke1;
      const bool rec = t >= 0 && t < a.n_rec;
      const double u = (P.uniforms && rec) ? P.uniforms[t * a.chains + c]
                                           : philox_uniform(a.seed, P.chain0 + c, iter);
      const double it_ = (a.inv_temp && rec) ? a.inv_temp[t] : 1.0;
      const bool finite = isfinite(H1);
      const bool acc = finite && (log(u) < (H0 - H1) * it_);
      const bool div = !finite || (H1 - H0 > 1000.0);
      sh_acc = acc ? 1 : 0;
      if (q == 0) {
        P.logpost[c] = acc ? logk1 : logk0;
        if (t >= 0 && t < a.n_rec) {
          const int64_t r = t * a.total_chains + P.chain0 + c;
          if (a.accepted) a.accepted[r] = acc ? 1 : 0;
          if (a.divergent) a.divergent[r] = div ? 1 : 0;
          if (a.H) { a.H[2 * r] = H0; a.H[2 * r + 1] = H1; }
        }
      }
    }
  }
  __syncthreads();
  const bool acc = sh_acc != 0;
  const int64_t e = (int64_t)q * 256 + threadIdx.x;
  if (e < pk) {
    const int64_t o = c * pk + e;
    float bnew;
    if (acc) {
      bnew = P.Bp[o];
      P.B[o] = bnew;
      P.G[o] = P.Gp[o];
    } else {
      bnew = P.B[o];
    }
    if (P.samples && t >= 0 && t < a.n_rec) P.samples[t * a.chains * pk + o] = bnew;
    if (P.moments) {
      P.moments[o] += (double)bnew;
      P.moments[a.chains * pk + o] += (double)bnew * (double)bnew;
    }
  }
}

// log K at the current state of every chain: sum of its log-likelihood and prior partials.
__global__ __launch_bounds__(64) void batch_final(BatchArgs a) {
  const int64_t it = blockIdx.x;
  const int b = find_problem(a.first_upd, a.nprob, it);
  const BatchProb& P = a.probs[b];
  const int64_t k = it - a.first_upd[b];
  if (k % P.nu) return;
  const int c = (int)(k / P.nu);
  const double v = wave_sum_strided(P.lpart + c, P.nrb, a.chains) +
                   wave_sum_strided(P.ppart + (int64_t)c * P.ne, P.ne, 1);
  if (threadIdx.x == 0) P.logpost[c] = v;
}

__global__ void counter_kernel(int64_t* ctr, int64_t v, int op) {
  if (threadIdx.x == 0) {
    if (op == 0) { ctr[0] = v; ctr[1] = v; }
    else ctr[0] += 1;
  }
}

}  // namespace

hipError_t launch_batch_start(const BatchArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(batch_start, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_batch_epilogue(const BatchArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(batch_epilogue, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_batch_accept(const BatchArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(batch_accept, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_batch_final(const BatchArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(batch_final, dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_counter(int64_t* ctr, int64_t set_to, int op, hipStream_t s) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, s, ctr, set_to, op);
  return hipGetLastError();
}

}  // namespace hmcx
