// Kernels around the fused pass: gradient epilogue with the leapfrog kicks and drift,
// trajectory start (momentum draw, opening half kick, drift), Metropolis accept and the
// log-posterior finalisation. All reductions run in float64 in a fixed order.
#include <math.h>

#include "device_common.h"

namespace hmcx {
namespace {

using namespace dev;

// Sum of one 256-thread block's values in a fixed order (lane tree, then wave order).
__device__ double block_sum256(double v, double* sh4) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh4[w] = v;
  __syncthreads();
  return ((sh4[0] + sh4[1]) + sh4[2]) + sh4[3];
}

// Prior, mask, the kicks and drift of `mode`, and the packed B operand for one gradient
// element e (< p K) whose likelihood part, summed over the partials, is gsum; pr and ke gain
// the element's prior log-density and kinetic energy.
template <typename T>
__device__ __forceinline__ void epi_element(const EpiArgs& a, int64_t e, T bt, T ev0, double gsum,
                                            double& pr, double& ke) {
  const int K = a.K;
  const bool pinned = a.pin && (int)(e % K) == K - 1;
  T* Bv = static_cast<T*>(a.B);
  T* Gv = static_cast<T*>(a.G);
  const double b = (double)bt;
  const T gt = pinned ? T(0) : (T)(gsum + prior_grad(b, a.prior, a.scale));
  Gv[e] = gt;
  pr = pinned ? 0.0 : prior_logd(b, a.prior, a.scale);
  if (a.mode != 0) {
    T* Ev = static_cast<T*>(a.eta);
    const T h = (T)a.h;
    T ev = ev0 + h * gt;                          // closing half kick, equation (hmc3)
    if (a.mode == 1) {
      ev = ev + h * gt;                           // opening half kick of the next update
      const T bn = pinned ? T(0) : bt + (T)a.eps * ev;   // full position step
      Bv[e] = bn;
      if constexpr (sizeof(T) == 4) {
        // the next pass's split-precision B operand, packed here instead of by a pass of its own
        if (a.bpk) store_packed_b(a.bpk, a.pack_nb, (int)(e % K) / 16, e / K, (int)(e % K) % 16, (float)bn);
      }
    } else {
      ke = 0.5 * (double)ev * (double)ev;
    }
    Ev[e] = ev;
  }
}

// 256 threads own 64 consecutive gradient elements. Thread t reads 16-byte groups
// (t % GROUPS) of the partials w = t / GROUPS, + SLICES, ... (every partial stride is a
// multiple of 64 elements, so the loads are aligned and many are in flight); the slices
// are then combined in a fixed order and wave 0 applies prior, mask and kicks.
template <typename T>
__global__ __launch_bounds__(256) void epilogue_kernel(EpiArgs a) {
  constexpr int VEC = 16 / sizeof(T);             // elements per 16-byte load
  constexpr int GROUPS = kEpiElems / VEC;         // 16-byte groups per 64 elements
  constexpr int SLICES = 256 / GROUPS;            // partials summed in parallel
  __shared__ double red[SLICES][kEpiElems];
  const int tid = threadIdx.x;
  const int K = a.K;
  const int64_t pk = (int64_t)a.p * K;
  const int64_t e0 = (int64_t)blockIdx.x * kEpiElems;
  const int el = tid & 63, q = tid >> 6;
  const int64_t e = e0 + el;
  // wave 0 fetches the position and momentum first, so their latency overlaps the partials
  T bt = T(0), ev0 = T(0);
  if (q == 0 && e < pk) {
    bt = static_cast<const T*>(a.B)[e];
    if (a.mode != 0) ev0 = static_cast<const T*>(a.eta)[e];
  }
  {
    const int grp = tid % GROUPS, sl = tid / GROUPS;
    double acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = 0.0;
    const T* gp = static_cast<const T*>(a.gpart) + e0 + grp * VEC;
    // Batches of BATCH loads are all issued before the first add, so their latencies
    // overlap (left to itself, the scheduler interleaves adds that wait for early loads).
    // Loads past the last partial re-read partial `sl` and add zero instead (a select, not
    // a branch, so no load is moved under a condition).
    typedef __attribute__((ext_vector_type(VEC))) T vec_t;
    constexpr int BATCH = 16;
    const int nw = a.nwg;
    for (int w0 = sl; w0 < nw; w0 += BATCH * SLICES) {
      vec_t q[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int w = w0 + u * SLICES;
        q[u] = *reinterpret_cast<const vec_t*>(gp + (int64_t)(w < nw ? w : sl) * a.gstride);
      }
      __builtin_amdgcn_sched_barrier(0);   // keep every add after the last load's issue
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const bool real = w0 + u * SLICES < nw;
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[v] += real ? (double)q[u][v] : 0.0;
      }
    }
#pragma unroll
    for (int v = 0; v < VEC; ++v) red[sl][grp * VEC + v] = acc[v];
  }
  __syncthreads();
  double pr = 0.0, ke = 0.0;
  if (q == 0 && e < pk) {
    double gsum = red[0][el];
#pragma unroll
    for (int sl = 1; sl < SLICES; ++sl) gsum += red[sl][el];
    epi_element<T>(a, e, bt, ev0, gsum, pr, ke);
  }
  if (q == 0) {
    pr = wave_sum(pr);
    ke = wave_sum(ke);
    if (el == 0) {
      a.ppart[blockIdx.x] = pr;
      if (a.mode == 2) a.kpart[blockIdx.x] = ke;
    }
  }
}

// Partial slices the main epilogue sums in parallel (16 for float, 8 for double).
template <typename T> constexpr int epi_slices() { return 256 * (16 / (int)sizeof(T)) / kEpiElems; }
// Partial counts up to which the one-thread-per-element epilogue runs (more partials keep the
// main kernel, whose threads load across partials in parallel).
constexpr int kEpiFewMax = 64;

// The same epilogue with one thread per gradient element, 256 elements per workgroup (a
// quarter of the workgroups, every thread busy), for partial counts up to kEpiFewMax. Wave w's
// 64 elements are the main kernel's group 4 blockIdx.x + w, whose partial-sum slot they fill.
// Each element keeps the main kernel's slice sums in registers: slice s adds partials s,
// s + S, s + 2 S, ... in turn from 0 (S = epi_slices<T>()), and the slices are added in order,
// which is exactly the main kernel's arithmetic (its loads past the last partial add +0 to a
// sum that started at +0 and so is never -0), so the results are bit for bit the same.
template <typename T>
__global__ __launch_bounds__(256) void epilogue_few(EpiArgs a) {
  constexpr int S = epi_slices<T>();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t pk = (int64_t)a.p * a.K;
  const int64_t e = (int64_t)blockIdx.x * 256 + tid;
  const bool ok = e < pk;
  const int64_t ec = ok ? e : 0;
  const T* gp = static_cast<const T*>(a.gpart) + ec;
  const T bt = ok ? static_cast<const T*>(a.B)[ec] : T(0);
  const T ev0 = (ok && a.mode != 0) ? static_cast<const T*>(a.eta)[ec] : T(0);
  const int nw = a.nwg;
  double sl[S];
#pragma unroll
  for (int u = 0; u < S; ++u) sl[u] = 0.0;
  int w0 = 0;
  for (; w0 + S <= nw; w0 += S) {
    T q[S];
#pragma unroll
    for (int u = 0; u < S; ++u) q[u] = gp[(int64_t)(w0 + u) * a.gstride];
#pragma unroll
    for (int u = 0; u < S; ++u) sl[u] += (double)q[u];
  }
  {
    T q[S];
#pragma unroll
    for (int u = 0; u < S; ++u) q[u] = gp[(int64_t)(w0 + u < nw ? w0 + u : 0) * a.gstride];
#pragma unroll
    for (int u = 0; u < S; ++u)
      if (w0 + u < nw) sl[u] += (double)q[u];
  }
  double gsum = sl[0];
#pragma unroll
  for (int u = 1; u < S; ++u) gsum += sl[u];
  double pr = 0.0, ke = 0.0;
  if (ok) epi_element<T>(a, e, bt, ev0, gsum, pr, ke);
  pr = wave_sum(pr);
  ke = wave_sum(ke);
  const int64_t g = (int64_t)blockIdx.x * 4 + w;
  if (lane == 0 && g * kEpiElems < pk) {
    a.ppart[g] = pr;
    if (a.mode == 2) a.kpart[g] = ke;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void start_kernel(StartArgs a) {
  __shared__ double sh4[4];
  const int K = a.K;
  const int64_t pk = (int64_t)a.p * K;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t iter = a.ctr ? a.ctr[0] : a.iter;
  const int64_t t = a.ctr ? a.ctr[0] - a.ctr[1] : a.t;
  double ke = 0.0;
  if (e < pk) {
    const bool pinned = a.pin && (int)(e % K) == K - 1;
    T* Ev = static_cast<T*>(a.eta);
    T ev;
    if (a.draw == 0) {
      ev = Ev[e];
    } else {
      const bool replay = a.draw == 1 && t >= 0 && t < a.n_rec;
      const double xi = replay ? a.normals[t * pk + e] : philox_normal(a.seed, a.chain, iter, e);
      ev = pinned ? T(0) : (T)xi;                   // eta = M * xi
      ke = 0.5 * (double)ev * (double)ev;
    }
    const T gt = static_cast<const T*>(a.G)[e];
    ev = ev + (T)a.h * gt;                          // opening half kick, equation (hmc1)
    const T bt = static_cast<const T*>(a.B)[e];
    static_cast<T*>(a.Bp)[e] = pinned ? T(0) : bt + (T)a.eps * ev;
    Ev[e] = ev;
  }
  if (a.draw != 0) {
    ke = block_sum256(ke, sh4);
    if (threadIdx.x == 0) {
      a.k0part[blockIdx.x] = ke;
      if (blockIdx.x == 0) a.scal[0] = *a.logpost;
    }
  }
}

// Fixed-order float64 sum of a small device array by one wave.
// Sum of v[0..n) by one wave in a fixed order: lane l adds v[l], v[l + 64], ... in turn, then
// the lanes are combined by wave_sum. Loads are issued eight at a time before their adds, so
// their latencies overlap (one at a time, a few thousand partials took tens of microseconds).
__device__ double wave_sum_array(const double* v, int n) {
  double s = 0.0;
  int i = threadIdx.x & 63;
  for (; i + 7 * 64 < n; i += 8 * 64) {
    double q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = v[i + 64 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += q[u];
  }
  for (; i < n; i += 64) s += v[i];
  return wave_sum(s);
}

template <typename T>
__global__ __launch_bounds__(256) void accept_kernel(AcceptArgs a) {
  __shared__ int sh_acc;
  __shared__ double sh_logk1;
  const int tid = threadIdx.x;
  const int64_t iter = a.ctr ? a.ctr[0] : a.iter;
  const int64_t t = a.ctr ? a.ctr[0] - a.ctr[1] : a.t;
  const bool rec = t >= 0 && t < a.n_rec;
  if (tid < 64) {
    const double logk1 = wave_sum_array(a.lpart, a.nl) + wave_sum_array(a.ppart, a.np);
    const double ke0 = wave_sum_array(a.k0part, a.nk0);
    const double ke1 = wave_sum_array(a.k1part, a.nk1);
    if (tid == 0) {
      const double logk0 = a.scal[0];
      const double H0 = -logk0 + ke0;
      const double H1 = -logk1 + ke1;
      const double u = (a.replay_u && rec) ? a.replay_u[t] : philox_uniform(a.seed, a.chain, iter);
      const double it = (a.inv_temp && rec) ? a.inv_temp[t] : 1.0;
      const bool finite = isfinite(H1);
      const bool acc = finite && (log(u) < (H0 - H1) * it);
      const bool div = !finite || (H1 - H0 > 1000.0);
      sh_acc = acc ? 1 : 0;
      sh_logk1 = logk1;
      if (blockIdx.x == 0) {
        *a.logpost = acc ? logk1 : logk0;
        if (rec) {
          if (a.accepted) a.accepted[t] = acc ? 1 : 0;
          if (a.divergent) a.divergent[t] = div ? 1 : 0;
          if (a.H) { a.H[2 * t] = H0; a.H[2 * t + 1] = H1; }
        }
      }
    }
  }
  __syncthreads();
  const bool acc = sh_acc != 0;
  const int64_t pk = (int64_t)a.p * a.K;
  const int64_t e = (int64_t)blockIdx.x * 256 + tid;
  if (e < pk) {
    T* Bv = static_cast<T*>(a.B);
    T bnew;
    if (acc) {
      bnew = static_cast<const T*>(a.Bp)[e];
      Bv[e] = bnew;
      static_cast<T*>(a.G)[e] = static_cast<const T*>(a.Gp)[e];
    } else {
      bnew = Bv[e];
    }
    if (a.sample && rec) static_cast<T*>(a.sample)[t * pk + e] = bnew;
  }
  (void)sh_logk1;
}

__global__ __launch_bounds__(64) void final_kernel(FinalArgs a) {
  const double v = wave_sum_array(a.lpart, a.nl) + wave_sum_array(a.ppart, a.np);
  if (threadIdx.x == 0) *a.logpost = v;
}

}  // namespace

template <typename T>
hipError_t launch_epilogue(const EpiArgs& a, int nwg, hipStream_t s) {
  if (a.nwg <= kEpiFewMax)
    hipLaunchKernelGGL(epilogue_few<T>, dim3((nwg + 3) / 4), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(epilogue_kernel<T>, dim3(nwg), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_start(const StartArgs& a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(start_kernel<T>, dim3(nwg), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_accept(const AcceptArgs& a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(accept_kernel<T>, dim3(nwg), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_final(const FinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(final_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_epilogue<float>(const EpiArgs&, int, hipStream_t);
template hipError_t launch_epilogue<double>(const EpiArgs&, int, hipStream_t);
template hipError_t launch_start<float>(const StartArgs&, int, hipStream_t);
template hipError_t launch_start<double>(const StartArgs&, int, hipStream_t);
template hipError_t launch_accept<float>(const AcceptArgs&, int, hipStream_t);
template hipError_t launch_accept<double>(const AcceptArgs&, int, hipStream_t);

}  // namespace hmcx
