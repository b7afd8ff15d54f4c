// Log-posterior + gradient for p too wide for one compute unit's row tile (p >> n).
//
// Same quantities as the fused pass (Section 2.1: logits X B, row softmax and
// log-likelihood, gradient X^T (Y - psi(XB)) plus the prior term), split into three
// kernels because a row's logits need all p columns before its residuals exist:
//   wide_logits   16-row x 1024-column blocks of X on MFMA -> per-chunk partial logits
//   wide_softmax  sums the chunk partials of a row, softmax, residuals R, log-likelihood
//   wide_grad     each workgroup owns an even share of the 16-column blocks, streams the
//                 rows of X and R (all of them, or one row slice) through MFMA
//                 (G block = X^T R); with all rows it then applies prior, mask and the
//                 leapfrog kicks and drift to its own columns (no cross-workgroup
//                 reduction), with row slices it writes partials for the shared epilogue.
// X is read twice per gradient. All loads go through buffer resources whose bounds
// make rows past n read as zero.
#include "device_common.h"

namespace hmcx {

using namespace dev;

namespace {

constexpr int kWideWaves = 4;

__device__ __forceinline__ float4 ld16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
template <typename T> __device__ __forceinline__ T ld1(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ float ld1<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ double ld1<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Partial logits over one column chunk for the row tiles tile0, tile0 + tstep, ...
// Wave w covers columns [chunk*CW + w*MBW*16, ... + MBW*16) in MBW blocks of 16. The chunk is
// the fast grid dimension, so the workgroups running together read the same rows (measured:
// with the chunk as the slow dimension the pass at n = 2000, p = 50000 took about 4% longer).
template <typename T, int NB>
__global__ __launch_bounds__(kWideWaves * 64) void wide_logits(WideArgs a) {
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int MBW = sizeof(T) == 4 ? 16 : 8;
  constexpr int CW = kWideWaves * MBW * 16;
  __shared__ __align__(16) T zb[kWideWaves * NB * 256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  const int p = a.p, K = a.K;
  const int64_t n = a.n, ldx = a.ldx;
  const int chunk = blockIdx.x;
  const int jw = chunk * CW + w * MBW * 16;              // first column of this wave
  const T* B = static_cast<const T*>(a.B);

  // the pinned column is read as zero (beta_K = 0 in the model)
  const int kmax = a.pin ? K - 1 : K;
  T bt[MBW][NB][4];
#pragma unroll
  for (int m = 0; m < MBW; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = jw + m * 16 + 4 * g + t, k = nb * 16 + c;
        bt[m][nb][t] = (j < p && k < kmax) ? B[(int64_t)j * K + k] : T(0);
      }
  const bool maskcols = ldx != p && jw + MBW * 16 > p;   // row padding inside this wave's span
  const uint64_t x_bytes = (uint64_t)((n - 1) * ldx + p) * sizeof(T);

  for (int64_t tile = blockIdx.y; tile * kTileRows < n; tile += gridDim.y) {
    const int64_t i0 = tile * kTileRows;
    const uint64_t base = (uint64_t)i0 * ldx * sizeof(T);
    const __amdgpu_buffer_rsrc_t xr =
        make_rsrc(static_cast<const char*>(a.X) + base, x_bytes - base);
    // A lane whose four columns all lie past p (the tail of the last chunk) loads from an
    // offset past the resource's end: zeros and no traffic where the rest of X is under 4 GB,
    // an in-bounds read of X's own elements otherwise (finite, and multiplied by coefficients
    // that are zero past p; with padded rows the wave's mask below zeroes them). Reading the
    // next rows there instead cost the last chunk as much traffic as a full one. The mask is
    // a wave-uniform branch: a per-lane one waits for each load before the next issues (2-7%
    // slower passes, measured).
    T av[MBW][4];
#pragma unroll
    for (int m = 0; m < MBW; ++m) {
      const int col0 = jw + m * 16 + 4 * g;
      const bool live = col0 < p;
      const uint32_t off = live ? (uint32_t)(((int64_t)c * ldx + col0) * sizeof(T)) : 0xFFFFFFE0u;
      if constexpr (sizeof(T) == 4) {
        const float4 q = ld16(xr, off);
        av[m][0] = q.x; av[m][1] = q.y; av[m][2] = q.z; av[m][3] = q.w;
      } else {
        const double2 q0 = __builtin_bit_cast(double2, ld16(xr, off));
        const double2 q1 = __builtin_bit_cast(double2, ld16(xr, off + 16));
        av[m][0] = q0.x; av[m][1] = q0.y; av[m][2] = q1.x; av[m][3] = q1.y;
      }
      if (maskcols) {
#pragma unroll
        for (int t = 0; t < 4; ++t) av[m][t] = (col0 + t < p) ? av[m][t] : T(0);
      }
    }
    acc_t z0[NB], z1[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) z0[nb] = z1[nb] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < MBW; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          if (m & 1) z1[nb] = M::run(av[m][t], bt[m][nb][t], z1[nb]);
          else       z0[nb] = M::run(av[m][t], bt[m][nb][t], z0[nb]);
        }
    __syncthreads();                                      // previous tile's exchange read
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) zb[((nb * 4 + r) * kWideWaves + w) * 64 + lane] = z0[nb][r] + z1[nb][r];
    __syncthreads();
    if (w == 0) {
      T* zp = static_cast<T*>(a.zpart) + (int64_t)chunk * n * (16 * NB);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T* src = zb + (nb * 4 + r) * kWideWaves * 64 + lane;
          const T v = ((src[0] + src[64]) + src[128]) + src[192];
          const int64_t i = i0 + M::row(r, g);
          if (i < n) zp[i * (16 * NB) + nb * 16 + c] = v;
        }
    }
  }
}

// Row softmax over the summed chunk partials: 4 rows per workgroup, 16 lanes per row. Wave g
// sums chunks g, g + 4, g + 8, ... of the four rows, the four sums are added in wave order
// through LDS, and wave 0 finishes the rows (a quarter of the dependent loads per thread of a
// one-wave-per-row-group form, whose chain over all chunks paced the kernel).
template <typename T, int NB>
__global__ __launch_bounds__(256) void wide_softmax(WideArgs a) {
  constexpr int KP = 16 * NB;
  __shared__ T zs[4][NB][64];
  const int tid = threadIdx.x, lane = tid & 63, grp = tid >> 6, c = lane & 15;
  const int K = a.K;
  const int64_t n = a.n;
  const int64_t i = (int64_t)blockIdx.x * 4 + (lane >> 4);
  const bool valid = i < n;
  const int64_t ic = valid ? i : n - 1;
  const T* zp = static_cast<const T*>(a.zpart) + ic * KP + c;
  T zz[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) zz[nb] = T(0);
#pragma unroll 4
  for (int ch = grp; ch < a.nchunk; ch += 4)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) zz[nb] += zp[(int64_t)ch * n * KP + nb * 16];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) zs[grp][nb][lane] = zz[nb];
  __syncthreads();
  if (grp != 0) return;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
    zz[nb] = ((zs[0][nb][lane] + zs[1][nb][lane]) + zs[2][nb][lane]) + zs[3][nb][lane];
  const int yi = a.y[ic];
  double l = 0.0;
  T* R = static_cast<T*>(a.R);
  if (a.link == 1) {
    // Poisson link, one coefficient column (lane c = 0): residual y - exp(z), term y z - exp(z)
    const T mu = dev_exp(zz[0]);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int k = nb * 16 + c;
      if (valid) R[i * KP + k] = k == 0 ? T(yi) - mu : T(0);
    }
    l = (valid && c == 0) ? (double)yi * (double)zz[0] - (double)mu : 0.0;
  } else if (a.link == 2) {
    // probit link, one coefficient column (lane c = 0): residual s phi(z) / Phi(s z) with
    // s = +1 for a success and -1 otherwise, term log Phi(s z)
    const T sg = yi == 1 ? T(1) : T(-1);
    T ratio;
    double lp;
    probit_row(sg * zz[0], ratio, lp);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int k = nb * 16 + c;
      if (valid) R[i * KP + k] = k == 0 ? sg * ratio : T(0);
    }
    l = (valid && c == 0) ? lp : 0.0;
  } else {
    T mx = -INFINITY;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
      if (nb * 16 + c < K) mx = fmax(mx, zz[nb]);
    mx = max16(mx);
    T ex[NB], se = T(0);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      ex[nb] = (nb * 16 + c < K) ? dev_exp(zz[nb] - mx) : T(0);
      se += ex[nb];
    }
    se = sum16(se);
    const T inv = dev_rcp(se);
    const T lse_shift = dev_log(se);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int k = nb * 16 + c;
      const bool hit = valid && k == yi;
      if (valid) R[i * KP + k] = (k < K) ? ((hit ? T(1) : T(0)) - ex[nb] * inv) : T(0);
      l += hit ? (double)((zz[nb] - mx) - lse_shift) : 0.0;
    }
  }
  l = wave_sum(l);
  if (lane == 0) a.lpart[blockIdx.x] = l;
}

// Blocks of 16 gradient columns a wave of the column-owner kernel can hold (accumulators and
// two load groups in registers): fewer for more class blocks and for float64.
template <typename T, int NB> constexpr int wide_wave_blocks() {
  return (sizeof(T) == 4 ? 4 : 2) / NB > 0 ? (sizeof(T) == 4 ? 4 : 2) / NB : 1;
}

// Column-owner gradient. The ceil(p/16) column blocks are shared out evenly: workgroup x owns
// blocks [x nblk / gridDim.x, (x + 1) nblk / gridDim.x) (at most 4 CB of them), and wave w
// takes the workgroup's blocks w, w + 4, ... (CB at most). An even share keeps every compute
// unit streaming the same number of columns, where whole 128-column workgroups left some units
// with two and others with one. With one row slice (gridDim.y == 1) the workgroup applies the
// leapfrog epilogue to its own columns; with several, slice blockIdx.y covers tiles_per_split
// 16-row tiles (a multiple of the U-tile load group) and writes its partial X^T R to gpart for
// the shared epilogue kernel.
template <typename T, int NB>
__global__ __launch_bounds__(kWideWaves * 64) void wide_grad(WideArgs a) {
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int KP = 16 * NB, CB = wide_wave_blocks<T, NB>(), U = 2;   // U row tiles per load group
  __shared__ double sh4[2][4];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  const int p = a.p, K = a.K;
  const int64_t n = a.n, ldx = a.ldx;
  const int64_t nblk = (p + 15) / 16;
  const int64_t b0 = (int64_t)blockIdx.x * nblk / gridDim.x;
  const int64_t b1 = (int64_t)(blockIdx.x + 1) * nblk / gridDim.x;
  // first column of this wave's block cb, and whether that block belongs to the workgroup
  int jb[CB];
  bool live[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int64_t b = b0 + w + kWideWaves * cb;
    live[cb] = b < b1;
    jb[cb] = (int)((live[cb] ? b : b0) * 16);
  }

  const uint64_t x_bytes = (uint64_t)((n - 1) * ldx + p) * sizeof(T);
  acc_t gacc[CB][NB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) gacc[cb][nb] = acc_t{0, 0, 0, 0};
  const int64_t ntiles = (n + kTileRows - 1) / kTileRows;
  const int64_t tbeg = (int64_t)blockIdx.y * a.tiles_per_split;
  const int64_t tend = gridDim.y == 1 ? ntiles : (tbeg + a.tiles_per_split < ntiles ? tbeg + a.tiles_per_split : ntiles);
  const int64_t ngroups = tend > tbeg ? (tend - tbeg + U - 1) / U : 0;

  // Groups of U row tiles are visited last to first: the logits pass has just read the
  // last rows of X, so the first groups here may still be held by the memory-side cache.
  // Group k - 1 is loaded while group k is multiplied; a group index below 0 gets
  // resources without records, so its loads return zeros without touching memory and
  // the issue stays free of branches. A block outside the workgroup's share loads from an
  // offset past every resource's end: zeros, no traffic.
  struct Regs { T xa[U][CB][4], ra[U][NB][4]; };
  auto load = [&](int64_t k, Regs& rg) {
    const bool real = k >= 0;
    const int64_t t0 = tbeg + (real ? k : 0) * U;
    const uint64_t base = (uint64_t)(t0 * kTileRows) * ldx * sizeof(T);
    const __amdgpu_buffer_rsrc_t xr =
        make_rsrc(static_cast<const char*>(a.X) + base, real ? x_bytes - base : 0);
    const __amdgpu_buffer_rsrc_t rr = make_rsrc(a.R, real ? (uint64_t)n * KP * sizeof(T) : 0);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int row = u * kTileRows + M::row(s, g);           // relative to t0's first row
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          rg.xa[u][cb][s] = ld1<T>(xr, live[cb] ? (uint32_t)(((int64_t)row * ldx + jb[cb] + c) * sizeof(T))
                                                : 0xFFFFFFF0u);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          rg.ra[u][nb][s] = ld1<T>(rr, (uint32_t)(((t0 * kTileRows + row) * KP + nb * 16 + c) * sizeof(T)));
      }
  };
  auto mma = [&](const Regs& rg) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            gacc[cb][nb] = M::run(rg.xa[u][cb][s], rg.ra[u][nb][s], gacc[cb][nb]);
  };
  // Explicit waits leave the group just issued in flight (the compiler, left to itself,
  // waits for every load before the first MFMA of the rotated loop).
  constexpr int GL = U * 4 * (CB + NB);                 // loads per group
  static_assert(GL < 64, "vmcnt range");
  // Groups are taken in pairs; with an odd count the last pair's second group is one of
  // zeros, whose products add nothing.
  Regs r0, r1;
  load(ngroups - 1, r0);
  for (int64_t k = ngroups - 1; k >= 0; k -= 2) {
    load(k - 1, r1);
    __builtin_amdgcn_s_waitcnt(wait_vm(GL));
    mma(r0);
    load(k - 2, r0);
    __builtin_amdgcn_s_waitcnt(wait_vm(GL));
    mma(r1);
  }

  if (gridDim.y > 1) {
    T* gp = static_cast<T*>(a.gpart) + (int64_t)blockIdx.y * a.gstride;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = jb[cb] + M::row(r, g), k = nb * 16 + c;
          if (live[cb] && j < p && k < K) gp[(int64_t)j * K + k] = gacc[cb][nb][r];
        }
    return;
  }

  // epilogue on this lane's elements (same arithmetic as the row-tile epilogue); the
  // position and momentum are read only now, after the stream
  T* Bv = static_cast<T*>(a.B);
  T* Ev = static_cast<T*>(a.eta);
  T* Gv = static_cast<T*>(a.G);
  double pr = 0.0, ke = 0.0;
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb[cb] + M::row(r, g), k = nb * 16 + c;
        if (!live[cb] || j >= p || k >= K) continue;
        const int64_t e = (int64_t)j * K + k;
        const bool pinned = a.pin && k == K - 1;
        const T bt = Bv[e];
        const double b = (double)bt;
        const T gt = pinned ? T(0) : (T)((double)gacc[cb][nb][r] + prior_grad(b, a.prior, a.scale));
        Gv[e] = gt;
        pr += pinned ? 0.0 : prior_logd(b, a.prior, a.scale);
        if (a.mode != 0) {
          const T h = (T)a.h;
          T ev = Ev[e] + h * gt;                               // closing half kick
          if (a.mode == 1) {
            ev = ev + h * gt;                                  // opening half kick
            Bv[e] = pinned ? T(0) : bt + (T)a.eps * ev;        // position step
          } else {
            ke += 0.5 * (double)ev * (double)ev;
          }
          Ev[e] = ev;
        }
      }
  pr = wave_sum(pr);
  ke = wave_sum(ke);
  if (lane == 0) { sh4[0][w] = pr; sh4[1][w] = ke; }
  __syncthreads();
  if (tid == 0) {
    a.ppart[blockIdx.x] = ((sh4[0][0] + sh4[0][1]) + sh4[0][2]) + sh4[0][3];
    if (a.mode == 2) a.kpart[blockIdx.x] = ((sh4[1][0] + sh4[1][1]) + sh4[1][2]) + sh4[1][3];
  }
}

}  // namespace

template <typename T>
int wide_chunk_cols() { return kWideWaves * (sizeof(T) == 4 ? 16 : 8) * 16; }
// Workgroups of the column-owner gradient for p columns and NB class blocks: enough that none
// holds more than 4 CB blocks of 16 columns, in whole rounds of 256 compute units from 256 on.
// Below that, 256 workgroups while that still gives every wave two blocks or more (at n = 2000,
// p = 50000, 256 workgroups of 12-13 blocks on two row slices streamed faster than 512 of 6 on
// one), and otherwise the fewest workgroups whose waves hold CB blocks each, the rows being
// split over more slices instead: a wave with one or two blocks keeps too few loads in flight
// (plan replays, FP32: n = 20000, K = 10 at p = 12000 / 16400 / 24000 took 458 / 618 / 910 us
// per gradient against 611 / 771 / 953 us with one block per wave in 256 workgroups, and the
// 36 problems of the batched workload with p > 1024 took 24% less time in all).
int wide_grad_groups(int64_t p, int nb, bool f64) {
  const int64_t nblk = (p + 15) / 16;
  const int cb = f64 ? (nb == 1 ? 2 : 1) : (nb == 1 ? 4 : nb == 2 ? 2 : 1);
  const int64_t need = (nblk + kWideWaves * cb - 1) / (kWideWaves * cb);
  if (need >= 256) return (int)((need + 255) / 256 * 256);
  if (nblk >= (int64_t)kWideWaves * 256 * 2) return 256;
  return (int)need;
}

template <typename T>
hipError_t launch_wide(const WideArgs& a, int nb, int logits_tiles_y, int softmax_wg, int grad_wg,
                       hipStream_t s) {
  const dim3 lg(a.nchunk, logits_tiles_y);
  const dim3 gg(grad_wg, a.nsplit);
#define HMC_WIDE(NB_)                                                                       \
  if (nb == NB_) {                                                                          \
    hipLaunchKernelGGL((wide_logits<T, NB_>), lg, dim3(kWideWaves * 64), 0, s, a);          \
    hipLaunchKernelGGL((wide_softmax<T, NB_>), dim3(softmax_wg), dim3(256), 0, s, a);       \
    hipLaunchKernelGGL((wide_grad<T, NB_>), gg, dim3(kWideWaves * 64), 0, s, a);           \
    return hipGetLastError();                                                               \
  }
  HMC_WIDE(1) HMC_WIDE(2) HMC_WIDE(4)
#undef HMC_WIDE
  return hipErrorInvalidValue;
}

template int wide_chunk_cols<float>();
template int wide_chunk_cols<double>();
template hipError_t launch_wide<float>(const WideArgs&, int, int, int, int, hipStream_t);
template hipError_t launch_wide<double>(const WideArgs&, int, int, int, int, hipStream_t);

}  // namespace hmcx
