// Fused log-posterior + gradient pass over X on CDNA4 matrix cores.
//
// For a 16-row tile X_t of X this computes, in one visit of the tile:
//   Z   = X_t B                        logits (Section 2.1, the XB product of (logkernelGPU))
//   l_i = z_{i,y_i} - logsumexp_k z_ik  log-likelihood terms (equations (loglike), (softmax))
//   R   = Y_t - softmax(Z)              residuals
//   G  += X_t^T R                       likelihood part of equation (gradient)
// so X is read from HBM once per gradient.
//
// Data movement. Tiles are copied HBM -> LDS by buffer loads that write LDS directly (no
// register staging); rows past n read as zero from the buffer bounds check. Two distinct
// static LDS tile buffers alternate (the tile loop is unrolled by two, so the compiler can
// prove a read of one buffer does not alias the copy into the other), and the copy of
// tile t+1 is issued between the logits MFMAs of tile t. The LDS tile is row-major without
// padding; the 16-byte chunk index inside a row is XOR-ed with (row mod 16), which makes
// both read patterns below free of bank conflicts.
//
// Math. NW waves (8 or 16: two or four per SIMD) split the 16-column blocks of a row
// padded to NW*MB*16 columns: wave w owns blocks w, w+NW, ... Logits: A operand = X rows (lane -> row l%16,
// 4 consecutive columns), B operand = this wave's coefficients, held in registers for the
// whole launch. Partial logits of the NW waves are summed through LDS in a fixed order;
// each of waves 0-3 then finishes the softmax of one accumulator register's rows (16
// lanes share a row; DPP reductions) and publishes R through LDS. Gradient: A operand =
// X^T (lane -> column l%16), B operand = R; choosing the k-index of each gradient MFMA to
// be the logits accumulator register lets R enter the second contraction in the layout
// the first one produced. Per-workgroup partial gradients are staged through LDS and
// written once, contiguously, at the end; the epilogue kernel reduces them in a fixed
// order, so results are bitwise reproducible.
#include "internal.h"

#include "device_common.h"

namespace hmcx {

using namespace dev;

template <typename T, int NW, int MB, int NB, int LINK>
__global__ __launch_bounds__(NW * 64) void fused_logpost_grad(FusedArgs a) {
  using M = Mma<T>;
  using acc_t = typename M::acc;
  constexpr int E = 16 / sizeof(T);               // elements per 16-byte chunk
  constexpr int COLS = NW * MB * 16;              // padded row length (elements)
  constexpr int CPR = COLS / E;                   // chunks per row
  constexpr int TILE = kTileRows * COLS;          // elements per tile buffer
  constexpr int LOADS = kTileRows * CPR / (64 * NW);   // direct loads per wave per tile
  constexpr int MSTEP = 16 * NW;                  // elements between a wave's blocks b, b + NW
  static_assert(NW >= 8, "waves 0-3 finish the softmax");
  static_assert(kTileRows * CPR % (64 * NW) == 0, "tile copy splits evenly over the waves");
  static_assert(LOADS % MB == 0, "whole copies between the logits MFMAs of a column block");

  __shared__ __align__(16) T xs0[TILE];
  __shared__ __align__(16) T xs1[TILE];
  __shared__ __align__(16) T zb[NW * NB * 256];   // partial logits: [nb][r][wave][lane]
  __shared__ __align__(16) T rb[NB * 256];        // residuals R, accumulator layout
  __shared__ double lred[4];
  __shared__ __align__(16) int yl0[64];           // labels of the tile in xs0 (first 16 used)
  __shared__ __align__(16) int yl1[64];           // labels of the tile in xs1

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  const int p = a.p, K = a.K;
  const int64_t n = a.n, ldx = a.ldx;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const T* __restrict__ B = static_cast<const T*>(a.B);

  // Tile-relative global byte offsets of this lane's direct loads (loop invariant):
  // LDS chunk q = (w*LOADS + k)*64 + lane holds row
  // r = q / CPR, chunk (q % CPR) ^ (r & 15). Bit k of zbits marks a chunk reaching past
  // column p: with padded rows (ldx > p) that padding is zeroed after it lands, so no
  // 0 * NaN can reach the logits; without padding those columns hold the next row's data.
  uint32_t goff[LOADS];
  uint32_t zbits = 0;
#pragma unroll
  for (int k = 0; k < LOADS; ++k) {
    const int q = (w * LOADS + k) * 64 + lane;
    const int r = q / CPR;
    const int c4 = (q % CPR) ^ (r & 15);
    goff[k] = (uint32_t)(((int64_t)r * ldx + (int64_t)c4 * E) * sizeof(T));
    if (c4 * E + E > p && ldx != p) zbits |= 1u << k;
  }
  const uint64_t x_bytes = (uint64_t)((n - 1) * ldx + p) * sizeof(T);

  // Lane-dependent parts of the two LDS read patterns (the swizzle only touches the low
  // four bits of the chunk index, so block b + NW is a fixed MSTEP elements further on).
  int rd1[E == 4 ? 1 : 2];            // logits A operand: row c, columns 16b + 4g + t
  if constexpr (E == 4) {
    rd1[0] = (c * CPR + ((4 * w + g) ^ c)) * E;
  } else {
    rd1[0] = (c * CPR + ((8 * w + 2 * g) ^ c)) * E;
    rd1[1] = (c * CPR + ((8 * w + 2 * g + 1) ^ c)) * E;
  }
  int rd2[4];                         // gradient A operand: row row(s, g), column 16b + c
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int row = M::row(s, g);
    if constexpr (E == 4)
      rd2[s] = (row * CPR + ((4 * w + (c >> 2)) ^ row)) * E + (c & 3);
    else
      rd2[s] = (row * CPR + ((8 * w + (c >> 1)) ^ row)) * E + (c & 1);
  }

  // Waves 0-3 own the softmax of accumulator register r = w: row my_row of the tile.
  const int my_row = w < 4 ? M::row(w, g) : 0;

  __amdgpu_buffer_rsrc_t xr_next;
  // Resource for the copy of tile t, plus the copy of its labels to LDS (64 lanes x 4 bytes
  // of which the first 16 belong to the tile; reads past n give 0). Past the last tile
  // the resource has no records: the copies then read zeros into the spare buffer, which
  // keeps the issue free of branches (the compiler tracks in-flight copies per buffer only
  // along straight-line code).
  // The label resource starts at the tile's first row, so its offsets stay small at any n.
  auto set_next = [&](int64_t t, int* ydst) {
    const bool real = t < a.ntiles;
    const uint64_t base_off = real ? (uint64_t)(t * kTileRows) * ldx * sizeof(T) : 0;
    xr_next = make_rsrc(reinterpret_cast<const char*>(X) + base_off, real ? x_bytes - base_off : 0);
    if (w == 0) {
      const int64_t r0 = real ? t * kTileRows : 0;
      const __amdgpu_buffer_rsrc_t yr = make_rsrc(a.y + r0, real ? (uint64_t)(n - r0) * 4 : 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(yr, (lds_void*)ydst, 4, lane * 4, 0, 0, 0);
    }
  };
#define HMC_ISSUE(K_, DST)                                                                   \
  __builtin_amdgcn_raw_ptr_buffer_load_lds(                                                 \
      xr_next, (lds_void*)((DST) + (w * LOADS + (K_)) * 64 * E), 16, (int)goff[K_], 0, 0, 0)

  // Every wave copies its share of the first tile before the coefficients are loaded.
  if ((int64_t)blockIdx.x < a.ntiles) {
    set_next(blockIdx.x, yl0);
#pragma unroll
    for (int k = 0; k < LOADS; ++k) HMC_ISSUE(k, xs0);
  }

  // Coefficients in B-operand layout: bt[m][nb][t] = beta[16 b + 4 g + t][16 nb + c],
  // block b = w + NW m; zero beyond p and K, and in the pinned column (beta_K = 0 in the
  // model, whatever the caller's buffer holds there).
  const int kmax = a.pin ? K - 1 : K;
  T bt[MB][NB][4];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int k = nb * 16 + c;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = (w + NW * m) * 16 + 4 * g + t;
        bt[m][nb][t] = (j < p && k < kmax) ? B[(int64_t)j * K + k] : T(0);
      }
    }
  }
  acc_t gacc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) gacc[m][nb] = acc_t{0, 0, 0, 0};
  double lacc = 0.0;

  // One tile: wait for its copy, then the math; the copy waves (4..) start the next
  // tile into `nxt` right after the first barrier.
  // Every LDS array reaches the step through a __restrict__ parameter: the resulting alias
  // scopes let the compiler see that reads of one buffer cannot observe the direct loads
  // into another, so it does not wait for the copy in flight before them.
  auto step = [&](int64_t tile, T* __restrict__ cur, T* __restrict__ nxt,
                  const int* __restrict__ ycur, int* __restrict__ ynxt, T* __restrict__ zx,
                  T* __restrict__ rx) {
    __builtin_amdgcn_s_waitcnt(kWaitVm0);               // this wave's copies of `tile` landed
    if (zbits) {
      // Columns past p hold the next row's data or row padding: zero them so no 0 * NaN
      // can reach the logits. Only lanes whose chunk reaches past p take this branch.
#pragma nounroll
      for (int k = 0; k < LOADS; ++k) {
        if ((zbits >> k) & 1u) {
          const int q = (w * LOADS + k) * 64 + lane;
          const int r = q / CPR;
          const int col = ((q % CPR) ^ (r & 15)) * E;
#pragma unroll
          for (int e = 0; e < E; ++e)
            if (col + e >= p) cur[q * E + e] = T(0);
        }
      }
    }
    __syncthreads();                                     // all copies landed; `nxt` is free
    set_next(tile + gridDim.x, ynxt);
    const int64_t i0 = tile * kTileRows;

    // ---- logits: Z = X_t B over this wave's column blocks (two accumulator chains)
    T av[MB][4];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      if constexpr (E == 4) {
        const float4 q = *reinterpret_cast<const float4*>(cur + rd1[0] + m * MSTEP);
        av[m][0] = q.x; av[m][1] = q.y; av[m][2] = q.z; av[m][3] = q.w;
      } else {
        const double2 q0 = *reinterpret_cast<const double2*>(cur + rd1[0] + m * MSTEP);
        const double2 q1 = *reinterpret_cast<const double2*>(cur + rd1[1] + m * MSTEP);
        av[m][0] = q0.x; av[m][1] = q0.y; av[m][2] = q1.x; av[m][3] = q1.y;
      }
    }
    // All operand reads are issued before the first MFMA: left to itself, the scheduler
    // waits for each read right before its four MFMAs, exposing every LDS latency.
    __builtin_amdgcn_sched_barrier(0);
    acc_t z0[NB], z1[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) z0[nb] = z1[nb] = acc_t{0, 0, 0, 0};
    // The copy of the next tile is issued in LOADS / MB pieces between the column blocks'
    // MFMAs, so the address unit works while the matrix core does.
#pragma unroll
    for (int m = 0; m < MB; ++m) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          if (m & 1) z1[nb] = M::run(av[m][t], bt[m][nb][t], z1[nb]);
          else       z0[nb] = M::run(av[m][t], bt[m][nb][t], z0[nb]);
        }
#pragma unroll
      for (int k = m * (LOADS / MB); k < (m + 1) * (LOADS / MB); ++k) HMC_ISSUE(k, nxt);
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      __builtin_amdgcn_sched_group_barrier(0x008, 4 * NB, 0);        // MFMA
      __builtin_amdgcn_sched_group_barrier(0x020, LOADS / MB, 0);    // VMEM read
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) zx[((nb * 4 + r) * NW + w) * 64 + lane] = z0[nb][r] + z1[nb][r];
    // LDS-only barriers below: a full __syncthreads() would also wait for the copy in flight.
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);

    // The gradient's X^T operands do not depend on the softmax: read them now, so the
    // reads overlap the barrier and the softmax.
    // In a partial last tile, rows past n are zeroed so that nothing in LDS beyond the
    // data (stale or uninitialised) can reach G through a 0 * NaN product.
    T xa[MB][4];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int s = 0; s < 4; ++s) xa[m][s] = cur[rd2[s] + m * MSTEP];
    __builtin_amdgcn_s_barrier();

    // ---- softmax and residuals for accumulator register r = w (waves 0-3)
    if (w < 4) {
      const int r = w;
      const int yi = ycur[my_row];
      T zz[NB], zpart[NB][NW];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const T* zp = zx + (nb * 4 + r) * NW * 64 + lane;   // wave w2's partial at zp[64 w2]
#pragma unroll
        for (int w2 = 0; w2 < NW; ++w2) zpart[nb][w2] = zp[64 * w2];
      }
      __builtin_amdgcn_sched_barrier(0);                  // all partial reads in flight
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        T sum = zpart[nb][0];
#pragma unroll
        for (int w2 = 1; w2 < NW; ++w2) sum += zpart[nb][w2];
        zz[nb] = sum;
      }
      const bool valid = i0 + my_row < n;
      if constexpr (LINK == 1) {
        // Poisson link, one coefficient column: lane c = 0 of each row holds z = x_i beta;
        // residual y_i - exp(z), log-likelihood term y_i z - exp(z) (no log y_i!)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bool use = valid && nb * 16 + c == 0;
          const T mu = use ? dev_exp(zz[nb]) : T(0);
          rx[(nb * 64 + lane) * 4 + r] = use ? T(yi) - mu : T(0);
          lacc += use ? (double)yi * (double)zz[nb] - (double)mu : 0.0;
        }
      } else if constexpr (LINK == 2) {
        // probit link, one coefficient column: lane c = 0 of each row holds z; with s = +1
        // for a success and -1 otherwise, residual s phi(z) / Phi(s z), term log Phi(s z)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const bool use = valid && nb * 16 + c == 0;
          const T s = yi == 1 ? T(1) : T(-1);
          T ratio;
          double lp;
          probit_row(use ? s * zz[nb] : T(0), ratio, lp);
          rx[(nb * 64 + lane) * 4 + r] = use ? s * ratio : T(0);
          lacc += use ? lp : 0.0;
        }
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
        const T lse_shift = dev_log(se);                  // LSE - max, in [0, log K]
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int k = nb * 16 + c;
          const bool hit = valid && k == yi;
          rx[(nb * 64 + lane) * 4 + r] =
              (valid && k < K) ? ((hit ? T(1) : T(0)) - ex[nb] * inv) : T(0);
          lacc += hit ? (double)((zz[nb] - mx) - lse_shift) : 0.0;
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_s_barrier();
    T rr[NB][4];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      if constexpr (E == 4) {
        const float4 q = *reinterpret_cast<const float4*>(rx + (nb * 64 + lane) * 4);
        rr[nb][0] = q.x; rr[nb][1] = q.y; rr[nb][2] = q.z; rr[nb][3] = q.w;
      } else {
        const double2 q0 = *reinterpret_cast<const double2*>(rx + (nb * 64 + lane) * 4);
        const double2 q1 = *reinterpret_cast<const double2*>(rx + (nb * 64 + lane) * 4 + 2);
        rr[nb][0] = q0.x; rr[nb][1] = q0.y; rr[nb][2] = q1.x; rr[nb][3] = q1.y;
      }
    }

    // ---- gradient: G_blk += X_t^T R; step s takes rows row(s, g), so R is register s.
    if (i0 + kTileRows > n) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (i0 + M::row(s, g) >= n)
#pragma unroll
          for (int m = 0; m < MB; ++m) xa[m][s] = T(0);
    }
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) gacc[m][nb] = M::run(xa[m][s], rr[nb][s], gacc[m][nb]);
  };

  int64_t tile = blockIdx.x;
  // Unrolled by two so each buffer is named statically in the code that reads it.
  while (tile < a.ntiles) {
    step(tile, xs0, xs1, yl0, yl1, zb, rb);
    tile += gridDim.x;
    if (tile >= a.ntiles) break;
    step(tile, xs1, xs0, yl1, yl0, zb, rb);
    tile += gridDim.x;
  }
#undef HMC_ISSUE

  // ---- per-workgroup partials: log-likelihood, then the p x K gradient block
  double lw = lacc;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) lw += __shfl_xor(lw, m, 64);
  __syncthreads();                                       // tile buffers free for staging
  if (w < 4 && lane == 0) lred[w] = lw;
  T* gp = static_cast<T*>(a.gpart) + (int64_t)blockIdx.x * a.gstride;
  if constexpr (NB <= 2) {
    // stage p x K in the two tile buffers (2 * TILE >= COLS * 16 * NB elements)
    T* st = xs0;
    static_assert(2 * TILE >= COLS * 16 * NB, "staging fits the tile buffers");
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int k = nb * 16 + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = (w + NW * m) * 16 + M::row(r, g);
          if (j < p && k < K) {
            T* dst = (j * K + k < TILE) ? xs0 + (j * K + k) : xs1 + (j * K + k - TILE);
            *dst = gacc[m][nb][r];
          }
        }
      }
    __syncthreads();
    // 16-byte non-temporal copies out (a partial starts 256-byte aligned; TILE is a multiple
    // of V, so no vector straddles the two buffers), then the few trailing elements one by
    // one. The partials are read once, by the epilogue kernel: streaming them past the
    // caches shortened the pass by 0.8 us (of 21).
    constexpr int V = 16 / sizeof(T);
    static_assert(TILE % V == 0, "vectors stay inside one staging buffer");
    typedef __attribute__((ext_vector_type(V))) T vec_t;
    const int pk = p * K, pkv = pk / V * V;
    for (int e = tid * V; e < pkv; e += NW * 64 * V)
      __builtin_nontemporal_store(*reinterpret_cast<const vec_t*>(e < TILE ? st + e : xs1 + (e - TILE)),
                                  reinterpret_cast<vec_t*>(gp + e));
    for (int e = pkv + tid; e < pk; e += NW * 64) gp[e] = (e < TILE) ? st[e] : xs1[e - TILE];
  } else {
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int k = nb * 16 + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = (w + NW * m) * 16 + M::row(r, g);
          if (j < p && k < K) gp[(int64_t)j * K + k] = gacc[m][nb][r];
        }
      }
    __syncthreads();
  }
  if (tid == 0) a.lpart[blockIdx.x] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
}

namespace {

// The link is a template parameter so that the softmax kernels carry no branch for it; the
// Poisson and probit links have one coefficient column, so only one-block variants exist
// for them.
template <typename T, int NW, int MB, int NB>
hipError_t launch_one(const FusedArgs& a, int nwg, hipStream_t s) {
  if (a.link == 1 || a.link == 2) {
    if constexpr (NB == 1) {
      if (a.link == 1)
        hipLaunchKernelGGL((fused_logpost_grad<T, NW, MB, 1, 1>), dim3(nwg), dim3(NW * 64), 0, s,
                           a);
      else
        hipLaunchKernelGGL((fused_logpost_grad<T, NW, MB, 1, 2>), dim3(nwg), dim3(NW * 64), 0, s,
                           a);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((fused_logpost_grad<T, NW, MB, NB, 0>), dim3(nwg), dim3(NW * 64), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// Instantiated variants: (waves, column blocks per wave, 16-class blocks). The static LDS
// of a variant is 2 tiles of 16 x (waves * blocks * 16) elements plus the exchanges.
#define HMC_FUSED_VARIANTS_F32(X_) \
  X_(16, 1, 1) X_(16, 2, 1) X_(16, 4, 1) \
  X_(8, 1, 1) X_(8, 2, 1) X_(8, 4, 1) X_(8, 8, 1) X_(8, 1, 2) X_(8, 2, 2) X_(8, 4, 2) \
  X_(8, 1, 4) X_(8, 2, 4) X_(8, 4, 4)
#define HMC_FUSED_VARIANTS_F64(X_) \
  X_(8, 1, 1) X_(8, 2, 1) X_(8, 4, 1) X_(8, 1, 2) X_(8, 2, 2) X_(8, 1, 4)

template <> bool fused_variant_exists<float>(int waves, int mb, int nb) {
#define HMC_CHECK(W_, MB_, NB_) if (waves == W_ && mb == MB_ && nb == NB_) return true;
  HMC_FUSED_VARIANTS_F32(HMC_CHECK)
  return false;
}
template <> bool fused_variant_exists<double>(int waves, int mb, int nb) {
  HMC_FUSED_VARIANTS_F64(HMC_CHECK)
#undef HMC_CHECK
  return false;
}

#define HMC_LAUNCH_T(T_, W_, MB_, NB_) \
  if (waves == W_ && mb == MB_ && nb == NB_) return launch_one<T_, W_, MB_, NB_>(a, nwg, s);
#define HMC_LAUNCH_F32(W_, MB_, NB_) HMC_LAUNCH_T(float, W_, MB_, NB_)
#define HMC_LAUNCH_F64(W_, MB_, NB_) HMC_LAUNCH_T(double, W_, MB_, NB_)

template <> hipError_t launch_fused<float>(const FusedArgs& a, int nwg, int waves, int mb, int nb,
                                           size_t, hipStream_t s) {
  HMC_FUSED_VARIANTS_F32(HMC_LAUNCH_F32)
  return hipErrorInvalidValue;
}
template <> hipError_t launch_fused<double>(const FusedArgs& a, int nwg, int waves, int mb, int nb,
                                            size_t, hipStream_t s) {
  HMC_FUSED_VARIANTS_F64(HMC_LAUNCH_F64)
  return hipErrorInvalidValue;
}
#undef HMC_LAUNCH_F64
#undef HMC_LAUNCH_F32
#undef HMC_LAUNCH_T

}  // namespace hmcx
