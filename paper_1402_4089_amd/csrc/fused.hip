// Fused log-posterior + gradient pass over X on CDNA4 matrix cores.
//
// For a 16-row tile X_t of X this computes, in one visit of the tile:
//   Z   = X_t B                        logits (Section 2.1, the XB product of (logkernelGPU))
//   l_i = z_{i,y_i} - logsumexp_k z_ik  log-likelihood terms (equations (loglike), (softmax))
//   R   = Y_t - softmax(Z)              residuals
//   G  += X_t^T R                       likelihood part of equation (gradient)
// so X is read from HBM once per gradient. The tile is staged in LDS and read twice in
// the two lane layouts the two contractions need:
//   * logits: A operand = X rows (lane -> row l%16, four consecutive columns), B operand
//     = coefficients held in registers for the wave's column blocks;
//   * gradient: A operand = X^T (lane -> column l%16, rows), B operand = R. R leaves the
//     logits MFMA in the accumulator layout; picking the k-index of each gradient MFMA
//     step to be the accumulator register lets R feed the second MFMA with no shuffle.
// Each wave owns column blocks b = w, w+NW, ... of 16 columns; partial logits of the NW
// waves are summed through LDS in a fixed order. Softmax row reductions run across the
// 16 lanes that share a row. Per-workgroup partial gradients are written once at the end
// and reduced by the epilogue kernel in a fixed order (bitwise reproducible).
#include "internal.h"

namespace hmcx {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef f32x4 acc;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // Output row held in accumulator register r by a lane of input block g (= lane / 16).
  static __device__ __forceinline__ int row(int r, int g) { return 4 * g + r; }
};
template <> struct Mma<double> {
  typedef f64x4 acc;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int g) { return 4 * r + g; }
};

template <typename T> struct alignas(16) Quad { T v[4]; };

template <typename T>
__device__ __forceinline__ Quad<T> load_quad_aligned(const T* p) {
  Quad<T> q;
  if constexpr (sizeof(T) == 4) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    q.v[0] = f.x; q.v[1] = f.y; q.v[2] = f.z; q.v[3] = f.w;
  } else {
    const double2 f0 = *reinterpret_cast<const double2*>(p);
    const double2 f1 = *reinterpret_cast<const double2*>(p + 2);
    q.v[0] = f0.x; q.v[1] = f0.y; q.v[2] = f1.x; q.v[3] = f1.y;
  }
  return q;
}

template <typename T> __device__ __forceinline__ T dev_exp(T x);
template <> __device__ __forceinline__ float dev_exp(float x) { return expf(x); }
template <> __device__ __forceinline__ double dev_exp(double x) { return exp(x); }
template <typename T> __device__ __forceinline__ T dev_log(T x);
template <> __device__ __forceinline__ float dev_log(float x) { return logf(x); }
template <> __device__ __forceinline__ double dev_log(double x) { return log(x); }

template <typename T>
__device__ __forceinline__ T max16(T v) {
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) v = fmax(v, __shfl_xor(v, m, 16));
  return v;
}
template <typename T>
__device__ __forceinline__ T sum16(T v) {
#pragma unroll
  for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 16);
  return v;
}

template <typename T, int NW, int MB, int NB>
__global__ __launch_bounds__(NW * 64) void fused_logpost_grad(FusedArgs a) {
  using M = Mma<T>;
  using acc_t = typename M::acc;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);               // kTileRows x pitch
  T* zb = xs + kTileRows * a.pitch;                      // NW x NB x 64 lanes x 4

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int p = a.p, K = a.K, nblk = a.nblk, pitch = a.pitch;
  const int cpr = nblk * 4;                              // 4-element chunks per tile row
  const int nch = kTileRows * cpr;
  const int64_t n = a.n, ldx = a.ldx;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const T* __restrict__ B = static_cast<const T*>(a.B);
  const int32_t* __restrict__ y = a.y;

  // Coefficients of this wave's column blocks in B-operand layout: bt[m][nb][t] is
  // beta[16 b + 4 g + t][16 nb + c] for block b = w + NW m.
  T bt[MB][NB][4];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int b = w + NW * m;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int k = nb * 16 + c;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = b * 16 + 4 * g + t;
        bt[m][nb][t] = (b < nblk && j < p && k < K) ? B[(int64_t)j * K + k] : T(0);
      }
    }
  }
  acc_t gacc[MB][NB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) gacc[m][nb] = acc_t{0, 0, 0, 0};
  double lacc = 0.0;

  // Register staging of the next tile (chunk q = tid + NW*64*s holds 4 elements).
  Quad<T> pf[MB];
  auto load_tile = [&](int64_t tile) {
    const int64_t i0 = tile * kTileRows;
#pragma unroll
    for (int s = 0; s < MB; ++s) {
      const int q = tid + NW * 64 * s;
      Quad<T> v;
      v.v[0] = v.v[1] = v.v[2] = v.v[3] = T(0);
      if (q < nch) {
        const int row = q / cpr, col = (q - row * cpr) * 4;
        const int64_t i = i0 + row;
        if (i < n) {
          const T* src = X + i * ldx + col;
          if (a.vec && col + 3 < p) {
            v = load_quad_aligned(src);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (col + e < p) v.v[e] = src[e];
          }
        }
      }
      pf[s] = v;
    }
  };
  auto store_tile = [&]() {
#pragma unroll
    for (int s = 0; s < MB; ++s) {
      const int q = tid + NW * 64 * s;
      if (q < nch) {
        const int row = q / cpr, col = (q - row * cpr) * 4;
        *reinterpret_cast<Quad<T>*>(xs + row * pitch + col) = pf[s];
      }
    }
  };

  int64_t tile = blockIdx.x;
  if (tile < a.ntiles) load_tile(tile);
  for (; tile < a.ntiles; tile += gridDim.x) {
    __syncthreads();                                     // previous tile fully consumed
    store_tile();
    __syncthreads();
    if (tile + gridDim.x < a.ntiles) load_tile(tile + gridDim.x);   // overlaps the math

    // ---- logits: Z = X_t B over this wave's column blocks
    acc_t z[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) z[nb] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int b = w + NW * m;
      if (b < nblk) {
        const Quad<T> av = *reinterpret_cast<const Quad<T>*>(xs + c * pitch + b * 16 + 4 * g);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) z[nb] = M::run(av.v[t], bt[m][nb][t], z[nb]);
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) zb[((w * NB + nb) * 64 + lane) * 4 + r] = z[nb][r];
    __syncthreads();

    // ---- softmax and residuals (every wave, redundantly; wave 0 also sums l_i)
    T rr[NB][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      T zz[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        T s = T(0);
#pragma unroll
        for (int w2 = 0; w2 < NW; ++w2) s += zb[((w2 * NB + nb) * 64 + lane) * 4 + r];
        zz[nb] = s;
      }
      const int64_t i = tile * kTileRows + M::row(r, g);
      const bool valid = i < n;
      const int yi = valid ? y[i] : -1;
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
      const T inv = T(1) / se;
      const T lse_shift = dev_log(se);                  // LSE - max, in [0, log K]
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int k = nb * 16 + c;
        const bool hit = valid && k == yi;
        rr[nb][r] = (valid && k < K) ? ((hit ? T(1) : T(0)) - ex[nb] * inv) : T(0);
        if (w == 0 && hit) lacc += (double)((zz[nb] - mx) - lse_shift);
      }
    }

    // ---- gradient: G_blk += X_t^T R, step s takes rows row(s, g) so R is register s
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int b = w + NW * m;
      if (b < nblk) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const T xa = xs[M::row(s, g) * pitch + b * 16 + c];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) gacc[m][nb] = M::run(xa, rr[nb][s], gacc[m][nb]);
        }
      }
    }
  }

  // ---- per-workgroup partials
  T* gp = static_cast<T*>(a.gpart) + (int64_t)blockIdx.x * p * K;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    const int b = w + NW * m;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int k = nb * 16 + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = b * 16 + M::row(r, g);
        if (b < nblk && j < p && k < K) gp[(int64_t)j * K + k] = gacc[m][nb][r];
      }
    }
  }
  if (w == 0) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) lacc += __shfl_xor(lacc, m, 64);
    if (lane == 0) a.lpart[blockIdx.x] = lacc;
  }
}

template <typename T, int NW, int MB, int NB>
hipError_t launch_one(const FusedArgs& a, int nwg, size_t lds, hipStream_t s) {
  auto fn = fused_logpost_grad<T, NW, MB, NB>;
  static size_t configured = 0;
  if (lds > 65536 && lds > configured) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    configured = lds;
  }
  hipLaunchKernelGGL(fn, dim3(nwg), dim3(NW * 64), lds, s, a);
  return hipGetLastError();
}

}  // namespace

// Instantiated variants: (waves, column blocks per wave, 16-class blocks).
#define HMC_FUSED_VARIANTS(X_) \
  X_(4, 1, 1) X_(4, 2, 1) X_(4, 4, 1) X_(4, 8, 1) X_(4, 16, 1) \
  X_(4, 1, 2) X_(4, 2, 2) X_(4, 4, 2) X_(4, 8, 2)              \
  X_(4, 1, 4) X_(4, 2, 4) X_(4, 4, 4)

template <typename T>
bool fused_variant_exists(int waves, int mb, int nb) {
#define HMC_CHECK(W_, MB_, NB_) \
  if (waves == W_ && mb == MB_ && nb == NB_) return !(sizeof(T) == 8 && MB_ * NB_ > 8);
  HMC_FUSED_VARIANTS(HMC_CHECK)
#undef HMC_CHECK
  return false;
}

template <typename T>
hipError_t launch_fused(const FusedArgs& a, int nwg, int waves, int mb, int nb, size_t lds,
                        hipStream_t s) {
#define HMC_LAUNCH(W_, MB_, NB_) \
  if (waves == W_ && mb == MB_ && nb == NB_) return launch_one<T, W_, MB_, NB_>(a, nwg, lds, s);
  HMC_FUSED_VARIANTS(HMC_LAUNCH)
#undef HMC_LAUNCH
  return hipErrorInvalidValue;
}

template bool fused_variant_exists<float>(int, int, int);
template bool fused_variant_exists<double>(int, int, int);
template hipError_t launch_fused<float>(const FusedArgs&, int, int, int, int, size_t, hipStream_t);
template hipError_t launch_fused<double>(const FusedArgs&, int, int, int, int, size_t, hipStream_t);

}  // namespace hmcx
