// Posterior-predictive classification (Section 3.2): for each row x_i of a data set, the
// mean over S coefficient samples B_s of the class probabilities softmax(x_i^T B_s),
// accumulated in float64, and the class of highest mean probability.
//
// One workgroup of 256 threads per 16-row tile: the tile of X is staged in LDS once and
// reused for every sample; each sample's coefficients are staged in LDS in turn. Thread
// (r, c) = (tid / 16, tid % 16) owns row r of the tile and the classes c, c + 16, ... of a
// sample's logits (the 16 lanes of a row form one DPP row, so the softmax max and sum are
// DPP reductions); the float64 running sums of the probabilities stay in its registers.
#include <math.h>

#include "device_common.h"

namespace hmcx {
namespace {

using namespace dev;

template <typename T, int NB>
__global__ __launch_bounds__(256) void predict_kernel(PredictArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* xs = reinterpret_cast<T*>(smem);                       // [16][p]
  T* bs = xs + 16 * (int64_t)a.p;                           // [p][K] of the current sample
  const int tid = threadIdx.x, r = tid >> 4, c = tid & 15;
  const int p = a.p, K = a.K;
  const int kmax = a.pin ? K - 1 : K;
  const int64_t n = a.n, ldx = a.ldx;
  const T* X = static_cast<const T*>(a.X);
  const T* S = static_cast<const T*>(a.samples);
  const int64_t pk = (int64_t)p * K;
  for (int64_t tile = blockIdx.x; tile * 16 < n; tile += gridDim.x) {
    const int64_t i0 = tile * 16;
    __syncthreads();                                        // previous tile's readers done
    for (int64_t e = tid; e < 16 * (int64_t)p; e += 256) {
      const int64_t rr = e / p, j = e - rr * p;
      xs[e] = (i0 + rr < n) ? X[(i0 + rr) * ldx + j] : T(0);
    }
    double acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = 0.0;
    for (int s = 0; s < a.n_samples; ++s) {
      __syncthreads();                                      // previous sample's readers done
      const T* Bs = S + (int64_t)s * pk;
      for (int64_t e = tid; e < pk; e += 256) bs[e] = Bs[e];
      __syncthreads();
      T z[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) z[q] = T(0);
      const T* xr = xs + (int64_t)r * p;
      for (int j = 0; j < p; ++j) {
        const T xv = xr[j];
        const T* br = bs + (int64_t)j * K;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const int k = 16 * q + c;
          z[q] += xv * (k < kmax ? br[k] : T(0));
        }
      }
      // softmax over the K classes of row r (the pinned class, if any, keeps logit 0)
      T mx = -INFINITY;
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (16 * q + c < K) mx = fmax(mx, z[q]);
      mx = max16(mx);
      T ex[NB], se = T(0);
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        ex[q] = (16 * q + c < K) ? exp(z[q] - mx) : T(0);
        se += ex[q];
      }
      se = sum16(se);
#pragma unroll
      for (int q = 0; q < NB; ++q) acc[q] += (double)ex[q] / (double)se;
    }
    // mean probabilities and the class of the largest (lowest index among exact ties)
    const int64_t i = i0 + r;
    const double inv = 1.0 / (double)a.n_samples;
    double best = -1.0;
    int bk = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int k = 16 * q + c;
      const double m = acc[q] * inv;
      if (k < K && i < n && a.mean_prob) a.mean_prob[i * K + k] = m;
      if (k < K && m > best) { best = m; bk = k; }
    }
    // argmax across the 16 lanes of the row: compare (value, -index) pairs
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) {
      const double ob = __shfl_xor(best, m, 64);
      const int ok = __shfl_xor(bk, m, 64);
      if (ob > best || (ob == best && ok < bk)) { best = ob; bk = ok; }
    }
    if (c == 0 && i < n && a.classes) a.classes[i] = bk;
  }
}

}  // namespace

size_t predict_lds_bytes(int64_t p, int K, bool f64) {
  return (size_t)(16 * p + p * K) * (f64 ? 8 : 4);
}

template <typename T>
hipError_t launch_predict(const PredictArgs& a, hipStream_t s) {
  const int64_t tiles = (a.n + 15) / 16;
  const int grid = (int)(tiles < 16384 ? tiles : 16384);
  const size_t lds = predict_lds_bytes(a.p, a.K, sizeof(T) == 8);
  const int nb = (a.K + 15) / 16;
#define HMC_PRED(NB_)                                                                     \
  if (nb == NB_) {                                                                        \
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&predict_kernel<T, NB_>), \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    if (e != hipSuccess) return e;                                                        \
    hipLaunchKernelGGL((predict_kernel<T, NB_>), dim3(grid), dim3(256), lds, s, a);       \
    return hipGetLastError();                                                             \
  }
  HMC_PRED(1) HMC_PRED(2) HMC_PRED(3) HMC_PRED(4)
#undef HMC_PRED
  return hipErrorInvalidValue;
}

template hipError_t launch_predict<float>(const PredictArgs&, hipStream_t);
template hipError_t launch_predict<double>(const PredictArgs&, hipStream_t);

}  // namespace hmcx
