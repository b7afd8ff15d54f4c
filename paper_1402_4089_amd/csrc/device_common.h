// Device-side helpers shared by the HIP kernels of libhmc (internal).
#pragma once
#include <math.h>

#include "internal.h"

namespace hmcx {
namespace dev {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;


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

// Softmax arithmetic. float: the hardware base-2 exponential and logarithm (about 1 ulp)
// on arguments scaled by log2(e), and the hardware reciprocal; the exponent argument is
// z - max <= 0, so its scaling error only touches classes of negligible probability.
// double: the correctly rounded library functions.
constexpr float kLog2e = 1.4426950408889634f, kLn2 = 0.6931471805599453f;
__device__ __forceinline__ float dev_exp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ __forceinline__ double dev_exp(double x) { return exp(x); }
__device__ __forceinline__ float dev_log(float x) { return __builtin_amdgcn_logf(x) * kLn2; }
__device__ __forceinline__ double dev_log(double x) { return log(x); }
__device__ __forceinline__ float dev_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double dev_rcp(double x) { return 1.0 / x; }

// Probit row term for w = s z (s = +1 for a success, -1 otherwise; z = x^T beta): the
// residual factor phi(w) / Phi(w) (the residual is s times it) and log Phi(w). With
// a = |w| / sqrt(2) and E = erfcx(a) = exp(a^2) erfc(a), in (0, 1], the lower tail is
// Phi(-|w|) = E exp(-a^2) / 2 =: t. Below w = 0: Phi(w) = t, so the ratio is
// sqrt(2 / pi) / E and log Phi(w) = log(E / 2) - a^2, both free of underflow however far
// out w lies. From w = 0 up: Phi(w) = 1 - t, the ratio is exp(-a^2) / (sqrt(2 pi) (1 - t))
// and log Phi(w) = log(1 - t), whose absolute error stays at rounding level even where t
// is below it. One erfcx, one exp and one log per row.
__device__ __forceinline__ void probit_row(double w, double& ratio, double& logp) {
  const double a = fabs(w) * 0.70710678118654752440;
  const double E = erfcx(a);
  const double ea = exp(-a * a);
  const double t = 0.5 * E * ea;
  const bool lower = w < 0.0;
  ratio = lower ? 0.79788456080286535588 / E : 0.39894228040143267794 * ea / (1.0 - t);
  logp = log(lower ? 0.5 * E : 1.0 - t) - (lower ? a * a : 0.0);
}
__device__ __forceinline__ void probit_row(float w, float& ratio, double& logp) {
  const float a = fabsf(w) * 0.70710678f;
  const float E = erfcxf(a);
  const float ea = dev_exp(-a * a);
  const float t = 0.5f * E * ea;
  const bool lower = w < 0.0f;
  ratio = lower ? 0.79788456f / E : 0.39894228f * ea / (1.0f - t);
  logp = (double)dev_log(lower ? 0.5f * E : 1.0f - t) - (lower ? (double)a * (double)a : 0.0);
}

// DPP move within a row of 16 lanes (quad_perm / half-row mirror / row mirror).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// s_waitcnt encodings (vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8) for waits
// the compiler's own counter tracking can see, unlike inline assembly.
constexpr int kWaitVm0 = 0x0F70;     // vmcnt(0)
constexpr int kWaitLgkm0 = 0xC07F;   // lgkmcnt(0)
// vmcnt(n): wait until at most n vector memory operations of this wave are in flight.
constexpr int wait_vm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x0F70; }
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kHalfMirror = 0x141, kRowMirror = 0x140;

// Reductions over the 16 lanes of a DPP row. Each stage combines a lane with a partner
// through a symmetric operation, so every lane ends with the bitwise-identical result.
template <typename T> __device__ __forceinline__ T max16(T v) {
  v = fmax(v, dpp<kQuadXor1>(v));
  v = fmax(v, dpp<kQuadXor2>(v));
  v = fmax(v, dpp<kHalfMirror>(v));
  return fmax(v, dpp<kRowMirror>(v));
}
template <typename T> __device__ __forceinline__ T sum16(T v) {
  v += dpp<kQuadXor1>(v);
  v += dpp<kQuadXor2>(v);
  v += dpp<kHalfMirror>(v);
  return v + dpp<kRowMirror>(v);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint64_t bytes) {
  const uint32_t nrec = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nrec, 0x00020000);
}


// Log prior density (constants dropped) and its derivative for one coefficient.
// Cauchy(0, s): -log(1 + (b/s)^2), derivative -2 b / (s^2 + b^2) (the Appendix's prior
// term with the sign of the derivative of -log(1 + b^2)); Gaussian N(0, s^2):
// -b^2 / (2 s^2), derivative -b / s^2.
__device__ __forceinline__ double prior_logd(double b, int prior, double s) {
  if (prior == 1) { const double r = b / s; return -log1p(r * r); }
  return -(b * b) / (2.0 * s * s);
}
__device__ __forceinline__ double prior_grad(double b, int prior, double s) {
  if (prior == 1) return -2.0 * b / (s * s + b * b);
  return -b / (s * s);
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 multiplies with the
// counter words, xor-mixed with the key; the key advances by two Weyl constants between
// rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}
__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
  const uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
  return ((double)v + 0.5) * 0x1.0p-53;
}
// Standard normal for flat coordinate e of (chain, iteration): Box-Muller on a pair.
__device__ __forceinline__ double philox_normal(uint64_t seed, int chain, int64_t iter, int64_t e) {
  uint32_t c[4] = {(uint32_t)(e >> 1), (uint32_t)iter, (uint32_t)chain, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double r = sqrt(-2.0 * log(u53(c[0], c[1])));
  double sn, cs;
  sincos(2.0 * M_PI * u53(c[2], c[3]), &sn, &cs);
  return (e & 1) ? r * sn : r * cs;
}
__device__ __forceinline__ double philox_uniform(uint64_t seed, int chain, int64_t iter) {
  uint32_t c[4] = {0u, (uint32_t)iter, (uint32_t)chain, 1u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  return u53(c[0], c[1]);
}

// bfloat16 of a float, rounded to nearest even.
__device__ __forceinline__ uint16_t bf16_from_f32(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float f32_from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Packed B operand of the split-precision contractions: for NB blocks of 16 classes, the
// fragment of k step j / 32 and block nb holds, for lane 16 ((j % 32) / 8) + (class % 16),
// the 8 coefficients of rows j - j % 8 .. j - j % 8 + 7 (the MFMA B input order), hi plane
// then lo plane 512 entries later. Index of the hi entry of (row j, class slot k16).
__device__ __forceinline__ int64_t packed_b_index(int NB, int nb, int64_t j, int k16) {
  const int64_t ks = j / 32;
  const int lane = 16 * (int)((j % 32) / 8) + k16;
  return ((ks * NB + nb) * 2) * 512 + lane * 8 + (j % 8);
}
// Store the bf16 hi/lo split of coefficient v at (row j, class slot k16 of block nb).
__device__ __forceinline__ void store_packed_b(uint16_t* bpk, int NB, int nb, int64_t j, int k16, float v) {
  const uint16_t h = bf16_from_f32(v);
  const int64_t i = packed_b_index(NB, nb, j, k16);
  bpk[i] = h;
  bpk[i + 512] = bf16_from_f32(v - f32_from_bf16(h));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

}  // namespace dev
}  // namespace hmcx
