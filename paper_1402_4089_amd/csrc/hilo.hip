// Split-precision form of the gradient pass. X is stored as two bfloat16 planes
// (hi = bf16(X), lo = bf16(X - hi)); the FP32 operands it meets (the coefficients B and
// the residuals R = Y - P) are split the same way on the fly, and each contraction sums
// the three products hi*hi + hi*lo + lo*hi on the BF16 matrix cores (v_mfma 16x16x32)
// with FP32 accumulation. Softmax statistics (log-sum-exp, the log-likelihood) are
// formed in FP64.
//
// The per-class gradient of this form does not fit one compute unit (p*K FP32
// accumulators exceed its register file), so the pass runs as two kernels: row blocks
// compute logits, softmax and the packed residual; column blocks then accumulate
// X^T R over a slice of rows each, and the shared epilogue sums the slices.
#include <math.h>

#include "device_common.h"

namespace hmcx {
namespace {

using namespace dev;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// bfloat16 of a double, rounded once to nearest even: 8 significant bits, the exponent
// range of binary32 (subnormals spaced 2^-133), +-inf past the largest finite value.
__device__ __forceinline__ u16 bf16_from_f64(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const u16 sign = (u16)((u >> 48) & 0x8000u);
  const int E = (int)((u >> 52) & 0x7FF);
  const uint64_t man = u & 0xFFFFFFFFFFFFFull;
  if (E == 0x7FF) return (u16)(sign | (man ? 0x7FC0u : 0x7F80u));
  const int e = E - 1023;
  if (e < -126) {
    // below the normal range: a multiple of 2^-133, found by exact scaling and rint
    const double t = rint(fabs(x) * 0x1.0p133);
    return (u16)(sign | (u16)t);
  }
  if (e > 127) return (u16)(sign | 0x7F80u);
  const uint32_t keep = (uint32_t)(man >> 45);
  const uint64_t rem = man & ((1ull << 45) - 1);
  const uint64_t half = 1ull << 44;
  uint32_t v = ((uint32_t)(e + 127) << 7) | keep;
  if (rem > half || (rem == half && (keep & 1u))) ++v;   // a carry moves into the exponent
  if (v > 0x7F80u) v = 0x7F80u;
  return (u16)(sign | v);
}


__device__ __forceinline__ uint32_t pack2(u16 a, u16 b) { return (uint32_t)a | ((uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 as_frag(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------------------
// Encoding of X: one thread per 8 output columns of a row; columns [p, ldo) are zeroed.
template <typename Tin>
__global__ __launch_bounds__(256) void split_kernel(const Tin* __restrict__ X, int64_t ldx,
                                                    int64_t n, int64_t p, u16* __restrict__ hi,
                                                    u16* __restrict__ lo, int64_t ldo) {
  const int64_t gpr = ldo / 8;
  const int64_t total = n * gpr;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int64_t i = t / gpr;
    const int64_t c0 = (t - i * gpr) * 8;
    u16 h[8], l[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      h[j] = 0;
      l[j] = 0;
      if (c0 + j < p) {
        const double x = (double)X[i * ldx + c0 + j];
        h[j] = bf16_from_f64(x);
        l[j] = bf16_from_f64(x - (double)f32_from_bf16(h[j]));
      }
    }
    const u32x4 hv = {pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
    *reinterpret_cast<u32x4*>(hi + i * ldo + c0) = hv;
    if (lo) {
      const u32x4 lv = {pack2(l[0], l[1]), pack2(l[2], l[3]), pack2(l[4], l[5]), pack2(l[6], l[7])};
      *reinterpret_cast<u32x4*>(lo + i * ldo + c0) = lv;
    }
  }
}

// ---------------------------------------------------------------------------------------
// One problem's operands for the split-precision bodies below. Class blocks: the padded
// class axis is NB blocks of 16, in softmax groups of GROUP blocks. With GROUP == NB the
// blocks are one problem's K <= 16 NB classes (one softmax per row); with GROUP < NB each
// group is a separate chain of the same problem with K <= 16 GROUP classes (NB / GROUP
// chains share every pass over X, one softmax per row and chain). A chain's state,
// gradient and partials are chain-major [chain][p][K].
struct Job {
  const u16* Xhi;
  const u16* Xlo;
  int64_t ldx;
  const int32_t* y;
  int64_t n;
  int p, K;
  const float* B;
  u16* Bpk;
  u16* Rpk;
  int pin;                 // 1: column K-1 of B is packed as zero (beta_K = 0)
};

// B -> packed hi/lo operand in the lane order of the MFMA B input: fragment (k-step s,
// class block nb, plane) holds, for lane l, the 8 values B[32 s + 8 (l / 16) + j][class
// 16 nb + l % 16 of the block's group], j = 0..7. Padding rows and classes are zero.
template <int NB, int GROUP>
__device__ __forceinline__ void pack_b_body(const Job& j, int64_t t) {
  const int lane = (int)(t & 63);
  const int nb = (int)((t >> 6) % NB);
  const int ks = (int)(t / (64 * NB));
  const int kk = 16 * (nb % GROUP) + (lane & 15);
  const int pb = 32 * ks + 8 * (lane >> 4);
  const float* B = j.B + (int64_t)(nb / GROUP) * j.p * j.K;
  const int kmax = j.pin ? j.K - 1 : j.K;
  u16 h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float v = (pb + e < j.p && kk < kmax) ? B[(int64_t)(pb + e) * j.K + kk] : 0.0f;
    h[e] = bf16_from_f32(v);
    l[e] = bf16_from_f32(v - f32_from_bf16(h[e]));
  }
  u16* dst = j.Bpk + packed_b_index(NB, nb, pb, lane & 15);
  *reinterpret_cast<u32x4*>(dst) = u32x4{pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]), pack2(h[6], h[7])};
  *reinterpret_cast<u32x4*>(dst + 512) = u32x4{pack2(l[0], l[1]), pack2(l[2], l[3]), pack2(l[4], l[5]), pack2(l[6], l[7])};
}

// Logits, softmax and packed residuals of row block rb (kHiloRows rows); every thread
// of the workgroup takes part (barriers inside).
//
// Wave w owns kHiloMB 16-row M blocks and all 16*NB padded classes. Its X operand
// comes straight from global memory, kBChunk - 1 k steps ahead of the MFMAs: lane l
// loads the 8 consecutive columns 32 s + 8 (l / 16) .. of row l % 16 of each M block,
// the A input layout of the MFMA. The packed B operand, shared by all waves, is staged in
// LDS (`bs`, two buffers of kBChunk k steps) one chunk ahead. After the k loop, lane l
// holds logits of rows 4 (l / 16) + i (i < 4) for class 16 nb + l % 16, so every row is
// spread over one 16-lane DPP row: max and sum are DPP reductions (across the GROUP
// blocks of a softmax group in-lane). The residual R = onehot(y) - P is split into bf16
// hi/lo and stored in the B-input lane order of the gradient kernel. lacc[group] gains
// this wave's log-likelihood terms (in the lane holding each row's label).
constexpr int kBChunk = 4;                       // k steps of B per LDS buffer
template <int NB> constexpr int bchunk_elems() { return kBChunk * NB * 1024; }

// Softmax over the K valid classes of each row and group of row block rb, FP64 statistics,
// and the packed residuals. After the 16-lane reductions every lane of a row holds the sums
// of exponentials of its 4 rows x NG groups; the FP64 log is taken once per (row, group) —
// lane m of the row takes sum number m — and read back by the lanes that need it with a
// shuffle. lacc[group] gains this wave's log-likelihood terms (in the label's lane).
template <int NB, int GROUP>
__device__ __forceinline__ void softmax_residuals(const Job& j, int64_t rb,
                                                  const f32x4 (&acc)[kHiloMB][NB],
                                                  const int (&ylab)[kHiloMB][4],
                                                  double (&lacc)[NB / GROUP]) {
  constexpr int NG = NB / GROUP;
  constexpr int MB = kHiloMB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int64_t n = j.n;
  const int K = j.K;
  const int64_t r0 = rb * kHiloRows + (int64_t)w * 16 * MB;
  constexpr int F = 4 * NG;
  static_assert(F <= 16, "one log per lane per M block");
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int64_t rblk = r0 / 32 + mb / 2;     // 32-row block of the gradient kernel
    uint32_t rh[NB][2], rl[NB][2];
    float zmx[4][NG];
    double ssum[4][NG];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        float zmax = -INFINITY;
#pragma unroll
        for (int b = 0; b < GROUP; ++b)
          if (16 * b + m < K) zmax = fmaxf(zmax, acc[mb][q * GROUP + b][i]);
        zmax = max16(zmax);
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < GROUP; ++b)
          if (16 * b + m < K) s += (double)dev_exp(acc[mb][q * GROUP + b][i] - zmax);
        zmx[i][q] = zmax;
        ssum[i][q] = sum16(s);
      }
    double v = 1.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < NG; ++q) v = (i * NG + q == m) ? ssum[i][q] : v;
    const double lg = log(v);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = r0 + 16 * mb + 4 * g + i;
      const bool valid = row < n;
      const int yi = valid ? ylab[mb][i] : -1;
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        const double lse = (double)zmx[i][q] + __shfl(lg, (lane & 48) | (i * NG + q), 64);
#pragma unroll
        for (int b = 0; b < GROUP; ++b) {
          const int kk = 16 * b + m, nb = q * GROUP + b;
          float r = 0.0f;
          if (valid && kk < K) {
            const double zl = (double)acc[mb][nb][i] - lse;     // log softmax
            if (kk == yi) lacc[q] += zl;                        // the label's lane only
            r = (kk == yi ? 1.0f : 0.0f) - dev_exp((float)zl);
          }
          const u16 h = bf16_from_f32(r);
          const u16 l = bf16_from_f32(r - f32_from_bf16(h));
          if (i & 1) {
            rh[nb][i >> 1] |= (uint32_t)h << 16;
            rl[nb][i >> 1] |= (uint32_t)l << 16;
          } else {
            rh[nb][i >> 1] = h;
            rl[nb][i >> 1] = l;
          }
        }
      }
    }
    // rows 16 (mb % 2) + 4 g + i of this 32-row block sit in lane 16 (2 (mb % 2) + g / 2)
    // + m, elements 4 (g % 2) + i, of the gradient kernel's fragments
    const int L = 16 * (2 * (mb & 1) + (g >> 1)) + m;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      u16* f = j.Rpk + (rblk * NB + nb) * 2 * 512 + L * 8 + 4 * (g & 1);
      *reinterpret_cast<uint2*>(f) = uint2{rh[nb][0], rh[nb][1]};
      *reinterpret_cast<uint2*>(f + 512) = uint2{rl[nb][0], rl[nb][1]};
    }
  }
}

template <int NB, int GROUP, bool LO>
__device__ __forceinline__ void logits_rows(const Job& j, int64_t rb, double (&lacc)[NB / GROUP],
                                            u16* __restrict__ bs) {
  constexpr int CH = bchunk_elems<NB>();         // u16 per chunk (hi and lo fragments)
  constexpr int PER = CH / 8 / (kHiloWaves * 64);   // 16-byte pieces per thread per chunk
  static_assert(CH / 8 % (kHiloWaves * 64) == 0, "a B chunk is a whole number of 16-byte pieces per thread");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int64_t n = j.n;
  const int p = j.p;
  const int nks = (p + 31) / 32;
  constexpr int MB = kHiloMB;
  f32x4 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // X fragments come from branch-free buffer loads whose resource starts at the row
  // block and ends at row n, so rows past n read as zero; columns past p are zeroed in
  // registers on the last (ragged) k step. Offsets fit 32 bits (ldx < 2^23).
  const int64_t rbase = rb * kHiloRows;
  const uint64_t rem = (uint64_t)(n - rbase) * j.ldx * 2;
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(j.Xhi + rbase * j.ldx, rem);
  const __amdgpu_buffer_rsrc_t rl = make_rsrc(LO ? j.Xlo + rbase * j.ldx : j.Xhi, LO ? rem : 0);
  uint32_t xoff[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
    xoff[mb] = (uint32_t)(((int64_t)(w * 16 * MB + 16 * mb + m) * j.ldx + 8 * g) * 2);
  // labels of this lane's rows, loaded now so their latency hides behind the k loop
  // (rows past n read as zero and are not used)
  const __amdgpu_buffer_rsrc_t yres = make_rsrc(j.y + rbase, (uint64_t)(n - rbase) * 4);
  int ylab[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      ylab[mb][i] = __builtin_amdgcn_raw_buffer_load_b32(
          yres, (int)((w * 16 * MB + 16 * mb + 4 * g + i) * 4), 0, 0);
  const int nch = (nks + kBChunk - 1) / kBChunk;
  const int64_t bp_total = (int64_t)nks * NB * 1024;
  u32x4 bst[PER];
  // every load below is issued unconditionally: buffer loads past a resource's end read
  // zero, and straight-line issue keeps the compiler's load counting exact (a load under a
  // branch makes it wait for everything at the join)
  const __amdgpu_buffer_rsrc_t bres = make_rsrc(j.Bpk, (uint64_t)bp_total * 2);
  auto fetch_b = [&](int c) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int64_t idx = (int64_t)c * CH + (int64_t)(i * kHiloWaves * 64 + threadIdx.x) * 8;
      bst[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(bres, (int)(idx * 2), 0, 0));
    }
  };
  auto stash_b = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i)
      *reinterpret_cast<u32x4*>(bs + buf * CH + (i * kHiloWaves * 64 + threadIdx.x) * 8) = bst[i];
  };

  // A fragments of k step ks. A step at or past nks (the ring's refills during the last
  // chunk) would read the next rows' bytes, real traffic that is thrown away: those loads
  // take an empty resource instead (still issued, so the issue stays branch-free).
  const __amdgpu_buffer_rsrc_t rz = make_rsrc(j.Xhi, 0);
  auto load_a = [&](int ks, u32x4 (&ah)[MB], u32x4 (&al)[MB]) {
    const bool live = ks < nks;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      ah[mb] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(live ? rh : rz, (int)(xoff[mb] + 64 * ks), 0, 0));
      if (LO) al[mb] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(live ? rl : rz, (int)(xoff[mb] + 64 * ks), 0, 0));
    }
  };
  // zero the elements of this lane's 8 columns 32 ks + 8 g .. that lie past p
  auto mask_tail = [&](int ks, u32x4 (&ah)[MB], u32x4 (&al)[MB]) {
    const int lim = p - (32 * ks + 8 * g);
    u32x4 mk;
#pragma unroll
    for (int d = 0; d < 4; ++d)
      mk[d] = (2 * d < lim ? 0x0000FFFFu : 0u) | (2 * d + 1 < lim ? 0xFFFF0000u : 0u);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      ah[mb] &= mk;
      if (LO) al[mb] &= mk;
    }
  };
  // X fragments kBChunk k steps ahead in a ring of kBChunk register sets: set kk holds
  // step ks = c kBChunk + kk of chunk c and is reloaded with step ks + kBChunk right after
  // its MFMAs, so kBChunk - 1 steps of loads stay in flight per wave while one is used.
  // The ring index is static in the unrolled chunk, so no register is copied (a copy of a
  // register a load has not yet filled would wait for that load).
  u32x4 xh[kBChunk][MB], xl[kBChunk][MB];
  fetch_b(0);
  stash_b(0);
#pragma unroll
  for (int kk = 0; kk < kBChunk; ++kk) load_a(kk, xh[kk], xl[kk]);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    fetch_b(c + 1);
    const u16* bc = bs + (c & 1) * CH + lane * 8;
#pragma unroll
    for (int kk = 0; kk < kBChunk; ++kk) {
      const int ks = c * kBChunk + kk;
      if (ks == nks - 1 && (p & 31)) mask_tail(ks, xh[kk], xl[kk]);
      bf16x8 bh[NB], bl[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const u16* f = bc + (kk * NB + nb) * 1024;
        bh[nb] = as_frag(*reinterpret_cast<const u32x4*>(f));
        bl[nb] = as_frag(*reinterpret_cast<const u32x4*>(f + 512));
      }
      if (ks < nks) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            acc[mb][nb] = mma(as_frag(xh[kk][mb]), bh[nb], acc[mb][nb]);
            acc[mb][nb] = mma(as_frag(xh[kk][mb]), bl[nb], acc[mb][nb]);
            if (LO) acc[mb][nb] = mma(as_frag(xl[kk][mb]), bh[nb], acc[mb][nb]);
          }
      }
      load_a(ks + kBChunk, xh[kk], xl[kk]);
    }
    stash_b((c + 1) & 1);
    __syncthreads();
  }

  softmax_residuals<NB, GROUP>(j, rb, acc, ylab, lacc);
}

// Gradient partial X^T R of the 128 columns from c0 over rows [rbeg, rend) (rbeg a
// multiple of 32), written to gp: element (column j, class kk of group q) at
// gp[q cstride + j K + kk].
//
// Stages of 32 rows (both X planes, 32 x 128 bf16 each, and the matching packed residual
// fragments) are loaded into registers two stages ahead of the math and stored to one of
// two LDS buffers one stage ahead, so two stages of loads stay in flight per workgroup.
// Wave w owns columns 32 w .. 32 w + 31 (two 16-column M blocks); the MFMA A input wants,
// per lane, 8 consecutive ROWS of one column, gathered from LDS with 16-bit reads. The
// 16-byte chunks of a staged row are XOR-swizzled by 2 ((row / 8) % 4) so that the four
// 8-row groups read at once fall in different banks. Rows outside the slice and columns
// past p load as zero.
template <int NB, bool LO> constexpr int grad_stage_elems() { return (LO ? 2 : 1) * 4096 + NB * 1024; }
template <int NB> struct RPiece;                    // residual u16 per thread and stage
template <> struct RPiece<1> { typedef uint2 type; static constexpr int N = 4; };
template <> struct RPiece<2> { typedef u32x4 type; static constexpr int N = 8; };
template <> struct RPiece<4> { typedef u32x4 type; static constexpr int N = 8; };

template <int NB, int GROUP, bool LO>
__device__ __forceinline__ void grad_cols(const Job& j, int64_t c0, int64_t rbeg, int64_t rend,
                                          float* __restrict__ gp, int64_t cstride,
                                          u16* __restrict__ xs) {
  constexpr int PL = LO ? 2 : 1;
  constexpr int XST = PL * 4096;                  // u16 of X per stage
  constexpr int ST = grad_stage_elems<NB, LO>();
  constexpr int RN = RPiece<NB>::N;               // residual u16 per thread per piece
  constexpr int RP = NB * 1024 / (256 * RN);      // residual pieces per thread per stage
  typedef typename RPiece<NB>::type rtype;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int p = j.p, K = j.K;
  const int64_t nst = rend > rbeg ? (rend - rbeg + 31) / 32 : 0;

  // staging: thread t moves 16-byte chunk sc of rows sr and sr + 16 of each plane, and
  // residual pieces t, t + 256, ...
  const int sr = threadIdx.x >> 4, sc = threadIdx.x & 15;
  const int64_t col = c0 + 8 * sc;
  struct Regs { u32x4 x[2][PL]; rtype r[RP]; };
  // Branch-free buffer loads: the X resource of a stage starts at its first row and ends
  // at the slice's last row (rows outside the slice read as zero; columns past p only feed
  // gradient columns that are not written); the residual resource covers the packed
  // buffer, so stages past the end read zero.
  const uint64_t rpk_bytes = (uint64_t)((j.n + kHiloRows - 1) / kHiloRows) * (kHiloRows / 32) * NB * 2048;
  const __amdgpu_buffer_rsrc_t rres = make_rsrc(j.Rpk, rpk_bytes);
  // a chunk at or past column p (the last column block of a problem whose p is not a
  // multiple of 128) would fetch the row's padding or the next row's bytes for columns that
  // are never written: its offset is put out of the resource's range, so it reads zero and
  // moves nothing
  uint32_t xo[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    xo[h] = col < p ? (uint32_t)(((int64_t)(sr + 16 * h) * j.ldx + col) * 2) : 0xFFFFFFF0u;
  auto fetch = [&](int64_t k, Regs& R) {
    const int64_t row0 = rbeg + 32 * k;
    const bool real = k < nst;
    const uint64_t xbytes = real ? (uint64_t)(rend - row0) * j.ldx * 2 : 0;
    const int64_t xbase = real ? row0 * j.ldx : 0;
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) {
      const __amdgpu_buffer_rsrc_t xr = make_rsrc((pl ? j.Xlo : j.Xhi) + xbase, xbytes);
      // X is read once here and its lines are used whole by this load: the non-temporal hint
      // (aux bit 1) lets the L2 evict them first, so the packed residual rows that the slice's
      // other column blocks re-read stay cached (measured: n=200000, p=4096 gradient pass
      // 1360 -> 1320 us; batched update 3535 -> 3465 us)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        R.x[h][pl] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, (int)xo[h], 0, 2));
    }
    const uint32_t roff = (uint32_t)((real ? row0 / 32 : (int64_t)(rpk_bytes / (NB * 2048))) * NB * 2048);
#pragma unroll
    for (int i = 0; i < RP; ++i) {
      const int off = (int)(roff + (i * 256 + threadIdx.x) * RN * 2);
      if constexpr (RN == 8)
        R.r[i] = __builtin_bit_cast(rtype, __builtin_amdgcn_raw_buffer_load_b128(rres, off, 0, 0));
      else
        R.r[i] = __builtin_bit_cast(rtype, __builtin_amdgcn_raw_buffer_load_b64(rres, off, 0, 0));
    }
  };
  auto stash = [&](const Regs& R, u16* buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = sr + 16 * h;
      const int pos = sc ^ (2 * ((q >> 3) & 3));
#pragma unroll
      for (int pl = 0; pl < PL; ++pl)
        *reinterpret_cast<u32x4*>(buf + pl * 4096 + q * 128 + 8 * pos) = R.x[h][pl];
    }
#pragma unroll
    for (int i = 0; i < RP; ++i)
      *reinterpret_cast<rtype*>(buf + XST + (i * 256 + threadIdx.x) * RN) = R.r[i];
  };

  f32x4 acc[2][NB];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](const u16* cur) {
    bf16x8 bh[NB], bl[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      bh[nb] = as_frag(*reinterpret_cast<const u32x4*>(cur + XST + nb * 1024 + lane * 8));
      bl[nb] = as_frag(*reinterpret_cast<const u32x4*>(cur + XST + nb * 1024 + 512 + lane * 8));
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const int cl = 32 * w + 16 * mb + m;
      const int off = ((cl >> 3) ^ (2 * g)) * 8 + (cl & 7);
      bf16x8 af[PL];
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) {
        const u16* t = cur + pl * 4096;
        u16 v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = t[(8 * g + e) * 128 + off];
        af[pl] = as_frag(u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])});
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        acc[mb][nb] = mma(af[0], bh[nb], acc[mb][nb]);
        acc[mb][nb] = mma(af[0], bl[nb], acc[mb][nb]);
        if (LO) acc[mb][nb] = mma(af[PL - 1], bh[nb], acc[mb][nb]);
      }
    }
  };

  // register sets: stage k in ra (k even) or rb (k odd), loaded two steps before its use
  Regs ra, rb;
  fetch(0, ra);
  fetch(1, rb);
  for (int64_t k = 0; k < nst; k += 2) {
    stash(ra, xs);
    __syncthreads();
    fetch(k + 2, ra);
    compute(xs);
    if (k + 1 >= nst) break;
    stash(rb, xs + ST);
    __syncthreads();
    fetch(k + 3, rb);
    compute(xs + ST);
  }
  __syncthreads();   // the buffers are reused by the caller's next item

  // lane l holds G[column 4 (l / 16) + i of the M block][class 16 nb + l % 16]
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t jc = c0 + 32 * w + 16 * mb + 4 * g + i;
      if (jc >= p) continue;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int kk = 16 * (nb % GROUP) + m;
        if (kk < K) gp[(nb / GROUP) * cstride + jc * K + kk] = acc[mb][nb][i];
      }
    }
}

// XCD-aware item order of the gradient kernels. Workgroup w of a launch runs on XCD w % 8,
// and consecutive items (the column blocks of one row slice) read the same packed residual
// rows, so they should share an XCD's L2: position `it` of the launch order is mapped to
// item (it % 8 + 8 (it / 8 / G)) G + (it / 8) % G, which gives XCD x the chunks x, x + 8, ...
// of G consecutive items. It is a bijection of [0, round_up(total, 8 G)); positions whose
// item is >= total do nothing.
__device__ __forceinline__ int64_t xcd_item(int64_t it, int G) {
  const int64_t x = it % kXcds, l = it / kXcds;
  return (x + kXcds * (l / G)) * G + l % G;
}

__device__ __forceinline__ Job job_of(const HiloArgs& a) {
  return Job{a.Xhi, a.Xlo, a.ldx, a.y, a.n, a.p, a.K, static_cast<const float*>(a.B), a.Bpk, a.Rpk, a.pin};
}

// ---------------------------------------------------------------------------------------
// Single-problem kernels (one softmax group spanning all NB class blocks).
template <int NB>
__global__ __launch_bounds__(256) void pack_b_kernel(HiloArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)((a.p + 31) / 32) * NB * 64) return;
  pack_b_body<NB, NB>(job_of(a), t);
}

template <int NB, bool LO>
__global__ __launch_bounds__(kHiloWaves * 64) void hilo_logits(HiloArgs a) {
  constexpr int ROWS = kHiloRows;
  __shared__ double lsum[kHiloWaves];
  __shared__ __attribute__((aligned(16))) u16 bs[2 * bchunk_elems<NB>()];
  const Job j = job_of(a);
  const int64_t nrb = (a.n + ROWS - 1) / ROWS;
  double lacc[1] = {0.0};
  for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) logits_rows<NB, NB, LO>(j, rb, lacc, bs);
  const double v = wave_sum(lacc[0]);
  if ((threadIdx.x & 63) == 0) lsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kHiloWaves; ++i) t += lsum[i];
    a.lpart[blockIdx.x] = t;
  }
}

// One workgroup per (128-column block, row slice) item, items slice-major (the column
// blocks of a slice consecutive) in the XCD-aware order; the launch has xcd_span(items,
// gcols) workgroups.
template <int NB, bool LO>
__global__ __launch_bounds__(256) void hilo_grad(HiloArgs a, int gcols) {
  __shared__ __attribute__((aligned(16))) u16 xs[2 * grad_stage_elems<NB, LO>()];
  const int64_t it = xcd_item(blockIdx.x, gcols);
  if (it >= (int64_t)gcols * a.nsplit) return;
  const int64_t cb = it % gcols, sl = it / gcols;
  const int64_t rbeg = sl * a.rows_per_split;
  const int64_t rend = rbeg + a.rows_per_split < a.n ? rbeg + a.rows_per_split : a.n;
  grad_cols<NB, NB, LO>(job_of(a), cb * 128, rbeg, rend, a.gpart + sl * a.gstride, 0, xs);
}

// ---------------------------------------------------------------------------------------
// Batched kernels: every problem of a batch, NB chains each (one class block per chain),
// in one persistent launch per phase. Work items are numbered table entry by table entry
// (the host orders the entries by decreasing p); item i belongs to entry b with
// first[b] <= i < first[b + 1].
__device__ __forceinline__ int find_problem(const int32_t* first, int nprob, int64_t item) {
  int lo = 0, hi = nprob;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ Job job_of(const BatchProb& b, const float* B) {
  return Job{b.Xhi, b.Xlo, b.ldx, b.y, b.n, b.p, b.K, B, b.Bpk, b.Rpk, b.pin};
}

template <int NB, int GROUP>
__global__ __launch_bounds__(256) void batch_pack(BatchArgs a) {
  const int64_t total = a.first_pack[a.nprob];
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int b = find_problem(a.first_pack, a.nprob, t);
    const BatchProb& P = a.probs[b];
    pack_b_body<NB, GROUP>(job_of(P, a.at_current ? P.B : P.Bp), t - a.first_pack[b]);
  }
}

template <int NB, int GROUP, bool LO>
__global__ __launch_bounds__(kHiloWaves * 64, 2) void batch_logits(BatchArgs a) {
  constexpr int NC = NB / GROUP;                  // chains
  __shared__ double lsum[kHiloWaves][NC];
  __shared__ __attribute__((aligned(16))) u16 bs[2 * bchunk_elems<NB>()];
  const int64_t total = a.first_logits[a.nprob];
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    const int b = find_problem(a.first_logits, a.nprob, it);
    const BatchProb& P = a.probs[b];
    const int64_t rb = it - a.first_logits[b];
    double lacc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) lacc[c] = 0.0;
    logits_rows<NB, GROUP, LO>(job_of(P, a.at_current ? P.B : P.Bp), rb, lacc, bs);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double v = wave_sum(lacc[c]);
      if ((threadIdx.x & 63) == 0) lsum[threadIdx.x >> 6][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
      double t = 0.0;
      for (int i = 0; i < kHiloWaves; ++i) t += lsum[i][threadIdx.x];
      P.lpart[rb * NC + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

template <int NB, int GROUP, bool LO>
__global__ __launch_bounds__(256) void batch_grad(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) u16 xs[2 * grad_stage_elems<NB, LO>()];
  const int64_t total = a.first_grad[a.nprob];
  const int64_t span = xcd_span(total, kGradChunk);
  for (int64_t pos = blockIdx.x; pos < span; pos += gridDim.x) {
    const int64_t it = xcd_item(pos, kGradChunk);
    if (it >= total) continue;
    const int b = find_problem(a.first_grad, a.nprob, it);
    const BatchProb& P = a.probs[b];
    const int64_t k = it - a.first_grad[b];
    const int64_t cb = k % P.gcols, s = k / P.gcols;
    const int64_t rbeg = s * P.rps;
    const int64_t rend = rbeg + P.rps < P.n ? rbeg + P.rps : P.n;
    grad_cols<NB, GROUP, LO>(job_of(P, a.at_current ? P.B : P.Bp), cb * 128, rbeg, rend,
                         P.gpart + s * P.gstride, P.cstride, xs);
  }
}

}  // namespace

template <typename Tin>
hipError_t launch_split(const Tin* X, int64_t ldx, int64_t n, int64_t p, uint16_t* hi,
                        uint16_t* lo, int64_t ldo, hipStream_t s) {
  const int64_t total = n * (ldo / 8);
  const int64_t want = (total + 255) / 256;
  const int grid = (int)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(split_kernel<Tin>, dim3(grid), dim3(256), 0, s, X, ldx, n, p, hi, lo, ldo);
  return hipGetLastError();
}
template hipError_t launch_split<float>(const float*, int64_t, int64_t, int64_t, uint16_t*, uint16_t*, int64_t, hipStream_t);
template hipError_t launch_split<double>(const double*, int64_t, int64_t, int64_t, uint16_t*, uint16_t*, int64_t, hipStream_t);

template <int NB, int GROUP, bool LO>
static hipError_t launch_batch_t(const BatchArgs& a, const int grid[3], bool pack, hipStream_t s) {
  if (pack) hipLaunchKernelGGL((batch_pack<NB, GROUP>), dim3(grid[0]), dim3(256), 0, s, a);
  hipLaunchKernelGGL((batch_logits<NB, GROUP, LO>), dim3(grid[1]), dim3(kHiloWaves * 64), 0, s, a);
  hipLaunchKernelGGL((batch_grad<NB, GROUP, LO>), dim3(grid[2]), dim3(256), 0, s, a);
  return hipGetLastError();
}

// chains x group class blocks (group = 16-class blocks per chain), at most 4 in all
hipError_t launch_batch_pass(const BatchArgs& a, int chains, int group, bool lo, const int grid[3], bool pack, hipStream_t s) {
#define HMC_BATCH(C_, G_)                                                                 \
  if (chains == C_ && group == G_)                                                        \
    return lo ? launch_batch_t<C_ * G_, G_, true>(a, grid, pack, s)                      \
              : launch_batch_t<C_ * G_, G_, false>(a, grid, pack, s);
  HMC_BATCH(1, 1) HMC_BATCH(2, 1) HMC_BATCH(4, 1) HMC_BATCH(1, 2) HMC_BATCH(2, 2) HMC_BATCH(1, 4)
#undef HMC_BATCH
  return hipErrorInvalidValue;
}

template <int NB, bool LO>
static hipError_t launch_hilo_t(const HiloArgs& a, int logits_wg, int grad_cols, bool pack, hipStream_t s) {
  const int nks = (a.p + 31) / 32;
  const int packs = (nks * NB * 64 + 255) / 256;
  if (pack) hipLaunchKernelGGL(pack_b_kernel<NB>, dim3(packs), dim3(256), 0, s, a);
  hipLaunchKernelGGL((hilo_logits<NB, LO>), dim3(logits_wg), dim3(kHiloWaves * 64), 0, s, a);
  const int64_t span = xcd_span((int64_t)grad_cols * a.nsplit, grad_cols);
  hipLaunchKernelGGL((hilo_grad<NB, LO>), dim3((unsigned)span), dim3(256), 0, s, a, grad_cols);
  return hipGetLastError();
}

hipError_t launch_hilo(const HiloArgs& a, int nb, bool lo, int logits_wg, int grad_cols, bool pack, hipStream_t s) {
  switch (nb * 2 + (lo ? 1 : 0)) {
    case 2: return launch_hilo_t<1, false>(a, logits_wg, grad_cols, pack, s);
    case 3: return launch_hilo_t<1, true>(a, logits_wg, grad_cols, pack, s);
    case 4: return launch_hilo_t<2, false>(a, logits_wg, grad_cols, pack, s);
    case 5: return launch_hilo_t<2, true>(a, logits_wg, grad_cols, pack, s);
    case 8: return launch_hilo_t<4, false>(a, logits_wg, grad_cols, pack, s);
    case 9: return launch_hilo_t<4, true>(a, logits_wg, grad_cols, pack, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace hmcx
