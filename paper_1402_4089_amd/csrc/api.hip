// C-ABI entry points of libhmc: argument checks, workspace layout and launch sequences.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "hmc.h"
#include "internal.h"

using namespace hmcx;

namespace {

thread_local std::string g_last_error;

// Event pool for hmc_profile_begin / hmc_profile_end.
struct Profiler {
  bool on = false;
  int cap = 0, used = 0;
  int repeat = 1;             // launches per event pair when the pass is idempotent
  hipEvent_t* ev = nullptr;   // 2 * cap events
  int* reps = nullptr;        // launches between each recorded pair
} g_prof;

hmc_status fail(hmc_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
hmc_status fail(hmc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

constexpr size_t kAlign = 256;
constexpr size_t kLdsLimit = 160 * 1024;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  bool f64;
  size_t ts;            // state element bytes
  int nblk, waves, mb, nb;
  size_t lds;
  int64_t ntiles;
  int nwg, nepi, nupd;
  int64_t gstride;      // elements between per-workgroup partial gradients
  bool wide;            // p beyond the row tile: chunked logits + column-owner gradient
  int nchunk, tiles_y, nsoft, ngrad, wsplit;
  int64_t wtps;         // wide gradient: 16-row tiles per row slice
  bool hilo, lo;        // bf16 split-precision form (lo: the low plane is present)
  int hl_logits_wg, hl_cols, hl_nsplit;
  int64_t hl_rps;       // rows per gradient slice
  size_t off_bpk, off_rpk;
  int nl, np;           // log-likelihood / prior (and kinetic) partial counts
  size_t off_zpart, off_R;
  size_t off_gpart, off_lpart, off_ppart, off_k0, off_k1, off_eta, off_bp, off_gp, off_scal, off_ctr, total;
};

int class_blocks(int K) { return K <= 16 ? 1 : K <= 32 ? 2 : 4; }

// LDS of the fused pass: two 16-row tile buffers of waves*mb*16 padded columns, plus the
// cross-wave logits and residual exchanges.
size_t lds_bytes(int waves, int mb, int nb, size_t ts) {
  return (size_t)2 * kTileRows * (waves * mb * 16) * ts + (size_t)(waves + 1) * nb * 256 * ts + 64;
}

// Pick the fused-kernel variant: the smallest column-block count covering p. FP32 with one
// class block runs 16 waves (four per SIMD) over the same padded row when that row has at
// least 16 column blocks: the extra waves hide more of the per-tile synchronisation
// (measured 20.1 -> 19.7 us per pass at n=20000, p=1000, K=10).
bool pick_variant(bool f64, int nblk, int nb, int* waves, int* mb) {
  int w = 8;
  const int need = (nblk + w - 1) / w;
  int m = 1;
  while (m < need) m <<= 1;
  if (!f64 && nb == 1 && m >= 2) { w = 16; m /= 2; }
  const bool ok = f64 ? fused_variant_exists<double>(w, m, nb) : fused_variant_exists<float>(w, m, nb);
  if (!ok || lds_bytes(w, m, nb, f64 ? 8 : 4) > kLdsLimit) return false;
  *waves = w;
  *mb = m;
  return true;
}

bool is_bf16(int32_t xfmt) { return xfmt == HMC_X_BF16_HILO || xfmt == HMC_X_BF16; }

// Largest row pitch whose in-kernel byte offsets fit 32 bits: 64 rows of FP32/FP64 X (the
// wide-p gradient's row groups; the row tile uses 16) and 128 rows of a bf16 plane (the
// split-precision logits blocks) must span less than 2^32 bytes.
int64_t max_ldx(int32_t xfmt) {
  if (is_bf16(xfmt)) return ((int64_t)1 << 23) - 8;
  return (((int64_t)1 << 26) / (xfmt == HMC_X_F64 ? 8 : 4)) - 1;
}

hmc_status check_problem(const hmc_problem* pr) {
  if (!pr) return fail(HMC_ERR_ARG, "problem descriptor is NULL");
  if (pr->xfmt != HMC_X_F64 && pr->xfmt != HMC_X_F32 && !is_bf16(pr->xfmt))
    return fail(HMC_ERR_DTYPE, "unsupported X format %d", pr->xfmt);
  if (pr->prior != HMC_PRIOR_GAUSS && pr->prior != HMC_PRIOR_CAUCHY)
    return fail(HMC_ERR_DTYPE, "unknown prior %d", pr->prior);
  if (pr->n < 1) return fail(HMC_ERR_SHAPE, "n = %lld must be >= 1", (long long)pr->n);
  if (pr->p < 1) return fail(HMC_ERR_SHAPE, "p = %lld must be >= 1", (long long)pr->p);
  if (pr->link != HMC_LINK_SOFTMAX && pr->link != HMC_LINK_POISSON && pr->link != HMC_LINK_PROBIT)
    return fail(HMC_ERR_DTYPE, "unknown link %d", pr->link);
  if (pr->link != HMC_LINK_SOFTMAX) {
    const char* name = pr->link == HMC_LINK_POISSON ? "Poisson" : "probit";
    if (pr->K != 1) return fail(HMC_ERR_SHAPE, "K = %d must be 1 for the %s link", pr->K, name);
    if (pr->pin_last_class != 0)
      return fail(HMC_ERR_ARG, "pin_last_class must be 0 for the %s link", name);
    if (is_bf16(pr->xfmt))
      return fail(HMC_ERR_UNSUPPORTED, "the %s link runs on FP64 or FP32 X only", name);
  } else if (pr->K < 2 || pr->K > 64) {
    return fail(HMC_ERR_SHAPE, "K = %d must be in [2, 64]", pr->K);
  }
  if (pr->ldx < pr->p)
    return fail(HMC_ERR_SHAPE, "ldx = %lld < p = %lld", (long long)pr->ldx, (long long)pr->p);
  if (pr->n > ((int64_t)1 << 40)) return fail(HMC_ERR_SHAPE, "n too large");
  if (!pr->X || !pr->y) return fail(HMC_ERR_ARG, "X and y must be device pointers");
  if (pr->xfmt == HMC_X_BF16_HILO) {
    if (!pr->X_lo) return fail(HMC_ERR_ARG, "X_lo must be a device pointer for HMC_X_BF16_HILO");
  } else if (pr->X_lo) {
    return fail(HMC_ERR_ARG, "X_lo must be NULL for this X format");
  }
  if (is_bf16(pr->xfmt)) {
    if (pr->ldx % 8) return fail(HMC_ERR_SHAPE, "ldx = %lld must be a multiple of 8 for bf16 X", (long long)pr->ldx);
    if ((uintptr_t)pr->X % 16 || (uintptr_t)pr->X_lo % 16)
      return fail(HMC_ERR_ARG, "bf16 X planes must be 16-byte aligned");
  }
  // The kernels address X through 32-bit buffer offsets from a row group's first row: up to
  // 128 rows (bf16 logits blocks) or 64 rows (FP32/FP64 wide-p gradient groups) of pitch ldx.
  if (pr->ldx > max_ldx(pr->xfmt))
    return fail(HMC_ERR_UNSUPPORTED, "ldx = %lld exceeds %lld, the row pitch 32-bit offsets reach for this format",
                (long long)pr->ldx, (long long)max_ldx(pr->xfmt));
  if (!(pr->prior_scale > 0.0) || !isfinite(pr->prior_scale))
    return fail(HMC_ERR_ARG, "prior_scale must be finite and > 0");
  if (pr->pin_last_class != 0 && pr->pin_last_class != 1)
    return fail(HMC_ERR_ARG, "pin_last_class must be 0 or 1");
  const int64_t maxp = hmc_max_p(pr->xfmt, pr->K);
  if (pr->p > maxp)
    return fail(HMC_ERR_UNSUPPORTED, "p = %lld exceeds %lld for this format and K = %d",
                (long long)pr->p, (long long)maxp, pr->K);
  return HMC_OK;
}

hmc_status make_layout(const hmc_problem* pr, Layout* L) {
  hmc_status st = check_problem(pr);
  if (st != HMC_OK) return st;
  L->f64 = pr->xfmt == HMC_X_F64;
  L->ts = L->f64 ? 8 : 4;
  L->nblk = (int)((pr->p + 15) / 16);
  L->nb = class_blocks(pr->K);
  L->hilo = is_bf16(pr->xfmt);
  L->lo = pr->xfmt == HMC_X_BF16_HILO;
  const hmc_tuning& tu = pr->tuning;
  if (tu.path < 0 || tu.path > 3) return fail(HMC_ERR_ARG, "tuning.path = %d must be 0..3", tu.path);
  if (tu.path == 0 && (tu.waves || tu.mb || tu.grid || tu.rows_per_slice))
    return fail(HMC_ERR_ARG, "tuning fields must be 0 with path 0 (the built-in rule)");
  if (tu.waves < 0 || tu.mb < 0 || tu.grid < 0 || tu.rows_per_slice < 0)
    return fail(HMC_ERR_ARG, "tuning fields must be >= 0");
  if (L->hilo != (tu.path == 3) && tu.path != 0)
    return fail(HMC_ERR_ARG, "tuning.path %d does not fit X format %d (path 3 is the bf16 formats' only path)",
                tu.path, pr->xfmt);
  if (tu.path == 1 || tu.path == 0) {
    const bool ruled = tu.waves == 0 && tu.mb == 0;
    bool ok;
    if (ruled) {
      ok = !L->hilo && pick_variant(L->f64, L->nblk, L->nb, &L->waves, &L->mb);
    } else {
      L->waves = tu.waves; L->mb = tu.mb;
      ok = (L->f64 ? fused_variant_exists<double>(tu.waves, tu.mb, L->nb)
                   : fused_variant_exists<float>(tu.waves, tu.mb, L->nb)) &&
           tu.waves * tu.mb >= L->nblk && lds_bytes(tu.waves, tu.mb, L->nb, L->ts) <= kLdsLimit;
      if (!ok) return fail(HMC_ERR_ARG, "row-tile variant (%d waves, %d blocks) does not exist or cover p = %lld",
                           tu.waves, tu.mb, (long long)pr->p);
    }
    if (tu.path == 1 && !ok)
      return fail(HMC_ERR_UNSUPPORTED, "p = %lld is beyond every row-tile variant at K = %d", (long long)pr->p, pr->K);
    L->wide = !L->hilo && !ok;
  } else {
    L->wide = tu.path == 2;
  }
  if (!L->wide && !L->hilo) L->lds = lds_bytes(L->waves, L->mb, L->nb, L->ts);
  L->ntiles = (pr->n + kTileRows - 1) / kTileRows;
  if (tu.grid && (tu.path == 1 || tu.path == 0)) {
    if (tu.grid > 4096) return fail(HMC_ERR_ARG, "tuning.grid = %d must be <= 4096 on the row tile", tu.grid);
    L->nwg = tu.grid;
  } else {
    // as few workgroups as keep the most tiles per workgroup at its minimum: fewer
    // partial gradients for the epilogue, same critical path (1250 tiles: 250 x 5)
    const int64_t per = (L->ntiles + kMaxFusedWG - 1) / kMaxFusedWG;
    L->nwg = (int)((L->ntiles + per - 1) / per);
  }
  if ((int64_t)L->nwg > L->ntiles) L->nwg = (int)L->ntiles;
  const int64_t pk = pr->p * (int64_t)pr->K;
  L->nepi = (int)((pk + kEpiElems - 1) / kEpiElems);
  L->nupd = (int)((pk + kUpdThreads - 1) / kUpdThreads);
  const int KP = 16 * L->nb;
  L->hl_logits_wg = L->hl_cols = L->hl_nsplit = 0;
  L->hl_rps = 0;
  if (L->hilo) {
    // logits: row blocks of kHiloRows rows; gradient: 128-column blocks times row
    // slices, about 2048 workgroups in all
    const int64_t rows = kHiloRows;
    const int64_t nrb = (pr->n + rows - 1) / rows;
    if (tu.grid > 65536) return fail(HMC_ERR_ARG, "tuning.grid = %d must be <= 65536", tu.grid);
    const int64_t lwg = tu.grid ? tu.grid : 2048;
    L->hl_logits_wg = (int)(nrb < lwg ? nrb : lwg);
    L->hl_cols = (int)((pr->p + 127) / 128);
    if (tu.rows_per_slice) {
      if (tu.rows_per_slice % 32) return fail(HMC_ERR_ARG, "tuning.rows_per_slice = %d must be a multiple of 32", tu.rows_per_slice);
      L->hl_rps = std::min<int64_t>(tu.rows_per_slice, (pr->n + 31) / 32 * 32);
    } else {
      int64_t want = (2048 + L->hl_cols - 1) / L->hl_cols;
      const int64_t n32 = (pr->n + 31) / 32;
      want = want < 1 ? 1 : want > 256 ? 256 : want;
      if (want > n32) want = n32;
      L->hl_rps = ((pr->n + want - 1) / want + 31) / 32 * 32;
    }
    L->hl_nsplit = (int)((pr->n + L->hl_rps - 1) / L->hl_rps);
    L->nchunk = L->tiles_y = L->nsoft = L->ngrad = 0;
    L->wsplit = 1; L->wtps = 0;
    L->nwg = L->hl_nsplit;
    L->nl = L->hl_logits_wg;
    L->np = L->nepi;
    L->gstride = (pk + 63) / 64 * 64;
  } else if (L->wide) {
    const int cw = L->f64 ? wide_chunk_cols<double>() : wide_chunk_cols<float>();
    L->nchunk = (int)((pr->p + cw - 1) / cw);
    // enough logits workgroups to fill the chip, at least 16 tile rows per chunk
    int64_t ty = (1024 + L->nchunk - 1) / L->nchunk;
    ty = ty < 16 ? 16 : ty;
    if (tu.grid) {
      if (tu.grid > 65535) return fail(HMC_ERR_ARG, "tuning.grid = %d must be <= 65535 on the wide-p path", tu.grid);
      ty = tu.grid;
    }
    L->tiles_y = (int)(L->ntiles < ty ? L->ntiles : ty);
    L->nsoft = (int)((pr->n + 3) / 4);               // softmax workgroups of 4 rows
    L->ngrad = wide_grad_groups(pr->p, L->nb, L->f64);
    // few column blocks: split the rows too (partials reduced by the shared epilogue)
    L->wsplit = 1;
    L->wtps = 0;
    if (tu.rows_per_slice) {
      if (tu.rows_per_slice % 64) return fail(HMC_ERR_ARG, "tuning.rows_per_slice = %d must be a multiple of 64 on the wide-p path", tu.rows_per_slice);
      const int64_t tps = tu.rows_per_slice / kTileRows;
      if (tps < L->ntiles) {
        L->wtps = tps;
        L->wsplit = (int)((L->ntiles + tps - 1) / tps);
      }
    } else if (L->ngrad < 512) {
      const int64_t groups = (L->ntiles + 3) / 4;                  // 4-tile groups (load pairs)
      int64_t want = (512 + L->ngrad - 1) / L->ngrad;
      want = want > groups ? groups : want;
      if (want > 1) {
        L->wtps = (groups + want - 1) / want * 4;
        L->wsplit = (int)((L->ntiles + L->wtps - 1) / L->wtps);
      }
    }
    L->nl = L->nsoft;
    L->np = L->wsplit > 1 ? L->nepi : L->ngrad;
    L->gstride = L->wsplit > 1 ? (pk + 63) / 64 * 64 : 0;
    L->nwg = L->wsplit > 1 ? L->wsplit : 0;
  } else {
    L->nchunk = L->tiles_y = L->nsoft = L->ngrad = 0;
    L->wsplit = 1; L->wtps = 0;
    L->nl = L->nwg;
    L->np = L->nepi;
    L->gstride = (pk + 63) / 64 * 64;
  }
  // 32-bit offsets into per-row buffers: the wide-p residuals [n][16 NB] (state type) and the
  // packed split-precision residuals (64 NB bytes per row)
  if (L->wide && (uint64_t)pr->n * KP * L->ts > 0xFFFFFFFFull)
    return fail(HMC_ERR_UNSUPPORTED, "n = %lld rows exceed the wide-p residual buffer's 32-bit offsets (%lld rows at K = %d)",
                (long long)pr->n, (long long)(0xFFFFFFFFll / (KP * (int64_t)L->ts)), pr->K);
  if (L->hilo && (uint64_t)(pr->n + kHiloRows) * 64 * L->nb > 0xFFFFFFFFull)
    return fail(HMC_ERR_UNSUPPORTED, "n = %lld rows exceed the packed residual's 32-bit offsets (%lld rows at K = %d)",
                (long long)pr->n, (long long)(0xFFFFFFFFll / (64 * L->nb) - kHiloRows), pr->K);
  size_t off = 0;
  L->off_gpart = off; off = align_up(off + (size_t)L->nwg * L->gstride * L->ts);
  L->off_zpart = off; off = align_up(off + (L->wide ? (size_t)L->nchunk * pr->n * KP * L->ts : 0));
  L->off_R = off;     off = align_up(off + (L->wide ? (size_t)pr->n * KP * L->ts : 0));
  {
    const size_t frag = 2 * 512 * sizeof(uint16_t);   // one hi/lo pair of 64-lane fragments
    const int64_t rows = kHiloRows;
    L->off_bpk = off; off = align_up(off + (L->hilo ? (size_t)((pr->p + 31) / 32) * L->nb * frag : 0));
    L->off_rpk = off;
    off = align_up(off + (L->hilo ? (size_t)((pr->n + rows - 1) / rows) * (rows / 32) * L->nb * frag : 0));
  }
  L->off_lpart = off; off = align_up(off + (size_t)L->nl * 8);
  L->off_ppart = off; off = align_up(off + (size_t)L->np * 8);
  L->off_k0 = off;    off = align_up(off + (size_t)L->nupd * 8);
  L->off_k1 = off;    off = align_up(off + (size_t)L->np * 8);
  L->off_eta = off;   off = align_up(off + (size_t)pk * L->ts);
  L->off_bp = off;    off = align_up(off + (size_t)pk * L->ts);
  L->off_gp = off;    off = align_up(off + (size_t)pk * L->ts);
  L->off_scal = off;  off = align_up(off + 8 * sizeof(double));
  L->off_ctr = off;   off = align_up(off + 2 * sizeof(int64_t));
  L->total = off;
  return HMC_OK;
}

hmc_status check_ws(const Layout& L, void* ws, size_t bytes) {
  if (!ws) return fail(HMC_ERR_WORKSPACE, "workspace pointer is NULL");
  if ((uintptr_t)ws % kAlign) return fail(HMC_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (bytes < L.total)
    return fail(HMC_ERR_WORKSPACE, "workspace of %zu bytes < required %zu", bytes, L.total);
  return HMC_OK;
}

// Candidate decompositions the autotuner times for a problem (see hmc_autotune).
std::vector<hmc_tuning> tuning_candidates(const hmc_problem* pr) {
  std::vector<hmc_tuning> out;
  hmc_problem q = *pr;
  q.tuning = hmc_tuning{};
  Layout rule;
  if (make_layout(&q, &rule) != HMC_OK) return out;
  const int64_t ntiles = rule.ntiles;
  if (rule.hilo) {
    const int64_t nrb = (pr->n + kHiloRows - 1) / kHiloRows;
    const int64_t rps = rule.hl_rps;
    for (int g : {1024, 2048, 4096}) {
      if (g > nrb && g != 1024) continue;
      for (int64_t r : {rps, rps / 2 / 32 * 32, rps * 2}) {
        if (r < 32 || r > ((int64_t)1 << 30)) continue;
        out.push_back(hmc_tuning{3, 0, 0, g, (int32_t)r});
      }
    }
    return out;
  }
  // row-tile variants that cover p, fewest padded columns first, at most three
  static const int kW[] = {16, 8}, kM[] = {1, 2, 4, 8};
  std::vector<std::pair<int, int>> vars;
  for (int m : kM)
    for (int w : kW) {
      const bool ok = (rule.f64 ? fused_variant_exists<double>(w, m, rule.nb) : fused_variant_exists<float>(w, m, rule.nb)) &&
                      w * m >= rule.nblk && lds_bytes(w, m, rule.nb, rule.ts) <= kLdsLimit;
      if (ok && vars.size() < 3) vars.push_back({w, m});
    }
  for (auto& v : vars) {
    const int64_t per = (ntiles + kMaxFusedWG - 1) / kMaxFusedWG;
    const int rule_g = (int)((ntiles + per - 1) / per);
    std::vector<int> grids = {rule_g};
    if (ntiles >= 256 && rule_g != 256) grids.push_back(256);
    if (rule_g / 2 >= 1) grids.push_back(rule_g / 2);
    for (int g : grids) out.push_back(hmc_tuning{1, v.first, v.second, g, 0});
  }
  // the wide-p path. Logits grid: the rule, twice and half of it, and the row-tile counts
  // that make the chunks x tiles grid just fill k rounds of 256 compute units; gradient row
  // slices: the rule's, one slice, twice the rule's, and 2..8 equal slices (the column-owner
  // grid times the slices is then close to a multiple of 256 for some count)
  if (pr->p > 256 || vars.empty()) {
    hmc_problem w = *pr;
    w.tuning = hmc_tuning{2, 0, 0, 0, 0};
    Layout wl;
    if (make_layout(&w, &wl) == HMC_OK) {
      const int ty = wl.tiles_y;
      const int64_t one = (pr->n + 63) / 64 * 64;
      const int64_t rs = wl.wsplit > 1 ? wl.wtps * kTileRows : one;
      std::vector<int> gs = {ty, 2 * ty, std::max(16, ty / 2)};
      for (int k = 1; k <= 8; ++k) {
        const int64_t g = (int64_t)k * 256 / wl.nchunk;
        if (g >= 1 && g <= ntiles) gs.push_back((int)g);
      }
      std::vector<int64_t> rss = {rs, one, 2 * rs};
      for (int sl = 2; sl <= 8; ++sl) {
        const int64_t r = ((pr->n + sl - 1) / sl + 63) / 64 * 64;
        if (r < one) rss.push_back(r);
      }
      std::sort(gs.begin(), gs.end());
      gs.erase(std::unique(gs.begin(), gs.end()), gs.end());
      std::sort(rss.begin(), rss.end());
      rss.erase(std::unique(rss.begin(), rss.end()), rss.end());
      for (int g : gs) {
        if (g > 65535) continue;
        for (int64_t r : rss) {
          if (r > ((int64_t)1 << 30)) continue;
          out.push_back(hmc_tuning{2, 0, 0, g, (int32_t)std::min<int64_t>(r, one)});
        }
      }
    }
  }
  return out;
}

template <typename P> P* at(void* ws, size_t off) {
  return reinterpret_cast<P*>(static_cast<char*>(ws) + off);
}

hmc_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return HMC_OK;
  return fail(HMC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HMC_TRY(expr)                     \
  do {                                    \
    hmc_status st_ = (expr);              \
    if (st_ != HMC_OK) return st_;        \
  } while (0)

// Runs `launch` (one gradient pass). While profiling, the pass is bracketed by a pair of
// events on its stream; an idempotent pass (one that only overwrites workspace) runs
// g_prof.repeat times back to back between the pair, which spreads the cost of recording
// the events over several launches.
template <typename F>
hmc_status timed_launch(hipStream_t s, bool idempotent, F&& launch) {
  if (!(g_prof.on && g_prof.used < g_prof.cap)) return launch();
  const int reps = idempotent ? g_prof.repeat : 1;
  HMC_TRY(hip_status(hipEventRecord(g_prof.ev[2 * g_prof.used], s), "profile event"));
  for (int r = 0; r < reps; ++r) HMC_TRY(launch());
  HMC_TRY(hip_status(hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s), "profile event"));
  g_prof.reps[g_prof.used] = reps;
  ++g_prof.used;
  return HMC_OK;
}

// One gradient evaluation at Bpos: fused pass, then the epilogue in `mode`.
// pack: the split-precision pass first packs Bpos into its B operand; a pass that follows a
// mode-1 epilogue of the same form finds it packed already (that epilogue wrote it).
template <typename T>
hmc_status gradient_step(const hmc_problem* pr, const Layout& L, const void* Bpos, void* G,
                         void* eta, int mode, double eps, void* ws, hipStream_t s, bool pack = true) {
  if (L.hilo) {
    HiloArgs h{};
    h.Xhi = static_cast<const uint16_t*>(pr->X);
    h.Xlo = static_cast<const uint16_t*>(pr->X_lo);
    h.ldx = pr->ldx; h.y = pr->y; h.B = Bpos;
    h.Bpk = at<uint16_t>(ws, L.off_bpk); h.Rpk = at<uint16_t>(ws, L.off_rpk);
    h.gpart = at<float>(ws, L.off_gpart); h.gstride = L.gstride;
    h.nsplit = L.hl_nsplit; h.rows_per_split = L.hl_rps;
    h.lpart = at<double>(ws, L.off_lpart);
    h.n = pr->n; h.p = (int32_t)pr->p; h.K = pr->K; h.pin = pr->pin_last_class;
    HMC_TRY(timed_launch(s, true, [&] {
      return hip_status(launch_hilo(h, L.nb, L.lo, L.hl_logits_wg, L.hl_cols, pack, s), "split-precision pass");
    }));
    EpiArgs e{};
    e.gpart = h.gpart; e.gstride = L.gstride; e.nwg = L.hl_nsplit; e.p = (int32_t)pr->p; e.K = pr->K;
    e.B = const_cast<void*>(Bpos); e.G = G; e.eta = eta;
    e.prior = pr->prior; e.scale = pr->prior_scale; e.pin = pr->pin_last_class;
    e.h = 0.5 * eps; e.eps = eps; e.mode = mode;
    e.ppart = at<double>(ws, L.off_ppart);
    e.kpart = at<double>(ws, L.off_k1);
    e.bpk = mode == 1 ? h.Bpk : nullptr;
    e.pack_nb = L.nb;
    return hip_status(launch_epilogue<T>(e, L.nepi, s), "gradient epilogue");
  }
  if (L.wide) {
    WideArgs w{};
    w.X = pr->X; w.ldx = pr->ldx; w.y = pr->y; w.B = const_cast<void*>(Bpos); w.eta = eta; w.G = G;
    w.link = pr->link;
    w.n = pr->n; w.p = (int32_t)pr->p; w.K = pr->K; w.nchunk = L.nchunk;
    w.zpart = at<void>(ws, L.off_zpart); w.R = at<void>(ws, L.off_R);
    w.lpart = at<double>(ws, L.off_lpart); w.ppart = at<double>(ws, L.off_ppart);
    w.kpart = at<double>(ws, L.off_k1);
    w.prior = pr->prior; w.scale = pr->prior_scale; w.pin = pr->pin_last_class;
    w.h = 0.5 * eps; w.eps = eps; w.mode = mode;
    w.nsplit = L.wsplit; w.tiles_per_split = L.wtps;
    w.gpart = at<void>(ws, L.off_gpart); w.gstride = L.gstride;
    // with one row slice the gradient kernel applies the leapfrog update itself: not idempotent
    HMC_TRY(timed_launch(s, L.wsplit > 1, [&] {
      return hip_status(launch_wide<T>(w, L.nb, L.tiles_y, L.nsoft, L.ngrad, s), "wide pass");
    }));
    if (L.wsplit == 1) return HMC_OK;
    EpiArgs e{};
    e.gpart = w.gpart; e.gstride = L.gstride; e.nwg = L.wsplit; e.p = (int32_t)pr->p; e.K = pr->K;
    e.B = const_cast<void*>(Bpos); e.G = G; e.eta = eta;
    e.prior = pr->prior; e.scale = pr->prior_scale; e.pin = pr->pin_last_class;
    e.h = 0.5 * eps; e.eps = eps; e.mode = mode;
    e.ppart = at<double>(ws, L.off_ppart);
    e.kpart = at<double>(ws, L.off_k1);
    return hip_status(launch_epilogue<T>(e, L.nepi, s), "gradient epilogue");
  }
  FusedArgs f;
  f.X = pr->X; f.ldx = pr->ldx; f.y = pr->y; f.B = Bpos; f.link = pr->link; f.pin = pr->pin_last_class;
  f.n = pr->n; f.p = (int32_t)pr->p; f.K = pr->K;
  f.ntiles = L.ntiles;
  f.gpart = at<void>(ws, L.off_gpart);
  f.gstride = L.gstride;
  f.lpart = at<double>(ws, L.off_lpart);
  HMC_TRY(timed_launch(s, true, [&] {
    return hip_status(launch_fused<T>(f, L.nwg, L.waves, L.mb, L.nb, L.lds, s), "fused pass");
  }));
  EpiArgs e{};
  e.gpart = f.gpart; e.gstride = L.gstride; e.nwg = L.nwg; e.p = (int32_t)pr->p; e.K = pr->K;
  e.B = const_cast<void*>(Bpos); e.G = G; e.eta = eta;
  e.prior = pr->prior; e.scale = pr->prior_scale; e.pin = pr->pin_last_class;
  e.h = 0.5 * eps; e.eps = eps; e.mode = mode;
  e.ppart = at<double>(ws, L.off_ppart);
  e.kpart = at<double>(ws, L.off_k1);
  return hip_status(launch_epilogue<T>(e, L.nepi, s), "gradient epilogue");
}

template <typename T>
hmc_status do_logpost_grad(const hmc_problem* pr, const Layout& L, const void* B, double* logpost,
                           void* G, void* ws, hipStream_t s) {
  HMC_TRY(gradient_step<T>(pr, L, B, G, nullptr, 0, 0.0, ws, s));
  FinalArgs fa{at<double>(ws, L.off_lpart), L.nl, at<double>(ws, L.off_ppart), L.np, logpost};
  return hip_status(launch_final(fa, s), "log-posterior final sum");
}

template <typename T>
hmc_status do_leapfrog(const hmc_problem* pr, const Layout& L, void* B, void* eta, void* G,
                       double* logpost, double eps, int L_steps, void* ws, hipStream_t s) {
  StartArgs sa{};
  sa.p = (int32_t)pr->p; sa.K = pr->K; sa.pin = pr->pin_last_class;
  sa.B = B; sa.G = G; sa.Bp = B; sa.eta = eta; sa.h = 0.5 * eps; sa.eps = eps; sa.draw = 0;
  HMC_TRY(hip_status(launch_start<T>(sa, L.nupd, s), "leapfrog start"));
  for (int st = 1; st <= L_steps; ++st)
    HMC_TRY(gradient_step<T>(pr, L, B, G, eta, st < L_steps ? 1 : 2, eps, ws, s, st == 1));
  FinalArgs fa{at<double>(ws, L.off_lpart), L.nl, at<double>(ws, L.off_ppart), L.np, logpost};
  return hip_status(launch_final(fa, s), "log-posterior final sum");
}

// One HMC iteration (momentum draw, L leapfrog updates, Metropolis test) enqueued on s.
// Record slot t and iteration first_iter + t come from the arguments, or, when ctr is a
// device counter {iteration, first iteration}, from device memory at run time (graphs).
template <typename T>
hmc_status enqueue_iteration(const hmc_problem* pr, const Layout& L, void* B, void* G,
                             double* logpost, const hmc_sample_args* ar, void* ws, hipStream_t s,
                             int64_t t, const int64_t* ctr) {
  void* eta = at<void>(ws, L.off_eta);
  void* Bp = at<void>(ws, L.off_bp);
  void* Gp = at<void>(ws, L.off_gp);
  double* scal = at<double>(ws, L.off_scal);
  const int64_t it = (int64_t)ar->first_iter + t;
  StartArgs sa{};
  sa.p = (int32_t)pr->p; sa.K = pr->K; sa.pin = pr->pin_last_class;
  sa.B = B; sa.G = G; sa.Bp = Bp; sa.eta = eta; sa.h = 0.5 * ar->eps; sa.eps = ar->eps;
  sa.draw = ar->replay_normals ? 1 : 2;
  sa.normals = ar->replay_normals;
  sa.seed = ar->seed; sa.chain = ar->chain; sa.iter = it; sa.t = t; sa.n_rec = ar->n_iter; sa.ctr = ctr;
  sa.k0part = at<double>(ws, L.off_k0); sa.logpost = logpost; sa.scal = scal;
  HMC_TRY(hip_status(launch_start<T>(sa, L.nupd, s), "trajectory start"));
  for (int st = 1; st <= ar->L; ++st)
    HMC_TRY(gradient_step<T>(pr, L, Bp, Gp, eta, st < ar->L ? 1 : 2, ar->eps, ws, s, st == 1));
  AcceptArgs aa{};
  aa.p = (int32_t)pr->p; aa.K = pr->K; aa.B = B; aa.G = G; aa.logpost = logpost;
  aa.Bp = Bp; aa.Gp = Gp;
  aa.lpart = at<double>(ws, L.off_lpart); aa.nl = L.nl;
  aa.ppart = at<double>(ws, L.off_ppart); aa.np = L.np;
  aa.k0part = at<double>(ws, L.off_k0); aa.nk0 = L.nupd;
  aa.k1part = at<double>(ws, L.off_k1); aa.nk1 = L.np;
  aa.scal = scal;
  aa.replay_u = ar->replay_uniforms;
  aa.inv_temp = ar->inv_temperature;
  aa.seed = ar->seed; aa.chain = ar->chain; aa.iter = it; aa.t = t; aa.n_rec = ar->n_iter; aa.ctr = ctr;
  aa.sample = ar->samples;
  aa.accepted = ar->accepted;
  aa.H = ar->H;
  aa.divergent = ar->divergent;
  return hip_status(launch_accept<T>(aa, L.nupd, s), "accept");
}

template <typename T>
hmc_status do_sample(const hmc_problem* pr, const Layout& L, void* B, void* G, double* logpost,
                     const hmc_sample_args* ar, void* ws, hipStream_t s) {
  for (int t = 0; t < ar->n_iter; ++t)
    HMC_TRY(enqueue_iteration<T>(pr, L, B, G, logpost, ar, ws, s, t, nullptr));
  return HMC_OK;
}

hmc_status check_sample_args(const hmc_sample_args* args) {
  if (!args) return fail(HMC_ERR_ARG, "args is NULL");
  if (!isfinite(args->eps) || args->eps == 0.0) return fail(HMC_ERR_ARG, "eps must be finite and non-zero");
  if (args->L < 1) return fail(HMC_ERR_ARG, "L = %d must be >= 1", args->L);
  if (args->n_iter < 1) return fail(HMC_ERR_ARG, "n_iter = %d must be >= 1", args->n_iter);
  if (args->first_iter < 0 || args->chain < 0) return fail(HMC_ERR_ARG, "first_iter and chain must be >= 0");
  if ((args->replay_normals == nullptr) != (args->replay_uniforms == nullptr))
    return fail(HMC_ERR_ARG, "replay_normals and replay_uniforms must both be set or both NULL");
  return HMC_OK;
}

// ---------------------------------------------------------------------------------------
// Batched form: many problems (bf16 formats), `chains` chains each; each chain takes
// ceil(max K / 16) class blocks (the batch's `group`), chains x group <= 4.

constexpr int kBatchMinRows = 1024;       // smallest gradient row slice the workspace holds
constexpr int kBatchDefaultRows = 4096;
constexpr int kBatchDefaultGrid = 2048;

struct BatchLayout {
  int nprob = 0, chains = 0, group = 1;   // group: 16-class blocks per chain
  bool lo = false;
  int rows = kBatchDefaultRows, grid = kBatchDefaultGrid;
  std::vector<BatchProb> table;           // entry t describes problem order[t]
  std::vector<int32_t> order;
  std::vector<int32_t> first[5];          // pack, logits, grad, epilogue, start/accept
  size_t off_table = 0, off_first = 0, off_ctr = 0, total = 0;
  int64_t n_epi = 0, n_upd = 0;
};

// Class blocks per chain of a batch: enough 16-class blocks for its largest K.
int batch_group(const hmc_problem* probs, int32_t n_prob) {
  int kmax = 0;
  for (int b = 0; b < n_prob; ++b) kmax = std::max(kmax, (int)probs[b].K);
  return class_blocks(kmax);
}

hmc_status check_batch(const hmc_problem* probs, int32_t n_prob, int32_t chains) {
  if (!probs) return fail(HMC_ERR_ARG, "problem array is NULL");
  if (n_prob < 1 || n_prob > 4096) return fail(HMC_ERR_SHAPE, "n_prob = %d must be in [1, 4096]", n_prob);
  if (chains != 1 && chains != 2 && chains != 4) return fail(HMC_ERR_SHAPE, "chains = %d must be 1, 2 or 4", chains);
  for (int b = 0; b < n_prob; ++b) {
    if (probs[b].K < 2 || probs[b].K > 64)
      return fail(HMC_ERR_SHAPE, "problem %d: K = %d must be in [2, 64] in the batched form", b, probs[b].K);
  }
  const int group = batch_group(probs, n_prob);
  if (chains * group > 4)
    return fail(HMC_ERR_SHAPE, "%d chains of %d class blocks each (K up to %d) exceed the 4 blocks of a batched pass",
                chains, group, 16 * group);
  for (int b = 0; b < n_prob; ++b) {
    HMC_TRY(check_problem(&probs[b]));
    if (!is_bf16(probs[b].xfmt))
      return fail(HMC_ERR_UNSUPPORTED, "problem %d: the batched form takes bf16 X (split X with hmc_split_bf16)", b);
    if (probs[b].xfmt != probs[0].xfmt)
      return fail(HMC_ERR_DTYPE, "problem %d: all problems of a batch must share one X format", b);
    // 32-bit offsets into the packed residuals of a problem's class blocks (64 bytes per
    // row and block)
    if ((uint64_t)(probs[b].n + kHiloRows) * 64 * (chains * group) > 0xFFFFFFFFull)
      return fail(HMC_ERR_UNSUPPORTED, "problem %d: n = %lld rows exceed the packed residual's 32-bit offsets",
                  b, (long long)probs[b].n);
  }
  return HMC_OK;
}

// Sizes and offsets of the batch workspace for gradient row slices of `rows` rows (the
// buffers are sized for kBatchMinRows, so any tuning >= it fits the same workspace).
hmc_status make_batch_layout(const hmc_problem* probs, int32_t n_prob, int32_t chains, int rows,
                             int grid, BatchLayout* B) {
  HMC_TRY(check_batch(probs, n_prob, chains));
  if (rows == 0) rows = kBatchDefaultRows;
  if (grid == 0) grid = kBatchDefaultGrid;
  if (rows < kBatchMinRows || rows % 32) return fail(HMC_ERR_ARG, "rows_per_slice = %d must be a multiple of 32, >= %d", rows, kBatchMinRows);
  if (grid < 64 || grid > 65536) return fail(HMC_ERR_ARG, "grid = %d must be in [64, 65536]", grid);
  B->nprob = n_prob; B->chains = chains; B->rows = rows; B->grid = grid;
  B->group = batch_group(probs, n_prob);
  const int blocks = chains * B->group;
  B->lo = probs[0].xfmt == HMC_X_BF16_HILO;
  B->table.assign(n_prob, BatchProb{});
  // Work items are numbered problem by problem in decreasing order of p (the cost of a
  // logits row block): the largest items start first and the smallest fill the tail.
  B->order.resize(n_prob);
  for (int b = 0; b < n_prob; ++b) B->order[b] = b;
  std::stable_sort(B->order.begin(), B->order.end(),
                   [&](int32_t u, int32_t v) { return probs[u].p > probs[v].p; });
  for (auto& f : B->first) f.assign(n_prob + 1, 0);
  size_t off = 0;
  B->off_table = off; off = align_up(off + sizeof(BatchProb) * n_prob);
  B->off_first = off; off = align_up(off + 5 * sizeof(int32_t) * (n_prob + 1));
  B->off_ctr = off;   off = align_up(off + 2 * sizeof(int64_t));
  const size_t frag = 2 * 512 * sizeof(uint16_t);
  const int64_t rb_rows = kHiloRows;
  int64_t items[5] = {0, 0, 0, 0, 0};
  for (int t = 0; t < n_prob; ++t) {
    const int b = B->order[t];
    const hmc_problem& pr = probs[b];
    BatchProb& P = B->table[t];
    const int64_t pk = pr.p * (int64_t)pr.K;
    P.n = pr.n; P.p = (int32_t)pr.p; P.K = pr.K;
    P.prior = pr.prior; P.pin = pr.pin_last_class; P.scale = pr.prior_scale;
    P.nrb = (int32_t)((pr.n + rb_rows - 1) / rb_rows);
    P.gcols = (int32_t)((pr.p + 127) / 128);
    P.rps = rows;
    P.nsplit = (int32_t)((pr.n + rows - 1) / rows);
    P.cstride = (pk + 63) / 64 * 64;
    P.gstride = chains * P.cstride;
    P.ne = (int32_t)((pk + 63) / 64);
    P.ne4 = (P.ne + 3) / 4;
    P.nu = (int32_t)((pk + 255) / 256);
    P.chain0 = b * chains;
    const int64_t nsplit_max = (pr.n + kBatchMinRows - 1) / kBatchMinRows;
    const int64_t nks = (pr.p + 31) / 32;
    // offsets relative to the workspace base, turned into pointers when bound
    auto put = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
    P.eta = reinterpret_cast<float*>(put(chains * pk * 4));
    P.Bp = reinterpret_cast<float*>(put(chains * pk * 4));
    P.Gp = reinterpret_cast<float*>(put(chains * pk * 4));
    P.Bpk = reinterpret_cast<uint16_t*>(put(nks * blocks * frag));
    P.Rpk = reinterpret_cast<uint16_t*>(put((size_t)P.nrb * (rb_rows / 32) * blocks * frag));
    P.gpart = reinterpret_cast<float*>(put(nsplit_max * P.gstride * 4));
    P.lpart = reinterpret_cast<double*>(put((size_t)P.nrb * chains * 8));
    P.ppart = reinterpret_cast<double*>(put((size_t)chains * P.ne * 8));
    P.k1part = reinterpret_cast<double*>(put((size_t)chains * P.ne * 8));
    P.k0part = reinterpret_cast<double*>(put((size_t)chains * P.nu * 8));
    P.scal = reinterpret_cast<double*>(put((size_t)chains * 8));
    const int64_t per[5] = {nks * blocks * 64, P.nrb, (int64_t)P.gcols * P.nsplit,
                            (int64_t)chains * P.ne4, (int64_t)chains * P.nu};
    for (int k = 0; k < 5; ++k) {
      B->first[k][t] = (int32_t)items[k];
      items[k] += per[k];
    }
  }
  for (int k = 0; k < 5; ++k) {
    if (items[k] > INT32_MAX) return fail(HMC_ERR_SHAPE, "batch too large for 32-bit item indices");
    B->first[k][n_prob] = (int32_t)items[k];
  }
  B->n_epi = items[3];
  B->n_upd = items[4];
  B->total = off;
  return HMC_OK;
}

// Resolve workspace offsets to device pointers, attach the caller's state and upload the
// table (a host-to-device copy on s; the host copy may be released when this returns).
hmc_status bind_batch(BatchLayout* BL, const hmc_problem* probs, void* const* B, void* const* G,
                      double* logpost, const hmc_batch_args* ar, void* ws, hipStream_t s) {
  const double* eps = ar ? ar->eps : nullptr;
  void* const* samples = ar ? ar->samples : nullptr;
  double* const* moments = ar ? ar->moments : nullptr;
  char* base = static_cast<char*>(ws);
  auto fix = [&](auto*& ptr) { ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(base + reinterpret_cast<size_t>(ptr)); };
  std::vector<BatchProb> tab = BL->table;
  for (int t = 0; t < BL->nprob; ++t) {
    const int b = BL->order[t];
    BatchProb& P = tab[t];
    const hmc_problem& pr = probs[b];
    if (!B[b] || !G[b]) return fail(HMC_ERR_ARG, "problem %d: B and G must be device pointers", b);
    P.Xhi = static_cast<const uint16_t*>(pr.X);
    P.Xlo = static_cast<const uint16_t*>(pr.X_lo);
    P.ldx = pr.ldx; P.y = pr.y;
    P.eps = eps ? eps[b] : 0.0;
    P.B = static_cast<float*>(B[b]); P.G = static_cast<float*>(G[b]);
    P.logpost = logpost + (int64_t)b * BL->chains;
    fix(P.eta); fix(P.Bp); fix(P.Gp); fix(P.Bpk); fix(P.Rpk); fix(P.gpart);
    fix(P.lpart); fix(P.ppart); fix(P.k1part); fix(P.k0part); fix(P.scal);
    P.samples = samples ? static_cast<float*>(samples[b]) : nullptr;
    P.moments = moments ? moments[b] : nullptr;
    P.normals = (ar && ar->replay_normals) ? ar->replay_normals[b] : nullptr;
    P.uniforms = (ar && ar->replay_uniforms) ? ar->replay_uniforms[b] : nullptr;
  }
  std::vector<int32_t> firsts;
  for (int k = 0; k < 5; ++k) firsts.insert(firsts.end(), BL->first[k].begin(), BL->first[k].end());
  HMC_TRY(hip_status(hipMemcpyAsync(base + BL->off_table, tab.data(), sizeof(BatchProb) * tab.size(),
                                    hipMemcpyHostToDevice, s), "batch table upload"));
  HMC_TRY(hip_status(hipMemcpyAsync(base + BL->off_first, firsts.data(), sizeof(int32_t) * firsts.size(),
                                    hipMemcpyHostToDevice, s), "batch item upload"));
  return HMC_OK;
}

BatchArgs batch_args(const BatchLayout& BL, void* ws) {
  char* base = static_cast<char*>(ws);
  BatchArgs a{};
  a.probs = reinterpret_cast<const BatchProb*>(base + BL.off_table);
  a.nprob = BL.nprob; a.chains = BL.chains; a.group = BL.group; a.total_chains = BL.nprob * BL.chains;
  const int32_t* f = reinterpret_cast<const int32_t*>(base + BL.off_first);
  a.first_pack = f; a.first_logits = f + (BL.nprob + 1); a.first_grad = f + 2 * (BL.nprob + 1);
  a.first_epi = f + 3 * (BL.nprob + 1); a.first_upd = f + 4 * (BL.nprob + 1);
  a.ctr = reinterpret_cast<int64_t*>(base + BL.off_ctr);
  return a;
}

int persistent_grid(int64_t items, int grid) { return (int)(items < grid ? (items > 0 ? items : 1) : grid); }

// One batched gradient evaluation (all chains of all problems) with its epilogue.
// pack: as for gradient_step (a mode-1 batched epilogue packs the next pass's B operand).
hmc_status batch_gradient(const BatchLayout& BL, BatchArgs a, int mode, hipStream_t s, bool pack = true) {
  a.mode = mode;
  const int grid[3] = {persistent_grid((BL.first[0][BL.nprob] + 255) / 256, BL.grid),
                       persistent_grid(BL.first[1][BL.nprob], BL.grid),
                       persistent_grid(xcd_span(BL.first[2][BL.nprob], kGradChunk), BL.grid)};
  HMC_TRY(timed_launch(s, true, [&] {
    return hip_status(launch_batch_pass(a, BL.chains, BL.group, BL.lo, grid, pack, s), "batched split-precision pass");
  }));
  return hip_status(launch_batch_epilogue(a, (int)BL.n_epi, s), "batched epilogue");
}

hmc_status batch_iteration(const BatchLayout& BL, BatchArgs a, int L_steps, hipStream_t s) {
  HMC_TRY(hip_status(launch_batch_start(a, (int)BL.n_upd, s), "batched start"));
  for (int st = 1; st <= L_steps; ++st) HMC_TRY(batch_gradient(BL, a, st < L_steps ? 1 : 2, s, st == 1));
  HMC_TRY(hip_status(launch_batch_accept(a, (int)BL.n_upd, s), "batched accept"));
  return hip_status(launch_counter(a.ctr, 0, 1, s), "iteration counter");
}

hmc_status check_batch_args(const hmc_batch_args* ar, int32_t n_prob) {
  if (!ar) return fail(HMC_ERR_ARG, "args is NULL");
  if (!ar->eps) return fail(HMC_ERR_ARG, "eps must be a host array of n_prob step sizes");
  for (int b = 0; b < n_prob; ++b)
    if (!isfinite(ar->eps[b]) || ar->eps[b] == 0.0)
      return fail(HMC_ERR_ARG, "eps[%d] must be finite and non-zero", b);
  if (ar->L < 1) return fail(HMC_ERR_ARG, "L = %d must be >= 1", ar->L);
  if (ar->n_iter < 1) return fail(HMC_ERR_ARG, "n_iter = %d must be >= 1", ar->n_iter);
  if (ar->first_iter < 0) return fail(HMC_ERR_ARG, "first_iter must be >= 0");
  if ((ar->replay_normals == nullptr) != (ar->replay_uniforms == nullptr))
    return fail(HMC_ERR_ARG, "replay_normals and replay_uniforms must both be set or both NULL");
  if (ar->replay_normals)
    for (int b = 0; b < n_prob; ++b)
      if (!ar->replay_normals[b] || !ar->replay_uniforms[b])
        return fail(HMC_ERR_ARG, "problem %d: replay arrays must be device pointers", b);
  return HMC_OK;
}

BatchArgs records(BatchArgs a, const hmc_batch_args* ar) {
  a.seed = ar->seed; a.n_rec = ar->n_iter;
  a.accepted = ar->accepted; a.H = ar->H; a.divergent = ar->divergent;
  a.inv_temp = ar->inv_temperature;
  return a;
}

}  // namespace

extern "C" {

int64_t hmc_max_p(int32_t xfmt, int32_t K) {
  if (xfmt != HMC_X_F64 && xfmt != HMC_X_F32 && !is_bf16(xfmt)) return 0;
  if (K < 1 || K > 64) return 0;
  // row-tile kernel up to its padded width; beyond it the wide-p kernels, bounded by
  // 32-bit element indexing of the p x K state and by the row pitch 32-bit buffer offsets
  // reach (p <= ldx)
  const int64_t by_state = ((int64_t)1 << 30) / K;
  return std::min(by_state, max_ldx(xfmt));
}

hmc_status hmc_workspace_bytes(const hmc_problem* prob, size_t* bytes) {
  if (!bytes) return fail(HMC_ERR_ARG, "bytes is NULL");
  Layout L;
  HMC_TRY(make_layout(prob, &L));
  *bytes = L.total;
  return HMC_OK;
}

hmc_status hmc_autotune_workspace_bytes(const hmc_problem* prob, size_t* bytes) {
  if (!bytes) return fail(HMC_ERR_ARG, "bytes is NULL");
  if (!prob) return fail(HMC_ERR_ARG, "problem descriptor is NULL");
  hmc_problem q = *prob;
  q.tuning = hmc_tuning{};
  Layout L;
  HMC_TRY(make_layout(&q, &L));
  size_t need = L.total;
  for (const hmc_tuning& t : tuning_candidates(&q)) {
    q.tuning = t;
    if (make_layout(&q, &L) == HMC_OK) need = std::max(need, L.total);
  }
  *bytes = need;
  return HMC_OK;
}

hmc_status hmc_autotune(const hmc_problem* prob, const void* B, double* logpost, void* G, void* ws,
                        size_t ws_bytes, void* stream, hmc_tuning* out, double* best_us) {
  if (!out) return fail(HMC_ERR_ARG, "out is NULL");
  if (!prob) return fail(HMC_ERR_ARG, "problem descriptor is NULL");
  if (!B || !logpost || !G) return fail(HMC_ERR_ARG, "B, logpost and G must be device pointers");
  hmc_problem q = *prob;
  q.tuning = hmc_tuning{};
  Layout L0;
  HMC_TRY(make_layout(&q, &L0));
  std::vector<hmc_tuning> cands = tuning_candidates(&q);
  cands.insert(cands.begin(), hmc_tuning{});                 // the rule itself
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  HMC_TRY(hip_status(hipEventCreate(&e0), "hipEventCreate"));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HMC_ERR_HIP, "hipEventCreate failed");
  }
  const bool prof = g_prof.on;
  g_prof.on = false;
  hmc_status st = HMC_OK;
  double best = -1.0;
  hmc_tuning pick{};
  auto run = [&](const Layout& L, int reps) -> hmc_status {
    for (int r = 0; r < reps; ++r)
      HMC_TRY(L.f64 ? do_logpost_grad<double>(&q, L, B, logpost, G, ws, s)
                    : do_logpost_grad<float>(&q, L, B, logpost, G, ws, s));
    return HMC_OK;
  };
  for (const hmc_tuning& t : cands) {
    q.tuning = t;
    Layout L;
    if (make_layout(&q, &L) != HMC_OK) continue;            // a candidate this shape cannot take
    if (check_ws(L, ws, ws_bytes) != HMC_OK) {
      st = fail(HMC_ERR_WORKSPACE, "workspace of %zu bytes < %zu needed by a candidate "
                "(size it with hmc_autotune_workspace_bytes)", ws_bytes, L.total);
      break;
    }
    // one untimed call, one timed call to size the measurement, then about 2 ms of calls
    float ms = 0.0f;
    st = run(L, 1);
    if (st == HMC_OK) st = hip_status(hipEventRecord(e0, s), "hipEventRecord");
    if (st == HMC_OK) st = run(L, 1);
    if (st == HMC_OK) st = hip_status(hipEventRecord(e1, s), "hipEventRecord");
    if (st == HMC_OK) st = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
    if (st == HMC_OK) st = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    if (st != HMC_OK) break;
    // three rounds of about 2 ms each; the fastest round counts (the others may include
    // interference)
    const int reps = (int)std::min(100.0, std::max(3.0, 2.0 / std::max((double)ms, 1e-3)));
    double us = -1.0;
    for (int round = 0; round < 3 && st == HMC_OK; ++round) {
      st = hip_status(hipEventRecord(e0, s), "hipEventRecord");
      if (st == HMC_OK) st = run(L, reps);
      if (st == HMC_OK) st = hip_status(hipEventRecord(e1, s), "hipEventRecord");
      if (st == HMC_OK) st = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
      if (st == HMC_OK) st = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (st == HMC_OK && (us < 0.0 || 1e3 * ms / reps < us)) us = 1e3 * ms / reps;
    }
    if (st != HMC_OK) break;
    if (best < 0.0 || us < best) { best = us; pick = t; }
  }
  g_prof.on = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != HMC_OK) return st;
  // leave G and logpost at B computed with the chosen decomposition
  q.tuning = pick;
  Layout L;
  HMC_TRY(make_layout(&q, &L));
  HMC_TRY(run(L, 1));
  *out = pick;
  if (best_us) *best_us = best;
  return HMC_OK;
}

hmc_status hmc_logpost_grad(const hmc_problem* prob, const void* B, double* logpost, void* G,
                            void* ws, size_t ws_bytes, void* stream) {
  Layout L;
  HMC_TRY(make_layout(prob, &L));
  if (!B || !logpost || !G) return fail(HMC_ERR_ARG, "B, logpost and G must be device pointers");
  HMC_TRY(check_ws(L, ws, ws_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return L.f64 ? do_logpost_grad<double>(prob, L, B, logpost, G, ws, s)
               : do_logpost_grad<float>(prob, L, B, logpost, G, ws, s);
}

}  // extern "C"

// Workspace of hmc_logpost_grad_noalloc: a device array of fixed size that every GPU the
// library runs on holds from module load until the process ends. In host code `scratch`
// names a host-side stand-in; its device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is passed to kernels.
namespace {
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hmc_status scratch_for_current_device(void** out) {
  int dev = 0;
  HMC_TRY(hip_status(hipGetDevice(&dev), "hipGetDevice"));
  if (dev < 0 || dev >= kMaxDevices) return fail(HMC_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HMC_TRY(hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
    if (!p) return fail(HMC_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HMC_OK;
}
}  // namespace

extern "C" {

hmc_status hmc_logpost_grad_noalloc(const hmc_problem* prob, const void* B, double* logpost,
                                    void* G, void* stream) {
  Layout L;
  HMC_TRY(make_layout(prob, &L));
  if (!B || !logpost || !G) return fail(HMC_ERR_ARG, "B, logpost and G must be device pointers");
  if (L.total > kScratchBytes)
    return fail(HMC_ERR_WORKSPACE, "this problem needs %zu bytes of workspace; the built-in scratch holds %zu "
                "(use hmc_logpost_grad with a caller workspace)", L.total, kScratchBytes);
  void* ws = nullptr;
  HMC_TRY(scratch_for_current_device(&ws));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return L.f64 ? do_logpost_grad<double>(prob, L, B, logpost, G, ws, s)
               : do_logpost_grad<float>(prob, L, B, logpost, G, ws, s);
}

hmc_status hmc_leapfrog(const hmc_problem* prob, void* B, void* eta, void* G, double* logpost,
                        double eps, int32_t L_steps, void* ws, size_t ws_bytes, void* stream) {
  Layout L;
  HMC_TRY(make_layout(prob, &L));
  if (!B || !eta || !G || !logpost) return fail(HMC_ERR_ARG, "B, eta, G and logpost must be device pointers");
  if (!isfinite(eps) || eps == 0.0) return fail(HMC_ERR_ARG, "eps must be finite and non-zero");
  if (L_steps < 1) return fail(HMC_ERR_ARG, "L = %d must be >= 1", L_steps);
  HMC_TRY(check_ws(L, ws, ws_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return L.f64 ? do_leapfrog<double>(prob, L, B, eta, G, logpost, eps, L_steps, ws, s)
               : do_leapfrog<float>(prob, L, B, eta, G, logpost, eps, L_steps, ws, s);
}

hmc_status hmc_sample(const hmc_problem* prob, void* B, void* G, double* logpost,
                      const hmc_sample_args* args, void* ws, size_t ws_bytes, void* stream) {
  Layout L;
  HMC_TRY(make_layout(prob, &L));
  HMC_TRY(check_sample_args(args));
  if (!B || !G || !logpost) return fail(HMC_ERR_ARG, "B, G and logpost must be device pointers");
  HMC_TRY(check_ws(L, ws, ws_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return L.f64 ? do_sample<double>(prob, L, B, G, logpost, args, ws, s)
               : do_sample<float>(prob, L, B, G, logpost, args, ws, s);
}

hmc_status hmc_batch_workspace_bytes(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                                     size_t* bytes) {
  if (!bytes) return fail(HMC_ERR_ARG, "bytes is NULL");
  BatchLayout BL;
  HMC_TRY(make_batch_layout(probs, n_prob, chains, 0, 0, &BL));
  *bytes = BL.total;
  return HMC_OK;
}

static hmc_status batch_common(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                               void* const* B, void* const* G, double* logpost,
                               const hmc_batch_tuning* tune, void* ws, size_t ws_bytes, BatchLayout* BL) {
  HMC_TRY(make_batch_layout(probs, n_prob, chains, tune ? tune->rows_per_slice : 0,
                            tune ? tune->grid : 0, BL));
  if (!B || !G || !logpost) return fail(HMC_ERR_ARG, "B, G (host arrays of device pointers) and logpost are required");
  if (!ws) return fail(HMC_ERR_WORKSPACE, "workspace pointer is NULL");
  if ((uintptr_t)ws % kAlign) return fail(HMC_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < BL->total)
    return fail(HMC_ERR_WORKSPACE, "workspace of %zu bytes < required %zu", ws_bytes, BL->total);
  return HMC_OK;
}

static hmc_status batch_logpost_grad(const BatchLayout& BL, void* ws, hipStream_t s) {
  BatchArgs a = batch_args(BL, ws);
  a.at_current = 1;
  HMC_TRY(batch_gradient(BL, a, 0, s));
  return hip_status(launch_batch_final(a, (int)BL.n_upd, s), "batched log-posterior sum");
}

hmc_status hmc_logpost_grad_batched(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                                    void* const* B, double* logpost, void* const* G,
                                    const hmc_batch_tuning* tune, void* ws, size_t ws_bytes,
                                    void* stream) {
  BatchLayout BL;
  HMC_TRY(batch_common(probs, n_prob, chains, B, G, logpost, tune, ws, ws_bytes, &BL));
  hipStream_t s = static_cast<hipStream_t>(stream);
  HMC_TRY(bind_batch(&BL, probs, B, G, logpost, nullptr, ws, s));
  return batch_logpost_grad(BL, ws, s);
}

hmc_status hmc_sample_batched(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                              void* const* B, void* const* G, double* logpost,
                              const hmc_batch_args* args, void* ws, size_t ws_bytes, void* stream) {
  HMC_TRY(check_batch_args(args, n_prob));
  BatchLayout BL;
  HMC_TRY(batch_common(probs, n_prob, chains, B, G, logpost, &args->tuning, ws, ws_bytes, &BL));
  hipStream_t s = static_cast<hipStream_t>(stream);
  HMC_TRY(bind_batch(&BL, probs, B, G, logpost, args, ws, s));
  BatchArgs a = records(batch_args(BL, ws), args);
  HMC_TRY(hip_status(launch_counter(a.ctr, args->first_iter, 0, s), "iteration counter"));
  for (int t = 0; t < args->n_iter; ++t) HMC_TRY(batch_iteration(BL, a, args->L, s));
  return HMC_OK;
}

hmc_status hmc_batch_autotune(const hmc_problem* probs, int32_t n_prob, int32_t chains,
                              void* const* B, void* const* G, double* logpost, void* ws,
                              size_t ws_bytes, void* stream, hmc_batch_tuning* out) {
  if (!out) return fail(HMC_ERR_ARG, "out is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  static const int kRows[] = {1024, 2048, 4096, 8192};
  static const int kGrid[] = {1024, 2048, 4096, 8192, 16384};
  hipEvent_t e0, e1;
  HMC_TRY(hip_status(hipEventCreate(&e0), "hipEventCreate"));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(HMC_ERR_HIP, "hipEventCreate failed");
  }
  const bool prof = g_prof.on;
  g_prof.on = false;
  hmc_status st = HMC_OK;
  float best = 0.0f;
  hmc_batch_tuning pick{kBatchDefaultRows, kBatchDefaultGrid};
  for (int r : kRows) {
    for (int g : kGrid) {
      hmc_batch_tuning t{r, g};
      BatchLayout BL;
      st = batch_common(probs, n_prob, chains, B, G, logpost, &t, ws, ws_bytes, &BL);
      if (st == HMC_OK) st = bind_batch(&BL, probs, B, G, logpost, nullptr, ws, s);
      if (st == HMC_OK) st = batch_logpost_grad(BL, ws, s);          // warm-up
      if (st == HMC_OK) st = hip_status(hipEventRecord(e0, s), "hipEventRecord");
      for (int k = 0; k < 3 && st == HMC_OK; ++k) st = batch_logpost_grad(BL, ws, s);
      if (st == HMC_OK) st = hip_status(hipEventRecord(e1, s), "hipEventRecord");
      if (st == HMC_OK) st = hip_status(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.0f;
      if (st == HMC_OK) st = hip_status(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (st != HMC_OK) break;
      if (best == 0.0f || ms < best) { best = ms; pick = t; }
    }
    if (st != HMC_OK) break;
  }
  g_prof.on = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == HMC_OK) *out = pick;
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Plans: one HMC iteration captured as a HIP graph and replayed; the iteration index
// lives in the workspace counter, advanced by the graph's last node.
struct hmc_plan {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t* ctr = nullptr;
  int64_t first_iter = 0, n_rec = 0, launched = 0;
  bool bounded = false;    // replay inputs or records in use: launches limited to n_rec
  bool started = false;
};

namespace {

template <typename F>
hmc_status capture(hmc_plan* P, F&& enqueue) {
  hipStream_t cs = nullptr;
  HMC_TRY(hip_status(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate"));
  const bool prof = g_prof.on;
  g_prof.on = false;
  hmc_status st = hip_status(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (st == HMC_OK) {
    st = enqueue(cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (st == HMC_OK) st = hip_status(e, "hipStreamEndCapture");
    if (st == HMC_OK) {
      P->graph = g;
      st = hip_status(hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  g_prof.on = prof;
  (void)hipStreamDestroy(cs);
  return st;
}

}  // namespace

extern "C" {

hmc_status hmc_plan_create(hmc_plan** plan, const hmc_problem* prob, void* B, void* G,
                           double* logpost, const hmc_sample_args* args, void* ws,
                           size_t ws_bytes, void* stream) {
  (void)stream;
  if (!plan) return fail(HMC_ERR_ARG, "plan is NULL");
  *plan = nullptr;
  Layout L;
  HMC_TRY(make_layout(prob, &L));
  HMC_TRY(check_sample_args(args));
  if (!B || !G || !logpost) return fail(HMC_ERR_ARG, "B, G and logpost must be device pointers");
  HMC_TRY(check_ws(L, ws, ws_bytes));
  hmc_plan* P = new hmc_plan;
  P->ctr = at<int64_t>(ws, L.off_ctr);
  P->first_iter = args->first_iter;
  P->n_rec = args->n_iter;
  P->bounded = args->replay_normals || args->samples || args->accepted || args->H || args->divergent ||
               args->inv_temperature;
  const hmc_sample_args ar = *args;
  const hmc_problem pr = *prob;
  hmc_status st = capture(P, [&](hipStream_t cs) -> hmc_status {
    HMC_TRY(L.f64 ? enqueue_iteration<double>(&pr, L, B, G, logpost, &ar, ws, cs, 0, P->ctr)
                  : enqueue_iteration<float>(&pr, L, B, G, logpost, &ar, ws, cs, 0, P->ctr));
    return hip_status(launch_counter(P->ctr, 0, 1, cs), "iteration counter");
  });
  if (st != HMC_OK) {
    hmc_plan_destroy(P);
    return st;
  }
  *plan = P;
  return HMC_OK;
}

hmc_status hmc_plan_create_batched(hmc_plan** plan, const hmc_problem* probs, int32_t n_prob,
                                   int32_t chains, void* const* B, void* const* G,
                                   double* logpost, const hmc_batch_args* args, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (!plan) return fail(HMC_ERR_ARG, "plan is NULL");
  *plan = nullptr;
  HMC_TRY(check_batch_args(args, n_prob));
  BatchLayout BL;
  HMC_TRY(batch_common(probs, n_prob, chains, B, G, logpost, &args->tuning, ws, ws_bytes, &BL));
  hipStream_t s = static_cast<hipStream_t>(stream);
  HMC_TRY(bind_batch(&BL, probs, B, G, logpost, args, ws, s));
  // the graph may be launched on another stream: the table must be in place first
  HMC_TRY(hip_status(hipStreamSynchronize(s), "hipStreamSynchronize"));
  hmc_plan* P = new hmc_plan;
  const BatchArgs a = records(batch_args(BL, ws), args);
  P->ctr = a.ctr;
  P->first_iter = args->first_iter;
  P->n_rec = args->n_iter;
  P->bounded = args->samples || args->accepted || args->H || args->divergent ||
               args->replay_normals || args->inv_temperature;
  const int L_steps = args->L;
  hmc_status st = capture(P, [&](hipStream_t cs) { return batch_iteration(BL, a, L_steps, cs); });
  if (st != HMC_OK) {
    hmc_plan_destroy(P);
    return st;
  }
  *plan = P;
  return HMC_OK;
}

hmc_status hmc_plan_launch(hmc_plan* plan, int32_t n_iter, void* stream) {
  if (!plan || !plan->exec) return fail(HMC_ERR_ARG, "plan is NULL or was not created");
  if (n_iter < 0) return fail(HMC_ERR_ARG, "n_iter = %d must be >= 0", n_iter);
  if (plan->bounded && plan->launched + n_iter > plan->n_rec)
    return fail(HMC_ERR_ARG, "%lld + %d iterations exceed the %lld the plan's records hold",
                (long long)plan->launched, n_iter, (long long)plan->n_rec);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!plan->started) {
    HMC_TRY(hip_status(launch_counter(plan->ctr, plan->first_iter, 0, s), "iteration counter"));
    plan->started = true;
  }
  for (int i = 0; i < n_iter; ++i) HMC_TRY(hip_status(hipGraphLaunch(plan->exec, s), "hipGraphLaunch"));
  plan->launched += n_iter;
  return HMC_OK;
}

hmc_status hmc_plan_destroy(hmc_plan* plan) {
  if (!plan) return HMC_OK;
  hmc_status st = HMC_OK;
  if (plan->exec && hipGraphExecDestroy(plan->exec) != hipSuccess) st = fail(HMC_ERR_HIP, "hipGraphExecDestroy failed");
  if (plan->graph && hipGraphDestroy(plan->graph) != hipSuccess) st = fail(HMC_ERR_HIP, "hipGraphDestroy failed");
  delete plan;
  return st;
}

hmc_status hmc_split_bf16(const void* X, int32_t src_fmt, int64_t n, int64_t p, int64_t ldx,
                          void* X_hi, void* X_lo, int64_t ld_out, void* stream) {
  if (src_fmt != HMC_X_F64 && src_fmt != HMC_X_F32)
    return fail(HMC_ERR_DTYPE, "source format %d must be HMC_X_F64 or HMC_X_F32", src_fmt);
  if (n < 1 || p < 1) return fail(HMC_ERR_SHAPE, "n and p must be >= 1");
  if (ldx < p) return fail(HMC_ERR_SHAPE, "ldx = %lld < p = %lld", (long long)ldx, (long long)p);
  if (ld_out < p || ld_out % 8)
    return fail(HMC_ERR_SHAPE, "ld_out = %lld must be >= p and a multiple of 8", (long long)ld_out);
  if (n > ((int64_t)1 << 40) || p > ((int64_t)1 << 31)) return fail(HMC_ERR_SHAPE, "n or p too large");
  if (!X || !X_hi) return fail(HMC_ERR_ARG, "X and X_hi must be device pointers");
  if ((uintptr_t)X_hi % 16 || (uintptr_t)X_lo % 16)
    return fail(HMC_ERR_ARG, "X_hi and X_lo must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint16_t* hi = static_cast<uint16_t*>(X_hi);
  uint16_t* lo = static_cast<uint16_t*>(X_lo);
  const hipError_t e = src_fmt == HMC_X_F64
      ? launch_split<double>(static_cast<const double*>(X), ldx, n, p, hi, lo, ld_out, s)
      : launch_split<float>(static_cast<const float*>(X), ldx, n, p, hi, lo, ld_out, s);
  return hip_status(e, "bf16 split");
}

hmc_status hmc_posterior_predictive(const hmc_problem* prob, const void* samples, int32_t n_samples,
                                    double* mean_prob, int32_t* classes, void* stream) {
  if (!prob) return fail(HMC_ERR_ARG, "problem descriptor is NULL");
  if (prob->xfmt != HMC_X_F64 && prob->xfmt != HMC_X_F32)
    return fail(HMC_ERR_UNSUPPORTED, "posterior-predictive classification takes FP64 or FP32 X");
  if (prob->link != HMC_LINK_SOFTMAX)
    return fail(HMC_ERR_UNSUPPORTED, "posterior-predictive classification is for the multinomial logit");
  if (prob->n < 1 || prob->p < 1) return fail(HMC_ERR_SHAPE, "n and p must be >= 1");
  if (prob->K < 2 || prob->K > 64) return fail(HMC_ERR_SHAPE, "K = %d must be in [2, 64]", prob->K);
  if (prob->ldx < prob->p) return fail(HMC_ERR_SHAPE, "ldx < p");
  if (prob->n > ((int64_t)1 << 40)) return fail(HMC_ERR_SHAPE, "n too large");
  if (prob->pin_last_class != 0 && prob->pin_last_class != 1)
    return fail(HMC_ERR_ARG, "pin_last_class must be 0 or 1");
  if (!prob->X || !samples) return fail(HMC_ERR_ARG, "X and samples must be device pointers");
  if (!mean_prob && !classes) return fail(HMC_ERR_ARG, "at least one of mean_prob and classes is required");
  if (n_samples < 1) return fail(HMC_ERR_ARG, "n_samples = %d must be >= 1", n_samples);
  const bool f64 = prob->xfmt == HMC_X_F64;
  if (predict_lds_bytes(prob->p, prob->K, f64) > kLdsLimit)
    return fail(HMC_ERR_UNSUPPORTED, "p = %lld with K = %d: a 16-row tile and one sample exceed the 160 KB LDS",
                (long long)prob->p, prob->K);
  PredictArgs a;
  a.X = prob->X; a.ldx = prob->ldx; a.n = prob->n;
  a.p = (int32_t)prob->p; a.K = prob->K; a.pin = prob->pin_last_class;
  a.samples = samples; a.n_samples = n_samples; a.mean_prob = mean_prob; a.classes = classes;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return hip_status(f64 ? launch_predict<double>(a, s) : launch_predict<float>(a, s),
                    "posterior-predictive classification");
}

hmc_status hmc_stream_read(const void* buf, size_t bytes, int32_t reps, void* sink, void* stream) {
  if (!buf) return fail(HMC_ERR_ARG, "buf must be a device pointer");
  if ((uintptr_t)buf % 16 || bytes % 16 || bytes == 0)
    return fail(HMC_ERR_ARG, "buf must be 16-byte aligned and bytes a positive multiple of 16");
  if (reps < 1 || reps > 1000) return fail(HMC_ERR_ARG, "reps = %d must be in [1, 1000]", reps);
  if (sink && (uintptr_t)sink % 4) return fail(HMC_ERR_ARG, "sink must be 4-byte aligned");
  return hip_status(launch_stream_read(buf, (int64_t)bytes, reps, static_cast<unsigned*>(sink),
                                       static_cast<hipStream_t>(stream)), "stream read");
}

hmc_status hmc_profile_begin(int32_t capacity, int32_t repeat) {
  if (g_prof.on) return fail(HMC_ERR_ARG, "profiling already active");
  if (capacity < 1 || capacity > (1 << 20)) return fail(HMC_ERR_ARG, "capacity out of range");
  if (repeat < 1 || repeat > 64) return fail(HMC_ERR_ARG, "repeat = %d must be in [1, 64]", repeat);
  g_prof.ev = new hipEvent_t[2 * (size_t)capacity];
  for (int i = 0; i < 2 * capacity; ++i) {
    hipError_t e = hipEventCreate(&g_prof.ev[i]);
    if (e != hipSuccess) {
      for (int k = 0; k < i; ++k) (void)hipEventDestroy(g_prof.ev[k]);
      delete[] g_prof.ev;
      g_prof.ev = nullptr;
      return hip_status(e, "hipEventCreate");
    }
  }
  g_prof.reps = new int[capacity];
  g_prof.repeat = repeat;
  g_prof.cap = capacity;
  g_prof.used = 0;
  g_prof.on = true;
  return HMC_OK;
}

hmc_status hmc_profile_end(int64_t* launches, double* mean_us, double* min_us, double* max_us) {
  if (!g_prof.on) return fail(HMC_ERR_ARG, "profiling not active");
  hmc_status st = HMC_OK;
  double sum = 0.0, mn = 0.0, mx = 0.0;
  if (g_prof.used > 0) {
    hipError_t e = hipEventSynchronize(g_prof.ev[2 * g_prof.used - 1]);
    if (e != hipSuccess) st = hip_status(e, "hipEventSynchronize");
    for (int i = 0; st == HMC_OK && i < g_prof.used; ++i) {
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]);
      if (e != hipSuccess) { st = hip_status(e, "hipEventElapsedTime"); break; }
      const double us = 1e3 * ms / g_prof.reps[i];
      sum += us;
      mn = i ? fmin(mn, us) : us;
      mx = i ? fmax(mx, us) : us;
    }
  }
  if (launches) *launches = g_prof.used;
  if (mean_us) *mean_us = g_prof.used ? sum / g_prof.used : 0.0;
  if (min_us) *min_us = mn;
  if (max_us) *max_us = mx;
  for (int i = 0; i < 2 * g_prof.cap; ++i) (void)hipEventDestroy(g_prof.ev[i]);
  delete[] g_prof.ev;
  delete[] g_prof.reps;
  g_prof.ev = nullptr;
  g_prof.reps = nullptr;
  g_prof.repeat = 1;
  g_prof.on = false;
  g_prof.cap = g_prof.used = 0;
  return st;
}

const char* hmc_status_string(hmc_status s) {
  switch (s) {
    case HMC_OK: return "ok";
    case HMC_ERR_ARG: return "invalid argument";
    case HMC_ERR_SHAPE: return "invalid shape";
    case HMC_ERR_DTYPE: return "invalid format";
    case HMC_ERR_HIP: return "HIP error";
    case HMC_ERR_WORKSPACE: return "invalid workspace";
    case HMC_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* hmc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
