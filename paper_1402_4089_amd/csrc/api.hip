// C-ABI entry points of libhmc: argument checks, workspace layout and launch sequences.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "hmc.h"
#include "internal.h"

using namespace hmcx;

namespace {

thread_local std::string g_last_error;

// Event pool for hmc_profile_begin / hmc_profile_end.
struct Profiler {
  bool on = false;
  int cap = 0, used = 0;
  hipEvent_t* ev = nullptr;   // 2 * cap events
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
  int nchunk, tiles_y, nsoft, ngrad;
  bool hilo, lo;        // bf16 split-precision form (lo: the low plane is present)
  int hl_logits_wg, hl_cols, hl_nsplit;
  int64_t hl_rps;       // rows per gradient slice
  size_t off_bpk, off_rpk;
  int nl, np;           // log-likelihood / prior (and kinetic) partial counts
  size_t off_zpart, off_R;
  size_t off_gpart, off_lpart, off_ppart, off_k0, off_k1, off_eta, off_bp, off_gp, off_scal, total;
};

int class_blocks(int K) { return K <= 16 ? 1 : K <= 32 ? 2 : 4; }

// LDS of the fused pass: two 16-row tile buffers of waves*mb*16 padded columns, plus the
// cross-wave logits and residual exchanges.
size_t lds_bytes(int waves, int mb, int nb, size_t ts) {
  return (size_t)2 * kTileRows * (waves * mb * 16) * ts + (size_t)(waves + 1) * nb * 256 * ts + 64;
}

// Pick the fused-kernel variant: the smallest column-block count covering p.
bool pick_variant(bool f64, int nblk, int nb, int* waves, int* mb) {
  const int w = 8;
  const int need = (nblk + w - 1) / w;
  int m = 1;
  while (m < need) m <<= 1;
  const bool ok = f64 ? fused_variant_exists<double>(w, m, nb) : fused_variant_exists<float>(w, m, nb);
  if (!ok || lds_bytes(w, m, nb, f64 ? 8 : 4) > kLdsLimit) return false;
  *waves = w;
  *mb = m;
  return true;
}

bool is_bf16(int32_t xfmt) { return xfmt == HMC_X_BF16_HILO || xfmt == HMC_X_BF16; }

hmc_status check_problem(const hmc_problem* pr) {
  if (!pr) return fail(HMC_ERR_ARG, "problem descriptor is NULL");
  if (pr->xfmt != HMC_X_F64 && pr->xfmt != HMC_X_F32 && !is_bf16(pr->xfmt))
    return fail(HMC_ERR_DTYPE, "unsupported X format %d", pr->xfmt);
  if (pr->prior != HMC_PRIOR_GAUSS && pr->prior != HMC_PRIOR_CAUCHY)
    return fail(HMC_ERR_DTYPE, "unknown prior %d", pr->prior);
  if (pr->n < 1) return fail(HMC_ERR_SHAPE, "n = %lld must be >= 1", (long long)pr->n);
  if (pr->p < 1) return fail(HMC_ERR_SHAPE, "p = %lld must be >= 1", (long long)pr->p);
  if (pr->K < 2 || pr->K > 64) return fail(HMC_ERR_SHAPE, "K = %d must be in [2, 64]", pr->K);
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
  L->wide = !L->hilo && !pick_variant(L->f64, L->nblk, L->nb, &L->waves, &L->mb);
  if (!L->wide && !L->hilo) L->lds = lds_bytes(L->waves, L->mb, L->nb, L->ts);
  L->ntiles = (pr->n + kTileRows - 1) / kTileRows;
  L->nwg = (int)(L->ntiles < kMaxFusedWG ? L->ntiles : kMaxFusedWG);
  const int64_t pk = pr->p * (int64_t)pr->K;
  L->nepi = (int)((pk + kEpiElems - 1) / kEpiElems);
  L->nupd = (int)((pk + kUpdThreads - 1) / kUpdThreads);
  const int KP = 16 * L->nb;
  L->hl_logits_wg = L->hl_cols = L->hl_nsplit = 0;
  L->hl_rps = 0;
  if (L->hilo) {
    // logits: row blocks of kHiloWaves * 32 rows; gradient: 128-column blocks times row
    // slices, about 2048 workgroups in all
    const int64_t rows = kHiloWaves * 32;
    const int64_t nrb = (pr->n + rows - 1) / rows;
    L->hl_logits_wg = (int)(nrb < 2048 ? nrb : 2048);
    L->hl_cols = (int)((pr->p + 127) / 128);
    int64_t want = (2048 + L->hl_cols - 1) / L->hl_cols;
    const int64_t n32 = (pr->n + 31) / 32;
    want = want < 1 ? 1 : want > 256 ? 256 : want;
    if (want > n32) want = n32;
    L->hl_rps = ((pr->n + want - 1) / want + 31) / 32 * 32;
    L->hl_nsplit = (int)((pr->n + L->hl_rps - 1) / L->hl_rps);
    L->nchunk = L->tiles_y = L->nsoft = L->ngrad = 0;
    L->nwg = L->hl_nsplit;
    L->nl = L->hl_logits_wg;
    L->np = L->nepi;
    L->gstride = (pk + 63) / 64 * 64;
  } else if (L->wide) {
    const int cw = L->f64 ? wide_chunk_cols<double>() : wide_chunk_cols<float>();
    L->nchunk = (int)((pr->p + cw - 1) / cw);
    L->tiles_y = (int)(L->ntiles < 16 ? L->ntiles : 16);
    L->nsoft = (int)((pr->n + 15) / 16);
    L->ngrad = (int)((pr->p + wide_grad_cols() - 1) / wide_grad_cols());
    L->nl = L->nsoft;
    L->np = L->ngrad;
    L->gstride = 0;
  } else {
    L->nchunk = L->tiles_y = L->nsoft = L->ngrad = 0;
    L->nl = L->nwg;
    L->np = L->nepi;
    L->gstride = (pk + 63) / 64 * 64;
  }
  size_t off = 0;
  L->off_gpart = off; off = align_up(off + (size_t)L->nwg * L->gstride * L->ts);
  L->off_zpart = off; off = align_up(off + (L->wide ? (size_t)L->nchunk * pr->n * KP * L->ts : 0));
  L->off_R = off;     off = align_up(off + (L->wide ? (size_t)pr->n * KP * L->ts : 0));
  {
    const size_t frag = 2 * 512 * sizeof(uint16_t);   // one hi/lo pair of 64-lane fragments
    const int64_t rows = kHiloWaves * 32;
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

// One gradient evaluation at Bpos: fused pass, then the epilogue in `mode`.
template <typename T>
hmc_status gradient_step(const hmc_problem* pr, const Layout& L, const void* Bpos, void* G,
                         void* eta, int mode, double eps, void* ws, hipStream_t s) {
  if (L.hilo) {
    HiloArgs h{};
    h.Xhi = static_cast<const uint16_t*>(pr->X);
    h.Xlo = static_cast<const uint16_t*>(pr->X_lo);
    h.ldx = pr->ldx; h.y = pr->y; h.B = Bpos;
    h.Bpk = at<uint16_t>(ws, L.off_bpk); h.Rpk = at<uint16_t>(ws, L.off_rpk);
    h.gpart = at<float>(ws, L.off_gpart); h.gstride = L.gstride;
    h.nsplit = L.hl_nsplit; h.rows_per_split = L.hl_rps;
    h.lpart = at<double>(ws, L.off_lpart);
    h.n = pr->n; h.p = (int32_t)pr->p; h.K = pr->K;
    const bool timed = g_prof.on && g_prof.used < g_prof.cap;
    if (timed) HMC_TRY(hip_status(hipEventRecord(g_prof.ev[2 * g_prof.used], s), "profile event"));
    HMC_TRY(hip_status(launch_hilo(h, L.nb, L.lo, L.hl_logits_wg, L.hl_cols, s), "split-precision pass"));
    if (timed) {
      HMC_TRY(hip_status(hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s), "profile event"));
      ++g_prof.used;
    }
    EpiArgs e;
    e.gpart = h.gpart; e.gstride = L.gstride; e.nwg = L.hl_nsplit; e.p = (int32_t)pr->p; e.K = pr->K;
    e.B = const_cast<void*>(Bpos); e.G = G; e.eta = eta;
    e.prior = pr->prior; e.scale = pr->prior_scale; e.pin = pr->pin_last_class;
    e.h = 0.5 * eps; e.eps = eps; e.mode = mode;
    e.ppart = at<double>(ws, L.off_ppart);
    e.kpart = at<double>(ws, L.off_k1);
    return hip_status(launch_epilogue<T>(e, L.nepi, s), "gradient epilogue");
  }
  if (L.wide) {
    WideArgs w{};
    w.X = pr->X; w.ldx = pr->ldx; w.y = pr->y; w.B = const_cast<void*>(Bpos); w.eta = eta; w.G = G;
    w.n = pr->n; w.p = (int32_t)pr->p; w.K = pr->K; w.nchunk = L.nchunk;
    w.zpart = at<void>(ws, L.off_zpart); w.R = at<void>(ws, L.off_R);
    w.lpart = at<double>(ws, L.off_lpart); w.ppart = at<double>(ws, L.off_ppart);
    w.kpart = at<double>(ws, L.off_k1);
    w.prior = pr->prior; w.scale = pr->prior_scale; w.pin = pr->pin_last_class;
    w.h = 0.5 * eps; w.eps = eps; w.mode = mode;
    const bool timed = g_prof.on && g_prof.used < g_prof.cap;
    if (timed) HMC_TRY(hip_status(hipEventRecord(g_prof.ev[2 * g_prof.used], s), "profile event"));
    HMC_TRY(hip_status(launch_wide<T>(w, L.nb, L.tiles_y, L.nsoft, L.ngrad, s), "wide pass"));
    if (timed) {
      HMC_TRY(hip_status(hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s), "profile event"));
      ++g_prof.used;
    }
    return HMC_OK;
  }
  FusedArgs f;
  f.X = pr->X; f.ldx = pr->ldx; f.y = pr->y; f.B = Bpos;
  f.n = pr->n; f.p = (int32_t)pr->p; f.K = pr->K;
  f.ntiles = L.ntiles;
  f.gpart = at<void>(ws, L.off_gpart);
  f.gstride = L.gstride;
  f.lpart = at<double>(ws, L.off_lpart);
  const bool timed = g_prof.on && g_prof.used < g_prof.cap;
  if (timed) HMC_TRY(hip_status(hipEventRecord(g_prof.ev[2 * g_prof.used], s), "profile event"));
  HMC_TRY(hip_status(launch_fused<T>(f, L.nwg, L.waves, L.mb, L.nb, L.lds, s), "fused pass"));
  if (timed) {
    HMC_TRY(hip_status(hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s), "profile event"));
    ++g_prof.used;
  }
  EpiArgs e;
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
    HMC_TRY(gradient_step<T>(pr, L, B, G, eta, st < L_steps ? 1 : 2, eps, ws, s));
  FinalArgs fa{at<double>(ws, L.off_lpart), L.nl, at<double>(ws, L.off_ppart), L.np, logpost};
  return hip_status(launch_final(fa, s), "log-posterior final sum");
}

template <typename T>
hmc_status do_sample(const hmc_problem* pr, const Layout& L, void* B, void* G, double* logpost,
                     const hmc_sample_args* ar, void* ws, hipStream_t s) {
  const int64_t pk = pr->p * (int64_t)pr->K;
  void* eta = at<void>(ws, L.off_eta);
  void* Bp = at<void>(ws, L.off_bp);
  void* Gp = at<void>(ws, L.off_gp);
  double* scal = at<double>(ws, L.off_scal);
  for (int t = 0; t < ar->n_iter; ++t) {
    const int64_t it = (int64_t)ar->first_iter + t;
    StartArgs sa{};
    sa.p = (int32_t)pr->p; sa.K = pr->K; sa.pin = pr->pin_last_class;
    sa.B = B; sa.G = G; sa.Bp = Bp; sa.eta = eta; sa.h = 0.5 * ar->eps; sa.eps = ar->eps;
    sa.draw = ar->replay_normals ? 1 : 2;
    sa.normals = ar->replay_normals ? ar->replay_normals + (int64_t)t * pk : nullptr;
    sa.seed = ar->seed; sa.chain = ar->chain; sa.iter = it;
    sa.k0part = at<double>(ws, L.off_k0); sa.logpost = logpost; sa.scal = scal;
    HMC_TRY(hip_status(launch_start<T>(sa, L.nupd, s), "trajectory start"));
    for (int st = 1; st <= ar->L; ++st)
      HMC_TRY(gradient_step<T>(pr, L, Bp, Gp, eta, st < ar->L ? 1 : 2, ar->eps, ws, s));
    AcceptArgs aa{};
    aa.p = (int32_t)pr->p; aa.K = pr->K; aa.B = B; aa.G = G; aa.logpost = logpost;
    aa.Bp = Bp; aa.Gp = Gp;
    aa.lpart = at<double>(ws, L.off_lpart); aa.nl = L.nl;
    aa.ppart = at<double>(ws, L.off_ppart); aa.np = L.np;
    aa.k0part = at<double>(ws, L.off_k0); aa.nk0 = L.nupd;
    aa.k1part = at<double>(ws, L.off_k1); aa.nk1 = L.np;
    aa.scal = scal;
    aa.replay_u = ar->replay_uniforms ? ar->replay_uniforms + t : nullptr;
    aa.inv_temp = ar->inv_temperature ? ar->inv_temperature + t : nullptr;
    aa.seed = ar->seed; aa.chain = ar->chain; aa.iter = it;
    aa.sample = ar->samples ? static_cast<char*>(ar->samples) + (size_t)t * pk * L.ts : nullptr;
    aa.accepted = ar->accepted ? ar->accepted + t : nullptr;
    aa.H = ar->H ? ar->H + 2 * (int64_t)t : nullptr;
    aa.divergent = ar->divergent ? ar->divergent + t : nullptr;
    HMC_TRY(hip_status(launch_accept<T>(aa, L.nupd, s), "accept"));
  }
  return HMC_OK;
}

}  // namespace

extern "C" {

int64_t hmc_max_p(int32_t xfmt, int32_t K) {
  if (xfmt != HMC_X_F64 && xfmt != HMC_X_F32 && !is_bf16(xfmt)) return 0;
  if (K < 2 || K > 64) return 0;
  const bool f64 = xfmt == HMC_X_F64;
  const int nb = class_blocks(K);
  (void)f64;
  (void)nb;
  // row-tile kernel up to its padded width; beyond it the wide-p kernels, bounded by
  // 32-bit element indexing of the p x K state
  return ((int64_t)1 << 30) / K;
}

hmc_status hmc_workspace_bytes(const hmc_problem* prob, size_t* bytes) {
  if (!bytes) return fail(HMC_ERR_ARG, "bytes is NULL");
  Layout L;
  HMC_TRY(make_layout(prob, &L));
  *bytes = L.total;
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
  if (!args) return fail(HMC_ERR_ARG, "args is NULL");
  if (!B || !G || !logpost) return fail(HMC_ERR_ARG, "B, G and logpost must be device pointers");
  if (!isfinite(args->eps) || args->eps == 0.0) return fail(HMC_ERR_ARG, "eps must be finite and non-zero");
  if (args->L < 1) return fail(HMC_ERR_ARG, "L = %d must be >= 1", args->L);
  if (args->n_iter < 1) return fail(HMC_ERR_ARG, "n_iter = %d must be >= 1", args->n_iter);
  if (args->first_iter < 0 || args->chain < 0) return fail(HMC_ERR_ARG, "first_iter and chain must be >= 0");
  if ((args->replay_normals == nullptr) != (args->replay_uniforms == nullptr))
    return fail(HMC_ERR_ARG, "replay_normals and replay_uniforms must both be set or both NULL");
  HMC_TRY(check_ws(L, ws, ws_bytes));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return L.f64 ? do_sample<double>(prob, L, B, G, logpost, args, ws, s)
               : do_sample<float>(prob, L, B, G, logpost, args, ws, s);
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

hmc_status hmc_profile_begin(int32_t capacity) {
  if (g_prof.on) return fail(HMC_ERR_ARG, "profiling already active");
  if (capacity < 1 || capacity > (1 << 20)) return fail(HMC_ERR_ARG, "capacity out of range");
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
      const double us = 1e3 * ms;
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
  g_prof.ev = nullptr;
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
