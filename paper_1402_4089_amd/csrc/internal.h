// Internal declarations shared by the HIP translation units of libhmc (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hmcx {

constexpr int kTileRows = 16;      // rows of X per tile: the M dimension of a 16x16 MFMA
constexpr int kMaxFusedWG = 256;   // one workgroup per MI355X compute unit
constexpr int kEpiElems = 64;      // gradient elements per epilogue workgroup
constexpr int kUpdThreads = 256;   // elements per refresh / accept workgroup

// Arguments of the fused log-posterior + gradient pass over X.
struct FusedArgs {
  const void* X;        // n x p, row pitch ldx, element type T
  int64_t ldx;
  const int32_t* y;     // n labels
  const void* B;        // p x K row-major, T
  int64_t n;
  int32_t p, K;
  int64_t ntiles;       // ceil(n / 16)
  void* gpart;          // [gridDim.x][gstride] T: per-workgroup partial X^T (Y - P), p x K
  int64_t gstride;      // elements between consecutive partials (p*K rounded up to 64)
  double* lpart;        // [gridDim.x]: per-workgroup partial log-likelihood
  int32_t link;         // hmc_link: 0 multinomial logit, 1 Poisson (K = 1)
  int32_t pin;          // 1: column K-1 of B is read as zero (its logit is the constant 0)
};

// Arguments of the gradient epilogue (partial reduction, prior, mask, leapfrog kicks).
struct EpiArgs {
  const void* gpart;
  int64_t gstride;      // elements between consecutive partials (multiple of 64)
  int32_t nwg;          // partial count
  int32_t p, K;
  void* B;              // position at which the gradient was taken (drifted when mode 1)
  void* G;              // out: gradient
  void* eta;            // momentum (modes 1, 2)
  int32_t prior;
  double scale;
  int32_t pin;
  double h, eps;        // half step, full step
  int32_t mode;         // 0 gradient only; 1 kick, kick, drift; 2 final kick + kinetic energy
  double* ppart;        // [gridDim.x] prior log-density partials at B (before any drift)
  double* kpart;        // [gridDim.x] kinetic partials (mode 2)
  uint16_t* bpk;        // mode 1, float state: packed split-precision B operand the drifted
                        // position is written into (for the next pass), or null
  int32_t pack_nb;      // its 16-class blocks
};

// Start of a trajectory: optional momentum draw, then the opening half kick and drift.
struct StartArgs {
  int32_t p, K, pin;
  const void* B;        // current position
  const void* G;        // gradient at B
  void* Bp;             // out: drifted position
  void* eta;            // in/out momentum (drawn here when draw != 0)
  double h, eps;
  int32_t draw;         // 0: use eta as given; 1: replay normals; 2: Philox
  const double* normals;   // replay [n_rec][p][K]
  uint64_t seed;
  int32_t chain;
  int64_t iter;         // global iteration index (Philox counter word 1) when ctr is null
  int64_t t;            // record slot when ctr is null
  int64_t n_rec;        // record / replay capacity in iterations
  const int64_t* ctr;   // device {iteration, first iteration} (graph replay), or null
  double* k0part;       // [gridDim.x] initial kinetic partials (draw != 0)
  const double* logpost;   // current log K (copied to scal[0] by block 0 when draw != 0)
  double* scal;
};

// Metropolis test, state selection and recording.
struct AcceptArgs {
  int32_t p, K;
  void* B; void* G; double* logpost;
  const void* Bp; const void* Gp;
  const double* lpart; int32_t nl;
  const double* ppart; int32_t np;
  const double* k0part; int32_t nk0;   // initial kinetic partials (start kernel)
  const double* k1part; int32_t nk1;   // final kinetic partials (last epilogue)
  const double* scal;       // scal[0] = log K at the current state
  const double* replay_u;   // [n_rec] uniforms, or null for Philox
  const double* inv_temp;   // [n_rec] values 1/T, or null
  uint64_t seed; int32_t chain; int64_t iter;
  int64_t t, n_rec;         // record slot (when ctr is null) and record capacity
  const int64_t* ctr;       // device {iteration, first iteration}, or null
  void* sample;             // [n_rec][p][K] records, or null
  int32_t* accepted; double* H; int32_t* divergent;   // [n_rec] records, or null
};

// Arguments of the wide-p kernels (logits by column chunk, row softmax, column-owner
// gradient with the leapfrog epilogue).
struct WideArgs {
  const void* X;        // n x p, row pitch ldx
  int64_t ldx;
  const int32_t* y;
  void* B;              // position (drifted by wide_grad in mode 1)
  void* eta;            // momentum (modes 1, 2)
  void* G;              // out: gradient
  int64_t n;
  int32_t p, K;
  int32_t nchunk;       // column chunks of wide_logits
  void* zpart;          // [nchunk][n][16*NB] partial logits
  void* R;              // [n][16*NB] residuals
  double* lpart;        // [ceil(n/16)] log-likelihood partials
  double* ppart;        // [gradient workgroups] prior log-density partials
  double* kpart;        // [gradient workgroups] kinetic partials (mode 2)
  int32_t prior;
  double scale;
  int32_t pin;
  double h, eps;
  int32_t mode;         // as EpiArgs::mode
  int32_t nsplit;       // row slices of wide_grad (1: it applies the epilogue itself)
  int64_t tiles_per_split;  // 16-row tiles per slice (a multiple of 4)
  void* gpart;          // [nsplit][gstride] partial gradients when nsplit > 1
  int64_t gstride;
  int32_t link;         // hmc_link: 0 multinomial logit, 1 Poisson (K = 1)
};

// Arguments of the split-precision (bf16 hi + lo) pass.
constexpr int kHiloWaves = 4;      // waves per logits workgroup
constexpr int kHiloMB = 2;         // 16-row M blocks per logits wave
constexpr int kHiloRows = kHiloWaves * 16 * kHiloMB;   // rows per logits row block

// XCD-aware order of the split-precision gradient items (hilo.hip): the launch order is
// split into chunks of G consecutive items dealt round-robin to the kXcds XCDs; the launch
// covers xcd_span(items, G) positions. kGradChunk is G for the batched kernel (the column
// blocks of one row slice of a problem with p <= 2048).
constexpr int kXcds = 8;
constexpr int kGradChunk = 16;
constexpr int64_t xcd_span(int64_t total, int G) {
  return (total + (int64_t)kXcds * G - 1) / ((int64_t)kXcds * G) * kXcds * G;
}
struct HiloArgs {
  const uint16_t* Xhi;  // n x p bf16 planes, row pitch ldx (a multiple of 8)
  const uint16_t* Xlo;  // null for the hi-only form
  int64_t ldx;
  const int32_t* y;
  const void* B;        // p x K float32 position
  uint16_t* Bpk;        // packed B operand [ceil(p/32)][NB][2][64][8]
  uint16_t* Rpk;        // packed residual operand [row blocks of 32][NB][2][64][8]
  float* gpart;         // [nsplit][gstride] partial X^T R, p x K
  int64_t gstride;
  int32_t nsplit;       // row slices of the gradient kernel
  int64_t rows_per_split;   // a multiple of 32
  double* lpart;        // [logits workgroups] log-likelihood partials
  int64_t n;
  int32_t p, K;
  int32_t pin;          // 1: column K-1 of B is packed as zero
};

// One problem of a batch (device table entry). Each problem runs `chains` chains that
// share every pass over its X: their states are chain-major [chains][p][K] float32.
struct BatchProb {
  const uint16_t* Xhi;
  const uint16_t* Xlo;      // null for the hi-only form
  int64_t ldx;
  const int32_t* y;
  int64_t n;
  int32_t p, K;             // K <= 16 * group
  int32_t prior, pin;
  double scale, eps;
  float* B; float* G;       // caller's current state and the gradient there
  double* logpost;          // caller's [chains] log K at the current state
  float* eta; float* Bp; float* Gp;   // workspace: momentum, proposal, gradient at proposal
  uint16_t* Bpk; uint16_t* Rpk;
  float* gpart;             // [nsplit][chains][cstride]
  int64_t gstride, cstride; // cstride = p K rounded up to 64; gstride = chains * cstride
  int32_t nsplit, gcols;
  int64_t rps;              // rows per gradient slice (a multiple of 32)
  int32_t nrb;              // logits row blocks of kHiloRows rows
  double* lpart;            // [nrb][chains]
  int32_t ne;               // partial-sum slots per chain (64 elements each)
  int32_t ne4;              // epilogue items per chain (256 elements, four slots, each)
  double* ppart; double* k1part;      // [chains][ne]
  int32_t nu;               // start / accept items per chain (256 elements each)
  double* k0part;           // [chains][nu]
  double* scal;             // [chains] log K at the current state (trajectory start)
  int32_t chain0;           // global index of chain 0 (Philox stream, records)
  float* samples;           // [n_iter][chains][p][K] or null
  double* moments;          // [2][chains][p][K] running sum and sum of squares, or null
  const double* normals;    // replayed momenta [n_iter][chains][p][K], or null for Philox
  const double* uniforms;   // replayed accept uniforms [n_iter][chains], or null for Philox
};

// Launch-wide arguments of the batched kernels. first_X[b] is the first work item of
// problem b in kernel X's item list (nprob + 1 entries).
struct BatchArgs {
  const BatchProb* probs;
  int32_t nprob, chains, total_chains;
  int32_t group;            // 16-class blocks per chain (class block c * group + k / 16)
  const int32_t* first_pack; const int32_t* first_logits; const int32_t* first_grad;
  const int32_t* first_epi; const int32_t* first_upd;
  int64_t* ctr;             // ctr[0]: global iteration index; ctr[1]: first iteration of the run
  uint64_t seed;
  int32_t mode;             // epilogue mode (as EpiArgs::mode)
  int32_t at_current;       // 1: gradient at (B, G) (log-posterior call); 0: at (Bp, Gp)
  int64_t n_rec;            // record capacity in iterations (records beyond it are dropped)
  int32_t* accepted; double* H; int32_t* divergent;   // [n_rec][total_chains] or null
  const double* inv_temp;   // [n_rec] values 1/T of the annealed acceptance, or null
};

// Posterior-predictive classification over coefficient samples.
struct PredictArgs {
  const void* X;        // n x p, row pitch ldx, element type T
  int64_t ldx, n;
  int32_t p, K, pin;
  const void* samples;  // [n_samples][p][K] T
  int32_t n_samples;
  double* mean_prob;    // [n][K] or null
  int32_t* classes;     // [n] or null
};

struct FinalArgs {
  const double* lpart; int32_t nl;
  const double* ppart; int32_t np;
  double* logpost;
};

// Launchers (return hipSuccess or the launch error). T is float or double.
template <typename T>
hipError_t launch_fused(const FusedArgs& a, int nwg, int waves, int mb, int nb, size_t lds,
                        hipStream_t s);
template <typename T> hipError_t launch_epilogue(const EpiArgs& a, int nwg, hipStream_t s);
template <typename T> hipError_t launch_start(const StartArgs& a, int nwg, hipStream_t s);
template <typename T> hipError_t launch_accept(const AcceptArgs& a, int nwg, hipStream_t s);
hipError_t launch_final(const FinalArgs& a, hipStream_t s);

template <typename T> int wide_chunk_cols();
int wide_grad_groups(int64_t p, int nb, bool f64);
template <typename T>
hipError_t launch_wide(const WideArgs& a, int nb, int logits_tiles_y, int softmax_wg, int grad_wg,
                       hipStream_t s);

hipError_t launch_hilo(const HiloArgs& a, int nb, bool lo, int logits_wg, int grad_cols, bool pack, hipStream_t s);
template <typename Tin>
hipError_t launch_split(const Tin* X, int64_t ldx, int64_t n, int64_t p, uint16_t* hi, uint16_t* lo,
                        int64_t ldo, hipStream_t s);

hipError_t launch_batch_pass(const BatchArgs& a, int chains, int group, bool lo, const int grid[3], bool pack, hipStream_t s);
// grid: {start/accept, epilogue} workgroup counts
hipError_t launch_batch_start(const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_batch_epilogue(const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_batch_accept(const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_batch_final(const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_counter(int64_t* ctr, int64_t set_to, int op, hipStream_t s);   // op 0 set, 1 advance

size_t predict_lds_bytes(int64_t p, int K, bool f64);
template <typename T> hipError_t launch_predict(const PredictArgs& a, hipStream_t s);

hipError_t launch_stream_read(const void* buf, int64_t bytes, int reps, unsigned* sink, hipStream_t s);

// Does a fused variant exist for (waves, mb, nb, T)?
template <typename T> bool fused_variant_exists(int waves, int mb, int nb);

}  // namespace hmcx
