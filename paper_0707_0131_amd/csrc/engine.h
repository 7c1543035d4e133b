// Solver engine of the eigCG library: context, device workspaces, and the
// CG / eigCG / init-CG / Incremental eigCG drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <map>
#include <string>
#include <array>
#include <vector>

#include "common.h"
#include "eigcg.h"
#include "kernels.h"

namespace eigcg {

using cplx = std::complex<double>;

struct HipError {
  hipError_t e;
  const char* what;
};
struct ApiError {
  int code;
  std::string msg;
};

// Device vectors of one batched solve (K columns, one precision).
struct Workspace {
  int K = 0;
  int Keig = 0;          // columns of the eigCG window arrays
  int prec = kF64;
  bool eig = false;
  int ring_len = 0;
  int nev = 0;
  void* b = nullptr;
  void* x = nullptr;
  void* r = nullptr;
  void* p = nullptr;
  void* tmp = nullptr;
  void* ring = nullptr;  // K * ring_len window residuals
  void* vr = nullptr;    // K * 2nev restarted window block
  void* tbuf = nullptr;  // K * 2 saved A p
  void* w = nullptr;     // K arrow-row vectors
  void* ritz = nullptr;  // K * nev Ritz vectors
  void* z = nullptr;     // K preconditioned residuals z = P^{-1} r (spectral preconditioner)
};

struct Ctx {
  eigcg_params P{};
  Geom g{};
  size_t cs = 0;         // complex elements per field (12 * vs)
  hipStream_t stream = nullptr;
  hipStream_t gstream = nullptr;  // capture-only stream for HIP graphs
  // captured CG segments (params.use_graphs), kept across solves; the key
  // holds what the captured kernels' arguments depend on beyond the context's
  // fixed buffers: iterations, precision, width, mask, eigCG and
  // preconditioner state and the workspace fields
  std::map<std::array<uint64_t, 14>, hipGraphExec_t> graphs;
  int device = 0;
  int comp64 = 0, comp32 = 0;
  int iprec = kF32;                // inner precision of mixed contexts (kF32 or kF16)
  int var64 = 1, var32 = 1;        // stencil kernel variants in use (var32: inner precision)
  int nc64 = 0, nc32 = 0;          // their columns per workgroup (0 = widest)
  double tune_ms[2 * kStencilVariants] = {};  // FP64 then FP32, per variant
  void* u64 = nullptr;
  void* u32 = nullptr;
  void* eo_tmp64 = nullptr;        // odd-even: odd-site intermediates (max_batch fields,
  size_t eo_cols64 = 0;            // or more for the batched init-CG guesses: eo_cols64)
  void* eo_tmp32 = nullptr;
  // bank (Section 4): U columns, H = U^H A U and its Cholesky factor
  int bank_prec = kF64;
  void* U = nullptr;
  void* bwork = nullptr;  // 2 nev fields: W = A Vbar and a temporary
  void* bwork64 = nullptr;  // FP32 banks: 2 FP64 fields for A v in FP64
  int l = 0;
  std::vector<cplx> H;    // max_bank x max_bank, ld = max_bank
  std::vector<cplx> L;    // Cholesky factor of H(0:l, 0:l)
  bool chol_ok = false;
  double amax = 0.0;      // largest Ritz value seen (norm of A estimate)
  int nlock = 0;          // leading columns of U locked out of building H (Section 4)
  uint64_t bank_gen = 0;  // bumped whenever U or H changes
  // Ritz values of the bank and their residual norms ||A u - theta u|| for the
  // dynamic init-CG restart threshold, valid while rm_gen == bank_gen
  uint64_t rm_gen = ~0ull;
  std::vector<double> rm_theta, rm_res;
  // spectral preconditioner P^{-1} = I + U_R D U_R^H (params.precond): the
  // bank in its Ritz basis, D = sigma / theta - 1, device staging of U_R^H r,
  // D U_R^H r and r^H U_R D U_R^H r per column
  void* UR = nullptr;
  int lR = 0;             // columns of U_R (0: P = I)
  bool spec_ok = false;   // U_R, D built for the current bank
  double spec_sigma = 0.0;
  double* d_specD = nullptr;
  double2* d_specG = nullptr;
  double2* d_specS = nullptr;
  double* d_specs = nullptr;
  void* bs = nullptr;      // BiCGSTAB on M or gamma5 M: eight FP64 work fields
  // scratch
  ColState* d_st = nullptr;
  ColState* h_st = nullptr;        // pinned: 2 x kMaxCols polls, kMaxCols upload slots
  double* d_hist = nullptr;
  double* h_hist = nullptr;        // pinned mirror
  int hist_stride = 0;             // doubles per column
  double* d_partial = nullptr;
  unsigned int* d_counter = nullptr;
  double2* d_gpart = nullptr;
  size_t gpart_elems = 0;
  double2* d_small = nullptr;      // small matrices (S, G) for GEMMs
  double2* h_small = nullptr;      // pinned mirror
  size_t small_elems = 0;
  double* d_norm = nullptr;        // kMaxCols norms
  double* h_norm = nullptr;
  Workspace ws64, ws32;
  Workspace wsg;                   // FP64 init-CG guesses of several right-hand sides at once
  size_t bytes = 0;
  std::string err;
  int sticky = 0;
  std::vector<double> last_ritz;
  std::map<int, double> iter_ms;   // measured CG iteration time per (precision, width)
  std::vector<hipEvent_t> events;
  // sampled stencil timings: events around the two passes of every
  // P.sample_every-th iteration, harvested when the pool is full or on request
  struct KSample {
    hipEvent_t e[4];  // start / end of pass 1, start / end of pass 2
    int prec;
    int ncols;
  };
  std::vector<KSample> ks_pool;
  int ks_used = 0;
  long ks_tick = 0;
  // harvested samples per precision: (pass 1 ms, pass 2 ms, columns)
  std::vector<std::array<float, 3>> ks_done[2];
  bool ks_harvest(bool wait);

  // memory
  void* dalloc(size_t bytes_);
  void dfree(void*& p);
  void check(hipError_t e, const char* what);
};

// Engine entry points (throw HipError / ApiError; the ABI layer converts).
void ctx_init(Ctx& c, const eigcg_params& p, const void* gauge_dev, hipStream_t s);
void ctx_release(Ctx& c);
void apply_op(Ctx& c, int op, int nrhs, const void* in_aos, void* out_aos);
// as apply_op for M, M^H, A in FP64, through a static device scratch array
// (no allocation); noalloc_scratch_bytes() is the array's size
void apply_op_noalloc(Ctx& c, int op, int nrhs, const void* in_aos, void* out_aos);
size_t noalloc_scratch_bytes();
void schur_rhs(Ctx& c, int nrhs, const void* b_full, void* rhs);
void schur_reconstruct(Ctx& c, int nrhs, const void* b_full, const void* x_even, void* x_full);
int solve(Ctx& c, int nrhs, const void* b_aos, void* x_aos, double tol, int mode,
          eigcg_stats* stats);
void deflate_init(Ctx& c, int nrhs, const void* b_aos, void* x_aos);
// Dynamic init-CG restart threshold from ascending Ritz values and their
// residual norms (host only): tau = 0 means no restart.
struct RestartPick {
  double tau, cost_none, cost_with;
};
RestartPick restart_model(int l, const double* theta, const double* res, double lam_max,
                          double tol, double restart_cost);
void bank_info(Ctx& c, int* l, double* vals, double* res);
int bank_lock(Ctx& c, double tol);
void bank_vectors(Ctx& c, int first, int count, void* out_aos);
int bank_load(Ctx& c, int count, const void* vecs_aos);
void bank_truncate(Ctx& c, int k);
void bank_restore(Ctx& c, int l, const void* vecs_aos, const double* h_host);
int solve_bicgstab(Ctx& c, int nrhs, const void* b_aos, void* x_aos, double tol, int flags,
                   int max_iter, eigcg_bicgstab_stats* stats);
double bench_kernels(Ctx& c, int what, int reps);
bool auto_continue(int done, int left, const double* iters, const double* secs, double iter_ms,
                   int bank_room);
void kernel_samples(Ctx& c, bool reset, double* out);
// device bytes an eigCG run of keig columns would still allocate for its window
size_t eig_window_bytes(const Ctx& c, int keig);
// drop this process's stencil tuning choices (the persisted file stays)
void tune_cache_reset();

// Engine helpers shared by the solver files (engine.cpp, bicgstab.cpp).
// Host-side bounds layer over the library's device allocations: every
// allocation is registered with its size, column pointers and the fields a
// launch touches are checked against it (ApiError EINVAL when they would
// reach past the end).
void register_span(const void* base, size_t bytes);
size_t unregister_span(const void* base);  // returns the registered size (0: unknown)
bool span_fits(const void* p, size_t bytes);
void check_span(const void* p, size_t bytes, const char* what);
void check_fields(const Ctx& c, const void* p, int prec, int ncols, const char* what);
void* col_ptr(void* base, int prec, size_t cs, size_t idx);
// out = op(in) (op = kOpM or kOpMdag) on ncols internal fields
void stencil_store(Ctx& c, int prec, int op, int ncols, const void* in, void* out);
// init-CG deflation of the masked columns, eq. (2.1): x += U H^{-1} U^H r with
// r = b - A x given (storage precision prec = the bank's)
void deflate_columns(Ctx& c, int prec, int ncols, uint32_t mask, void* x, const void* r);

// Serving sessions (continuous batching over max_batch slots of one context).
struct Session;
struct SessionDone {
  uint64_t tag;
  int status;
  int iters;
  int outer;
  int first_leg;  // iterations before the first init-CG restart (= iters when none)
  double restart_tau;  // the FP64 init-CG restart threshold it was given (0: none)
  double true_rel_res;
};
Session* session_open(Ctx& c);
int session_free_slot(Session* s);
int session_active(Session* s);
int session_admit(Session* s, const void* b_aos, void* x_aos, double tol, uint64_t tag,
                  std::vector<SessionDone>& done);
void session_step(Session* s, std::vector<SessionDone>& done);
void session_close(Session* s);

}  // namespace eigcg

// The opaque handle of the C ABI.
struct eigcg_ctx {
  eigcg::Ctx c;
};
