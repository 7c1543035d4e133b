/* eigCG on MI355X: C ABI of the HIP library libeigcg.so.
 *
 * Method: A. Stathopoulos and K. Orginos, "Computing and deflating eigenvalues
 * while solving multiple right hand side linear systems with an application
 * to Quantum Chromodynamics" (arXiv:0707.0131).
 *
 * The library solves A x = b with A = M^H M, where M is the Wilson-Dirac
 * operator on a periodic 4D lattice with SU(3) links (Section 1 of the paper:
 * M = m_q I - D is gamma5-Hermitian and CG runs on the normal equations):
 *
 *   (M psi)(x) = (4 + m_q) psi(x)
 *     - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *
 * with Euclidean chiral gamma matrices g_k = [[0, -i s_k], [i s_k, 0]]
 * (k = x, y, z; s_k Pauli), g_t = [[0, I], [I, 0]], gamma5 = diag(1,1,-1,-1).
 *
 * Three solve modes follow the paper:
 *   EIGCG_MODE_CG      plain CG (Figure 3.1, left box);
 *   EIGCG_MODE_EIGCG   one step of Incremental eigCG (Section 4): init-CG
 *                      guess from the current bank U (eq. (2.1)), eigCG(nev, m)
 *                      (Figure 3.1), then the nev Ritz vectors are
 *                      orthonormalised against U and appended, H = U^H A U
 *                      grows by nev rows and columns;
 *   EIGCG_MODE_INITCG  init-CG (eq. (2.1)) with the bank, restarted once near
 *                      machine precision (Section 5.3);
 *   EIGCG_MODE_AUTO    the nrhs right-hand sides of the call are one sequence:
 *                      Incremental eigCG while it pays, then init-CG for the
 *                      rest (Section 5.5: the best number of eigCG solves grows
 *                      with the number of right-hand sides; chosen at run time
 *                      from measured iterations and times, see
 *                      eigcg_host_auto_continue).  Init-CG only with 16-bit
 *                      inner solves.
 *
 * Odd-even preconditioning (params.schur = 1; the operator of the paper's
 * lattice runs, compared in Section 3.1 and used in the QCD tests of Section
 * 5.1, which halves the system): sites split by the
 * parity of x + y + z + t, D couples opposite parities only, and with
 * d = 4 + m_q the context's operator becomes A = Mhat^H Mhat on the even
 * sites, where Mhat = d - D_eo D_oe / (4 d) is the Schur complement of the
 * odd block of M.  Solving M x = b: eigcg_schur_rhs gives the right-hand side
 * Mhat^H (b_e + D_eo b_o / (2 d)), eigcg_solve returns x_e, and
 * eigcg_schur_reconstruct adds x_o = (b_o + D_oe x_e / 2) / d.
 *
 * Boundary layout (always FP64, owned by the caller, device pointers):
 *   spinor fields: complex128 [nrhs][Lt][Lz][Ly][Lx][4 spin][3 colour]; in an
 *                  odd-even context the solver's fields (b, x, bank vectors,
 *                  eigcg_apply) are [nrhs][V/2 even sites][4][3], the even
 *                  sites in lexicographic order (site s is entry s / 2)
 *   gauge field:   complex128 [Lt][Lz][Ly][Lx][4 mu][3][3], U_mu(x)[a][b] row-major,
 *                  mu = 0..3 is x, y, z, t.
 * Internal precision (EIGCG_FP64 or EIGCG_MIXED_FP32) never changes the
 * boundary layout.  All device work is enqueued on the stream given at create
 * time; calls return when their results are final unless stated otherwise.
 *
 * Errors are negative return codes; eigcg_last_error() gives a message.
 * EIGCG_EHIP is sticky: after it only eigcg_destroy is valid.  A context is
 * not thread-safe; distinct contexts may be used from distinct threads.
 */
#ifndef EIGCG_H
#define EIGCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eigcg_ctx eigcg_ctx;

enum {
  EIGCG_OK = 0,
  EIGCG_EINVAL = -1,      /* bad argument (dims, nev/m, NaN/Inf in b, ...) */
  EIGCG_ENOMEM = -2,      /* HBM budget exceeded or hipMalloc failed */
  EIGCG_ENOTCONV = -3,    /* max_iter reached; x holds the last iterate */
  EIGCG_EBREAKDOWN = -4,  /* p^H A p <= 0 or non-finite scalars */
  EIGCG_EHIP = -5,        /* HIP runtime failure (sticky) */
  EIGCG_EBUSY = -6        /* serving: ticket not finished yet */
};

enum { EIGCG_FP64 = 0, EIGCG_MIXED_FP32 = 1, EIGCG_MIXED_HALF = 2 };
enum { EIGCG_MODE_CG = 0, EIGCG_MODE_EIGCG = 1, EIGCG_MODE_INITCG = 2, EIGCG_MODE_AUTO = 3 };
enum { EIGCG_OP_M = 0, EIGCG_OP_MDAG = 1, EIGCG_OP_A = 2, EIGCG_OP_INNER = 3 };
enum { EIGCG_PRECOND_NONE = 0, EIGCG_PRECOND_SPECTRAL = 1 };
enum { EIGCG_RESTART_FIXED = 0, EIGCG_RESTART_DYNAMIC = 1 };

typedef struct {
  int32_t dims[4];        /* Lx, Ly, Lz, Lt; each >= 2, periodic */
  double mass;            /* m_q */
  int32_t nev, m;         /* eigCG(nev, m); requires m > 2 nev >= 2 (Figure 3.1) */
  int32_t max_bank;       /* most columns of U (<= 256) */
  int32_t precision;      /* EIGCG_FP64; EIGCG_MIXED_FP32 (FP32 iterations, FP64
                             reliable updates in CG and eigCG modes, FP64
                             refinement in init-CG mode); EIGCG_MIXED_HALF
                             (16-bit links and vectors with FP32 arithmetic and
                             an FP32 iterate, each inner solve rescaled, FP64
                             refinement; CG and init-CG modes only; needs
                             compress_links and SU(3) links, else EINVAL) */
  int32_t max_batch;      /* right-hand sides per batched launch, 1..12 */
  int32_t reliable_every; /* mixed precision: FP64 reliable update period */
  int32_t max_iter;       /* per right-hand side */
  double restart_tol;     /* init-CG restart threshold on ||r||/||b||:
                             0 -> 10 u ||A|| with u = 2^-24, single precision as
                             in the paper's runs (Sections 5.1, 5.3; ||A|| = the
                             largest Ritz value seen), < 0 -> never */
  uint64_t hbm_budget;    /* bytes this context may allocate, 0 = no cap */
  int32_t compress_links; /* 1: store links as two rows when they are SU(3) */
  int32_t check_every;    /* iterations between host convergence polls */
  int32_t use_graphs;     /* 1: segments of CG iterations (stencil passes,
                             finalize and update kernels) are replayed from HIP
                             graphs captured once per context and segment shape;
                             iterations that sample_every times run on their own */
  int32_t stencil_variant;/* 0: pick the fastest stencil kernel by timing at create
                             (cached per lattice shape and precision in the process);
                             1..15: force a variant (see eigcg_layout_info) */
  int32_t plane_pad;      /* extra sites (in units of 64) after each SoA plane so
                             that planes do not start on the same memory channel:
                             0 = library default, < 0 = none */
  int32_t sample_every;   /* > 0: time the two stencil passes of every n-th CG
                             iteration with events on the context's stream
                             (read with eigcg_kernel_samples); 0 = off */
  int32_t schur;          /* 1: odd-even preconditioned operator on the even
                             sites (every extent even); 0: A = M^H M */
  int32_t precond;        /* EIGCG_PRECOND_NONE, or EIGCG_PRECOND_SPECTRAL: CG and
                             eigCG iterations use z = P^{-1} r with the bank as a
                             spectral preconditioner (Section 2.1's alternative to
                             init-CG; Section 4's example), P^{-1} = I + U_R
                             (sigma Theta^{-1} - I) U_R^H with U_R, Theta the bank's
                             Ritz vectors and values (U_R^H A U_R = Theta), rebuilt
                             when the bank changes; eigCG then runs in the
                             preconditioned form of Section 3 (window V = P^{-1} R,
                             Ritz pairs of the pencil A y = lambda P y).  Costs two
                             passes over U per iteration.  FP64 contexts only
                             (EINVAL otherwise); an empty bank means P = I */
  double precond_sigma;   /* sigma of the spectral preconditioner (the value the
                             Ritz directions are mapped to); <= 0: the largest
                             Ritz value seen, else (8 + |m_q|)^2 */
  int32_t restart_rule;   /* EIGCG_RESTART_FIXED: the init-CG restart threshold is
                             restart_tol as above; EIGCG_RESTART_DYNAMIC: FP64
                             init-CG chooses it per solve from the bank's Ritz
                             values and residual norms (the open choice at the end
                             of Section 5.3) with the cost model of
                             eigcg_restart_model, lambda_max the largest Ritz value
                             seen (else (8 + |m|)^2); the inputs are recomputed
                             after the bank changes (l applications of A);
                             restart_tol < 0 still disables the restart */
  double restart_cost;    /* iterations the dynamic rule charges for one restart;
                             <= 0: the library's estimate from algorithmic bytes
                             (an application of A plus two passes over the l bank
                             vectors, against one FP64 CG iteration) */
} eigcg_params;

typedef struct {
  int32_t iters;          /* CG iterations (inner iterations in mixed mode) */
  int32_t restarts;       /* eigCG window restarts */
  int32_t outer_steps;    /* init-CG restarts / reliable updates / refinements */
  int32_t status;         /* EIGCG_OK, EIGCG_ENOTCONV or EIGCG_EBREAKDOWN */
  double true_rel_res;    /* ||b - A x|| / ||b|| recomputed in FP64 */
  double seconds;         /* wall time of this right-hand side's batch */
  int32_t bank_added;     /* vectors appended to U (EIGCG mode) */
  int32_t nritz;          /* Ritz pairs produced by eigCG (EIGCG mode) */
  int32_t mode_used;      /* mode this right-hand side was solved in (EIGCG_MODE_AUTO
                             resolves to EIGCG or INITCG) */
  int32_t first_leg_iters;/* FP64 init-CG: iterations completed when the restart of
                             Section 5.3 re-deflated the iterate (= iters when it did
                             not restart); other schemes: iters */
  double restart_tau;     /* FP64 init-CG: the restart threshold on ||r||/||b|| this
                             right-hand side was given (0: no restart planned);
                             other schemes: 0 */
} eigcg_stats;

/* Fill *p with defaults (nev 10, m 100, bank 240, FP64, batch 1, ...). */
int eigcg_default_params(eigcg_params* p);

/* Create a context for one gauge field and mass.  gauge_dev: device pointer to
 * the boundary gauge layout (deep-copied and converted; the caller may free it
 * afterwards).  hip_stream: hipStream_t or NULL for the default stream.
 * Errors: EINVAL (dims, nev/m, sizes), ENOMEM, EHIP. */
int eigcg_create(const eigcg_params* p, const void* gauge_dev, void* hip_stream,
                 eigcg_ctx** out);

/* Solve A x_i = b_i for nrhs right-hand sides (batched by max_batch).
 * b_dev, x_dev: boundary spinor layout; x_dev holds the initial guess on entry
 * (zero it for a cold start) and the solution on exit.  Success means the FP64
 * true residual ||b - A x|| / ||b|| <= tol.  stats: nrhs entries or NULL.
 * b = 0 gives x = 0 after 0 iterations.  Returns the worst per-RHS status. */
int eigcg_solve(eigcg_ctx* ctx, int32_t nrhs, const void* b_dev, void* x_dev, double tol,
                int32_t mode, eigcg_stats* stats);

/* init-CG guess of eq. (2.1): x <- x + U H^{-1} U^H (b - A x) for nrhs columns
 * (x_dev: in x~0, out x0).  With an empty bank x is unchanged. */
int eigcg_deflate_init(eigcg_ctx* ctx, int32_t nrhs, const void* b_dev, void* x_dev);

/* Free everything the context owns. */
int eigcg_destroy(eigcg_ctx* ctx);

/* ---- deflated BiCGSTAB on the Dirac system ------------------------------------
 * Section 1: the eigenvectors of A = M^H M are eigenvectors of the Hermitian
 * Q = gamma5 M (Q^2 = A), so the bank built by eigCG can deflate a
 * nonsymmetric solver for further right-hand sides.  eigcg_solve_bicgstab
 * solves M x_i = b_i (in an odd-even context Mhat x_e = b_e on even-site
 * fields) for nrhs columns, one after the other, in FP64 on the context's FP64
 * operator, with BiCGSTAB (van der Vorst 1992; shadow residual r_0, half step
 * taken when ||s|| meets the tolerance, restart from the current iterate when
 * the recursive residual converged but the true one did not).
 * flags: EIGCG_BICG_GAMMA5 iterates on Q x = gamma5 b instead of M x = b (same
 * solution and residual norm; the form whose spectrum the bank deflates);
 * EIGCG_BICG_DEFLATE first moves x to the minimiser of ||b - M x|| over
 * x + span(U): since (M U)^H (M U) = U^H A U = H, this is the init-CG step of
 * eq. (2.1) for A x = M^H b, x <- x + U H^{-1} U^H M^H (b - M x), with the bank's
 * H and Cholesky factor (for exact eigenvectors it is the Galerkin projection
 * of Q x = gamma5 b onto span(U)).  An empty bank leaves x unchanged.
 * EIGCG_BICG_GUESS_ONLY returns after that step (iters 0; true_rel_res and
 * guess_rel_res = the starting point's residual; status OK if it meets tol,
 * else ENOTCONV).
 * b_dev, x_dev: boundary spinor layout, x holds the starting guess on entry.
 * max_iter <= 0: the context's max_iter.  Success means the FP64 true residual
 * ||b - M x|| / ||b|| <= tol.  stats: nrhs entries or NULL.  Returns the worst
 * per-column status (ENOTCONV at max_iter, EBREAKDOWN on a zero rho, r^_0^H v or
 * t^H t, on non-finite scalars, or when H is not positive definite). */
enum { EIGCG_BICG_GAMMA5 = 1, EIGCG_BICG_DEFLATE = 2, EIGCG_BICG_GUESS_ONLY = 4 };
typedef struct {
  int32_t iters;          /* BiCGSTAB iterations (two applications of M each) */
  int32_t restarts;       /* restarts after a true-residual check */
  int32_t status;         /* EIGCG_OK, EIGCG_ENOTCONV or EIGCG_EBREAKDOWN */
  int32_t bank_used;      /* bank columns in the deflated guess (0: none) */
  double true_rel_res;    /* ||b - M x|| / ||b|| in FP64 */
  double guess_rel_res;   /* the same for the starting guess after deflation */
  double seconds;         /* wall time of this column */
} eigcg_bicgstab_stats;
int eigcg_solve_bicgstab(eigcg_ctx* ctx, int32_t nrhs, const void* b_dev, void* x_dev,
                         double tol, int32_t flags, int32_t max_iter,
                         eigcg_bicgstab_stats* stats);

/* out = op(in) for op = M, M^H or A = M^H M in FP64 (test support); in an
 * odd-even context Mhat, Mhat^H and Mhat^H Mhat on even-site fields.
 * op + 3 (EIGCG_OP_INNER): the same with the inner-precision kernels of a
 * mixed context (input rounded to FP32 or 16 bits, result widened to FP64);
 * EINVAL in an FP64 context. */
int eigcg_apply(eigcg_ctx* ctx, int32_t op, int32_t nrhs, const void* in_dev, void* out_dev);

/* eigcg_apply without allocating: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  out = op(in) for op = EIGCG_OP_M, EIGCG_OP_MDAG or
 * EIGCG_OP_A in FP64 (not EIGCG_OP_INNER), the same kernels and results as
 * eigcg_apply, one column at a time through two staging fields held in a
 * fixed device array of the library (one per GPU, kept until the process
 * ends; its size from eigcg_noalloc_scratch_bytes, 64 MiB: lattices up to
 * 2 x 12 x 16 B x (padded sites) within it, e.g. 16^3 x 32).  EINVAL for a
 * larger lattice, another op, or when the context's device is not current.
 * Calls on one GPU share its array: calls that overlap on one GPU (several
 * threads or streams) race and must be serialised by the caller.
 * Synchronises the context's stream. */
int eigcg_apply_noalloc(eigcg_ctx* ctx, int32_t op, int32_t nrhs, const void* in_dev,
                        void* out_dev);
int eigcg_noalloc_scratch_bytes(uint64_t* bytes);

/* Odd-even contexts only (EINVAL otherwise), for nrhs full-lattice fields
 * b_full_dev (boundary layout [nrhs][Lt][Lz][Ly][Lx][4][3]):
 * eigcg_schur_rhs writes rhs_dev (even-site layout) = Mhat^H (b_e + D_eo b_o / (2 d)),
 * the right-hand side whose solution x_e is the even part of the solution of
 * M x = b; eigcg_schur_reconstruct writes x_full_dev (full layout) with even part
 * x_even_dev and odd part (b_o + D_oe x_e / 2) / d.  Both synchronise. */
int eigcg_schur_rhs(eigcg_ctx* ctx, int32_t nrhs, const void* b_full_dev, void* rhs_dev);
int eigcg_schur_reconstruct(eigcg_ctx* ctx, int32_t nrhs, const void* b_full_dev,
                            const void* x_even_dev, void* x_full_dev);

/* Rayleigh-Ritz on the bank (Section 5.2): *l = columns of U; ritz_vals
 * (l doubles, ascending) = eigenvalues of H = U^H A U; ritz_res (l doubles or
 * NULL) = ||A u - theta u|| of each Ritz vector (l extra applications of A). */
int eigcg_bank_info(eigcg_ctx* ctx, int32_t* l, double* ritz_vals, double* ritz_res);

/* Copy bank columns [first, first+count) to out_dev in the boundary spinor
 * layout (count fields). */
int eigcg_bank_vectors(eigcg_ctx* ctx, int32_t first, int32_t count, void* out_dev);

/* Append count given fields (boundary layout) to the bank: each group of nev
 * is orthonormalised against U and within itself (classical Gram-Schmidt
 * twice, columns whose norm drops below 1e-10 of their input norm are
 * skipped) and H grows by U^H A Vbar, as in the Section 4 update.  *added
 * (may be NULL) receives the number of vectors kept.  Serves checkpoint /
 * restore of a bank and tests with prescribed deflation spaces. */
int eigcg_bank_load(eigcg_ctx* ctx, int32_t count, const void* vecs_dev, int32_t* added);

/* Copy H = U^H A U (l x l, column-major complex128) to host memory h_host. */
int eigcg_bank_matrix(eigcg_ctx* ctx, double* h_host);

/* Ritz values (ascending, nev per column) produced by the last EIGCG-mode
 * solve; *count = values written (<= cap). */
int eigcg_last_ritz(eigcg_ctx* ctx, double* vals, int32_t cap, int32_t* count);

/* Drop every bank vector (l = 0). */
int eigcg_bank_reset(eigcg_ctx* ctx);

/* Truncate U to its k lowest Ritz vectors (the Section 4 discussion of
 * limiting the size of U): with H Y = Y Theta, U <- U Y_k and H <- Theta_k
 * (k >= l leaves the bank unchanged, k = 0 empties it).  Needs k fields of
 * device memory for the duration of the call.  EINVAL for k < 0. */
int eigcg_bank_truncate(eigcg_ctx* ctx, int32_t k);

/* Lock accurate eigenvectors out of U (the Section 4 discussion of lowering
 * the cost of growing U): Rayleigh-Ritz on the unlocked columns, U_u <- U_u Y
 * with H_u Y = Y Theta (H_u the block of H on the unlocked columns; its
 * coupling with the locked block is zero by construction), and every Ritz
 * vector with ||A u - theta u|| <= tol (absolute, in the bank precision) is
 * locked.  Locked columns come first (the earlier ones, then the new ones in
 * ascending Ritz value), the unlocked Ritz vectors follow in ascending order,
 * and H becomes diag(Theta) on the rotated columns.  Later bank updates leave
 * the locked rows of U^H A Vbar at zero instead of forming them (each skipped
 * entry is r^H v, at most tol in modulus) while still orthonormalising new
 * vectors against every column.  Needs l - nlocked fields of device memory
 * during the call and one application of A per unlocked column.  *nlocked
 * (may be null) receives the number of locked columns.  Truncation,
 * restore and reset unlock everything.  EINVAL for tol < 0 or non-finite. */
int eigcg_bank_lock(eigcg_ctx* ctx, double tol, int32_t* nlocked);
/* Number of locked leading columns of U (>= 0), or EINVAL. */
int eigcg_bank_locked(eigcg_ctx* ctx);

/* Restore a saved bank (checkpoint / resume): U <- l fields from vecs_dev
 * (boundary layout, as eigcg_bank_vectors wrote them; stored in the bank's
 * precision) and H <- h_host (l x l complex128 column-major, as
 * eigcg_bank_matrix wrote it).  Nothing is re-orthonormalised and A is not
 * applied, so the restored context deflates exactly as the saved one did.
 * EINVAL when l > max_bank or H is not Hermitian positive definite. */
int eigcg_bank_restore(eigcg_ctx* ctx, int32_t l, const void* vecs_dev, const double* h_host);

/* Bytes of device memory the context holds. */
int eigcg_memory(eigcg_ctx* ctx, uint64_t* bytes);

/* info[0] = lattice sites V, info[1] = padded plane stride, info[2] = 1 when
 * the FP64 links are stored as two rows (12 reals), info[3] likewise for the
 * FP32 links of a mixed-precision context, info[4] / info[5] = stencil
 * variant used for FP64 / FP32, info[6] / info[7] = columns per workgroup
 * those variants run with (0 = the widest the batch allows: 2 for FP64, 4
 * for FP32); info needs 8 entries.  Variants:
 *   1  thread per site, 256-site units dealt round-robin to workgroups
 *   2  thread per site, XCD-contiguous chunks of units
 *   3  two waves per 64-site tile (directions split, LDS exchange), XCD chunks
 *   4  as 3 with streaming (nontemporal) epilogue loads and stores
 *   5  as 4 with a grid of the resident size (one sweeping front per XCD)
 *   6  as 5 with at most two workgroups per compute unit
 *   7  as 5 with one workgroup per compute unit
 *   8  as 5, each XCD sweeping its t-slab in (z, t, xy) tile order
 *   9  as 8 with at most two workgroups per compute unit
 *  10  as 9 with cached (not streaming) epilogue loads and stores
 *  11  z-march: each lane marches the z-planes of one (x, y, t) column, so
 *      the z-hops reuse spinors and links from registers; XCD x owns a t-slab
 *  12  as 11 with the z-range in 2 chunks; 13: in 4 chunks (more waves)
 *  14  as 9, the t-slab swept in blocks of 4, 3 or 2 z-planes (dividing Lz):
 *      (z-block, t, z, xy) order, z-neighbours one xy-plane apart in the sweep
 *  15  as 14 with cached (not streaming) epilogue loads and stores
 * (8-15 need Lx Ly divisible by 64 and Lt by 8, else they run as 5 / 6 / 6;
 * 16-bit storage runs 1-4 as 5, 10 as 9 and 15 as 14; odd-even contexts run
 * 1-2 as 3 and 11-13 as 6).
 * eigcg_tune_report: tune_ms (30 doubles) receives the ms that variants 1..15
 * took (best over columns per workgroup) for one CG-shaped pair of stencil
 * passes over a full batch at create, FP64 then FP32 (0 where not timed, e.g.
 * a forced variant). */
int eigcg_layout_info(eigcg_ctx* ctx, int32_t* info);
int eigcg_tune_report(eigcg_ctx* ctx, double* tune_ms);

/* The stencil tuner's choices per (lattice, plane stride, geometry,
 * precision, link storage, batch width) are kept for the process and
 * persisted in a text file (one line per choice: device and library build,
 * the key, the variant, columns per workgroup and the timings), so that
 * later processes skip the timing: the file is the environment variable
 * EIGCG_TUNE_CACHE (empty or "off": no file), else
 * $XDG_CACHE_HOME/eigcg/stencil_tune.txt or ~/.cache/eigcg/stencil_tune.txt.
 * eigcg_tune_cache_reset drops the process's choices (the file stays), so the
 * next create reads the file again or re-tunes. */
int eigcg_tune_cache_reset(void);

/* Average device time (ms) of one launch, from HIP events on the context's
 * stream around reps back-to-back launches: what 0 = FP64 stencil M, 1 = plain
 * copy of one FP64 field (12 V complex numbers read and written; a reference
 * for memory counters), 2 = one full FP64 CG iteration (three kernels),
 * 3 = FP32 stencil M (mixed contexts).  Runs on the context's internal work
 * vectors (their contents change); reps + 8 must not exceed max_iter. */
int eigcg_time_kernel(eigcg_ctx* ctx, int32_t what, int32_t reps, double* ms);

/* Sampled stencil timings (params.sample_every; each sampled kernel carries
 * start/stop events filled by its own dispatch).  out[0..3] for FP64 and
 * out[4..7] for FP32 iterations: number of sampled iterations in which the
 * kernels ran, mean duration in ms of the first pass (M p with the p^H A p
 * partials), mean duration of the second pass (M^H fused with the residual
 * update and its norm, without the per-column finalize kernel), mean batch
 * width.  A sample whose second pass took under half the median of all
 * samples is a launch after every column of it had stopped (the kernels exit
 * at once) and is left out of all four.  Waits for the context's stream;
 * reset != 0 clears the accumulated samples. */
int eigcg_kernel_samples(eigcg_ctx* ctx, int32_t reset, double* out);

/* Text of the context's last error; with ctx == NULL, of this thread's last
 * failed eigcg_create. */
const char* eigcg_last_error(const eigcg_ctx* ctx);

/* ---- serving: continuous batching over several contexts --------------------
 * A server admits solve requests for any registered context (gauge field).
 * Every field has a worker thread and a HIP stream of its own, so the work of
 * different fields overlaps on the device.  A field's requests are served in
 * submission order: init-CG requests run as columns of a shared batched
 * iteration (new requests join and finished ones leave between iteration
 * segments) deflated with the field's resident bank (eq. (2.1)); eigCG
 * requests (eigcg_submit_mode with EIGCG_MODE_EIGCG: one step of Incremental
 * eigCG, Section 4) wait for the running slots to finish, then grow the
 * field's bank by their Ritz vectors, so later requests are deflated with
 * the grown bank.  Admission is subject to the HBM budget: each context's
 * resident memory is charged once, every active init-CG request its working
 * set, an eigCG request the field's eigCG window while it is not allocated
 * (it waits for other fields' requests to finish, and fails with
 * EIGCG_ENOMEM when the window cannot fit even then).  Results do not depend
 * on which other requests share a batch or run at the same time. */
typedef struct eigcg_server eigcg_server;

int eigcg_server_create(uint64_t hbm_budget, eigcg_server** out);
/* Register a context; *field_id receives its index.  The context must stay
 * alive until the server is destroyed and must not be used directly meanwhile. */
int eigcg_server_add(eigcg_server* srv, eigcg_ctx* ctx, int32_t* field_id);
/* Enqueue one solve (mode EIGCG_MODE_INITCG semantics, cold start).  b_dev and
 * x_dev (one field each, boundary layout) must stay valid until done. */
int eigcg_submit(eigcg_server* srv, int32_t field_id, const void* b_dev, void* x_dev, double tol,
                 uint64_t* ticket);
/* As eigcg_submit with mode EIGCG_MODE_INITCG or EIGCG_MODE_EIGCG (the latter
 * grows the field's bank; EINVAL in a 16-bit context). */
int eigcg_submit_mode(eigcg_server* srv, int32_t field_id, const void* b_dev, void* x_dev,
                      double tol, int32_t mode, uint64_t* ticket);
/* EIGCG_EBUSY while running; otherwise the solve status with *st filled
 * (st->seconds = submit-to-completion latency). */
int eigcg_poll(eigcg_server* srv, uint64_t ticket, eigcg_stats* st);
/* Block until every submitted request has completed. */
int eigcg_server_drain(eigcg_server* srv);
int eigcg_server_destroy(eigcg_server* srv);

/* ---- device probes (test support) -------------------------------------------
 * eigcg_debug_mfma_probe: runs the FP64 and FP32 16x16x4 matrix-core
 * instructions on index-encoding inputs; out_dev (device, 1024 doubles)
 * receives, per lane and accumulator register, the (row + 1, column + 1) of
 * the product entry it holds (FP64 first, then FP32).
 * eigcg_debug_gemm: the library's complex tall-skinny products on contiguous
 * device columns of n complex entries (prec 0: complex128, 1: complex64):
 * kind 0: out (n x N) = in (n x K) s (K x N, complex128 column-major);
 * kind 2: out += in s; kind 3: out -= in s (out holds its old values);
 * kind 1: out (K x N, complex128 column-major) = in^H r (r: n x N), using
 * scratch_dev (scratch_elems doubles) for chunk partials.  K <= 256,
 * N <= 24 (kinds 0, 2, 3) or 16 (kind 1).  All synchronise the device. */
int eigcg_debug_mfma_probe(double* out_dev);
/* eigcg_debug_span: the host-side bounds layer (no GPU needed).  The library
 * registers each of its device allocations with its size and refuses, with
 * EINVAL before any launch, a column pointer or a launch whose fields would
 * reach past the end of the allocation they start in.  op 0 registers
 * [addr, addr + bytes) as an allocation, op 1 removes the allocation at addr,
 * op 2 checks an access of bytes at addr: EIGCG_OK when it ends inside the
 * allocation containing addr (or addr lies in none), EIGCG_EINVAL when it
 * reaches past that allocation's end.  Addresses are never dereferenced. */
int eigcg_debug_span(int32_t op, uint64_t addr, uint64_t bytes);
int eigcg_debug_gemm(int32_t prec, int32_t kind, uint64_t n, int32_t K, int32_t N,
                     const void* in_dev, const void* r_dev, const double* s_dev, void* out_dev,
                     double* scratch_dev, uint64_t scratch_elems);

/* ---- host linear algebra (test support; no GPU needed) ---------------------- */
/* Ascending eigenvalues w (n) and eigenvectors of the k lowest (z, n x k
 * column-major complex128) of the Hermitian n x n matrix a (column-major
 * complex128, upper triangle read). */
int eigcg_host_eig_lowest(int32_t n, const double* a, int32_t k, double* w, double* z);
/* Thin QR of the m x n complex matrix a: q (m x n) and r (n x n). */
int eigcg_host_qr(int32_t m, int32_t n, const double* a, double* q, double* r);
/* Solve H X = B (H n x n HPD, B n x nrhs; complex128 column-major). */
int eigcg_host_chol_solve(int32_t n, const double* h, int32_t nrhs, double* b);
/* The rule of EIGCG_MODE_AUTO: after `done` eigCG groups (batches of right-
 * hand sides) with mean iteration counts iters[done] and wall times
 * secs[done] (seconds), `left` groups still to solve (the next included),
 * iter_ms the measured time of one CG iteration of a group and bank_room the
 * nev-blocks U can still take: 1 when the next group should run eigCG (its
 * overhead over plain CG, estimated by the last group as
 * secs - iters * iter_ms, is smaller than the iterations it is predicted to
 * save the left - 1 later groups: the mean drop in iterations over the last
 * three groups, or fewer while done < 4), else 0.  Always 1 for done < 3
 * (with left > 1 and room), always 0 for left <= 1 or no room. */
int eigcg_host_auto_continue(int32_t done, int32_t left, const double* iters, const double* secs,
                             double iter_ms, int32_t bank_room);
/* The dynamic init-CG restart threshold (EIGCG_RESTART_DYNAMIC), the open
 * choice at the end of Section 5.3, on given inputs: l Ritz values theta
 * (ascending, positive) with residual norms res = ||A u - theta u||, the norm
 * estimate lambda_max, the solve tolerance tol and the cost of one restart in
 * iterations.  Model: with R_k the residuals of the k lowest pairs, the
 * residual left by a Galerkin projection (eq. (2.1)) regains components along
 * their true eigenvectors once CG has reduced it by s_k = ||R_k||_F / lambda_max
 * (the lower end of the angle bracket [||R_k|| / lambda_max, ||R_k|| / gap_k];
 * s_0 = 0); the bulk starts at theta_b, b = 1 + max{k : ||R_k||_F /
 * (theta_{k+1} - theta_k) < 1}; a CG leg reducing the residual by f costs
 * |O| + sqrt(lambda_max/theta_b)/2 (ln(2/f) + sum over the outliers
 * O = {k'+1 .. b-1}, k' = max{k < b : s_k <= f}, of ln(lambda_max/theta_j - 1))
 * iterations (the CG bound with outlying eigenvalues); one restart at tau
 * costs leg(tau) + restart_cost + leg(tol/tau), constant between the break
 * points {s_k, tol/s_k}: equal neighbouring intervals merge, the cheapest wins
 * (then the wider in ln tau, then the larger tau), and tau is its geometric
 * midpoint, planned only when strictly cheaper than no restart.  out[0] = tau
 * (0: no restart), out[1] = predicted iterations without a restart, out[2] =
 * with the planned one (= out[1] if none).  Host only; EINVAL for l < 0,
 * unsorted or non-positive theta, or non-finite inputs. */
int eigcg_restart_model(int32_t l, const double* theta, const double* res, double lambda_max,
                        double tol, double restart_cost, double* out);

#ifdef __cplusplus
}
#endif

#endif /* EIGCG_H */
