// Host-side launchers of the HIP kernels (declarations).  Every launcher
// enqueues on the given stream and returns hipSuccess or the launch error.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace eigcg {

enum Prec { kF64 = 0, kF32 = 1, kF16 = 2 };  // kF16: IEEE half storage, FP32 arithmetic
enum StencilOp { kOpM = 0, kOpMdag = 1 };
// epilogues of the stencil launch
enum StencilEpi {
  kEpiStore = 0,   // out = op(in)
  kEpiNorm = 1,    // out = op(in); partials of ||out||^2 = p^H A p (first CG pass)
  kEpiCGR = 2,     // alpha from the first pass; t = op(in); r -= alpha t; r^H r; then a
                   // finalize kernel updates alpha, beta and the stop tests
  kEpiRes = 3,     // r = b - op(in); r^H r -> rho (true residual, with finalize)
};

// Stencil kernel variants (StencilLaunch::variant):
//  1: thread per site, 256-site units dealt round-robin to workgroups
//  2: thread per site, XCD-contiguous chunks of units
//  3: two waves per 64-site tile (directions split, LDS exchange), XCD chunks
//  4: as 3 with streaming (nontemporal) epilogue loads and stores
//  5: as 4 with a resident-size grid (one contiguous front per XCD)
//  6: as 5 with at most two workgroups per CU
//  7: as 5 with one workgroup per CU
//  8: as 5, each XCD sweeping a t-slab in (z, t, xy) tile order
//  9: as 8 with at most two workgroups per CU
// 10: as 9 with cached (not streaming) epilogue loads and stores
// 11: z-march: each lane marches the z-planes of one (x, y, t) column, the
//     z-hops from registers, XCD x owning a t-slab (stencil_impl.h)
// 12, 13: as 11 with the z-range split in 2 or 4 chunks (more waves)
// 14: as 9 with the slab swept in blocks of z-planes (4, 3 or 2 dividing Lz):
//     (z-block, t, z, xy) order, so z-neighbours inside a block are one
//     xy-plane apart in the sweep and t-neighbours one block of planes
// 15: as 14 with cached (not streaming) epilogue loads and stores
// 8-15 need whole 64-site tiles per xy-plane and Lt divisible by 8; other
// lattices run 5 and 6 (10-15 as 6) instead; the odd-even geometry runs
// 11-13 as 6.
constexpr int kStencilVariants = 15;

struct StencilLaunch {
  int prec;                 // kF64 / kF32 (vectors and links)
  int op;                   // kOpM / kOpMdag
  int epi;                  // StencilEpi
  int compressed;           // links stored as two rows
  int variant;              // stencil kernel variant 1..kStencilVariants (0 = 1)
  const void* in; size_t in_cs;     // column stride in complex elements
  void* out; size_t out_cs;         // kEpiStore / kEpiNorm target
  const void* u;
  const Geom* g;
  double diag;              // 4 + m_q
  int ncols;
  uint32_t mask;            // columns to process
  ColState* st;             // per-column state (kEpiNorm / kEpiCGR / kEpiRes)
  double* partial;          // 2 * kMaxCols * kMaxGrid doubles (first/second pass)
  unsigned int* counter;    // unused by the stencil (kept for the launch ABI)
  void* r; size_t r_cs;     // kEpiCGR residual, kEpiRes residual output
  const void* b; size_t b_cs;       // kEpiRes right-hand side
  void* tbuf; size_t t_cs;  // kEpiCGR: two t slots per column (slot = j & 1)
  double* hist; int hist_stride;    // kEpiCGR: per column 3 doubles per iteration
  hipEvent_t ev_start = nullptr;    // when set: timestamps of the stencil kernel's own
  hipEvent_t ev_stop = nullptr;     // start and end, taken by its dispatch
  int* grid_out = nullptr;          // when set: receives the grid's x extent (the number
                                    // of partials per column the pass writes)
  int defer_finalize = 0;           // kEpiCGR: leave the finalize kernel to the caller
                                    // (launch_finalize_cg), e.g. after a preconditioner
  int nc = 0;                       // variants 3..10: columns per workgroup (1, 2, or 4
                                    // for FP32); 0 = widest that ncols allows
  // Odd-even geometry (g->eo): op is the even-site Schur complement
  // Mhat = diag - D_eo D_oe / (4 diag) or its adjoint (D: hopping sum of M
  // or M^H), applied in two passes: t = D_oe in / (2 diag) into eo_tmp (odd
  // sites, ncols fields), then diag in - D_eo t / 2 with the epilogue.
  // Variants 1 and 2 run as 3.
  void* eo_tmp = nullptr; size_t eo_tmp_cs = 0;
  // eo_raw = 1: one pass only, out (parity eo_par) = eo_dg in2 + eo_ch D in,
  // in on the other parity (in2 may be null: eo_dg ignored)
  int eo_raw = 0;
  int eo_par = 0;
  const void* in2 = nullptr; size_t in2_cs = 0;
  double eo_dg = 0.0, eo_ch = 0.0;
};

hipError_t launch_stencil(const StencilLaunch& L, hipStream_t s);
// per-precision entry points (one translation unit each)
hipError_t launch_stencil_f64(const StencilLaunch& L, hipStream_t s);
hipError_t launch_stencil_f32(const StencilLaunch& L, hipStream_t s);
hipError_t launch_stencil_f16(const StencilLaunch& L, hipStream_t s);
hipError_t launch_stencil_eo_f64(const StencilLaunch& L, hipStream_t s);
hipError_t launch_stencil_eo_f32(const StencilLaunch& L, hipStream_t s);
hipError_t launch_stencil_eo_f16(const StencilLaunch& L, hipStream_t s);

// End of a CG iteration: x += alpha p; (running) p = r + beta p; optional window append
// V_ring[(iter + 1) % ring] = r / sqrt(rho).
struct UpdateLaunch {
  int prec;
  int ncols;
  uint32_t mask;
  ColState* st;
  const Geom* g;
  void* x; size_t x_cs;
  void* p; size_t p_cs;
  const void* r; size_t r_cs;
  void* ring; size_t ring_cs; int ring_len; size_t ring_col_cs;  // slot stride, column stride
};
hipError_t launch_cg_update(const UpdateLaunch& L, hipStream_t s);

// The CG scalars after the second stencil pass (what a kEpiCGR launch does
// itself unless defer_finalize): p^H A p from part_a (alpha or breakdown),
// ||r||^2 from part_b (stop tests); with spec_s the preconditioned rho_new =
// r^H z = ||r||^2 + spec_s[col] sets beta, rho and the history.  nb partials
// per column (the passes' grid extent).
hipError_t launch_finalize_cg(ColState* st, int ncols, uint32_t mask, const double* part_a,
                              const double* part_b, int nb, double* hist, int hist_stride,
                              const double* spec_s, hipStream_t s);
// Spectral preconditioner z = r + U_R (D (U_R^H r)) (blas.hip): from G =
// U_R^H r (l x ncols, complex, column-major), S = D G and s = G^H D G per
// column (fixed order); then z = r and the caller adds U_R S.
hipError_t launch_spec_scale(const double2* G, const double* D, int l, int ncols, double2* S,
                             double* s_out, hipStream_t s);
// rho += s[col] for running masked columns (the start of a preconditioned CG:
// rho = r^H z after the true residual's ||r||^2)
hipError_t launch_spec_rho(ColState* st, int ncols, uint32_t mask, const double* s_in,
                           hipStream_t s);

// Initial CG state: p = r (rho already in st), optional ring slot 1 write;
// per column: rho = r^H r given by kEpiRes.
hipError_t launch_cg_start(const UpdateLaunch& L, hipStream_t s);

// After a true-residual computation (kEpiRes): per masked column in state
// Run, or stopped for a restart, decide converged (rho <= res_stop2) or
// running again (with the refinement's next inner stop when inner_rel2 > 0).
hipError_t launch_post_residual(ColState* st, int ncols, uint32_t mask, hipStream_t s);
// After a reliable update (r = FP64 true residual, rho = r^H r in the states,
// post_residual done): p <- p - (r^H p / rho - 1) r for running masked
// columns, so that r^H p = r^H r as the next step length assumes (FP32 or
// FP64 vectors; partial: 2 kMaxCols kMaxGrid doubles).
hipError_t launch_reliable_fix_p(int prec, int ncols, uint32_t mask, size_t n, const void* r,
                                 void* p, size_t cs, const ColState* st, double* partial,
                                 hipStream_t s);
// Set state/reason of masked columns (host-driven transitions).
hipError_t launch_set_state(ColState* st, int ncols, uint32_t mask, int state, int reason,
                            int clear_restart, hipStream_t s);

// Layout conversion between the boundary (AoS complex128, [site][spin][colour])
// and the internal SoA planes; prec selects the internal storage.
hipError_t launch_spinor_to_soa(const double2* aos, void* soa, int prec, const Geom* g, int ncols,
                                size_t soa_cs, hipStream_t s);
hipError_t launch_spinor_from_soa(const void* soa, double2* aos, int prec, const Geom* g,
                                  int ncols, size_t soa_cs, hipStream_t s);
// gauge AoS [site][mu][a][b] -> SoA planes (full 9 or compressed 6 per mu;
// parity blocks in the odd-even geometry)
hipError_t launch_gauge_to_soa(const double2* aos, void* soa, int prec, int compressed,
                               const Geom* g, hipStream_t s);
// max over links of |U U^H - 1| and |det U - 1| (unitarity check), one double each
hipError_t launch_gauge_check(const double2* aos, const Geom* g, double* out2, hipStream_t s);
// Odd-even geometry, FP64: full-lattice AoS fields <-> their even and odd
// half-site SoA fields (ncols columns; soa_cs per half field)
hipError_t launch_split_eo(const double2* aos, void* even, void* odd, const Geom* g, int ncols,
                           size_t soa_cs, hipStream_t s);
hipError_t launch_merge_eo(const void* even, const void* odd, double2* aos, const Geom* g,
                           int ncols, size_t soa_cs, hipStream_t s);

// Generic BLAS1 over n complex entries per column (FP64 or FP32 storage).
// y = a*x + y with per-column complex a (device array of 2*ncols doubles or
// host scalar when a_dev is null).
hipError_t launch_axpy(int prec, int ncols, size_t n, const double* a_dev, double a_re,
                       double a_im, const void* x, size_t x_cs, void* y, size_t y_cs,
                       hipStream_t s);
// y = x (with conversion between precisions: src_prec -> dst_prec)
hipError_t launch_copy(int src_prec, int dst_prec, int ncols, size_t n, const void* x,
                       size_t x_cs, void* y, size_t y_cs, hipStream_t s,
                       uint32_t mask = 0xffffffffu);
// norms2[c] = ||x_c||^2 in FP64, deterministic; partial/counter as for stencils
hipError_t launch_norm2(int prec, int ncols, size_t n, const void* x, size_t x_cs,
                        double* partial, unsigned int* counter, double* out, hipStream_t s);
// y_c *= scale[c] (scale from device, FP64)
hipError_t launch_scale(int prec, int ncols, size_t n, const double* scale_dev, void* y,
                        size_t y_cs, hipStream_t s);
// w = t1 - beta * t0 per column with beta = hist-derived scalar from device
hipError_t launch_xpby(int prec, int ncols, size_t n, const void* t1, const void* t0,
                       size_t t_cs, const double* beta_dev, void* w, size_t w_cs,
                       hipStream_t s);
// mixed precision accumulation: x64 += (double) e32 / scale ; e32 = 0, where
// scale is the column's inner-solve scale from scale_st (1 when null)
hipError_t launch_accum_f32_into_f64(int ncols, size_t n, void* x64, size_t x_cs, void* e32,
                                     size_t e_cs, hipStream_t s, uint32_t mask = 0xffffffffu,
                                     const ColState* scale_st = nullptr);
// 16-bit inner solves: per running column, scale = c0 / sqrt(rho); rho and
// restart2 are rescaled to the inner solve's units
hipError_t launch_set_scale(ColState* st, int ncols, uint32_t mask, double c0, hipStream_t s);
// y16 = scale * x64 for running masked columns (16-bit storage)
hipError_t launch_to_inner16(int ncols, size_t n, const void* x64, size_t x_cs, void* y16,
                             size_t y_cs, uint32_t mask, const ColState* st, hipStream_t s);

// Tall-skinny products on MFMA (complex):
//   Out(n x N) = beta*Out + In(n x K) * S(K x N)
// In columns come from a device array of column pointers (K entries), Out
// columns likewise (N entries); S is column-major complex FP64 on the device
// (ld = K).  beta is 0 (overwrite) or 1 (accumulate).  Out may alias In
// columns (each output row depends only on the same input row).
hipError_t launch_gemm_tall(int prec, size_t n, int K, int N, const void* const* in_cols,
                            void* const* out_cols, const double2* S, int beta_one, int negate,
                            hipStream_t s);
// Reduction products: G(K x N) = In(n x K)^H * R(n x N), column pointer
// arrays as above; deterministic two-pass (chunk partials then fixed-order
// sum); result FP64 complex column-major (ld = K) on the device.
hipError_t launch_gemm_reduce(int prec, size_t n, int K, int N, const void* const* in_cols,
                              const void* const* r_cols, double2* partial, size_t partial_elems,
                              double2* G, hipStream_t s);

// BiCGSTAB vectors (FP64, n complex entries; bicgstab_blas.hip).
// launch_bicg_dots: out[i] = a_i^H b_i for np <= kBicgMaxDots pairs, deterministic
// (workgroup partials in `partial`, kBicgMaxDots * kBicgDotBlocks entries, then a
// fixed-order sum).
constexpr int kBicgMaxDots = 4;
constexpr int kBicgDotBlocks = 1024;
hipError_t launch_bicg_dots(int np, size_t n, const void* const* a, const void* const* b,
                            double2* partial, double2* out, hipStream_t s);

// Device-resident BiCGSTAB recurrence (one right-hand side): the scalars live
// in a BicgState on the device and every kernel of an iteration reads them
// there, so the host polls only between segments of iterations.  A kernel does
// nothing once state != kBicgRun.
enum BicgRun { kBicgRun = 0, kBicgConv = 1, kBicgHalf = 2, kBicgBreak = 3, kBicgMaxIt = 4 };
struct BicgState {
  double2 rho, rho_old, alpha, omega, beta;
  double stop2;      // (tol ||b||)^2
  int it, max_iter;  // iterations completed, cap
  int state;         // BicgRun
  int half;          // the current iteration ends with the half step
};
// p = r + beta (p - omega v)
hipError_t launch_bicg_p_dev(size_t n, void* p, const void* r, const void* v,
                             const BicgState* st, hipStream_t s);
// alpha = rho / (rh^H v)
hipError_t launch_bicg_alpha(size_t n, const void* rh, const void* v, double2* partial,
                             BicgState* st, hipStream_t s);
// s = r - alpha v
hipError_t launch_bicg_s_dev(size_t n, void* sv, const void* r, const void* v,
                             const BicgState* st, hipStream_t s);
// t^H s, s^H s, t^H t: the half-step test on ||s||, else omega = t^H s / t^H t
hipError_t launch_bicg_omega(size_t n, const void* t, const void* sv, double2* partial,
                             BicgState* st, hipStream_t s);
// x += alpha p + omega s, r = s - omega t (half step: x += alpha p, r = s),
// then rho, the convergence test on ||r||, the iteration cap and beta
hipError_t launch_bicg_xr_dev(size_t n, void* x, void* r, const void* p, const void* sv,
                              const void* t, const void* rh, double2* partial, BicgState* st,
                              hipStream_t s);

// Test support: MFMA lane-layout probe (1024 doubles written to out_dev).
hipError_t launch_mfma_probe(double* out_dev, hipStream_t s);

}  // namespace eigcg
