// BiCGSTAB on the Dirac system with a deflated starting guess from the eigCG
// bank.  Section 1 of the paper: the eigenvectors of A = M^H M are also
// eigenvectors of the Hermitian Q = gamma5 M (Q^2 = A), so the vectors eigCG
// accumulates can deflate a nonsymmetric solver for later right-hand sides.
//
// The iteration is van der Vorst's BiCGSTAB (1992) with shadow residual r_0,
// on M x = b or on Q x = gamma5 b.  The guess minimises ||b - M x|| over
// x + span(U): the normal equations of that least-squares problem have the
// matrix (M U)^H (M U) = U^H A U = H, the bank's own, so the guess is the
// init-CG step of eq. (2.1) applied to A x = M^H b and reuses its Cholesky
// factor.  For exact eigenvectors it equals the Galerkin projection of
// Q x = gamma5 b onto span(U).
//
// Every vector operation runs in the library's kernels: the two-tile stencil,
// the fused BiCGSTAB updates and inner products (bicgstab_blas.hip), BLAS1 and
// the MFMA products of the deflation.  The recurrence's scalars (rho, alpha,
// omega, beta), its stop tests and the iteration count live in a BicgState on
// the device, updated by one-workgroup kernels after each inner product; the
// host reads the state once per segment of iterations (kernels of a stopped
// recurrence do nothing), and itself only starts and restarts the iteration
// and checks the true residual.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <utility>
#include <vector>

#include "engine.h"

namespace eigcg {
namespace {

constexpr int kMaxRestarts = 8;

enum { kX, kB, kR, kRh, kP, kV, kS, kT, kFields };

size_t prec_bytes(int prec) { return prec == kF64 ? 16 : (prec == kF32 ? 8 : 4); }

double wall_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

bool finite(cplx z) { return std::isfinite(z.real()) && std::isfinite(z.imag()); }

double2 d2(cplx z) { return make_double2(z.real(), z.imag()); }

constexpr size_t kPartialBytes = sizeof(double2) * kBicgMaxDots * kBicgDotBlocks;
constexpr int kSegment = 8;  // iterations enqueued between reads of the device state

struct Bicg {
  Ctx& c;
  bool g5;               // iterate on gamma5 M
  void* f[kFields];
  double2* partial;      // inner-product partials
  double2* out;          // inner products (kBicgMaxDots)
  BicgState* dst;        // the recurrence's device state

  Bicg(Ctx& c_, bool g5_) : c(c_), g5(g5_) {
    const size_t fb = c.cs * prec_bytes(kF64);
    const size_t bytes = fb * kFields + kPartialBytes + sizeof(double2) * kBicgMaxDots +
                         sizeof(BicgState);
    if (!c.bs) {
      c.bs = c.dalloc(bytes);
      // plane padding stays zero: kernels below never write it
      c.check(hipMemsetAsync(c.bs, 0, bytes, c.stream), "clear");
    }
    for (int i = 0; i < kFields; ++i) f[i] = col_ptr(c.bs, kF64, c.cs, i);
    partial = (double2*)((char*)c.bs + fb * kFields);
    out = partial + kBicgMaxDots * kBicgDotBlocks;
    dst = (BicgState*)(out + kBicgMaxDots);
  }
  void put_state(const BicgState& h) {
    c.check(hipMemcpyAsync(dst, &h, sizeof(BicgState), hipMemcpyHostToDevice, c.stream), "state");
    c.check(hipStreamSynchronize(c.stream), "sync");
  }
  BicgState get_state() {
    BicgState h;
    c.check(hipMemcpyAsync(&h, dst, sizeof(BicgState), hipMemcpyDeviceToHost, c.stream), "state");
    c.check(hipStreamSynchronize(c.stream), "sync");
    return h;
  }

  // y <- gamma5 y: in the chiral basis gamma5 = diag(1, 1, -1, -1), so the
  // planes of spins 2 and 3 (the second half of the field) change sign
  void gamma5(void* y) {
    const size_t half = c.cs / 2;
    void* lo = (char*)y + half * prec_bytes(kF64);
    c.check(launch_axpy(kF64, 1, half, nullptr, -2.0, 0.0, lo, half, lo, half, c.stream),
            "gamma5");
  }
  // out = M in, or gamma5 M in
  void op(const void* in, void* out, bool with_g5) {
    stencil_store(c, kF64, kOpM, 1, in, out);
    if (with_g5) gamma5(out);
  }
  void axpy(cplx a, const void* x, void* y) {
    c.check(launch_axpy(kF64, 1, c.cs, nullptr, a.real(), a.imag(), x, c.cs, y, c.cs, c.stream),
            "axpy");
  }
  void copy(const void* x, void* y) {
    c.check(launch_copy(kF64, kF64, 1, c.cs, x, c.cs, y, c.cs, c.stream), "copy");
  }
  void zero(void* y) {
    c.check(hipMemsetAsync(y, 0, c.cs * prec_bytes(kF64), c.stream), "zero");
  }
  // the np inner products in `out`, read back (synchronous)
  std::vector<cplx> fetch(int np) {
    c.check(hipMemcpyAsync(c.h_norm, out, sizeof(double2) * np, hipMemcpyDeviceToHost, c.stream),
            "memcpy");
    c.check(hipStreamSynchronize(c.stream), "sync");
    std::vector<cplx> G(np);
    for (int i = 0; i < np; ++i) G[i] = cplx(c.h_norm[2 * i], c.h_norm[2 * i + 1]);
    return G;
  }
  // a_i^H b_i
  std::vector<cplx> dots(std::vector<const void*> a, std::vector<const void*> b) {
    c.check(launch_bicg_dots((int)a.size(), c.cs, a.data(), b.data(), partial, out, c.stream),
            "dots");
    return fetch((int)a.size());
  }
  // r = rhs - Op x (rhs = f[kB]: b, or gamma5 b on the gamma5 system)
  void residual(void* r) {
    op(f[kX], f[kT], g5);
    copy(f[kB], r);
    axpy(-1.0, f[kT], r);
  }
};

// x <- x + U H^{-1} U^H M^H (b - M x)
void deflated_guess(Ctx& c, Bicg& B) {
  B.residual(B.f[kR]);            // rhs - Op x
  if (B.g5) B.gamma5(B.f[kR]);    // b - M x either way
  stencil_store(c, kF64, kOpMdag, 1, B.f[kR], B.f[kT]);  // M^H (b - M x)
  if (c.bank_prec == kF64) {
    deflate_columns(c, kF64, 1, 1u, B.f[kX], B.f[kT]);
  } else {  // FP32 bank: the products run in FP32, the correction is added in FP64
    void* r32 = B.f[kR];
    void* e32 = B.f[kV];
    c.check(launch_copy(kF64, kF32, 1, c.cs, B.f[kT], c.cs, r32, c.cs, c.stream), "narrow");
    c.check(hipMemsetAsync(e32, 0, c.cs * prec_bytes(kF32), c.stream), "zero");
    deflate_columns(c, kF32, 1, 1u, e32, r32);
    c.check(launch_accum_f32_into_f64(1, c.cs, B.f[kX], c.cs, e32, c.cs, c.stream), "accum");
  }
}

int solve_column(Ctx& c, Bicg& B, double tol, int max_iter, bool defl, bool guess_only,
                 eigcg_bicgstab_stats& st) {
  std::vector<cplx> G = B.dots({B.f[kB]}, {B.f[kB]});
  const double bb = G[0].real();
  if (!std::isfinite(bb)) throw ApiError{EIGCG_EINVAL, "right-hand side is not finite"};
  if (bb == 0.0) {  // b = 0: x = 0
    B.zero(B.f[kX]);
    return EIGCG_OK;
  }
  const double bnorm = std::sqrt(bb);
  const double stop = tol * bnorm;
  if (B.g5) B.gamma5(B.f[kB]);
  if (defl) {
    deflated_guess(c, B);
    st.bank_used = c.l;
  }
  int status = EIGCG_OK;
  int it = 0;
  bool first = true;
  if (guess_only) {  // the deflated starting point alone
    B.residual(B.f[kR]);
    G = B.dots({B.f[kR]}, {B.f[kR]});
    st.guess_rel_res = st.true_rel_res = std::sqrt(G[0].real()) / bnorm;
    return st.true_rel_res <= tol ? EIGCG_OK : EIGCG_ENOTCONV;
  }
  void* R = B.f[kR];
  void* S = B.f[kS];
  void* P = B.f[kP];
  void* V = B.f[kV];
  while (true) {
    B.residual(R);
    B.copy(R, B.f[kRh]);
    G = B.dots({B.f[kRh], R}, {R, R});
    cplx rho = G[0];
    const double rr = G[1].real();
    if (first) st.guess_rel_res = std::sqrt(rr) / bnorm;
    first = false;
    if (std::sqrt(rr) <= stop) break;
    if (st.restarts > kMaxRestarts) break;
    if (it >= max_iter) {
      status = EIGCG_ENOTCONV;
      break;
    }
    if (rho == 0.0 || !finite(rho)) {
      status = EIGCG_EBREAKDOWN;
      break;
    }
    B.zero(V);
    B.zero(P);
    // rho_old = alpha = omega = 1, so beta = rho (p = r in the first step)
    BicgState h{};
    h.rho = d2(rho);
    h.rho_old = h.alpha = h.omega = make_double2(1.0, 0.0);
    h.beta = d2(rho);
    h.stop2 = stop * stop;
    h.it = it;
    h.max_iter = max_iter;
    h.state = kBicgRun;
    h.half = 0;
    B.put_state(h);
    while (h.state == kBicgRun) {
      for (int k = 0; k < kSegment; ++k) {
        c.check(launch_bicg_p_dev(c.cs, P, R, V, B.dst, c.stream), "p");
        B.op(P, V, B.g5);
        c.check(launch_bicg_alpha(c.cs, B.f[kRh], V, B.partial, B.dst, c.stream), "alpha");
        c.check(launch_bicg_s_dev(c.cs, S, R, V, B.dst, c.stream), "s");
        B.op(S, B.f[kT], B.g5);
        c.check(launch_bicg_omega(c.cs, B.f[kT], S, B.partial, B.dst, c.stream), "omega");
        c.check(launch_bicg_xr_dev(c.cs, B.f[kX], R, P, S, B.f[kT], B.f[kRh], B.partial, B.dst,
                                   c.stream),
                "x, r");
      }
      h = B.get_state();
    }
    it = h.it;
    if (h.state == kBicgBreak) {
      status = EIGCG_EBREAKDOWN;
      break;
    }
    if (h.state == kBicgMaxIt) {
      status = EIGCG_ENOTCONV;
      break;
    }
    // the recursion met the tolerance (after a full or a half step): the
    // true residual decides
    B.residual(R);
    G = B.dots({R}, {R});
    if (std::sqrt(G[0].real()) <= stop) break;
    ++st.restarts;
  }
  st.iters = it;
  B.residual(R);
  G = B.dots({R}, {R});
  st.true_rel_res = std::sqrt(G[0].real()) / bnorm;
  if (status == EIGCG_OK && !(st.true_rel_res <= tol)) status = EIGCG_ENOTCONV;
  return status;
}

}  // namespace

int solve_bicgstab(Ctx& c, int nrhs, const void* b_aos, void* x_aos, double tol, int flags,
                   int max_iter, eigcg_bicgstab_stats* stats) {
  const bool g5 = (flags & EIGCG_BICG_GAMMA5) != 0;
  const bool defl = (flags & EIGCG_BICG_DEFLATE) != 0 && c.l > 0;
  const bool guess_only = (flags & EIGCG_BICG_GUESS_ONLY) != 0;
  if (max_iter <= 0) max_iter = c.P.max_iter;
  Bicg B(c, g5);
  int worst = EIGCG_OK;
  const size_t col_elems = (size_t)12 * c.g.V;
  for (int j = 0; j < nrhs; ++j) {
    const double t0 = wall_s();
    eigcg_bicgstab_stats st{};
    const double2* bsrc = (const double2*)b_aos + (size_t)j * col_elems;
    double2* xdst = (double2*)x_aos + (size_t)j * col_elems;
    c.check(launch_spinor_to_soa(bsrc, B.f[kB], kF64, &c.g, 1, c.cs, c.stream), "to soa");
    c.check(launch_spinor_to_soa(xdst, B.f[kX], kF64, &c.g, 1, c.cs, c.stream), "to soa");
    st.status = solve_column(c, B, tol, max_iter, defl, guess_only, st);
    c.check(launch_spinor_from_soa(B.f[kX], xdst, kF64, &c.g, 1, c.cs, c.stream), "from soa");
    c.check(hipStreamSynchronize(c.stream), "sync");
    st.seconds = wall_s() - t0;
    if (stats) stats[j] = st;
    if (st.status != EIGCG_OK && (worst == EIGCG_OK || st.status < worst)) worst = st.status;
  }
  return worst;
}

}  // namespace eigcg
