// extern "C" boundary of libeigcg.so: argument validation, error codes and
// exception translation around the engine (engine.cpp) and the host linear
// algebra (hostla.cpp).
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "engine.h"
#include "hostla.h"

using eigcg::ApiError;
using eigcg::Ctx;
using eigcg::HipError;


namespace {

int fail(eigcg_ctx* ctx, int code, const std::string& msg) {
  if (ctx) {
    ctx->c.err = msg;
    if (code == EIGCG_EHIP) ctx->c.sticky = 1;
  }
  return code;
}

// message of this thread's last failed eigcg_create (no context to hold it)
std::string& create_error() {
  static thread_local std::string e = "no context";
  return e;
}

template <typename F> int guarded(eigcg_ctx* ctx, F&& f) {
  if (ctx && ctx->c.sticky) return fail(ctx, EIGCG_EHIP, "context unusable after a HIP error");
  try {
    return f();
  } catch (const HipError& e) {
    (void)hipGetLastError();
    return fail(ctx, EIGCG_EHIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const ApiError& e) {
    return fail(ctx, e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(ctx, EIGCG_ENOMEM, "host allocation failed");
  }
}

int validate(const eigcg_params* p, std::string& why) {
  if (!p) { why = "null params"; return EIGCG_EINVAL; }
  long long V = 1;
  for (int i = 0; i < 4; ++i) {
    if (p->dims[i] < 2 || p->dims[i] > 4096) { why = "lattice extent out of range"; return EIGCG_EINVAL; }
    V *= p->dims[i];
  }
  if (V * 12 * 16 > (1ll << 40) || V >= (1ll << 30)) { why = "lattice too large"; return EIGCG_EINVAL; }
  if (!std::isfinite(p->mass)) { why = "mass not finite"; return EIGCG_EINVAL; }
  if (!(p->m > 2 * p->nev && p->nev >= 1)) { why = "eigCG needs m > 2 nev >= 2"; return EIGCG_EINVAL; }
  if ((long long)p->m * 2 * p->nev > 4096 || p->nev > 32 || p->m > 256) {
    why = "window too large (m * 2 nev <= 4096, nev <= 32, m <= 256)";
    return EIGCG_EINVAL;
  }
  if (p->max_bank < 0 || p->max_bank > 256) { why = "max_bank must be in [0, 256]"; return EIGCG_EINVAL; }
  if (p->precision != EIGCG_FP64 && p->precision != EIGCG_MIXED_FP32 &&
      p->precision != EIGCG_MIXED_HALF) { why = "bad precision"; return EIGCG_EINVAL; }
  if (p->max_batch < 1 || p->max_batch > 12) { why = "max_batch must be in [1, 12]"; return EIGCG_EINVAL; }
  if (p->max_iter < 1 || p->max_iter > 10000000) { why = "bad max_iter"; return EIGCG_EINVAL; }
  if (p->check_every < 1) { why = "check_every must be >= 1"; return EIGCG_EINVAL; }
  if (p->stencil_variant < 0 || p->stencil_variant > eigcg::kStencilVariants) { why = "stencil_variant out of range"; return EIGCG_EINVAL; }
  if (p->plane_pad > 4096) { why = "plane_pad too large"; return EIGCG_EINVAL; }
  if (p->sample_every < 0) { why = "sample_every must be >= 0"; return EIGCG_EINVAL; }
  if (p->schur != 0 && p->schur != 1) { why = "schur must be 0 or 1"; return EIGCG_EINVAL; }
  if (p->schur && (p->dims[0] % 2 || p->dims[1] % 2 || p->dims[2] % 2 || p->dims[3] % 2)) {
    why = "odd-even preconditioning needs every lattice extent even";
    return EIGCG_EINVAL;
  }
  if (p->precision == EIGCG_MIXED_FP32 && p->reliable_every < 1) { why = "reliable_every must be >= 1"; return EIGCG_EINVAL; }
  if (p->precond != EIGCG_PRECOND_NONE && p->precond != EIGCG_PRECOND_SPECTRAL) { why = "bad precond"; return EIGCG_EINVAL; }
  if (p->precond == EIGCG_PRECOND_SPECTRAL && p->precision != EIGCG_FP64) {
    why = "the spectral preconditioner runs in FP64 contexts only";
    return EIGCG_EINVAL;
  }
  if (!std::isfinite(p->precond_sigma)) { why = "precond_sigma not finite"; return EIGCG_EINVAL; }
  if (p->restart_rule != EIGCG_RESTART_FIXED && p->restart_rule != EIGCG_RESTART_DYNAMIC) {
    why = "bad restart_rule";
    return EIGCG_EINVAL;
  }
  if (!std::isfinite(p->restart_cost)) { why = "restart_cost not finite"; return EIGCG_EINVAL; }
  if (!std::isfinite(p->restart_tol)) { why = "restart_tol not finite"; return EIGCG_EINVAL; }
  return EIGCG_OK;
}

}  // namespace

extern "C" {

int eigcg_default_params(eigcg_params* p) {
  if (!p) return EIGCG_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->dims[0] = p->dims[1] = p->dims[2] = p->dims[3] = 4;
  p->mass = 0.0;
  p->nev = 10;
  p->m = 100;
  p->max_bank = 240;
  p->precision = EIGCG_FP64;
  p->max_batch = 1;
  p->reliable_every = 50;
  p->max_iter = 20000;
  p->restart_tol = 0.0;
  p->hbm_budget = 0;
  p->compress_links = 1;
  p->check_every = 16;
  p->use_graphs = 0;
  p->stencil_variant = 0;
  p->plane_pad = 0;
  p->sample_every = 0;
  return EIGCG_OK;
}

int eigcg_create(const eigcg_params* p, const void* gauge_dev, void* hip_stream, eigcg_ctx** out) {
  if (!out) return EIGCG_EINVAL;
  *out = nullptr;
  std::string why;
  int v = validate(p, why);
  if (v != EIGCG_OK) {
    create_error() = why;
    return v;
  }
  if (!gauge_dev) {
    create_error() = "null gauge field";
    return EIGCG_EINVAL;
  }
  eigcg_ctx* ctx = new (std::nothrow) eigcg_ctx();
  if (!ctx) return EIGCG_ENOMEM;
  int rc = guarded(ctx, [&] {
    eigcg::ctx_init(ctx->c, *p, gauge_dev, (hipStream_t)hip_stream);
    return EIGCG_OK;
  });
  if (rc != EIGCG_OK) {
    create_error() = ctx->c.err;
    eigcg::ctx_release(ctx->c);
    delete ctx;
    return rc;
  }
  *out = ctx;
  return EIGCG_OK;
}

int eigcg_destroy(eigcg_ctx* ctx) {
  if (!ctx) return EIGCG_EINVAL;
  eigcg::ctx_release(ctx->c);
  delete ctx;
  return EIGCG_OK;
}

int eigcg_solve(eigcg_ctx* ctx, int32_t nrhs, const void* b_dev, void* x_dev, double tol,
                int32_t mode, eigcg_stats* stats) {
  if (!ctx) return EIGCG_EINVAL;
  if (nrhs < 0 || (nrhs > 0 && (!b_dev || !x_dev)))
    return fail(ctx, EIGCG_EINVAL, "bad right-hand side arguments");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(ctx, EIGCG_EINVAL, "tol must be > 0");
  if (mode < EIGCG_MODE_CG || mode > EIGCG_MODE_AUTO) return fail(ctx, EIGCG_EINVAL, "bad mode");
  if (nrhs == 0) return EIGCG_OK;
  return guarded(ctx, [&] { return eigcg::solve(ctx->c, nrhs, b_dev, x_dev, tol, mode, stats); });
}

int eigcg_deflate_init(eigcg_ctx* ctx, int32_t nrhs, const void* b_dev, void* x_dev) {
  if (!ctx) return EIGCG_EINVAL;
  if (nrhs < 0 || (nrhs > 0 && (!b_dev || !x_dev)))
    return fail(ctx, EIGCG_EINVAL, "bad arguments");
  if (nrhs == 0) return EIGCG_OK;
  return guarded(ctx, [&] {
    eigcg::deflate_init(ctx->c, nrhs, b_dev, x_dev);
    return EIGCG_OK;
  });
}

int eigcg_solve_bicgstab(eigcg_ctx* ctx, int32_t nrhs, const void* b_dev, void* x_dev,
                         double tol, int32_t flags, int32_t max_iter,
                         eigcg_bicgstab_stats* stats) {
  if (!ctx) return EIGCG_EINVAL;
  if (nrhs < 0 || (nrhs > 0 && (!b_dev || !x_dev)))
    return fail(ctx, EIGCG_EINVAL, "bad right-hand side arguments");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(ctx, EIGCG_EINVAL, "tol must be > 0");
  if (flags & ~(EIGCG_BICG_GAMMA5 | EIGCG_BICG_DEFLATE | EIGCG_BICG_GUESS_ONLY))
    return fail(ctx, EIGCG_EINVAL, "bad flags");
  if (nrhs == 0) return EIGCG_OK;
  return guarded(ctx, [&] {
    return eigcg::solve_bicgstab(ctx->c, nrhs, b_dev, x_dev, tol, flags, max_iter, stats);
  });
}

int eigcg_apply(eigcg_ctx* ctx, int32_t op, int32_t nrhs, const void* in_dev, void* out_dev) {
  if (!ctx) return EIGCG_EINVAL;
  if (op < EIGCG_OP_M || op > EIGCG_OP_A + 3) return fail(ctx, EIGCG_EINVAL, "bad op");
  if (nrhs < 0 || (nrhs > 0 && (!in_dev || !out_dev))) return fail(ctx, EIGCG_EINVAL, "bad arguments");
  if (nrhs == 0) return EIGCG_OK;
  return guarded(ctx, [&] {
    eigcg::apply_op(ctx->c, op, nrhs, in_dev, out_dev);
    return EIGCG_OK;
  });
}

int eigcg_apply_noalloc(eigcg_ctx* ctx, int32_t op, int32_t nrhs, const void* in_dev,
                        void* out_dev) {
  if (!ctx) return EIGCG_EINVAL;
  if (op < EIGCG_OP_M || op > EIGCG_OP_A) return fail(ctx, EIGCG_EINVAL, "bad op");
  if (nrhs < 0 || (nrhs > 0 && (!in_dev || !out_dev))) return fail(ctx, EIGCG_EINVAL, "bad arguments");
  if (nrhs == 0) return EIGCG_OK;
  return guarded(ctx, [&] {
    eigcg::apply_op_noalloc(ctx->c, op, nrhs, in_dev, out_dev);
    return EIGCG_OK;
  });
}

int eigcg_noalloc_scratch_bytes(uint64_t* bytes) {
  if (!bytes) return EIGCG_EINVAL;
  *bytes = eigcg::noalloc_scratch_bytes();
  return EIGCG_OK;
}

int eigcg_schur_rhs(eigcg_ctx* ctx, int32_t nrhs, const void* b_full_dev, void* rhs_dev) {
  if (!ctx) return EIGCG_EINVAL;
  if (!ctx->c.g.eo) return fail(ctx, EIGCG_EINVAL, "context is not odd-even preconditioned");
  if (nrhs < 0 || (nrhs > 0 && (!b_full_dev || !rhs_dev))) return fail(ctx, EIGCG_EINVAL, "bad arguments");
  if (nrhs == 0) return EIGCG_OK;
  return guarded(ctx, [&] {
    eigcg::schur_rhs(ctx->c, nrhs, b_full_dev, rhs_dev);
    return EIGCG_OK;
  });
}

int eigcg_schur_reconstruct(eigcg_ctx* ctx, int32_t nrhs, const void* b_full_dev,
                            const void* x_even_dev, void* x_full_dev) {
  if (!ctx) return EIGCG_EINVAL;
  if (!ctx->c.g.eo) return fail(ctx, EIGCG_EINVAL, "context is not odd-even preconditioned");
  if (nrhs < 0 || (nrhs > 0 && (!b_full_dev || !x_even_dev || !x_full_dev)))
    return fail(ctx, EIGCG_EINVAL, "bad arguments");
  if (nrhs == 0) return EIGCG_OK;
  return guarded(ctx, [&] {
    eigcg::schur_reconstruct(ctx->c, nrhs, b_full_dev, x_even_dev, x_full_dev);
    return EIGCG_OK;
  });
}

int eigcg_bank_info(eigcg_ctx* ctx, int32_t* l, double* ritz_vals, double* ritz_res) {
  if (!ctx || !l) return EIGCG_EINVAL;
  return guarded(ctx, [&] {
    int ll = 0;
    eigcg::bank_info(ctx->c, &ll, ritz_vals, ritz_res);
    *l = ll;
    return EIGCG_OK;
  });
}

int eigcg_bank_vectors(eigcg_ctx* ctx, int32_t first, int32_t count, void* out_dev) {
  if (!ctx) return EIGCG_EINVAL;
  if (first < 0 || count < 0 || first + count > ctx->c.l || (count > 0 && !out_dev))
    return fail(ctx, EIGCG_EINVAL, "bank range out of bounds");
  return guarded(ctx, [&] {
    eigcg::bank_vectors(ctx->c, first, count, out_dev);
    return EIGCG_OK;
  });
}

int eigcg_bank_load(eigcg_ctx* ctx, int32_t count, const void* vecs_dev, int32_t* added) {
  if (!ctx || count < 0 || (count > 0 && !vecs_dev)) return EIGCG_EINVAL;
  return guarded(ctx, [&] {
    int a = eigcg::bank_load(ctx->c, count, vecs_dev);
    if (added) *added = a;
    return EIGCG_OK;
  });
}

int eigcg_bank_matrix(eigcg_ctx* ctx, double* h_host) {
  if (!ctx || !h_host) return EIGCG_EINVAL;
  const int l = ctx->c.l, ld = ctx->c.P.max_bank;
  for (int j = 0; j < l; ++j)
    for (int i = 0; i < l; ++i) {
      const auto v = ctx->c.H[(size_t)j * ld + i];
      h_host[2 * ((size_t)j * l + i)] = v.real();
      h_host[2 * ((size_t)j * l + i) + 1] = v.imag();
    }
  return EIGCG_OK;
}

int eigcg_last_ritz(eigcg_ctx* ctx, double* vals, int32_t cap, int32_t* count) {
  if (!ctx || !count || cap < 0 || (cap > 0 && !vals)) return EIGCG_EINVAL;
  const int n = std::min<int>(cap, (int)ctx->c.last_ritz.size());
  for (int i = 0; i < n; ++i) vals[i] = ctx->c.last_ritz[i];
  *count = n;
  return EIGCG_OK;
}

int eigcg_bank_truncate(eigcg_ctx* ctx, int32_t k) {
  if (!ctx) return EIGCG_EINVAL;
  if (k < 0) return fail(ctx, EIGCG_EINVAL, "negative bank size");
  return guarded(ctx, [&] {
    eigcg::bank_truncate(ctx->c, k);
    return EIGCG_OK;
  });
}

int eigcg_bank_lock(eigcg_ctx* ctx, double tol, int32_t* nlocked) {
  if (!ctx) return EIGCG_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol))
    return fail(ctx, EIGCG_EINVAL, "lock tolerance must be finite and >= 0");
  return guarded(ctx, [&] {
    const int n = eigcg::bank_lock(ctx->c, tol);
    if (nlocked) *nlocked = n;
    return EIGCG_OK;
  });
}

int eigcg_bank_locked(eigcg_ctx* ctx) {
  if (!ctx) return EIGCG_EINVAL;
  return ctx->c.nlock;
}

int eigcg_bank_restore(eigcg_ctx* ctx, int32_t l, const void* vecs_dev, const double* h_host) {
  if (!ctx) return EIGCG_EINVAL;
  if (l < 0 || (l > 0 && (!vecs_dev || !h_host))) return fail(ctx, EIGCG_EINVAL, "bad arguments");
  return guarded(ctx, [&] {
    eigcg::bank_restore(ctx->c, l, vecs_dev, h_host);
    return EIGCG_OK;
  });
}

int eigcg_bank_reset(eigcg_ctx* ctx) {
  if (!ctx) return EIGCG_EINVAL;
  ctx->c.l = 0;
  ctx->c.nlock = 0;
  ctx->c.chol_ok = false;
  ctx->c.spec_ok = false;
  ++ctx->c.bank_gen;
  return EIGCG_OK;
}

int eigcg_memory(eigcg_ctx* ctx, uint64_t* bytes) {
  if (!ctx || !bytes) return EIGCG_EINVAL;
  *bytes = ctx->c.bytes;
  return EIGCG_OK;
}

int eigcg_debug_span(int32_t op, uint64_t addr, uint64_t bytes) {
  const void* p = reinterpret_cast<const void*>((uintptr_t)addr);
  if (op == 0) {
    if (!addr || !bytes) return EIGCG_EINVAL;
    eigcg::register_span(p, (size_t)bytes);
    return EIGCG_OK;
  }
  if (op == 1) return eigcg::unregister_span(p) ? EIGCG_OK : EIGCG_EINVAL;
  if (op == 2) return eigcg::span_fits(p, (size_t)bytes) ? EIGCG_OK : EIGCG_EINVAL;
  return EIGCG_EINVAL;
}

int eigcg_tune_cache_reset(void) {
  eigcg::tune_cache_reset();
  return EIGCG_OK;
}

int eigcg_layout_info(eigcg_ctx* ctx, int32_t* info) {
  if (!ctx || !info) return EIGCG_EINVAL;
  info[0] = ctx->c.g.V;
  info[1] = ctx->c.g.vs;
  info[2] = ctx->c.comp64;
  info[3] = ctx->c.comp32;
  info[4] = ctx->c.var64;
  info[5] = ctx->c.var32;
  info[6] = ctx->c.nc64;
  info[7] = ctx->c.nc32;
  return EIGCG_OK;
}

int eigcg_tune_report(eigcg_ctx* ctx, double* tune_ms) {
  if (!ctx || !tune_ms) return EIGCG_EINVAL;
  for (int i = 0; i < 2 * eigcg::kStencilVariants; ++i) tune_ms[i] = ctx->c.tune_ms[i];
  return EIGCG_OK;
}

int eigcg_time_kernel(eigcg_ctx* ctx, int32_t what, int32_t reps, double* ms) {
  if (!ctx || !ms || reps < 1 || what < 0 || what > 3) return EIGCG_EINVAL;
  return guarded(ctx, [&] {
    *ms = eigcg::bench_kernels(ctx->c, what, reps);
    return EIGCG_OK;
  });
}

int eigcg_kernel_samples(eigcg_ctx* ctx, int32_t reset, double* out) {
  if (!ctx || !out) return EIGCG_EINVAL;
  return guarded(ctx, [&] {
    eigcg::kernel_samples(ctx->c, reset != 0, out);
    return EIGCG_OK;
  });
}

const char* eigcg_last_error(const eigcg_ctx* ctx) {
  if (!ctx) return create_error().c_str();
  return ctx->c.err.c_str();
}

// ---- device kernel probes (test support) ---------------------------------------

int eigcg_debug_mfma_probe(double* out_dev) {
  if (!out_dev) return EIGCG_EINVAL;
  if (eigcg::launch_mfma_probe(out_dev, nullptr) != hipSuccess) return EIGCG_EHIP;
  return hipDeviceSynchronize() == hipSuccess ? EIGCG_OK : EIGCG_EHIP;
}

int eigcg_debug_gemm(int32_t prec, int32_t kind, uint64_t n, int32_t K, int32_t N,
                     const void* in_dev, const void* r_dev, const double* s_dev, void* out_dev,
                     double* scratch_dev, uint64_t scratch_elems) {
  if (K <= 0 || N <= 0 || K > 256 || N > 24 || !in_dev || !out_dev || n == 0) return EIGCG_EINVAL;
  const size_t eb = prec == 0 ? 16 : 8;
  std::vector<const void*> in(K);
  for (int i = 0; i < K; ++i) in[i] = (const char*)in_dev + (size_t)i * n * eb;
  hipError_t e;
  if (kind == 0 || kind == 2 || kind == 3) {  // out (n x N) (+-)= in (n x K) * S (K x N)
    if (!s_dev) return EIGCG_EINVAL;
    std::vector<void*> out(N);
    for (int j = 0; j < N; ++j) out[j] = (char*)out_dev + (size_t)j * n * eb;
    e = eigcg::launch_gemm_tall(prec == 0 ? eigcg::kF64 : eigcg::kF32, n, K, N, in.data(),
                                out.data(), (const double2*)s_dev, kind != 0, kind == 3, nullptr);
  } else if (kind == 1) {  // out (K x N complex FP64) = in^H r
    if (!r_dev || N > 16 || !scratch_dev) return EIGCG_EINVAL;
    std::vector<const void*> rc(N);
    for (int j = 0; j < N; ++j) rc[j] = (const char*)r_dev + (size_t)j * n * eb;
    e = eigcg::launch_gemm_reduce(prec == 0 ? eigcg::kF64 : eigcg::kF32, n, K, N, in.data(),
                                  rc.data(), (double2*)scratch_dev, scratch_elems / 2,
                                  (double2*)out_dev, nullptr);
  } else {
    return EIGCG_EINVAL;
  }
  if (e != hipSuccess) return EIGCG_EHIP;
  return hipDeviceSynchronize() == hipSuccess ? EIGCG_OK : EIGCG_EHIP;
}

// ---- host linear algebra exports (test support) ------------------------------

int eigcg_host_eig_lowest(int32_t n, const double* a, int32_t k, double* w, double* z) {
  if (n <= 0 || k < 0 || k > n || !a || !w || (k > 0 && !z)) return EIGCG_EINVAL;
  const auto* A = reinterpret_cast<const eigcg::hostla::cplx*>(a);
  auto* Z = reinterpret_cast<eigcg::hostla::cplx*>(z);
  return eigcg::hostla::herm_eig_lowest(n, A, n, k, w, Z, n) == 0 ? EIGCG_OK : EIGCG_EBREAKDOWN;
}

int eigcg_host_qr(int32_t m, int32_t n, const double* a, double* q, double* r) {
  if (m <= 0 || n <= 0 || n > m || !a || !q) return EIGCG_EINVAL;
  eigcg::hostla::qr_thin(m, n, reinterpret_cast<const eigcg::hostla::cplx*>(a), m,
                         reinterpret_cast<eigcg::hostla::cplx*>(q), m,
                         reinterpret_cast<eigcg::hostla::cplx*>(r), n);
  return EIGCG_OK;
}

int eigcg_host_chol_solve(int32_t n, const double* h, int32_t nrhs, double* b) {
  if (n <= 0 || nrhs < 0 || !h || (nrhs > 0 && !b)) return EIGCG_EINVAL;
  std::vector<eigcg::hostla::cplx> L(reinterpret_cast<const eigcg::hostla::cplx*>(h),
                                     reinterpret_cast<const eigcg::hostla::cplx*>(h) + (size_t)n * n);
  if (eigcg::hostla::cholesky(n, L.data(), n) != 0) return EIGCG_EBREAKDOWN;
  eigcg::hostla::cholesky_solve(n, L.data(), n, nrhs, reinterpret_cast<eigcg::hostla::cplx*>(b), n);
  return EIGCG_OK;
}

int eigcg_host_auto_continue(int32_t done, int32_t left, const double* iters, const double* secs,
                             double iter_ms, int32_t bank_room) {
  if (done < 0 || (done > 0 && (!iters || !secs))) return EIGCG_EINVAL;
  return eigcg::auto_continue(done, left, iters, secs, iter_ms, bank_room) ? 1 : 0;
}

int eigcg_restart_model(int32_t l, const double* theta, const double* res, double lambda_max,
                        double tol, double restart_cost, double* out) {
  if (l < 0 || !out || (l > 0 && (!theta || !res))) return EIGCG_EINVAL;
  if (!(lambda_max > 0.0) || !std::isfinite(lambda_max) || !(tol > 0.0) || !(tol < 1.0) ||
      !std::isfinite(restart_cost))
    return EIGCG_EINVAL;
  for (int i = 0; i < l; ++i) {
    if (!std::isfinite(theta[i]) || !std::isfinite(res[i]) || res[i] < 0.0) return EIGCG_EINVAL;
    if (!(theta[i] > 0.0) || (i > 0 && theta[i] < theta[i - 1])) return EIGCG_EINVAL;
  }
  const eigcg::RestartPick r = eigcg::restart_model(l, theta, res, lambda_max, tol, restart_cost);
  out[0] = r.tau;
  out[1] = r.cost_none;
  out[2] = r.cost_with;
  return EIGCG_OK;
}

}  // extern "C"
