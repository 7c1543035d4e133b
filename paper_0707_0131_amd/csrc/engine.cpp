// Solver engine: context set-up, batched CG / eigCG / init-CG drivers and the
// Incremental eigCG bank (Figure 3.1, eq. (2.1) and Section 4 of the paper).
//
// Execution model.  The CG scalars live on the device (ColState); a CG
// iteration is three kernels (stencil M with ||M p||^2 -> alpha; stencil M^H
// fused with r -= alpha t and r^H r -> beta and the stop test; x/p update with
// the eigCG window append), so the host never waits inside the iteration.  The
// host enqueues segments of iterations, each followed by an asynchronous copy
// of the column states (and of the alpha/beta history for eigCG) and an event,
// and processes segment s while segment s+1 already runs.  eigCG restarts fall
// on segment ends: the host builds the window matrix T from the history,
// computes the restart coefficients in FP64 (eq. (2.3)), uploads QZ and
// enqueues the MFMA product V <- V (QZ) while the GPU keeps iterating; the
// window is a ring of residual slots large enough for that lag.  The arrow
// row w^H V uses t saved by the device on a schedule it advances itself.
#include "engine.h"

#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

#include "hostla.h"

namespace eigcg {

namespace {

// Registry of the library's device allocations (base address -> bytes),
// shared by every thread and context: the byte accounting of dfree and the
// host-side bounds checks below read it.
struct AllocRegistry {
  std::mutex mu;
  std::map<uintptr_t, size_t> m;
};
AllocRegistry& allocs() {
  static AllocRegistry r;
  return r;
}

size_t round_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Partition of the small-matrix staging area (d_small / h_small, 2^17
// complex entries): per-column restart coefficients QZ, per-column arrow rows,
// and a generic region for synchronous products.
constexpr size_t kSmallElems = (size_t)1 << 17;
constexpr size_t kQzSlot = kSmallElems / 2 / kMaxCols;  // m * 2 nev <= 4096
inline size_t qz_off(int col) { return (size_t)col * kQzSlot; }
inline size_t arrow_off(int col) { return kSmallElems / 2 + (size_t)col * 64; }
constexpr size_t kGenericOff = kSmallElems * 3 / 4;

}  // namespace

void Ctx::check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{e, what};
}

void* Ctx::dalloc(size_t n) {
  n = round_up(n, 256);
  if (P.hbm_budget && bytes + n > P.hbm_budget)
    throw ApiError{EIGCG_ENOMEM, "HBM budget of the context exceeded"};
  void* p = nullptr;
  if (hipMalloc(&p, n) != hipSuccess) {
    (void)hipGetLastError();
    throw ApiError{EIGCG_ENOMEM, "hipMalloc failed"};
  }
  check(hipMemsetAsync(p, 0, n, stream), "hipMemsetAsync");
  bytes += n;
  register_span(p, n);
  return p;
}

void Ctx::dfree(void*& p) {
  if (!p) return;
  const size_t n = unregister_span(p);
  bytes -= std::min(bytes, n);
  (void)hipFree(p);
  p = nullptr;
}

void register_span(const void* base, size_t bytes) {
  AllocRegistry& r = allocs();
  std::lock_guard<std::mutex> lk(r.mu);
  r.m[(uintptr_t)base] = bytes;
}

size_t unregister_span(const void* base) {
  AllocRegistry& r = allocs();
  std::lock_guard<std::mutex> lk(r.mu);
  auto it = r.m.find((uintptr_t)base);
  if (it == r.m.end()) return 0;
  const size_t n = it->second;
  r.m.erase(it);
  return n;
}

// Host-side bounds check of a device access: when p lies inside one of the
// library's allocations, [p, p + bytes) must end inside it.  Pointers outside
// every allocation (the caller's tensors) are not the library's to check.
bool span_fits(const void* p, size_t bytes) {
  AllocRegistry& r = allocs();
  std::lock_guard<std::mutex> lk(r.mu);
  const uintptr_t a = (uintptr_t)p;
  auto it = r.m.upper_bound(a);
  if (it == r.m.begin()) return true;
  --it;
  const uintptr_t end = it->first + it->second;
  if (a >= end) return true;
  return bytes <= end - a;
}

void check_span(const void* p, size_t bytes, const char* what) {
  if (!span_fits(p, bytes))
    throw ApiError{EIGCG_EINVAL, std::string("internal: ") + what +
                                     " reaches past the end of its device allocation"};
}

static size_t elem_bytes(int prec) { return prec == kF64 ? 16 : (prec == kF32 ? 8 : 4); }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

static void ws_ensure(Ctx& c, Workspace& w, int prec, bool eig, int keig = 0);
static StencilLaunch stencil_base(Ctx& c, int prec);
static void bank_ritz_residuals(Ctx& c, int j0, int n, const std::vector<double>& th,
                                const std::vector<cplx>& Y, double* res);

// Stencil autotuner: times every kernel variant (the search space: site
// mapping and sweep order, workgroups per CU, z-march chunking) and, for the
// two-tile variants, every number of columns per workgroup, on this lattice
// at the context's batch width, and keeps the fastest.  The choice is cached
// per (lattice shape, plane stride, geometry, precision, link storage, batch
// width) for the process and persisted in a file keyed by the device and the
// library build, so later processes skip the timing.  Variants differ in
// summation order at the rounding level; columns per workgroup do not change
// any column's arithmetic.  A forced variant in the parameters wins (with
// the widest column grouping).
namespace {

struct TunePick {
  std::vector<double> ms;  // best time per variant
  int var, nc;
};

std::mutex g_tune_mu;
std::map<std::vector<int>, TunePick> g_tune;  // this process's choices

// File of persisted choices: EIGCG_TUNE_CACHE (empty or "off": none), else
// $XDG_CACHE_HOME/eigcg/stencil_tune.txt or ~/.cache/eigcg/stencil_tune.txt.
std::string tune_cache_path() {
  const char* e = std::getenv("EIGCG_TUNE_CACHE");
  if (e) return (*e == 0 || std::strcmp(e, "off") == 0) ? std::string() : std::string(e);
  const char* x = std::getenv("XDG_CACHE_HOME");
  const char* h = std::getenv("HOME");
  std::string dir;
  if (x && *x) dir = std::string(x);
  else if (h && *h) dir = std::string(h) + "/.cache";
  else return std::string();
  (void)mkdir(dir.c_str(), 0755);
  dir += "/eigcg";
  (void)mkdir(dir.c_str(), 0755);
  return dir + "/stencil_tune.txt";
}

// The device and this build of the kernels: a persisted choice is used only
// by the same library build on the same kind of device.
std::string tune_tag(int device) {
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char& ch : arch)
    if (ch == ' ' || ch == ':') ch = '_';
  std::string build = __DATE__ "_" __TIME__;
  for (char& ch : build)
    if (ch == ' ' || ch == ':') ch = '_';
  return arch + "/" + std::to_string(cus) + "cu/v" + std::to_string(kStencilVariants) + "/" + build;
}

std::string tune_line_key(const std::string& tag, const std::vector<int>& key) {
  std::string k = tag;
  for (int v : key) k += " " + std::to_string(v);
  return k;
}

bool tune_file_lookup(const std::string& path, const std::string& lk, TunePick& pk) {
  if (path.empty()) return false;
  std::FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char buf[2048];
  bool found = false;
  while (std::fgets(buf, sizeof(buf), f)) {  // the last matching line wins
    std::string line(buf);
    const size_t sep = line.find(" : ");
    if (sep == std::string::npos || line.substr(0, sep) != lk) continue;
    std::vector<double> vals;
    const char* q = line.c_str() + sep + 3;
    char* end = nullptr;
    for (;;) {
      const double v = std::strtod(q, &end);
      if (end == q) break;
      vals.push_back(v);
      q = end;
    }
    if ((int)vals.size() != 2 + kStencilVariants) continue;
    const int var = (int)vals[0];
    if (var < 1 || var > kStencilVariants) continue;
    pk.var = var;
    pk.nc = (int)vals[1];
    pk.ms.assign(vals.begin() + 2, vals.end());
    found = true;
  }
  std::fclose(f);
  return found;
}

void tune_file_append(const std::string& path, const std::string& lk, const TunePick& pk) {
  if (path.empty()) return;
  std::string line = lk + " : " + std::to_string(pk.var) + " " + std::to_string(pk.nc);
  char num[64];
  for (double v : pk.ms) {
    std::snprintf(num, sizeof(num), " %.6g", v);
    line += num;
  }
  line += "\n";
  std::FILE* f = std::fopen(path.c_str(), "a");  // one short append per choice
  if (!f) return;
  std::fputs(line.c_str(), f);
  std::fclose(f);
}

}  // namespace

void tune_cache_reset() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

static void autotune_stencil(Ctx& c, int prec) {
  using Pick = TunePick;
  std::mutex& mu = g_tune_mu;
  auto& cache = g_tune;
  int& var = prec == kF64 ? c.var64 : c.var32;
  int& ncs = prec == kF64 ? c.nc64 : c.nc32;
  double* tms = c.tune_ms + (prec == kF64 ? 0 : kStencilVariants);
  if (c.P.stencil_variant > 0) {
    var = c.P.stencil_variant;
    ncs = 0;
    return;
  }
  const std::vector<int> key = {c.g.L[0], c.g.L[1], c.g.L[2], c.g.L[3], c.g.vs, c.g.eo, prec,
                                prec == kF64 ? c.comp64 : c.comp32, c.P.max_batch};
  auto apply = [&](const Pick& pk) {
    for (int v = 1; v <= kStencilVariants; ++v) tms[v - 1] = pk.ms[v - 1];
    var = pk.var;
    ncs = pk.nc;
  };
  const std::string path = tune_cache_path();
  const std::string lkey = tune_line_key(tune_tag(c.device), key);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
      Pick pf;
      if (tune_file_lookup(path, lkey, pf)) it = cache.emplace(key, pf).first;
    }
    if (it != cache.end()) {
      apply(it->second);
      return;
    }
  }
  // Each candidate runs the two passes of a CG iteration with their memory
  // traffic: M p -> t with the partial-sum epilogue, then M^H t against a
  // right-hand side with the residual epilogue (reads b, writes r), on the
  // context's scratch vectors and state slots, for a full batch of
  // max_batch columns (the width the solver launches).
  Workspace& w = prec == kF64 ? c.ws64 : c.ws32;
  ws_ensure(c, w, prec, false);
  hipEvent_t e0, e1;
  c.check(hipEventCreate(&e0), "ev");
  c.check(hipEventCreate(&e1), "ev");
  Pick pk;
  pk.ms.assign(kStencilVariants, 0.0);
  pk.var = 1;
  pk.nc = 0;
  double best = 1e300;
  const int ncmax = (w.K >= 4 && prec != kF64) ? 4 : (w.K >= 2 ? 2 : 1);
  for (int v = c.g.eo ? 3 : 1; v <= kStencilVariants; ++v) {  // odd-even runs 1, 2 as 3
    if (c.g.eo && v >= 11 && v <= 13) continue;  // the z-march needs the full geometry
    for (int nc = 1; nc <= ncmax; nc *= 2) {
      if ((v < 3 || (v >= 11 && v <= 13)) && nc > 1) break;
      StencilLaunch L1 = stencil_base(c, prec);
      L1.variant = v;
      L1.nc = nc;
      L1.op = kOpM;
      L1.epi = kEpiNorm;
      L1.in = w.b; L1.in_cs = c.cs;
      L1.out = w.tmp; L1.out_cs = c.cs;
      L1.ncols = w.K;
      L1.mask = w.K >= 32 ? 0xffffffffu : ((1u << w.K) - 1u);
      StencilLaunch L2 = L1;
      L2.op = kOpMdag;
      L2.epi = kEpiRes;
      L2.in = w.tmp;
      L2.b = w.p; L2.b_cs = c.cs;
      L2.r = w.r; L2.r_cs = c.cs;
      auto pair = [&]() {
        c.check(launch_stencil(L1, c.stream), "tune");
        c.check(launch_stencil(L2, c.stream), "tune");
      };
      for (int i = 0; i < 2; ++i) pair();
      const int reps = 8;
      c.check(hipEventRecord(e0, c.stream), "ev");
      for (int i = 0; i < reps; ++i) pair();
      c.check(hipEventRecord(e1, c.stream), "ev");
      c.check(hipEventSynchronize(e1), "ev");
      float ms = 0.f;
      c.check(hipEventElapsedTime(&ms, e0, e1), "ev");
      const double t = (double)ms / reps;
      if (pk.ms[v - 1] == 0.0 || t < pk.ms[v - 1]) pk.ms[v - 1] = t;
      if (t < best) {
        best = t;
        pk.var = v;
        pk.nc = nc;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (void* v : {w.tmp, w.r}) c.check(hipMemsetAsync(v, 0, c.cs * elem_bytes(prec) * w.K, c.stream), "clear");
  c.check(hipStreamSynchronize(c.stream), "sync");
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it == cache.end()) {
    it = cache.emplace(key, pk).first;
    tune_file_append(path, lkey, pk);
  }
  apply(it->second);
}

void ctx_init(Ctx& c, const eigcg_params& p, const void* gauge_dev, hipStream_t s) {
  c.P = p;
  c.stream = s;
  c.check(hipGetDevice(&c.device), "hipGetDevice");
  Geom& g = c.g;
  for (int i = 0; i < 4; ++i) g.L[i] = p.dims[i];
  g.Vfull = p.dims[0] * p.dims[1] * p.dims[2] * p.dims[3];
  // odd-even preconditioning: the solver's vectors live on the even sites
  g.eo = p.schur ? 1 : 0;
  g.V = g.eo ? g.Vfull / 2 : g.Vfull;
  g.dxh = FastDiv((uint32_t)std::max(1, p.dims[0] / 2));
  // plane stride: V rounded up to 64 sites, plus an odd number of 64-site
  // blocks by default so that the 12 spinor planes and the link planes of a
  // site start on different memory channels
  const int pad = p.plane_pad < 0 ? 0 : (p.plane_pad == 0 ? 1 : p.plane_pad);
  g.vs = (int)round_up((size_t)g.V, 64) + 64 * pad;
  g.stride[0] = 1;
  g.stride[1] = p.dims[0];
  g.stride[2] = p.dims[0] * p.dims[1];
  g.stride[3] = p.dims[0] * p.dims[1] * p.dims[2];
  g.dx = FastDiv((uint32_t)p.dims[0]);
  g.dy = FastDiv((uint32_t)p.dims[1]);
  g.dz = FastDiv((uint32_t)p.dims[2]);
  c.cs = (size_t)12 * g.vs;

  // scratch
  c.hist_stride = 3 * (p.max_iter + 8);
  c.d_st = (ColState*)c.dalloc(sizeof(ColState) * kMaxCols);
  c.check(hipHostMalloc((void**)&c.h_st, sizeof(ColState) * kMaxCols * 4, 0), "hipHostMalloc");
  c.d_hist = (double*)c.dalloc(sizeof(double) * (size_t)kMaxCols * c.hist_stride);
  c.check(hipHostMalloc((void**)&c.h_hist, sizeof(double) * (size_t)kMaxCols * c.hist_stride, 0),
          "hipHostMalloc");
  c.d_partial = (double*)c.dalloc(sizeof(double) * (size_t)(kMaxCols + 2) * kMaxGrid * 2);
  c.d_counter = (unsigned int*)c.dalloc(256);
  c.gpart_elems = (size_t)1 << 21;  // 32 MiB of double2 chunk partials
  c.d_gpart = (double2*)c.dalloc(sizeof(double2) * c.gpart_elems);
  c.small_elems = kSmallElems;
  c.d_small = (double2*)c.dalloc(sizeof(double2) * c.small_elems);
  c.check(hipHostMalloc((void**)&c.h_small, sizeof(double2) * c.small_elems, 0), "hipHostMalloc");
  c.d_norm = (double*)c.dalloc(sizeof(double) * kMaxCols * 4);
  c.check(hipHostMalloc((void**)&c.h_norm, sizeof(double) * kMaxCols * 4, 0), "hipHostMalloc");

  // gauge field: unitarity check decides two-row storage
  double* chk = c.d_partial;  // out2 + partials + counter (see launch_gauge_check)
  c.check(launch_gauge_check((const double2*)gauge_dev, &g, chk, s), "gauge check");
  double h2[2];
  c.check(hipMemcpyAsync(h2, chk, sizeof(h2), hipMemcpyDeviceToHost, s), "memcpy");
  c.check(hipStreamSynchronize(s), "sync");
  const bool su3 = h2[0] < 1e-12 && h2[1] < 1e-12;
  c.comp64 = (p.compress_links && su3) ? 1 : 0;
  const size_t link_blocks = g.eo ? 2 : 1;  // odd-even: one block of link planes per parity
  c.u64 = c.dalloc(link_blocks * 4 * (c.comp64 ? 6 : 9) * g.vs * 16);
  c.check(launch_gauge_to_soa((const double2*)gauge_dev, c.u64, kF64, c.comp64, &g, s),
          "gauge to soa");
  if (p.precision != EIGCG_FP64) {  // inner links: FP32, or 16-bit for the half mode
    c.iprec = p.precision == EIGCG_MIXED_HALF ? kF16 : kF32;
    c.comp32 = (p.compress_links && h2[0] < 1e-6 && h2[1] < 1e-6) ? 1 : 0;
    if (c.iprec == kF16 && !c.comp32)
      throw ApiError{EIGCG_EINVAL, "16-bit storage needs two-row links: compress_links = 1 and "
                                   "links unitary with determinant 1 to 1e-6"};
    c.u32 = c.dalloc(link_blocks * 4 * (c.comp32 ? 6 : 9) * g.vs * elem_bytes(c.iprec));
    c.check(launch_gauge_to_soa((const double2*)gauge_dev, c.u32, c.iprec, c.comp32, &g, s),
            "gauge to soa inner");
  }
  if (g.eo) {  // odd-site intermediate of the two-pass Schur operator, per batch column
    c.eo_tmp64 = c.dalloc((size_t)p.max_batch * c.cs * 16);
    c.eo_cols64 = (size_t)p.max_batch;
    if (p.precision != EIGCG_FP64)
      c.eo_tmp32 = c.dalloc((size_t)p.max_batch * c.cs * elem_bytes(c.iprec));
  }
  c.bank_prec = p.precision == EIGCG_FP64 ? kF64 : kF32;
  c.H.assign((size_t)p.max_bank * p.max_bank, cplx(0.0, 0.0));
  c.L.assign((size_t)p.max_bank * p.max_bank, cplx(0.0, 0.0));
  c.events.resize(4 + 3 * kMaxCols);
  for (auto& e : c.events) c.check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  c.check(hipStreamSynchronize(s), "sync");
  autotune_stencil(c, kF64);
  if (p.precision != EIGCG_FP64) autotune_stencil(c, c.iprec);
}

static void ws_release(Ctx& c, Workspace& w) {
  c.dfree(w.b); c.dfree(w.x); c.dfree(w.r); c.dfree(w.p); c.dfree(w.tmp);
  c.dfree(w.ring); c.dfree(w.vr); c.dfree(w.tbuf); c.dfree(w.w); c.dfree(w.ritz); c.dfree(w.z);
  w.K = 0;
  w.eig = false;
}

void ctx_release(Ctx& c) {
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  ws_release(c, c.ws64);
  ws_release(c, c.ws32);
  ws_release(c, c.wsg);
  c.dfree(c.U);
  c.dfree(c.UR);
  {
    void* v2;
    v2 = c.d_specD; c.dfree(v2);
    v2 = c.d_specG; c.dfree(v2);
    v2 = c.d_specS; c.dfree(v2);
    v2 = c.d_specs; c.dfree(v2);
  }
  c.dfree(c.bwork);
  c.dfree(c.bwork64);
  c.dfree(c.u64);
  c.dfree(c.u32);
  c.dfree(c.eo_tmp64);
  c.dfree(c.eo_tmp32);
  c.dfree(c.bs);
  void* v;
  v = c.d_st; c.dfree(v);
  v = c.d_hist; c.dfree(v);
  v = c.d_partial; c.dfree(v);
  v = c.d_counter; c.dfree(v);
  v = c.d_gpart; c.dfree(v);
  v = c.d_small; c.dfree(v);
  v = c.d_norm; c.dfree(v);
  if (c.h_st) (void)hipHostFree(c.h_st);
  if (c.h_hist) (void)hipHostFree(c.h_hist);
  if (c.h_small) (void)hipHostFree(c.h_small);
  if (c.h_norm) (void)hipHostFree(c.h_norm);
  for (auto& e : c.events) (void)hipEventDestroy(e);
  c.events.clear();
  for (auto& k : c.ks_pool)
    for (auto& e : k.e) (void)hipEventDestroy(e);
  c.ks_pool.clear();
  for (auto& kv : c.graphs) (void)hipGraphExecDestroy(kv.second);
  c.graphs.clear();
  if (c.gstream) (void)hipStreamDestroy(c.gstream);
  c.gstream = nullptr;
}

// Fold the recorded stencil samples into the running sums.  All samples were
// recorded on one in-order stream, so the last one completing means all have.
bool Ctx::ks_harvest(bool wait) {
  if (ks_used == 0) return true;
  hipEvent_t last = ks_pool[ks_used - 1].e[3];
  if (wait) {
    check(hipEventSynchronize(last), "sample wait");
  } else {
    const hipError_t q = hipEventQuery(last);
    if (q == hipErrorNotReady) return false;
    check(q, "sample query");
  }
  for (int i = 0; i < ks_used; ++i) {
    KSample& k = ks_pool[i];
    float a = 0.f, b = 0.f;
    check(hipEventElapsedTime(&a, k.e[0], k.e[1]), "sample time");
    check(hipEventElapsedTime(&b, k.e[2], k.e[3]), "sample time");
    const int p = k.prec == kF64 ? 0 : 1;
    ks_done[p].push_back({a, b, (float)k.ncols});
  }
  ks_used = 0;
  return true;
}

// Means over the sampled iterations whose kernels ran: a sample whose second
// pass took under half the median of all samples is a launch whose columns had
// all stopped (the kernel exits at once) and is left out.
void kernel_samples(Ctx& c, bool reset, double* out) {
  c.ks_harvest(true);
  for (int p = 0; p < 2; ++p) {
    const auto& v = c.ks_done[p];
    double n = 0.0, s1 = 0.0, s2 = 0.0, sc = 0.0;
    if (!v.empty()) {
      std::vector<float> b2(v.size());
      for (size_t i = 0; i < v.size(); ++i) b2[i] = v[i][1];
      std::nth_element(b2.begin(), b2.begin() + b2.size() / 2, b2.end());
      const float cut = 0.5f * b2[b2.size() / 2];
      for (const auto& k : v) {
        if (k[1] < cut) continue;
        n += 1.0;
        s1 += k[0];
        s2 += k[1];
        sc += k[2];
      }
    }
    out[4 * p + 0] = n;
    out[4 * p + 1] = n > 0 ? s1 / n : 0.0;
    out[4 * p + 2] = n > 0 ? s2 / n : 0.0;
    out[4 * p + 3] = n > 0 ? sc / n : 0.0;
  }
  if (reset) {
    for (int p = 0; p < 2; ++p) c.ks_done[p].clear();
  }
}

static int seg_len_eig(const eigcg_params& P) {
  int d = (P.m - 2 * P.nev - 1) / 2;
  d = std::min(d, std::max(1, P.check_every));
  return std::max(1, d);
}

// Restart products V <- V (QZ) run in column groups whose m x group
// coefficients fit the tall kernel's 64 KB of LDS; with more than one group
// the restarted block cannot be overwritten in place (every output column
// reads all of the old block), so it alternates between two halves.
static int restart_group(const eigcg_params& P) { return std::max(1, std::min(24, 4096 / P.m)); }
static bool restart_pingpong(const eigcg_params& P) { return 2 * P.nev > restart_group(P); }

// Device bytes of the eigCG window arrays (residual ring, restarted block,
// saved A p, arrow vector, Ritz vectors) for keig columns in precision prec.
static size_t window_bytes(const Ctx& c, int prec, int keig) {
  const size_t vb = c.cs * elem_bytes(prec);
  const size_t ring_len = (size_t)(c.P.m + seg_len_eig(c.P) + 2);
  const size_t per = ring_len + (size_t)2 * c.P.nev * (restart_pingpong(c.P) ? 2 : 1) + 2 + 1 +
                     (size_t)c.P.nev;
  return vb * per * (size_t)keig;
}

size_t eig_window_bytes(const Ctx& c, int keig) {
  if (c.P.precision == EIGCG_MIXED_HALF) return 0;  // no eigCG iterations
  size_t b = 0;
  if (c.P.precision == EIGCG_FP64) {
    if (!c.ws64.eig || c.ws64.Keig < keig) b += window_bytes(c, kF64, keig);
  } else if (!c.ws32.eig || c.ws32.Keig < keig) {
    b += window_bytes(c, c.iprec, keig);
  }
  return b;
}

// Work vectors of max_batch columns; with eig, the eigCG window arrays for
// keig columns (default max_batch), reallocated when a wider run needs them.
static void ws_ensure(Ctx& c, Workspace& w, int prec, bool eig, int keig) {
  const int K = c.P.max_batch;
  if (keig <= 0 || keig > K) keig = K;
  const size_t vb = c.cs * elem_bytes(prec);
  if (w.K == 0) {
    w.prec = prec;
    w.K = K;
    w.b = c.dalloc(vb * K);
    // the iterate of a 16-bit inner solve accumulates in FP32
    w.x = c.dalloc((prec == kF16 ? c.cs * 8 : vb) * K);
    w.r = c.dalloc(vb * K);
    w.p = c.dalloc(vb * K);
    w.tmp = c.dalloc(vb * K);
    if (c.P.precond == EIGCG_PRECOND_SPECTRAL && prec == kF64) w.z = c.dalloc(vb * K);
  }
  if (eig && w.eig && w.Keig < keig) {  // a wider eigCG run than the window holds
    c.dfree(w.ring); c.dfree(w.vr); c.dfree(w.tbuf); c.dfree(w.w); c.dfree(w.ritz);
    w.eig = false;
  }
  if (eig && !w.eig) {
    w.nev = c.P.nev;
    w.Keig = keig;
    w.ring_len = c.P.m + seg_len_eig(c.P) + 2;
    w.ring = c.dalloc(vb * (size_t)keig * w.ring_len);
    w.vr = c.dalloc(vb * (size_t)keig * 2 * c.P.nev * (restart_pingpong(c.P) ? 2 : 1));
    w.tbuf = c.dalloc(vb * (size_t)keig * 2);
    w.w = c.dalloc(vb * (size_t)keig);
    w.ritz = c.dalloc(vb * (size_t)keig * c.P.nev);
    w.eig = true;
  }
}

// Field idx of a run of fields starting at base; the field must end inside
// base's allocation.
void* col_ptr(void* base, int prec, size_t cs, size_t idx) {
  check_span(base, (idx + 1) * cs * elem_bytes(prec), "column");
  return (char*)base + idx * cs * elem_bytes(prec);
}

// ncols whole fields of precision prec start at p (inside p's allocation)
void check_fields(const Ctx& c, const void* p, int prec, int ncols, const char* what) {
  if (p && ncols > 0) check_span(p, (size_t)ncols * c.cs * elem_bytes(prec), what);
}

// ---------------------------------------------------------------------------
// operator application
// ---------------------------------------------------------------------------

static StencilLaunch stencil_base(Ctx& c, int prec) {
  StencilLaunch L{};
  L.prec = prec;
  L.compressed = prec == kF64 ? c.comp64 : c.comp32;
  L.variant = prec == kF64 ? c.var64 : c.var32;
  L.nc = prec == kF64 ? c.nc64 : c.nc32;
  L.u = prec == kF64 ? c.u64 : c.u32;
  L.g = &c.g;
  L.diag = 4.0 + c.P.mass;
  L.eo_tmp = prec == kF64 ? c.eo_tmp64 : c.eo_tmp32;
  L.eo_tmp_cs = c.cs;
  L.st = c.d_st;
  L.partial = c.d_partial;
  L.counter = c.d_counter;
  L.hist = c.d_hist;
  L.hist_stride = c.hist_stride;
  return L;
}

// out = op(in) (op = M or M^H) on ncols internal fields
// The odd-even operator's two passes keep ncols odd-site intermediates.
static void check_eo_tmp(const Ctx& c, int prec, int ncols) {
  if (c.g.eo) check_fields(c, prec == kF64 ? c.eo_tmp64 : c.eo_tmp32, prec, ncols,
                           "odd-even intermediate");
}

void stencil_store(Ctx& c, int prec, int op, int ncols, const void* in, void* out) {
  check_fields(c, in, prec, ncols, "stencil input");
  check_fields(c, out, prec, ncols, "stencil output");
  check_eo_tmp(c, prec, ncols);
  StencilLaunch L = stencil_base(c, prec);
  L.op = op;
  L.epi = kEpiStore;
  L.in = in; L.in_cs = c.cs;
  L.out = out; L.out_cs = c.cs;
  L.ncols = ncols;
  L.mask = (ncols >= 32) ? 0xffffffffu : ((1u << ncols) - 1);
  c.check(launch_stencil(L, c.stream), "stencil");
}

// r = b - A x for masked columns, rho = ||r||^2 into the column states
static void true_residual(Ctx& c, int prec, int ncols, uint32_t mask, const void* x,
                          const void* b, void* r, void* tmp) {
  for (const void* f : {x, b, (const void*)r, (const void*)tmp})
    check_fields(c, f, prec, ncols, "true-residual field");
  check_eo_tmp(c, prec, ncols);
  StencilLaunch L = stencil_base(c, prec);
  L.op = kOpM;
  L.epi = kEpiStore;
  L.in = x; L.in_cs = c.cs;
  L.out = tmp; L.out_cs = c.cs;
  L.ncols = ncols;
  L.mask = mask;
  c.check(launch_stencil(L, c.stream), "stencil M");
  L.op = kOpMdag;
  L.epi = kEpiRes;
  L.in = tmp;
  L.r = r; L.r_cs = c.cs;
  L.b = b; L.b_cs = c.cs;
  c.check(launch_stencil(L, c.stream), "stencil Mdag res");
}

void apply_op(Ctx& c, int op, int nrhs, const void* in_aos, void* out_aos) {
  if (op >= 3) {  // the inner precision's kernels (input rounded to it, result widened)
    if (c.P.precision == EIGCG_FP64) throw ApiError{EIGCG_EINVAL, "not a mixed-precision context"};
    const int ip = c.iprec;
    Workspace& w64 = c.ws64;
    Workspace& w = c.ws32;
    ws_ensure(c, w64, kF64, false);
    ws_ensure(c, w, ip, false);
    for (int c0 = 0; c0 < nrhs; c0 += w.K) {
      const int k = std::min(w.K, nrhs - c0);
      const uint32_t m = (k >= 32) ? 0xffffffffu : ((1u << k) - 1);
      const double2* src = (const double2*)in_aos + (size_t)c0 * 12 * c.g.V;
      double2* dst = (double2*)out_aos + (size_t)c0 * 12 * c.g.V;
      c.check(launch_spinor_to_soa(src, w64.x, kF64, &c.g, k, c.cs, c.stream), "to soa");
      c.check(launch_copy(kF64, ip, k, c.cs, w64.x, c.cs, w.p, c.cs, c.stream, m), "narrow");
      if (op == EIGCG_OP_A + 3) {
        stencil_store(c, ip, kOpM, k, w.p, w.tmp);
        stencil_store(c, ip, kOpMdag, k, w.tmp, w.r);
      } else {
        stencil_store(c, ip, op == EIGCG_OP_M + 3 ? kOpM : kOpMdag, k, w.p, w.r);
      }
      c.check(launch_copy(ip, kF64, k, c.cs, w.r, c.cs, w64.r, c.cs, c.stream, m), "widen");
      c.check(launch_spinor_from_soa(w64.r, dst, kF64, &c.g, k, c.cs, c.stream), "from soa");
    }
    c.check(hipStreamSynchronize(c.stream), "sync");
    return;
  }
  Workspace& w = c.ws64;
  ws_ensure(c, w, kF64, false);
  for (int c0 = 0; c0 < nrhs; c0 += w.K) {
    const int k = std::min(w.K, nrhs - c0);
    const double2* src = (const double2*)in_aos + (size_t)c0 * 12 * c.g.V;
    double2* dst = (double2*)out_aos + (size_t)c0 * 12 * c.g.V;
    check_fields(c, w.x, kF64, k, "operator input");
    c.check(launch_spinor_to_soa(src, w.x, kF64, &c.g, k, c.cs, c.stream), "to soa");
    if (op == EIGCG_OP_A) {
      stencil_store(c, kF64, kOpM, k, w.x, w.tmp);
      stencil_store(c, kF64, kOpMdag, k, w.tmp, w.r);
    } else {
      stencil_store(c, kF64, op == EIGCG_OP_M ? kOpM : kOpMdag, k, w.x, w.r);
    }
    c.check(launch_spinor_from_soa(w.r, dst, kF64, &c.g, k, c.cs, c.stream), "from soa");
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
}

// Odd-even preconditioning: maps between the full system M x = b and the
// even-site system.  One raw pass: out (parity par) = dg in2 + ch D in.
static void eo_pass(Ctx& c, int k, int par, const void* in, const void* in2, double dg, double ch,
                    void* out) {
  StencilLaunch L = stencil_base(c, kF64);
  L.op = kOpM;
  L.epi = kEpiStore;
  L.in = in; L.in_cs = c.cs;
  L.out = out; L.out_cs = c.cs;
  L.ncols = k;
  L.mask = (k >= 32) ? 0xffffffffu : ((1u << k) - 1);
  L.eo_raw = 1;
  L.eo_par = par;
  L.in2 = in2; L.in2_cs = c.cs;
  L.eo_dg = dg;
  L.eo_ch = ch;
  c.check(launch_stencil(L, c.stream), "odd-even pass");
}

// rhs = Mhat^H (b_e + D_eo b_o / (2 d)): the right-hand side of the
// preconditioned normal equations for M x = b
void schur_rhs(Ctx& c, int nrhs, const void* b_full, void* rhs) {
  if (!c.g.eo) throw ApiError{EIGCG_EINVAL, "context is not odd-even preconditioned"};
  Workspace& w = c.ws64;
  ws_ensure(c, w, kF64, false);
  const double d = 4.0 + c.P.mass;
  for (int c0 = 0; c0 < nrhs; c0 += w.K) {
    const int k = std::min(w.K, nrhs - c0);
    const double2* src = (const double2*)b_full + (size_t)c0 * 12 * c.g.Vfull;
    double2* dst = (double2*)rhs + (size_t)c0 * 12 * c.g.V;
    c.check(launch_split_eo(src, w.b, w.p, &c.g, k, c.cs, c.stream), "split");
    eo_pass(c, k, 0, w.p, w.b, 1.0, 0.5 / d, w.x);
    stencil_store(c, kF64, kOpMdag, k, w.x, w.r);
    c.check(launch_spinor_from_soa(w.r, dst, kF64, &c.g, k, c.cs, c.stream), "from soa");
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
}

// x = (x_e, (b_o + D_oe x_e / 2) / d) on the full lattice
void schur_reconstruct(Ctx& c, int nrhs, const void* b_full, const void* x_even, void* x_full) {
  if (!c.g.eo) throw ApiError{EIGCG_EINVAL, "context is not odd-even preconditioned"};
  Workspace& w = c.ws64;
  ws_ensure(c, w, kF64, false);
  const double d = 4.0 + c.P.mass;
  for (int c0 = 0; c0 < nrhs; c0 += w.K) {
    const int k = std::min(w.K, nrhs - c0);
    const double2* bsrc = (const double2*)b_full + (size_t)c0 * 12 * c.g.Vfull;
    const double2* xsrc = (const double2*)x_even + (size_t)c0 * 12 * c.g.V;
    double2* dst = (double2*)x_full + (size_t)c0 * 12 * c.g.Vfull;
    c.check(launch_split_eo(bsrc, w.b, w.p, &c.g, k, c.cs, c.stream), "split");
    c.check(launch_spinor_to_soa(xsrc, w.x, kF64, &c.g, k, c.cs, c.stream), "to soa");
    eo_pass(c, k, 1, w.x, w.p, 1.0 / d, 0.5 / d, w.r);
    c.check(launch_merge_eo(w.x, w.r, dst, &c.g, k, c.cs, c.stream), "merge");
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
}

// ---------------------------------------------------------------------------
// small device products with host-side coefficient matrices
// ---------------------------------------------------------------------------

// G (K x N) = In^H R on the device, copied to host (synchronous)
static void reduce_to_host(Ctx& c, int prec, int K, int N, const std::vector<const void*>& in,
                           const std::vector<const void*>& rc, std::vector<cplx>& G) {
  G.assign((size_t)K * N, cplx(0.0, 0.0));
  for (int k0 = 0; k0 < K; k0 += 256) {
    const int kk = std::min(256, K - k0);
    for (int n0 = 0; n0 < N; n0 += 16) {
      const int nn = std::min(16, N - n0);
      double2* dg = c.d_small + kGenericOff;
      double2* hg = c.h_small + kGenericOff;
      c.check(launch_gemm_reduce(prec, c.cs, kk, nn, in.data() + k0, rc.data() + n0, c.d_gpart,
                                 c.gpart_elems, dg, c.stream),
              "gemm reduce");
      c.check(hipMemcpyAsync(hg, dg, sizeof(double2) * kk * nn, hipMemcpyDeviceToHost, c.stream),
              "memcpy");
      c.check(hipStreamSynchronize(c.stream), "sync");
      for (int j = 0; j < nn; ++j)
        for (int i = 0; i < kk; ++i) {
          double2 v = hg[(size_t)j * kk + i];
          G[(size_t)(n0 + j) * K + k0 + i] = cplx(v.x, v.y);
        }
    }
  }
}

// Out (+)= In * S with host S (K x N, ld K); uses the staging area at
// element offset `slot` of d_small / h_small.  Synchronous staging.
static void tall_from_host(Ctx& c, int prec, int K, int N, const std::vector<const void*>& in,
                           const std::vector<void*>& out, const cplx* S, int beta_one,
                           int negate) {
  for (int k0 = 0; k0 < K; k0 += 256) {
    const int kk = std::min(256, K - k0);
    // the kernel holds the kk x nn coefficients in 64 KB of LDS
    const int nmax = std::max(1, std::min(24, 4096 / kk));
    for (int n0 = 0; n0 < N; n0 += nmax) {
      const int nn = std::min(nmax, N - n0);
      c.check(hipStreamSynchronize(c.stream), "sync");
      double2* dg = c.d_small + kGenericOff;
      double2* hg = c.h_small + kGenericOff;
      for (int j = 0; j < nn; ++j)
        for (int i = 0; i < kk; ++i) {
          cplx v = S[(size_t)(n0 + j) * K + k0 + i];
          hg[(size_t)j * kk + i] = make_double2(v.real(), v.imag());
        }
      c.check(hipMemcpyAsync(dg, hg, sizeof(double2) * kk * nn, hipMemcpyHostToDevice, c.stream),
              "memcpy");
      c.check(launch_gemm_tall(prec, c.cs, kk, nn, in.data() + k0, out.data() + n0, dg,
                               (beta_one || k0 > 0) ? 1 : 0, negate, c.stream),
              "gemm tall");
    }
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
}

// ---------------------------------------------------------------------------
// init-CG deflation, eq. (2.1): x += U H^{-1} U^H (b - A x)
// ---------------------------------------------------------------------------

static void ensure_chol(Ctx& c) {
  if (c.chol_ok) return;
  const int l = c.l, ld = c.P.max_bank;
  for (int j = 0; j < l; ++j)
    for (int i = 0; i < l; ++i) c.L[(size_t)j * ld + i] = c.H[(size_t)j * ld + i];
  if (hostla::cholesky(l, c.L.data(), ld) != 0)
    throw ApiError{EIGCG_EBREAKDOWN, "H = U^H A U is not positive definite"};
  c.chol_ok = true;
}

// columns of ws (prec) given by mask; r holds b - A x on entry (prec storage)
void deflate_columns(Ctx& c, int prec, int ncols, uint32_t mask, void* x, const void* r) {
  if (c.l == 0) return;
  ensure_chol(c);
  const int l = c.l;
  std::vector<int> cols;
  for (int j = 0; j < ncols; ++j)
    if ((mask >> j) & 1u) cols.push_back(j);
  if (cols.empty()) return;
  if (prec != c.bank_prec) throw ApiError{EIGCG_EINVAL, "bank precision mismatch"};
  std::vector<const void*> in(l), rc;
  for (int i = 0; i < l; ++i) in[i] = col_ptr(c.U, c.bank_prec, c.cs, i);
  for (int j : cols) rc.push_back(col_ptr(const_cast<void*>(r), prec, c.cs, j));
  std::vector<cplx> G;
  reduce_to_host(c, prec, l, (int)cols.size(), in, rc, G);
  hostla::cholesky_solve(l, c.L.data(), c.P.max_bank, (int)cols.size(), G.data(), l);
  std::vector<void*> out;
  for (int j : cols) out.push_back(col_ptr(x, prec, c.cs, j));
  tall_from_host(c, prec, l, (int)cols.size(), in, out, G.data(), 1, 0);
}

// ---------------------------------------------------------------------------
// spectral preconditioner (params.precond): P^{-1} = I + U_R D U_R^H
// ---------------------------------------------------------------------------

// From the current bank: Rayleigh-Ritz on H (host FP64, H Y = Y Theta), the
// Ritz basis U_R = U Y on the device, D = sigma / theta - 1 (Section 2.1's
// spectral preconditioner; sigma from the parameters, else the largest Ritz
// value seen, else (8 + |m|)^2).  An empty bank leaves P = I.
static void ensure_spectral(Ctx& c) {
  if (c.P.precond != EIGCG_PRECOND_SPECTRAL || c.spec_ok) return;
  const int l = c.l, ld = c.P.max_bank;
  c.lR = 0;
  if (l > 0) {
    std::vector<double> th(l);
    std::vector<cplx> Y((size_t)l * l);
    if (hostla::herm_eig_lowest(l, c.H.data(), ld, l, th.data(), Y.data(), l) != 0)
      throw ApiError{EIGCG_EBREAKDOWN, "bank eigensolver failed"};
    if (!(th[0] > 0.0))
      throw ApiError{EIGCG_EBREAKDOWN, "the spectral preconditioner needs positive Ritz values"};
    const double am = std::fabs(c.P.mass);
    const double sigma = c.P.precond_sigma > 0 ? c.P.precond_sigma
                                               : (c.amax > 0 ? c.amax : (8.0 + am) * (8.0 + am));
    const size_t nb = (size_t)c.P.max_bank;
    if (!c.UR) c.UR = c.dalloc(c.cs * 16 * nb);
    if (!c.d_specD) {
      c.d_specD = (double*)c.dalloc(sizeof(double) * nb);
      c.d_specG = (double2*)c.dalloc(sizeof(double2) * nb * kMaxCols);
      c.d_specS = (double2*)c.dalloc(sizeof(double2) * nb * kMaxCols);
      c.d_specs = (double*)c.dalloc(sizeof(double) * kMaxCols);
    }
    std::vector<const void*> in(l);
    std::vector<void*> out(l);
    for (int i = 0; i < l; ++i) {
      in[i] = col_ptr(c.U, kF64, c.cs, i);
      out[i] = col_ptr(c.UR, kF64, c.cs, i);
    }
    tall_from_host(c, kF64, l, l, in, out, Y.data(), 0, 0);
    std::vector<double> D(l);
    for (int i = 0; i < l; ++i) D[i] = sigma / th[i] - 1.0;
    c.check(hipMemcpy(c.d_specD, D.data(), sizeof(double) * l, hipMemcpyHostToDevice), "D");
    c.spec_sigma = sigma;
    c.lR = l;
  }
  c.spec_ok = true;
}

// z = P^{-1} r = r + U_R (D (U_R^H r)) for K columns (enqueued on stream s;
// capturable); also leaves s_j = r_j^H U_R D U_R^H r_j in d_specs, so that
// r^H z = ||r||^2 + s_j.
static hipError_t apply_spectral(Ctx& c, hipStream_t s, int K, uint32_t mask, const void* r,
                                 void* z) {
  const int l = c.lR;
  std::vector<const void*> in(l), rc(K);
  std::vector<void*> zc(K);
  for (int i = 0; i < l; ++i) in[i] = col_ptr(c.UR, kF64, c.cs, i);
  for (int j = 0; j < K; ++j) {
    rc[j] = col_ptr(const_cast<void*>(r), kF64, c.cs, j);
    zc[j] = col_ptr(z, kF64, c.cs, j);
  }
  hipError_t e = launch_gemm_reduce(kF64, c.cs, l, K, in.data(), rc.data(), c.d_gpart,
                                    c.gpart_elems, c.d_specG, s);
  if (e == hipSuccess) e = launch_spec_scale(c.d_specG, c.d_specD, l, K, c.d_specS, c.d_specs, s);
  if (e == hipSuccess) e = launch_copy(kF64, kF64, K, c.cs, r, c.cs, z, c.cs, s, mask);
  const int nmax = std::max(1, std::min(24, 4096 / l));
  for (int n0 = 0; n0 < K && e == hipSuccess; n0 += nmax) {
    const int nn = std::min(nmax, K - n0);
    e = launch_gemm_tall(kF64, c.cs, l, nn, in.data(), zc.data() + n0, c.d_specS + (size_t)n0 * l,
                         1, 0, s);
  }
  return e;
}

// ---------------------------------------------------------------------------
// eigCG window bookkeeping (host side, one per column)
// ---------------------------------------------------------------------------

struct EigCol {
  int k_lo = 1;            // first residual index in the window
  bool has_vr = false;     // restarted block present (2 nev columns)
  int vr_half = 0;         // which half of the column's restart area holds it
  std::vector<double> Mv;  // its Ritz values (diagonal of T)
  std::vector<cplx> arrow; // arrow row, T(2nev, 0:2nev)
  int arrow_J = 0;         // iteration whose residual carries the arrow row
  int arrow_state = 0;     // 0 none, 1 needs enqueue, 2 enqueued, 3 read
  int next_full = 0;       // iteration after which the window is full
  int restarts = 0;
  bool finalized = false;
  std::vector<double> ritz_vals;
  int nritz = 0;
};

struct Run {
  Ctx& c;
  Workspace& w;
  int prec;
  int K;
  uint32_t mask;
  bool eig;
  int nev, m, period;
  std::vector<EigCol> ec;
  std::vector<int> hist_read;    // iterations of history copied to the host
  std::vector<int> done;         // column processed as stopped
  std::vector<int> reason;
  std::vector<int> iters;
  std::vector<int> outer;        // host-driven restarts
  std::vector<int> first_leg;    // iterations before the first init-CG restart (-1: none)
  std::vector<int> stale_until;  // snapshots of segments <= this id predate a host restart
  int enq_iter = 0;              // iterations enqueued (all columns in lockstep)
  bool spec = false;             // iterations preconditioned with z = P^{-1} r
  int seg_id = 0;                // id of the last enqueued segment

  Run(Ctx& c_, Workspace& w_, int prec_, int K_, uint32_t mask_, bool eig_)
      : c(c_), w(w_), prec(prec_), K(K_), mask(mask_), eig(eig_) {
    nev = c.P.nev;
    m = c.P.m;
    period = m - 2 * nev;
    ec.resize(K);
    hist_read.assign(K, 0);
    done.assign(K, 0);
    reason.assign(K, 0);
    iters.assign(K, 0);
    outer.assign(K, 0);
    first_leg.assign(K, -1);
    stale_until.assign(K, -1);
    for (int j = 0; j < K; ++j) ec[j].next_full = m;
    spec = c.P.precond == EIGCG_PRECOND_SPECTRAL && prec == kF64 && c.spec_ok && c.lR > 0;
    if (spec) check_fields(c, w.z, kF64, K, "preconditioned residuals");
    // every launch of the run covers K columns of the workspace
    if (K > w.K) throw ApiError{EIGCG_EINVAL, "internal: run wider than its workspace"};
    for (const void* f : {w.b, w.r, w.p, w.tmp}) check_fields(c, f, prec, K, "run field");
    check_fields(c, w.x, prec == kF16 ? kF32 : prec, K, "run iterate");
    check_eo_tmp(c, prec, K);
    if (eig) {
      if (K > w.Keig) throw ApiError{EIGCG_EINVAL, "internal: eigCG run wider than its window"};
      check_fields(c, w.ring, prec, K * w.ring_len, "window ring");
    }
  }
  Run(const Run&) = delete;
  Run& operator=(const Run&) = delete;

  void* ringslot(int col, int k) const {
    const int slot = k % w.ring_len;
    return col_ptr(w.ring, prec, c.cs, (size_t)col * w.ring_len + slot);
  }
  // column i of the restarted block of column col (half: of the two
  // alternating areas when restart_pingpong)
  void* vrcol_half(int col, int half, int i) const {
    const size_t per = (size_t)2 * nev * (restart_pingpong(c.P) ? 2 : 1);
    return col_ptr(w.vr, prec, c.cs, (size_t)col * per + (size_t)half * 2 * nev + i);
  }
  void* vrcol(int col, int i) const { return vrcol_half(col, ec[col].vr_half, i); }

  // alpha_k, beta_k, rho_k from the host history copy (k is 1-based)
  double alpha(int col, int k) const { return c.h_hist[(size_t)col * c.hist_stride + 3 * (k - 1)]; }
  double beta(int col, int k) const {
    return k <= 1 ? 0.0 : c.h_hist[(size_t)col * c.hist_stride + 3 * (k - 2) + 1];
  }
  double rho(int col, int k) const {
    return c.h_hist[(size_t)col * c.hist_stride + 3 * (k - 2) + 2];  // k >= 2
  }

  // event triple for this iteration when it is sampled, else null
  Ctx::KSample* sample_slot() {
    const int every = c.P.sample_every;
    if (every <= 0 || (c.ks_tick++ % every) != 0) return nullptr;
    constexpr int kPool = 256;
    if (c.ks_pool.empty()) {
      c.ks_pool.resize(kPool);
      for (auto& k : c.ks_pool)
        for (auto& e : k.e) c.check(hipEventCreate(&e), "sample event");
    }
    if (c.ks_used == kPool && !c.ks_harvest(false)) return nullptr;
    Ctx::KSample* k = &c.ks_pool[c.ks_used++];
    k->prec = prec;
    k->ncols = __builtin_popcount(mask);
    return k;
  }

  void enqueue_iters(int n) {
    StencilLaunch L1 = stencil_base(c, prec);
    L1.op = kOpM;
    L1.epi = kEpiNorm;
    L1.in = w.p; L1.in_cs = c.cs;
    L1.out = w.tmp; L1.out_cs = c.cs;
    L1.ncols = K;
    L1.mask = mask;
    StencilLaunch L2 = L1;
    L2.op = kOpMdag;
    L2.epi = kEpiCGR;
    L2.in = w.tmp;
    L2.r = w.r; L2.r_cs = c.cs;
    L2.tbuf = eig ? w.tbuf : nullptr;
    L2.t_cs = c.cs;
    UpdateLaunch L3{};
    L3.prec = prec;
    L3.ncols = K;
    L3.mask = mask;
    L3.st = c.d_st;
    L3.g = &c.g;
    L3.x = w.x; L3.x_cs = c.cs;
    L3.p = w.p; L3.p_cs = c.cs;
    L3.r = w.r; L3.r_cs = c.cs;
    L3.ring = eig ? w.ring : nullptr;
    L3.ring_cs = c.cs;
    L3.ring_len = w.ring_len;
    L3.ring_col_cs = (size_t)w.ring_len * c.cs;
    // preconditioned iterations: after the second pass z = P^{-1} r, then the
    // CG scalars with rho = r^H z, then p = z + beta p and the window from z
    int nb2 = 0;
    double* part_a = c.d_partial;
    double* part_b = c.d_partial + (size_t)kMaxCols * kMaxGrid;
    if (spec) {
      L2.defer_finalize = 1;
      L2.grid_out = &nb2;
      L3.r = w.z;
    }
    auto precond_step = [&](hipStream_t st) -> hipError_t {
      hipError_t e = apply_spectral(c, st, K, mask, w.r, w.z);
      if (e == hipSuccess)
        e = launch_finalize_cg(c.d_st, K, mask, part_a, part_b, nb2, c.d_hist, c.hist_stride,
                               c.d_specs, st);
      return e;
    };
    // one iteration on its own; a sampled one times each stencil kernel by its
    // own dispatch timestamps (no extra packets between the kernels)
    auto eager = [&]() {
      Ctx::KSample* ks = sample_slot();
      L1.ev_start = ks ? ks->e[0] : nullptr;
      L1.ev_stop = ks ? ks->e[1] : nullptr;
      L2.ev_start = ks ? ks->e[2] : nullptr;
      L2.ev_stop = ks ? ks->e[3] : nullptr;
      c.check(launch_stencil(L1, c.stream), "K1");
      c.check(launch_stencil(L2, c.stream), "K2");
      if (spec) c.check(precond_step(c.stream), "preconditioner");
      c.check(launch_cg_update(L3, c.stream), "K3");
      L1.ev_start = L1.ev_stop = L2.ev_start = L2.ev_stop = nullptr;
    };
    // len iterations replayed from a graph captured once per context
    auto replay = [&](int len) {
      const std::array<uint64_t, 14> key = {
          (uint64_t)len, (uint64_t)prec, (uint64_t)K, (uint64_t)mask, (uint64_t)eig,
          (uint64_t)spec, spec ? (uint64_t)c.bank_gen : 0u, (uint64_t)(uintptr_t)w.p,
          (uint64_t)(uintptr_t)w.r, (uint64_t)(uintptr_t)w.x, (uint64_t)(uintptr_t)w.tmp,
          (uint64_t)(uintptr_t)w.ring, (uint64_t)(uintptr_t)w.tbuf,
          (uint64_t)(uintptr_t)w.z ^ ((uint64_t)w.ring_len << 48)};
      auto it = c.graphs.find(key);
      if (it == c.graphs.end()) {
        // bounded: graphs of earlier workspaces, banks or masks are dropped
        if (c.graphs.size() >= 64) {
          c.check(hipStreamSynchronize(c.stream), "sync");
          for (auto& kv : c.graphs) (void)hipGraphExecDestroy(kv.second);
          c.graphs.clear();
        }
        // captured on a private stream (the context's stream may be the null
        // stream, which cannot be captured); replayed on the context's stream
        if (!c.gstream) c.check(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking), "stream");
        hipGraph_t gr = nullptr;
        hipGraphExec_t ex = nullptr;
        c.check(hipStreamBeginCapture(c.gstream, hipStreamCaptureModeThreadLocal), "capture");
        hipError_t e = hipSuccess;
        for (int i = 0; i < len && e == hipSuccess; ++i) {
          e = launch_stencil(L1, c.gstream);
          if (e == hipSuccess) e = launch_stencil(L2, c.gstream);
          if (e == hipSuccess && spec) e = precond_step(c.gstream);
          if (e == hipSuccess) e = launch_cg_update(L3, c.gstream);
        }
        const hipError_t e2 = hipStreamEndCapture(c.gstream, &gr);
        c.check(e, "captured launch");
        c.check(e2, "end capture");
        const hipError_t e3 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        c.check(e3, "graph instantiate");
        it = c.graphs.emplace(key, ex).first;
      }
      c.check(hipGraphLaunch(it->second, c.stream), "graph launch");
    };
    if (c.P.use_graphs && n > 0) {
      // runs of unsampled iterations from graphs, sampled ones on their own
      for (int i = 0; i < n;) {
        int run = n - i;
        if (c.P.sample_every > 0) {
          const long every = c.P.sample_every;
          run = (int)std::min<long>(run, (every - c.ks_tick % every) % every);
        }
        if (run > 0) {
          replay(run);
          c.ks_tick += run;
          i += run;
        } else {
          eager();
          ++i;
        }
      }
      enq_iter += n;
      return;
    }
    for (int i = 0; i < n; ++i) eager();
    enq_iter += n;
  }

  // states (slot) and history up to `upto` iterations, then an event
  void enqueue_poll(int slot, int upto) {
    c.check(hipMemcpyAsync(c.h_st + slot * kMaxCols, c.d_st, sizeof(ColState) * K,
                           hipMemcpyDeviceToHost, c.stream),
            "poll states");
    if (eig) {
      for (int j = 0; j < K; ++j) {
        if (!((mask >> j) & 1u) || done[j]) continue;
        const int from = hist_read[j];
        if (upto <= from) continue;
        const size_t off = (size_t)j * c.hist_stride + 3 * (size_t)from;
        c.check(hipMemcpyAsync(c.h_hist + off, c.d_hist + off, sizeof(double) * 3 * (upto - from),
                               hipMemcpyDeviceToHost, c.stream),
                "poll hist");
        hist_read[j] = upto;
      }
    }
    c.check(hipEventRecord(c.events[slot], c.stream), "event");
  }

  // full window matrix T (i x i) of column col given iterations up to j_last
  // (diagonal of the last residual filled when with_last_diag)
  int build_T(int col, int k_hi, std::vector<cplx>& T, int ld) {
    EigCol& e = ec[col];
    const int base = e.has_vr ? 2 * nev : 0;
    const int i = base + (k_hi - e.k_lo + 1);
    T.assign((size_t)ld * ld, cplx(0.0, 0.0));
    if (e.has_vr) {
      for (int q = 0; q < 2 * nev; ++q) T[(size_t)q * ld + q] = e.Mv[q];
      // column-major: T(row, col) = T[col * ld + row]; arrow[q] = T(q, base)
      for (int q = 0; q < 2 * nev; ++q) {
        T[(size_t)base * ld + q] = e.arrow[q];
        T[(size_t)q * ld + base] = std::conj(e.arrow[q]);
      }
    }
    for (int k = e.k_lo; k <= k_hi; ++k) {
      const int pidx = base + (k - e.k_lo);
      const double a = alpha(col, k);
      double d = 1.0 / a;
      if (k >= 2) d += beta(col, k) / alpha(col, k - 1);
      T[(size_t)pidx * ld + pidx] = d;
      if (k > e.k_lo) {
        const double off = -std::sqrt(beta(col, k)) / alpha(col, k - 1);
        T[(size_t)pidx * ld + pidx - 1] = off;
        T[(size_t)(pidx - 1) * ld + pidx] = off;
      }
    }
    return i;
  }

  void window_cols(int col, int k_hi, std::vector<const void*>& in) {
    EigCol& e = ec[col];
    in.clear();
    if (e.has_vr)
      for (int q = 0; q < 2 * nev; ++q) in.push_back(vrcol(col, q));
    for (int k = e.k_lo; k <= k_hi; ++k) in.push_back(ringslot(col, k));
  }

  void wait_arrow(int col) {
    EigCol& e = ec[col];
    if (e.arrow_state == 2) {
      c.check(hipEventSynchronize(c.events[4 + kMaxCols + col]), "arrow wait");
      e.arrow.resize(2 * nev);
      const double inv = 1.0 / std::sqrt(rho(col, e.arrow_J));
      for (int q = 0; q < 2 * nev; ++q) {
        // the device computed v_q^H w, i.e. T(q, 2nev) sqrt(rho) (T = V^H A V, A r = w)
        double2 v = c.h_small[arrow_off(col) + q];
        e.arrow[q] = cplx(v.x, v.y) * inv;
      }
      e.arrow_state = 3;
    }
  }

  // Figure 3.1 restart (eq. (2.3)) for one column whose window filled at E
  void do_restart(int col, int E) {
    EigCol& e = ec[col];
    if (e.has_vr) wait_arrow(col);
    std::vector<cplx> T;
    const int i = build_T(col, E, T, m);
    if (i != m) throw ApiError{EIGCG_EINVAL, "internal: window size mismatch at restart"};
    // restart coefficients: Ritz vectors of T_m and T_{m-1}, orth, Rayleigh-Ritz
    std::vector<double> w1(m), w2(m);
    std::vector<cplx> Y((size_t)m * nev), Yb((size_t)m * nev, cplx(0.0, 0.0));
    if (hostla::herm_eig_lowest(m, T.data(), m, nev, w1.data(), Y.data(), m) != 0)
      throw ApiError{EIGCG_EBREAKDOWN, "window eigensolver failed"};
    c.amax = std::max(c.amax, w1[m - 1]);
    if (hostla::herm_eig_lowest(m - 1, T.data(), m, nev, w2.data(), Yb.data(), m) != 0)
      throw ApiError{EIGCG_EBREAKDOWN, "window eigensolver failed"};
    for (int q = 0; q < nev; ++q) Yb[(size_t)q * m + (m - 1)] = 0.0;  // pad Ybar
    std::vector<cplx> YY((size_t)m * 2 * nev);
    std::copy(Y.begin(), Y.end(), YY.begin());
    std::copy(Yb.begin(), Yb.end(), YY.begin() + (size_t)m * nev);
    std::vector<cplx> Q((size_t)m * 2 * nev);
    hostla::qr_thin(m, 2 * nev, YY.data(), m, Q.data(), m, nullptr, 0);  // orth([Y, Ybar])
    std::vector<cplx> TQ((size_t)m * 2 * nev), Hs((size_t)4 * nev * nev);
    hostla::matmul_sparse_a(m, 2 * nev, m, T.data(), m, Q.data(), m, TQ.data(), m);
    hostla::matmul_ah_b(2 * nev, 2 * nev, m, Q.data(), m, TQ.data(), m, Hs.data(), 2 * nev);
    std::vector<double> Mv(2 * nev);
    std::vector<cplx> Z((size_t)4 * nev * nev);
    if (hostla::herm_eig_lowest(2 * nev, Hs.data(), 2 * nev, 2 * nev, Mv.data(), Z.data(),
                                2 * nev) != 0)  // Q^H T_m Q = Z M Z^H
      throw ApiError{EIGCG_EBREAKDOWN, "restart eigensolver failed"};
    std::vector<cplx> QZ((size_t)m * 2 * nev);
    hostla::matmul_sparse_a(m, 2 * nev, 2 * nev, Q.data(), m, Z.data(), 2 * nev, QZ.data(), m);
    // V <- V (QZ) on the device, in place over the restart block
    hipEvent_t ev = c.events[4 + col];
    c.check(hipEventSynchronize(ev), "qz slot wait");
    double2* hq = c.h_small + qz_off(col);
    double2* dq = c.d_small + qz_off(col);
    for (size_t q = 0; q < QZ.size(); ++q) hq[q] = make_double2(QZ[q].real(), QZ[q].imag());
    c.check(hipMemcpyAsync(dq, hq, sizeof(double2) * QZ.size(), hipMemcpyHostToDevice, c.stream),
            "qz upload");
    std::vector<const void*> in;
    window_cols(col, E, in);
    const bool pp = restart_pingpong(c.P);
    const int nh = pp ? 1 - e.vr_half : e.vr_half;  // output half
    std::vector<void*> out(2 * nev);
    for (int q = 0; q < 2 * nev; ++q) out[q] = vrcol_half(col, nh, q);
    const int nmax = restart_group(c.P);
    for (int n0 = 0; n0 < 2 * nev; n0 += nmax) {
      const int nn = std::min(nmax, 2 * nev - n0);
      c.check(launch_gemm_tall(prec, c.cs, m, nn, in.data(), out.data() + n0, dq + (size_t)n0 * m,
                               0, 0, c.stream),
              "restart gemm");
    }
    c.check(hipEventRecord(ev, c.stream), "event");
    e.vr_half = nh;
    e.has_vr = true;
    e.Mv = Mv;
    e.k_lo = E + 1;
    e.arrow_J = E + 1;
    e.arrow_state = 1;
    e.next_full = E + period;
    e.restarts++;
  }

  // arrow row: w = t_J - beta_J t_{J-1} = A r; arrow = V^H w (conj-transposed later)
  void enqueue_arrow(int col) {
    EigCol& e = ec[col];
    const int J = e.arrow_J;
    const double bJ = beta(col, J);
    void* tJ = col_ptr(w.tbuf, prec, c.cs, (size_t)col * 2 + (J & 1));
    void* tJ1 = col_ptr(w.tbuf, prec, c.cs, (size_t)col * 2 + ((J - 1) & 1));
    void* wv = col_ptr(w.w, prec, c.cs, col);
    // w = tJ - bJ tJ1: copy, then axpy
    c.check(launch_copy(prec, prec, 1, c.cs, tJ, c.cs, wv, c.cs, c.stream), "copy");
    c.check(launch_axpy(prec, 1, c.cs, nullptr, -bJ, 0.0, tJ1, c.cs, wv, c.cs, c.stream), "axpy");
    std::vector<const void*> in(2 * nev), rc(1, wv);
    for (int q = 0; q < 2 * nev; ++q) in[q] = vrcol(col, q);
    double2* G = c.d_small + arrow_off(col);
    c.check(launch_gemm_reduce(prec, c.cs, 2 * nev, 1, in.data(), rc.data(), c.d_gpart,
                               c.gpart_elems, G, c.stream),
            "arrow gemm");
    c.check(hipMemcpyAsync(c.h_small + arrow_off(col), G,
                           sizeof(double2) * 2 * nev, hipMemcpyDeviceToHost, c.stream),
            "arrow copy");
    c.check(hipEventRecord(c.events[4 + kMaxCols + col], c.stream), "event");
    e.arrow_state = 2;
  }

  // final Rayleigh-Ritz on T_i and the nev Ritz vectors (eigCG output)
  void finalize_eig(int col, int j) {
    EigCol& e = ec[col];
    if (e.finalized) return;
    e.finalized = true;
    if (j < 1) return;
    if (e.has_vr && e.arrow_state == 1) enqueue_arrow(col);
    if (e.has_vr) wait_arrow(col);
    std::vector<cplx> T;
    const int i = build_T(col, j, T, m);
    const int k = std::min(nev, i);
    std::vector<double> th(i);
    std::vector<cplx> Y((size_t)i * k);
    if (hostla::herm_eig_lowest(i, T.data(), m, k, th.data(), Y.data(), i) != 0)
      throw ApiError{EIGCG_EBREAKDOWN, "final eigensolver failed"};
    c.amax = std::max(c.amax, th[i - 1]);
    e.ritz_vals.assign(th.begin(), th.begin() + k);
    e.nritz = k;
    std::vector<const void*> in;
    window_cols(col, j, in);
    std::vector<void*> out(k);
    for (int q = 0; q < k; ++q) out[q] = col_ptr(w.ritz, prec, c.cs, (size_t)col * nev + q);
    c.check(hipStreamSynchronize(c.stream), "sync");
    tall_from_host(c, prec, i, k, in, out, Y.data(), 0, 0);
  }
};

// ---------------------------------------------------------------------------
// the batched iteration driver
// ---------------------------------------------------------------------------

// Precision schemes of a run.  FP64: the whole iteration in FP64 (init-CG
// restart of Section 5.3 host-driven).  Reliable: FP32 inner CG, every
// reliable_every iterations of the run x64 += x32 and r is replaced by the
// FP64 true residual (all columns in lockstep); a column whose recursive
// residual reaches the target waits and is updated alone at the next segment
// boundary, so a column's arithmetic does not depend on the others.  Refine: FP32 inner CG
// per column until its residual falls by inner_rel, then an FP64 outer step
// x64 += e, r = b - A x64, deflation re-applied (each column on its own
// schedule, which keeps results independent of the batch composition).
enum Scheme { kSchemeF64 = 0, kSchemeReliable = 1, kSchemeRefine = 2 };
constexpr double kRefineRel = 1e-4;
// 16-bit storage keeps ~3 decimal digits: inner solves reduce their residual
// by 1e-2 before the next FP64 outer step
constexpr double kRefineRelHalf = 1e-2;

static void cg_start(Run& R, uint32_t mask) {
  if (R.spec) {  // z = P^{-1} r and rho = r^H z = ||r||^2 + s for the first direction
    R.c.check(apply_spectral(R.c, R.c.stream, R.K, mask, R.w.r, R.w.z), "preconditioner");
    R.c.check(launch_spec_rho(R.c.d_st, R.K, mask, R.c.d_specs, R.c.stream), "rho");
  }
  UpdateLaunch L{};
  L.prec = R.prec;
  L.ncols = R.K;
  L.mask = mask;
  L.st = R.c.d_st;
  L.g = &R.c.g;
  L.p = R.w.p; L.p_cs = R.c.cs;
  L.r = R.spec ? R.w.z : R.w.r; L.r_cs = R.c.cs;
  L.ring = R.eig ? R.w.ring : nullptr;
  L.ring_cs = R.c.cs;
  L.ring_len = R.w.ring_len;
  L.ring_col_cs = (size_t)R.w.ring_len * R.c.cs;
  R.c.check(launch_cg_start(L, R.c.stream), "cg start");
}

static int status_of(int reason) {
  if (reason == ReasonConverged) return EIGCG_OK;
  if (reason == ReasonBreakdown) return EIGCG_EBREAKDOWN;
  return EIGCG_ENOTCONV;
}

struct Driver {
  Run R;
  int scheme;
  Workspace& w64;
  int seg, relf;
  uint32_t rel_wait = 0;  // columns waiting for a reliable update
  uint32_t f64_wait = 0;  // FP64 columns stopped at their restart point, waiting for the batch
  bool wait_restarts = false;  // a fixed batch (a solve call): restarts wait for each other
  bool pending = false;
  int pslot = 0, pend = 0, pid = 0, slot = 0;

  Driver(Ctx& c, Workspace& w, Workspace& w64_, int prec, int K, bool eig, int scheme_)
      : R(c, w, prec, K, K >= 32 ? 0xffffffffu : ((1u << K) - 1), eig), scheme(scheme_), w64(w64_) {
    seg = eig ? seg_len_eig(c.P) : std::max(1, c.P.check_every);
    relf = scheme == kSchemeReliable ? std::max(1, c.P.reliable_every) : 0;
  }

  Ctx& c() { return R.c; }
  void* colp(void* base, int prec, int j) { return col_ptr(base, prec, R.c.cs, j); }

  // write the state of the masked columns (pinned staging per column)
  void upload_states(uint32_t m, const std::vector<ColState>& st) {
    Ctx& cx = c();
    for (int j = 0; j < R.K; ++j) {
      if (!((m >> j) & 1u)) continue;
      hipEvent_t ev = cx.events[4 + 2 * kMaxCols + j];
      cx.check(hipEventSynchronize(ev), "upload slot");
      ColState* h = cx.h_st + 2 * kMaxCols + j;
      *h = st[j];
      cx.check(hipMemcpyAsync(cx.d_st + j, h, sizeof(ColState), hipMemcpyHostToDevice, cx.stream),
               "state upload");
      cx.check(hipEventRecord(ev, cx.stream), "event");
    }
  }

  // Start the masked columns: b and the initial guess x are in the FP64 work
  // vectors (internal layout).  With deflate, x += U H^-1 U^H (b - A x).
  void start_columns(uint32_t m, const std::vector<double>& bn2, double tol, double restart_tol,
                     bool deflate) {
    Ctx& cx = c();
    std::vector<ColState> st(R.K);
    for (int j = 0; j < R.K; ++j) {
      if (!((m >> j) & 1u)) continue;
      ColState& S = st[j];
      std::memset(&S, 0, sizeof(S));
      S.max_iter = cx.P.max_iter;
      S.scale = 1.0;
      S.state = ColRun;
      const double t2 = tol * tol * bn2[j];
      S.res_stop2 = t2;
      if (scheme == kSchemeF64) {
        S.stop2 = t2;
        S.restart2 = restart_tol > tol ? restart_tol * restart_tol * bn2[j] : 0.0;
      } else if (scheme == kSchemeRefine) {
        const double rel = restart_tol > 0 ? restart_tol : kRefineRel;
        S.inner_rel2 = rel * rel;
      } else {
        // reliable updates: a column whose recursive residual reaches the
        // target waits for the next FP64 update (run at once), which decides
        // convergence on the true residual; iterating on would take the
        // inner recursion towards FP32 underflow
        S.restart2 = t2;
      }
      if (R.eig) {
        S.save_t0 = R.m;
        S.save_t1 = R.m + 1;
        S.tperiod = R.period;
      }
    }
    upload_states(m, st);
    Workspace& w = R.w;
    if (scheme == kSchemeF64) {
      if (deflate && cx.l > 0) {
        true_residual(cx, kF64, R.K, m, w.x, w.b, w.r, w.tmp);
        deflate_columns(cx, kF64, R.K, m, w.x, w.r);
      }
      true_residual(cx, kF64, R.K, m, w.x, w.b, w.r, w.tmp);
    } else {
      for (int j = 0; j < R.K; ++j)
        if ((m >> j) & 1u)
          cx.check(hipMemsetAsync(colp(w.x, kF32, j), 0, cx.cs * 8, cx.stream), "zero e");
      true_residual(cx, kF64, R.K, m, w64.x, w64.b, w64.r, w64.tmp);
      if (deflate && cx.l > 0) deflate_mixed(m);
      if (R.prec == kF32)
        cx.check(launch_copy(kF64, kF32, R.K, cx.cs, w64.r, cx.cs, w.r, cx.cs, cx.stream, m), "copy");
    }
    cx.check(launch_post_residual(cx.d_st, R.K, m, cx.stream), "post");
    if (R.prec == kF16) to_inner16(m);
    cg_start(R, m);
    for (int j = 0; j < R.K; ++j) {
      if (!((m >> j) & 1u)) continue;
      R.done[j] = 0;
      R.reason[j] = 0;
      R.iters[j] = 0;
      R.outer[j] = 0;
      R.first_leg[j] = -1;
      R.ec[j] = EigCol();
      R.ec[j].next_full = R.m;
      R.hist_read[j] = 0;
      R.stale_until[j] = R.seg_id;  // snapshots already in flight predate this start
    }
  }

  // FP32 residual scratch for the deflation of a mixed-precision column: the
  // inner residual itself for FP32 iterations, the FP64 tmp field (viewed as
  // FP32 columns) for 16-bit ones
  void* r32_scratch() { return R.prec == kF32 ? R.w.r : w64.tmp; }

  // init-CG deflation (eq. (2.1)) of the masked columns with the FP32 bank:
  // x64 += U H^-1 U^H r64, then the FP64 true residual again
  void deflate_mixed(uint32_t m) {
    Ctx& cx = c();
    void* r32 = r32_scratch();
    cx.check(launch_copy(kF64, kF32, R.K, cx.cs, w64.r, cx.cs, r32, cx.cs, cx.stream, m), "copy");
    deflate_columns(cx, kF32, R.K, m, R.w.x, r32);
    cx.check(launch_accum_f32_into_f64(R.K, cx.cs, w64.x, cx.cs, R.w.x, cx.cs, cx.stream, m),
             "accum");
    true_residual(cx, kF64, R.K, m, w64.x, w64.b, w64.r, w64.tmp);
  }

  // 16-bit inner solve of the masked running columns: scale the FP64
  // residual to an RMS entry of 2^-5 (well inside the half range while the
  // inner solve reduces it by its tolerance) and store it in 16 bits
  void to_inner16(uint32_t m) {
    Ctx& cx = c();
    const double c0 = std::sqrt((double)cx.cs) / 32.0;
    cx.check(launch_set_scale(cx.d_st, R.K, m, c0, cx.stream), "scale");
    cx.check(launch_to_inner16(R.K, cx.cs, w64.r, cx.cs, R.w.r, cx.cs, m, cx.d_st, cx.stream),
             "to f16");
  }

  // inner correction into the FP64 iterate (undoing the 16-bit scale)
  void accum_inner(uint32_t m) {
    Ctx& cx = c();
    cx.check(launch_accum_f32_into_f64(R.K, cx.cs, w64.x, cx.cs, R.w.x, cx.cs, cx.stream, m,
                                       R.prec == kF16 ? cx.d_st : nullptr),
             "accum");
  }

  // FP64 reliable update of the masked columns (every column of the run in
  // lockstep at the periodic updates; a waiting column alone otherwise)
  void reliable_update(uint32_t m) {
    Ctx& cx = c();
    for (int j = 0; j < R.K; ++j)
      if (((m >> j) & 1u) && !R.done[j]) R.outer[j]++;
    cx.check(launch_accum_f32_into_f64(R.K, cx.cs, w64.x, cx.cs, R.w.x, cx.cs, cx.stream, m), "accum");
    true_residual(cx, kF64, R.K, m, w64.x, w64.b, w64.r, w64.tmp);
    cx.check(launch_copy(kF64, kF32, R.K, cx.cs, w64.r, cx.cs, R.w.r, cx.cs, cx.stream, m), "copy");
    cx.check(launch_post_residual(cx.d_st, R.K, m, cx.stream), "post");
    cx.check(launch_reliable_fix_p(kF32, R.K, m, cx.cs, R.w.r, R.w.p, cx.cs, cx.d_st, cx.d_partial,
                                   cx.stream),
             "fix p");
  }

  // init-CG restart (Section 5.3) of the masked FP64 columns: deflate their
  // current iterates again (one pass over the bank for all of them; each
  // column's arithmetic is that of its own deflation) and restart CG from them
  void host_restart(uint32_t m) {
    Ctx& cx = c();
    Workspace& w = R.w;
    true_residual(cx, kF64, R.K, m, w.x, w.b, w.r, w.tmp);
    deflate_columns(cx, kF64, R.K, m, w.x, w.r);
    true_residual(cx, kF64, R.K, m, w.x, w.b, w.r, w.tmp);
    cx.check(launch_set_state(cx.d_st, R.K, m, ColRun, ReasonNone, 1, cx.stream), "state");
    cx.check(launch_post_residual(cx.d_st, R.K, m, cx.stream), "post");
    cg_start(R, m);
    for (int j = 0; j < R.K; ++j) {
      if (!((m >> j) & 1u)) continue;
      R.outer[j]++;
      R.stale_until[j] = R.seg_id;
    }
  }

  // FP64 restarts wait for the batch: a column stopped at its restart point
  // keeps its iterate until no other column can still reach its own, then all
  // of them restart together.  A waiting column's restart is the one it would
  // have had at once (its x and r do not change while it waits).
  bool restarts_ready() const {
    for (int j = 0; j < R.K; ++j) {
      if (!((R.mask >> j) & 1u) || R.done[j] || ((f64_wait >> j) & 1u)) continue;
      if (R.outer[j] == 0) return false;  // running, restart still ahead
    }
    return true;
  }

  // FP64 outer step of iterative refinement for the masked mixed-precision
  // columns, together (one pass over the bank U deflates all of them);
  // returns the mask of columns that have converged.
  uint32_t host_refine(uint32_t m) {
    Ctx& cx = c();
    Workspace& w = R.w;
    accum_inner(m);
    true_residual(cx, kF64, R.K, m, w64.x, w64.b, w64.r, w64.tmp);
    cx.check(launch_post_residual(cx.d_st, R.K, m, cx.stream), "post");
    ColState* hs = cx.h_st + 3 * kMaxCols;  // read-back area (not an upload slot)
    cx.check(hipMemcpyAsync(hs, cx.d_st, sizeof(ColState) * R.K, hipMemcpyDeviceToHost, cx.stream),
             "state");
    cx.check(hipStreamSynchronize(cx.stream), "sync");
    uint32_t conv = 0, run = 0;
    for (int j = 0; j < R.K; ++j) {
      if (!((m >> j) & 1u)) continue;
      R.outer[j]++;
      if (hs[j].state == ColStopped && hs[j].reason == ReasonConverged) conv |= 1u << j;
      else run |= 1u << j;
    }
    if (run) {
      if (cx.l > 0) {  // deflation per outer step
        deflate_mixed(run);
        cx.check(launch_post_residual(cx.d_st, R.K, run, cx.stream), "post");
      }
      if (R.prec == kF32)
        cx.check(launch_copy(kF64, kF32, R.K, cx.cs, w64.r, cx.cs, w.r, cx.cs, cx.stream, run),
                 "copy");
      else
        to_inner16(run);
      cg_start(R, run);
      for (int j = 0; j < R.K; ++j)
        if ((run >> j) & 1u) R.stale_until[j] = R.seg_id;
    }
    return conv;
  }

  void process(int pslot_, int end, int id) {
    Ctx& cx = c();
    cx.check(hipEventSynchronize(cx.events[pslot_]), "poll wait");
    const ColState* hs = cx.h_st + pslot_ * kMaxCols;
    uint32_t mref = 0;  // columns due for an FP64 refinement step
    for (int j = 0; j < R.K; ++j) {
      if (!((R.mask >> j) & 1u) || R.done[j]) continue;
      if (id <= R.stale_until[j]) continue;
      const ColState S = hs[j];
      R.iters[j] = S.iter;
      if (R.eig) {
        EigCol& e = R.ec[j];
        if (e.arrow_state == 1 && S.iter >= e.arrow_J) R.enqueue_arrow(j);
        if (S.state == ColRun && S.iter == end && e.next_full == end) R.do_restart(j, end);
      }
      if (S.state == ColRun) continue;
      if (S.reason == ReasonRestart) {
        if (scheme == kSchemeF64) {
          if (R.first_leg[j] < 0) R.first_leg[j] = S.iter;
          f64_wait |= 1u << j;
          if (!wait_restarts) {  // serving slots: other requests keep arriving
            cx.check(hipStreamSynchronize(cx.stream), "sync");
            host_restart(f64_wait);
            f64_wait = 0;
          }
          continue;
        }
        if (scheme == kSchemeRefine) {
          mref |= 1u << j;
          continue;
        }
        rel_wait |= 1u << j;  // kSchemeReliable
        continue;
      }
      R.done[j] = 1;
      R.reason[j] = S.reason;
      if (R.eig) R.finalize_eig(j, S.iter);
    }
    if (f64_wait && restarts_ready()) {
      cx.check(hipStreamSynchronize(cx.stream), "sync");
      host_restart(f64_wait);
      f64_wait = 0;
    }
    if (mref) {
      cx.check(hipStreamSynchronize(cx.stream), "sync");
      const uint32_t conv = host_refine(mref);
      for (int j = 0; j < R.K; ++j) {
        if (!((conv >> j) & 1u)) continue;
        R.done[j] = 1;
        R.reason[j] = ReasonConverged;
      }
    }
  }

  // plan, enqueue and poll one segment; process the previous one
  void step() {
    if (rel_wait) {  // between segments: every column's update is at an iteration boundary
      reliable_update(rel_wait & R.mask);
      rel_wait = 0;
    }
    int end = R.enq_iter + seg;
    if (R.eig)
      for (int j = 0; j < R.K; ++j)
        if (((R.mask >> j) & 1u) && !R.done[j] && R.ec[j].next_full > R.enq_iter)
          end = std::min(end, R.ec[j].next_full);
    if (relf) end = std::min(end, (R.enq_iter / relf + 1) * relf);
    R.enqueue_iters(end - R.enq_iter);
    if (relf && end % relf == 0) reliable_update(R.mask);
    R.enqueue_poll(slot, end);
    const int id = ++R.seg_id;
    if (pending) process(pslot, pend, pid);
    pending = true;
    pslot = slot;
    pend = end;
    pid = id;
    slot ^= 1;
  }

  void finish() {
    c().check(hipStreamSynchronize(c().stream), "sync");
    if (pending) process(pslot, pend, pid);
    pending = false;
    c().check(hipStreamSynchronize(c().stream), "sync");
  }

  bool all_done(uint32_t m) const {
    for (int j = 0; j < R.K; ++j)
      if (((m >> j) & 1u) && !R.done[j]) return false;
    return true;
  }

  // columns not seen stopped (iteration cap of the host loop): final states
  void settle(uint32_t m) {
    Ctx& cx = c();
    cx.check(hipMemcpy(cx.h_st, cx.d_st, sizeof(ColState) * R.K, hipMemcpyDeviceToHost), "states");
    for (int j = 0; j < R.K; ++j) {
      if (!((m >> j) & 1u) || R.done[j]) continue;
      R.iters[j] = cx.h_st[j].iter;
      R.reason[j] = cx.h_st[j].reason == ReasonNone ? ReasonMaxIter : cx.h_st[j].reason;
      R.done[j] = 1;
      if (R.eig) R.finalize_eig(j, cx.h_st[j].iter);
    }
  }

  // final FP64 true residuals of the masked columns (x already final in w64)
  std::vector<double> final_residuals(uint32_t m, const std::vector<double>& bn2) {
    Ctx& cx = c();
    if (scheme != kSchemeF64) accum_inner(m);
    cx.check(launch_set_state(cx.d_st, R.K, m, ColStopped, ReasonConverged, 0, cx.stream), "st");
    true_residual(cx, kF64, R.K, m, w64.x, w64.b, w64.r, w64.tmp);
    cx.check(hipMemcpy(cx.h_st, cx.d_st, sizeof(ColState) * R.K, hipMemcpyDeviceToHost), "states");
    std::vector<double> res(R.K, 0.0);
    for (int j = 0; j < R.K; ++j)
      if ((m >> j) & 1u) res[j] = std::sqrt(cx.h_st[j].rho / bn2[j]);
    return res;
  }
};

// ---------------------------------------------------------------------------
// Dynamic init-CG restart threshold.  Section 5.3 restarts once near machine
// precision and leaves open a threshold chosen from the bank's Ritz values and
// residual norms, trading the condition number that re-deflation restores
// against the cost of restarting.  The rule taken here is a cost model:
//  * contamination: with R_k the residuals of the k lowest Ritz pairs, the sine
//    of the angle between their span and the true invariant subspace lies
//    between ||R_k|| / lambda_max and the Davis-Kahan bound ||R_k|| / gap_k;
//    after a Galerkin projection, eq. (2.1), the residual's components along
//    those eigenvectors are at most that fraction of it, usually far less since
//    a Ritz vector's error spreads over the spectrum.  The model takes the
//    lower end, s_k = ||R_k||_F / lambda_max (s_0 = 0): those directions
//    reappear once CG has reduced the residual by s_k, which is also Section
//    5.3's observation that Ritz vectors keep deflating down to their own
//    residual norm scaled by the norm of A;
//  * bulk: the span is resolved while ||R_k||_F / (theta_{k+1} - theta_k) < 1;
//    b = 1 + the largest such k, kappa = lambda_max / theta_b;
//  * a leg that reduces the residual by f keeps the lowest
//    k'(f) = max{k < b : s_k <= f} directions deflated; the others are outlying
//    eigenvalues in the CG bound:
//    n(f) = |O| + sqrt(kappa)/2 (ln(2/f) + sum_O ln(lambda_max/theta_j - 1));
//  * one restart at tau costs n(tau) + R + n(tol/tau), which is constant
//    between the break points {s_k, tol/s_k}; equal neighbours merge, the
//    cheapest interval wins (then the wider in ln tau, then the larger tau),
//    tau is its geometric midpoint, and the restart is planned only when it is
//    strictly cheaper than n(tol).
// ---------------------------------------------------------------------------
namespace {

struct LegModel {
  const double* th = nullptr;
  std::vector<double> s;
  int b = 1;
  double lam_max = 0.0;
  double cost(double f) const {
    int kp = 0;
    for (int k = 0; k < b; ++k)
      if (s[k] <= f) kp = k;
    const double kappa = lam_max / th[b - 1];
    double extra = 0.0;
    for (int j = kp + 1; j < b; ++j) extra += std::log(std::max(lam_max / th[j - 1] - 1.0, 1.0));
    return (double)(b - 1 - kp) + 0.5 * std::sqrt(kappa) * (std::log(2.0 / f) + extra);
  }
};

}  // namespace

RestartPick restart_model(int l, const double* theta, const double* res, double lam_max,
                          double tol, double restart_cost) {
  RestartPick out{0.0, 0.0, 0.0};
  if (l <= 0) return out;
  LegModel m;
  m.th = theta;
  m.lam_max = lam_max;
  m.s.assign(l, 0.0);
  for (int k = 1; k < l; ++k) {
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += res[j] * res[j];
    const double rk = std::sqrt(acc);
    m.s[k] = rk / lam_max;
    const double gap = theta[k] - theta[k - 1];
    if (gap > 0.0 && rk / gap < 1.0) m.b = k + 1;
  }
  const double none = m.cost(tol);
  std::vector<double> pts{tol, 1.0};
  for (int k = 1; k < l; ++k) {
    const double cand[2] = {m.s[k], m.s[k] > 0.0 ? tol / m.s[k] : 0.0};
    for (double p : cand)
      if (tol < p && p < 1.0) pts.push_back(p);
  }
  std::sort(pts.begin(), pts.end());
  pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
  struct Iv { double lo, hi, c; };
  std::vector<Iv> merged;
  for (size_t i = 0; i + 1 < pts.size(); ++i) {
    const double lo = pts[i], hi = pts[i + 1];
    const double mid = std::sqrt(lo * hi);
    const double c = m.cost(mid) + restart_cost + m.cost(tol / mid);
    if (!merged.empty() && std::fabs(merged.back().c - c) <= 1e-12 * std::max(1.0, std::fabs(c)))
      merged.back().hi = hi;
    else
      merged.push_back({lo, hi, c});
  }
  const Iv* best = nullptr;
  for (const Iv& v : merged) {
    if (!best) { best = &v; continue; }
    const double wv = -std::log(v.hi / v.lo), wb = -std::log(best->hi / best->lo);
    if (v.c < best->c || (v.c == best->c && (wv < wb || (wv == wb && -v.hi < -best->hi))))
      best = &v;
  }
  out.cost_none = none;
  out.cost_with = none;
  if (best && best->c < none) {
    out.tau = std::sqrt(best->lo * best->hi);
    out.cost_with = best->c;
  }
  return out;
}

namespace {

void check_finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) throw ApiError{EIGCG_EINVAL, "right-hand side has NaN or Inf"};
}

std::vector<double> col_norms(Ctx& c, int prec, int k, const void* base) {
  c.check(launch_norm2(prec, k, c.cs, base, c.cs, c.d_partial, c.d_counter, c.d_norm, c.stream),
          "norm");
  c.check(hipMemcpyAsync(c.h_norm, c.d_norm, sizeof(double) * k, hipMemcpyDeviceToHost, c.stream),
          "norm copy");
  c.check(hipStreamSynchronize(c.stream), "sync");
  return std::vector<double>(c.h_norm, c.h_norm + k);
}

int scheme_for(const Ctx& c, int mode) {
  if (c.P.precision == EIGCG_FP64) return kSchemeF64;
  if (c.P.precision == EIGCG_MIXED_HALF) return kSchemeRefine;  // rescaled 16-bit inner solves
  return mode == EIGCG_MODE_INITCG ? kSchemeRefine : kSchemeReliable;
}

// Section 5.3's fixed threshold: within an order of magnitude of machine
// precision scaled by the norm of A.  The paper's runs are in single precision
// (Section 5.1) and its convergence figure restarts close to single machine
// precision, which is where a bank of Ritz vectors of that accuracy stops
// deflating: 10 u ||A|| with u = 2^-24, ||A|| estimated by the largest Ritz
// value seen (or (8+|m|)^2)
double anorm_estimate(const Ctx& c) {
  const double am = std::fabs(c.P.mass);
  return c.amax > 0 ? c.amax : (8.0 + am) * (8.0 + am);
}

double fixed_restart_tol(const Ctx& c) { return 10.0 * 5.9604644775390625e-8 * anorm_estimate(c); }

// Iterations one init-CG restart costs, from algorithmic bytes per site: the
// restart recomputes r = b - A x (one application of A), forms U^H r and
// x += U y (two passes over the l bank columns) and touches x, r and b; one
// FP64 CG iteration is an application of A (two stencil passes: spinor in and
// out, four links) plus its BLAS passes (nine spinors).
double restart_cost_estimate(const Ctx& c) {
  const double vec = 192.0;
  const double vbank = c.bank_prec == kF64 ? 192.0 : 96.0;
  const double links = c.comp64 ? 4.0 * 96.0 : 4.0 * 144.0;
  const double apply_a = 2.0 * (2.0 * vec + links);
  const double iteration = apply_a + 9.0 * vec;
  const double restart = apply_a + 2.0 * c.l * vbank + 4.0 * vec;
  return restart / iteration;
}

// Ritz values and residual norms of the bank, recomputed when U or H changed
// (l applications of A).  Uses the bank-precision workspace: call only while no
// solve holds live columns in it.
void ensure_restart_inputs(Ctx& c) {
  if (c.rm_gen == c.bank_gen) return;
  const int l = c.l, ld = c.P.max_bank;
  c.rm_theta.assign(l, 0.0);
  c.rm_res.assign(l, 0.0);
  if (l > 0) {
    std::vector<cplx> Y((size_t)l * l);
    if (hostla::herm_eig_lowest(l, c.H.data(), ld, l, c.rm_theta.data(), Y.data(), l) != 0)
      throw ApiError{EIGCG_EBREAKDOWN, "bank eigensolver failed"};
    bank_ritz_residuals(c, 0, l, c.rm_theta, Y, c.rm_res.data());
  }
  c.rm_gen = c.bank_gen;
}

double restart_tol_for(Ctx& c, int mode, int scheme, double tol, bool may_compute) {
  if (scheme == kSchemeRefine)
    return c.P.restart_tol > 0 ? c.P.restart_tol
                               : (c.P.precision == EIGCG_MIXED_HALF ? kRefineRelHalf : kRefineRel);
  if (mode != EIGCG_MODE_INITCG || c.P.restart_tol < 0) return 0.0;
  if (c.P.restart_rule == EIGCG_RESTART_DYNAMIC) {
    if (c.l < 2) return 0.0;
    if (c.rm_gen != c.bank_gen) {
      if (!may_compute)
        throw ApiError{EIGCG_EINVAL, "internal: restart-model inputs are stale inside a session"};
      ensure_restart_inputs(c);
    }
    if (!(c.rm_theta[0] > 0.0)) return fixed_restart_tol(c);  // H not numerically SPD
    const double cost = c.P.restart_cost > 0 ? c.P.restart_cost : restart_cost_estimate(c);
    return restart_model(c.l, c.rm_theta.data(), c.rm_res.data(), anorm_estimate(c), tol, cost)
        .tau;
  }
  if (c.P.restart_tol > 0) return c.P.restart_tol;
  return fixed_restart_tol(c);
}

}  // namespace

// Section 4: orthonormalise the Ritz vectors of one column against U and among
// themselves (classical Gram-Schmidt twice), W = A Vbar, grow H by the new
// rows/columns and append Vbar to U.  Returns the number of vectors added.
void ensure_bank(Ctx& c) {
  if (!c.U) c.U = c.dalloc(c.cs * elem_bytes(c.bank_prec) * (size_t)c.P.max_bank);
  if (!c.bwork) c.bwork = c.dalloc(c.cs * elem_bytes(c.bank_prec) * (size_t)2 * c.P.nev);
  if (c.bank_prec == kF32 && !c.bwork64) c.bwork64 = c.dalloc(c.cs * 16 * (size_t)2);
}

// Number of leading columns of the Hermitian H (n x n, column-major, ld)
// whose Cholesky pivots exceed rel * H_jj: the largest leading block that is
// numerically positive definite at that relative accuracy.
static int chol_leading(const std::vector<cplx>& H, int n, int ld, double rel) {
  std::vector<cplx> L((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = j; i < n; ++i) L[(size_t)j * n + i] = H[(size_t)j * ld + i];
  for (int j = 0; j < n; ++j) {
    double s = L[(size_t)j * n + j].real();
    for (int k = 0; k < j; ++k) s -= std::norm(L[(size_t)k * n + j]);
    if (!(s > rel * H[(size_t)j * ld + j].real())) return j;
    const double ljj = std::sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      cplx t = L[(size_t)j * n + i];
      for (int k = 0; k < j; ++k) t -= L[(size_t)k * n + i] * std::conj(L[(size_t)k * n + j]);
      L[(size_t)j * n + i] = t / ljj;
    }
  }
  return n;
}

// src: k contiguous fields (bank precision) of new directions; they may
// already sit in the bank slots l..l+k-1.
int bank_append_from(Ctx& c, const void* src, int nsrc) {
  const int prec = c.bank_prec;
  const int nev = c.P.nev;
  const int room = c.P.max_bank - c.l;
  const int k = std::min(nsrc, room);
  if (k <= 0) return 0;
  ensure_bank(c);
  const int l = c.l;
  // norms before projection (drop test), then copy into the bank slots
  c.check(launch_norm2(prec, k, c.cs, src, c.cs, c.d_partial, c.d_counter, c.d_norm, c.stream),
          "norm");
  c.check(hipMemcpyAsync(c.h_norm, c.d_norm, sizeof(double) * k, hipMemcpyDeviceToHost, c.stream),
          "norm copy");
  c.check(hipStreamSynchronize(c.stream), "sync");
  std::vector<double> n0(c.h_norm, c.h_norm + k);
  void* vb = col_ptr(c.U, prec, c.cs, l);
  if (vb != src) c.check(launch_copy(prec, prec, k, c.cs, src, c.cs, vb, c.cs, c.stream), "copy");
  std::vector<const void*> ucols(l);
  for (int i = 0; i < l; ++i) ucols[i] = col_ptr(c.U, prec, c.cs, i);
  // CGS2 against U
  if (l > 0) {
    std::vector<const void*> rc(k);
    std::vector<void*> out(k);
    for (int q = 0; q < k; ++q) {
      rc[q] = col_ptr(c.U, prec, c.cs, l + q);
      out[q] = col_ptr(c.U, prec, c.cs, l + q);
    }
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<cplx> G;
      reduce_to_host(c, prec, l, k, ucols, rc, G);
      tall_from_host(c, prec, l, k, ucols, out, G.data(), 1, 1);
    }
  }
  // CGS2 inside the new block, column by column, with the drop rule
  int kept = 0;
  for (int q = 0; q < k; ++q) {
    void* v = col_ptr(c.U, prec, c.cs, l + q);
    void* dst = col_ptr(c.U, prec, c.cs, l + kept);
    if (kept > 0) {
      std::vector<const void*> prev(kept), rc(1, v);
      std::vector<void*> out(1, v);
      for (int i = 0; i < kept; ++i) prev[i] = col_ptr(c.U, prec, c.cs, l + i);
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<cplx> g;
        reduce_to_host(c, prec, kept, 1, prev, rc, g);
        tall_from_host(c, prec, kept, 1, prev, out, g.data(), 1, 1);
      }
    }
    c.check(launch_norm2(prec, 1, c.cs, v, c.cs, c.d_partial, c.d_counter, c.d_norm, c.stream),
            "norm");
    c.check(hipMemcpyAsync(c.h_norm, c.d_norm, sizeof(double), hipMemcpyDeviceToHost, c.stream),
            "norm copy");
    c.check(hipStreamSynchronize(c.stream), "sync");
    const double nrm = std::sqrt(c.h_norm[0]);
    // drop rule of Section 4 (1e-10 of the input norm) for an FP64 bank.  An
    // FP32 bank's projection coefficients carry FP32 dot-product errors
    // (~1e-6 of the input norm), which a small remainder would amplify into
    // large overlaps with U after normalisation: remainders below 1e-2 of the
    // input are dropped
    const double drop = prec == kF64 ? 1e-10 : 1e-2;
    if (!(nrm > drop * std::sqrt(n0[q]))) continue;
    const double inv = 1.0 / nrm;
    // scale into its final slot
    if (dst != v) c.check(launch_copy(prec, prec, 1, c.cs, v, c.cs, dst, c.cs, c.stream), "copy");
    c.h_norm[1] = inv;
    c.check(hipMemcpyAsync(c.d_norm + 1, c.h_norm + 1, sizeof(double), hipMemcpyHostToDevice,
                           c.stream),
            "scale upload");
    c.check(launch_scale(prec, 1, c.cs, c.d_norm + 1, dst, c.cs, c.stream), "scale");
    c.check(hipStreamSynchronize(c.stream), "sync");
    ++kept;
  }
  if (kept == 0) return 0;
  // W = A Vbar, then [U Vbar]^H W (kept <= nev; the work area holds 2 nev fields)
  void* W = c.bwork;
  void* tmp = col_ptr(c.bwork, prec, c.cs, nev);
  for (int q = 0; q < kept; ++q) {
    if (prec == kF64) {
      stencil_store(c, prec, kOpM, 1, col_ptr(c.U, prec, c.cs, l + q), tmp);
      stencil_store(c, prec, kOpMdag, 1, tmp, col_ptr(W, prec, c.cs, q));
    } else {
      // FP32 bank: A v in FP64 on the exact FP64 image of the stored vector,
      // so low modes (|A v| ~ lambda_min |v|) do not lose their digits to
      // FP32 cancellation; W is then rounded relative to its own size
      void* v64 = c.bwork64;
      void* t64 = col_ptr(c.bwork64, kF64, c.cs, 1);
      c.check(launch_copy(kF32, kF64, 1, c.cs, col_ptr(c.U, prec, c.cs, l + q), c.cs, v64, c.cs,
                          c.stream),
              "to f64");
      stencil_store(c, kF64, kOpM, 1, v64, t64);
      stencil_store(c, kF64, kOpMdag, 1, t64, v64);
      c.check(launch_copy(kF64, kF32, 1, c.cs, v64, c.cs, col_ptr(W, prec, c.cs, q), c.cs,
                          c.stream),
              "to f32");
    }
  }
  // locked columns (Section 4) take no part: their rows of U^H W stay zero
  const int nl = std::min(c.nlock, l);
  const int na = l + kept - nl;
  std::vector<const void*> all(na), wc(kept);
  for (int i = 0; i < na; ++i) all[i] = col_ptr(c.U, prec, c.cs, nl + i);
  for (int q = 0; q < kept; ++q) wc[q] = col_ptr(W, prec, c.cs, q);
  std::vector<cplx> G2;
  reduce_to_host(c, prec, na, kept, all, wc, G2);
  const int ld = c.P.max_bank;
  for (int q = 0; q < kept; ++q) {
    for (int i = 0; i < l + kept; ++i) {
      // (U Vbar)_i^H A vbar_q
      const cplx v = i < nl ? cplx(0.0, 0.0) : G2[(size_t)q * na + (i - nl)];
      c.H[(size_t)(l + q) * ld + i] = v;
      if (i < l) c.H[(size_t)i * ld + (l + q)] = std::conj(v);
    }
  }
  for (int a = 0; a < kept; ++a)  // Hermitian part of the new diagonal block
    for (int b = a; b < kept; ++b) {
      const cplx x = c.H[(size_t)(l + b) * ld + (l + a)];
      const cplx y = c.H[(size_t)(l + a) * ld + (l + b)];
      const cplx h = 0.5 * (x + std::conj(y));
      c.H[(size_t)(l + b) * ld + (l + a)] = h;
      c.H[(size_t)(l + a) * ld + (l + b)] = std::conj(h);
    }
  for (int a = 0; a < kept; ++a) {
    cplx& d = c.H[(size_t)(l + a) * ld + (l + a)];
    d = cplx(d.real(), 0.0);
  }
  // keep the bank a basis on which H stays numerically positive definite (A
  // is HPD, so a failing pivot means a new direction is not independent of
  // the others to the bank's precision): truncate at the first such column
  const int good = chol_leading(c.H, l + kept, ld, prec == kF64 ? 1e-13 : 1e-6);
  if (good < l + kept) kept = std::max(0, good - l);
  c.l = l + kept;
  c.chol_ok = false;
  c.spec_ok = false;
  ++c.bank_gen;
  return kept;
}

// Time of one CG iteration (stencil passes, finalize, update) of a batch of K
// columns in precision prec, from events around reps iterations on the
// context's work vectors (cached per precision and width).
static double cg_iteration_ms(Ctx& c, int prec, int K) {
  const int key = prec * 64 + K;
  auto it = c.iter_ms.find(key);
  if (it != c.iter_ms.end()) return it->second;
  Workspace& w = prec == kF64 ? c.ws64 : c.ws32;
  ws_ensure(c, w, prec, false);
  const size_t vb = c.cs * elem_bytes(prec);
  for (void* v : {w.x, w.p, w.r, w.tmp})
    c.check(hipMemsetAsync(v, 0x3F, vb * w.K, c.stream), "fill");
  const std::vector<double> rn = col_norms(c, prec, K, w.r);
  c.check(launch_copy(prec, prec, K, c.cs, w.r, c.cs, w.p, c.cs, c.stream), "copy");
  std::vector<ColState> st(K);
  std::memset(st.data(), 0, sizeof(ColState) * K);
  for (int j = 0; j < K; ++j) {  // a consistent CG state (r = p) that never stops
    st[j].state = ColRun;
    st[j].rho = rn[j];
    st[j].stop2 = st[j].restart2 = st[j].res_stop2 = -1.0;
    st[j].max_iter = 0x3fffffff;
    st[j].scale = 1.0;
  }
  std::memcpy(c.h_st, st.data(), sizeof(ColState) * K);
  c.check(hipMemcpy(c.d_st, c.h_st, sizeof(ColState) * K, hipMemcpyHostToDevice), "st");
  const int reps = 10;
  ensure_spectral(c);
  Run R(c, w, prec, K, K >= 32 ? 0xffffffffu : ((1u << K) - 1), false);
  hipEvent_t e0, e1;
  c.check(hipEventCreate(&e0), "ev");
  c.check(hipEventCreate(&e1), "ev");
  R.enqueue_iters(2);
  c.check(hipEventRecord(e0, c.stream), "ev");
  R.enqueue_iters(reps);
  c.check(hipEventRecord(e1, c.stream), "ev");
  c.check(hipEventSynchronize(e1), "ev");
  float ms = 0.f;
  c.check(hipEventElapsedTime(&ms, e0, e1), "ev");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (void* v : {w.x, w.p, w.r, w.tmp}) c.check(hipMemsetAsync(v, 0, vb * w.K, c.stream), "clear");
  c.check(hipStreamSynchronize(c.stream), "sync");
  const double t = (double)ms / reps;
  c.iter_ms[key] = t;
  return t;
}

// The dynamic switch from Incremental eigCG to init-CG (Section 5.5: run
// eigCG for the number of right-hand sides that minimises the total time,
// monitored at run time).  After `done` eigCG groups with mean iterations
// iters[] and wall times secs[], with `left` groups still to solve (the next
// one included) and room for `bank_room` more nev-blocks in U: one more eigCG
// group pays its overhead over plain iterations (estimated by the last group:
// secs - iters * iter_ms) to shorten each of the later left - 1 groups by the
// next drop in iterations, predicted as the mean drop over the last (up to
// three) groups, which smooths the spread of iteration counts between
// right-hand sides.  Returns true to run the next group with eigCG.
bool auto_continue(int done, int left, const double* iters, const double* secs, double iter_ms,
                   int bank_room) {
  if (bank_room <= 0 || left <= 1) return false;
  if (done < 3) return true;  // the first drops are measured over three groups
  const int w = std::min(done - 1, 3);
  const double d = (iters[done - 1 - w] - iters[done - 1]) / w;
  if (!(d > 0.0)) return false;
  const double gain_s = (left - 1) * d * iter_ms * 1e-3;
  const double over_s = std::max(0.0, secs[done - 1] - iters[done - 1] * iter_ms * 1e-3);
  return over_s < gain_s;
}

// FP64 init-CG guesses, eq. (2.1), of right-hand sides [first, first +
// count) in groups of up to kMaxCols columns: x <- x + U H^-1 U^H (b - A x)
// in the caller's x, so that one pass over the bank U serves a group instead
// of one right-hand side.  Each column's arithmetic is that of its own
// deflation (the stencil and both products treat columns independently).
// Returns false, having changed nothing, when the group workspace cannot be
// allocated.
// The FP64 workspace of several columns at once (b, x, r, tmp; up to kMaxCols
// columns, fewer when memory is short), allocated on first use; in an odd-even
// context the operator's intermediate grows to its width.  False when not even
// two columns fit.
static bool ensure_wsg(Ctx& c) {
  Workspace& g = c.wsg;
  if (g.K == 0) {
    const size_t vb = c.cs * 16;
    for (int k = kMaxCols; k >= 2 && g.K == 0; k /= 2) {
      try {
        g.b = c.dalloc(vb * k);
        g.x = c.dalloc(vb * k);
        g.r = c.dalloc(vb * k);
        g.tmp = c.dalloc(vb * k);
        g.K = k;
        g.prec = kF64;
      } catch (const ApiError&) {  // budget or device memory: try fewer columns
        c.dfree(g.b); c.dfree(g.x); c.dfree(g.r); c.dfree(g.tmp);
      }
    }
    if (g.K == 0) return false;
  }
  // the odd-even operator's intermediate holds max_batch columns; the
  // group's residual pass needs g.K of them
  if (c.g.eo && (size_t)g.K > c.eo_cols64) {
    void* t = nullptr;
    try {
      t = c.dalloc((size_t)g.K * c.cs * 16);
    } catch (const ApiError&) {
      return false;
    }
    c.dfree(c.eo_tmp64);
    c.eo_tmp64 = t;
    c.eo_cols64 = (size_t)g.K;
  }
  return true;
}

// FP64 init-CG guesses, eq. (2.1), for count right-hand sides from first, a
// group of workspace columns per pass over U
static bool batched_guess(Ctx& c, int first, int count, const void* b_aos, void* x_aos) {
  if (!ensure_wsg(c)) return false;
  Workspace& g = c.wsg;
  std::vector<ColState> st(kMaxCols);
  std::memset(st.data(), 0, sizeof(ColState) * kMaxCols);
  for (auto& s : st) s.state = ColStopped;
  for (int c0 = first; c0 < first + count; c0 += g.K) {
    const int k = std::min(g.K, first + count - c0);
    const uint32_t mask = k >= 32 ? 0xffffffffu : ((1u << k) - 1u);
    const double2* bsrc = (const double2*)b_aos + (size_t)c0 * 12 * c.g.V;
    double2* xdst = (double2*)x_aos + (size_t)c0 * 12 * c.g.V;
    check_fields(c, g.b, kF64, k, "guess right-hand sides");
    check_fields(c, g.x, kF64, k, "guess iterates");
    // the residual pass leaves its norms in the column states: keep them idle
    std::memcpy(c.h_st, st.data(), sizeof(ColState) * k);
    c.check(hipMemcpyAsync(c.d_st, c.h_st, sizeof(ColState) * k, hipMemcpyHostToDevice, c.stream),
            "states");
    c.check(launch_spinor_to_soa(bsrc, g.b, kF64, &c.g, k, c.cs, c.stream), "to soa");
    c.check(launch_spinor_to_soa(xdst, g.x, kF64, &c.g, k, c.cs, c.stream), "to soa");
    true_residual(c, kF64, k, mask, g.x, g.b, g.r, g.tmp);
    deflate_columns(c, kF64, k, mask, g.x, g.r);
    c.check(launch_spinor_from_soa(g.x, xdst, kF64, &c.g, k, c.cs, c.stream), "from soa");
    c.check(hipStreamSynchronize(c.stream), "sync");
  }
  return true;
}

int solve(Ctx& c, int nrhs, const void* b_aos, void* x_aos, double tol, int mode,
          eigcg_stats* stats) {
  const bool mixed = c.P.precision != EIGCG_FP64;
  // 16-bit inner solves cannot run eigCG: the automatic mode is init-CG there
  if (mode == EIGCG_MODE_AUTO && c.P.precision == EIGCG_MIXED_HALF) mode = EIGCG_MODE_INITCG;
  const bool automatic = mode == EIGCG_MODE_AUTO;
  if (mode == EIGCG_MODE_EIGCG && c.P.precision == EIGCG_MIXED_HALF)
    throw ApiError{EIGCG_EINVAL, "eigCG mode needs FP64 or FP32 iterations (16-bit inner solves "
                                 "restart at every refinement step)"};
  const bool any_eig = mode == EIGCG_MODE_EIGCG || mode == EIGCG_MODE_AUTO;
  const int prec = mixed ? c.iprec : kF64;
  // eigCG groups run min(max_batch, nrhs) columns: the window holds that many
  const int keig = std::min(c.P.max_batch, nrhs);
  ws_ensure(c, c.ws64, kF64, any_eig && !mixed, keig);
  if (mixed) ws_ensure(c, c.ws32, c.iprec, any_eig, keig);
  Workspace& w = mixed ? c.ws32 : c.ws64;
  Workspace& w64 = c.ws64;
  int worst = EIGCG_OK;
  c.last_ritz.clear();
  std::vector<double> auto_iters, auto_secs;  // eigCG groups of the automatic mode
  bool auto_eig = true;
  int guessed_from = nrhs;  // right-hand sides from here on carry their deflated guess
  for (int c0 = 0; c0 < nrhs; c0 += w.K) {
    const int K = std::min(w.K, nrhs - c0);
    int gmode = mode;
    if (automatic) {
      if (auto_eig) {
        const int left = (nrhs - c0 + w.K - 1) / w.K;
        const int room = (c.P.max_bank - c.l) / std::max(1, c.P.nev * K);
        const double it_ms = auto_iters.size() >= 3 ? cg_iteration_ms(c, prec, K) : 0.0;
        auto_eig = auto_continue((int)auto_iters.size(), left, auto_iters.data(),
                                 auto_secs.data(), it_ms, room);
      }
      gmode = auto_eig ? EIGCG_MODE_EIGCG : EIGCG_MODE_INITCG;
    }
    const bool eig = gmode == EIGCG_MODE_EIGCG;
    const int scheme = scheme_for(c, gmode);
    // FP64 init-CG over more than one batch: the bank is fixed from here on,
    // so the guesses of all remaining right-hand sides are formed in groups
    if (gmode == EIGCG_MODE_INITCG && scheme == kSchemeF64 && c.l > 0 && c0 < guessed_from &&
        nrhs - c0 > w.K && batched_guess(c, c0, nrhs - c0, b_aos, x_aos))
      guessed_from = c0;
    const double rtol = restart_tol_for(c, gmode, scheme, tol, true);
    const double t0 = now_s();
    const double2* bsrc = (const double2*)b_aos + (size_t)c0 * 12 * c.g.V;
    double2* xdst = (double2*)x_aos + (size_t)c0 * 12 * c.g.V;
    check_fields(c, w64.b, kF64, K, "right-hand sides");
    check_fields(c, w64.x, kF64, K, "iterates");
    c.check(launch_spinor_to_soa(bsrc, w64.b, kF64, &c.g, K, c.cs, c.stream), "to soa");
    c.check(launch_spinor_to_soa(xdst, w64.x, kF64, &c.g, K, c.cs, c.stream), "to soa");
    std::vector<double> bn2 = col_norms(c, kF64, K, w64.b);
    check_finite(bn2);
    uint32_t mask = 0;
    for (int j = 0; j < K; ++j) {
      if (bn2[j] > 0.0) {
        mask |= 1u << j;
      } else {  // b = 0: x = 0
        c.check(hipMemsetAsync(col_ptr(w64.x, kF64, c.cs, j), 0, c.cs * 16, c.stream), "zero");
      }
    }
    ensure_spectral(c);  // the bank may have grown since the last group
    Driver D(c, w, w64, prec, K, eig, scheme);
    D.wait_restarts = true;
    {  // columns with b = 0 never run
      std::vector<ColState> idle(K);
      std::memset(idle.data(), 0, sizeof(ColState) * K);
      for (auto& s : idle) {
        s.state = ColStopped;
        s.reason = ReasonConverged;
      }
      D.upload_states(D.R.mask & ~mask, idle);
    }
    std::vector<double> res(K, 0.0);
    if (mask) {
      D.start_columns(mask, bn2, tol, rtol, gmode != EIGCG_MODE_CG && c0 < guessed_from);
      const int hard_cap = c.P.max_iter + 4 * D.seg + 8;
      while (!D.all_done(mask) && D.R.enq_iter <= hard_cap) D.step();
      D.finish();
      D.settle(mask);
      res = D.final_residuals(mask, bn2);
    }
    c.check(launch_spinor_from_soa(w64.x, xdst, kF64, &c.g, K, c.cs, c.stream), "from soa");
    c.check(hipStreamSynchronize(c.stream), "sync");
    // Incremental eigCG: append each column's Ritz vectors in column order
    std::vector<int> added(K, 0);
    if (eig) {
      for (int j = 0; j < K; ++j) {
        if (!((mask >> j) & 1u)) continue;
        const EigCol& e = D.R.ec[j];
        for (double v : e.ritz_vals) c.last_ritz.push_back(v);
        for (int q0 = 0; q0 < e.nritz; q0 += c.P.nev)
          added[j] += bank_append_from(c, col_ptr(w.ritz, prec, c.cs, (size_t)j * c.P.nev + q0),
                                       std::min(c.P.nev, e.nritz - q0));
      }
    }
    const double dt = now_s() - t0;
    if (automatic && eig && mask) {
      double it = 0.0;
      int n = 0;
      for (int j = 0; j < K; ++j)
        if ((mask >> j) & 1u) { it += D.R.iters[j]; ++n; }
      auto_iters.push_back(it / std::max(1, n));
      auto_secs.push_back(dt);
    }
    for (int j = 0; j < K; ++j) {
      int stt = EIGCG_OK;
      if ((mask >> j) & 1u) {
        stt = status_of(D.R.reason[j]);
        if (stt == EIGCG_OK && !(res[j] <= tol)) stt = EIGCG_ENOTCONV;
      }
      if (stt < worst) worst = stt;
      if (stats) {
        eigcg_stats& s = stats[c0 + j];
        s.iters = D.R.iters[j];
        s.restarts = eig ? D.R.ec[j].restarts : 0;
        s.outer_steps = D.R.outer[j];
        s.status = stt;
        s.true_rel_res = res[j];
        s.seconds = dt;
        s.bank_added = added[j];
        s.nritz = eig ? D.R.ec[j].nritz : 0;
        s.mode_used = gmode;
        s.first_leg_iters = D.R.first_leg[j] >= 0 ? D.R.first_leg[j] : D.R.iters[j];
        s.restart_tau = scheme == kSchemeF64 && gmode == EIGCG_MODE_INITCG ? rtol : 0.0;
      }
    }
  }
  return worst;
}

// ---------------------------------------------------------------------------
// serving sessions: a persistent batched init-CG over max_batch slots
// ---------------------------------------------------------------------------

struct Session {
  Ctx& c;
  Driver D;
  int K;
  std::vector<int> active;
  std::vector<uint64_t> tag;
  std::vector<double> tol, bn2, t_admit, rtau;
  std::vector<void*> xdst;
  Session(Ctx& c_, Workspace& w, Workspace& w64, int prec, int scheme)
      : c(c_), D(c_, w, w64, prec, c_.P.max_batch, false, scheme), K(c_.P.max_batch) {
    active.assign(K, 0);
    tag.assign(K, 0);
    tol.assign(K, 0.0);
    bn2.assign(K, 0.0);
    t_admit.assign(K, 0.0);
    rtau.assign(K, 0.0);
    xdst.assign(K, nullptr);
  }
};

Session* session_open(Ctx& c) {
  const bool mixed = c.P.precision != EIGCG_FP64;
  const int prec = mixed ? c.iprec : kF64;
  ws_ensure(c, c.ws64, kF64, false);
  if (mixed) ws_ensure(c, c.ws32, c.iprec, false);
  ensure_spectral(c);
  // the dynamic restart rule reads the bank's Ritz pairs, computed here while
  // no request holds workspace columns (the bank is fixed while the session lives)
  if (c.P.restart_rule == EIGCG_RESTART_DYNAMIC && c.P.restart_tol >= 0 &&
      scheme_for(c, EIGCG_MODE_INITCG) == kSchemeF64 && c.l >= 2)
    ensure_restart_inputs(c);
  Session* s = new Session(c, mixed ? c.ws32 : c.ws64, c.ws64, prec,
                           scheme_for(c, EIGCG_MODE_INITCG));
  std::vector<ColState> idle(s->K);
  std::memset(idle.data(), 0, sizeof(ColState) * s->K);
  for (auto& st : idle) {
    st.state = ColStopped;
    st.reason = ReasonConverged;
  }
  s->D.upload_states(s->D.R.mask, idle);
  for (int j = 0; j < s->K; ++j) s->D.R.done[j] = 1;
  return s;
}

int session_free_slot(Session* s) {
  for (int j = 0; j < s->K; ++j)
    if (!s->active[j]) return j;
  return -1;
}

int session_active(Session* s) {
  int n = 0;
  for (int j = 0; j < s->K; ++j) n += s->active[j];
  return n;
}

// Admit one request into a free slot (cold start x = 0, init-CG deflation).
// Returns the slot, or -1 when full.  A zero right-hand side completes at once
// (reported through the done list of the next step).
int session_admit(Session* s, const void* b_aos, void* x_aos, double tol, uint64_t tg,
                  std::vector<SessionDone>& done) {
  Ctx& c = s->c;
  const int j = session_free_slot(s);
  if (j < 0) return -1;
  Workspace& w64 = s->D.w64;
  c.check(launch_spinor_to_soa((const double2*)b_aos, col_ptr(w64.b, kF64, c.cs, j), kF64, &c.g, 1,
                               c.cs, c.stream),
          "to soa");
  c.check(hipMemsetAsync(col_ptr(w64.x, kF64, c.cs, j), 0, c.cs * 16, c.stream), "zero x");
  std::vector<double> n = col_norms(c, kF64, 1, col_ptr(w64.b, kF64, c.cs, j));
  check_finite(n);
  if (!(n[0] > 0.0)) {
    c.check(hipMemsetAsync(x_aos, 0, (size_t)12 * c.g.V * 16, c.stream), "zero");
    c.check(hipStreamSynchronize(c.stream), "sync");
    SessionDone d{};
    d.tag = tg;
    d.status = EIGCG_OK;
    done.push_back(d);
    return j;
  }
  std::vector<double> bn2(s->K, 1.0);
  bn2[j] = n[0];
  s->bn2[j] = n[0];
  s->tol[j] = tol;
  s->tag[j] = tg;
  s->xdst[j] = x_aos;
  s->t_admit[j] = now_s();
  try {
    const double rtol = restart_tol_for(c, EIGCG_MODE_INITCG, s->D.scheme, tol, false);
    s->rtau[j] = s->D.scheme == kSchemeF64 ? rtol : 0.0;
    s->D.start_columns(1u << j, bn2, tol, rtol, true);
  } catch (...) {
    // the slot stays free and idle; the caller reports the request as failed
    std::vector<ColState> idle(s->K);
    std::memset(idle.data(), 0, sizeof(ColState) * s->K);
    idle[j].state = ColStopped;
    idle[j].reason = ReasonConverged;
    s->D.upload_states(1u << j, idle);
    s->D.R.done[j] = 1;
    throw;
  }
  s->active[j] = 1;
  return j;
}

// One segment; finished requests are written back and reported.
void session_step(Session* s, std::vector<SessionDone>& done) {
  Ctx& c = s->c;
  if (session_active(s) == 0) return;
  s->D.step();
  uint32_t fin = 0;
  for (int j = 0; j < s->K; ++j)
    if (s->active[j] && s->D.R.done[j]) fin |= 1u << j;
  if (!fin) return;
  std::vector<double> res = s->D.final_residuals(fin, s->bn2);
  for (int j = 0; j < s->K; ++j) {
    if (!((fin >> j) & 1u)) continue;
    c.check(launch_spinor_from_soa(col_ptr(s->D.w64.x, kF64, c.cs, j), (double2*)s->xdst[j], kF64,
                                   &c.g, 1, c.cs, c.stream),
            "from soa");
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
  for (int j = 0; j < s->K; ++j) {
    if (!((fin >> j) & 1u)) continue;
    SessionDone d{};
    d.tag = s->tag[j];
    int stt = status_of(s->D.R.reason[j]);
    if (stt == EIGCG_OK && !(res[j] <= s->tol[j])) stt = EIGCG_ENOTCONV;
    d.status = stt;
    d.iters = s->D.R.iters[j];
    d.outer = s->D.R.outer[j];
    d.first_leg = s->D.R.first_leg[j] >= 0 ? s->D.R.first_leg[j] : s->D.R.iters[j];
    d.restart_tau = s->rtau[j];
    d.true_rel_res = res[j];
    done.push_back(d);
    s->active[j] = 0;
  }
}

void session_close(Session* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->c.stream);
  delete s;
}

void deflate_init(Ctx& c, int nrhs, const void* b_aos, void* x_aos) {
  const bool mixed = c.P.precision != EIGCG_FP64;
  ws_ensure(c, c.ws64, kF64, false);
  if (mixed) ws_ensure(c, c.ws32, c.iprec, false);
  Workspace& w64 = c.ws64;
  for (int c0 = 0; c0 < nrhs; c0 += w64.K) {
    const int K = std::min(w64.K, nrhs - c0);
    const uint32_t mask = (K >= 32) ? 0xffffffffu : ((1u << K) - 1);
    const double2* bsrc = (const double2*)b_aos + (size_t)c0 * 12 * c.g.V;
    double2* xdst = (double2*)x_aos + (size_t)c0 * 12 * c.g.V;
    check_fields(c, w64.b, kF64, K, "right-hand sides");
    check_fields(c, w64.x, kF64, K, "iterates");
    c.check(launch_spinor_to_soa(bsrc, w64.b, kF64, &c.g, K, c.cs, c.stream), "to soa");
    c.check(launch_spinor_to_soa(xdst, w64.x, kF64, &c.g, K, c.cs, c.stream), "to soa");
    if (c.l > 0) {
      std::vector<ColState> st(K);
      std::memset(st.data(), 0, sizeof(ColState) * K);
      for (auto& s : st) s.state = ColStopped;
      std::memcpy(c.h_st, st.data(), sizeof(ColState) * K);
      c.check(hipMemcpy(c.d_st, c.h_st, sizeof(ColState) * K, hipMemcpyHostToDevice), "st");
      true_residual(c, kF64, K, mask, w64.x, w64.b, w64.r, w64.tmp);
      if (!mixed) {
        deflate_columns(c, kF64, K, mask, w64.x, w64.r);
      } else {
        Workspace& w = c.ws32;  // FP32 iterate (also for 16-bit inner solves)
        void* r32 = c.iprec == kF32 ? w.r : w64.tmp;  // FP32 residual scratch
        c.check(hipMemsetAsync(w.x, 0, c.cs * 8 * K, c.stream), "zero");
        c.check(launch_copy(kF64, kF32, K, c.cs, w64.r, c.cs, r32, c.cs, c.stream), "copy");
        deflate_columns(c, kF32, K, mask, w.x, r32);
        c.check(launch_accum_f32_into_f64(K, c.cs, w64.x, c.cs, w.x, c.cs, c.stream), "accum");
      }
    }
    c.check(launch_spinor_from_soa(w64.x, xdst, kF64, &c.g, K, c.cs, c.stream), "from soa");
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
}

// Residual norms ||A u_q - theta_q u_q|| of the Ritz vectors u_q = U_n y_q of
// the n bank columns U_n = U[:, j0 : j0 + n] (Y column-major, n x n), in the
// bank precision, a workspace-width block of Ritz vectors per pass over U_n.
static void bank_ritz_residuals(Ctx& c, int j0, int n, const std::vector<double>& th,
                                const std::vector<cplx>& Y, double* res) {
  const int prec = c.bank_prec;
  // an FP64 bank uses the wide FP64 workspace (up to kMaxCols Ritz vectors per
  // pass over U_n) when it exists or the context's own is narrower than four
  // columns; otherwise the bank-precision workspace, where a 16-bit inner
  // workspace holds half as many FP32 fields per buffer
  Workspace* wp = nullptr;
  int wide = 0;
  if (prec == kF64 && (c.wsg.K > 0 || c.P.max_batch < 4) && ensure_wsg(c)) {
    wp = &c.wsg;
    wide = c.wsg.K;
  } else {
    wp = prec == kF64 ? &c.ws64 : &c.ws32;
    ws_ensure(c, *wp, prec, false);
    wide = wp->prec == prec ? wp->K : wp->K / 2;
  }
  Workspace& w = *wp;
  const int kb = std::max(1, std::min(wide, n));
  std::vector<const void*> in(n);
  for (int i = 0; i < n; ++i) in[i] = col_ptr(c.U, prec, c.cs, j0 + i);
  for (int q0 = 0; q0 < n; q0 += kb) {
    const int nq = std::min(kb, n - q0);
    std::vector<void*> out(nq);
    for (int j = 0; j < nq; ++j) out[j] = col_ptr(w.x, prec, c.cs, j);
    tall_from_host(c, prec, n, nq, in, out, Y.data() + (size_t)q0 * n, 0, 0);
    stencil_store(c, prec, kOpM, nq, w.x, w.tmp);
    stencil_store(c, prec, kOpMdag, nq, w.tmp, w.r);
    for (int j = 0; j < nq; ++j)
      c.check(launch_axpy(prec, 1, c.cs, nullptr, -th[q0 + j], 0.0, col_ptr(w.x, prec, c.cs, j),
                          c.cs, col_ptr(w.r, prec, c.cs, j), c.cs, c.stream),
              "axpy");
    std::vector<double> nn = col_norms(c, prec, nq, w.r);
    for (int j = 0; j < nq; ++j) res[q0 + j] = std::sqrt(nn[j]);
  }
}

void bank_info(Ctx& c, int* l_out, double* vals, double* res) {
  const int l = c.l, ld = c.P.max_bank;
  *l_out = l;
  if (l == 0 || !vals) return;
  std::vector<double> th(l);
  std::vector<cplx> Y((size_t)l * l);
  if (hostla::herm_eig_lowest(l, c.H.data(), ld, res ? l : 0, th.data(), res ? Y.data() : nullptr,
                              l) != 0)
    throw ApiError{EIGCG_EBREAKDOWN, "bank eigensolver failed"};
  for (int i = 0; i < l; ++i) vals[i] = th[i];
  if (res) bank_ritz_residuals(c, 0, l, th, Y, res);
}

int bank_load(Ctx& c, int count, const void* vecs_aos) {
  ensure_bank(c);
  int added = 0;
  const int nev = c.P.nev;
  for (int q0 = 0; q0 < count && c.l < c.P.max_bank; q0 += nev) {
    const int k = std::min(std::min(nev, count - q0), c.P.max_bank - c.l);
    void* slot = col_ptr(c.U, c.bank_prec, c.cs, c.l);
    const double2* src = (const double2*)vecs_aos + (size_t)q0 * 12 * c.g.V;
    c.check(launch_spinor_to_soa(src, slot, c.bank_prec, &c.g, k, c.cs, c.stream), "to soa");
    added += bank_append_from(c, slot, k);
  }
  return added;
}

// Truncation of U to its k lowest Ritz vectors (the Section 4 discussion of
// limiting U): with H Y = Y Theta, U <- U Y_k and H <- Theta_k.  The product
// goes through a temporary of k fields (the bank's own columns are inputs).
void bank_truncate(Ctx& c, int k) {
  if (k < 0) throw ApiError{EIGCG_EINVAL, "negative bank size"};
  if (k >= c.l) return;
  if (k == 0) {
    c.l = 0;
    c.nlock = 0;
    c.chol_ok = false;
    c.spec_ok = false;
    ++c.bank_gen;
    return;
  }
  const int l = c.l, ld = c.P.max_bank, prec = c.bank_prec;
  std::vector<double> th(l);
  std::vector<cplx> Y((size_t)l * k);
  if (hostla::herm_eig_lowest(l, c.H.data(), ld, k, th.data(), Y.data(), l) != 0)
    throw ApiError{EIGCG_EBREAKDOWN, "bank eigensolver failed"};
  void* tmp = c.dalloc(c.cs * elem_bytes(prec) * (size_t)k);
  try {
    std::vector<const void*> in(l);
    for (int i = 0; i < l; ++i) in[i] = col_ptr(c.U, prec, c.cs, i);
    std::vector<void*> out(k);
    for (int j = 0; j < k; ++j) out[j] = col_ptr(tmp, prec, c.cs, j);
    tall_from_host(c, prec, l, k, in, out, Y.data(), 0, 0);
    c.check(launch_copy(prec, prec, k, c.cs, tmp, c.cs, c.U, c.cs, c.stream), "copy");
    c.check(hipStreamSynchronize(c.stream), "sync");
  } catch (...) {
    c.dfree(tmp);
    throw;
  }
  c.dfree(tmp);
  std::fill(c.H.begin(), c.H.end(), cplx(0.0, 0.0));
  for (int i = 0; i < k; ++i) c.H[(size_t)i * ld + i] = cplx(th[i], 0.0);
  c.l = k;
  c.nlock = 0;
  c.chol_ok = false;
  c.spec_ok = false;
  ++c.bank_gen;
}

// Section 4: lock accurate eigenvectors out of U so that they take no part in
// building H.  Rayleigh-Ritz on the unlocked columns (their coupling with the
// locked block is zero by construction), H_u Y = Y Theta and U_u <- U_u Y; the
// Ritz vectors with ||A u - theta u|| <= tol are locked.  Locked columns come
// first (the earlier ones, then the new ones in ascending Ritz value), the
// unlocked Ritz vectors follow in ascending order, and H becomes diag(theta)
// on every rotated column.  Bank updates then leave the locked rows of
// U^H A Vbar at zero: each skipped entry is r^H v for a locked residual r and
// a new v orthogonal to it, at most tol in modulus.
int bank_lock(Ctx& c, double tol) {
  if (!(tol >= 0.0) || !std::isfinite(tol))
    throw ApiError{EIGCG_EINVAL, "lock tolerance must be finite and >= 0"};
  const int l = c.l, nl = c.nlock, n = l - nl, ld = c.P.max_bank, prec = c.bank_prec;
  if (n <= 0) return nl;
  std::vector<cplx> Hu((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Hu[(size_t)j * n + i] = c.H[(size_t)(nl + j) * ld + nl + i];
  std::vector<double> th(n);
  std::vector<cplx> Y((size_t)n * n);
  if (hostla::herm_eig_lowest(n, Hu.data(), n, n, th.data(), Y.data(), n) != 0)
    throw ApiError{EIGCG_EBREAKDOWN, "bank eigensolver failed"};
  std::vector<double> res(n);
  bank_ritz_residuals(c, nl, n, th, Y, res.data());
  std::vector<int> order;
  for (int j = 0; j < n; ++j)
    if (res[j] <= tol) order.push_back(j);
  const int nnew = (int)order.size();
  for (int j = 0; j < n; ++j)
    if (!(res[j] <= tol)) order.push_back(j);
  std::vector<cplx> Yp((size_t)n * n);
  for (int q = 0; q < n; ++q)
    std::copy(Y.begin() + (size_t)order[q] * n, Y.begin() + (size_t)(order[q] + 1) * n,
              Yp.begin() + (size_t)q * n);
  void* tmp = c.dalloc(c.cs * elem_bytes(prec) * (size_t)n);
  try {
    std::vector<const void*> in(n);
    for (int i = 0; i < n; ++i) in[i] = col_ptr(c.U, prec, c.cs, nl + i);
    std::vector<void*> out(n);
    for (int j = 0; j < n; ++j) out[j] = col_ptr(tmp, prec, c.cs, j);
    tall_from_host(c, prec, n, n, in, out, Yp.data(), 0, 0);
    c.check(launch_copy(prec, prec, n, c.cs, tmp, c.cs, col_ptr(c.U, prec, c.cs, nl), c.cs,
                        c.stream),
            "copy");
    c.check(hipStreamSynchronize(c.stream), "sync");
  } catch (...) {
    c.dfree(tmp);
    throw;
  }
  c.dfree(tmp);
  for (int j = nl; j < l; ++j)
    for (int i = 0; i < l; ++i) {
      c.H[(size_t)j * ld + i] = cplx(0.0, 0.0);
      c.H[(size_t)i * ld + j] = cplx(0.0, 0.0);
    }
  for (int q = 0; q < n; ++q) c.H[(size_t)(nl + q) * ld + nl + q] = cplx(th[order[q]], 0.0);
  c.nlock = nl + nnew;
  c.chol_ok = false;
  c.spec_ok = false;
  ++c.bank_gen;
  return c.nlock;
}

// Restore a saved bank: U <- the given fields (in the bank's precision) and
// H <- h (l x l, column-major), both as eigcg_bank_vectors and
// eigcg_bank_matrix returned them; no orthonormalisation, no applications of A.
void bank_restore(Ctx& c, int l, const void* vecs_aos, const double* h_host) {
  if (l < 0 || l > c.P.max_bank) throw ApiError{EIGCG_EINVAL, "bank size out of range"};
  ensure_bank(c);
  const int ld = c.P.max_bank;
  const cplx* h = reinterpret_cast<const cplx*>(h_host);
  std::vector<cplx> Hn((size_t)ld * ld, cplx(0.0, 0.0));
  for (int j = 0; j < l; ++j)
    for (int i = 0; i < l; ++i) Hn[(size_t)j * ld + i] = h[(size_t)j * l + i];
  std::vector<cplx> Lt = Hn;  // H must be Hermitian positive definite
  if (l > 0 && hostla::cholesky(l, Lt.data(), ld) != 0)
    throw ApiError{EIGCG_EINVAL, "bank matrix is not positive definite"};
  for (int q0 = 0; q0 < l; q0 += 16) {
    const int k = std::min(16, l - q0);
    const double2* src = (const double2*)vecs_aos + (size_t)q0 * 12 * c.g.V;
    c.check(launch_spinor_to_soa(src, col_ptr(c.U, c.bank_prec, c.cs, q0), c.bank_prec, &c.g, k,
                                 c.cs, c.stream),
            "to soa");
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
  c.H = Hn;
  c.l = l;
  c.nlock = 0;
  c.chol_ok = false;
  c.spec_ok = false;
  ++c.bank_gen;
}

void bank_vectors(Ctx& c, int first, int count, void* out_aos) {
  for (int q = 0; q < count; ++q) {
    double2* dst = (double2*)out_aos + (size_t)q * 12 * c.g.V;
    c.check(launch_spinor_from_soa(col_ptr(c.U, c.bank_prec, c.cs, first + q), dst, c.bank_prec,
                                   &c.g, 1, c.cs, c.stream),
            "from soa");
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
}

// Kernel timing on the context's stream (HIP events around `reps` launches):
// what 0: FP64 stencil M (store); 1: plain copy of one FP64 field; 2: one
// FP64 CG iteration (four kernels); 3: FP32 stencil M (store; mixed-precision
// contexts only).
double bench_kernels(Ctx& c, int what, int reps) {
  const int prec = what == 3 ? c.iprec : kF64;
  if (what == 3 && !c.u32) throw ApiError{EIGCG_EINVAL, "context has no inner-precision links"};
  Workspace& w = prec == kF64 ? c.ws64 : c.ws32;
  ws_ensure(c, w, prec, false);
  // non-zero, finite work vectors (byte pattern 0x3F) and a state that never
  // stops, so every timed launch does its full work
  const size_t vb = c.cs * elem_bytes(prec);
  for (void* v : {w.x, w.p, w.r, w.tmp}) c.check(hipMemsetAsync(v, 0x3F, vb, c.stream), "fill");
  std::vector<ColState> st(1);
  std::memset(st.data(), 0, sizeof(ColState));
  st[0].state = ColRun;
  if (what == 2) {
    st[0].rho = col_norms(c, prec, 1, w.r)[0];  // a consistent CG state: r = p
    c.check(launch_copy(prec, prec, 1, c.cs, w.r, c.cs, w.p, c.cs, c.stream), "copy");
  }
  st[0].stop2 = -1.0;
  st[0].restart2 = -1.0;
  st[0].res_stop2 = -1.0;
  st[0].max_iter = 0x3fffffff;
  std::memcpy(c.h_st, st.data(), sizeof(ColState));
  c.check(hipMemcpy(c.d_st, c.h_st, sizeof(ColState), hipMemcpyHostToDevice), "st");
  ensure_spectral(c);
  Run R(c, w, prec, 1, 1u, false);
  hipEvent_t e0, e1;
  c.check(hipEventCreate(&e0), "ev");
  c.check(hipEventCreate(&e1), "ev");
  auto launch = [&]() {
    if (what == 0 || what == 3) {
      stencil_store(c, prec, kOpM, 1, w.x, w.tmp);
    } else if (what == 1) {
      c.check(launch_copy(prec, prec, 1, c.cs, w.x, c.cs, w.tmp, c.cs, c.stream), "copy");
    } else {
      R.enqueue_iters(1);
    }
  };
  if (reps + 8 > c.P.max_iter) throw ApiError{EIGCG_EINVAL, "reps must stay below max_iter"};
  for (int i = 0; i < 3; ++i) launch();
  c.check(hipEventRecord(e0, c.stream), "ev");
  for (int i = 0; i < reps; ++i) launch();
  c.check(hipEventRecord(e1, c.stream), "ev");
  c.check(hipEventSynchronize(e1), "ev");
  float ms = 0.f;
  c.check(hipEventElapsedTime(&ms, e0, e1), "ev");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (void* v : {w.x, w.p, w.r, w.tmp}) c.check(hipMemsetAsync(v, 0, vb, c.stream), "clear");
  c.check(hipStreamSynchronize(c.stream), "sync");
  return (double)ms / reps;
}

}  // namespace eigcg

