// Wilson-Dirac stencil kernels with fused CG epilogues (gfx950).
//
// One thread per lattice site (grid-stride over sites), one right-hand side
// per blockIdx.y.  Loads are SoA planes, so each of the 12 spinor components
// and each link entry is a contiguous 64-lane access; the 8 neighbour spinors
// of a site are shared with 8 other sites through L2.  Reductions
// (||M p||^2 and r^H r) are deterministic: fixed-order wave/workgroup sums,
// workgroup partials in a fixed slot, and the last workgroup to finish sums
// the partials in index order and updates the CG scalars of every column.
#include "kernels.h"
#include "wilson.h"

namespace eigcg {

namespace {

struct DevArgs {
  const void* in; size_t in_cs;
  void* out; size_t out_cs;
  const void* u;
  Geom g;
  double diag;
  int ncols;
  uint32_t mask;
  ColState* st;
  double* partial;
  unsigned int* counter;
  void* r; size_t r_cs;
  const void* b; size_t b_cs;
  void* tbuf; size_t t_cs;
  double* hist; int hist_stride;
};

template <typename VS, typename LS, bool COMP, bool DAG, int EPI>
__global__ __launch_bounds__(kBlock) void k_wilson(DevArgs a) {
  using R = typename Storage<VS>::real;
  __shared__ double lds4[kBlock / 64];
  __shared__ R ldsr[kBlock / 64];
  const int col = blockIdx.y;
  bool active = ((a.mask >> col) & 1u) != 0;
  if (active && (EPI == kEpiNorm || EPI == kEpiCGR)) active = a.st[col].state == ColRun;
  R alpha = R(0);
  bool save_t = false;
  int save_slot = 0;
  if (EPI == kEpiCGR && active) {
    alpha = (R)a.st[col].alpha;
    const int j = a.st[col].iter + 1;  // iteration being completed
    save_t = a.tbuf != nullptr && (j == a.st[col].save_t0 || j == a.st[col].save_t1);
    save_slot = j & 1;
  }
  const VS* in = reinterpret_cast<const VS*>(a.in) + (size_t)col * a.in_cs;
  const LS* u = reinterpret_cast<const LS*>(a.u);
  const size_t vs = (size_t)a.g.vs;
  R acc2 = R(0);
  if (active) {
    for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)a.g.V;
         s += gridDim.x * kBlock) {
      cpx<R> h[12];
      hopping_site<VS, LS, COMP, DAG ? 1 : -1>(in, u, a.g, s, h);
      const R d = (R)a.diag;
      cpx<R> o[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) {
        cpx<R> v = Storage<VS>::ld(in, (size_t)e * vs + s);
        o[e] = {d * v.re - R(0.5) * h[e].re, d * v.im - R(0.5) * h[e].im};
      }
      if (EPI == kEpiStore || EPI == kEpiNorm) {
        VS* out = reinterpret_cast<VS*>(a.out) + (size_t)col * a.out_cs;
#pragma unroll
        for (int e = 0; e < 12; ++e) {
          Storage<VS>::st(out, (size_t)e * vs + s, o[e]);
          if (EPI == kEpiNorm) acc2 += o[e].re * o[e].re + o[e].im * o[e].im;
        }
      } else if (EPI == kEpiCGR) {
        VS* r = reinterpret_cast<VS*>(a.r) + (size_t)col * a.r_cs;
        if (save_t) {
          VS* t = reinterpret_cast<VS*>(a.tbuf) + ((size_t)col * 2 + save_slot) * a.t_cs;
#pragma unroll
          for (int e = 0; e < 12; ++e) Storage<VS>::st(t, (size_t)e * vs + s, o[e]);
        }
#pragma unroll
        for (int e = 0; e < 12; ++e) {
          cpx<R> rv = Storage<VS>::ld(r, (size_t)e * vs + s);
          rv.re -= alpha * o[e].re;
          rv.im -= alpha * o[e].im;
          Storage<VS>::st(r, (size_t)e * vs + s, rv);
          acc2 += rv.re * rv.re + rv.im * rv.im;
        }
      } else {  // kEpiRes: r = b - op(in)
        VS* r = reinterpret_cast<VS*>(a.r) + (size_t)col * a.r_cs;
        const VS* b = reinterpret_cast<const VS*>(a.b) + (size_t)col * a.b_cs;
#pragma unroll
        for (int e = 0; e < 12; ++e) {
          cpx<R> bv = Storage<VS>::ld(b, (size_t)e * vs + s);
          cpx<R> rv = {bv.re - o[e].re, bv.im - o[e].im};
          Storage<VS>::st(r, (size_t)e * vs + s, rv);
          acc2 += rv.re * rv.re + rv.im * rv.im;
        }
      }
    }
  }
  if (EPI == kEpiStore) return;
  // deterministic reduction: workgroup sum in R, partial slot per workgroup
  R bs = block_sum(acc2, ldsr);
  if (threadIdx.x == 0) a.partial[(size_t)col * gridDim.x + blockIdx.x] = (double)bs;
  if (!elect_last_block(a.counter)) return;
  for (int c = 0; c < a.ncols; ++c) {
    const bool on = ((a.mask >> c) & 1u) != 0;
    if (!on) continue;
    const double tot = reduce_partials(a.partial + (size_t)c * gridDim.x, gridDim.x, lds4);
    if (threadIdx.x != 0) continue;
    ColState& S = a.st[c];
    if (EPI == kEpiNorm) {
      if (S.state != ColRun) continue;
      S.pap = tot;
      if (tot > 0.0 && tot < INFINITY) {
        S.alpha = S.rho / tot;
      } else {
        S.alpha = 0.0;
        S.state = ColStopPending;
        S.reason = ReasonBreakdown;
      }
    } else if (EPI == kEpiCGR) {
      if (S.state == ColRun) {
        const int j = S.iter + 1;
        const double rho_new = tot;
        const double beta = rho_new / S.rho;
        if (a.hist) {
          double* h = a.hist + (size_t)c * a.hist_stride + (size_t)3 * (j - 1);
          h[0] = S.alpha;
          h[1] = beta;
          h[2] = rho_new;
        }
        S.iter = j;
        if (j == S.save_t1 && S.tperiod > 0) {
          S.save_t0 += S.tperiod;
          S.save_t1 += S.tperiod;
        }
        S.rho_prev = S.rho;
        S.rho = rho_new;
        S.beta = beta;
        if (!(rho_new < INFINITY)) {
          S.state = ColStopPending;
          S.reason = ReasonBreakdown;
        } else if (rho_new <= S.stop2) {
          S.state = ColStopPending;
          S.reason = ReasonConverged;
        } else if (rho_new <= S.restart2) {
          S.state = ColStopPending;
          S.reason = ReasonRestart;
        } else if (j >= S.max_iter) {
          S.state = ColStopPending;
          S.reason = ReasonMaxIter;
        }
      } else if (S.state == ColStopPending) {
        S.state = ColStopped;
      }
    } else {  // kEpiRes
      S.rho = tot;
    }
  }
}

template <typename VS, typename LS>
hipError_t launch_typed(const StencilLaunch& L, hipStream_t s) {
  DevArgs a;
  a.in = L.in; a.in_cs = L.in_cs; a.out = L.out; a.out_cs = L.out_cs; a.u = L.u; a.g = *L.g;
  a.diag = L.diag; a.ncols = L.ncols; a.mask = L.mask; a.st = L.st; a.partial = L.partial;
  a.counter = L.counter; a.r = L.r; a.r_cs = L.r_cs; a.b = L.b; a.b_cs = L.b_cs;
  a.tbuf = L.tbuf; a.t_cs = L.t_cs; a.hist = L.hist; a.hist_stride = L.hist_stride;
  int gx = (L.g->V + kBlock - 1) / kBlock;
  if (gx > kMaxGrid) gx = kMaxGrid;
  dim3 grid(gx, L.ncols), block(kBlock);
#define EIGCG_DISPATCH(COMP, DAG, EPI) \
  hipLaunchKernelGGL((k_wilson<VS, LS, COMP, DAG, EPI>), grid, block, 0, s, a)
#define EIGCG_EPI(COMP, DAG)                                  \
  switch (L.epi) {                                            \
    case kEpiStore: EIGCG_DISPATCH(COMP, DAG, kEpiStore); break; \
    case kEpiNorm: EIGCG_DISPATCH(COMP, DAG, kEpiNorm); break;   \
    case kEpiCGR: EIGCG_DISPATCH(COMP, DAG, kEpiCGR); break;     \
    default: EIGCG_DISPATCH(COMP, DAG, kEpiRes); break;          \
  }
  if (L.compressed) {
    if (L.op == kOpMdag) { EIGCG_EPI(true, true) } else { EIGCG_EPI(true, false) }
  } else {
    if (L.op == kOpMdag) { EIGCG_EPI(false, true) } else { EIGCG_EPI(false, false) }
  }
#undef EIGCG_EPI
#undef EIGCG_DISPATCH
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stencil(const StencilLaunch& L, hipStream_t s) {
  if (L.ncols <= 0 || L.ncols > kMaxCols) return hipErrorInvalidValue;
  if (L.prec == kF64) return launch_typed<double2, double2>(L, s);
  return launch_typed<float2, float2>(L, s);
}

}  // namespace eigcg
