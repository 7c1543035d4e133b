// Streaming BLAS1 kernels of the CG/eigCG iteration, layout conversions and
// small helpers (gfx950).  All are HBM-bound; every access is a contiguous
// 64-lane load or store of one SoA plane, and every reduction is
// deterministic (fixed-order sums, see common.h).
#include <float.h>

#include "kernels.h"

namespace eigcg {

namespace {

inline int grid_for(size_t n) {
  size_t g = (n + kBlock - 1) / kBlock;
  if (g > (size_t)kMaxGrid) g = kMaxGrid;
  if (g == 0) g = 1;
  return (int)g;
}

// End of a CG iteration (Figure 3.1) and the start of the next: x += alpha p;
// p = r + beta p; window slot (iter+1) % ring = r / sqrt(rho).
template <typename VS, typename XS>
__global__ __launch_bounds__(kBlock) void k_cg_update(UpdateLaunch a, Geom g) {
  using R = typename Storage<VS>::real;
  const int col = blockIdx.y;
  if (!((a.mask >> col) & 1u)) return;
  const ColState S = a.st[col];
  if (S.state == ColStopped) return;
  const bool run = S.state == ColRun;
  const R alpha = (R)S.alpha, beta = (R)S.beta;
  const R inv = run ? (R)(1.0 / sqrt(S.rho)) : R(0);
  XS* x = reinterpret_cast<XS*>(a.x) + (size_t)col * a.x_cs;
  VS* p = reinterpret_cast<VS*>(a.p) + (size_t)col * a.p_cs;
  const VS* r = reinterpret_cast<const VS*>(a.r) + (size_t)col * a.r_cs;
  VS* v = nullptr;
  if (run && a.ring) {
    const int slot = (S.iter + 1) % a.ring_len;
    v = reinterpret_cast<VS*>(a.ring) + (size_t)col * a.ring_col_cs + (size_t)slot * a.ring_cs;
  }
  const size_t vs = (size_t)g.vs;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)g.V; s += gridDim.x * kBlock) {
    // four components at a time, every load of a group before its first
    // store (a store could alias a later load for all the compiler knows,
    // which would serialise the memory round trips component by component)
#pragma unroll
    for (int e0 = 0; e0 < 12; e0 += 4) {
      cpx<R> pv[4], xv[4], rv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const size_t i = (size_t)(e0 + k) * vs + s;
        pv[k] = Storage<VS>::ld(p, i);
        xv[k] = Storage<XS>::ld(x, i);
        if (run) rv[k] = Storage<VS>::ld(r, i);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const size_t i = (size_t)(e0 + k) * vs + s;
        xv[k].re += alpha * pv[k].re;
        xv[k].im += alpha * pv[k].im;
        Storage<XS>::st(x, i, xv[k]);
        if (run) {
          Storage<VS>::st(p, i, {rv[k].re + beta * pv[k].re, rv[k].im + beta * pv[k].im});
          if (v) Storage<VS>::st(v, i, {rv[k].re * inv, rv[k].im * inv});
        }
      }
    }
  }
}

// CG start: p = r; window slot 1 = r / sqrt(rho) (first eigCG column).
template <typename VS>
__global__ __launch_bounds__(kBlock) void k_cg_start(UpdateLaunch a, Geom g) {
  using R = typename Storage<VS>::real;
  const int col = blockIdx.y;
  if (!((a.mask >> col) & 1u)) return;
  const ColState S = a.st[col];
  if (S.state != ColRun) return;
  const R inv = (R)(1.0 / sqrt(S.rho));
  VS* p = reinterpret_cast<VS*>(a.p) + (size_t)col * a.p_cs;
  const VS* r = reinterpret_cast<const VS*>(a.r) + (size_t)col * a.r_cs;
  VS* v = nullptr;
  if (a.ring) {
    const int slot = (S.iter + 1) % a.ring_len;
    v = reinterpret_cast<VS*>(a.ring) + (size_t)col * a.ring_col_cs + (size_t)slot * a.ring_cs;
  }
  const size_t vs = (size_t)g.vs;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)g.V; s += gridDim.x * kBlock) {
#pragma unroll
    for (int e = 0; e < 12; ++e) {
      const size_t i = (size_t)e * vs + s;
      cpx<R> rv = Storage<VS>::ld(r, i);
      Storage<VS>::st(p, i, rv);
      if (v) Storage<VS>::st(v, i, {rv.re * inv, rv.im * inv});
    }
  }
}

template <typename VS>
__global__ __launch_bounds__(kBlock) void k_to_soa(const double2* __restrict__ aos, VS* soa,
                                                   Geom g, size_t soa_cs) {
  using R = typename Storage<VS>::real;
  const int col = blockIdx.y;
  const double2* src = aos + (size_t)col * 12 * g.V;
  VS* dst = soa + (size_t)col * soa_cs;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)g.V; s += gridDim.x * kBlock) {
#pragma unroll
    for (int e = 0; e < 12; ++e) {
      double2 v = src[(size_t)s * 12 + e];
      Storage<VS>::st(dst, (size_t)e * g.vs + s, {(R)v.x, (R)v.y});
    }
  }
}

template <typename VS>
__global__ __launch_bounds__(kBlock) void k_from_soa(const VS* __restrict__ soa, double2* aos,
                                                     Geom g, size_t soa_cs) {
  const int col = blockIdx.y;
  double2* dst = aos + (size_t)col * 12 * g.V;
  const VS* src = soa + (size_t)col * soa_cs;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)g.V; s += gridDim.x * kBlock) {
#pragma unroll
    for (int e = 0; e < 12; ++e) {
      auto v = Storage<VS>::ld(src, (size_t)e * g.vs + s);
      dst[(size_t)s * 12 + e] = make_double2((double)v.re, (double)v.im);
    }
  }
}

// parity of lattice site s, (x + y + z + t) mod 2
__device__ __forceinline__ uint32_t site_parity(const Geom& g, uint32_t s) {
  const uint32_t xyz = g.dx.div(s);
  const uint32_t x = s - xyz * (uint32_t)g.L[0];
  const uint32_t zt = g.dy.div(xyz);
  const uint32_t y = xyz - zt * (uint32_t)g.L[1];
  const uint32_t t = g.dz.div(zt);
  const uint32_t z = zt - t * (uint32_t)g.L[2];
  return (x + y + z + t) & 1u;
}

template <typename LS>
__global__ __launch_bounds__(kBlock) void k_gauge_to_soa(const double2* __restrict__ aos, LS* soa,
                                                         Geom g, int comp) {
  using R = typename Storage<LS>::real;
  const int per = comp ? 6 : 9;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)g.Vfull;
       s += gridDim.x * kBlock) {
    // odd-even geometry: the block of the site's parity, at its half index
    const size_t base = g.eo ? (size_t)site_parity(g, s) * 4 * per * g.vs : 0;
    const uint32_t i = g.eo ? s >> 1 : s;
    for (int mu = 0; mu < 4; ++mu) {
      for (int e = 0; e < per; ++e) {
        double2 v = aos[((size_t)s * 4 + mu) * 9 + e];
        Storage<LS>::st(soa, base + (size_t)(mu * per + e) * g.vs + i, {(R)v.x, (R)v.y});
      }
    }
  }
}

// full-lattice AoS field <-> even and odd half-site SoA fields (FP64)
__global__ __launch_bounds__(kBlock) void k_split_eo(const double2* __restrict__ aos, double2* even,
                                                     double2* odd, Geom g, size_t soa_cs) {
  const int col = blockIdx.y;
  const double2* src = aos + (size_t)col * 12 * g.Vfull;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)g.Vfull;
       s += gridDim.x * kBlock) {
    double2* dst = (site_parity(g, s) ? odd : even) + (size_t)col * soa_cs;
#pragma unroll
    for (int e = 0; e < 12; ++e) dst[(size_t)e * g.vs + (s >> 1)] = src[(size_t)s * 12 + e];
  }
}

__global__ __launch_bounds__(kBlock) void k_merge_eo(const double2* __restrict__ even,
                                                     const double2* __restrict__ odd, double2* aos,
                                                     Geom g, size_t soa_cs) {
  const int col = blockIdx.y;
  double2* dst = aos + (size_t)col * 12 * g.Vfull;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)g.Vfull;
       s += gridDim.x * kBlock) {
    const double2* src = (site_parity(g, s) ? odd : even) + (size_t)col * soa_cs;
#pragma unroll
    for (int e = 0; e < 12; ++e) dst[(size_t)s * 12 + e] = src[(size_t)e * g.vs + (s >> 1)];
  }
}

// max |U U^H - I| and max |det U - 1| over all links (unitarity check that
// decides whether links may be stored as two rows).
__global__ __launch_bounds__(kBlock) void k_gauge_check(const double2* __restrict__ aos, Geom g,
                                                        double* partial) {
  __shared__ double lds[2][kBlock];
  double m1 = 0.0, m2 = 0.0;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < (uint32_t)g.Vfull;
       s += gridDim.x * kBlock) {
    for (int mu = 0; mu < 4; ++mu) {
      cpx<double> U[9];
      for (int e = 0; e < 9; ++e) {
        double2 v = aos[((size_t)s * 4 + mu) * 9 + e];
        U[e] = {v.x, v.y};
      }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          cpx<double> t = {0.0, 0.0};
          for (int c = 0; c < 3; ++c) {
            // (U U^H)_ab = sum_c U_ac conj(U_bc)
            cpx<double> p = cmulc(U[b * 3 + c], U[a * 3 + c]);
            t = cadd(t, p);
          }
          if (a == b) t.re -= 1.0;
          m1 = fmax(m1, sqrt(t.re * t.re + t.im * t.im));
        }
      cpx<double> det = cmul(U[0], csub(cmul(U[4], U[8]), cmul(U[5], U[7])));
      det = csub(det, cmul(U[1], csub(cmul(U[3], U[8]), cmul(U[5], U[6]))));
      det = cadd(det, cmul(U[2], csub(cmul(U[3], U[7]), cmul(U[4], U[6]))));
      det.re -= 1.0;
      m2 = fmax(m2, sqrt(det.re * det.re + det.im * det.im));
    }
  }
  lds[0][threadIdx.x] = m1;
  lds[1][threadIdx.x] = m2;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      lds[0][threadIdx.x] = fmax(lds[0][threadIdx.x], lds[0][threadIdx.x + off]);
      lds[1][threadIdx.x] = fmax(lds[1][threadIdx.x], lds[1][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = lds[0][0];
    partial[2 * blockIdx.x + 1] = lds[1][0];
  }
}

__global__ void k_gauge_check_final(const double* partial, int nb, double* out2) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < nb; ++i) {
    a = fmax(a, partial[2 * i]);
    b = fmax(b, partial[2 * i + 1]);
  }
  out2[0] = a;
  out2[1] = b;
}

// ---- generic BLAS1 over n complex entries per column ------------------------

template <typename VS>
__global__ __launch_bounds__(kBlock) void k_axpy(size_t n, const double* a_dev, double are,
                                                 double aim, const VS* x, size_t x_cs, VS* y,
                                                 size_t y_cs) {
  using R = typename Storage<VS>::real;
  const int col = blockIdx.y;
  double ar = are, ai = aim;
  if (a_dev) { ar = a_dev[2 * col]; ai = a_dev[2 * col + 1]; }
  const cpx<R> a = {(R)ar, (R)ai};
  const VS* xc = x + (size_t)col * x_cs;
  VS* yc = y + (size_t)col * y_cs;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    cpx<R> yv = Storage<VS>::ld(yc, i);
    Storage<VS>::st(yc, i, cadd(yv, cmul(a, Storage<VS>::ld(xc, i))));
  }
}

template <typename SS, typename DS>
__global__ __launch_bounds__(kBlock) void k_copy(size_t n, const SS* x, size_t x_cs, DS* y,
                                                 size_t y_cs, uint32_t mask) {
  using R = typename Storage<DS>::real;
  const int col = blockIdx.y;
  if (!((mask >> col) & 1u)) return;
  const SS* xc = x + (size_t)col * x_cs;
  DS* yc = y + (size_t)col * y_cs;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    auto v = Storage<SS>::ld(xc, i);
    Storage<DS>::st(yc, i, {(R)v.re, (R)v.im});
  }
}

template <typename VS>
__global__ __launch_bounds__(kBlock) void k_norm2(size_t n, const VS* x, size_t x_cs,
                                                  double* partial) {
  __shared__ double lds4[kBlock / 64];
  const int col = blockIdx.y;
  const VS* xc = x + (size_t)col * x_cs;
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    auto v = Storage<VS>::ld(xc, i);
    acc += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
  }
  double bs = block_sum(acc, lds4);
  if (threadIdx.x == 0) partial[(size_t)col * gridDim.x + blockIdx.x] = bs;
}

__global__ __launch_bounds__(kBlock) void k_norm2_final(const double* partial, int nb, int ncols,
                                                        double* out) {
  __shared__ double lds4[kBlock / 64];
  const int c = blockIdx.x;  // one workgroup per column
  if (c >= ncols) return;
  const double t = reduce_partials(partial + (size_t)c * nb, nb, lds4);
  if (threadIdx.x == 0) out[c] = t;
}

template <typename VS>
__global__ __launch_bounds__(kBlock) void k_scale(size_t n, const double* sc, VS* y, size_t y_cs) {
  using R = typename Storage<VS>::real;
  const int col = blockIdx.y;
  const R f = (R)sc[col];
  VS* yc = y + (size_t)col * y_cs;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    auto v = Storage<VS>::ld(yc, i);
    Storage<VS>::st(yc, i, {v.re * f, v.im * f});
  }
}

template <typename VS>
__global__ __launch_bounds__(kBlock) void k_xpby(size_t n, const VS* t1, const VS* t0,
                                                 size_t t_cs, const double* beta, VS* w,
                                                 size_t w_cs) {
  using R = typename Storage<VS>::real;
  const int col = blockIdx.y;
  const R b = (R)beta[col];
  const VS* a1 = t1 + (size_t)col * t_cs;
  const VS* a0 = t0 + (size_t)col * t_cs;
  VS* wc = w + (size_t)col * w_cs;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    auto u1 = Storage<VS>::ld(a1, i);
    auto u0 = Storage<VS>::ld(a0, i);
    Storage<VS>::st(wc, i, {u1.re - b * u0.re, u1.im - b * u0.im});
  }
}

// x64 += e32 (divided by the column's inner scale when st is given); e32 = 0
__global__ __launch_bounds__(kBlock) void k_accum(size_t n, double2* x, size_t x_cs, float2* e,
                                                  size_t e_cs, uint32_t mask, const ColState* st) {
  const int col = blockIdx.y;
  if (!((mask >> col) & 1u)) return;
  const double inv = st ? 1.0 / st[col].scale : 1.0;
  double2* xc = x + (size_t)col * x_cs;
  float2* ec = e + (size_t)col * e_cs;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    float2 ev = ec[i];
    double2 xv = xc[i];
    if (st) {
      xv.x += (double)ev.x * inv;
      xv.y += (double)ev.y * inv;
    } else {
      xv.x += (double)ev.x;
      xv.y += (double)ev.y;
    }
    xc[i] = xv;
    ec[i] = make_float2(0.f, 0.f);
  }
}

// Inner-solve scaling of 16-bit iterations: for every masked running column
// s = c0 / sqrt(rho) (rho = FP64 true r^H r), so the scaled residual has an
// RMS entry of c0 / sqrt(n); rho and the inner stop move to the scaled units.
__global__ void k_set_scale(ColState* st, int ncols, uint32_t mask, double c0) {
  const int c = threadIdx.x;
  if (c >= ncols || !((mask >> c) & 1u)) return;
  ColState& S = st[c];
  if (S.state != ColRun) return;
  const double s = S.rho > 0.0 ? c0 / sqrt(S.rho) : 1.0;
  S.scale = s;
  S.rho *= s * s;
  S.restart2 *= s * s;
}

// y (16-bit) = scale_col * x (FP64) for running columns
__global__ __launch_bounds__(kBlock) void k_to_inner16(size_t n, const double2* x, size_t x_cs,
                                                       f16x2* y, size_t y_cs, uint32_t mask,
                                                       const ColState* st) {
  const int col = blockIdx.y;
  if (!((mask >> col) & 1u)) return;
  if (st[col].state != ColRun) return;
  const double f = st[col].scale;
  const double2* xc = x + (size_t)col * x_cs;
  f16x2* yc = y + (size_t)col * y_cs;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const double2 v = xc[i];
    Storage<f16x2>::st(yc, i, {(float)(v.x * f), (float)(v.y * f)});
  }
}

__global__ void k_post_residual(ColState* st, int ncols, uint32_t mask) {
  const int c = threadIdx.x;
  if (c >= ncols || !((mask >> c) & 1u)) return;
  ColState& S = st[c];
  const bool waiting = S.state != ColRun && S.reason == ReasonRestart;
  if (S.state != ColRun && !waiting) return;
  if (S.rho <= S.res_stop2) {
    S.state = ColStopped;
    S.reason = ReasonConverged;
  } else {
    S.state = ColRun;
    S.reason = ReasonNone;
    if (S.inner_rel2 > 0.0) S.restart2 = fmax(S.inner_rel2 * S.rho, 0.25 * S.res_stop2);
  }
}

__global__ void k_set_state(ColState* st, int ncols, uint32_t mask, int state, int reason,
                            int clear_restart) {
  const int c = threadIdx.x;
  if (c >= ncols || !((mask >> c) & 1u)) return;
  st[c].state = state;
  st[c].reason = reason;
  if (clear_restart) st[c].restart2 = 0.0;
}

// After a reliable update has replaced r by the FP64 true residual, restore
// the premise of the next step length alpha = r^H r / p^H A p, namely
// r^H p = r^H r: p <- p - (r^H p / r^H r - 1) r (the component of p along
// the new r becomes exactly r).  Running columns only; r^H r is the state's rho.
template <typename VS>
__global__ __launch_bounds__(kBlock) void k_dot_rp(size_t n, const VS* r, const VS* p, size_t cs,
                                                   uint32_t mask, const ColState* st,
                                                   double* part_re, double* part_im) {
  using R = typename Storage<VS>::real;
  __shared__ double lds4[kBlock / 64];
  const int col = blockIdx.y;
  if (!((mask >> col) & 1u) || st[col].state != ColRun) return;
  const VS* rc = r + (size_t)col * cs;
  const VS* pc = p + (size_t)col * cs;
  double sr = 0.0, si = 0.0;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const cpx<R> a = Storage<VS>::ld(rc, i), b = Storage<VS>::ld(pc, i);
    sr += (double)a.re * (double)b.re + (double)a.im * (double)b.im;
    si += (double)a.re * (double)b.im - (double)a.im * (double)b.re;
  }
  sr = block_sum(sr, lds4);
  si = block_sum(si, lds4);
  if (threadIdx.x == 0) {
    part_re[(size_t)col * gridDim.x + blockIdx.x] = sr;
    part_im[(size_t)col * gridDim.x + blockIdx.x] = si;
  }
}

template <typename VS>
__global__ __launch_bounds__(kBlock) void k_fix_p(size_t n, const VS* r, VS* p, size_t cs,
                                                  uint32_t mask, const ColState* st,
                                                  const double* part_re, const double* part_im) {
  using R = typename Storage<VS>::real;
  __shared__ double lds4[kBlock / 64];
  const int col = blockIdx.y;
  if (!((mask >> col) & 1u) || st[col].state != ColRun) return;
  const double dr = reduce_partials(part_re + (size_t)col * gridDim.x, gridDim.x, lds4);
  const double di = reduce_partials(part_im + (size_t)col * gridDim.x, gridDim.x, lds4);
  const double rho = st[col].rho;
  if (!(rho > 0.0 && rho < INFINITY)) return;
  const R cr = (R)(dr / rho - 1.0), ci = (R)(di / rho);
  const VS* rc = r + (size_t)col * cs;
  VS* pc = p + (size_t)col * cs;
  for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const cpx<R> a = Storage<VS>::ld(rc, i);
    cpx<R> b = Storage<VS>::ld(pc, i);
    b.re -= cr * a.re - ci * a.im;
    b.im -= cr * a.im + ci * a.re;
    Storage<VS>::st(pc, i, b);
  }
}

}  // namespace

hipError_t launch_reliable_fix_p(int prec, int ncols, uint32_t mask, size_t n, const void* r,
                                 void* p, size_t cs, const ColState* st, double* partial,
                                 hipStream_t s) {
  if (prec != kF32 && prec != kF64) return hipErrorInvalidValue;
  const int gx = grid_for(n);
  dim3 grid(gx, ncols);
  double* pre = partial;
  double* pim = partial + (size_t)kMaxCols * kMaxGrid;
  if (prec == kF32) {
    hipLaunchKernelGGL(k_dot_rp<float2>, grid, dim3(kBlock), 0, s, n, (const float2*)r,
                       (const float2*)p, cs, mask, st, pre, pim);
    hipLaunchKernelGGL(k_fix_p<float2>, grid, dim3(kBlock), 0, s, n, (const float2*)r, (float2*)p,
                       cs, mask, st, pre, pim);
  } else {
    hipLaunchKernelGGL(k_dot_rp<double2>, grid, dim3(kBlock), 0, s, n, (const double2*)r,
                       (const double2*)p, cs, mask, st, pre, pim);
    hipLaunchKernelGGL(k_fix_p<double2>, grid, dim3(kBlock), 0, s, n, (const double2*)r,
                       (double2*)p, cs, mask, st, pre, pim);
  }
  return hipGetLastError();
}

hipError_t launch_post_residual(ColState* st, int ncols, uint32_t mask, hipStream_t s) {
  hipLaunchKernelGGL(k_post_residual, dim3(1), dim3(64), 0, s, st, ncols, mask);
  return hipGetLastError();
}

hipError_t launch_set_state(ColState* st, int ncols, uint32_t mask, int state, int reason,
                            int clear_restart, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, s, st, ncols, mask, state, reason,
                     clear_restart);
  return hipGetLastError();
}

namespace {

// Spectral preconditioner, middle step: S = D G and s = G^H D G per column
// (G = U_R^H r, l x ncols complex column-major; D = sigma / theta - 1).  One
// workgroup; column j's sum runs over i in a fixed order in thread j.
__global__ __launch_bounds__(kBlock) void k_spec_scale(const double2* G, const double* D, int l,
                                                       int ncols, double2* S, double* s_out) {
  for (int e = threadIdx.x; e < l * ncols; e += kBlock) {
    const double2 g = G[e];
    const double d = D[e % l];
    S[e] = make_double2(d * g.x, d * g.y);
  }
  if (threadIdx.x < ncols) {
    const int j = threadIdx.x;
    double acc = 0.0;
    for (int i = 0; i < l; ++i) {
      const double2 g = G[(size_t)j * l + i];
      acc += D[i] * (g.x * g.x + g.y * g.y);
    }
    s_out[j] = acc;
  }
}

__global__ void k_spec_rho(ColState* st, int ncols, uint32_t mask, const double* s_in) {
  const int c = threadIdx.x;
  if (c >= ncols || !((mask >> c) & 1u)) return;
  if (st[c].state == ColRun) st[c].rho += s_in[c];
}

}  // namespace

hipError_t launch_spec_scale(const double2* G, const double* D, int l, int ncols, double2* S,
                             double* s_out, hipStream_t s) {
  if (l <= 0 || ncols <= 0 || ncols > kBlock) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_spec_scale, dim3(1), dim3(kBlock), 0, s, G, D, l, ncols, S, s_out);
  return hipGetLastError();
}

hipError_t launch_spec_rho(ColState* st, int ncols, uint32_t mask, const double* s_in,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_spec_rho, dim3(1), dim3(64), 0, s, st, ncols, mask, s_in);
  return hipGetLastError();
}

hipError_t launch_cg_update(const UpdateLaunch& L, hipStream_t s) {
  // one site per thread (the kernel writes no per-workgroup partials, so the
  // grid is not held to kMaxGrid): a capped grid left a fraction of the
  // threads a second site each, a tail the rest of the GPU waited for
  const size_t wgs = ((size_t)L.g->V + kBlock - 1) / kBlock;
  dim3 grid((unsigned)std::min<size_t>(wgs, 1u << 20), L.ncols);
  if (L.prec == kF64)
    hipLaunchKernelGGL((k_cg_update<double2, double2>), grid, dim3(kBlock), 0, s, L, *L.g);
  else if (L.prec == kF32)
    hipLaunchKernelGGL((k_cg_update<float2, float2>), grid, dim3(kBlock), 0, s, L, *L.g);
  else  // 16-bit p, r; the iterate accumulates in FP32
    hipLaunchKernelGGL((k_cg_update<f16x2, float2>), grid, dim3(kBlock), 0, s, L, *L.g);
  return hipGetLastError();
}

hipError_t launch_cg_start(const UpdateLaunch& L, hipStream_t s) {
  dim3 grid(grid_for(L.g->V), L.ncols);
  if (L.prec == kF64)
    hipLaunchKernelGGL(k_cg_start<double2>, grid, dim3(kBlock), 0, s, L, *L.g);
  else if (L.prec == kF32)
    hipLaunchKernelGGL(k_cg_start<float2>, grid, dim3(kBlock), 0, s, L, *L.g);
  else
    hipLaunchKernelGGL(k_cg_start<f16x2>, grid, dim3(kBlock), 0, s, L, *L.g);
  return hipGetLastError();
}

hipError_t launch_set_scale(ColState* st, int ncols, uint32_t mask, double c0, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scale, dim3(1), dim3(64), 0, s, st, ncols, mask, c0);
  return hipGetLastError();
}

hipError_t launch_to_inner16(int ncols, size_t n, const void* x64, size_t x_cs, void* y16,
                             size_t y_cs, uint32_t mask, const ColState* st, hipStream_t s) {
  dim3 grid(grid_for(n), ncols);
  hipLaunchKernelGGL(k_to_inner16, grid, dim3(kBlock), 0, s, n, (const double2*)x64, x_cs,
                     (f16x2*)y16, y_cs, mask, st);
  return hipGetLastError();
}

hipError_t launch_spinor_to_soa(const double2* aos, void* soa, int prec, const Geom* g, int ncols,
                                size_t soa_cs, hipStream_t s) {
  dim3 grid(grid_for(g->V), ncols);
  if (prec == kF64)
    hipLaunchKernelGGL(k_to_soa<double2>, grid, dim3(kBlock), 0, s, aos, (double2*)soa, *g, soa_cs);
  else
    hipLaunchKernelGGL(k_to_soa<float2>, grid, dim3(kBlock), 0, s, aos, (float2*)soa, *g, soa_cs);
  return hipGetLastError();
}

hipError_t launch_spinor_from_soa(const void* soa, double2* aos, int prec, const Geom* g,
                                  int ncols, size_t soa_cs, hipStream_t s) {
  dim3 grid(grid_for(g->V), ncols);
  if (prec == kF64)
    hipLaunchKernelGGL(k_from_soa<double2>, grid, dim3(kBlock), 0, s, (const double2*)soa, aos, *g,
                       soa_cs);
  else
    hipLaunchKernelGGL(k_from_soa<float2>, grid, dim3(kBlock), 0, s, (const float2*)soa, aos, *g,
                       soa_cs);
  return hipGetLastError();
}

hipError_t launch_gauge_to_soa(const double2* aos, void* soa, int prec, int compressed,
                               const Geom* g, hipStream_t s) {
  dim3 grid(grid_for(g->Vfull));
  if (prec == kF64)
    hipLaunchKernelGGL(k_gauge_to_soa<double2>, grid, dim3(kBlock), 0, s, aos, (double2*)soa, *g,
                       compressed);
  else if (prec == kF32)
    hipLaunchKernelGGL(k_gauge_to_soa<float2>, grid, dim3(kBlock), 0, s, aos, (float2*)soa, *g,
                       compressed);
  else
    hipLaunchKernelGGL(k_gauge_to_soa<f16x2>, grid, dim3(kBlock), 0, s, aos, (f16x2*)soa, *g,
                       compressed);
  return hipGetLastError();
}

hipError_t launch_split_eo(const double2* aos, void* even, void* odd, const Geom* g, int ncols,
                           size_t soa_cs, hipStream_t s) {
  if (!g->eo) return hipErrorInvalidValue;
  dim3 grid(grid_for(g->Vfull), ncols);
  hipLaunchKernelGGL(k_split_eo, grid, dim3(kBlock), 0, s, aos, (double2*)even, (double2*)odd, *g,
                     soa_cs);
  return hipGetLastError();
}

hipError_t launch_merge_eo(const void* even, const void* odd, double2* aos, const Geom* g,
                           int ncols, size_t soa_cs, hipStream_t s) {
  if (!g->eo) return hipErrorInvalidValue;
  dim3 grid(grid_for(g->Vfull), ncols);
  hipLaunchKernelGGL(k_merge_eo, grid, dim3(kBlock), 0, s, (const double2*)even,
                     (const double2*)odd, aos, *g, soa_cs);
  return hipGetLastError();
}

hipError_t launch_gauge_check(const double2* aos, const Geom* g, double* out2, hipStream_t s) {
  // scratch after the two outputs: one (max, max) pair per workgroup
  int gx = grid_for(g->Vfull);
  double* partial = out2 + 2;
  hipLaunchKernelGGL(k_gauge_check, dim3(gx), dim3(kBlock), 0, s, aos, *g, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gauge_check_final, dim3(1), dim3(64), 0, s, partial, gx, out2);
  return hipGetLastError();
}

hipError_t launch_axpy(int prec, int ncols, size_t n, const double* a_dev, double a_re,
                       double a_im, const void* x, size_t x_cs, void* y, size_t y_cs,
                       hipStream_t s) {
  dim3 grid(grid_for(n), ncols);
  if (prec == kF64)
    hipLaunchKernelGGL(k_axpy<double2>, grid, dim3(kBlock), 0, s, n, a_dev, a_re, a_im,
                       (const double2*)x, x_cs, (double2*)y, y_cs);
  else
    hipLaunchKernelGGL(k_axpy<float2>, grid, dim3(kBlock), 0, s, n, a_dev, a_re, a_im,
                       (const float2*)x, x_cs, (float2*)y, y_cs);
  return hipGetLastError();
}

hipError_t launch_copy(int src_prec, int dst_prec, int ncols, size_t n, const void* x,
                       size_t x_cs, void* y, size_t y_cs, hipStream_t s, uint32_t mask) {
  dim3 grid(grid_for(n), ncols);
  if (src_prec == kF16 || dst_prec == kF16) {  // 16-bit storage: to and from FP64 only
    if (src_prec == kF64 && dst_prec == kF16)
      hipLaunchKernelGGL((k_copy<double2, f16x2>), grid, dim3(kBlock), 0, s, n, (const double2*)x,
                         x_cs, (f16x2*)y, y_cs, mask);
    else if (src_prec == kF16 && dst_prec == kF64)
      hipLaunchKernelGGL((k_copy<f16x2, double2>), grid, dim3(kBlock), 0, s, n, (const f16x2*)x,
                         x_cs, (double2*)y, y_cs, mask);
    else
      return hipErrorInvalidValue;
  } else if (src_prec == kF64 && dst_prec == kF64)
    hipLaunchKernelGGL((k_copy<double2, double2>), grid, dim3(kBlock), 0, s, n, (const double2*)x,
                       x_cs, (double2*)y, y_cs, mask);
  else if (src_prec == kF64)
    hipLaunchKernelGGL((k_copy<double2, float2>), grid, dim3(kBlock), 0, s, n, (const double2*)x,
                       x_cs, (float2*)y, y_cs, mask);
  else if (dst_prec == kF64)
    hipLaunchKernelGGL((k_copy<float2, double2>), grid, dim3(kBlock), 0, s, n, (const float2*)x,
                       x_cs, (double2*)y, y_cs, mask);
  else
    hipLaunchKernelGGL((k_copy<float2, float2>), grid, dim3(kBlock), 0, s, n, (const float2*)x,
                       x_cs, (float2*)y, y_cs, mask);
  return hipGetLastError();
}

hipError_t launch_norm2(int prec, int ncols, size_t n, const void* x, size_t x_cs,
                        double* partial, unsigned int* counter, double* out, hipStream_t s) {
  (void)counter;
  const int gx = grid_for(n);
  dim3 grid(gx, ncols);
  if (prec == kF64)
    hipLaunchKernelGGL(k_norm2<double2>, grid, dim3(kBlock), 0, s, n, (const double2*)x, x_cs,
                       partial);
  else
    hipLaunchKernelGGL(k_norm2<float2>, grid, dim3(kBlock), 0, s, n, (const float2*)x, x_cs,
                       partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_norm2_final, dim3(ncols), dim3(kBlock), 0, s, partial, gx, ncols, out);
  return hipGetLastError();
}

hipError_t launch_scale(int prec, int ncols, size_t n, const double* scale_dev, void* y,
                        size_t y_cs, hipStream_t s) {
  dim3 grid(grid_for(n), ncols);
  if (prec == kF64)
    hipLaunchKernelGGL(k_scale<double2>, grid, dim3(kBlock), 0, s, n, scale_dev, (double2*)y, y_cs);
  else
    hipLaunchKernelGGL(k_scale<float2>, grid, dim3(kBlock), 0, s, n, scale_dev, (float2*)y, y_cs);
  return hipGetLastError();
}

hipError_t launch_xpby(int prec, int ncols, size_t n, const void* t1, const void* t0,
                       size_t t_cs, const double* beta_dev, void* w, size_t w_cs,
                       hipStream_t s) {
  dim3 grid(grid_for(n), ncols);
  if (prec == kF64)
    hipLaunchKernelGGL(k_xpby<double2>, grid, dim3(kBlock), 0, s, n, (const double2*)t1,
                       (const double2*)t0, t_cs, beta_dev, (double2*)w, w_cs);
  else
    hipLaunchKernelGGL(k_xpby<float2>, grid, dim3(kBlock), 0, s, n, (const float2*)t1,
                       (const float2*)t0, t_cs, beta_dev, (float2*)w, w_cs);
  return hipGetLastError();
}

hipError_t launch_accum_f32_into_f64(int ncols, size_t n, void* x64, size_t x_cs, void* e32,
                                     size_t e_cs, hipStream_t s, uint32_t mask,
                                     const ColState* scale_st) {
  dim3 grid(grid_for(n), ncols);
  hipLaunchKernelGGL(k_accum, grid, dim3(kBlock), 0, s, n, (double2*)x64, x_cs, (float2*)e32,
                     e_cs, mask, scale_st);
  return hipGetLastError();
}

}  // namespace eigcg
