// Wilson-Dirac stencil building blocks (device side).
//
//   (M psi)(x) = (4 + m_q) psi(x)
//                - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu) ]
//
// and M^H, which swaps the two projectors (gamma5-Hermiticity, Section 1 of the
// paper).  Gamma matrices are Euclidean and chiral: g_mu = [[0, B_mu], [B_mu^H, 0]]
// with B_k = -i sigma_k (k = x, y, z) and B_t = I, so gamma5 = diag(1, 1, -1, -1).
//
// Spin projection: for psi = (u, l) (upper / lower spin pairs) and s = +-1,
// (1 + s g_mu) psi = (h, s B_mu^H h) with h = u + s B_mu l, because B_mu is
// unitary.  A hop therefore loads the neighbour spinor, forms the 2x3 half
// spinor h, applies the 3x3 link to its two spin rows and rebuilds the lower
// half from the upper one: 2 SU(3) mat-vecs instead of 4.
#pragma once

#include "common.h"

namespace eigcg {

// h = u + s B_mu l for one colour (spin components c0..c3 of the neighbour).
template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cpx<R> u0, const cpx<R> u1, const cpx<R> l0,
                                        const cpx<R> l1, cpx<R>& h0, cpx<R>& h1) {
  cpx<R> b0, b1;  // B_mu l
  if (MU == 0) { b0 = cmi(l1); b1 = cmi(l0); }
  else if (MU == 1) { b0 = cneg(l1); b1 = l0; }
  else if (MU == 2) { b0 = cmi(l0); b1 = ci(l1); }
  else { b0 = l0; b1 = l1; }
  if (S > 0) { h0 = cadd(u0, b0); h1 = cadd(u1, b1); }
  else { h0 = csub(u0, b0); h1 = csub(u1, b1); }
}

// acc += (g, s B_mu^H g) for one colour.
template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate(cpx<R>* acc, int a, const cpx<R> g0, const cpx<R> g1) {
  cpx<R> d0, d1;  // B_mu^H g
  if (MU == 0) { d0 = ci(g1); d1 = ci(g0); }
  else if (MU == 1) { d0 = g1; d1 = cneg(g0); }
  else if (MU == 2) { d0 = ci(g0); d1 = cmi(g1); }
  else { d0 = g0; d1 = g1; }
  acc[0 * 3 + a] = cadd(acc[0 * 3 + a], g0);
  acc[1 * 3 + a] = cadd(acc[1 * 3 + a], g1);
  if (S > 0) {
    acc[2 * 3 + a] = cadd(acc[2 * 3 + a], d0);
    acc[3 * 3 + a] = cadd(acc[3 * 3 + a], d1);
  } else {
    acc[2 * 3 + a] = csub(acc[2 * 3 + a], d0);
    acc[3 * 3 + a] = csub(acc[3 * 3 + a], d1);
  }
}

// Load link U_mu(site) as 9 complex numbers (row-major [a][b]).
template <typename LS, bool COMP>
__device__ __forceinline__ void load_link(const LS* __restrict__ u, int mu, size_t vs,
                                          uint32_t site, cpx<typename Storage<LS>::real>* U) {
  using R = typename Storage<LS>::real;
  if (!COMP) {
#pragma unroll
    for (int e = 0; e < 9; ++e) U[e] = Storage<LS>::ld(u, (size_t)(mu * 9 + e) * vs + site);
  } else {
#pragma unroll
    for (int e = 0; e < 6; ++e) U[e] = Storage<LS>::ld(u, (size_t)(mu * 6 + e) * vs + site);
    // third row = conj(row0 x row1) for a special unitary matrix
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
      cpx<R> t = csub(cmul(U[b1], U[3 + b2]), cmul(U[b2], U[3 + b1]));
      U[6 + b] = {t.re, -t.im};
    }
  }
}

// Site coordinates of lexicographic site index s (x fastest).
__device__ __forceinline__ void site_coords(const Geom& g, uint32_t s, uint32_t* coord) {
  const uint32_t xyz = g.dx.div(s);
  coord[0] = s - xyz * (uint32_t)g.L[0];
  const uint32_t zt = g.dy.div(xyz);
  coord[1] = xyz - zt * (uint32_t)g.L[1];
  coord[3] = g.dz.div(zt);
  coord[2] = zt - coord[3] * (uint32_t)g.L[2];
}

// Odd-even geometry: coordinates and lattice site index of half-lattice
// site h of parity par (x = 2 (h mod Lx/2) + (y + z + t + par) mod 2).
__device__ __forceinline__ uint32_t eo_site_coords(const Geom& g, uint32_t h, uint32_t par,
                                                   uint32_t* coord) {
  const uint32_t row = g.dxh.div(h);
  const uint32_t xh = h - row * (uint32_t)(g.L[0] >> 1);
  const uint32_t zt = g.dy.div(row);
  coord[1] = row - zt * (uint32_t)g.L[1];
  coord[3] = g.dz.div(zt);
  coord[2] = zt - coord[3] * (uint32_t)g.L[2];
  coord[0] = 2u * xh + ((coord[1] + coord[2] + coord[3] + par) & 1u);
  return row * (uint32_t)g.L[0] + coord[0];
}

// Both hops of direction MU for one site, accumulated into acc:
// acc += (1 + sf g_mu) U_mu(x) psi(x+mu) + (1 - sf g_mu) U_mu(x-mu)^+ psi(x-mu),
// sf = -1 for M, +1 for M^H.
template <int MU, typename VS, typename LS, bool COMP, int SF>
__device__ __forceinline__ void hop_dir(const VS* __restrict__ in, const LS* __restrict__ u,
                                        const Geom& g, uint32_t s, const uint32_t* coord,
                                        cpx<typename Storage<VS>::real>* acc) {
  using R = typename Storage<VS>::real;
  const size_t vs = (size_t)g.vs;
  const uint32_t c_ = coord[MU];
  const uint32_t st_ = (uint32_t)g.stride[MU];
  const uint32_t span_ = (uint32_t)(g.L[MU] - 1) * st_;
  const uint32_t sf_ = (c_ + 1 < (uint32_t)g.L[MU]) ? s + st_ : s - span_;
  const uint32_t sb_ = (c_ > 0) ? s - st_ : s + span_;
  {
    cpx<R> U[9];
    load_link<LS, COMP>(u, MU, vs, s, U);
    cpx<R> h[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<R> u0 = Storage<VS>::ld(in, (size_t)(0 + a) * vs + sf_);
      cpx<R> u1 = Storage<VS>::ld(in, (size_t)(3 + a) * vs + sf_);
      cpx<R> l0 = Storage<VS>::ld(in, (size_t)(6 + a) * vs + sf_);
      cpx<R> l1 = Storage<VS>::ld(in, (size_t)(9 + a) * vs + sf_);
      project<MU, SF>(u0, u1, l0, l1, h[a], h[3 + a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<R> g0 = cmul(U[a * 3 + 0], h[0]);
      cpx<R> g1 = cmul(U[a * 3 + 0], h[3]);
      g0 = cadd(g0, cmul(U[a * 3 + 1], h[1]));
      g1 = cadd(g1, cmul(U[a * 3 + 1], h[4]));
      g0 = cadd(g0, cmul(U[a * 3 + 2], h[2]));
      g1 = cadd(g1, cmul(U[a * 3 + 2], h[5]));
      accumulate<MU, SF>(acc, a, g0, g1);
    }
  }
  {
    cpx<R> U[9];
    load_link<LS, COMP>(u, MU, vs, sb_, U);
    cpx<R> h[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<R> u0 = Storage<VS>::ld(in, (size_t)(0 + a) * vs + sb_);
      cpx<R> u1 = Storage<VS>::ld(in, (size_t)(3 + a) * vs + sb_);
      cpx<R> l0 = Storage<VS>::ld(in, (size_t)(6 + a) * vs + sb_);
      cpx<R> l1 = Storage<VS>::ld(in, (size_t)(9 + a) * vs + sb_);
      project<MU, -SF>(u0, u1, l0, l1, h[a], h[3 + a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<R> g0 = cmulc(U[0 * 3 + a], h[0]);
      cpx<R> g1 = cmulc(U[0 * 3 + a], h[3]);
      g0 = cadd(g0, cmulc(U[1 * 3 + a], h[1]));
      g1 = cadd(g1, cmulc(U[1 * 3 + a], h[4]));
      g0 = cadd(g0, cmulc(U[2 * 3 + a], h[2]));
      g1 = cadd(g1, cmulc(U[2 * 3 + a], h[5]));
      accumulate<MU, -SF>(acc, a, g0, g1);
    }
  }
}

// Rebuild the third row of a two-row link: conj(row0 x row1) for SU(3).
template <typename R>
__device__ __forceinline__ void link_third_row(cpx<R>* U) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
    cpx<R> t = csub(cmul(U[b1], U[3 + b2]), cmul(U[b2], U[3 + b1]));
    U[6 + b] = {t.re, -t.im};
  }
}

// One hop of hop_dir_n.  The link at link_site and a column's neighbour spinor
// at nb are loaded before either is used, so a wave keeps every load of the
// hop in flight at once (one memory round trip per hop and column); the
// scheduling barriers stop the compiler from interleaving the loads with the
// arithmetic.  Further columns (NC > 1) load their spinor after the previous
// column's arithmetic, which bounds the live registers to one spinor.
// BWD: backward hop (U^+ and the opposite projector).  The arithmetic and its
// order are those of hop_dir.
template <int MU, typename VS, typename LS, bool COMP, int SF, int NC, bool BWD>
__device__ __forceinline__ void hop_one_n(const VS* __restrict__ in, size_t in_cs, uint32_t act,
                                          const LS* __restrict__ u, size_t vs,
                                          uint32_t link_site, uint32_t nb,
                                          cpx<typename Storage<VS>::real> (*acc)[12]) {
  using R = typename Storage<VS>::real;
  constexpr int NL = COMP ? 6 : 9;
  cpx<R> U[9];
#pragma unroll
  for (int e = 0; e < NL; ++e) U[e] = Storage<LS>::ld(u, (size_t)(MU * NL + e) * vs + link_site);
  bool first = true;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (!((act >> c) & 1u)) continue;
    const VS* ic = in + (size_t)c * in_cs;
    cpx<R> v[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) v[e] = Storage<VS>::ld(ic, (size_t)e * vs + nb);
    __builtin_amdgcn_sched_barrier(0);
    if (COMP && first) link_third_row(U);
    first = false;
    cpx<R> h[6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      project<MU, BWD ? -SF : SF>(v[0 + a], v[3 + a], v[6 + a], v[9 + a], h[a], h[3 + a]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<R> g0, g1;
      if (!BWD) {
        g0 = cmul(U[a * 3 + 0], h[0]);
        g1 = cmul(U[a * 3 + 0], h[3]);
        g0 = cadd(g0, cmul(U[a * 3 + 1], h[1]));
        g1 = cadd(g1, cmul(U[a * 3 + 1], h[4]));
        g0 = cadd(g0, cmul(U[a * 3 + 2], h[2]));
        g1 = cadd(g1, cmul(U[a * 3 + 2], h[5]));
      } else {
        g0 = cmulc(U[0 * 3 + a], h[0]);
        g1 = cmulc(U[0 * 3 + a], h[3]);
        g0 = cadd(g0, cmulc(U[1 * 3 + a], h[1]));
        g1 = cadd(g1, cmulc(U[1 * 3 + a], h[4]));
        g0 = cadd(g0, cmulc(U[2 * 3 + a], h[2]));
        g1 = cadd(g1, cmulc(U[2 * 3 + a], h[5]));
      }
      accumulate<MU, BWD ? -SF : SF>(acc[c], a, g0, g1);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// hop_dir for NC right-hand sides at once: each link is loaded (and its third
// row rebuilt) once and applied to the NC columns in == in0 + c in_cs whose
// bit is set in act.  Per column the arithmetic is exactly hop_dir's.
// EO: odd-even geometry; s is the lattice site, in holds the other parity's
// half sites, u this parity's link block and u2 the other parity's.
template <int MU, typename VS, typename LS, bool COMP, int SF, int NC, bool EO = false>
__device__ __forceinline__ void hop_dir_n(const VS* __restrict__ in, size_t in_cs, uint32_t act,
                                          const LS* __restrict__ u, const LS* __restrict__ u2,
                                          const Geom& g, uint32_t s, const uint32_t* coord,
                                          cpx<typename Storage<VS>::real> (*acc)[12]) {
  const size_t vs = (size_t)g.vs;
  const uint32_t c_ = coord[MU];
  const uint32_t st_ = (uint32_t)g.stride[MU];
  const uint32_t span_ = (uint32_t)(g.L[MU] - 1) * st_;
  const uint32_t sf_ = EO ? ((c_ + 1 < (uint32_t)g.L[MU]) ? s + st_ : s - span_) >> 1
                          : ((c_ + 1 < (uint32_t)g.L[MU]) ? s + st_ : s - span_);
  const uint32_t sb_ = EO ? ((c_ > 0) ? s - st_ : s + span_) >> 1
                          : ((c_ > 0) ? s - st_ : s + span_);
  hop_one_n<MU, VS, LS, COMP, SF, NC, false>(in, in_cs, act, u, vs, EO ? s >> 1 : s, sf_, acc);
  hop_one_n<MU, VS, LS, COMP, SF, NC, true>(in, in_cs, act, EO ? u2 : u, vs, sb_, sb_, acc);
}

// Hopping sum over all four directions for one site.
template <typename VS, typename LS, bool COMP, int SF>
__device__ __forceinline__ void hopping_site(const VS* __restrict__ in,
                                             const LS* __restrict__ u, const Geom& g,
                                             uint32_t s, cpx<typename Storage<VS>::real>* acc) {
  using R = typename Storage<VS>::real;
  uint32_t coord[4];
  site_coords(g, s, coord);
#pragma unroll
  for (int e = 0; e < 12; ++e) acc[e] = {R(0), R(0)};
  hop_dir<0, VS, LS, COMP, SF>(in, u, g, s, coord, acc);
  hop_dir<1, VS, LS, COMP, SF>(in, u, g, s, coord, acc);
  hop_dir<2, VS, LS, COMP, SF>(in, u, g, s, coord, acc);
  hop_dir<3, VS, LS, COMP, SF>(in, u, g, s, coord, acc);
}

}  // namespace eigcg
