#pragma once
// Wilson-Dirac stencil kernels with fused CG epilogues (gfx950).  Included
// by one translation unit per storage precision (dslash_f64/f32/f16.hip), each
// instantiating launch_typed for its type, so the kernels build in parallel.
//
// One thread per lattice site (grid-stride over sites), one right-hand side
// per blockIdx.y.  Loads are SoA planes, so each of the 12 spinor components
// and each link entry is a contiguous 64-lane access; the 8 neighbour spinors
// of a site are shared with 8 other sites through L2.  Reductions
// (||M p||^2 and r^H r) are deterministic and fence-free: fixed-order
// wave/workgroup sums into one partial slot per workgroup; the second pass
// sums the first pass's partials itself (same order in every workgroup) to
// get alpha, and a one-workgroup finalize kernel, ordered by the stream,
// updates the CG scalars of every column.
#include <algorithm>
#include <type_traits>

#include <mutex>

#include <hip/hip_ext.h>

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
  double* partial;          // this pass's per-workgroup partials
  const double* partial_in;  // kEpiCGR: partials of the first pass (p^H A p)
  void* r; size_t r_cs;
  const void* b; size_t b_cs;
  void* tbuf; size_t t_cs;
  double* hist; int hist_stride;
  uint32_t ord_P, ord_Ls;   // slab sweep: 64-site tiles per xy-plane, t-slices per XCD
  uint32_t ord_Bz;          // slab sweep: z-planes per block (divides Lz; 1 = no blocks)
  uint32_t zc_n, zc_len;    // z-march: z-chunks per (xy tile, t) column and their length
  // odd-even geometry: output parity, the other parity's link block, and
  // out = dg in2 + ch (hopping sum of in) at the centre (in2 may be null)
  uint32_t par;
  const void* u2;
  const void* in2; size_t in2_cs;
  double dg, ch;
};

// Work units (blocks of sites) handed to workgroups.  With xcd set, the
// units are split into eight contiguous chunks and workgroup b (which the
// hardware places on XCD b % 8) walks chunk b % 8, so the workgroups sharing
// an XCD's L2 sweep neighbouring sites together.
struct Units {
  uint32_t u, end, step;
  __device__ __forceinline__ Units(uint32_t T, bool xcd) {
    if (!xcd) {
      u = blockIdx.x;
      end = T;
      step = gridDim.x;
    } else {
      const uint32_t x = blockIdx.x & 7u, q = blockIdx.x >> 3;
      const uint32_t C = (T + 7u) >> 3;
      u = x * C + q;
      end = min((x + 1) * C, T);
      step = gridDim.x >> 3;
    }
  }
};

// CG epilogue for components [C0, C0 + NC) of site s, given o = op(in) there.
template <typename VS, int EPI, int C0, int NC, bool NT = false>
__device__ __forceinline__ void epilogue(const DevArgs& a, int col, uint32_t s,
                                         const cpx<typename Storage<VS>::real>* o,
                                         typename Storage<VS>::real alpha, bool save_t,
                                         int save_slot, typename Storage<VS>::real& acc2) {
  using R = typename Storage<VS>::real;
  const size_t vs = (size_t)a.g.vs;
  if (EPI == kEpiStore || EPI == kEpiNorm) {
    VS* out = reinterpret_cast<VS*>(a.out) + (size_t)col * a.out_cs;
#pragma unroll
    for (int e = C0; e < C0 + NC; ++e) {
      if (NT) Storage<VS>::st_nt(out, (size_t)e * vs + s, o[e]);
      else Storage<VS>::st(out, (size_t)e * vs + s, o[e]);
      if (EPI == kEpiNorm) acc2 += o[e].re * o[e].re + o[e].im * o[e].im;
    }
  } else if (EPI == kEpiCGR) {
    VS* r = reinterpret_cast<VS*>(a.r) + (size_t)col * a.r_cs;
    if (save_t) {
      VS* t = reinterpret_cast<VS*>(a.tbuf) + ((size_t)col * 2 + save_slot) * a.t_cs;
#pragma unroll
      for (int e = C0; e < C0 + NC; ++e) Storage<VS>::st(t, (size_t)e * vs + s, o[e]);
    }
    // every component of r is loaded before the first store: a store to r
    // could alias a later load for all the compiler knows, which would
    // otherwise serialise one memory round trip per component
    cpx<R> rv[NC];
#pragma unroll
    for (int e = C0; e < C0 + NC; ++e)
      rv[e - C0] = NT ? Storage<VS>::ld_nt(r, (size_t)e * vs + s) : Storage<VS>::ld(r, (size_t)e * vs + s);
#pragma unroll
    for (int e = C0; e < C0 + NC; ++e) {
      cpx<R> v = rv[e - C0];
      v.re -= alpha * o[e].re;
      v.im -= alpha * o[e].im;
      if (NT) Storage<VS>::st_nt(r, (size_t)e * vs + s, v);
      else Storage<VS>::st(r, (size_t)e * vs + s, v);
      acc2 += v.re * v.re + v.im * v.im;
    }
  } else {  // kEpiRes: r = b - op(in)
    VS* r = reinterpret_cast<VS*>(a.r) + (size_t)col * a.r_cs;
    const VS* b = reinterpret_cast<const VS*>(a.b) + (size_t)col * a.b_cs;
    cpx<R> bv[NC];  // loaded before the first store to r (see above)
#pragma unroll
    for (int e = C0; e < C0 + NC; ++e)
      bv[e - C0] = NT ? Storage<VS>::ld_nt(b, (size_t)e * vs + s) : Storage<VS>::ld(b, (size_t)e * vs + s);
#pragma unroll
    for (int e = C0; e < C0 + NC; ++e) {
      cpx<R> rv = {bv[e - C0].re - o[e].re, bv[e - C0].im - o[e].im};
      if (NT) Storage<VS>::st_nt(r, (size_t)e * vs + s, rv);
      else Storage<VS>::st(r, (size_t)e * vs + s, rv);
      acc2 += rv.re * rv.re + rv.im * rv.im;
    }
  }
}

// Column activity and (second pass) alpha for this workgroup's column.
template <typename VS, int EPI>
__device__ __forceinline__ bool column_setup(const DevArgs& a, int col, double* lds4,
                                             typename Storage<VS>::real& alpha, bool& save_t,
                                             int& save_slot) {
  using R = typename Storage<VS>::real;
  bool active = ((a.mask >> col) & 1u) != 0;
  if (active && (EPI == kEpiNorm || EPI == kEpiCGR)) active = a.st[col].state == ColRun;
  alpha = R(0);
  save_t = false;
  save_slot = 0;
  if (EPI == kEpiCGR) {
    // alpha = rho / ||M p||^2 from the first pass's partials, summed in the
    // same fixed order by every workgroup (and by the finalize kernel)
    const double pap = reduce_partials(a.partial_in + (size_t)col * gridDim.x, gridDim.x, lds4);
    if (active) {
      if (pap > 0.0 && pap < INFINITY) {
        alpha = (R)(a.st[col].rho / pap);
        const int j = a.st[col].iter + 1;  // iteration being completed
        save_t = a.tbuf != nullptr && (j == a.st[col].save_t0 || j == a.st[col].save_t1);
        save_slot = j & 1;
      } else {
        active = false;  // breakdown: the finalize kernel stops the column
      }
    }
  }
  return active;
}

// Variants 1 and 2: one thread per site, all eight hops; 256 sites per unit,
// round-robin (1) or XCD-contiguous (2) unit mapping.
template <typename VS, typename LS, bool COMP, bool DAG, int EPI, bool XCD>
__global__ __launch_bounds__(kBlock) void k_wilson(DevArgs a) {
  using R = typename Storage<VS>::real;
  __shared__ double lds4[kBlock / 64];
  __shared__ R ldsr[kBlock / 64];
  const int col = blockIdx.y;
  R alpha;
  bool save_t;
  int save_slot;
  const bool active = column_setup<VS, EPI>(a, col, lds4, alpha, save_t, save_slot);
  const VS* in = reinterpret_cast<const VS*>(a.in) + (size_t)col * a.in_cs;
  const LS* u = reinterpret_cast<const LS*>(a.u);
  const size_t vs = (size_t)a.g.vs;
  R acc2 = R(0);
  if (active) {
    const uint32_t T = ((uint32_t)a.g.V + kBlock - 1) / kBlock;
    for (Units it(T, XCD); it.u < it.end; it.u += it.step) {
      const uint32_t s = it.u * kBlock + threadIdx.x;
      if (s >= (uint32_t)a.g.V) continue;
      cpx<R> h[12];
      hopping_site<VS, LS, COMP, DAG ? 1 : -1>(in, u, a.g, s, h);
      const R d = (R)a.diag;
      cpx<R> o[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) {
        cpx<R> v = Storage<VS>::ld(in, (size_t)e * vs + s);
        o[e] = {d * v.re - R(0.5) * h[e].re, d * v.im - R(0.5) * h[e].im};
      }
      epilogue<VS, EPI, 0, 12>(a, col, s, o, alpha, save_t, save_slot, acc2);
    }
  }
  if (EPI == kEpiStore) return;
  R bs = block_sum(acc2, ldsr);
  if (threadIdx.x == 0) a.partial[(size_t)col * gridDim.x + blockIdx.x] = (double)bs;
}

// Variants 3..10: a unit is two 64-site tiles; each tile is handled by a pair
// of waves, the even wave doing directions x and y, the odd wave z and t.
// They swap half of their partial sums through LDS and each finishes six of
// the twelve output components, so per-thread state is half of variant 1's
// and twice as many waves stream the lattice.  A workgroup serves NC columns
// (right-hand sides blockIdx.y NC .. + NC - 1): every link is loaded once per
// site and applied to all of them, and each column's arithmetic and
// reduction order are those of NC = 1, so results do not depend on NC.
// EO: odd-even geometry, one pass of the Schur complement (sites of parity
// a.par, neighbours read from the other parity's half field).
template <typename VS, typename LS, bool COMP, bool DAG, int EPI, bool NT, int ORD, int NC,
          bool EO = false>
__global__ __launch_bounds__(kBlock) void k_wilson_pair(DevArgs a) {
  using R = typename Storage<VS>::real;
  __shared__ double lds4[kBlock / 64];
  __shared__ R ldsr[kBlock / 64];
  __shared__ cpx<R> xbuf[2][2][NC][6][64];  // [tile][writer parity][column][component][lane]
  const int col0 = blockIdx.y * NC;
  R alpha[NC];
  bool save_t[NC];
  int save_slot[NC];
  uint32_t act = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    bool on = false;
    alpha[c] = R(0);
    save_t[c] = false;
    save_slot[c] = 0;
    if (col0 + c < a.ncols) on = column_setup<VS, EPI>(a, col0 + c, lds4, alpha[c], save_t[c],
                                                       save_slot[c]);
    if (on) act |= 1u << c;
  }
  const VS* in = reinterpret_cast<const VS*>(a.in) + (size_t)col0 * a.in_cs;
  const LS* u = reinterpret_cast<const LS*>(a.u);
  const LS* u2 = reinterpret_cast<const LS*>(a.u2);
  const VS* in2 = EO && a.in2 ? reinterpret_cast<const VS*>(a.in2) + (size_t)col0 * a.in2_cs
                              : nullptr;
  const size_t vs = (size_t)a.g.vs;
  const int tile = threadIdx.x >> 7;
  const int odd = (threadIdx.x >> 6) & 1;
  const int lane = threadIdx.x & 63;
  R acc2[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc2[c] = R(0);
  // one 128-site unit: tile `tile` of this workgroup covers sites s (valid)
  auto unit = [&](uint32_t s, bool valid) {
      cpx<R> acc[NC][12];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int e = 0; e < 12; ++e) acc[c][e] = {R(0), R(0)};
      if (valid) {
        uint32_t coord[4];
        uint32_t sl = s;  // lattice site
        if (EO) sl = eo_site_coords(a.g, s, a.par, coord);
        else site_coords(a.g, s, coord);
        if (!odd) {
          hop_dir_n<0, VS, LS, COMP, DAG ? 1 : -1, NC, EO>(in, a.in_cs, act, u, u2, a.g, sl, coord, acc);
          hop_dir_n<1, VS, LS, COMP, DAG ? 1 : -1, NC, EO>(in, a.in_cs, act, u, u2, a.g, sl, coord, acc);
        } else {
          hop_dir_n<2, VS, LS, COMP, DAG ? 1 : -1, NC, EO>(in, a.in_cs, act, u, u2, a.g, sl, coord, acc);
          hop_dir_n<3, VS, LS, COMP, DAG ? 1 : -1, NC, EO>(in, a.in_cs, act, u, u2, a.g, sl, coord, acc);
        }
      }
      // hand the partner the half it finishes: even keeps 0..5, odd keeps 6..11
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (odd) {
#pragma unroll
          for (int e = 0; e < 6; ++e) xbuf[tile][1][c][e][lane] = acc[c][e];
        } else {
#pragma unroll
          for (int e = 0; e < 6; ++e) xbuf[tile][0][c][e][lane] = acc[c][6 + e];
        }
      }
      __syncthreads();
      const R d = EO ? (R)a.dg : (R)a.diag;
      const R ch = (R)a.ch;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (!((act >> c) & 1u)) continue;
        const VS* ic = EO ? (in2 ? in2 + (size_t)c * a.in2_cs : nullptr) : in + (size_t)c * a.in_cs;
        const bool ld_c = valid && (!EO || ic != nullptr);
        cpx<R> o[12];
        if (!odd) {
#pragma unroll
          for (int e = 0; e < 6; ++e) {
            const cpx<R> p = xbuf[tile][1][c][e][lane];
            cpx<R> v = ld_c ? Storage<VS>::ld(ic, (size_t)e * vs + s) : cpx<R>{R(0), R(0)};
            const R hr = acc[c][e].re + p.re, hi = acc[c][e].im + p.im;
            if constexpr (EO) o[e] = {d * v.re + ch * hr, d * v.im + ch * hi};
            else o[e] = {d * v.re - R(0.5) * hr, d * v.im - R(0.5) * hi};
          }
          if (valid)
            epilogue<VS, EPI, 0, 6, NT>(a, col0 + c, s, o, alpha[c], save_t[c], save_slot[c],
                                        acc2[c]);
        } else {
#pragma unroll
          for (int e = 6; e < 12; ++e) {
            const cpx<R> p = xbuf[tile][0][c][e - 6][lane];
            cpx<R> v = ld_c ? Storage<VS>::ld(ic, (size_t)e * vs + s) : cpx<R>{R(0), R(0)};
            const R hr = p.re + acc[c][e].re, hi = p.im + acc[c][e].im;
            if constexpr (EO) o[e] = {d * v.re + ch * hr, d * v.im + ch * hi};
            else o[e] = {d * v.re - R(0.5) * hr, d * v.im - R(0.5) * hi};
          }
          if (valid)
            epilogue<VS, EPI, 6, 6, NT>(a, col0 + c, s, o, alpha[c], save_t[c], save_slot[c],
                                        acc2[c]);
        }
      }
      __syncthreads();
  };
  if (act) {
    if (ORD == 0) {
      const uint32_t T = ((uint32_t)a.g.V + 127u) / 128u;
      for (Units it(T, true); it.u < it.end; it.u += it.step) {
        const uint32_t s = it.u * 128u + tile * 64u + lane;
        unit(s, s < (uint32_t)a.g.V);
      }
    } else {
      // XCD x owns the t-slab [x Ls, (x + 1) Ls) and visits its 64-site tiles
      // (P per xy-plane) in (z-block, t, z, xy) order with blocks of Bz
      // z-planes: t-neighbours are Bz P tiles apart in the sweep and
      // z-neighbours inside a block P tiles apart, so they are still in the
      // XCD's L2 when the sweeping front reaches them.  With Bz = 1 the order
      // is (z, t, xy) and z-neighbours are Ls P tiles apart.
      const uint32_t x = blockIdx.x & 7u, step = gridDim.x >> 3;
      const uint32_t P = a.ord_P, Ls = a.ord_Ls, Bz = a.ord_Bz;
      const uint32_t ntx = P * Ls * (uint32_t)a.g.L[2];
      const uint32_t units = (ntx + 1u) >> 1;
      for (uint32_t un = blockIdx.x >> 3; un < units; un += step) {
        const uint32_t pos = 2u * un + (uint32_t)tile;
        const bool valid = pos < ntx;
        uint32_t s = 0;
        if (valid) {
          const uint32_t xyt = pos % P, rest = pos / P;
          const uint32_t zi = rest % Bz, r2 = rest / Bz;
          const uint32_t t = x * Ls + r2 % Ls, z = (r2 / Ls) * Bz + zi;
          s = ((t * (uint32_t)a.g.L[2] + z) * P + xyt) * 64u + (uint32_t)lane;
        }
        unit(s, valid);
      }
    }
  }
  if (EPI == kEpiStore) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    R bs = block_sum(acc2[c], ldsr);
    if (threadIdx.x == 0 && col0 + c < a.ncols)
      a.partial[(size_t)(col0 + c) * gridDim.x + blockIdx.x] = (double)bs;
  }
}

// Variants 11..13: z-march.  Lane l of a wave owns the sites (xy = 64 tile +
// l, z, t) of one t-slice and marches z through a chunk of zc_len planes.
// The z-hops come from registers: the forward hop's link U_z(s) also forms
// the backward hop of site s + z, U_z(s)^+ (1 -+ g_z) psi(s), which is carried
// to the next plane, so along z every spinor and link is loaded once by its
// own lane.  The x, y and t neighbours of a plane are the sites the other
// lanes and waves march over at the same time (all waves start at the first
// plane of their chunk together), so they are L2 hits.  XCD x owns the
// t-slab [x Ls, (x + 1) Ls) (workgroup b runs on XCD b mod 8), so the working
// set of one plane step on an XCD is one z-plane of its slab.  Per site the
// hops are accumulated in the order of variant 1 (x, y, z forward then
// backward, t) with the same expressions: a site's output equals variant 1's
// bit for bit; only the order of the partial sums of the reductions differs.
template <typename VS, typename LS, bool COMP, bool DAG, int EPI>
__global__ __launch_bounds__(kBlock) void k_wilson_zmarch(DevArgs a) {
  using R = typename Storage<VS>::real;
  constexpr int SF = DAG ? 1 : -1;
  __shared__ double lds4[kBlock / 64];
  __shared__ R ldsr[kBlock / 64];
  const int col = blockIdx.y;
  R alpha;
  bool save_t;
  int save_slot;
  const bool active = column_setup<VS, EPI>(a, col, lds4, alpha, save_t, save_slot);
  const VS* in = reinterpret_cast<const VS*>(a.in) + (size_t)col * a.in_cs;
  const LS* u = reinterpret_cast<const LS*>(a.u);
  const size_t vs = (size_t)a.g.vs;
  R acc2 = R(0);
  const uint32_t P = a.ord_P, Ls = a.ord_Ls;
  const uint32_t wv = (blockIdx.x >> 3) * (kBlock / 64) + (threadIdx.x >> 6);  // wave of the XCD
  if (active && wv < P * Ls * a.zc_n) {
    const uint32_t tile = wv % P, rest = wv / P;
    const uint32_t t = (blockIdx.x & 7u) * Ls + rest % Ls;
    const uint32_t zc = rest / Ls;
    const uint32_t xy = tile * 64u + (threadIdx.x & 63u);
    const uint32_t Lz = (uint32_t)a.g.L[2];
    const uint32_t plane = (uint32_t)a.g.stride[2];  // Lx Ly
    const uint32_t z0 = zc * a.zc_len;
    const uint32_t z1 = min(z0 + a.zc_len, Lz);
    uint32_t coord[4];
    coord[1] = a.g.dx.div(xy);
    coord[0] = xy - coord[1] * (uint32_t)a.g.L[0];
    coord[3] = t;
    const uint32_t base = t * Lz * plane + xy;  // site at z = 0
    // carried backward z-hop: g = U_z(s - z)^+ h(psi(s - z)), two spin rows x 3 colours
    cpx<R> cg[6];
    auto carry = [&](uint32_t sb, const cpx<R>* U) {
      cpx<R> h[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cpx<R> u0 = Storage<VS>::ld(in, (size_t)(0 + c) * vs + sb);
        cpx<R> u1 = Storage<VS>::ld(in, (size_t)(3 + c) * vs + sb);
        cpx<R> l0 = Storage<VS>::ld(in, (size_t)(6 + c) * vs + sb);
        cpx<R> l1 = Storage<VS>::ld(in, (size_t)(9 + c) * vs + sb);
        project<2, -SF>(u0, u1, l0, l1, h[c], h[3 + c]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cpx<R> g0 = cmulc(U[0 * 3 + c], h[0]);
        cpx<R> g1 = cmulc(U[0 * 3 + c], h[3]);
        g0 = cadd(g0, cmulc(U[1 * 3 + c], h[1]));
        g1 = cadd(g1, cmulc(U[1 * 3 + c], h[4]));
        g0 = cadd(g0, cmulc(U[2 * 3 + c], h[2]));
        g1 = cadd(g1, cmulc(U[2 * 3 + c], h[5]));
        cg[c] = g0;
        cg[3 + c] = g1;
      }
    };
    if (z0 < z1) {  // prologue: the backward hop into the chunk's first plane
      const uint32_t sb = base + ((z0 > 0 ? z0 : Lz) - 1u) * plane;
      cpx<R> U[9];
      load_link<LS, COMP>(u, 2, vs, sb, U);
      carry(sb, U);
    }
    for (uint32_t z = z0; z < z1; ++z) {
      const uint32_t s = base + z * plane;
      coord[2] = z;
      cpx<R> acc[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) acc[e] = {R(0), R(0)};
      hop_dir<0, VS, LS, COMP, SF>(in, u, a.g, s, coord, acc);
      hop_dir<1, VS, LS, COMP, SF>(in, u, a.g, s, coord, acc);
      {
        cpx<R> U[9];
        load_link<LS, COMP>(u, 2, vs, s, U);
        const uint32_t sf = z + 1u < Lz ? s + plane : base;
        cpx<R> h[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cpx<R> u0 = Storage<VS>::ld(in, (size_t)(0 + c) * vs + sf);
          cpx<R> u1 = Storage<VS>::ld(in, (size_t)(3 + c) * vs + sf);
          cpx<R> l0 = Storage<VS>::ld(in, (size_t)(6 + c) * vs + sf);
          cpx<R> l1 = Storage<VS>::ld(in, (size_t)(9 + c) * vs + sf);
          project<2, SF>(u0, u1, l0, l1, h[c], h[3 + c]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cpx<R> g0 = cmul(U[c * 3 + 0], h[0]);
          cpx<R> g1 = cmul(U[c * 3 + 0], h[3]);
          g0 = cadd(g0, cmul(U[c * 3 + 1], h[1]));
          g1 = cadd(g1, cmul(U[c * 3 + 1], h[4]));
          g0 = cadd(g0, cmul(U[c * 3 + 2], h[2]));
          g1 = cadd(g1, cmul(U[c * 3 + 2], h[5]));
          accumulate<2, SF>(acc, c, g0, g1);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) accumulate<2, -SF>(acc, c, cg[c], cg[3 + c]);
        carry(s, U);  // the backward hop into plane z + 1
      }
      hop_dir<3, VS, LS, COMP, SF>(in, u, a.g, s, coord, acc);
      const R d = (R)a.diag;
      cpx<R> o[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) {
        cpx<R> v = Storage<VS>::ld(in, (size_t)e * vs + s);
        o[e] = {d * v.re - R(0.5) * acc[e].re, d * v.im - R(0.5) * acc[e].im};
      }
      epilogue<VS, EPI, 0, 12, true>(a, col, s, o, alpha, save_t, save_slot, acc2);
    }
  }
  if (EPI == kEpiStore) return;
  R bs = block_sum(acc2, ldsr);
  if (threadIdx.x == 0) a.partial[(size_t)col * gridDim.x + blockIdx.x] = (double)bs;
}

// CG scalars after the second stencil pass (one workgroup): p^H A p from the
// first pass's partials (alpha, or breakdown), r^H r from the second pass's
// partials (beta, history, stop tests, eigCG t-save schedule).  With a
// preconditioner (spec_s): the stop tests keep ||r||^2 and the CG scalar
// becomes r^H z = ||r||^2 + spec_s[c].
__global__ __launch_bounds__(kBlock) void k_finalize_cg(ColState* st, int ncols, uint32_t mask,
                                                        const double* part_a, const double* part_b,
                                                        int nb, double* hist, int hist_stride,
                                                        const double* spec_s) {
  __shared__ double lds4[kBlock / 64];
  {
    const int c = blockIdx.x;  // one workgroup per column
    if (c >= ncols || !((mask >> c) & 1u)) return;
    const double pap = reduce_partials(part_a + (size_t)c * nb, nb, lds4);
    const double rr_new = reduce_partials(part_b + (size_t)c * nb, nb, lds4);
    const double rho_new = spec_s ? rr_new + spec_s[c] : rr_new;
    if (threadIdx.x != 0) return;
    ColState& S = st[c];
    if (S.state == ColRun) {
      S.pap = pap;
      if (!(pap > 0.0 && pap < INFINITY)) {
        S.alpha = 0.0;
        S.state = ColStopPending;
        S.reason = ReasonBreakdown;
        return;
      }
      S.alpha = S.rho / pap;
      const int j = S.iter + 1;
      const double beta = rho_new / S.rho;
      if (hist) {
        double* h = hist + (size_t)c * hist_stride + (size_t)3 * (j - 1);
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
      } else if (rr_new <= S.stop2) {
        S.state = ColStopPending;
        S.reason = ReasonConverged;
      } else if (rr_new <= S.restart2) {
        S.state = ColStopPending;
        S.reason = ReasonRestart;
      } else if (j >= S.max_iter) {
        S.state = ColStopPending;
        S.reason = ReasonMaxIter;
      }
    } else if (S.state == ColStopPending) {
      S.state = ColStopped;
    }
  }
}

// rho = ||b - A x||^2 of a true-residual pass
__global__ __launch_bounds__(kBlock) void k_finalize_res(ColState* st, int ncols, uint32_t mask,
                                                         const double* part, int nb) {
  __shared__ double lds4[kBlock / 64];
  const int c = blockIdx.x;  // one workgroup per column
  if (c >= ncols || !((mask >> c) & 1u)) return;
  const double tot = reduce_partials(part + (size_t)c * nb, nb, lds4);
  if (threadIdx.x == 0) st[c].rho = tot;
}

// Two-tile kernel occupancy control.  `per_cu` > 0 caps the workgroups that
// share a CU by reserving LDS (fewer misses in flight per XCD, so stencil
// neighbours stay in the L2 until their second use); 0 leaves the natural
// occupancy.  Returns the dynamic LDS bytes to request and sets the number of
// workgroups resident on the whole device (a multiple of 8).
template <typename VS, typename LS, bool EO>
size_t pair_occupancy(int per_cu, int* resident) {
  struct Info { size_t lds; int resident; };
  static Info cache[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  Info& I = cache[per_cu & 3];
  if (I.resident == 0) {
    auto kern = k_wilson_pair<VS, LS, true, false, kEpiCGR, true, 0, 1, EO>;
    int dev = 0, cus = 0, lds_cu = 0, lds_wg = 0, per = 0;
    hipFuncAttributes fa{};
    size_t extra = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess &&
        hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
            hipSuccess &&
        hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern)) == hipSuccess) {
      if (per_cu > 0) {
        // smallest per-workgroup LDS that lets only per_cu workgroups fit
        const size_t want = (size_t)lds_cu / (size_t)(per_cu + 1) + 1024;
        if (want > fa.sharedSizeBytes && want <= (size_t)lds_wg) extra = want - fa.sharedSizeBytes;
      }
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kBlock, extra) != hipSuccess)
        per = 0;
    }
    I.lds = extra;
    I.resident = (per > 0 && cus > 0) ? std::max(8, std::min(kMaxGrid, (per * cus) & ~7))
                                      : kMaxGrid;
  }
  *resident = I.resident;
  return I.lds;
}

// One stencil pass.  EO: one pass of the odd-even operator with the output
// parity, second input and coefficients of L's eo_* fields.
template <typename VS, typename LS, bool EO = false>
hipError_t launch_typed(const StencilLaunch& L, hipStream_t s) {
  constexpr int NC4 = sizeof(typename Storage<VS>::real) == 4 ? 4 : 2;
  if ((L.g->eo != 0) != EO) return hipErrorInvalidValue;
  DevArgs a;
  a.in = L.in; a.in_cs = L.in_cs; a.out = L.out; a.out_cs = L.out_cs; a.u = L.u; a.g = *L.g;
  a.diag = L.diag; a.ncols = L.ncols; a.mask = L.mask; a.st = L.st;
  a.par = 0; a.u2 = nullptr; a.in2 = nullptr; a.in2_cs = 0; a.dg = 0.0; a.ch = -0.5;
  if (EO) {
    // link parity blocks: 4 directions x (6 or 9) planes each
    const size_t blk = (size_t)4 * (L.compressed ? 6 : 9) * L.g->vs;
    const LS* ub = reinterpret_cast<const LS*>(L.u);
    a.par = (uint32_t)(L.eo_par & 1);
    a.u = ub + (a.par ? blk : 0);
    a.u2 = ub + (a.par ? 0 : blk);
    a.in2 = L.in2; a.in2_cs = L.in2_cs;
    a.dg = L.in2 ? L.eo_dg : 0.0;
    a.ch = L.eo_ch;
  }
  // first pass (kEpiNorm) writes partial slot A, second pass (kEpiCGR, kEpiRes) slot B
  double* part_a = L.partial;
  double* part_b = L.partial + (size_t)kMaxCols * kMaxGrid;
  a.partial = (L.epi == kEpiNorm) ? part_a : part_b;
  a.partial_in = part_a;
  a.r = L.r; a.r_cs = L.r_cs; a.b = L.b; a.b_cs = L.b_cs;
  a.tbuf = L.tbuf; a.t_cs = L.t_cs; a.hist = L.hist; a.hist_stride = L.hist_stride;
  // 16-bit storage instantiates only the streaming two-tile kernels with
  // two-row links: other variants run as 5, uncompressed links are refused
  constexpr bool kHalf = std::is_same<VS, f16x2>::value;
  int variant = L.variant <= 0 ? 1 : L.variant;
  if (EO && variant < 3) variant = 3;  // the odd-even passes use the two-tile kernels
  if (kHalf) {
    if (!L.compressed) return hipErrorInvalidValue;
    if (variant < 5) variant = 5;
    if (variant == 10) variant = 9;
    if (variant == 15) variant = 14;
  }
  const uint32_t plane = (uint32_t)(L.g->L[0] * L.g->L[1]) >> (EO ? 1 : 0);
  a.ord_P = plane / 64u;
  a.ord_Ls = (uint32_t)L.g->L[3] / 8u;
  a.ord_Bz = 1;
  if (variant == 14 || variant == 15) {  // z-blocked slab sweep: the largest of 4, 3, 2 dividing Lz
    const uint32_t Lz = (uint32_t)L.g->L[2];
    a.ord_Bz = Lz % 4u == 0 ? 4u : Lz % 3u == 0 ? 3u : Lz % 2u == 0 ? 2u : 1u;
  }
  a.zc_n = 1;
  a.zc_len = (uint32_t)L.g->L[2];
  int gx = 0;
  if (variant >= 11 && variant <= 13) {
    // z-march: 1, 2 or 4 z-chunks per column; needs the full geometry, whole
    // 64-site tiles per xy-plane, a t-slab per XCD and a grid within kMaxGrid
    const uint32_t n = variant == 11 ? 1u : variant == 12 ? 2u : 4u;
    const uint32_t Lz = (uint32_t)L.g->L[2];
    a.zc_n = std::min(n, Lz);
    a.zc_len = (Lz + a.zc_n - 1) / a.zc_n;
    a.zc_n = (Lz + a.zc_len - 1) / a.zc_len;  // no empty chunk
    const uint32_t waves = a.ord_P * a.ord_Ls * a.zc_n;
    gx = (int)(8u * ((waves + kBlock / 64 - 1) / (kBlock / 64)));
    if (EO || plane % 64u != 0 || L.g->L[3] % 8 != 0 || gx > kMaxGrid) variant = 6;
  }
  if ((variant >= 8 && variant <= 10 || variant >= 14) &&
      (plane % 64u != 0 || L.g->L[3] % 8 != 0))
    variant = variant == 8 ? 5 : 6;  // the slab sweep needs whole tiles per plane, 8 slabs
  const uint32_t unit = variant >= 3 ? 128u : (uint32_t)kBlock;
  const uint32_t T = ((uint32_t)L.g->V + unit - 1) / unit;
  size_t dyn_lds = 0;
  if (variant >= 11 && variant <= 13) {
    // grid set above
  } else if (variant == 1) {
    gx = (int)std::min<uint32_t>(T, kMaxGrid);
  } else if (variant >= 5) {
    // as many workgroups as are resident at once (multiple of 8), so each
    // XCD's workgroups sweep one contiguous front of its chunk
    int res = 0;
    const int per_cu = (variant == 6 || variant >= 9) ? 2 : variant == 7 ? 1 : 0;
    dyn_lds = pair_occupancy<VS, LS, EO>(per_cu, &res);
    gx = (int)std::min<uint32_t>((T + 7u) & ~7u, (uint32_t)res);
  } else {
    gx = (int)std::min<uint32_t>((T + 7u) & ~7u, kMaxGrid);  // a multiple of 8 (XCDs)
  }
  // columns per workgroup of the two-tile kernels (links loaded once per
  // site for all of them); the grid's x extent and the site-to-workgroup map
  // do not depend on it, so every column's reductions are the same for any
  // batch width.  FP64 takes at most 2 (LDS of the exchange buffer).
  int nc = 1;
  if (variant >= 3 && (variant <= 10 || variant >= 14) && L.compressed && L.ncols >= 2) {
    const int widest = (L.ncols >= 4 && sizeof(typename Storage<VS>::real) == 4) ? 4 : 2;
    nc = L.nc > 0 ? std::min(L.nc, widest) : widest;
    if (nc == 3) nc = 2;
  }
  if (nc > 1) dyn_lds = 0;  // the larger exchange buffer already caps occupancy
  dim3 grid(gx, (L.ncols + nc - 1) / nc), block(kBlock);
#define EIGCG_LAUNCH(KERNEL, LDS)                                                     \
  hipExtLaunchKernelGGL(KERNEL, grid, block, LDS, s, L.ev_start, L.ev_stop, 0, a);
#define EIGCG_PAIR(COMP, DAG, EPI, NT, ORD)                                           \
  if (nc == 4) {                                                                     \
    EIGCG_LAUNCH((k_wilson_pair<VS, LS, COMP, DAG, EPI, NT, ORD, NC4, EO>), dyn_lds) \
  } else if (nc == 2) {                                                              \
    EIGCG_LAUNCH((k_wilson_pair<VS, LS, COMP, DAG, EPI, NT, ORD, 2, EO>), dyn_lds)   \
  } else {                                                                           \
    EIGCG_LAUNCH((k_wilson_pair<VS, LS, COMP, DAG, EPI, NT, ORD, 1, EO>), dyn_lds)   \
  }
#define EIGCG_K(COMP, DAG, EPI)                                                      \
  if (variant >= 11 && variant <= 13) {                                              \
    if constexpr (!EO) {                                                             \
      EIGCG_LAUNCH((k_wilson_zmarch<VS, LS, COMP, DAG, EPI>), 0)                     \
    }                                                                                \
  } else if (variant == 10 || variant == 15) {                                       \
    EIGCG_PAIR(COMP, DAG, EPI, false, 1)                                             \
  } else if (variant >= 8) {                                                         \
    EIGCG_PAIR(COMP, DAG, EPI, true, 1)                                              \
  } else if (variant >= 4) {                                                         \
    EIGCG_PAIR(COMP, DAG, EPI, true, 0)                                              \
  } else if (variant == 3) {                                                         \
    EIGCG_PAIR(COMP, DAG, EPI, false, 0)                                             \
  } else if constexpr (!EO) {                                                        \
    if (variant == 2) {                                                              \
      EIGCG_LAUNCH((k_wilson<VS, LS, COMP, DAG, EPI, true>), 0)                      \
    } else {                                                                         \
      EIGCG_LAUNCH((k_wilson<VS, LS, COMP, DAG, EPI, false>), 0)                     \
    }                                                                                \
  }
#define EIGCG_EPI(COMP, DAG)                                  \
  switch (L.epi) {                                            \
    case kEpiStore: { EIGCG_K(COMP, DAG, kEpiStore) } break;  \
    case kEpiNorm: { EIGCG_K(COMP, DAG, kEpiNorm) } break;    \
    case kEpiCGR: { EIGCG_K(COMP, DAG, kEpiCGR) } break;      \
    default: { EIGCG_K(COMP, DAG, kEpiRes) } break;           \
  }
  if constexpr (kHalf) {
#define EIGCG_KH(COMP, DAG, EPI)                                                     \
  if (variant >= 11 && variant <= 13) {                                              \
    if constexpr (!EO) {                                                             \
      EIGCG_LAUNCH((k_wilson_zmarch<VS, LS, COMP, DAG, EPI>), 0)                     \
    }                                                                                \
  } else if (variant >= 8) {                                                         \
    EIGCG_PAIR(COMP, DAG, EPI, true, 1)                                              \
  } else {                                                                           \
    EIGCG_PAIR(COMP, DAG, EPI, true, 0)                                              \
  }
    switch ((L.op == kOpMdag ? 4 : 0) + L.epi) {
      case 0: { EIGCG_KH(true, false, kEpiStore) } break;
      case 1: { EIGCG_KH(true, false, kEpiNorm) } break;
      case 2: { EIGCG_KH(true, false, kEpiCGR) } break;
      case 3: { EIGCG_KH(true, false, kEpiRes) } break;
      case 4: { EIGCG_KH(true, true, kEpiStore) } break;
      case 5: { EIGCG_KH(true, true, kEpiNorm) } break;
      case 6: { EIGCG_KH(true, true, kEpiCGR) } break;
      default: { EIGCG_KH(true, true, kEpiRes) } break;
    }
#undef EIGCG_KH
  } else {
    if (L.compressed) {
      if (L.op == kOpMdag) { EIGCG_EPI(true, true) } else { EIGCG_EPI(true, false) }
    } else {
      if (L.op == kOpMdag) { EIGCG_EPI(false, true) } else { EIGCG_EPI(false, false) }
    }
  }
#undef EIGCG_EPI
#undef EIGCG_K
#undef EIGCG_PAIR
#undef EIGCG_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (L.grid_out) *L.grid_out = gx;
  if (L.epi == kEpiCGR) {
    if (!L.defer_finalize)
      hipLaunchKernelGGL(k_finalize_cg, dim3(L.ncols), dim3(kBlock), 0, s, L.st, L.ncols, L.mask,
                         part_a, part_b, gx, L.hist, L.hist_stride, (const double*)nullptr);
  } else if (L.epi == kEpiRes)
    hipLaunchKernelGGL(k_finalize_res, dim3(L.ncols), dim3(kBlock), 0, s, L.st, L.ncols, L.mask, part_b,
                       gx);
  return hipGetLastError();
}

// Odd-even operator: Mhat (or Mhat^H) = diag - D_eo D_oe / (4 diag) as two
// passes through L.eo_tmp, the epilogue on the second; or one raw pass.
// Sampling events bracket both passes.
template <typename VS, typename LS>
hipError_t launch_eo(const StencilLaunch& L, hipStream_t s) {
  if (L.eo_raw) return launch_typed<VS, LS, true>(L, s);
  if (!L.eo_tmp) return hipErrorInvalidValue;
  StencilLaunch A = L;  // t = D_oe in / (2 diag) on the odd sites
  A.epi = kEpiStore;
  A.out = L.eo_tmp; A.out_cs = L.eo_tmp_cs;
  A.eo_par = 1;
  A.in2 = nullptr; A.in2_cs = 0;
  A.eo_dg = 0.0;
  A.eo_ch = 0.5 / L.diag;
  A.ev_stop = nullptr;
  StencilLaunch B = L;  // diag in - D_eo t / 2 on the even sites, with L's epilogue
  B.in = L.eo_tmp; B.in_cs = L.eo_tmp_cs;
  B.eo_par = 0;
  B.in2 = L.in; B.in2_cs = L.in_cs;
  B.eo_dg = L.diag;
  B.eo_ch = -0.5;
  B.ev_start = nullptr;
  hipError_t e = launch_typed<VS, LS, true>(A, s);
  if (e != hipSuccess) return e;
  return launch_typed<VS, LS, true>(B, s);
}

}  // namespace

}  // namespace eigcg
