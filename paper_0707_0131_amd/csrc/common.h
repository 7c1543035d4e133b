// Shared device/host definitions of the eigCG HIP library (gfx950).
//
// Internal data layout (all vectors and links live in HBM in this form):
//
//  * sites are numbered lexicographically with x fastest, then y, z, t;
//  * a spinor field is 12 complex planes (component c = 3*spin + colour),
//    each plane holding `vs` sites (vs = V rounded up to a multiple of 64,
//    the pad is kept zero), so lane i of a wavefront reads site s0+i of one
//    plane: every load of the stencil and of BLAS1 is a contiguous 64-lane
//    access;
//  * several right-hand sides are separate fields one after the other
//    (column stride 12*vs complex);
//  * links are 4 directions x 9 (full) or 6 (first two rows, third row
//    rebuilt from unitarity) complex planes of vs sites.
//
// Odd-even geometry (Geom::eo = 1): vectors live on one parity of sites
// ((x + y + z + t) even for the solver's fields); site s of parity p has
// half index h = s / 2 (Lx even), V and vs count half sites, and the links
// are two parity blocks of planes (even sites' links first), each link at
// the half index of the site it starts from.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eigcg {

constexpr int kBlock = 256;        // threads per workgroup of the streaming kernels
constexpr int kMaxGrid = 2048;     // cap on workgroups of grid-stride kernels
constexpr int kMaxCols = 16;       // most right-hand sides a kernel handles at once

// Exact unsigned division by a runtime constant: q = (n * mul) >> shift for
// every n < 2^31 (round-up method of Granlund and Montgomery).
struct FastDiv {
  uint64_t mul;
  uint32_t shift;
  uint32_t d;
  FastDiv() : mul(1), shift(0), d(1) {}
  explicit FastDiv(uint32_t div) : d(div) {
    uint32_t l = 0;
    while ((1ull << l) < div) ++l;
    shift = 32 + l;
    mul = ((1ull << shift) / div) + 1;
  }
  __host__ __device__ inline uint32_t div(uint32_t n) const {
    return (uint32_t)(((uint64_t)n * mul) >> shift);
  }
};

struct Geom {
  int L[4];        // Lx, Ly, Lz, Lt
  int V;           // sites of a vector (half of Vfull in the odd-even geometry)
  int vs;          // plane stride (sites, multiple of 64)
  int stride[4];   // lattice site-index step of a unit hop: 1, Lx, Lx*Ly, Lx*Ly*Lz
  FastDiv dx, dy, dz;  // Lx, Ly, Lz
  int eo;          // 1: odd-even geometry (vectors on one parity)
  int Vfull;       // lattice sites
  FastDiv dxh;     // Lx / 2 (odd-even geometry)
};

// Per right-hand-side solver state on the device.  Scalars of the CG
// recurrence are FP64 in every precision mode.
struct ColState {
  double rho;       // r^H r of the current residual
  double rho_prev;
  double alpha;     // alpha of the last completed iteration
  double beta;      // beta for the next search direction
  double pap;       // p^H A p of the current iteration
  double stop2;     // recursive r^H r at or below this: converged
  double restart2;  // recursive r^H r at or below this: stop for a host-driven
                    // restart (init-CG re-deflation, mixed-precision update)
  double res_stop2; // true-residual r^H r at or below this: converged
  double inner_rel2;// iterative refinement: after a true residual rho, the inner
                    // solve stops at restart2 = max(inner_rel2 rho, res_stop2 / 4)
  int iter;         // completed iterations
  int max_iter;
  int state;        // ColRun / ColStopPending / ColStopped
  int reason;       // ReasonNone / Converged / MaxIter / Breakdown / Restart
  int save_t0;      // iterations j whose t_j = A p_j is kept (the eigCG restart's
  int save_t1;      // arrow row needs A r = t_J - beta_J t_{J-1}); slot j & 1; 0 = none
  int tperiod;      // after saving at save_t1 both advance by this (m - 2 nev)
  int pad_;
  double scale;     // 16-bit inner solves: the inner system is A e = scale r
};

enum { ColRun = 0, ColStopPending = 1, ColStopped = 2 };
enum { ReasonNone = 0, ReasonConverged = 1, ReasonMaxIter = 2, ReasonBreakdown = 3,
       ReasonRestart = 4 };

// --- small complex helpers -------------------------------------------------
template <typename R> struct cpx { R re, im; };

template <typename R> __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R> __device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
  // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> __device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename R> __device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename R> __device__ __forceinline__ cpx<R> ci(cpx<R> a) {  // i*a
  return {-a.im, a.re};
}
template <typename R> __device__ __forceinline__ cpx<R> cmi(cpx<R> a) {  // -i*a
  return {a.im, -a.re};
}
template <typename R> __device__ __forceinline__ cpx<R> cneg(cpx<R> a) { return {-a.re, -a.im}; }

// --- storage types -----------------------------------------------------------
template <typename S> struct Storage;
// ld_nt / st_nt: streaming (nontemporal) access for data touched once per
// launch, so that it does not displace reused stencil data from the L2.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
template <> struct Storage<double2> {
  using real = double;
  __device__ static __forceinline__ cpx<double> ld(const double2* p, size_t i) {
    double2 v = p[i];
    return {v.x, v.y};
  }
  __device__ static __forceinline__ void st(double2* p, size_t i, cpx<double> v) {
    p[i] = make_double2(v.re, v.im);
  }
  __device__ static __forceinline__ cpx<double> ld_nt(const double2* p, size_t i) {
    const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p) + i);
    return {v.x, v.y};
  }
  __device__ static __forceinline__ void st_nt(double2* p, size_t i, cpx<double> v) {
    nt_d2 w;
    w.x = v.re;
    w.y = v.im;
    __builtin_nontemporal_store(w, reinterpret_cast<nt_d2*>(p) + i);
  }
};
// 16-bit storage (IEEE half pairs), FP32 arithmetic
struct __attribute__((aligned(4))) f16x2 {
  _Float16 x, y;
};
template <> struct Storage<f16x2> {
  using real = float;
  __device__ static __forceinline__ cpx<float> ld(const f16x2* p, size_t i) {
    const f16x2 v = p[i];
    return {(float)v.x, (float)v.y};
  }
  __device__ static __forceinline__ void st(f16x2* p, size_t i, cpx<float> v) {
    f16x2 w;
    w.x = (_Float16)v.re;
    w.y = (_Float16)v.im;
    p[i] = w;
  }
  __device__ static __forceinline__ cpx<float> ld_nt(const f16x2* p, size_t i) {
    const unsigned int u = __builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p) + i);
    f16x2 v;
    __builtin_memcpy(&v, &u, 4);
    return {(float)v.x, (float)v.y};
  }
  __device__ static __forceinline__ void st_nt(f16x2* p, size_t i, cpx<float> v) {
    f16x2 w;
    w.x = (_Float16)v.re;
    w.y = (_Float16)v.im;
    unsigned int u;
    __builtin_memcpy(&u, &w, 4);
    __builtin_nontemporal_store(u, reinterpret_cast<unsigned int*>(p) + i);
  }
};
template <> struct Storage<float2> {
  using real = float;
  __device__ static __forceinline__ cpx<float> ld(const float2* p, size_t i) {
    float2 v = p[i];
    return {v.x, v.y};
  }
  __device__ static __forceinline__ void st(float2* p, size_t i, cpx<float> v) {
    p[i] = make_float2(v.re, v.im);
  }
  __device__ static __forceinline__ cpx<float> ld_nt(const float2* p, size_t i) {
    const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p) + i);
    return {v.x, v.y};
  }
  __device__ static __forceinline__ void st_nt(float2* p, size_t i, cpx<float> v) {
    nt_f2 w;
    w.x = v.re;
    w.y = v.im;
    __builtin_nontemporal_store(w, reinterpret_cast<nt_f2*>(p) + i);
  }
};

// --- deterministic reductions --------------------------------------------------
// Sum over a 256-thread workgroup in a fixed order (wavefront butterfly, then
// the four wave partials in order).  Every thread gets the total.
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T> __device__ __forceinline__ T block_sum(T v, T* lds4) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds4[w] = v;
  __syncthreads();
  T s = lds4[0];
#pragma unroll
  for (int i = 1; i < kBlock / 64; ++i) s += lds4[i];
  return s;
}

// Fixed-order sum of n partials (written by an earlier kernel of the same
// stream) by one workgroup; every workgroup that calls it gets the same bits.
__device__ __forceinline__ double reduce_partials(const double* part, int n, double* lds4) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += part[i];
  return block_sum(s, lds4);
}

}  // namespace eigcg
