// Vector kernels of the BiCGSTAB solver on FP64 fields of n complex entries
// (SoA planes, so entry e of every field is the same site and component).
//
// Inner products are deterministic: each workgroup reduces its grid-stride
// share in a fixed tree and writes one partial per product; a one-workgroup
// kernel sums the partials in a fixed order.  The update kernels fuse the
// recurrences of one iteration so that each field is read once per pass.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace eigcg {
namespace {

struct DotPtrs {
  const double2* a[kBicgMaxDots];
  const double2* b[kBicgMaxDots];
};

__device__ inline double2 conj_mul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

int blocks_for(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  return (int)(b < (size_t)kBicgDotBlocks ? b : (size_t)kBicgDotBlocks);
}

// fixed-order tree over the workgroup, one partial per product
template <int NP>
__device__ void write_partials(double2 (&acc)[NP], double2* partial) {
  __shared__ double2 red[NP][kBlock];
#pragma unroll
  for (int i = 0; i < NP; ++i) red[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int i = 0; i < NP; ++i) red[i][threadIdx.x] = add(red[i][threadIdx.x], red[i][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NP; ++i) partial[(size_t)blockIdx.x * NP + i] = red[i][0];
  }
}

template <int NP>
__global__ __launch_bounds__(kBlock) void k_dots(size_t n, DotPtrs d, double2* partial) {
  double2 acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = make_double2(0.0, 0.0);
  for (size_t e = blockIdx.x * (size_t)kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = add(acc[i], conj_mul(d.a[i][e], d.b[i][e]));
  }
  write_partials<NP>(acc, partial);
}

__global__ __launch_bounds__(kBlock) void k_dots_final(int np, int nblk, const double2* partial,
                                                       double2* out) {
  __shared__ double2 red[kBlock];
  for (int i = 0; i < np; ++i) {
    double2 s = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < nblk; b += kBlock) s = add(s, partial[(size_t)b * np + i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] = add(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
    __syncthreads();
  }
}

// Complex quotient a / b by Smith's method (scaled by the larger component of
// b, so that |b|^2 is never formed).
__device__ inline double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.x * r + b.y;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ inline bool cfinite(double2 z) { return isfinite(z.x) && isfinite(z.y); }
__device__ inline bool czero(double2 z) { return z.x == 0.0 && z.y == 0.0; }

// the fixed-order sum of k_dots_final for np products, into out (thread 0 has it)
__device__ void sum_partials(int np, int nblk, const double2* partial, double2* out) {
  __shared__ double2 red[kBlock];
  for (int i = 0; i < np; ++i) {
    double2 s = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < nblk; b += kBlock) s = add(s, partial[(size_t)b * np + i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] = add(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_bicg_p_dev(size_t n, double2* __restrict__ p,
                                                       const double2* __restrict__ r,
                                                       const double2* __restrict__ v,
                                                       const BicgState* st) {
  if (st->state != kBicgRun) return;
  const double2 beta = st->beta, omega = st->omega;
  for (size_t e = blockIdx.x * (size_t)kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock)
    p[e] = add(r[e], mul(beta, sub(p[e], mul(omega, v[e]))));
}

template <int NP>
__global__ __launch_bounds__(kBlock) void k_dots_dev(size_t n, DotPtrs d, double2* partial,
                                                     const BicgState* st) {
  if (st->state != kBicgRun) return;
  double2 acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = make_double2(0.0, 0.0);
  for (size_t e = blockIdx.x * (size_t)kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = add(acc[i], conj_mul(d.a[i][e], d.b[i][e]));
  }
  write_partials<NP>(acc, partial);
}

__global__ __launch_bounds__(kBlock) void k_bicg_alpha(int nblk, const double2* partial,
                                                       BicgState* st) {
  if (st->state != kBicgRun) return;
  double2 rv[1];
  sum_partials(1, nblk, partial, rv);
  if (threadIdx.x != 0) return;
  if (czero(rv[0]) || !cfinite(rv[0])) {
    st->state = kBicgBreak;
    return;
  }
  st->alpha = cdiv(st->rho, rv[0]);
}

__global__ __launch_bounds__(kBlock) void k_bicg_s_dev(size_t n, double2* __restrict__ s,
                                                       const double2* __restrict__ r,
                                                       const double2* __restrict__ v,
                                                       const BicgState* st) {
  if (st->state != kBicgRun) return;
  const double2 alpha = st->alpha;
  for (size_t e = blockIdx.x * (size_t)kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock)
    s[e] = sub(r[e], mul(alpha, v[e]));
}

__global__ __launch_bounds__(kBlock) void k_bicg_omega(int nblk, const double2* partial,
                                                       BicgState* st) {
  if (st->state != kBicgRun) return;
  double2 g[3];  // t^H s, s^H s, t^H t
  sum_partials(3, nblk, partial, g);
  if (threadIdx.x != 0) return;
  st->it += 1;
  if (g[1].x <= st->stop2) {  // ||s|| <= tol ||b||: half step
    st->half = 1;
    return;
  }
  if (czero(g[2]) || !cfinite(g[2]) || !cfinite(g[0])) {
    st->state = kBicgBreak;
    return;
  }
  st->omega = cdiv(g[0], g[2]);
}

// x += alpha p + omega s; r = s - omega t; partials of rh^H r and r^H r.  The
// half step instead sets x += alpha p and r = s.
__global__ __launch_bounds__(kBlock) void k_bicg_xr_dev(size_t n, double2* __restrict__ x,
                                                        double2* __restrict__ r,
                                                        const double2* __restrict__ p,
                                                        const double2* __restrict__ s,
                                                        const double2* __restrict__ t,
                                                        const double2* __restrict__ rh,
                                                        double2* partial, const BicgState* st) {
  if (st->state != kBicgRun) return;
  const double2 alpha = st->alpha;
  if (st->half) {
    for (size_t e = blockIdx.x * (size_t)kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
      x[e] = add(x[e], mul(alpha, p[e]));
      r[e] = s[e];
    }
    return;
  }
  const double2 omega = st->omega;
  double2 acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  for (size_t e = blockIdx.x * (size_t)kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
    const double2 se = s[e];
    x[e] = add(add(x[e], mul(alpha, p[e])), mul(omega, se));
    const double2 re = sub(se, mul(omega, t[e]));
    r[e] = re;
    acc[0] = add(acc[0], conj_mul(rh[e], re));
    acc[1] = add(acc[1], conj_mul(re, re));
  }
  write_partials<2>(acc, partial);
}

__global__ __launch_bounds__(kBlock) void k_bicg_rho(int nblk, const double2* partial,
                                                     BicgState* st) {
  if (st->state != kBicgRun) return;
  if (st->half) {
    if (threadIdx.x == 0) st->state = kBicgHalf;
    return;
  }
  double2 g[2];  // rh^H r, r^H r
  sum_partials(2, nblk, partial, g);
  if (threadIdx.x != 0) return;
  st->rho_old = st->rho;
  st->rho = g[0];
  if (g[1].x <= st->stop2) {
    st->state = kBicgConv;
    return;
  }
  if (st->it >= st->max_iter) {
    st->state = kBicgMaxIt;
    return;
  }
  // the next iteration's breakdown test and beta
  if (czero(st->rho) || czero(st->omega) || !cfinite(st->rho)) {
    st->state = kBicgBreak;
    return;
  }
  st->beta = mul(cdiv(st->rho, st->rho_old), cdiv(st->alpha, st->omega));
}

}  // namespace

hipError_t launch_bicg_p_dev(size_t n, void* p, const void* r, const void* v,
                             const BicgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_p_dev, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, (double2*)p,
                     (const double2*)r, (const double2*)v, st);
  return hipGetLastError();
}

hipError_t launch_bicg_alpha(size_t n, const void* rh, const void* v, double2* partial,
                             BicgState* st, hipStream_t s) {
  DotPtrs d{};
  d.a[0] = (const double2*)rh;
  d.b[0] = (const double2*)v;
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_dots_dev<1>, dim3(nb), dim3(kBlock), 0, s, n, d, partial, st);
  hipLaunchKernelGGL(k_bicg_alpha, dim3(1), dim3(kBlock), 0, s, nb, partial, st);
  return hipGetLastError();
}

hipError_t launch_bicg_s_dev(size_t n, void* sv, const void* r, const void* v,
                             const BicgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_s_dev, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, (double2*)sv,
                     (const double2*)r, (const double2*)v, st);
  return hipGetLastError();
}

hipError_t launch_bicg_omega(size_t n, const void* t, const void* sv, double2* partial,
                             BicgState* st, hipStream_t s) {
  DotPtrs d{};
  d.a[0] = (const double2*)t;  d.b[0] = (const double2*)sv;
  d.a[1] = (const double2*)sv; d.b[1] = (const double2*)sv;
  d.a[2] = (const double2*)t;  d.b[2] = (const double2*)t;
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_dots_dev<3>, dim3(nb), dim3(kBlock), 0, s, n, d, partial, st);
  hipLaunchKernelGGL(k_bicg_omega, dim3(1), dim3(kBlock), 0, s, nb, partial, st);
  return hipGetLastError();
}

hipError_t launch_bicg_xr_dev(size_t n, void* x, void* r, const void* p, const void* sv,
                              const void* t, const void* rh, double2* partial, BicgState* st,
                              hipStream_t s) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_bicg_xr_dev, dim3(nb), dim3(kBlock), 0, s, n, (double2*)x, (double2*)r,
                     (const double2*)p, (const double2*)sv, (const double2*)t,
                     (const double2*)rh, partial, st);
  hipLaunchKernelGGL(k_bicg_rho, dim3(1), dim3(kBlock), 0, s, nb, partial, st);
  return hipGetLastError();
}

hipError_t launch_bicg_dots(int np, size_t n, const void* const* a, const void* const* b,
                            double2* partial, double2* out, hipStream_t s) {
  if (np < 1 || np > kBicgMaxDots) return hipErrorInvalidValue;
  DotPtrs d{};
  for (int i = 0; i < np; ++i) {
    d.a[i] = (const double2*)a[i];
    d.b[i] = (const double2*)b[i];
  }
  const int nb = blocks_for(n);
  switch (np) {
    case 1: hipLaunchKernelGGL(k_dots<1>, dim3(nb), dim3(kBlock), 0, s, n, d, partial); break;
    case 2: hipLaunchKernelGGL(k_dots<2>, dim3(nb), dim3(kBlock), 0, s, n, d, partial); break;
    case 3: hipLaunchKernelGGL(k_dots<3>, dim3(nb), dim3(kBlock), 0, s, n, d, partial); break;
    default: hipLaunchKernelGGL(k_dots<4>, dim3(nb), dim3(kBlock), 0, s, n, d, partial); break;
  }
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(kBlock), 0, s, np, nb, partial, out);
  return hipGetLastError();
}

}  // namespace eigcg
