// Complex tall-skinny products on the gfx950 matrix cores (MFMA 16x16x4).
//
//  * launch_gemm_tall:   Out(n x N) (+)= In(n x K) S(K x N)
//      eigCG restart V <- V (QZ) (Figure 3.1), Ritz vectors V Y,
//      the init-CG lift X += U C (eq. (2.1)) and the Gram-Schmidt update
//      Vbar -= U (U^H Vbar) of the Incremental eigCG bank (Section 4).
//  * launch_gemm_reduce: G(K x N) = In(n x K)^H R(n x N)
//      U^H R of init-CG, U^H Vbar / U^H W / Vbar^H W of the bank update and
//      the arrow row w^H V of the restart.
//
// Complex arithmetic is embedded in real MFMA tiles.  For the tall product the
// real K index interleaves (Re, Im) of each input column and the real output
// columns interleave (Re, Im) of each output column, so the 2x2 real block of
// S = a + ib is [[a, b], [-b, a]]; lanes 2q and 2q+1 of an accumulator tile
// then hold Re and Im of the same output element.  For the reduction the
// conjugate-transpose puts In on the M side: the real block is
// [[Re R, Im R], [Im R, -Re R]].
//
// MFMA lane layout of the 16x16x4 single-block instructions: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register r of lane l
// holds D[4 (l / 16) + r][l % 16] for FP32 and D[l / 16 + 4 r][l % 16] for
// FP64 (measured by the lane-layout probe, which a unit test runs).
#include "kernels.h"

namespace eigcg {

namespace {

constexpr int kMaxK = 256;
constexpr int kMaxN = 24;

struct TallArgs {
  const void* in[kMaxK];
  void* out[kMaxN];
};

template <typename R> struct Mfma;
template <> struct Mfma<double> {
  using acc_t = __attribute__((__vector_size__(4 * sizeof(double)))) double;
  __device__ static __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of accumulator register r in lane group g = lane / 16
  __device__ static __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <> struct Mfma<float> {
  using acc_t = __attribute__((__vector_size__(4 * sizeof(float)))) float;
  __device__ static __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

// The column pointers are staged in LDS, which loses their address space:
// loads and stores through a generic pointer become flat instructions, whose
// completion every LDS wait must also wait for, so the products read and write
// device memory through global pointers.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> as_global(T* p) { return (gptr<T>)p; }
template <typename R> struct Vec2;
template <> struct Vec2<double> { using t = nt_d2; };
template <> struct Vec2<float> { using t = nt_f2; };
template <typename VS>
__device__ __forceinline__ cpx<typename Storage<VS>::real> ldg(const VS* p, size_t i) {
  using V = typename Vec2<typename Storage<VS>::real>::t;
  const V v = as_global(reinterpret_cast<const V*>(p))[i];
  return {v.x, v.y};
}

// Out rows [row0, row0 + 64) per wave; 4 waves per workgroup.
template <typename VS, int NT>
__global__ __launch_bounds__(256) void k_gemm_tall(size_t n, int K, int N, const double2* S,
                                                   int beta_one, int negate, TallArgs cols) {
  using R = typename Storage<VS>::real;
  using M = Mfma<R>;
  extern __shared__ double2 sS[];  // K x N complex, column-major (ld K)
  __shared__ const VS* sin[kMaxK];
  __shared__ R* sout[kMaxN];
  for (int i = threadIdx.x; i < K * N; i += blockDim.x) {
    double2 v = S[i];
    sS[i] = negate ? make_double2(-v.x, -v.y) : v;
  }
  for (int i = threadIdx.x; i < K; i += blockDim.x) sin[i] = reinterpret_cast<const VS*>(cols.in[i]);
  for (int i = threadIdx.x; i < N; i += blockDim.x) sout[i] = reinterpret_cast<R*>(cols.out[i]);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const size_t row0 = ((size_t)blockIdx.x * 4 + wave) * 64;
  if (row0 >= n) return;
  const int li = lane & 15;   // A row within a 16-row subtile / B column within a tile
  const int lk = lane >> 4;   // real k within the 4-step
  const int kpart = lk & 1;   // 0: Re, 1: Im of the input entry
  const int kcol = lk >> 1;   // which of the two complex input columns of the step

  typename M::acc_t acc[4][NT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = typename M::acc_t{};

  // A fragments of input columns k0 + kcol: one real part per lane (lanes of
  // the two parts of a complex entry read adjacent words).  Lanes past column
  // K - 1 read that column and lanes past row n - 1 read that row: the B
  // entries of a column past K - 1 are zero and an output row past n - 1 is
  // not stored, so the loop body is free of branches and the loaded values
  // are first used by the products.
  const R* const* sinr = reinterpret_cast<const R* const*>(sin);
  const bool full = row0 + 64 <= n;  // wave-uniform
  auto load_a = [&](int k0, R* af) {
    const int kc = k0 + kcol;
    const gptr<const R> src = as_global(sinr[kc < K ? kc : K - 1]);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      size_t row = row0 + m * 16 + li;
      if (!full && row >= n) row = n - 1;
      af[m] = src[2 * row + kpart];
    }
  };
  auto step = [&](int k0, const R* af) {
    const int kc = k0 + kcol;
    const bool kvalid = kc < K;
    // B fragments: real column jj = 16 t + li -> output column j = 8 t + li/2, part li&1
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      // lanes past column N - 1 or K - 1 read an entry in range and take zero
      const int j = 8 * t + (li >> 1);
      const double2 s = sS[(size_t)(j < N ? j : N - 1) * K + (kvalid ? kc : K - 1)];
      // [[a, b], [-b, a]] with rows (Re-in, Im-in), cols (Re-out, Im-out)
      R bv = kpart == 0 ? ((li & 1) ? (R)s.y : (R)s.x) : ((li & 1) ? (R)s.x : (R)(-s.y));
      bv = (kvalid && j < N) ? bv : R(0);
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m][t] = M::op(af[m], bv, acc[m][t]);
    }
  };
  // software pipeline: the A fragments of the next kPre steps are in flight
  // while the current step's products run.  The steps run in groups of kPre;
  // steps of the last group past column K - 1 multiply by zero B entries.
  constexpr int kPre = 4;
  R af[kPre][4];
#pragma unroll
  for (int q = 0; q < kPre; ++q) load_a(2 * q, af[q]);
  for (int k0 = 0; k0 < K; k0 += 2 * kPre) {
#pragma unroll
    for (int q = 0; q < kPre; ++q) {
      const int kq = k0 + 2 * q;
      step(kq, af[q]);
      // the step's registers take the fragments kPre steps ahead (a copy of
      // them would make every iteration wait for its own loads); the barrier
      // keeps the scheduler from sinking the loads towards their use
      load_a(kq + 2 * kPre, af[q]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // epilogue: register r of the lane holds D[M::row(lane/16, r)][li] of each
  // tile.  With beta = 1 a tile's old output values are all loaded before its
  // first store.  Lanes past column N - 1 (and, in the last wave, past row
  // n - 1) address column N - 1 (row n - 1) and store nothing.
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = 8 * t + (li >> 1);
    const bool jv = j < N;
    const gptr<R> dst = as_global(sout[jv ? j : N - 1]) + (li & 1);
    if (beta_one) {
      R old[4][4];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          size_t row = row0 + m * 16 + M::row(lk, r);
          if (!full && row >= n) row = n - 1;
          old[m][r] = dst[2 * row];
        }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][t][r] += old[m][r];
    }
    if (!jv) continue;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t row = row0 + m * 16 + M::row(lk, r);
        if (full || row < n) dst[2 * row] = acc[m][t][r];
      }
  }
}

// Reduction product partials: wave handles (row chunk, 16 input columns).
// The workgroup stages tiles of TR rows through LDS with coalesced loads
// (each input column's rows are contiguous; one wave load reads TR rows of
// 64 / TR columns, or 64 rows of one) and shares the R tile between its four waves; the products
// then run over the tile's rows in pairs, in the same order as a direct
// row-pair sweep of the chunk (so TR does not change any result).  Dynamic
// LDS: 4 x 16 columns of input entries, then 16 columns of R, each column
// TR + 1 entries long (the pad spreads the 16 lanes that read one row of 16
// columns over the LDS banks).
template <typename VS, int NT, int TR>
__global__ __launch_bounds__(256) void k_gemm_reduce(size_t n, int K, int N, size_t chunk,
                                                     TallArgs cols, double* partial) {
  using R = typename Storage<VS>::real;
  using M = Mfma<R>;
  constexpr int kLanesPerCol = TR < 64 ? TR : 64;  // lanes loading one column's tile rows
  constexpr int kColsPerLoad = 64 / kLanesPerCol;  // columns one wave load covers
  constexpr int kLoads = 16 / kColsPerLoad * (TR / kLanesPerCol);
  __shared__ const VS* sin[kMaxK];
  __shared__ const VS* sr[kMaxN];
  extern __shared__ double2 lds_dyn[];
  constexpr int CS = TR + 1;                          // column stride in LDS
  cpx<R>* tU = reinterpret_cast<cpx<R>*>(lds_dyn);  // [wave][input column][row]
  cpx<R>* tR = tU + 4 * 16 * CS;                     // [output column][row], N <= 16
  for (int i = threadIdx.x; i < K; i += blockDim.x) sin[i] = reinterpret_cast<const VS*>(cols.in[i]);
  for (int i = threadIdx.x; i < N; i += blockDim.x) sr[i] = reinterpret_cast<const VS*>(cols.out[i]);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int mtile = blockIdx.y * 4 + wave;
  const int mtiles = (K + 15) / 16;
  const bool mact = mtile < mtiles;  // every wave takes part in the loads and barriers
  const int li = lane & 15;
  const int lk = lane >> 4;
  const int kpart = lk & 1;
  const int krow = lk >> 1;
  const int lsub = lane / kLanesPerCol;  // loads: column within a load
  const int lrow = lane % kLanesPerCol;  // loads: row within a load
  const size_t r0 = (size_t)blockIdx.x * chunk;
  size_t r1 = r0 + chunk;
  if (r1 > n) r1 = n;
  cpx<R>* tUw = tU + (size_t)wave * 16 * CS;

  typename M::acc_t acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = typename M::acc_t{};

  // load q covers columns (q % (16 / kColsPerLoad)) * kColsPerLoad + lsub and
  // rows (q / (16 / kColsPerLoad)) * kLanesPerCol + lrow of the tile
  constexpr int kColGroups = 16 / kColsPerLoad;
  // the next tile's entries are loaded into registers while the current
  // tile's products run
  cpx<R> pu[kLoads];
  constexpr int kRLoads = (16 * TR) / 256;  // R tile entries per thread
  cpx<R> pr[kRLoads];
  // each thread's load columns are the same for every tile: their pointers
  // are read from LDS once (null for a column past K - 1 or N - 1)
  const VS* ucol[kLoads];
  const VS* rcol[kRLoads];
#pragma unroll
  for (int q = 0; q < kLoads; ++q) {
    const int col = mtile * 16 + (q % kColGroups) * kColsPerLoad + lsub;
    ucol[q] = (mact && col < K) ? sin[col] : nullptr;
  }
#pragma unroll
  for (int q = 0; q < kRLoads; ++q) {
    const int j = (q * 256 + (int)threadIdx.x) / TR;
    rcol[q] = j < N ? sr[j] : nullptr;
  }
  auto fetch = [&](size_t rb) {
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      const size_t row = rb + (size_t)(q / kColGroups) * kLanesPerCol + lrow;
      pu[q] = {R(0), R(0)};
      if (ucol[q] && row < r1) pu[q] = ldg(ucol[q], row);
    }
#pragma unroll
    for (int q = 0; q < kRLoads; ++q) {
      const int e = q * 256 + (int)threadIdx.x;  // entry of the 16 x TR tile
      const size_t row = rb + e % TR;
      pr[q] = {R(0), R(0)};
      if (rcol[q] && row < r1) pr[q] = ldg(rcol[q], row);
    }
  };
  if (r0 < r1) fetch(r0);
  for (size_t rb = r0; rb < r1; rb += TR) {
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      const int c = (q % kColGroups) * kColsPerLoad + lsub;
      const int tr = (q / kColGroups) * kLanesPerCol + lrow;
      tUw[c * CS + tr] = pu[q];
    }
#pragma unroll
    for (int q = 0; q < kRLoads; ++q) {
      const int e = q * 256 + (int)threadIdx.x;  // entry e = j * TR + row
      tR[(e / TR) * CS + e % TR] = pr[q];
    }
    __syncthreads();
    if (rb + TR < r1) fetch(rb + TR);
    if (mact) {
      // every row pair of the tile: rows beyond the chunk are zero in both
      // staged tiles, so their products add nothing, and the fixed trip count
      // lets the LDS reads of several pairs be in flight together
#pragma unroll 4
      for (int s = 0; s < TR; s += 2) {
        const int tr = s + krow;
        const cpx<R> z = tUw[li * CS + tr];
        const R a = kpart ? z.im : z.re;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int j = 8 * t + (li >> 1);  // < 16: inside the staged R tile
          const cpx<R> y = tR[j * CS + tr];
          // [[Re R, Im R], [Im R, -Re R]] with rows (Re-in, Im-in), cols (Re-out, Im-out)
          R bv = kpart == 0 ? ((li & 1) ? y.im : y.re) : ((li & 1) ? -y.re : y.im);
          bv = j < N ? bv : R(0);
          acc[t] = M::op(a, bv, acc[t]);
        }
      }
    }
    __syncthreads();
  }
  if (!mact) return;
  // partial layout: [chunk][i in 0..K)][jj in 0..2N) doubles
  double* dst = partial + (size_t)blockIdx.x * K * 2 * N;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int jj = 16 * t + li;
    if (jj >= 2 * N) continue;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int i = mtile * 16 + M::row(lk, rr);
      if (i < K) dst[(size_t)i * 2 * N + jj] = (double)acc[t][rr];
    }
  }
}

// One workgroup per output G[i, j]: thread t sums chunks t, t + 256, ... in
// order, then the workgroup combines the 256 sums in a fixed order, so the
// result depends only on the chunking (which does not depend on N).
__global__ __launch_bounds__(256) void k_gemm_reduce_final(int K, int N, int nchunk,
                                                           const double* partial, double2* G) {
  __shared__ double lds[2][4];
  const int idx = blockIdx.x;  // over K*N complex outputs
  const int i = idx % K, j = idx / K;
  const size_t stride = (size_t)K * 2 * N;
  double re = 0.0, im = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 256) {
    const double* p = partial + (size_t)c * stride + (size_t)i * 2 * N + 2 * j;
    re += p[0];
    im += p[1];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off, 64);
    im += __shfl_xor(im, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    lds[0][w] = re;
    lds[1][w] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    G[(size_t)j * K + i] = make_double2(lds[0][0] + lds[0][1] + lds[0][2] + lds[0][3],
                                        lds[1][0] + lds[1][1] + lds[1][2] + lds[1][3]);
}

template <typename VS>
hipError_t tall_typed(size_t n, int K, int N, const void* const* in_cols, void* const* out_cols,
                      const double2* S, int beta_one, int negate, hipStream_t s) {
  TallArgs a;
  for (int i = 0; i < K; ++i) a.in[i] = in_cols[i];
  for (int j = 0; j < N; ++j) a.out[j] = out_cols[j];
  const int nt = (N + 7) / 8;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  size_t lds = (size_t)K * N * sizeof(double2);
  if (nt == 1)
    hipLaunchKernelGGL((k_gemm_tall<VS, 1>), grid, block, lds, s, n, K, N, S, beta_one, negate, a);
  else if (nt == 2)
    hipLaunchKernelGGL((k_gemm_tall<VS, 2>), grid, block, lds, s, n, K, N, S, beta_one, negate, a);
  else
    hipLaunchKernelGGL((k_gemm_tall<VS, 3>), grid, block, lds, s, n, K, N, S, beta_one, negate, a);
  return hipGetLastError();
}

template <typename VS>
hipError_t reduce_typed(size_t n, int K, int N, const void* const* in_cols,
                        const void* const* r_cols, double2* partial, size_t partial_elems,
                        double2* G, hipStream_t s) {
  TallArgs a;
  for (int i = 0; i < K; ++i) a.in[i] = in_cols[i];
  for (int j = 0; j < N; ++j) a.out[j] = const_cast<void*>(r_cols[j]);
  // chunk so that the partial buffer (nchunk * K * 2N doubles) fits for the
  // widest N, so the chunking (and every column's summation order) does not
  // depend on how many columns are reduced together
  if (N > kMaxN) return hipErrorInvalidValue;
  size_t per_chunk = (size_t)K * kMaxN;  // double2 elements per chunk
  size_t max_chunks = partial_elems / per_chunk;
  if (max_chunks == 0) return hipErrorInvalidValue;
  size_t want = 1024;
  if (want > max_chunks) want = max_chunks;
  size_t chunk = (n + want - 1) / want;
  if (chunk < 256) chunk = 256;
  chunk = (chunk + 1) & ~(size_t)1;
  const int nchunk = (int)((n + chunk - 1) / chunk);
  const int nt = (N + 7) / 8;
  dim3 grid(nchunk, ((K + 15) / 16 + 3) / 4), block(256);
  double* part = reinterpret_cast<double*>(partial);
  // 32-row tiles: 512 B (FP64) or 256 B (FP32) contiguous per column, 42 KB /
  // 21 KB of LDS, so three / seven workgroups share a CU
  constexpr int kTR = 32;
  const size_t lds = (4 * 16 + 16) * (kTR + 1) * sizeof(cpx<typename Storage<VS>::real>);
  if (nt == 1)
    hipLaunchKernelGGL((k_gemm_reduce<VS, 1, kTR>), grid, block, lds, s, n, K, N, chunk, a, part);
  else
    hipLaunchKernelGGL((k_gemm_reduce<VS, 2, kTR>), grid, block, lds, s, n, K, N, chunk, a, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int outs = K * N;
  hipLaunchKernelGGL(k_gemm_reduce_final, dim3(outs), dim3(256), 0, s, K, N, nchunk, part, G);
  return hipGetLastError();
}

// Lane-layout probe of the 16x16x4 MFMA instructions: two products whose
// results encode the row index (A[i][0] = i + 1, B[0][j] = 1) and the column
// index (A[i][0] = 1, B[0][j] = j + 1) of every accumulator entry.
// out: 64 lanes x 4 registers x 2 (row, column) for FP64, then the same for FP32.
__global__ void k_mfma_probe(double* out) {
  const int l = threadIdx.x;
  const int i = l & 15, k = l >> 4;
  using A64 = Mfma<double>;
  using A32 = Mfma<float>;
  typename A64::acc_t r64 = A64::op(k == 0 ? double(i + 1) : 0.0, k == 0 ? 1.0 : 0.0,
                                    typename A64::acc_t{});
  typename A64::acc_t c64 = A64::op(k == 0 ? 1.0 : 0.0, k == 0 ? double(i + 1) : 0.0,
                                    typename A64::acc_t{});
  typename A32::acc_t r32 = A32::op(k == 0 ? float(i + 1) : 0.f, k == 0 ? 1.f : 0.f,
                                    typename A32::acc_t{});
  typename A32::acc_t c32 = A32::op(k == 0 ? 1.f : 0.f, k == 0 ? float(i + 1) : 0.f,
                                    typename A32::acc_t{});
  for (int r = 0; r < 4; ++r) {
    out[(l * 4 + r) * 2 + 0] = r64[r];
    out[(l * 4 + r) * 2 + 1] = c64[r];
    out[512 + (l * 4 + r) * 2 + 0] = (double)r32[r];
    out[512 + (l * 4 + r) * 2 + 1] = (double)c32[r];
  }
}

}  // namespace

hipError_t launch_mfma_probe(double* out_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, s, out_dev);
  return hipGetLastError();
}

hipError_t launch_gemm_tall(int prec, size_t n, int K, int N, const void* const* in_cols,
                            void* const* out_cols, const double2* S, int beta_one, int negate,
                            hipStream_t s) {
  if (K <= 0 || N <= 0 || K > kMaxK || N > kMaxN || (size_t)K * N * 16 > 65536)
    return hipErrorInvalidValue;
  if (prec == kF64)
    return tall_typed<double2>(n, K, N, in_cols, out_cols, S, beta_one, negate, s);
  return tall_typed<float2>(n, K, N, in_cols, out_cols, S, beta_one, negate, s);
}

hipError_t launch_gemm_reduce(int prec, size_t n, int K, int N, const void* const* in_cols,
                              const void* const* r_cols, double2* partial, size_t partial_elems,
                              double2* G, hipStream_t s) {
  if (K <= 0 || N <= 0 || K > kMaxK || N > 16) return hipErrorInvalidValue;
  if (prec == kF64)
    return reduce_typed<double2>(n, K, N, in_cols, r_cols, partial, partial_elems, G, s);
  return reduce_typed<float2>(n, K, N, in_cols, r_cols, partial, partial_elems, G, s);
}

}  // namespace eigcg
