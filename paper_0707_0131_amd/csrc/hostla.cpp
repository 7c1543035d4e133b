// Host FP64 dense linear algebra (see hostla.h).
//
// Methods (textbook, written for this library):
//  * Householder reduction of a Hermitian matrix to real symmetric tridiagonal
//    form, processing columns from the last to the first;
//  * implicit QL iteration with Wilkinson shifts for the tridiagonal
//    eigenvalues (Bowdler, Martin, Reinsch and Wilkinson, 1968);
//  * inverse iteration with partial-pivoting tridiagonal LU for the wanted
//    eigenvectors, with eigenvalue separation and Gram-Schmidt inside clusters
//    (as in Peters and Wilkinson's inverse iteration);
//  * Householder thin QR and a lower Cholesky factorisation.
#include "hostla.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <vector>

namespace eigcg {
namespace hostla {

namespace {

inline double sign_of(double a, double b) { return b >= 0.0 ? std::fabs(a) : -std::fabs(a); }

// Elementary reflector H = I - tau v v^H with v = [x; 1] (last entry implicit)
// such that H^H [x; alpha] = [0; beta], beta real.  x is overwritten by the
// scaled reflector entries.  Returns tau; alpha becomes beta.
cplx make_reflector(int nx, cplx& alpha, cplx* x) {
  double xnorm2 = 0.0;
  for (int i = 0; i < nx; ++i) xnorm2 += std::norm(x[i]);
  double ar = alpha.real(), ai = alpha.imag();
  if (xnorm2 == 0.0 && ai == 0.0) return cplx(0.0, 0.0);
  double beta = -sign_of(std::sqrt(ar * ar + ai * ai + xnorm2), ar);
  cplx tau((beta - ar) / beta, -ai / beta);
  cplx scal = 1.0 / (alpha - beta);
  for (int i = 0; i < nx; ++i) x[i] *= scal;
  alpha = cplx(beta, 0.0);
  return tau;
}

// Tridiagonal reduction: W (n x n, full Hermitian storage, column-major) is
// overwritten; d[n], e[n-1] real; reflector i (for column i+1) lives in
// W(0:i-1, i+1) with implicit unit entry at row i, tau[i].
void tridiagonalize(int n, cplx* W, int ldw, double* d, double* e, cplx* tau) {
  std::vector<cplx> x(n), v(n);
  for (int i = n - 2; i >= 0; --i) {
    cplx* col = W + (size_t)(i + 1) * ldw;  // column i+1
    cplx alpha = col[i];
    cplx t = make_reflector(i, alpha, col);  // x = col[0..i-1]
    e[i] = alpha.real();
    if (t != cplx(0.0, 0.0)) {
      // v = [col[0..i-1], 1]
      for (int r = 0; r < i; ++r) v[r] = col[r];
      v[i] = 1.0;
      // x = tau * A v  (A = W(0:i, 0:i), Hermitian, full storage)
      for (int r = 0; r <= i; ++r) x[r] = 0.0;
      for (int c = 0; c <= i; ++c) {
        const cplx vc = v[c];
        if (vc == cplx(0.0, 0.0)) continue;
        const cplx* wc = W + (size_t)c * ldw;
        for (int r = 0; r <= i; ++r) x[r] += wc[r] * vc;
      }
      for (int r = 0; r <= i; ++r) x[r] *= t;
      // alpha2 = -1/2 tau (x^H v)
      cplx xv = 0.0;
      for (int r = 0; r <= i; ++r) xv += std::conj(x[r]) * v[r];
      cplx a2 = -0.5 * t * xv;
      for (int r = 0; r <= i; ++r) x[r] += a2 * v[r];
      // W -= v x^H + x v^H
      for (int c = 0; c <= i; ++c) {
        cplx* wc = W + (size_t)c * ldw;
        const cplx xc = std::conj(x[c]), vc = std::conj(v[c]);
        for (int r = 0; r <= i; ++r) wc[r] -= v[r] * xc + x[r] * vc;
      }
    }
    tau[i] = t;
    d[i + 1] = W[(size_t)(i + 1) * ldw + (i + 1)].real();
  }
  d[0] = W[0].real();
}

// Eigenvalues of the symmetric tridiagonal (d, e) by implicit QL; d is
// overwritten with the unsorted eigenvalues.  e has n entries (e[n-1] scratch).
int tridiag_ql_values(int n, double* d, double* e) {
  if (n <= 1) return 0;
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    int mm;
    do {
      for (mm = l; mm < n - 1; ++mm) {
        double dd = std::fabs(d[mm]) + std::fabs(d[mm + 1]);
        if (std::fabs(e[mm]) <= DBL_EPSILON * dd) break;
      }
      if (mm != l) {
        if (iter++ == 80) return -1;
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = std::hypot(g, 1.0);
        g = d[mm] - d[l] + e[l] / (g + sign_of(r, g));
        double s = 1.0, c = 1.0, p = 0.0;
        int i;
        bool early = false;
        for (i = mm - 1; i >= l; --i) {
          double f = s * e[i];
          double b = c * e[i];
          r = std::hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] -= p;
            e[mm] = 0.0;
            early = true;
            break;
          }
          s = f / r;
          c = g / r;
          g = d[i + 1] - p;
          r = (d[i] - g) * s + 2.0 * c * b;
          p = s * r;
          d[i + 1] = g + p;
          g = c * r - b;
        }
        if (early) continue;
        d[l] -= p;
        e[l] = g;
        e[mm] = 0.0;
      }
    } while (mm != l);
  }
  return 0;
}

// One inverse-iteration solve (T - lambda I) y = b for symmetric tridiagonal
// (d, e) by Gaussian elimination with partial pivoting.  b is overwritten.
void tridiag_shift_solve(int n, const double* d, const double* e, double lambda, double tiny,
                         double* b, std::vector<double>& u0, std::vector<double>& u1,
                         std::vector<double>& u2, std::vector<double>& lmul,
                         std::vector<char>& piv) {
  // Row i of T - lambda I: sub e[i-1], diag d[i]-lambda, super e[i].
  // Factorisation rows: U has diagonal u0, first super u1, second super u2.
  double a = d[0] - lambda;       // current pivot-row diagonal
  double bsup = n > 1 ? e[0] : 0; // current pivot-row superdiagonal
  for (int i = 0; i < n - 1; ++i) {
    double c = e[i];                  // sub-diagonal entry of row i+1
    double anext = d[i + 1] - lambda; // diagonal of row i+1
    double bnext = (i + 1 < n - 1) ? e[i + 1] : 0.0;
    if (std::fabs(a) >= std::fabs(c)) {
      piv[i] = 0;
      double l = (a == 0.0) ? 0.0 : c / a;
      if (a == 0.0) a = tiny;
      lmul[i] = l;
      u0[i] = a;
      u1[i] = bsup;
      u2[i] = 0.0;
      a = anext - l * bsup;
      bsup = bnext;
    } else {
      piv[i] = 1;
      double l = a / c;
      lmul[i] = l;
      u0[i] = c;
      u1[i] = anext;
      u2[i] = bnext;
      a = bsup - l * anext;
      bsup = -l * bnext;
    }
  }
  if (a == 0.0) a = tiny;
  u0[n - 1] = a;
  // forward: apply row swaps and multipliers to b
  for (int i = 0; i < n - 1; ++i) {
    if (piv[i]) std::swap(b[i], b[i + 1]);
    b[i + 1] -= lmul[i] * b[i];
  }
  // back substitution
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    if (i + 1 < n) s -= u1[i] * b[i + 1];
    if (i + 2 < n) s -= u2[i] * b[i + 2];
    double p = u0[i];
    if (std::fabs(p) < tiny) p = (p >= 0 ? tiny : -tiny);
    b[i] = s / p;
  }
}

}  // namespace

int herm_eig_lowest(int n, const cplx* A, int lda, int k, double* w, cplx* Z, int ldz) {
  if (n <= 0) return 0;
  k = std::min(k, n);
  std::vector<cplx> W((size_t)n * n);
  // full Hermitian copy from the upper triangle
  for (int c = 0; c < n; ++c) {
    for (int r = 0; r <= c; ++r) {
      cplx v = A[(size_t)c * lda + r];
      W[(size_t)c * n + r] = v;
      W[(size_t)r * n + c] = std::conj(v);
    }
    W[(size_t)c * n + c] = cplx(A[(size_t)c * lda + c].real(), 0.0);
  }
  std::vector<double> d(n), e(n, 0.0);
  std::vector<cplx> tau(n > 1 ? n - 1 : 1);
  tridiagonalize(n, W.data(), n, d.data(), e.data(), tau.data());
  std::vector<double> dv(d), ev(e);
  if (tridiag_ql_values(n, dv.data(), ev.data()) != 0) return -1;
  std::sort(dv.begin(), dv.end());
  for (int i = 0; i < n; ++i) w[i] = dv[i];
  if (k == 0 || Z == nullptr) return 0;

  double tnorm = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = std::fabs(d[i]);
    if (i > 0) s += std::fabs(e[i - 1]);
    if (i < n - 1) s += std::fabs(e[i]);
    tnorm = std::max(tnorm, s);
  }
  if (tnorm == 0.0) tnorm = 1.0;
  const double tiny = DBL_EPSILON * tnorm;
  const double sep = 10.0 * DBL_EPSILON * tnorm;
  const double ortol = 1e-3 * tnorm;

  std::vector<double> Y((size_t)n * k);
  std::vector<double> u0(n), u1(n), u2(n), lm(n), b(n);
  std::vector<char> piv(n);
  uint64_t seed = 0x9E3779B97F4A7C15ull;
  int cluster_start = 0;
  double lam_prev = 0.0;
  for (int j = 0; j < k; ++j) {
    double lam = w[j];
    if (j > 0) {
      if (lam - lam_prev < sep) lam = lam_prev + sep;  // separate close eigenvalues
      if (w[j] - w[j - 1] > ortol) cluster_start = j;
    }
    lam_prev = lam;
    for (int i = 0; i < n; ++i) {
      seed = seed * 6364136223846793005ull + 1442695040888963407ull;
      b[i] = ((double)(seed >> 11) * (1.0 / 9007199254740992.0)) - 0.5;
    }
    for (int it = 0; it < 4; ++it) {
      tridiag_shift_solve(n, d.data(), e.data(), lam, tiny, b.data(), u0, u1, u2, lm, piv);
      // Gram-Schmidt against earlier vectors of the same cluster (twice)
      for (int pass = 0; pass < 2; ++pass) {
        for (int q = cluster_start; q < j; ++q) {
          const double* yq = Y.data() + (size_t)q * n;
          double dot = 0.0;
          for (int i = 0; i < n; ++i) dot += yq[i] * b[i];
          for (int i = 0; i < n; ++i) b[i] -= dot * yq[i];
        }
      }
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += b[i] * b[i];
      nrm = std::sqrt(nrm);
      if (nrm == 0.0) {
        b[j % n] = 1.0;
        nrm = 1.0;
      }
      for (int i = 0; i < n; ++i) b[i] /= nrm;
    }
    // fix the sign convention: largest-magnitude entry positive
    int imax = 0;
    for (int i = 1; i < n; ++i)
      if (std::fabs(b[i]) > std::fabs(b[imax])) imax = i;
    double sg = b[imax] < 0 ? -1.0 : 1.0;
    double* yj = Y.data() + (size_t)j * n;
    for (int i = 0; i < n; ++i) yj[i] = sg * b[i];
  }
  // back-transform z = H(n-2) ... H(0) y  (apply H(0) first)
  for (int j = 0; j < k; ++j) {
    cplx* z = Z + (size_t)j * ldz;
    const double* yj = Y.data() + (size_t)j * n;
    for (int i = 0; i < n; ++i) z[i] = yj[i];
    for (int i = 0; i <= n - 2; ++i) {
      const cplx t = tau[i];
      if (t == cplx(0.0, 0.0)) continue;
      const cplx* v = W.data() + (size_t)(i + 1) * n;  // v[0..i-1], v[i] = 1
      cplx s = z[i];
      for (int r = 0; r < i; ++r) s += std::conj(v[r]) * z[r];
      s *= t;
      for (int r = 0; r < i; ++r) z[r] -= v[r] * s;
      z[i] -= s;
    }
  }
  return 0;
}

void qr_thin(int m, int n, const cplx* A, int lda, cplx* Q, int ldq, cplx* R, int ldr) {
  std::vector<cplx> W((size_t)m * n);
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < m; ++r) W[(size_t)c * m + r] = A[(size_t)c * lda + r];
  std::vector<cplx> tau(n);
  std::vector<cplx> v(m);
  for (int j = 0; j < n; ++j) {
    cplx* col = W.data() + (size_t)j * m;
    // reflector on col[j..m-1] with the pivot first: reorder so that the
    // "last" entry of make_reflector is col[j]
    int nx = m - j - 1;
    cplx alpha = col[j];
    std::vector<cplx> x(col + j + 1, col + m);
    cplx t = make_reflector(nx, alpha, x.data());
    for (int r = 0; r < nx; ++r) col[j + 1 + r] = x[r];
    col[j] = alpha;
    tau[j] = t;
    // apply H^H = I - conj(tau) v v^H to W(j:m, j+1:n), v = [1; x]
    if (t != cplx(0.0, 0.0)) {
      for (int c = j + 1; c < n; ++c) {
        cplx* wc = W.data() + (size_t)c * m;
        cplx s = wc[j];
        for (int r = 0; r < nx; ++r) s += std::conj(col[j + 1 + r]) * wc[j + 1 + r];
        s *= std::conj(t);
        wc[j] -= s;
        for (int r = 0; r < nx; ++r) wc[j + 1 + r] -= col[j + 1 + r] * s;
      }
    }
  }
  if (R) {
    for (int c = 0; c < n; ++c)
      for (int r = 0; r < n; ++r)
        R[(size_t)c * ldr + r] = (r <= c) ? W[(size_t)c * m + r] : cplx(0.0, 0.0);
  }
  // Q = H(0) H(1) ... H(n-1) [I_n; 0]
  for (int c = 0; c < n; ++c) {
    cplx* q = Q + (size_t)c * ldq;
    for (int r = 0; r < m; ++r) q[r] = (r == c) ? 1.0 : 0.0;
    for (int j = n - 1; j >= 0; --j) {
      const cplx t = tau[j];
      if (t == cplx(0.0, 0.0)) continue;
      const cplx* col = W.data() + (size_t)j * m;
      int nx = m - j - 1;
      cplx s = q[j];
      for (int r = 0; r < nx; ++r) s += std::conj(col[j + 1 + r]) * q[j + 1 + r];
      s *= t;
      q[j] -= s;
      for (int r = 0; r < nx; ++r) q[j + 1 + r] -= col[j + 1 + r] * s;
    }
  }
}

int cholesky(int n, cplx* A, int lda) {
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * lda + j].real();
    for (int k = 0; k < j; ++k) s -= std::norm(A[(size_t)k * lda + j]);
    if (!(s > 0.0)) return j + 1;
    double ljj = std::sqrt(s);
    A[(size_t)j * lda + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      cplx t = A[(size_t)j * lda + i];
      for (int k = 0; k < j; ++k) t -= A[(size_t)k * lda + i] * std::conj(A[(size_t)k * lda + j]);
      A[(size_t)j * lda + i] = t / ljj;
    }
  }
  return 0;
}

void cholesky_solve(int n, const cplx* L, int ldl, int nrhs, cplx* B, int ldb) {
  for (int c = 0; c < nrhs; ++c) {
    cplx* b = B + (size_t)c * ldb;
    for (int i = 0; i < n; ++i) {  // L y = b
      cplx s = b[i];
      for (int k = 0; k < i; ++k) s -= L[(size_t)k * ldl + i] * b[k];
      b[i] = s / L[(size_t)i * ldl + i].real();
    }
    for (int i = n - 1; i >= 0; --i) {  // L^H x = y
      cplx s = b[i];
      for (int k = i + 1; k < n; ++k) s -= std::conj(L[(size_t)i * ldl + k]) * b[k];
      b[i] = s / L[(size_t)i * ldl + i].real();
    }
  }
}

void matmul_sparse_a(int m, int n, int k, const cplx* A, int lda, const cplx* B, int ldb,
                     cplx* C, int ldc) {
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < m; ++r) C[(size_t)c * ldc + r] = 0.0;
  for (int p = 0; p < k; ++p) {
    const cplx* ap = A + (size_t)p * lda;
    for (int r = 0; r < m; ++r) {
      const cplx a = ap[r];
      if (a == cplx(0.0, 0.0)) continue;
      for (int c = 0; c < n; ++c) C[(size_t)c * ldc + r] += a * B[(size_t)c * ldb + p];
    }
  }
}

void matmul_ah_b(int m, int n, int k, const cplx* A, int lda, const cplx* B, int ldb, cplx* C,
                 int ldc) {
  for (int c = 0; c < n; ++c) {
    const cplx* bc = B + (size_t)c * ldb;
    for (int r = 0; r < m; ++r) {
      const cplx* ar = A + (size_t)r * lda;
      cplx s = 0.0;
      for (int p = 0; p < k; ++p) s += std::conj(ar[p]) * bc[p];
      C[(size_t)c * ldc + r] = s;
    }
  }
}

}  // namespace hostla
}  // namespace eigcg
