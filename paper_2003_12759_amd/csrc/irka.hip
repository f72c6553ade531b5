// IRKA-style outer loop with computed shifts: Algorithm 2 (BIRKA) without
// its bilinear terms.  Each round solves the shifted pairs at the current
// shifts on the device (morx_solve_shifts, Algorithm 4's chains, the vertical
// link carried from one round to the next), projects (morx_project), and
// takes the next shifts as the mirror images -lambda_i of the eigenvalues of
// the reduced pencil (Ar, Er) (line 3 of Algorithm 2: the eigendecomposition
// of the reduced matrix).  The MIMO form takes from the same
// eigendecomposition the tangential directions of the next round's
// right-hand sides (one per shift, solved by morx_solve_pairs), its
// eigenvectors found by inverse iteration.  The r x r eigenvalue problem runs on the host:
// Er^{-1} Ar by LU with partial pivoting, Householder reduction to upper
// Hessenberg form, then Francis double-shift QR steps with deflation
// (J. G. F. Francis, "The QR transformation", Computer J. 4 (1961-62); the
// step as in Golub and Van Loan, Matrix Computations, Section 7.5).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace {

constexpr double kEps = 2.220446049250313e-16;

// H = Er^{-1} Ar (r x r, column-major inputs, row-major H); false if a pivot
// of Er vanishes relative to its largest entry
bool pencil_to_standard(int r, const double* Ar, const double* Er, std::vector<double>& H) {
  std::vector<double> M((size_t)r * r), R((size_t)r * r);
  double emax = 0.0;
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      M[(size_t)i * r + j] = Er[(size_t)j * r + i];
      R[(size_t)i * r + j] = Ar[(size_t)j * r + i];
      emax = std::max(emax, fabs(M[(size_t)i * r + j]));
    }
  if (!(emax > 0.0)) return false;
  for (int k = 0; k < r; ++k) {
    int p = k;
    for (int i = k + 1; i < r; ++i)
      if (fabs(M[(size_t)i * r + k]) > fabs(M[(size_t)p * r + k])) p = i;
    if (!(fabs(M[(size_t)p * r + k]) > 1e3 * kEps * emax)) return false;
    if (p != k)
      for (int j = 0; j < r; ++j) {
        std::swap(M[(size_t)p * r + j], M[(size_t)k * r + j]);
        std::swap(R[(size_t)p * r + j], R[(size_t)k * r + j]);
      }
    for (int i = k + 1; i < r; ++i) {
      const double f = M[(size_t)i * r + k] / M[(size_t)k * r + k];
      M[(size_t)i * r + k] = 0.0;
      for (int j = k + 1; j < r; ++j) M[(size_t)i * r + j] -= f * M[(size_t)k * r + j];
      for (int j = 0; j < r; ++j) R[(size_t)i * r + j] -= f * R[(size_t)k * r + j];
    }
  }
  // back substitution, one right-hand-side column at a time
  H.assign((size_t)r * r, 0.0);
  for (int j = 0; j < r; ++j)
    for (int i = r - 1; i >= 0; --i) {
      double s = R[(size_t)i * r + j];
      for (int l = i + 1; l < r; ++l) s -= M[(size_t)i * r + l] * H[(size_t)l * r + j];
      H[(size_t)i * r + j] = s / M[(size_t)i * r + i];
    }
  return true;
}

// Householder vector of u (length len <= 3): v with v[0] = u[0] - alpha,
// alpha = -sign(u[0]) |u|; returns beta = 2 / v^T v, or 0 when u = 0
double householder(const double* u, int len, double* v) {
  double nrm = 0.0;
  for (int i = 0; i < len; ++i) nrm += u[i] * u[i];
  nrm = sqrt(nrm);
  if (nrm == 0.0) return 0.0;
  const double alpha = u[0] >= 0.0 ? -nrm : nrm;
  for (int i = 0; i < len; ++i) v[i] = u[i];
  v[0] -= alpha;
  double vv = 0.0;
  for (int i = 0; i < len; ++i) vv += v[i] * v[i];
  return vv > 0.0 ? 2.0 / vv : 0.0;
}

// rows r0..r0+len-1 of H (row-major, n columns) times (I - beta v v^T) from
// the left, on columns c0..c1
void reflect_rows(std::vector<double>& H, int n, int r0, int len, const double* v, double beta,
                  int c0, int c1) {
  for (int j = c0; j <= c1; ++j) {
    double s = 0.0;
    for (int i = 0; i < len; ++i) s += v[i] * H[(size_t)(r0 + i) * n + j];
    s *= beta;
    for (int i = 0; i < len; ++i) H[(size_t)(r0 + i) * n + j] -= s * v[i];
  }
}

// columns k0..k0+len-1 times (I - beta v v^T) from the right, on rows r0..r1
void reflect_cols(std::vector<double>& H, int n, int k0, int len, const double* v, double beta,
                  int r0, int r1) {
  for (int i = r0; i <= r1; ++i) {
    double s = 0.0;
    for (int j = 0; j < len; ++j) s += H[(size_t)i * n + k0 + j] * v[j];
    s *= beta;
    for (int j = 0; j < len; ++j) H[(size_t)i * n + k0 + j] -= s * v[j];
  }
}

// eigenvalues of the 2 x 2 block [[a, b], [c, d]]
void eig2(double a, double b, double c, double d, double* wr, double* wi) {
  const double p = 0.5 * (a - d);
  const double disc = p * p + b * c;
  if (disc >= 0.0) {
    const double q = p + (p >= 0.0 ? sqrt(disc) : -sqrt(disc));  // no cancellation
    wr[0] = d + q;
    wr[1] = q != 0.0 ? d - b * c / q : d + q;
    wi[0] = wi[1] = 0.0;
  } else {
    wr[0] = wr[1] = d + p;
    wi[0] = sqrt(-disc);
    wi[1] = -wi[0];
  }
}

// Eigenvalues of the real n x n matrix H (row-major, overwritten): Householder
// reduction to upper Hessenberg form, then implicitly shifted double-shift QR
// steps (shifts: the eigenvalues of the trailing 2 x 2 block; every tenth
// step on one block the exceptional shift of EISPACK's HQR, Martin, Peters and
// Wilkinson, "The QR algorithm for real Hessenberg matrices", Numer. Math. 14
// (1970): shift sum 1.5 w and product w^2 from the last two subdiagonal
// magnitudes) with deflation at negligible subdiagonal entries.  false if a
// block has not split after 60 n steps.
bool hessenberg_qr(int n, std::vector<double>& H, double* wr, double* wi) {
  for (int k = 0; k + 2 < n; ++k) {
    double u[64], v[64];
    const int len = n - k - 1;
    for (int i = 0; i < len; ++i) u[i] = H[(size_t)(k + 1 + i) * n + k];
    double nrm = 0.0;
    for (int i = 0; i < len; ++i) nrm += u[i] * u[i];
    nrm = sqrt(nrm);
    if (nrm == 0.0) continue;
    const double alpha = u[0] >= 0.0 ? -nrm : nrm;
    for (int i = 0; i < len; ++i) v[i] = u[i];
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < len; ++i) vv += v[i] * v[i];
    if (!(vv > 0.0)) continue;
    const double beta = 2.0 / vv;
    reflect_rows(H, n, k + 1, len, v, beta, k, n - 1);
    reflect_cols(H, n, k + 1, len, v, beta, 0, n - 1);
    H[(size_t)(k + 1) * n + k] = alpha;
    for (int i = k + 2; i < n; ++i) H[(size_t)i * n + k] = 0.0;
  }
  double norm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = std::max(0, i - 1); j < n; ++j) norm += fabs(H[(size_t)i * n + j]);
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
  int hi = n - 1, its = 0, total = 0;
  while (hi >= 0) {
    int l = hi;
    while (l > 0) {
      double s = fabs(h(l - 1, l - 1)) + fabs(h(l, l));
      if (s == 0.0) s = norm;
      if (fabs(h(l, l - 1)) <= kEps * s) {
        h(l, l - 1) = 0.0;
        break;
      }
      --l;
    }
    if (l == hi) {  // 1 x 1 block
      wr[hi] = h(hi, hi);
      wi[hi] = 0.0;
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {  // 2 x 2 block
      eig2(h(hi - 1, hi - 1), h(hi - 1, hi), h(hi, hi - 1), h(hi, hi), wr + hi - 1, wi + hi - 1);
      hi -= 2;
      its = 0;
      continue;
    }
    if (++total > 60 * n) return false;
    ++its;
    // the double shift: sum and product of the trailing 2 x 2 block's eigenvalues
    double s = h(hi - 1, hi - 1) + h(hi, hi);
    double t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
    if (its % 10 == 0) {
      const double w = fabs(h(hi, hi - 1)) + fabs(h(hi - 1, hi - 2));
      s = 1.5 * w;
      t = w * w;
    }
    // first column of H^2 - s H + t I on the active block (three entries)
    double x = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - s * h(l, l) + t;
    double y = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - s);
    double z = h(l + 1, l) * h(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      const double u[3] = {x, y, z};
      double v[3];
      const double beta = householder(u, 3, v);
      if (beta > 0.0) {
        reflect_rows(H, n, k, 3, v, beta, std::max(l, k - 1), hi);
        reflect_cols(H, n, k, 3, v, beta, l, std::min(k + 3, hi));
      }
      x = h(k + 1, k);
      y = h(k + 2, k);
      if (k < hi - 2) z = h(k + 3, k);
    }
    const double u[2] = {x, y};
    double v[2];
    const double beta = householder(u, 2, v);
    if (beta > 0.0) {
      reflect_rows(H, n, hi - 1, 2, v, beta, hi - 2, hi);
      reflect_cols(H, n, hi - 1, 2, v, beta, l, hi);
    }
  }
  return true;
}

morx_status pencil_eigs(int r, const double* Ar, const double* Er, double* wr, double* wi) {
  std::vector<double> H;
  MORX_REQUIRE(pencil_to_standard(r, Ar, Er, H), MORX_E_INVALID,
               "reduced pencil: Er is singular");
  MORX_REQUIRE(hessenberg_qr(r, H, wr, wi), MORX_E_NOT_CONVERGED,
               "reduced pencil: QR iterations did not converge");
  // ascending real part (then imaginary part)
  std::vector<int> ord(r);
  for (int i = 0; i < r; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) {
    return wr[a] < wr[b] || (wr[a] == wr[b] && wi[a] < wi[b]);
  });
  std::vector<double> a(wr, wr + r), b(wi, wi + r);
  for (int i = 0; i < r; ++i) {
    wr[i] = a[ord[i]];
    wi[i] = b[ord[i]];
  }
  return MORX_OK;
}

// LU with partial pivoting of the row-major r x r matrix M, in place; pivots
// smaller than tiny are set to tiny (inverse iteration factors the matrix at
// an eigenvalue, where a pivot vanishes)
void lu_factor(int r, std::vector<double>& M, std::vector<int>& piv, double tiny) {
  piv.resize(r);
  for (int k = 0; k < r; ++k) {
    int p = k;
    for (int i = k + 1; i < r; ++i)
      if (fabs(M[(size_t)i * r + k]) > fabs(M[(size_t)p * r + k])) p = i;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < r; ++j) std::swap(M[(size_t)p * r + j], M[(size_t)k * r + j]);
    double& d = M[(size_t)k * r + k];
    if (fabs(d) < tiny) d = d < 0.0 ? -tiny : tiny;
    for (int i = k + 1; i < r; ++i) {
      const double f = M[(size_t)i * r + k] / d;
      M[(size_t)i * r + k] = f;
      for (int j = k + 1; j < r; ++j) M[(size_t)i * r + j] -= f * M[(size_t)k * r + j];
    }
  }
}

// x <- M^{-1} x with the factors of lu_factor (P M = L U, the interchanges
// applied to whole rows, so all of them come before the forward substitution)
void lu_solve(int r, const std::vector<double>& LU, const std::vector<int>& piv, double* x) {
  for (int k = 0; k < r; ++k) std::swap(x[k], x[piv[k]]);
  for (int k = 0; k < r; ++k)
    for (int i = k + 1; i < r; ++i) x[i] -= LU[(size_t)i * r + k] * x[k];
  for (int i = r - 1; i >= 0; --i) {
    double t = x[i];
    for (int j = i + 1; j < r; ++j) t -= LU[(size_t)i * r + j] * x[j];
    x[i] = t / LU[(size_t)i * r + i];
  }
}

// unit length, largest-magnitude entry positive
void normalise_dir(double* v, int len) {
  double nrm = 0.0, big = 0.0;
  int at = 0;
  for (int i = 0; i < len; ++i) {
    nrm += v[i] * v[i];
    if (fabs(v[i]) > big) {
      big = fabs(v[i]);
      at = i;
    }
  }
  nrm = sqrt(nrm);
  if (!(nrm > 0.0)) return;
  const double f = (v[at] < 0.0 ? -1.0 : 1.0) / nrm;
  for (int i = 0; i < len; ++i) v[i] *= f;
}

// Tangential directions of the reduced model (column-major Ar, Er (r x r),
// Br (r x m), Cr (r x q)) at its real eigenvalues lam[0..r): with
// Er^{-1} Ar = R diag(lam) R^{-1} (R's columns by inverse iteration),
// bdir_i = row i of R^{-1} Er^{-1} Br and cdir_i = column i of Cr^T R
morx_status tangent_dirs(int r, int m, int q, const double* Ar, const double* Er,
                         const double* Br, const double* Cr, const double* lam, double* bdir,
                         double* cdir) {
  std::vector<double> H;
  MORX_REQUIRE(pencil_to_standard(r, Ar, Er, H), MORX_E_INVALID, "reduced pencil: Er is singular");
  double hn = 0.0;
  for (double v : H) hn = std::max(hn, fabs(v));
  std::vector<double> R((size_t)r * r), M((size_t)r * r), x(r);
  std::vector<int> piv;
  for (int i = 0; i < r; ++i) {
    M = H;
    for (int d = 0; d < r; ++d) M[(size_t)d * r + d] -= lam[i];
    lu_factor(r, M, piv, 1e-14 * std::max(hn, fabs(lam[i])));
    for (int d = 0; d < r; ++d) x[d] = 1.0 + 0.01 * d;
    for (int it = 0; it < 3; ++it) {
      lu_solve(r, M, piv, x.data());
      double nrm = 0.0;
      for (double v : x) nrm += v * v;
      nrm = sqrt(nrm);
      MORX_REQUIRE(std::isfinite(nrm) && nrm > 0.0, MORX_E_NOT_CONVERGED,
                   "reduced pencil: inverse iteration failed at eigenvalue %d", i);
      for (double& v : x) v /= nrm;
    }
    for (int d = 0; d < r; ++d) R[(size_t)d * r + i] = x[d];  // row-major, column i
  }
  // Er^{-1} Br, then R^{-1} of that
  std::vector<double> Ef((size_t)r * r), Rf(R);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) Ef[(size_t)i * r + j] = Er[(size_t)j * r + i];
  std::vector<int> pe, pr;
  lu_factor(r, Ef, pe, 1e-300);
  lu_factor(r, Rf, pr, 1e-300);
  for (int k = 0; k < m; ++k) {
    for (int d = 0; d < r; ++d) x[d] = Br[(size_t)k * r + d];
    lu_solve(r, Ef, pe, x.data());
    lu_solve(r, Rf, pr, x.data());
    for (int i = 0; i < r; ++i) bdir[(size_t)i * m + k] = x[i];
  }
  for (int i = 0; i < r; ++i)
    for (int k = 0; k < q; ++k) {
      double t = 0.0;
      for (int d = 0; d < r; ++d) t += Cr[(size_t)k * r + d] * R[(size_t)d * r + i];
      cdir[(size_t)i * q + k] = t;
    }
  for (int i = 0; i < r; ++i) {
    normalise_dir(bdir + (size_t)i * m, m);
    normalise_dir(cdir + (size_t)i * q, q);
    for (int k = 0; k < m; ++k)
      MORX_REQUIRE(std::isfinite(bdir[(size_t)i * m + k]), MORX_E_NOT_CONVERGED,
                   "reduced pencil: eigenvector matrix is singular");
    for (int k = 0; k < q; ++k)
      MORX_REQUIRE(std::isfinite(cdir[(size_t)i * q + k]), MORX_E_NOT_CONVERGED,
                   "reduced pencil: eigenvector matrix is singular");
  }
  return MORX_OK;
}

// out[:, j] = M dir_j for the r columns j (M: n x k, dir: k x r column-major)
__global__ __launch_bounds__(256) void k_tangent(const double* __restrict__ M, int64_t ldm, int k,
                                                 const double* __restrict__ dir,
                                                 double* __restrict__ out, int64_t ldo,
                                                 int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = blockIdx.y;
  double s = 0.0;
  for (int c = 0; c < k; ++c) s = fma(M[(int64_t)c * ldm + i], dir[(int64_t)j * k + c], s);
  out[(int64_t)j * ldo + i] = s;
}

}  // namespace

extern "C" morx_status morx_pencil_eigvals(int32_t r, const double* Ar, const double* Er,
                                           double* wr, double* wi) {
  MORX_REQUIRE(r >= 1 && r <= 64, MORX_E_INVALID, "morx_pencil_eigvals: r must be 1..64");
  MORX_REQUIRE(Ar && Er && wr && wi, MORX_E_INVALID, "morx_pencil_eigvals: null argument");
  for (int64_t i = 0; i < (int64_t)r * r; ++i)
    MORX_REQUIRE(std::isfinite(Ar[i]) && std::isfinite(Er[i]), MORX_E_NONFINITE,
                 "morx_pencil_eigvals: non-finite entry");
  return pencil_eigs(r, Ar, Er, wr, wi);
}

extern "C" morx_status morx_irka(morx_system sys, int32_t r, double* sigmas, const double* b,
                                 const double* c, int32_t max_rounds, double tol,
                                 const morx_opts* opts, double* Ar, double* Er, double* Br,
                                 double* Cr, double* poles_re, double* poles_im, int32_t* rounds,
                                 double* change, morx_col_stats* stats, void* stream) {
  MORX_REQUIRE(sys && sigmas && b && c && Ar && Er && Br && Cr && poles_re && poles_im && rounds &&
                   change,
               MORX_E_INVALID, "morx_irka: null argument");
  MORX_REQUIRE(r >= 1 && r <= 64, MORX_E_INVALID, "morx_irka: r must be 1..64");
  MORX_REQUIRE(max_rounds >= 1, MORX_E_INVALID, "morx_irka: max_rounds must be >= 1");
  MORX_REQUIRE(tol >= 0.0 && std::isfinite(tol), MORX_E_INVALID, "morx_irka: bad tolerance");
  morx_opts o;
  if (opts) o = *opts;
  else morx_opts_default(&o);
  MORX_REQUIRE(o.chain == MORX_CHAIN_RESET || o.chain == MORX_CHAIN_NEXT_ROUND, MORX_E_INVALID,
               "morx_irka: the rounds keep Algorithm 4's vertical chain (RESET or NEXT_ROUND)");
  std::vector<double> sig(sigmas, sigmas + r);
  for (double s : sig) MORX_REQUIRE(std::isfinite(s), MORX_E_NONFINITE, "morx_irka: shift not finite");
  std::sort(sig.begin(), sig.end());
  for (int i = 1; i < r; ++i)
    MORX_REQUIRE(sig[i] > sig[i - 1], MORX_E_INVALID, "morx_irka: shifts must be distinct");
  const int64_t n = sys->n;
  MORX_HIP(hipSetDevice(sys->ctx->device));
  DevBuf xy;
  MORX_TRY(dev_alloc(xy, (size_t)2 * r * n * sizeof(double)));
  double* X = (double*)xy.p;
  double* Y = X + (int64_t)r * n;
  std::vector<morx_col_stats> st(r);
  std::vector<double> wr(r), wi(r);
  morx_status s = MORX_OK;
  *rounds = 0;
  *change = INFINITY;
  for (int z = 1; z <= max_rounds; ++z) {
    // round 1 follows the caller's policy; later rounds link vertically
    // from the previous round's first shift (Algorithm 4 across rounds)
    morx_opts oz = o;
    oz.want_dual = 1;
    if (z > 1) oz.chain = MORX_CHAIN_NEXT_ROUND;
    s = morx_solve_shifts(sys, r, sig.data(), 1, b, n, c, n, X, n, Y, n, &oz, st.data(), stream);
    if (s != MORX_OK) break;
    s = morx_project(sys, r, X, n, Y, n, 1, b, n, 1, c, n, Ar, Er, Br, Cr, 1, stream);
    if (s != MORX_OK) break;
    *rounds = z;
    for (int i = 0; i < r; ++i) sigmas[i] = sig[i];
    s = pencil_eigs(r, Ar, Er, wr.data(), wi.data());
    if (s != MORX_OK) break;
    for (int i = 0; i < r; ++i) {
      poles_re[i] = wr[i];
      poles_im[i] = wi[i];
    }
    double amax = 0.0, imax = 0.0;
    for (int i = 0; i < r; ++i) {
      amax = std::max(amax, hypot(wr[i], wi[i]));
      imax = std::max(imax, fabs(wi[i]));
    }
    if (imax > 1e-10 * amax) {
      morx_set_error("morx_irka: the reduced pencil has a complex pole pair in round %d "
                     "(real shifts only)", z);
      s = MORX_E_UNSUPPORTED;
      break;
    }
    // next shifts: the mirror images, ascending (wr is ascending)
    std::vector<double> next(r);
    for (int i = 0; i < r; ++i) next[i] = -wr[r - 1 - i];
    double ch = 0.0;
    for (int i = 0; i < r; ++i) ch = std::max(ch, fabs(next[i] - sig[i]) / fabs(sig[i]));
    *change = ch;
    if (ch <= tol) break;
    if (z == max_rounds) {
      morx_set_error("morx_irka: shifts still moving after %d rounds (relative change %.3g)", z,
                     ch);
      s = MORX_E_NOT_CONVERGED;
      break;
    }
    bool distinct = true;
    for (int i = 1; i < r; ++i) distinct = distinct && next[i] > next[i - 1];
    if (!distinct) {
      morx_set_error("morx_irka: repeated mirror images in round %d", z);
      s = MORX_E_UNSUPPORTED;
      break;
    }
    sig = next;
  }
  if (stats)
    for (int i = 0; i < r; ++i) stats[i] = st[i];
  dev_free(xy);
  return s;
}

extern "C" morx_status morx_irka_tangential(morx_system sys, int32_t r, double* sigmas,
                                            int32_t m, const double* B, int64_t ldb, int32_t q,
                                            const double* C, int64_t ldc, double* bdir,
                                            double* cdir, int32_t max_rounds, double tol,
                                            const morx_opts* opts, double* Ar, double* Er,
                                            double* Br, double* Cr, double* poles_re,
                                            double* poles_im, int32_t* rounds, double* change,
                                            morx_col_stats* stats, void* stream) {
  const char* who = "morx_irka_tangential";
  MORX_REQUIRE(sys && sigmas && B && C && bdir && cdir && Ar && Er && Br && Cr && poles_re &&
                   poles_im && rounds && change,
               MORX_E_INVALID, "%s: null argument", who);
  MORX_REQUIRE(r >= 1 && r <= 64 && m >= 1 && m <= 64 && q >= 1 && q <= 64, MORX_E_INVALID,
               "%s: r, m and q must be 1..64", who);
  MORX_REQUIRE(ldb >= sys->n && ldc >= sys->n, MORX_E_INVALID, "%s: bad leading dimension", who);
  MORX_REQUIRE(max_rounds >= 1, MORX_E_INVALID, "%s: max_rounds must be >= 1", who);
  MORX_REQUIRE(tol >= 0.0 && std::isfinite(tol), MORX_E_INVALID, "%s: bad tolerance", who);
  morx_opts o;
  if (opts) o = *opts;
  else morx_opts_default(&o);
  MORX_REQUIRE(o.chain == MORX_CHAIN_RESET || o.chain == MORX_CHAIN_NEXT_ROUND, MORX_E_INVALID,
               "%s: the rounds keep Algorithm 4's vertical chain (RESET or NEXT_ROUND)", who);
  // shifts ascending, each with its directions
  std::vector<int> ord(r);
  for (int i = 0; i < r; ++i) {
    ord[i] = i;
    MORX_REQUIRE(std::isfinite(sigmas[i]), MORX_E_NONFINITE, "%s: shift not finite", who);
  }
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return sigmas[a] < sigmas[b]; });
  std::vector<double> sig(r), bd((size_t)r * m), cd((size_t)r * q);
  for (int i = 0; i < r; ++i) {
    sig[i] = sigmas[ord[i]];
    double nb = 0.0, nc = 0.0;
    for (int k = 0; k < m; ++k) {
      bd[(size_t)i * m + k] = bdir[(size_t)ord[i] * m + k];
      nb += fabs(bd[(size_t)i * m + k]);
    }
    for (int k = 0; k < q; ++k) {
      cd[(size_t)i * q + k] = cdir[(size_t)ord[i] * q + k];
      nc += fabs(cd[(size_t)i * q + k]);
    }
    MORX_REQUIRE(std::isfinite(nb) && std::isfinite(nc), MORX_E_NONFINITE,
                 "%s: direction not finite", who);
    MORX_REQUIRE(nb > 0.0 && nc > 0.0, MORX_E_INVALID, "%s: zero direction", who);
  }
  for (int i = 1; i < r; ++i)
    MORX_REQUIRE(sig[i] > sig[i - 1], MORX_E_INVALID, "%s: shifts must be distinct", who);
  const int64_t n = sys->n;
  MORX_HIP(hipSetDevice(sys->ctx->device));
  hipStream_t hs = (hipStream_t)stream;
  DevBuf buf;
  MORX_TRY(dev_alloc(buf, ((size_t)4 * r * n + (size_t)r * (m + q)) * sizeof(double)));
  double* X = (double*)buf.p;
  double* Y = X + (int64_t)r * n;
  double* Bt = Y + (int64_t)r * n;
  double* Ct = Bt + (int64_t)r * n;
  double* ddir = Ct + (int64_t)r * n;
  std::vector<morx_col_stats> st(r);
  std::vector<double> wr(r), wi(r), lam(r), nbd((size_t)r * m), ncd((size_t)r * q);
  morx_status s = MORX_OK;
  *rounds = 0;
  *change = INFINITY;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)r);
  for (int z = 1; z <= max_rounds; ++z) {
    // right-hand sides B bdir_i and C cdir_i
    if (hipMemcpyAsync(ddir, bd.data(), bd.size() * sizeof(double), hipMemcpyHostToDevice, hs) !=
            hipSuccess ||
        hipMemcpyAsync(ddir + (size_t)r * m, cd.data(), cd.size() * sizeof(double),
                       hipMemcpyHostToDevice, hs) != hipSuccess) {
      morx_set_error("%s: copying the directions failed", who);
      s = MORX_E_HIP;
      break;
    }
    k_tangent<<<grid, 256, 0, hs>>>(B, ldb, m, ddir, Bt, n, n);
    k_tangent<<<grid, 256, 0, hs>>>(C, ldc, q, ddir + (size_t)r * m, Ct, n, n);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(hs) != hipSuccess) {
      morx_set_error("%s: forming the right-hand sides failed", who);
      s = MORX_E_HIP;
      break;
    }
    morx_opts oz = o;
    oz.want_dual = 1;
    if (z > 1) oz.chain = MORX_CHAIN_NEXT_ROUND;
    s = morx_solve_pairs(sys, r, sig.data(), Bt, n, Ct, n, X, n, Y, n, &oz, st.data(), stream);
    if (s != MORX_OK) break;
    s = morx_project(sys, r, X, n, Y, n, m, B, ldb, q, C, ldc, Ar, Er, Br, Cr, 1, stream);
    if (s != MORX_OK) break;
    *rounds = z;
    for (int i = 0; i < r; ++i) sigmas[i] = sig[i];
    memcpy(bdir, bd.data(), bd.size() * sizeof(double));
    memcpy(cdir, cd.data(), cd.size() * sizeof(double));
    s = pencil_eigs(r, Ar, Er, wr.data(), wi.data());
    if (s != MORX_OK) break;
    for (int i = 0; i < r; ++i) {
      poles_re[i] = wr[i];
      poles_im[i] = wi[i];
    }
    double amax = 0.0, imax = 0.0;
    for (int i = 0; i < r; ++i) {
      amax = std::max(amax, hypot(wr[i], wi[i]));
      imax = std::max(imax, fabs(wi[i]));
    }
    if (imax > 1e-10 * amax) {
      morx_set_error("%s: the reduced pencil has a complex pole pair in round %d "
                     "(real shifts only)", who, z);
      s = MORX_E_UNSUPPORTED;
      break;
    }
    // next shifts: the mirror images, ascending; lam[i] the pole of shift i
    std::vector<double> next(r);
    for (int i = 0; i < r; ++i) {
      lam[i] = wr[r - 1 - i];
      next[i] = -lam[i];
    }
    double ch = 0.0;
    for (int i = 0; i < r; ++i) ch = std::max(ch, fabs(next[i] - sig[i]) / fabs(sig[i]));
    *change = ch;
    if (ch <= tol) break;
    if (z == max_rounds) {
      morx_set_error("%s: shifts still moving after %d rounds (relative change %.3g)", who, z, ch);
      s = MORX_E_NOT_CONVERGED;
      break;
    }
    bool distinct = true;
    for (int i = 1; i < r; ++i) distinct = distinct && next[i] > next[i - 1];
    if (!distinct) {
      morx_set_error("%s: repeated mirror images in round %d", who, z);
      s = MORX_E_UNSUPPORTED;
      break;
    }
    s = tangent_dirs(r, m, q, Ar, Er, Br, Cr, lam.data(), nbd.data(), ncd.data());
    if (s != MORX_OK) break;
    sig = next;
    bd = nbd;
    cd = ncd;
  }
  if (stats)
    for (int i = 0; i < r; ++i) stats[i] = st[i];
  hipStreamSynchronize(hs);
  dev_free(buf);
  return s;
}
