// Restarted GMRES(m) with right preconditioning: the solver of the paper's
// experiments (Section IV), here a comparator of the BiCG path on the same
// factor chains (Algorithm 4 or a comparator schedule).  Every system, the
// primal (sigma E - A) x = b with P and the transposed one with P^T, runs its
// own GMRES, one system at a time (the paper solves them in sequence):
//   Arnoldi on A_s P, classical Gram-Schmidt applied twice (dot products and
//   updates on the device, all basis vectors of a pass at once),
//   the Hessenberg matrix, Givens rotations and the triangular solve of at
//   most (m+1) x m on the host (one synchronisation per Arnoldi step),
//   x += P (V y) at the end of a cycle, then the true residual decides:
//   done, restart (after m steps), or a refinement restart (the estimate
//   passed but the true residual did not; at most max_restarts of those).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "krylov.h"

morx_status launch_shifted_apply(morx_system sys, double sigma, bool trans, int ncol,
                                 const double* X, int64_t ldx, double* Y, int64_t ldy,
                                 hipStream_t st);
morx_status launch_factor_apply(morx_system sys, morx_factor f, bool trans, int ncol,
                                const double* X, int64_t ldx, double* Y, int64_t ldy,
                                hipStream_t st);

namespace {

constexpr int kBlock = 256;
constexpr int kGroup = 8;       // basis vectors per thread in the dot kernel
constexpr int kDotBlocks = 512;  // row blocks of the dot kernel (partials per vector)
constexpr int kMaxRestart = 64;

// partial sums of v_q . w for q < k (v_q = V + q * ldv); blockIdx.y picks a
// group of kGroup vectors
__global__ __launch_bounds__(kBlock) void k_gm_dots(const double* __restrict__ V, int64_t ldv,
                                                    int k, const double* __restrict__ w,
                                                    int64_t n, double* __restrict__ part) {
  __shared__ double sh[kBlock / 64][kGroup];
  const int q0 = blockIdx.y * kGroup;
  double acc[kGroup];
#pragma unroll
  for (int q = 0; q < kGroup; ++q) acc[q] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double wi = w[i];
#pragma unroll
    for (int q = 0; q < kGroup; ++q)
      if (q0 + q < k) acc[q] = fma(V[(int64_t)(q0 + q) * ldv + i], wi, acc[q]);
  }
#pragma unroll
  for (int q = 0; q < kGroup; ++q) {
    const double s = wave_sum(acc[q]);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kGroup && q0 + (int)threadIdx.x < k) {
    const int q = threadIdx.x;
    part[(int64_t)(q0 + q) * gridDim.x + blockIdx.x] = (sh[0][q] + sh[1][q]) + (sh[2][q] + sh[3][q]);
  }
}

// out[q] (+)= sum of the partials of vector q, in a fixed order; one wave per vector
__global__ __launch_bounds__(1024) void k_gm_fin(const double* __restrict__ part, int nblk, int k,
                                                 double* __restrict__ out, int accumulate) {
  const int lane = threadIdx.x & 63;
  for (int q = threadIdx.x >> 6; q < k; q += 16) {
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += part[(int64_t)q * nblk + b];
    s = wave_sum(s);
    if (lane == 0) out[q] = accumulate ? out[q] + s : s;
  }
}

// w -= sum_q h[q] v_q, q < k
__global__ __launch_bounds__(kBlock) void k_gm_update(const double* __restrict__ V, int64_t ldv,
                                                      int k, const double* __restrict__ h,
                                                      double* __restrict__ w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = w[i];
  for (int q = 0; q < k; ++q) s = fma(-h[q], V[(int64_t)q * ldv + i], s);
  w[i] = s;
}

// y = a * x
__global__ __launch_bounds__(kBlock) void k_gm_scale(const double* __restrict__ x, double a,
                                                     double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// u = sum_q y[q] v_q, q < k
__global__ __launch_bounds__(kBlock) void k_gm_combine(const double* __restrict__ V, int64_t ldv,
                                                       int k, const double* __restrict__ y,
                                                       double* __restrict__ u, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < k; ++q) s = fma(y[q], V[(int64_t)q * ldv + i], s);
  u[i] = s;
}

// x += z; r = b - q (q = A_s x computed beforehand)
__global__ __launch_bounds__(kBlock) void k_gm_axpy(const double* __restrict__ z,
                                                    double* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] += z[i];
}

__global__ __launch_bounds__(kBlock) void k_gm_residual(const double* __restrict__ b,
                                                        const double* __restrict__ q,
                                                        double* __restrict__ r, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) r[i] = b[i] - q[i];
}

__global__ void k_gm_zero(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// device workspace of one system's GMRES
struct GmWork {
  morx_system sys;
  hipStream_t st;
  int64_t n, ld;
  int m;
  double *V, *Z, *T0, *T1, *W, *U, *R, *part, *hd;  // hd: 3 (m+1) coefficients + norm
};

// z = P v (forward chain: factors first to last) or P^T v (transposed chain:
// transposed factors last to first), never forming the product
morx_status chain_apply(const GmWork& g, const std::vector<morx_factor>& chain, bool trans,
                        const double* v, double* z) {
  const int L = (int)chain.size();
  const double* src = v;
  for (int p = 0; p < L; ++p) {
    morx_factor f = trans ? chain[L - 1 - p] : chain[p];
    double* dst = (p == L - 1) ? z : ((p & 1) ? g.T1 : g.T0);
    MORX_TRY(launch_factor_apply(g.sys, f, trans, 1, src, g.ld, dst, g.ld, g.st));
    src = dst;
  }
  return MORX_OK;
}

// h (device, k values) = V(:, 0:k)^T w, accumulated onto h when acc != 0
morx_status dots(const GmWork& g, const double* V, int k, const double* w, double* h, int acc) {
  const int nblk = (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (g.n + kBlock - 1) / kBlock));
  k_gm_dots<<<dim3(nblk, (k + kGroup - 1) / kGroup), kBlock, 0, g.st>>>(V, g.ld, k, w, g.n, g.part);
  k_gm_fin<<<1, 1024, 0, g.st>>>(g.part, nblk, k, h, acc);
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

void givens(double a, double b, double* c, double* s) {
  if (b == 0.0) {
    *c = 1.0;
    *s = 0.0;
    return;
  }
  const double r = std::hypot(a, b);
  *c = a / r;
  *s = b / r;
}

struct GmResult {
  int status, iters, restarts;
  double relres;
};

// One system: A_s x = b (trans = 0) or A_s^T x = b (trans = 1), x (dev) out.
morx_status gmres_one(const GmWork& g, double sigma, bool trans,
                      const std::vector<morx_factor>& chain, const double* b, double nb, double* x,
                      const morx_opts& o, int maxit, GmResult* res) {
  const int m = g.m;
  const int64_t n = g.n;
  res->iters = 0;
  res->restarts = 0;
  res->status = MORX_E_NOT_CONVERGED;
  k_gm_zero<<<blocks_for(n), kBlock, 0, g.st>>>(x, n);
  if (nb == 0.0) {
    res->status = MORX_OK;
    res->relres = 0.0;
    return MORX_OK;
  }
  // r = b
  MORX_HIP(hipMemcpyAsync(g.R, b, n * sizeof(double), hipMemcpyDeviceToDevice, g.st));
  double beta = nb;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
  std::vector<double> hh(3 * (m + 1) + 1);
  const double stop = o.tol * nb;
  while (true) {
    // v_0 = r / beta
    k_gm_scale<<<blocks_for(n), kBlock, 0, g.st>>>(g.R, 1.0 / beta, g.V, n);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k = 0;
    double est = beta;
    for (int j = 0; j < m; ++j) {
      double* vj = g.V + (int64_t)j * g.ld;
      MORX_TRY(chain_apply(g, chain, trans, vj, g.Z));
      MORX_TRY(launch_shifted_apply(g.sys, sigma, trans, 1, g.Z, g.ld, g.W, g.ld, g.st));
      // classical Gram-Schmidt, twice: h1 = V^T w, w -= V h1, h2 = V^T w, w -= V h2
      double* h1 = g.hd;
      double* h2 = g.hd + (m + 1);
      MORX_TRY(dots(g, g.V, j + 1, g.W, h1, 0));
      k_gm_update<<<blocks_for(n), kBlock, 0, g.st>>>(g.V, g.ld, j + 1, h1, g.W, n);
      MORX_TRY(dots(g, g.V, j + 1, g.W, h2, 0));
      k_gm_update<<<blocks_for(n), kBlock, 0, g.st>>>(g.V, g.ld, j + 1, h2, g.W, n);
      double* nw = g.hd + 2 * (m + 1);
      MORX_TRY(dots(g, g.W, 1, g.W, nw, 0));
      MORX_HIP(hipMemcpyAsync(hh.data(), g.hd, (3 * (m + 1)) * sizeof(double),
                              hipMemcpyDeviceToHost, g.st));
      MORX_HIP(hipStreamSynchronize(g.st));
      const double hn = std::sqrt(std::max(hh[2 * (m + 1)], 0.0));
      double* Hj = &H[(size_t)j * (m + 1)];  // column j, rows 0..j+1
      for (int i = 0; i <= j; ++i) Hj[i] = hh[i] + hh[(m + 1) + i];
      Hj[j + 1] = hn;
      if (!(hn >= 0.0) || !std::isfinite(hn)) {
        morx_set_error("gmres: non-finite Arnoldi vector");
        return MORX_E_NONFINITE;
      }
      if (hn > 0.0)
        k_gm_scale<<<blocks_for(n), kBlock, 0, g.st>>>(g.W, 1.0 / hn, g.V + (int64_t)(j + 1) * g.ld,
                                                       n);
      for (int i = 0; i < j; ++i) {  // earlier rotations on the new column
        const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = t;
      }
      givens(Hj[j], Hj[j + 1], &cs[j], &sn[j]);
      Hj[j] = cs[j] * Hj[j] + sn[j] * Hj[j + 1];
      Hj[j + 1] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      k = j + 1;
      est = std::fabs(gv[k]);
      if (est <= stop || Hj[j] == 0.0) break;
    }
    res->iters += k;
    // y from the rotated (upper triangular) H; x += P (V y)
    for (int i = k - 1; i >= 0; --i) {
      double s = gv[i];
      for (int q = i + 1; q < k; ++q) s -= H[(size_t)q * (m + 1) + i] * y[q];
      y[i] = s / H[(size_t)i * (m + 1) + i];
    }
    MORX_HIP(hipMemcpyAsync(g.hd, y.data(), k * sizeof(double), hipMemcpyHostToDevice, g.st));
    k_gm_combine<<<blocks_for(n), kBlock, 0, g.st>>>(g.V, g.ld, k, g.hd, g.U, n);
    MORX_TRY(chain_apply(g, chain, trans, g.U, g.Z));
    k_gm_axpy<<<blocks_for(n), kBlock, 0, g.st>>>(g.Z, x, n);
    // true residual
    MORX_TRY(launch_shifted_apply(g.sys, sigma, trans, 1, x, g.ld, g.W, g.ld, g.st));
    k_gm_residual<<<blocks_for(n), kBlock, 0, g.st>>>(b, g.W, g.R, n);
    double* nr = g.hd + 2 * (m + 1);
    MORX_TRY(dots(g, g.R, 1, g.R, nr, 0));
    double rr = 0.0;
    MORX_HIP(hipMemcpyAsync(&rr, nr, sizeof(double), hipMemcpyDeviceToHost, g.st));
    MORX_HIP(hipStreamSynchronize(g.st));
    beta = std::sqrt(std::max(rr, 0.0));
    res->relres = beta / nb;
    if (res->relres <= o.tol) {
      res->status = MORX_OK;
      return MORX_OK;
    }
    if (res->iters >= maxit || !std::isfinite(beta)) return MORX_OK;
    if (est <= stop || k < m) {
      // the estimate passed (or the cycle broke down) but the true residual did not
      if (res->restarts >= o.max_restarts) return MORX_OK;
      res->restarts += 1;
    }
  }
}

}  // namespace

extern "C" morx_status morx_gmres_shifts(morx_system sys, int32_t nshift, const double* sigmas,
                                         int32_t m, const double* B, int64_t ldb, const double* C,
                                         int64_t ldc, int32_t restart, double* X, int64_t ldx,
                                         double* Y, int64_t ldy, const morx_opts* opts,
                                         morx_col_stats* stats, void* stream) {
  MORX_REQUIRE(sys, MORX_E_INVALID, "morx_gmres_shifts: null system");
  morx_opts o;
  if (opts) o = *opts;
  else morx_opts_default(&o);
  const bool want_dual = o.want_dual != 0;
  MORX_REQUIRE(nshift >= 1 && sigmas && m >= 1, MORX_E_INVALID,
               "morx_gmres_shifts: need at least one shift and one column");
  MORX_REQUIRE(restart >= 1 && restart <= kMaxRestart, MORX_E_INVALID,
               "morx_gmres_shifts: restart length must be 1..%d", kMaxRestart);
  MORX_REQUIRE(B && X && ldb >= sys->n && ldx >= sys->n, MORX_E_INVALID,
               "morx_gmres_shifts: bad B or X");
  MORX_REQUIRE(!want_dual || (C && Y && ldc >= sys->n && ldy >= sys->n), MORX_E_INVALID,
               "morx_gmres_shifts: want_dual needs C and Y");
  MORX_REQUIRE(o.precond_prec >= MORX_F64 && o.precond_prec <= MORX_BF16, MORX_E_INVALID,
               "morx_gmres_shifts: bad precision");
  MORX_REQUIRE(o.chain >= MORX_CHAIN_RESET && o.chain <= MORX_CHAIN_FIRST, MORX_E_INVALID,
               "morx_gmres_shifts: unknown chain policy %d", o.chain);
  MORX_REQUIRE(o.tol >= 0.0 && o.max_restarts >= 0, MORX_E_INVALID,
               "morx_gmres_shifts: bad tolerance or restart limit");
  for (int i = 0; i < nshift; ++i)
    MORX_REQUIRE(std::isfinite(sigmas[i]), MORX_E_NONFINITE,
                 "morx_gmres_shifts: shift %d not finite", i);
  MORX_REQUIRE(sys->ls_supported, MORX_E_UNSUPPORTED,
               "factor pattern exceeds the local least-squares limits");
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  MORX_TRY(stream_enter(ctx, caller));
  hipStream_t st = ctx->stream;

  std::vector<morx_factor> fresh, horizontal;
  ChainPlan plan;
  DevBuf work, norms;
  GmWork g{};
  g.sys = sys;
  g.st = st;
  g.n = sys->n;
  g.ld = sys->n_pad;
  g.m = restart;
  const int nblk = kDotBlocks;
  const size_t vecs = (size_t)(restart + 1) + 7;  // V (m+1), Z, T0, T1, W, U, R + partials
  morx_status s = dev_alloc(work, vecs * g.ld * sizeof(double) +
                                      ((size_t)(restart + 1) * nblk + 3 * (restart + 1) + 1 +
                                       kMaxRestart) * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(norms, (size_t)2 * m * sizeof(double));
  if (s == MORX_OK) s = plan_chains(sys, nshift, sigmas, o, fresh, plan);
  if (s == MORX_OK) s = factor_build_many(sys, o.precond_prec, plan.jobs.data(), nshift, st);
  if (s == MORX_OK) {
    double* base = (double*)work.p;
    g.V = base;
    g.Z = base + (int64_t)(restart + 1) * g.ld;
    g.T0 = g.Z + g.ld;
    g.T1 = g.T0 + g.ld;
    g.W = g.T1 + g.ld;
    g.U = g.W + g.ld;
    g.R = g.U + g.ld;
    g.part = g.R + g.ld;
    g.hd = g.part + (int64_t)(restart + 1) * nblk;
    const int maxit = o.maxit > 0 ? o.maxit : (int)std::min<int64_t>(sys->n, 20000);
    // right-hand-side norms
    std::vector<double> nb(m, 0.0), nc(m, 0.0);
    for (int c = 0; c < m && s == MORX_OK; ++c) {
      s = dots(g, B + (int64_t)c * ldb, 1, B + (int64_t)c * ldb, (double*)norms.p + c, 0);
      if (s == MORX_OK && want_dual)
        s = dots(g, C + (int64_t)c * ldc, 1, C + (int64_t)c * ldc, (double*)norms.p + m + c, 0);
    }
    std::vector<double> hn(2 * m, 0.0);
    if (s == MORX_OK &&
        (hipMemcpyAsync(hn.data(), norms.p, 2 * m * sizeof(double), hipMemcpyDeviceToHost, st) !=
             hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess)) {
      morx_set_error("gmres: norms");
      s = MORX_E_HIP;
    }
    for (int c = 0; c < m; ++c) {
      nb[c] = std::sqrt(hn[c]);
      nc[c] = std::sqrt(hn[m + c]);
      if (!std::isfinite(nb[c]) || !std::isfinite(nc[c])) {
        morx_set_error("B or C holds NaN or Inf");
        s = MORX_E_NONFINITE;
      }
    }
    for (int i = 0; i < nshift && s == MORX_OK; ++i)
      for (int c = 0; c < m && s == MORX_OK; ++c) {
        const int64_t k = (int64_t)i * m + c;
        GmResult rp{}, rd{};
        s = gmres_one(g, sigmas[i], false, plan.chains[i], B + (int64_t)c * ldb, nb[c],
                      X + k * ldx, o, maxit, &rp);
        if (s == MORX_OK && want_dual)
          s = gmres_one(g, sigmas[i], true, plan.chains[i], C + (int64_t)c * ldc, nc[c],
                        Y + k * ldy, o, maxit, &rd);
        if (s == MORX_OK && stats) {
          morx_col_stats& cs = stats[k];
          memset(&cs, 0, sizeof(cs));
          cs.status = rp.status != MORX_OK ? rp.status : (want_dual ? rd.status : MORX_OK);
          cs.iters = rp.iters + (want_dual ? rd.iters : 0);
          cs.restarts = rp.restarts + (want_dual ? rd.restarts : 0);
          cs.relres_primal = rp.relres;
          cs.relres_dual = want_dual ? rd.relres : 0.0;
        }
      }
  }
  hipStreamSynchronize(st);
  if (s == MORX_OK) commit_chains(sys, plan, sigmas, o.precond_prec, fresh, horizontal);
  for (morx_factor f : horizontal) factor_release(f);
  for (morx_factor f : fresh) factor_release(f);
  dev_free(work);
  dev_free(norms);
  morx_status s2 = stream_leave(ctx, caller);
  if (s != MORX_OK) return s;
  if (s2 != MORX_OK) return s2;
  morx_status worst = MORX_OK;
  if (stats)
    for (int64_t k = 0; k < (int64_t)nshift * m; ++k)
      if (stats[k].status != MORX_OK) worst = (morx_status)stats[k].status;
  return worst;
}
