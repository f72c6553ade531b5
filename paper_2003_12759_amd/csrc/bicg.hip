// Right-preconditioned two-sided BiCG for a batch of shifted systems
// (sigma_c E - A) x_c = b_c and (sigma_c E - A)^T y_c = c_c, one recurrence per
// column pair (Section III-A: Krylov methods with right preconditioning,
// x = P x~; the shadow recurrence of BiCG is the transposed system with P^T).
//
// Preconditioner of column c: the first L_c factors of one factor list G,
// applied G[0] first (Algorithm 4: P_1^(1), Q_1^(2..z), Q_2^(z), ...).  All
// columns of a batch share G, so chain step s reads factor s once for every
// column whose chain contains it, and the transposed chain reads it once in
// the reverse order.
//
// One iteration = L_max chain launches (forward and transposed halves side
// by side) + one launch for p, p~ and both shifted products + one update
// launch.  Scalars (rho, beta, delta, alpha, norms, state) stay on the
// device; each reduction ends in the last block to arrive, which sums the
// per-block partials in a fixed order (deterministic) and advances the
// column's state.  The host only polls the states every few iterations.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

struct ColInfo {
  double sigma;
  double nb, nc;      // norms of the primal and dual right-hand sides
  double tol;
  double rho, rho_prev, alpha, beta, delta;
  double rr, rtrt;    // squared norms of the current residuals
  double relp, reld;  // true relative residuals at the last check
  const double* bsrc;  // primal right-hand side (dev)
  const double* csrc;  // dual (or shadow) right-hand side (dev)
  double* xout;        // caller's output columns (dev) or null
  double* yout;
  int32_t state, L, first, it_cycle, iters, restarts, max_restarts, maxit;
  int32_t check_p, check_d, broke, status;
  int32_t out_x, out_y;  // 0: write zeros, 1: primal iterate, 2: dual iterate
  int32_t pad0, pad1;
};

enum Vec : int {
  V_X, V_XT, V_R, V_RT, V_P0, V_P1, V_PT0, V_PT1, V_Z, V_ZT, V_Q, V_QT,
  V_T0, V_T1, V_TT0, V_TT1, kNumVec
};

struct Workspace {
  int64_t ld = 0;
  int cap = 0;
  int nblk_cap = 0;
  DevBuf vec, cols, partial, counters;
  ColInfo* hcols = nullptr;  // pinned host mirror
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kNC = 4;           // columns per thread
constexpr int kMaxBlocks = 2048;  // row blocks (grid-stride beyond)
constexpr double kBreakdown = 1e-14;

struct IterArgs {
  int64_t n, ld;
  int cap, nc, nblk;
  const int32_t *off, *col, *offT, *colT;
  const double *valA, *valAT, *e;
  double* vec;
  ColInfo* cols;
  double* partial;
  unsigned* counter;
};

__device__ __forceinline__ double* vptr(const IterArgs& a, int slot, int c) {
  return a.vec + ((int64_t)slot * a.cap + c) * a.ld;
}

// ---- reductions --------------------------------------------------------------

// reduce NQ values per column over the block and store one partial per block
template <int NQ>
__device__ void block_partials(double (&v)[kNC][NQ], unsigned mask, const IterArgs& a, int c0) {
  __shared__ double sh[kWaves][kNC * NQ];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kNC; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = wave_sum(v[j][q]);
      if (lane == 0) sh[w][j * NQ + q] = s;
    }
  __syncthreads();
  if (threadIdx.x < kNC * NQ) {
    const int j = threadIdx.x / NQ, q = threadIdx.x % NQ;
    double t = 0.0;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) t += sh[ww][threadIdx.x];
    if (mask & (1u << j)) a.partial[((int64_t)q * a.cap + c0 + j) * a.nblk + blockIdx.x] = t;
  }
}

__device__ bool arrive_last(unsigned* counter, unsigned total) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == total - 1u);
    if (last) atomicExch(counter, 0u);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// one wave sums the nblk partials of quantity q of column c (fixed order)
__device__ __forceinline__ double wave_total(const IterArgs& a, int q, int c) {
  const double* p = a.partial + ((int64_t)q * a.cap + c) * a.nblk;
  double s = 0.0;
  for (int b = threadIdx.x & 63; b < a.nblk; b += 64) s += p[b];
  return wave_sum(s);
}

__device__ __forceinline__ bool passed(const ColInfo& ci, double rr, double rtrt) {
  return (!ci.check_p || sqrt(rr) <= ci.tol * ci.nb) && (!ci.check_d || sqrt(rtrt) <= ci.tol * ci.nc);
}

// ---- kernels -------------------------------------------------------------------

// x = x~ = 0, r = b, r~ = c; norms of b and c
__global__ __launch_bounds__(kBlock) void k_init(IterArgs a) {
  const int c0 = blockIdx.y * kNC;
  unsigned mask = 0;
  const double* b[kNC];
  const double* cc[kNC];
  double* x[kNC];
  double* xt[kNC];
  double* r[kNC];
  double* rt[kNC];
  double v[kNC][2];
#pragma unroll
  for (int j = 0; j < kNC; ++j) {
    const int c = min(c0 + j, a.nc - 1);
    if (c0 + j < a.nc && a.cols[c].state == COL_ACTIVE) mask |= 1u << j;
    b[j] = a.cols[c].bsrc;
    cc[j] = a.cols[c].csrc;
    x[j] = vptr(a, V_X, c);
    xt[j] = vptr(a, V_XT, c);
    r[j] = vptr(a, V_R, c);
    rt[j] = vptr(a, V_RT, c);
    v[j][0] = v[j][1] = 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n; i += (int64_t)a.nblk * kBlock) {
#pragma unroll
    for (int j = 0; j < kNC; ++j)
      if (mask & (1u << j)) {
        const double bi = b[j][i], ci = cc[j][i];
        x[j][i] = 0.0;
        xt[j][i] = 0.0;
        r[j][i] = bi;
        rt[j][i] = ci;
        v[j][0] = fma(bi, bi, v[j][0]);
        v[j][1] = fma(ci, ci, v[j][1]);
      }
  }
  block_partials<2>(v, mask, a, c0);
  if (!arrive_last(a.counter, gridDim.x * gridDim.y)) return;
  for (int c = threadIdx.x >> 6; c < a.nc; c += kWaves) {
    ColInfo& ci = a.cols[c];
    if (ci.state != COL_ACTIVE) continue;
    const double bb = wave_total(a, 0, c), cc2 = wave_total(a, 1, c);
    if ((threadIdx.x & 63) == 0) {
      ci.nb = sqrt(bb);
      ci.nc = sqrt(cc2);
      ci.rr = bb;
      ci.rtrt = cc2;
      ci.first = 1;
      ci.it_cycle = 0;
      if (passed(ci, bb, cc2)) {
        ci.state = COL_DONE;
        ci.relp = ci.nb > 0.0 ? 1.0 : 0.0;
        ci.reld = ci.nc > 0.0 ? 1.0 : 0.0;
        if (ci.check_p && ci.nb == 0.0) ci.relp = 0.0;
        if (ci.check_d && ci.nc == 0.0) ci.reld = 0.0;
      }
    }
  }
}

// one chain step: forward half applies G[s] (rows of S), transposed half
// applies G[maxL-1-s]^T (rows of S^T); the last step also forms rho = z~^T r
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_chain_step(IterArgs a, const VT* __restrict__ fval,
                                                       const VT* __restrict__ bval, int s, int maxL,
                                                       int do_rho) {
  const int c0 = blockIdx.y * kNC;
  const bool bwd = blockIdx.z == 1;
  const int jf = bwd ? maxL - 1 - s : s;  // factor index applied by this half
  unsigned mask = 0;
  const double* src[kNC];
  double* dst[kNC];
  const double* rv[kNC];
#pragma unroll
  for (int j = 0; j < kNC; ++j) {
    const int c = min(c0 + j, a.nc - 1);
    const ColInfo& ci = a.cols[c];
    const int L = ci.L;
    if (c0 + j < a.nc && ci.state == COL_ACTIVE && L > jf) mask |= 1u << j;
    if (!bwd) {
      src[j] = (jf == 0) ? vptr(a, V_R, c) : vptr(a, V_T0 + ((jf - 1) & 1), c);
      dst[j] = (jf == L - 1) ? vptr(a, V_Z, c) : vptr(a, V_T0 + (jf & 1), c);
    } else {
      const int t = L - 1 - jf;  // how many transposed factors this column applied before
      src[j] = (t <= 0) ? vptr(a, V_RT, c) : vptr(a, V_TT0 + ((t - 1) & 1), c);
      dst[j] = (jf == 0) ? vptr(a, V_ZT, c) : vptr(a, V_TT0 + ((t < 0 ? 0 : t) & 1), c);
    }
    rv[j] = vptr(a, V_R, c);
  }
  const int32_t* off = bwd ? a.offT : a.off;
  const int32_t* col = bwd ? a.colT : a.col;
  const VT* val = bwd ? bval : fval;
  const bool rho_half = bwd && do_rho;
  double v[kNC][3];
#pragma unroll
  for (int j = 0; j < kNC; ++j) v[j][0] = v[j][1] = v[j][2] = 0.0;
  if (mask) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
         i += (int64_t)a.nblk * kBlock) {
      double acc[kNC];
#pragma unroll
      for (int j = 0; j < kNC; ++j) acc[j] = 0.0;
      sell_row<VT, kNC>(off, col, val, i, src, mask, acc);
#pragma unroll
      for (int j = 0; j < kNC; ++j)
        if (mask & (1u << j)) {
          dst[j][i] = acc[j];
          if (rho_half) {
            const double ri = rv[j][i];
            v[j][0] = fma(acc[j], ri, v[j][0]);
            v[j][1] = fma(acc[j], acc[j], v[j][1]);
            v[j][2] = fma(ri, ri, v[j][2]);
          }
        }
    }
  }
  if (!rho_half) return;
  block_partials<3>(v, mask, a, c0);
  if (!arrive_last(a.counter, gridDim.x * gridDim.y)) return;
  for (int c = threadIdx.x >> 6; c < a.nc; c += kWaves) {
    ColInfo& ci = a.cols[c];
    if (ci.state != COL_ACTIVE) continue;
    const double rho = wave_total(a, 0, c), zz = wave_total(a, 1, c), rr = wave_total(a, 2, c);
    if ((threadIdx.x & 63) == 0) {
      if (fabs(rho) <= kBreakdown * sqrt(zz) * sqrt(rr)) {
        ci.state = COL_BREAKDOWN;
        ci.broke = 1;
      } else {
        ci.beta = ci.first ? 0.0 : rho / ci.rho_prev;
        ci.rho = rho;
      }
    }
  }
}

// p = z + beta p, p~ = z~ + beta p~ (formed on the fly at every gathered
// index), q = (sigma E - A) p, q~ = (sigma E - A)^T p~, delta = p~^T q
__global__ __launch_bounds__(kBlock) void k_spmv_pair(IterArgs a, int par) {
  const int c0 = blockIdx.y * kNC;
  unsigned mask = 0;
  const double *z[kNC], *zt[kNC], *po[kNC], *pto[kNC];
  double *pn[kNC], *ptn[kNC], *q[kNC], *qt[kNC];
  double beta[kNC], sig[kNC];
  bool first[kNC];
#pragma unroll
  for (int j = 0; j < kNC; ++j) {
    const int c = min(c0 + j, a.nc - 1);
    const ColInfo& ci = a.cols[c];
    if (c0 + j < a.nc && ci.state == COL_ACTIVE) mask |= 1u << j;
    z[j] = vptr(a, V_Z, c);
    zt[j] = vptr(a, V_ZT, c);
    po[j] = vptr(a, V_P0 + (par ^ 1), c);
    pto[j] = vptr(a, V_PT0 + (par ^ 1), c);
    pn[j] = vptr(a, V_P0 + par, c);
    ptn[j] = vptr(a, V_PT0 + par, c);
    q[j] = vptr(a, V_Q, c);
    qt[j] = vptr(a, V_QT, c);
    beta[j] = ci.beta;
    sig[j] = ci.sigma;
    first[j] = ci.first != 0;
  }
  double v[kNC][3];
#pragma unroll
  for (int j = 0; j < kNC; ++j) v[j][0] = v[j][1] = v[j][2] = 0.0;
  if (mask) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
         i += (int64_t)a.nblk * kBlock) {
      double acc[kNC], acct[kNC];
#pragma unroll
      for (int j = 0; j < kNC; ++j) acc[j] = acct[j] = 0.0;
      const int64_t sl = i >> 6;
      const int32_t lane = (int32_t)(i & 63);
      {
        const int32_t o1 = a.off[sl + 1];
        for (int32_t p = a.off[sl] + lane; p < o1; p += kSlice) {
          const int32_t cidx = a.col[p];
          const double av = a.valA[p];
#pragma unroll
          for (int j = 0; j < kNC; ++j)
            if (mask & (1u << j)) {
              const double pc = first[j] ? z[j][cidx] : fma(beta[j], po[j][cidx], z[j][cidx]);
              acc[j] = fma(av, pc, acc[j]);
            }
        }
      }
      {
        const int32_t o1 = a.offT[sl + 1];
        for (int32_t p = a.offT[sl] + lane; p < o1; p += kSlice) {
          const int32_t cidx = a.colT[p];
          const double av = a.valAT[p];
#pragma unroll
          for (int j = 0; j < kNC; ++j)
            if (mask & (1u << j)) {
              const double pc = first[j] ? zt[j][cidx] : fma(beta[j], pto[j][cidx], zt[j][cidx]);
              acct[j] = fma(av, pc, acct[j]);
            }
        }
      }
      const double ei = a.e[i];
#pragma unroll
      for (int j = 0; j < kNC; ++j)
        if (mask & (1u << j)) {
          const double pi = first[j] ? z[j][i] : fma(beta[j], po[j][i], z[j][i]);
          const double pti = first[j] ? zt[j][i] : fma(beta[j], pto[j][i], zt[j][i]);
          const double qi = fma(sig[j] * ei, pi, -acc[j]);
          const double qti = fma(sig[j] * ei, pti, -acct[j]);
          pn[j][i] = pi;
          ptn[j][i] = pti;
          q[j][i] = qi;
          qt[j][i] = qti;
          v[j][0] = fma(pti, qi, v[j][0]);
          v[j][1] = fma(pti, pti, v[j][1]);
          v[j][2] = fma(qi, qi, v[j][2]);
        }
    }
  }
  block_partials<3>(v, mask, a, c0);
  if (!arrive_last(a.counter, gridDim.x * gridDim.y)) return;
  for (int c = threadIdx.x >> 6; c < a.nc; c += kWaves) {
    ColInfo& ci = a.cols[c];
    if (ci.state != COL_ACTIVE) continue;
    const double delta = wave_total(a, 0, c), pp = wave_total(a, 1, c), qq = wave_total(a, 2, c);
    if ((threadIdx.x & 63) == 0) {
      if (fabs(delta) <= kBreakdown * sqrt(pp) * sqrt(qq)) {
        ci.state = COL_BREAKDOWN;
        ci.broke = 1;
      } else {
        ci.delta = delta;
        ci.alpha = ci.rho / delta;
      }
    }
  }
}

// x += alpha p, x~ += alpha p~, r -= alpha q, r~ -= alpha q~; convergence test
__global__ __launch_bounds__(kBlock) void k_update(IterArgs a, int par) {
  const int c0 = blockIdx.y * kNC;
  unsigned mask = 0;
  double *x[kNC], *xt[kNC], *r[kNC], *rt[kNC];
  const double *p[kNC], *pt[kNC], *q[kNC], *qt[kNC];
  double al[kNC];
#pragma unroll
  for (int j = 0; j < kNC; ++j) {
    const int c = min(c0 + j, a.nc - 1);
    const ColInfo& ci = a.cols[c];
    if (c0 + j < a.nc && ci.state == COL_ACTIVE) mask |= 1u << j;
    x[j] = vptr(a, V_X, c);
    xt[j] = vptr(a, V_XT, c);
    r[j] = vptr(a, V_R, c);
    rt[j] = vptr(a, V_RT, c);
    p[j] = vptr(a, V_P0 + par, c);
    pt[j] = vptr(a, V_PT0 + par, c);
    q[j] = vptr(a, V_Q, c);
    qt[j] = vptr(a, V_QT, c);
    al[j] = ci.alpha;
  }
  double v[kNC][2];
#pragma unroll
  for (int j = 0; j < kNC; ++j) v[j][0] = v[j][1] = 0.0;
  if (mask) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
         i += (int64_t)a.nblk * kBlock) {
#pragma unroll
      for (int j = 0; j < kNC; ++j)
        if (mask & (1u << j)) {
          x[j][i] = fma(al[j], p[j][i], x[j][i]);
          xt[j][i] = fma(al[j], pt[j][i], xt[j][i]);
          const double ri = fma(-al[j], q[j][i], r[j][i]);
          const double rti = fma(-al[j], qt[j][i], rt[j][i]);
          r[j][i] = ri;
          rt[j][i] = rti;
          v[j][0] = fma(ri, ri, v[j][0]);
          v[j][1] = fma(rti, rti, v[j][1]);
        }
    }
  }
  block_partials<2>(v, mask, a, c0);
  if (!arrive_last(a.counter, gridDim.x * gridDim.y)) return;
  for (int c = threadIdx.x >> 6; c < a.nc; c += kWaves) {
    ColInfo& ci = a.cols[c];
    if (ci.state != COL_ACTIVE) continue;
    const double rr = wave_total(a, 0, c), rtrt = wave_total(a, 1, c);
    if ((threadIdx.x & 63) == 0) {
      ci.rr = rr;
      ci.rtrt = rtrt;
      ci.it_cycle += 1;
      ci.iters += 1;
      ci.rho_prev = ci.rho;
      ci.first = 0;
      if (passed(ci, rr, rtrt)) ci.state = COL_CONVERGED;
      else if (ci.it_cycle >= ci.maxit) ci.state = COL_MAXIT;
    }
  }
}

// true residuals r = b - A_s x, r~ = c - A_s^T x~ for columns that stopped
// iterating; accept, restart from the current iterates, or give up
__global__ __launch_bounds__(kBlock) void k_true_residual(IterArgs a) {
  const int c0 = blockIdx.y * kNC;
  unsigned mask = 0;
  const double *x[kNC], *xt[kNC], *b[kNC], *cc[kNC];
  double *r[kNC], *rt[kNC];
  double sig[kNC];
#pragma unroll
  for (int j = 0; j < kNC; ++j) {
    const int c = min(c0 + j, a.nc - 1);
    const ColInfo& ci = a.cols[c];
    const int st = ci.state;
    if (c0 + j < a.nc && (st == COL_CONVERGED || st == COL_BREAKDOWN || st == COL_MAXIT))
      mask |= 1u << j;
    x[j] = vptr(a, V_X, c);
    xt[j] = vptr(a, V_XT, c);
    r[j] = vptr(a, V_R, c);
    rt[j] = vptr(a, V_RT, c);
    b[j] = ci.bsrc;
    cc[j] = ci.csrc;
    sig[j] = ci.sigma;
  }
  double v[kNC][2];
#pragma unroll
  for (int j = 0; j < kNC; ++j) v[j][0] = v[j][1] = 0.0;
  if (mask) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
         i += (int64_t)a.nblk * kBlock) {
      double acc[kNC], acct[kNC];
#pragma unroll
      for (int j = 0; j < kNC; ++j) acc[j] = acct[j] = 0.0;
      const double* xs[kNC];
      const double* xts[kNC];
#pragma unroll
      for (int j = 0; j < kNC; ++j) {
        xs[j] = x[j];
        xts[j] = xt[j];
      }
      sell_row<double, kNC>(a.off, a.col, a.valA, i, xs, mask, acc);
      sell_row<double, kNC>(a.offT, a.colT, a.valAT, i, xts, mask, acct);
      const double ei = a.e[i];
#pragma unroll
      for (int j = 0; j < kNC; ++j)
        if (mask & (1u << j)) {
          // b - (sigma E x - A x) = b - sigma e x + A x
          const double ri = b[j][i] - fma(sig[j] * ei, x[j][i], -acc[j]);
          const double rti = cc[j][i] - fma(sig[j] * ei, xt[j][i], -acct[j]);
          r[j][i] = ri;
          rt[j][i] = rti;
          v[j][0] = fma(ri, ri, v[j][0]);
          v[j][1] = fma(rti, rti, v[j][1]);
        }
    }
  }
  block_partials<2>(v, mask, a, c0);
  if (!arrive_last(a.counter, gridDim.x * gridDim.y)) return;
  for (int c = threadIdx.x >> 6; c < a.nc; c += kWaves) {
    ColInfo& ci = a.cols[c];
    const int st = ci.state;
    if (!(st == COL_CONVERGED || st == COL_BREAKDOWN || st == COL_MAXIT)) continue;
    const double rr = wave_total(a, 0, c), rtrt = wave_total(a, 1, c);
    if ((threadIdx.x & 63) == 0) {
      ci.rr = rr;
      ci.rtrt = rtrt;
      ci.relp = ci.nb > 0.0 ? sqrt(rr) / ci.nb : 0.0;
      ci.reld = ci.nc > 0.0 ? sqrt(rtrt) / ci.nc : 0.0;
      if (passed(ci, rr, rtrt)) {
        ci.state = COL_DONE;
        ci.status = MORX_OK;
      } else if (ci.restarts < ci.max_restarts) {
        ci.restarts += 1;
        ci.state = COL_ACTIVE;
        ci.first = 1;
        ci.it_cycle = 0;
      } else {
        ci.state = COL_FAILED;
        ci.status = (st == COL_BREAKDOWN) ? MORX_E_BREAKDOWN : MORX_E_NOT_CONVERGED;
      }
    }
  }
}

// copy the iterates to the caller's columns (or zeros)
__global__ __launch_bounds__(kBlock) void k_copy_out(IterArgs a, int64_t ldx, int64_t ldy) {
  const int c = blockIdx.y;
  const ColInfo& ci = a.cols[c];
  const double* xs = vptr(a, V_X, c);
  const double* ys = vptr(a, V_XT, c);
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    if (ci.xout) ci.xout[i] = ci.out_x == 1 ? xs[i] : (ci.out_x == 2 ? ys[i] : 0.0);
    if (ci.yout) ci.yout[i] = ci.out_y == 1 ? xs[i] : (ci.out_y == 2 ? ys[i] : 0.0);
  }
  (void)ldx;
  (void)ldy;
}

__global__ void k_zero(double* p, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// column norms of a dense block, one block per column (fixed order)
__global__ __launch_bounds__(kBlock) void k_colnorm(const double* X, int64_t ld, int64_t n,
                                                    double* out) {
  __shared__ double sh[kWaves];
  const double* x = X + (int64_t)blockIdx.x * ld;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) s = fma(x[i], x[i], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += sh[w];
    out[blockIdx.x] = sqrt(t);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

void workspace_free(Workspace* ws) {
  if (!ws) return;
  if (ws->exec) hipGraphExecDestroy(ws->exec);
  if (ws->graph) hipGraphDestroy(ws->graph);
  dev_free(ws->vec);
  dev_free(ws->cols);
  dev_free(ws->partial);
  dev_free(ws->counters);
  if (ws->hcols) hipHostFree(ws->hcols);
  delete ws;
}

static morx_status workspace_reserve(morx_system sys, int ncol) {
  Workspace* ws = sys->ws;
  if (ws && ws->cap >= ncol && ws->ld == sys->n_pad) return MORX_OK;
  int cap = std::max(ncol, ws ? 2 * ws->cap : 4);
  cap = std::max(cap, ncol);
  if (ws) {
    MORX_HIP(hipStreamSynchronize(sys->ctx->stream));
    workspace_free(ws);
  }
  sys->ws = nullptr;
  ws = new Workspace();
  ws->ld = sys->n_pad;
  ws->cap = cap;
  ws->nblk_cap = kMaxBlocks;
  morx_status s = dev_alloc(ws->vec, (size_t)kNumVec * cap * ws->ld * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(ws->cols, (size_t)cap * sizeof(ColInfo));
  if (s == MORX_OK) s = dev_alloc(ws->partial, (size_t)4 * cap * kMaxBlocks * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(ws->counters, 64 * sizeof(unsigned));
  if (s == MORX_OK && hipHostMalloc((void**)&ws->hcols, (size_t)cap * sizeof(ColInfo)) != hipSuccess)
    s = MORX_E_NOMEM;
  if (s != MORX_OK) {
    workspace_free(ws);
    morx_set_error("BiCG workspace allocation failed (%d columns)", ncol);
    return MORX_E_NOMEM;
  }
  hipStream_t st = sys->ctx->stream;
  int64_t cnt = (int64_t)(ws->vec.bytes / sizeof(double));
  k_zero<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>((double*)ws->vec.p, cnt);
  int64_t cc = 64 / 2;  // counters: 64 unsigned = 32 doubles of zero bits
  k_zero<<<1, 256, 0, st>>>((double*)ws->counters.p, cc);
  MORX_HIP(hipGetLastError());
  sys->ws = ws;
  return MORX_OK;
}

struct BatchCol {
  double sigma;
  int L;
  const double* b;
  const double* c;
  double* xout;
  double* yout;
  int check_p, check_d, out_x, out_y;
  morx_col_stats* stats;
};

static IterArgs make_args(morx_system sys, Workspace* ws, int nc, int slot) {
  IterArgs a;
  a.n = sys->n;
  a.ld = ws->ld;
  a.cap = ws->cap;
  a.nc = nc;
  a.nblk = (int)std::min<int64_t>((sys->n + kBlock - 1) / kBlock, kMaxBlocks);
  a.off = sys->sell.off;
  a.col = sys->sell.col;
  a.offT = sys->sellT.off;
  a.colT = sys->sellT.col;
  a.valA = sys->sell_val;
  a.valAT = sys->sellT_val;
  a.e = sys->e;
  a.vec = (double*)ws->vec.p;
  a.cols = (ColInfo*)ws->cols.p;
  a.partial = (double*)ws->partial.p;
  a.counter = (unsigned*)ws->counters.p + slot;
  return a;
}

template <typename VT>
static void enqueue_chain(IterArgs a, const std::vector<morx_factor>& G, int maxL, dim3 grid,
                          hipStream_t st) {
  for (int s = 0; s < maxL; ++s) {
    const VT* fv = (const VT*)G[s]->vals.p;
    const VT* bv = (const VT*)G[maxL - 1 - s]->valsT.p;
    k_chain_step<VT><<<grid, kBlock, 0, st>>>(a, fv, bv, s, maxL, s == maxL - 1 ? 1 : 0);
  }
}

static morx_status enqueue_iterations(morx_system sys, Workspace* ws, int nc,
                                      const std::vector<morx_factor>& G, int maxL, int prec,
                                      int iters, hipStream_t st) {
  IterArgs a_chain = make_args(sys, ws, nc, 0);
  IterArgs a_spmv = make_args(sys, ws, nc, 1);
  IterArgs a_upd = make_args(sys, ws, nc, 2);
  const unsigned chunks = (unsigned)((nc + kNC - 1) / kNC);
  dim3 g2(a_chain.nblk, chunks, 2), g1(a_chain.nblk, chunks, 1);
  for (int it = 0; it < iters; ++it) {
    const int par = it & 1;
    if (prec == MORX_F64) enqueue_chain<double>(a_chain, G, maxL, g2, st);
    else if (prec == MORX_F32) enqueue_chain<float>(a_chain, G, maxL, g2, st);
    else enqueue_chain<uint16_t>(a_chain, G, maxL, g2, st);
    k_spmv_pair<<<g1, kBlock, 0, st>>>(a_spmv, par);
    k_update<<<g1, kBlock, 0, st>>>(a_upd, par);
  }
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

// Solve one batch of columns sharing the factor list G (every chain is a prefix).
static morx_status solve_batch(morx_system sys, std::vector<BatchCol>& cols,
                               const std::vector<morx_factor>& G, int prec, const morx_opts& o,
                               hipStream_t st) {
  const int nc = (int)cols.size();
  if (nc == 0) return MORX_OK;
  int maxL = 0;
  for (auto& c : cols) maxL = std::max(maxL, c.L);
  MORX_REQUIRE(maxL >= 1 && maxL <= (int)G.size(), MORX_E_INVALID, "bad chain length");
  MORX_TRY(workspace_reserve(sys, nc));
  Workspace* ws = sys->ws;
  const int maxit = o.maxit > 0 ? o.maxit : (int)std::min<int64_t>(sys->n, 20000);
  for (int c = 0; c < nc; ++c) {
    ColInfo ci;
    ColInfo zero_ci = {};
    ci = zero_ci;
    ci.sigma = cols[c].sigma;
    ci.tol = o.tol;
    ci.bsrc = cols[c].b;
    ci.csrc = cols[c].c;
    ci.xout = cols[c].xout;
    ci.yout = cols[c].yout;
    ci.state = COL_ACTIVE;
    ci.L = cols[c].L;
    ci.first = 1;
    ci.max_restarts = o.max_restarts;
    ci.maxit = maxit;
    ci.check_p = cols[c].check_p;
    ci.check_d = cols[c].check_d;
    ci.out_x = cols[c].out_x;
    ci.out_y = cols[c].out_y;
    ci.status = MORX_E_NOT_CONVERGED;
    ws->hcols[c] = ci;
  }
  MORX_HIP(hipMemcpyAsync(ws->cols.p, ws->hcols, nc * sizeof(ColInfo), hipMemcpyHostToDevice, st));
  IterArgs a0 = make_args(sys, ws, nc, 3);
  const unsigned chunks = (unsigned)((nc + kNC - 1) / kNC);
  k_init<<<dim3(a0.nblk, chunks, 1), kBlock, 0, st>>>(a0);
  MORX_HIP(hipGetLastError());

  int seg = std::max(2, o.poll_iters > 0 ? o.poll_iters : 8);
  seg += seg & 1;  // even: the p buffers alternate by iteration parity
  bool graph_ready = false;
  if (ws->exec) {
    hipGraphExecDestroy(ws->exec);
    ws->exec = nullptr;
  }
  if (ws->graph) {
    hipGraphDestroy(ws->graph);
    ws->graph = nullptr;
  }
  if (o.use_graph) {
    MORX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    morx_status s = enqueue_iterations(sys, ws, nc, G, maxL, prec, seg, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    MORX_TRY(s);
    MORX_REQUIRE(e == hipSuccess, MORX_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    ws->graph = g;
    MORX_HIP(hipGraphInstantiate(&ws->exec, g, nullptr, nullptr, 0));
    graph_ready = true;
  }
  const int64_t guard_max = (int64_t)(o.max_restarts + 1) * (maxit + seg) / seg + 4;
  for (int64_t guard = 0; guard <= guard_max * 2; ++guard) {
    MORX_HIP(hipMemcpyAsync(ws->hcols, ws->cols.p, nc * sizeof(ColInfo), hipMemcpyDeviceToHost, st));
    MORX_HIP(hipStreamSynchronize(st));
    int active = 0, stopped = 0;
    for (int c = 0; c < nc; ++c) {
      const int s = ws->hcols[c].state;
      if (s == COL_ACTIVE) ++active;
      else if (s == COL_CONVERGED || s == COL_BREAKDOWN || s == COL_MAXIT) ++stopped;
    }
    if (active == 0 && stopped == 0) break;
    if (active == 0) {
      k_true_residual<<<dim3(a0.nblk, chunks, 1), kBlock, 0, st>>>(a0);
      MORX_HIP(hipGetLastError());
      continue;
    }
    if (graph_ready) {
      MORX_HIP(hipGraphLaunch(ws->exec, st));
    } else {
      MORX_TRY(enqueue_iterations(sys, ws, nc, G, maxL, prec, seg, st));
    }
  }
  // outputs
  k_copy_out<<<dim3((unsigned)std::min<int64_t>((sys->n + kBlock - 1) / kBlock, 1024), nc, 1),
               kBlock, 0, st>>>(a0, 0, 0);
  MORX_HIP(hipGetLastError());
  MORX_HIP(hipMemcpyAsync(ws->hcols, ws->cols.p, nc * sizeof(ColInfo), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipStreamSynchronize(st));
  for (int c = 0; c < nc; ++c) {
    const ColInfo& ci = ws->hcols[c];
    morx_col_stats* out = cols[c].stats;
    if (!out) continue;
    out->status = ci.state == COL_DONE ? MORX_OK : (ci.state == COL_FAILED ? ci.status : MORX_E_NOT_CONVERGED);
    out->iters = ci.iters;
    out->restarts = ci.restarts;
    out->relres_primal = cols[c].out_x == 2 ? ci.reld : (cols[c].out_x == 1 ? ci.relp : 0.0);
    out->relres_dual = cols[c].out_y == 2 ? ci.reld : (cols[c].out_y == 1 ? ci.relp : 0.0);
  }
  return MORX_OK;
}

// ---------------------------------------------------------------------------
// morx_solve_shifts: Algorithm 4's factor schedule around the batched solver

static int worse(int a, int b) {
  // the more severe of two statuses (0 is best)
  auto rank = [](int s) {
    switch (s) {
      case MORX_OK: return 0;
      case MORX_E_NOT_CONVERGED: return 1;
      case MORX_E_BREAKDOWN: return 2;
      default: return 3;
    }
  };
  return rank(b) > rank(a) ? b : a;
}

static morx_status solve_shifts_impl(morx_system sys, int32_t nshift, const double* sigmas,
                                     int32_t m, const double* B, int64_t ldb, const double* C,
                                     int64_t ldc, double* X, int64_t ldx, double* Y, int64_t ldy,
                                     const morx_opts& o, morx_col_stats* stats, hipStream_t st,
                                     std::vector<morx_factor>& horizontal) {
  const bool want_dual = o.want_dual != 0;
  const int prec = o.precond_prec;
  MORX_REQUIRE(sys->ls_supported, MORX_E_UNSUPPORTED,
               "factor pattern exceeds the local least-squares limits");
  // right-hand-side norms decide how each column pair runs
  DevBuf nb;
  MORX_TRY(dev_alloc(nb, (size_t)2 * m * sizeof(double)));
  k_colnorm<<<m, kBlock, 0, st>>>(B, ldb, sys->n, (double*)nb.p);
  if (want_dual) k_colnorm<<<m, kBlock, 0, st>>>(C, ldc, sys->n, (double*)nb.p + m);
  std::vector<double> norms(2 * m, 0.0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(norms.data(), nb.p, 2 * m * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dev_free(nb);
  MORX_REQUIRE(e == hipSuccess, MORX_E_HIP, "norms: %s", hipGetErrorString(e));
  for (int j = 0; j < 2 * m; ++j)
    MORX_REQUIRE(std::isfinite(norms[j]), MORX_E_NONFINITE, "B or C holds NaN or Inf");

  // factor list: vertical chain (+ this call's first factor), then horizontal
  const bool reset = (o.chain == MORX_CHAIN_RESET) || sys->vertical.empty();
  if (!reset)
    MORX_REQUIRE(sys->vertical_prec == prec, MORX_E_INVALID,
                 "MORX_CHAIN_NEXT_ROUND needs the precision of the previous round");
  if (reset) {
    for (morx_factor f : sys->vertical) factor_release(f);
    sys->vertical.clear();
  }
  std::vector<FactorJob> jobs;
  std::vector<morx_factor> fresh;
  for (int i = 0; i < nshift; ++i) {
    morx_factor f = nullptr;
    MORX_TRY(factor_alloc(sys, prec, &f));
    fresh.push_back(f);
    FactorJob jb;
    if (i == 0) {
      jb.is_spai = reset ? 1 : 0;
      jb.sigma_prev = reset ? 0.0 : sys->last_first_shift;
    } else {
      jb.is_spai = 0;
      jb.sigma_prev = sigmas[i - 1];
    }
    jb.sigma_new = sigmas[i];
    jb.vals = f->vals.p;
    jb.valsT = f->valsT.p;
    f->is_spai = jb.is_spai != 0;
    f->sigma_prev = jb.sigma_prev;
    f->sigma_new = jb.sigma_new;
    jobs.push_back(jb);
  }
  auto zero_cols = [&](int i, int j) {
    BatchCol bc{};
    bc.sigma = sigmas[i];
    bc.xout = X + (int64_t)(i * m + j) * ldx;
    bc.yout = want_dual ? Y + (int64_t)(i * m + j) * ldy : nullptr;
    return bc;
  };
  auto make_col = [&](int i, int j, int L) -> BatchCol {
    BatchCol bc = zero_cols(i, j);
    bc.L = L;
    bc.stats = stats ? &stats[i * m + j] : nullptr;
    const bool bz = norms[j] == 0.0;
    const bool cz = !want_dual || norms[m + j] == 0.0;
    if (!bz) {
      bc.b = B + (int64_t)j * ldb;
      bc.c = cz ? bc.b : C + (int64_t)j * ldc;  // shadow right-hand side b when c is absent
      bc.check_p = 1;
      bc.check_d = cz ? 0 : 1;
      bc.out_x = 1;
      bc.out_y = cz ? 0 : 2;
    } else {
      // only the transposed system is nontrivial: its recurrence is the shadow one
      bc.b = C + (int64_t)j * ldc;
      bc.c = bc.b;
      bc.check_p = 0;
      bc.check_d = 1;
      bc.out_x = 0;
      bc.out_y = 2;
    }
    return bc;
  };
  morx_status worst = MORX_OK;
  std::vector<BatchCol> trivial;
  for (int i = 0; i < nshift; ++i)
    for (int j = 0; j < m; ++j)
      if (norms[j] == 0.0 && (!want_dual || norms[m + j] == 0.0)) {
        BatchCol bc = zero_cols(i, j);
        bc.stats = stats ? &stats[i * m + j] : nullptr;
        trivial.push_back(bc);
      }

  auto finish_status = [&](int i0, int i1) {
    if (!stats) return;
    for (int i = i0; i < i1; ++i)
      for (int j = 0; j < m; ++j) worst = (morx_status)worse(worst, stats[i * m + j].status);
  };

  if (o.batched) {
    MORX_TRY(factor_build_many(sys, prec, jobs.data(), nshift, st));
    sys->vertical.push_back(fresh[0]);
    for (int i = 1; i < nshift; ++i) horizontal.push_back(fresh[i]);
    std::vector<morx_factor> G = sys->vertical;
    const int Lv = (int)sys->vertical.size();
    for (int i = 1; i < nshift; ++i) G.push_back(fresh[i]);
    std::vector<BatchCol> cols;
    for (int i = 0; i < nshift; ++i)
      for (int j = 0; j < m; ++j)
        if (!(norms[j] == 0.0 && (!want_dual || norms[m + j] == 0.0)))
          cols.push_back(make_col(i, j, Lv + i));
    MORX_TRY(solve_batch(sys, cols, G, prec, o, st));
  } else {
    // one shift at a time, one column at a time (factor i built just before
    // the solves that first need it, as in Algorithm 4)
    std::vector<morx_factor> G;
    for (int i = 0; i < nshift; ++i) {
      MORX_TRY(factor_build_many(sys, prec, &jobs[i], 1, st));
      if (i == 0) {
        sys->vertical.push_back(fresh[0]);
        G = sys->vertical;
      } else {
        horizontal.push_back(fresh[i]);
        G.push_back(fresh[i]);
      }
      for (int j = 0; j < m; ++j) {
        if (norms[j] == 0.0 && (!want_dual || norms[m + j] == 0.0)) continue;
        std::vector<BatchCol> one{make_col(i, j, (int)G.size())};
        MORX_TRY(solve_batch(sys, one, G, prec, o, st));
      }
    }
  }
  sys->vertical_prec = prec;
  sys->last_first_shift = sigmas[0];
  finish_status(0, nshift);
  // trivial columns: zero solutions
  for (auto& bc : trivial) {
    MORX_HIP(hipMemsetAsync(bc.xout, 0, sys->n * sizeof(double), st));
    if (bc.yout) MORX_HIP(hipMemsetAsync(bc.yout, 0, sys->n * sizeof(double), st));
    if (bc.stats) {
      bc.stats->status = MORX_OK;
      bc.stats->iters = 0;
      bc.stats->restarts = 0;
      bc.stats->relres_primal = 0.0;
      bc.stats->relres_dual = 0.0;
    }
  }
  MORX_HIP(hipStreamSynchronize(st));
  return worst;
}

extern "C" morx_status morx_solve_shifts(morx_system sys, int32_t nshift, const double* sigmas,
                                         int32_t m, const double* B, int64_t ldb, const double* C,
                                         int64_t ldc, double* X, int64_t ldx, double* Y,
                                         int64_t ldy, const morx_opts* opts,
                                         morx_col_stats* stats, void* stream) {
  MORX_REQUIRE(sys, MORX_E_INVALID, "morx_solve_shifts: null system");
  morx_opts o;
  if (opts) o = *opts;
  else morx_opts_default(&o);
  const bool want_dual = o.want_dual != 0;
  MORX_REQUIRE(nshift >= 1 && sigmas && m >= 1, MORX_E_INVALID,
               "morx_solve_shifts: need at least one shift and one column");
  MORX_REQUIRE(B && X && ldb >= sys->n && ldx >= sys->n, MORX_E_INVALID,
               "morx_solve_shifts: bad B or X");
  MORX_REQUIRE(!want_dual || (C && Y && ldc >= sys->n && ldy >= sys->n), MORX_E_INVALID,
               "morx_solve_shifts: want_dual needs C and Y");
  MORX_REQUIRE(o.precond_prec >= MORX_F64 && o.precond_prec <= MORX_BF16, MORX_E_INVALID,
               "morx_solve_shifts: bad precision");
  MORX_REQUIRE(o.tol >= 0.0 && o.max_restarts >= 0, MORX_E_INVALID,
               "morx_solve_shifts: bad tolerance or restart limit");
  for (int i = 0; i < nshift; ++i)
    MORX_REQUIRE(std::isfinite(sigmas[i]), MORX_E_NONFINITE, "morx_solve_shifts: shift %d not finite", i);
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  MORX_TRY(stream_enter(ctx, caller));
  std::vector<morx_factor> horizontal;
  morx_status s = solve_shifts_impl(sys, nshift, sigmas, m, B, ldb, want_dual ? C : nullptr, ldc,
                                    X, ldx, want_dual ? Y : nullptr, ldy, o, stats, ctx->stream,
                                    horizontal);
  hipStreamSynchronize(ctx->stream);
  for (morx_factor f : horizontal) factor_release(f);
  morx_status s2 = stream_leave(ctx, caller);
  return s != MORX_OK ? s : s2;
}
