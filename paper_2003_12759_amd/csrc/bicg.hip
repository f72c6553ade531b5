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
// One iteration is
//   L_max chain launches (forward and transposed halves side by side; the
//   last one also forms the partial sums of rho = z~^T r),
//   fin_rho   (one block: convergence test on the previous update, rho, beta),
//   form_p    (p = z + beta p, p~ = z~ + beta p~),
//   spmv_pair (q = A_s p, q~ = A_s^T p~, delta sums),
//   fin_delta (one block: alpha),
//   update    (x, x~, r, r~ and the partial sums of their norms).
// Scalars stay on the device; every reduction is block partials summed in a
// fixed order by the next one-block kernel (deterministic, and no grid-wide
// fences inside a kernel).  The host polls the column states every few
// iterations.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>
#include <vector>

#include <hip/hip_ext.h>

#include "chain_kernels.h"
#include "krylov.h"

static int apply_vecs(int aprec) { return aprec == MORX_F64 ? 6 : 8; }

// trace counters (algorithmic bytes per kernel class)
enum TraceClass : int {
  TR_CHAIN = 0, TR_SPMV = 1, TR_UPDATE = 2, TR_FACTOR = 3, TR_FORMP = 4, kTraceClasses = 8
};

namespace {

// ---- kernels -------------------------------------------------------------------

// x = x~ = 0, r = b, r~ = c; partial norms of b and c
template <int NC>
__global__ __launch_bounds__(kBlock) void k_init(IterArgs a) {
  const WaveCtx t = wave_ctx(a);
  const int c0 = blockIdx.y * NC;
  unsigned valid = 0;
#pragma unroll
  for (int j = 0; j < NC; ++j)
    if (c0 + j < a.nc && a.cols[c0 + j].state == COL_INIT) valid |= 1u << j;
  double v[NC][2];
#pragma unroll
  for (int j = 0; j < NC; ++j) v[j][0] = v[j][1] = 0.0;
  for (int64_t sl = t.s_begin; sl < t.s_end; ++sl) {
    const int64_t i = sl * kSlice + t.lane;
    if (i >= a.n) continue;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (!(valid & (1u << j))) continue;
      const int c = c0 + j;
      const ColInfo& ci = a.cols[c];
      const double bi = ci.bsrc[i], cv = ci.csrc[i];
      vptr(a, V_X, c)[i] = 0.0;
      vptr(a, V_XT, c)[i] = 0.0;
      vptr(a, V_R, c)[i] = bi;
      vptr(a, V_RT, c)[i] = cv;
      store_rcopy(a, c, i, bi, cv);
      v[j][0] = fma(bi, bi, v[j][0]);
      v[j][1] = fma(cv, cv, v[j][1]);
    }
  }
  block_partials<NC, 2>(a, t, c0, valid, v, a.part_norm);
}

__global__ __launch_bounds__(kFinThreads) void k_fin_init(IterArgs a) {
  for (int c = threadIdx.x >> 6; c < a.nc; c += kFinThreads / 64) {
    ColInfo& ci = a.cols[c];
    if (ci.state != COL_INIT) continue;
    double t2[2];
    wave_totals<2>(a, a.part_norm, c, t2);
    if ((threadIdx.x & 63) == 0) {
      ci.nb = sqrt(t2[0]);
      ci.nc = sqrt(t2[1]);
      ci.first = 1;
      ci.it_cycle = 0;
      ci.state = COL_ACTIVE;
    }
  }
}

// vector `slot` of column c in the apply precision
__device__ __forceinline__ void* apply_ptr(const IterArgs& a, int slot, int c) {
  return (char*)a.avec + ((int64_t)slot * a.cap + c) * a.ld * a.abytes;
}

// what the first factor pass of a chain reads: r (r~), or its FP32 copy
__device__ __forceinline__ const void* chain_in(const IterArgs& a, int c, bool bwd) {
  if (a.abytes == 8) return vptr(a, bwd ? V_RT : V_R, c);
  return apply_ptr(a, bwd ? A_RT : A_R, c);
}

// Work lists of the next iteration's chain steps.  Step s lists the forward
// pairs (active columns with L > s: factor s of the chain) and then the
// transposed pairs (L > maxL-1-s: factor maxL-1-s transposed), each half
// padded with c = -1 to a multiple of the tile width ncv, then c = -1 up to
// the grid's ymax chunks; plan_cnt[s] is the number of chunks.  One wave per
// step, columns 64 at a time in slot order.  Called by every thread of a
// one-block kernel after that kernel's last change of a column state.
__device__ void build_plan(const IterArgs& a) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  // step maxL: the shifted pair's list (every active column, both halves),
  // kept after the chain steps' lists, at index lcap
  for (int s = threadIdx.x >> 6; s <= a.maxL; s += kFinThreads / 64) {
    const bool spmv = s == a.maxL;
    const int list = spmv ? a.lcap : s;
    const int nv = spmv ? a.ncv_spmv : a.ncv;  // chunk width of this list
    const int fill = spmv ? a.plan_ld : min(a.plan_ld, a.ymax * a.ncv);
    ChainItem* out = a.plan + (int64_t)list * a.plan_ld;
    int pos = 0;
    for (int h = 0; h < 2; ++h) {
      const int jf = h ? a.maxL - 1 - s : s;
      for (int c0 = 0; c0 < a.nc; c0 += 64) {
        const int c = c0 + lane;
        int L = 0;
        bool on = false;
        if (c < a.nc) {
          const ColInfo& ci = a.cols[c];
          L = ci.L;
          on = ci.state == COL_ACTIVE && (spmv || L > jf);
        }
        const unsigned long long m = __ballot(on);
        if (on && spmv) {
          out[pos + __popcll(m & below)] = ChainItem{nullptr, nullptr, nullptr, c, h};
        } else if (on) {
          ChainItem e;
          e.c = c;
          e.flags = h;
          e.fv = a.ftab[((int64_t)(h ? a.cap : 0) + c) * a.lcap + jf];
          if (!h) {
            e.src = jf == 0 ? chain_in(a, c, false) : apply_ptr(a, A_T0 + ((jf - 1) & 1), c);
            e.dst = jf == L - 1 ? apply_ptr(a, A_Z, c) : apply_ptr(a, A_T0 + (jf & 1), c);
          } else {
            const int k = L - 1 - jf;  // transposed factors this column applied before
            e.src = k == 0 ? chain_in(a, c, true) : apply_ptr(a, A_TT0 + ((k - 1) & 1), c);
            e.dst = jf == 0 ? apply_ptr(a, A_ZT, c) : apply_ptr(a, A_TT0 + (k & 1), c);
          }
          out[pos + __popcll(m & below)] = e;
        }
        pos += __popcll(m);
      }
      const int pad = (nv - pos % nv) % nv;
      if (lane < pad) out[pos + lane] = ChainItem{nullptr, nullptr, nullptr, -1, h};
      pos += pad;
      if (h == 0 && lane == 0) a.plan_cnt[a.lcap + 1 + list] = pos / nv;  // forward chunks
    }
    for (int q = pos + lane; q < fill; q += 64) out[q] = ChainItem{nullptr, nullptr, nullptr, -1, 0};
    if (lane == 0) a.plan_cnt[list] = pos / nv;
  }
  __syncthreads();
  // chunk summaries on each chunk's first pair (the same wave per step)
  for (int s = threadIdx.x >> 6; s <= a.maxL; s += kFinThreads / 64) {
    const int list = s == a.maxL ? a.lcap : s;
    const int nv = s == a.maxL ? a.ncv_spmv : a.ncv;
    ChainItem* out = a.plan + (int64_t)list * a.plan_ld;
    const int nch = a.plan_cnt[list];
    for (int q = lane; q < nch; q += 64) {
      ChainItem* ck = out + (int64_t)q * nv;
      const void* f0 = ck[0].fv;
      int ncol = 0;
      bool same = true;
      for (int j = 0; j < nv; ++j)
        if (ck[j].c >= 0) {
          ++ncol;
          same = same && ck[j].fv == f0;
        }
      ck[0].flags = (ck[0].flags & 1) | (same ? 2 : 0) | (ncol << 8);
    }
  }
}

__global__ __launch_bounds__(kFinThreads) void k_plan(IterArgs a) { build_plan(a); }

// convergence test on the residuals of the previous update (or of the start
// of the cycle), the iteration limit, then rho and beta
__global__ __launch_bounds__(kFinThreads) void k_fin_rho(IterArgs a) {
  __shared__ double chain_cols, act_cols, vec_cols, first_cols;
  if (threadIdx.x == 0) chain_cols = act_cols = vec_cols = first_cols = 0.0;
  __syncthreads();
  for (int c = threadIdx.x >> 6; c < a.nc; c += kFinThreads / 64) {
    ColInfo& ci = a.cols[c];
    if (ci.state != COL_ACTIVE) continue;
    double tn[2], tr[2];
    wave_totals<2>(a, a.part_norm, c, tn);
    wave_totals<2>(a, a.part_rho, c, tr);
    const double rr = tn[0], rtrt = tn[1], rho = tr[0], zz = tr[1];
    if ((threadIdx.x & 63) == 0) {
      if (a.trace) {
        atomicAdd(&chain_cols, (double)ci.L);
        atomicAdd(&act_cols, 1.0);
      }
      ci.rr = rr;
      ci.rtrt = rtrt;
      if (passed(ci, rr, rtrt)) {
        ci.state = COL_CONVERGED;
      } else if (ci.it_cycle >= ci.maxit) {
        ci.state = COL_MAXIT;
      } else if (fabs(rho) <= kBreakdown * sqrt(zz) * sqrt(rr)) {
        ci.state = COL_BREAKDOWN;
        ci.broke = 1;
      } else {
        ci.beta = ci.first ? 0.0 : rho / ci.rho_prev;
        ci.rho = rho;
        if (a.trace) {
          atomicAdd(&vec_cols, 1.0);
          if (ci.first) atomicAdd(&first_cols, 1.0);
        }
      }
    }
  }
  if (!a.trace) return;
  __syncthreads();
  if (threadIdx.x == 0) {
    // algorithmic bytes of this iteration's chain launches and of spmv_pair
    const double n = (double)a.n, nnz = (double)a.nnzS;
    const double mat = (double)(a.vbytes + 4) * nnz + 4.0 * (n + 1.0);
    const double ab = (double)a.abytes;
    if (chain_cols > 0.0) {
      // maxL factor passes per direction; per (column, factor, direction) one
      // n-vector read and one written; r read once per column for rho
      a.trace[TR_CHAIN] += 2.0 * a.maxL * mat + 2.0 * 2.0 * ab * n * chain_cols + 8.0 * n * act_cols;
    }
    if (vec_cols > 0.0) {
      // both operator passes (values, 4-byte indices, row offsets), e read;
      // per column p, p~ read and q, q~ written
      const double amat = 2.0 * (12.0 * nnz + 4.0 * (n + 1.0)) + 8.0 * n;
      a.trace[TR_SPMV] += amat + 32.0 * n * vec_cols;
      // form_p: z, z~ read; p, p~ of the last step read (not on a cycle's
      // first step); p, p~ written
      a.trace[TR_FORMP] += (2.0 * ab + 32.0) * n * vec_cols - 16.0 * n * first_cols;
    }
  }
}

// p = z + beta p_old, p~ = z~ + beta p~_old (p = z on a cycle's first
// step), formed once per row so that the shifted products gather p itself
// (and the partial sums of ||p~||^2, slot 1 of the delta partials)
template <typename AT>
__global__ __launch_bounds__(kBlock) void k_form_p(IterArgs a, int par) {
  const WaveCtx t = wave_ctx(a);
  const int c = blockIdx.y;
  const ColInfo& ci = a.cols[c];
  if (ci.state != COL_ACTIVE) return;
  const double beta = ci.beta;
  const bool first = ci.first != 0;
  const AT* z = aptr<AT>(a, A_Z, c);
  const AT* zt = aptr<AT>(a, A_ZT, c);
  const double* po = vptr(a, V_P0 + (par ^ 1), c);
  const double* pto = vptr(a, V_PT0 + (par ^ 1), c);
  double* pn = vptr(a, V_P0 + par, c);
  double* ptn = vptr(a, V_PT0 + par, c);
  double v[1][1] = {{0.0}};
  for (int64_t sl = t.s_begin; sl < t.s_end; ++sl) {
    const int64_t i = sl * kSlice + t.lane;
    if (i >= a.n) continue;
    const double zi = (double)z[i], zti = (double)zt[i];
    pn[i] = first ? zi : fma(beta, po[i], zi);
    const double pti = first ? zti : fma(beta, pto[i], zti);
    ptn[i] = pti;
    v[0][0] = fma(pti, pti, v[0][0]);
  }
  block_partials<1, 1>(a, t, c, 1u, v, a.part_delta + (int64_t)a.cap * a.nblk);
}

// q = (sigma E - A) p, q~ = (sigma E - A)^T p~, partial sums of
// delta = p~^T q and ||q||^2
template <int NC>
__global__ __launch_bounds__(kBlock) void k_spmv_pair(IterArgs a, int par) {
  constexpr int kU = ChunkLen<NC>::value;
  const WaveCtx t = wave_ctx(a);
  const int c0 = blockIdx.y * NC;
  unsigned valid = 0;
  double sig[NC];
  const double *p[NC], *pt[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int c = min(c0 + j, a.nc - 1);
    const ColInfo& ci = a.cols[c];
    if (c0 + j < a.nc && ci.state == COL_ACTIVE) valid |= 1u << j;
    sig[j] = ci.sigma;
    p[j] = vptr(a, V_P0 + par, c);
    pt[j] = vptr(a, V_PT0 + par, c);
  }
  // valid is the same for the whole block; columns past the batch read the
  // last column's vectors and their results are dropped
  if (!valid) return;
  double v[NC][2];
#pragma unroll
  for (int j = 0; j < NC; ++j) v[j][0] = v[j][1] = 0.0;
  for (int64_t sl = t.s_begin; sl < t.s_end; ++sl) {
    const int64_t i = sl * kSlice + t.lane;
    double acc[NC], acct[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] = acct[j] = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int32_t* off = h ? a.offT : a.off;
      const int32_t* col = h ? a.colT : a.col;
      const double* val = h ? a.valAT : a.valA;
      const int32_t base = gld(off + sl);
      const int32_t w = (gld(off + sl + 1) - base) >> 6;
      const int32_t p0 = base + t.lane;
      int32_t nix[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) nix[u] = gld(col + p0 + (u < w ? u * kSlice : 0));
      for (int32_t m0 = 0; m0 < w; m0 += kU) {
        int32_t cix[kU];
        double vv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const bool ok = m0 + u < w;
          const int32_t pp = p0 + (ok ? (m0 + u) * kSlice : 0);
          cix[u] = nix[u];
          const double raw = gld(val + pp);
          vv[u] = ok ? raw : 0.0;
        }
        if (m0 + kU < w) {
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int32_t mn = m0 + kU + u;
            nix[u] = gld(col + p0 + (mn < w ? mn * kSlice : 0));
          }
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const double* pv = h ? pt[j] : p[j];
          double sacc = h ? acct[j] : acc[j];
#pragma unroll
          for (int u = 0; u < kU; ++u) sacc = fma(vv[u], gld(pv + cix[u]), sacc);
          if (h) acct[j] = sacc;
          else acc[j] = sacc;
        }
      }
    }
    if (i < a.n) {
      const double ei = gld(a.e + i);
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (valid & (1u << j)) {
          const int c = c0 + j;
          const double pi = gld(p[j] + i);
          const double pti = gld(pt[j] + i);
          const double se = sig[j] * ei;
          const double qi = fma(se, pi, -acc[j]);
          const double qti = fma(se, pti, -acct[j]);
          gst(vptr(a, V_Q, c) + i, qi);
          gst(vptr(a, V_QT, c) + i, qti);
          v[j][0] = fma(pti, qi, v[j][0]);
          v[j][1] = fma(qi, qi, v[j][1]);
        }
    }
  }
  // delta and ||q||^2 in slots 0 and 2 (form_p fills slot 1 with ||p~||^2)
  block_partials<NC, 2, 2>(a, t, c0, valid, v, a.part_delta);
}

__global__ __launch_bounds__(kFinThreads) void k_fin_delta(IterArgs a) {
  __shared__ double upd_cols;
  if (threadIdx.x == 0) upd_cols = 0.0;
  __syncthreads();
  for (int c = threadIdx.x >> 6; c < a.nc; c += kFinThreads / 64) {
    ColInfo& ci = a.cols[c];
    if (ci.state != COL_ACTIVE) continue;
    double td[3];
    wave_totals<3>(a, a.part_delta, c, td);
    const double delta = td[0], pp = td[1], qq = td[2];
    if ((threadIdx.x & 63) == 0) {
      if (fabs(delta) <= kBreakdown * sqrt(pp) * sqrt(qq)) {
        ci.state = COL_BREAKDOWN;
        ci.broke = 1;
      } else {
        ci.delta = delta;
        ci.alpha = ci.rho / delta;
        ci.it_cycle += 1;
        ci.iters += 1;
        ci.rho_prev = ci.rho;
        ci.first = 0;
        if (a.trace) atomicAdd(&upd_cols, 1.0);
      }
    }
  }
  __syncthreads();
  build_plan(a);  // chain steps of the next iteration
  if (!a.trace) return;
  // x, x~, r, r~ read and written, p, p~, q, q~ read (+ the FP32 copies of r, r~)
  const double rcopy = a.abytes == 4 ? 8.0 : 0.0;
  if (threadIdx.x == 0) a.trace[TR_UPDATE] += (96.0 + rcopy) * (double)a.n * upd_cols;
}

// x += alpha p, x~ += alpha p~, r -= alpha q, r~ -= alpha q~; partial norms
template <int NC>
__global__ __launch_bounds__(kBlock) void k_update(IterArgs a, int par) {
  const WaveCtx t = wave_ctx(a);
  const int c0 = blockIdx.y * NC;
  unsigned valid = 0;
  double al[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int c = min(c0 + j, a.nc - 1);
    if (c0 + j < a.nc && a.cols[c].state == COL_ACTIVE) valid |= 1u << j;
    al[j] = a.cols[c].alpha;
  }
  double v[NC][2];
#pragma unroll
  for (int j = 0; j < NC; ++j) v[j][0] = v[j][1] = 0.0;
  for (int64_t sl = t.s_begin; sl < t.s_end; ++sl) {
    const int64_t i = sl * kSlice + t.lane;
    if (i >= a.n) continue;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (!(valid & (1u << j))) continue;
      const int c = c0 + j;
      double* x = vptr(a, V_X, c);
      double* xt = vptr(a, V_XT, c);
      double* r = vptr(a, V_R, c);
      double* rt = vptr(a, V_RT, c);
      x[i] = fma(al[j], vptr(a, V_P0 + par, c)[i], x[i]);
      xt[i] = fma(al[j], vptr(a, V_PT0 + par, c)[i], xt[i]);
      const double ri = fma(-al[j], vptr(a, V_Q, c)[i], r[i]);
      const double rti = fma(-al[j], vptr(a, V_QT, c)[i], rt[i]);
      r[i] = ri;
      rt[i] = rti;
      store_rcopy(a, c, i, ri, rti);
      v[j][0] = fma(ri, ri, v[j][0]);
      v[j][1] = fma(rti, rti, v[j][1]);
    }
  }
  block_partials<NC, 2>(a, t, c0, valid, v, a.part_norm);
}

// true residuals r = b - A_s x, r~ = c - A_s^T x~ of the columns that stopped
template <int NC>
__global__ __launch_bounds__(kBlock) void k_true_residual(IterArgs a) {
  const WaveCtx t = wave_ctx(a);
  const int c0 = blockIdx.y * NC;
  unsigned valid = 0;
#pragma unroll
  for (int j = 0; j < NC; ++j)
    if (c0 + j < a.nc && stopped(a.cols[c0 + j].state)) valid |= 1u << j;
  double v[NC][2];
#pragma unroll
  for (int j = 0; j < NC; ++j) v[j][0] = v[j][1] = 0.0;
  if (valid) {
    for (int64_t sl = t.s_begin; sl < t.s_end; ++sl) {
      const int64_t i = sl * kSlice + t.lane;
      double acc[NC], acct[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) acc[j] = acct[j] = 0.0;
      {
        const int32_t base = a.off[sl];
        const int32_t w = (a.off[sl + 1] - base) >> 6;
        for (int32_t m0 = 0; m0 < w; m0 += kUnroll) {
          SliceChunk ch;
          double vv[kUnroll];
          load_chunk<double>(a.col, a.valA, base + t.lane, w, m0, ch, vv);
#pragma unroll
          for (int j = 0; j < NC; ++j)
            if (valid & (1u << j)) acc[j] = chunk_dot(ch, vv, m0, w, vptr(a, V_X, c0 + j), acc[j]);
        }
      }
      {
        const int32_t base = a.offT[sl];
        const int32_t w = (a.offT[sl + 1] - base) >> 6;
        for (int32_t m0 = 0; m0 < w; m0 += kUnroll) {
          SliceChunk ch;
          double vv[kUnroll];
          load_chunk<double>(a.colT, a.valAT, base + t.lane, w, m0, ch, vv);
#pragma unroll
          for (int j = 0; j < NC; ++j)
            if (valid & (1u << j)) acct[j] = chunk_dot(ch, vv, m0, w, vptr(a, V_XT, c0 + j), acct[j]);
        }
      }
      if (i >= a.n) continue;
      const double ei = a.e[i];
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (valid & (1u << j)) {
          const int c = c0 + j;
          const ColInfo& ci = a.cols[c];
          const double se = ci.sigma * ei;
          // b - (sigma E x - A x)
          const double ri = ci.bsrc[i] - fma(se, vptr(a, V_X, c)[i], -acc[j]);
          const double rti = ci.csrc[i] - fma(se, vptr(a, V_XT, c)[i], -acct[j]);
          vptr(a, V_R, c)[i] = ri;
          vptr(a, V_RT, c)[i] = rti;
          store_rcopy(a, c, i, ri, rti);
          v[j][0] = fma(ri, ri, v[j][0]);
          v[j][1] = fma(rti, rti, v[j][1]);
        }
    }
  }
  block_partials<NC, 2>(a, t, c0, valid, v, a.part_norm);
}

// accept, restart from the current iterates (true residuals are in r, r~ and
// their norms in the norm partials, read by the next fin_rho), or give up
__global__ __launch_bounds__(kFinThreads) void k_fin_true(IterArgs a) {
  for (int c = threadIdx.x >> 6; c < a.nc; c += kFinThreads / 64) {
    ColInfo& ci = a.cols[c];
    const int st = ci.state;
    if (!stopped(st)) continue;
    double tn[2];
    wave_totals<2>(a, a.part_norm, c, tn);
    const double rr = tn[0], rtrt = tn[1];
    if ((threadIdx.x & 63) == 0) {
      ci.rr = rr;
      ci.rtrt = rtrt;
      ci.relp = ci.nb > 0.0 ? sqrt(rr) / ci.nb : sqrt(rr);
      ci.reld = ci.nc > 0.0 ? sqrt(rtrt) / ci.nc : sqrt(rtrt);
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

// copy the iterates of the listed slots to their output columns (or zeros)
struct SlotList {
  int n;
  int s[64];
};

__global__ __launch_bounds__(256) void k_copy_out(IterArgs a, SlotList sl) {
  const int c = sl.s[blockIdx.y];
  const ColInfo& ci = a.cols[c];
  const double* xs = vptr(a, V_X, c);
  const double* ys = vptr(a, V_XT, c);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * 256) {
    if (ci.xout) ci.xout[i] = ci.out_x == 1 ? xs[i] : (ci.out_x == 2 ? ys[i] : 0.0);
    if (ci.yout) ci.yout[i] = ci.out_y == 1 ? xs[i] : (ci.out_y == 2 ? ys[i] : 0.0);
  }
}

// Inputs of a product run outside a solve: column c of X into slot vector
// vf (and its FP32 copy when the apply is FP32), of Xt into vb; missing
// sides are zero
__global__ __launch_bounds__(256) void k_probe_in(IterArgs a, int vf, int vb, const double* X,
                                                  int64_t ldx, const double* Xt, int64_t ldxt,
                                                  int rcopy) {
  const int c = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * 256) {
    const double x = X ? X[(int64_t)c * ldx + i] : 0.0;
    const double xt = Xt ? Xt[(int64_t)c * ldxt + i] : 0.0;
    vptr(a, vf, c)[i] = x;
    vptr(a, vb, c)[i] = xt;
    if (rcopy) store_rcopy(a, c, i, x, xt);
  }
}

// Outputs of such a product: the chain results z, z~ (apply precision,
// widened) when `chain`, else the shifted pair's q, q~
__global__ __launch_bounds__(256) void k_probe_out(IterArgs a, int chain, double* Y, int64_t ldy,
                                                   double* Yt, int64_t ldyt) {
  const int c = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * 256) {
    double y, yt;
    if (!chain) {
      y = vptr(a, V_Q, c)[i];
      yt = vptr(a, V_QT, c)[i];
    } else if (a.abytes == 4) {
      y = (double)aptr<float>(a, A_Z, c)[i];
      yt = (double)aptr<float>(a, A_ZT, c)[i];
    } else {
      y = aptr<double>(a, A_Z, c)[i];
      yt = aptr<double>(a, A_ZT, c)[i];
    }
    if (Y) Y[(int64_t)c * ldy + i] = y;
    if (Yt) Yt[(int64_t)c * ldyt + i] = yt;
  }
}

__global__ void k_zero(double* p, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// column norms of a dense block: partial sums over row slabs, then one wave per column
constexpr int kNormSlabs = 64;
__global__ __launch_bounds__(256) void k_colnorm_part(const double* X, int64_t ld, int64_t n,
                                                      double* part) {
  __shared__ double sh[4];
  const double* x = X + (int64_t)blockIdx.y * ld;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s = fma(x[i], x[i], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(kFinThreads) void k_colnorm_fin(const double* part, int ncol,
                                                             double* out) {
  for (int c = threadIdx.x >> 6; c < ncol; c += kFinThreads / 64) {
    const int lane = threadIdx.x & 63;
    const double v = lane < kNormSlabs ? part[(int64_t)c * kNormSlabs + lane] : 0.0;
    const double s = wave_sum(v);
    if (lane == 0) out[c] = sqrt(s);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// tracing: per-class launch events and algorithmic bytes

struct TraceState {
  bool on = false;
  DevBuf counters;  // double[kTraceClasses]
  struct Pending {
    int cls;
    hipEvent_t a, b;
    int count = 1;  // launches bracketed by the pair
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  double ms[kTraceClasses] = {0};
  int64_t launches[kTraceClasses] = {0};
};

static TraceState* trace_of(morx_ctx ctx) {
  static std::mutex mu;
  static std::vector<std::pair<morx_ctx, TraceState*>> all;
  std::lock_guard<std::mutex> lk(mu);
  for (auto& p : all)
    if (p.first == ctx) return p.second;
  all.push_back({ctx, new TraceState()});
  return all.back().second;
}

static hipEvent_t trace_event(TraceState* t) {
  if (!t->free_events.empty()) {
    hipEvent_t e = t->free_events.back();
    t->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch a kernel; when tracing, through hipExtLaunchKernelGGL so that the
// start and stop events time the dispatch itself (no inter-kernel gap).
template <typename... KArgs, typename... Args>
static void launch(TraceState* t, int cls, void (*kernel)(KArgs...), dim3 g, dim3 b,
                   hipStream_t st, Args... args) {
  if (!t || !t->on) {
    hipLaunchKernelGGL(kernel, g, b, 0, st, args...);
    return;
  }
  hipEvent_t e0 = trace_event(t), e1 = trace_event(t);
  hipExtLaunchKernelGGL(kernel, g, b, 0, st, e0, e1, 0, args...);
  if (e0 && e1) t->pending.push_back({cls, e0, e1, 1});
}

static void trace_collect(TraceState* t) {
  for (auto& p : t->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      t->ms[p.cls] += ms;
      t->launches[p.cls] += p.count;
    }
    t->free_events.push_back(p.a);
    t->free_events.push_back(p.b);
  }
  t->pending.clear();
}

static const char* kTraceNames[kTraceClasses] = {"chain_step", "spmv_pair", "update", "factor_ls",
                                                 "form_p", "", "", ""};

TraceState* trace_state_if_on(morx_ctx ctx) {
  TraceState* t = trace_of(ctx);
  return t->on ? t : nullptr;
}

static double* trace_counters(morx_ctx ctx) {
  TraceState* t = trace_of(ctx);
  return t->on ? (double*)t->counters.p : nullptr;
}

extern "C" morx_status morx_trace_enable(morx_ctx ctx, int32_t enable) {
  MORX_REQUIRE(ctx, MORX_E_INVALID, "morx_trace_enable: null context");
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  TraceState* t = trace_of(ctx);
  if (enable && !t->counters.p) MORX_TRY(dev_alloc(t->counters, kTraceClasses * sizeof(double)));
  if (enable) {
    MORX_HIP(hipStreamSynchronize(ctx->stream));
    k_zero<<<1, 64, 0, ctx->stream>>>((double*)t->counters.p, kTraceClasses);
    MORX_HIP(hipGetLastError());
    MORX_HIP(hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < kTraceClasses; ++c) {
      t->ms[c] = 0.0;
      t->launches[c] = 0;
    }
  }
  t->on = enable != 0;
  return MORX_OK;
}

extern "C" morx_status morx_trace_read(morx_ctx ctx, morx_trace_entry* out, int32_t cap,
                                       int32_t* count) {
  MORX_REQUIRE(ctx && count, MORX_E_INVALID, "morx_trace_read: null argument");
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  TraceState* t = trace_of(ctx);
  double bytes[kTraceClasses] = {0};
  if (t->counters.p) {
    MORX_HIP(hipStreamSynchronize(ctx->stream));
    MORX_HIP(hipMemcpy(bytes, t->counters.p, sizeof(bytes), hipMemcpyDeviceToHost));
  }
  int k = 0;
  for (int c = 0; c < kTraceClasses; ++c) {
    if (!kTraceNames[c][0]) continue;
    if (out && k < cap) {
      memset(&out[k], 0, sizeof(out[k]));
      strncpy(out[k].name, kTraceNames[c], sizeof(out[k].name) - 1);
      out[k].launches = t->launches[c];
      out[k].total_ms = t->ms[c];
      out[k].alg_bytes = bytes[c];
    }
    ++k;
  }
  *count = k;
  return MORX_OK;
}

// factor construction launches are traced from factor.hip through these
void trace_factor_begin(morx_ctx ctx, hipStream_t st, void** token) {
  *token = nullptr;
  TraceState* t = trace_state_if_on(ctx);
  if (!t) return;
  hipEvent_t a = trace_event(t);
  if (a) hipEventRecord(a, st);
  *token = a;
}

void trace_factor_end(morx_ctx ctx, hipStream_t st, void* token) {
  TraceState* t = trace_state_if_on(ctx);
  if (!t || !token) return;
  hipEvent_t b = trace_event(t);
  if (!b) return;
  hipEventRecord(b, st);
  t->pending.push_back({TR_FACTOR, (hipEvent_t)token, b, 1});
}

// ---------------------------------------------------------------------------
// host side: the slot batch

void batch_free(KrylovBatch& b) {
  for (auto& g : b.graphs) {
    if (g.x) hipGraphExecDestroy(g.x);
    if (g.g) hipGraphDestroy(g.g);
  }
  b.graphs.clear();
  dev_free(b.vec);
  dev_free(b.avec);
  dev_free(b.cols);
  dev_free(b.part);
  dev_free(b.ftab);
  dev_free(b.plan);
  if (b.hcols) hipHostFree(b.hcols);
  if (b.hftab) hipHostFree(b.hftab);
  b.hcols = nullptr;
  b.hftab = nullptr;
  b.cap = b.lcap = 0;
}

void krylov_batch_delete(KrylovBatch* kb) {
  if (!kb) return;
  batch_free(*kb);
  delete kb;
}

// work-list entries per chain step: both halves, each padded to the tile width
static int plan_ld(int cap) { return 2 * cap + 2 * kMaxNC; }
// lcap chain-step lists and the shifted pair's, then their chunk counts
static size_t plan_bytes(int cap, int lcap) {
  return (size_t)(lcap + 1) * plan_ld(cap) * sizeof(ChainItem) +
         2 * (size_t)(lcap + 1) * sizeof(int32_t);
}

size_t batch_bytes(morx_system sys, int cap, int aprec) {
  const size_t ld = (size_t)sys->n_pad;
  return (size_t)kNumVec * cap * ld * sizeof(double) +
         (size_t)apply_vecs(aprec) * cap * ld * prec_bytes(aprec) +
         (size_t)8 * cap * kMaxBlocks * sizeof(double) + plan_bytes(cap, 64);
}

morx_status batch_alloc(KrylovBatch& b, morx_system sys, int cap, int lcap, int prec, int aprec,
                        hipStream_t st) {
  batch_free(b);
  b.sys = sys;
  b.cap = cap;
  b.lcap = lcap;
  b.prec = prec;
  b.aprec = aprec;
  b.ld = sys->n_pad;
  morx_status s = dev_alloc(b.vec, (size_t)kNumVec * cap * b.ld * sizeof(double));
  if (s == MORX_OK)
    s = dev_alloc(b.avec, (size_t)apply_vecs(aprec) * cap * b.ld * prec_bytes(aprec));
  if (s == MORX_OK) s = dev_alloc(b.cols, (size_t)cap * sizeof(ColInfo));
  if (s == MORX_OK) s = dev_alloc(b.part, (size_t)8 * cap * kMaxBlocks * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(b.ftab, (size_t)2 * cap * lcap * sizeof(void*));
  if (s == MORX_OK) s = dev_alloc(b.plan, plan_bytes(cap, lcap));
  if (s == MORX_OK && hipHostMalloc((void**)&b.hcols, (size_t)cap * sizeof(ColInfo)) != hipSuccess)
    s = MORX_E_NOMEM;
  if (s == MORX_OK &&
      hipHostMalloc((void**)&b.hftab, (size_t)2 * cap * lcap * sizeof(void*)) != hipSuccess)
    s = MORX_E_NOMEM;
  if (s != MORX_OK) {
    batch_free(b);
    morx_set_error("BiCG slot allocation failed (%d slots)", cap);
    return MORX_E_NOMEM;
  }
  for (int c = 0; c < cap; ++c) {
    ColInfo ci = {};
    ci.state = COL_IDLE;
    b.hcols[c] = ci;
  }
  memset(b.hftab, 0, (size_t)2 * cap * lcap * sizeof(void*));
  const int64_t cnt = (int64_t)(b.vec.bytes / sizeof(double));
  k_zero<<<(unsigned)((cnt + 255) / 256), 256, 0, st>>>((double*)b.vec.p, cnt);
  const int64_t acnt = (int64_t)(b.avec.bytes / sizeof(double));
  k_zero<<<(unsigned)((acnt + 255) / 256), 256, 0, st>>>((double*)b.avec.p, acnt);
  MORX_HIP(hipGetLastError());
  MORX_HIP(hipMemcpyAsync(b.cols.p, b.hcols, (size_t)cap * sizeof(ColInfo), hipMemcpyHostToDevice, st));
  MORX_HIP(hipMemcpyAsync(b.ftab.p, b.hftab, (size_t)2 * cap * lcap * sizeof(void*),
                          hipMemcpyHostToDevice, st));
  return MORX_OK;
}

morx_status batch_upload(KrylovBatch& b, int first, int count, hipStream_t st) {
  if (count <= 0) return MORX_OK;
  MORX_HIP(hipMemcpyAsync((ColInfo*)b.cols.p + first, b.hcols + first, count * sizeof(ColInfo),
                          hipMemcpyHostToDevice, st));
  for (int h = 0; h < 2; ++h) {
    const size_t off = ((size_t)h * b.cap + first) * b.lcap;
    MORX_HIP(hipMemcpyAsync((void**)b.ftab.p + off, b.hftab + off, (size_t)count * b.lcap * sizeof(void*),
                            hipMemcpyHostToDevice, st));
  }
  return MORX_OK;
}

morx_status batch_download(KrylovBatch& b, hipStream_t st) {
  MORX_HIP(hipMemcpyAsync(b.hcols, b.cols.p, (size_t)b.cap * sizeof(ColInfo), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipStreamSynchronize(st));
  return MORX_OK;
}

// columns per wave: the batch split into equal chunks of at most ncmax,
// rounded up to an instantiated tile width (1..8, 10, 12, 16; the extra
// columns of a chunk are past the batch and masked)
static int pick_nc(int nc, int ncmax) {
  const int chunks = (nc + ncmax - 1) / ncmax;
  const int w = (nc + chunks - 1) / chunks;
  return w <= 8 ? w : (w <= 10 ? 10 : (w <= 12 ? 12 : 16));
}

// whether both orders of the pattern carry a halo layout the chain step can
// take: lists of at most kHaloCap entries, or kHaloCapNarrow for patterns of
// at most kNarrow slots (their halo kernel keeps fewer slots and list entries)
static bool pattern_narrow(morx_system sys) {
  return std::max(sys->sell.max_width, sys->sellT.max_width) <= kNarrow;
}
static bool halo_available(morx_system sys) {
  if (sys->sell.hmax <= 0 || sys->sellT.hmax <= 0) return false;
  return !pattern_narrow(sys) || std::max(sys->sell.hmax, sys->sellT.hmax) <= kHaloCapNarrow;
}
// the chain step runs on the halo layout: by default for wide patterns, on
// request (chain_kernel 1) for narrow ones
static bool halo_in_use(morx_system sys) {
  if (!halo_available(sys)) return false;
  return sys->tune_chain == 1 || (sys->tune_chain == -1 && !pattern_narrow(sys));
}

static IterArgs make_args(KrylovBatch& b, int nc, int maxL) {
  morx_system sys = b.sys;
  IterArgs a;
  a.n = sys->n;
  a.ld = b.ld;
  a.nnzS = sys->nnzS;
  a.nslices = sys->nslice;
  a.cap = b.cap;
  a.nc = nc;
  // slices per wave: as few as the partial-sum budget allows (or the tuned
  // value); blocks: a multiple of 8 for the XCD remap
  const int64_t per_blk_min = (a.nslices + kMaxBlocks - 1) / kMaxBlocks;
  a.spw = (int)std::max<int64_t>(1, (per_blk_min + kWavesPerBlock - 1) / kWavesPerBlock);
  if (sys->tune_spw > 0) a.spw = std::max(a.spw, (int)sys->tune_spw);
  a.ncmax = sys->tune_nc > 0 ? (int)sys->tune_nc : kDefaultNC;
  a.ncmax_spmv = sys->tune_nc_spmv > 0 ? (int)sys->tune_nc_spmv : a.ncmax;
  a.ncv = pick_nc(nc, a.ncmax);
  // the shifted pair's tile on the halo layout: A is read once per chunk of
  // columns, and a chunk's staged vectors share the L2 (the autotuner weighs
  // the two)
  a.ncv_spmv = pick_nc(nc, a.ncmax_spmv);
  // chain grid: the most chunks of (half, column) pairs any step has, from
  // the chain lengths of the occupied slots; a batch whose slots change
  // between segments (serving) takes the bound for nc columns instead, so
  // its graphs do not depend on the mix
  int ymax = 2 * ((nc + a.ncv - 1) / a.ncv);
  if (b.profile_grid) {
    ymax = 1;
    for (int s = 0; s < maxL; ++s) {
      int f = 0, r = 0;
      for (int c = 0; c < nc; ++c) {
        const ColInfo& ci = b.hcols[c];
        if (ci.state == COL_IDLE) continue;
        f += ci.L > s;
        r += ci.L > maxL - 1 - s;
      }
      ymax = std::max(ymax, (f + a.ncv - 1) / a.ncv + (r + a.ncv - 1) / a.ncv);
    }
  }
  a.ymax = ymax;
  a.plan_ld = plan_ld(b.cap);
  int64_t nb = (a.nslices + (int64_t)kWavesPerBlock * a.spw - 1) / ((int64_t)kWavesPerBlock * a.spw);
  nb = std::max<int64_t>(8, (nb + 7) / 8 * 8);
  a.nblk = (int)nb;
  a.vbytes = (int)prec_bytes(b.prec);
  a.maxL = maxL;
  a.lcap = b.lcap;
  a.off = sys->sell.off;
  a.col = sys->sell.col;
  a.nsell = sys->sell.nnz_sell;
  a.nsellT = sys->sellT.nnz_sell;
  a.narrow = std::max(sys->sell.max_width, sys->sellT.max_width) <= kNarrow;
  a.hmax = halo_in_use(sys) ? std::max(sys->sell.hmax, sys->sellT.hmax) : 0;
  // strided row blocks when the groups of hstride * spw row blocks tile the
  // pattern exactly (the grid's blocks then cover every row block once)
  {
    const int64_t nrb = (a.nslices + kHaloSlices - 1) / kHaloSlices;
    const int64_t S = sys->sell.hstride;
    a.hstride = (S > 1 && nrb % (S * a.spw) == 0 && nrb / a.spw == a.nblk) ? (int)S : 1;
    // the chain steps before an iteration's last form no partial sums, so
    // their grid is not bound by the partial-sum budget: one slice per wave,
    // the most workgroups, so that the last round of resident workgroups
    // leaves little of the chip idle (27-point job: 1,024 workgroups in 1.3
    // rounds of the 768 resident, 272 us per launch; 8,192 workgroups, 254 us)
    a.spw_chain = 1;
    int64_t nbc = (a.nslices + (int64_t)kWavesPerBlock * a.spw_chain - 1) /
                  ((int64_t)kWavesPerBlock * a.spw_chain);
    nbc = std::max<int64_t>(8, (nbc + 7) / 8 * 8);
    a.nblk_chain = (int)nbc;
    a.hstride_chain = (S > 1 && nrb % (S * a.spw_chain) == 0 && nrb / a.spw_chain == nbc) ? (int)S : 1;
  }
  a.hoff = sys->sell.hoff;
  a.hcol = sys->sell.hcol;
  a.lidx = sys->sell.lidx;
  a.hoffT = sys->sellT.hoff;
  a.hcolT = sys->sellT.hcol;
  a.hrun = sys->sell.hrun;
  a.hrunT = sys->sellT.hrun;
  a.lidxT = sys->sellT.lidx;
  a.offT = sys->sellT.off;
  a.colT = sys->sellT.col;
  a.valA = sys->sell_val;
  a.valAT = sys->sellT_val;
  a.e = sys->e;
  a.vec = (double*)b.vec.p;
  a.avec = b.avec.p;
  a.abytes = (int)prec_bytes(b.aprec);
  a.cols = (ColInfo*)b.cols.p;
  a.ftab = (const void* const*)b.ftab.p;
  double* part = (double*)b.part.p;
  const int64_t slab = (int64_t)b.cap * kMaxBlocks;
  a.part_rho = part;
  a.part_delta = part + 3 * slab;
  a.part_norm = part + 6 * slab;
  a.trace = trace_counters(sys->ctx);
  a.plan = (ChainItem*)b.plan.p;
  a.plan_cnt = (int32_t*)((ChainItem*)b.plan.p + (size_t)(b.lcap + 1) * a.plan_ld);
  return a;
}

static dim3 grid_of(const IterArgs& a, int ncv, int halves) {
  return dim3((unsigned)a.nblk, (unsigned)((a.nc + ncv - 1) / ncv), (unsigned)halves);
}

// The maxL chain launches of an iteration run back to back; when tracing, one
// event pair brackets the whole run and counts maxL launches, so the event
// overhead is spread over the run instead of added to every launch.
static void enqueue_chain(const IterArgs& a, int prec, hipStream_t st, TraceState* t) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (t) {
    e0 = trace_event(t);
    e1 = trace_event(t);
    if (e0) hipEventRecord(e0, st);
  }
  if (prec == MORX_F64) chain_launch_f64(a, st);
  else if (prec == MORX_F32) chain_launch_f32(a, st);
  else chain_launch_bf16(a, st);
  if (t && e0 && e1) {
    hipEventRecord(e1, st);
    t->pending.push_back({TR_CHAIN, e0, e1, a.maxL});
  }
}

// q = A_s p, q~ = A_s^T p~ of an iteration (p in the parity-`par` slots):
// on the halo layout the chain step's kernel in its shifted-pair form (tile
// of the chain step), else the row-gather kernel
static void enqueue_spmv(const IterArgs& a, int par, hipStream_t st, TraceState* t) {
  if (a.hmax > 0) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (t) {
      e0 = trace_event(t);
      e1 = trace_event(t);
      if (e0) hipEventRecord(e0, st);
    }
    spmv_halo_launch(a, par, st);
    if (t && e0 && e1) {
      hipEventRecord(e1, st);
      t->pending.push_back({TR_SPMV, e0, e1, 1});
    }
    return;
  }
  const int ncs = pick_nc(a.nc, a.ncmax_spmv);
  MORX_NC_DISPATCH(ncs, {
    launch(t, TR_SPMV, k_spmv_pair<NC>, grid_of(a, NC, 1), dim3(kBlock), st, a, par);
  });
}

static morx_status enqueue_iterations(const IterArgs& a, int prec, int iters, hipStream_t st,
                                      TraceState* t) {
  const bool f32 = a.abytes == 4;
  // the first iteration's work lists (fin_delta writes the later ones)
  k_plan<<<1, kFinThreads, 0, st>>>(a);
  for (int it = 0; it < iters; ++it) {
    const int par = it & 1;
    enqueue_chain(a, prec, st, t);
    k_fin_rho<<<1, kFinThreads, 0, st>>>(a);
    if (f32) launch(t, TR_FORMP, k_form_p<float>, grid_of(a, 1, 1), dim3(kBlock), st, a, par);
    else launch(t, TR_FORMP, k_form_p<double>, grid_of(a, 1, 1), dim3(kBlock), st, a, par);
    enqueue_spmv(a, par, st, t);
    k_fin_delta<<<1, kFinThreads, 0, st>>>(a);
    // elementwise: one column per wave, nothing to share between columns
    launch(t, TR_UPDATE, k_update<1>, grid_of(a, 1, 1), dim3(kBlock), st, a, par);
  }
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

morx_status batch_launch_init(KrylovBatch& b, int nc, hipStream_t st) {
  const IterArgs a = make_args(b, nc, 1);
  k_init<1><<<grid_of(a, 1, 1), kBlock, 0, st>>>(a);
  k_fin_init<<<1, kFinThreads, 0, st>>>(a);
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

morx_status batch_launch_true(KrylovBatch& b, int nc, hipStream_t st) {
  const IterArgs a = make_args(b, nc, 1);
  MORX_NC_DISPATCH(pick_nc(nc, a.ncmax_spmv),
                   k_true_residual<NC><<<grid_of(a, NC, 1), kBlock, 0, st>>>(a));
  k_fin_true<<<1, kFinThreads, 0, st>>>(a);
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

morx_status batch_launch_copy_out(KrylovBatch& b, const int* slots, int count, hipStream_t st) {
  const IterArgs a = make_args(b, b.cap, 1);
  for (int k0 = 0; k0 < count; k0 += 64) {
    SlotList sl;
    sl.n = std::min(64, count - k0);
    for (int k = 0; k < sl.n; ++k) sl.s[k] = slots[k0 + k];
    k_copy_out<<<dim3((unsigned)std::min<int64_t>((a.n + 255) / 256, 1024), sl.n, 1), 256, 0, st>>>(a, sl);
  }
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

// one segment of `iters` iterations; graphs are cached per (nc, maxL, iters)
// and launch shape
morx_status batch_launch_segment(KrylovBatch& b, int nc, int maxL, int iters, bool use_graph,
                                 hipStream_t st, TraceState* t) {
  const IterArgs a = make_args(b, nc, maxL);
  if (!use_graph || t) return enqueue_iterations(a, b.prec, iters, st, t);
  const int64_t key =
      ((((((int64_t)iters * 1024 + nc) * 128 + a.spw) * 16 + a.ncmax) * 16 + a.ncmax_spmv) * 4096 +
       a.ymax) * 2 + (a.hmax > 0);
  for (auto& g : b.graphs)
    if (g.maxL == maxL && g.key == key) {
      MORX_HIP(hipGraphLaunch(g.x, st));
      return MORX_OK;
    }
  if (b.graphs.size() >= 24) {
    hipGraphExecDestroy(b.graphs.front().x);
    hipGraphDestroy(b.graphs.front().g);
    b.graphs.erase(b.graphs.begin());
  }
  MORX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  morx_status s = enqueue_iterations(a, b.prec, iters, st, nullptr);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  MORX_TRY(s);
  MORX_REQUIRE(e == hipSuccess, MORX_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    morx_set_error("graph instantiation failed: %s", hipGetErrorString(e));
    return MORX_E_HIP;
  }
  b.graphs.push_back({maxL, key, g, x});
  MORX_HIP(hipGraphLaunch(x, st));
  return MORX_OK;
}

void trace_collect_pending(TraceState* t) {
  if (t) trace_collect(t);
}

struct BatchCol {
  double sigma;
  int L;
  const std::vector<morx_factor>* chain;  // factors applied first to last (L of them)
  const double* b;
  const double* c;
  double* xout;
  double* yout;
  int check_p, check_d, out_x, out_y;
  morx_col_stats* stats;
};

// Solve a set of columns, each preconditioned by its own factor chain (in a
// batched multi-shift solve the chains are prefixes of one factor list, so
// the chain step shares every factor load among the columns of a wave).
static morx_status solve_batch(morx_system sys, std::vector<BatchCol>& cols, int prec,
                               const morx_opts& o, hipStream_t st) {
  const int aprec = o.apply_prec;
  const int nc = (int)cols.size();
  if (nc == 0) return MORX_OK;
  int maxL = 0;
  for (auto& c : cols) {
    MORX_REQUIRE(c.chain && c.L >= 1 && c.L <= (int)c.chain->size(), MORX_E_INVALID,
                 "bad chain length");
    maxL = std::max(maxL, c.L);
  }
  if (!sys->kb) sys->kb = new KrylovBatch();
  KrylovBatch& b = *sys->kb;
  b.profile_grid = true;
  if (b.cap < nc || b.lcap < maxL || b.prec != prec || b.aprec != aprec || b.ld != sys->n_pad) {
    MORX_HIP(hipStreamSynchronize(st));
    MORX_TRY(batch_alloc(b, sys, std::max(nc, b.cap), std::max(maxL, b.lcap), prec, aprec, st));
  }
  TraceState* t = trace_state_if_on(sys->ctx);
  const int maxit = o.maxit > 0 ? o.maxit : (int)std::min<int64_t>(sys->n, 20000);
  for (int c = 0; c < nc; ++c) {
    ColInfo ci = {};
    ci.sigma = cols[c].sigma;
    ci.tol = o.tol;
    ci.bsrc = cols[c].b;
    ci.csrc = cols[c].c;
    ci.xout = cols[c].xout;
    ci.yout = cols[c].yout;
    ci.state = COL_INIT;
    ci.L = cols[c].L;
    ci.first = 1;
    ci.max_restarts = o.max_restarts;
    ci.maxit = maxit;
    ci.check_p = cols[c].check_p;
    ci.check_d = cols[c].check_d;
    ci.out_x = cols[c].out_x;
    ci.out_y = cols[c].out_y;
    ci.status = MORX_E_NOT_CONVERGED;
    b.hcols[c] = ci;
    for (int s = 0; s < b.lcap; ++s) {
      const bool in = s < cols[c].L;
      b.hftab[(size_t)c * b.lcap + s] = in ? (*cols[c].chain)[s]->vals.p : nullptr;
      b.hftab[((size_t)b.cap + c) * b.lcap + s] = in ? (*cols[c].chain)[s]->valsT.p : nullptr;
    }
  }
  MORX_TRY(batch_upload(b, 0, nc, st));
  MORX_TRY(batch_launch_init(b, nc, st));

  int seg = std::max(2, o.poll_iters > 0 ? o.poll_iters : 8);
  seg += seg & 1;  // even: the p buffers alternate by iteration parity
  const int64_t guard_max = 2 * ((int64_t)(o.max_restarts + 1) * (maxit + seg) / seg + 4);
  for (int64_t guard = 0; guard <= guard_max; ++guard) {
    MORX_TRY(batch_download(b, st));
    if (t) trace_collect(t);
    int active = 0, stop = 0;
    for (int c = 0; c < nc; ++c) {
      const int s = b.hcols[c].state;
      if (s == COL_ACTIVE) ++active;
      else if (s == COL_CONVERGED || s == COL_BREAKDOWN || s == COL_MAXIT) ++stop;
    }
    if (active == 0 && stop == 0) break;
    if (active == 0) {
      MORX_TRY(batch_launch_true(b, nc, st));
      continue;
    }
    MORX_TRY(batch_launch_segment(b, nc, maxL, seg, o.use_graph != 0, st, t));
  }
  std::vector<int> all(nc);
  for (int c = 0; c < nc; ++c) all[c] = c;
  MORX_TRY(batch_launch_copy_out(b, all.data(), nc, st));
  MORX_TRY(batch_download(b, st));
  if (t) trace_collect(t);
  for (int c = 0; c < nc; ++c) {
    ColInfo& ci = b.hcols[c];
    morx_col_stats* out = cols[c].stats;
    if (out) {
      out->status = ci.state == COL_DONE ? MORX_OK
                                         : (ci.state == COL_FAILED ? ci.status : MORX_E_NOT_CONVERGED);
      out->iters = ci.iters;
      out->restarts = ci.restarts;
      out->relres_primal = cols[c].out_x == 2 ? ci.reld : (cols[c].out_x == 1 ? ci.relp : 0.0);
      out->relres_dual = cols[c].out_y == 2 ? ci.reld : (cols[c].out_y == 1 ? ci.relp : 0.0);
    }
    ci.state = COL_IDLE;
  }
  return batch_upload(b, 0, nc, st);
}

// ---------------------------------------------------------------------------
// morx_solve_shifts: Algorithm 4's factor schedule around the batched solver

static int worse(int a, int b) {
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

static morx_status rhs_norms(morx_system sys, const double* X, int64_t ld, int m, double* out_host,
                             hipStream_t st) {
  DevBuf part, res;
  MORX_TRY(dev_alloc(part, (size_t)m * kNormSlabs * sizeof(double)));
  morx_status s = dev_alloc(res, (size_t)m * sizeof(double));
  if (s == MORX_OK) {
    k_colnorm_part<<<dim3(kNormSlabs, m), 256, 0, st>>>(X, ld, sys->n, (double*)part.p);
    k_colnorm_fin<<<1, kFinThreads, 0, st>>>((double*)part.p, m, (double*)res.p);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(out_host, res.p, m * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      morx_set_error("norms: %s", hipGetErrorString(e));
      s = MORX_E_HIP;
    }
  }
  dev_free(part);
  dev_free(res);
  return s;
}

namespace {

// out[:, c] = e .* in[:, c] for ncol columns (the next moment's right-hand side)
__global__ __launch_bounds__(256) void k_scale_cols(const double* __restrict__ e,
                                                    const double* __restrict__ in, int64_t ldi,
                                                    double* __restrict__ out, int64_t ldo,
                                                    int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t c = blockIdx.y;
  out[c * ldo + i] = e[i] * in[c * ldi + i];
}

}  // namespace

// One column pair of a solve: how it runs follows from its right-hand-side
// norms (a zero primal side runs the transposed system as the shadow
// recurrence; a missing or zero dual side uses b as the shadow right-hand side).
static BatchCol pair_col(double sigma, const std::vector<morx_factor>* chain, const double* b,
                         const double* c, double nb, double nc, bool want_dual, double* xout,
                         double* yout, morx_col_stats* st) {
  BatchCol bc{};
  bc.sigma = sigma;
  bc.xout = xout;
  bc.yout = want_dual ? yout : nullptr;
  bc.chain = chain;
  bc.L = (int)chain->size();
  bc.stats = st;
  const bool cz = !want_dual || nc == 0.0;
  if (nb != 0.0) {
    bc.b = b;
    bc.c = cz ? b : c;
    bc.check_p = 1;
    bc.check_d = cz ? 0 : 1;
    bc.out_x = 1;
    bc.out_y = cz ? 0 : 2;
  } else {
    bc.b = c;
    bc.c = c;
    bc.check_p = 0;
    bc.check_d = 1;
    bc.out_x = 0;
    bc.out_y = 2;
  }
  return bc;
}

// Factor jobs and each shift's chain.  Algorithm 4 (RESET / NEXT_ROUND): the
// vertical chain (plus, for the next round, this call's first factor), then
// the horizontal updates.  Comparators: a SPAI per shift (DIRECT), or Table
// 2's first approach, P_i = Q_i P_1 with Q_i taken from sigmas[0] (FIRST);
// neither keeps a vertical chain.  Factors are allocated into `fresh`, not
// built.
morx_status plan_chains(morx_system sys, int nshift, const double* sigmas, const morx_opts& o,
                        std::vector<morx_factor>& fresh, ChainPlan& plan) {
  const int prec = o.precond_prec;
  const int policy = o.chain;
  const bool reuse = policy == MORX_CHAIN_RESET || policy == MORX_CHAIN_NEXT_ROUND;
  const bool reset = !reuse || policy == MORX_CHAIN_RESET || sys->vertical.empty();
  plan.reuse = reuse;
  if (!reset)
    MORX_REQUIRE(sys->vertical_prec == prec, MORX_E_INVALID,
                 "MORX_CHAIN_NEXT_ROUND needs the precision of the previous round");
  if (reset) {
    for (morx_factor f : sys->vertical) factor_release(f);
    sys->vertical.clear();
  }
  plan.jobs.clear();
  for (int i = 0; i < nshift; ++i) {
    morx_factor f = nullptr;
    MORX_TRY(factor_alloc(sys, prec, &f));
    fresh.push_back(f);
    FactorJob jb;
    if (policy == MORX_CHAIN_DIRECT || i == 0) {
      const bool spai = !reuse || reset;
      jb.is_spai = spai ? 1 : 0;
      jb.sigma_prev = spai ? 0.0 : sys->last_first_shift;
    } else {
      jb.is_spai = 0;
      jb.sigma_prev = policy == MORX_CHAIN_FIRST ? sigmas[0] : sigmas[i - 1];
    }
    jb.sigma_new = sigmas[i];
    jb.vals = f->vals.p;
    jb.valsT = f->valsT.p;
    f->is_spai = jb.is_spai != 0;
    f->sigma_prev = jb.sigma_prev;
    f->sigma_new = jb.sigma_new;
    plan.jobs.push_back(jb);
  }
  plan.chains.assign(nshift, {});
  for (int i = 0; i < nshift; ++i) {
    if (policy == MORX_CHAIN_DIRECT) {
      plan.chains[i] = {fresh[i]};
    } else if (policy == MORX_CHAIN_FIRST) {
      plan.chains[i] = {fresh[0]};
      if (i > 0) plan.chains[i].push_back(fresh[i]);
    } else {
      plan.chains[i] = sys->vertical;
      for (int k = 0; k <= i; ++k) plan.chains[i].push_back(fresh[k]);
    }
  }
  // what each shift's chain is, for morx_last_chains
  sys->last_chains.assign(nshift, {});
  for (int i = 0; i < nshift; ++i)
    for (morx_factor f : plan.chains[i]) {
      morx_factor_spec sp{};
      sp.is_spai = f->is_spai ? 1 : 0;
      sp.sigma_prev = f->is_spai ? 0.0 : f->sigma_prev;
      sp.sigma_new = f->sigma_new;
      sys->last_chains[i].push_back(sp);
    }
  sys->has_last_chains = true;
  return MORX_OK;
}

// After a successful call: the first factor joins the vertical chain
// (Algorithm 4); the rest are released when the call returns.
void commit_chains(morx_system sys, const ChainPlan& plan, const double* sigmas, int prec,
                   std::vector<morx_factor>& fresh, std::vector<morx_factor>& horizontal) {
  size_t keep_from = 0;
  if (plan.reuse && !fresh.empty()) {
    sys->vertical.push_back(fresh[0]);
    keep_from = 1;
  }
  for (size_t k = keep_from; k < fresh.size(); ++k) horizontal.push_back(fresh[k]);
  fresh.clear();
  sys->vertical_prec = plan.reuse ? prec : -1;
  sys->last_first_shift = sigmas[0];
}

// Shifted solves of nmom moments: moment 0 solves (sigma_i E - A) x = b_c and
// the transposed systems with c_c; moment j solves the same systems with
// E times moment j-1 as right-hand sides.  The factors and chains (policy
// o.chain) are built once and serve every moment.  X holds moment j of
// column c of shift i at column (j * nshift + i) * m + c (Y, stats alike).
// per_shift: column i of B and C is the right-hand side of shift i only (m = 1,
// nmom = 1); otherwise every shift takes all m columns
static morx_status solve_shifts_impl(morx_system sys, int32_t nshift, const double* sigmas,
                                     int32_t m, const double* B, int64_t ldb, const double* C,
                                     int64_t ldc, int32_t nmom, double* X, int64_t ldx, double* Y,
                                     int64_t ldy, const morx_opts& o, morx_col_stats* stats,
                                     hipStream_t st, std::vector<morx_factor>& horizontal,
                                     std::vector<morx_factor>& fresh, bool per_shift = false) {
  const bool want_dual = o.want_dual != 0;
  const int prec = o.precond_prec;
  MORX_REQUIRE(sys->ls_supported, MORX_E_UNSUPPORTED,
               "factor pattern exceeds the local least-squares limits");
  MORX_REQUIRE(!per_shift || (m == 1 && nmom == 1), MORX_E_INVALID,
               "per-shift right-hand sides take one column and one moment");
  // right-hand-side norms decide how each column pair runs
  const int nrhs = per_shift ? nshift : m;
  std::vector<double> norms(2 * nrhs, 0.0);
  MORX_TRY(rhs_norms(sys, B, ldb, nrhs, norms.data(), st));
  if (want_dual) MORX_TRY(rhs_norms(sys, C, ldc, nrhs, norms.data() + nrhs, st));
  for (int j = 0; j < 2 * nrhs; ++j)
    MORX_REQUIRE(std::isfinite(norms[j]), MORX_E_NONFINITE, "B or C holds NaN or Inf");

  ChainPlan plan;
  MORX_TRY(plan_chains(sys, nshift, sigmas, o, fresh, plan));
  const std::vector<FactorJob>& jobs = plan.jobs;
  const std::vector<std::vector<morx_factor>>& chains = plan.chains;

  // right-hand sides of moments j >= 1: E times the previous moment
  const int64_t nm = (int64_t)nshift * m;
  DevBuf rb, rc;
  if (nmom > 1) {
    MORX_TRY(dev_alloc(rb, (size_t)nm * sys->n_pad * sizeof(double)));
    if (want_dual) {
      const morx_status sa = dev_alloc(rc, (size_t)nm * sys->n_pad * sizeof(double));
      if (sa != MORX_OK) {
        dev_free(rb);
        return sa;
      }
    }
  }
  std::vector<double> nb(nm), nc(nm, 0.0);  // per (shift, column) of the current moment
  for (int i = 0; i < nshift; ++i)
    for (int c = 0; c < m; ++c) {
      const int k = per_shift ? i : c;
      nb[i * m + c] = norms[k];
      nc[i * m + c] = want_dual ? norms[nrhs + k] : 0.0;
    }
  auto trivial = [&](int64_t k) { return nb[k] == 0.0 && (!want_dual || nc[k] == 0.0); };
  morx_status s = MORX_OK;
  for (int mom = 0; mom < nmom && s == MORX_OK; ++mom) {
    double* Xm = X + (int64_t)mom * nm * ldx;
    double* Ym = want_dual ? Y + (int64_t)mom * nm * ldy : nullptr;
    morx_col_stats* Sm = stats ? stats + (int64_t)mom * nm : nullptr;
    if (mom > 0) {
      const dim3 g((unsigned)((sys->n + 255) / 256), (unsigned)nm);
      k_scale_cols<<<g, 256, 0, st>>>(sys->e, X + (int64_t)(mom - 1) * nm * ldx, ldx,
                                      (double*)rb.p, sys->n_pad, sys->n);
      if (want_dual)
        k_scale_cols<<<g, 256, 0, st>>>(sys->e, Y + (int64_t)(mom - 1) * nm * ldy, ldy,
                                        (double*)rc.p, sys->n_pad, sys->n);
      MORX_HIP(hipGetLastError());
      s = rhs_norms(sys, (const double*)rb.p, sys->n_pad, (int)nm, nb.data(), st);
      if (s == MORX_OK && want_dual)
        s = rhs_norms(sys, (const double*)rc.p, sys->n_pad, (int)nm, nc.data(), st);
      if (s != MORX_OK) break;
    }
    auto col = [&](int i, int c) -> BatchCol {
      const int64_t k = (int64_t)i * m + c;
      const int64_t j = per_shift ? i : c;  // the right-hand-side column
      const double* b = mom == 0 ? B + j * ldb : (const double*)rb.p + k * sys->n_pad;
      const double* cc = !want_dual ? nullptr
                         : mom == 0 ? C + j * ldc
                                    : (const double*)rc.p + k * sys->n_pad;
      return pair_col(sigmas[i], &chains[i], b, cc, nb[k], nc[k], want_dual, Xm + k * ldx,
                      Ym ? Ym + k * ldy : nullptr, Sm ? &Sm[k] : nullptr);
    };
    if (o.batched) {
      // every factor in one launch, every column pair of a moment in one batch
      if (mom == 0) s = factor_build_many(sys, prec, jobs.data(), nshift, st);
      std::vector<BatchCol> cols;
      for (int i = 0; i < nshift; ++i)
        for (int c = 0; c < m; ++c)
          if (!trivial((int64_t)i * m + c)) cols.push_back(col(i, c));
      if (s == MORX_OK) s = solve_batch(sys, cols, prec, o, st);
    } else {
      // one shift at a time, one column at a time (factor i built just before
      // the solves that first need it, as in Algorithm 4)
      for (int i = 0; i < nshift && s == MORX_OK; ++i) {
        if (mom == 0) s = factor_build_many(sys, prec, &jobs[i], 1, st);
        for (int c = 0; c < m && s == MORX_OK; ++c) {
          if (trivial((int64_t)i * m + c)) continue;
          std::vector<BatchCol> one{col(i, c)};
          s = solve_batch(sys, one, prec, o, st);
        }
      }
    }
    // trivial column pairs have the zero solution
    for (int64_t k = 0; k < nm && s == MORX_OK; ++k) {
      if (!trivial(k)) continue;
      if (hipMemsetAsync(Xm + k * ldx, 0, sys->n * sizeof(double), st) != hipSuccess ||
          (want_dual && hipMemsetAsync(Ym + k * ldy, 0, sys->n * sizeof(double), st) != hipSuccess)) {
        morx_set_error("solve: clearing a zero column failed");
        s = MORX_E_HIP;
        break;
      }
      if (Sm) {
        Sm[k].status = MORX_OK;
        Sm[k].iters = 0;
        Sm[k].restarts = 0;
        Sm[k].relres_primal = 0.0;
        Sm[k].relres_dual = 0.0;
      }
    }
  }
  hipStreamSynchronize(st);
  dev_free(rb);
  dev_free(rc);
  MORX_TRY(s);
  commit_chains(sys, plan, sigmas, prec, fresh, horizontal);
  morx_status worst = MORX_OK;
  if (stats)
    for (int64_t k = 0; k < (int64_t)nmom * nm; ++k) worst = (morx_status)worse(worst, stats[k].status);
  MORX_HIP(hipStreamSynchronize(st));
  return worst;
}

static morx_status solve_entry(const char* who, morx_system sys, int32_t nshift,
                               const double* sigmas, int32_t m, const double* B, int64_t ldb,
                               const double* C, int64_t ldc, int32_t nmom, double* X, int64_t ldx,
                               double* Y, int64_t ldy, const morx_opts* opts,
                               morx_col_stats* stats, void* stream, bool per_shift = false) {
  MORX_REQUIRE(sys, MORX_E_INVALID, "%s: null system", who);
  morx_opts o;
  if (opts) o = *opts;
  else morx_opts_default(&o);
  const bool want_dual = o.want_dual != 0;
  MORX_REQUIRE(nshift >= 1 && sigmas && m >= 1, MORX_E_INVALID,
               "%s: need at least one shift and one column", who);
  MORX_REQUIRE(nmom >= 1 && (int64_t)nmom * nshift * m <= (1 << 20), MORX_E_INVALID,
               "%s: bad number of moments", who);
  MORX_REQUIRE(B && X && ldb >= sys->n && ldx >= sys->n, MORX_E_INVALID, "%s: bad B or X", who);
  MORX_REQUIRE(!want_dual || (C && Y && ldc >= sys->n && ldy >= sys->n), MORX_E_INVALID,
               "%s: want_dual needs C and Y", who);
  MORX_REQUIRE(o.precond_prec >= MORX_F64 && o.precond_prec <= MORX_BF16, MORX_E_INVALID,
               "%s: bad precision", who);
  MORX_REQUIRE(o.apply_prec == MORX_F64 || o.apply_prec == MORX_F32, MORX_E_INVALID,
               "%s: apply precision must be MORX_F64 or MORX_F32", who);
  MORX_REQUIRE(o.chain >= MORX_CHAIN_RESET && o.chain <= MORX_CHAIN_FIRST, MORX_E_INVALID,
               "%s: unknown chain policy %d", who, o.chain);
  MORX_REQUIRE(o.tol >= 0.0 && o.max_restarts >= 0, MORX_E_INVALID,
               "%s: bad tolerance or restart limit", who);
  for (int i = 0; i < nshift; ++i)
    MORX_REQUIRE(std::isfinite(sigmas[i]), MORX_E_NONFINITE, "%s: shift %d not finite", who, i);
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  MORX_TRY(stream_enter(ctx, caller));
  std::vector<morx_factor> horizontal, fresh;
  morx_status s = solve_shifts_impl(sys, nshift, sigmas, m, B, ldb, want_dual ? C : nullptr, ldc,
                                    nmom, X, ldx, want_dual ? Y : nullptr, ldy, o, stats,
                                    ctx->stream, horizontal, fresh, per_shift);
  hipStreamSynchronize(ctx->stream);
  for (morx_factor f : horizontal) factor_release(f);
  for (morx_factor f : fresh) factor_release(f);
  morx_status s2 = stream_leave(ctx, caller);
  return s != MORX_OK ? s : s2;
}

extern "C" morx_status morx_solve_shifts(morx_system sys, int32_t nshift, const double* sigmas,
                                         int32_t m, const double* B, int64_t ldb, const double* C,
                                         int64_t ldc, double* X, int64_t ldx, double* Y,
                                         int64_t ldy, const morx_opts* opts,
                                         morx_col_stats* stats, void* stream) {
  return solve_entry("morx_solve_shifts", sys, nshift, sigmas, m, B, ldb, C, ldc, 1, X, ldx, Y,
                     ldy, opts, stats, stream);
}

extern "C" morx_status morx_solve_moments(morx_system sys, int32_t nshift, const double* sigmas,
                                          int32_t m, const double* B, int64_t ldb,
                                          const double* C, int64_t ldc, int32_t nmom, double* X,
                                          int64_t ldx, double* Y, int64_t ldy,
                                          const morx_opts* opts, morx_col_stats* stats,
                                          void* stream) {
  return solve_entry("morx_solve_moments", sys, nshift, sigmas, m, B, ldb, C, ldc, nmom, X, ldx,
                     Y, ldy, opts, stats, stream);
}

extern "C" morx_status morx_solve_pairs(morx_system sys, int32_t nshift, const double* sigmas,
                                        const double* B, int64_t ldb, const double* C, int64_t ldc,
                                        double* X, int64_t ldx, double* Y, int64_t ldy,
                                        const morx_opts* opts, morx_col_stats* stats,
                                        void* stream) {
  return solve_entry("morx_solve_pairs", sys, nshift, sigmas, 1, B, ldb, C, ldc, 1, X, ldx, Y, ldy,
                     opts, stats, stream, true);
}

namespace {

// X[:, c] *= f for the gridDim.y columns of a block
__global__ __launch_bounds__(256) void k_scale_block(double* __restrict__ X, int64_t ld, int64_t n,
                                                     double f) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  X[(int64_t)blockIdx.y * ld + i] *= f;
}

}  // namespace

// With proportional damping the second-order matrix is a multiple of a
// first-order one: s^2 M + s (alpha M + beta K) + K = c(s) (sigma(s) M + K),
// c(s) = 1 + beta s, sigma(s) = (s^2 + alpha s) / c(s).  The system holds
// E = M and A = -K, so every point is the first-order pair at sigma(s_i), and
// moment j there, Z_j = (sigma E - A)^{-1} E Z_{j-1}, gives the second-order
// one as X_j = (-1)^j c^{-(j+1)} Z_j (likewise Y_j).  Relative residuals are
// invariant under that scaling.  The least-squares problems scale too: the
// SPAI of c A_1 is P / c, and min ||c' A' - c A Q|| is solved by (c' / c) Q,
// so every chain is the first-order chain times a positive or negative
// scalar, and right-preconditioned BiCG runs the same iterates.
extern "C" morx_status morx_solve_second_order(morx_system sys, double alpha, double beta,
                                               int32_t npoint, const double* points, int32_t m,
                                               const double* F, int64_t ldf, const double* C,
                                               int64_t ldc, int32_t nmom, double* X, int64_t ldx,
                                               double* Y, int64_t ldy, const morx_opts* opts,
                                               morx_col_stats* stats, void* stream) {
  const char* who = "morx_solve_second_order";
  MORX_REQUIRE(sys, MORX_E_INVALID, "%s: null system", who);
  MORX_REQUIRE(std::isfinite(alpha) && std::isfinite(beta), MORX_E_NONFINITE,
               "%s: alpha and beta must be finite", who);
  MORX_REQUIRE(npoint >= 1 && points && m >= 1 && nmom >= 1 &&
                   (int64_t)nmom * npoint * m <= (1 << 20),
               MORX_E_INVALID, "%s: need at least one point, column and moment", who);
  std::vector<double> sig(npoint), cs(npoint);
  for (int i = 0; i < npoint; ++i) {
    const double s = points[i];
    MORX_REQUIRE(std::isfinite(s), MORX_E_NONFINITE, "%s: point %d not finite", who, i);
    cs[i] = 1.0 + beta * s;
    MORX_REQUIRE(cs[i] != 0.0, MORX_E_INVALID, "%s: 1 + beta s is zero at point %d", who, i);
    sig[i] = (s * s + alpha * s) / cs[i];
    MORX_REQUIRE(std::isfinite(sig[i]), MORX_E_INVALID,
                 "%s: the first-order shift of point %d overflows", who, i);
  }
  morx_opts o;
  if (opts) o = *opts;
  else morx_opts_default(&o);
  const morx_status st = solve_entry(who, sys, npoint, sig.data(), m, F, ldf, C, ldc, nmom, X, ldx,
                                     Y, ldy, &o, stats, stream);
  // column statuses leave every result in place; other failures return as they are
  if (st != MORX_OK && st != MORX_E_NOT_CONVERGED && st != MORX_E_BREAKDOWN) return st;
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t hs = (hipStream_t)stream;
  const int64_t n = sys->n;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)m);
  for (int j = 0; j < nmom; ++j)
    for (int i = 0; i < npoint; ++i) {
      const double f = (j % 2 ? -1.0 : 1.0) * std::pow(cs[i], -(double)(j + 1));
      if (f == 1.0) continue;
      const int64_t col = ((int64_t)j * npoint + i) * m;
      k_scale_block<<<grid, 256, 0, hs>>>(X + col * ldx, ldx, n, f);
      if (o.want_dual) k_scale_block<<<grid, 256, 0, hs>>>(Y + col * ldy, ldy, n, f);
    }
  MORX_HIP(hipGetLastError());
  MORX_HIP(hipStreamSynchronize(hs));
  return st;
}


// ---------------------------------------------------------------------------
// launch shapes: get, set, autotune

extern "C" morx_status morx_system_get_tune(morx_system sys, morx_tune* out) {
  MORX_REQUIRE(sys && out, MORX_E_INVALID, "morx_system_get_tune: null argument");
  memset(out, 0, sizeof(*out));
  out->factor_kernel = sys->tune_factor_rows;
  out->cols_per_wave = sys->tune_nc;
  out->slices_per_wave = sys->tune_spw;
  out->spmv_cols_per_wave = sys->tune_nc_spmv;
  out->chain_kernel = halo_in_use(sys) ? 1 : 0;
  out->halo_stride = halo_in_use(sys) ? sys->sell.hstride : 1;
  return MORX_OK;
}

extern "C" morx_status morx_chain_kernel_name(morx_system sys, int32_t ncol, int32_t prec,
                                              int32_t apply_prec, char* buf, int32_t cap) {
  MORX_REQUIRE(sys && buf && cap > 0 && ncol >= 1, MORX_E_INVALID,
               "morx_chain_kernel_name: bad argument");
  MORX_REQUIRE(prec >= MORX_F64 && prec <= MORX_BF16 &&
                   (apply_prec == MORX_F64 || apply_prec == MORX_F32),
               MORX_E_INVALID, "morx_chain_kernel_name: bad precision");
  std::lock_guard<std::mutex> lk(sys->ctx->mu);
  const char* vt = prec == MORX_F64 ? "double" : (prec == MORX_F32 ? "float" : "unsigned short");
  const char* at = apply_prec == MORX_F64 ? "double" : "float";
  const int nc = pick_nc(ncol, sys->tune_nc > 0 ? (int)sys->tune_nc : kDefaultNC);
  const bool narrow = pattern_narrow(sys);
  char tmp[128];
  if (halo_in_use(sys))
    snprintf(tmp, sizeof(tmp), "k_chain_halo<%s, %s, %d, %d, %d, %d>", vt, at, nc, (int)kHaloChain,
             narrow ? kNarrow : kHaloMaxW, narrow ? kHaloCapNarrow : kHaloCap);
  else
    snprintf(tmp, sizeof(tmp), "%s<%s, %s, %d, false>", narrow ? "k_chain_narrow" : "k_chain_step",
             vt, at, nc);
  MORX_REQUIRE((int)strlen(tmp) < cap, MORX_E_INVALID, "morx_chain_kernel_name: buffer too small");
  memcpy(buf, tmp, strlen(tmp) + 1);
  return MORX_OK;
}

extern "C" morx_status morx_system_set_tune(morx_system sys, const morx_tune* t) {
  MORX_REQUIRE(sys && t, MORX_E_INVALID, "morx_system_set_tune: null argument");
  MORX_REQUIRE(t->factor_kernel == -1 || factor_kernel_supported(sys, t->factor_kernel),
               MORX_E_INVALID, "morx_system_set_tune: factor kernel %d does not fit the pattern",
               t->factor_kernel);
  MORX_REQUIRE(t->cols_per_wave == -1 || (t->cols_per_wave >= 1 && t->cols_per_wave <= kMaxNC),
               MORX_E_INVALID, "morx_system_set_tune: cols_per_wave must be -1 or 1..%d", kMaxNC);
  MORX_REQUIRE(t->slices_per_wave == -1 || (t->slices_per_wave >= 1 && t->slices_per_wave <= 64),
               MORX_E_INVALID, "morx_system_set_tune: slices_per_wave must be -1 or 1..64");
  MORX_REQUIRE(t->spmv_cols_per_wave == -1 ||
                   (t->spmv_cols_per_wave >= 1 && t->spmv_cols_per_wave <= kMaxNC),
               MORX_E_INVALID, "morx_system_set_tune: spmv_cols_per_wave must be -1 or 1..%d",
               kMaxNC);
  MORX_REQUIRE(t->chain_kernel >= -1 && t->chain_kernel <= 1, MORX_E_INVALID,
               "morx_system_set_tune: chain_kernel must be -1, 0 or 1");
  MORX_REQUIRE(t->chain_kernel != 1 || halo_available(sys), MORX_E_UNSUPPORTED,
               "morx_system_set_tune: the pattern has no halo layout (rows of more than %d "
               "entries, or a block of 256 rows touching more than %d columns, %d for rows "
               "of at most %d entries)",
               kHaloMaxW, kHaloCap, kHaloCapNarrow, kNarrow);
  std::lock_guard<std::mutex> lk(sys->ctx->mu);
  sys->tune_factor_rows = t->factor_kernel;
  sys->tune_chain = t->chain_kernel;
  sys->tune_nc = t->cols_per_wave;
  sys->tune_spw = t->slices_per_wave;
  sys->tune_nc_spmv = t->spmv_cols_per_wave;
  return MORX_OK;
}

namespace {

// deterministic, nonzero right-hand sides for timing runs
__global__ void k_tune_rhs(double* p, int64_t n, int64_t ld, int ncol) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < ncol; ++c) {
    const uint32_t h = (uint32_t)(i * 2654435761u) ^ (uint32_t)(c * 40503u + 17u);
    p[(int64_t)c * ld + i] = 0.5 + (double)(h & 0xffffu) / 65536.0;
  }
}

}  // namespace

// systems above this size skip the Householder least-squares candidates when
// the normal equations apply
constexpr int64_t kTuneHouseholderMaxN = (int64_t)1 << 17;
// relative slowdown that ends a tile's row-block search (single timings of
// 6 iterations vary by about 1 % between launches)
constexpr double kTuneMargin = 0.03;
// a tile this much slower than the best shape so far ends the search over
// narrower tiles of that chain kernel: a narrower tile reads every factor
// value for fewer columns, and once that cost shows it only grows
constexpr double kTuneTileCut = 1.25;

static morx_status time_events(hipEvent_t a, hipEvent_t b, hipStream_t st, double* ms) {
  MORX_HIP(hipStreamSynchronize(st));
  float f = 0.f;
  MORX_HIP(hipEventElapsedTime(&f, a, b));
  *ms = f;
  return MORX_OK;
}

static morx_status autotune_impl(morx_system sys, double sigma, int ncols, int chain_len,
                                 int prec, morx_tune* out, hipStream_t st, hipEvent_t e0,
                                 hipEvent_t e1, std::vector<morx_factor>& keep) {
  // 1. least-squares kernel: per candidate one build of as many shifts as a
  // round has (each shift is a job of the same launch, as in a solve; the
  // jobs here are identical SPAI problems writing the same storage)
  double best_f = 1e300;
  int best_rows = -1;
  morx_factor f = nullptr;
  MORX_TRY(factor_alloc(sys, prec, &f));
  keep.push_back(f);
  // (capped near 8M column problems per candidate, so tuning a large system
  // stays short)
  const int64_t cap_jobs = std::max<int64_t>(2, ((int64_t)8 << 20) / std::max<int64_t>(sys->n, 1));
  const int njobs = (int)std::max<int64_t>(1, std::min<int64_t>({chain_len, 16, cap_jobs}));
  std::vector<FactorJob> fjobs(njobs, FactorJob{sigma, 0.0, 1, f->vals.p, f->valsT.p});
  const int saved_rows = sys->tune_factor_rows;
  // Where the normal equations apply, a column costs them two m x m
  // matrices and an m x m Cholesky per shift against a Householder QR of the
  // |I_k| x m local matrix (|I_k| about 4m for stencils): measured 5-9x
  // faster.  On large systems the Householder candidates, each a full build,
  // are therefore not timed.
  const bool ne_ok = factor_kernel_supported(sys, 2);
  for (int rows : {2, 0, 1, 8, 16}) {
    if (!factor_kernel_supported(sys, rows)) continue;
    if (rows != 2 && ne_ok && sys->n > kTuneHouseholderMaxN) continue;
    sys->tune_factor_rows = rows;
    MORX_HIP(hipEventRecord(e0, st));
    morx_status s = factor_build_many(sys, prec, fjobs.data(), njobs, st);
    MORX_HIP(hipEventRecord(e1, st));
    double ms = 0.0;
    MORX_TRY(time_events(e0, e1, st, &ms));
    if (s != MORX_OK) {
      sys->tune_factor_rows = saved_rows;
      return s;
    }
    if (ms < best_f) {
      best_f = ms;
      best_rows = rows;
    }
  }
  sys->tune_factor_rows = best_rows;
  f->is_spai = true;
  f->sigma_new = sigma;

  // 2. iteration shapes: BiCG iterations of ncols pairs preconditioned by
  // prefixes of one list of chain_len distinct copies of f, column c taking
  // 1 + c * chain_len / ncols factors (the chains of one round of
  // Algorithm 4; a single factor reused would stay in the last-level cache)
  std::vector<morx_factor> chain{f};
  for (int j = 1; j < chain_len; ++j) {
    morx_factor g = nullptr;
    MORX_TRY(factor_alloc(sys, prec, &g));
    keep.push_back(g);
    MORX_HIP(hipMemcpyAsync(g->vals.p, f->vals.p, f->vals.bytes, hipMemcpyDeviceToDevice, st));
    MORX_HIP(hipMemcpyAsync(g->valsT.p, f->valsT.p, f->valsT.bytes, hipMemcpyDeviceToDevice, st));
    chain.push_back(g);
  }
  KrylovBatch kb;
  kb.profile_grid = true;
  MORX_TRY(batch_alloc(kb, sys, ncols, chain_len, prec, MORX_F64, st));
  DevBuf rhs;
  morx_status s = dev_alloc(rhs, (size_t)ncols * sys->n_pad * sizeof(double));
  if (s != MORX_OK) {
    batch_free(kb);
    return s;
  }
  k_tune_rhs<<<(unsigned)((sys->n + 255) / 256), 256, 0, st>>>((double*)rhs.p, sys->n, sys->n_pad,
                                                                ncols);
  const int saved_nc = sys->tune_nc, saved_spw = sys->tune_spw, saved_ncs = sys->tune_nc_spmv;
  const int saved_chain = sys->tune_chain;
  sys->tune_nc = -1;
  sys->tune_spw = -1;
  sys->tune_nc_spmv = -1;
  sys->tune_chain = -1;
  const IterArgs a0 = make_args(kb, ncols, chain_len);
  const int spw0 = a0.spw;
  constexpr int kWarm = 2, kTimed = 6;
  // ms per iteration at one shape (fresh recurrences every time)
  auto time_shape = [&](int ncmax, int spw, int ncs, double* ms) -> morx_status {
    sys->tune_nc = ncmax;
    sys->tune_spw = spw;
    sys->tune_nc_spmv = ncs;
    for (int c = 0; c < ncols; ++c) {
      ColInfo ci = {};
      ci.sigma = sigma;
      ci.tol = 0.0;  // never converges: every timed iteration does full work
      ci.bsrc = (const double*)rhs.p + (int64_t)c * sys->n_pad;
      ci.csrc = ci.bsrc;
      ci.state = COL_INIT;
      ci.L = 1 + (int)(((int64_t)c * chain_len) / ncols);
      ci.first = 1;
      ci.maxit = 1 << 20;
      ci.check_p = ci.check_d = 1;
      kb.hcols[c] = ci;
      for (int j = 0; j < chain_len; ++j) {
        const bool in = j < ci.L;
        kb.hftab[(size_t)c * kb.lcap + j] = in ? chain[j]->vals.p : nullptr;
        kb.hftab[((size_t)kb.cap + c) * kb.lcap + j] = in ? chain[j]->valsT.p : nullptr;
      }
    }
    MORX_TRY(batch_upload(kb, 0, ncols, st));
    MORX_TRY(batch_launch_init(kb, ncols, st));
    const IterArgs a = make_args(kb, ncols, chain_len);
    MORX_TRY(enqueue_iterations(a, prec, kWarm, st, nullptr));
    MORX_HIP(hipEventRecord(e0, st));
    MORX_TRY(enqueue_iterations(a, prec, kTimed, st, nullptr));
    MORX_HIP(hipEventRecord(e1, st));
    MORX_TRY(time_events(e0, e1, st, ms));
    *ms /= kTimed;
    return MORX_OK;
  };
  double best_i = 1e300;
  int best_nc = -1, best_spw = -1, best_ncs = -1, best_chain = -1;
  // chain kernel (the built-in one, and where the pattern has a halo layout
  // the other: row gathers for wide patterns, the halo layout for narrow
  // ones), chain tile and row block; the shifted pair follows the chain tile
  // and kernel ...
  std::vector<int> kernels{-1};
  if (halo_available(sys)) kernels.push_back(pattern_narrow(sys) ? 1 : 0);
  for (int kern : kernels) {
    sys->tune_chain = kern;
    std::vector<int> seen;
    for (int ncmax : {16, 12, 8, 6, 4, 3, 2, 1}) {
      const int ncv = pick_nc(ncols, ncmax);
      if (std::find(seen.begin(), seen.end(), ncv) != seen.end()) continue;
      seen.push_back(ncv);
      double prev = 1e300, tile_best = 1e300;
      for (int mult : {1, 2, 4}) {
        const int spw = spw0 * mult;
        if (mult > 1 && (sys->nslice + (int64_t)kWavesPerBlock * spw - 1) /
                                ((int64_t)kWavesPerBlock * spw) < 256)
          break;  // too few row blocks to fill the chip
        double ms = 0.0;
        s = time_shape(ncmax, spw, -1, &ms);
        if (s != MORX_OK) break;
        if (ms < best_i) {
          best_i = ms;
          best_nc = ncmax;
          best_spw = spw;
          best_chain = kern;
        }
        tile_best = std::min(tile_best, ms);
        // a wider row block lost at this tile (beyond launch-to-launch jitter)
        if (ms > prev * (1.0 + kTuneMargin)) break;
        prev = std::min(prev, ms);
      }
      if (s != MORX_OK) break;
      if (tile_best > best_i * kTuneTileCut) break;
    }
    if (s != MORX_OK) break;
  }
  sys->tune_chain = best_chain;
  // ... and the shifted pair's own tile with the chain shape and kernel fixed
  if (s == MORX_OK) {
    std::vector<int> seen{pick_nc(ncols, best_nc)};
    for (int ncs : {16, 8, 4, 2, 1}) {
      const int ncv = pick_nc(ncols, ncs);
      if (std::find(seen.begin(), seen.end(), ncv) != seen.end()) continue;
      seen.push_back(ncv);
      double ms = 0.0;
      s = time_shape(best_nc, best_spw, ncs, &ms);
      if (s != MORX_OK) break;
      if (ms < best_i) {
        best_i = ms;
        best_ncs = ncs;
      }
    }
  }
  hipStreamSynchronize(st);
  dev_free(rhs);
  batch_free(kb);
  if (s != MORX_OK) {
    sys->tune_nc = saved_nc;
    sys->tune_spw = saved_spw;
    sys->tune_nc_spmv = saved_ncs;
    sys->tune_chain = saved_chain;
    return s;
  }
  sys->tune_nc = best_nc;
  sys->tune_spw = best_spw;
  sys->tune_nc_spmv = best_ncs;
  sys->tune_chain = best_chain;
  memset(out, 0, sizeof(*out));
  out->factor_kernel = best_rows;
  out->cols_per_wave = best_nc;
  out->slices_per_wave = best_spw;
  out->spmv_cols_per_wave = best_ncs;
  out->chain_kernel = halo_in_use(sys) ? 1 : 0;
  out->halo_stride = halo_in_use(sys) ? sys->sell.hstride : 1;
  out->factor_ms = best_f;
  out->iter_ms = best_i;
  return MORX_OK;
}

extern "C" morx_status morx_autotune(morx_system sys, double sigma, int32_t ncols,
                                     int32_t chain_len, int32_t prec, morx_tune* out,
                                     void* stream) {
  MORX_REQUIRE(sys && out, MORX_E_INVALID, "morx_autotune: null argument");
  MORX_REQUIRE(ncols >= 1 && ncols <= 1024, MORX_E_INVALID, "morx_autotune: ncols must be 1..1024");
  MORX_REQUIRE(chain_len >= 1 && chain_len <= 64, MORX_E_INVALID,
               "morx_autotune: chain_len must be 1..64");
  MORX_REQUIRE(prec >= MORX_F64 && prec <= MORX_BF16, MORX_E_INVALID, "morx_autotune: bad precision");
  MORX_REQUIRE(std::isfinite(sigma), MORX_E_NONFINITE, "morx_autotune: shift not finite");
  MORX_REQUIRE(sys->ls_supported, MORX_E_UNSUPPORTED,
               "factor pattern exceeds the local least-squares limits");
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  MORX_TRY(stream_enter(ctx, caller));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  morx_status s = MORX_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    morx_set_error("morx_autotune: event creation failed");
    s = MORX_E_HIP;
  }
  std::vector<morx_factor> fs;
  if (s == MORX_OK)
    s = autotune_impl(sys, sigma, ncols, chain_len, prec, out, ctx->stream, e0, e1, fs);
  hipStreamSynchronize(ctx->stream);
  for (morx_factor f : fs) factor_release(f);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  morx_status s2 = stream_leave(ctx, caller);
  return s != MORX_OK ? s : s2;
}

// ---------------------------------------------------------------------------
// the chain step and the shifted pair of a solve, on caller columns
//
// A temporary slot batch holds the columns as active BiCG slots: the inputs
// go where an iteration's first chain pass (r, r~) or the shifted pair (p,
// p~) reads them, the work lists come from the same device-side builder, and
// the launches are the ones an iteration enqueues for that many columns,
// with the system's launch shapes.

static dim3 probe_grid(const morx_system sys, int ncol) {
  return dim3((unsigned)std::min<int64_t>((sys->n + 255) / 256, 2048), (unsigned)ncol, 1);
}

morx_status hot_chain_apply(morx_system sys, int ncol, int lcap, const morx_factor* chains,
                            const int32_t* lens, const double* X, int64_t ldx, double* Y,
                            int64_t ldy, const double* Xt, int64_t ldxt, double* Yt, int64_t ldyt,
                            int aprec, hipStream_t st) {
  const int prec = chains[0]->prec;
  int maxL = 0;
  for (int c = 0; c < ncol; ++c) maxL = std::max(maxL, (int)lens[c]);
  KrylovBatch b;
  b.profile_grid = true;
  MORX_TRY(batch_alloc(b, sys, ncol, maxL, prec, aprec, st));
  for (int c = 0; c < ncol; ++c) {
    ColInfo ci = {};
    ci.state = COL_ACTIVE;
    ci.L = lens[c];
    b.hcols[c] = ci;
    for (int s = 0; s < b.lcap; ++s) {
      morx_factor f = s < lens[c] ? chains[(size_t)c * lcap + s] : nullptr;
      b.hftab[(size_t)c * b.lcap + s] = f ? f->vals.p : nullptr;
      b.hftab[((size_t)b.cap + c) * b.lcap + s] = f ? f->valsT.p : nullptr;
    }
  }
  morx_status s = batch_upload(b, 0, ncol, st);
  if (s == MORX_OK) {
    const IterArgs a = make_args(b, ncol, maxL);
    k_probe_in<<<probe_grid(sys, ncol), 256, 0, st>>>(a, V_R, V_RT, X, ldx, Xt, ldxt,
                                                       aprec == MORX_F32);
    k_plan<<<1, kFinThreads, 0, st>>>(a);
    enqueue_chain(a, prec, st, nullptr);
    k_probe_out<<<probe_grid(sys, ncol), 256, 0, st>>>(a, 1, Y, ldy, Yt, ldyt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      morx_set_error("chain apply: %s", hipGetErrorString(e));
      s = MORX_E_HIP;
    }
  }
  hipStreamSynchronize(st);
  batch_free(b);
  return s;
}

morx_status hot_shifted_pair(morx_system sys, int ncol, const double* sigmas, const double* X,
                             int64_t ldx, double* Y, int64_t ldy, const double* Xt, int64_t ldxt,
                             double* Yt, int64_t ldyt, hipStream_t st) {
  KrylovBatch b;
  b.profile_grid = true;
  MORX_TRY(batch_alloc(b, sys, ncol, 1, MORX_F64, MORX_F64, st));
  for (int c = 0; c < ncol; ++c) {
    ColInfo ci = {};
    ci.state = COL_ACTIVE;
    ci.sigma = sigmas[c];
    ci.L = 1;
    b.hcols[c] = ci;
  }
  morx_status s = batch_upload(b, 0, ncol, st);
  if (s == MORX_OK) {
    const IterArgs a = make_args(b, ncol, 1);
    k_probe_in<<<probe_grid(sys, ncol), 256, 0, st>>>(a, V_P0, V_PT0, X, ldx, Xt, ldxt, 0);
    k_plan<<<1, kFinThreads, 0, st>>>(a);  // the halo form takes its columns from a work list
    enqueue_spmv(a, 0, st, nullptr);
    k_probe_out<<<probe_grid(sys, ncol), 256, 0, st>>>(a, 0, Y, ldy, Yt, ldyt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      morx_set_error("shifted pair: %s", hipGetErrorString(e));
      s = MORX_E_HIP;
    }
  }
  hipStreamSynchronize(st);
  batch_free(b);
  return s;
}

extern "C" morx_status morx_chain_apply_batch(morx_system sys, int32_t ncol, int32_t lcap,
                                              const morx_factor* chains, const int32_t* lens,
                                              const double* X, int64_t ldx, double* Y,
                                              int64_t ldy, const double* Xt, int64_t ldxt,
                                              double* Yt, int64_t ldyt, int32_t apply_prec,
                                              void* stream) {
  MORX_REQUIRE(sys && chains && lens, MORX_E_INVALID, "morx_chain_apply_batch: null argument");
  MORX_REQUIRE(ncol >= 1 && ncol <= 1024 && lcap >= 1 && lcap <= 64, MORX_E_INVALID,
               "morx_chain_apply_batch: ncol must be 1..1024 and lcap 1..64");
  MORX_REQUIRE((X == nullptr) == (Y == nullptr) && (Xt == nullptr) == (Yt == nullptr),
               MORX_E_INVALID, "morx_chain_apply_batch: an input without its output");
  MORX_REQUIRE(!X || (ldx >= sys->n && ldy >= sys->n), MORX_E_INVALID,
               "morx_chain_apply_batch: leading dimension below n");
  MORX_REQUIRE(!Xt || (ldxt >= sys->n && ldyt >= sys->n), MORX_E_INVALID,
               "morx_chain_apply_batch: leading dimension below n");
  MORX_REQUIRE(apply_prec == MORX_F64 || apply_prec == MORX_F32, MORX_E_INVALID,
               "morx_chain_apply_batch: apply precision must be MORX_F64 or MORX_F32");
  int prec = -1;
  for (int c = 0; c < ncol; ++c) {
    MORX_REQUIRE(lens[c] >= 1 && lens[c] <= lcap, MORX_E_INVALID,
                 "morx_chain_apply_batch: chain length %d of column %d outside 1..%d", lens[c], c,
                 lcap);
    for (int k = 0; k < lens[c]; ++k) {
      const morx_factor f = chains[(size_t)c * lcap + k];
      MORX_REQUIRE(f && f->sys == sys, MORX_E_INVALID,
                   "morx_chain_apply_batch: factor %d of column %d does not belong to this system",
                   k, c);
      MORX_REQUIRE(prec < 0 || f->prec == prec, MORX_E_INVALID,
                   "morx_chain_apply_batch: factors of different storage precisions");
      prec = f->prec;
    }
  }
  std::lock_guard<std::mutex> lk(sys->ctx->mu);
  MORX_HIP(hipSetDevice(sys->ctx->device));
  std::vector<morx_factor> tab(chains, chains + (size_t)ncol * lcap);
  for (int c = 0; c < ncol; ++c)
    for (int k = lens[c]; k < lcap; ++k) tab[(size_t)c * lcap + k] = nullptr;
  return hot_chain_apply(sys, ncol, lcap, tab.data(), lens, X, ldx, Y, ldy, Xt, ldxt, Yt, ldyt,
                         apply_prec, (hipStream_t)stream);
}

extern "C" morx_status morx_shifted_apply_pair(morx_system sys, int32_t ncol, const double* sigmas,
                                               const double* X, int64_t ldx, double* Y,
                                               int64_t ldy, const double* Xt, int64_t ldxt,
                                               double* Yt, int64_t ldyt, void* stream) {
  MORX_REQUIRE(sys && sigmas, MORX_E_INVALID, "morx_shifted_apply_pair: null argument");
  MORX_REQUIRE(ncol >= 1 && ncol <= 1024, MORX_E_INVALID,
               "morx_shifted_apply_pair: ncol must be 1..1024");
  MORX_REQUIRE((X == nullptr) == (Y == nullptr) && (Xt == nullptr) == (Yt == nullptr),
               MORX_E_INVALID, "morx_shifted_apply_pair: an input without its output");
  MORX_REQUIRE(!X || (ldx >= sys->n && ldy >= sys->n), MORX_E_INVALID,
               "morx_shifted_apply_pair: leading dimension below n");
  MORX_REQUIRE(!Xt || (ldxt >= sys->n && ldyt >= sys->n), MORX_E_INVALID,
               "morx_shifted_apply_pair: leading dimension below n");
  for (int c = 0; c < ncol; ++c)
    MORX_REQUIRE(std::isfinite(sigmas[c]), MORX_E_NONFINITE,
                 "morx_shifted_apply_pair: shift %d not finite", c);
  std::lock_guard<std::mutex> lk(sys->ctx->mu);
  MORX_HIP(hipSetDevice(sys->ctx->device));
  return hot_shifted_pair(sys, ncol, sigmas, X, ldx, Y, ldy, Xt, ldxt, Yt, ldyt,
                          (hipStream_t)stream);
}

extern "C" morx_status morx_last_chains(morx_system sys, int32_t cap_shifts, int32_t ldspec,
                                        int32_t* nshift, int32_t* lens, morx_factor_spec* specs) {
  MORX_REQUIRE(sys && nshift, MORX_E_INVALID, "morx_last_chains: null argument");
  MORX_REQUIRE(cap_shifts >= 0 && ldspec >= 0 && (cap_shifts == 0 || (lens && specs)),
               MORX_E_INVALID, "morx_last_chains: bad output arrays");
  std::lock_guard<std::mutex> lk(sys->ctx->mu);
  MORX_REQUIRE(sys->has_last_chains, MORX_E_INVALID, "morx_last_chains: no solve has run");
  *nshift = (int32_t)sys->last_chains.size();
  for (int i = 0; i < cap_shifts && i < (int)sys->last_chains.size(); ++i) {
    const auto& ch = sys->last_chains[i];
    lens[i] = (int32_t)ch.size();
    for (int k = 0; k < (int)ch.size() && k < ldspec; ++k) specs[(size_t)i * ldspec + k] = ch[k];
  }
  return MORX_OK;
}
