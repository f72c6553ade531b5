// SPAI and reuse-update factors as n independent column least-squares
// problems, one wavefront per column (Section III-A, eq. gen-precond-par; the
// note under Algorithm 4 says the update minimisations are solved the same way).
//
// Column k of a factor is supported on J_k = column k of S.  Its problem only
// touches the rows I_k of S[:, J_k]; the wave gathers those nonzeros, sorts
// their row indices to get I_k, builds the dense |I_k| x |J_k| matrix of
// A_s = sigma E - A in LDS and solves it with Householder QR:
//   SPAI:    min || e_k        - A_new[I_k, J_k] p ||
//   update:  min || A_prev[I_k, k] - A_new[I_k, J_k] q ||
// One wave handles several shifts for the same column, so the gather and sort
// are done once per column.
#include <math.h>

#include <algorithm>
#include <cmath>

#include "common.h"

namespace {

constexpr int kLdsBudget = 60 * 1024;  // dynamic LDS, below the 64 KiB workgroup limit

struct LsLayout {
  int Tpad, Tmax, ldm, mmax;
  size_t off_keys, off_tri, off_tv, off_uniq, off_J, off_q, off_M, bytes;
};

LsLayout ls_layout(int maxJ, int maxT, int maxI) {
  LsLayout L;
  L.Tmax = std::max(maxT, 1);
  L.Tpad = 64;
  while (L.Tpad < L.Tmax) L.Tpad <<= 1;
  L.ldm = std::max(maxI, 1) | 1;  // odd stride: fewer LDS bank conflicts
  L.mmax = std::max(maxJ, 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 15) / 16 * 16;
    return r;
  };
  L.off_keys = take((size_t)L.Tpad * 4);
  L.off_tri = take((size_t)L.Tmax * 4);
  L.off_tv = take((size_t)L.Tmax * 8);
  L.off_uniq = take((size_t)std::max(maxI, 1) * 4);
  L.off_J = take(32 * 4);
  L.off_q = take(32 * 8);
  L.off_M = take((size_t)L.ldm * (L.mmax + 1) * 8);
  L.bytes = o;
  return L;
}

__device__ __forceinline__ int wave_excl_scan(int v, int lane, int* total) {
  int inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  *total = __shfl(inc, 63, 64);
  return inc - v;
}

// Gather the nonzeros of S[:, J_k] (rows into keys[], (row-local, col) later),
// sort the rows and compact them into uniq[].  Returns m = |J_k|, T, nI.
__device__ void gather_sort_unique(const int32_t* __restrict__ trowptr,
                                   const int32_t* __restrict__ tcol,
                                   const double* __restrict__ tval, int64_t k, int lane, int Tpad,
                                   int* keys, int* tri, double* tv, int* uniq, int* J, int* m_out,
                                   int* T_out, int* nI_out) {
  const int lo = trowptr[k];
  const int m = trowptr[k + 1] - lo;
  int len = 0, j = 0;
  if (lane < m) {
    j = tcol[lo + lane];
    J[lane] = j;
    len = trowptr[j + 1] - trowptr[j];
  }
  int T;
  int off = wave_excl_scan(len, lane, &T);
  if (lane < m) {
    const int b = trowptr[j];
    for (int u = 0; u < len; ++u) {
      keys[off + u] = tcol[b + u];
      tri[off + u] = lane;  // local column; the local row is added below
      if (tv) tv[off + u] = tval[b + u];
    }
  }
  for (int t = T + lane; t < Tpad; t += 64) keys[t] = 0x7fffffff;
  __syncthreads();
  // bitonic sort of the row indices (ascending)
  for (int size = 2; size <= Tpad; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = lane; t < Tpad; t += 64) {
        int p = t ^ stride;
        if (p > t) {
          int a = keys[t], b = keys[p];
          bool up = ((t & size) == 0);
          if ((a > b) == up) {
            keys[t] = b;
            keys[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  // compact unique rows
  int base = 0;
  for (int t0 = 0; t0 < T; t0 += 64) {
    int t = t0 + lane;
    bool first = (t < T) && (t == 0 || keys[t] != keys[t - 1]);
    unsigned long long mask = __ballot(first);
    int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
    if (first) uniq[pos] = keys[t];
    base += __popcll(mask);
  }
  __syncthreads();
  *m_out = m;
  *T_out = T;
  *nI_out = base;
}

__device__ __forceinline__ int find_row(const int* uniq, int nI, int row) {
  int lo = 0, hi = nI - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (uniq[mid] < row) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_ls_count(const int32_t* __restrict__ trowptr,
                                                  const int32_t* __restrict__ tcol, int64_t n,
                                                  int* __restrict__ stats) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int lo = trowptr[k], m = trowptr[k + 1] - lo;
  int T = 0;
  for (int a = 0; a < m; ++a) {
    int j = tcol[lo + a];
    T += trowptr[j + 1] - trowptr[j];
  }
  atomicMax(&stats[0], m);
  atomicMax(&stats[1], T);
}

__global__ __launch_bounds__(64) void k_ls_unique(const int32_t* __restrict__ trowptr,
                                                  const int32_t* __restrict__ tcol, int64_t n,
                                                  LsLayout L, int* __restrict__ stats) {
  extern __shared__ __align__(16) unsigned char lds[];
  int* keys = (int*)(lds + L.off_keys);
  int* tri = (int*)(lds + L.off_tri);
  int* uniq = (int*)(lds + L.off_uniq);
  int* J = (int*)(lds + L.off_J);
  const int lane = threadIdx.x;
  for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
    int m, T, nI;
    gather_sort_unique(trowptr, tcol, nullptr, k, lane, L.Tpad, keys, tri, nullptr, uniq, J, &m,
                       &T, &nI);
    if (lane == 0) atomicMax(&stats[2], nI);
    __syncthreads();
  }
}

template <typename VT>
__global__ __launch_bounds__(64) void k_factor_ls(
    const int32_t* __restrict__ trowptr, const int32_t* __restrict__ tcol,
    const double* __restrict__ tval, const double* __restrict__ e,
    const int32_t* __restrict__ tp2s, const int32_t* __restrict__ sellT_off, int64_t n,
    const FactorJob* __restrict__ jobs, int njobs, LsLayout L, int* __restrict__ status,
    const int32_t* __restrict__ list, const int* __restrict__ list_count) {
  extern __shared__ __align__(16) unsigned char lds[];
  int* keys = (int*)(lds + L.off_keys);
  int* tri = (int*)(lds + L.off_tri);
  double* tv = (double*)(lds + L.off_tv);
  int* uniq = (int*)(lds + L.off_uniq);
  int* J = (int*)(lds + L.off_J);
  double* q = (double*)(lds + L.off_q);
  double* M = (double*)(lds + L.off_M);
  const int lane = threadIdx.x;
  const int ldm = L.ldm;
  // every column, or the columns listed (those the normal equations gave up)
  const int64_t count = list ? (int64_t)*list_count : n;

  for (int64_t it = blockIdx.x; it < count; it += gridDim.x) {
    const int64_t k = list ? (int64_t)list[it] : it;
    int m, T, nI;
    gather_sort_unique(trowptr, tcol, tval, k, lane, L.Tpad, keys, tri, tv, uniq, J, &m, &T, &nI);
    // local row of every gathered nonzero (keys[] is sorted now, so walk the
    // columns again in gather order)
    {
      int len = 0, j = 0;
      if (lane < m) {
        j = J[lane];
        len = trowptr[j + 1] - trowptr[j];
      }
      int Tt;
      int off = wave_excl_scan(len, lane, &Tt);
      if (lane < m) {
        const int b = trowptr[j];
        for (int u = 0; u < len; ++u) {
          int li = find_row(uniq, nI, tcol[b + u]);
          tri[off + u] = (li << 5) | lane;
        }
      }
    }
    __shared__ int s_kloc, s_ak;
    if (lane == 0) s_kloc = find_row(uniq, nI, (int)k);
    if (lane < m && J[lane] == (int)k) s_ak = lane;
    __syncthreads();
    const int kloc = s_kloc, ak = s_ak;
    const double ek = e[k];
    int CG = 1;
    while (CG < m + 1) CG <<= 1;
    const int RG = 64 / CG;
    const int cc = lane % CG, g = lane / CG;

    for (int jb = 0; jb < njobs; ++jb) {
      const FactorJob job = jobs[jb];
      const double sn = job.sigma_new;
      // dense local matrix [A_new(I_k, J_k) | rhs], column-major with stride ldm
      for (int t = lane; t < (m + 1) * ldm; t += 64) M[t] = 0.0;
      __syncthreads();
      for (int t = lane; t < T; t += 64) {
        int a = tri[t] & 31, li = tri[t] >> 5;
        double v = -tv[t];
        if (uniq[li] == J[a]) v += sn * e[J[a]];
        M[a * ldm + li] = v;
      }
      __syncthreads();
      if (job.is_spai) {
        if (lane == 0) M[m * ldm + kloc] = 1.0;
      } else {
        for (int r = lane; r < nI; r += 64) M[m * ldm + r] = M[ak * ldm + r];
        __syncthreads();
        if (lane == 0) M[m * ldm + kloc] -= (sn - job.sigma_prev) * ek;
      }
      __syncthreads();
      // Householder QR of the m columns, applied to the right-hand side too
      bool singular = false;
      for (int c = 0; c < m; ++c) {
        double s = 0.0;
        if (cc >= c && cc <= m) {
          for (int r = c + g; r < nI; r += RG) s += M[c * ldm + r] * M[cc * ldm + r];
        }
        for (int off = CG; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
        s = __shfl(s, cc, 64);  // one value per column for every row group
        const double norm2 = __shfl(s, c, 64);
        const double x0 = M[c * ldm + c];
        double scale = 0.0;
        for (int a = 0; a <= c; ++a) scale = fmax(scale, fabs(M[a * ldm + a]));
        if (!(norm2 > 0.0) || sqrt(norm2) <= 1e-14 * fmax(scale, 1e-300)) singular = true;
        const double alpha = (x0 > 0.0) ? -sqrt(norm2) : sqrt(norm2);
        const double vtv = 2.0 * alpha * (alpha - x0);
        if (cc > c && cc <= m && vtv > 0.0) {
          const double d = s - alpha * M[cc * ldm + c];
          const double tau = 2.0 * d / vtv;
          for (int r = c + g; r < nI; r += RG) {
            const double vr = (r == c) ? (x0 - alpha) : M[c * ldm + r];
            M[cc * ldm + r] -= tau * vr;
          }
        }
        __syncthreads();
        if (lane == 0) M[c * ldm + c] = alpha;
        __syncthreads();
      }
      // back substitution R q = (Q^T rhs)(0:m)
      if (lane == 0) {
        for (int i = m - 1; i >= 0; --i) {
          double acc = M[m * ldm + i];
          for (int j2 = i + 1; j2 < m; ++j2) acc -= M[j2 * ldm + i] * q[j2];
          q[i] = singular ? 0.0 : acc / M[i * ldm + i];
        }
      }
      __syncthreads();
      if (lane < m) {
        const double v = q[lane];
        const int64_t posT = (int64_t)sellT_off[k / kSlice] + (int64_t)lane * kSlice + (k % kSlice);
        store_val<VT>((VT*)job.valsT + posT, v);
        store_val<VT>((VT*)job.vals + tp2s[trowptr[k] + lane], v);
      }
      if (singular && lane == 0) atomicOr(status, 1);
      __syncthreads();
    }
  }
}

__global__ void k_fill_zero_bytes(uint32_t* p, int64_t words) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0u;
}

// Imported values: CSR(S) order -> SELL(S) order, rounded to the storage type
template <typename VT>
__global__ void k_import_sell(const double* __restrict__ val, const int32_t* __restrict__ csr2sell,
                              int64_t nnz, VT* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) store_val<VT>(out + csr2sell[p], val[p]);
}

// ... and SELL(S) -> SELL(S^T): row k of S^T lists column k of S; its entry m
// sits at SELL(S^T) position off[k / 64] + 64 m + k % 64
template <typename VT>
__global__ void k_import_sellT(const VT* __restrict__ sellv, const int32_t* __restrict__ trowptr,
                               const int32_t* __restrict__ tp2s, const int32_t* __restrict__ offT,
                               int64_t n, VT* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t p0 = trowptr[k], p1 = trowptr[k + 1];
  const int64_t base = offT[k >> 6] + (k & 63);
  for (int32_t p = p0; p < p1; ++p) out[base + (int64_t)(p - p0) * 64] = sellv[tp2s[p]];
}

template <typename VT>
__global__ void k_factor_to_csr(const VT* __restrict__ vals, const int32_t* __restrict__ csr2sell,
                                int64_t nnz, double* __restrict__ out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) out[p] = load_val<VT>(vals + csr2sell[p]);
}

// ---- normal-equations kernel (factor_kernel 2) -----------------------------
//
// With M(s) = s E(I_k, J_k) - A(I_k, J_k), m = |J_k| and a the position of k
// in J_k, every product the normal equations of a column need comes from two
// m x m matrices:
//   G0  = A(I_k, J_k)^T A(I_k, J_k) = (A^T A)(J_k, J_k)  (I_k holds every row of
//         those columns of A),
//   Ajj = A(J_k, J_k),
// since E(I_k, J_k) has one entry E_j per column, in row J_j:
//   M(s1)^T M(s2) = G0 - s2 Ajj^T E_J - s1 E_J Ajj + s1 s2 E_J^2.
// A SPAI column solves G(s) q = M(s)^T e_k with M(s)^T e_k = s E_k e_a -
// Ajj(a, :)^T; an update column solves G(sn) q = M(sn)^T M(sp) e_a (its
// right-hand side is column k of sp E - A).  Neither I_k nor the dense
// |I_k| x m matrix is formed: the block gathers the m columns of A, and one
// merge per column pair over their sorted rows gives G0 and the two entries of
// Ajj, hence H = E_J Ajj + Ajj^T E_J (G(s) = G0 - s H + s^2 E_J^2, both
// symmetric; Ajj itself is kept only in row and column a), and then groups
// of CG lanes, lane i holding row i, each take one shift: Cholesky
// factorisation and the two triangular solves in registers, each column of L
// passed to the group's lanes through LDS.  Lane i skips its own update at
// step i, so its entries past i keep L(i, i) times column i of L, which the
// solve with L^T then reads from the lane's registers.  The normal equations
// square the condition
// number, so a column with a pivot below kNeTol times the diagonal entry it
// started from is listed for the Householder kernel, which rebuilds every
// shift of that column (and reports a rank-deficient problem as the other
// kernels do).
constexpr double kNeTol = 1e-6;
constexpr int kNeGather = 16;  // entries of a column loaded together in the set-up

struct NeLayout {
  int T, G;  // gathered entries, lane groups per block
  size_t off_J, off_off, off_E, off_H, off_G0, off_A, off_crow, off_cval, off_L, bytes;
};

// A normal-equations block has nw waves (one to four), whose 64 nw / CG lane
// groups solve as many shifts of one column problem at a time and share the
// LDS copy of its matrices; the launch picks nw for the number of shifts.
constexpr int kNeMaxWaves = 4;

NeLayout ne_layout(int maxT, int CG, int nw) {
  NeLayout L;
  L.T = std::max(maxT, 1);
  L.G = nw * 64 / CG;
  const size_t mat = (size_t)CG * (CG + 1) * 8;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 15) / 16 * 16;
    return r;
  };
  L.off_J = take((size_t)CG * 4);
  L.off_off = take((size_t)(CG + 1) * 4);
  L.off_E = take((size_t)CG * 8);
  L.off_H = take(mat);
  L.off_G0 = take(mat);
  L.off_A = take((size_t)2 * CG * 8);
  // the gathered columns, later in the same space one column of L per group
  const size_t base = o;
  L.off_crow = base;
  L.off_cval = base + ((size_t)L.T * 4 + 15) / 16 * 16;
  L.off_L = base;
  const size_t gather = L.off_cval - base + (size_t)L.T * 8;
  o += std::max(gather, (size_t)L.G * CG * 8);
  L.bytes = o;
  return L;
}

// Lane gbase + c's value for every lane of a group of CG lanes (a group lies
// within one wave): lane reads of the scalar unit for groups of 16 or 32
// lanes, an LDS permute for narrower ones
template <int CG>
__device__ __forceinline__ double group_bcast(double v, int gbase, int c) {
  if constexpr (CG >= 16) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    double out = 0.0;
    const int wl = (int)(threadIdx.x & 63);
#pragma unroll
    for (int g2 = 0; g2 < 64 / CG; ++g2) {
      const double x = __hiloint2double(__builtin_amdgcn_readlane(hi, g2 * CG + c),
                                        __builtin_amdgcn_readlane(lo, g2 * CG + c));
      out = (wl / CG == g2) ? x : out;
    }
    return out;
  } else {
    return __shfl(v, gbase + c, 64);
  }
}

// 1 / sqrt(x) for positive normal x: the hardware estimate (about 23 bits)
// refined by two Newton steps for 1 / y^2 = x, y <- y (3 - x y^2) / 2, each of
// which doubles the correct bits
__device__ __forceinline__ double rsqrt_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int it = 0; it < 2; ++it) y = fma(y, fma(-h * y, y, 0.5), y);
  return y;
}

// Orders the LDS writes of a group before its lanes' reads: every group lies
// within one wave, so a wavefront-scope fence replaces a block barrier
__device__ __forceinline__ void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// (at most 128 registers, four waves per SIMD: a few set-up values spill)
template <typename VT, int CG>
__global__ __launch_bounds__(kNeMaxWaves * 64, 4) void k_factor_ne(
    const int32_t* __restrict__ trowptr, const int32_t* __restrict__ tcol,
    const double* __restrict__ tval, const double* __restrict__ e,
    const int32_t* __restrict__ tp2s, const int32_t* __restrict__ sellT_off, int64_t n,
    const FactorJob* __restrict__ jobs, int njobs, NeLayout L, int* __restrict__ fb_count,
    int32_t* __restrict__ fb_list) {
  constexpr int LD = CG + 1;  // stride of the m x m matrices in LDS
  const int nthr = (int)blockDim.x, G = L.G;
  __shared__ int a_sh, bad_sh;  // the diagonal's position in J; a shift's fallback
  extern __shared__ __align__(16) unsigned char lds[];
  int* J = (int*)(lds + L.off_J);
  int* coff = (int*)(lds + L.off_off);
  double* EJ = (double*)(lds + L.off_E);
  double* H = (double*)(lds + L.off_H);
  double* G0 = (double*)(lds + L.off_G0);
  double* rowA = (double*)(lds + L.off_A);  // Ajj(a, :)
  double* colA = rowA + CG;                 // Ajj(:, a)
  int* crow = (int*)(lds + L.off_crow);
  double* cval = (double*)(lds + L.off_cval);
  const int lane = threadIdx.x, wl = lane & 63, wave = lane >> 6, nw = nthr >> 6;
  const int g = lane / CG, i = lane % CG, gbase = (g * CG) & 63;  // group's first lane in its wave
  if (lane == 0) bad_sh = 0;
  double* Lc = (double*)(lds + L.off_L) + (size_t)g * CG;  // the group's current column of L

  for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
    const int lo = trowptr[k];
    const int m = trowptr[k + 1] - lo;  // <= CG (checked on the host)
    // gather the columns J_k of A in order (rows sorted within a column):
    // every wave scans the column lengths, wave w copies the entries
    // w kNeGather, (w + nw) kNeGather, ... of each column, with all of a
    // group's loads in flight before the first store
    int len = 0, jc = -1, cb = 0;
    if (wl < m) {
      jc = tcol[lo + wl];
      cb = trowptr[jc];
      len = trowptr[jc + 1] - cb;
    }
    int T;
    const int off = wave_excl_scan(len, wl, &T);
    if (wave == 0) {
      if (wl < m) {
        J[wl] = jc;
        EJ[wl] = e[jc];
        coff[wl] = off;
      }
      if (wl == 0) coff[m] = T;
      const unsigned long long am = __ballot(jc == (int)k);
      if (wl == 0) a_sh = am ? (int)__ffsll((long long)am) - 1 : 0;  // the diagonal is in S
    }
    for (int u0 = wave * kNeGather; u0 < len; u0 += nw * kNeGather) {
      int rr[kNeGather];
      double vv[kNeGather];
#pragma unroll
      for (int u = 0; u < kNeGather; ++u) {
        const int uu = min(u0 + u, len - 1);
        rr[u] = tcol[cb + uu];
        vv[u] = tval[cb + uu];
      }
#pragma unroll
      for (int u = 0; u < kNeGather; ++u)
        if (u0 + u < len) {
          crow[off + u0 + u] = rr[u];
          cval[off + u0 + u] = vv[u];
        }
    }
    __syncthreads();
    const int a = a_sh;
    // one pass per column pair r <= l over the union of their sorted rows:
    // G0(r, l) sums the products at common rows; the entry of column l at row
    // J_r is Ajj(r, l) = A(J_r, J_l), the entry of column r at row J_l is
    // Ajj(l, r).  H(r, l) = E_r Ajj(r, l) + E_l Ajj(l, r); row and column a of
    // Ajj are kept for the right-hand sides.
    const int npair = m * (m + 1) / 2;
    for (int p = lane; p < npair; p += nthr) {
      int r = 0, q = p;
      while (q >= m - r) {
        q -= m - r;
        ++r;
      }
      const int l = r + q;
      // Column r holds row J_r (its diagonal) and column l row J_l, so when
      // either list ends the other's entries at those rows, if any, have been
      // passed: the merge stops there.
      int x = coff[r], y = coff[l];
      const int xe = coff[r + 1], ye = coff[l + 1];
      const int jr = J[r], jl = J[l];
      double sg = 0.0, arl = 0.0, alr = 0.0;
      while (x < xe && y < ye) {
        const int rx = crow[x], ry = crow[y];
        const double vx = cval[x], vy = cval[y];
        if (rx == ry) sg = fma(vx, vy, sg);
        if (ry == jr) arl = vy;
        if (rx == jl) alr = vx;
        x += rx <= ry;
        y += ry <= rx;
      }
      G0[r * LD + l] = sg;
      G0[l * LD + r] = sg;
      const double h = fma(EJ[r], arl, EJ[l] * alr);
      H[r * LD + l] = h;
      H[l * LD + r] = h;
      if (r == a) {
        rowA[l] = arl;
        colA[l] = alr;
      }
      if (l == a) {
        colA[r] = arl;
        rowA[r] = alr;
      }
    }
    __syncthreads();  // the gathered columns are dead: their space holds L's columns now
    // per lane: Ajj(a, i), Ajj(i, a), G0(i, a), G0(i, i), H(i, i)
    const bool row = i < m;
    const double ei = row ? EJ[i] : 0.0, ek = EJ[a];
    const double aai = row ? rowA[i] : 0.0;
    const double aia = row ? colA[i] : 0.0;
    const double g0a = row ? G0[i * LD + a] : 0.0;
    const double g0i = row ? G0[i * LD + i] : 0.0;
    const double hii = row ? H[i * LD + i] : 0.0;
    bool bad = false;
    for (int r0 = 0; r0 < njobs; r0 += G) {
      const bool live = r0 + g < njobs;
      const FactorJob job = jobs[live ? r0 + g : njobs - 1];
      const double sn = job.sigma_new, sp = job.sigma_prev;
      // row i of G(sn) = G0 - sn H + sn^2 E_J^2 (identity rows past m) and
      // the right-hand side
      const double dsh = sn * sn * ei * ei;
      double gr[CG];
#pragma unroll
      for (int l = 0; l < CG; ++l) {
        double v = 0.0;
        if (row && l < m) v = fma(-sn, H[i * LD + l], G0[i * LD + l]);
        gr[l] = v + (l == i ? (row ? sn * sn * ei * ei : 1.0) : 0.0);
      }
      const double gd = fma(-sn, hii, g0i) + dsh;  // G(sn)(i, i) as built in gr
      double y = 0.0;
      if (row) {
        if (job.is_spai)
          y = (i == a ? sn * ek : 0.0) - aai;
        else
          y = g0a - sp * ek * aai - sn * ei * aia + (i == a ? sn * sp * ek * ek : 0.0);
      }
      // Cholesky G = L L^T.  After step c lane r >= c holds L(r, c) in
      // gr[c]; lane c skips its update at step c, so after the loop lane i
      // holds L(i, i) L(l, i) in gr[l], l > i, and 1 / L(i, i) in inv (the
      // loops run over all CG positions with uniform guards, so that they
      // unroll completely and gr stays in registers)
      double inv = 0.0;
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        if (c < m) {
          const double piv = group_bcast<CG>(gr[c], gbase, c);
          const double rd = piv > 0.0 ? rsqrt_newton(piv) : 1.0;
          const double d = piv > 0.0 ? piv * rd : 1.0;
          if (i == c && live) bad = bad || !(piv > kNeTol * gd);
          if (i == c) inv = rd;
          const double lic = i > c ? gr[c] * rd : (i == c ? d : 0.0);
          if (i >= c) gr[c] = lic;
          Lc[i] = lic;
          group_sync();
          const double mult = i > c ? lic : 0.0;
#pragma unroll
          for (int l = c + 1; l < CG; ++l)
            if (l < m) gr[l] = fma(-mult, Lc[l], gr[l]);
        }
      }
      // L z = y, then L^T q = z (lane i < c takes L(c, i) q_c as gr[c] q_c
      // and divides the sum by L(i, i) once)
#pragma unroll
      for (int c = 0; c < CG; ++c) {
        if (c < m) {
          const double zc = group_bcast<CG>(y * inv, gbase, c);
          if (i == c) y = zc;
          else if (i > c) y = fma(-gr[c], zc, y);
        }
      }
      double sacc = 0.0;
#pragma unroll
      for (int c = CG - 1; c >= 0; --c) {
        if (c < m) {
          const double qc = group_bcast<CG>(fma(-sacc, inv, y) * inv, gbase, c);
          if (i == c) y = qc;
          else if (i < c) sacc = fma(gr[c], qc, sacc);
        }
      }
      if (row && live) {
        const int64_t posT = (int64_t)sellT_off[k / kSlice] + (int64_t)i * kSlice + (k % kSlice);
        store_val<VT>((VT*)job.valsT + posT, y);
        store_val<VT>((VT*)job.vals + tp2s[lo + i], y);
      }
    }
    if (__ballot(bad) != 0ull && (lane & 63) == 0) atomicOr(&bad_sh, 1);
    __syncthreads();
    if (lane == 0 && bad_sh) {
      fb_list[atomicAdd(fb_count, 1)] = (int32_t)k;
      bad_sh = 0;
    }
  }
}

// ---- block kernel for larger local problems ------------------------------------
//
// One block of BC x BR threads per column (BC = 32: four or eight waves; BC
// = 8 or 16: one wave, for small column patterns).  The dense
// |I_k| x (|J_k| + 1) matrix is held in registers: thread (cc, g) =
// (tid % BC, tid / BC) owns column cc (column |J_k| is the right-hand side)
// at the local rows r = s * BR + g, s < S.  A Householder step stages only the reflector column, row c of
// every column and the per-row-group partial dot products in LDS (double
// buffered by step parity, two barriers per step); the gathered triples stay
// in LDS so every shift rebuilds its matrix without touching global memory.
constexpr int kBCmax = 32;  // column lanes: |J_k| + 1 <= 32

struct BlkLayout {
  int Tpad, Tmax, maxI, S, BR, BC;
  size_t off_keys, off_trow, off_tv, off_uniq, off_R, off_col, off_v, off_rowc, off_part, bytes;
};

BlkLayout blk_layout(int maxT, int maxI, int S, int BR, int BC) {
  BlkLayout L;
  L.Tmax = std::max(maxT, 1);
  L.Tpad = 64;
  while (L.Tpad < L.Tmax) L.Tpad <<= 1;
  L.maxI = std::max(maxI, 1);
  L.S = S;
  L.BR = BR;
  L.BC = BC;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 15) / 16 * 16;
    return r;
  };
  // Per column: the gather and sort arrays (keys, triples, values, rows I_k),
  // then in the same space the dense -A(I_k, J_k), BC columns of S * BR rows,
  // which every shift reads to build its matrix.
  size_t gather = 0;
  auto add = [&](size_t bytes) {
    size_t r = gather;
    gather += (bytes + 15) / 16 * 16;
    return r;
  };
  L.off_keys = add((size_t)L.Tpad * 4);
  L.off_trow = add((size_t)L.Tmax * 4);
  L.off_tv = add((size_t)L.Tmax * 8);
  L.off_uniq = add((size_t)L.maxI * 4);
  take(std::max(gather, (size_t)BC * S * BR * 8));
  L.off_R = take((size_t)BC * (BC + 1) * 8);  // R staging of the back substitution
  L.off_col = take((size_t)(3 * BC + 8) * 4);  // J, triple offsets (+1), diagonal rows, misc
  L.off_v = take((size_t)2 * S * BR * 8);
  L.off_rowc = take((size_t)2 * BC * 8);
  L.off_part = take((size_t)2 * BR * BC * 8);
  L.bytes = o;
  return L;
}

// (up to 16 slots: at least 3 blocks per CU; the steps are latency bound, so
// blocks in flight matter more than registers)
template <typename VT, int S, int BR, int BC>
__global__ __launch_bounds__(BC * BR, (S <= 16 ? 3 : 1)) void k_factor_ls_blk(
    const int32_t* __restrict__ trowptr, const int32_t* __restrict__ tcol,
    const double* __restrict__ tval, const double* __restrict__ e,
    const int32_t* __restrict__ tp2s, const int32_t* __restrict__ sellT_off, int64_t n,
    const FactorJob* __restrict__ jobs, int njobs, BlkLayout L, int* __restrict__ status) {
  constexpr int kBC = BC;
  constexpr int kRld = BC + 1;  // row stride of the R staging buffer
  extern __shared__ __align__(16) unsigned char lds[];
  int* keys = (int*)(lds + L.off_keys);
  double* base = (double*)lds;  // -A(I_k, J_k) once the gather arrays are done
  double* R = (double*)(lds + L.off_R);
  int* trow = (int*)(lds + L.off_trow);
  double* tv = (double*)(lds + L.off_tv);
  int* uniq = (int*)(lds + L.off_uniq);
  int* colJ = (int*)(lds + L.off_col);
  int* coloff = colJ + kBC;        // kBC + 1 entries
  int* coldiag = colJ + 2 * kBC + 1;
  int* misc = colJ + 3 * kBC + 1;  // T, nI, kloc, ak
  double* vbuf = (double*)(lds + L.off_v);
  double* rowc = (double*)(lds + L.off_rowc);
  double* part = (double*)(lds + L.off_part);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cc = tid % kBC, g = tid / kBC;
  constexpr int kBR = BR;
  constexpr int kBT = kBC * BR;
  constexpr int VS = S * kBR;  // rows held per column (>= |I_k|)

  for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
    const int lo = trowptr[k];
    const int m = trowptr[k + 1] - lo;
    // gather the nonzeros of S[:, J_k] in column order (wave 0)
    if (wave == 0) {
      int len = 0, j = 0;
      if (lane < m) {
        j = tcol[lo + lane];
        colJ[lane] = j;
        len = trowptr[j + 1] - trowptr[j];
      }
      int T;
      const int off = wave_excl_scan(len, lane, &T);
      if (lane < m) {
        coloff[lane] = off;
        const int b = trowptr[j];
        for (int u = 0; u < len; ++u) {
          const int row = tcol[b + u];
          trow[off + u] = row;
          keys[off + u] = row;
          tv[off + u] = tval[b + u];
        }
      }
      if (lane == 0) {
        coloff[m] = T;
        misc[0] = T;
      }
    }
    __syncthreads();
    const int T = misc[0];
    for (int t = T + tid; t < L.Tpad; t += kBT) keys[t] = 0x7fffffff;
    __syncthreads();
    // bitonic sort of the row indices
    for (int size = 2; size <= L.Tpad; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int t = tid; t < L.Tpad; t += kBT) {
          const int p = t ^ stride;
          if (p > t) {
            const int a = keys[t], b = keys[p];
            const bool up = ((t & size) == 0);
            if ((a > b) == up) {
              keys[t] = b;
              keys[p] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    // unique rows I_k (wave 0)
    if (wave == 0) {
      int base = 0;
      for (int t0 = 0; t0 < T; t0 += 64) {
        const int t = t0 + lane;
        const bool first = (t < T) && (t == 0 || keys[t] != keys[t - 1]);
        const unsigned long long mask = __ballot(first);
        const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (first) uniq[pos] = keys[t];
        base += __popcll(mask);
      }
      if (lane == 0) misc[1] = base;
    }
    __syncthreads();
    const int nI = misc[1];
    // every triple as (local row << 5) | local column, in column order (rows
    // ascending within a column); the local row of every column's own index
    for (int t = tid; t < T; t += kBT) {
      int a = 0;
      while (a + 1 < m && coloff[a + 1] <= t) ++a;
      trow[t] = (find_row(uniq, nI, trow[t]) << 5) | a;
    }
    if (tid < m) {
      coldiag[tid] = find_row(uniq, nI, colJ[tid]);
      if (colJ[tid] == (int)k) misc[3] = tid;
    }
    if (tid == 0) misc[2] = find_row(uniq, nI, (int)k);
    __syncthreads();
    const int kloc = misc[2], ak = misc[3];
    // dense -A(I_k, J_k): each thread merges its column's triples (rows
    // ascending) into its rows, then stores them over the gather arrays
    {
      double B0[S];
      int p = cc < m ? coloff[cc] : 0;
      const int pe = cc < m ? coloff[cc + 1] : 0;
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) {
        const int r = s2 * kBR + g;
        double x = 0.0;
        while (p < pe && (trow[p] >> 5) < r) ++p;
        if (p < pe && (trow[p] >> 5) == r) x = -tv[p];
        B0[s2] = x;
      }
      __syncthreads();
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) base[cc * VS + s2 * kBR + g] = B0[s2];
      __syncthreads();
    }
    // the shifted diagonal entry of this thread's column: column cc of
    // A_new, or for an update's right-hand side A_prev(I_k, k) = column ak
    const int acol = (cc == m) ? ak : min(cc, max(m - 1, 0));
    const int dl = (cc <= m) ? coldiag[acol] : -1;
    const double ej = (cc <= m) ? e[colJ[acol]] : 0.0;

    for (int jb = 0; jb < njobs; ++jb) {
      const FactorJob job = jobs[jb];
      // this thread's column of [A_new(I_k, J_k) | rhs]
      double M[S];
      const bool rhs = (cc == m);
      if (cc < m || (rhs && !job.is_spai)) {
        const double dv = (rhs ? job.sigma_prev : job.sigma_new) * ej;
#pragma unroll
        for (int s2 = 0; s2 < S; ++s2) {
          const int r = s2 * kBR + g;
          const double x = base[acol * VS + r];
          M[s2] = (r == dl) ? x + dv : x;
        }
      } else {
#pragma unroll
        for (int s2 = 0; s2 < S; ++s2) M[s2] = (rhs && s2 * kBR + g == kloc) ? 1.0 : 0.0;
      }
      // Householder QR of the m columns, applied to the right-hand side too
      bool singular = false;
      double rmax = 0.0;  // largest |R_aa| so far
      for (int c = 0; c < m; ++c) {
        const int buf = c & 1;
        double* vb = vbuf + buf * VS;
        if (cc == c) {
#pragma unroll
          for (int s2 = 0; s2 < S; ++s2) vb[s2 * kBR + g] = M[s2];
        }
        if (g == c % kBR) {
          double x = 0.0;
#pragma unroll
          for (int s2 = 0; s2 < S; ++s2) x = (s2 == c / kBR) ? M[s2] : x;
          rowc[buf * kBC + cc] = x;
        }
        __syncthreads();
        const double x0 = vb[c];
        double pp[2] = {0.0, 0.0};  // two chains: even and odd slots
#pragma unroll
        for (int s2 = 0; s2 < S; ++s2) {
          const int r = s2 * kBR + g;
          const double x = (r >= c) ? vb[r] : 0.0;
          pp[s2 & 1] = fma(x, M[s2], pp[s2 & 1]);
        }
        part[(buf * kBR + g) * kBC + cc] = pp[0] + pp[1];
        __syncthreads();
        double sc = 0.0, n2 = 0.0;
        {
          double a4[4] = {0.0, 0.0, 0.0, 0.0}, b4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int g2 = 0; g2 < kBR; ++g2) {
            a4[g2 & 3] += part[(buf * kBR + g2) * kBC + cc];
            b4[g2 & 3] += part[(buf * kBR + g2) * kBC + c];
          }
          sc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
          n2 = (b4[0] + b4[1]) + (b4[2] + b4[3]);
        }
        const double scale = fmax(rmax, fabs(x0));
        if (!(n2 > 0.0) || sqrt(n2) <= 1e-14 * fmax(scale, 1e-300)) singular = true;
        const double alpha = (x0 > 0.0) ? -sqrt(n2) : sqrt(n2);
        const double vtv = 2.0 * alpha * (alpha - x0);
        if (cc > c && cc <= m && vtv > 0.0) {
          const double d = sc - alpha * rowc[buf * kBC + cc];
          const double tau = 2.0 * d / vtv;
#pragma unroll
          for (int s2 = 0; s2 < S; ++s2) {
            const int r = s2 * kBR + g;
            const double w = (r == c) ? (x0 - alpha) : ((r > c) ? vb[r] : 0.0);
            M[s2] = fma(-tau, w, M[s2]);
          }
        }
        if (cc == c) {
#pragma unroll
          for (int s2 = 0; s2 < S; ++s2) M[s2] = (s2 * kBR + g == c) ? alpha : M[s2];
        }
        rmax = fmax(rmax, fabs(alpha));
      }
      // back substitution R q = (Q^T rhs)(0:m), one wave, column by column
      __syncthreads();
      if (cc <= m) {
#pragma unroll
        for (int s2 = 0; s2 < S; ++s2) {
          const int r = s2 * kBR + g;
          if (r < m) R[r * kRld + cc] = M[s2];
        }
      }
      __syncthreads();
      if (wave == 0) {
        double y = (lane < m) ? R[lane * kRld + m] : 0.0;
        // reciprocals of R's diagonal up front, off the loop's critical path
        const double rinv = (lane < m) ? 1.0 / R[lane * kRld + lane] : 0.0;
        double q = 0.0;
        for (int i = m - 1; i >= 0; --i) {
          const double qi = __shfl(y, i, 64) * __shfl(rinv, i, 64);
          if (lane == i) q = qi;
          if (lane < i) y = fma(-R[lane * kRld + i], qi, y);
        }
        if (lane < m) {
          const double v = singular ? 0.0 : q;
          const int64_t posT =
              (int64_t)sellT_off[k / kSlice] + (int64_t)lane * kSlice + (k % kSlice);
          store_val<VT>((VT*)job.valsT + posT, v);
          store_val<VT>((VT*)job.vals + tp2s[trowptr[k] + lane], v);
        }
        if (singular && lane == 0) atomicOr(status, 1);
      }
      __syncthreads();
    }
  }
}

// Register slots per thread of the register kernels: rows per column / BR.
int blk_slots(int maxI, int BR) {
  int S = 2;
  while (S * BR < maxI) S <<= 1;
  return S;
}

// Shape of a register least-squares variant: factor_kernel 1 is one wave per
// column (BC = 8 or 16 column lanes), 8 and 16 one block of 32 x BR threads.
struct BlkShape {
  int BC, BR, S;
};

bool blk_shape(morx_system sys, int variant, BlkShape* out) {
  BlkShape b{};
  if (variant == 1) {
    if (sys->max_J + 1 > 16) return false;
    b.BC = sys->max_J + 1 <= 8 ? 8 : 16;
    b.BR = 64 / b.BC;
    b.S = blk_slots(sys->max_I, b.BR);
    if (b.S > (b.BC == 8 ? 16 : 32)) return false;
  } else if (variant == 8 || variant == 16) {
    if (sys->max_J + 1 > kBCmax) return false;
    b.BC = kBCmax;
    b.BR = variant;
    b.S = std::max(4, blk_slots(sys->max_I, b.BR));
    if (b.S > (variant == 16 ? 16 : 32)) return false;
  } else {
    return false;
  }
  if (blk_layout(sys->max_T, sys->max_I, b.S, b.BR, b.BC).bytes > (size_t)kLdsBudget) return false;
  *out = b;
  return true;
}

// The register variant that builds this system's factors, or 0 for the
// per-wave LDS kernel.  The system's tuned choice wins when it is set;
// otherwise small column patterns keep the per-wave kernel and larger ones
// take the 32 x 16 block.
int blk_variant(morx_system sys) {
  int v = sys->tune_factor_rows;
  if (v == 2) return 0;
  if (v < 0) v = sys->max_J < 12 ? 0 : 16;
  BlkShape b;
  if (v == 16 && !blk_shape(sys, 16, &b)) v = 8;
  return (v != 0 && blk_shape(sys, v, &b)) ? v : 0;
}

int ls_grid(morx_system sys) {
  int64_t cap = (int64_t)std::max(sys->ctx->num_cu, 1) * 64;
  return (int)std::min<int64_t>(sys->n, std::max<int64_t>(cap, 1));
}

}  // namespace

// column lanes of the normal-equations kernel, or 0 when it does not apply
static int ne_lanes(morx_system sys) {
  if (!sys->ls_supported || sys->max_J > 32) return 0;
  const int cg = sys->max_J <= 8 ? 8 : (sys->max_J <= 16 ? 16 : 32);
  return ne_layout(sys->max_T, cg, 1).bytes <= (size_t)kLdsBudget ? cg : 0;
}

// Waves per normal-equations block: the count whose resident blocks per CU
// finish the most columns per unit of time.  A block's time per column is its
// set-up (gathers, G0, H; shared by its waves) plus one round of shifts per
// G of them; on the 27-point job (|J_k| = 27) the set-up measured 1.37 rounds
// with one wave, about nw^-0.6 of that with nw (builds of 1, 4, 6 and 12
// shifts: 96.6, 78.6, 85.0 and 133.6 ms at one, two, three and three waves)
template <typename VT, int CG>
static int ne_waves(int njobs, int maxT) {
  int best_nw = 1;
  double best = -1.0;
  for (int nw = 1; nw <= kNeMaxWaves; ++nw) {
    const NeLayout N = ne_layout(maxT, CG, nw);
    if (N.bytes > (size_t)kLdsBudget) break;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_factor_ne<VT, CG>, nw * 64,
                                                     N.bytes) != hipSuccess)
      nb = 0;
    const int rounds = (njobs + N.G - 1) / N.G;
    const double score = nb / (1.37 * pow((double)nw, -0.6) + rounds);
    if (score > best + 1e-9) {
      best = score;
      best_nw = nw;
    }
  }
  return best_nw;
}

bool factor_kernel_supported(morx_system sys, int variant) {
  if (!sys->ls_supported) return false;
  if (variant == 0) return true;
  if (variant == 2) return ne_lanes(sys) > 0;
  BlkShape b;
  return blk_shape(sys, variant, &b);
}

morx_status ls_pattern_stats(morx_system sys, hipStream_t st) {
  DevBuf sb;
  MORX_TRY(dev_alloc(sb, 4 * sizeof(int)));
  MORX_HIP(hipMemsetAsync(sb.p, 0, 4 * sizeof(int), st));
  int* stats = (int*)sb.p;
  k_ls_count<<<(unsigned)((sys->n + 255) / 256), 256, 0, st>>>(sys->trowptr, sys->tcol, sys->n,
                                                              stats);
  int h[4] = {0, 0, 0, 0};
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) err = hipMemcpyAsync(h, stats, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  if (err != hipSuccess) {
    dev_free(sb);
    morx_set_error("ls_pattern_stats: %s", hipGetErrorString(err));
    return MORX_E_HIP;
  }
  sys->max_J = h[0];
  sys->max_T = h[1];
  sys->ls_supported = (h[0] <= kMaxJ && h[1] <= kMaxTriples);
  if (sys->ls_supported) {
    // the unique-row pass needs room for up to T rows and no dense matrix
    LsLayout L = ls_layout(h[0], h[1], h[1]);
    L.bytes = L.off_M;
    k_ls_unique<<<ls_grid(sys), 64, L.bytes, st>>>(sys->trowptr, sys->tcol, sys->n, L, stats);
    err = hipGetLastError();
    if (err == hipSuccess) err = hipMemcpyAsync(h, stats, 4 * sizeof(int), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) {
      dev_free(sb);
      morx_set_error("ls_pattern_stats: %s", hipGetErrorString(err));
      return MORX_E_HIP;
    }
    sys->max_I = h[2];
    LsLayout L2 = ls_layout(sys->max_J, sys->max_T, sys->max_I);
    sys->ls_supported = (sys->max_I <= kMaxI) && (L2.bytes <= (size_t)kLdsBudget);
  }
  dev_free(sb);
  return MORX_OK;
}

morx_status factor_alloc(morx_system sys, int32_t prec, morx_factor* out) {
  for (size_t i = 0; i < sys->factor_pool.size(); ++i) {
    if (sys->factor_pool[i]->prec == prec) {
      *out = sys->factor_pool[i];
      sys->factor_pool.erase(sys->factor_pool.begin() + i);
      return MORX_OK;
    }
  }
  morx_factor f = new morx_factor_s();
  f->sys = sys;
  f->prec = prec;
  f->pooled = true;
  const size_t b = prec_bytes(prec);
  morx_status s = dev_alloc(f->vals, (size_t)(sys->sell.nnz_sell + kSellPad) * b);
  if (s == MORX_OK) s = dev_alloc(f->valsT, (size_t)(sys->sellT.nnz_sell + kSellPad) * b);
  if (s != MORX_OK) {
    dev_free(f->vals);
    dev_free(f->valsT);
    delete f;
    return s;
  }
  // padding slots are never written by the least-squares kernel: zero them once
  hipStream_t st = sys->ctx->stream;
  int64_t w1 = (int64_t)(f->vals.bytes / 4), w2 = (int64_t)(f->valsT.bytes / 4);
  k_fill_zero_bytes<<<(unsigned)((w1 + 255) / 256), 256, 0, st>>>((uint32_t*)f->vals.p, w1);
  k_fill_zero_bytes<<<(unsigned)((w2 + 255) / 256), 256, 0, st>>>((uint32_t*)f->valsT.p, w2);
  MORX_HIP(hipGetLastError());
  // the factor may be built on another stream: the zeros must land first
  MORX_HIP(hipStreamSynchronize(st));
  *out = f;
  return MORX_OK;
}

void factor_release(morx_factor f) {
  if (!f) return;
  f->sys->factor_pool.push_back(f);
}

void factor_discard(morx_factor f) {
  if (!f) return;
  dev_free(f->vals);
  dev_free(f->valsT);
  delete f;
}

morx_status factor_build_many(morx_system sys, int32_t prec, const FactorJob* jobs, int njobs,
                              hipStream_t st) {
  MORX_REQUIRE(sys->ls_supported, MORX_E_UNSUPPORTED,
               "factor pattern exceeds the local least-squares limits (|J_k|=%d, triples=%d, "
               "|I_k|=%d)",
               sys->max_J, sys->max_T, sys->max_I);
  if (njobs <= 0) return MORX_OK;
  LsLayout L = ls_layout(sys->max_J, sys->max_T, sys->max_I);
  DevBuf jb, sb;
  MORX_TRY(dev_alloc(jb, njobs * sizeof(FactorJob)));
  MORX_TRY(dev_alloc(sb, 2 * sizeof(int)));  // rank-deficient flag, normal-equations fallbacks
  MORX_HIP(hipMemcpyAsync(jb.p, jobs, njobs * sizeof(FactorJob), hipMemcpyHostToDevice, st));
  MORX_HIP(hipMemsetAsync(sb.p, 0, 2 * sizeof(int), st));
  const int grid = ls_grid(sys);
  void* token = nullptr;
  trace_factor_begin(sys->ctx, st, &token);
  const int variant = blk_variant(sys);
  const int cg = (sys->tune_factor_rows == 2 || sys->tune_factor_rows < 0) ? ne_lanes(sys) : 0;
  int32_t* fb_list = nullptr;
  if (cg > 0) {
    if (!sys->ls_fallback) {
      DevBuf fb;
      MORX_TRY(dev_alloc(fb, (size_t)sys->n * sizeof(int32_t)));
      sys->owned.push_back(fb);
      sys->resident_bytes += (int64_t)fb.bytes;
      sys->ls_fallback = (int32_t*)fb.p;
    }
    fb_list = sys->ls_fallback;
  }
  BlkShape bs{};
  if (cg > 0) {
    // many short-lived workgroups (about 16 columns each on the 27-point job):
    // 512 per CU built the 12-shift set in 134 ms, 128 per CU in 136 ms, 32
    // per CU in 141 ms, one per resident slot in 155 ms
    const int ngrid = (int)std::min<int64_t>(sys->n, (int64_t)std::max(sys->ctx->num_cu, 1) * 512);
    int* fb_count = (int*)sb.p + 1;
#define MORX_NE_LAUNCH(VT, CGV)                                                                 \
  do {                                                                                          \
    const int nw = ne_waves<VT, CGV>(njobs, sys->max_T);                                        \
    const NeLayout N = ne_layout(sys->max_T, CGV, nw);                                          \
    k_factor_ne<VT, CGV><<<ngrid, nw * 64, N.bytes, st>>>(sys->trowptr, sys->tcol, sys->tval,   \
                                                          sys->e, sys->tp2s, sys->sellT.off,    \
                                                          sys->n, (FactorJob*)jb.p, njobs, N,   \
                                                          fb_count, fb_list);                   \
  } while (0)
#define MORX_NE_CG(VT)                 \
  if (cg == 8) MORX_NE_LAUNCH(VT, 8);   \
  else if (cg == 16) MORX_NE_LAUNCH(VT, 16); \
  else MORX_NE_LAUNCH(VT, 32);
    // then the Householder kernel on the columns the normal equations listed
#define MORX_NE_FALLBACK(VT)                                                                    \
  k_factor_ls<VT><<<grid, 64, L.bytes, st>>>(sys->trowptr, sys->tcol, sys->tval, sys->e,         \
                                            sys->tp2s, sys->sellT.off, sys->n, (FactorJob*)jb.p, \
                                            njobs, L, (int*)sb.p, fb_list, fb_count)
    if (prec == MORX_F64) { MORX_NE_CG(double) MORX_NE_FALLBACK(double); }
    else if (prec == MORX_F32) { MORX_NE_CG(float) MORX_NE_FALLBACK(float); }
    else { MORX_NE_CG(uint16_t) MORX_NE_FALLBACK(uint16_t); }
#undef MORX_NE_FALLBACK
#undef MORX_NE_CG
#undef MORX_NE_LAUNCH
  } else if (variant > 0 && blk_shape(sys, variant, &bs)) {
    const int S = bs.S, BR = bs.BR, BC = bs.BC;
    const BlkLayout B = blk_layout(sys->max_T, sys->max_I, S, BR, BC);
    // one-wave blocks: more of them to fill the CUs
    const int per_cu = BC == kBCmax ? 8 : 32;
    const int bgrid =
        (int)std::min<int64_t>(sys->n, (int64_t)std::max(sys->ctx->num_cu, 1) * per_cu);
#define MORX_BLK_LAUNCH(VT, SV, BRV, BCV)                                                 \
  k_factor_ls_blk<VT, SV, BRV, BCV><<<bgrid, BCV * BRV, B.bytes, st>>>(                    \
      sys->trowptr, sys->tcol, sys->tval, sys->e, sys->tp2s, sys->sellT.off, sys->n,      \
      (FactorJob*)jb.p, njobs, B, (int*)sb.p)
#define MORX_BLK_S(VT)                                                   \
  if (BC == 8) {                                                         \
    switch (S) {                                                         \
      case 2: MORX_BLK_LAUNCH(VT, 2, 8, 8); break;                       \
      case 4: MORX_BLK_LAUNCH(VT, 4, 8, 8); break;                       \
      case 8: MORX_BLK_LAUNCH(VT, 8, 8, 8); break;                       \
      default: MORX_BLK_LAUNCH(VT, 16, 8, 8); break;                     \
    }                                                                    \
  } else if (BC == 16) {                                                 \
    switch (S) {                                                         \
      case 2: case 4: MORX_BLK_LAUNCH(VT, 4, 4, 16); break;              \
      case 8: MORX_BLK_LAUNCH(VT, 8, 4, 16); break;                      \
      case 16: MORX_BLK_LAUNCH(VT, 16, 4, 16); break;                    \
      default: MORX_BLK_LAUNCH(VT, 32, 4, 16); break;                    \
    }                                                                    \
  } else if (BR == 8) {                                                  \
    switch (S) {                                                         \
      case 4: MORX_BLK_LAUNCH(VT, 4, 8, 32); break;                      \
      case 8: MORX_BLK_LAUNCH(VT, 8, 8, 32); break;                      \
      case 16: MORX_BLK_LAUNCH(VT, 16, 8, 32); break;                    \
      default: MORX_BLK_LAUNCH(VT, 32, 8, 32); break;                    \
    }                                                                    \
  } else {                                                               \
    switch (S) {                                                         \
      case 4: MORX_BLK_LAUNCH(VT, 4, 16, 32); break;                     \
      case 8: MORX_BLK_LAUNCH(VT, 8, 16, 32); break;                     \
      default: MORX_BLK_LAUNCH(VT, 16, 16, 32); break;                   \
    }                                                                    \
  }
    if (prec == MORX_F64) { MORX_BLK_S(double) }
    else if (prec == MORX_F32) { MORX_BLK_S(float) }
    else { MORX_BLK_S(uint16_t) }
#undef MORX_BLK_S
#undef MORX_BLK_LAUNCH
  } else switch (prec) {
    case MORX_F64:
      k_factor_ls<double><<<grid, 64, L.bytes, st>>>(sys->trowptr, sys->tcol, sys->tval, sys->e,
                                                     sys->tp2s, sys->sellT.off, sys->n,
                                                     (FactorJob*)jb.p, njobs, L, (int*)sb.p,
                                                     nullptr, nullptr);
      break;
    case MORX_F32:
      k_factor_ls<float><<<grid, 64, L.bytes, st>>>(sys->trowptr, sys->tcol, sys->tval, sys->e,
                                                    sys->tp2s, sys->sellT.off, sys->n,
                                                    (FactorJob*)jb.p, njobs, L, (int*)sb.p,
                                                    nullptr, nullptr);
      break;
    default:
      k_factor_ls<uint16_t><<<grid, 64, L.bytes, st>>>(sys->trowptr, sys->tcol, sys->tval,
                                                       sys->e, sys->tp2s, sys->sellT.off, sys->n,
                                                       (FactorJob*)jb.p, njobs, L, (int*)sb.p,
                                                       nullptr, nullptr);
  }
  trace_factor_end(sys->ctx, st, token);
  MORX_HIP(hipGetLastError());
  int singular = 0;
  MORX_HIP(hipMemcpyAsync(&singular, sb.p, sizeof(int), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipStreamSynchronize(st));
  dev_free(jb);
  dev_free(sb);
  MORX_REQUIRE(!singular, MORX_E_SINGULAR_LS, "a local least-squares matrix is rank deficient");
  return MORX_OK;
}

// ---------------------------------------------------------------------------

static morx_status factor_make(morx_system sys, bool spai, double sp, double sn, int32_t prec,
                               void* stream, morx_factor* out) {
  MORX_REQUIRE(sys && out, MORX_E_INVALID, "factor: null argument");
  MORX_REQUIRE(prec >= MORX_F64 && prec <= MORX_BF16, MORX_E_INVALID, "factor: bad precision");
  MORX_REQUIRE(std::isfinite(sn) && (spai || std::isfinite(sp)), MORX_E_NONFINITE, "factor: shift not finite");
  *out = nullptr;
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  MORX_TRY(stream_enter(ctx, (hipStream_t)stream));
  morx_factor f = nullptr;
  MORX_TRY(factor_alloc(sys, prec, &f));
  f->is_spai = spai;
  f->sigma_prev = sp;
  f->sigma_new = sn;
  FactorJob job{sn, sp, spai ? 1 : 0, f->vals.p, f->valsT.p};
  morx_status s = factor_build_many(sys, prec, &job, 1, ctx->stream);
  if (s != MORX_OK) {
    factor_release(f);
    return s;
  }
  MORX_TRY(stream_leave(ctx, (hipStream_t)stream));
  *out = f;
  return MORX_OK;
}

extern "C" morx_status morx_factor_spai(morx_system sys, double sigma, int32_t prec, void* stream,
                                        morx_factor* out) {
  return factor_make(sys, true, 0.0, sigma, prec, stream, out);
}

extern "C" morx_status morx_factor_update(morx_system sys, double sigma_prev, double sigma_new,
                                          int32_t prec, void* stream, morx_factor* out) {
  return factor_make(sys, false, sigma_prev, sigma_new, prec, stream, out);
}

extern "C" morx_status morx_factor_values(morx_factor f, double* val, void* stream) {
  MORX_REQUIRE(f && val, MORX_E_INVALID, "morx_factor_values: null argument");
  morx_system sys = f->sys;
  std::lock_guard<std::mutex> lk(sys->ctx->mu);
  MORX_HIP(hipSetDevice(sys->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  unsigned g = (unsigned)((sys->nnzS + 255) / 256);
  switch (f->prec) {
    case MORX_F64:
      k_factor_to_csr<double><<<g, 256, 0, st>>>((double*)f->vals.p, sys->csr2sell, sys->nnzS, val);
      break;
    case MORX_F32:
      k_factor_to_csr<float><<<g, 256, 0, st>>>((float*)f->vals.p, sys->csr2sell, sys->nnzS, val);
      break;
    default:
      k_factor_to_csr<uint16_t><<<g, 256, 0, st>>>((uint16_t*)f->vals.p, sys->csr2sell, sys->nnzS,
                                                    val);
  }
  MORX_HIP(hipGetLastError());
  MORX_HIP(hipStreamSynchronize(st));
  return MORX_OK;
}

extern "C" morx_status morx_factor_destroy(morx_factor f) {
  if (!f) return MORX_OK;
  std::lock_guard<std::mutex> lk(f->sys->ctx->mu);
  hipSetDevice(f->sys->ctx->device);
  hipStreamSynchronize(f->sys->ctx->stream);
  factor_release(f);
  return MORX_OK;
}

extern "C" morx_status morx_factor_build(morx_system sys, int32_t njobs,
                                         const morx_factor_spec* jobs, int32_t prec, void* stream,
                                         morx_factor* out) {
  MORX_REQUIRE(sys && jobs && out, MORX_E_INVALID, "morx_factor_build: null argument");
  MORX_REQUIRE(njobs >= 1 && njobs <= 4096, MORX_E_INVALID, "morx_factor_build: njobs must be 1..4096");
  MORX_REQUIRE(prec >= MORX_F64 && prec <= MORX_BF16, MORX_E_INVALID, "morx_factor_build: bad precision");
  for (int j = 0; j < njobs; ++j)
    MORX_REQUIRE(std::isfinite(jobs[j].sigma_new) && (jobs[j].is_spai || std::isfinite(jobs[j].sigma_prev)),
                 MORX_E_NONFINITE, "morx_factor_build: shift of job %d not finite", j);
  for (int j = 0; j < njobs; ++j) out[j] = nullptr;
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  MORX_TRY(stream_enter(ctx, (hipStream_t)stream));
  std::vector<morx_factor> fs;
  std::vector<FactorJob> fj;
  morx_status s = MORX_OK;
  for (int j = 0; j < njobs && s == MORX_OK; ++j) {
    morx_factor f = nullptr;
    s = factor_alloc(sys, prec, &f);
    if (s != MORX_OK) break;
    f->is_spai = jobs[j].is_spai != 0;
    f->sigma_prev = f->is_spai ? 0.0 : jobs[j].sigma_prev;
    f->sigma_new = jobs[j].sigma_new;
    fs.push_back(f);
    fj.push_back(FactorJob{f->sigma_new, f->sigma_prev, f->is_spai ? 1 : 0, f->vals.p, f->valsT.p});
  }
  if (s == MORX_OK) s = factor_build_many(sys, prec, fj.data(), njobs, ctx->stream);
  if (s != MORX_OK) {
    hipStreamSynchronize(ctx->stream);
    for (morx_factor f : fs) factor_release(f);
    return s;
  }
  MORX_TRY(stream_leave(ctx, (hipStream_t)stream));
  for (int j = 0; j < njobs; ++j) out[j] = fs[j];
  return MORX_OK;
}

extern "C" morx_status morx_factor_import(morx_system sys, const double* val, int32_t prec,
                                          void* stream, morx_factor* out) {
  MORX_REQUIRE(sys && val && out, MORX_E_INVALID, "morx_factor_import: null argument");
  MORX_REQUIRE(prec >= MORX_F64 && prec <= MORX_BF16, MORX_E_INVALID, "morx_factor_import: bad precision");
  *out = nullptr;
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  morx_factor f = nullptr;
  MORX_TRY(factor_alloc(sys, prec, &f));
  f->is_spai = true;
  f->sigma_prev = 0.0;
  f->sigma_new = 0.0;
  const unsigned g1 = (unsigned)((sys->nnzS + 255) / 256), g2 = (unsigned)((sys->n + 255) / 256);
  switch (prec) {
    case MORX_F64:
      k_import_sell<double><<<g1, 256, 0, st>>>(val, sys->csr2sell, sys->nnzS, (double*)f->vals.p);
      k_import_sellT<double><<<g2, 256, 0, st>>>((const double*)f->vals.p, sys->trowptr, sys->tp2s,
                                                 sys->sellT.off, sys->n, (double*)f->valsT.p);
      break;
    case MORX_F32:
      k_import_sell<float><<<g1, 256, 0, st>>>(val, sys->csr2sell, sys->nnzS, (float*)f->vals.p);
      k_import_sellT<float><<<g2, 256, 0, st>>>((const float*)f->vals.p, sys->trowptr, sys->tp2s,
                                                sys->sellT.off, sys->n, (float*)f->valsT.p);
      break;
    default:
      k_import_sell<uint16_t><<<g1, 256, 0, st>>>(val, sys->csr2sell, sys->nnzS,
                                                  (uint16_t*)f->vals.p);
      k_import_sellT<uint16_t><<<g2, 256, 0, st>>>((const uint16_t*)f->vals.p, sys->trowptr,
                                                   sys->tp2s, sys->sellT.off, sys->n,
                                                   (uint16_t*)f->valsT.p);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    factor_release(f);
    morx_set_error("morx_factor_import: %s", hipGetErrorString(e));
    return MORX_E_HIP;
  }
  *out = f;
  return MORX_OK;
}
