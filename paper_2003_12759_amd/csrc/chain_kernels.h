// Iteration state shared by the BiCG driver (bicg.hip) and the chain-step
// translation units (chain_f64.hip, chain_f32.hip, chain_bf16.hip): the
// launch arguments, the device helpers, and the three chain kernels (row
// gathers for patterns up to eight slots wide, row gathers for wider ones,
// and the halo layout in LDS).  The chain kernels are instantiated once per
// factor storage precision, each in its own file, so that they compile side
// by side.
#pragma once

#include <math.h>

#include <type_traits>

#include "krylov.h"

// FP64 Krylov vectors of a slot
enum Vec : int { V_X, V_XT, V_R, V_RT, V_P0, V_P1, V_PT0, V_PT1, V_Q, V_QT, kNumVec };
// vectors of the preconditioner apply, in the apply precision: z, z~, the
// ping-pong intermediates of both chains and (FP32 apply only) the rounded
// copies of r, r~ that the first factor pass reads
enum ApplyVec : int { A_Z, A_ZT, A_T0, A_T1, A_TT0, A_TT1, A_R, A_RT };

constexpr int kMaxNC = 16;         // columns per wave (tuned)
constexpr int kDefaultNC = 8;      // columns per wave without tuning
constexpr int kMaxBlocks = 1024;   // row blocks per launch (partials per column)
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;
constexpr int kFinThreads = 1024;  // finalize kernels: one wave per column
constexpr double kBreakdown = 1e-14;

// Launch geometry shared by every iteration kernel.  A block has four waves;
// each wave owns spw consecutive 64-row slices and handles the NC columns
// blockIdx.y * NC ... of the batch on them, so index and value loads of the
// matrix or factor are shared by all NC columns.  Block indices are remapped
// so that consecutive row ranges run on one XCD (workgroups are dealt to the
// 8 XCDs round robin), keeping a range's stencil neighbours in that XCD's L2.
// one (half, column) pair of a chain step: the factor it applies and the
// vectors it reads and writes
struct ChainItem {
  const void* fv;   // factor values, forward or transposed order
  const void* src;  // input (apply precision)
  void* dst;        // output (apply precision)
  int32_t c;        // column slot; -1: padding or past the list
  // bit 0: transposed chain on the rows of S^T; on the first pair of a chunk
  // also bit 1: every pair of the chunk applies the same factor, and bits
  // 8 and up: pairs in the chunk
  int32_t flags;
};

struct IterArgs {
  int64_t n, ld, nnzS, nslices;
  int64_t nsell, nsellT;  // entries of the sliced-ELL arrays of S and S^T
  int cap, nc, nblk, spw, vbytes, maxL, lcap;
  int ncmax;       // most columns per wave, chain step
  int ncmax_spmv;  // most columns per wave, shifted pair and true residual
  int ncv;         // chain tile width of this launch sequence
  int ncv_spmv;    // shifted pair on the halo layout: columns per block (chunks of its list)
  int ymax;        // chain launches: chunks of ncv (half, column) pairs in the grid
  int plan_ld;     // work-list entries per step
  int narrow;      // every slice of S and S^T at most kNarrow slots wide
  int hmax;        // chain step on the halo layout: longest list of S and S^T; 0: gathers
                   // (narrow patterns: the W = 8 kernel, lists of at most kHaloCapNarrow)
  int hstride;     // halo kernels: a block's row blocks are hstride apart (1: consecutive)
  // chain steps without partial sums on the halo layout: their own, smaller
  // row blocks (more workgroups than the partial-sum budget allows the others)
  int spw_chain, nblk_chain, hstride_chain;
  const int32_t *hoff, *hcol, *hoffT, *hcolT;
  const int32_t *hrun, *hrunT;  // the lists as runs (kHaloRunInts per row block)
  const uint16_t *lidx, *lidxT;
  const int32_t *off, *col, *offT, *colT;
  const double *valA, *valAT, *e;
  double* vec;
  void* avec;    // apply vectors (element type double or float)
  int abytes;    // 8 or 4
  ColInfo* cols;
  const void* const* ftab;  // [2][cap][lcap]: factor values, forward then transposed order
  double* part_rho;    // [2][cap][nblk] (room for 3)
  double* part_delta;  // [3][cap][nblk]
  double* part_norm;   // [2][cap][nblk]
  double* trace;       // [kTraceClasses] or null
  ChainItem* plan;     // [lcap][plan_ld] work lists of the chain steps
  int32_t* plan_cnt;   // [2][lcap + 1]: chunks per list, then the forward ones
};

namespace {

__device__ __forceinline__ double* vptr(const IterArgs& a, int slot, int c) {
  return a.vec + ((int64_t)slot * a.cap + c) * a.ld;
}

template <typename AT>
__device__ __forceinline__ AT* aptr(const IterArgs& a, int slot, int c) {
  return (AT*)a.avec + ((int64_t)slot * a.cap + c) * a.ld;
}

// the FP32 copies of r and r~ (apply precision FP32 only)
__device__ __forceinline__ void store_rcopy(const IterArgs& a, int c, int64_t i, double ri,
                                            double rti) {
  if (a.abytes == 4) {
    aptr<float>(a, A_R, c)[i] = (float)ri;
    aptr<float>(a, A_RT, c)[i] = (float)rti;
  }
}

struct WaveCtx {
  int lane, wave, blk;
  int64_t s_begin, s_end;
};

__device__ __forceinline__ WaveCtx wave_ctx(const IterArgs& a) {
  WaveCtx t;
  t.wave = threadIdx.x >> 6;
  t.lane = threadIdx.x & 63;
  const int per_xcd = a.nblk >> 3;  // nblk is a multiple of 8
  t.blk = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  t.s_begin = ((int64_t)t.blk * kWavesPerBlock + t.wave) * a.spw;
  t.s_end = min(a.nslices, t.s_begin + a.spw);
  return t;
}

// ---- reductions --------------------------------------------------------------

// Sum NQ per-lane values of each of the NC columns over the block and store
// one partial per (quantity, column, block); quantity q goes to slot q * QS.
// Every thread calls it.
template <int NC, int NQ, int QS = 1>
__device__ void block_partials_cols(const IterArgs& a, const WaveCtx& t, const int (&cols)[NC],
                                    unsigned valid, double (&v)[NC][NQ], double* part) {
  __shared__ double sh[kWavesPerBlock][NC][NQ];
#pragma unroll
  for (int j = 0; j < NC; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double s = wave_sum(v[j][q]);
      if (t.lane == 0) sh[t.wave][j][q] = s;
    }
  __syncthreads();
  if (threadIdx.x < NC * NQ) {
    const int j = threadIdx.x / NQ, q = threadIdx.x % NQ;
    if (valid & (1u << j)) {
      double tot = 0.0;
#pragma unroll
      for (int w = 0; w < kWavesPerBlock; ++w) tot += sh[w][j][q];
      part[((int64_t)q * QS * a.cap + cols[j]) * a.nblk + t.blk] = tot;
    }
  }
}

// the same for the columns c0 ... c0 + NC - 1
template <int NC, int NQ, int QS = 1>
__device__ void block_partials(const IterArgs& a, const WaveCtx& t, int c0, unsigned valid,
                               double (&v)[NC][NQ], double* part) {
  int cols[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) cols[j] = c0 + j;
  block_partials_cols<NC, NQ, QS>(a, t, cols, valid, v, part);
}

// One wave sums the nblk partials of NQ quantities of column c, every load of
// the column issued before the first add (nblk <= 1024: 16 per lane and
// quantity), then a fixed-order reduction.
template <int NQ>
__device__ __forceinline__ void wave_totals(const IterArgs& a, const double* part, int c,
                                            double (&out)[NQ]) {
  const int lane = threadIdx.x & 63;
  double v[NQ][kMaxBlocks / 64];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double* p = part + ((int64_t)q * a.cap + c) * a.nblk;
#pragma unroll
    for (int k = 0; k < kMaxBlocks / 64; ++k) {
      const int b = lane + 64 * k;
      v[q][k] = b < a.nblk ? p[b] : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxBlocks / 64; ++k) s += v[q][k];
    out[q] = wave_sum(s);
  }
}

__device__ __forceinline__ bool passed(const ColInfo& ci, double rr, double rtrt) {
  return (!ci.check_p || sqrt(rr) <= ci.tol * ci.nb) && (!ci.check_d || sqrt(rtrt) <= ci.tol * ci.nc);
}

__device__ __forceinline__ bool stopped(int st) {
  return st == COL_CONVERGED || st == COL_BREAKDOWN || st == COL_MAXIT;
}

// Slots of a slice are processed kUnroll at a time: the index and value loads
// of a chunk are issued together, then every column's gathers for the chunk.
constexpr int kUnroll = 8;

struct SliceChunk {
  int32_t c[kUnroll];
  int32_t w;  // slots of the slice
};

template <typename VT>
__device__ __forceinline__ void load_chunk(const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, int32_t p0, int32_t w,
                                           int32_t m0, SliceChunk& ch, double (&v)[kUnroll]) {
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const bool ok = m0 + u < w;
    const int32_t p = p0 + (ok ? (m0 + u) * kSlice : 0);
    ch.c[u] = col[p];
    v[u] = ok ? load_val<VT>(val + p) : 0.0;
  }
}

template <typename XT>
__device__ __forceinline__ double chunk_dot(const SliceChunk& ch, const double (&v)[kUnroll],
                                            int32_t m0, int32_t w, const XT* __restrict__ x,
                                            double acc) {
  double g[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) g[u] = (double)x[ch.c[u]];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) acc = (m0 + u < w) ? fma(v[u], g[u], acc) : acc;
  return acc;
}

// the same with p = z + beta * p_old formed at every gathered index
template <typename AT>
__device__ __forceinline__ double chunk_dot_p(const SliceChunk& ch, const double (&v)[kUnroll],
                                              int32_t m0, int32_t w, const AT* __restrict__ z,
                                              const double* __restrict__ po, double beta,
                                              bool first, double acc) {
  double g[kUnroll];
  if (first) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) g[u] = (double)z[ch.c[u]];
  } else {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) g[u] = fma(beta, po[ch.c[u]], (double)z[ch.c[u]]);
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) acc = (m0 + u < w) ? fma(v[u], g[u], acc) : acc;
  return acc;
}

// One chain step s applies, for every column whose chain is long enough,
// factor s of the forward chain on the rows of S and factor maxL-1-s of the
// transposed chain on the rows of S^T; the last step also forms the partial
// sums of rho = z~^T r and ||z~||^2.  The (half, column) pairs that
// have work at a step come from the step's work list, built on the device by
// the one-block kernels before the iteration (build_plan): blockIdx.y picks a
// chunk of NC pairs of one half, so no block is launched for a column whose
// chain is shorter than the step, and columns of a chunk that apply the same
// factor share its value loads.
// AT is the apply precision: each pass sums in FP64 and stores its result
// rounded to AT; with AT = float the first pass reads the FP32 copy of r.

// Offsets of slots past a slice's width point past every array, so their
// loads return 0 without a memory access and add 0 to the row sums.
constexpr uint32_t kOutside = 0xfffffff0u;

// Slots per chunk of the product loops: every index, value and gather load of
// a chunk is issued before its first use; wide tiles take shorter chunks to
// stay within the register budget.
template <int NC>
struct ChunkLen {
  static constexpr int value = NC <= 4 ? 8 : (NC <= 8 ? 4 : 2);
};

// RHO: the iteration's last chain launch, whose transposed half also forms
// the partial sums of rho (a separate instantiation, so the other launches
// do not hold those accumulators in registers)
template <typename VT, typename AT, int NC, bool RHO>
__global__ __launch_bounds__(kBlock) void k_chain_step(IterArgs a, int s) {
  constexpr int kU = ChunkLen<NC>::value;
  const WaveCtx t = wave_ctx(a);
  const ChainItem* plan = a.plan + (int64_t)s * a.plan_ld;
  const int nchunks = gld(a.plan_cnt + s);
  const int nsl = (int)max<int64_t>(t.s_end - t.s_begin, 0);
  // slice starts of the wave's slices, lane l holding slice s_begin + wb + l
  // for both orders (a window of 64, refilled as the wave moves past it)
  const int wl = min(t.lane, nsl);
  int32_t owF = nsl > 0 ? gld(a.off + t.s_begin + wl) : 0;
  int32_t owB = nsl > 0 ? gld(a.offT + t.s_begin + wl) : 0;
  for (int y = blockIdx.y;; y += gridDim.y) {
    ChainItem it[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) it[j] = plan[y * NC + j];
    if (it[0].c < 0) break;  // past the last chunk (uniform over the block)
    const bool bwd = (it[0].flags & 1) != 0;
    const bool rho_half = RHO && bwd;
    unsigned valid = 0;
    const AT* src[NC];
    AT* dst[NC];
    const VT* fv[NC];
    bool shared = true;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const bool on = it[j].c >= 0;  // padding at the end of a half's list
      if (on) valid |= 1u << j;
      // padding runs along with the chunk's first pair (cache hits, results
      // dropped), so the slot loop has no per-column branch
      src[j] = (const AT*)(on ? it[j].src : it[0].src);
      dst[j] = (AT*)it[j].dst;
      fv[j] = (const VT*)(on ? it[j].fv : it[0].fv);
      shared = shared && fv[j] == (const VT*)it[0].fv;
    }
    const VT* fv0 = (const VT*)it[0].fv;
    const int32_t* off = bwd ? a.offT : a.off;
    const int32_t* col = bwd ? a.colT : a.col;
    int32_t ow = bwd ? owB : owF;
    int wb = 0;
    double v[RHO ? NC : 1][2];
#pragma unroll
    for (int j = 0; j < (RHO ? NC : 1); ++j) v[j][0] = v[j][1] = 0.0;
    if (nsl > 0) {
      // bounds of relative slice k; refills the window so that k and k+1 are in it
      auto bounds = [&](int k, int32_t& base, int32_t& w) {
        if (k + 1 - wb > 63) {
          wb = k;
          ow = gld(off + t.s_begin + wb + min(t.lane, nsl - wb));
        }
        base = __shfl(ow, k - wb, 64);
        w = (__shfl(ow, k + 1 - wb, 64) - base) >> 6;
      };
      // (slice, chunk) cursor over the wave's slices; the column indices of
      // the next chunk, possibly in the next slice, are loaded while the
      // current chunk's values and gathers are in flight
      int k = 0, m0 = 0;
      int32_t base, w;
      bounds(0, base, w);
      int32_t nix[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) nix[u] = gld(col + base + t.lane + (u < w ? u * kSlice : 0));
      double acc[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) acc[j] = 0.0;
      while (true) {
        const int32_t p0 = base + t.lane;
        int32_t pp[kU], cix[kU];
        bool ok[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          ok[u] = m0 + u < w;
          pp[u] = p0 + (ok[u] ? (m0 + u) * kSlice : 0);  // past the row: slot 0, value dropped
          cix[u] = nix[u];
        }
        int k2 = k, m2 = m0 + kU;
        int32_t base2 = base, w2 = w;
        if (m2 >= w) {
          k2 = k + 1;
          m2 = 0;
          if (k2 < nsl) bounds(k2, base2, w2);
        }
        if (k2 < nsl) {
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int32_t mn = m2 + u;
            nix[u] = gld(col + base2 + t.lane + (mn < w2 ? mn * kSlice : 0));
          }
        }
        if (shared) {
          double vv[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const double raw = gload_val<VT>(fv0 + pp[u]);
            vv[u] = ok[u] ? raw : 0.0;
          }
#pragma unroll
          for (int j = 0; j < NC; ++j)
#pragma unroll
            for (int u = 0; u < kU; ++u) acc[j] = fma(vv[u], (double)gld(src[j] + cix[u]), acc[j]);
        } else {
#pragma unroll
          for (int j = 0; j < NC; ++j)
#pragma unroll
            for (int u = 0; u < kU; ++u) {
              const double raw = gload_val<VT>(fv[j] + pp[u]);
              acc[j] = fma(ok[u] ? raw : 0.0, (double)gld(src[j] + cix[u]), acc[j]);
            }
        }
        if (m2 == 0) {  // slice k done
          const int64_t i = (t.s_begin + k) * kSlice + t.lane;
          if (i < a.n) {
#pragma unroll
            for (int j = 0; j < NC; ++j)
              if (valid & (1u << j)) {
                const AT zs = (AT)acc[j];
                gst(dst[j] + i, zs);
                if constexpr (RHO) {
                  if (rho_half) {
                    const double zi = (double)zs;
                    const double ri = gld(vptr(a, V_R, it[j].c) + i);
                    v[j][0] = fma(zi, ri, v[j][0]);
                    v[j][1] = fma(zi, zi, v[j][1]);
                  }
                }
              }
          }
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[j] = 0.0;
          if (k2 >= nsl) break;
        }
        k = k2;
        m0 = m2;
        base = base2;
        w = w2;
      }
    }
    if constexpr (RHO)
      if (rho_half) {
        int cols[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) cols[j] = it[j].c;
        block_partials_cols<NC, 2>(a, t, cols, valid, v, a.part_rho);
      }
    if (y + (int)gridDim.y >= nchunks) break;
  }
}

// The chain step for patterns whose slices are at most kNarrow slots wide
// (stencils with up to eight entries per row).  Per slice the column indices
// (and a chunk's shared factor values) stay in registers while the chunk's
// pairs run one after the other, two gather buffers alternating so that
// pair j+1's gathers are in flight during pair j's sums.  Registers do not
// grow with the tile width, and a wide tile reads the slice's indices and
// values once for all its pairs.  Slots past a slice's width are not loaded;
// each row sums its slots in order from zero, as the general kernel does.
// The rho partials (last step) are summed per lane over the wave's slices
// and then over the block, as in the general kernel.
constexpr int kNarrow = 8;

// A pointer every lane holds the same value of, kept in scalar registers
// (a buffer descriptor built from a vector register would need a loop over
// its distinct values)
template <typename T>
__device__ __forceinline__ T* uniform(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}

template <typename VT>
using NarrowVal = typename std::conditional<sizeof(VT) == 8, double, float>::type;

template <typename VT>
__device__ __forceinline__ NarrowVal<VT> buf_raw(BufRes r, uint32_t off);
template <>
__device__ __forceinline__ double buf_raw<double>(BufRes r, uint32_t off) {
  return buf_val<double>(r, off);
}
template <>
__device__ __forceinline__ float buf_raw<float>(BufRes r, uint32_t off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_raw<uint16_t>(BufRes r, uint32_t off) {
  return __uint_as_float(((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0)) << 16);
}

template <typename VT, typename AT, int NC, bool RHO, bool SHARED>
__device__ __forceinline__ void narrow_slice(const IterArgs& a, const WaveCtx& t,
                                             const ChainItem* ck, int ncol, BufRes rcol,
                                             int32_t base, int w, int64_t i, int64_t fbytes,
                                             int64_t vbytes, bool rho_half,
                                             double (&v)[RHO ? NC : 1][2]) {
  using FT = NarrowVal<VT>;
  constexpr uint32_t kVB = sizeof(VT), kAB = sizeof(AT);
  const uint32_t oi = (uint32_t)(base + t.lane) * 4u;
  const uint32_t ov = (uint32_t)(base + t.lane) * kVB;
  uint32_t go[kNarrow], fo[kNarrow];  // byte offsets of the gathers and of the values
#pragma unroll
  for (int u = 0; u < kNarrow; ++u) {
    const bool in = u < w;
    go[u] = (uint32_t)buf_i32(rcol, in ? oi + u * kSlice * 4 : kOutside);
    fo[u] = in ? ov + u * kSlice * kVB : kOutside;
  }
#pragma unroll
  for (int u = 0; u < kNarrow; ++u) go[u] = u < w ? go[u] * kAB : kOutside;
  FT fb[SHARED ? 1 : 2][kNarrow];
  AT gb[2][kNarrow];
  double rb[2] = {0.0, 0.0};  // r_i of the pair (rho partials, last step only)
  auto issue = [&](int j, int q) {
    const ChainItem* e = ck + j;
    if (!SHARED || j == 0) {
      const BufRes rf = buf_res(uniform(e->fv), fbytes);
#pragma unroll
      for (int u = 0; u < kNarrow; ++u) fb[SHARED ? 0 : q][u] = buf_raw<VT>(rf, fo[u]);
    }
    const BufRes rs = buf_res(uniform(e->src), vbytes);
#pragma unroll
    for (int u = 0; u < kNarrow; ++u) gb[q][u] = (AT)buf_val<AT>(rs, go[u]);
    if constexpr (RHO) {
      const double* rp = vptr(a, V_R, __builtin_amdgcn_readfirstlane(e->c));
      if (rho_half && i < a.n) rb[q] = gld(rp + i);
    }
  };
  auto finish = [&](int j, int q) {
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kNarrow; ++u)
      acc = fma((double)fb[SHARED ? 0 : q][u], (double)gb[q][u], acc);
    AT* dst = (AT*)uniform(ck[j].dst);
    const AT zs = (AT)acc;
    if (i < a.n) gst(dst + i, zs);
    if constexpr (RHO) {
      if (rho_half) {
        if (i < a.n) {
          const double zi = (double)zs, ri = rb[q];
          v[j][0] = fma(zi, ri, v[j][0]);
          v[j][1] = fma(zi, zi, v[j][1]);
        }
      }
    }
  };
  // pair j+1's loads are issued before pair j's sums (two buffers alternate)
  issue(0, 0);
  if constexpr (NC <= 8) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (j >= ncol) break;
      if (j + 1 < ncol) issue(j + 1, (j + 1) & 1);
      finish(j, j & 1);
    }
  } else {
    // wide tiles: uniform guards rather than an early exit, so that the loop
    // still unrolls completely and the buffers stay in registers
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (j < ncol) {
        if (j + 1 < ncol) issue(j + 1, (j + 1) & 1);
        finish(j, j & 1);
      }
    }
  }
}

template <typename VT, typename AT, int NC, bool RHO>
__global__ __launch_bounds__(kBlock) void k_chain_narrow(IterArgs a, int s) {
  const WaveCtx t = wave_ctx(a);
  const ChainItem* plan = a.plan + (int64_t)s * a.plan_ld;
  const int nchunks = gld(a.plan_cnt + s);
  const int nsl = (int)max<int64_t>(t.s_end - t.s_begin, 0);
  const int wl = min(t.lane, nsl);
  const int32_t owF = nsl > 0 ? gld(a.off + t.s_begin + wl) : 0;
  const int32_t owB = nsl > 0 ? gld(a.offT + t.s_begin + wl) : 0;
  for (int y = blockIdx.y;; y += gridDim.y) {
    const ChainItem* ck = plan + (int64_t)y * NC;
    const int c0 = ck->c;
    if (c0 < 0) break;  // past the last chunk (uniform over the block)
    const int flags = ck->flags;
    const bool bwd = (flags & 1) != 0;
    const bool shared = (flags & 2) != 0;  // every pair of the chunk applies one factor
    const int ncol = flags >> 8;           // pairs of the chunk
    const bool rho_half = RHO && bwd;
    double v[RHO ? NC : 1][2];  // per-lane rho partials of the chunk's pairs
#pragma unroll
    for (int j = 0; j < (RHO ? NC : 1); ++j) v[j][0] = v[j][1] = 0.0;
    const int64_t nsell = bwd ? a.nsellT : a.nsell;
    const int64_t fbytes = nsell * (int64_t)sizeof(VT), vbytes = a.ld * (int64_t)sizeof(AT);
    const BufRes rcol = buf_res(bwd ? a.colT : a.col, nsell * 4);
    const int32_t* off = bwd ? a.offT : a.off;
    int32_t ow = bwd ? owB : owF;
    int wb = 0;
    for (int k = 0; k < nsl; ++k) {
      if (k + 1 - wb > 63) {  // keep slices k and k+1 in the window
        wb = k;
        ow = gld(off + t.s_begin + wb + min(t.lane, nsl - wb));
      }
      const int32_t base = __builtin_amdgcn_readfirstlane(__shfl(ow, k - wb, 64));
      const int w = (__builtin_amdgcn_readfirstlane(__shfl(ow, k + 1 - wb, 64)) - base) >> 6;
      const int64_t i = (t.s_begin + k) * kSlice + t.lane;
      if (shared)
        narrow_slice<VT, AT, NC, RHO, true>(a, t, ck, ncol, rcol, base, w, i, fbytes, vbytes,
                                            rho_half, v);
      else
        narrow_slice<VT, AT, NC, RHO, false>(a, t, ck, ncol, rcol, base, w, i, fbytes, vbytes,
                                             rho_half, v);
    }
    if constexpr (RHO)
      if (rho_half) {
        int cols[NC];
        unsigned valid = 0;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          cols[j] = j < ncol ? ck[j].c : 0;
          if (j < ncol) valid |= 1u << j;
        }
        block_partials_cols<NC, 2>(a, t, cols, valid, v, a.part_rho);
        __syncthreads();  // the shared partials are reused by the next chunk
      }
    if (y + (int)gridDim.y >= nchunks) break;
  }
}

// The chain step on the halo layout, for patterns whose blocks of
// kHaloSlices slices touch at most kHaloCap distinct columns (a 27-point
// stencil: 1,536 for 256 rows; a 7-point one: about 900).  A block's four
// waves take one such row block at a time: the entries of CB input vectors
// at the row block's distinct columns are copied into LDS, then every row
// sums its slots from LDS through the entries' 16-bit local indices.  The
// 27 x 256 gathers of a 27-point row block read 1,536 distinct entries, so
// vector reads through the L1 path fall about 4.5-fold (7-point: about
// 2-fold) and the index stream halves.  Each row sums its slots in order
// from zero, as the gather kernels do, so the results are the same.  Two
// forms: W = 32 slots with lists of at most kHaloCap, and W = kNarrow slots
// with lists of at most kHaloCapNarrow (fewer registers, half the LDS).
template <int NC>
struct HaloGroup {
  static constexpr int value = NC < 3 ? NC : 3;  // input vectors per LDS round
};

template <typename VT>
__device__ __forceinline__ NarrowVal<VT> gload_narrow(const VT* p) {
  if constexpr (sizeof(VT) == 2) return __uint_as_float(((uint32_t)gld(p)) << 16);
  else return gld(p);
}

// Loads of a stream read once per launch (factor or matrix values, local
// indices), marked non-temporal so that they do not push the staged vectors,
// which neighbouring row blocks read again, out of the L2
template <typename T>
__device__ __forceinline__ T gld_stream(const T* p) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}
template <typename VT>
__device__ __forceinline__ NarrowVal<VT> gload_stream(const VT* p) {
  if constexpr (sizeof(VT) == 2) return __uint_as_float(((uint32_t)gld_stream(p)) << 16);
  else return gld_stream(p);
}

// What a halo launch computes.  kHaloChain: one chain step (factor s
// forward, factor maxL-1-s transposed); kHaloRho: the same, and its
// transposed half also forms the partial sums of rho = z~^T r and ||z~||^2
// (the iteration's last chain launch); kHaloSpmv: the shifted pair
// q = (sigma E - A) p on the rows of S and q~ = (sigma E - A)^T p~ on the rows
// of S^T, A's values taking the place of a factor shared by every column (p
// of parity s & 1), with the partial sums of delta = p~^T q and ||q||^2 on
// the forward half.
enum HaloMode : int { kHaloChain = 0, kHaloRho = 1, kHaloSpmv = 2 };

// W: slots a slice may have (8 or W); HC: list cap (LDS entries)
template <typename VT, typename AT, int NC, int MODE, int W, int HC>
__global__ __launch_bounds__(kBlock) void k_chain_halo(IterArgs a, int s) {
  constexpr bool RHO = MODE == kHaloRho;
  constexpr bool SPMV = MODE == kHaloSpmv;  // VT = AT = double
  constexpr bool PART = RHO || SPMV;
  constexpr int CB = HaloGroup<NC>::value;
  constexpr int kPT = HC / kBlock;  // list entries per thread
  constexpr int kSG = 4;                  // list entries per thread in flight while staging
  constexpr int kGW = 8;                  // slots per group of the row sums
  using FT = NarrowVal<VT>;
  // [CB][HC]: each vector's entries at the list positions, one vector after
  // the other, so that the rows of a slice (consecutive list positions in a
  // stencil's interior) read consecutive LDS words, and one LDS address per
  // slot serves every vector of the round through the instruction's offset
  // (c * HC entries); every position a staging round covers is written (past
  // the list: zeros), so the stores need no guard
  __shared__ AT xs[CB * HC];
  const WaveCtx t = wave_ctx(a);
  const int64_t nrb = (a.nslices + kHaloSlices - 1) / kHaloSlices;
  // the block's row blocks: rb0 + k * hstride, k < spw (hstride 1: the
  // block's own slices; hstride S: the blocks of a group of S * spw row blocks
  // take its S strided sequences, neighbours in the group side by side)
  const int64_t hs = a.hstride;
  const int64_t rb0 = hs > 1 ? ((int64_t)t.blk / hs) * hs * a.spw + t.blk % hs
                             : (int64_t)t.blk * a.spw;
  const int nrbk = hs > 1 ? (rb0 < nrb ? a.spw : 0)
                          : (int)max<int64_t>(0, min<int64_t>(a.spw, nrb - rb0));
  // the shifted pair's work list follows the chain steps' lists
  const int list = SPMV ? a.lcap : s;
  const int par = s & 1;  // (shifted pair) parity of the p vectors
  const ChainItem* plan = a.plan + (int64_t)list * a.plan_ld;
  const int nchunks = gld(a.plan_cnt + list);
  const uint32_t vbytes = (uint32_t)(a.ld * (int64_t)sizeof(AT));
  // A narrow chain step without partial sums walks every chunk of its half
  // inside each row block (grid y = the half), so that the row block's local
  // indices, list and shared factor values are loaded once for all of the
  // half's columns (the wide form keeps one chunk per grid row: walking costs
  // it registers past three waves per SIMD); the other modes take one chunk
  // per grid row.  The list holds the forward chunks first.
  constexpr bool WALK = MODE == kHaloChain && W == kNarrow;
  int nfwd = 0;
  if constexpr (WALK) nfwd = __builtin_amdgcn_readfirstlane(gld(a.plan_cnt + a.lcap + 1 + list));
  const int ngroups = WALK ? 2 : nchunks;
  for (int y = blockIdx.y;; y += gridDim.y) {
    if (y >= ngroups) break;  // uniform over the block
    const int g0 = WALK ? (y == 0 ? 0 : nfwd) : y;
    const int g1 = WALK ? (y == 0 ? nfwd : nchunks) : y + 1;
    if (g0 >= g1) {
      if (y + (int)gridDim.y >= ngroups) break;
      continue;
    }
    const ChainItem* ck = plan + (int64_t)g0 * NC;
    if (ck->c < 0) break;  // past the last chunk (uniform over the block)
    int flags = ck->flags;
    const bool bwd = (flags & 1) != 0;
    // (shared) the group's first chunk's factor, loaded once per row block
    const bool gshared = SPMV || (flags & 2) != 0;
    bool shared = gshared;
    int ncol = flags >> 8;
    const bool part_half = (RHO && bwd) || (SPMV && !bwd);
    // partial sums per pair: rho = z~^T r and ||z~||^2 (last chain step), or
    // delta = p~^T q and ||q||^2 (shifted pair; ||p~||^2 comes from form_p);
    // ||r||^2 comes from the update pass, which writes r
    constexpr int NQ = 2;
    // (shifted pair) the list was built before this iteration's convergence
    // test: columns that have stopped since are skipped
    unsigned live = (1u << ncol) - 1u;
    if constexpr (SPMV) {
      live = 0;
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (j < ncol && a.cols[ck[j].c].state == COL_ACTIVE) live |= 1u << j;
      live = __builtin_amdgcn_readfirstlane(live);
    }
    double v[PART ? NC : 1][NQ];
#pragma unroll
    for (int j = 0; j < (PART ? NC : 1); ++j)
#pragma unroll
      for (int q = 0; q < NQ; ++q) v[j][q] = 0.0;
    const int32_t* off = bwd ? a.offT : a.off;
    const int32_t* hoff = bwd ? a.hoffT : a.hoff;
    const int32_t* hcol = bwd ? a.hcolT : a.hcol;
    const int32_t* hrun = bwd ? a.hrunT : a.hrun;
    const uint16_t* lidx = bwd ? a.lidxT : a.lidx;
    const VT* fv0 = SPMV ? (const VT*)(bwd ? a.valAT : a.valA) : (const VT*)uniform(ck->fv);
    // the input and output vectors of pair j (the shifted pair's come from the slots)
    auto col_of = [&](int j) -> int { return __builtin_amdgcn_readfirstlane(ck[j].c); };
    auto src_of = [&](int j) -> const AT* {
      if constexpr (SPMV) return (const AT*)vptr(a, (bwd ? V_PT0 : V_P0) + par, col_of(j));
      else return (const AT*)uniform(ck[j].src);
    };
    auto dst_of = [&](int j) -> AT* {
      if constexpr (SPMV) return (AT*)vptr(a, bwd ? V_QT : V_Q, col_of(j));
      else return (AT*)uniform(ck[j].dst);
    };
    for (int k = 0; k < nrbk; ++k) {
      const int64_t rb = rb0 + k * hs;
      const int64_t sl = rb * kHaloSlices + t.wave;  // this wave's slice (none past the last)
      const int64_t slc = min<int64_t>(sl, a.nslices - 1);
      const int32_t base = __builtin_amdgcn_readfirstlane(gld(off + slc));
      const int w = sl < a.nslices
                        ? (__builtin_amdgcn_readfirstlane(gld(off + slc + 1)) - base) >> 6
                        : 0;
      const int ngw = __builtin_amdgcn_readfirstlane((w + kGW - 1) / kGW);  // slot groups
      const int64_t i = sl * kSlice + t.lane;
      double ei = 0.0;
      if constexpr (SPMV) ei = i < a.n ? gld(a.e + i) : 0.0;
      const int32_t h0 = __builtin_amdgcn_readfirstlane(gld(hoff + rb));
      const int H = __builtin_amdgcn_readfirstlane(gld(hoff + rb + 1)) - h0;
      // the list entries of this thread: from the block's runs (entry e of
      // run r is column s_r + e - o_r), or read from the list (which carries
      // kHaloCap >= HC entries of padding)
      int32_t hv[kPT];
      const int32_t* rp = hrun + rb * kHaloRunInts;
      const int nrun = __builtin_amdgcn_readfirstlane(gld(rp));
      if (nrun > 0) {
        int32_t rd[kHaloRuns], ro[kHaloRuns];
#pragma unroll
        for (int r = 0; r < kHaloRuns; ++r) {
          ro[r] = __builtin_amdgcn_readfirstlane(gld(rp + 2 + 2 * r));
          rd[r] = __builtin_amdgcn_readfirstlane(gld(rp + 1 + 2 * r)) - ro[r];
        }
#pragma unroll
        for (int q = 0; q < kPT; ++q) {
          const int e = (int)threadIdx.x + kBlock * q;
          int32_t c = e + rd[0];
#pragma unroll
          for (int r = 1; r < kHaloRuns; ++r)
            if (r < nrun && e >= ro[r]) c = e + rd[r];
          hv[q] = e < H ? c : 0;
        }
      } else {
        const int32_t* hp = hcol + h0 + threadIdx.x;
#pragma unroll
        for (int q = 0; q < kPT; ++q) {
          const int32_t r = gld(hp + kBlock * q);
          hv[q] = (int)threadIdx.x + kBlock * q < H ? r : 0;
        }
      }
      // local indices, kept as LDS byte offsets, and (shared factor)
      // values: all W slots read from one address (slot m at a
      // constant offset; the arrays carry padding past the last slice), and
      // slots past the width replaced by list position 0 and value 0, which
      // add nothing
      const uint16_t* lp = lidx + base + t.lane;
      uint32_t la[W];
      FT fb[W];
#pragma unroll
      for (int m = 0; m < W; ++m) {
        const uint32_t r = gld_stream(lp + m * kSlice);
        la[m] = m < w ? r * (uint32_t)sizeof(AT) : 0u;
      }
#pragma unroll
      for (int m = 0; m < W; ++m) fb[m] = (FT)0;
      if (gshared) {
        const VT* fp = fv0 + base + t.lane;
#pragma unroll
        for (int m = 0; m < W; ++m) {
          const FT r = gload_stream<VT>(fp + m * kSlice);
          fb[m] = m < w ? r : (FT)0;
        }
      }
      bool fb_ok = gshared;  // fb holds the values of fv0
      for (int yc = g0; yc < g1; ++yc) {
      if constexpr (WALK) {
        ck = plan + (int64_t)yc * NC;
        flags = ck->flags;
        ncol = flags >> 8;
        // a chunk whose pairs share fv0 reads fb; any other reads its pairs'
        // own values (which overwrite fb)
        shared = (flags & 2) != 0 && uniform(ck->fv) == (const void*)fv0;
        if (shared && !fb_ok) {
          const VT* fp = fv0 + base + t.lane;
#pragma unroll
          for (int m = 0; m < W; ++m) {
            const FT r = gload_stream<VT>(fp + m * kSlice);
            fb[m] = m < w ? r : (FT)0;
          }
          fb_ok = true;
        }
        if (!shared) fb_ok = false;
      }
#pragma unroll
      for (int j0 = 0; j0 < NC; j0 += CB) {
        if (j0 >= ncol) break;  // uniform
        if (((live >> j0) & ((1u << CB) - 1u)) == 0u) continue;  // uniform
        // the CB input vectors at the row block's distinct columns: kSG
        // entries per thread loaded, then stored, at a time
        BufRes rs[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) rs[c] = buf_res(src_of(min(j0 + c, ncol - 1)), vbytes);
#pragma unroll
        for (int q0 = 0; q0 < kPT; q0 += kSG) {
          if (q0 * kBlock >= H) break;  // uniform
          double sv[kSG][CB];
#pragma unroll
          for (int q = 0; q < kSG; ++q) {
            const int e = (int)threadIdx.x + kBlock * (q0 + q);
            const uint32_t o = e < H ? (uint32_t)hv[q0 + q] * (uint32_t)sizeof(AT) : kOutside;
#pragma unroll
            for (int c = 0; c < CB; ++c) sv[q][c] = buf_val<AT>(rs[c], o);
          }
#pragma unroll
          for (int q = 0; q < kSG; ++q) {
            const int e = (int)threadIdx.x + kBlock * (q0 + q);
#pragma unroll
            for (int c = 0; c < CB; ++c) xs[c * HC + e] = (AT)sv[q][c];
          }
        }
        // values at the row itself, in flight during the sums: (last chain
        // step) r_i of the round's pairs; (shifted pair) p_i or p~_i, and on
        // the forward half p~_i
        double rr[PART ? CB : 1], ri2[SPMV ? CB : 1];
        if constexpr (PART) {
#pragma unroll
          for (int c = 0; c < CB; ++c) {
            rr[c] = 0.0;
            if constexpr (SPMV) ri2[c] = 0.0;
            if (j0 + c < ncol && i < a.n) {
              const int cc = col_of(j0 + c);
              if constexpr (RHO) {
                if (part_half) rr[c] = gld(vptr(a, V_R, cc) + i);
              } else {
                rr[c] = gld((const double*)src_of(j0 + c) + i);
                if (!bwd) ri2[c] = gld(vptr(a, V_PT0 + par, cc) + i);
              }
            }
          }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          const int j = j0 + c;
          if (j < NC && j < ncol && ((live >> j) & 1u)) {
            const char* xc = (const char*)(xs + c * HC);
            if (!shared) {  // this pair's own factor values
              const VT* fp = (const VT*)uniform(ck[j].fv) + base + t.lane;
#pragma unroll
              for (int m = 0; m < W; ++m) {
                const FT r = gload_stream<VT>(fp + m * kSlice);
                fb[m] = m < w ? r : (FT)0;
              }
            }
            // slots in groups of kGW, all LDS reads of a group issued
            // together; slots past the width multiply 0 with the row
            // block's first staged entry
            double acc = 0.0;
#pragma unroll
            for (int g = 0; g < W / kGW; ++g) {
              if (g >= ngw) break;  // uniform
              AT xg[kGW];
#pragma unroll
              for (int u = 0; u < kGW; ++u) xg[u] = *(const AT*)(xc + la[g * kGW + u]);
#pragma unroll
              for (int u = 0; u < kGW; ++u) acc = fma((double)fb[g * kGW + u], (double)xg[u], acc);
            }
            if (i < a.n) {  // rows past n, and waves past the last slice
              AT* dst = dst_of(j);
              if constexpr (SPMV) {
                const double se = a.cols[col_of(j)].sigma * ei;
                const double qi = fma(se, rr[c], -acc);
                gst(dst + i, (AT)qi);
                if (part_half) {
                  v[j][0] = fma(ri2[c], qi, v[j][0]);
                  v[j][NQ - 1] = fma(qi, qi, v[j][NQ - 1]);
                }
              } else {
                const AT zs = (AT)acc;
                gst(dst + i, zs);
                if constexpr (RHO) {
                  if (part_half) {
                    const double zi = (double)zs;
                    const double ri = rr[c];
                    v[j][0] = fma(zi, ri, v[j][0]);
                    v[j][1] = fma(zi, zi, v[j][1]);
                  }
                }
              }
            }
          }
        }
        __syncthreads();  // before the next round overwrites the LDS copies
      }
      }  // chunks of the group
    }
    if constexpr (PART)
      if (part_half) {
        int cols[NC];
        unsigned valid = 0;
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          cols[j] = j < ncol ? ck[j].c : 0;
          if (j < ncol && ((live >> j) & 1u)) valid |= 1u << j;
        }
        if constexpr (SPMV) block_partials_cols<NC, NQ, 2>(a, t, cols, valid, v, a.part_delta);
        else block_partials_cols<NC, NQ>(a, t, cols, valid, v, a.part_rho);
        __syncthreads();  // the shared partials are reused by the next chunk
      }
    if (y + (int)gridDim.y >= ngroups) break;
  }
}

#define MORX_NC_DISPATCH(NCV, ...)                         \
  switch (NCV) {                                           \
    case 1: { constexpr int NC = 1; __VA_ARGS__; } break;  \
    case 2: { constexpr int NC = 2; __VA_ARGS__; } break;  \
    case 3: { constexpr int NC = 3; __VA_ARGS__; } break;  \
    case 4: { constexpr int NC = 4; __VA_ARGS__; } break;  \
    case 5: { constexpr int NC = 5; __VA_ARGS__; } break;  \
    case 6: { constexpr int NC = 6; __VA_ARGS__; } break;  \
    case 7: { constexpr int NC = 7; __VA_ARGS__; } break;  \
    case 8: { constexpr int NC = 8; __VA_ARGS__; } break;  \
    case 10: { constexpr int NC = 10; __VA_ARGS__; } break; \
    case 12: { constexpr int NC = 12; __VA_ARGS__; } break; \
    default: { constexpr int NC = 16; __VA_ARGS__; } break; \
  }

// the maxL chain launches of one iteration, factors stored as VT
template <typename VT, typename AT, int NC>
void chain_run(const IterArgs& a, hipStream_t st) {
  const dim3 g((unsigned)a.nblk, (unsigned)a.ymax, 1);
  // the steps before the last (no partial sums) on their own row blocks
  IterArgs c = a;
  c.spw = a.spw_chain;
  c.nblk = a.nblk_chain;
  c.hstride = a.hstride_chain;
  const dim3 gc((unsigned)c.nblk, (unsigned)a.ymax, 1);
  const dim3 gw((unsigned)c.nblk, 2u, 1);  // the narrow halo chain steps walk their half's chunks
  if (a.hmax > 0 && a.narrow) {
    for (int s = 0; s + 1 < a.maxL; ++s)
      k_chain_halo<VT, AT, NC, kHaloChain, kNarrow, kHaloCapNarrow><<<gw, kBlock, 0, st>>>(c, s);
    k_chain_halo<VT, AT, NC, kHaloRho, kNarrow, kHaloCapNarrow><<<g, kBlock, 0, st>>>(a, a.maxL - 1);
  } else if (a.hmax > 0) {
    for (int s = 0; s + 1 < a.maxL; ++s)
      k_chain_halo<VT, AT, NC, kHaloChain, kHaloMaxW, kHaloCap><<<gc, kBlock, 0, st>>>(c, s);
    k_chain_halo<VT, AT, NC, kHaloRho, kHaloMaxW, kHaloCap><<<g, kBlock, 0, st>>>(a, a.maxL - 1);
  } else if (a.narrow) {
    for (int s = 0; s + 1 < a.maxL; ++s) k_chain_narrow<VT, AT, NC, false><<<g, kBlock, 0, st>>>(a, s);
    k_chain_narrow<VT, AT, NC, true><<<g, kBlock, 0, st>>>(a, a.maxL - 1);
  } else {
    for (int s = 0; s + 1 < a.maxL; ++s) k_chain_step<VT, AT, NC, false><<<g, kBlock, 0, st>>>(a, s);
    k_chain_step<VT, AT, NC, true><<<g, kBlock, 0, st>>>(a, a.maxL - 1);
  }
}

template <typename VT>
void chain_launch_vt(const IterArgs& a, hipStream_t st) {
  MORX_NC_DISPATCH(a.ncv, {
    if (a.abytes == 4) chain_run<VT, float, NC>(a, st);
    else chain_run<VT, double, NC>(a, st);
  });
}

}  // namespace

// The shifted pair on the halo layout (kHaloSpmv), p of parity par, columns
// in chunks of a.ncv_spmv; the grid's y extent covers both halves of every
// column
template <int NC>
void spmv_halo_run(const IterArgs& a, int par, hipStream_t st) {
  const dim3 g((unsigned)a.nblk, (unsigned)(2 * ((a.nc + NC - 1) / NC)), 1);
  if (a.narrow)
    k_chain_halo<double, double, NC, kHaloSpmv, kNarrow, kHaloCapNarrow><<<g, kBlock, 0, st>>>(a, par);
  else
    k_chain_halo<double, double, NC, kHaloSpmv, kHaloMaxW, kHaloCap><<<g, kBlock, 0, st>>>(a, par);
}

// one per file: the chain launches of an iteration for factors stored in
// FP64, FP32 or BF16 (the apply precision comes from the arguments)
void chain_launch_f64(const IterArgs& a, hipStream_t st);
// (in the FP64 file) the shifted pair on the halo layout, tile a.ncv
void spmv_halo_launch(const IterArgs& a, int par, hipStream_t st);
void chain_launch_f32(const IterArgs& a, hipStream_t st);
void chain_launch_bf16(const IterArgs& a, hipStream_t st);
