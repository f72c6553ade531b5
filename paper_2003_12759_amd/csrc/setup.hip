// System set-up: copy A and E, form the factor pattern S = pattern(A) + diag,
// its transpose, and the sliced-ELL (height 64) layouts used by every
// product kernel.  All of it is integer and copy work done once per system.
//
// The SPAI column problems (Section III-A, eq. gen-precond-par) and the reuse
// updates (Section III-C) all read column k of S and the columns of S listed
// there, so the transpose of S is kept in CSR form as well.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>

#include "common.h"

namespace {

constexpr int kBlock = 256;

// ---- prefix sums (int64, exclusive) ---------------------------------------

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void k_scan_tile(const int64_t* __restrict__ in,
                                                      int64_t* __restrict__ out,
                                                      int64_t* __restrict__ tile_sums,
                                                      int64_t count) {
  __shared__ int64_t sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t run = 0;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    int64_t i = base + t;
    v[t] = (i < count) ? in[i] : 0;
    run += v[t];
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int off = 1; off < kBlock; off <<= 1) {
    int64_t add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t prefix = sh[threadIdx.x] - run;
#pragma unroll
  for (int t = 0; t < kScanItems; ++t) {
    int64_t i = base + t;
    if (i < count) out[i] = prefix;
    prefix += v[t];
  }
  if (threadIdx.x == kBlock - 1) tile_sums[blockIdx.x] = sh[kBlock - 1];
}

__global__ void k_scan_add(int64_t* __restrict__ out, const int64_t* __restrict__ tile_off,
                           int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] += tile_off[i / kScanTile];
}

// exclusive scan of `count` values; total returned through `total_dev` (out[count])
morx_status scan_exclusive(const int64_t* in, int64_t* out, int64_t count, hipStream_t st,
                           std::vector<DevBuf>& tmp) {
  if (count <= 0) return MORX_OK;
  int64_t tiles = (count + kScanTile - 1) / kScanTile;
  DevBuf sums, offs;
  MORX_TRY(dev_alloc(sums, (tiles + 1) * sizeof(int64_t)));
  MORX_TRY(dev_alloc(offs, (tiles + 1) * sizeof(int64_t)));
  tmp.push_back(sums);
  tmp.push_back(offs);
  k_scan_tile<<<dim3((unsigned)tiles), dim3(kBlock), 0, st>>>(in, out, (int64_t*)sums.p, count);
  MORX_HIP(hipGetLastError());
  if (tiles > 1) {
    MORX_TRY(scan_exclusive((int64_t*)sums.p, (int64_t*)offs.p, tiles, st, tmp));
    k_scan_add<<<dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, st>>>(
        out, (int64_t*)offs.p, count);
    MORX_HIP(hipGetLastError());
  }
  return MORX_OK;
}

// ---- validation and pattern S ----------------------------------------------

enum : int { ERR_INVALID = 1, ERR_NONFINITE = 2 };

__global__ void k_check_rows(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             const double* __restrict__ val, const double* __restrict__ e,
                             int64_t n, int64_t nnz, int64_t* __restrict__ lenS,
                             int* __restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t lo = rowptr[i], hi = rowptr[i + 1];
  int bad = 0;
  if (lo < 0 || hi < lo || hi > nnz) bad |= ERR_INVALID;
  if (i == 0 && lo != 0) bad |= ERR_INVALID;
  if (i == n - 1 && hi != nnz) bad |= ERR_INVALID;
  bool has_diag = false;
  if (!(bad & ERR_INVALID)) {
    int64_t prev = -1;
    for (int64_t p = lo; p < hi; ++p) {
      int64_t c = col[p];
      if (c < 0 || c >= n || c <= prev) bad |= ERR_INVALID;
      if (c == i) has_diag = true;
      if (!isfinite(val[p])) bad |= ERR_NONFINITE;
      prev = c;
    }
  }
  if (!isfinite(e[i])) bad |= ERR_NONFINITE;
  lenS[i] = (bad & ERR_INVALID) ? 0 : (hi - lo) + (has_diag ? 0 : 1);
  if (bad) atomicOr(err, bad);
}

__global__ void k_fill_S(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                         const double* __restrict__ val, const int64_t* __restrict__ offS,
                         int64_t n, int32_t* __restrict__ rowptrS, int32_t* __restrict__ colS,
                         double* __restrict__ valS) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  rowptrS[i] = (int32_t)offS[i];
  if (i == n) return;
  int64_t q = offS[i];
  bool placed = false;
  for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    int32_t c = col[p];
    if (!placed && c > i) {
      colS[q] = (int32_t)i;
      valS[q] = 0.0;
      ++q;
      placed = true;
    }
    if (c == i) placed = true;
    colS[q] = c;
    valS[q] = val[p];
    ++q;
  }
  if (!placed) {
    colS[q] = (int32_t)i;
    valS[q] = 0.0;
  }
}

// ---- transpose of S ----------------------------------------------------------

__global__ void k_count_cols(const int32_t* __restrict__ colS, int64_t nnzS,
                             int32_t* __restrict__ cnt) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnzS) atomicAdd(&cnt[colS[p]], 1);
}

__global__ void k_widen(const int32_t* __restrict__ in, int64_t* __restrict__ out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

__global__ void k_scatter_T(const int32_t* __restrict__ rowptrS, const int32_t* __restrict__ colS,
                            int64_t n, const int64_t* __restrict__ toff,
                            int32_t* __restrict__ cursor, int32_t* __restrict__ tcol,
                            int32_t* __restrict__ tsrc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t p = rowptrS[i]; p < rowptrS[i + 1]; ++p) {
    int32_t c = colS[p];
    int32_t slot = atomicAdd(&cursor[c], 1);
    int64_t q = toff[c] + slot;
    tcol[q] = (int32_t)i;
    tsrc[q] = p;
  }
}

// rows of S^T are filled in arbitrary order by the scatter; sort each by
// column so the layout (and every result) is deterministic
__global__ void k_sort_T_rows(const int64_t* __restrict__ toff, int64_t n,
                              int32_t* __restrict__ tcol, int32_t* __restrict__ tsrc,
                              int32_t* __restrict__ trowptr, const double* __restrict__ valS,
                              double* __restrict__ tval) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > n) return;
  trowptr[k] = (int32_t)toff[k];
  if (k == n) return;
  int64_t lo = toff[k], hi = toff[k + 1];
  for (int64_t a = lo + 1; a < hi; ++a) {
    int32_t c = tcol[a], s = tsrc[a];
    int64_t b = a - 1;
    while (b >= lo && tcol[b] > c) {
      tcol[b + 1] = tcol[b];
      tsrc[b + 1] = tsrc[b];
      --b;
    }
    tcol[b + 1] = c;
    tsrc[b + 1] = s;
  }
  for (int64_t a = lo; a < hi; ++a) tval[a] = valS[tsrc[a]];
}

__global__ void k_compare(const int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t n,
                          int* __restrict__ diff) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && a[i] != b[i]) atomicOr(diff, 1);
}

// ---- sliced ELL ------------------------------------------------------------------

__global__ void k_slice_width(const int32_t* __restrict__ rowptr, int64_t n, int64_t nslice,
                              int64_t* __restrict__ w64) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslice) return;
  int32_t w = 0;
  for (int64_t r = s * kSlice; r < (s + 1) * kSlice && r < n; ++r)
    w = max(w, rowptr[r + 1] - rowptr[r]);
  w64[s] = (int64_t)w * kSlice;
}

__global__ void k_narrow_off(const int64_t* __restrict__ in, int32_t* __restrict__ out,
                             int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (int32_t)in[i];
}

// fill the ELL arrays; padding uses an in-range column (the row itself, or 0
// for rows past n) with a zero value so gathers never leave [0, n)
__global__ void k_fill_sell(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, int64_t n, int64_t n_pad,
                            const int32_t* __restrict__ off, int32_t* __restrict__ scol,
                            double* __restrict__ sval, int32_t* __restrict__ csr2sell) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  int64_t s = i / kSlice, lane = i % kSlice;
  int32_t w = (off[s + 1] - off[s]) / kSlice;
  int32_t len = (i < n) ? rowptr[i + 1] - rowptr[i] : 0;
  int32_t lo = (i < n) ? rowptr[i] : 0;
  for (int32_t m = 0; m < w; ++m) {
    int64_t pos = (int64_t)off[s] + (int64_t)m * kSlice + lane;
    if (m < len) {
      scol[pos] = col[lo + m];
      if (sval) sval[pos] = val[lo + m];
      if (csr2sell) csr2sell[lo + m] = (int32_t)pos;
    } else {
      scol[pos] = (i < n) ? (int32_t)i : 0;
      if (sval) sval[pos] = 0.0;
    }
  }
}

__global__ void k_compose(const int32_t* __restrict__ tsrc, const int32_t* __restrict__ csr2sell,
                          int64_t nnz, int32_t* __restrict__ tp2s) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) tp2s[p] = csr2sell[tsrc[p]];
}

__global__ void k_copy_pad(const double* __restrict__ in, double* __restrict__ out, int64_t n,
                           int64_t n_pad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_pad) out[i] = (i < n) ? in[i] : 0.0;
}

inline unsigned nblk(int64_t count) { return (unsigned)((count + kBlock - 1) / kBlock); }

// ---- halo layout -------------------------------------------------------------------

constexpr int kHaloEnt = kHaloSlices * kSlice * kHaloMaxW;  // entries of a block, at most
constexpr int kHaloThreads = 256;

// One workgroup per block of kHaloSlices slices: sort the block's column
// indices (bitonic, in LDS), keep the distinct ones, and give every entry the
// position of its column in that ascending list.  cnt[b] receives the list's
// length; the list goes to tmp[b * kHaloCap ...] when it fits the cap.
__global__ __launch_bounds__(kHaloThreads) void k_halo_block(const int32_t* __restrict__ off,
                                                             const int32_t* __restrict__ col,
                                                             int64_t nslice,
                                                             int32_t* __restrict__ cnt,
                                                             int32_t* __restrict__ tmp,
                                                             uint16_t* __restrict__ lidx) {
  __shared__ int32_t keys[kHaloEnt];
  __shared__ int32_t uniq[kHaloCap];
  __shared__ int32_t part[kHaloThreads + 1];
  const int64_t b = blockIdx.x;
  const int64_t s0 = b * kHaloSlices, s1 = min(nslice, s0 + kHaloSlices);
  const int32_t e0 = off[s0];
  const int E = off[s1] - e0;  // <= kHaloEnt: slices are at most kHaloMaxW wide
  int P = 1;
  while (P < E) P <<= 1;
  for (int q = threadIdx.x; q < P; q += kHaloThreads) keys[q] = q < E ? col[e0 + q] : 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = threadIdx.x; q < P / 2; q += kHaloThreads) {
        const int i = 2 * q - (q & (j - 1)), l = i + j;  // i has bit j clear
        const bool up = (i & k) == 0;
        const int32_t x = keys[i], y = keys[l];
        if ((x > y) == up) {
          keys[i] = y;
          keys[l] = x;
        }
      }
      __syncthreads();
    }
  // first occurrences, counted per thread over a contiguous range, then placed
  const int per = (P + kHaloThreads - 1) / kHaloThreads;
  const int q0 = min(P, (int)threadIdx.x * per), q1 = min(P, q0 + per);
  auto first = [&](int q) { return keys[q] != 0x7fffffff && (q == 0 || keys[q] != keys[q - 1]); };
  int c = 0;
  for (int q = q0; q < q1; ++q) c += first(q);
  part[threadIdx.x + 1] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    part[0] = 0;
    for (int t = 1; t <= kHaloThreads; ++t) part[t] += part[t - 1];
  }
  __syncthreads();
  const int H = part[kHaloThreads];
  if (threadIdx.x == 0) cnt[b] = H;
  if (H > kHaloCap) return;  // uniform: the layout is not built
  int pos = part[threadIdx.x];
  for (int q = q0; q < q1; ++q)
    if (first(q)) {
      uniq[pos] = keys[q];
      tmp[b * kHaloCap + pos] = keys[q];
      ++pos;
    }
  __syncthreads();
  for (int q = threadIdx.x; q < E; q += kHaloThreads) {
    const int32_t cq = col[e0 + q];
    int lo = 0, hi = H - 1;  // cq is in uniq[0, H)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (uniq[mid] < cq) lo = mid + 1;
      else hi = mid;
    }
    lidx[e0 + q] = (uint16_t)lo;
  }
}

__global__ __launch_bounds__(kHaloThreads) void k_halo_pack(const int32_t* __restrict__ hoff,
                                                            const int32_t* __restrict__ tmp,
                                                            int32_t* __restrict__ hcol) {
  const int64_t b = blockIdx.x;
  const int32_t h0 = hoff[b], H = hoff[b + 1] - h0;
  for (int q = threadIdx.x; q < H; q += kHaloThreads) hcol[h0 + q] = tmp[b * kHaloCap + q];
}

// Each block's list as runs of consecutive columns (one wave per block): a
// run starts where a column is not its predecessor plus one; more than
// kHaloRuns runs leave the count 0 and the list is read as it is
__global__ __launch_bounds__(64) void k_halo_runs(const int32_t* __restrict__ lists,
                                                  const int32_t* __restrict__ cnt,
                                                  int32_t* __restrict__ hrun) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x;
  const int H = cnt[b];
  const int32_t* L = lists + b * kHaloCap;
  int32_t* out = hrun + b * kHaloRunInts;
  const unsigned long long below = (1ull << lane) - 1ull;
  int nr = 0;
  for (int q0 = 0; q0 < H; q0 += 64) {
    const int q = q0 + lane;
    const bool brk = q < H && (q == 0 || L[q] != L[q - 1] + 1);
    const unsigned long long m = __ballot(brk);
    if (brk) {
      const int r = nr + __popcll(m & below);
      if (r < kHaloRuns) {
        out[1 + 2 * r] = L[q];
        out[2 + 2 * r] = q;
      }
    }
    nr += __popcll(m);
  }
  if (lane == 0) out[0] = nr <= kHaloRuns ? nr : 0;
}

template <typename T>
morx_status owned_alloc(morx_system sys, T** p, int64_t count) {
  DevBuf b;
  MORX_TRY(dev_alloc(b, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
  sys->owned.push_back(b);
  sys->resident_bytes += (int64_t)b.bytes;
  *p = (T*)b.p;
  return MORX_OK;
}

morx_status build_sell(morx_system sys, const int32_t* rowptr, const int32_t* col,
                       const double* val, Sell& out, double** sval, int32_t* csr2sell,
                       hipStream_t st, std::vector<DevBuf>& tmp) {
  const int64_t n = sys->n, ns = sys->nslice;
  DevBuf w64, off64;
  MORX_TRY(dev_alloc(w64, (ns + 1) * sizeof(int64_t)));
  MORX_TRY(dev_alloc(off64, (ns + 1) * sizeof(int64_t)));
  tmp.push_back(w64);
  tmp.push_back(off64);
  MORX_HIP(hipMemsetAsync(w64.p, 0, (ns + 1) * sizeof(int64_t), st));
  k_slice_width<<<nblk(ns), kBlock, 0, st>>>(rowptr, n, ns, (int64_t*)w64.p);
  MORX_HIP(hipGetLastError());
  std::vector<int64_t> hw((size_t)ns);
  MORX_HIP(hipMemcpyAsync(hw.data(), w64.p, (size_t)ns * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MORX_TRY(scan_exclusive((int64_t*)w64.p, (int64_t*)off64.p, ns + 1, st, tmp));
  int64_t total = 0;
  MORX_HIP(hipMemcpyAsync(&total, (int64_t*)off64.p + ns, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipStreamSynchronize(st));
  int64_t wmax = 0;
  for (int64_t w : hw) wmax = std::max(wmax, w / kSlice);
  out.max_width = (int32_t)wmax;
  // the iteration kernels address these arrays (and n-vectors, n <= total)
  // with 32-bit byte offsets of 8-byte elements
  MORX_REQUIRE(total < ((int64_t)1 << 29) - 4096, MORX_E_UNSUPPORTED,
               "sliced-ELL size %lld exceeds 2^29 entries", (long long)total);
  out.nnz_sell = total;
  MORX_TRY(owned_alloc(sys, &out.off, ns + 1));
  MORX_TRY(owned_alloc(sys, &out.col, total));
  MORX_TRY(owned_alloc(sys, sval, total + kSellPad));  // halo kernels read past the end
  k_narrow_off<<<nblk(ns + 1), kBlock, 0, st>>>((int64_t*)off64.p, out.off, ns + 1);
  k_fill_sell<<<nblk(sys->n_pad), kBlock, 0, st>>>(rowptr, col, val, n, sys->n_pad, out.off,
                                                   out.col, *sval, csr2sell);
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

// The row-block distance d (1..kHaloStrideMax) whose lists share the most
// columns with row block r's, over a few sample blocks in the middle of the
// pattern: consecutive row blocks of a grid row share part of their lists,
// but for a lexicographically ordered 3-D stencil the block one plane further
// shares more (the halo kernels then walk row blocks a plane apart, and the
// shared entries are still in the cache when the next row block stages them).
constexpr int kHaloStrideMax = 512;
morx_status halo_stride(Sell& sl, int64_t nrb, const int32_t* lists, const std::vector<int32_t>& hc,
                        hipStream_t st) {
  sl.hstride = 1;
  if (nrb < 4 * 8) return MORX_OK;
  const int64_t dmax = std::min<int64_t>(kHaloStrideMax, nrb / 4);
  std::vector<int64_t> score(dmax + 1, 0);
  std::vector<int32_t> buf((size_t)(dmax + 1) * kHaloCap);
  for (const int64_t r0 : {nrb / 2 - dmax / 2, nrb / 3, (2 * nrb) / 3 - dmax}) {
    if (r0 < 0 || r0 + dmax >= nrb) continue;
    MORX_HIP(hipMemcpyAsync(buf.data(), lists + r0 * kHaloCap, buf.size() * sizeof(int32_t),
                            hipMemcpyDeviceToHost, st));
    MORX_HIP(hipStreamSynchronize(st));
    const int32_t* a = buf.data();
    const int na = hc[r0];
    for (int64_t d = 1; d <= dmax; ++d) {
      const int32_t* b = buf.data() + d * kHaloCap;
      const int nb = hc[r0 + d];
      int i = 0, j = 0, common = 0;  // both lists ascending
      while (i < na && j < nb) {
        if (a[i] == b[j]) {
          ++common;
          ++i;
          ++j;
        } else if (a[i] < b[j]) {
          ++i;
        } else {
          ++j;
        }
      }
      score[d] += common;
    }
  }
  int64_t best = 1;
  for (int64_t d = 2; d <= dmax; ++d)
    if (score[d] > score[best]) best = d;
  sl.hstride = (int32_t)best;
  return MORX_OK;
}

// Halo layout of a pattern whose slices are at most kHaloMaxW slots wide; a
// pattern with a block of more than kHaloCap distinct columns keeps none
// (hmax = 0) and the chain step gathers from the vectors instead.
morx_status build_halo(morx_system sys, Sell& sl, hipStream_t st, std::vector<DevBuf>& tmp) {
  sl.hmax = 0;
  if (sl.max_width > kHaloMaxW) return MORX_OK;
  const int64_t nrb = (sys->nslice + kHaloSlices - 1) / kHaloSlices;
  DevBuf cnt, lists, lidx;
  MORX_TRY(dev_alloc(cnt, nrb * sizeof(int32_t)));
  MORX_TRY(dev_alloc(lists, nrb * kHaloCap * sizeof(int32_t)));
  tmp.push_back(cnt);
  tmp.push_back(lists);
  MORX_TRY(dev_alloc(lidx, (sl.nnz_sell + kSellPad) * sizeof(uint16_t)));
  MORX_HIP(hipMemsetAsync(lidx.p, 0, (sl.nnz_sell + kSellPad) * sizeof(uint16_t), st));
  k_halo_block<<<(unsigned)nrb, kHaloThreads, 0, st>>>(sl.off, sl.col, sys->nslice,
                                                       (int32_t*)cnt.p, (int32_t*)lists.p,
                                                       (uint16_t*)lidx.p);
  MORX_HIP(hipGetLastError());
  std::vector<int32_t> hc((size_t)nrb);
  MORX_HIP(hipMemcpyAsync(hc.data(), cnt.p, nrb * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipStreamSynchronize(st));
  int32_t hmax = 0;
  std::vector<int32_t> hoff((size_t)nrb + 1, 0);
  for (int64_t b = 0; b < nrb; ++b) {
    hmax = std::max(hmax, hc[b]);
    hoff[b + 1] = hoff[b] + hc[b];
  }
  if (hmax > kHaloCap) {
    tmp.push_back(lidx);
    return MORX_OK;
  }
  sys->owned.push_back(lidx);
  sys->resident_bytes += (int64_t)lidx.bytes;
  sl.lidx = (uint16_t*)lidx.p;
  MORX_TRY(owned_alloc(sys, &sl.hoff, nrb + 1));
  // list reads run up to kHaloCap entries past a block's start
  MORX_TRY(owned_alloc(sys, &sl.hcol, hoff[nrb] + kHaloCap));
  MORX_HIP(hipMemcpyAsync(sl.hoff, hoff.data(), (nrb + 1) * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
  k_halo_pack<<<(unsigned)nrb, kHaloThreads, 0, st>>>(sl.hoff, (int32_t*)lists.p, sl.hcol);
  MORX_HIP(hipGetLastError());
  MORX_TRY(owned_alloc(sys, &sl.hrun, nrb * kHaloRunInts));
  MORX_HIP(hipMemsetAsync(sl.hrun, 0, (size_t)nrb * kHaloRunInts * sizeof(int32_t), st));
  k_halo_runs<<<(unsigned)nrb, 64, 0, st>>>((const int32_t*)lists.p, (const int32_t*)cnt.p,
                                            sl.hrun);
  MORX_HIP(hipGetLastError());
  MORX_TRY(halo_stride(sl, nrb, (const int32_t*)lists.p, hc, st));
  MORX_HIP(hipStreamSynchronize(st));  // hoff's host copy goes out of scope
  sl.hmax = hmax;
  return MORX_OK;
}

}  // namespace

// ---------------------------------------------------------------------------

morx_status ls_pattern_stats(morx_system sys, hipStream_t st);  // factor.hip

static morx_status system_build(morx_system sys, const int32_t* rowptr, const int32_t* colind,
                                const double* val, const double* e_diag, hipStream_t st,
                                std::vector<DevBuf>& tmp) {
  const int64_t n = sys->n, nnz = sys->nnz_in;
  DevBuf lenS, offS, errb;
  MORX_TRY(dev_alloc(lenS, (n + 1) * sizeof(int64_t)));
  MORX_TRY(dev_alloc(offS, (n + 1) * sizeof(int64_t)));
  MORX_TRY(dev_alloc(errb, sizeof(int)));
  tmp.push_back(lenS);
  tmp.push_back(offS);
  tmp.push_back(errb);
  MORX_HIP(hipMemsetAsync(errb.p, 0, sizeof(int), st));
  MORX_HIP(hipMemsetAsync(lenS.p, 0, (n + 1) * sizeof(int64_t), st));
  k_check_rows<<<nblk(n), kBlock, 0, st>>>(rowptr, colind, val, e_diag, n, nnz,
                                           (int64_t*)lenS.p, (int*)errb.p);
  MORX_HIP(hipGetLastError());
  int err = 0;
  MORX_HIP(hipMemcpyAsync(&err, errb.p, sizeof(int), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipStreamSynchronize(st));
  MORX_REQUIRE(!(err & ERR_INVALID), MORX_E_INVALID,
               "CSR of A is malformed (rowptr not monotone from 0 to nnz, or column indices "
               "out of range / not strictly increasing within a row)");
  MORX_REQUIRE(!(err & ERR_NONFINITE), MORX_E_NONFINITE, "A or E holds NaN or Inf");

  MORX_TRY(scan_exclusive((int64_t*)lenS.p, (int64_t*)offS.p, n + 1, st, tmp));
  int64_t nnzS = 0;
  MORX_HIP(hipMemcpyAsync(&nnzS, (int64_t*)offS.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipStreamSynchronize(st));
  MORX_REQUIRE(nnzS < (int64_t)INT32_MAX, MORX_E_UNSUPPORTED, "nnz(S) >= 2^31");
  sys->nnzS = nnzS;

  MORX_TRY(owned_alloc(sys, &sys->rowptr, n + 1));
  MORX_TRY(owned_alloc(sys, &sys->colind, nnzS));
  MORX_TRY(owned_alloc(sys, &sys->valA, nnzS));
  k_fill_S<<<nblk(n + 1), kBlock, 0, st>>>(rowptr, colind, val, (int64_t*)offS.p, n, sys->rowptr,
                                           sys->colind, sys->valA);
  MORX_HIP(hipGetLastError());

  // transpose
  DevBuf cnt, cnt64, toff, tsrc;
  MORX_TRY(dev_alloc(cnt, (n + 1) * sizeof(int32_t)));
  MORX_TRY(dev_alloc(cnt64, (n + 1) * sizeof(int64_t)));
  MORX_TRY(dev_alloc(toff, (n + 1) * sizeof(int64_t)));
  tmp.push_back(cnt);
  tmp.push_back(cnt64);
  tmp.push_back(toff);
  MORX_HIP(hipMemsetAsync(cnt.p, 0, (n + 1) * sizeof(int32_t), st));
  k_count_cols<<<nblk(nnzS), kBlock, 0, st>>>(sys->colind, nnzS, (int32_t*)cnt.p);
  k_widen<<<nblk(n + 1), kBlock, 0, st>>>((int32_t*)cnt.p, (int64_t*)cnt64.p, n + 1);
  MORX_HIP(hipGetLastError());
  MORX_TRY(scan_exclusive((int64_t*)cnt64.p, (int64_t*)toff.p, n + 1, st, tmp));
  MORX_TRY(owned_alloc(sys, &sys->trowptr, n + 1));
  MORX_TRY(owned_alloc(sys, &sys->tcol, nnzS));
  MORX_TRY(owned_alloc(sys, &sys->tval, nnzS));
  int32_t* tsrcp = nullptr;
  MORX_TRY(dev_alloc(tsrc, nnzS * sizeof(int32_t)));
  tmp.push_back(tsrc);
  tsrcp = (int32_t*)tsrc.p;
  MORX_HIP(hipMemsetAsync(cnt.p, 0, (n + 1) * sizeof(int32_t), st));
  k_scatter_T<<<nblk(n), kBlock, 0, st>>>(sys->rowptr, sys->colind, n, (int64_t*)toff.p,
                                          (int32_t*)cnt.p, sys->tcol, tsrcp);
  k_sort_T_rows<<<nblk(n + 1), kBlock, 0, st>>>((int64_t*)toff.p, n, sys->tcol, tsrcp,
                                                sys->trowptr, sys->valA, sys->tval);
  MORX_HIP(hipGetLastError());

  // structural symmetry: S^T has exactly the rows of S
  MORX_HIP(hipMemsetAsync(errb.p, 0, sizeof(int), st));
  k_compare<<<nblk(n + 1), kBlock, 0, st>>>(sys->rowptr, sys->trowptr, n + 1, (int*)errb.p);
  k_compare<<<nblk(nnzS), kBlock, 0, st>>>(sys->colind, sys->tcol, nnzS, (int*)errb.p);
  MORX_HIP(hipGetLastError());
  int diff = 0;
  MORX_HIP(hipMemcpyAsync(&diff, errb.p, sizeof(int), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipStreamSynchronize(st));
  sys->symmetric_pattern = (diff == 0);

  // sliced ELL for S (values of A) and S^T (values of A^T)
  MORX_TRY(owned_alloc(sys, &sys->csr2sell, nnzS));
  MORX_TRY(build_sell(sys, sys->rowptr, sys->colind, sys->valA, sys->sell, &sys->sell_val,
                      sys->csr2sell, st, tmp));
  MORX_TRY(build_sell(sys, sys->trowptr, sys->tcol, sys->tval, sys->sellT, &sys->sellT_val,
                      nullptr, st, tmp));
  MORX_TRY(build_halo(sys, sys->sell, st, tmp));
  MORX_TRY(build_halo(sys, sys->sellT, st, tmp));
  MORX_TRY(owned_alloc(sys, &sys->tp2s, nnzS));
  k_compose<<<nblk(nnzS), kBlock, 0, st>>>(tsrcp, sys->csr2sell, nnzS, sys->tp2s);
  MORX_TRY(owned_alloc(sys, &sys->e, sys->n_pad));
  k_copy_pad<<<nblk(sys->n_pad), kBlock, 0, st>>>(e_diag, sys->e, n, sys->n_pad);
  MORX_HIP(hipGetLastError());

  MORX_TRY(ls_pattern_stats(sys, st));
  MORX_HIP(hipStreamSynchronize(st));
  return MORX_OK;
}

extern "C" morx_status morx_system_create(morx_ctx ctx, int64_t n, int64_t nnz,
                                          const int32_t* rowptr, const int32_t* colind,
                                          const double* val, const double* e_diag, void* stream,
                                          morx_system* out) {
  MORX_REQUIRE(ctx && out, MORX_E_INVALID, "morx_system_create: null context or output");
  *out = nullptr;
  MORX_REQUIRE(n > 0 && n < (int64_t)INT32_MAX - kSlice, MORX_E_INVALID,
               "morx_system_create: n=%lld out of range", (long long)n);
  MORX_REQUIRE(nnz >= 0 && nnz < (int64_t)INT32_MAX, MORX_E_INVALID,
               "morx_system_create: nnz=%lld out of range", (long long)nnz);
  MORX_REQUIRE(rowptr && e_diag && (nnz == 0 || (colind && val)), MORX_E_INVALID,
               "morx_system_create: null input pointer");
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  MORX_TRY(stream_enter(ctx, caller));
  morx_system sys = new morx_system_s();
  sys->ctx = ctx;
  sys->n = n;
  sys->n_pad = (n + kSlice - 1) / kSlice * kSlice;
  sys->nslice = sys->n_pad / kSlice;
  sys->nnz_in = nnz;
  std::vector<DevBuf> tmp;
  morx_status s = system_build(sys, rowptr, colind, val, e_diag, ctx->stream, tmp);
  hipStreamSynchronize(ctx->stream);
  for (auto& b : tmp) dev_free(b);
  if (s != MORX_OK) {
    morx_system_destroy(sys);
    return s;
  }
  MORX_TRY(stream_leave(ctx, caller));
  *out = sys;
  return MORX_OK;
}

extern "C" morx_status morx_system_destroy(morx_system sys) {
  if (!sys) return MORX_OK;
  hipSetDevice(sys->ctx->device);
  hipStreamSynchronize(sys->ctx->stream);
  hipStreamSynchronize(sys->ctx->stream2);
  for (morx_factor f : sys->vertical) factor_release(f);
  sys->vertical.clear();
  for (morx_factor f : sys->factor_pool) {
    dev_free(f->vals);
    dev_free(f->valsT);
    delete f;
  }
  sys->factor_pool.clear();
  if (sys->kb) krylov_batch_delete(sys->kb);
  for (auto& b : sys->owned) dev_free(b);
  delete sys;
  return MORX_OK;
}

extern "C" morx_status morx_system_info(morx_system sys, int64_t* nnz_pattern,
                                        int64_t* resident_bytes) {
  MORX_REQUIRE(sys, MORX_E_INVALID, "morx_system_info: null system");
  if (nnz_pattern) *nnz_pattern = sys->nnzS;
  if (resident_bytes) *resident_bytes = sys->resident_bytes;
  return MORX_OK;
}

extern "C" morx_status morx_system_pattern(morx_system sys, int32_t* rowptr, int32_t* colind,
                                           void* stream) {
  MORX_REQUIRE(sys && rowptr && colind, MORX_E_INVALID, "morx_system_pattern: null argument");
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  MORX_HIP(hipMemcpyAsync(rowptr, sys->rowptr, (sys->n + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, st));
  MORX_HIP(hipMemcpyAsync(colind, sys->colind, sys->nnzS * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, st));
  MORX_HIP(hipStreamSynchronize(st));
  return MORX_OK;
}
