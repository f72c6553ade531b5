// Two-sided Petrov-Galerkin projection of the shifted-solve results
// (Section II, the reduced model after Algorithm 2; descriptor form):
//   V = orth(X), W = orth(Y), Ar = W^T A V, Er = W^T E V, Br = W^T B, Cr = V^T C.
//
// Every n-long contraction U^T diag(w) V (U: n x r1, V: n x r2, r <= 64) runs
// on FP64 MFMA (16x16x4 blocks): one wave per 16 x 16 output tile, each
// workgroup over one slab of rows, then a fixed-order sum of the slab
// partials.  orth is shifted Cholesky-QR with two more Cholesky-QR passes
// (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci. Comput.
// 2020), which stays stable for ill-conditioned X; it spans the same space as
// the Householder QR of the reference formulas, so the reduced transfer
// function is the same.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// partial[b] = U[rows_b]^T diag(w[rows_b]) V~[rows_b], column-major r1 x r2,
// where V~ is V, or with SPARSE the product A V formed row by row on the fly
// (A's rows on the sliced-ELL layout of S; the product is never stored).  One
// block of four waves per slab of rows: kGR rows of U and V~ at a time are
// staged in LDS, then every wave runs the 16 x 16 x 4 FP64 MFMA steps of its
// output tiles from LDS.  Thread t stages row t % kGR of columns t / kGR + 8 u
// (u < 8): a wave's loads of a column are consecutive rows, and a sparse row's
// slots are loaded once and serve all of the thread's columns, with every
// gather of a slot group in flight together.  The next step's loads are issued
// before the current step's MFMA work.  Slabs are numbered so that
// consecutive slabs run on one XCD (workgroups go round robin over the 8
// XCDs): a stencil row's neighbours one plane away lie a few slabs over, so
// the V entries they share are read through that XCD's L2.
constexpr int kGR = 32;        // rows staged per step
constexpr int kGLd = 64 + 2;   // LDS row stride (doubles)
constexpr int kGThreads = 256;
constexpr int kGItems = kGR * 64 / kGThreads;  // columns per thread
constexpr int kGSlots = 8;                     // sparse slots loaded together

template <bool SPARSE>
__device__ __forceinline__ void gram_load(const double* __restrict__ U, int64_t ldu, int r1,
                                          const double* __restrict__ V, int64_t ldv, int r2,
                                          const double* __restrict__ w, int64_t row, bool in,
                                          int c0, const int32_t* __restrict__ off,
                                          const int32_t* __restrict__ col,
                                          const double* __restrict__ val, double (&a)[kGItems],
                                          double (&b)[kGItems]) {
  const double wr = (w && in) ? w[row] : 1.0;
#pragma unroll
  for (int u = 0; u < kGItems; ++u) {
    const int c = c0 + 8 * u;
    a[u] = (in && c < r1) ? U[(int64_t)c * ldu + row] * wr : 0.0;
    b[u] = 0.0;
  }
  if constexpr (SPARSE) {
    if (!in) return;
    const int64_t sl = row >> 6;
    const int32_t p0 = off[sl] + (int32_t)(row & 63);
    const int width = (off[sl + 1] - off[sl]) >> 6;  // uniform over the 32 rows of a step
    for (int m0 = 0; m0 < width; m0 += kGSlots) {
      int32_t cc[kGSlots];
      double vv[kGSlots];
#pragma unroll
      for (int m = 0; m < kGSlots; ++m) {
        const bool ok = m0 + m < width;
        cc[m] = ok ? col[p0 + (m0 + m) * kSlice] : 0;
        vv[m] = ok ? val[p0 + (m0 + m) * kSlice] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kGItems; ++u) {
        const int c = c0 + 8 * u;
        if (c < r2) {  // uniform over the 32 lanes of a column
          const double* vc = V + (int64_t)c * ldv;
          double x[kGSlots];
#pragma unroll
          for (int m = 0; m < kGSlots; ++m) x[m] = vc[cc[m]];
#pragma unroll
          for (int m = 0; m < kGSlots; ++m) b[u] = fma(vv[m], x[m], b[u]);
        }
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < kGItems; ++u) {
      const int c = c0 + 8 * u;
      if (in && c < r2) b[u] = V[(int64_t)c * ldv + row];
    }
  }
}

template <bool SPARSE>
__global__ __launch_bounds__(kGThreads) void k_gram_mfma(
    const double* __restrict__ U, int64_t ldu, int r1, const double* __restrict__ V, int64_t ldv,
    int r2, const double* __restrict__ w, int64_t n, int64_t rows_per_block, int nb,
    const int32_t* __restrict__ off, const int32_t* __restrict__ col,
    const double* __restrict__ val, double* __restrict__ partial) {
  __shared__ double su[kGR * kGLd];
  __shared__ double sv[kGR * kGLd];
  // slab of this block: the grid is a multiple of 8 blocks, XCD-major
  const int slab = (int)(blockIdx.x & 7) * (int)(gridDim.x >> 3) + (int)(blockIdx.x >> 3);
  if (slab >= nb) return;  // uniform: the padding blocks of the grid
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t1n = (r1 + 15) >> 4, t2n = (r2 + 15) >> 4, ntile = t1n * t2n;
  const int kk = lane >> 4, li = lane & 15;
  const int rr = threadIdx.x % kGR, c0 = threadIdx.x / kGR;
  const int64_t r0 = (int64_t)slab * rows_per_block;
  const int64_t rend = min(n, r0 + rows_per_block);
  v4d acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  double a[kGItems], b[kGItems];
  gram_load<SPARSE>(U, ldu, r1, V, ldv, r2, w, r0 + rr, r0 + rr < rend, c0, off, col, val, a, b);
  for (int64_t base = r0; base < rend; base += kGR) {
    // rows base .. base + kGR - 1 (zeros past the slab and past r)
#pragma unroll
    for (int u = 0; u < kGItems; ++u) {
      su[rr * kGLd + c0 + 8 * u] = a[u];
      sv[rr * kGLd + c0 + 8 * u] = b[u];
    }
    __syncthreads();
    if (base + kGR < rend) {
      const int64_t row = base + kGR + rr;
      gram_load<SPARSE>(U, ldu, r1, V, ldv, r2, w, row, row < rend, c0, off, col, val, a, b);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int tile = wave + 4 * q;
      if (tile < ntile) {  // uniform over the wave
        const int ti = tile / t2n, tj = tile % t2n;
#pragma unroll
        for (int k = 0; k < kGR; k += 4) {
          const double x = su[(k + kk) * kGLd + ti * 16 + li];
          const double y = sv[(k + kk) * kGLd + tj * 16 + li];
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[q], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // output block: element t of lane l holds D[(l >> 4) + 4t][l & 15]
  double* out = partial + (int64_t)slab * r1 * r2;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int tile = wave + 4 * q;
    if (tile >= ntile) continue;
    const int ti = tile / t2n, tj = tile % t2n;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ii = ti * 16 + kk + 4 * t, jj = tj * 16 + li;
      if (ii < r1 && jj < r2) out[ii + (int64_t)jj * r1] = acc[q][t];
    }
  }
}

// out[k] = scale * sum_b partial[b][k]: one wave per output entry, fixed order
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int nb,
                                                      int cnt, double* __restrict__ out,
                                                      double scale) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= cnt) return;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += partial[(int64_t)b * cnt + k];
  s = wave_sum(s);
  if (lane == 0) out[k] = scale * s;
}

// upper Cholesky G + shift*I = R^T R of an r x r Gram matrix (one workgroup);
// status[0] = 1 when a pivot is not positive
__global__ __launch_bounds__(256) void k_chol(const double* __restrict__ G, int r, double shift_coef,
                                              double* __restrict__ R, int* __restrict__ status) {
  __shared__ double a[64 * 64];
  __shared__ double tr;
  for (int k = threadIdx.x; k < r * r; k += blockDim.x) a[k] = G[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int d = 0; d < r; ++d) t += a[d + d * r];
    tr = t;
  }
  __syncthreads();
  const double shift = shift_coef * tr;
  if ((int)threadIdx.x < r) a[threadIdx.x + threadIdx.x * r] += shift;
  __syncthreads();
  // column-major a; compute upper R in place (R[i][j] at a[i + j*r], i <= j)
  for (int k = 0; k < r; ++k) {
    if (threadIdx.x == 0) {
      double d = a[k + k * r];
      if (!(d > 0.0)) {
        status[0] = 1;
        d = 1.0;
      }
      a[k + k * r] = sqrt(d);
    }
    __syncthreads();
    const double rkk = a[k + k * r];
    for (int j = k + 1 + threadIdx.x; j < r; j += blockDim.x) a[k + j * r] /= rkk;
    __syncthreads();
    for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
      const int i = idx % r, j = idx / r;
      if (i > k && j >= i) a[i + j * r] -= a[k + i * r] * a[k + j * r];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
    const int i = idx % r, j = idx / r;
    R[idx] = (i <= j) ? a[idx] : 0.0;
  }
}

// X <- X R^{-1} row by row (R upper triangular, r <= RM, RM in {16, 32, 64}:
// the loops unroll over RM, so a small basis runs a short kernel)
template <int RM>
__global__ __launch_bounds__(256) void k_trsm_rows(double* __restrict__ X, int64_t ld, int64_t n,
                                                   int r, const double* __restrict__ R) {
  __shared__ double sr[RM * RM];  // R with row stride RM, zeros past r
  for (int k = threadIdx.x; k < RM * RM; k += blockDim.x) {
    const int l = k % RM, j = k / RM;
    sr[k] = (l < r && j < r) ? R[l + j * r] : 0.0;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x[RM];
#pragma unroll
  for (int j = 0; j < RM; ++j) x[j] = j < r ? X[(int64_t)j * ld + i] : 0.0;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    if (j < r) {
      double s = x[j];
#pragma unroll
      for (int l = 0; l < j; ++l) s -= x[l] * sr[l + j * RM];
      x[j] = s / sr[j + j * RM];
    }
  }
#pragma unroll
  for (int j = 0; j < RM; ++j)
    if (j < r) X[(int64_t)j * ld + i] = x[j];
}

__global__ void k_copy_cols(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                            int64_t ldd, int64_t n, int r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < n && c < r) dst[(int64_t)c * ldd + i] = src[(int64_t)c * lds + i];
}

// Partial sums of one n-long contraction: one partial r1 x r2 block per slab
// of rows (a multiple of kGR rows each), at most kPartialDoubles doubles of
// partials in all and about four slabs per CU.
constexpr size_t kPartialDoubles = (size_t)256 * 64 * 64;

struct Gram {
  morx_system sys;
  double* partial = nullptr;  // kPartialDoubles
};

struct GramShape {
  int64_t rows_per_block;
  int nb;    // slabs
  int grid;  // nb rounded up to a multiple of 8
};

GramShape gram_shape(const Gram& g, int r1, int r2) {
  const int64_t n = g.sys->n;
  const int64_t cap = (int64_t)(kPartialDoubles / ((size_t)r1 * r2));
  const int64_t target =
      std::max<int64_t>(1, std::min<int64_t>(cap, 4 * (int64_t)std::max(1, g.sys->ctx->num_cu)));
  const int64_t per = (n + target - 1) / target;
  GramShape s;
  s.rows_per_block = std::max<int64_t>(kGR, (per + kGR - 1) / kGR * kGR);
  s.nb = (int)std::max<int64_t>(1, (n + s.rows_per_block - 1) / s.rows_per_block);
  s.grid = (s.nb + 7) / 8 * 8;
  return s;
}

// out_dev = scale * U^T diag(w) V~ (V~ = V, or A V when sparse)
morx_status gram(const Gram& g, const double* U, int64_t ldu, int r1, const double* V,
                 int64_t ldv, int r2, const double* w, bool sparse, double* out_dev,
                 double scale, hipStream_t st) {
  const int64_t n = g.sys->n;
  morx_system sys = g.sys;
  const GramShape s = gram_shape(g, r1, r2);
  if (sparse)
    k_gram_mfma<true><<<s.grid, kGThreads, 0, st>>>(U, ldu, r1, V, ldv, r2, w, n,
                                                     s.rows_per_block, s.nb, sys->sell.off,
                                                     sys->sell.col, sys->sell_val, g.partial);
  else
    k_gram_mfma<false><<<s.grid, kGThreads, 0, st>>>(U, ldu, r1, V, ldv, r2, w, n,
                                                      s.rows_per_block, s.nb, nullptr, nullptr,
                                                      nullptr, g.partial);
  const int cnt = r1 * r2;
  k_sum_partials<<<(cnt + 3) / 4, 256, 0, st>>>(g.partial, s.nb, cnt, out_dev, scale);
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

// shifted Cholesky-QR, then two Cholesky-QR passes, in place on X (n x r, ld)
morx_status orth_scqr3(const Gram& g, double* X, int64_t ld, int r, double* G, double* R,
                       int* status, hipStream_t st) {
  const int64_t n = g.sys->n;
  const double u = 1.1102230246251565e-16;
  const double coef = 11.0 * ((double)n * r + (double)r * (r + 1)) * u;
  for (int pass = 0; pass < 3; ++pass) {
    MORX_TRY(gram(g, X, ld, r, X, ld, r, nullptr, false, G, 1.0, st));
    k_chol<<<1, 256, 0, st>>>(G, r, pass == 0 ? coef : 0.0, R, status);
    const unsigned tg = (unsigned)((n + 255) / 256);
    if (r <= 16) k_trsm_rows<16><<<tg, 256, 0, st>>>(X, ld, n, r, R);
    else if (r <= 32) k_trsm_rows<32><<<tg, 256, 0, st>>>(X, ld, n, r, R);
    else k_trsm_rows<64><<<tg, 256, 0, st>>>(X, ld, n, r, R);
    MORX_HIP(hipGetLastError());
  }
  return MORX_OK;
}

// the four products of the reduced model into res = [Ar | Er | Br | Cr]
// (4096 doubles each, column-major with ld r)
morx_status project_products(const Gram& g, int r, const double* Vd, int64_t ldv,
                             const double* Wd, int64_t ldw, int m, const double* B, int64_t ldb,
                             int q, const double* C, int64_t ldc, double* res, hipStream_t st) {
  MORX_TRY(gram(g, Wd, ldw, r, Vd, ldv, r, nullptr, true, res, 1.0, st));             // W^T A V
  MORX_TRY(gram(g, Wd, ldw, r, Vd, ldv, r, g.sys->e, false, res + 4096, 1.0, st));     // W^T E V
  if (m > 0) MORX_TRY(gram(g, Wd, ldw, r, B, ldb, m, nullptr, false, res + 8192, 1.0, st));
  if (q > 0) MORX_TRY(gram(g, Vd, ldv, r, C, ldc, q, nullptr, false, res + 12288, 1.0, st));
  return MORX_OK;
}

morx_status check_project_args(morx_system sys, int32_t r, const double* V, int64_t ldv,
                               const double* W, int64_t ldw, int32_t m, const double* B,
                               int64_t ldb, int32_t q, const double* C, int64_t ldc, double* Ar,
                               double* Er, double* Br, double* Cr, const char* who) {
  MORX_REQUIRE(sys, MORX_E_INVALID, "%s: null system", who);
  MORX_REQUIRE(r >= 1 && r <= 64 && m >= 0 && m <= 64 && q >= 0 && q <= 64, MORX_E_INVALID,
               "%s: r, m, q must be in [1, 64], [0, 64], [0, 64]", who);
  MORX_REQUIRE(V && W && ldv >= sys->n && ldw >= sys->n && Ar && Er, MORX_E_INVALID,
               "%s: bad V, W or outputs", who);
  MORX_REQUIRE(m == 0 || (B && Br && ldb >= sys->n), MORX_E_INVALID, "%s: bad B", who);
  MORX_REQUIRE(q == 0 || (C && Cr && ldc >= sys->n), MORX_E_INVALID, "%s: bad C", who);
  return MORX_OK;
}

// the device results (ld r) into the caller's host arrays
morx_status copy_results(const double* res, int r, int m, int q, double* Ar, double* Er,
                         double* Br, double* Cr, hipStream_t st) {
  MORX_HIP(hipMemcpyAsync(Ar, res, (size_t)r * r * sizeof(double), hipMemcpyDeviceToHost, st));
  MORX_HIP(hipMemcpyAsync(Er, res + 4096, (size_t)r * r * sizeof(double), hipMemcpyDeviceToHost, st));
  if (m > 0)
    MORX_HIP(hipMemcpyAsync(Br, res + 8192, (size_t)r * m * sizeof(double), hipMemcpyDeviceToHost, st));
  if (q > 0)
    MORX_HIP(hipMemcpyAsync(Cr, res + 12288, (size_t)r * q * sizeof(double), hipMemcpyDeviceToHost, st));
  return MORX_OK;
}

// Scratch of the allocation-free projection: the slab partials of one
// contraction at a time, then the four results.  Every GPU the library runs
// on holds its own copy until the process ends.
constexpr size_t kScratchPartial = kPartialDoubles;
constexpr size_t kScratchResults = 4 * 4096;                        // doubles
__device__ __align__(256) double scratch[kScratchPartial + kScratchResults];

}  // namespace

// Called by morx_create with the context's device current: the device
// address of this GPU's scratch (host code never passes the array's name).
morx_status project_scratch_init(morx_ctx ctx) {
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  MORX_REQUIRE(e == hipSuccess && ptr, MORX_E_HIP, "projection scratch address: %s",
               hipGetErrorString(e));
  ctx->proj_scratch = (double*)ptr;
  return MORX_OK;
}

extern "C" morx_status morx_project(morx_system sys, int32_t r, const double* V, int64_t ldv,
                                    const double* W, int64_t ldw, int32_t m, const double* B,
                                    int64_t ldb, int32_t q, const double* C, int64_t ldc,
                                    double* Ar, double* Er, double* Br, double* Cr,
                                    int32_t orthonormalize, void* stream) {
  MORX_TRY(check_project_args(sys, r, V, ldv, W, ldw, m, B, ldb, q, C, ldc, Ar, Er, Br, Cr,
                              "morx_project"));
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  MORX_TRY(stream_enter(ctx, caller));
  hipStream_t st = ctx->stream;
  const int64_t n = sys->n, ld = sys->n_pad;
  DevBuf part, vv, ww, small, stat;
  morx_status s = dev_alloc(part, kPartialDoubles * sizeof(double));
  const Gram g{sys, (double*)part.p};
  if (s == MORX_OK && orthonormalize) s = dev_alloc(vv, (size_t)ld * r * sizeof(double));
  if (s == MORX_OK && orthonormalize) s = dev_alloc(ww, (size_t)ld * r * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(small, (size_t)6 * 4096 * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(stat, sizeof(int));
  int status = 0;
  if (s == MORX_OK) {
    double* S = (double*)small.p;
    double *res = S, *G = S + 4 * 4096, *R = S + 5 * 4096;
    const double* Vd = V;
    const double* Wd = W;
    int64_t ldvd = ldv, ldwd = ldw;
    hipError_t e = hipMemsetAsync(stat.p, 0, sizeof(int), st);
    if (e != hipSuccess) s = MORX_E_HIP;
    if (s == MORX_OK && orthonormalize) {
      // orthonormal bases of the columns of V and W, in copies
      dim3 cg((unsigned)((n + 255) / 256), r);
      k_copy_cols<<<cg, 256, 0, st>>>(V, ldv, (double*)vv.p, ld, n, r);
      k_copy_cols<<<cg, 256, 0, st>>>(W, ldw, (double*)ww.p, ld, n, r);
      s = orth_scqr3(g, (double*)vv.p, ld, r, G, R, (int*)stat.p, st);
      if (s == MORX_OK) s = orth_scqr3(g, (double*)ww.p, ld, r, G, R, (int*)stat.p, st);
      Vd = (const double*)vv.p;
      Wd = (const double*)ww.p;
      ldvd = ldwd = ld;
    }
    if (s == MORX_OK) s = project_products(g, r, Vd, ldvd, Wd, ldwd, m, B, ldb, q, C, ldc, res, st);
    if (s == MORX_OK) s = copy_results(res, r, m, q, Ar, Er, Br, Cr, st);
    if (s == MORX_OK) {
      e = hipMemcpyAsync(&status, stat.p, sizeof(int), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        morx_set_error("morx_project: %s", hipGetErrorString(e));
        s = MORX_E_HIP;
      }
    }
  }
  hipStreamSynchronize(st);
  dev_free(part);
  dev_free(vv);
  dev_free(ww);
  dev_free(small);
  dev_free(stat);
  if (s != MORX_OK) return s;
  MORX_REQUIRE(status == 0, MORX_E_SINGULAR_LS,
               "morx_project: Cholesky-QR failed (V or W numerically rank deficient)");
  return stream_leave(ctx, caller);
}

extern "C" morx_status morx_project_noalloc(morx_system sys, int32_t r, const double* V,
                                            int64_t ldv, const double* W, int64_t ldw, int32_t m,
                                            const double* B, int64_t ldb, int32_t q,
                                            const double* C, int64_t ldc, double* Ar, double* Er,
                                            double* Br, double* Cr, void* stream) {
  MORX_TRY(check_project_args(sys, r, V, ldv, W, ldw, m, B, ldb, q, C, ldc, Ar, Er, Br, Cr,
                              "morx_project_noalloc"));
  morx_ctx ctx = sys->ctx;
  MORX_REQUIRE(ctx->proj_scratch, MORX_E_HIP, "morx_project_noalloc: no scratch on device %d",
               ctx->device);
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const Gram g{sys, ctx->proj_scratch};
  double* res = ctx->proj_scratch + kScratchPartial;
  MORX_TRY(project_products(g, r, V, ldv, W, ldw, m, B, ldb, q, C, ldc, res, st));
  MORX_TRY(copy_results(res, r, m, q, Ar, Er, Br, Cr, st));
  MORX_HIP(hipStreamSynchronize(st));
  return MORX_OK;
}
