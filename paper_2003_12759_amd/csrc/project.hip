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

// partial[b] = U[rows_b]^T diag(w[rows_b]) V[rows_b], column-major r1 x r2
__global__ __launch_bounds__(1024) void k_gram_mfma(const double* __restrict__ U, int64_t ldu,
                                                    int r1, const double* __restrict__ V,
                                                    int64_t ldv, int r2,
                                                    const double* __restrict__ w, int64_t n,
                                                    int64_t rows_per_block,
                                                    double* __restrict__ partial) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t2n = (r2 + 15) >> 4;
  const int ti = wave / t2n, tj = wave % t2n;
  const int i = ti * 16 + (lane & 15), j = tj * 16 + (lane & 15), kk = lane >> 4;
  const bool iv = i < r1, jv = j < r2;
  const double* up = U + (int64_t)min(i, r1 - 1) * ldu;
  const double* vp = V + (int64_t)min(j, r2 - 1) * ldv;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t rend = min(n, r0 + rows_per_block);
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  // uniform trip count: every lane issues every MFMA
  for (int64_t base = r0; base < r0 + rows_per_block; base += 4) {
    const int64_t row = base + kk;
    const bool in = row < rend;
    double a = (in && iv) ? up[row] : 0.0;
    if (w && in) a *= w[row];
    const double b = (in && jv) ? vp[row] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  // output block: element t of lane l holds D[(l >> 4) + 4t][l & 15]
  double* out = partial + (int64_t)blockIdx.x * r1 * r2;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int ii = ti * 16 + (lane >> 4) + 4 * t, jj = tj * 16 + (lane & 15);
    if (ii < r1 && jj < r2) out[ii + (int64_t)jj * r1] = acc[t];
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

// X <- X R^{-1} row by row (R upper triangular, r <= 64)
__global__ __launch_bounds__(256) void k_trsm_rows(double* __restrict__ X, int64_t ld, int64_t n,
                                                   int r, const double* __restrict__ R) {
  __shared__ double sr[64 * 64];
  for (int k = threadIdx.x; k < r * r; k += blockDim.x) sr[k] = R[k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x[64];
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < r) x[j] = X[(int64_t)j * ld + i];
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    if (j < r) {
      double s = x[j];
#pragma unroll
      for (int l = 0; l < 64; ++l)
        if (l < j) s -= x[l] * sr[l + j * r];
      x[j] = s / sr[j + j * r];
    }
  }
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < r) X[(int64_t)j * ld + i] = x[j];
}

__global__ void k_copy_cols(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                            int64_t ldd, int64_t n, int r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i < n && c < r) dst[(int64_t)c * ldd + i] = src[(int64_t)c * lds + i];
}

struct Gram {
  morx_system sys;
  DevBuf partial;
  int64_t rows_per_block = 0;
  int nb = 0;
};

morx_status gram(Gram& g, const double* U, int64_t ldu, int r1, const double* V, int64_t ldv,
                 int r2, const double* w, double* out_dev, double scale, hipStream_t st) {
  const int64_t n = g.sys->n;
  const int waves = ((r1 + 15) / 16) * ((r2 + 15) / 16);
  k_gram_mfma<<<g.nb, 64 * waves, 0, st>>>(U, ldu, r1, V, ldv, r2, w, n, g.rows_per_block,
                                          (double*)g.partial.p);
  const int cnt = r1 * r2;
  k_sum_partials<<<(cnt + 3) / 4, 256, 0, st>>>((double*)g.partial.p, g.nb, cnt, out_dev, scale);
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

// shifted Cholesky-QR, then two Cholesky-QR passes, in place on X (n x r, ld)
morx_status orth_scqr3(Gram& g, double* X, int64_t ld, int r, double* G, double* R, int* status,
                       hipStream_t st) {
  const int64_t n = g.sys->n;
  const double u = 1.1102230246251565e-16;
  const double coef = 11.0 * ((double)n * r + (double)r * (r + 1)) * u;
  for (int pass = 0; pass < 3; ++pass) {
    MORX_TRY(gram(g, X, ld, r, X, ld, r, nullptr, G, 1.0, st));
    k_chol<<<1, 256, 0, st>>>(G, r, pass == 0 ? coef : 0.0, R, status);
    k_trsm_rows<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(X, ld, n, r, R);
    MORX_HIP(hipGetLastError());
  }
  return MORX_OK;
}

}  // namespace

extern "C" morx_status morx_project(morx_system sys, int32_t r, const double* V, int64_t ldv,
                                    const double* W, int64_t ldw, int32_t m, const double* B,
                                    int64_t ldb, int32_t q, const double* C, int64_t ldc,
                                    double* Ar, double* Er, double* Br, double* Cr,
                                    int32_t orthonormalize, void* stream) {
  MORX_REQUIRE(sys, MORX_E_INVALID, "morx_project: null system");
  MORX_REQUIRE(r >= 1 && r <= 64 && m >= 0 && m <= 64 && q >= 0 && q <= 64, MORX_E_INVALID,
               "morx_project: r, m, q must be in [1, 64], [0, 64], [0, 64]");
  MORX_REQUIRE(V && W && ldv >= sys->n && ldw >= sys->n && Ar && Er, MORX_E_INVALID,
               "morx_project: bad V, W or outputs");
  MORX_REQUIRE(m == 0 || (B && Br && ldb >= sys->n), MORX_E_INVALID, "morx_project: bad B");
  MORX_REQUIRE(q == 0 || (C && Cr && ldc >= sys->n), MORX_E_INVALID, "morx_project: bad C");
  morx_ctx ctx = sys->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  MORX_HIP(hipSetDevice(ctx->device));
  hipStream_t caller = (hipStream_t)stream;
  MORX_TRY(stream_enter(ctx, caller));
  hipStream_t st = ctx->stream;
  const int64_t n = sys->n, ld = sys->n_pad;
  Gram g;
  g.sys = sys;
  const int64_t target_blocks = std::max(1, 2 * ctx->num_cu);
  g.rows_per_block = std::max<int64_t>(256, ((n + target_blocks - 1) / target_blocks + 3) / 4 * 4);
  g.nb = (int)((n + g.rows_per_block - 1) / g.rows_per_block);
  DevBuf vv, ww, tt, small, stat;
  morx_status s = dev_alloc(g.partial, (size_t)g.nb * 64 * 64 * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(vv, (size_t)ld * r * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(ww, (size_t)ld * r * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(tt, (size_t)ld * r * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(small, (size_t)8 * 64 * 64 * sizeof(double));
  if (s == MORX_OK) s = dev_alloc(stat, sizeof(int));
  std::vector<double> h(4 * 64 * 64);
  int status = 0;
  if (s == MORX_OK) {
    double* Vd = (double*)vv.p;
    double* Wd = (double*)ww.p;
    double* T = (double*)tt.p;
    double* S = (double*)small.p;
    double *G = S, *R = S + 4096, *oA = S + 2 * 4096, *oE = S + 3 * 4096, *oB = S + 4 * 4096,
           *oC = S + 5 * 4096;
    hipError_t e = hipMemsetAsync(stat.p, 0, sizeof(int), st);
    dim3 cg((unsigned)((n + 255) / 256), r);
    k_copy_cols<<<cg, 256, 0, st>>>(V, ldv, Vd, ld, n, r);
    k_copy_cols<<<cg, 256, 0, st>>>(W, ldw, Wd, ld, n, r);
    if (e != hipSuccess) s = MORX_E_HIP;
    if (s == MORX_OK && orthonormalize) {
      s = orth_scqr3(g, Vd, ld, r, G, R, (int*)stat.p, st);
      if (s == MORX_OK) s = orth_scqr3(g, Wd, ld, r, G, R, (int*)stat.p, st);
    }
    // T = (0 E - A) V = -A V, so Ar = -W^T T
    if (s == MORX_OK) s = launch_shifted_apply(sys, 0.0, false, r, Vd, ld, T, ld, st);
    if (s == MORX_OK) s = gram(g, Wd, ld, r, T, ld, r, nullptr, oA, -1.0, st);
    if (s == MORX_OK) s = gram(g, Wd, ld, r, Vd, ld, r, sys->e, oE, 1.0, st);
    if (s == MORX_OK && m > 0) s = gram(g, Wd, ld, r, B, ldb, m, nullptr, oB, 1.0, st);
    if (s == MORX_OK && q > 0) s = gram(g, Vd, ld, r, C, ldc, q, nullptr, oC, 1.0, st);
    if (s == MORX_OK) {
      e = hipMemcpyAsync(h.data(), oA, 4 * 4096 * sizeof(double), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(&status, stat.p, sizeof(int), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        morx_set_error("morx_project: %s", hipGetErrorString(e));
        s = MORX_E_HIP;
      }
    }
  }
  hipStreamSynchronize(st);
  dev_free(g.partial);
  dev_free(vv);
  dev_free(ww);
  dev_free(tt);
  dev_free(small);
  dev_free(stat);
  if (s != MORX_OK) return s;
  MORX_REQUIRE(status == 0, MORX_E_SINGULAR_LS,
               "morx_project: Cholesky-QR failed (V or W numerically rank deficient)");
  std::copy(h.begin(), h.begin() + r * r, Ar);
  std::copy(h.begin() + 4096, h.begin() + 4096 + r * r, Er);
  if (m > 0) std::copy(h.begin() + 2 * 4096, h.begin() + 2 * 4096 + r * m, Br);
  if (q > 0) std::copy(h.begin() + 3 * 4096, h.begin() + 3 * 4096 + r * q, Cr);
  return stream_leave(ctx, caller);
}
