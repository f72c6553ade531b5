// Shifted operator and single-factor products on the sliced-ELL layouts.
//
//   Y = (sigma E - A) X        rows of S with A's values, E's diagonal fused
//   Y = (sigma E - A)^T X      rows of S^T with A^T's values
//   Y = F X, Y = F^T X         a SPAI or update factor (FP64/FP32/BF16 values)
//
// One thread per row, up to NC columns per thread; the shifted matrix and the
// preconditioner product are never formed (Section III-B; appendix B form).
// These simple kernels serve the GMRES comparator and the projection; the
// public product entry points below run the solve's own kernels instead.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace {

constexpr int kBlock = 256;

template <int NC>
__global__ __launch_bounds__(kBlock) void k_shifted(const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ e, double sigma,
                                                    int64_t n, int ncol, const double* X,
                                                    int64_t ldx, double* Y, int64_t ldy) {
  const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int c0 = blockIdx.y * NC;
  if (row >= n) return;
  const double* x[NC];
  double acc[NC];
  unsigned mask = 0;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    x[j] = X + (int64_t)std::min(c0 + j, ncol - 1) * ldx;
    acc[j] = 0.0;
    if (c0 + j < ncol) mask |= 1u << j;
  }
  sell_row<double, NC>(off, col, val, row, x, mask, acc);
  const double se = sigma * e[row];
#pragma unroll
  for (int j = 0; j < NC; ++j)
    if (mask & (1u << j)) Y[(int64_t)(c0 + j) * ldy + row] = fma(se, x[j][row], -acc[j]);
}

template <typename VT, int NC>
__global__ __launch_bounds__(kBlock) void k_factor(const int32_t* __restrict__ off,
                                                   const int32_t* __restrict__ col,
                                                   const VT* __restrict__ val, int64_t n,
                                                   int ncol, const double* X, int64_t ldx,
                                                   double* Y, int64_t ldy) {
  const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int c0 = blockIdx.y * NC;
  if (row >= n) return;
  const double* x[NC];
  double acc[NC];
  unsigned mask = 0;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    x[j] = X + (int64_t)std::min(c0 + j, ncol - 1) * ldx;
    acc[j] = 0.0;
    if (c0 + j < ncol) mask |= 1u << j;
  }
  sell_row<VT, NC>(off, col, val, row, x, mask, acc);
#pragma unroll
  for (int j = 0; j < NC; ++j)
    if (mask & (1u << j)) Y[(int64_t)(c0 + j) * ldy + row] = acc[j];
}

constexpr int kNC = 4;

inline dim3 grid_for(int64_t n, int ncol) {
  return dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)((ncol + kNC - 1) / kNC));
}

}  // namespace

morx_status launch_shifted_apply(morx_system sys, double sigma, bool trans, int ncol,
                                 const double* X, int64_t ldx, double* Y, int64_t ldy,
                                 hipStream_t st) {
  if (ncol <= 0) return MORX_OK;
  const Sell& L = trans ? sys->sellT : sys->sell;
  const double* v = trans ? sys->sellT_val : sys->sell_val;
  k_shifted<kNC><<<grid_for(sys->n, ncol), kBlock, 0, st>>>(L.off, L.col, v, sys->e, sigma, sys->n,
                                                            ncol, X, ldx, Y, ldy);
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

morx_status launch_factor_apply(morx_system sys, morx_factor f, bool trans, int ncol,
                                const double* X, int64_t ldx, double* Y, int64_t ldy,
                                hipStream_t st) {
  if (ncol <= 0) return MORX_OK;
  const Sell& L = trans ? sys->sellT : sys->sell;
  const void* v = trans ? f->valsT.p : f->vals.p;
  dim3 g = grid_for(sys->n, ncol);
  switch (f->prec) {
    case MORX_F64:
      k_factor<double, kNC><<<g, kBlock, 0, st>>>(L.off, L.col, (const double*)v, sys->n, ncol, X,
                                                  ldx, Y, ldy);
      break;
    case MORX_F32:
      k_factor<float, kNC><<<g, kBlock, 0, st>>>(L.off, L.col, (const float*)v, sys->n, ncol, X,
                                                 ldx, Y, ldy);
      break;
    default:
      k_factor<uint16_t, kNC><<<g, kBlock, 0, st>>>(L.off, L.col, (const uint16_t*)v, sys->n, ncol,
                                                    X, ldx, Y, ldy);
  }
  MORX_HIP(hipGetLastError());
  return MORX_OK;
}

// The public single products run the solve's kernels (bicg.hip), in chunks
// of at most 1024 columns.
constexpr int kProbeChunk = 1024;

extern "C" morx_status morx_shifted_apply(morx_system sys, double sigma, int32_t trans,
                                          int32_t ncol, const double* X, int64_t ldx, double* Y,
                                          int64_t ldy, void* stream) {
  MORX_REQUIRE(sys, MORX_E_INVALID, "morx_shifted_apply: null system");
  MORX_REQUIRE(ncol >= 0 && (ncol == 0 || (X && Y)), MORX_E_INVALID,
               "morx_shifted_apply: bad columns or null pointer");
  MORX_REQUIRE(ldx >= sys->n && ldy >= sys->n, MORX_E_INVALID,
               "morx_shifted_apply: leading dimension below n");
  MORX_REQUIRE(std::isfinite(sigma), MORX_E_NONFINITE, "morx_shifted_apply: shift not finite");
  if (ncol == 0) return MORX_OK;
  std::lock_guard<std::mutex> lk(sys->ctx->mu);
  MORX_HIP(hipSetDevice(sys->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const std::vector<double> sig(std::min(ncol, kProbeChunk), sigma);
  for (int c0 = 0; c0 < ncol; c0 += kProbeChunk) {
    const int nc = std::min(kProbeChunk, ncol - c0);
    const double* x = X + (int64_t)c0 * ldx;
    double* y = Y + (int64_t)c0 * ldy;
    if (trans) MORX_TRY(hot_shifted_pair(sys, nc, sig.data(), nullptr, 0, nullptr, 0, x, ldx, y, ldy, st));
    else MORX_TRY(hot_shifted_pair(sys, nc, sig.data(), x, ldx, y, ldy, nullptr, 0, nullptr, 0, st));
  }
  return MORX_OK;
}

extern "C" morx_status morx_chain_apply(morx_system sys, int32_t nfactor, const morx_factor* chain,
                                        int32_t trans, int32_t ncol, const double* X, int64_t ldx,
                                        double* Y, int64_t ldy, void* stream) {
  MORX_REQUIRE(sys && nfactor >= 1 && nfactor <= 64 && chain, MORX_E_INVALID,
               "morx_chain_apply: bad chain");
  MORX_REQUIRE(ncol >= 0 && (ncol == 0 || (X && Y)), MORX_E_INVALID,
               "morx_chain_apply: bad columns or null pointer");
  MORX_REQUIRE(ldx >= sys->n && ldy >= sys->n, MORX_E_INVALID,
               "morx_chain_apply: leading dimension below n");
  for (int i = 0; i < nfactor; ++i) {
    MORX_REQUIRE(chain[i] && chain[i]->sys == sys, MORX_E_INVALID,
                 "morx_chain_apply: factor %d does not belong to this system", i);
    MORX_REQUIRE(chain[i]->prec == chain[0]->prec, MORX_E_INVALID,
                 "morx_chain_apply: factors of different storage precisions");
  }
  if (ncol == 0) return MORX_OK;
  std::lock_guard<std::mutex> lk(sys->ctx->mu);
  MORX_HIP(hipSetDevice(sys->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int nmax = std::min(ncol, kProbeChunk);
  std::vector<morx_factor> tab((size_t)nmax * nfactor);
  for (int c = 0; c < nmax; ++c)
    for (int k = 0; k < nfactor; ++k) tab[(size_t)c * nfactor + k] = chain[k];
  const std::vector<int32_t> lens(nmax, nfactor);
  for (int c0 = 0; c0 < ncol; c0 += kProbeChunk) {
    const int nc = std::min(kProbeChunk, ncol - c0);
    const double* x = X + (int64_t)c0 * ldx;
    double* y = Y + (int64_t)c0 * ldy;
    if (trans)
      MORX_TRY(hot_chain_apply(sys, nc, nfactor, tab.data(), lens.data(), nullptr, 0, nullptr, 0,
                               x, ldx, y, ldy, MORX_F64, st));
    else
      MORX_TRY(hot_chain_apply(sys, nc, nfactor, tab.data(), lens.data(), x, ldx, y, ldy, nullptr,
                               0, nullptr, 0, MORX_F64, st));
  }
  return MORX_OK;
}
