// Internal declarations shared by the libmorx sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/morx.h"

// ---------------------------------------------------------------------------
// error plumbing

void morx_set_error(const char* fmt, ...);

#define MORX_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      morx_set_error("%s:%d: %s -> %s", __FILE__, __LINE__, #call, hipGetErrorString(e_)); \
      return MORX_E_HIP;                                                            \
    }                                                                               \
  } while (0)

#define MORX_TRY(expr)                 \
  do {                                 \
    morx_status s_ = (expr);           \
    if (s_ != MORX_OK) return s_;      \
  } while (0)

#define MORX_REQUIRE(cond, code, ...)  \
  do {                                 \
    if (!(cond)) {                     \
      morx_set_error(__VA_ARGS__);     \
      return code;                     \
    }                                  \
  } while (0)

// ---------------------------------------------------------------------------
// constants

constexpr int kSlice = 64;         // sliced-ELL slice height = one wavefront
// Halo layout of a wide pattern: rows are grouped in blocks of kHaloSlices
// slices; each block lists the distinct columns its entries touch (at most
// kHaloCap), and each entry stores its column's position in that list.
constexpr int kHaloSlices = 4;
constexpr int kHaloCap = 2048;
constexpr int kHaloCapNarrow = 1024;  // list cap of the kernel for slices of <= 8 slots
constexpr int kHaloMaxW = 32;      // widest slice the halo layout takes
// A block's list in runs of consecutive columns (a stencil's block lists one
// run per grid plane): kHaloRunInts integers per block, the run count (0: the
// list has more than kHaloRuns runs and is read as it is) then per run its
// first column and its first list position
constexpr int kHaloRuns = 7;
constexpr int kHaloRunInts = 16;
// Entries past the end of a sliced-ELL value or local-index array: the halo
// chain step reads all kHaloMaxW slots of a slice with one address and
// discards those past its width, so the last slice may read this far beyond.
constexpr int64_t kSellPad = (int64_t)kHaloMaxW * kSlice;
constexpr int kMaxJ = 31;          // max entries of one column of S
constexpr int kMaxI = 512;         // max rows of one local least-squares matrix
constexpr int kMaxTriples = 2048;  // max nonzeros gathered for one column problem

// per-column BiCG status values kept on the device
enum ColState : int32_t {
  COL_ACTIVE = 0,
  COL_CONVERGED = 1,   // recursive residuals passed, true residual not yet checked
  COL_BREAKDOWN = 2,   // near-breakdown seen: restart from true residuals
  COL_MAXIT = 3,       // iteration limit of the cycle reached
  COL_DONE = 4,        // true residuals passed
  COL_FAILED = 5,      // gave up (see host-side status)
  COL_IDLE = 6,        // free slot
  COL_INIT = 7         // filled slot waiting for its first initialisation
};

// ---------------------------------------------------------------------------
// device buffer helper

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

morx_status dev_alloc(DevBuf& b, size_t bytes);
void dev_free(DevBuf& b);

// sliced ELL (height 64) of a square pattern: slice s covers rows 64s..64s+63,
// entry m of row i sits at off[s] + m*64 + (i % 64).
struct Sell {
  int32_t* off = nullptr;  // [nslice+1]
  int32_t* col = nullptr;  // [nnz_sell]
  int64_t nnz_sell = 0;
  int32_t max_width = 0;
  // halo layout (patterns wider than eight slots): per block of kHaloSlices
  // slices, its ascending distinct columns hcol[hoff[b] .. hoff[b+1]), and
  // per entry the position of its column in its block's list
  int32_t* hoff = nullptr;   // [ceil(nslice / kHaloSlices) + 1]
  int32_t* hcol = nullptr;
  uint16_t* lidx = nullptr;  // [nnz_sell]
  int32_t* hrun = nullptr;   // [blocks * kHaloRunInts]: the lists as runs
  int32_t hmax = 0;          // longest list; 0: no halo layout
  // row-block distance whose lists share the most columns (a grid plane
  // for lexicographically ordered stencils); 1 when no longer one shares more
  // than the next row block
  int32_t hstride = 1;
};

struct morx_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;   // internal work stream (capturable)
  hipStream_t stream2 = nullptr;  // factor construction overlapped with solves
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_aux = nullptr;
  int num_cu = 0;
  double* proj_scratch = nullptr;  // this device's allocation-free projection scratch
  std::mutex mu;
};

struct morx_factor_s {
  morx_system sys = nullptr;
  int32_t prec = MORX_F64;
  double sigma_prev = 0.0, sigma_new = 0.0;
  bool is_spai = true;
  DevBuf vals;      // SELL(S) order, for F x
  DevBuf valsT;     // SELL(S^T) order, for F^T x
  bool pooled = false;
};

struct KrylovBatch;  // BiCG slots (krylov.h)

struct morx_system_s {
  morx_ctx ctx = nullptr;
  int64_t n = 0, n_pad = 0, nslice = 0;
  int64_t nnz_in = 0, nnzS = 0;
  // CSR of S (A's values, explicit zero where the diagonal was inserted)
  int32_t* rowptr = nullptr;
  int32_t* colind = nullptr;
  double* valA = nullptr;
  // CSR of S^T: row k lists column k of S; tval = A(i,k) at entry (k,i)
  int32_t* trowptr = nullptr;
  int32_t* tcol = nullptr;
  double* tval = nullptr;
  int32_t* tp2s = nullptr;      // CSR(S^T) position -> SELL(S) position
  int32_t* csr2sell = nullptr;  // CSR(S) position -> SELL(S) position
  // sliced ELL layouts
  Sell sell, sellT;
  double* sell_val = nullptr;   // A on SELL(S)
  double* sellT_val = nullptr;  // A^T on SELL(S^T)
  bool symmetric_pattern = false;
  double* e = nullptr;          // [n_pad], zero padded
  // local least-squares sizes
  int32_t max_J = 0, max_T = 0, max_I = 0;
  bool ls_supported = true;
  // launch shapes (morx_tune): -1 means the built-in heuristic
  int32_t tune_factor_rows = -1;  // least-squares kernel (morx_tune.factor_kernel)
  int32_t* ls_fallback = nullptr;  // columns the normal equations leave to Householder QR
  int32_t tune_nc = -1;           // chain step: most columns per wave (1..8)
  int32_t tune_nc_spmv = -1;      // shifted pair, true residual: the same (-1: tune_nc)
  int32_t tune_spw = -1;          // iteration kernels: 64-row slices per wave
  int32_t tune_chain = -1;        // chain step: 0 row gathers, 1 halo in LDS (-1: built-in)
  std::vector<DevBuf> owned;
  // chain state between morx_solve_shifts calls (Algorithm 4)
  std::vector<morx_factor> vertical;  // P_1^(1), Q_1^(2), ..., Q_1^(z)
  double last_first_shift = 0.0;
  int32_t vertical_prec = -1;
  // factor chains of the last solve call, per shift in application order
  std::vector<std::vector<morx_factor_spec>> last_chains;
  bool has_last_chains = false;
  // recycled factor storage and BiCG workspace
  std::vector<morx_factor> factor_pool;
  KrylovBatch* kb = nullptr;
  int64_t resident_bytes = 0;
};

// ---------------------------------------------------------------------------
// internal entry points between translation units

// factor.hip
struct FactorJob {
  double sigma_new;
  double sigma_prev;  // ignored for SPAI
  int32_t is_spai;
  void* vals;
  void* valsT;
};
morx_status factor_alloc(morx_system sys, int32_t prec, morx_factor* out);
// whether the least-squares kernel variant (0, 8 or 16 row groups) handles the pattern
bool factor_kernel_supported(morx_system sys, int rows);
void factor_release(morx_factor f);  // back to the system's pool
void factor_discard(morx_factor f);  // device memory freed (no work may still use it)
morx_status factor_build_many(morx_system sys, int32_t prec, const FactorJob* jobs, int njobs,
                              hipStream_t st);

// bicg.hip: the solve's chain and shifted-pair kernels on caller columns
morx_status hot_chain_apply(morx_system sys, int ncol, int lcap, const morx_factor* chains,
                            const int32_t* lens, const double* X, int64_t ldx, double* Y,
                            int64_t ldy, const double* Xt, int64_t ldxt, double* Yt, int64_t ldyt,
                            int aprec, hipStream_t st);
morx_status hot_shifted_pair(morx_system sys, int ncol, const double* sigmas, const double* X,
                             int64_t ldx, double* Y, int64_t ldy, const double* Xt, int64_t ldxt,
                             double* Yt, int64_t ldyt, hipStream_t st);

// spmm.hip (single-column helpers of the GMRES comparator and the projection)
morx_status launch_shifted_apply(morx_system sys, double sigma, bool trans, int ncol,
                                 const double* X, int64_t ldx, double* Y, int64_t ldy,
                                 hipStream_t st);
morx_status launch_factor_apply(morx_system sys, morx_factor f, bool trans, int ncol,
                                const double* X, int64_t ldx, double* Y, int64_t ldy,
                                hipStream_t st);

// project.hip
morx_status project_scratch_init(morx_ctx ctx);

// bicg.hip
void krylov_batch_delete(KrylovBatch* kb);
void trace_factor_begin(morx_ctx ctx, hipStream_t st, void** token);
void trace_factor_end(morx_ctx ctx, hipStream_t st, void* token);

// streams: make `inner` wait for `outer` and back
morx_status stream_enter(morx_ctx ctx, hipStream_t outer);
morx_status stream_leave(morx_ctx ctx, hipStream_t outer);

// ---------------------------------------------------------------------------
// device helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return __shfl(v, 0, 64);  // every lane takes lane 0's association order
}

template <typename T>
__device__ __forceinline__ double load_val(const T* p);
template <>
__device__ __forceinline__ double load_val<double>(const double* p) { return *p; }
template <>
__device__ __forceinline__ double load_val<float>(const float* p) { return (double)*p; }
template <>
__device__ __forceinline__ double load_val<uint16_t>(const uint16_t* p) {
  uint32_t b = ((uint32_t)*p) << 16;
  return (double)__uint_as_float(b);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (uint16_t)((b >> 16) | 0x40u);
  uint32_t lsb = (b >> 16) & 1u;
  b += 0x7fffu + lsb;
  return (uint16_t)(b >> 16);
}

template <typename T>
__device__ __forceinline__ void store_val(T* p, double v);
template <>
__device__ __forceinline__ void store_val<double>(double* p, double v) { *p = v; }
template <>
__device__ __forceinline__ void store_val<float>(float* p, double v) { *p = (float)v; }
template <>
__device__ __forceinline__ void store_val<uint16_t>(uint16_t* p, double v) {
  *p = f32_to_bf16_rne((float)v);
}

// Loads and stores through the global address space.  Pointers that come out
// of device memory (factor tables, slot descriptors) or out of selects are
// generic to the compiler, which then emits flat instructions that also count
// against the LDS wait counter; these casts keep them global.
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
template <typename T>
__device__ __forceinline__ double gload_val(const T* p);
template <>
__device__ __forceinline__ double gload_val<double>(const double* p) { return gld(p); }
template <>
__device__ __forceinline__ double gload_val<float>(const float* p) { return (double)gld(p); }
template <>
__device__ __forceinline__ double gload_val<uint16_t>(const uint16_t* p) {
  return (double)__uint_as_float(((uint32_t)gld(p)) << 16);
}

// Buffer loads: a wave-uniform base and byte size in a resource descriptor
// and a 32-bit per-lane byte offset (plus a wave-uniform one), so a load
// needs one address register instead of two; the hardware checks the offset
// against the size and reads past it return 0.  Every array read this way is
// below 4 GiB (checked when a system is created).
using BufRes = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ BufRes buf_res(const void* p, int64_t bytes) {
  const uint32_t n = bytes >= 0xffffffffLL ? 0xffffffffu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, 0x00020000);
}
__device__ __forceinline__ int32_t buf_i32(BufRes r, uint32_t off, uint32_t soff = 0) {
  return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, 0);
}
template <typename T>
__device__ __forceinline__ double buf_val(BufRes r, uint32_t off, uint32_t soff = 0);
template <>
__device__ __forceinline__ double buf_val<double>(BufRes r, uint32_t off, uint32_t soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0);
  return __hiloint2double((int)v[1], (int)v[0]);
}
template <>
__device__ __forceinline__ double buf_val<float>(BufRes r, uint32_t off, uint32_t soff) {
  return (double)__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, 0));
}
template <>
__device__ __forceinline__ double buf_val<uint16_t>(BufRes r, uint32_t off, uint32_t soff) {
  const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, (int)soff, 0);
  return (double)__uint_as_float(h << 16);
}

inline size_t prec_bytes(int32_t prec) { return prec == MORX_F64 ? 8 : (prec == MORX_F32 ? 4 : 2); }

// One row of a sliced-ELL product for up to NC columns: acc[j] += sum_m v_m * x_j[col_m].
// Lanes of a slice read consecutive addresses for each slot m (coalesced).
template <typename VT, int NC>
__device__ __forceinline__ void sell_row(const int32_t* __restrict__ off,
                                         const int32_t* __restrict__ col,
                                         const VT* __restrict__ val, int64_t row,
                                         const double* const (&x)[NC], unsigned mask,
                                         double (&acc)[NC]) {
  const int64_t s = row >> 6;
  const int32_t o1 = off[s + 1];
  for (int32_t p = off[s] + (int32_t)(row & 63); p < o1; p += kSlice) {
    const int32_t c = col[p];
    const double v = load_val<VT>(val + p);
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (mask & (1u << j)) acc[j] = fma(v, x[j][c], acc[j]);
  }
}
