// Context, streams, device memory and error reporting of libmorx.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "common.h"

static thread_local char g_err[512] = "";

void morx_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

morx_status dev_alloc(DevBuf& b, size_t bytes) {
  b.p = nullptr;
  b.bytes = 0;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    hipGetLastError();
    morx_set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return MORX_E_NOMEM;
  }
  b.bytes = bytes;
  return MORX_OK;
}

void dev_free(DevBuf& b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

morx_status stream_enter(morx_ctx ctx, hipStream_t outer) {
  MORX_HIP(hipEventRecord(ctx->ev_in, outer));
  MORX_HIP(hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0));
  MORX_HIP(hipStreamWaitEvent(ctx->stream2, ctx->ev_in, 0));
  return MORX_OK;
}

morx_status stream_leave(morx_ctx ctx, hipStream_t outer) {
  MORX_HIP(hipEventRecord(ctx->ev_out, ctx->stream));
  MORX_HIP(hipStreamWaitEvent(outer, ctx->ev_out, 0));
  MORX_HIP(hipEventRecord(ctx->ev_aux, ctx->stream2));
  MORX_HIP(hipStreamWaitEvent(outer, ctx->ev_aux, 0));
  return MORX_OK;
}

extern "C" void morx_opts_default(morx_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-10;
  o->maxit = 0;
  o->max_restarts = 3;
  o->precond_prec = MORX_F64;
  o->chain = MORX_CHAIN_RESET;
  o->want_dual = 1;
  o->batched = 1;
  o->poll_iters = 8;
  o->use_graph = 1;
}

extern "C" const char* morx_status_str(int32_t s) {
  switch (s) {
    case MORX_OK: return "ok";
    case MORX_E_INVALID: return "invalid argument";
    case MORX_E_NOMEM: return "out of memory";
    case MORX_E_HIP: return "HIP runtime error";
    case MORX_E_SINGULAR_LS: return "rank-deficient local least-squares problem";
    case MORX_E_NOT_CONVERGED: return "not converged";
    case MORX_E_BREAKDOWN: return "BiCG breakdown";
    case MORX_E_NONFINITE: return "non-finite input";
    case MORX_E_ADMISSION: return "request exceeds the memory budget";
    case MORX_E_UNSUPPORTED: return "unsupported pattern";
    case MORX_E_PENDING: return "pending";
    default: return "unknown status";
  }
}

extern "C" const char* morx_last_error(void) { return g_err; }

extern "C" morx_status morx_create(morx_ctx* out, int device) {
  MORX_REQUIRE(out, MORX_E_INVALID, "morx_create: null output");
  *out = nullptr;
  int count = 0;
  MORX_HIP(hipGetDeviceCount(&count));
  MORX_REQUIRE(device >= 0 && device < count, MORX_E_INVALID, "morx_create: device %d of %d",
               device, count);
  MORX_HIP(hipSetDevice(device));
  morx_ctx ctx = new morx_ctx_s();
  ctx->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cu = prop.multiProcessorCount;
  if (ctx->num_cu <= 0) ctx->num_cu = 256;
  hipError_t e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->stream2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_aux, hipEventDisableTiming);
  if (e != hipSuccess) {
    morx_set_error("morx_create: %s", hipGetErrorString(e));
    morx_destroy(ctx);
    return MORX_E_HIP;
  }
  const morx_status s = project_scratch_init(ctx);  // with the device current
  if (s != MORX_OK) {
    morx_destroy(ctx);
    return s;
  }
  *out = ctx;
  return MORX_OK;
}

extern "C" morx_status morx_destroy(morx_ctx ctx) {
  if (!ctx) return MORX_OK;
  hipSetDevice(ctx->device);
  if (ctx->stream) {
    hipStreamSynchronize(ctx->stream);
    hipStreamDestroy(ctx->stream);
  }
  if (ctx->stream2) {
    hipStreamSynchronize(ctx->stream2);
    hipStreamDestroy(ctx->stream2);
  }
  if (ctx->ev_in) hipEventDestroy(ctx->ev_in);
  if (ctx->ev_out) hipEventDestroy(ctx->ev_out);
  if (ctx->ev_aux) hipEventDestroy(ctx->ev_aux);
  delete ctx;
  return MORX_OK;
}
