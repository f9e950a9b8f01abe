// Context, error reporting, parameters and workspaces of libancka.
#include <cstdarg>
#include <cmath>

#include "common.h"

ancka_status set_err(ancka_ctx* ctx, ancka_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

ancka_status ws_get(ancka_ctx* ctx, const char* name, size_t bytes, void** out) {
  DevBuf& b = ctx->ws[name];
  if (bytes == 0) bytes = 256;
  if (b.bytes < bytes) {
    if (b.ptr) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      HIP_TRY(ctx, hipFree(b.ptr));
      b.ptr = nullptr;
      b.bytes = 0;
    }
    size_t want = bytes + bytes / 8;
    HIP_TRY(ctx, hipMalloc(&b.ptr, want));
    b.bytes = want;
  }
  *out = b.ptr;
  return ANCKA_OK;
}

ancka_status ctx_side_stream(ancka_ctx* ctx, hipStream_t* s, hipEvent_t* e) {
  if (!ctx->side) {
    HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    HIP_TRY(ctx, hipEventCreateWithFlags(&ctx->side_ev, hipEventDisableTiming));
  }
  *s = ctx->side;
  *e = ctx->side_ev;
  return ANCKA_OK;
}

ancka_status ctx_events(ancka_ctx* ctx, hipEvent_t** out) {
  if (!ctx->ev_ready) {
    for (auto& e : ctx->ev) HIP_TRY(ctx, hipEventCreate(&e));
    ctx->ev_ready = true;
  }
  *out = ctx->ev;
  return ANCKA_OK;
}

ancka_status op_alloc(ancka_ctx* ctx, ancka_op* op, size_t bytes, void** out) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  HIP_TRY(ctx, hipMalloc(&p, bytes));
  op->owned.push_back(p);
  *out = p;
  return ANCKA_OK;
}

extern "C" {

ancka_status ancka_create(ancka_ctx** out, int32_t device, void* hip_stream) {
  if (!out) return ANCKA_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return ANCKA_ERR_INVALID_ARG;
  ancka_ctx* c = new ancka_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return ANCKA_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return ANCKA_ERR_HIP;
  }
  if (prop.warpSize != ANCKA_WAVE) {
    delete c;
    return ANCKA_ERR_UNSUPPORTED;
  }
  c->num_cu = prop.multiProcessorCount;
  const ancka_status ss = disc_scratch_setup(c);
  if (ss != ANCKA_OK) {
    delete c;
    return ss;
  }
  *out = c;
  return ANCKA_OK;
}

void ancka_destroy(ancka_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
    (void)hipEventDestroy(ctx->side_ev);
  }
  for (auto& kv : ctx->ws)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  if (ctx->ev_ready)
    for (auto& e : ctx->ev) (void)hipEventDestroy(e);
  delete ctx;
}

const char* ancka_last_error(const ancka_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ancka_params ancka_default_params(void) {
  ancka_params p;
  p.k = 0;
  p.K = 10;
  p.alpha = 0.2;
  p.beta = 0.5;
  p.gamma = 3;
  p.tau = 5;
  p.T_i = 25;
  p.T_a = 1000;
  p.eps_q = 0.005;
  p.disc_max_iter = 30;
  p.knn_mode = ANCKA_KNN_EXACT_F32;
  p.q_dtype = ANCKA_F32;
  p.early_stop = 1;
  p.ivf_nlist = 1024;
  p.ivf_nprobe = 32;
  return p;
}

ancka_status ancka_device_info(ancka_ctx* ctx, int32_t* num_cu, int32_t* warp_size) {
  if (!ctx) return ANCKA_ERR_INVALID_ARG;
  if (num_cu) *num_cu = ctx->num_cu;
  if (warp_size) *warp_size = ANCKA_WAVE;
  return ANCKA_OK;
}

}  // extern "C"
