// Learned warm start (MLP d -> h1 -> h2 -> k).  Placeholder entry points until the kernels land.
#include "common.h"

extern "C" {

ancka_status ancka_ws_create(ancka_ctx* ctx, int32_t, int32_t, int32_t, int32_t, uint64_t, ancka_ws** out) {
  if (out) *out = nullptr;
  return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "warm start not built");
}
void ancka_ws_destroy(ancka_ws*) {}
ancka_status ancka_ws_features(ancka_ctx* ctx, const ancka_op*, const void*, int32_t, int64_t, int64_t, float*) {
  return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "warm start not built");
}
ancka_status ancka_ws_forward(ancka_ctx* ctx, ancka_ws*, const float*, int64_t, float*, int32_t) {
  return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "warm start not built");
}
ancka_status ancka_ws_backward(ancka_ctx* ctx, ancka_ws*, const float*, const float*, int64_t, double*) {
  return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "warm start not built");
}
ancka_status ancka_ws_step(ancka_ctx* ctx, ancka_ws*, double) {
  return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "warm start not built");
}
ancka_status ancka_ws_get_params(ancka_ctx* ctx, ancka_ws*, int32_t, float*, int64_t*) {
  return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "warm start not built");
}
ancka_status ancka_ws_set_params(ancka_ctx* ctx, ancka_ws*, const float*) {
  return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "warm start not built");
}

}  // extern "C"
