// Internal declarations shared by the HIP sources of libancka (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/ancka.h"

#define ANCKA_WAVE 64

// ------------------------------------------------------------------------------------------
// context and operator

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct ancka_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  std::string err;
  std::map<std::string, DevBuf> ws;   // grow-only named workspaces
  hipEvent_t ev[8] = {};               // timing events, created on first use
  bool ev_ready = false;
  hipStream_t side = nullptr;          // second stream of the clustering loop (default priority)
  hipEvent_t side_ev = nullptr;        // orders it after the main stream
};

// the context's timing events (created once)
ancka_status ctx_events(ancka_ctx* ctx, hipEvent_t** out);
// the context's second stream and its ordering event (created once)
ancka_status ctx_side_stream(ancka_ctx* ctx, hipStream_t* s, hipEvent_t* e);

struct ancka_op {
  int kind = 0;
  int dtype = ANCKA_F32;              // ANCKA_F32 / ANCKA_F64 (values and blocks)
  int64_t n = 0, m = 0;
  int L = 1;
  // topology rows.  graph / multiplex: n*L segments (row i, layer l) = segment i*L + l.
  // hypergraph: node -> incident hyperedges (n segments).
  int64_t* tptr = nullptr;
  int32_t* tidx = nullptr;
  void* tscale = nullptr;             // per segment: (1-beta_i)/(L_i deg_l(i)); hypergraph (1-beta_u)/delta(u)
  void* tcol = nullptr;               // transposed walk scales: graph/multiplex per (j,l) 1/(L_j deg_l(j)); hypergraph 1/delta(v)
  // hypergraph hyperedge -> members
  int64_t* eptr = nullptr;
  int32_t* eidx = nullptr;
  void* escale = nullptr;             // 1/|e|
  // KNN part: values beta_i A_K[i,j] / D_K[i]
  int64_t* kptr = nullptr;
  int32_t* kidx = nullptr;
  void* kval = nullptr;
  void* self = nullptr;               // per row: 1 where P[i,i] = 1 is added, else 0
  double* beta = nullptr;
  int64_t* delta = nullptr;
  double* dk = nullptr;
  int32_t* rorder = nullptr;          // node rows in processing order (coarse attribute cells), nullable
  int64_t nnz_knn = 0, nnz_topo = 0, nnz_edge = 0;
  std::vector<void*> owned;
};

// ------------------------------------------------------------------------------------------
// error handling

ancka_status set_err(ancka_ctx* ctx, ancka_status st, const char* fmt, ...);

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return set_err((ctx), _e == hipErrorOutOfMemory ? ANCKA_ERR_OOM : ANCKA_ERR_HIP,        \
                     "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
  } while (0)

#define ST_TRY(expr)                       \
  do {                                     \
    ancka_status _s = (expr);              \
    if (_s != ANCKA_OK) return _s;         \
  } while (0)

#define LAUNCH_CHECK(ctx) HIP_TRY(ctx, hipGetLastError())

// named, grow-only device workspace (contents undefined on return)
ancka_status ws_get(ancka_ctx* ctx, const char* name, size_t bytes, void** out);
template <typename T>
inline ancka_status ws_get_t(ancka_ctx* ctx, const char* name, size_t count, T** out) {
  void* p = nullptr;
  ancka_status s = ws_get(ctx, name, count * sizeof(T), &p);
  *out = (T*)p;
  return s;
}
// Looks up, once per device, the address of the Discretize state that
// ancka_discretize_noalloc uses on the context's device (discretize.hip).
ancka_status disc_scratch_setup(ancka_ctx* ctx);
// allocation owned by an operator
ancka_status op_alloc(ancka_ctx* ctx, ancka_op* op, size_t bytes, void** out);

// ------------------------------------------------------------------------------------------
// primitives (prim.hip)

// out[0..count] = exclusive prefix sum of in[0..count-1]; out[count] = total.
ancka_status scan_excl_i64(ancka_ctx* ctx, const int64_t* in, int64_t* out, int64_t count);
// Stable LSD radix sort of (keys, vals) by the low `bits` bits of the keys; vals nullable.
ancka_status radix_sort_u64(ancka_ctx* ctx, uint64_t* keys, uint64_t* vals, int64_t count, int bits);
// Merge runs of equal keys of a sorted array: unique keys, values summed in run order as
// double (vals/out_vals nullable).  *out_count is written on the host (synchronises).
ancka_status unique_sorted(ancka_ctx* ctx, const uint64_t* keys, const uint64_t* vals, int vals_are_double,
                           int64_t count, uint64_t* out_keys, double* out_vals, int64_t* out_count);
// row_ptr[r] = first position p with (keys[p] >> col_bits) >= r, for r in 0..rows.
ancka_status csr_ptr_from_sorted(ancka_ctx* ctx, const uint64_t* keys, int64_t count, int col_bits,
                                 int64_t rows, int64_t* row_ptr);
ancka_status fill_zero(ancka_ctx* ctx, void* p, size_t bytes);

// Rows of X (n x d, xdtype) ordered by coarse cell (most similar of 64 evenly spaced pivot
// rows), then by norm: order[p] = row at position p (knn.hip).
ancka_status cell_order(ancka_ctx* ctx, const void* X, int xdtype, int64_t n, int64_t d, int64_t ldx, int32_t* order);

// ------------------------------------------------------------------------------------------
// sparse products (spmm.hip)

// Z = P Q for an n x cols block (op->dtype); internal entry used by every phase.
ancka_status op_apply(ancka_ctx* ctx, const ancka_op* op, const void* Q, void* Z, int cols, int64_t ld);
// Z = (1-alpha) P Q + alpha * Yh(labels) (MHC recursion step; Yh from labels and counts).
ancka_status op_apply_mhc(ancka_ctx* ctx, const ancka_op* op, const void* Q, void* Z, int cols, int64_t ld,
                          double alpha, const int32_t* labels, const int32_t* counts, const void* f0val = nullptr);
// Pi^T <- (1-alpha) P_N^T Pi^T + alpha Z0^T on the topology walk (InitBCM step).
ancka_status op_apply_init(ancka_ctx* ctx, const ancka_op* op, const void* Pin, void* Pout, int cols,
                           int64_t ld, double alpha, const int32_t* centres);
// U = (X^ + P_N X^)/2 over a float n x cols block with row scales (warm-start features).
ancka_status op_apply_features(ancka_ctx* ctx, const ancka_op* op, const float* Xh, float* U, int cols,
                               int64_t ld);

// ------------------------------------------------------------------------------------------
// QR (qr.hip)

// Orthonormalise an n x kp block in place (CholQR; second pass if needed or FP64).
// R_out: device kp*kp double (upper, row-major) or nullptr.  dq2: device double* accumulating
// ||Qnew - Qprev||_F^2 (Qprev nullable).
ancka_status qr_block(ancka_ctx* ctx, int dtype, const void* Z, void* Qout, int64_t n, int kp, int64_t ld,
                      const void* Qprev, double* dq2_dev, double* R_out);
// counts[c] = number of rows with label c (device); *bad |= 1 on a label outside [0, k)
ancka_status count_labels(ancka_ctx* ctx, const int32_t* labels, int64_t n, int k, int32_t* counts, int* bad);
// starting block of Alg. 4, starting block (see ancka_initial_block)
ancka_status initial_block(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels, const float* zwarm, int k,
                           void* Q, int64_t ldq);
// Discretize of Alg. 5 (see ancka_discretize); synchronises
ancka_status discretize_internal(ancka_ctx* ctx, const void* Q, int qdtype, int64_t n, int k, int64_t ldq,
                                 int max_iter, int32_t* labels, double* R, double* obj, int32_t* iters);

// ------------------------------------------------------------------------------------------
// small device helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__host__ __device__ static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

