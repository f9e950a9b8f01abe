// Device construction of the walk operator P = (I - B) P_N + B P_K (Eq. p-mat-ancka) without
// forming P: the KNN graph A_K = W + W^T of Eq. (AK), the topology CSRs of Eqs. (rw-hg),
// (rw-ag), (rw-mg), beta_i of Eq. (beta_i) and the per-row scales that the SpMM kernels apply.
// Every CSR is produced by a stable radix sort of (row, column) keys, so the column order of
// each row -- and with it every later floating-point sum -- is deterministic.
#include <cmath>

#include "common.h"

namespace {

constexpr uint64_t SENTINEL = ~0ull;

__host__ __device__ inline int bits_for(int64_t v) {  // smallest b with 2^b > v
  int b = 0;
  while (b < 63 && (int64_t(1) << b) <= v) b++;
  return b;
}

template <typename TS>
__global__ void emit_knn_kernel(const int32_t* __restrict__ nbr_idx, const TS* __restrict__ nbr_sim, int64_t n, int K,
                                int cb, uint64_t* __restrict__ keys, uint64_t* __restrict__ vals,
                                int* __restrict__ bad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n * K) return;
  const int64_t i = p / K;
  const int32_t j = nbr_idx[p];
  const TS s = nbr_sim[p];
  uint64_t k1 = SENTINEL, k2 = SENTINEL, v = 0;
  if (j < -1 || j >= n) atomicOr(bad, 1);
  if (j >= 0 && j < n && j != i && s > (TS)0) {
    k1 = ((uint64_t)i << cb) | (uint64_t)j;
    k2 = ((uint64_t)j << cb) | (uint64_t)i;
    if (sizeof(TS) == 8) v = (uint64_t)__double_as_longlong((double)s);
    else v = (uint64_t)__float_as_uint((float)s);
  }
  keys[2 * p] = k1;
  keys[2 * p + 1] = k2;
  vals[2 * p] = v;
  vals[2 * p + 1] = v;
}

// graph / multiplex layer l: both directions of every edge, segment key (i*L + l, j)
__global__ void emit_graph_kernel(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t n, int L,
                                  int l, int cb, uint64_t* __restrict__ keys, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = ptr[i], e = ptr[i + 1];
  for (int64_t p = b; p < e; p++) {
    const int32_t j = idx[p];
    uint64_t k1 = SENTINEL, k2 = SENTINEL;
    if (j < 0 || j >= n) {
      atomicOr(bad, 1);
    } else if (j != i) {
      k1 = ((uint64_t)(i * L + l) << cb) | (uint64_t)j;
      k2 = ((uint64_t)((int64_t)j * L + l) << cb) | (uint64_t)i;
    }
    keys[2 * p] = k1;
    keys[2 * p + 1] = k2;
  }
}

// hypergraph: (e, v) keys for hyperedge rows and (v, e) keys for node rows
__global__ void emit_hyper_kernel(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t n,
                                  int64_t m, int cbn, int cbm, uint64_t* __restrict__ ekeys,
                                  uint64_t* __restrict__ vkeys, int* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int64_t b = ptr[e], f = ptr[e + 1];
  if (f <= b) atomicOr(bad, 2);
  for (int64_t p = b; p < f; p++) {
    const int32_t v = idx[p];
    if (v < 0 || v >= n) {
      atomicOr(bad, 1);
      ekeys[p] = SENTINEL;
      vkeys[p] = SENTINEL;
    } else {
      ekeys[p] = ((uint64_t)e << cbn) | (uint64_t)v;
      vkeys[p] = ((uint64_t)v << cbm) | (uint64_t)e;
    }
  }
}

// CSR sanity: ptr[0] = 0, non-decreasing, ptr[rows] = nnz, every index in [0, ncols).
// Runs (and is checked on the host) before any kernel follows the caller's pointers.
__global__ void validate_csr_kernel(const int64_t* __restrict__ ptr, int64_t rows, int64_t nnz,
                                    const int32_t* __restrict__ idx, int64_t ncols, int* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < rows) {
    const int64_t a = ptr[t], b = ptr[t + 1];
    if (a > b || b > nnz || a < 0) atomicOr(bad, 4);
    if (t == 0 && a != 0) atomicOr(bad, 4);
    if (t == rows - 1 && b != nnz) atomicOr(bad, 4);
  }
  if (t < nnz) {
    const int32_t j = idx[t];
    if (j < 0 || j >= ncols) atomicOr(bad, 1);
  }
}

__global__ void key_cols_kernel(const uint64_t* __restrict__ keys, int64_t count, int cb, int32_t* __restrict__ col) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < count) col[p] = (int32_t)(keys[p] & ((1ull << cb) - 1));
}

// D_K[i] = sum of row i of A_K, in column order
__global__ void knn_rowsum_kernel(const int64_t* __restrict__ kptr, const double* __restrict__ kv, int64_t n,
                                  double* __restrict__ dk) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t p = kptr[i]; p < kptr[i + 1]; p++) s += kv[p];
  dk[i] = s;
}

// per node: delta, beta, self loop, topology scales
template <typename T>
__global__ void node_scales_kernel(int kind, int64_t n, int L, const int64_t* __restrict__ tptr,
                                   const double* __restrict__ dk, double beta_param, double* __restrict__ beta,
                                   int64_t* __restrict__ delta, T* __restrict__ self, T* __restrict__ tscale,
                                   T* __restrict__ tcol) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t del = 0;
  int active = 0;
  const int segs = (kind == ANCKA_HYPERGRAPH) ? 1 : L;
  for (int l = 0; l < segs; l++) {
    const int64_t dl = tptr[i * segs + l + 1] - tptr[i * segs + l];
    del += dl;
    active += dl > 0;
  }
  const double b = (dk[i] == 0.0) ? 0.0 : (del == 0 ? 1.0 : beta_param);
  beta[i] = b;
  delta[i] = del;
  self[i] = (b == 0.0 && del == 0) ? (T)1 : (T)0;
  for (int l = 0; l < segs; l++) {
    const int64_t dl = tptr[i * segs + l + 1] - tptr[i * segs + l];
    // graph / multiplex: average over the layers where i has edges; hypergraph: 1/delta(v)
    const double w = dl > 0 ? 1.0 / ((double)active * (double)dl) : 0.0;
    tscale[i * segs + l] = (T)((1.0 - b) * w);
    tcol[i * segs + l] = (T)w;
  }
}

template <typename T>
__global__ void edge_scales_kernel(const int64_t* __restrict__ eptr, int64_t m, T* __restrict__ escale) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) escale[e] = (T)(1.0 / (double)(eptr[e + 1] - eptr[e]));
}

template <typename T>
__global__ void knn_values_kernel(const int64_t* __restrict__ kptr, const double* __restrict__ kv,
                                  const double* __restrict__ dk, const double* __restrict__ beta, int64_t n,
                                  T* __restrict__ kval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = dk[i] > 0.0 ? beta[i] / dk[i] : 0.0;
  for (int64_t p = kptr[i]; p < kptr[i + 1]; p++) kval[p] = (T)(kv[p] * sc);
}

__global__ void last_key_kernel(const uint64_t* __restrict__ keys, int64_t count, uint64_t* __restrict__ out) {
  out[0] = count > 0 ? keys[count - 1] : 0ull;
}

unsigned nb256(int64_t c) { return (unsigned)cdiv(c > 0 ? c : 1, 256); }

// sort keys (+ values), merge duplicates, drop a trailing SENTINEL run.  Returns the unique
// count; keys_out / vals_out receive the merged arrays.
ancka_status sort_unique(ancka_ctx* ctx, uint64_t* keys, uint64_t* vals, int vals_double, int64_t count, int bits,
                         uint64_t* keys_out, double* vals_out, int64_t* out_count) {
  // SENTINEL sorts last because its low `bits` bits are all ones and every valid key is smaller
  ST_TRY(radix_sort_u64(ctx, keys, vals, count, bits));
  int64_t u = 0;
  ST_TRY(unique_sorted(ctx, keys, vals, vals_double, count, keys_out, vals_out, &u));
  if (u > 0) {
    uint64_t* lk = nullptr;
    ST_TRY(ws_get_t(ctx, "op_lastkey", 1, &lk));
    last_key_kernel<<<1, 1, 0, ctx->stream>>>(keys_out, u, lk);
    LAUNCH_CHECK(ctx);
    uint64_t h = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&h, lk, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    if ((h & mask) == mask) u--;
  }
  *out_count = u;
  return ANCKA_OK;
}

template <typename T>
ancka_status build_typed(ancka_ctx* ctx, const ancka_network* net, const int32_t* nbr_idx, const void* nbr_sim,
                         int sim_dtype, int K, double beta, ancka_op* op) {
  const int64_t n = net->n;
  const int cb = bits_for(n);
  int* bad = nullptr;
  ST_TRY(ws_get_t(ctx, "op_bad", 4, &bad));
  ST_TRY(fill_zero(ctx, bad, 16));
  {
    // validate the caller's topology before any kernel follows its pointers
    const int layers = net->kind == ANCKA_HYPERGRAPH ? 1 : net->L;
    for (int l = 0; l < layers; l++) {
      const int64_t rows = net->kind == ANCKA_HYPERGRAPH ? net->m : n;
      const int64_t nnz = net->nnz[l];
      validate_csr_kernel<<<nb256(rows > nnz ? rows : nnz), 256, 0, ctx->stream>>>(net->ptr[l], rows, nnz, net->idx[l], n,
                                                                                   bad);
      LAUNCH_CHECK(ctx);
    }
    int hb = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (hb & 4) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: inconsistent CSR row pointers");
    if (hb & 1) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: node index out of range");
  }

  // ---- A_K = W + W^T
  {
    const int64_t cnt = 2 * n * K;
    uint64_t *keys = nullptr, *vals = nullptr, *ukeys = nullptr;
    double* uvals = nullptr;
    ST_TRY(ws_get_t(ctx, "op_keys", (size_t)cnt, &keys));
    ST_TRY(ws_get_t(ctx, "op_vals", (size_t)cnt, &vals));
    ST_TRY(ws_get_t(ctx, "op_ukeys", (size_t)cnt, &ukeys));
    ST_TRY(ws_get_t(ctx, "op_uvals", (size_t)cnt, &uvals));
    if (sim_dtype == ANCKA_F64)
      emit_knn_kernel<double><<<nb256(n * K), 256, 0, ctx->stream>>>(nbr_idx, (const double*)nbr_sim, n, K, cb, keys,
                                                                       vals, bad);
    else
      emit_knn_kernel<float><<<nb256(n * K), 256, 0, ctx->stream>>>(nbr_idx, (const float*)nbr_sim, n, K, cb, keys,
                                                                      vals, bad);
    LAUNCH_CHECK(ctx);
    int64_t u = 0;
    ST_TRY(sort_unique(ctx, keys, vals, sim_dtype == ANCKA_F64, cnt, 2 * cb, ukeys, uvals, &u));
    op->nnz_knn = u;
    void* p;
    ST_TRY(op_alloc(ctx, op, sizeof(int64_t) * (n + 1), &p));
    op->kptr = (int64_t*)p;
    ST_TRY(op_alloc(ctx, op, sizeof(int32_t) * (u + 1), &p));
    op->kidx = (int32_t*)p;
    ST_TRY(op_alloc(ctx, op, sizeof(T) * (u + 1), &p));
    op->kval = p;
    ST_TRY(op_alloc(ctx, op, sizeof(double) * n, &p));
    op->dk = (double*)p;
    ST_TRY(csr_ptr_from_sorted(ctx, ukeys, u, cb, n, op->kptr));
    key_cols_kernel<<<nb256(u), 256, 0, ctx->stream>>>(ukeys, u, cb, op->kidx);
    LAUNCH_CHECK(ctx);
    knn_rowsum_kernel<<<nb256(n), 256, 0, ctx->stream>>>(op->kptr, uvals, n, op->dk);
    LAUNCH_CHECK(ctx);
    // keep A_K values until the betas are known
    double* akv = nullptr;
    ST_TRY(ws_get_t(ctx, "op_akv", (size_t)(u + 1), &akv));
    HIP_TRY(ctx, hipMemcpyAsync(akv, uvals, sizeof(double) * u, hipMemcpyDeviceToDevice, ctx->stream));
  }

  // ---- topology
  void* p;
  if (net->kind == ANCKA_HYPERGRAPH) {
    const int64_t m = net->m;
    const int64_t nnz = net->nnz[0];
    const int cbm = bits_for(m);
    uint64_t *ek = nullptr, *vk = nullptr, *uk = nullptr;
    ST_TRY(ws_get_t(ctx, "op_keys", (size_t)nnz, &ek));
    ST_TRY(ws_get_t(ctx, "op_vals", (size_t)nnz, &vk));
    ST_TRY(ws_get_t(ctx, "op_ukeys", (size_t)nnz, &uk));
    emit_hyper_kernel<<<nb256(m), 256, 0, ctx->stream>>>(net->ptr[0], net->idx[0], n, m, cb, cbm, ek, vk, bad);
    LAUNCH_CHECK(ctx);
    // hyperedge -> members
    int64_t ue = 0;
    ST_TRY(sort_unique(ctx, ek, nullptr, 0, nnz, cbm + cb, uk, nullptr, &ue));
    op->nnz_edge = ue;
    ST_TRY(op_alloc(ctx, op, sizeof(int64_t) * (m + 1), &p));
    op->eptr = (int64_t*)p;
    ST_TRY(op_alloc(ctx, op, sizeof(int32_t) * (ue + 1), &p));
    op->eidx = (int32_t*)p;
    ST_TRY(csr_ptr_from_sorted(ctx, uk, ue, cb, m, op->eptr));
    key_cols_kernel<<<nb256(ue), 256, 0, ctx->stream>>>(uk, ue, cb, op->eidx);
    LAUNCH_CHECK(ctx);
    // node -> incident hyperedges
    int64_t uv = 0;
    ST_TRY(sort_unique(ctx, vk, nullptr, 0, nnz, cb + cbm, uk, nullptr, &uv));
    op->nnz_topo = uv;
    ST_TRY(op_alloc(ctx, op, sizeof(int64_t) * (n + 1), &p));
    op->tptr = (int64_t*)p;
    ST_TRY(op_alloc(ctx, op, sizeof(int32_t) * (uv + 1), &p));
    op->tidx = (int32_t*)p;
    ST_TRY(csr_ptr_from_sorted(ctx, uk, uv, cbm, n, op->tptr));
    key_cols_kernel<<<nb256(uv), 256, 0, ctx->stream>>>(uk, uv, cbm, op->tidx);
    LAUNCH_CHECK(ctx);
    ST_TRY(op_alloc(ctx, op, sizeof(T) * (m + 1), &p));
    op->escale = p;
    edge_scales_kernel<T><<<nb256(m), 256, 0, ctx->stream>>>(op->eptr, m, (T*)op->escale);
    LAUNCH_CHECK(ctx);
  } else {
    const int L = net->L;
    int64_t tot = 0;
    for (int l = 0; l < L; l++) tot += net->nnz[l];
    uint64_t *keys = nullptr, *uk = nullptr;
    ST_TRY(ws_get_t(ctx, "op_keys", (size_t)(2 * tot + 1), &keys));
    ST_TRY(ws_get_t(ctx, "op_ukeys", (size_t)(2 * tot + 1), &uk));
    int64_t off = 0;
    for (int l = 0; l < L; l++) {
      // offset the per-row emission by the layer's start in the concatenated key array
      emit_graph_kernel<<<nb256(n), 256, 0, ctx->stream>>>(net->ptr[l], net->idx[l], n, L, l, cb, keys + 2 * off, bad);
      LAUNCH_CHECK(ctx);
      off += net->nnz[l];
    }
    const int sb = bits_for(n * L);
    int64_t u = 0;
    ST_TRY(sort_unique(ctx, keys, nullptr, 0, 2 * tot, sb + cb, uk, nullptr, &u));
    op->nnz_topo = u;
    ST_TRY(op_alloc(ctx, op, sizeof(int64_t) * (n * L + 1), &p));
    op->tptr = (int64_t*)p;
    ST_TRY(op_alloc(ctx, op, sizeof(int32_t) * (u + 1), &p));
    op->tidx = (int32_t*)p;
    ST_TRY(csr_ptr_from_sorted(ctx, uk, u, cb, n * L, op->tptr));
    key_cols_kernel<<<nb256(u), 256, 0, ctx->stream>>>(uk, u, cb, op->tidx);
    LAUNCH_CHECK(ctx);
  }

  // ---- per-node data
  const int segs = net->kind == ANCKA_HYPERGRAPH ? 1 : net->L;
  ST_TRY(op_alloc(ctx, op, sizeof(double) * n, &p));
  op->beta = (double*)p;
  ST_TRY(op_alloc(ctx, op, sizeof(int64_t) * n, &p));
  op->delta = (int64_t*)p;
  ST_TRY(op_alloc(ctx, op, sizeof(T) * n, &p));
  op->self = p;
  ST_TRY(op_alloc(ctx, op, sizeof(T) * n * segs, &p));
  op->tscale = p;
  ST_TRY(op_alloc(ctx, op, sizeof(T) * n * segs, &p));
  op->tcol = p;
  node_scales_kernel<T><<<nb256(n), 256, 0, ctx->stream>>>(net->kind, n, net->L, op->tptr, op->dk, beta, op->beta,
                                                           op->delta, (T*)op->self, (T*)op->tscale, (T*)op->tcol);
  LAUNCH_CHECK(ctx);
  double* akv = nullptr;
  ST_TRY(ws_get_t(ctx, "op_akv", (size_t)(op->nnz_knn + 1), &akv));
  knn_values_kernel<T><<<nb256(n), 256, 0, ctx->stream>>>(op->kptr, akv, op->dk, op->beta, n, (T*)op->kval);
  LAUNCH_CHECK(ctx);

  // processing order of node rows for the sparse products: rows of one coarse attribute cell
  // are handled together, so the rows they gather (mostly in the same cell) stay in cache
  if (net->X && net->d >= 1 && net->ldx >= net->d) {
    ST_TRY(op_alloc(ctx, op, sizeof(int32_t) * n, &p));
    op->rorder = (int32_t*)p;
    ST_TRY(cell_order(ctx, net->X, net->xdtype, n, net->d, net->ldx, op->rorder));
  }

  int hbad = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (hbad & 1) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: node index out of range");
  if (hbad & 2) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: empty hyperedge");
  return ANCKA_OK;
}

}  // namespace

extern "C" {

ancka_status ancka_build_operator(ancka_ctx* ctx, const ancka_network* net, const int32_t* nbr_idx,
                                  const void* nbr_sim, int32_t sim_dtype, int32_t K, double beta, int32_t op_dtype,
                                  ancka_op** out) {
  if (!ctx) return ANCKA_ERR_INVALID_ARG;
  if (!net || !out || !nbr_idx || !nbr_sim || net->n < 2 || net->n > INT32_MAX - 1 || K < 1 || beta < 0.0 ||
      beta > 1.0 || (sim_dtype != ANCKA_F64 && sim_dtype != ANCKA_F32) ||
      (op_dtype != ANCKA_F64 && op_dtype != ANCKA_F32))
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: invalid arguments");
  if (net->kind == ANCKA_HYPERGRAPH) {
    if (net->L != 1 || net->m < 1 || net->m > INT32_MAX - 1 || !net->ptr[0] || !net->idx[0] || net->nnz[0] < 1)
      return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: hypergraph needs L=1, m>=1 and its incidence");
  } else if (net->kind == ANCKA_GRAPH || net->kind == ANCKA_MULTIPLEX) {
    if (net->L < 1 || net->L > ANCKA_MAX_LAYERS || (net->kind == ANCKA_GRAPH && net->L != 1))
      return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: invalid layer count %d", net->L);
    for (int l = 0; l < net->L; l++)
      if (!net->ptr[l] || (net->nnz[l] > 0 && !net->idx[l]) || net->nnz[l] < 0)
        return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: layer %d CSR missing", l);
  } else {
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_build_operator: unknown kind %d", net->kind);
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  *out = nullptr;
  ancka_op* op = new ancka_op();
  op->kind = net->kind;
  op->dtype = op_dtype;
  op->n = net->n;
  op->m = net->kind == ANCKA_HYPERGRAPH ? net->m : 0;
  op->L = net->kind == ANCKA_HYPERGRAPH ? 1 : net->L;
  ancka_status st = op_dtype == ANCKA_F64 ? build_typed<double>(ctx, net, nbr_idx, nbr_sim, sim_dtype, K, beta, op)
                                          : build_typed<float>(ctx, net, nbr_idx, nbr_sim, sim_dtype, K, beta, op);
  if (st != ANCKA_OK) {
    ancka_op_destroy(op);
    return st;
  }
  *out = op;
  return ANCKA_OK;
}

void ancka_op_destroy(ancka_op* op) {
  if (!op) return;
  for (void* p : op->owned) (void)hipFree(p);
  delete op;
}

ancka_status ancka_op_info(ancka_ctx* ctx, const ancka_op* op, double* beta, int64_t* delta, double* dk,
                           int64_t* nnz_knn, int64_t* nnz_topo) {
  if (!ctx || !op) return ANCKA_ERR_INVALID_ARG;
  const int64_t n = op->n;
  if (beta) HIP_TRY(ctx, hipMemcpyAsync(beta, op->beta, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  if (delta) HIP_TRY(ctx, hipMemcpyAsync(delta, op->delta, sizeof(int64_t) * n, hipMemcpyDeviceToHost, ctx->stream));
  if (dk) HIP_TRY(ctx, hipMemcpyAsync(dk, op->dk, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (nnz_knn) *nnz_knn = op->nnz_knn;
  if (nnz_topo) *nnz_topo = op->nnz_topo;
  return ANCKA_OK;
}

}  // extern "C"
