// Greedy initial BCM (Alg. 3 and the greedy start of Alg. 4), multi-hop conductance (Alg. 2 and its
// use in Alg. 4) and the whole method (Alg. 4) on gfx950.  The host only sequences kernels and reads a
// few scalars every tau iterations (phi, ||Q^(t) - Q^(t-1)||_F, the Discretize flag).
#include <chrono>
#include <cmath>
#include <limits>
#include <vector>

#include "common.h"

namespace {

constexpr int TOPK_T = 256;
constexpr int TOPK_CHUNK = 4096;

// key = (degree << 32) | (0xffffffff - index): the largest key is the largest degree with the
// smallest index, the centre order of Alg. 4, choice of the centres
__device__ __forceinline__ unsigned long long centre_key(int64_t deg, int64_t i) {
  return ((unsigned long long)deg << 32) | (unsigned long long)(0xffffffffu - (uint32_t)i);
}

__device__ unsigned long long block_max_u64(unsigned long long v, unsigned long long* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = TOPK_T / 2; s > 0; s >>= 1) {
    if (tid < s && red[tid + s] > red[tid]) red[tid] = red[tid + s];
    __syncthreads();
  }
  const unsigned long long r = red[0];
  __syncthreads();
  return r;
}

// each block: the k largest keys of its chunk (k rounds of a block maximum)
__global__ __launch_bounds__(TOPK_T) void topk_block_kernel(const int64_t* __restrict__ delta, int64_t n, int k,
                                                            unsigned long long* __restrict__ out) {
  __shared__ unsigned long long keys[TOPK_CHUNK];
  __shared__ unsigned long long red[TOPK_T];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * TOPK_CHUNK;
  for (int e = tid; e < TOPK_CHUNK; e += TOPK_T) {
    const int64_t i = base + e;
    keys[e] = (i < n) ? centre_key(delta[i], i) : 0ull;
  }
  __syncthreads();
  for (int r = 0; r < k; r++) {
    unsigned long long m = 0ull;
    for (int e = tid; e < TOPK_CHUNK; e += TOPK_T) m = keys[e] > m ? keys[e] : m;
    const unsigned long long best = block_max_u64(m, red);
    for (int e = tid; e < TOPK_CHUNK; e += TOPK_T)
      if (keys[e] == best) keys[e] = 0ull;
    if (tid == 0) out[(int64_t)blockIdx.x * k + r] = best;
    __syncthreads();
  }
}

// single block: the k largest of all block candidates, then centre indices sorted ascending
__global__ __launch_bounds__(TOPK_T) void topk_final_kernel(unsigned long long* __restrict__ cand, int64_t count, int k,
                                                            int64_t /*n*/, int32_t* __restrict__ centres,
                                                            int32_t* __restrict__ centre_of) {
  __shared__ unsigned long long red[TOPK_T];
  __shared__ int32_t sel[64];
  const int tid = threadIdx.x;
  for (int r = 0; r < k; r++) {
    unsigned long long m = 0ull;
    for (int64_t e = tid; e < count; e += TOPK_T) m = cand[e] > m ? cand[e] : m;
    const unsigned long long best = block_max_u64(m, red);
    for (int64_t e = tid; e < count; e += TOPK_T)
      if (cand[e] == best) cand[e] = 0ull;
    if (tid == 0) sel[r] = (int32_t)(0xffffffffu - (uint32_t)(best & 0xffffffffull));
    __syncthreads();
  }
  if (tid == 0) {
    for (int a = 1; a < k; a++) {
      const int32_t v = sel[a];
      int b = a - 1;
      while (b >= 0 && sel[b] > v) {
        sel[b + 1] = sel[b];
        b--;
      }
      sel[b + 1] = v;
    }
    for (int j = 0; j < k; j++) {
      centres[j] = sel[j];
      centre_of[sel[j]] = j;
    }
  }
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t count, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// Pi^T(0) = alpha Z0^T
template <typename T>
__global__ void init_pi_kernel(T* __restrict__ P, int64_t n, int64_t ld, const int32_t* __restrict__ centre_of, T alpha) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = centre_of[i];
  for (int64_t j = 0; j < ld; j++) P[i * ld + j] = (j == c) ? alpha : (T)0;
}

// label = first maximum over the k columns of a row (all-zero row -> 0)
template <typename T>
__global__ void row_argmax_kernel(const T* __restrict__ P, int64_t n, int k, int64_t ld, int32_t* __restrict__ labels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int b = 0;
  T bv = P[i * ld];
  for (int j = 1; j < k; j++) {
    const T v = P[i * ld + j];
    if (v > bv) {
      bv = v;
      b = j;
    }
  }
  labels[i] = b;
}

// the non-zero of each row of F(0) = alpha Yh: alpha / sqrt(|C_l|) (the expression of mhc_f0_kernel)
template <typename T>
__global__ void mhc_f0v_kernel(T* __restrict__ v, int64_t n, const int32_t* __restrict__ labels,
                               const int32_t* __restrict__ counts, T alpha) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  v[i] = alpha / sqrt((T)counts[labels[i]]);
}

// F(0) = alpha Yh
template <typename T>
__global__ void mhc_f0_kernel(T* __restrict__ F, int64_t n, int64_t ld, const int32_t* __restrict__ labels,
                              const int32_t* __restrict__ counts, T alpha) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int l = labels[i];
  const T v = alpha / sqrt((T)counts[l]);
  for (int64_t j = 0; j < ld; j++) F[i * ld + j] = (j == l) ? v : (T)0;
}

// per-block partial of trace(Yh^T F) = sum_i F[i, l_i] / sqrt(|C_{l_i}|)
template <typename T>
__global__ __launch_bounds__(256) void mhc_trace_kernel(const T* __restrict__ F, int64_t n, int64_t ld,
                                                        const int32_t* __restrict__ labels,
                                                        const int32_t* __restrict__ counts, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const int l = labels[i];
    v = (double)F[i * ld + l] / sqrt((double)counts[l]);
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void mhc_final_kernel(const double* __restrict__ part, int64_t count, int k, double* __restrict__ phi) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) phi[0] = 1.0 - red[0] / (double)k;
}

__global__ void copy_i32_kernel(const int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) b[i] = a[i];
}

__global__ void warm_argmax_kernel(const float* __restrict__ Z, int64_t n, int k, int32_t* __restrict__ labels) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int b = 0;
  float bv = Z[i * k];
  for (int j = 1; j < k; j++)
    if (Z[i * k + j] > bv) {
      bv = Z[i * k + j];
      b = j;
    }
  labels[i] = b;
}

unsigned nb256(int64_t c) { return (unsigned)cdiv(c > 0 ? c : 1, 256); }
// Leading dimension of the n x cols blocks the sparse products gather rows from: rows of at most
// 128 bytes are padded to a power of two of bytes (16..128) and longer rows to a multiple of 128
// bytes, so a row gather never straddles more cache lines than its size requires.
int64_t pad_ld(int cols, int dtype) {
  const int es = dtype == ANCKA_F64 ? 8 : 4;
  int64_t bytes = (int64_t)cols * es;
  if (bytes <= 128) {
    int64_t p2 = 16;
    while (p2 < bytes) p2 *= 2;
    bytes = p2;
  } else {
    bytes = (bytes + 127) / 128 * 128;
  }
  return bytes / es;
}

template <typename T>
ancka_status init_bcm_typed(ancka_ctx* ctx, const ancka_op* op, int k, double alpha, int T_i, int32_t* labels) {
  const int64_t n = op->n;
  const int64_t nblk = cdiv(n, TOPK_CHUNK);
  unsigned long long* cand = nullptr;
  int32_t *centres = nullptr, *centre_of = nullptr;
  ST_TRY(ws_get_t(ctx, "ib_cand", (size_t)nblk * k, &cand));
  ST_TRY(ws_get_t(ctx, "ib_centres", 64, &centres));
  ST_TRY(ws_get_t(ctx, "ib_centre_of", (size_t)n, &centre_of));
  topk_block_kernel<<<(unsigned)nblk, TOPK_T, 0, ctx->stream>>>(op->delta, n, k, cand);
  LAUNCH_CHECK(ctx);
  fill_i32_kernel<<<nb256(n), 256, 0, ctx->stream>>>(centre_of, n, -1);
  LAUNCH_CHECK(ctx);
  topk_final_kernel<<<1, TOPK_T, 0, ctx->stream>>>(cand, nblk * k, k, n, centres, centre_of);
  LAUNCH_CHECK(ctx);
  const int64_t ld = pad_ld(k, op->dtype);
  T *P0 = nullptr, *P1 = nullptr;
  ST_TRY(ws_get_t(ctx, "ib_P0", (size_t)n * ld, &P0));
  ST_TRY(ws_get_t(ctx, "ib_P1", (size_t)n * ld, &P1));
  // Pi(0) = alpha Z0 is one-hot: the first step reads it through centre_of
  if (T_i == 0) {
    init_pi_kernel<T><<<nb256(n), 256, 0, ctx->stream>>>(P0, n, ld, centre_of, (T)alpha);
    LAUNCH_CHECK(ctx);
  }
  for (int t = 0; t < T_i; t++) {
    ST_TRY(op_apply_init(ctx, op, t == 0 ? nullptr : P0, P1, k, ld, alpha, centre_of));
    std::swap(P0, P1);
  }
  row_argmax_kernel<T><<<nb256(n), 256, 0, ctx->stream>>>(P0, n, k, ld, labels);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

ancka_status init_bcm(ancka_ctx* ctx, const ancka_op* op, int k, double alpha, int T_i, int32_t* labels) {
  if (op->dtype == ANCKA_F64) return init_bcm_typed<double>(ctx, op, k, alpha, T_i, labels);
  return init_bcm_typed<float>(ctx, op, k, alpha, T_i, labels);
}

// phi into a device double (no synchronisation)
template <typename T>
ancka_status mhc_typed(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels, int k, double alpha, int gamma,
                       double* phi_dev, int* bad, bool validate) {
  const int64_t n = op->n;
  int32_t* counts = nullptr;
  ST_TRY(ws_get_t(ctx, "mhc_counts", 64, &counts));
  ST_TRY(count_labels(ctx, labels, n, k, counts, bad));
  if (validate) {
    // labels index the counts in every kernel below: check them first
    int hb = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (hb) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "mhc: label outside [0, k)");
  }
  const int64_t ld = pad_ld(k, op->dtype);
  T *F0 = nullptr, *F1 = nullptr;
  double* part = nullptr;
  ST_TRY(ws_get_t(ctx, "mhc_F0", (size_t)n * ld, &F0));
  ST_TRY(ws_get_t(ctx, "mhc_F1", (size_t)n * ld, &F1));
  ST_TRY(ws_get_t(ctx, "mhc_part", (size_t)cdiv(n, 256), &part));
  // F(0) = alpha Yh is one-hot: the first product reads it through the labels and the value
  // alpha / sqrt(|C_l|) of each row
  T* f0v = nullptr;
  ST_TRY(ws_get_t(ctx, "mhc_f0v", (size_t)n, &f0v));
  mhc_f0v_kernel<T><<<nb256(n), 256, 0, ctx->stream>>>(f0v, n, labels, counts, (T)alpha);
  LAUNCH_CHECK(ctx);
  if (gamma == 0) {
    mhc_f0_kernel<T><<<nb256(n), 256, 0, ctx->stream>>>(F0, n, ld, labels, counts, (T)alpha);
    LAUNCH_CHECK(ctx);
  }
  for (int l = 0; l < gamma; l++) {
    ST_TRY(op_apply_mhc(ctx, op, l == 0 ? nullptr : F0, F1, k, ld, alpha, labels, counts, f0v));
    std::swap(F0, F1);
  }
  mhc_trace_kernel<T><<<nb256(n), 256, 0, ctx->stream>>>(F0, n, ld, labels, counts, part);
  LAUNCH_CHECK(ctx);
  mhc_final_kernel<<<1, 256, 0, ctx->stream>>>(part, cdiv(n, 256), k, phi_dev);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

ancka_status mhc_dev(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels, int k, double alpha, int gamma,
                     double* phi_dev, int* bad, bool validate = true) {
  if (op->dtype == ANCKA_F64) return mhc_typed<double>(ctx, op, labels, k, alpha, gamma, phi_dev, bad, validate);
  return mhc_typed<float>(ctx, op, labels, k, alpha, gamma, phi_dev, bad, validate);
}

ancka_status mhc_host(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels, int k, double alpha, int gamma,
                      double* phi) {
  double* dphi = nullptr;
  int* bad = nullptr;
  ST_TRY(ws_get_t(ctx, "mhc_phi", 1, &dphi));
  ST_TRY(ws_get_t(ctx, "mhc_bad", 4, &bad));
  ST_TRY(fill_zero(ctx, bad, 16));
  ST_TRY(mhc_dev(ctx, op, labels, k, alpha, gamma, dphi, bad));
  int hbad = 0;
  HIP_TRY(ctx, hipMemcpyAsync(phi, dphi, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (hbad) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "mhc: label outside [0, k)");
  return ANCKA_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

ancka_status ancka_init_bcm(ancka_ctx* ctx, const ancka_op* op, int32_t k, double alpha, int32_t T_i, int32_t* labels) {
  if (!ctx || !op || !labels) return ANCKA_ERR_INVALID_ARG;
  if (k < 1 || k > 64 || k > op->n || alpha < 0.0 || alpha > 1.0 || T_i < 0)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_init_bcm: k=%d alpha=%g T_i=%d", k, alpha, T_i);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  return init_bcm(ctx, op, k, alpha, T_i, labels);
}

ancka_status ancka_mhc(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels, int32_t k, double alpha,
                       int32_t gamma, double* phi) {
  if (!ctx || !op || !labels || !phi) return ANCKA_ERR_INVALID_ARG;
  if (k < 1 || k > 64 || alpha < 0.0 || alpha > 1.0 || gamma < 1)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_mhc: k=%d alpha=%g gamma=%d", k, alpha, gamma);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  return mhc_host(ctx, op, labels, k, alpha, gamma, phi);
}

}  // extern "C"

namespace {

// Alg. 4 from the greedy start on on a built operator.  R: report with its trace buffers set; ph: phase times
// (the KNN and operator slots are left to the caller).
ancka_status cluster_loop(ancka_ctx* ctx, const ancka_op* op, const ancka_params& p, const float* zwarm,
                          int32_t* labels, ancka_report* R, double* ph) {
  const int64_t n = op->n;
  const int k = p.k;
  const int cap = R->trace_capacity;
  int32_t* tr_t = R->trace_t;
  double* tr_phi = R->trace_phi;
  auto trace = [&](int t, double phi) {
    if (R->trace_len < cap && tr_t && tr_phi) {
      tr_t[R->trace_len] = t;
      tr_phi[R->trace_len] = phi;
    }
    R->trace_len++;
  };
  double t0 = 0.0;

  // ---- initial BCM (Alg. 4, greedy start) and its MHC
  t0 = now_ms();
  const int64_t ldq = pad_ld(k + 1, p.q_dtype);
  const size_t es = p.q_dtype == ANCKA_F64 ? 8 : 4;
  int32_t *ycur = nullptr, *ybest = nullptr, *ywarm = nullptr;
  ST_TRY(ws_get_t(ctx, "cl_ycur", (size_t)n, &ycur));
  ST_TRY(ws_get_t(ctx, "cl_ybest", (size_t)n, &ybest));
  ST_TRY(init_bcm(ctx, op, k, p.alpha, p.T_i, ybest));
  double phi0 = 0.0;
  hipStream_t side_s = nullptr;
  hipEvent_t side_ev = nullptr;
  ST_TRY(ctx_side_stream(ctx, &side_s, &side_ev));
  double* dphi0 = nullptr;
  bool phi0_pending = false;
  if (!zwarm) {
    // the greedy start's conductance is first needed at the first check: it runs on the side
    // stream beside the starting block and the first block of iterations
    int* dbad0 = nullptr;
    ST_TRY(ws_get_t(ctx, "cl_phi0", 1, &dphi0));
    ST_TRY(ws_get_t(ctx, "cl_bad0", 4, &dbad0));
    HIP_TRY(ctx, hipEventRecord(side_ev, ctx->stream));
    HIP_TRY(ctx, hipStreamWaitEvent(side_s, side_ev, 0));
    hipStream_t main0 = ctx->stream;
    ctx->stream = side_s;
    ancka_status st = fill_zero(ctx, dbad0, 16);
    if (st == ANCKA_OK) st = mhc_dev(ctx, op, ybest, k, p.alpha, p.gamma, dphi0, dbad0, false);   // labels from init_bcm
    ctx->stream = main0;
    ST_TRY(st);
    phi0_pending = true;
  } else {
    ST_TRY(mhc_host(ctx, op, ybest, k, p.alpha, p.gamma, &phi0));
    R->phi_init_cold = phi0;
  }
  ph[ANCKA_PHASE_INIT] = now_ms() - t0;
  bool warm = false;
  if (zwarm) {
    t0 = now_ms();
    ST_TRY(ws_get_t(ctx, "cl_ywarm", (size_t)n, &ywarm));
    warm_argmax_kernel<<<nb256(n), 256, 0, ctx->stream>>>(zwarm, n, k, ywarm);
    LAUNCH_CHECK(ctx);
    double phw = 0.0;
    ST_TRY(mhc_host(ctx, op, ywarm, k, p.alpha, p.gamma, &phw));
    R->phi_init_warm = phw;
    if (phw <= phi0) {
      warm = true;
      phi0 = phw;
      copy_i32_kernel<<<nb256(n), 256, 0, ctx->stream>>>(ywarm, ybest, n);
      LAUNCH_CHECK(ctx);
    }
    ph[ANCKA_PHASE_WARM] += now_ms() - t0;
  }
  R->init_used = warm ? 1 : 0;

  // ---- starting block (Alg. 4, starting block)
  t0 = now_ms();
  void *Q = nullptr, *Qn = nullptr, *Z = nullptr;
  double* dq2 = nullptr;
  int* qflags = nullptr;
  ST_TRY(ws_get(ctx, "cl_Q", (size_t)n * ldq * es, &Q));
  ST_TRY(ws_get(ctx, "cl_Qn", (size_t)n * ldq * es, &Qn));
  ST_TRY(ws_get(ctx, "cl_Z", (size_t)n * ldq * es, &Z));
  // padding columns stay zero through every product (they are never written by the QR)
  ST_TRY(fill_zero(ctx, Q, (size_t)n * ldq * es));
  ST_TRY(fill_zero(ctx, Qn, (size_t)n * ldq * es));
  ST_TRY(fill_zero(ctx, Z, (size_t)n * ldq * es));
  ST_TRY(ws_get_t(ctx, "cl_dq2", 2, &dq2));
  ST_TRY(initial_block(ctx, op, warm ? nullptr : ybest, warm ? zwarm : nullptr, k, Q, ldq));
  ST_TRY(ws_get_t(ctx, "qr_flags", 4, &qflags));
  ST_TRY(fill_zero(ctx, qflags, 16));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ph[warm ? ANCKA_PHASE_WARM : ANCKA_PHASE_INIT] += now_ms() - t0;

  // ---- main loop (Alg. 4, main loop)
  // The iterations run on the main stream in blocks of tau.  At a check t the block Q(t) is
  // copied aside; unless Eq. (tcond-1) already ends the run, the next block is queued on the
  // main stream at once, and the Discretize and MHC of check t run on the side stream meanwhile
  // (the next iterations need only Q(t)).  Results, checks and stopping points are those of
  // running everything in order; a check that could end the run is not overlapped.
  hipStream_t main_s = ctx->stream;
  hipEvent_t snap_ev = side_ev;
  void* Qs = nullptr;
  ST_TRY(ws_get(ctx, "cl_Qs", (size_t)n * ldq * es, &Qs));
  double best_phi = phi0;
  int best_t = 0;
  std::vector<double> hist{phi0};
  // the greedy start's conductance from the side stream (before the first check uses it)
  auto resolve_phi0 = [&]() -> ancka_status {
    if (!phi0_pending) return ANCKA_OK;
    HIP_TRY(ctx, hipMemcpyAsync(&phi0, dphi0, sizeof(double), hipMemcpyDeviceToHost, side_s));
    HIP_TRY(ctx, hipStreamSynchronize(side_s));
    phi0_pending = false;
    R->phi_init_cold = phi0;
    best_phi = phi0;
    hist[0] = phi0;
    trace(0, phi0);
    return ANCKA_OK;
  };
  if (!phi0_pending) trace(0, phi0);
  int reason = ANCKA_STOP_MAX_ITER;
  int t = 0;
  int enq = 0;   // iterations queued on the main stream
  auto queue_to = [&](int upto) -> ancka_status {
    for (; enq < upto;) {
      enq++;
      const bool check = (enq % p.tau) == 0;
      ST_TRY(op_apply(ctx, op, Q, Z, k + 1, ldq));
      ST_TRY(qr_block(ctx, p.q_dtype, Z, Qn, n, k + 1, ldq, check ? Q : nullptr, check ? dq2 : nullptr, nullptr));
      std::swap(Q, Qn);
    }
    return ANCKA_OK;
  };
  double ti = now_ms();   // start of the current wait for the main stream
  ST_TRY(queue_to(p.T_a < p.tau ? p.T_a : p.tau));
  for (int tc = p.tau;; tc += p.tau) {
    if (tc > p.T_a) {   // no check left: the trailing iterations, then stop at T_a
      ST_TRY(queue_to(p.T_a));
      HIP_TRY(ctx, hipStreamSynchronize(main_s));
      ph[ANCKA_PHASE_ITER] += now_ms() - ti;
      t = p.T_a;
      break;
    }
    ST_TRY(resolve_phi0());
    double hdq2 = 0.0;
    int hflags[4] = {0, 0, 0, 0};
    HIP_TRY(ctx, hipMemcpyAsync(&hdq2, dq2, sizeof(double), hipMemcpyDeviceToHost, main_s));
    HIP_TRY(ctx, hipMemcpyAsync(hflags, qflags, sizeof(hflags), hipMemcpyDeviceToHost, main_s));
    HIP_TRY(ctx, hipStreamSynchronize(main_s));
    ph[ANCKA_PHASE_ITER] += now_ms() - ti;
    if (hflags[1] & 2) return set_err(ctx, ANCKA_ERR_NUMERICAL, "ancka_cluster: Cholesky QR broke down at t=%d", tc);
    const bool converged = p.early_stop && sqrt(hdq2) < p.eps_q;
    // Q(t) aside, then the next block of iterations (not when this check ends the run)
    HIP_TRY(ctx, hipMemcpyAsync(Qs, Q, (size_t)n * ldq * es, hipMemcpyDeviceToDevice, main_s));
    HIP_TRY(ctx, hipEventRecord(snap_ev, main_s));
    ti = now_ms();
    // Eq. (tcond-2) can end the run at this check only if the conductance already rose at the
    // previous one; the next block is queued ahead only when this check cannot end the run
    const size_t hn = hist.size();
    const bool may_stop = converged || (p.early_stop && hn >= 2 && hist[hn - 2] < hist[hn - 1]);
    if (!may_stop) ST_TRY(queue_to(tc + p.tau <= p.T_a ? tc + p.tau : p.T_a));
    // Discretize columns 2..k+1 (the constant eigenvector is dropped), then MHC, on the side
    HIP_TRY(ctx, hipStreamWaitEvent(side_s, snap_ev, 0));
    ctx->stream = side_s;
    double td = now_ms();
    int32_t dit = 0;
    double phi = 0.0;
    ancka_status st = discretize_internal(ctx, (const char*)Qs + es, p.q_dtype, n, k, ldq, p.disc_max_iter, ycur,
                                          nullptr, nullptr, &dit);
    double tm = now_ms();
    if (st == ANCKA_OK) st = mhc_host(ctx, op, ycur, k, p.alpha, p.gamma, &phi);
    if (st == ANCKA_OK && phi < best_phi) {
      copy_i32_kernel<<<nb256(n), 256, 0, side_s>>>(ycur, ybest, n);
      if (hipGetLastError() != hipSuccess) st = set_err(ctx, ANCKA_ERR_HIP, "ancka_cluster: launch failed");
    }
    ctx->stream = main_s;
    if (st != ANCKA_OK) {
      (void)hipStreamSynchronize(main_s);
      return st;
    }
    R->disc_iters_total += dit;
    ph[ANCKA_PHASE_DISCRETIZE] += tm - td;
    ph[ANCKA_PHASE_MHC] += now_ms() - tm;
    trace(tc, phi);
    if (phi < best_phi) {
      best_phi = phi;
      best_t = tc;
    }
    hist.push_back(phi);
    if (converged) {
      reason = ANCKA_STOP_CONVERGED;
      t = tc;
      break;
    }
    if (p.early_stop) {
      const size_t h = hist.size();
      if (h >= 3 && hist[h - 3] < hist[h - 2] && hist[h - 2] < hist[h - 1]) {
        reason = ANCKA_STOP_EARLY;
        t = tc;
        break;
      }
    }
    // the run goes on: queue the next block now if it was held back
    ti = now_ms();
    if (may_stop) ST_TRY(queue_to(tc + p.tau <= p.T_a ? tc + p.tau : p.T_a));
  }
  // the side stream's last copy into ybest, and any queued block, finish before the labels
  ST_TRY(resolve_phi0());
  HIP_TRY(ctx, hipStreamSynchronize(side_s));
  HIP_TRY(ctx, hipStreamSynchronize(main_s));
  copy_i32_kernel<<<nb256(n), 256, 0, ctx->stream>>>(ybest, labels, n);
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  R->iterations = t;
  R->stop_reason = reason;
  R->best_phi = best_phi;
  R->best_t = best_t;
  return ANCKA_OK;
}

bool params_ok(const ancka_params& p, int64_t n) {
  const int k = p.k;
  return !(k < 1 || k + 1 > 64 || k > n || p.K < 1 || p.K > n - 1 || p.alpha < 0.0 || p.alpha > 1.0 || p.beta < 0.0 ||
           p.beta > 1.0 || p.gamma < 1 || p.tau < 1 || p.T_i < 0 || p.T_a < 0 || p.disc_max_iter < 1 ||
           (p.q_dtype != ANCKA_F32 && p.q_dtype != ANCKA_F64));
}

void report_init(ancka_report* R) {
  const int cap = R->trace_capacity;
  int32_t* tr_t = R->trace_t;
  double* tr_phi = R->trace_phi;
  *R = ancka_report{};
  R->trace_capacity = cap;
  R->trace_t = tr_t;
  R->trace_phi = tr_phi;
  R->phi_init_warm = std::numeric_limits<double>::quiet_NaN();
}

}  // namespace

extern "C" {

ancka_status ancka_cluster_op(ancka_ctx* ctx, const ancka_op* op, const ancka_params* prm, const float* zwarm,
                              int32_t* labels, ancka_report* rep) {
  if (!ctx || !op || !prm || !labels) return ANCKA_ERR_INVALID_ARG;
  if (!params_ok(*prm, op->n) || prm->q_dtype != op->dtype)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_cluster_op: invalid parameters (n=%lld k=%d, q_dtype %d, op %d)",
                   (long long)op->n, prm->k, prm->q_dtype, op->dtype);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  ancka_report local;
  local.trace_capacity = 0;
  local.trace_t = nullptr;
  local.trace_phi = nullptr;
  ancka_report* R = rep ? rep : &local;
  report_init(R);
  double ph[ANCKA_NPHASES] = {0};
  ST_TRY(cluster_loop(ctx, op, *prm, zwarm, labels, R, ph));
  for (int i = 0; i < ANCKA_NPHASES; i++) R->phase_ms[i] = ph[i];
  return ANCKA_OK;
}

ancka_status ancka_cluster(ancka_ctx* ctx, const ancka_network* net, const ancka_params* prm, const float* zwarm,
                           int32_t* labels, ancka_report* rep) {
  if (!ctx || !net || !prm || !labels) return ANCKA_ERR_INVALID_ARG;
  const ancka_params& p = *prm;
  const int64_t n = net->n;
  if (!params_ok(p, n) || !net->X)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_cluster: invalid parameters (n=%lld k=%d K=%d)", (long long)n,
                   p.k, p.K);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  double ph[ANCKA_NPHASES] = {0};
  ancka_report local;
  local.trace_capacity = 0;
  local.trace_t = nullptr;
  local.trace_phi = nullptr;
  ancka_report* R = rep ? rep : &local;
  report_init(R);

  // ---- KNN graph (Alg. 6)
  double t0 = now_ms();
  const bool f64sim = p.knn_mode == ANCKA_KNN_EXACT_F64;
  int32_t* nidx = nullptr;
  void* nsim = nullptr;
  ST_TRY(ws_get_t(ctx, "cl_nidx", (size_t)n * p.K, &nidx));
  ST_TRY(ws_get(ctx, "cl_nsim", (size_t)n * p.K * (f64sim ? 8 : 4), &nsim));
  if (p.knn_mode == ANCKA_KNN_IVF_BF16)
    ST_TRY(ancka_knn_ivf(ctx, net->X, net->xdtype, n, net->d, net->ldx, p.K, p.ivf_nlist, p.ivf_nprobe, nidx, nsim,
                         &R->knn));
  else
    ST_TRY(ancka_knn(ctx, net->X, net->xdtype, n, net->d, net->ldx, p.K, p.knn_mode, nidx, nsim, &R->knn));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ph[ANCKA_PHASE_KNN] = now_ms() - t0;

  // ---- operator (Alg. 4, operator construction)
  t0 = now_ms();
  ancka_op* op = nullptr;
  ST_TRY(ancka_build_operator(ctx, net, nidx, nsim, f64sim ? ANCKA_F64 : ANCKA_F32, p.K, p.beta, p.q_dtype, &op));
  struct OpGuard {
    ancka_op* o;
    ~OpGuard() { ancka_op_destroy(o); }
  } guard{op};
  ph[ANCKA_PHASE_OPERATOR] = now_ms() - t0;

  ST_TRY(cluster_loop(ctx, op, p, zwarm, labels, R, ph));
  for (int i = 0; i < ANCKA_NPHASES; i++) R->phase_ms[i] = ph[i];
  return ANCKA_OK;
}

}  // extern "C"
