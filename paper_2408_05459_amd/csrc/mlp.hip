// Learned warm start on gfx950: one-hop feature aggregation, a three-layer perceptron
// d -> h1 -> h2 -> k with BF16 MFMA products (FP32 accumulation), its backward pass, Adam, and
// the rotation that turns an eigenblock into a training target.
//
// Every product is C[M][N] = A[M][K] B[N][K]^T with both operands K-contiguous, so one MFMA
// kernel covers all of them:
//   forward        H = act(U W + b):     A = U or H (n rows),  B = W^T (out, in)
//   input gradient G = (G' W^T) * [H>0]: A = G' (n rows),      B = W (in, out)
//   weight grad    dW = H^T G:           A = H^T (in, n),      B = G^T (out, n), split over n
// The epilogues that produce an activation or a gradient also write its transposed BF16 copy,
// which is the K-contiguous operand of the weight-gradient product.  Split-K partial sums are
// reduced in a fixed order, so every result is deterministic.
#include <cmath>
#include <cstring>

#include "common.h"

struct ancka_ws {
  int device = 0;
  int d = 0, h1 = 0, h2 = 0, k = 0;
  int dK = 0;                         // d rounded up to 16
  int k16 = 0;                        // k rounded up to 16
  int64_t count = 0;                  // packed parameters
  int64_t off[6] = {};                // W1 b1 W2 b2 W3 b3 in the packed vector
  float* master = nullptr;            // FP32 master parameters (packed)
  float* grad = nullptr;              // gradients (packed)
  float* am = nullptr;                // Adam first moment
  float* av = nullptr;                // Adam second moment
  float* pack = nullptr;              // staging for get_params(0)
  int64_t t = 0;                      // Adam step count
  uint16_t* W1T = nullptr;            // [h1][dK] forward operand (out, in)
  uint16_t* W2T = nullptr;            // [h2][h1]
  uint16_t* W3T = nullptr;            // [k][h2]
  uint16_t* W2N = nullptr;            // [h1][h2] input-gradient operand (in, out)
  uint16_t* W3N = nullptr;            // [h2][k16]
  // forward activations (row-major), grown to capf rows
  int64_t capf = 0;
  uint16_t* H1 = nullptr;             // [capf][h1]
  uint16_t* H2 = nullptr;             // [capf][h2]
  // training buffers, grown to capb rows (npad = leading dimension of the transposed copies)
  int64_t capb = 0, npad = 0;
  uint16_t* UT = nullptr;             // [d][npad]
  uint16_t* H1T = nullptr;            // [h1][npad]
  uint16_t* H2T = nullptr;            // [h2][npad]
  uint16_t* G3 = nullptr;             // [capb][k16]
  uint16_t* G3T = nullptr;            // [k][npad]
  uint16_t* G2 = nullptr;             // [capb][h2]
  uint16_t* G2T = nullptr;            // [h2][npad]
  uint16_t* G1T = nullptr;            // [h1][npad]
  float* part = nullptr;              // split-K partials
  size_t part_elems = 0;
  double* lpart = nullptr;            // loss partials
  double* lsum = nullptr;
  int64_t kept_n = 0;                 // rows of the activations kept by the last forward
  std::vector<void*> owned;
};

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int KSPLIT_MAX = 64;

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// 8 consecutive K elements of one operand row as a BF16 fragment; elements at or beyond `lim`
// (relative to p) read as zero.
template <typename TA>
__device__ __forceinline__ bf16x8 load_frag(const TA* p, bool row_ok, int64_t lim);

template <>
__device__ __forceinline__ bf16x8 load_frag<uint16_t>(const uint16_t* p, bool row_ok, int64_t lim) {
  uint4 v = make_uint4(0, 0, 0, 0);
  if (row_ok) {
    if (lim >= 8) {
      v = *(const uint4*)p;
    } else {
      uint16_t e[8];
#pragma unroll
      for (int u = 0; u < 8; u++) e[u] = (u < lim) ? p[u] : (uint16_t)0;
      v.x = e[0] | ((uint32_t)e[1] << 16);
      v.y = e[2] | ((uint32_t)e[3] << 16);
      v.z = e[4] | ((uint32_t)e[5] << 16);
      v.w = e[6] | ((uint32_t)e[7] << 16);
    }
  }
  return __builtin_bit_cast(bf16x8, v);
}

template <>
__device__ __forceinline__ bf16x8 load_frag<float>(const float* p, bool row_ok, int64_t lim) {
  float e[8];
  if (row_ok && lim >= 8) {
    const float4 a = *(const float4*)p;
    const float4 b = *(const float4*)(p + 4);
    e[0] = a.x; e[1] = a.y; e[2] = a.z; e[3] = a.w;
    e[4] = b.x; e[5] = b.y; e[6] = b.z; e[7] = b.w;
  } else {
#pragma unroll
    for (int u = 0; u < 8; u++) e[u] = (row_ok && u < lim) ? p[u] : 0.0f;
  }
  uint4 v;
  v.x = bf16_rne(e[0]) | ((uint32_t)bf16_rne(e[1]) << 16);
  v.y = bf16_rne(e[2]) | ((uint32_t)bf16_rne(e[3]) << 16);
  v.z = bf16_rne(e[4]) | ((uint32_t)bf16_rne(e[5]) << 16);
  v.w = bf16_rne(e[6]) | ((uint32_t)bf16_rne(e[7]) << 16);
  return __builtin_bit_cast(bf16x8, v);
}

struct GemmArgs {
  const void* A;           // [M][K] row-major, leading dimension lda (float or bf16)
  int64_t lda;
  const uint16_t* B;       // [N][K] row-major bf16, leading dimension ldb
  int64_t ldb;
  int64_t M;
  int N;
  int64_t K;
  int64_t kchunk;          // K range of one blockIdx.z (multiple of 16)
  const float* bias;       // [N] or null
  int relu;
  const uint16_t* mask;    // [M][ldm] bf16: result kept where mask > 0 (null: no mask)
  int64_t ldm;
  float* C;                // f32 out, C[z * csplit + row * ldc + col] (null: none)
  int64_t ldc, csplit;
  uint16_t* Cb;            // bf16 row-major out (null: none)
  int64_t ldcb;
  uint16_t* Ct;            // bf16 transposed out, Ct[col * ldct + row] (null: none)
  int64_t ldct;
};

// Workgroup of 4 waves stacked along M; a wave owns a (32 MB) x (32 NB) block of C and keeps
// MB x NB 32x32 FP32 accumulators.  Operand fragments are read straight from global memory
// (16 bytes per lane per k-step); rows of one fragment are neighbours, so the 4 k-steps of a
// 128-byte line hit the same cache line.
template <typename TA, int MB, int NB>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(const GemmArgs g) {
  const int wave = threadIdx.x / ANCKA_WAVE;
  const int lane = threadIdx.x % ANCKA_WAVE;
  const int l32 = lane % 32;
  const int half = lane / 32;
  const int64_t r0 = (int64_t)blockIdx.x * (128 * MB) + wave * (32 * MB);
  const int c0 = blockIdx.y * (32 * NB);
  const int64_t kb = (int64_t)blockIdx.z * g.kchunk;
  const int64_t ke = (kb + g.kchunk < g.K) ? kb + g.kchunk : g.K;
  const TA* A = (const TA*)g.A;

  f32x16 acc[MB][NB];
#pragma unroll
  for (int mb = 0; mb < MB; mb++)
#pragma unroll
    for (int nb = 0; nb < NB; nb++)
#pragma unroll
      for (int i = 0; i < 16; i++) acc[mb][nb][i] = 0.0f;

  const TA* arow[MB];
  bool aok[MB];
#pragma unroll
  for (int mb = 0; mb < MB; mb++) {
    const int64_t row = r0 + mb * 32 + l32;
    aok[mb] = row < g.M;
    arow[mb] = A + (aok[mb] ? row : 0) * g.lda;
  }
  const uint16_t* brow[NB];
  bool bok[NB];
#pragma unroll
  for (int nb = 0; nb < NB; nb++) {
    const int col = c0 + nb * 32 + l32;
    bok[nb] = col < g.N;
    brow[nb] = g.B + (int64_t)(bok[nb] ? col : 0) * g.ldb;
  }

#pragma unroll 2
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    const int64_t kk = k0 + half * 8;
    const int64_t lim = ke - kk;
    bf16x8 a[MB], b[NB];
#pragma unroll
    for (int mb = 0; mb < MB; mb++) a[mb] = load_frag<TA>(arow[mb] + kk, aok[mb], lim);
#pragma unroll
    for (int nb = 0; nb < NB; nb++) b[nb] = load_frag<uint16_t>(brow[nb] + kk, bok[nb], lim);
#pragma unroll
    for (int mb = 0; mb < MB; mb++)
#pragma unroll
      for (int nb = 0; nb < NB; nb++)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
  }

  // epilogue: acc[mb][nb][4q + e] is C[r0 + 32 mb + 8 q + 4 half + e][c0 + 32 nb + l32]
#pragma unroll
  for (int nb = 0; nb < NB; nb++) {
    const int col = c0 + nb * 32 + l32;
    if (col >= g.N) continue;
    const float bias = g.bias ? g.bias[col] : 0.0f;
#pragma unroll
    for (int mb = 0; mb < MB; mb++) {
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int64_t rb = r0 + mb * 32 + 8 * q + 4 * half;
        uint16_t hv[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int64_t row = rb + e;
          float v = acc[mb][nb][4 * q + e] + bias;
          if (g.relu) v = fmaxf(v, 0.0f);
          if (g.mask && row < g.M) {
            const uint16_t m = g.mask[row * g.ldm + col];
            if (m == 0 || (m & 0x8000u)) v = 0.0f;
          }
          hv[e] = bf16_rne(v);
          if (row < g.M) {
            if (g.C) g.C[(int64_t)blockIdx.z * g.csplit + row * g.ldc + col] = v;
            if (g.Cb) g.Cb[row * g.ldcb + col] = hv[e];
          }
        }
        if (g.Ct) {
          uint16_t* dst = g.Ct + (int64_t)col * g.ldct + rb;
          if (rb + 3 < g.M) {
            uint2 w;
            w.x = hv[0] | ((uint32_t)hv[1] << 16);
            w.y = hv[2] | ((uint32_t)hv[3] << 16);
            *(uint2*)dst = w;
          } else {
#pragma unroll
            for (int e = 0; e < 4; e++)
              if (rb + e < g.M) dst[e] = hv[e];
          }
        }
      }
    }
  }
}

// sum of split-K partials in split order: out[e] = sum_z part[z * stride + e]
__global__ __launch_bounds__(256) void split_reduce_kernel(const float* __restrict__ part, int splits, int64_t stride,
                                                           float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= stride) return;
  float s = 0.0f;
  for (int z = 0; z < splits; z++) s += part[(int64_t)z * stride + e];
  out[e] = s;
}

// out[r] = sum_{i < n} bf16 Y[r][i] (bias gradients; one workgroup per row, fixed order)
__global__ __launch_bounds__(256) void row_sum_kernel(const uint16_t* __restrict__ Y, int64_t ld, int64_t n,
                                                      float* __restrict__ out) {
  __shared__ float red[4];
  const uint16_t* y = Y + (int64_t)blockIdx.x * ld;
  float s = 0.0f;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += bf16_val(y[i]);
  s = wave_sum(s);
  if (threadIdx.x % ANCKA_WAVE == 0) red[threadIdx.x / ANCKA_WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// G3 = bf16(2 (Z - T) / n) into [n][k16] and its transpose [k][npad]; per-block sums of (Z-T)^2
__global__ __launch_bounds__(256) void loss_grad_kernel(const float* __restrict__ Z, const float* __restrict__ T,
                                                        int64_t n, int k, float scale, uint16_t* __restrict__ G3,
                                                        int k16, uint16_t* __restrict__ G3T, int64_t npad,
                                                        double* __restrict__ lpart) {
  __shared__ double red[4];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double sq = 0.0;
  if (e < n * k) {
    const int64_t i = e / k;
    const int o = (int)(e % k);
    const float diff = Z[e] - T[e];
    sq = (double)diff * (double)diff;
    const uint16_t h = bf16_rne(diff * scale);
    G3[i * k16 + o] = h;
    G3T[(int64_t)o * npad + i] = h;
  }
  sq = wave_sum(sq);
  if (threadIdx.x % ANCKA_WAVE == 0) red[threadIdx.x / ANCKA_WAVE] = sq;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ p, int64_t count,
                                                           double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) s += p[i];
  s = wave_sum(s);
  if (threadIdx.x % ANCKA_WAVE == 0) red[threadIdx.x / ANCKA_WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

// UT[c][i] = bf16(U[i][c]) for c < d, i < n, through a 64 x 64 LDS tile
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const float* __restrict__ U, int64_t ldu, int64_t n, int d,
                                                             uint16_t* __restrict__ UT, int64_t ldt) {
  __shared__ uint16_t tile[64][66];
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r;
    const int c = c0 + tx;
    tile[r][tx] = (i < n && c < d) ? bf16_rne(U[i * ldu + c]) : (uint16_t)0;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int c = c0 + r;
    const int64_t i = i0 + tx;
    if (c < d && i < n) UT[(int64_t)c * ldt + i] = tile[tx][r];
  }
}

// dst[r][c] = bf16(src(r, c)) for r < R, c < Cpad (zero for c >= C); src(r, c) = src[c*lds + r]
// when trans, else src[r*lds + c]
__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ src, int64_t lds, int trans, int R,
                                                      int C, int Cpad, uint16_t* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)R * Cpad) return;
  const int r = (int)(e / Cpad), c = (int)(e % Cpad);
  float v = 0.0f;
  if (c < C) v = trans ? src[(int64_t)c * lds + r] : src[(int64_t)r * lds + c];
  dst[e] = bf16_rne(v);
}

// out(r, c) = float(bf16 WT[c][r]) for r < R (in), c < C (out): the forward weights as (in, out)
__global__ __launch_bounds__(256) void from_bf16_t_kernel(const uint16_t* __restrict__ WT, int64_t ldw, int R, int C,
                                                          float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)R * C) return;
  const int r = (int)(e / C), c = (int)(e % C);
  out[e] = bf16_val(WT[(int64_t)c * ldw + r]);
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t count, float lr,
                                                   float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const float gi = g[e];
  const float mi = 0.9f * m[e] + 0.1f * gi;
  const float vi = 0.999f * v[e] + 0.001f * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// X^ rows (unit L2 norm, zero rows stay zero) as float n x ld; columns d .. round4(d)-1 zero
template <typename TX>
__device__ __forceinline__ float load_f(const TX* p, int64_t i);
template <>
__device__ __forceinline__ float load_f<double>(const double* p, int64_t i) { return (float)p[i]; }
template <>
__device__ __forceinline__ float load_f<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ float load_f<uint16_t>(const uint16_t* p, int64_t i) { return bf16_val(p[i]); }
template <typename TX>
__device__ __forceinline__ double load_d(const TX* p, int64_t i) {
  if constexpr (sizeof(TX) == 8) return (double)p[i];
  else return (double)load_f<TX>(p, i);
}

template <typename TX>
__global__ __launch_bounds__(256) void normalize_rows_kernel(const TX* __restrict__ X, int64_t n, int64_t d,
                                                             int64_t ldx, float* __restrict__ Xh, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / ANCKA_WAVE;
  const int lane = threadIdx.x % ANCKA_WAVE;
  if (i >= n) return;
  const TX* x = X + i * ldx;
  double s = 0.0;
  for (int64_t c = lane; c < d; c += ANCKA_WAVE) {
    const double v = load_d<TX>(x, c);
    s += v * v;
  }
  s = wave_sum(s);
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  const int64_t dp = (d + 3) / 4 * 4;
  for (int64_t c = lane; c < dp; c += ANCKA_WAVE)
    Xh[i * ld + c] = (c < d) ? (float)(load_d<TX>(x, c) * inv) : 0.0f;
}

// T[i][colmap[c]] = sum_j Q~[i][j] R[j][c], Q~ = row of Q scaled to unit norm (zero stays zero)
template <typename TQ>
__global__ __launch_bounds__(256) void target_kernel(const TQ* __restrict__ Q, int64_t n, int k, int64_t ldq,
                                                     const double* __restrict__ R, const int32_t* __restrict__ colmap,
                                                     float* __restrict__ T) {
  __shared__ double Rs[64 * 64];
  __shared__ int cm[64];
  for (int e = threadIdx.x; e < k * k; e += 256) Rs[e] = R[e];
  if ((int)threadIdx.x < k) cm[threadIdx.x] = colmap[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const TQ* q = Q + i * ldq;
  double s = 0.0;
  for (int j = 0; j < k; j++) s += (double)q[j] * (double)q[j];
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int c = 0; c < k; c++) {
    double y = 0.0;
    for (int j = 0; j < k; j++) y += (double)q[j] * Rs[j * k + c];
    T[i * k + cm[c]] = (float)(y * inv);
  }
}

// --------------------------------------------------------------------------------------------

inline int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

ancka_status ws_alloc(ancka_ctx* ctx, ancka_ws* ws, size_t bytes, void** out) {
  void* p = nullptr;
  HIP_TRY(ctx, hipMalloc(&p, bytes > 0 ? bytes : 16));
  ws->owned.push_back(p);
  *out = p;
  return ANCKA_OK;
}
template <typename T>
ancka_status ws_alloc_t(ancka_ctx* ctx, ancka_ws* ws, size_t count, T** out) {
  void* p = nullptr;
  ancka_status s = ws_alloc(ctx, ws, count * sizeof(T), &p);
  *out = (T*)p;
  return s;
}
// release a buffer owned by ws (after the stream has drained)
void ws_release(ancka_ws* ws, void* p) {
  if (!p) return;
  for (size_t i = 0; i < ws->owned.size(); i++)
    if (ws->owned[i] == p) {
      (void)hipFree(p);
      ws->owned.erase(ws->owned.begin() + i);
      return;
    }
}

unsigned nblk(int64_t c) { return (unsigned)cdiv(c > 0 ? c : 1, 256); }

ancka_status launch_gemm(ancka_ctx* ctx, const GemmArgs& g, bool a_f32, int splits) {
  if (g.M <= 0 || g.N <= 0) return ANCKA_OK;
  // 64-column tiles for wide outputs, 32 for the k-column output layer
  const bool wide = g.N > 32;
  const int MB = 2;
  const unsigned gx = (unsigned)cdiv(g.M, 128 * MB);
  const unsigned gy = (unsigned)cdiv(g.N, wide ? 64 : 32);
  dim3 grid(gx, gy, (unsigned)splits);
  if (a_f32) {
    if (wide) mlp_gemm_kernel<float, 2, 2><<<grid, 256, 0, ctx->stream>>>(g);
    else mlp_gemm_kernel<float, 2, 1><<<grid, 256, 0, ctx->stream>>>(g);
  } else {
    if (wide) mlp_gemm_kernel<uint16_t, 2, 2><<<grid, 256, 0, ctx->stream>>>(g);
    else mlp_gemm_kernel<uint16_t, 2, 1><<<grid, 256, 0, ctx->stream>>>(g);
  }
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

GemmArgs gemm_blank() {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  return g;
}

// refresh the BF16 operand copies from the master weights
ancka_status refresh_bf16(ancka_ctx* ctx, ancka_ws* ws) {
  const float* W1 = ws->master + ws->off[0];
  const float* W2 = ws->master + ws->off[2];
  const float* W3 = ws->master + ws->off[4];
  to_bf16_kernel<<<nblk((int64_t)ws->h1 * ws->dK), 256, 0, ctx->stream>>>(W1, ws->h1, 1, ws->h1, ws->d, ws->dK, ws->W1T);
  to_bf16_kernel<<<nblk((int64_t)ws->h2 * ws->h1), 256, 0, ctx->stream>>>(W2, ws->h2, 1, ws->h2, ws->h1, ws->h1, ws->W2T);
  to_bf16_kernel<<<nblk((int64_t)ws->k * ws->h2), 256, 0, ctx->stream>>>(W3, ws->k, 1, ws->k, ws->h2, ws->h2, ws->W3T);
  to_bf16_kernel<<<nblk((int64_t)ws->h1 * ws->h2), 256, 0, ctx->stream>>>(W2, ws->h2, 0, ws->h1, ws->h2, ws->h2, ws->W2N);
  to_bf16_kernel<<<nblk((int64_t)ws->h2 * ws->k16), 256, 0, ctx->stream>>>(W3, ws->k, 0, ws->h2, ws->k, ws->k16, ws->W3N);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

ancka_status ensure_fwd(ancka_ctx* ctx, ancka_ws* ws, int64_t n) {
  if (n <= ws->capf) return ANCKA_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ws_release(ws, ws->H1);
  ws_release(ws, ws->H2);
  ws->H1 = ws->H2 = nullptr;
  ws->capf = 0;
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)n * ws->h1, &ws->H1));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)n * ws->h2, &ws->H2));
  ws->capf = n;
  return ANCKA_OK;
}

ancka_status ensure_bwd(ancka_ctx* ctx, ancka_ws* ws, int64_t n) {
  if (n <= ws->capb) return ANCKA_OK;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  uint16_t** bufs[] = {&ws->UT, &ws->H1T, &ws->H2T, &ws->G3, &ws->G3T, &ws->G2, &ws->G2T, &ws->G1T};
  for (uint16_t** b : bufs) {
    ws_release(ws, *b);
    *b = nullptr;
  }
  ws_release(ws, ws->lpart);
  ws->lpart = nullptr;
  ws->capb = 0;
  ws->kept_n = 0;
  const int64_t np = rup(n, 64);
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)ws->d * np, &ws->UT));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)ws->h1 * np, &ws->H1T));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)ws->h2 * np, &ws->H2T));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)n * ws->k16, &ws->G3));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)ws->k * np, &ws->G3T));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)n * ws->h2, &ws->G2));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)ws->h2 * np, &ws->G2T));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)ws->h1 * np, &ws->G1T));
  ST_TRY(ws_alloc_t(ctx, ws, (size_t)cdiv(n * ws->k, 256), &ws->lpart));
  ws->npad = np;
  ws->capb = n;
  return ANCKA_OK;
}

// dW[M][N] = A^T-product over n rows, split over n, reduced into out (packed gradient slot)
ancka_status weight_grad(ancka_ctx* ctx, ancka_ws* ws, const uint16_t* AT, int64_t M, const uint16_t* BT, int N,
                         int64_t n, float* out) {
  // about 4 workgroups per compute unit, each over at least 256 rows of n
  const int64_t tiles = cdiv(M, 256) * cdiv(N, N > 32 ? 64 : 32);
  int64_t splits = cdiv(4 * (int64_t)(ctx->num_cu > 0 ? ctx->num_cu : 256), tiles);
  splits = splits < 1 ? 1 : (splits > KSPLIT_MAX ? KSPLIT_MAX : splits);
  int64_t chunk = rup(cdiv(n, splits), 16);
  if (chunk < 256) chunk = 256;
  splits = cdiv(n, chunk);
  GemmArgs g = gemm_blank();
  g.A = AT;
  g.lda = ws->npad;
  g.B = BT;
  g.ldb = ws->npad;
  g.M = M;
  g.N = N;
  g.K = n;
  g.kchunk = chunk;
  g.C = ws->part;
  g.ldc = N;
  g.csplit = M * N;
  if ((size_t)(splits * M * N) > ws->part_elems) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws: partial buffer");
  ST_TRY(launch_gemm(ctx, g, false, (int)splits));
  split_reduce_kernel<<<nblk(M * N), 256, 0, ctx->stream>>>(ws->part, (int)splits, M * N, out);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

// SplitMix64 (Steele, Lea and Flood 2014) 53-bit uniforms in [0, 1)
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

ancka_status check_ws(ancka_ctx* ctx, ancka_ws* ws) {
  if (!ctx) return ANCKA_ERR_INVALID_ARG;
  if (!ws) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws: null model");
  if (ws->device != ctx->device) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws: model belongs to another device");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  return ANCKA_OK;
}

}  // namespace

extern "C" {

void ancka_ws_destroy(ancka_ws* ws) {
  if (!ws) return;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ws->device);
  (void)hipDeviceSynchronize();
  for (void* p : ws->owned) (void)hipFree(p);
  (void)hipSetDevice(prev);
  delete ws;
}

ancka_status ancka_ws_create(ancka_ctx* ctx, int32_t d_in, int32_t h1, int32_t h2, int32_t k, uint64_t seed,
                             ancka_ws** out) {
  if (!ctx || !out) return ANCKA_ERR_INVALID_ARG;
  *out = nullptr;
  if (d_in < 1 || d_in > 4096 || h1 < 16 || h1 > 1024 || h1 % 16 || h2 < 16 || h2 > 1024 || h2 % 16 || k < 1 ||
      k > 64)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_create: d_in=%d h1=%d h2=%d k=%d", d_in, h1, h2, k);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  ancka_ws* ws = new ancka_ws();
  ws->device = ctx->device;
  ws->d = d_in;
  ws->h1 = h1;
  ws->h2 = h2;
  ws->k = k;
  ws->dK = (int)rup(d_in, 16);
  ws->k16 = (int)rup(k, 16);
  const int64_t sizes[6] = {(int64_t)d_in * h1, h1, (int64_t)h1 * h2, h2, (int64_t)h2 * k, k};
  int64_t o = 0;
  for (int i = 0; i < 6; i++) {
    ws->off[i] = o;
    o += sizes[i];
  }
  ws->count = o;
  ancka_status st = ANCKA_OK;
  auto fail = [&](ancka_status s) {
    ancka_ws_destroy(ws);
    return s;
  };
  if ((st = ws_alloc_t(ctx, ws, (size_t)o, &ws->master)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)o, &ws->grad)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)o, &ws->am)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)o, &ws->av)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)o, &ws->pack)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)h1 * ws->dK, &ws->W1T)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)h2 * h1, &ws->W2T)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)k * h2, &ws->W3T)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)h1 * h2, &ws->W2N)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, (size_t)h2 * ws->k16, &ws->W3N)) != ANCKA_OK) return fail(st);
  if ((st = ws_alloc_t(ctx, ws, 1, &ws->lsum)) != ANCKA_OK) return fail(st);
  // partials of the largest weight gradient at the largest split count
  int64_t mn = (int64_t)d_in * h1;
  if ((int64_t)h1 * h2 > mn) mn = (int64_t)h1 * h2;
  if ((int64_t)h2 * k > mn) mn = (int64_t)h2 * k;
  ws->part_elems = (size_t)(mn * KSPLIT_MAX);
  if ((st = ws_alloc_t(ctx, ws, ws->part_elems, &ws->part)) != ANCKA_OK) return fail(st);

  std::vector<float> host((size_t)o, 0.0f);
  SplitMix64 rng{seed};
  const int64_t wi[3] = {0, 2, 4};
  const int fan[3] = {d_in, h1, h2};
  for (int l = 0; l < 3; l++) {
    const double a = 1.0 / std::sqrt((double)fan[l]);
    for (int64_t e = 0; e < sizes[wi[l]]; e++) host[ws->off[wi[l]] + e] = (float)((2.0 * rng.uniform() - 1.0) * a);
  }
  if ((st = ancka_ws_set_params(ctx, ws, host.data())) != ANCKA_OK) return fail(st);
  *out = ws;
  return ANCKA_OK;
}

ancka_status ancka_ws_set_params(ancka_ctx* ctx, ancka_ws* ws, const float* host) {
  ST_TRY(check_ws(ctx, ws));
  if (!host) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_set_params: null host buffer");
  HIP_TRY(ctx, hipMemcpyAsync(ws->master, host, (size_t)ws->count * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ST_TRY(fill_zero(ctx, ws->am, (size_t)ws->count * sizeof(float)));
  ST_TRY(fill_zero(ctx, ws->av, (size_t)ws->count * sizeof(float)));
  ST_TRY(fill_zero(ctx, ws->grad, (size_t)ws->count * sizeof(float)));
  ws->t = 0;
  return refresh_bf16(ctx, ws);
}

ancka_status ancka_ws_get_params(ancka_ctx* ctx, ancka_ws* ws, int32_t which, float* host, int64_t* count) {
  ST_TRY(check_ws(ctx, ws));
  if (count) *count = ws->count;
  if (which < 0 || which > 2) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_get_params: which=%d", which);
  if (!host) return ANCKA_OK;
  const float* src = which == 1 ? ws->grad : ws->master;
  if (which == 0) {
    HIP_TRY(ctx, hipMemcpyAsync(ws->pack, ws->master, (size_t)ws->count * sizeof(float), hipMemcpyDeviceToDevice,
                                ctx->stream));
    from_bf16_t_kernel<<<nblk((int64_t)ws->d * ws->h1), 256, 0, ctx->stream>>>(ws->W1T, ws->dK, ws->d, ws->h1,
                                                                             ws->pack + ws->off[0]);
    from_bf16_t_kernel<<<nblk((int64_t)ws->h1 * ws->h2), 256, 0, ctx->stream>>>(ws->W2T, ws->h1, ws->h1, ws->h2,
                                                                              ws->pack + ws->off[2]);
    from_bf16_t_kernel<<<nblk((int64_t)ws->h2 * ws->k), 256, 0, ctx->stream>>>(ws->W3T, ws->h2, ws->h2, ws->k,
                                                                             ws->pack + ws->off[4]);
    LAUNCH_CHECK(ctx);
    src = ws->pack;
  }
  HIP_TRY(ctx, hipMemcpyAsync(host, src, (size_t)ws->count * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return ANCKA_OK;
}

ancka_status ancka_ws_features(ancka_ctx* ctx, const ancka_op* op, const void* X, int32_t xdtype, int64_t d,
                               int64_t ldx, float* U, int64_t ldu) {
  if (!ctx) return ANCKA_ERR_INVALID_ARG;
  if (!op || !X || !U) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_features: null argument");
  if (d < 1 || ldx < d || ldu < d || ldu % 4 != 0)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_features: d=%lld ldx=%lld ldu=%lld (ldu must be a multiple of 4)",
                   (long long)d, (long long)ldx, (long long)ldu);
  if (xdtype != ANCKA_F64 && xdtype != ANCKA_F32 && xdtype != ANCKA_BF16)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_features: xdtype %d", xdtype);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  const int64_t n = op->n;
  float* Xh = nullptr;
  ST_TRY(ws_get_t(ctx, "ws_xh", (size_t)n * ldu, &Xh));
  const unsigned grid = (unsigned)cdiv(n, 4);
  if (xdtype == ANCKA_F64)
    normalize_rows_kernel<double><<<grid, 256, 0, ctx->stream>>>((const double*)X, n, d, ldx, Xh, ldu);
  else if (xdtype == ANCKA_F32)
    normalize_rows_kernel<float><<<grid, 256, 0, ctx->stream>>>((const float*)X, n, d, ldx, Xh, ldu);
  else
    normalize_rows_kernel<uint16_t><<<grid, 256, 0, ctx->stream>>>((const uint16_t*)X, n, d, ldx, Xh, ldu);
  LAUNCH_CHECK(ctx);
  return op_apply_features(ctx, op, Xh, U, (int)((d + 3) / 4 * 4), ldu);
}

ancka_status ancka_ws_forward(ancka_ctx* ctx, ancka_ws* ws, const float* U, int64_t n, int64_t ldu, float* zhat,
                              int32_t keep_acts) {
  ST_TRY(check_ws(ctx, ws));
  if (!U || !zhat) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_forward: null argument");
  if (n < 1 || n > INT32_MAX || ldu < ws->d || ldu % 4 != 0 || ((uintptr_t)U % 16) != 0)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG,
                   "ws_forward: n=%lld ldu=%lld (ldu >= %d, multiple of 4, U 16-byte aligned)", (long long)n,
                   (long long)ldu, ws->d);
  ST_TRY(ensure_fwd(ctx, ws, n));
  if (keep_acts) {
    ST_TRY(ensure_bwd(ctx, ws, n));
    dim3 tg((unsigned)cdiv(n, 64), (unsigned)cdiv(ws->d, 64));
    transpose_bf16_kernel<<<tg, 256, 0, ctx->stream>>>(U, ldu, n, ws->d, ws->UT, ws->npad);
    LAUNCH_CHECK(ctx);
  }
  ws->kept_n = 0;
  // layer 1: H1 = bf16(relu(bf16(U) W1 + b1))
  GemmArgs g = gemm_blank();
  g.A = U;
  g.lda = ldu;
  g.B = ws->W1T;
  g.ldb = ws->dK;
  g.M = n;
  g.N = ws->h1;
  g.K = ws->d;
  g.kchunk = rup(ws->d, 16);
  g.bias = ws->master + ws->off[1];
  g.relu = 1;
  g.Cb = ws->H1;
  g.ldcb = ws->h1;
  g.Ct = keep_acts ? ws->H1T : nullptr;
  g.ldct = ws->npad;
  ST_TRY(launch_gemm(ctx, g, true, 1));
  // layer 2: H2 = bf16(relu(H1 W2 + b2))
  g = gemm_blank();
  g.A = ws->H1;
  g.lda = ws->h1;
  g.B = ws->W2T;
  g.ldb = ws->h1;
  g.M = n;
  g.N = ws->h2;
  g.K = ws->h1;
  g.kchunk = ws->h1;
  g.bias = ws->master + ws->off[3];
  g.relu = 1;
  g.Cb = ws->H2;
  g.ldcb = ws->h2;
  g.Ct = keep_acts ? ws->H2T : nullptr;
  g.ldct = ws->npad;
  ST_TRY(launch_gemm(ctx, g, false, 1));
  // layer 3: Zhat = H2 W3 + b3 (FP32)
  g = gemm_blank();
  g.A = ws->H2;
  g.lda = ws->h2;
  g.B = ws->W3T;
  g.ldb = ws->h2;
  g.M = n;
  g.N = ws->k;
  g.K = ws->h2;
  g.kchunk = ws->h2;
  g.bias = ws->master + ws->off[5];
  g.C = zhat;
  g.ldc = ws->k;
  ST_TRY(launch_gemm(ctx, g, false, 1));
  if (keep_acts) ws->kept_n = n;
  return ANCKA_OK;
}

ancka_status ancka_ws_backward(ancka_ctx* ctx, ancka_ws* ws, const float* zhat, const float* T, int64_t n,
                               double* loss) {
  ST_TRY(check_ws(ctx, ws));
  if (!zhat || !T) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_backward: null argument");
  if (n < 1 || n != ws->kept_n)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_backward: no activations kept for n=%lld (kept %lld)",
                   (long long)n, (long long)ws->kept_n);
  const int k = ws->k;
  const int64_t lblocks = cdiv(n * k, 256);
  loss_grad_kernel<<<(unsigned)lblocks, 256, 0, ctx->stream>>>(zhat, T, n, k, (float)(2.0 / (double)n), ws->G3, ws->k16,
                                                               ws->G3T, ws->npad, ws->lpart);
  LAUNCH_CHECK(ctx);
  if (loss) {
    sum_partials_kernel<<<1, 256, 0, ctx->stream>>>(ws->lpart, lblocks, ws->lsum);
    LAUNCH_CHECK(ctx);
  }
  float* gr = ws->grad;
  // layer 3: dW3 = H2^T G3, db3 = sum G3
  ST_TRY(weight_grad(ctx, ws, ws->H2T, ws->h2, ws->G3T, k, n, gr + ws->off[4]));
  row_sum_kernel<<<(unsigned)k, 256, 0, ctx->stream>>>(ws->G3T, ws->npad, n, gr + ws->off[5]);
  LAUNCH_CHECK(ctx);
  // G2 = bf16((G3 W3^T) * [H2 > 0])
  GemmArgs g = gemm_blank();
  g.A = ws->G3;
  g.lda = ws->k16;
  g.B = ws->W3N;
  g.ldb = ws->k16;
  g.M = n;
  g.N = ws->h2;
  g.K = k;
  g.kchunk = rup(k, 16);
  g.mask = ws->H2;
  g.ldm = ws->h2;
  g.Cb = ws->G2;
  g.ldcb = ws->h2;
  g.Ct = ws->G2T;
  g.ldct = ws->npad;
  ST_TRY(launch_gemm(ctx, g, false, 1));
  // layer 2: dW2 = H1^T G2, db2 = sum G2
  ST_TRY(weight_grad(ctx, ws, ws->H1T, ws->h1, ws->G2T, ws->h2, n, gr + ws->off[2]));
  row_sum_kernel<<<(unsigned)ws->h2, 256, 0, ctx->stream>>>(ws->G2T, ws->npad, n, gr + ws->off[3]);
  LAUNCH_CHECK(ctx);
  // G1 = bf16((G2 W2^T) * [H1 > 0]), transposed copy only
  g = gemm_blank();
  g.A = ws->G2;
  g.lda = ws->h2;
  g.B = ws->W2N;
  g.ldb = ws->h2;
  g.M = n;
  g.N = ws->h1;
  g.K = ws->h2;
  g.kchunk = ws->h2;
  g.mask = ws->H1;
  g.ldm = ws->h1;
  g.Ct = ws->G1T;
  g.ldct = ws->npad;
  ST_TRY(launch_gemm(ctx, g, false, 1));
  // layer 1: dW1 = bf16(U)^T G1, db1 = sum G1
  ST_TRY(weight_grad(ctx, ws, ws->UT, ws->d, ws->G1T, ws->h1, n, gr + ws->off[0]));
  row_sum_kernel<<<(unsigned)ws->h1, 256, 0, ctx->stream>>>(ws->G1T, ws->npad, n, gr + ws->off[1]);
  LAUNCH_CHECK(ctx);
  if (loss) {
    double s = 0.0;
    HIP_TRY(ctx, hipMemcpyAsync(&s, ws->lsum, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    *loss = s / (double)n;
  }
  return ANCKA_OK;
}

ancka_status ancka_ws_step(ancka_ctx* ctx, ancka_ws* ws, double lr) {
  ST_TRY(check_ws(ctx, ws));
  if (!(lr > 0.0)) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_step: lr=%g", lr);
  ws->t += 1;
  const double c1 = 1.0 / (1.0 - std::pow(0.9, (double)ws->t));
  const double c2 = 1.0 / (1.0 - std::pow(0.999, (double)ws->t));
  adam_kernel<<<nblk(ws->count), 256, 0, ctx->stream>>>(ws->master, ws->grad, ws->am, ws->av, ws->count, (float)lr,
                                                        (float)c1, (float)c2);
  LAUNCH_CHECK(ctx);
  return refresh_bf16(ctx, ws);
}

ancka_status ancka_ws_target(ancka_ctx* ctx, const void* Q, int32_t qdtype, int64_t n, int32_t k, int64_t ldq,
                             const double* R, const int32_t* colmap, float* T) {
  if (!ctx) return ANCKA_ERR_INVALID_ARG;
  if (!Q || !R || !colmap || !T) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_target: null argument");
  if (k < 1 || k > 64 || n < 1 || ldq < k || (qdtype != ANCKA_F32 && qdtype != ANCKA_F64))
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_target: n=%lld k=%d ldq=%lld qdtype=%d", (long long)n, k,
                   (long long)ldq, qdtype);
  std::vector<int> seen(k, 0);
  for (int c = 0; c < k; c++) {
    if (colmap[c] < 0 || colmap[c] >= k || seen[colmap[c]]++)
      return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ws_target: colmap is not a permutation of 0..%d", k - 1);
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  double* Rd = nullptr;
  int32_t* cmd = nullptr;
  ST_TRY(ws_get_t(ctx, "ws_target_R", (size_t)k * k, &Rd));
  ST_TRY(ws_get_t(ctx, "ws_target_map", (size_t)k, &cmd));
  HIP_TRY(ctx, hipMemcpyAsync(Rd, R, (size_t)k * k * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(cmd, colmap, (size_t)k * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  if (qdtype == ANCKA_F64)
    target_kernel<double><<<nblk(n), 256, 0, ctx->stream>>>((const double*)Q, n, k, ldq, Rd, cmd, T);
  else
    target_kernel<float><<<nblk(n), 256, 0, ctx->stream>>>((const float*)Q, n, k, ldq, Rd, cmd, T);
  LAUNCH_CHECK(ctx);
  // the host arrays may be reused once the copies have been consumed
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return ANCKA_OK;
}

}  // extern "C"
