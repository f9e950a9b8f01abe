// Thin QR of the iterated block (Eq. ortho-iter) by Cholesky QR with an FP64 Gram matrix and
// FP64 Cholesky, and the orthogonal iteration / starting block built on it (Alg. 4 lines
// 12-15).
//
// Q R = Z with diag(R) > 0 is unique for a full-rank Z.  With the Gram G = Z^T Z formed in
// FP64 from FP32 data (exact products, FP64 sums) one Cholesky pass loses only about
// kappa(Z)^2 u_64 of orthogonality, below the FP32 rounding of the stored Q; a second pass
// (Q <- Q R2^-1, R <- R2 R1) runs on the device whenever the first factorisation needed a
// diagonal shift or saw a pivot below 1e-8 of its diagonal entry, and always for FP64 blocks.
// The second-pass kernels read a device flag and exit at once when it is not set, so the
// whole step is enqueued without a host synchronisation.
#include <cmath>
#include <vector>

#include "common.h"

namespace {

constexpr int GR_ROWS = 32;  // rows staged per step of the Gram kernel

// Partial Gram of a row range.  The kp x kp result is cut into 4 x 4 blocks; only the blocks on
// or above the diagonal are computed (nt (nt + 1) / 2 of them, nt = ceil(kp / 4), one per thread,
// packed into the first threads) and each is also written mirrored.  fma is symmetric in its
// two factors and every block adds the rows in the same order, so the mirrored values are the
// bits the block below the diagonal would have produced.  Entries beyond kp are written as 0.
template <typename T>
__global__ __launch_bounds__(256) void gram_partial_kernel(const T* __restrict__ Z, int64_t n, int kp, int64_t ld,
                                                           int64_t rows_per_block, double* __restrict__ part,
                                                           const int* __restrict__ active) {
  if (active && *active == 0) return;
  __shared__ __align__(16) double zs[GR_ROWS][64 + 2];   // 16-byte aligned rows
  const int tid = threadIdx.x;
  const int nt = (kp + 3) / 4;
  const int npairs = nt * (nt + 1) / 2;
  int ty = 0, tx = tid;   // the thread's block (ty <= tx) when tid < npairs
  while (ty < nt && tx >= nt - ty) {
    tx -= nt - ty;
    ty++;
  }
  tx += ty;
  const bool mine = tid < npairs;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = (r0 + rows_per_block < n) ? r0 + rows_per_block : n;
  // the next chunk of rows is loaded into registers while the current one is multiplied
  constexpr int PER = GR_ROWS * 64 / 256;
  T pre[PER];
  auto load = [&](int64_t s) {
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      const int rr = e / 64, cc = e % 64;
      const int64_t row = s + rr;
      pre[u] = (row < r1 && cc < kp) ? Z[row * ld + cc] : (T)0;
    }
  };
  if (r0 < r1) load(r0);
  for (int64_t s = r0; s < r1; s += GR_ROWS) {
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      zs[e / 64][e % 64] = (double)pre[u];
    }
    __syncthreads();
    if (s + GR_ROWS < r1) load(s + GR_ROWS);
    if (mine) {
      for (int rr = 0; rr < GR_ROWS; rr++) {
        const double2 a01 = *(const double2*)&zs[rr][ty * 4];
        const double2 a23 = *(const double2*)&zs[rr][ty * 4 + 2];
        const double2 b01 = *(const double2*)&zs[rr][tx * 4];
        const double2 b23 = *(const double2*)&zs[rr][tx * 4 + 2];
        const double a[4] = {a01.x, a01.y, a23.x, a23.y};
        const double b[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++) acc[i][j] = fma(a[i], b[j], acc[i][j]);
      }
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.x * 64 * 64;
  if (mine) {
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        out[(ty * 4 + i) * 64 + tx * 4 + j] = acc[i][j];
        out[(tx * 4 + j) * 64 + ty * 4 + i] = acc[i][j];
      }
  }
  // blocks outside the nt x nt grid: zeros (thread = block (tid / 16, tid % 16) of the 16 x 16 grid)
  const int oy = tid / 16, ox = tid % 16;
  if (oy >= nt || ox >= nt) {
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) out[(oy * 4 + i) * 64 + ox * 4 + j] = 0.0;
  }
}

// fixed-order sum of the per-block partials
__global__ void gram_reduce_kernel(const double* __restrict__ part, int nblocks, double* __restrict__ G,
                                   const int* __restrict__ active) {
  if (active && *active == 0) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 64 * 64) return;
  // eight loads in flight ahead of the additions, which keep their order (bit-identical sums)
  double s = 0.0;
  int b = 0;
  for (; b + 8 <= nblocks; b += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = part[(int64_t)(b + u) * 64 * 64 + e];
#pragma unroll
    for (int u = 0; u < 8; u++) s += v[u];
  }
  for (; b < nblocks; b++) s += part[(int64_t)b * 64 * 64 + e];
  G[e] = s;
}

// Cholesky G = R^T R on one workgroup; writes R (upper, kp x kp in a 64x64 array) and R^-1.
// flags[0] (out): 1 when a second pass is required; flags[1] |= 1 on breakdown after a shift.
// force2: the second pass is always requested.  active: nullable device flag.
__global__ __launch_bounds__(256) void chol_kernel(const double* __restrict__ Gin, int kp, int64_t n,
                                                   double* __restrict__ R, double* __restrict__ Rinv,
                                                   int* __restrict__ flags, int force2, const int* __restrict__ active,
                                                   int set_flag) {
  if (active && *active == 0) return;
  __shared__ double G[64][65];
  __shared__ double L[64][65];
  __shared__ int s_bad;
  __shared__ double s_minratio;
  const int tid = threadIdx.x;
  int shifted = 0;
  for (int attempt = 0; attempt < 2; attempt++) {
    shifted = attempt;
    for (int e = tid; e < 64 * 64; e += 256) {
      const int i = e / 64, j = e % 64;
      G[i][j] = (i < kp && j < kp) ? Gin[i * 64 + j] : 0.0;
      L[i][j] = 0.0;
    }
    if (tid == 0) {
      s_bad = 0;
      s_minratio = 1.0;
    }
    __syncthreads();
    if (attempt == 1) {
      // shift of Fukaya et al. (shifted Cholesky QR): s = 11 (n kp + kp (kp + 1)) u tr(G)
      double tr = 0.0;
      for (int j = 0; j < kp; j++) tr += G[j][j];
      const double sft = 11.0 * ((double)n * kp + (double)kp * (kp + 1)) * ldexp(1.0, -53) * tr;
      __syncthreads();
      if (tid < kp) G[tid][tid] += sft;
      __syncthreads();
    }
    for (int j = 0; j < kp; j++) {
      if (tid == 0) {
        const double d = G[j][j];
        const double orig = Gin[j * 64 + j];
        if (!(d > 0.0) || !(d > 1e-15 * orig)) {
          s_bad = 1;
          L[j][j] = 1.0;
        } else {
          L[j][j] = sqrt(d);
          const double ratio = orig > 0.0 ? d / orig : 0.0;
          if (ratio < s_minratio) s_minratio = ratio;
        }
      }
      __syncthreads();
      const double ljj = L[j][j];
      for (int i = j + 1 + tid; i < kp; i += 256) L[i][j] = G[i][j] / ljj;
      __syncthreads();
      const int rem = kp - j - 1;
      for (int e = tid; e < rem * rem; e += 256) {
        const int i = j + 1 + e / rem, k = j + 1 + e % rem;
        G[i][k] -= L[i][j] * L[k][j];
      }
      __syncthreads();
    }
    if (s_bad == 0) break;
    if (attempt == 1) break;
    __syncthreads();
  }
  // R = L^T; Rinv = R^-1 column by column (upper triangular), columns held in G's storage
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    R[e] = (i < kp && j < kp && i <= j) ? L[j][i] : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    const int c = tid;
    // back substitution R x = e_c, x_i = 0 for i > c; thread c touches only column c of G
    for (int i = 63; i >= 0; i--) {
      double v = 0.0;
      if (i <= c && c < kp) {
        v = (i == c) ? 1.0 : 0.0;
        for (int k = i + 1; k <= c; k++) v -= L[k][i] * G[k][c];
        v /= L[i][i];
      }
      G[i][c] = v;
    }
    for (int i = 0; i < 64; i++) Rinv[i * 64 + c] = G[i][c];
  }
  if (tid == 0 && set_flag) {
    const bool need2 = force2 || s_bad || shifted || s_minratio < 1e-8;
    flags[0] = need2 ? 1 : 0;
    if (s_bad) flags[1] |= 1;   // shifted (first pass) or broke down (second pass)
  }
  if (tid == 0 && !set_flag && s_bad) flags[1] |= 2;
}

// Q[i, :] = Z[i, :] R^-1 in FP64 arithmetic; dq partial = sum ||Q_i - Qprev_i||^2 per block.
// 16-byte vector of T
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; static constexpr int W = 4; };
template <> struct Vec16<double> { typedef double2 type; static constexpr int W = 2; };

template <typename T>
__device__ __forceinline__ T vget(const typename Vec16<T>::type& v, int i);
template <>
__device__ __forceinline__ float vget<float>(const float4& v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
template <>
__device__ __forceinline__ double vget<double>(const double2& v, int i) {
  return i == 0 ? v.x : v.y;
}

// Q = Z R^{-1} row by row in FP64 (one thread per row).  With vec, rows are read (Z and Q(t-1))
// and written (whole vectors below kp) in 16-byte vectors: ld is then a multiple of the vector
// width, at least KPM, and the base pointers are 16-byte aligned.
template <typename T, int KPM>
__global__ __launch_bounds__(256) void apply_rinv_kernel(const T* __restrict__ Z, T* __restrict__ Q, int64_t n, int kp,
                                                         int64_t ld, const double* __restrict__ Rinv,
                                                         const T* __restrict__ Qprev, double* __restrict__ dq_part,
                                                         const int* __restrict__ active, int vec) {
  if (active && *active == 0) return;
  __shared__ double red[256];
  const int tid = threadIdx.x;
  // R^-1 is read with addresses that are the same in every lane (scalar loads); only entries
  // (c, j) with c <= j < kp reach a stored output
  const double* __restrict__ Rg = Rinv;
#define Rs(c, j) Rg[(c) * 64 + (j)]
  const int64_t r = (int64_t)blockIdx.x * 256 + tid;
  double dq = 0.0;
  // (the last row goes element by element: its vectors could run past kp to the end of ld, which
  // a caller's buffer need not hold for the last row)
  if (r + 1 < n && vec) {
    typedef typename Vec16<T>::type VT;
    constexpr int VW = Vec16<T>::W;
    double z[KPM];
#pragma unroll
    for (int c0 = 0; c0 < KPM; c0 += VW) {
      const VT v = *(const VT*)(Z + r * ld + c0);
#pragma unroll
      for (int u = 0; u < VW; u++) z[c0 + u] = (c0 + u < kp) ? (double)vget<T>(v, u) : 0.0;
    }
#pragma unroll
    for (int j0 = 0; j0 < KPM; j0 += VW) {
      T qv[VW];
      // the VW sums advance together over c (each keeps its own order c = 0 .. j)
      double sv[VW];
#pragma unroll
      for (int u = 0; u < VW; u++) sv[u] = 0.0;
#pragma unroll
      for (int c = 0; c < j0 + VW; c++)
#pragma unroll
        for (int u = 0; u < VW; u++)
          if (c <= j0 + u) sv[u] = fma(z[c], Rs(c, j0 + u), sv[u]);
#pragma unroll
      for (int u = 0; u < VW; u++) qv[u] = (T)sv[u];
      if (j0 < kp) {
        if (Qprev) {
          const VT pv = *(const VT*)(Qprev + r * ld + j0);
#pragma unroll
          for (int u = 0; u < VW; u++)
            if (j0 + u < kp) {
              const double dd = (double)qv[u] - (double)vget<T>(pv, u);
              dq = fma(dd, dd, dq);
            }
        }
        if (j0 + VW <= kp) {
          VT o;
          T* op = (T*)&o;
#pragma unroll
          for (int u = 0; u < VW; u++) op[u] = qv[u];
          *(VT*)(Q + r * ld + j0) = o;
        } else {
#pragma unroll
          for (int u = 0; u < VW; u++)
            if (j0 + u < kp) Q[r * ld + j0 + u] = qv[u];
        }
      }
    }
  } else if (r < n) {
    double z[KPM];
#pragma unroll
    for (int c = 0; c < KPM; c++) z[c] = (c < kp) ? (double)Z[r * ld + c] : 0.0;
#pragma unroll
    for (int j = 0; j < KPM; j++) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c <= j; c++) s = fma(z[c], Rs(c, j), s);
      if (j < kp) {
        const T qv = (T)s;
        if (Qprev) {
          const double dd = (double)qv - (double)Qprev[r * ld + j];
          dq = fma(dd, dd, dq);
        }
        Q[r * ld + j] = qv;
      }
    }
  }
  if (dq_part) {
    red[tid] = dq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) dq_part[blockIdx.x] = red[0];
  }
#undef Rs
}

__global__ void sum_partials_kernel(const double* __restrict__ part, int64_t count, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// R = R2 R1 when the second pass ran, else R1 (both upper, 64x64 storage)
__global__ void combine_r_kernel(const double* __restrict__ R1, const double* __restrict__ R2, int kp,
                                 const int* __restrict__ flags, double* __restrict__ R) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 64 * 64) return;
  const int i = e / 64, j = e % 64;
  if (flags[0] == 0) {
    R[e] = R1[e];
    return;
  }
  double s = 0.0;
  for (int k = i; k <= j && k < kp; k++) s += R2[i * 64 + k] * R1[k * 64 + j];
  R[e] = (i < kp && j < kp) ? s : 0.0;
}

template <typename T>
ancka_status launch_apply(ancka_ctx* ctx, const T* Z, T* Q, int64_t n, int kp, int64_t ld, const double* Rinv,
                          const T* Qprev, double* dq_part, const int* active) {
  const unsigned grid = (unsigned)cdiv(n, 256);
  // the kernel computes every column below KPM (fully unrolled), so KPM follows kp closely
  const int kpm = kp <= 8 ? 8 : kp <= 16 ? 16 : kp <= 32 ? 32 : kp <= 40 ? 40 : kp <= 48 ? 48 : kp <= 52 ? 52 : kp <= 56 ? 56 : 64;
  const int vw = 16 / (int)sizeof(T);
  const auto al16 = [](const void* p) { return p == nullptr || ((uintptr_t)p % 16) == 0; };
  const int vec = (ld % vw == 0 && ld >= kpm && al16(Z) && al16(Q) && al16(Qprev)) ? 1 : 0;
  if (kp <= 8)
    apply_rinv_kernel<T, 8><<<grid, 256, 0, ctx->stream>>>(Z, Q, n, kp, ld, Rinv, Qprev, dq_part, active, vec);
  else if (kp <= 16)
    apply_rinv_kernel<T, 16><<<grid, 256, 0, ctx->stream>>>(Z, Q, n, kp, ld, Rinv, Qprev, dq_part, active, vec);
  else if (kp <= 32)
    apply_rinv_kernel<T, 32><<<grid, 256, 0, ctx->stream>>>(Z, Q, n, kp, ld, Rinv, Qprev, dq_part, active, vec);
  else if (kp <= 40)
    apply_rinv_kernel<T, 40><<<grid, 256, 0, ctx->stream>>>(Z, Q, n, kp, ld, Rinv, Qprev, dq_part, active, vec);
  else if (kp <= 48)
    apply_rinv_kernel<T, 48><<<grid, 256, 0, ctx->stream>>>(Z, Q, n, kp, ld, Rinv, Qprev, dq_part, active, vec);
  else if (kp <= 52)
    apply_rinv_kernel<T, 52><<<grid, 256, 0, ctx->stream>>>(Z, Q, n, kp, ld, Rinv, Qprev, dq_part, active, vec);
  else if (kp <= 56)
    apply_rinv_kernel<T, 56><<<grid, 256, 0, ctx->stream>>>(Z, Q, n, kp, ld, Rinv, Qprev, dq_part, active, vec);
  else
    apply_rinv_kernel<T, 64><<<grid, 256, 0, ctx->stream>>>(Z, Q, n, kp, ld, Rinv, Qprev, dq_part, active, vec);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

template <typename T>
ancka_status gram(ancka_ctx* ctx, const T* Z, int64_t n, int kp, int64_t ld, double* G, const int* active) {
  int64_t nblocks = 4 * (int64_t)ctx->num_cu;
  int64_t rpb = cdiv(n, nblocks);
  rpb = cdiv(rpb, GR_ROWS) * GR_ROWS;
  nblocks = cdiv(n, rpb);
  double* part = nullptr;
  ST_TRY(ws_get_t(ctx, "qr_gpart", (size_t)nblocks * 64 * 64, &part));
  gram_partial_kernel<T><<<(unsigned)nblocks, 256, 0, ctx->stream>>>(Z, n, kp, ld, rpb, part, active);
  LAUNCH_CHECK(ctx);
  gram_reduce_kernel<<<16, 256, 0, ctx->stream>>>(part, (int)nblocks, G, active);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

template <typename T>
ancka_status qr_typed(ancka_ctx* ctx, const T* Z, T* Qout, int64_t n, int kp, int64_t ld, const T* Qprev,
                      double* dq2_dev, double* R_out, bool force2) {
  double *G = nullptr, *R1 = nullptr, *Ri1 = nullptr, *R2 = nullptr, *Ri2 = nullptr, *dqp = nullptr;
  int* flags = nullptr;
  ST_TRY(ws_get_t(ctx, "qr_mats", (size_t)5 * 64 * 64, &G));
  R1 = G + 64 * 64;
  Ri1 = R1 + 64 * 64;
  R2 = Ri1 + 64 * 64;
  Ri2 = R2 + 64 * 64;
  ST_TRY(ws_get_t(ctx, "qr_flags", 4, &flags));
  const int64_t nb = cdiv(n, 256);
  if (dq2_dev) ST_TRY(ws_get_t(ctx, "qr_dqpart", (size_t)nb, &dqp));
  // pass 1
  ST_TRY(gram<T>(ctx, Z, n, kp, ld, G, nullptr));
  chol_kernel<<<1, 256, 0, ctx->stream>>>(G, kp, n, R1, Ri1, flags, force2 ? 1 : 0, nullptr, 1);
  LAUNCH_CHECK(ctx);
  ST_TRY(launch_apply<T>(ctx, Z, Qout, n, kp, ld, Ri1, Qprev, dqp, nullptr));
  // pass 2 (device-conditional)
  ST_TRY(gram<T>(ctx, Qout, n, kp, ld, G, flags));
  chol_kernel<<<1, 256, 0, ctx->stream>>>(G, kp, n, R2, Ri2, flags, 0, flags, 0);
  LAUNCH_CHECK(ctx);
  ST_TRY(launch_apply<T>(ctx, Qout, Qout, n, kp, ld, Ri2, Qprev, dqp, flags));
  if (dq2_dev) {
    sum_partials_kernel<<<1, 256, 0, ctx->stream>>>(dqp, nb, dq2_dev);
    LAUNCH_CHECK(ctx);
  }
  if (R_out) {
    combine_r_kernel<<<16, 256, 0, ctx->stream>>>(R1, R2, kp, flags, R_out);
    LAUNCH_CHECK(ctx);
  }
  return ANCKA_OK;
}

// Q0 = [1/sqrt(n) 1 | h(Y)] with fill columns, or [1/sqrt(n) 1 | Zwarm]
template <typename T>
__global__ void build_q0_kernel(T* __restrict__ Q, int64_t n, int k, int64_t ld, const int32_t* __restrict__ labels,
                                const int32_t* __restrict__ counts, const float* __restrict__ zwarm,
                                const int* __restrict__ fill_col) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Q[i * ld] = (T)(1.0 / sqrt((double)n));
  for (int j = 1; j <= k; j++) {
    double v;
    if (fill_col[j]) {
      v = cos(M_PI * ((double)i + 0.5) * (double)j / (double)n);
    } else if (zwarm) {
      v = (double)zwarm[i * k + (j - 1)];
    } else {
      v = (labels[i] == j - 1) ? 1.0 / sqrt((double)counts[j - 1]) : 0.0;
    }
    Q[i * ld + j] = (T)v;
  }
  for (int64_t j = k + 1; j < ld; j++) Q[i * ld + j] = (T)0;
}

// per-block histogram in LDS, then one global add per non-empty bin (integer: order-free)
__global__ __launch_bounds__(256) void count_labels_kernel(const int32_t* __restrict__ labels, int64_t n, int k,
                                                           int32_t* __restrict__ counts, int* __restrict__ bad) {
  __shared__ int h[64];
  if (threadIdx.x < 64) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * 4096;
  for (int u = 0; u < 16; u++) {
    const int64_t i = base + (int64_t)u * 256 + threadIdx.x;
    if (i >= n) break;
    const int l = labels[i];
    if (l < 0 || l >= k) atomicOr(bad, 1);
    else atomicAdd(&h[l], 1);
  }
  __syncthreads();
  if ((int)threadIdx.x < k && h[threadIdx.x] != 0) atomicAdd(&counts[threadIdx.x], h[threadIdx.x]);
}

}  // namespace

ancka_status qr_block(ancka_ctx* ctx, int dtype, const void* Z, void* Qout, int64_t n, int kp, int64_t ld,
                      const void* Qprev, double* dq2_dev, double* R_out) {
  if (dtype == ANCKA_F64)
    return qr_typed<double>(ctx, (const double*)Z, (double*)Qout, n, kp, ld, (const double*)Qprev, dq2_dev, R_out,
                            true);
  return qr_typed<float>(ctx, (const float*)Z, (float*)Qout, n, kp, ld, (const float*)Qprev, dq2_dev, R_out, false);
}

// counts[c] = |{i : labels[i] = c}| (device); *bad set for out-of-range labels
ancka_status count_labels(ancka_ctx* ctx, const int32_t* labels, int64_t n, int k, int32_t* counts, int* bad) {
  ST_TRY(fill_zero(ctx, counts, sizeof(int32_t) * k));
  count_labels_kernel<<<(unsigned)cdiv(n, 4096), 256, 0, ctx->stream>>>(labels, n, k, counts, bad);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

ancka_status initial_block(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels, const float* zwarm, int k,
                           void* Q, int64_t ldq) {
  const int64_t n = op->n;
  int32_t* counts = nullptr;
  int* bad = nullptr;
  int* fill = nullptr;
  ST_TRY(ws_get_t(ctx, "ib_counts", 64, &counts));
  ST_TRY(ws_get_t(ctx, "ib_bad", 4, &bad));
  ST_TRY(ws_get_t(ctx, "ib_fill", 72, &fill));
  std::vector<int> hfill(72, 0);
  if (labels) {
    ST_TRY(fill_zero(ctx, bad, 16));
    ST_TRY(count_labels(ctx, labels, n, k, counts, bad));
    std::vector<int32_t> hc(k);
    int hbad = 0;
    HIP_TRY(ctx, hipMemcpyAsync(hc.data(), counts, sizeof(int32_t) * k, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (hbad) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "initial block: label outside [0, k)");
    // zero columns (empty clusters) and the column of the last non-empty cluster, which lies in
    // the span of the constant column and the other cluster columns, take the fill vector
    int last = -1;
    for (int c = 0; c < k; c++) {
      if (hc[c] == 0) hfill[c + 1] = 1;
      else last = c;
    }
    if (last >= 0) hfill[last + 1] = 1;
  }
  HIP_TRY(ctx, hipMemcpyAsync(fill, hfill.data(), sizeof(int) * 72, hipMemcpyHostToDevice, ctx->stream));
  // the host array dies with this call: the copy must have read it before returning
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  void* Z = nullptr;
  const size_t es = op->dtype == ANCKA_F64 ? 8 : 4;
  ST_TRY(ws_get(ctx, "ib_Z", (size_t)n * ldq * es, &Z));
  if (op->dtype == ANCKA_F64)
    build_q0_kernel<double><<<(unsigned)cdiv(n, 256), 256, 0, ctx->stream>>>((double*)Z, n, k, ldq, labels, counts, zwarm,
                                                                             fill);
  else
    build_q0_kernel<float><<<(unsigned)cdiv(n, 256), 256, 0, ctx->stream>>>((float*)Z, n, k, ldq, labels, counts, zwarm,
                                                                            fill);
  LAUNCH_CHECK(ctx);
  // two Cholesky QR passes: the first, on a block that mixes a constant column with cluster
  // indicators, is only moderately conditioned
  if (op->dtype == ANCKA_F64)
    return qr_typed<double>(ctx, (const double*)Z, (double*)Q, n, k + 1, ldq, nullptr, nullptr, nullptr, true);
  return qr_typed<float>(ctx, (const float*)Z, (float*)Q, n, k + 1, ldq, nullptr, nullptr, nullptr, true);
}

extern "C" {

ancka_status ancka_initial_block(ancka_ctx* ctx, const ancka_op* op, const int32_t* labels, const float* zwarm,
                                 int32_t k, void* Q, int64_t ldq) {
  if (!ctx || !op || !Q || (!labels && !zwarm)) return ANCKA_ERR_INVALID_ARG;
  const int vw = op->dtype == ANCKA_F64 ? 2 : 4;
  if (k < 1 || k + 1 > 64 || k > op->n || ldq < k + 1 || ldq % vw != 0)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_initial_block: k=%d ldq=%lld", k, (long long)ldq);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  return initial_block(ctx, op, labels, zwarm, k, Q, ldq);
}

ancka_status ancka_orth_iter(ancka_ctx* ctx, const ancka_op* op, void* Q, int64_t ldq, int32_t kp1, int32_t iters,
                             double* R_last, double* dq_fro) {
  if (!ctx || !op || !Q) return ANCKA_ERR_INVALID_ARG;
  const int vw = op->dtype == ANCKA_F64 ? 2 : 4;
  if (kp1 < 2 || kp1 > 64 || ldq < kp1 || ldq % vw != 0 || iters < 0)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_orth_iter: kp1=%d ldq=%lld iters=%d", kp1, (long long)ldq, iters);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  const int64_t n = op->n;
  const size_t es = op->dtype == ANCKA_F64 ? 8 : 4;
  void *Z = nullptr, *Qp = nullptr;
  double* dev = nullptr;
  int* flags = nullptr;
  ST_TRY(ws_get(ctx, "oi_Z", (size_t)n * ldq * es, &Z));
  ST_TRY(ws_get(ctx, "oi_Qprev", (size_t)n * ldq * es, &Qp));
  ST_TRY(ws_get_t(ctx, "oi_out", 64 * 64 + 2, &dev));
  ST_TRY(ws_get_t(ctx, "qr_flags", 4, &flags));
  ST_TRY(fill_zero(ctx, flags, 16));
  for (int t = 0; t < iters; t++) {
    const bool last = t == iters - 1;
    ST_TRY(op_apply(ctx, op, Q, Z, kp1, ldq));
    if (last && dq_fro) HIP_TRY(ctx, hipMemcpyAsync(Qp, Q, (size_t)n * ldq * es, hipMemcpyDeviceToDevice, ctx->stream));
    ST_TRY(qr_block(ctx, op->dtype, Z, Q, n, kp1, ldq, (last && dq_fro) ? Qp : nullptr, (last && dq_fro) ? dev : nullptr,
                    (last && R_last) ? dev + 2 : nullptr));
  }
  std::vector<double> h(64 * 64 + 2, 0.0);
  int hflags[4] = {0, 0, 0, 0};
  HIP_TRY(ctx, hipMemcpyAsync(h.data(), dev, sizeof(double) * (64 * 64 + 2), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (hflags[1] & 2) return set_err(ctx, ANCKA_ERR_NUMERICAL, "ancka_orth_iter: Cholesky QR broke down");
  if (iters > 0) {
    if (dq_fro) *dq_fro = sqrt(h[0]);
    if (R_last)
      for (int i = 0; i < kp1; i++)
        for (int j = 0; j < kp1; j++) R_last[i * kp1 + j] = h[2 + i * 64 + j];
  }
  return ANCKA_OK;
}

}  // extern "C"
