// Discretize (Sec. 7: Definition 2, Eqs. updateY and svd-in-discr, Alg. 5) on gfx950.
//
// Per step two kernels run:
//  disc_pass  one thread per row: q~ = q / |q| (zero rows stay zero), t = q~ R, label = first
//             argmax of t; the row is added to its cluster's sum S[label] and count.  The sums
//             are kept in 2^-s fixed point (|q~_c| <= 1) with 64-bit integer atomics, so
//             they are exact and independent of the order in which rows arrive; s = 40, or
//             62 - ceil(log2 n) when n > 2^22, so that n rows of magnitude <= 2^s cannot
//             reach 2^63.
//  disc_svd   one workgroup: M = S / count (rows of M are cluster means of q~, i.e. Y~^T Q~ with
//             the column sums of Y as divisors); R = V U^T and trace(Omega) of M = U Omega V^T,
//             in FP64; obj = n - 2 trace(Omega); sets a device flag when |obj - obj_prev| <=
//             1e-12 max(1, |obj|).  Later steps see the flag and return at once, so labels
//             keep the values of the last argmax, as Alg. 5 returns them.  R is the orthogonal
//             polar factor of M^T: with every cluster non-empty it comes from a Newton-Schulz
//             iteration (k x k products), otherwise -- or if that does not converge -- from a
//             one-sided Jacobi SVD (Hestenes).
// In the Jacobi SVD, singular vectors of (numerically) zero singular values -- e.g. an empty
// cluster -- are completed deterministically: each takes the standard basis vector with the
// largest residual against the columns before it (smaller index on ties), orthogonalised twice.
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"

namespace {

// 2^s of the fixed-point cluster sums: n (2^s + 1) < 2^63 for every n < 2^31.
inline double fix_scale(int64_t n) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < n) b++;   // 2^b >= n
  const int s = b > 22 ? 62 - b : 40;
  return std::ldexp(1.0, s);
}

struct DiscState {
  int done;
  int iters;
  double obj;
  double obj_prev;
};

// OFF = 0 or 1: the rows of Q are read in 16-byte vectors from Q - OFF (16-byte aligned, ldq a
// multiple of the vector width, OFF + k <= ldq; the block's first column is then usually the
// column before Q); OFF = -1: element by element.
template <typename T, int KM, int OFF>
__global__ __launch_bounds__(256) void disc_pass_kernel(const T* __restrict__ Q, int64_t n, int k, int64_t ldq,
                                                        const T* __restrict__ R, int32_t* __restrict__ labels,
                                                        unsigned long long* __restrict__ Sg,
                                                        unsigned int* __restrict__ cg,
                                                        const DiscState* __restrict__ st, double fscale) {
  if (st->done) return;
  __shared__ unsigned long long Ss[KM * KM];   // Ss[c][label]: lanes of different labels hit different banks
  __shared__ unsigned int cs[KM];
  const int tid = threadIdx.x;
  for (int e = tid; e < KM * KM; e += 256) Ss[e] = 0ull;
  if (tid < KM) cs[tid] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  if (i < n) {
    T q[KM];
    double nr = 0.0;
    // (the last row is read element by element: its vectors could run past the rows' k columns
    // to the end of ldq, which a caller's buffer need not hold for the last row)
    if (OFF >= 0 && i + 1 < n) {
      constexpr int W = 16 / sizeof(T);
      constexpr int OF = OFF >= 0 ? OFF : 0;
      constexpr int NV = (KM + OF + W - 1) / W;
      T raw[NV * W];
      const T* base = Q - OF + i * ldq;
#pragma unroll
      for (int v = 0; v < NV; v++) {
        if (v * W < OF + k) {
          if constexpr (W == 4) {
            const float4 x = *(const float4*)(base + v * W);
            raw[v * W] = x.x; raw[v * W + 1] = x.y; raw[v * W + 2] = x.z; raw[v * W + 3] = x.w;
          } else {
            const double2 x = *(const double2*)(base + v * W);
            raw[v * W] = x.x; raw[v * W + 1] = x.y;
          }
        } else {
#pragma unroll
          for (int u = 0; u < W; u++) raw[v * W + u] = (T)0;
        }
      }
#pragma unroll
      for (int c = 0; c < KM; c++) q[c] = (c < k) ? raw[c + OF] : (T)0;
    } else {
#pragma unroll
      for (int c = 0; c < KM; c++) q[c] = (c < k) ? Q[i * ldq + c] : (T)0;
    }
#pragma unroll
    for (int c = 0; c < KM; c++) nr += (double)q[c] * (double)q[c];
    if (nr > 0.0) {
      const T inv = (T)(1.0 / sqrt(nr));
#pragma unroll
      for (int c = 0; c < KM; c++) q[c] *= inv;
    }
    int best = 0;
    T bv = (T)0;
    constexpr int VW = 16 / sizeof(T);   // R entries per 16-byte LDS read
#pragma unroll
    for (int j = 0; j < KM; j++) {
      if (j < k) {
        T t = (T)0;
#pragma unroll
        for (int c = 0; c < KM; c += VW) {
          if (c >= k) continue;   // R^T rows are zero beyond column k
          // R^T row j from global memory at addresses every lane shares (scalar loads: a
          // broadcast read of LDS would cost a full 64-lane transfer per 16 bytes)
          T r[VW];
          if constexpr (VW == 4) {
            const float4 v = *(const float4*)(R + j * KM + c);
            r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w;
          } else {
            const double2 v = *(const double2*)(R + j * KM + c);
            r[0] = v.x; r[1] = v.y;
          }
#pragma unroll
          for (int u = 0; u < VW; u++) t = fma(q[c + u], r[u], t);
        }
        if (j == 0 || t > bv) {
          bv = t;
          best = j;
        }
      }
    }
    labels[i] = best;
    atomicAdd(&cs[best], 1u);
#pragma unroll
    for (int c = 0; c < KM; c++)
      if (c < k) {
        const long long f = llrint((double)q[c] * fscale);
        if (f != 0) atomicAdd(&Ss[c * KM + best], (unsigned long long)f);
      }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += 256) {
    const int a = e / k, b = e % k;
    const unsigned long long v = Ss[b * KM + a];
    if (v != 0ull) atomicAdd(&Sg[e], v);
  }
  if (tid < k && cs[tid] != 0u) atomicAdd(&cg[tid], cs[tid]);
}

__device__ __forceinline__ double sgn1(double x) { return x < 0.0 ? -1.0 : 1.0; }

// Columns of a k x k orthogonal factor stored as B[j][i].  Each column flagged in isnull is
// replaced, in increasing j, by the standard basis vector with the largest residual against the
// columns already in place (all non-null ones and the null ones completed before it), projected
// twice and normalised.  The k residual norms are computed by k threads at once (each in the
// same order as a serial loop); the choice and the projection are made by thread 0.  All threads
// of the workgroup call it (it has barriers); placed and n2 are k ints / doubles of LDS.
template <int KM>
__device__ void complete_null_cols(double (*B)[KM + 1], int k, const int* isnull, int tid, int* placed,
                                   double* n2) {
  if (tid < k) placed[tid] = !isnull[tid];
  __syncthreads();
  for (int j = 0; j < k; j++) {
    if (!isnull[j]) continue;
    if (tid < k) {
      const int i = tid;
      double s2 = 0.0;
      for (int a = 0; a < k; a++) {
        double w = (a == i) ? 1.0 : 0.0;
        for (int c = 0; c < k; c++)
          if (placed[c]) w -= B[c][a] * B[c][i];
        s2 += w * w;
      }
      n2[i] = s2;
    }
    __syncthreads();
    if (tid == 0) {
      int bi = 0;
      double bn = -1.0;
      for (int i = 0; i < k; i++)
        if (n2[i] > bn) {
          bn = n2[i];
          bi = i;
        }
      double w[KM];
      for (int a = 0; a < k; a++) w[a] = (a == bi) ? 1.0 : 0.0;
      for (int pass = 0; pass < 2; pass++)
        for (int c = 0; c < k; c++) {
          if (!placed[c]) continue;
          double dp = 0.0;
          for (int a = 0; a < k; a++) dp += B[c][a] * w[a];
          for (int a = 0; a < k; a++) w[a] -= dp * B[c][a];
        }
      double nn = 0.0;
      for (int a = 0; a < k; a++) nn += w[a] * w[a];
      nn = sqrt(nn);
      for (int a = 0; a < k; a++) B[j][a] = w[a] / nn;
      placed[j] = 1;
    }
    __syncthreads();
  }
}

// Sum and maximum over the 256 threads of a workgroup, the same value in every thread; the wave
// partials are combined in a fixed order, so repeated runs give the same bits.  red: 4 doubles
// of LDS.  The maximum keeps a NaN.
__device__ double block_sum4(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ __forceinline__ double max_nan(double a, double b) { return (a >= b || a != a) ? a : b; }

__device__ double block_max4(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max_nan(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return max_nan(max_nan(red[0], red[1]), max_nan(red[2], red[3]));
}

constexpr int NS_MAX_ITERS = 100;
constexpr double NS_TOL = 1e-10;   // max |X^T X - I| before the last update

template <typename T, int KM>
__global__ __launch_bounds__(256) void disc_svd_kernel(unsigned long long* __restrict__ Sg, unsigned int* __restrict__ cg,
                                                       int k, int64_t n, double* __restrict__ Rd, T* __restrict__ Rt,
                                                       DiscState* __restrict__ st, double fscale) {
  if (st->done) return;
  __shared__ double A[KM][KM + 1];   // A[j][i] = column j of M (then of M V)
  __shared__ double V[KM][KM + 1];   // V[j][i] = column j of V; X^T X in the Newton-Schulz path
  __shared__ double Xs[2][KM][KM + 1];
  __shared__ double red[4];
  __shared__ double sig[KM];
  __shared__ int isnull[KM];
  __shared__ int placed[KM];
  __shared__ double n2[KM];
  __shared__ int s_rot;
  const int tid = threadIdx.x;
  const int empty = __syncthreads_or(tid < k && cg[tid] == 0u);
  // M[c][j] = S[c][j] / (2^s count[c]); then clear S and counts for the next step
  for (int e = tid; e < KM * KM; e += 256) {
    const int c = e / KM, j = e % KM;
    double v = 0.0;
    if (c < k && j < k) {
      const unsigned int cnt = cg[c];
      const long long s = (long long)Sg[c * k + j];
      v = cnt ? ((double)s / fscale) / (double)cnt : 0.0;
    }
    A[j][c] = v;
    V[j][c] = (c == j && c < k) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += 256) Sg[e] = 0ull;
  if (tid < k) cg[tid] = 0u;

  // R = V U^T is the orthogonal polar factor of M^T, and trace(Omega) = trace(R M).  With every
  // cluster non-empty M is (in practice) nonsingular, and the Newton-Schulz iteration
  // X <- X (3I - X^T X) / 2 from X = M^T / s, s >= sigma_max(M) (singular values in (0, 1]),
  // converges to that factor: the singular vectors stay, the singular values go to 1.  Its steps
  // are scaled as by Chen and Chow (a stable scaling of Newton-Schulz), which speeds up the
  // growth of small singular values.  One plain update follows the first step with
  // max |X^T X - I| <= 1e-10.  If it does not get there (a singular M) the one-sided Jacobi SVD
  // below is used.
  double ssum = 0.0;
  bool polar = false;
  if (!empty) {
    // each thread owns rows tr + 16 r and columns tc + 16 s (r, s < 4) of the k x k products;
    // the iterates and V are zero outside the leading k x k block, so the products read them
    // without bounds checks (only a column index of KM or more, for KM < 64, is skipped)
    const int tr = tid >> 4, tc = tid & 15;
    auto at = [&](double (*X)[KM + 1], int i, int j) -> double {
      if constexpr (KM >= 64) return X[i][j];
      else return j < KM ? X[i][j] : 0.0;
    };
    // g = the thread's 4 x 4 block of X^T X
    auto gram = [&](double (*X)[KM + 1], double (&g)[4][4]) {
#pragma unroll
      for (int r = 0; r < 4; r++)
#pragma unroll
        for (int c = 0; c < 4; c++) g[r][c] = 0.0;
#pragma unroll 2
      for (int i = 0; i < k; i++) {
        double xa[4], xb[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          xa[r] = at(X, i, tr + 16 * r);
          xb[r] = at(X, i, tc + 16 * r);
        }
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
          for (int c = 0; c < 4; c++) g[r][c] = fma(xa[r], xb[c], g[r][c]);
      }
    };
    // Scale: sigma_max(M)^2 <= max_a sum_b |(M M^T)_ab| (Gershgorin on the Gram of X = M^T), which
    // is sharp when the cluster means are near orthogonal, so the iteration starts close to 1.
    double g[4][4];
    gram(A, g);
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
      for (int c = 0; c < 4; c++)
        if (tr + 16 * r < k && tc + 16 * c < k) V[tr + 16 * r][tc + 16 * c] = fabs(g[r][c]);
    __syncthreads();
    double rs = 0.0;
    if (tid < k)
      for (int b = 0; b < k; b++) rs += V[tid][b];
    const double bnd = block_max4(rs, red);
    // Gershgorin also bounds sigma_min^2 from below: min_a (2 G_aa - sum_b |G_ab|), when positive
    const double lneg = block_max4(tid < k ? rs - 2.0 * V[tid][tid] : -INFINITY, red);
    if (bnd > 0.0) {
      const double inv = 1.0 / sqrt(bnd);
      // ell: the assumed lower end of the singular values of X (all lie in (0, 1]); the bound
      // above, or 1e-3 when it is smaller (a guess: a wrong one costs steps, not accuracy)
      double ell = lneg < 0.0 ? sqrt(-lneg / bnd) : 0.0;
      ell = fmin(fmax(ell, 1e-3), 1.0);
      for (int e = tid; e < KM * KM; e += 256) {
        const int a = e / KM, b = e % KM;
        Xs[0][a][b] = (a < k && b < k) ? A[a][b] * inv : 0.0;
        Xs[1][a][b] = 0.0;
      }
      __syncthreads();
      int cur = 0;
      for (int it = 0; it < NS_MAX_ITERS; it++) {
        double (*X)[KM + 1] = Xs[cur];
        double (*Y)[KM + 1] = Xs[cur ^ 1];
        gram(X, g);
        double dm = 0.0;
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
          for (int c = 0; c < 4; c++) {
            const int a = tr + 16 * r, b = tc + 16 * c;
            if (a < k && b < k) {
              V[a][b] = g[r][c];
              dm = max_nan(dm, fabs(g[r][c] - (a == b ? 1.0 : 0.0)));
            }
          }
        dm = block_max4(dm, red);   // its barriers also publish V = X^T X
        const bool last = dm <= NS_TOL;
        // scaled step X <- (a/2) X (3I - a^2 X^T X) with a = sqrt(3 / (1 + ell + ell^2)): it maps
        // [ell, 1] onto [ell', 1] with ell' = f(ell) = f(1), and grows small singular values
        // by up to 3 sqrt(3) / 2 per step instead of 3/2; a -> 1 as ell -> 1.  The last step is
        // the plain one (a = 1).
        const double sa = last ? 1.0 : sqrt(3.0 / (1.0 + ell + ell * ell));
        const double c1 = 1.5 * sa, c3 = 0.5 * sa * sa * sa;
        ell = 0.5 * sa * ell * (3.0 - sa * sa * ell * ell);
        double y[4][4];
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
          for (int c = 0; c < 4; c++) y[r][c] = 0.0;
#pragma unroll 2
        for (int a = 0; a < k; a++) {
          double xr[4], gc[4];
#pragma unroll
          for (int r = 0; r < 4; r++) {
            xr[r] = (KM >= 64 || tr + 16 * r < KM) ? X[tr + 16 * r][a] : 0.0;
            gc[r] = at(V, a, tc + 16 * r);
          }
#pragma unroll
          for (int r = 0; r < 4; r++)
#pragma unroll
            for (int c = 0; c < 4; c++) y[r][c] = fma(xr[r], gc[c], y[r][c]);
        }
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
          for (int c = 0; c < 4; c++) {
            const int i = tr + 16 * r, b = tc + 16 * c;
            if (i < k && b < k) Y[i][b] = c1 * X[i][b] - c3 * y[r][c];
          }
        __syncthreads();
        cur ^= 1;
        if (last) {
          polar = true;
          break;
        }
      }
      if (polar) {
        double (*X)[KM + 1] = Xs[cur];
        double t = 0.0;
        for (int e = tid; e < k * k; e += 256) {
          const int a = e / k, b = e % k;
          t += X[a][b] * A[a][b];   // R[a][b] M[b][a]
          Rd[e] = X[a][b];
          Rt[b * KM + a] = (T)X[a][b];
        }
        ssum = block_sum4(t, red);
      }
    }
    if (!polar) {
      // V held scratch values: back to V = I for the Jacobi SVD
      for (int e = tid; e < KM * KM; e += 256) V[e / KM][e % KM] = (e / KM == e % KM && e / KM < k) ? 1.0 : 0.0;
      __syncthreads();
    }
  }

  if (!polar) {
    // one-sided Jacobi on the columns of A (round-robin pairs; k padded to even with a zero column)
    const int kk = k + (k & 1);
    const int npairs = kk / 2;
    const int tpp = 256 / 32;  // 8 threads per pair (npairs <= 32)
    const int pair = tid / tpp, sub = tid % tpp;
    for (int sweep = 0; sweep < 40; sweep++) {
      if (tid == 0) s_rot = 0;
      __syncthreads();
      for (int step = 0; step < kk - 1; step++) {
        if (pair < npairs) {
          const int m = pair;
          auto pos = [&](int x) { return x == 0 ? 0 : ((x - 1 + step) % (kk - 1)) + 1; };
          int p = pos(m), q = pos(kk - 1 - m);
          if (p > q) {
            const int t = p;
            p = q;
            q = t;
          }
          double al = 0.0, be = 0.0, ga = 0.0;
          if (q < k) {
            for (int i = sub; i < k; i += tpp) {
              const double x = A[p][i], y = A[q][i];
              al += x * x;
              be += y * y;
              ga += x * y;
            }
          }
          // reduce over the 8 lanes of the pair (consecutive lanes of one wave)
          for (int o = tpp / 2; o > 0; o >>= 1) {
            al += __shfl_xor(al, o, tpp);
            be += __shfl_xor(be, o, tpp);
            ga += __shfl_xor(ga, o, tpp);
          }
          if (q < k && ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = sgn1(zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double s = c * t;
            for (int i = sub; i < k; i += tpp) {
              const double x = A[p][i], y = A[q][i];
              A[p][i] = c * x - s * y;
              A[q][i] = s * x + c * y;
              const double vx = V[p][i], vy = V[q][i];
              V[p][i] = c * vx - s * vy;
              V[q][i] = s * vx + c * vy;
            }
            if (sub == 0) s_rot = 1;
          }
        }
        __syncthreads();
      }
      if (s_rot == 0) break;
      __syncthreads();
    }
    // singular values sigma_j = |a_j|; left vectors u_j = a_j / sigma_j in place.  R = sum_j v_j u_j^T
    // does not depend on the order of the pairs, so no sort is needed.
    if (tid < k) {
      double s2 = 0.0;
      for (int i = 0; i < k; i++) s2 += A[tid][i] * A[tid][i];
      sig[tid] = sqrt(s2);
    }
    __syncthreads();
    double smax = 0.0;
    for (int i = 0; i < k; i++) {
      smax = fmax(smax, sig[i]);
      ssum += sig[i];
    }
    int nnull = 0;
    if (tid < k) {
      const bool nz = smax > 0.0 && sig[tid] > 1e-12 * smax;
      isnull[tid] = nz ? 0 : 1;
      for (int i = 0; i < k; i++) A[tid][i] = nz ? A[tid][i] / sig[tid] : 0.0;
    }
    __syncthreads();
    for (int i = 0; i < k; i++) nnull += isnull[i];
    if (nnull > 0) {
      complete_null_cols<KM>(A, k, isnull, tid, placed, n2);
      complete_null_cols<KM>(V, k, isnull, tid, placed, n2);
    }
    __syncthreads();
    // R = V U^T
    for (int e = tid; e < k * k; e += 256) {
      const int a = e / k, b = e % k;
      double s = 0.0;
      for (int j = 0; j < k; j++) s += V[j][a] * A[j][b];
      Rd[e] = s;
      Rt[b * KM + a] = (T)s;
    }
  }
  if (tid == 0) {
    const double obj = (double)n - 2.0 * ssum;
    st->iters += 1;
    if (st->iters > 1 && fabs(obj - st->obj) <= 1e-12 * fmax(1.0, fabs(obj))) st->done = 1;
    st->obj_prev = st->obj;
    st->obj = obj;
  }
}

template <typename T>
__global__ void disc_init_kernel(int k, int km, double* __restrict__ Rd, T* __restrict__ Rt, DiscState* __restrict__ st,
                                 unsigned long long* __restrict__ Sg, unsigned int* __restrict__ cg) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < k * k) {
    const double v = (e / k == e % k) ? 1.0 : 0.0;
    Rd[e] = v;
    Sg[e] = 0ull;
  }
  // R^T with row stride km, zero outside k x k (the row pass reads whole 16-byte groups)
  if (e < km * km) Rt[e] = (e / km == e % km && e / km < k) ? (T)1 : (T)0;
  if (e < k) cg[e] = 0u;
  if (e == 0) {
    st->done = 0;
    st->iters = 0;
    st->obj = 0.0;
    st->obj_prev = 0.0;
  }
}

// Device state of one Discretize call: R (FP64 and in the block's type), the fixed-point
// cluster sums, the counts and the loop state.  Every entry point passes memory of at least
// DISC_STATE_BYTES, 256-byte aligned.
struct DiscBufs {
  double* Rd;
  void* Rt;
  unsigned long long* Sg;
  unsigned int* cg;
  DiscState* st;
};
constexpr size_t DISC_R_BYTES = 64 * 64 * sizeof(double);
constexpr size_t DISC_STATE_BYTES = 3 * DISC_R_BYTES + 256 + 256;

DiscBufs disc_bufs_at(void* base) {
  char* b = (char*)base;
  DiscBufs d;
  d.Rd = (double*)b;
  d.Rt = (void*)(b + DISC_R_BYTES);
  d.Sg = (unsigned long long*)(b + 2 * DISC_R_BYTES);
  d.cg = (unsigned int*)(b + 3 * DISC_R_BYTES);
  d.st = (DiscState*)(b + 3 * DISC_R_BYTES + 256);
  return d;
}

template <typename T, int KM>
ancka_status disc_launch(ancka_ctx* ctx, const T* Q, int64_t n, int k, int64_t ldq, int max_iter, int32_t* labels,
                         double* Rh, double* obj, int32_t* iters, const DiscBufs& b) {
  double* Rd = b.Rd;
  T* Rt = (T*)b.Rt;
  unsigned long long* Sg = b.Sg;
  unsigned int* cg = b.cg;
  DiscState* st = b.st;
  const double fscale = fix_scale(n);
  static_assert(KM * KM <= 16 * 256, "disc_init_kernel covers R^T with 16 x 256 threads");
  disc_init_kernel<T><<<16, 256, 0, ctx->stream>>>(k, KM, Rd, Rt, st, Sg, cg);
  LAUNCH_CHECK(ctx);
  const unsigned grid = (unsigned)cdiv(n, 256);
  // vector reads from Q - voff when that is 16-byte aligned (voff = 0 or 1 columns back)
  int voff = -1;
  const int64_t vw = 16 / (int64_t)sizeof(T);
  if (ldq % vw == 0)
    for (int o = 0; o <= 1 && voff < 0; o++)
      if (((uintptr_t)(Q - o) % 16) == 0 && o + k <= ldq) voff = o;
  DiscState hs{0, 0, 0.0, 0.0};
  for (int it = 0; it < max_iter; it++) {
    if (voff == 0)
      disc_pass_kernel<T, KM, 0><<<grid, 256, 0, ctx->stream>>>(Q, n, k, ldq, Rt, labels, Sg, cg, st, fscale);
    else if (voff == 1)
      disc_pass_kernel<T, KM, 1><<<grid, 256, 0, ctx->stream>>>(Q, n, k, ldq, Rt, labels, Sg, cg, st, fscale);
    else
      disc_pass_kernel<T, KM, -1><<<grid, 256, 0, ctx->stream>>>(Q, n, k, ldq, Rt, labels, Sg, cg, st, fscale);
    LAUNCH_CHECK(ctx);
    disc_svd_kernel<T, KM><<<1, 256, 0, ctx->stream>>>(Sg, cg, k, n, Rd, Rt, st, fscale);
    LAUNCH_CHECK(ctx);
    if ((it % 4) == 3 || it == max_iter - 1) {
      HIP_TRY(ctx, hipMemcpyAsync(&hs, st, sizeof(DiscState), hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      if (hs.done) break;
    }
  }
  if (Rh) {
    HIP_TRY(ctx, hipMemcpyAsync(Rh, Rd, sizeof(double) * k * k, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  if (obj) *obj = hs.obj;
  if (iters) *iters = hs.iters;
  return ANCKA_OK;
}

template <typename T>
ancka_status disc_typed(ancka_ctx* ctx, const T* Q, int64_t n, int k, int64_t ldq, int max_iter, int32_t* labels,
                        double* Rh, double* obj, int32_t* iters, const DiscBufs& b) {
  if (k <= 8) return disc_launch<T, 8>(ctx, Q, n, k, ldq, max_iter, labels, Rh, obj, iters, b);
  if (k <= 16) return disc_launch<T, 16>(ctx, Q, n, k, ldq, max_iter, labels, Rh, obj, iters, b);
  if (k <= 32) return disc_launch<T, 32>(ctx, Q, n, k, ldq, max_iter, labels, Rh, obj, iters, b);
  return disc_launch<T, 64>(ctx, Q, n, k, ldq, max_iter, labels, Rh, obj, iters, b);
}

ancka_status disc_dispatch(ancka_ctx* ctx, const void* Q, int qdtype, int64_t n, int k, int64_t ldq, int max_iter,
                           int32_t* labels, double* R, double* obj, int32_t* iters, const DiscBufs& b) {
  if (qdtype == ANCKA_F64)
    return disc_typed<double>(ctx, (const double*)Q, n, k, ldq, max_iter, labels, R, obj, iters, b);
  return disc_typed<float>(ctx, (const float*)Q, n, k, ldq, max_iter, labels, R, obj, iters, b);
}

ancka_status disc_check_args(ancka_ctx* ctx, const char* fn, const void* Q, int32_t qdtype, int64_t n, int32_t k,
                             int64_t ldq, int32_t max_iter, const int32_t* labels) {
  if (!ctx) return ANCKA_ERR_INVALID_ARG;
  if (!Q || !labels || k < 1 || k > 64 || n < 1 || n >= ((int64_t)1 << 31) || ldq < k || max_iter < 1 ||
      (qdtype != ANCKA_F32 && qdtype != ANCKA_F64))
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "%s: n=%lld k=%d ldq=%lld max_iter=%d qdtype=%d (need 1 <= k <= 64, "
                   "1 <= n < 2^31, ldq >= k, max_iter >= 1, F32 or F64)", fn, (long long)n, k, (long long)ldq,
                   max_iter, qdtype);
  return ANCKA_OK;
}

// The library's own Discretize state for ancka_discretize_noalloc: one copy per GPU (a
// device-side array), at the address hipGetSymbolAddress reports on that GPU.  Host code uses
// only that address, never the array's name (which names host memory in host code).
__device__ __align__(256) unsigned char scratch[DISC_STATE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

ancka_status disc_scratch_setup(ancka_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
    return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "device %d beyond the %d devices the library tracks", ctx->device,
                   MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    HIP_TRY(ctx, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));   // the current device is ctx->device
    g_scratch_ptr[ctx->device] = p;
  }
  return ANCKA_OK;
}

ancka_status discretize_internal(ancka_ctx* ctx, const void* Q, int qdtype, int64_t n, int k, int64_t ldq,
                                 int max_iter, int32_t* labels, double* R, double* obj, int32_t* iters) {
  void* base = nullptr;
  ST_TRY(ws_get(ctx, "disc_state", DISC_STATE_BYTES, &base));
  return disc_dispatch(ctx, Q, qdtype, n, k, ldq, max_iter, labels, R, obj, iters, disc_bufs_at(base));
}

extern "C" ancka_status ancka_discretize(ancka_ctx* ctx, const void* Q, int32_t qdtype, int64_t n, int32_t k,
                                         int64_t ldq, int32_t max_iter, int32_t* labels, double* R, double* obj,
                                         int32_t* iters) {
  ST_TRY(disc_check_args(ctx, "ancka_discretize", Q, qdtype, n, k, ldq, max_iter, labels));
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  return discretize_internal(ctx, Q, qdtype, n, k, ldq, max_iter, labels, R, obj, iters);
}

extern "C" ancka_status ancka_discretize_noalloc(ancka_ctx* ctx, const void* Q, int32_t qdtype, int64_t n, int32_t k,
                                                 int64_t ldq, int32_t max_iter, int32_t* labels, double* R,
                                                 double* obj, int32_t* iters) {
  ST_TRY(disc_check_args(ctx, "ancka_discretize_noalloc", Q, qdtype, n, k, ldq, max_iter, labels));
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[ctx->device];
  }
  if (!base) return set_err(ctx, ANCKA_ERR_HIP, "ancka_discretize_noalloc: no state address for device %d", ctx->device);
  return disc_dispatch(ctx, Q, qdtype, n, k, ldq, max_iter, labels, R, obj, iters, disc_bufs_at(base));
}
