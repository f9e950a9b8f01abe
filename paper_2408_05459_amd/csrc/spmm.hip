// Sparse products with the walk operator (Eqs. zt, mhc-comp-ancka, pi_c_t) on gfx950.
//
// One kernel covers every product the method needs.  For output row r:
//   acc = sum_seg tscale[seg] * sum_{p in seg} tcol[idx[p]*segs + l] * tsrc[idx[p]]     (topology)
//       + sum_{p in knn row r} kval[p] * ksrc[kidx[p]]                                   (KNN walk)
//       + self[r] * ssrc[r]                                                              (self term)
//   out[r] = a * acc + epilogue(r)
// A row is owned by LPR lanes; each lane owns VW consecutive columns and loads them with one
// 16-byte access per gathered row, so a gather of row j is one coalesced 16*LPR-byte request.
// Neighbour indices are read cooperatively (one per lane) and broadcast inside the lane group.
// Sums run in CSR order, so results are deterministic.
#include "common.h"

namespace {

template <typename T>
struct V16;
template <>
struct V16<float> {
  typedef float4 type;
  static constexpr int W = 4;
};
template <>
struct V16<double> {
  typedef double2 type;
  static constexpr int W = 2;
};

template <typename T>
__device__ __forceinline__ void vload(const T* p, T (&v)[V16<T>::W]) {
  const typename V16<T>::type x = *(const typename V16<T>::type*)p;
  if constexpr (V16<T>::W == 4) {
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
  } else {
    v[0] = x.x;
    v[1] = x.y;
  }
}
template <typename T>
__device__ __forceinline__ void vstore(T* p, const T (&v)[V16<T>::W]) {
  typename V16<T>::type x;
  if constexpr (V16<T>::W == 4) {
    x.x = v[0];
    x.y = v[1];
    x.z = v[2];
    x.w = v[3];
  } else {
    x.x = v[0];
    x.y = v[1];
  }
  *(typename V16<T>::type*)p = x;
}

// a source row's W columns from coff: TS = T, or bf16 storage (TS = uint16_t, T = float: four
// columns in one 8-byte load, widened exactly)
template <typename T, typename TS>
__device__ __forceinline__ void src_load(const TS* p, T (&v)[V16<T>::W]) {
  if constexpr (sizeof(TS) == sizeof(T)) {
    vload<T>((const T*)p, v);
  } else {
    static_assert(V16<T>::W == 4, "bf16 sources with FP32 blocks only");
    const uint2 x = *(const uint2*)p;
    v[0] = __uint_as_float(x.x << 16);
    v[1] = __uint_as_float(x.x & 0xffff0000u);
    v[2] = __uint_as_float(x.y << 16);
    v[3] = __uint_as_float(x.y & 0xffff0000u);
  }
}

enum { EPI_NONE = 0, EPI_MHC = 1, EPI_INIT = 2 };

template <typename T>
struct SpmmArgs {
  int64_t rows;
  int segs;
  const int64_t* tptr;
  const int32_t* tidx;
  const T* tscale;   // per segment, nullable (= 1)
  const T* tcol;     // per (source row, layer), nullable (= 1)
  const T* tsrc;
  int64_t tld;       // leading dimension of tsrc
  const int64_t* kptr;  // nullable: no KNN part
  const int32_t* kidx;
  const T* kval;
  const T* ksrc;
  const T* self;     // nullable
  T selfu;           // uniform self coefficient when self == nullptr
  const T* ssrc;     // nullable: no self term
  T* out;
  int64_t ld;        // leading dimension of out, ksrc and ssrc
  int cols;
  T a;
  int epi;
  const int32_t* labels;   // EPI_MHC: label of each row; EPI_INIT: centre index of each row or -1
  const int32_t* counts;   // EPI_MHC: cluster sizes
  T b;
  const int32_t* rorder;   // nullable: output row handled by slot w is rorder[w]
  // nullable: the sources ksrc and ssrc (and tsrc when oh_t) are one-hot blocks given by their
  // labels: row j holds oh_val[j] (oh_alpha when oh_val is null) in column oh_lab[j] and zeros
  // elsewhere (oh_lab[j] < 0: a zero row).  The products then read a label and a value per
  // gathered row instead of the row, with the same arithmetic: the skipped terms are exact zeros.
  const int32_t* oh_lab;
  const T* oh_val;
  T oh_alpha;
  int oh_t;
};

// row j of a one-hot source, the lanes' W columns from coff
template <typename T>
__device__ __forceinline__ void onehot_row(const int32_t* __restrict__ lab, const T* __restrict__ val, T alpha,
                                           int64_t j, int coff, T (&v)[V16<T>::W]) {
  constexpr int W = V16<T>::W;
  const int l = lab[j];
  const T x = val ? val[j] : alpha;
#pragma unroll
  for (int c = 0; c < W; c++) v[c] = (coff + c == l) ? x : (T)0;
}

template <typename T, int LPR, typename TS = T>
__device__ __forceinline__ void gather_segment(const int64_t beg, const int64_t end, const int32_t* __restrict__ idx,
                                               const T* __restrict__ colw, int colw_stride, int colw_off,
                                               const T* __restrict__ vals, const TS* __restrict__ src, int64_t ld,
                                               int sub, bool col_ok, int coff, T (&acc)[V16<T>::W],
                                               const int32_t* __restrict__ olab, const T* __restrict__ oval,
                                               T oalpha) {
  constexpr int W = V16<T>::W;
  for (int64_t p0 = beg; p0 < end; p0 += LPR) {
    const int64_t myp = p0 + sub;
    int32_t jm = 0;
    T wm = (T)0;
    int32_t lm = -1;   // one-hot source: label and value of row jm, loaded by the lane that owns jm
    T xm = (T)0;
    if (myp < end) {
      jm = idx[myp];
      wm = vals ? vals[myp] : (T)1;
      if (colw) wm *= colw[(int64_t)jm * colw_stride + colw_off];
      if (olab) {
        lm = olab[jm];
        xm = oval ? oval[jm] : oalpha;
      }
    }
    const int cnt = (int)((end - p0) < LPR ? (end - p0) : LPR);
    int u = 0;
    for (; u + 4 <= cnt; u += 4) {
      int32_t j[4];
      T w[4];
      T v[4][W];
      int l[4];
      T x[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        // every lane of the group takes part in the broadcasts (no shuffle under a lane branch)
        j[q] = __shfl(jm, u + q, LPR);
        w[q] = __shfl(wm, u + q, LPR);
        l[q] = olab ? __shfl(lm, u + q, LPR) : -1;
        x[q] = olab ? __shfl(xm, u + q, LPR) : (T)0;
      }
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if (col_ok && olab) {
#pragma unroll
          for (int c = 0; c < W; c++) v[q][c] = (coff + c == l[q]) ? x[q] : (T)0;
        } else if (col_ok) src_load<T, TS>(src + (int64_t)j[q] * ld + coff, v[q]);
        else {
#pragma unroll
          for (int c = 0; c < W; c++) v[q][c] = (T)0;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int c = 0; c < W; c++) acc[c] = fma(w[q], v[q][c], acc[c]);
    }
    for (; u < cnt; u++) {
      const int32_t j = __shfl(jm, u, LPR);
      const T w = __shfl(wm, u, LPR);
      const int l = olab ? __shfl(lm, u, LPR) : -1;
      const T x = olab ? __shfl(xm, u, LPR) : (T)0;
      T v[W];
      if (col_ok) {
        if (olab) {
#pragma unroll
          for (int c = 0; c < W; c++) v[c] = (coff + c == l) ? x : (T)0;
        } else {
          src_load<T, TS>(src + (int64_t)j * ld + coff, v);
        }
#pragma unroll
        for (int c = 0; c < W; c++) acc[c] = fma(w, v[c], acc[c]);
      }
    }
  }
}

// TS: storage type of the gathered sources (T, or bf16 for FP32 blocks; the pointers of A are then
// bf16 arrays of the same leading dimensions)
template <typename T, int LPR, typename TS = T>
__global__ __launch_bounds__(256) void spmm_kernel(const SpmmArgs<T> A) {
  constexpr int W = V16<T>::W;
  constexpr int RPB = 256 / LPR;
  const int sub = threadIdx.x % LPR;
  const int64_t w = (int64_t)blockIdx.x * RPB + threadIdx.x / LPR;
  if (w >= A.rows) return;   // whole lane groups exit together
  const int64_t r = A.rorder ? (int64_t)A.rorder[w] : w;
  const int coff = sub * W;
  const bool col_ok = coff < A.cols;
  T acc[W];
#pragma unroll
  for (int c = 0; c < W; c++) acc[c] = (T)0;

  for (int l = 0; l < A.segs; l++) {
    const int64_t seg = r * A.segs + l;
    const int64_t b = A.tptr[seg], e = A.tptr[seg + 1];
    if (b == e) continue;
    T part[W];
#pragma unroll
    for (int c = 0; c < W; c++) part[c] = (T)0;
    gather_segment<T, LPR, TS>(b, e, A.tidx, A.tcol, A.segs, l, nullptr, (const TS*)A.tsrc, A.tld, sub, col_ok, coff,
                               part, A.oh_t ? A.oh_lab : nullptr, A.oh_val, A.oh_alpha);
    const T s = A.tscale ? A.tscale[seg] : (T)1;
#pragma unroll
    for (int c = 0; c < W; c++) acc[c] = fma(s, part[c], acc[c]);
  }
  if (A.kptr) {
    gather_segment<T, LPR, TS>(A.kptr[r], A.kptr[r + 1], A.kidx, nullptr, 0, 0, A.kval, (const TS*)A.ksrc, A.ld, sub,
                               col_ok, coff, acc, A.oh_lab, A.oh_val, A.oh_alpha);
  }
  if ((A.ssrc || A.oh_lab) && col_ok && (A.self || A.selfu != (T)0)) {
    const T sc = A.self ? A.self[r] : A.selfu;
    if (sc != (T)0) {
      T v[W];
      if (A.oh_lab) onehot_row<T>(A.oh_lab, A.oh_val, A.oh_alpha, r, coff, v);
      else src_load<T, TS>((const TS*)A.ssrc + r * A.ld + coff, v);
#pragma unroll
      for (int c = 0; c < W; c++) acc[c] = fma(sc, v[c], acc[c]);
    }
  }
  if (!col_ok) return;
  T o[W];
#pragma unroll
  for (int c = 0; c < W; c++) o[c] = A.a * acc[c];
  if (A.epi == EPI_MHC) {
    const int lab = A.labels[r];
    const int c = lab - coff;
    if (c >= 0 && c < W) o[c] += A.b / sqrt((T)A.counts[lab]);
  } else if (A.epi == EPI_INIT) {
    const int cj = A.labels[r];
    const int c = cj - coff;
    if (cj >= 0 && c >= 0 && c < W) o[c] += A.b;
  }
  vstore<T>(A.out + r * A.ld + coff, o);
}

template <typename T, typename TS = T>
ancka_status launch_spmm(ancka_ctx* ctx, SpmmArgs<T> A) {
  if (A.rows <= 0) return ANCKA_OK;
  constexpr int W = V16<T>::W;
  const int need = (A.cols + W - 1) / W;
  int lpr = 2;
  while (lpr < need) lpr *= 2;
  if (lpr > 64) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "spmm: %d columns exceed one wave", A.cols);
  const unsigned grid = (unsigned)cdiv(A.rows, 256 / lpr);
  switch (lpr) {
    case 2: spmm_kernel<T, 2, TS><<<grid, 256, 0, ctx->stream>>>(A); break;
    case 4: spmm_kernel<T, 4, TS><<<grid, 256, 0, ctx->stream>>>(A); break;
    case 8: spmm_kernel<T, 8, TS><<<grid, 256, 0, ctx->stream>>>(A); break;
    case 16: spmm_kernel<T, 16, TS><<<grid, 256, 0, ctx->stream>>>(A); break;
    case 32: spmm_kernel<T, 32, TS><<<grid, 256, 0, ctx->stream>>>(A); break;
    default: spmm_kernel<T, 64, TS><<<grid, 256, 0, ctx->stream>>>(A); break;
  }
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

template <typename T>
SpmmArgs<T> blank(int64_t rows, T* out, int64_t ld, int cols) {
  SpmmArgs<T> A;
  A.rows = rows;
  A.segs = 1;
  A.tptr = nullptr;
  A.tidx = nullptr;
  A.tscale = nullptr;
  A.tcol = nullptr;
  A.tsrc = nullptr;
  A.tld = ld;
  A.kptr = nullptr;
  A.kidx = nullptr;
  A.kval = nullptr;
  A.ksrc = nullptr;
  A.self = nullptr;
  A.selfu = (T)0;
  A.ssrc = nullptr;
  A.out = out;
  A.ld = ld;
  A.cols = cols;
  A.a = (T)1;
  A.epi = EPI_NONE;
  A.labels = nullptr;
  A.counts = nullptr;
  A.b = (T)0;
  A.rorder = nullptr;
  A.oh_lab = nullptr;
  A.oh_val = nullptr;
  A.oh_alpha = (T)0;
  A.oh_t = 0;
  return A;
}

// P Q with optional epilogue (EPI_NONE: plain; EPI_MHC: (1-alpha) P F + alpha Yh)
// (Q null: the source is the one-hot block of oh_lab / oh_val / oh_alpha)
template <typename T>
ancka_status apply_typed(ancka_ctx* ctx, const ancka_op* op, const T* Q, T* Z, int cols, int64_t ld, T a, int epi,
                         const int32_t* labels, const int32_t* counts, T b, const int32_t* oh_lab = nullptr,
                         const T* oh_val = nullptr, T oh_alpha = (T)0, const char* ename = "spmm_E") {
  const int64_t n = op->n;
  const T* topo_src = Q;
  bool topo_onehot = oh_lab != nullptr;
  if (op->kind == ANCKA_HYPERGRAPH) {
    T* E = nullptr;
    ST_TRY(ws_get_t(ctx, ename, (size_t)op->m * ld, &E));
    SpmmArgs<T> S1 = blank<T>(op->m, E, ld, cols);
    S1.tptr = op->eptr;
    S1.tidx = op->eidx;
    S1.tscale = (const T*)op->escale;
    S1.tsrc = Q;
    S1.oh_lab = oh_lab;
    S1.oh_val = oh_val;
    S1.oh_alpha = oh_alpha;
    S1.oh_t = 1;
    ST_TRY(launch_spmm<T>(ctx, S1));
    topo_src = E;
    topo_onehot = false;
  }
  SpmmArgs<T> S = blank<T>(n, Z, ld, cols);
  S.segs = op->kind == ANCKA_HYPERGRAPH ? 1 : op->L;
  S.tptr = op->tptr;
  S.rorder = op->rorder;
  S.tidx = op->tidx;
  S.tscale = (const T*)op->tscale;
  S.tsrc = topo_src;
  S.kptr = op->kptr;
  S.kidx = op->kidx;
  S.kval = (const T*)op->kval;
  S.ksrc = Q;
  S.self = (const T*)op->self;
  S.ssrc = Q;
  S.a = a;
  S.epi = epi;
  S.labels = labels;
  S.counts = counts;
  S.b = b;
  S.oh_lab = oh_lab;
  S.oh_val = oh_val;
  S.oh_alpha = oh_alpha;
  S.oh_t = topo_onehot ? 1 : 0;
  return launch_spmm<T>(ctx, S);
}

// (Pin null: the source is one-hot, alpha in column centre_of[j] of the centres' rows)
template <typename T>
ancka_status init_typed(ancka_ctx* ctx, const ancka_op* op, const T* Pin, T* Pout, int cols, int64_t ld, T a,
                        const int32_t* centre_of, T b) {
  const int64_t n = op->n;
  const int32_t* oh = Pin ? nullptr : centre_of;
  if (op->kind == ANCKA_HYPERGRAPH) {
    T* E = nullptr;
    ST_TRY(ws_get_t(ctx, "spmm_E", (size_t)op->m * ld, &E));
    SpmmArgs<T> S1 = blank<T>(op->m, E, ld, cols);
    S1.tptr = op->eptr;
    S1.tidx = op->eidx;
    S1.tscale = (const T*)op->escale;
    S1.tcol = (const T*)op->tcol;   // 1/delta(v) of the source node
    S1.tsrc = Pin;
    S1.oh_lab = oh;
    S1.oh_alpha = b;
    S1.oh_t = 1;
    ST_TRY(launch_spmm<T>(ctx, S1));
    SpmmArgs<T> S2 = blank<T>(n, Pout, ld, cols);
    S2.tptr = op->tptr;
    S2.rorder = op->rorder;
    S2.tidx = op->tidx;
    S2.tsrc = E;
    S2.a = a;
    S2.epi = EPI_INIT;
    S2.labels = centre_of;
    S2.b = b;
    return launch_spmm<T>(ctx, S2);
  }
  SpmmArgs<T> S = blank<T>(n, Pout, ld, cols);
  S.segs = op->L;
  S.tptr = op->tptr;
  S.rorder = op->rorder;
  S.tidx = op->tidx;
  S.tcol = (const T*)op->tcol;      // 1/(L_j deg_l(j)) of the source node in layer l
  S.tsrc = Pin;
  S.oh_lab = oh;
  S.oh_alpha = b;
  S.oh_t = 1;
  S.a = a;
  S.epi = EPI_INIT;
  S.labels = centre_of;
  S.b = b;
  return launch_spmm<T>(ctx, S);
}

}  // namespace

ancka_status op_apply(ancka_ctx* ctx, const ancka_op* op, const void* Q, void* Z, int cols, int64_t ld) {
  if (op->dtype == ANCKA_F64)
    return apply_typed<double>(ctx, op, (const double*)Q, (double*)Z, cols, ld, 1.0, EPI_NONE, nullptr, nullptr, 0.0);
  return apply_typed<float>(ctx, op, (const float*)Q, (float*)Z, cols, ld, 1.0f, EPI_NONE, nullptr, nullptr, 0.0f);
}

// Z = P Q with Q stored in bf16 (graph / multiplex operators of FP32 values; FP32 accumulation)
ancka_status op_apply_bf16(ancka_ctx* ctx, const ancka_op* op, const uint16_t* Q, float* Z, int cols, int64_t ld) {
  SpmmArgs<float> S = blank<float>(op->n, Z, ld, cols);
  S.segs = op->L;
  S.tptr = op->tptr;
  S.rorder = op->rorder;
  S.tidx = op->tidx;
  S.tscale = (const float*)op->tscale;
  S.tsrc = (const float*)(const void*)Q;
  S.kptr = op->kptr;
  S.kidx = op->kidx;
  S.kval = (const float*)op->kval;
  S.ksrc = (const float*)(const void*)Q;
  S.self = (const float*)op->self;
  S.ssrc = (const float*)(const void*)Q;
  S.a = 1.0f;
  return launch_spmm<float, uint16_t>(ctx, S);
}

ancka_status op_apply_mhc(ancka_ctx* ctx, const ancka_op* op, const void* Q, void* Z, int cols, int64_t ld,
                          double alpha, const int32_t* labels, const int32_t* counts, const void* f0val) {
  // Q null: the source is F(0) = alpha Yh, row j holding f0val[j] in column labels[j]
  if (op->dtype == ANCKA_F64)
    return apply_typed<double>(ctx, op, (const double*)Q, (double*)Z, cols, ld, 1.0 - alpha, EPI_MHC, labels, counts,
                               alpha, Q ? nullptr : labels, (const double*)f0val, alpha, "spmm_E_mhc");
  return apply_typed<float>(ctx, op, (const float*)Q, (float*)Z, cols, ld, (float)(1.0 - alpha), EPI_MHC, labels,
                            counts, (float)alpha, Q ? nullptr : labels, (const float*)f0val, (float)alpha,
                            "spmm_E_mhc");
}

ancka_status op_apply_init(ancka_ctx* ctx, const ancka_op* op, const void* Pin, void* Pout, int cols, int64_t ld,
                           double alpha, const int32_t* centre_of) {
  if (op->dtype == ANCKA_F64)
    return init_typed<double>(ctx, op, (const double*)Pin, (double*)Pout, cols, ld, 1.0 - alpha, centre_of, alpha);
  return init_typed<float>(ctx, op, (const float*)Pin, (float*)Pout, cols, ld, (float)(1.0 - alpha), centre_of,
                           (float)alpha);
}

ancka_status op_apply_features(ancka_ctx* ctx, const ancka_op* op, const float* Xh, float* U, int cols, int64_t ld) {
  // U = 0.5 Xh + 0.5 P_N Xh, column panels of at most 64
  for (int c0 = 0; c0 < cols; c0 += 64) {
    const int w = (cols - c0) < 64 ? (cols - c0) : 64;
    const float* src = Xh + c0;
    float* dst = U + c0;
    if (op->kind == ANCKA_HYPERGRAPH) {
      float* E = nullptr;
      ST_TRY(ws_get_t(ctx, "spmm_Ef", (size_t)op->m * 64, &E));
      SpmmArgs<float> S1 = blank<float>(op->m, E, 64, w);
      S1.tptr = op->eptr;
      S1.tidx = op->eidx;
      S1.tscale = (const float*)op->escale;
      S1.tsrc = src;
      S1.tld = ld;
      ST_TRY(launch_spmm<float>(ctx, S1));
      SpmmArgs<float> S2 = blank<float>(op->n, dst, ld, w);
      S2.tptr = op->tptr;
      S2.rorder = op->rorder;
      S2.tidx = op->tidx;
      S2.tscale = (const float*)op->tcol;   // 1/delta(u) per node
      S2.tsrc = E;
      S2.tld = 64;
      S2.ssrc = src;
      S2.selfu = 1.0f;
      S2.a = 0.5f;
      ST_TRY(launch_spmm<float>(ctx, S2));
    } else {
      SpmmArgs<float> S = blank<float>(op->n, dst, ld, w);
      S.segs = op->L;
      S.tptr = op->tptr;
      S.rorder = op->rorder;
      S.tidx = op->tidx;
      S.tscale = (const float*)op->tcol;    // 1/(L_i deg_l(i)) per segment
      S.tsrc = src;
      S.ssrc = src;
      S.selfu = 1.0f;
      S.a = 0.5f;
      ST_TRY(launch_spmm<float>(ctx, S));
    }
  }
  return ANCKA_OK;
}

extern "C" ancka_status ancka_apply_p(ancka_ctx* ctx, const ancka_op* op, const void* Q, void* Z, int32_t cols,
                                      int64_t ld) {
  if (!ctx || !op || !Q || !Z) return ANCKA_ERR_INVALID_ARG;
  const int vw = op->dtype == ANCKA_F64 ? 2 : 4;
  if (cols < 1 || cols > 64 || ld < cols || ld % vw != 0)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_apply_p: cols=%d ld=%lld (ld must be a multiple of %d)", cols,
                   (long long)ld, vw);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  return op_apply(ctx, op, Q, Z, cols, ld);
}

extern "C" ancka_status ancka_apply_p_bf16(ancka_ctx* ctx, const ancka_op* op, const void* Q, float* Z, int32_t cols,
                                           int64_t ld) {
  if (!ctx || !op || !Q || !Z) return ANCKA_ERR_INVALID_ARG;
  if (cols < 1 || cols > 64 || ld < cols || ld % 4 != 0)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_apply_p_bf16: cols=%d ld=%lld (ld must be a multiple of 4)",
                   cols, (long long)ld);
  if (op->dtype != ANCKA_F32 || op->kind == ANCKA_HYPERGRAPH)
    return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "ancka_apply_p_bf16: FP32 graph or multiplex operators only");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  return op_apply_bf16(ctx, op, (const uint16_t*)Q, Z, cols, ld);
}
