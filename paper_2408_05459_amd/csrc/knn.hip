// K nearest neighbours by cosine similarity (Sec. 3.1; Alg. 6, neighbour search) on gfx950.
//
// Modes
//  EXACT_F64     FP64 tiles; the top-K list is final (similarity = dot / sqrt(|x_i|^2 |x_j|^2)).
//  EXACT_F32     FP32 tiles -> top-2K candidates -> FP64 rescoring -> top-K + certificate.
//  BF16_RESCORE  BF16 MFMA tiles (FP32 accumulation of exact products) -> as EXACT_F32.
//
// Certificate: a candidate outside the 2K list has an approximate score no larger than the
// 2K-th listed one, a; its exact score is at most a + eps, eps bounding the tile arithmetic
// (fp32 accumulation: gamma_d = d u / (1 - d u) plus the roundings of the inverse norms, with a
// safety factor 4).  When the K-th rescored similarity exceeds a + eps no outside candidate can
// enter the top K, otherwise the row is recomputed exactly over all n candidates.
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <vector>
#include <algorithm>

#include "common.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_to_f32(uint16_t v) { return __uint_as_float(((uint32_t)v) << 16); }

template <typename TX>
__device__ __forceinline__ double load_as_double(const TX* p, int64_t i);
template <>
__device__ __forceinline__ double load_as_double<double>(const double* p, int64_t i) { return p[i]; }
template <>
__device__ __forceinline__ double load_as_double<float>(const float* p, int64_t i) { return (double)p[i]; }
template <>
__device__ __forceinline__ double load_as_double<uint16_t>(const uint16_t* p, int64_t i) {
  return (double)bf16_to_f32(p[i]);
}

// key order: larger similarity first, then smaller index
template <typename T>
__device__ __forceinline__ bool better(T s, int j, T s2, int j2) {
  return s > s2 || (s == s2 && j < j2);
}

// ---- prologue: |x_i|^2 in FP64, 1/|x_i|, |x_i|, optional zero-padded bf16 copy -----------
template <typename TX>
__global__ __launch_bounds__(256) void knn_prologue_kernel(const TX* __restrict__ X, int64_t n, int64_t d, int64_t ldx,
                                                           double* __restrict__ sq, float* __restrict__ invn,
                                                           float* __restrict__ nrm, uint16_t* __restrict__ Xp, int DP,
                                                           unsigned long long* __restrict__ zero_count) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / ANCKA_WAVE;
  const int lane = threadIdx.x % ANCKA_WAVE;
  if (row >= n) return;
  const TX* xr = X + row * ldx;
  double acc = 0.0;
  for (int64_t c = lane; c < d; c += ANCKA_WAVE) {
    const double v = load_as_double<TX>(xr, c);
    acc += v * v;
  }
  acc = wave_sum(acc);
  if (Xp) {
    uint16_t* xp = Xp + row * (int64_t)DP;
    for (int c = lane; c < DP; c += ANCKA_WAVE) {
      uint16_t v = 0;
      if (c < d) v = ((const uint16_t*)(const void*)xr)[c];
      xp[c] = v;
    }
  }
  if (lane == 0) {
    sq[row] = acc;
    const double nr = sqrt(acc);
    invn[row] = acc > 0.0 ? (float)(1.0 / nr) : 0.0f;
    nrm[row] = (float)nr;
    if (acc == 0.0) atomicAdd(zero_count, 1ull);
  }
}

// ---- exact tiles with vector FMA (EXACT_F64 / EXACT_F32) -----------------------------------
// 64 queries x 64 candidates per step, 4x4 outputs per thread, d streamed in chunks of 16.
// The score tile goes to LDS; thread r < 64 owns query r's list of length KP (sorted).
constexpr int VT_Q = 64;
constexpr int VT_C = 64;
constexpr int VT_D = 16;

template <typename T, typename TX>
__global__ __launch_bounds__(256) void knn_vector_kernel(const TX* __restrict__ X, int64_t n, int64_t d, int64_t ldx,
                                                         const double* __restrict__ sq, const float* __restrict__ invn,
                                                         int KP, int exact_div, int32_t* __restrict__ cand_idx,
                                                         T* __restrict__ cand_sim) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = (T*)smem;                       // [VT_D][VT_Q]
  T* Bs = As + VT_D * VT_Q;               // [VT_D][VT_C]
  T* S = Bs + VT_D * VT_C;                // [VT_Q][VT_C + 1]
  T* lsim = S + VT_Q * (VT_C + 1);        // [VT_Q][KP]
  int* lidx = (int*)(lsim + VT_Q * KP);   // [VT_Q][KP]

  const int tid = threadIdx.x;
  const int ty = tid / 16, tx = tid % 16;
  const int64_t q0 = (int64_t)blockIdx.x * VT_Q;

  for (int e = tid; e < VT_Q * KP; e += 256) {
    lsim[e] = -INFINITY;
    lidx[e] = INT_MAX;
  }
  // query owner state
  const int64_t my_q = q0 + tid;
  const bool owner = tid < VT_Q && my_q < n;
  T my_sq = 0, my_inv = 0;
  if (owner) {
    my_sq = (T)sq[my_q];
    my_inv = (T)invn[my_q];
  }
  const bool my_zero = owner && sq[my_q] == 0.0;
  __syncthreads();

  const int64_t ntiles = cdiv(n, VT_C);
  for (int64_t t = 0; t < ntiles; t++) {
    const int64_t c0 = t * VT_C;
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) acc[i][j] = 0;
    for (int64_t k0 = 0; k0 < d; k0 += VT_D) {
      // thread loads 4 elements of one row of each tile: row = tid / 4, cols (tid % 4) * 4 ..
      const int lr = tid / 4, lc = (tid % 4) * 4;
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int64_t kk = k0 + lc + u;
        const int64_t qr = q0 + lr, cr = c0 + lr;
        As[(lc + u) * VT_Q + lr] = (qr < n && kk < d) ? (T)load_as_double<TX>(X, qr * ldx + kk) : (T)0;
        Bs[(lc + u) * VT_C + lr] = (cr < n && kk < d) ? (T)load_as_double<TX>(X, cr * ldx + kk) : (T)0;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < VT_D; kk++) {
        T a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; i++) a[i] = As[kk * VT_Q + ty * 4 + i];
#pragma unroll
        for (int j = 0; j < 4; j++) b[j] = Bs[kk * VT_C + tx * 4 + j];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
          for (int j = 0; j < 4; j++) acc[i][j] = fma(a[i], b[j], acc[i][j]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int j = 0; j < 4; j++) S[(ty * 4 + i) * (VT_C + 1) + tx * 4 + j] = acc[i][j];
    __syncthreads();
    if (owner && !my_zero) {
      T* ls = lsim + tid * KP;
      int* li = lidx + tid * KP;
      T thr = ls[KP - 1];
      int thr_i = li[KP - 1];
      for (int c = 0; c < VT_C; c++) {
        const int64_t j = c0 + c;
        if (j >= n || j == my_q) continue;
        const double sqj = sq[j];
        if (sqj == 0.0) continue;
        const T dot = S[tid * (VT_C + 1) + c];
        T s;
        if (exact_div) s = dot / sqrt(my_sq * (T)sqj);
        else s = dot * (my_inv * (T)invn[j]);
        const int jj = (int)j;
        if (!better<T>(s, jj, thr, thr_i)) continue;
        int p = KP - 1;
        while (p > 0 && better<T>(s, jj, ls[p - 1], li[p - 1])) {
          ls[p] = ls[p - 1];
          li[p] = li[p - 1];
          p--;
        }
        ls[p] = s;
        li[p] = jj;
        thr = ls[KP - 1];
        thr_i = li[KP - 1];
      }
    }
    __syncthreads();
  }
  if (owner) {
    for (int r = 0; r < KP; r++) {
      const int j = lidx[tid * KP + r];
      cand_idx[my_q * KP + r] = (j == INT_MAX) ? -1 : j;
      cand_sim[my_q * KP + r] = (j == INT_MAX) ? (T)0 : lsim[tid * KP + r];
    }
  }
}

// ---- BF16 MFMA tiles ------------------------------------------------------------------------
// Scan order.  Rows are grouped into coarse cells (the most similar of NPIV pivot rows), in
// norm order inside a cell; queries and candidates share this order (a bf16 copy Xs, padded to
// whole blocks of QB = 4*QW rows).  Workgroup I owns block I of QB consecutive queries, and its
// window is a block range lo .. hi around I (the blocks of the cells its rows belong to), with
// J in I's window exactly when I is in J's.
// Two passes cover every unordered pair of rows.
//  Window pass: block I scans the tiles of its window, starting at its own cell; the most
//    similar rows lie there, so each list ends close to its final state.  A bound pass over the
//    same tiles first finds a lower bound of each query's KP-th score, where its list starts.
//  Symmetric pass: block I scans blocks hi+1 .. I+h (h = half the ring; for an even block count
//    the opposite block is scanned only from the lower half), so each pair of blocks outside
//    each other's windows meets once.  A tile score a = x_i.x_j serves both rows: the query side updates the lists
//    of block I in LDS as in the window pass; on the candidate side, a pair whose score reaches
//    the candidate row's threshold after the window pass (the worst entry of its list then)
//    is handed over through a global buffer and merged into that row's list afterwards.  The
//    candidate-side test is a necessary condition for entering the final list, so the merged
//    lists equal those of a full scan of all pairs.
// When a window would exceed a quarter of the ring the window pass is the whole scan and the
// symmetric pass is skipped.
// The order changes nothing in the result (lists are ordered by the (similarity, index) key).
// Tiles.  Wave w holds its QW queries as MFMA B operands in registers for the whole kernel;
// 64-row candidate tiles (two 32-row A blocks) stream through double-buffered LDS.
// Epilogue.  A lane holds 16 candidates of one query per (A block, B block).  The maximum raw
// dot of its 32 candidates is compared with the query's threshold times the tile's smallest
// norm -- necessary for any of them to enter the list, and tight because a tile's norms are
// close.  Passing lanes score their candidates exactly (dot / |x_j|) and insert them into the
// query's sorted list in LDS; the two half-waves, which hold different candidates of the same
// queries, insert one after the other.
constexpr int BT_C = 64;   // candidates per tile
constexpr int TAU_T = 11;   // bound pass: values kept per lane (lists up to 2 TAU_T - 1 = 21 long)
constexpr int TAU_T2 = 21;  // the bound pass for lists of 22 .. 41 entries
enum { SCAN_WIN = 0, SCAN_SYM = 1, SCAN_TAU = 2 };
constexpr int NPIV = 64;   // coarse cells of the scan order

// One query's candidate list, unsorted: kpp slots (the list length rounded up to 4; padding
// slots hold (+inf, -1) and are never the worst), in LDS or in global memory.  The caller keeps
// the list's worst entry (score ws, index wj, slot wp) under the order (score desc, index asc) in
// registers.  list_worst finds it with 16-byte reads, eight entries per step; list_replace_worst
// puts (s, jj) in its place and returns the new worst.  The list ends as the top entries of that
// total order whatever order candidates arrive in.
__device__ __forceinline__ void list_worst(const float* ls, const int* li, int kpp, float& ws, int& wj, int& wp) {
  float bs = INFINITY;
  int bj = INT_MIN, bp = 0;
  for (int r = 0; r < kpp; r += 8) {
    const float4 sa = *(const float4*)(ls + r);
    const int4 ja = *(const int4*)(li + r);
    float4 sb = make_float4(INFINITY, INFINITY, INFINITY, INFINITY);
    int4 jb = make_int4(-1, -1, -1, -1);
    if (r + 4 < kpp) {
      sb = *(const float4*)(ls + r + 4);
      jb = *(const int4*)(li + r + 4);
    }
    if (sa.x < bs || (sa.x == bs && ja.x > bj)) { bs = sa.x; bj = ja.x; bp = r; }
    if (sa.y < bs || (sa.y == bs && ja.y > bj)) { bs = sa.y; bj = ja.y; bp = r + 1; }
    if (sa.z < bs || (sa.z == bs && ja.z > bj)) { bs = sa.z; bj = ja.z; bp = r + 2; }
    if (sa.w < bs || (sa.w == bs && ja.w > bj)) { bs = sa.w; bj = ja.w; bp = r + 3; }
    if (sb.x < bs || (sb.x == bs && jb.x > bj)) { bs = sb.x; bj = jb.x; bp = r + 4; }
    if (sb.y < bs || (sb.y == bs && jb.y > bj)) { bs = sb.y; bj = jb.y; bp = r + 5; }
    if (sb.z < bs || (sb.z == bs && jb.z > bj)) { bs = sb.z; bj = jb.z; bp = r + 6; }
    if (sb.w < bs || (sb.w == bs && jb.w > bj)) { bs = sb.w; bj = jb.w; bp = r + 7; }
  }
  ws = bs;
  wj = bj;
  wp = bp;
}

// Empty slots (-inf, INT_MAX) are the worst entries there are, and list_worst returns the first
// of equal worst entries, so a list fills its slots in order: the empty slots are always a
// suffix.  Filling an empty slot then leaves the next slot as the new worst when that one is
// empty too, and no scan is needed.  Kept out of line: the insertion runs at 32 places of each
// epilogue, and inlined copies crowd the kernel's registers.
struct ListWorst {
  float s;
  int j;
  int p;
};
__device__ __noinline__ ListWorst list_replace_worst(float* ls, int* li, int kpp, float s, int jj, ListWorst w) {
  const bool was_empty = w.j == INT_MAX;
  ls[w.p] = s;
  li[w.p] = jj;
  if (was_empty && w.p + 1 < kpp && li[w.p + 1] == INT_MAX) return ListWorst{-INFINITY, INT_MAX, w.p + 1};
  ListWorst r;
  list_worst(ls, li, kpp, r.s, r.j, r.p);
  return r;
}

// Arguments of both passes.  Lists are kept per sorted row p in [0, npad): KPP slots (KP rounded
// up to 4; slots KP.. hold (+inf, -1)), unsorted, original row indices (INT_MAX: empty slot) and
// raw scores x_p.x_j / |x_j| (the cosine times |x_p|, which orders a row's candidates like the
// cosine).
struct ScanArgs {
  const uint16_t* Xs;        // [npad][DP] bf16 rows in scan order, zero padded
  const float* invs;         // [npad] 1/|x|, 0 for zero and padding rows
  const int32_t* perm;       // [npad] original index, -1 for padding rows
  const float* tile_min;     // [ntp] smallest norm of a non-zero row of each tile (+inf if none)
  const int32_t* wg_start;   // [nwg] first tile of the cell of each block's first row
  int64_t nwg;               // blocks of QB rows (workgroups)
  int64_t ntp;               // tiles in the padded ring, nwg * QB / BT_C
  int w;                     // -1: the window is the whole ring (no symmetric pass); else >= 0
  const int32_t* wlo;        // [nwg] window of block I: blocks wlo[I] .. whi[I] (unwrapped, taken
  const int32_t* whi;        //   mod nwg); wlo <= I <= whi, and J in I's window iff I in J's
  int KP;                    // list length
  int32_t* lidx;             // [npad][KPP] lists (written by the window pass, updated in place)
  float* lsim;               // [npad][KPP]
  float* colthr;             // [npad] candidate-side threshold: the list's worst raw score after
                             // the window pass (-inf if not full; +inf for zero and padding rows)
  const float* tile_thr;     // [ntp] smallest colthr of each tile (symmetric pass)
  const float* tile_cinv;    // [ntp] smallest 1/|x| of a non-zero row of each tile (bound pass)
  float* tau;                // [npad] lower bound of each row's KP-th best raw score (bound pass
                             //   writes it, window pass starts from it); nullptr: none
  uint64_t* hkey;            // hand-over buffer: sorted row that receives the candidate
  uint64_t* hval;            //   (original index of the candidate << 32) | raw score bits
  unsigned long long* hcount;  // entries produced (may exceed hcap: then the buffer overflowed)
  int64_t hcap;
  // IVF (nullable): block I scans the tiles tlist[toff[I]] .. tlist[toff[I+1] - 1] (the tiles of
  // the cells it probes, its own cell's first) instead of a ring range; window and bound passes only
  const int32_t* tlist;
  const int64_t* toff;
};

// LG: the lists stay in global memory (args.lsim / args.lidx) instead of LDS, for list lengths
// whose LDS copy would leave room for fewer than two workgroups per CU.
template <int DP, int QW, int NBUF, int MODE, bool LG, int TT = TAU_T>
__global__ __launch_bounds__(256, (DP <= 128 ? 2 : 1)) void knn_bf16_kernel(ScanArgs args) {
  constexpr bool SYM = MODE == SCAN_SYM;
  constexpr bool TAU = MODE == SCAN_TAU;
  constexpr bool LDSL = !TAU && !LG;    // lists in LDS
  constexpr int KS = DP / 16;           // MFMA k-steps
  constexpr int NQB = QW / 32;          // query blocks per wave
  constexpr int QB = 4 * QW;            // queries per workgroup
  constexpr int TPB = QB / BT_C;        // tiles per block
  constexpr int LDR = DP + 8;           // LDS row stride in bf16 (16-byte pad)
  constexpr int CHUNKS = BT_C * DP / 8; // 16-byte chunks per tile
  constexpr int CPT = CHUNKS / 256;     // chunks per thread
  static_assert(CHUNKS % 256 == 0, "tile chunks");
  static_assert(QB % BT_C == 0, "padding to whole workgroups covers whole tiles");

  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* tileb = (uint16_t*)smem;                         // [NBUF][BT_C][LDR]
  float* tinv = (float*)(tileb + NBUF * BT_C * LDR);         // [NBUF][BT_C]
  int* tperm = (int*)(tinv + NBUF * BT_C);                   // [NBUF][BT_C]
  float* tmn = (float*)(tperm + NBUF * BT_C);                // [NBUF] smallest norm, [2 + NBUF] tile_thr
  const int KP = args.KP;
  const int KPP = (KP + 3) & ~3;                             // list slots per query
  float* tthr = tmn + 4;                                     // [NBUF][BT_C] colthr (symmetric pass)
  float* lsim = tthr + NBUF * BT_C;                          // [QB][KPP] lists in LDS (LDSL)
  int* lidx = (int*)(lsim + (LDSL ? QB * KPP : 0));          // [QB][KPP]

  const int tid = threadIdx.x;
  const int wave = tid / ANCKA_WAVE;
  const int lane = tid % ANCKA_WAVE;
  const int l32 = lane % 32;
  const int half = lane / 32;
  const int64_t blk = blockIdx.x;
  const int64_t q0 = blk * QB;
  // list of the workgroup's query q (LDS, or the global copy of its sorted row)
  auto list_s = [&](int q) { return LDSL ? lsim + q * KPP : args.lsim + (q0 + q) * (int64_t)KPP; };
  auto list_i = [&](int q) { return LDSL ? lidx + q * KPP : args.lidx + (q0 + q) * (int64_t)KPP; };

  // the window pass starts from empty lists; the symmetric pass from the window pass's lists
  if (MODE == SCAN_WIN) {
    for (int e = tid; e < QB * KPP; e += 256) {
      const bool pad = (e % KPP) >= KP;
      if (LDSL) {
        lsim[e] = pad ? INFINITY : -INFINITY;
        lidx[e] = pad ? -1 : INT_MAX;
      } else {
        args.lsim[q0 * KPP + e] = pad ? INFINITY : -INFINITY;
        args.lidx[q0 * KPP + e] = pad ? -1 : INT_MAX;
      }
    }
  } else if (SYM && LDSL) {
    for (int e = tid; e < QB * KPP; e += 256) {
      lsim[e] = args.lsim[q0 * KPP + e];
      lidx[e] = args.lidx[q0 * KPP + e];
    }
  }
  __syncthreads();   // (also orders the global initialisation of LG lists before their first reads)

  // query fragments: lane holds 8 bf16 of query row (l32) at k = ks*16 + half*8
  bf16x8 bq[NQB][KS];
  float thr[NQB];
  float tq[NQB];     // window pass: the bound pass's lower bound, a floor for the threshold
  float colq[NQB];   // symmetric pass: 1/|x_i| of the lane's query (0: the query takes no part)
  float rt[NQB][TT];  // bound pass: the lane's TT largest bound scores, descending
  float wv[NQB];     // worst entry of the query's list: score, index, slot (both halves hold it)
  int wi[NQB], wp[NQB];
  int qloc[NQB];
  int qorig[NQB];
  // Xs, invs and perm are padded with zero rows (invs 0, perm -1) to whole workgroups, so no
  // load below needs a bounds check; padding rows never become candidates (invs 0) and their
  // queries never accept one (threshold +inf).
#pragma unroll
  for (int qb = 0; qb < NQB; qb++) {
    qloc[qb] = wave * QW + qb * 32 + l32;
    const int64_t qs = q0 + qloc[qb];
    qorig[qb] = args.perm[qs];
    const float iq = args.invs[qs];
    tq[qb] = (MODE == SCAN_WIN && args.tau) ? args.tau[qs] : -INFINITY;
    // worst entry of the query's list: the first empty slot of a new list; found in the window
    // pass's list by the symmetric pass (the bound pass has no lists)
    wv[qb] = -INFINITY;
    wi[qb] = INT_MAX;
    wp[qb] = 0;
    if (SYM) list_worst(list_s(qloc[qb]), list_i(qloc[qb]), KPP, wv[qb], wi[qb], wp[qb]);
    thr[qb] = iq > 0.0f ? (SYM ? wv[qb] : tq[qb]) : INFINITY;
    colq[qb] = iq;
#pragma unroll
    for (int j = 0; j < TT; j++) rt[qb][j] = -INFINITY;
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
      const uint4 v = *(const uint4*)(args.Xs + qs * DP + ks * 16 + half * 8);
      bq[qb][ks] = __builtin_bit_cast(bf16x8, v);
    }
  }

  // this workgroup's scan: L tiles of the ring starting at tile ws, beginning at offset s0
  // tile indices fit in 32 bits (ntp < 2^26 for n < 2^31 rows); fewer 64-bit scalars keeps the
  // loop's scalar registers from spilling
  const int ntp = (int)args.ntp;
  int ws, L, s0;
  int64_t tl0 = 0;   // IVF: this block's first entry of the tile list
  if (!SYM && args.tlist) {
    tl0 = args.toff[blk];
    ws = 0;
    L = (int)(args.toff[blk + 1] - tl0);
    s0 = 0;
  } else if (!SYM) {
    if (args.w < 0) {
      ws = 0;
      L = ntp;
      s0 = args.wg_start[blk];
    } else {
      const int lo = args.wlo[blk], hi = args.whi[blk];
      int b0 = lo;
      if (b0 < 0) b0 += args.nwg;
      ws = b0 * TPB;
      L = (hi - lo + 1) * TPB;
      s0 = args.wg_start[blk] - ws;
      if (s0 < 0) s0 += ntp;
      if (s0 >= L) s0 = (blk - lo) * TPB;
    }
  } else {
    const int nwg = (int)args.nwg, bk = (int)blk;
    const int hb = (nwg % 2 == 0 && bk >= nwg / 2) ? nwg / 2 - 1 : nwg / 2;
    const int hi = args.whi[blk];
    ws = ((hi + 1) % args.nwg) * TPB;
    L = blk + hb > hi ? (blk + hb - hi) * TPB : 0;
    s0 = 0;
  }
  const int ntiles = L;
  const uint16_t* __restrict__ Xs = args.Xs;
  const float* __restrict__ invs = args.invs;
  const int32_t* __restrict__ perm = args.perm;
  const float* __restrict__ tile_min = args.tile_min;
  // this thread's 16-byte chunks of a tile: element offsets in global memory and in LDS
  int goff[CPT], loff[CPT];
#pragma unroll
  for (int u = 0; u < CPT; u++) {
    const int c = u * 256 + tid;
    const int r = c / (DP / 8), c8 = c % (DP / 8);
    goff[u] = r * DP + c8 * 8;
    loff[u] = r * LDR + c8 * 8;
  }
  // One register set of the prefetched tile (a native vector type: the HIP uint4 struct keeps
  // such arrays out of registers): step t commits tile t+1 to LDS after its epilogue and then
  // loads tile t+2, so each load has a whole step to arrive.  (A second set, two steps ahead,
  // costs 20 VGPRs and was slower.)
  u32x4 pre[CPT];
  float pre_inv, pre_tmn, pre_thr, pre_tthr;
  int pre_perm;
  // tile of step t of this workgroup's scan: ws + ((s0 + t) mod L), taken mod ntp.  Every step
  // prefetches and commits a tile (past the end the last tile is loaded again, into a buffer no
  // one reads): with no conditional load the compiler needs no wait for stale loads.
#define KNN_TILE_AT(t)                                                                        \
  ([&](int t_) {                                                                          \
    if (!SYM && args.tlist) return (int)args.tlist[tl0 + t_];                                 \
    int u_ = s0 + t_;                                                                         \
    if (u_ >= L) u_ -= L;                                                                     \
    u_ += ws;                                                                                 \
    return u_ >= ntp ? u_ - ntp : u_;                                                         \
  })(t)
#define KNN_STEP_CLAMP(x) ((x) < L ? (x) : (L > 0 ? L - 1 : 0))
#define KNN_PREFETCH(tt)                                                                      \
  {                                                                                           \
    const int tt_ = (tt);                                                                     \
    pre_tmn = tile_min[tt_];                                                                  \
    if (SYM) pre_tthr = args.tile_thr[tt_];                                                   \
    if (TAU) pre_tthr = args.tile_cinv[tt_];                                                  \
    const uint16_t* src_ = Xs + tt_ * (int64_t)(BT_C * DP);                                   \
    _Pragma("unroll") for (int u = 0; u < CPT; u++) pre[u] = *(const u32x4*)(src_ + goff[u]); \
    const int r_ = tt_ * BT_C + (tid & (BT_C - 1));                                           \
    pre_inv = invs[r_];                                                                       \
    pre_perm = perm[r_];                                                                      \
    if (SYM) pre_thr = args.colthr[r_];                                                       \
  }
#define KNN_COMMIT(b)                                                                         \
  {                                                                                           \
    const int b_ = (b);                                                                       \
    uint16_t* dst_ = tileb + b_ * BT_C * LDR;                                                 \
    _Pragma("unroll") for (int u = 0; u < CPT; u++) *(u32x4*)(dst_ + loff[u]) = pre[u];       \
    if (tid < BT_C) {                                                                         \
      tinv[b_ * BT_C + tid] = pre_inv;                                                        \
      tperm[b_ * BT_C + tid] = pre_perm;                                                      \
      if (SYM) tthr[b_ * BT_C + tid] = pre_thr;                                               \
    }                                                                                         \
    if (tid == 0) {                                                                           \
      tmn[b_] = pre_tmn;                                                                      \
      if (SYM || TAU) tmn[2 + b_] = pre_tthr;                                                 \
    }                                                                                         \
  }

  // step 0's tile to buffer 0; the tile of step 1 in flight
  KNN_PREFETCH(KNN_TILE_AT(0));
  KNN_COMMIT(0);
  KNN_PREFETCH(KNN_TILE_AT(KNN_STEP_CLAMP(1)));
  __syncthreads();

  // steps in pairs, so that the LDS buffer s of step t = t0 + s is a compile-time index; an odd
  // last step is followed by one whose epilogue is skipped
  int t0 = 0;
  // the step body, inlined twice per pass of the loop below with its buffer s fixed
  auto step = [&](auto s_tag) __attribute__((always_inline)) {
    constexpr int s = decltype(s_tag)::value;
    const int t = t0 + s;
    const int buf = NBUF == 2 ? s : 0;

    f32x16 acc[2][NQB];
#pragma unroll
    for (int cb = 0; cb < 2; cb++)
#pragma unroll
      for (int qb = 0; qb < NQB; qb++)
#pragma unroll
        for (int i = 0; i < 16; i++) acc[cb][qb][i] = 0.0f;

    const uint16_t* tb = tileb + buf * BT_C * LDR;
    // The tile's A fragments are read from LDS two k-steps ahead of the MFMAs that use them (the
    // scheduling barriers keep the compiler from serialising each read with its MFMAs), and the
    // wave raises its issue priority while it feeds the matrix cores, so that the other wave on
    // the SIMD runs its epilogue meanwhile.
    __builtin_amdgcn_s_setprio(1);
    bf16x8 a[3][2];
#pragma unroll
    for (int kk = 0; kk < 2; kk++)
#pragma unroll
      for (int cb = 0; cb < 2; cb++)
        a[kk][cb] = __builtin_bit_cast(bf16x8, *(const uint4*)(tb + (cb * 32 + l32) * LDR + kk * 16 + half * 8));
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
      if (ks + 2 < KS) {
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
          a[(ks + 2) % 3][cb] =
              __builtin_bit_cast(bf16x8, *(const uint4*)(tb + (cb * 32 + l32) * LDR + (ks + 2) * 16 + half * 8));
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int cb = 0; cb < 2; cb++)
#pragma unroll
        for (int qb = 0; qb < NQB; qb++)
          acc[cb][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks % 3][cb], bq[qb][ks], acc[cb][qb], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_setprio(0);

    // ---- epilogue: filter, then exact insertion for the rare hits
    if (t < ntiles) {
    const float mn = tmn[buf];
    const int tcur_tile = SYM ? KNN_TILE_AT(t) : 0;
#pragma unroll
    for (int qb = 0; qb < NQB; qb++) {
      float m = -INFINITY;
#pragma unroll
      for (int cb = 0; cb < 2; cb++)
#pragma unroll
        for (int i = 0; i < 16; i++) m = fmaxf(m, acc[cb][qb][i]);
      if (TAU) {
        // the lane keeps the TT largest list scores a / |x_j| (a > 0) it sees; a * c, c the
        // tile's smallest 1/|x_j|, is no larger (rounding is monotone) and screens candidates
        // before 1/|x_j| is read
        const float c = tmn[2 + buf];
        if (__ballot(m * c > rt[qb][TT - 1])) {
#pragma unroll
          for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int g = 0; g < 4; g++) {
              const float g4 = fmaxf(fmaxf(acc[cb][qb][4 * g], acc[cb][qb][4 * g + 1]),
                                     fmaxf(acc[cb][qb][4 * g + 2], acc[cb][qb][4 * g + 3]));
              if (g4 * c > rt[qb][TT - 1]) {
#pragma unroll
                for (int r = 0; r < 4; r++) {
                  const float av = acc[cb][qb][4 * g + r];
                  float x = av * tinv[buf * BT_C + cb * 32 + 8 * g + 4 * half + r];
                  if (av > 0.0f && av * c > rt[qb][TT - 1] && x > rt[qb][TT - 1]) {
#pragma unroll
                    for (int j = 0; j < TT; j++) {
                      const float hi = fmaxf(rt[qb][j], x);
                      x = fminf(rt[qb][j], x);
                      rt[qb][j] = hi;
                    }
                  }
                }
              }
            }
        }
        continue;
      }
      const float th = thr[qb];
      const float fth = (th >= 0.0f) ? th * mn * (1.0f - 1e-6f) : (th == INFINITY ? INFINITY : -INFINITY);
      const bool hit = m >= fth;
      if (__ballot(hit)) {
        const int q = qloc[qb];
        const int qi = qorig[qb];
        float* ls = list_s(q);
        int* li = list_i(q);
        for (int h = 0; h < 2; h++) {
          if (hit && half == h) {
            float tcur = wv[qb];
            int tcur_i = wi[qb];
            int wslot = wp[qb];
            // a candidate can enter only if its raw score reaches the tile bound fth (fth is at
            // most the list's worst score times the smallest candidate norm of the tile), so the
            // norm and index of a candidate are read only when that test passes
            // groups of 4 candidates are skipped whole when their largest score misses fth
#pragma unroll
            for (int cb = 0; cb < 2; cb++) {
#pragma unroll
              for (int g = 0; g < 4; g++) {
                const float g4 = fmaxf(fmaxf(acc[cb][qb][4 * g], acc[cb][qb][4 * g + 1]),
                                       fmaxf(acc[cb][qb][4 * g + 2], acc[cb][qb][4 * g + 3]));
                if (g4 >= fth) {
#pragma unroll
                  for (int r = 0; r < 4; r++) {
                    const int i = 4 * g + r;
                    const float a = acc[cb][qb][i];
                    if (a >= fth) {
                      const int cl = buf * BT_C + cb * 32 + 8 * g + 4 * half + r;
                      const float iv = tinv[cl];
                      const int jp = tperm[cl];
                      const float sc = a * iv;
                      // below the bound tq no candidate can end in the list
                      if (iv > 0.0f && jp != qi && sc >= tq[qb] && better<float>(sc, jp, tcur, tcur_i)) {
                        const ListWorst nw = list_replace_worst(ls, li, KPP, sc, jp, ListWorst{tcur, tcur_i, wslot});
                        tcur = nw.s;
                        tcur_i = nw.j;
                        wslot = nw.p;
                      }
                    }
                  }
                }
              }
            }
            wv[qb] = tcur;
            wi[qb] = tcur_i;
            wp[qb] = wslot;
          }
          // the two halves of the wave update the same lists in turn; the other half's lanes
          // take over the worst-entry record (lane l and l ^ 32 hold the same query).  LDS
          // operations of one wave execute in program order, so only the compiler must keep
          // them in order; a memory fence here would also wait for the next tile's global loads.
          // Lists in global memory need that fence: the other half reads what this one wrote.
          if (LG) __threadfence_block();
          {
            const float ov = __shfl_xor(wv[qb], 32, ANCKA_WAVE);
            const int oi = __shfl_xor(wi[qb], 32, ANCKA_WAVE);
            const int op = __shfl_xor(wp[qb], 32, ANCKA_WAVE);
            if (half != h) {
              wv[qb] = ov;
              wi[qb] = oi;
              wp[qb] = op;
            }
          }
          asm volatile("" ::: "memory");
        }
        if (thr[qb] != INFINITY) thr[qb] = fmaxf(wv[qb], tq[qb]);
      }
      if (SYM) {
        // candidate side: the lane's query i is a candidate of the 32 tile rows j it holds
        // scores for, with raw score a / |x_i| in row j's units.  Since rounding is monotone,
        // fl(m / |x_i|) below the tile's smallest threshold excludes all 32.
        const float cq = colq[qb];
        const bool ch = cq > 0.0f && m * cq >= tmn[2 + buf];
        if (__ballot(ch)) {
          uint32_t mask = 0;
          if (ch) {
#pragma unroll 1
            for (int b = 0; b < 32; b++) {
              const int i = b & 15;
              const float sc = (b < 16 ? acc[0][qb][i] : acc[1][qb][i]) * cq;
              if (sc >= tthr[buf * BT_C + (b >> 4) * 32 + 8 * (i / 4) + 4 * half + (i % 4)]) mask |= 1u << b;
            }
          }
          // slots in the hand-over buffer: wave prefix sum of the counts, one atomic per wave
          const int cnt = __popc(mask);
          int incl = cnt;
#pragma unroll
          for (int o = 1; o < ANCKA_WAVE; o <<= 1) {
            const int v = __shfl_up(incl, o, ANCKA_WAVE);
            if (lane >= o) incl += v;
          }
          const int tot = __shfl(incl, ANCKA_WAVE - 1, ANCKA_WAVE);
          unsigned long long base = 0;
          if (lane == ANCKA_WAVE - 1 && tot > 0) base = atomicAdd(args.hcount, (unsigned long long)tot);
          const unsigned lo = __shfl((unsigned)(base & 0xffffffffu), ANCKA_WAVE - 1, ANCKA_WAVE);
          const unsigned hi = __shfl((unsigned)(base >> 32), ANCKA_WAVE - 1, ANCKA_WAVE);
          uint64_t slot = (((uint64_t)hi << 32) | lo) + (uint64_t)(incl - cnt);
          const uint64_t row0 = (uint64_t)tcur_tile * BT_C + 4 * half;
          const uint64_t hv = (uint64_t)(uint32_t)qorig[qb] << 32;
          // a wave-uniform loop over the 32 positions keeps this rare path compact
#pragma unroll 1
          for (int b = 0; b < 32; b++) {
            if (mask & (1u << b)) {
              const int i = b & 15;
              const float sc = (b < 16 ? acc[0][qb][i] : acc[1][qb][i]) * cq;
              if (slot < (uint64_t)args.hcap) {
                args.hkey[slot] = row0 + (b >> 4) * 32 + 8 * (i / 4) + (i % 4);
                args.hval[slot] = hv | __float_as_uint(sc);
              }
              slot++;
            }
          }
        }
      }
    }

    }  // t < ntiles

    if (NBUF == 2) {
      KNN_COMMIT(buf ^ 1);
      __syncthreads();
    } else {
      __syncthreads();            // every wave is done with the single buffer
      KNN_COMMIT(0);
      __syncthreads();
    }
    KNN_PREFETCH(KNN_TILE_AT(KNN_STEP_CLAMP(t + 2)));
  };
  for (; t0 < ntiles; t0 += 2) {
    step(std::integral_constant<int, 0>{});
    step(std::integral_constant<int, 1>{});
  }

  if (TAU) {
    // The two halves of a lane pair hold disjoint candidates of one query, so their 2 TT
    // values belong to 2 TT distinct candidates (at most one of them the query itself), each
    // with a list score at least the smaller of the two TT-th values.  With 2 TT - 1 >= KP
    // that value is a lower bound of the query's KP-th best list score; -inf when a half saw
    // fewer than TT positive scores, or when KP is too long for TT.
#pragma unroll
    for (int qb = 0; qb < NQB; qb++) {
      const float own = rt[qb][TT - 1];
      const float other = __shfl_xor(own, 32, ANCKA_WAVE);
      const float t = fminf(own, other);
      if (half == 0) args.tau[q0 + qloc[qb]] = (2 * TT - 1 >= KP && t > 0.0f) ? t : -INFINITY;
    }
    return;
  }
  // store the lists (unsorted; the merge kernel sorts them) and, in the window pass, the
  // candidate-side threshold of each row: the worst entry of a full list, at least the bound of
  // the bound pass (both are lower bounds of the row's final KP-th score)
  if (LDSL) {
    __syncthreads();
    for (int e = tid; e < QB * KPP; e += 256) {
      args.lsim[q0 * KPP + e] = lsim[e];
      args.lidx[q0 * KPP + e] = lidx[e];
    }
  }
  if (!SYM) {
#pragma unroll
    for (int qb = 0; qb < NQB; qb++) {
      if (half == 0) {
        const int64_t qs = q0 + qloc[qb];
        const float lw = wi[qb] != INT_MAX ? wv[qb] : -INFINITY;
        args.colthr[qs] = colq[qb] > 0.0f ? fmaxf(lw, tq[qb]) : INFINITY;
      }
    }
  }
}

#undef KNN_TILE_AT
#undef KNN_STEP_CLAMP
#undef KNN_PREFETCH
#undef KNN_COMMIT

__global__ void fill_i64_kernel(int64_t* __restrict__ a, int64_t count, int64_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) a[i] = v;
}

// smallest candidate-side threshold of each tile
__global__ void tile_thr_kernel(const float* __restrict__ colthr, int64_t ntp, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntp) return;
  float m = INFINITY;
  for (int r = 0; r < BT_C; r++) m = fminf(m, colthr[t * BT_C + r]);
  out[t] = m;
}

// first hand-over entry of each row in the sorted keys (rows without entries keep -1)
__global__ void handover_starts_kernel(const uint64_t* __restrict__ hkey, int64_t hn, int64_t* __restrict__ start) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= hn) return;
  if (e == 0 || hkey[e] != hkey[e - 1]) start[hkey[e]] = e;
}

// Final lists: row p's list merged with the hand-over entries of row p (hkey sorted, hn
// entries, the first at start[p]), sorted best first, then written at the original index with
// scores scaled by 1/|x_p| to cosines.  One thread per row, RB rows per workgroup; the result
// is the top KP of the union under the (score, index) order, whatever order the entries arrive in.
__global__ __launch_bounds__(256) void knn_merge_kernel(int64_t n, int KP, int RB, const int32_t* __restrict__ lidx,
                                                        const float* __restrict__ lsim, const float* __restrict__ invs,
                                                        const int32_t* __restrict__ perm,
                                                        const uint64_t* __restrict__ hkey,
                                                        const uint64_t* __restrict__ hval, int64_t hn,
                                                        const int64_t* __restrict__ start,
                                                        int32_t* __restrict__ cand_idx, float* __restrict__ cand_sim) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int KPP = (KP + 3) & ~3;
  const int64_t p0 = (int64_t)blockIdx.x * RB;
  const int64_t p = p0 + threadIdx.x;
  float* lsb = (float*)smem;
  int* lib = (int*)((float*)smem + RB * KPP);
  // the block's RB lists are contiguous (KPP slots each): load them into LDS with consecutive
  // threads on consecutive entries
  const int64_t rows = (n - p0) < RB ? (n - p0) : RB;
  for (int e = threadIdx.x; e < RB * KPP; e += RB) {
    const bool in = e / KPP < rows;
    lsb[e] = in ? lsim[p0 * KPP + e] : INFINITY;
    lib[e] = in ? lidx[p0 * KPP + e] : -1;
  }
  __syncthreads();
  if (p >= n) return;   // no barrier below: each thread works on its own slice of LDS
  float* ls = lsb + threadIdx.x * KPP;
  int* li = lib + threadIdx.x * KPP;
  const int64_t e0 = hn > 0 ? start[p] : -1;
  if (e0 >= 0) {
    float ws;
    int wj, wp;
    list_worst(ls, li, KPP, ws, wj, wp);
    for (int64_t e = e0; e < hn && hkey[e] == (uint64_t)p; e++) {
      const uint64_t v = hval[e];
      const float s = __uint_as_float((uint32_t)(v & 0xffffffffu));
      const int j = (int)(v >> 32);
      if (better<float>(s, j, ws, wj)) {
        const ListWorst nw = list_replace_worst(ls, li, KPP, s, j, ListWorst{ws, wj, wp});
        ws = nw.s;
        wj = nw.j;
        wp = nw.p;
      }
    }
  }
  // (slots KP.. hold (+inf, -1) and are never replaced: the list is the first KP slots)
  for (int r = 1; r < KP; r++) {
    const float sr = ls[r];
    const int jr = li[r];
    int b = r;
    while (b > 0 && better<float>(sr, jr, ls[b - 1], li[b - 1])) {
      ls[b] = ls[b - 1];
      li[b] = li[b - 1];
      b--;
    }
    ls[b] = sr;
    li[b] = jr;
  }
  const int qi = perm[p];
  const float iq = invs[p];
  for (int r = 0; r < KP; r++) {
    const int j = li[r];
    cand_idx[(int64_t)qi * KP + r] = (j == INT_MAX) ? -1 : j;
    cand_sim[(int64_t)qi * KP + r] = (j == INT_MAX) ? 0.0f : ls[r] * iq;
  }
}

// cell of each row: the most similar of npiv pivots (dot with the pivot scaled by its inverse
// norm; ties to the smaller pivot).  Pivots come as a bf16 matrix Pm (npiv x dp, dp = d rounded up
// to 8, zero padded) with inverse norms pinv_g; they are held in LDS NPIV at a time; a thread owns
// a row and sweeps it 8 elements at a time against every pivot of the chunk.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

template <typename TX>
__global__ __launch_bounds__(256) void cell_assign_kernel(const TX* __restrict__ X, int64_t n, int64_t d,
                                                          int64_t ldx, const uint16_t* __restrict__ Pm,
                                                          const float* __restrict__ pinv_g, int npiv,
                                                          uint64_t* __restrict__ keys,
                                                          const float* __restrict__ nrm, uint64_t* __restrict__ vals) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int dp = (int)((d + 7) / 8 * 8);
  uint16_t* P = (uint16_t*)smem;            // [NPIV][dp]
  float* pinv = (float*)(P + NPIV * dp);    // [NPIV]
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const TX* xr = X + (i < n ? i : 0) * ldx;
  int best = 0;
  float bv = -INFINITY;
  for (int p0 = 0; p0 < npiv; p0 += NPIV) {
    const int np = npiv - p0 < NPIV ? npiv - p0 : NPIV;
    __syncthreads();   // the previous chunk is no longer read
    for (int e = threadIdx.x; e < NPIV * dp; e += 256) {
      const int p = e / dp;
      P[e] = p < np ? Pm[(int64_t)p0 * dp + e] : (uint16_t)0;
    }
    if (threadIdx.x < NPIV) pinv[threadIdx.x] = threadIdx.x < np ? pinv_g[p0 + threadIdx.x] : 0.0f;
    __syncthreads();
    if (i < n) {
      float acc[NPIV];
#pragma unroll
      for (int p = 0; p < NPIV; p++) acc[p] = 0.0f;
      for (int c0 = 0; c0 < dp; c0 += 8) {
        float xv[8];
#pragma unroll
        for (int u = 0; u < 8; u++) xv[u] = (c0 + u < d) ? (float)load_as_double<TX>(xr, c0 + u) : 0.0f;
#pragma unroll
        for (int p = 0; p < NPIV; p++) {
          const uint4 pv = *(const uint4*)(P + p * dp + c0);
          const uint32_t w[4] = {pv.x, pv.y, pv.z, pv.w};
#pragma unroll
          for (int u = 0; u < 4; u++) {
            acc[p] = fmaf(xv[2 * u], __uint_as_float(w[u] << 16), acc[p]);
            acc[p] = fmaf(xv[2 * u + 1], __uint_as_float(w[u] & 0xffff0000u), acc[p]);
          }
        }
      }
#pragma unroll
      for (int p = 0; p < NPIV; p++) {
        const float v = acc[p] * pinv[p];
        if (p < np && (v > bv || (p0 == 0 && p == 0))) {
          bv = v;
          best = p0 + p;
        }
      }
    }
  }
  if (i >= n) return;
  keys[i] = ((uint64_t)best << 32) | (uint64_t)__float_as_uint(nrm[i]);
  vals[i] = (uint64_t)i;
}

// ---- IVF coarse quantiser (the approximate branch of Alg. 6, for n beyond the exact n^2 budget) -
// Pivot c is the first non-zero row at or after row c n / nlist (rows are in no particular order,
// so this is a sample of the rows); each row's list is its most similar pivot (cell_assign_kernel).
__global__ void ivf_pivots_kernel(const float* __restrict__ invn, int64_t n, int nlist, int64_t* __restrict__ piv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nlist) return;
  const int64_t r0 = (int64_t)((double)c * (double)n / nlist);
  int64_t r = r0;
  while (r < n && !(invn[r] > 0.0f)) r++;
  piv[c] = r < n ? r : r0;
}

// Training sample of the coarse quantiser: row s n / S of X for s < S (a sample of the rows, which
// are in no particular order), with its inverse norm and norm
__global__ void ivf_sample_kernel(const uint16_t* __restrict__ X, int64_t n, int64_t d, int64_t ldx, int64_t S,
                                  const float* __restrict__ invn, const float* __restrict__ nrm,
                                  uint16_t* __restrict__ Xsm, float* __restrict__ invs_s, float* __restrict__ nrm_s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * d) return;
  const int64_t s = e / d, c = e % d;
  const int64_t r = (int64_t)((double)s * (double)n / (double)S);
  Xsm[e] = X[r * ldx + c];
  if (c == 0) {
    invs_s[s] = invn[r];
    nrm_s[s] = nrm[r];
  }
}

// Pm[p] = row piv[p] of X rounded to bf16 (zero padded to dp), pinv[p] = its inverse norm
template <typename TX>
__global__ void gather_pivots_kernel(const TX* __restrict__ X, int64_t d, int64_t ldx, const float* __restrict__ invn,
                                     const int64_t* __restrict__ piv, int npiv, int dp, uint16_t* __restrict__ Pm,
                                     float* __restrict__ pinv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)npiv * dp) return;
  const int p = (int)(e / dp), c = (int)(e % dp);
  Pm[e] = c < d ? f32_to_bf16_rne((float)load_as_double<TX>(X, piv[p] * ldx + c)) : (uint16_t)0;
  if (c == 0) pinv[p] = invn[piv[p]];
}

// One Lloyd step of the spherical k-means that trains the coarse quantiser: centroid c = the
// normalised sum of the unit rows of list c (rows order[cs[c]] .. order[cs[c+1]-1], summed in that
// order by each column's thread), rounded to bf16, with the inverse norm of the rounded vector.
// An empty list keeps its centroid.  One workgroup per list.
__global__ __launch_bounds__(256) void ivf_centroid_kernel(const uint16_t* __restrict__ X, int64_t d, int64_t ldx,
                                                           const float* __restrict__ invn,
                                                           const uint64_t* __restrict__ order,
                                                           const int64_t* __restrict__ cs, int dp,
                                                           uint16_t* __restrict__ Pm, float* __restrict__ pinv) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  const int64_t b = cs[c], e = cs[c + 1];
  if (e <= b) return;
  float acc[2] = {0.0f, 0.0f};   // columns threadIdx.x and threadIdx.x + 256 (d <= 512)
  for (int64_t p = b; p < e; p++) {
    const int64_t r = (int64_t)order[p];
    const float iv = invn[r];
#pragma unroll
    for (int u = 0; u < 2; u++) {
      const int col = threadIdx.x + 256 * u;
      if (col < d) acc[u] = fmaf(bf16_to_f32(X[r * ldx + col]), iv, acc[u]);
    }
  }
  uint16_t q[2];
  float sq = 0.0f;
  red[threadIdx.x] = acc[0] * acc[0] + acc[1] * acc[1];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const float nr = sqrtf(red[0]);
  __syncthreads();
  if (!(nr > 0.0f)) return;
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const int col = threadIdx.x + 256 * u;
    q[u] = f32_to_bf16_rne(acc[u] / nr);
    const float v = bf16_to_f32(q[u]);
    if (col < d) sq = fmaf(v, v, sq);
    if (col < dp) Pm[(int64_t)c * dp + col] = col < d ? q[u] : (uint16_t)0;
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) pinv[c] = red[0] > 0.0f ? 1.0f / sqrtf(red[0]) : 0.0f;
}

// Probe lists: for pivot c, the nprobe pivots of largest cosine with it (c itself first: its
// cosine is 1), ties to the smaller pivot.  One thread per pivot, the list in LDS.
__global__ __launch_bounds__(64) void ivf_probe_kernel(const uint16_t* __restrict__ Pm, const float* __restrict__ pinv,
                                                      int64_t d, int dp, int nlist, int nprobe,
                                                      int32_t* __restrict__ probes) {
  __shared__ float ls[64][65];
  __shared__ int li[64][65];
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= nlist) return;
  float* s = ls[threadIdx.x];
  int* l = li[threadIdx.x];
  int cnt = 0;
  const uint16_t* xc = Pm + (int64_t)c * dp;
  const float ic = pinv[c];
  for (int j = 0; j < nlist; j++) {
    float v;
    if (j == c) {
      v = INFINITY;   // the own cell first
    } else {
      const uint16_t* xj = Pm + (int64_t)j * dp;
      float dot = 0.0f;
      for (int64_t e = 0; e < d; e++) dot = fmaf(bf16_to_f32(xc[e]), bf16_to_f32(xj[e]), dot);
      v = dot * ic * pinv[j];
    }
    // insertion into the sorted list (value desc, index asc) of at most nprobe entries
    if (cnt < nprobe || v > s[cnt - 1]) {
      int q = cnt < nprobe ? cnt++ : nprobe - 1;
      while (q > 0 && v > s[q - 1]) {
        s[q] = s[q - 1];
        l[q] = l[q - 1];
        q--;
      }
      s[q] = v;
      l[q] = j;
    }
  }
  for (int q = 0; q < nprobe; q++) probes[(int64_t)c * nprobe + q] = q < cnt ? l[q] : -1;
}

// ---- pivots of the coarse cells: farthest-point sampling -------------------------------------
// Over S evenly spaced rows (sample s is row s*n/S): the first pivot is the first non-zero sample;
// each next one is the sample whose largest cosine with the pivots chosen so far is smallest
// (ties to the smaller sample).  Zero rows are never chosen.  Well-separated groups of rows then
// each receive a pivot before any group receives a second one, so a coarse cell rarely mixes
// groups.  Iteration `it` folds pivot it into every sample's largest cosine (it = -1: start)
// and leaves each block's arg-min; the select kernel takes the overall arg-min as pivot it+1.
constexpr int FPS_S = 8192;

__global__ __launch_bounds__(256) void fps_update_kernel(const uint16_t* __restrict__ X, int64_t n, int64_t d,
                                                         int64_t ldx, int vec, const float* __restrict__ invn, int S,
                                                         const int64_t* __restrict__ piv, int it,
                                                         float* __restrict__ ms, float* __restrict__ bval,
                                                         int* __restrict__ bidx) {
  __shared__ float pv[512];
  __shared__ float wv[4];
  __shared__ int wi[4];
  const int tid = threadIdx.x;
  const int s = blockIdx.x * 256 + tid;
  if (it >= 0) {
    const int64_t pr = piv[it];
    const float pi = invn[pr];
    for (int c = tid; c < d; c += 256) pv[c] = bf16_to_f32(X[pr * ldx + c]) * pi;
  }
  __syncthreads();
  float v = INFINITY;
  int si = INT_MAX;
  if (s < S) {
    const int64_t r = (int64_t)s * n / S;
    float m;
    if (it < 0) {
      m = invn[r] > 0.0f ? -INFINITY : INFINITY;
    } else {
      m = ms[s];
      if (m != INFINITY) {
        const uint16_t* xr = X + r * ldx;
        float dot = 0.0f;
        int64_t c = 0;
        if (vec) {
          for (; c + 8 <= d; c += 8) {
            const uint4 w = *(const uint4*)(xr + c);
            const uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int u = 0; u < 4; u++) {
              dot = fmaf(__uint_as_float(q[u] << 16), pv[c + 2 * u], dot);
              dot = fmaf(__uint_as_float(q[u] & 0xffff0000u), pv[c + 2 * u + 1], dot);
            }
          }
        }
        for (; c < d; c++) dot = fmaf(bf16_to_f32(xr[c]), pv[c], dot);
        m = fmaxf(m, dot * invn[r]);
      }
      ms[s] = m;
    }
    if (it < 0) ms[s] = m;
    v = m;
    si = s;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(v, o, ANCKA_WAVE);
    const int oi = __shfl_xor(si, o, ANCKA_WAVE);
    if (ov < v || (ov == v && oi < si)) {
      v = ov;
      si = oi;
    }
  }
  if (tid % ANCKA_WAVE == 0) {
    wv[tid / ANCKA_WAVE] = v;
    wi[tid / ANCKA_WAVE] = si;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; w++)
      if (wv[w] < v || (wv[w] == v && wi[w] < si)) {
        v = wv[w];
        si = wi[w];
      }
    bval[blockIdx.x] = v;
    bidx[blockIdx.x] = si;
  }
}

// pivot it = the sample with the smallest value over the nb (<= 64) block candidates
__global__ void fps_select_kernel(const float* __restrict__ bval, const int* __restrict__ bidx, int nb, int64_t n,
                                  int S, int64_t* __restrict__ piv, int it) {
  const int lane = threadIdx.x;
  float v = lane < nb ? bval[lane] : INFINITY;
  int si = lane < nb ? bidx[lane] : INT_MAX;
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(v, o, ANCKA_WAVE);
    const int oi = __shfl_xor(si, o, ANCKA_WAVE);
    if (ov < v || (ov == v && oi < si)) {
      v = ov;
      si = oi;
    }
  }
  if (lane == 0) piv[it] = si == INT_MAX ? 0 : (int64_t)si * n / S;
}

// Xs[p] = zero-padded bf16 row X[perm[p]], invs[p] = 1/|x_perm[p]|, perm[p]; rows n..npad-1
// are zero with invs 0 and perm -1
__global__ __launch_bounds__(256) void gather_sorted_kernel(const uint16_t* __restrict__ X, int64_t n, int64_t npad,
                                                            int64_t d,
                                                            int64_t ldx, const uint64_t* __restrict__ order,
                                                            const float* __restrict__ invn, int DP,
                                                            uint16_t* __restrict__ Xs, float* __restrict__ invs,
                                                            int32_t* __restrict__ perm) {
  const int64_t p = (int64_t)blockIdx.x * 4 + threadIdx.x / ANCKA_WAVE;
  const int lane = threadIdx.x % ANCKA_WAVE;
  if (p >= npad) return;
  uint16_t* xs = Xs + p * (int64_t)DP;
  if (p >= n) {   // padding row
    for (int c = lane; c < DP; c += ANCKA_WAVE) xs[c] = (uint16_t)0;
    if (lane == 0) {
      invs[p] = 0.0f;
      perm[p] = -1;
    }
    return;
  }
  const int64_t i = (int64_t)order[p];
  const uint16_t* xr = X + i * ldx;
  for (int c = lane; c < DP; c += ANCKA_WAVE) xs[c] = (c < d) ? xr[c] : (uint16_t)0;
  if (lane == 0) {
    invs[p] = invn[i];
    perm[p] = (int32_t)i;
  }
}

// per tile of ordered candidates: the smallest norm of a non-zero row (+inf if none) and the
// smallest inverse norm of a non-zero row (0 if none)
__global__ void tile_min_sorted_kernel(const float* __restrict__ invs, int64_t n, int tile, float* __restrict__ out,
                                       float* __restrict__ cinv, int64_t ntiles) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  float m = INFINITY, c = INFINITY;
  for (int64_t j = t * tile; j < n && j < (t + 1) * tile; j++) {
    const float iv = invs[j];
    if (iv > 0.0f) {
      m = fminf(m, 1.0f / iv);
      c = fminf(c, iv);
    }
  }
  // 1/iv rounds; shrink by a few ulps so the bound stays below every |x_j| as seen through 1/|x_j|
  out[t] = m * (1.0f - 4e-7f);
  cinv[t] = c == INFINITY ? 0.0f : c;
}

// cs[c] = first sorted position of cell c (keys sorted by cell << 32 | norm), cs[ncell] = n
__global__ void cell_starts_kernel(const uint64_t* __restrict__ keys, int64_t n, int ncell, int64_t* __restrict__ cs) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > ncell) return;
  const uint64_t target = (uint64_t)c << 32;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  cs[c] = lo;
}

// first tile of each workgroup's scan: the tile holding the first row of the group of its first
// query (the cell: the sorted key shifted right by `shift`)
__global__ void wg_start_kernel(const uint64_t* __restrict__ keys, int64_t n, int qb, int64_t nwg, int shift,
                                int32_t* __restrict__ start) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nwg) return;
  const uint64_t cell = keys[b * qb] >> shift;
  const uint64_t target = cell << shift;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  start[b] = (int32_t)(lo / BT_C);
}

__global__ void u64_to_i32_kernel(const uint64_t* __restrict__ a, int64_t n, int32_t* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (int32_t)a[i];
}

// ---- FP64 rescoring of the candidate lists + certificate --------------------------------------
// One wave per row.  s_ij = dot / sqrt(|x_i|^2 |x_j|^2) with the dot accumulated in FP64 by
// lanes over d and reduced by a butterfly (identical for (i,j) and (j,i)).
template <typename TX>
__device__ __forceinline__ double exact_dot(const TX* __restrict__ X, int64_t ldx, int64_t d, int64_t i, int64_t j,
                                            int lane) {
  double acc = 0.0;
  const TX* xi = X + i * ldx;
  const TX* xj = X + j * ldx;
  for (int64_t c = lane; c < d; c += ANCKA_WAVE) acc += load_as_double<TX>(xi, c) * load_as_double<TX>(xj, c);
  return wave_sum(acc);
}

// bitonic sort of 64 (s, j) pairs across a wave, best first
__device__ __forceinline__ void wave_sort_desc(double& s, int& j, int lane) {
  for (int k = 2; k <= 64; k <<= 1) {
    for (int st = k >> 1; st > 0; st >>= 1) {
      const double so = __shfl_xor(s, st, 64);
      const int jo = __shfl_xor(j, st, 64);
      const bool up = ((lane & k) == 0);          // this block sorted best-first
      const bool lower = ((lane & st) == 0);
      const bool mine_better = better<double>(s, j, so, jo);
      // lower element of the pair should hold the better one in an "up" block
      const bool keep = (lower == up) ? mine_better : !mine_better;
      if (!keep) {
        s = so;
        j = jo;
      }
    }
  }
}

// bitonic sort of 128 (s, j) pairs across a wave, two per lane: element e = slot * 64 + lane
// (slot 0: (s0, j0), slot 1: (s1, j1)); best first in e order, so the best 64 end in slot 0
__device__ __forceinline__ void wave_sort_desc128(double& s0, int& j0, double& s1, int& j1, int lane) {
  for (int k = 2; k <= 128; k <<= 1) {
    for (int st = k >> 1; st > 0; st >>= 1) {
      if (st == 64) {
        // partner of element e is e ^ 64: the other slot of the same lane; k = 128 (one block)
        if (better<double>(s1, j1, s0, j0)) {
          const double ts = s0;
          const int tj = j0;
          s0 = s1;
          j0 = j1;
          s1 = ts;
          j1 = tj;
        }
        continue;
      }
#pragma unroll
      for (int slot = 0; slot < 2; slot++) {
        double& s = slot ? s1 : s0;
        int& j = slot ? j1 : j0;
        const int e = slot * 64 + lane;
        const double so = __shfl_xor(s, st, 64);
        const int jo = __shfl_xor(j, st, 64);
        const bool up = ((e & k) == 0);
        const bool lower = ((e & st) == 0);
        const bool mine_better = better<double>(s, j, so, jo);
        const bool keep = (lower == up) ? mine_better : !mine_better;
        if (!keep) {
          s = so;
          j = jo;
        }
      }
    }
  }
}

template <typename TX>
__global__ __launch_bounds__(256) void knn_rescore_kernel(const TX* __restrict__ X, int64_t n, int64_t d, int64_t ldx,
                                                          const double* __restrict__ sq, int KP, int K,
                                                          const int32_t* __restrict__ cand_idx,
                                                          const float* __restrict__ cand_sim, double eps,
                                                          int32_t* __restrict__ nbr_idx, float* __restrict__ nbr_sim,
                                                          int32_t* __restrict__ uncert_rows,
                                                          unsigned int* __restrict__ uncert_count) {
  const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / ANCKA_WAVE;
  const int lane = threadIdx.x % ANCKA_WAVE;
  if (i >= n) return;
  // candidate r is held by lane r % 64 in slot r / 64 (KP <= 128)
  double my_s = -INFINITY, my_s2 = -INFINITY;
  int my_j = INT_MAX, my_j2 = INT_MAX;
  int valid = 0;
  const double sqi = sq[i];
  const TX* xi = X + i * ldx;
  // four candidates at a time, so that their row gathers and reductions overlap; each dot is
  // accumulated exactly as exact_dot does (lane order over d, then the butterfly)
  for (int r0 = 0; r0 < KP; r0 += 4) {
    int jj[4];
    double acc[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      jj[q] = (r0 + q < KP) ? cand_idx[i * KP + r0 + q] : -1;
      acc[q] = 0.0;
    }
    for (int64_t c = lane; c < d; c += ANCKA_WAVE) {
      const double a = load_as_double<TX>(xi, c);
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (jj[q] >= 0) acc[q] += a * load_as_double<TX>(X + (int64_t)jj[q] * ldx, c);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const double dot = wave_sum(acc[q]);
      if (jj[q] < 0) continue;
      valid++;
      const double s = dot / sqrt(sqi * sq[jj[q]]);
      if (lane == r0 + q) {
        my_s = s;
        my_j = jj[q];
      } else if (lane + 64 == r0 + q) {
        my_s2 = s;
        my_j2 = jj[q];
      }
    }
  }
  if (KP <= 64) wave_sort_desc(my_s, my_j, lane);
  else wave_sort_desc128(my_s, my_j, my_s2, my_j2, lane);
  if (lane < K) {   // K <= KP / 2 <= 64: the best K are in slot 0
    const bool ok = my_j != INT_MAX;
    nbr_idx[i * K + lane] = ok ? my_j : -1;
    nbr_sim[i * K + lane] = ok ? (float)my_s : 0.0f;
  }
  // certificate (only when the list was full: otherwise it holds every candidate)
  const double sK = __shfl(my_s, K - 1, 64);
  if (lane == 0 && valid == KP) {
    const double a = (double)cand_sim[i * KP + KP - 1];
    if (!(sK > a + eps)) {
      const unsigned int slot = atomicAdd(uncert_count, 1u);
      uncert_rows[slot] = (int32_t)i;
    }
  }
}

// ---- exact recompute of uncertified rows: one workgroup per row, every candidate ------------
template <typename TX>
__global__ __launch_bounds__(256) void knn_exact_rows_kernel(const TX* __restrict__ X, int64_t n, int64_t d,
                                                             int64_t ldx, const double* __restrict__ sq, int K,
                                                             const int32_t* __restrict__ rows,
                                                             int32_t* __restrict__ nbr_idx, float* __restrict__ nbr_sim) {
  __shared__ double ls[4][64];
  __shared__ int li[4][64];
  const int wave = threadIdx.x / ANCKA_WAVE;
  const int lane = threadIdx.x % ANCKA_WAVE;
  const int64_t i = rows[blockIdx.x];
  const double sqi = sq[i];
  // wave-private list in lanes: (s, j) sorted best-first across lanes 0..K-1
  double s_l = -INFINITY;
  int j_l = INT_MAX;
  double thr = -INFINITY;
  int thr_i = INT_MAX;
  for (int64_t j = wave; j < n; j += 4) {
    if (j == i) continue;
    const double sqj = sq[j];
    if (sqj == 0.0) continue;
    const double dot = exact_dot<TX>(X, ldx, d, i, j, lane);
    const double s = dot / sqrt(sqi * sqj);
    if (better<double>(s, (int)j, thr, thr_i)) {
      // insert: lanes with a worse element shift down by one
      const bool worse = !better<double>(s_l, j_l, s, (int)j);
      const double s_up = __shfl_up(s_l, 1, 64);
      const int j_up = __shfl_up(j_l, 1, 64);
      const bool worse_up = lane > 0 && !better<double>(s_up, j_up, s, (int)j);
      if (worse) {
        if (worse_up) {
          s_l = s_up;
          j_l = j_up;
        } else {
          s_l = s;
          j_l = (int)j;
        }
      }
      thr = __shfl(s_l, K - 1, 64);
      thr_i = __shfl(j_l, K - 1, 64);
    }
  }
  ls[wave][lane] = (lane < K) ? s_l : -INFINITY;
  li[wave][lane] = (lane < K) ? j_l : INT_MAX;
  __syncthreads();
  if (wave == 0) {
    // merge the 4 lists of K <= 64: the best 64 of lists 0 and 1, of lists 2 and 3, then of
    // those two; the best K end in lanes 0 .. K-1 of slot 0
    double a0 = ls[0][lane], a1 = ls[1][lane], b0 = ls[2][lane], b1 = ls[3][lane];
    int ia0 = li[0][lane], ia1 = li[1][lane], ib0 = li[2][lane], ib1 = li[3][lane];
    wave_sort_desc128(a0, ia0, a1, ia1, lane);
    wave_sort_desc128(b0, ib0, b1, ib1, lane);
    wave_sort_desc128(a0, ia0, b0, ib0, lane);
    if (lane < K) {
      nbr_idx[i * K + lane] = (ia0 == INT_MAX) ? -1 : ia0;
      nbr_sim[i * K + lane] = (ia0 == INT_MAX) ? 0.0f : (float)a0;
    }
  }
}

template <typename TX>
ancka_status run_vector(ancka_ctx* ctx, const TX* X, int64_t n, int64_t d, int64_t ldx, const double* sq,
                        const float* invn, int KP, bool f64, int32_t* cidx, void* csim) {
  const unsigned grid = (unsigned)cdiv(n, VT_Q);
  HIP_TRY(ctx, hipFuncSetAttribute((const void*)knn_vector_kernel<double, TX>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIP_TRY(ctx, hipFuncSetAttribute((const void*)knn_vector_kernel<float, TX>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  if (f64) {
    const size_t sm = sizeof(double) * (2 * VT_D * VT_Q + VT_Q * (VT_C + 1) + VT_Q * KP) + sizeof(int) * VT_Q * KP;
    knn_vector_kernel<double, TX><<<grid, 256, sm, ctx->stream>>>(X, n, d, ldx, sq, invn, KP, 1, cidx, (double*)csim);
  } else {
    const size_t sm = sizeof(float) * (2 * VT_D * VT_Q + VT_Q * (VT_C + 1) + VT_Q * KP) + sizeof(int) * VT_Q * KP;
    knn_vector_kernel<float, TX><<<grid, 256, sm, ctx->stream>>>(X, n, d, ldx, sq, invn, KP, 0, cidx, (float*)csim);
  }
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

template <int DP, int QW>
constexpr int bf16_qb() {
  return 4 * QW;
}
int bf16_qw(int DP) { return DP <= 256 ? 64 : 32; }

template <int DP, int QW, int NBUF, int MODE, bool LG, int TT = TAU_T>
ancka_status launch_bf16(ancka_ctx* ctx, const ScanArgs& args, size_t sm) {
  // the LDS limit is a per-device attribute of the function: set it on every call (cheap), so a
  // context on another device sees it too
  HIP_TRY(ctx, hipFuncSetAttribute((const void*)knn_bf16_kernel<DP, QW, NBUF, MODE, LG, TT>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  knn_bf16_kernel<DP, QW, NBUF, MODE, LG, TT><<<(unsigned)args.nwg, 256, sm, ctx->stream>>>(args);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

template <int DP, int QW, int NBUF, int MODE>
ancka_status run_bf16_t(ancka_ctx* ctx, const ScanArgs& args) {
  constexpr int QB = 4 * QW;
  const int KPP = (args.KP + 3) & ~3;
  const size_t base = (size_t)NBUF * BT_C * (DP + 8) * 2 + 2 * NBUF * BT_C * 4 + 16 + (size_t)NBUF * BT_C * 4;
  const size_t lists = (size_t)QB * KPP * 8;
  // lists stay in LDS while the workgroups per CU the kernel is built for (two up to d = 128, else
  // one) still fit; longer lists are kept in global memory
  const size_t budget = (size_t)160 * 1024 / (DP <= 128 ? 2 : 1);
  if constexpr (MODE == SCAN_TAU) {
    // 2 TT - 1 values bound the list's last entry: 11 per lane up to 21 entries, else 21
    if (args.KP <= 2 * TAU_T - 1) return launch_bf16<DP, QW, NBUF, MODE, false, TAU_T>(ctx, args, base);
    return launch_bf16<DP, QW, NBUF, MODE, false, TAU_T2>(ctx, args, base);
  } else {
    if (base + lists <= budget) return launch_bf16<DP, QW, NBUF, MODE, false>(ctx, args, base + lists);
    return launch_bf16<DP, QW, NBUF, MODE, true>(ctx, args, base);
  }
}

template <int MODE>
ancka_status run_bf16(ancka_ctx* ctx, int DP, const ScanArgs& args) {
  switch (DP) {
    case 32: return run_bf16_t<32, 64, 2, MODE>(ctx, args);
    case 64: return run_bf16_t<64, 64, 2, MODE>(ctx, args);
    case 128: return run_bf16_t<128, 64, 2, MODE>(ctx, args);
    case 256: return run_bf16_t<256, 64, 2, MODE>(ctx, args);
    case 512: return run_bf16_t<512, 32, 1, MODE>(ctx, args);
    default: return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "knn: bf16 path supports d <= 512 (got padded %d)", DP);
  }
}

// Windows of the window pass, per block I as an unwrapped block range [lo, hi] with lo <= I <= hi.
// Default: the blocks of the coarse cells that block I's rows belong to (cells are contiguous
// row ranges cs[c] .. cs[c+1] of the scan order), so a row's window holds its whole cell.  With
// ANCKA_KNN_WINDOW = w: blocks I-w .. I+w.  Both are symmetric (J in I's window iff I in J's).
// Returns false (whole-ring scan instead) when a window would exceed a quarter of the ring, as
// the symmetric pass assumes.
bool scan_windows(int64_t n, int64_t nwg, int QB, const int64_t* hcs, std::vector<int32_t>& lo,
                  std::vector<int32_t>& hi) {
  lo.assign(nwg, 0);
  hi.assign(nwg, 0);
  const int64_t cap = nwg / 4;
  if (const char* e = getenv("ANCKA_KNN_WINDOW")) {
    int64_t w = atoll(e);
    if (w < 0) w = 0;
    if (2 * w + 1 > cap) return false;
    for (int64_t I = 0; I < nwg; I++) {
      lo[I] = (int32_t)(I - w);
      hi[I] = (int32_t)(I + w);
    }
    return true;
  }
  auto cell_of = [&](int64_t p) {   // last cell c with hcs[c] <= p (empty cells skipped)
    int c = 0;
    while (c + 1 < NPIV && hcs[c + 1] <= p) c++;
    return c;
  };
  for (int64_t I = 0; I < nwg; I++) {
    const int64_t p0 = I * QB, p1 = std::min(n, (I + 1) * QB) - 1;
    const int c0 = cell_of(p0), c1 = cell_of(p1);
    lo[I] = (int32_t)(hcs[c0] / QB);
    hi[I] = (I == nwg - 1) ? (int32_t)(nwg - 1) : (int32_t)((hcs[c1 + 1] - 1) / QB);
    if (hi[I] - lo[I] + 1 > cap) return false;
  }
  return true;
}

// Capacity (entries) of the hand-over buffer: ANCKA_KNN_HANDOVER or max(16 n, 2^22).
int64_t handover_capacity(int64_t n) {
  int64_t c = 16 * n > ((int64_t)1 << 22) ? 16 * n : ((int64_t)1 << 22);
  if (const char* e = getenv("ANCKA_KNN_HANDOVER")) c = atoll(e);
  return c < 1 ? 1 : c;
}

// BF16 tile phase: window pass, symmetric pass, sort of the hand-over entries by row, merge.
// If the hand-over buffer overflows the window pass is redone over the whole ring instead.
ancka_status bf16_scan(ancka_ctx* ctx, int DP, ScanArgs args, const std::vector<int32_t>& hlo,
                       const std::vector<int32_t>& hhi, int64_t n, int32_t* cidx, float* csim, ancka_knn_stats* st) {
  hipEvent_t* ev = nullptr;
  ST_TRY(ctx_events(ctx, &ev));
  int64_t hn = 0;
  int64_t* hstart = nullptr;
  bool timed_sym = false;
  if (args.w >= 0 && args.tau) ST_TRY(run_bf16<SCAN_TAU>(ctx, DP, args));
  ST_TRY(run_bf16<SCAN_WIN>(ctx, DP, args));
  if (args.w >= 0) {
    tile_thr_kernel<<<(unsigned)cdiv(args.ntp, 256), 256, 0, ctx->stream>>>(args.colthr, args.ntp,
                                                                             (float*)args.tile_thr);
    LAUNCH_CHECK(ctx);
    ST_TRY(fill_zero(ctx, args.hcount, sizeof(unsigned long long)));
    HIP_TRY(ctx, hipEventRecord(ev[4], ctx->stream));
    ST_TRY(run_bf16<SCAN_SYM>(ctx, DP, args));
    HIP_TRY(ctx, hipEventRecord(ev[5], ctx->stream));
    timed_sym = true;
    unsigned long long hc = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&hc, args.hcount, sizeof(hc), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (st) st->handed_over = (int64_t)hc;
    if ((int64_t)hc > args.hcap) {
      args.w = -1;
      ST_TRY(run_bf16<SCAN_WIN>(ctx, DP, args));
      if (st) st->rescanned = 1;
    } else {
      hn = (int64_t)hc;
      const int64_t npad = args.nwg * 4 * bf16_qw(DP);
      int bits = 1;
      while (bits < 63 && ((int64_t)1 << bits) < npad) bits++;
      ST_TRY(radix_sort_u64(ctx, args.hkey, args.hval, hn, bits));
      ST_TRY(ws_get_t(ctx, "knn_hstart", (size_t)npad, &hstart));
      fill_i64_kernel<<<(unsigned)cdiv(npad, 256), 256, 0, ctx->stream>>>(hstart, npad, -1);
      LAUNCH_CHECK(ctx);
      if (hn > 0) {
        handover_starts_kernel<<<(unsigned)cdiv(hn, 256), 256, 0, ctx->stream>>>(args.hkey, hn, hstart);
        LAUNCH_CHECK(ctx);
      }
    }
  }
  const int KPP = (args.KP + 3) & ~3;
  const int RB = KPP <= 40 ? 256 : 64;   // rows per workgroup: RB lists of KPP slots in LDS
  HIP_TRY(ctx, hipFuncSetAttribute((const void*)knn_merge_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024));
  knn_merge_kernel<<<(unsigned)cdiv(n, RB), RB, (size_t)RB * KPP * 8, ctx->stream>>>(
      n, args.KP, RB, args.lidx, args.lsim, args.invs, args.perm, args.hkey, args.hval, hn, hstart, cidx, csim);
  LAUNCH_CHECK(ctx);
  if (st) {
    int32_t wmax = -1;
    if (args.w >= 0)
      for (size_t I = 0; I < hlo.size(); I++) wmax = std::max(wmax, hhi[I] - hlo[I] + 1);
    st->window = wmax;
    if (timed_sym) {
      HIP_TRY(ctx, hipEventSynchronize(ev[5]));
      float ms = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, ev[4], ev[5]));
      st->sym_ms = ms;
      // unordered pairs of rows the symmetric pass scores (padding rows included)
      const int64_t QB = 4 * bf16_qw(DP), nwg = args.nwg;
      int64_t blocks = 0;
      for (int64_t I = 0; I < nwg; I++) {
        const int64_t hb = (nwg % 2 == 0 && I >= nwg / 2) ? nwg / 2 - 1 : nwg / 2;
        if (I + hb > hhi[I]) blocks += I + hb - hhi[I];
      }
      st->sym_pairs = blocks * QB * QB;
    }
  }
  return ANCKA_OK;
}

template <typename TX>
ancka_status rescore_and_fix(ancka_ctx* ctx, const TX* X, int64_t n, int64_t d, int64_t ldx, const double* sq, int KP,
                             int K, const int32_t* cidx, const float* csim, int32_t* nbr_idx, float* nbr_sim,
                             ancka_knn_stats* st, bool recompute = true) {
  int32_t* urows = nullptr;
  unsigned int* ucount = nullptr;
  ST_TRY(ws_get_t(ctx, "knn_urows", (size_t)n, &urows));
  ST_TRY(ws_get_t(ctx, "knn_ucount", 4, &ucount));
  ST_TRY(fill_zero(ctx, ucount, 4 * sizeof(unsigned int)));
  const double u = ldexp(1.0, -24);
  const double gd = (double)d * u / (1.0 - (double)d * u);
  const double eps = 4.0 * (gd + 4.0 * u);
  knn_rescore_kernel<TX><<<(unsigned)cdiv(n, 4), 256, 0, ctx->stream>>>(X, n, d, ldx, sq, KP, K, cidx, csim, eps,
                                                                        nbr_idx, nbr_sim, urows, ucount);
  LAUNCH_CHECK(ctx);
  unsigned int hcount = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&hcount, ucount, sizeof(unsigned int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (hcount > 0 && recompute) {
    knn_exact_rows_kernel<TX><<<hcount, 256, 0, ctx->stream>>>(X, n, d, ldx, sq, K, urows, nbr_idx, nbr_sim);
    LAUNCH_CHECK(ctx);
  }
  if (st) {
    st->uncertified_rows = hcount;
    st->recomputed_rows = recompute ? hcount : 0;
  }
  return ANCKA_OK;
}

template <typename TX>
ancka_status knn_typed(ancka_ctx* ctx, const TX* X, int64_t n, int64_t d, int64_t ldx, int K, int mode,
                       int32_t* nbr_idx, void* nbr_sim, ancka_knn_stats* st) {
  double* sq = nullptr;
  float *invn = nullptr, *nrm = nullptr;
  unsigned long long* zc = nullptr;
  ST_TRY(ws_get_t(ctx, "knn_sq", (size_t)n, &sq));
  ST_TRY(ws_get_t(ctx, "knn_invn", (size_t)n, &invn));
  ST_TRY(ws_get_t(ctx, "knn_nrm", (size_t)n, &nrm));
  ST_TRY(ws_get_t(ctx, "knn_zero", 2, &zc));
  ST_TRY(fill_zero(ctx, zc, 16));
  int DP = 0;
  if (mode == ANCKA_KNN_BF16_RESCORE) {
    DP = 32;
    while (DP < d) DP *= 2;
    if (DP > 512) return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "knn: bf16 path supports d <= 512");
  }
  hipEvent_t* ev = nullptr;
  ST_TRY(ctx_events(ctx, &ev));
  HIP_TRY(ctx, hipEventRecord(ev[0], ctx->stream));
  knn_prologue_kernel<TX><<<(unsigned)cdiv(n, 4), 256, 0, ctx->stream>>>(X, n, d, ldx, sq, invn, nrm, nullptr, 0, zc);
  LAUNCH_CHECK(ctx);

  if (mode == ANCKA_KNN_EXACT_F64) {
    int KP = K;
    HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
    ST_TRY(run_vector<TX>(ctx, X, n, d, ldx, sq, invn, KP, true, nbr_idx, nbr_sim));
    HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
    if (st) st->uncertified_rows = st->recomputed_rows = 0;
  } else {
    const int KP = 2 * K;
    int32_t* cidx = nullptr;
    float* csim = nullptr;
    ST_TRY(ws_get_t(ctx, "knn_cidx", (size_t)n * KP, &cidx));
    ST_TRY(ws_get_t(ctx, "knn_csim", (size_t)n * KP, &csim));
    if (mode == ANCKA_KNN_EXACT_F32) {
      HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
      ST_TRY(run_vector<TX>(ctx, X, n, d, ldx, sq, invn, KP, false, cidx, csim));
      HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
    } else {
      // scan order: rows grouped by coarse cell (nearest of NPIV pivot rows), by norm inside a
      // cell; a zero-padded bf16 copy Xs in that order serves as queries and candidates
      const int QB = 4 * bf16_qw(DP);
      const int64_t nwg = cdiv(n, QB);
      const int64_t nt = nwg * (QB / BT_C);   // tiles of the padded ring
      float *tmin = nullptr, *invs = nullptr;
      uint64_t *keys = nullptr, *order = nullptr;
      int64_t* piv = nullptr;
      int32_t *perm = nullptr, *wgs = nullptr;
      uint16_t* Xs = nullptr;
      ST_TRY(ws_get_t(ctx, "knn_tmin", (size_t)nt, &tmin));
      ST_TRY(ws_get_t(ctx, "knn_keys", (size_t)n, &keys));
      ST_TRY(ws_get_t(ctx, "knn_order", (size_t)n, &order));
      ST_TRY(ws_get_t(ctx, "knn_piv", NPIV, &piv));
      // sorted copies padded to whole workgroups (QB is a multiple of the tile height)
      const int64_t npad = nwg * QB;
      ST_TRY(ws_get_t(ctx, "knn_invs", (size_t)npad, &invs));
      ST_TRY(ws_get_t(ctx, "knn_perm", (size_t)npad, &perm));
      ST_TRY(ws_get_t(ctx, "knn_wgs", (size_t)nwg, &wgs));
      ST_TRY(ws_get_t(ctx, "knn_xs", (size_t)npad * DP, &Xs));
      // pivots: farthest-point sampling over FPS_S evenly spaced rows
      {
        const int S = (int)std::min<int64_t>(n, FPS_S);
        const int nb = (int)cdiv(S, 256);
        float *fms = nullptr, *fbv = nullptr;
        int* fbi = nullptr;
        ST_TRY(ws_get_t(ctx, "knn_fps_ms", (size_t)S, &fms));
        ST_TRY(ws_get_t(ctx, "knn_fps_bv", (size_t)nb, &fbv));
        ST_TRY(ws_get_t(ctx, "knn_fps_bi", (size_t)nb, &fbi));
        const int vec = (ldx % 8 == 0 && ((uintptr_t)X % 16) == 0) ? 1 : 0;
        const uint16_t* Xb = (const uint16_t*)(const void*)X;
        for (int it = -1; it < NPIV - 1; it++) {
          fps_update_kernel<<<(unsigned)nb, 256, 0, ctx->stream>>>(Xb, n, d, ldx, vec, invn, S, piv, it, fms, fbv,
                                                                   fbi);
          LAUNCH_CHECK(ctx);
          fps_select_kernel<<<1, ANCKA_WAVE, 0, ctx->stream>>>(fbv, fbi, nb, n, S, piv, it + 1);
          LAUNCH_CHECK(ctx);
        }
      }
      const int dp8 = (int)((d + 7) / 8 * 8);
      const size_t csm = (size_t)NPIV * dp8 * 2 + NPIV * 4;
      uint16_t* Pm = nullptr;
      float* pinv = nullptr;
      ST_TRY(ws_get_t(ctx, "knn_pm", (size_t)NPIV * dp8, &Pm));
      ST_TRY(ws_get_t(ctx, "knn_pinv", NPIV, &pinv));
      gather_pivots_kernel<uint16_t><<<(unsigned)cdiv((int64_t)NPIV * dp8, 256), 256, 0, ctx->stream>>>(
          (const uint16_t*)(const void*)X, d, ldx, invn, piv, NPIV, dp8, Pm, pinv);
      LAUNCH_CHECK(ctx);
      HIP_TRY(ctx, hipFuncSetAttribute((const void*)cell_assign_kernel<uint16_t>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
      cell_assign_kernel<uint16_t><<<(unsigned)cdiv(n, 256), 256, csm, ctx->stream>>>(
          (const uint16_t*)(const void*)X, n, d, ldx, Pm, pinv, NPIV, keys, nrm, order);
      LAUNCH_CHECK(ctx);
      ST_TRY(radix_sort_u64(ctx, keys, order, n, 40));
      // cell ranges of the scan order (rows of a cell in norm order: a 64-row tile then spans a
      // narrow band of norms, which keeps the tile filters tight)
      int64_t* cstart = nullptr;
      ST_TRY(ws_get_t(ctx, "knn_cstart", NPIV + 1, &cstart));
      cell_starts_kernel<<<1, 128, 0, ctx->stream>>>(keys, n, NPIV, cstart);
      LAUNCH_CHECK(ctx);
      int64_t hcs[NPIV + 1];
      HIP_TRY(ctx, hipMemcpyAsync(hcs, cstart, sizeof(hcs), hipMemcpyDeviceToHost, ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      gather_sorted_kernel<<<(unsigned)cdiv(npad, 4), 256, 0, ctx->stream>>>((const uint16_t*)(const void*)X, n, npad,
                                                                             d, ldx, order, invn, DP, Xs, invs, perm);
      LAUNCH_CHECK(ctx);
      float* tcinv = nullptr;
      ST_TRY(ws_get_t(ctx, "knn_tcinv", (size_t)nt, &tcinv));
      tile_min_sorted_kernel<<<(unsigned)cdiv(nt, 256), 256, 0, ctx->stream>>>(invs, n, BT_C, tmin, tcinv, nt);
      LAUNCH_CHECK(ctx);
      wg_start_kernel<<<(unsigned)cdiv(nwg, 256), 256, 0, ctx->stream>>>(keys, n, QB, nwg, 32, wgs);
      LAUNCH_CHECK(ctx);
      ScanArgs sa{};
      sa.Xs = Xs;
      sa.invs = invs;
      sa.perm = perm;
      sa.tile_min = tmin;
      sa.wg_start = wgs;
      sa.nwg = nwg;
      sa.ntp = nt;
      std::vector<int32_t> hlo, hhi;
      sa.w = scan_windows(n, nwg, QB, hcs, hlo, hhi) ? 0 : -1;
      sa.KP = KP;

      const int KPP = (KP + 3) & ~3;
      ST_TRY(ws_get_t(ctx, "knn_lidx", (size_t)npad * KPP, &sa.lidx));
      ST_TRY(ws_get_t(ctx, "knn_lsim", (size_t)npad * KPP, &sa.lsim));
      ST_TRY(ws_get_t(ctx, "knn_colthr", (size_t)npad, &sa.colthr));
      if (sa.w >= 0) {
        int32_t *wlo = nullptr, *whi = nullptr;
        ST_TRY(ws_get_t(ctx, "knn_wlo", (size_t)nwg, &wlo));
        ST_TRY(ws_get_t(ctx, "knn_whi", (size_t)nwg, &whi));
        HIP_TRY(ctx, hipMemcpyAsync(wlo, hlo.data(), nwg * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync(whi, hhi.data(), nwg * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        sa.wlo = wlo;
        sa.whi = whi;
        float* tthr = nullptr;
        ST_TRY(ws_get_t(ctx, "knn_tthr", (size_t)nt, &tthr));
        sa.tile_thr = tthr;
        sa.tile_cinv = tcinv;
        if (2 * TAU_T2 - 1 >= KP) ST_TRY(ws_get_t(ctx, "knn_tau", (size_t)npad, &sa.tau));
        sa.hcap = handover_capacity(n);
        ST_TRY(ws_get_t(ctx, "knn_hkey", (size_t)sa.hcap, &sa.hkey));
        ST_TRY(ws_get_t(ctx, "knn_hval", (size_t)sa.hcap, &sa.hval));
        ST_TRY(ws_get_t(ctx, "knn_hcount", 1, &sa.hcount));
      }
      HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
      ST_TRY(bf16_scan(ctx, DP, sa, hlo, hhi, n, cidx, csim, st));
      HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
    }
    ST_TRY(rescore_and_fix<TX>(ctx, X, n, d, ldx, sq, KP, K, cidx, csim, nbr_idx, (float*)nbr_sim, st));
  }
  HIP_TRY(ctx, hipEventRecord(ev[3], ctx->stream));
  if (st) {
    unsigned long long hz = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&hz, zc, sizeof(hz), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    st->zero_rows = (int64_t)hz;
    float a = 0.f, b = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&a, ev[1], ev[2]));
    HIP_TRY(ctx, hipEventElapsedTime(&b, ev[0], ev[3]));
    st->tile_ms = a;
    st->total_ms = b;
  }
  return ANCKA_OK;
}

// ---- IVF search (approximate; the paper's large-n branch of Alg. 6) ------------------------------
constexpr int IVF_LLOYD = 4;     // spherical k-means steps that refine the pivot rows
constexpr int IVF_SAMPLE = 256;  // training rows per list
// Coarse quantiser of nlist pivot rows; rows sorted by (list, norm) form the scan order; block I of
// QB rows scans the tiles of the lists its rows belong to and of the nprobe - 1 lists whose pivots
// are most similar to each of those lists' pivot (own list first), with the window pass's BF16
// tiles and top-2K lists; then FP64 rescoring of the 2K candidates and top K.  Candidates outside
// the probed lists are never seen, so the result is approximate (no exact recompute).
ancka_status ivf_knn(ancka_ctx* ctx, const uint16_t* X, int64_t n, int64_t d, int64_t ldx, int K, int nlist,
                     int nprobe, int32_t* nbr_idx, float* nbr_sim, ancka_knn_stats* st) {
  double* sq = nullptr;
  float *invn = nullptr, *nrm = nullptr;
  unsigned long long* zc = nullptr;
  ST_TRY(ws_get_t(ctx, "knn_sq", (size_t)n, &sq));
  ST_TRY(ws_get_t(ctx, "knn_invn", (size_t)n, &invn));
  ST_TRY(ws_get_t(ctx, "knn_nrm", (size_t)n, &nrm));
  ST_TRY(ws_get_t(ctx, "knn_zero", 2, &zc));
  ST_TRY(fill_zero(ctx, zc, 16));
  int DP = 32;
  while (DP < d) DP *= 2;
  if (DP > 512) return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "ancka_knn_ivf: d <= 512");
  hipEvent_t* ev = nullptr;
  ST_TRY(ctx_events(ctx, &ev));
  HIP_TRY(ctx, hipEventRecord(ev[0], ctx->stream));
  knn_prologue_kernel<uint16_t><<<(unsigned)cdiv(n, 4), 256, 0, ctx->stream>>>(X, n, d, ldx, sq, invn, nrm, nullptr, 0,
                                                                               zc);
  LAUNCH_CHECK(ctx);
  const int KP = 2 * K;
  const int KPP = (KP + 3) & ~3;
  const int QB = 4 * bf16_qw(DP);
  const int64_t nwg = cdiv(n, QB);
  const int64_t nt = nwg * (QB / BT_C);
  const int64_t npad = nwg * QB;
  int64_t* piv = nullptr;
  uint64_t *keys = nullptr, *order = nullptr;
  int64_t* cstart = nullptr;
  int32_t* probes = nullptr;
  ST_TRY(ws_get_t(ctx, "ivf_piv", (size_t)nlist, &piv));
  ST_TRY(ws_get_t(ctx, "knn_keys", (size_t)n, &keys));
  ST_TRY(ws_get_t(ctx, "knn_order", (size_t)n, &order));
  ST_TRY(ws_get_t(ctx, "ivf_cstart", (size_t)nlist + 1, &cstart));
  ST_TRY(ws_get_t(ctx, "ivf_probes", (size_t)nlist * nprobe, &probes));
  ivf_pivots_kernel<<<(unsigned)cdiv(nlist, 256), 256, 0, ctx->stream>>>(invn, n, nlist, piv);
  LAUNCH_CHECK(ctx);
  // coarse quantiser: the pivot rows refined by IVF_LLOYD steps of spherical k-means
  const int dp8 = (int)((d + 7) / 8 * 8);
  uint16_t* Pm = nullptr;
  float* pinv = nullptr;
  ST_TRY(ws_get_t(ctx, "ivf_pm", (size_t)nlist * dp8, &Pm));
  ST_TRY(ws_get_t(ctx, "ivf_pinv", (size_t)nlist, &pinv));
  gather_pivots_kernel<uint16_t><<<(unsigned)cdiv((int64_t)nlist * dp8, 256), 256, 0, ctx->stream>>>(
      X, d, ldx, invn, piv, nlist, dp8, Pm, pinv);
  LAUNCH_CHECK(ctx);
  const size_t csm = (size_t)NPIV * dp8 * 2 + NPIV * 4;
  HIP_TRY(ctx, hipFuncSetAttribute((const void*)cell_assign_kernel<uint16_t>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024));
  int cbits = 1;
  while ((1 << cbits) < nlist) cbits++;
  // k-means steps on a training sample of IVF_SAMPLE rows per list (all rows when n is smaller)
  const int64_t S = std::min<int64_t>(n, (int64_t)IVF_SAMPLE * nlist);
  uint16_t* Xsm = nullptr;
  float *invs_s = nullptr, *nrm_s = nullptr;
  uint64_t *keys_s = nullptr, *order_s = nullptr;
  ST_TRY(ws_get_t(ctx, "ivf_xsm", (size_t)S * d, &Xsm));
  ST_TRY(ws_get_t(ctx, "ivf_invs_s", (size_t)S, &invs_s));
  ST_TRY(ws_get_t(ctx, "ivf_nrm_s", (size_t)S, &nrm_s));
  ST_TRY(ws_get_t(ctx, "ivf_keys_s", (size_t)S, &keys_s));
  ST_TRY(ws_get_t(ctx, "ivf_order_s", (size_t)S, &order_s));
  ivf_sample_kernel<<<(unsigned)cdiv(S * d, 256), 256, 0, ctx->stream>>>(X, n, d, ldx, S, invn, nrm, Xsm, invs_s,
                                                                         nrm_s);
  LAUNCH_CHECK(ctx);
  for (int it = 0; it < IVF_LLOYD; it++) {
    cell_assign_kernel<uint16_t><<<(unsigned)cdiv(S, 256), 256, csm, ctx->stream>>>(Xsm, S, d, d, Pm, pinv, nlist,
                                                                                  keys_s, nrm_s, order_s);
    LAUNCH_CHECK(ctx);
    ST_TRY(radix_sort_u64(ctx, keys_s, order_s, S, 32 + cbits));
    cell_starts_kernel<<<(unsigned)cdiv(nlist + 1, 256), 256, 0, ctx->stream>>>(keys_s, S, nlist, cstart);
    LAUNCH_CHECK(ctx);
    ivf_centroid_kernel<<<(unsigned)nlist, 256, 0, ctx->stream>>>(Xsm, d, d, invs_s, order_s, cstart, dp8, Pm, pinv);
    LAUNCH_CHECK(ctx);
  }
  // every row to its list
  cell_assign_kernel<uint16_t><<<(unsigned)cdiv(n, 256), 256, csm, ctx->stream>>>(X, n, d, ldx, Pm, pinv, nlist,
                                                                                keys, nrm, order);
  LAUNCH_CHECK(ctx);
  ST_TRY(radix_sort_u64(ctx, keys, order, n, 32 + cbits));
  cell_starts_kernel<<<(unsigned)cdiv(nlist + 1, 256), 256, 0, ctx->stream>>>(keys, n, nlist, cstart);
  LAUNCH_CHECK(ctx);
  ivf_probe_kernel<<<(unsigned)cdiv(nlist, 64), 64, 0, ctx->stream>>>(Pm, pinv, d, dp8, nlist, nprobe, probes);
  LAUNCH_CHECK(ctx);
  std::vector<int64_t> hcs(nlist + 1);
  std::vector<int32_t> hpr((size_t)nlist * nprobe);
  HIP_TRY(ctx, hipMemcpyAsync(hcs.data(), cstart, sizeof(int64_t) * (nlist + 1), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(hpr.data(), probes, sizeof(int32_t) * hpr.size(), hipMemcpyDeviceToHost, ctx->stream));
  // sorted copies (bf16 rows, inverse norms, original indices) and per-tile smallest norms
  float *tmin = nullptr, *invs = nullptr, *tcinv = nullptr;
  int32_t* perm = nullptr;
  uint16_t* Xs = nullptr;
  ST_TRY(ws_get_t(ctx, "knn_tmin", (size_t)nt, &tmin));
  ST_TRY(ws_get_t(ctx, "knn_tcinv", (size_t)nt, &tcinv));
  ST_TRY(ws_get_t(ctx, "knn_invs", (size_t)npad, &invs));
  ST_TRY(ws_get_t(ctx, "knn_perm", (size_t)npad, &perm));
  ST_TRY(ws_get_t(ctx, "knn_xs", (size_t)npad * DP, &Xs));
  gather_sorted_kernel<<<(unsigned)cdiv(npad, 4), 256, 0, ctx->stream>>>(X, n, npad, d, ldx, order, invn, DP, Xs, invs,
                                                                         perm);
  LAUNCH_CHECK(ctx);
  tile_min_sorted_kernel<<<(unsigned)cdiv(nt, 256), 256, 0, ctx->stream>>>(invs, n, BT_C, tmin, tcinv, nt);
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  // tile lists of the blocks: the lists of the block's rows (cells c0 .. c1), then the lists each
  // of them probes, in probe order; each tile once
  std::vector<int64_t> toff(nwg + 1, 0);
  std::vector<int32_t> tl;
  tl.reserve((size_t)nwg * nprobe * (size_t)std::max<int64_t>(1, n / nlist / BT_C + 2));
  std::vector<int64_t> seen(nt, -1);
  auto cell_of = [&](int64_t p) {   // last cell c with hcs[c] <= p
    return (int)(std::upper_bound(hcs.begin(), hcs.end(), p) - hcs.begin()) - 1;
  };
  for (int64_t I = 0; I < nwg; I++) {
    const int64_t p0 = I * QB, p1 = std::min(n, (I + 1) * QB) - 1;
    const int c0 = cell_of(p0), c1 = cell_of(p1);
    auto add_cell = [&](int c) {
      if (c < 0 || c >= nlist || hcs[c + 1] <= hcs[c]) return;
      for (int64_t t = hcs[c] / BT_C; t <= (hcs[c + 1] - 1) / BT_C; t++)
        if (seen[t] != I) {
          seen[t] = I;
          tl.push_back((int32_t)t);
        }
    };
    for (int c = c0; c <= c1; c++) add_cell(c);
    for (int q = 1; q < nprobe; q++)
      for (int c = c0; c <= c1; c++) add_cell(hpr[(size_t)c * nprobe + q]);
    toff[I + 1] = (int64_t)tl.size();
    if (toff[I + 1] == toff[I]) return set_err(ctx, ANCKA_ERR_NUMERICAL, "ancka_knn_ivf: block %lld has no tiles", (long long)I);
  }
  int32_t* dtl = nullptr;
  int64_t* dtoff = nullptr;
  ST_TRY(ws_get_t(ctx, "ivf_tlist", tl.size(), &dtl));
  ST_TRY(ws_get_t(ctx, "ivf_toff", (size_t)nwg + 1, &dtoff));
  HIP_TRY(ctx, hipMemcpyAsync(dtl, tl.data(), sizeof(int32_t) * tl.size(), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(dtoff, toff.data(), sizeof(int64_t) * (nwg + 1), hipMemcpyHostToDevice, ctx->stream));
  ScanArgs sa{};
  sa.Xs = Xs;
  sa.invs = invs;
  sa.perm = perm;
  sa.tile_min = tmin;
  sa.tile_cinv = tcinv;
  sa.nwg = nwg;
  sa.ntp = nt;
  sa.w = 0;
  sa.KP = KP;
  sa.tlist = dtl;
  sa.toff = dtoff;
  int32_t* wgs = nullptr;
  ST_TRY(ws_get_t(ctx, "knn_wgs", (size_t)nwg, &wgs));
  ST_TRY(fill_zero(ctx, wgs, sizeof(int32_t) * nwg));
  sa.wg_start = wgs;
  ST_TRY(ws_get_t(ctx, "knn_lidx", (size_t)npad * KPP, &sa.lidx));
  ST_TRY(ws_get_t(ctx, "knn_lsim", (size_t)npad * KPP, &sa.lsim));
  ST_TRY(ws_get_t(ctx, "knn_colthr", (size_t)npad, &sa.colthr));
  if (2 * TAU_T2 - 1 >= KP) ST_TRY(ws_get_t(ctx, "knn_tau", (size_t)npad, &sa.tau));
  int32_t* cidx = nullptr;
  float* csim = nullptr;
  ST_TRY(ws_get_t(ctx, "knn_cidx", (size_t)n * KP, &cidx));
  ST_TRY(ws_get_t(ctx, "knn_csim", (size_t)n * KP, &csim));
  HIP_TRY(ctx, hipEventRecord(ev[1], ctx->stream));
  if (sa.tau) ST_TRY(run_bf16<SCAN_TAU>(ctx, DP, sa));
  ST_TRY(run_bf16<SCAN_WIN>(ctx, DP, sa));
  const int RB = KPP <= 40 ? 256 : 64;
  HIP_TRY(ctx, hipFuncSetAttribute((const void*)knn_merge_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024));
  knn_merge_kernel<<<(unsigned)cdiv(n, RB), RB, (size_t)RB * KPP * 8, ctx->stream>>>(
      n, KP, RB, sa.lidx, sa.lsim, invs, perm, nullptr, nullptr, 0, nullptr, cidx, csim);
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipEventRecord(ev[2], ctx->stream));
  ST_TRY(rescore_and_fix<uint16_t>(ctx, X, n, d, ldx, sq, KP, K, cidx, csim, nbr_idx, nbr_sim, st, false));
  HIP_TRY(ctx, hipEventRecord(ev[3], ctx->stream));
  if (st) {
    unsigned long long hz = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&hz, zc, sizeof(hz), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    st->zero_rows = (int64_t)hz;
    float a = 0.f, b = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&a, ev[1], ev[2]));
    HIP_TRY(ctx, hipEventElapsedTime(&b, ev[0], ev[3]));
    st->tile_ms = a;
    st->total_ms = b;
    st->window = -1;
    // pairs scored: sum over blocks of QB x 64 x tiles (ordered pairs, padding included)
    st->sym_pairs = (int64_t)tl.size() * BT_C * QB;
  }
  return ANCKA_OK;
}

template <typename TX>
ancka_status cell_order_typed(ancka_ctx* ctx, const TX* X, int64_t n, int64_t d, int64_t ldx, int32_t* order_out) {
  double* sq = nullptr;
  float *invn = nullptr, *nrm = nullptr;
  unsigned long long* zc = nullptr;
  uint64_t *keys = nullptr, *vals = nullptr;
  int64_t* piv = nullptr;
  ST_TRY(ws_get_t(ctx, "co_sq", (size_t)n, &sq));
  ST_TRY(ws_get_t(ctx, "co_invn", (size_t)n, &invn));
  ST_TRY(ws_get_t(ctx, "co_nrm", (size_t)n, &nrm));
  ST_TRY(ws_get_t(ctx, "co_zero", 2, &zc));
  ST_TRY(ws_get_t(ctx, "co_keys", (size_t)n, &keys));
  ST_TRY(ws_get_t(ctx, "co_vals", (size_t)n, &vals));
  ST_TRY(ws_get_t(ctx, "co_piv", NPIV, &piv));
  knn_prologue_kernel<TX><<<(unsigned)cdiv(n, 4), 256, 0, ctx->stream>>>(X, n, d, ldx, sq, invn, nrm, nullptr, 0, zc);
  LAUNCH_CHECK(ctx);
  int64_t hp[NPIV];
  for (int p = 0; p < NPIV; p++) hp[p] = (int64_t)((double)p * (double)n / NPIV);
  HIP_TRY(ctx, hipMemcpyAsync(piv, hp, sizeof(hp), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));   // hp is a stack array
  const int dp8 = (int)((d + 7) / 8 * 8);
  const size_t csm = (size_t)NPIV * dp8 * 2 + NPIV * 4;
  if (csm > 160 * 1024) return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "cell order: d too large");
  uint16_t* Pm = nullptr;
  float* pinv = nullptr;
  ST_TRY(ws_get_t(ctx, "co_pm", (size_t)NPIV * dp8, &Pm));
  ST_TRY(ws_get_t(ctx, "co_pinv", NPIV, &pinv));
  gather_pivots_kernel<TX><<<(unsigned)cdiv((int64_t)NPIV * dp8, 256), 256, 0, ctx->stream>>>(X, d, ldx, invn, piv,
                                                                                            NPIV, dp8, Pm, pinv);
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipFuncSetAttribute((const void*)cell_assign_kernel<TX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024));
  cell_assign_kernel<TX><<<(unsigned)cdiv(n, 256), 256, csm, ctx->stream>>>(X, n, d, ldx, Pm, pinv, NPIV, keys, nrm,
                                                                           vals);
  LAUNCH_CHECK(ctx);
  ST_TRY(radix_sort_u64(ctx, keys, vals, n, 40));
  u64_to_i32_kernel<<<(unsigned)cdiv(n, 256), 256, 0, ctx->stream>>>(vals, n, order_out);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

}  // namespace

extern "C" ancka_status ancka_knn(ancka_ctx* ctx, const void* X, int32_t xdtype, int64_t n, int64_t d, int64_t ldx,
                                  int32_t K, int32_t mode, int32_t* nbr_idx, void* nbr_sim, ancka_knn_stats* stats) {
  if (!ctx) return ANCKA_ERR_INVALID_ARG;
  if (!X || !nbr_idx || !nbr_sim || n < 2 || d < 1 || ldx < d || K < 1 || K > n - 1 || n > INT32_MAX - 64 ||
      K > 64)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_knn: invalid arguments (n=%lld d=%lld ldx=%lld K=%d)",
                   (long long)n, (long long)d, (long long)ldx, K);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  if (mode == ANCKA_KNN_BF16_RESCORE && xdtype != ANCKA_BF16)
    return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "ancka_knn: BF16_RESCORE needs bf16 attributes");
  if (mode < 0 || mode > 2) return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_knn: unknown mode %d", mode);
  if (stats) *stats = ancka_knn_stats{0, 0, 0, 0.0, 0.0, 0.0, 0, 0, -1, 0};
  switch (xdtype) {
    case ANCKA_F64: return knn_typed<double>(ctx, (const double*)X, n, d, ldx, K, mode, nbr_idx, nbr_sim, stats);
    case ANCKA_F32: return knn_typed<float>(ctx, (const float*)X, n, d, ldx, K, mode, nbr_idx, nbr_sim, stats);
    case ANCKA_BF16: return knn_typed<uint16_t>(ctx, (const uint16_t*)X, n, d, ldx, K, mode, nbr_idx, nbr_sim, stats);
    default: return set_err(ctx, ANCKA_ERR_INVALID_ARG, "ancka_knn: unknown dtype %d", xdtype);
  }
}

extern "C" ancka_status ancka_knn_ivf(ancka_ctx* ctx, const void* X, int32_t xdtype, int64_t n, int64_t d,
                                      int64_t ldx, int32_t K, int32_t nlist, int32_t nprobe, int32_t* nbr_idx,
                                      void* nbr_sim, ancka_knn_stats* stats) {
  if (!ctx) return ANCKA_ERR_INVALID_ARG;
  if (!X || !nbr_idx || !nbr_sim || n < 2 || d < 1 || ldx < d || K < 1 || K > n - 1 || n > INT32_MAX - 64 ||
      K > 64 || nlist < 1 || nlist > 4096 || nlist > n || nprobe < 1 || nprobe > 64 || nprobe > nlist)
    return set_err(ctx, ANCKA_ERR_INVALID_ARG,
                   "ancka_knn_ivf: invalid arguments (n=%lld d=%lld ldx=%lld K=%d nlist=%d nprobe=%d; need "
                   "1 <= K <= min(n-1, 64), 1 <= nlist <= min(n, 4096), 1 <= nprobe <= min(nlist, 64))",
                   (long long)n, (long long)d, (long long)ldx, K, nlist, nprobe);
  if (xdtype != ANCKA_BF16) return set_err(ctx, ANCKA_ERR_UNSUPPORTED, "ancka_knn_ivf: bf16 attributes only");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, ANCKA_ERR_HIP, "hipSetDevice");
  if (stats) *stats = ancka_knn_stats{0, 0, 0, 0.0, 0.0, 0.0, 0, 0, -1, 0};
  return ivf_knn(ctx, (const uint16_t*)X, n, d, ldx, K, nlist, nprobe, nbr_idx, (float*)nbr_sim, stats);
}

ancka_status cell_order(ancka_ctx* ctx, const void* X, int xdtype, int64_t n, int64_t d, int64_t ldx, int32_t* order) {
  switch (xdtype) {
    case ANCKA_F64: return cell_order_typed<double>(ctx, (const double*)X, n, d, ldx, order);
    case ANCKA_F32: return cell_order_typed<float>(ctx, (const float*)X, n, d, ldx, order);
    case ANCKA_BF16: return cell_order_typed<uint16_t>(ctx, (const uint16_t*)X, n, d, ldx, order);
    default: return set_err(ctx, ANCKA_ERR_INVALID_ARG, "cell order: unknown dtype %d", xdtype);
  }
}
