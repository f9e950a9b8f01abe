// Device primitives: exclusive scan, stable LSD radix sort, run merging, CSR row pointers.
// Every result is deterministic: integer counting only, ranks derived from wave ballots.
#include "common.h"

namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_I = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_I;

__global__ __launch_bounds__(SCAN_T) void scan_tile_kernel(const int64_t* __restrict__ in, int64_t* __restrict__ out,
                                                           int64_t count, int64_t* __restrict__ sums) {
  __shared__ int64_t s[SCAN_T];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)tid * SCAN_I;
  int64_t v[SCAN_I];
  int64_t tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_I; i++) {
    v[i] = (base + i < count) ? in[base + i] : 0;
    tot += v[i];
  }
  s[tid] = tot;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    int64_t add = (tid >= off) ? s[tid - off] : 0;
    __syncthreads();
    s[tid] += add;
    __syncthreads();
  }
  int64_t run = s[tid] - tot;
#pragma unroll
  for (int i = 0; i < SCAN_I; i++) {
    if (base + i < count) out[base + i] = run;
    run += v[i];
  }
  if (tid == SCAN_T - 1) sums[blockIdx.x] = s[tid];
}

__global__ void scan_add_kernel(int64_t* __restrict__ out, int64_t count, const int64_t* __restrict__ sums_scan) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < count) out[p] += sums_scan[p / SCAN_TILE];
  if (p == 0) out[count] = sums_scan[cdiv(count, SCAN_TILE)];
}

ancka_status scan_level(ancka_ctx* ctx, const int64_t* in, int64_t* out, int64_t count, int level) {
  const int64_t nb = cdiv(count, SCAN_TILE);
  if (nb <= 1) {
    scan_tile_kernel<<<1, SCAN_T, 0, ctx->stream>>>(in, out, count, out + count);
    LAUNCH_CHECK(ctx);
    return ANCKA_OK;
  }
  char name[32];
  snprintf(name, sizeof(name), "scan_sums_%d", level);
  int64_t* sums = nullptr;
  ST_TRY(ws_get_t(ctx, name, 2 * (nb + 1), &sums));
  int64_t* sums_scan = sums + (nb + 1);
  scan_tile_kernel<<<(unsigned)nb, SCAN_T, 0, ctx->stream>>>(in, out, count, sums);
  LAUNCH_CHECK(ctx);
  ST_TRY(scan_level(ctx, sums, sums_scan, nb, level + 1));
  scan_add_kernel<<<(unsigned)cdiv(count, 256), 256, 0, ctx->stream>>>(out, count, sums_scan);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

// ---- radix sort ---------------------------------------------------------------------------
constexpr int RS_T = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_T * RS_ITEMS;
constexpr int RS_BINS = 256;

__global__ __launch_bounds__(RS_T) void rs_hist_kernel(const uint64_t* __restrict__ keys, int64_t count, int shift,
                                                       int64_t ntiles, int64_t* __restrict__ hist) {
  __shared__ int h[RS_BINS];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; r++) {
    const int64_t p = base + (int64_t)r * RS_T + tid;
    if (p < count) atomicAdd(&h[(keys[p] >> shift) & (RS_BINS - 1)], 1);
  }
  __syncthreads();
  hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(RS_T) void rs_scatter_kernel(const uint64_t* __restrict__ kin, const uint64_t* __restrict__ vin,
                                                          uint64_t* __restrict__ kout, uint64_t* __restrict__ vout,
                                                          int64_t count, int shift, int64_t ntiles,
                                                          const int64_t* __restrict__ offs) {
  __shared__ int64_t running[RS_BINS];
  __shared__ int wc[RS_T / ANCKA_WAVE][RS_BINS];
  const int tid = threadIdx.x;
  const int w = tid / ANCKA_WAVE;
  const int lane = tid % ANCKA_WAVE;
  running[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; r++) {
    for (int j = tid; j < (RS_T / ANCKA_WAVE) * RS_BINS; j += RS_T) (&wc[0][0])[j] = 0;
    __syncthreads();
    const int64_t p = base + (int64_t)r * RS_T + tid;
    const bool act = p < count;
    const uint64_t key = act ? kin[p] : 0ull;
    const uint64_t val = (act && vin) ? vin[p] : 0ull;
    const int d = (int)((key >> shift) & (RS_BINS - 1));
    uint64_t m = __ballot(act);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const uint64_t bal = __ballot(act && ((d >> b) & 1));
      m &= ((d >> b) & 1) ? bal : ~bal;
    }
    const int rank = __popcll(m & below);
    if (act && rank == 0) wc[w][d] = __popcll(m);
    __syncthreads();
    if (act) {
      int64_t pos = running[d] + rank;
      for (int w2 = 0; w2 < w; w2++) pos += wc[w2][d];
      kout[pos] = key;
      if (vin) vout[pos] = val;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int w2 = 0; w2 < RS_T / ANCKA_WAVE; w2++) add += wc[w2][tid];
    running[tid] += add;
    __syncthreads();
  }
}

__global__ void copy_u64_kernel(const uint64_t* __restrict__ a, uint64_t* __restrict__ b, int64_t count) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < count) b[p] = a[p];
}

__global__ void uniq_flag_kernel(const uint64_t* __restrict__ keys, int64_t count, int64_t* __restrict__ flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < count) flags[p] = (p == 0 || keys[p] != keys[p - 1]) ? 1 : 0;
}

__global__ void uniq_write_kernel(const uint64_t* __restrict__ keys, const uint64_t* __restrict__ vals, int vals_double,
                                  int64_t count, const int64_t* __restrict__ pos, uint64_t* __restrict__ out_keys,
                                  double* __restrict__ out_vals) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const uint64_t k = keys[p];
  if (p != 0 && keys[p - 1] == k) return;
  const int64_t q = pos[p];
  out_keys[q] = k;
  if (vals && out_vals) {
    double s = 0.0;
    for (int64_t r = p; r < count && keys[r] == k; r++) {
      const uint64_t v = vals[r];
      s += vals_double ? __longlong_as_double((long long)v) : (double)__uint_as_float((uint32_t)v);
    }
    out_vals[q] = s;
  }
}

__global__ void csr_ptr_kernel(const uint64_t* __restrict__ keys, int64_t count, int col_bits, int64_t rows,
                               int64_t* __restrict__ row_ptr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > rows) return;
  const uint64_t target = (uint64_t)r << col_bits;
  int64_t lo = 0, hi = count;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  row_ptr[r] = lo;
}

__global__ void fill_zero_kernel(uint32_t* __restrict__ p, int64_t words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0u;
}

}  // namespace

ancka_status scan_excl_i64(ancka_ctx* ctx, const int64_t* in, int64_t* out, int64_t count) {
  if (count <= 0) {
    return fill_zero(ctx, out, sizeof(int64_t));
  }
  return scan_level(ctx, in, out, count, 0);
}

ancka_status radix_sort_u64(ancka_ctx* ctx, uint64_t* keys, uint64_t* vals, int64_t count, int bits) {
  if (count <= 1 || bits <= 0) return ANCKA_OK;
  const int64_t ntiles = cdiv(count, RS_TILE);
  int64_t *hist = nullptr, *offs = nullptr;
  uint64_t *k2 = nullptr, *v2 = nullptr;
  ST_TRY(ws_get_t(ctx, "rs_hist", (size_t)RS_BINS * ntiles, &hist));
  ST_TRY(ws_get_t(ctx, "rs_offs", (size_t)RS_BINS * ntiles + 1, &offs));
  ST_TRY(ws_get_t(ctx, "rs_keys", (size_t)count, &k2));
  if (vals) ST_TRY(ws_get_t(ctx, "rs_vals", (size_t)count, &v2));
  uint64_t *ka = keys, *kb = k2, *va = vals, *vb = v2;
  for (int shift = 0; shift < bits; shift += 8) {
    rs_hist_kernel<<<(unsigned)ntiles, RS_T, 0, ctx->stream>>>(ka, count, shift, ntiles, hist);
    LAUNCH_CHECK(ctx);
    ST_TRY(scan_excl_i64(ctx, hist, offs, (int64_t)RS_BINS * ntiles));
    rs_scatter_kernel<<<(unsigned)ntiles, RS_T, 0, ctx->stream>>>(ka, va, kb, vb, count, shift, ntiles, offs);
    LAUNCH_CHECK(ctx);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    copy_u64_kernel<<<(unsigned)cdiv(count, 256), 256, 0, ctx->stream>>>(ka, keys, count);
    LAUNCH_CHECK(ctx);
    if (vals) {
      copy_u64_kernel<<<(unsigned)cdiv(count, 256), 256, 0, ctx->stream>>>(va, vals, count);
      LAUNCH_CHECK(ctx);
    }
  }
  return ANCKA_OK;
}

ancka_status unique_sorted(ancka_ctx* ctx, const uint64_t* keys, const uint64_t* vals, int vals_are_double,
                           int64_t count, uint64_t* out_keys, double* out_vals, int64_t* out_count) {
  if (count == 0) {
    *out_count = 0;
    return ANCKA_OK;
  }
  int64_t *flags = nullptr, *pos = nullptr;
  ST_TRY(ws_get_t(ctx, "uq_flags", (size_t)count, &flags));
  ST_TRY(ws_get_t(ctx, "uq_pos", (size_t)count + 1, &pos));
  const unsigned nb = (unsigned)cdiv(count, 256);
  uniq_flag_kernel<<<nb, 256, 0, ctx->stream>>>(keys, count, flags);
  LAUNCH_CHECK(ctx);
  ST_TRY(scan_excl_i64(ctx, flags, pos, count));
  uniq_write_kernel<<<nb, 256, 0, ctx->stream>>>(keys, vals, vals_are_double, count, pos, out_keys, out_vals);
  LAUNCH_CHECK(ctx);
  HIP_TRY(ctx, hipMemcpyAsync(out_count, pos + count, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return ANCKA_OK;
}

ancka_status csr_ptr_from_sorted(ancka_ctx* ctx, const uint64_t* keys, int64_t count, int col_bits, int64_t rows,
                                 int64_t* row_ptr) {
  csr_ptr_kernel<<<(unsigned)cdiv(rows + 1, 256), 256, 0, ctx->stream>>>(keys, count, col_bits, rows, row_ptr);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}

ancka_status fill_zero(ancka_ctx* ctx, void* p, size_t bytes) {
  const int64_t words = (int64_t)((bytes + 3) / 4);
  if (words == 0) return ANCKA_OK;
  fill_zero_kernel<<<(unsigned)cdiv(words, 256), 256, 0, ctx->stream>>>((uint32_t*)p, words);
  LAUNCH_CHECK(ctx);
  return ANCKA_OK;
}
