// Stable LSD radix sort of (khi, klo, val) records and an exclusive scan.
//
// One pass per 8-bit digit: a 256-bin histogram per tile of 4096 records,
// an exclusive scan of the digit-major histogram table (rows, then digit
// offsets), and a stable scatter
// that ranks records inside each tile with wave ballots (8 ballots give every
// lane the set of lanes holding the same digit).  Records in a tile are taken
// in index order (round r covers records r*256 .. r*256+255), so equal digits
// keep their input order and the sort is stable and deterministic.
#include "common.hpp"
#include "ctx.hpp"

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t* __restrict__ klo,
                                                        const uint64_t* __restrict__ khi, int64_t n,
                                                        int word, int shift,
                                                        uint32_t* __restrict__ hist,
                                                        int64_t nblocks) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t idx = base + (int64_t)r * RS_THREADS + tid;
    if (idx < n) {
      uint64_t key = word ? khi[idx] : klo[idx];
      atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)tid * nblocks + blockIdx.x] = h[tid];
}

// Exclusive scan of the digit-major table in two steps: one block per digit
// scans its row of tile counts (coalesced, 256 at a time) and leaves the row
// total in rowsum; then one block turns the 256 totals into digit offsets.
// The scatter adds a digit's offset to its row entry.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scan_rows(uint32_t* __restrict__ hist,
                                                             int64_t nblocks,
                                                             uint32_t* __restrict__ rowsum) {
  __shared__ uint32_t wsum[RS_THREADS / REC_WAVE];
  __shared__ uint32_t run;
  const int tid = threadIdx.x, lane = tid & (REC_WAVE - 1), wave = tid / REC_WAVE;
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  if (tid == 0) run = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nblocks; c0 += RS_THREADS) {
    const int64_t k = c0 + tid;
    const uint32_t v = k < nblocks ? row[k] : 0u;
    // inclusive scan inside the wave, then across the waves
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < REC_WAVE; o <<= 1) {
      uint32_t y = __shfl_up(x, o, REC_WAVE);
      if (lane >= o) x += y;
    }
    if (lane == REC_WAVE - 1) wsum[wave] = x;
    __syncthreads();
    uint32_t before = run;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (k < nblocks) row[k] = before + x - v;
    __syncthreads();
    if (tid == 0) {
      uint32_t t = 0;
      for (int w = 0; w < RS_THREADS / REC_WAVE; ++w) t += wsum[w];
      run += t;
    }
    __syncthreads();
  }
  if (tid == 0) rowsum[blockIdx.x] = run;
}

__global__ __launch_bounds__(256) void k_rs_scan_bins(uint32_t* __restrict__ rowsum) {
  __shared__ uint32_t sh[256];
  const int tid = threadIdx.x;
  const uint32_t v = rowsum[tid];
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    uint32_t a = tid >= o ? sh[tid - o] : 0u;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  rowsum[tid] = sh[tid] - v;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint64_t* __restrict__ klo_in, const uint64_t* __restrict__ khi_in,
    const uint32_t* __restrict__ val_in, uint64_t* __restrict__ klo_out,
    uint64_t* __restrict__ khi_out, uint32_t* __restrict__ val_out, int64_t n, int word, int shift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ binoff, int64_t nblocks,
    int use_hi, int use_val) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t cnt[RS_THREADS / REC_WAVE][256];
  const int tid = threadIdx.x;
  const int wave = tid / REC_WAVE;
  const int lane = tid % REC_WAVE;
  base[tid] = hist[(int64_t)tid * nblocks + blockIdx.x] + binoff[tid];
  for (int w = 0; w < RS_THREADS / REC_WAVE; ++w) cnt[w][tid] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
  const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t idx = tbase + (int64_t)r * RS_THREADS + tid;
    bool valid = idx < n;
    uint64_t lo = 0, hi = 0;
    uint32_t v = 0;
    int d = 0;
    if (valid) {
      lo = klo_in[idx];
      if (use_hi) hi = khi_in[idx];
      if (use_val) v = val_in[idx];
      d = (int)(((word ? hi : lo) >> shift) & 255u);
    }
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1;
      uint64_t bal = __ballot(valid && bit);
      mask &= bit ? bal : ~bal;
    }
    int rank = __popcll(mask & lt);
    if (valid && rank == 0) cnt[wave][d] = (uint32_t)__popcll(mask);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + rank;
      for (int w = 0; w < wave; ++w) pos += cnt[w][d];
      klo_out[pos] = lo;
      if (use_hi) khi_out[pos] = hi;
      if (use_val) val_out[pos] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < RS_THREADS / REC_WAVE; ++w) { add += cnt[w][tid]; cnt[w][tid] = 0; }
    base[tid] += add;
    __syncthreads();
  }
}

// ----- exclusive scan of int64 -----
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 4;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

__device__ int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 1; o < SC_THREADS; o <<= 1) {
    int64_t a = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += a;
    __syncthreads();
  }
  int64_t incl = sh[tid];
  *total = sh[SC_THREADS - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_tiles(const int64_t* in, int64_t* out,
                                                           int64_t n, int64_t* tile_sums) {
  __shared__ int64_t sh[SC_THREADS];
  const int tid = threadIdx.x;
  int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)tid * SC_ITEMS;
  int64_t x[SC_ITEMS];
  int64_t s = 0;
  for (int k = 0; k < SC_ITEMS; ++k) {
    x[k] = base + k < n ? in[base + k] : 0;
    s += x[k];
  }
  int64_t tot;
  int64_t ex = block_excl_scan(s, sh, &tot);
  for (int k = 0; k < SC_ITEMS; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += x[k];
  }
  if (tid == 0) tile_sums[blockIdx.x] = tot;
}

// single block: exclusive scan of the tile sums (serial chunks per thread)
__global__ __launch_bounds__(SC_THREADS) void k_scan_sums(int64_t* sums, int64_t nt,
                                                          int64_t* total) {
  __shared__ int64_t sh[SC_THREADS];
  const int tid = threadIdx.x;
  int64_t per = (nt + SC_THREADS - 1) / SC_THREADS;
  int64_t b = (int64_t)tid * per, e = b + per < nt ? b + per : nt;
  int64_t s = 0;
  for (int64_t k = b; k < e; ++k) s += sums[k];
  int64_t tot;
  int64_t run = block_excl_scan(s, sh, &tot);
  for (int64_t k = b; k < e; ++k) {
    int64_t v = sums[k];
    sums[k] = run;
    run += v;
  }
  if (tid == 0 && total) *total = tot;
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_add(int64_t* out, int64_t n,
                                                         const int64_t* tile_sums) {
  int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
  int64_t a = tile_sums[blockIdx.x];
  for (int k = 0; k < SC_ITEMS; ++k)
    if (base + k < n) out[base + k] += a;
}

}  // namespace

rec_status rec_radix_sort(rec_ctx* ctx, int64_t n, const Digit* digits, int nd, int* cur) {
  if (n <= 0 || nd <= 0) return REC_OK;
  if (n > ctx->sb.cap) {
    ctx->err = "sort buffer too small";
    return REC_E_NOMEM;
  }
  int64_t nblocks = (n + RS_TILE - 1) / RS_TILE;
  int use_hi = 0;
  for (int d = 0; d < nd; ++d) use_hi |= digits[d].word;
  int c = *cur;
  for (int d = 0; d < nd; ++d) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(RS_THREADS), 0, ctx->stream,
                       ctx->sb.klo[c], ctx->sb.khi[c], n, digits[d].word, digits[d].shift,
                       ctx->sb.hist, nblocks);
    uint32_t* binoff = ctx->sb.hist + 256 * nblocks;   // the table's spare row of 256
    hipLaunchKernelGGL(k_rs_scan_rows, dim3(256), dim3(RS_THREADS), 0, ctx->stream, ctx->sb.hist,
                       nblocks, binoff);
    hipLaunchKernelGGL(k_rs_scan_bins, dim3(1), dim3(256), 0, ctx->stream, binoff);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(RS_THREADS), 0, ctx->stream,
                       ctx->sb.klo[c], ctx->sb.khi[c], ctx->sb.val[c], ctx->sb.klo[1 - c],
                       ctx->sb.khi[1 - c], ctx->sb.val[1 - c], n, digits[d].word,
                       digits[d].shift, ctx->sb.hist, binoff, nblocks, use_hi, 1);
    c = 1 - c;
  }
  *cur = c;
  REC_HIP(hipGetLastError());
  return REC_OK;
}

rec_status rec_exclusive_scan(rec_ctx* ctx, const int64_t* in, int64_t* out, int64_t n,
                              int64_t* total_dev) {
  if (n <= 0) return REC_OK;
  int64_t nt = (n + SC_TILE - 1) / SC_TILE;
  hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(SC_THREADS), 0, ctx->stream, in, out, n,
                     ctx->scan_tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SC_THREADS), 0, ctx->stream, ctx->scan_tmp, nt,
                     total_dev);
  hipLaunchKernelGGL(k_scan_add, dim3(nt), dim3(SC_THREADS), 0, ctx->stream, out, n,
                     ctx->scan_tmp);
  REC_HIP(hipGetLastError());
  return REC_OK;
}
