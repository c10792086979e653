// Tile binning and depth sorting (the tiling / sorting stages the paper's
// App. A lists beside preprocessing; the blending of Eq. 4 needs the
// primitives of every pixel in depth order).
//
//   depth  : (for many pairs) stable LSD radix sort of the (view, primitive)
//            pairs by their float32 depth bits (ties keep the index order)
//   scan   : exclusive prefix sum of the tile counts in that order
//   emit   : one (key, value) instance per covered tile, primitives in depth
//            order, key = (global tile id << 31) | float32 depth bits,
//            value = primitive id
//   sort   : stable LSD radix sort of the instances by the tile bits of the
//            key only: the input is already in depth order and every pass
//            is stable, so the result is ordered by the whole key (and by
//            primitive index for equal depths), as a sort over all bits
//            would order it, with 2-3 passes over the instances instead of
//            6 (8-bit digits, 3 kernels per pass: digit histogram per block,
//            scan, stable scatter).  For few pairs the extra launches of the
//            depth sort cost more than the passes saved: the pairs stay in
//            primitive order and the sort covers depth and tile bits.
//   ranges : [start, end) of every global tile in the sorted array
//
// Sizes only known on the device (the instance count) are read from device
// memory; launches are sized by the workspace capacity, so the sequence can
// be captured in a graph.  Writes past the capacity are dropped and flagged.
#include "snp_internal.h"

namespace snp {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int64_t kScanChunk = (int64_t)kScanThreads * kScanItems;  // 4096

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int64_t kSortChunk = (int64_t)kSortThreads * kSortRounds;  // 4096
constexpr int kRadix = 256;

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan: uint32 values -> uint32 offsets, uint64 block totals
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t block_exclusive_scan_u64(uint64_t x, uint64_t* total, uint64_t* s_warp) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_warp[w] = inc;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int k = 0; k < kScanThreads / 64; ++k) {
    if (k < w) base += s_warp[k];
    tot += s_warp[k];
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

template <typename TI>
__global__ void __launch_bounds__(kScanThreads) scan_block_kernel(const TI* in, uint64_t* out64,
                                                                  uint32_t* out32, int64_t n,
                                                                  uint64_t* block_sums) {
  __shared__ uint64_t s_warp[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? (uint64_t)in[i] : 0;
    sum += v[k];
  }
  uint64_t total;
  uint64_t run = block_exclusive_scan_u64(sum, &total, s_warp);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) {
      if (out64) out64[i] = run;
      if (out32) out32[i] = (uint32_t)run;
    }
    run += v[k];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) scan_add_kernel(uint64_t* out64, uint32_t* out32, int64_t n,
                                                                const uint64_t* __restrict__ block_off) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const uint64_t off = block_off[blockIdx.x];
  for (int k = threadIdx.x; k < kScanChunk; k += kScanThreads) {
    const int64_t i = base + k;
    if (i < n) {
      if (out64) out64[i] += off;
      if (out32) out32[i] = (uint32_t)(out32[i] + off);
    }
  }
}

__global__ void store_total_kernel(const uint64_t* sums, uint64_t* total_out) { *total_out = sums[0]; }

// Scratch needed by scan_exclusive for n elements (bytes).
size_t scan_scratch_bytes(int64_t n) {
  size_t bytes = 0;
  while (true) {
    const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
    bytes += ((size_t)nb * 8 + 255) / 256 * 256;
    if (nb <= 1) break;
    n = nb;
  }
  return bytes + 256;
}

// Exclusive scan of n uint32 values into out32 (wrapping) and the exact
// total into *total_out (uint64, device) if non-null.
template <typename TI>
static hipError_t scan_level(const TI* in, uint64_t* out64, uint32_t* out32, int64_t n, char* scratch,
                             uint64_t* total_out, hipStream_t st) {
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  uint64_t* sums = reinterpret_cast<uint64_t*>(scratch);
  char* next = scratch + ((size_t)nb * 8 + 255) / 256 * 256;
  hipLaunchKernelGGL(scan_block_kernel<TI>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, out64, out32, n, sums);
  if (nb > 1) {
    // sums -> exclusive offsets in place (through a uint64 copy level)
    hipError_t e = scan_level<uint64_t>(sums, sums, nullptr, nb, next, total_out, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, st, out64, out32, n, sums);
  } else if (total_out) {
    hipLaunchKernelGGL(store_total_kernel, dim3(1), dim3(1), 0, st, sums, total_out);
  }
  return hipGetLastError();
}

hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* scratch, uint64_t* total_out,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  return scan_level<uint32_t>(in, nullptr, out, n, reinterpret_cast<char*>(scratch), total_out, st);
}

// ---------------------------------------------------------------------------
// emit instances
// ---------------------------------------------------------------------------

// (depth bits, index) of every (view, primitive) pair, the input of the depth sort
__global__ void __launch_bounds__(256) depth_keys_kernel(const uint32_t* __restrict__ depth_bits, int64_t n,
                                                         unsigned long long* __restrict__ keys,
                                                         uint32_t* __restrict__ idx, unsigned long long* n_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *n_out = (unsigned long long)n;
  if (i >= n) return;
  keys[i] = depth_bits[i];
  idx[i] = (uint32_t)i;
}

// tile counts in depth order
__global__ void __launch_bounds__(256) gather_counts_kernel(const uint32_t* __restrict__ order,
                                                            const uint32_t* __restrict__ counts, int64_t n,
                                                            uint32_t* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = counts[order[j]];
}

hipError_t launch_depth_keys(const uint32_t* depth_bits, int64_t n, unsigned long long* keys, uint32_t* idx,
                             unsigned long long* n_out, hipStream_t st) {
  hipLaunchKernelGGL(depth_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, depth_bits, n, keys, idx,
                     n_out);
  return hipGetLastError();
}

hipError_t launch_gather_counts(const uint32_t* order, const uint32_t* counts, int64_t n, uint32_t* out,
                                hipStream_t st) {
  hipLaunchKernelGGL(gather_counts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, order, counts, n, out);
  return hipGetLastError();
}

// Instances of the pairs j (in depth order, or primitive order when order is
// null) at offsets[j] on.  A wave takes 64 consecutive pairs, whose
// instances are one contiguous output range, and writes that range 64
// instances at a time (lane l writes position base + l), so the writes are
// coalesced: each lane finds its pair by a binary search over the wave's
// offsets in LDS and its tile from the pair's tile rectangle.
__global__ void __launch_bounds__(256) emit_kernel(EmitArgs a) {
  constexpr int NW = 4;
  __shared__ uint32_t s_off[NW][65];   // first instance of each pair, relative to the wave's base; [64] = end
  __shared__ int32_t s_tx0[NW][64], s_nx[NW][64], s_ty0[NW][64], s_v[NW][64];
  __shared__ uint32_t s_p[NW][64], s_d[NW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t n = a.P * a.V;
  const int64_t j0 = ((int64_t)blockIdx.x * NW + w) * 64;
  const bool wave_has_pairs = j0 < n;  // wave-uniform; every wave still reaches the barrier
  const int64_t j = j0 + lane;
  uint32_t cnt = 0;
  if (j < n) {
    const int64_t i = a.order ? (int64_t)a.order[j] : j;
    cnt = a.tile_counts[i];
    const int v = (int)(i / a.P);
    const CamDev& cam = a.cams[v];
    const int tx0 = a.rects[4 * i] / cam.tile_w, tx1 = a.rects[4 * i + 1] / cam.tile_w;
    s_tx0[w][lane] = tx0;
    s_nx[w][lane] = tx1 - tx0 + 1;
    s_ty0[w][lane] = a.rects[4 * i + 2] / cam.tile_h;
    s_v[w][lane] = v;
    s_p[w][lane] = (uint32_t)(i - (int64_t)v * a.P);
    s_d[w][lane] = a.depth_bits[i];
  }
  // the wave's offsets are the exclusive scan values of its pairs (uint32
  // arithmetic: the differences stay exact if the scan wrapped)
  const uint32_t base = wave_has_pairs ? a.offsets[j0] : 0u;
  const int last = wave_has_pairs ? (int)min((int64_t)63, n - 1 - j0) : 0;
  s_off[w][lane] = j < n ? a.offsets[j] - base : 0xFFFFFFFFu;
  if (wave_has_pairs && lane == last) s_off[w][64] = (a.offsets[j] - base) + cnt;
  __syncthreads();
  const uint32_t total = wave_has_pairs ? s_off[w][64] : 0u;
  for (uint32_t o0 = 0; o0 < total; o0 += 64) {
    const uint32_t o = o0 + lane;
    if (o < total) {
      // the last pair k with s_off[k] <= o (pairs without instances share
      // their offset with the next one and are skipped by taking the last)
      int lo = 0, hi = last;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[w][mid] <= o) lo = mid; else hi = mid - 1;
      }
      const uint32_t k = o - s_off[w][lo];
      const int nx = s_nx[w][lo];
      const int ty = s_ty0[w][lo] + (int)(k / (uint32_t)nx);
      const int tx = s_tx0[w][lo] + (int)(k % (uint32_t)nx);
      const CamDev& cam = a.cams[s_v[w][lo]];
      const int64_t pos = (int64_t)base + (int64_t)o;
      if (pos < a.capacity) {
        const unsigned long long tile = (unsigned long long)(cam.tile_base + ty * cam.ntx + tx);
        a.keys[pos] = (tile << 31) | (unsigned long long)s_d[w][lo];
        a.values[pos] = s_p[w][lo];
      }
    }
  }
}

__global__ void check_capacity_kernel(unsigned long long* counters, int64_t capacity) {
  if (counters[CNT_INSTANCES] > (unsigned long long)capacity) counters[CNT_OVERFLOW] = 1ull;
}

hipError_t launch_emit(const EmitArgs& a, unsigned long long* counters, hipStream_t st) {
  const int64_t n = a.P * a.V;
  if (n > 0) hipLaunchKernelGGL(emit_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(check_capacity_kernel, dim3(1), dim3(1), 0, st, counters, a.capacity);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stable LSD radix sort
// ---------------------------------------------------------------------------
// number of elements to sort: *count, at most the capacity of the buffers
__device__ __forceinline__ int64_t sort_count(const unsigned long long* count, int64_t capacity) {
  const unsigned long long n = *count;
  return n > (unsigned long long)capacity ? capacity : (int64_t)n;
}

__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const unsigned long long* __restrict__ keys,
                                                                  const unsigned long long* count,
                                                                  int64_t capacity, int shift,
                                                                  uint32_t* __restrict__ hist, int64_t nblocks) {
  __shared__ uint32_t s_h[kRadix];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = sort_count(count, capacity);
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & 0xFF], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = s_h[threadIdx.x];
}

// Stable scatter of one block's chunk.  The chunk's keys are first placed
// in LDS in digit order (the block's own digit counts from the histogram
// give each digit's local start; ballot ranks keep the input order within a
// digit), then written out from LDS in that order, so consecutive threads
// write consecutive addresses of a digit's output run (runs of about
// chunk / 256 keys) instead of one scattered key each.
__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const unsigned long long* __restrict__ kin, const uint32_t* __restrict__ vin,
    unsigned long long* __restrict__ kout, uint32_t* __restrict__ vout, const unsigned long long* count,
    int64_t capacity, int shift, const uint32_t* __restrict__ offs, const uint32_t* __restrict__ hist,
    int64_t nblocks) {
  constexpr int NW = kSortThreads / 64;
  __shared__ unsigned long long s_key[kSortChunk];
  __shared__ uint32_t s_val[kSortChunk];
  __shared__ uint32_t s_lstart[kRadix];     // first local position of each digit
  __shared__ uint32_t s_run[kRadix];        // running local position of each digit
  __shared__ uint32_t s_goff[kRadix];       // global start of each digit for this block
  __shared__ uint32_t s_wcnt[NW][kRadix];   // per-wave digit counts in the current round
  __shared__ uint32_t s_wsum[NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // local digit starts: exclusive scan of this block's digit counts
  const uint32_t c = hist[(int64_t)t * nblocks + blockIdx.x];
  uint32_t inc = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_wsum[w] = inc;
  s_goff[t] = offs[(int64_t)t * nblocks + blockIdx.x];
  __syncthreads();
  uint32_t wbase = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) wbase += k < w ? s_wsum[k] : 0u;
  s_lstart[t] = wbase + inc - c;
  s_run[t] = wbase + inc - c;
  const int64_t n = sort_count(count, capacity);
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // all of this thread's keys and values first, so their loads are in flight together
  unsigned long long rkey[kSortRounds];
  uint32_t rval[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + t;
    rkey[r] = i < n ? kin[i] : 0ull;
    rval[r] = i < n ? vin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t rbase = base + (int64_t)r * kSortThreads;
    if (rbase >= n) break;  // uniform over the block
#pragma unroll
    for (int k = 0; k < NW; ++k) s_wcnt[k][t] = 0;
    __syncthreads();
    const int64_t i = rbase + t;
    const bool valid = i < n;
    const unsigned long long key = rkey[r];
    const uint32_t val = rval[r];
    const uint32_t d = valid ? (uint32_t)((key >> shift) & 0xFF) : 0u;
    // lanes of this wave holding the same digit
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank_w = (uint32_t)__popcll(peers & lt_mask);
    if (valid && rank_w == 0) s_wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    // per digit: prefix over the waves, advance the running local position
    {
      uint32_t run = s_run[t];
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const uint32_t cw = s_wcnt[k][t];
        s_wcnt[k][t] = run;
        run += cw;
      }
      s_run[t] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t lpos = s_wcnt[w][d] + rank_w;
      s_key[lpos] = key;
      s_val[lpos] = val;
    }
    __syncthreads();
  }
  // write the chunk out in digit order
  const int64_t nloc = n - base < kSortChunk ? n - base : kSortChunk;
  for (int q = t; q < nloc; q += kSortThreads) {
    const unsigned long long key = s_key[q];
    const uint32_t d = (uint32_t)((key >> shift) & 0xFF);
    const uint32_t pos = s_goff[d] + ((uint32_t)q - s_lstart[d]);
    kout[pos] = key;
    vout[pos] = s_val[q];
  }
}

size_t sort_scratch_bytes(int64_t capacity) {
  const int64_t nblocks = (capacity + kSortChunk - 1) / kSortChunk;
  const int64_t nh = nblocks * kRadix;
  return ((size_t)nh * 4 + 255) / 256 * 256 * 2 + scan_scratch_bytes(nh);
}

// Sorts the first min(*count, capacity) keys/values by bits [lo_bit, lo_bit +
// key_bits), stably.  Buffers ping-pong between (k0,v0) and (k1,v1); the
// input is in (k0,v0) and the result ends in (k0,v0) if the number of passes
// is even, else in (k1,v1).
hipError_t radix_sort(unsigned long long* k0, uint32_t* v0, unsigned long long* k1, uint32_t* v1, int64_t capacity,
                      const unsigned long long* count, int lo_bit, int key_bits, void* scratch, hipStream_t st) {
  const int64_t nblocks = (capacity + kSortChunk - 1) / kSortChunk;
  if (nblocks <= 0) return hipSuccess;
  const int64_t nh = nblocks * kRadix;
  char* sp = reinterpret_cast<char*>(scratch);
  uint32_t* hist = reinterpret_cast<uint32_t*>(sp);
  uint32_t* offs = reinterpret_cast<uint32_t*>(sp + ((size_t)nh * 4 + 255) / 256 * 256);
  char* scan_scr = sp + ((size_t)nh * 4 + 255) / 256 * 256 * 2;
  const int passes = (key_bits + 7) / 8;
  unsigned long long *ki = k0, *ko = k1;
  uint32_t *vi = v0, *vo = v1;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = lo_bit + 8 * ps;
    hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nblocks), dim3(kSortThreads), 0, st, ki, count, capacity,
                       shift, hist, nblocks);
    hipError_t e = scan_exclusive_u32(hist, offs, nh, scan_scr, nullptr, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nblocks), dim3(kSortThreads), 0, st, ki, vi, ko, vo,
                       count, capacity, shift, offs, hist, nblocks);
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  return hipGetLastError();
}

int radix_passes(int key_bits) { return (key_bits + 7) / 8; }

// ---------------------------------------------------------------------------
// tile ranges
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) ranges_kernel(const unsigned long long* __restrict__ keys,
                                                     const unsigned long long* counters, int64_t capacity,
                                                     uint32_t* __restrict__ ranges) {
  const int64_t n = sort_count(counters + CNT_INSTANCES, capacity);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const unsigned long long tile = keys[i] >> 31;
    if (i == 0 || (keys[i - 1] >> 31) != tile) ranges[2 * tile] = (uint32_t)i;
    if (i == n - 1 || (keys[i + 1] >> 31) != tile) ranges[2 * tile + 1] = (uint32_t)(i + 1);
  }
}

// (16-bit key, tile id) for the order in which persistent rasterizers take
// the tiles: key = 2^16 - 1 - min(instances, 2^16 - 1), so an ascending
// stable sort puts the tiles with the most instances first (equal or
// saturated counts in tile order); two radix passes
__global__ void __launch_bounds__(256) tile_keys_kernel(const uint32_t* __restrict__ ranges, int64_t n,
                                                        unsigned long long* __restrict__ keys,
                                                        uint32_t* __restrict__ ids, unsigned long long* n_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *n_out = (unsigned long long)n;
  if (t >= n) return;
  const uint32_t cnt = ranges[2 * t + 1] - ranges[2 * t];
  keys[t] = 0xFFFFull - (unsigned long long)(cnt < 0xFFFFu ? cnt : 0xFFFFu);
  ids[t] = (uint32_t)t;
}

hipError_t launch_tile_keys(const uint32_t* ranges, int64_t n_tiles, unsigned long long* keys, uint32_t* ids,
                            unsigned long long* n_out, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(tile_keys_kernel, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, st, ranges, n_tiles,
                     keys, ids, n_out);
  return hipGetLastError();
}

hipError_t launch_ranges(const unsigned long long* keys, const unsigned long long* counters, int64_t capacity,
                         uint32_t* ranges, int64_t n_tiles, hipStream_t st) {
  hipError_t e = fill_u32(ranges, 2 * n_tiles, 0u, st);
  if (e != hipSuccess) return e;
  int64_t blocks = (capacity + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)blocks), dim3(256), 0, st, keys, counters, capacity, ranges);
  return hipGetLastError();
}

}  // namespace snp
