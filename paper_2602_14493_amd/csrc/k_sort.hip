// LSD onesweep radix sort of the (tile << 32 | depth) instance keys with their face-view values,
// 8-bit digits over the low `key_bits` bits (32 depth bits + enough bits for the batch's tiles),
// then the per-tile [start, end) ranges.
//
//  k_sort_hist    one read of the keys builds the digit histograms of every pass at once
//  k_sort_digits  exclusive scan of each pass's 256-bin histogram -> global digit offsets
//  k_sort_pass    per pass: each workgroup takes a partition ticket (so every earlier partition
//                 already runs), ranks its 4096 keys stably in LDS with wavefront ballots (8
//                 ballots per 64 keys match equal digits), publishes its digit counts, resolves
//                 its global offsets by decoupled look-back over earlier partitions' descriptors,
//                 stages the keys in LDS in digit order and writes them out in coalesced runs.
// Descriptor word: bits 31..30 = {0 empty, 1 aggregate, 2 inclusive prefix}, bits 29..0 = count,
// so one 32-bit atomic load observes flag and value together.  Two descriptor buffers alternate:
// each pass clears, for its own partitions, the buffer the next pass will use.
#include "gmr_common.h"
#include "gmr_launch.h"

namespace gmr {

__global__ __launch_bounds__(256) void k_sort_hist(const uint64_t* __restrict__ keys, const WsHdr* __restrict__ hdr,
                                                   uint32_t* __restrict__ hist, int passes,
                                                   uint32_t* __restrict__ desc0, int64_t desc_words) {
  __shared__ uint32_t s_h[kMaxPasses * 256];
  for (int i = threadIdx.x; i < kMaxPasses * 256; i += blockDim.x) s_h[i] = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < desc_words; i += (int64_t)gridDim.x * blockDim.x)
    desc0[i] = 0;
  __syncthreads();
  const uint32_t n = min(hdr->count, hdr->capacity);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    for (int p = 0; p < passes; ++p) atomicAdd(&s_h[p * 256 + ((k >> (8 * p)) & 255u)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < passes * 256; i += blockDim.x)
    if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

__global__ __launch_bounds__(256) void k_sort_digits(const uint32_t* __restrict__ hist, uint32_t* __restrict__ dig,
                                                     int passes) {
  __shared__ uint32_t s_w[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int p = 0; p < passes; ++p) {
    const uint32_t x = hist[p * 256 + threadIdx.x];
    uint32_t inc = x;
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t y = __shfl_up(inc, d, 64);
      if (lane >= d) inc += y;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += s_w[k];
    dig[p * 256 + threadIdx.x] = before + inc - x;
    __syncthreads();
  }
}

__device__ inline uint32_t desc_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void desc_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kSortBlock) void k_sort_pass(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                          uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          WsHdr* hdr, const uint32_t* __restrict__ dig,
                                                          uint32_t* desc_cur, uint32_t* desc_next, int pass) {
  __shared__ uint64_t s_keys[kSortPart];
  __shared__ uint32_t s_vals[kSortPart];
  __shared__ uint32_t s_wcnt[kSortBlock / kWave][256];
  __shared__ uint32_t s_bstart[256];
  __shared__ uint32_t s_gbase[256];
  __shared__ uint32_t s_wsum[kSortBlock / kWave];
  __shared__ uint32_t s_part;

  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int shift = 8 * pass;
  if (threadIdx.x == 0) s_part = atomicAdd(&hdr->part_ctr[pass], 1u);
  for (int i = threadIdx.x; i < (kSortBlock / kWave) * 256; i += kSortBlock) (&s_wcnt[0][0])[i] = 0;
  __syncthreads();
  const uint32_t n = min(hdr->count, hdr->capacity);
  const uint32_t part = s_part;
  const uint32_t nparts = (n + kSortPart - 1) / kSortPart;
  if (part >= nparts) return;  // uniform across the workgroup
  const uint32_t base = part * kSortPart;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  uint64_t k[kSortItems];
  uint32_t v[kSortItems];
  uint32_t rank[kSortItems];
  // ---- stable ranking inside the partition: wavefront w owns keys [w*1024, (w+1)*1024), 64 at a time
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t idx = base + (uint32_t)w * (kSortItems * kWave) + (uint32_t)i * kWave + (uint32_t)lane;
    const bool have = idx < n;
    k[i] = have ? kin[idx] : 0ull;
    v[i] = have ? vin[idx] : 0u;
    const uint32_t d = (uint32_t)(k[i] >> shift) & 255u;
    uint64_t peers = __ballot(have);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    uint32_t old = 0;
    if (have) old = s_wcnt[w][d];
    wave_lds_sync();
    if (have && below == 0) s_wcnt[w][d] = old + (uint32_t)__popcll(peers);
    wave_lds_sync();
    rank[i] = old + below;
  }
  __syncthreads();

  // ---- per digit (thread = digit): wavefront-exclusive offsets, publish, look back
  const int d = threadIdx.x;
  uint32_t tot = 0;
  for (int ww = 0; ww < kSortBlock / kWave; ++ww) {
    const uint32_t c = s_wcnt[ww][d];
    s_wcnt[ww][d] = tot;
    tot += c;
  }
  uint32_t* my = desc_cur + (size_t)part * 256 + d;
  desc_store(my, (part == 0 ? kFlagInc : kFlagAgg) | tot);
  desc_next[(size_t)part * 256 + d] = 0u;
  uint32_t excl = 0;
  if (part > 0) {
    int j = (int)part - 1;
    while (true) {
      const uint32_t x = desc_load(desc_cur + (size_t)j * 256 + d);
      if ((x & ~kValMask) == 0u) {
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += x & kValMask;
      if (x & kFlagInc) break;
      --j;
    }
    desc_store(my, kFlagInc | (excl + tot));
  }
  s_gbase[d] = dig[pass * 256 + d] + excl;
  // block-local exclusive scan over digits -> s_bstart
  {
    uint32_t inc = tot;
    for (int s = 1; s < kWave; s <<= 1) {
      const uint32_t y = __shfl_up(inc, s, kWave);
      if (lane >= s) inc += y;
    }
    if (lane == kWave - 1) s_wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int ww = 0; ww < w; ++ww) before += s_wsum[ww];
    s_bstart[d] = before + inc - tot;
  }
  __syncthreads();

  // ---- stage in digit order, then write out in coalesced runs
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t idx = base + (uint32_t)w * (kSortItems * kWave) + (uint32_t)i * kWave + (uint32_t)lane;
    if (idx < n) {
      const uint32_t dd = (uint32_t)(k[i] >> shift) & 255u;
      const uint32_t pos = s_bstart[dd] + s_wcnt[w][dd] + rank[i];
      s_keys[pos] = k[i];
      s_vals[pos] = v[i];
    }
  }
  __syncthreads();
  const uint32_t nb = min((uint32_t)kSortPart, n - base);
  for (uint32_t s = threadIdx.x; s < nb; s += kSortBlock) {
    const uint64_t key = s_keys[s];
    const uint32_t dd = (uint32_t)(key >> shift) & 255u;
    const uint32_t g = s_gbase[dd] + (s - s_bstart[dd]);
    kout[g] = key;
    vout[g] = s_vals[s];
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = val;
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint64_t* __restrict__ keys, const WsHdr* __restrict__ hdr,
                                                     uint32_t* __restrict__ ranges) {
  const uint32_t n = min(hdr->count, hdr->capacity);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t t = (uint32_t)(keys[i] >> 32);
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[2 * (size_t)t] = i;
    if (i + 1 == n || (uint32_t)(keys[i + 1] >> 32) != t) ranges[2 * (size_t)t + 1] = i + 1;
  }
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)nb), dim3(256), 0, s, p, n, val);
}

void launch_sort_hist(const uint64_t* keys0, const WsHdr* hdr, uint32_t* hist, uint32_t* dig, uint32_t* desc0,
                      int64_t parts_max, int passes, int hist_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_hist, dim3(hist_blocks), dim3(256), 0, s, keys0, hdr, hist, passes, desc0, parts_max * 256);
  hipLaunchKernelGGL(k_sort_digits, dim3(1), dim3(256), 0, s, hist, dig, passes);
}

// One onesweep pass p: reads buffer (p & 1), writes buffer (p & 1) ^ 1.
void launch_sort_pass(uint64_t* keys0, uint32_t* vals0, uint64_t* keys1, uint32_t* vals1, WsHdr* hdr, const uint32_t* dig,
                      uint32_t* desc0, uint32_t* desc1, int64_t parts_max, int p, hipStream_t s) {
  if (parts_max <= 0) return;
  const bool odd = p & 1;
  hipLaunchKernelGGL(k_sort_pass, dim3((unsigned)parts_max), dim3(kSortBlock), 0, s, odd ? keys1 : keys0,
                     odd ? vals1 : vals0, odd ? keys0 : keys1, odd ? vals0 : vals1, hdr, dig, odd ? desc1 : desc0,
                     odd ? desc0 : desc1, p);
}

void launch_tile_ranges(const uint64_t* sorted_keys, const WsHdr* hdr, uint32_t* ranges, int64_t tiles_total,
                        int blocks, hipStream_t s) {
  launch_fill_u32(ranges, 2 * tiles_total, 0u, s);
  hipLaunchKernelGGL(k_tile_ranges, dim3(blocks), dim3(256), 0, s, sorted_keys, hdr, ranges);
}

}  // namespace gmr
