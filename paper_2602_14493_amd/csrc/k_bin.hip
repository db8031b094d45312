// Tile binning: exclusive scan of tiles-touched over face-views, then emission of one
// (key, value) instance per (face-view, tile): key = global tile << 32 | float32 depth bits,
// value = face-view index.  Emission order is face-view order, so a stable sort on the key breaks
// depth ties by ascending global id.
//
// Scan: reduce (per 4096 face-views) -> single-block scan of the block sums -> emit, which redoes
// the block-local scan on wavefront shuffles.  Face-view t of block b, wave w, round i, lane l is
// b*4096 + w*1024 + i*64 + l: every load is a coalesced 64-wide run.
#include "gmr_common.h"
#include "gmr_launch.h"

namespace gmr {

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ inline uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint32_t* __restrict__ cnt, int64_t n,
                                                            uint32_t* __restrict__ bsum) {
  __shared__ uint32_t s_w[kScanBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)w * (kScanItems * kWave) + lane;
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + (int64_t)i * kWave;
    if (idx < n) acc += cnt[idx];
  }
  acc = wave_sum(acc);
  if (lane == 0) s_w[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < kScanBlock / kWave; ++k) t += s_w[k];
    bsum[blockIdx.x] = t;
  }
}

// Single workgroup: exclusive scan of the block sums (64-bit), instance total and overflow flag;
// also clears the sort histograms and the per-pass partition tickets for this pass of the pipeline.
__global__ __launch_bounds__(1024) void k_scan_top(const uint32_t* __restrict__ bsum, int nb, uint64_t* __restrict__ boff,
                                                   WsHdr* hdr, uint32_t* __restrict__ hist, int hist_n, uint32_t cap,
                                                   uint32_t passes) {
  __shared__ uint64_t s_part[1024 / kWave];
  __shared__ uint64_t s_carry;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < hist_n; i += blockDim.x) hist[i] = 0;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    const int idx = base + threadIdx.x;
    const uint64_t x = idx < nb ? bsum[idx] : 0;
    uint64_t inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      uint64_t y = __shfl_up(inc, d, kWave);
      if (lane >= d) inc += y;
    }
    if (lane == kWave - 1) s_part[w] = inc;
    __syncthreads();
    uint64_t before = s_carry;
    for (int k = 0; k < w; ++k) before += s_part[k];
    if (idx < nb) boff[idx] = before + inc - x;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t t = 0;
      for (int k = 0; k < 1024 / kWave; ++k) t += s_part[k];
      s_carry += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint64_t total = s_carry;
    hdr->capacity = cap;
    hdr->passes = passes;
    hdr->count = total > 0xffffffffull ? 0xffffffffu : (uint32_t)total;
    hdr->overflow = total > cap ? 1u : 0u;
    for (int p = 0; p < kMaxPasses; ++p) hdr->part_ctr[p] = 0;
    hdr->work_fwd = 0;
    hdr->work_bwd = 0;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_emit(const uint32_t* __restrict__ cnt, const uint4* __restrict__ bin,
                                                     int64_t n, const uint64_t* __restrict__ boff, const WsHdr* __restrict__ hdr,
                                                     uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_w[kScanBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)w * (kScanItems * kWave) + lane;
  uint32_t c[kScanItems];
  uint32_t wtot = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + (int64_t)i * kWave;
    c[i] = idx < n ? cnt[idx] : 0u;
    wtot += c[i];
  }
  wtot = wave_sum(wtot);
  if (lane == 0) s_w[w] = wtot;
  __syncthreads();
  uint64_t off = boff[blockIdx.x];
  for (int k = 0; k < w; ++k) off += s_w[k];
  const uint64_t cap = hdr->capacity;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const uint32_t inc = wave_incl_scan(c[i], lane);
    const uint64_t my = off + inc - c[i];
    off += __shfl(inc, kWave - 1, kWave);
    if (c[i] == 0) continue;
    const int64_t fv = base + (int64_t)i * kWave;
    const uint4 b = bin[fv];
    const uint32_t nx = b.y & 0xffffu, ny = b.y >> 16;
    uint64_t pos = my;
    for (uint32_t ty = 0; ty < ny; ++ty) {
      for (uint32_t tx = 0; tx < nx; ++tx, ++pos) {
        if (pos < cap) {
          const uint32_t tile = b.x + ty * b.z + tx;
          keys[pos] = ((uint64_t)tile << 32) | (uint64_t)b.w;
          vals[pos] = (uint32_t)fv;
        }
      }
    }
  }
}

void launch_bin(const uint32_t* cnt, const uint4* bin, int64_t n, uint32_t* bsum, uint64_t* boff, int nb, WsHdr* hdr,
                uint32_t* hist, int hist_n, uint32_t cap, uint32_t passes, uint64_t* keys, uint32_t* vals,
                hipStream_t s) {
  if (nb > 0) hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBlock), 0, s, cnt, n, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, nb, boff, hdr, hist, hist_n, cap, passes);
  if (nb > 0) hipLaunchKernelGGL(k_emit, dim3(nb), dim3(kScanBlock), 0, s, cnt, bin, n, boff, hdr, keys, vals);
}

}  // namespace gmr
