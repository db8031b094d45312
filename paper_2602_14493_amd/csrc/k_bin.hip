// Tile binning over the depth-sorted face-view elements: exclusive scan of tiles-touched, then
// emission of one instance {tile, face-view} per (face-view, tile) in that order.  Emission order
// is (float32 depth, face-view), so a stable sort on the tile id alone completes the
// (tile, depth, id) order.  The emitter also accumulates the histograms of the tile digits and
// clears the first tile pass's descriptors.
//
// Scan: reduce (per 4096 elements) -> single-block scan of the block sums -> emit, which redoes the
// block-local scan on wavefront shuffles.  Element t of block b, wave w, round i, lane l is
// b*4096 + w*1024 + i*64 + l: every load is a coalesced 64-wide run.
#include "gmr_common.h"
#include "gmr_launch.h"

namespace gmr {

__device__ inline uint32_t el_count(const uint4& e) { return (e.w & 0xffffu) * (e.w >> 16); }

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

template <int kItems>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint4* __restrict__ el_a,
                                                            const uint4* __restrict__ el_b, const WsHdr* __restrict__ hdr,
                                                            int64_t n, uint32_t* __restrict__ bsum) {
  __shared__ uint32_t s_w[kScanBlock / kWave];
  const uint4* __restrict__ el = depth_keys_narrow(hdr) ? el_b : el_a;  // where the depth passes ended
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * (kScanBlock * kItems) + (int64_t)w * (kItems * kWave) + lane;
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const int64_t idx = base + (int64_t)i * kWave;
    if (idx < n) acc += el_count(el[idx]);
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

// Single workgroup: exclusive scan of the block sums (64-bit), instance total and overflow flag.
__global__ __launch_bounds__(1024) void k_scan_top(const uint32_t* __restrict__ bsum, int nb, uint64_t* __restrict__ boff,
                                                   WsHdr* hdr, uint32_t cap) {
  __shared__ uint64_t s_part[1024 / kWave];
  __shared__ uint64_t s_carry;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
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
    hdr->count = total > 0xffffffffull ? 0xffffffffu : (uint32_t)total;
    hdr->overflow = total > cap ? 1u : 0u;
  }
}

template <int kItems>
__global__ __launch_bounds__(kScanBlock) void k_emit(const void* __restrict__ table, const uint4* __restrict__ el_a,
                                                     const uint4* __restrict__ el_b, int64_t n,
                                                     const uint64_t* __restrict__ boff, const WsHdr* __restrict__ hdr,
                                                     uint2* __restrict__ inst, uint32_t* __restrict__ hist, TilePasses tp,
                                                     uint32_t* __restrict__ desc0, uint32_t desc0_words) {
  const uint4* __restrict__ el = depth_keys_narrow(hdr) ? el_b : el_a;  // where the depth passes ended
  __shared__ uint32_t s_w[kScanBlock / kWave];
  __shared__ uint32_t s_h[kMaxPasses - kTileRow0][kHistStride];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const ViewDev* views = table_views(table);
  const int nv = static_cast<const TableHdr*>(table)->num_views;
  for (int i = threadIdx.x; i < tp.n * kHistStride; i += kScanBlock) (&s_h[0][0])[i] = 0u;
  {  // this workgroup's slice of the first tile pass's descriptors
    const uint32_t chunk = (desc0_words + gridDim.x - 1) / gridDim.x;
    const uint32_t b0 = blockIdx.x * chunk;
    const uint32_t b1 = min(desc0_words, b0 + chunk);
    for (uint32_t i = b0 + threadIdx.x; i < b1; i += kScanBlock) desc0[i] = 0u;
  }
  const int64_t base = (int64_t)blockIdx.x * (kScanBlock * kItems) + (int64_t)w * (kItems * kWave) + lane;
  uint32_t c[kItems];
  uint32_t wtot = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const int64_t idx = base + (int64_t)i * kWave;
    c[i] = idx < n ? el_count(el[idx]) : 0u;
    wtot += c[i];
  }
  wtot = wave_sum(wtot);
  if (lane == 0) s_w[w] = wtot;
  __syncthreads();
  uint64_t off = boff[blockIdx.x];
  for (int k = 0; k < w; ++k) off += s_w[k];
  const uint64_t cap = hdr->capacity;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t inc = wave_incl_scan(c[i], lane);
    const uint64_t my = off + inc - c[i];
    off += __shfl(inc, kWave - 1, kWave);
    if (c[i] == 0) continue;
    const uint4 e = el[base + (int64_t)i * kWave];
    const uint32_t nx = e.w & 0xffffu, ny = e.w >> 16;
    const uint32_t tiles_x = (uint32_t)views[find_view_by_fv(views, nv, (int64_t)e.y)].tiles_x;
    uint64_t pos = my;
    for (uint32_t ty = 0; ty < ny; ++ty) {
      for (uint32_t tx = 0; tx < nx; ++tx, ++pos) {
        if (pos < cap) {
          const uint32_t tile = e.z + ty * tiles_x + tx;
          inst[pos] = make_uint2(tile, e.y);
          for (int p = 0; p < tp.n; ++p) atomicAdd(&s_h[p][(tile >> tp.shift[p]) & tp.mask[p]], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < tp.n * kHistStride; i += kScanBlock)
    if ((&s_h[0][0])[i]) atomicAdd(&hist[kTileRow0 * kHistStride + i], (&s_h[0][0])[i]);
}

void launch_bin(const void* table, const uint4* el_a, const uint4* el_b, int64_t n, int items, uint32_t* bsum, uint64_t* boff, int nb,
                WsHdr* hdr, uint32_t cap, uint2* inst, uint32_t* hist, const TilePasses& tp, uint32_t* desc0,
                uint32_t desc0_words, hipStream_t s) {
  const bool large = items == kScanItemsLarge;
  if (nb > 0) {
    if (large) hipLaunchKernelGGL(k_scan_reduce<kScanItemsLarge>, dim3(nb), dim3(kScanBlock), 0, s, el_a, el_b, hdr, n, bsum);
    else hipLaunchKernelGGL(k_scan_reduce<kScanItemsSmall>, dim3(nb), dim3(kScanBlock), 0, s, el_a, el_b, hdr, n, bsum);
  }
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, nb, boff, hdr, cap);
  if (nb > 0) {
    if (large)
      hipLaunchKernelGGL(k_emit<kScanItemsLarge>, dim3(nb), dim3(kScanBlock), 0, s, table, el_a, el_b, n, boff, hdr, inst, hist,
                         tp, desc0, desc0_words);
    else
      hipLaunchKernelGGL(k_emit<kScanItemsSmall>, dim3(nb), dim3(kScanBlock), 0, s, table, el_a, el_b, n, boff, hdr, inst, hist,
                         tp, desc0, desc0_words);
  }
}

}  // namespace gmr
