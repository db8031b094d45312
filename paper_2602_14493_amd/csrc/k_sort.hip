// LSD onesweep radix sort and tile ranges.
//
// The (tile | depth) key of an instance is sorted least significant digit first.  The depth digits
// are identical for every instance of a face-view, so their passes run on the face-views, before
// instances are emitted (4 passes of 8 bits over 16 B face-view elements {depth bits, face-view,
// first tile, nx | ny << 16}); emission then walks face-views in depth order, and the tile digits
// are sorted on the instances (uint2 {tile, face-view}, passes of up to 9 bits).  The result is the
// stable sort of the instances by (tile, float32 depth, face-view), i.e. ties in depth broken by
// ascending global id, with far fewer bytes moved than sorting 64-bit keys per instance.  When the
// visible face-views' keys span fewer than 256 values of their high 16 bits (depths within a
// factor of ~3.7, the usual object-centric view), the third depth pass sorts on the offset
// (key >> 16) - min, which orders those bits exactly, and the fourth pass exits at once.
//
// k_onesweep (one launch per pass): each workgroup takes a partition ticket, so every earlier
// partition is already resident; it loads its partition (4096 elements, or 1024 for small inputs),
// ranks them stably in LDS with wavefront ballots (one ballot per digit bit matches equal digits
// among 64 lanes), publishes its digit counts, resolves its global offsets by decoupled look-back
// over the earlier partitions' descriptors, stages the elements in LDS in digit order and writes
// them out in coalesced runs.
// Descriptor word: bits 31..30 = {0 empty, 1 aggregate, 2 inclusive prefix}, bits 29..0 = count,
// so a single 32-bit atomic load observes flag and value together.  Each pass also clears its
// share of the descriptor buffer the next pass will use, and scans its own digit histogram.
#include "gmr_common.h"
#include "gmr_launch.h"

namespace gmr {

__device__ inline uint32_t elem_key(const uint4& e) { return e.x; }
__device__ inline uint32_t elem_key(const uint2& e) { return e.x; }

__device__ inline uint32_t desc_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void desc_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// kSplit: write keys and values to separate uint32 arrays (the last instance pass).
// kItems: elements per thread; a partition holds kSortBlock * kItems elements.
template <typename E, int kRadix, bool kSplit, int kItems>
__global__ __launch_bounds__(kSortBlock) void k_onesweep(const E* __restrict__ in, E* __restrict__ out,
                                                         uint32_t* __restrict__ out_k, uint32_t* __restrict__ out_v,
                                                         const uint32_t* __restrict__ n_dev, uint32_t n_max,
                                                         const uint32_t* __restrict__ hist, uint32_t* desc_cur,
                                                         uint32_t* desc_next, uint32_t next_words, uint32_t* ticket,
                                                         int shift, uint32_t mask, const WsHdr* range_hdr,
                                                         int depth_pass) {
  constexpr int kNW = kSortBlock / kWave;
  constexpr int kBits = kRadix == 256 ? 8 : 9;
  constexpr int kPart = kSortBlock * kItems;
  __shared__ E s_el[kPart];
  __shared__ uint32_t s_wcnt[kNW][kRadix];
  __shared__ uint32_t s_bstart[kRadix];
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_wsum[kNW];
  __shared__ uint32_t s_hsum[kNW];
  __shared__ uint32_t s_part;

  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  // narrow depth range: the third depth pass sorts on (key >> 16) - key_hi_min, the fourth is void
  uint32_t sub = 0u;
  if (range_hdr && depth_pass >= 2 && depth_keys_narrow(range_hdr)) {
    if (depth_pass == 3) return;
    sub = key_hi_min(range_hdr);
  }
  // clear this workgroup's slice of the next pass's descriptors (every workgroup, before any exit)
  {
    const uint32_t chunk = (next_words + gridDim.x - 1) / gridDim.x;
    const uint32_t b0 = blockIdx.x * chunk;
    const uint32_t b1 = min(next_words, b0 + chunk);
    for (uint32_t i = b0 + threadIdx.x; i < b1; i += kSortBlock) desc_next[i] = 0u;
  }
  if (threadIdx.x == 0) s_part = atomicAdd(ticket, 1u);
  for (int i = threadIdx.x; i < kNW * kRadix; i += kSortBlock) (&s_wcnt[0][0])[i] = 0u;
  // global start of this thread's digit: exclusive scan of the pass's digit histogram
  const int d = threadIdx.x;
  uint32_t hcount = 0u;
  if (d < kRadix) {
    const uint32_t bin = sub ? ((uint32_t)d + sub) & 0xffu : (uint32_t)d;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) hcount += hist[c * kHistWords + bin];
  }
  uint32_t hinc = hcount;
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) {
    const uint32_t y = __shfl_up(hinc, s, kWave);
    if (lane >= s) hinc += y;
  }
  if (lane == kWave - 1) s_hsum[w] = hinc;
  __syncthreads();
  uint32_t dig_d = hinc - hcount;
  for (int ww = 0; ww < w; ++ww) dig_d += s_hsum[ww];
  const uint32_t n = n_dev ? min(*n_dev, n_max) : n_max;
  const uint32_t part = s_part;
  const uint32_t nparts = (n + kPart - 1) / kPart;
  if (part >= nparts) return;  // uniform across the workgroup
  const uint32_t base = part * kPart;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  // ---- load every element first (all loads in flight together)
  E e[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t idx = base + (uint32_t)w * (kItems * kWave) + (uint32_t)i * kWave + (uint32_t)lane;
    if (idx < n) e[i] = in[idx];
    else e[i] = E{};
  }
  // ---- stable ranking: wavefront w owns elements [w*ITEMS*64, (w+1)*ITEMS*64), 64 at a time
  uint32_t rank[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t idx = base + (uint32_t)w * (kItems * kWave) + (uint32_t)i * kWave + (uint32_t)lane;
    const bool have = idx < n;
    const uint32_t d = ((elem_key(e[i]) >> shift) - sub) & mask;
    // lanes whose digit equals this lane's: per bit, keep the lanes whose bit agrees with ours --
    // peers &= ~(ballot(bit) ^ (bit ? ~0 : 0)), on the two 32-bit halves (m = the bit sign-extended)
    const uint64_t h = __ballot(have);
    uint32_t plo = (uint32_t)h, phi = (uint32_t)(h >> 32);
#pragma unroll
    for (int b = 0; b < kBits; ++b) {
      const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);
      const uint64_t bb = __ballot(m != 0u);
      plo &= ~((uint32_t)bb ^ m);
      phi &= ~((uint32_t)(bb >> 32) ^ m);
    }
    const uint64_t peers = (uint64_t)plo | ((uint64_t)phi << 32);
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    uint32_t old = 0;
    if (have) old = s_wcnt[w][d];
    wave_lds_sync();
    if (have && below == 0) s_wcnt[w][d] = old + (uint32_t)__popcll(peers);
    wave_lds_sync();
    rank[i] = old + below;
  }
  __syncthreads();

  // ---- per digit: wavefront-exclusive offsets, publish, look back
  uint32_t tot = 0;
  if (d < kRadix) {
    for (int ww = 0; ww < kNW; ++ww) {
      const uint32_t c = s_wcnt[ww][d];
      s_wcnt[ww][d] = tot;
      tot += c;
    }
    uint32_t* my = desc_cur + (size_t)part * kRadix + d;
    desc_store(my, (part == 0 ? kFlagInc : kFlagAgg) | tot);
    uint32_t excl = 0;
    if (part > 0) {
      // look back kLook predecessors at a time (all loads in flight together), consuming them in
      // order until an inclusive prefix; an empty descriptor ends the window and is read again
      constexpr int kLook = 8;
      int j = (int)part - 1;
      while (true) {
        uint32_t x[kLook];
#pragma unroll
        for (int i = 0; i < kLook; ++i)  // below partition 0 (never reached: it is inclusive) read nothing
          x[i] = j - i >= 0 ? desc_load(desc_cur + (size_t)(j - i) * kRadix + d) : kFlagInc;
        int used = 0;
        bool done = false, empty = false;
#pragma unroll
        for (int i = 0; i < kLook; ++i) {
          if (done || empty) continue;
          if ((x[i] & ~kValMask) == 0u) {
            empty = true;
            continue;
          }
          excl += x[i] & kValMask;
          ++used;
          done = (x[i] & kFlagInc) != 0u;
        }
        if (done) break;
        j -= used;
        if (empty) __builtin_amdgcn_s_sleep(1);
      }
      desc_store(my, kFlagInc | (excl + tot));
    }
    s_gbase[d] = dig_d + excl;
  }
  // block-local exclusive scan of the digit totals (threads >= kRadix contribute 0)
  {
    uint32_t inc = tot;
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
      const uint32_t y = __shfl_up(inc, s, kWave);
      if (lane >= s) inc += y;
    }
    if (lane == kWave - 1) s_wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int ww = 0; ww < w; ++ww) before += s_wsum[ww];
    if (d < kRadix) s_bstart[d] = before + inc - tot;
  }
  __syncthreads();

  // ---- stage in digit order, then write out in coalesced runs
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t idx = base + (uint32_t)w * (kItems * kWave) + (uint32_t)i * kWave + (uint32_t)lane;
    if (idx < n) {
      const uint32_t dd = ((elem_key(e[i]) >> shift) - sub) & mask;
      s_el[s_bstart[dd] + s_wcnt[w][dd] + rank[i]] = e[i];
    }
  }
  __syncthreads();
  const uint32_t nb = min((uint32_t)kPart, n - base);
  for (uint32_t s = threadIdx.x; s < nb; s += kSortBlock) {
    const E x = s_el[s];
    const uint32_t dd = ((elem_key(x) >> shift) - sub) & mask;
    const uint32_t g = s_gbase[dd] + (s - s_bstart[dd]);
    if (g >= n) continue;  // only if the histogram disagreed with n: never write past the input's size
    if constexpr (kSplit) {
      out_k[g] = elem_key(x);
      out_v[g] = reinterpret_cast<const uint32_t*>(&x)[1];
    } else {
      out[g] = x;
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = val;
}

// Start / end of each tile's run in the sorted keys (their tile-id bits: tmask; the bits above
// carry the raster-block masks).  A thread takes 8 consecutive keys with two 16-B loads plus its two
// neighbours, so the kernel streams the keys once at full width.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* __restrict__ keys, uint32_t tmask,
                                                     const WsHdr* __restrict__ hdr, uint32_t* __restrict__ ranges) {
  constexpr uint32_t kNone = 0xFFFFFFFFu;  // tile ids are < 2^30: never equal to a masked key
  const uint32_t n = min(hdr->count, hdr->capacity);
  const uint32_t groups = (n + 7u) / 8u;
  for (uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x; gi < groups; gi += gridDim.x * blockDim.x) {
    const uint32_t i0 = 8u * gi;
    uint32_t k[10];
    if (i0 + 8u <= n) {
      const uint4 a = reinterpret_cast<const uint4*>(keys + i0)[0];
      const uint4 b = reinterpret_cast<const uint4*>(keys + i0)[1];
      k[1] = a.x & tmask; k[2] = a.y & tmask; k[3] = a.z & tmask; k[4] = a.w & tmask;
      k[5] = b.x & tmask; k[6] = b.y & tmask; k[7] = b.z & tmask; k[8] = b.w & tmask;
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) k[1 + j] = i0 + j < n ? keys[i0 + j] & tmask : kNone;
    }
    k[0] = i0 > 0u ? keys[i0 - 1u] & tmask : kNone;
    k[9] = i0 + 8u < n ? keys[i0 + 8u] & tmask : kNone;
#pragma unroll
    for (int j = 1; j <= 8; ++j) {
      const uint32_t t = k[j];
      if (t == kNone) break;
      const uint32_t i = i0 + (uint32_t)(j - 1);
      if (k[j - 1] != t) ranges[2 * (size_t)t] = i;
      if (k[j + 1] != t) ranges[2 * (size_t)t + 1] = i + 1u;
    }
  }
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)nb), dim3(256), 0, s, p, n, val);
}

template <int kItems>
static void sort_fv_pass(const uint4* in, uint4* out, uint32_t n, const uint32_t* hist, uint32_t* desc_cur,
                         uint32_t* desc_next, uint32_t next_words, uint32_t* ticket, int pass, const WsHdr* hdr,
                         hipStream_t s) {
  const uint32_t parts = (n + kSortBlock * kItems - 1) / (kSortBlock * kItems);
  if (parts == 0) return;
  hipLaunchKernelGGL((k_onesweep<uint4, 256, false, kItems>), dim3(parts), dim3(kSortBlock), 0, s, in, out, nullptr,
                     nullptr, nullptr, n, hist, desc_cur, desc_next, next_words, ticket, 8 * pass, 255u, hdr, pass);
}

void launch_sort_fv_pass(const uint4* in, uint4* out, uint32_t n, const uint32_t* hist, uint32_t* desc_cur,
                         uint32_t* desc_next, uint32_t next_words, uint32_t* ticket, int pass, const WsHdr* hdr,
                         int items, hipStream_t s) {
  if (items == kSortItemsSmall)
    sort_fv_pass<kSortItemsSmall>(in, out, n, hist, desc_cur, desc_next, next_words, ticket, pass, hdr, s);
  else
    sort_fv_pass<kSortItemsLarge>(in, out, n, hist, desc_cur, desc_next, next_words, ticket, pass, hdr, s);
}

template <int kRadix, int kItems>
static void sort_inst_pass(const uint2* in, uint2* out, uint32_t* out_k, uint32_t* out_v, const uint32_t* n_dev,
                           uint32_t cap, const uint32_t* hist, uint32_t* desc_cur, uint32_t* desc_next,
                           uint32_t next_words, uint32_t* ticket, int shift, uint32_t mask, hipStream_t s) {
  const uint32_t parts = (cap + kSortBlock * kItems - 1) / (kSortBlock * kItems);
  if (parts == 0) return;
  if (out_k)
    hipLaunchKernelGGL((k_onesweep<uint2, kRadix, true, kItems>), dim3(parts), dim3(kSortBlock), 0, s, in, out, out_k,
                       out_v, n_dev, cap, hist, desc_cur, desc_next, next_words, ticket, shift, mask, nullptr, -1);
  else
    hipLaunchKernelGGL((k_onesweep<uint2, kRadix, false, kItems>), dim3(parts), dim3(kSortBlock), 0, s, in, out, out_k,
                       out_v, n_dev, cap, hist, desc_cur, desc_next, next_words, ticket, shift, mask, nullptr, -1);
}

void launch_sort_inst_pass(const uint2* in, uint2* out, uint32_t* out_k, uint32_t* out_v, const uint32_t* n_dev,
                           uint32_t cap, const uint32_t* hist, uint32_t* desc_cur, uint32_t* desc_next,
                           uint32_t next_words, uint32_t* ticket, int shift, uint32_t mask, int items, hipStream_t s) {
  // digits of <= 8 bits use the 256-bin variant (fewer ballots, half the descriptors)
  const bool narrow = mask <= 255u, small = items == kSortItemsSmall;
  if (narrow && small)
    sort_inst_pass<256, kSortItemsSmall>(in, out, out_k, out_v, n_dev, cap, hist, desc_cur, desc_next, next_words,
                                         ticket, shift, mask, s);
  else if (narrow)
    sort_inst_pass<256, kSortItemsLarge>(in, out, out_k, out_v, n_dev, cap, hist, desc_cur, desc_next, next_words,
                                         ticket, shift, mask, s);
  else if (small)
    sort_inst_pass<512, kSortItemsSmall>(in, out, out_k, out_v, n_dev, cap, hist, desc_cur, desc_next, next_words,
                                         ticket, shift, mask, s);
  else
    sort_inst_pass<512, kSortItemsLarge>(in, out, out_k, out_v, n_dev, cap, hist, desc_cur, desc_next, next_words,
                                         ticket, shift, mask, s);
}

// ranges[] was zeroed by the list-building prologue (tiles without instances stay [0, 0)).
void launch_tile_ranges(const uint32_t* sorted_keys, uint32_t tile_mask, const WsHdr* hdr, uint32_t* ranges, int blocks,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_tile_ranges, dim3(blocks), dim3(256), 0, s, sorted_keys, tile_mask, hdr, ranges);
}

}  // namespace gmr
