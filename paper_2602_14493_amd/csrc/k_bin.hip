// Tile binning over the depth-sorted face-view elements: exclusive scan of tiles-touched, then
// emission of one instance {tile, face-view} per (face-view, tile) in that order (the key carrying,
// above the tile id, the instance's raster-block mask when the table enables them).  Emission order
// is (float32 depth, face-view), so a stable sort on the tile id alone completes the
// (tile, depth, id) order.  The emitter also accumulates the histograms of the tile digits and
// clears the first tile pass's descriptors.
//
// One pass: each workgroup takes a ticket b (so every earlier block is already resident), counts
// the instances of its face-views, publishes that aggregate, finds its exclusive offset by
// decoupled look-back over the earlier blocks' descriptors (one wavefront reads 64 of them at a
// time) and emits, from the elements it kept in registers.  Large inputs: the wavefront writes the
// runs of its 64 face-views 64 instances at a time (coalesced stores, every lane busy); small,
// latency-bound inputs: each lane writes its own face-view's run.  Element t of block b, wave w,
// round i, lane l is b*256*I + w*64*I + i*64 + l (I face-views per thread): every load is a
// coalesced 64-wide run.  Descriptor (64-bit): bits
// 63..62 = {0 empty, 1 aggregate, 2 inclusive prefix}, bits 61..0 = count; the list-building
// prologue clears them.  The last block writes the instance total and the overflow flag.
#include "gmr_common.h"
#include "gmr_launch.h"

namespace gmr {

// Instances of a face-view from its packed tile extent (nx, ny fields of the element's last word).
__device__ inline uint32_t wh_count(uint32_t wh) { return el_nx(wh) * el_ny(wh); }

// The face-view's block columns / rows in its first and last tiles, and ny, packed for the emission:
// clo | chi << 3 | rlo << 6 | rhi << 9 | ny << 16 (from the element's last two words).
__device__ inline uint32_t emit_bits(uint32_t ez, uint32_t ew) {
  return ((ew >> 13) & 7u) | (((ez >> 26) & 7u) << 3) | ((ew >> 29) << 6) | ((ez >> 29) << 9) | (el_ny(ew) << 16);
}

// Raster-block mask of the instance in tile column tx (of nx) and row ty of the face-view's range.
__device__ inline uint32_t emit_mask(uint32_t bits, uint32_t tx, uint32_t ty, uint32_t nx, uint32_t sub_x,
                                     uint32_t sub_y) {
  const uint32_t ny = bits >> 16;
  const uint32_t clo = tx == 0u ? (bits & 7u) : 0u, chi = tx + 1u == nx ? ((bits >> 3) & 7u) : sub_x - 1u;
  const uint32_t rlo = ty == 0u ? ((bits >> 6) & 7u) : 0u, rhi = ty + 1u == ny ? ((bits >> 9) & 7u) : sub_y - 1u;
  return block_mask(clo, chi, rlo, rhi, sub_x);
}

// Per-wavefront staging of one round's 64 face-views for the cooperative emission.
struct EmitLds {
  uint32_t fv[kWave], t0[kWave], nxtx[kWave], ex[kWave];  // face-view, first tile, nx | tiles_x << 16, run start
  uint32_t bits[kWave];                                    // emit_bits of the face-view
  int32_t mark[kWave];                                     // source lane of the run starting at a window slot
};

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

__device__ inline uint64_t wave_sum64(uint64_t x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

constexpr uint64_t kBinAgg = 1ull << 62, kBinInc = 2ull << 62, kBinVal = (1ull << 62) - 1ull;

__device__ inline uint64_t bdesc_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void bdesc_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront 0 of block b (b > 0): the sum of the counts of blocks [0, b).  Lane l reads the
// descriptor of block j - l; the nearest inclusive prefix ends the walk, and an empty descriptor
// (its block has not published yet) ends the window, to be read again.
__device__ inline uint64_t bin_lookback(const uint64_t* desc, uint32_t b, int lane) {
  uint64_t excl = 0;
  int64_t j = (int64_t)b - 1;
  while (true) {
    const int64_t q = j - lane;
    // below block 0 nothing is read: block 0 publishes an inclusive prefix, which ends the walk first
    const uint64_t x = q >= 0 ? bdesc_load(desc + q) : kBinInc;
    const uint64_t inc_m = __ballot((x & ~kBinVal) == kBinInc);
    const uint64_t stop = inc_m | __ballot((x & ~kBinVal) == 0ull);
    const int f = stop ? __builtin_ctzll(stop) : kWave;  // nearest lane that is not a plain aggregate
    const bool inclusive = f < kWave && ((inc_m >> f) & 1ull);
    const int upto = inclusive ? f + 1 : f;
    excl += wave_sum64(lane < upto ? (x & kBinVal) : 0ull);
    if (inclusive) return excl;
    j -= f;
    if (f < kWave) __builtin_amdgcn_s_sleep(1);
  }
}

template <int kItems>
__global__ __launch_bounds__(kScanBlock) void k_emit(const void* __restrict__ table, const uint4* __restrict__ el_a,
                                                     const uint4* __restrict__ el_b, int64_t n, uint32_t nb,
                                                     uint64_t* bdesc, WsHdr* hdr, uint32_t cap32,
                                                     uint2* __restrict__ inst, uint32_t* __restrict__ hist, TilePasses tp,
                                                     uint32_t* __restrict__ desc0, uint32_t desc0_words) {
  const uint4* __restrict__ el = depth_keys_narrow(hdr) ? el_b : el_a;  // where the depth passes ended
  const TableHdr* th = static_cast<const TableHdr*>(table);
  const int bsh = th->bm_shift1 - 1;  // key bit of the raster-block masks (< 0: none)
  const uint32_t sub_x = (uint32_t)th->sub_x, sub_y = (uint32_t)th->sub_y;
  __shared__ uint32_t s_w[kScanBlock / kWave];
  __shared__ uint32_t s_h[kMaxPasses - kTileRow0][kHistStride];
  __shared__ uint32_t s_b;
  __shared__ uint64_t s_excl;
  __shared__ EmitLds s_lds[kScanBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (threadIdx.x == 0) s_b = atomicAdd(&hdr->emit_ctr, 1u);
  const ViewDev* views = table_views(table);
  const int nv = th->num_views;
  for (int i = threadIdx.x; i < tp.n * kHistStride; i += kScanBlock) (&s_h[0][0])[i] = 0u;
  {  // this workgroup's slice of the first tile pass's descriptors
    const uint32_t chunk = (desc0_words + gridDim.x - 1) / gridDim.x;
    const uint32_t b0 = blockIdx.x * chunk;
    const uint32_t b1 = min(desc0_words, b0 + chunk);
    for (uint32_t i = b0 + threadIdx.x; i < b1; i += kScanBlock) desc0[i] = 0u;
  }
  __syncthreads();  // s_b (and the cleared histogram)
  const uint32_t b = s_b;
  const int64_t base = (int64_t)b * (kScanBlock * kItems) + (int64_t)w * (kItems * kWave) + lane;
  // the elements stay in registers from the count to the emission: {face-view, first tile, nx | ny << 16}
  uint32_t ef[kItems], et[kItems], ew[kItems];
  uint32_t wtot = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const int64_t idx = base + (int64_t)i * kWave;
    ew[i] = 0u;
    ef[i] = et[i] = 0u;
    if (idx < n) {
      const uint4 e = el[idx];
      ef[i] = e.y; et[i] = e.z; ew[i] = e.w;
    }
    wtot += wh_count(ew[i]);
  }
  wtot = wave_sum(wtot);
  if (lane == 0) s_w[w] = wtot;
  __syncthreads();
  if (w == 0) {
    uint64_t tot = 0;
    for (int k = 0; k < kScanBlock / kWave; ++k) tot += s_w[k];
    if (lane == 0) bdesc_store(bdesc + b, (b == 0 ? kBinInc : kBinAgg) | tot);
    const uint64_t excl = b > 0 ? bin_lookback(bdesc, b, lane) : 0ull;
    if (lane == 0) {
      if (b > 0) bdesc_store(bdesc + b, kBinInc | (excl + tot));
      s_excl = excl;
      if (b + 1 == nb) {
        const uint64_t total = excl + tot;
        hdr->count = total > 0xffffffffull ? 0xffffffffu : (uint32_t)total;
        hdr->overflow = total > cap32 ? 1u : 0u;
        hdr->peak_count = max(hdr->peak_count, hdr->count);
      }
    }
  }
  __syncthreads();
  uint64_t off = s_excl;
  for (int k = 0; k < w; ++k) off += s_w[k];
  const uint64_t cap = cap32;
  if constexpr (kItems == kScanItemsSmall) {
    // small inputs (latency-bound): each lane writes its own face-view's run
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const uint32_t c = wh_count(ew[i]);
      const uint32_t inc = wave_incl_scan(c, lane);
      uint64_t pos = off + inc - c;
      off += __shfl(inc, kWave - 1, kWave);
      if (c == 0u) continue;
      const uint32_t nx = el_nx(ew[i]), ny = el_ny(ew[i]);
      const uint32_t tiles_x = (uint32_t)views[find_view_by_fv(views, nv, (int64_t)ef[i])].tiles_x;
      const uint32_t bits = emit_bits(et[i], ew[i]), tile0 = bsh >= 0 ? et[i] & kElTileMask : et[i];
      for (uint32_t ty = 0; ty < ny; ++ty) {
        for (uint32_t tx = 0; tx < nx; ++tx, ++pos) {
          if (pos < cap) {
            const uint32_t tile = tile0 + ty * tiles_x + tx;
            const uint32_t key = bsh >= 0 ? tile | (emit_mask(bits, tx, ty, nx, sub_x, sub_y) << bsh) : tile;
            inst[pos] = make_uint2(key, ef[i]);
            for (int q = 0; q < tp.n; ++q) atomicAdd(&s_h[q][(tile >> tp.shift[q]) & tp.mask[q]], 1u);
          }
        }
      }
    }
  } else {
    EmitLds& L = s_lds[w];
    const uint64_t le_mask = (2ull << lane) - 1ull;  // slots 0..lane
    // Large inputs: each round's 64 face-views own consecutive runs of the output, and the wavefront
    // writes them 64 instances at a time (coalesced, every lane busy): slot t of a window holds
    // output j0 + t, whose face-view is the one whose run starts at the last marked slot <= t (each
    // run marks its first slot in the window).
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const uint32_t c = wh_count(ew[i]);
      const uint32_t inc = wave_incl_scan(c, lane);
      const uint32_t total = __shfl(inc, kWave - 1, kWave);
      if (total == 0u) continue;  // wave-uniform
      const uint32_t excl = inc - c;
      const uint32_t nx = el_nx(ew[i]);
      const uint32_t tiles_x = c ? (uint32_t)views[find_view_by_fv(views, nv, (int64_t)ef[i])].tiles_x : 0u;
      L.fv[lane] = ef[i];
      L.t0[lane] = bsh >= 0 ? et[i] & kElTileMask : et[i];
      L.nxtx[lane] = nx | (tiles_x << 16);
      L.ex[lane] = excl;
      L.bits[lane] = emit_bits(et[i], ew[i]);
      for (uint32_t j0 = 0; j0 < total; j0 += kWave) {
        L.mark[lane] = -1;
        wave_lds_sync();
        if (c > 0u && excl < j0 + kWave && excl + c > j0) L.mark[excl > j0 ? excl - j0 : 0u] = lane;
        wave_lds_sync();
        const int mk = L.mark[lane];
        const uint64_t heads = __ballot(mk >= 0) & le_mask;  // slot 0 is always marked
        const int ps = 63 - __builtin_clzll(heads);
        const int src = ps == lane ? mk : L.mark[ps];
        const uint32_t j = j0 + (uint32_t)lane;
        if (j < total) {
          const uint32_t k = j - L.ex[src];
          const uint32_t nt = L.nxtx[src], nxs = nt & 0xffffu;
          // k / nxs: a float estimate (k < 2^24 is exact in float), then exact integer correction
          uint32_t ty = (uint32_t)((float)k * __builtin_amdgcn_rcpf((float)nxs));
          int32_t r = (int32_t)(k - ty * nxs);
          while (r < 0) { --ty; r += (int32_t)nxs; }
          while (r >= (int32_t)nxs) { ++ty; r -= (int32_t)nxs; }
          const uint64_t pos = off + j;
          if (pos < cap) {
            const uint32_t tile = L.t0[src] + ty * (nt >> 16) + (uint32_t)r;
            const uint32_t key =
                bsh >= 0 ? tile | (emit_mask(L.bits[src], (uint32_t)r, ty, nxs, sub_x, sub_y) << bsh) : tile;
            inst[pos] = make_uint2(key, L.fv[src]);
            for (int q = 0; q < tp.n; ++q) {
              const uint32_t dg = (tile >> tp.shift[q]) & tp.mask[q];
              if (q == 0) {  // the low digit of a run of neighbouring tiles: spread over the bins
                atomicAdd(&s_h[q][dg], 1u);
              } else {
                // higher digits: the window's tiles mostly share them, and same-address LDS atomics
                // serialise -- the lanes holding the first active lane's digit add once
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
                const uint64_t same = __ballot(dg == d0);
                if (dg != d0) atomicAdd(&s_h[q][dg], 1u);
                else if (lane == __builtin_ctzll(same)) atomicAdd(&s_h[q][d0], (uint32_t)__popcll(same));
              }
            }
          }
        }
        wave_lds_sync();  // the next window (or round) rewrites the slots
      }
      off += total;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < tp.n * kHistStride; i += kScanBlock)
    if ((&s_h[0][0])[i])
      atomicAdd(&hist[(blockIdx.x % kHistCopies) * kHistWords + kTileRow0 * kHistStride + i], (&s_h[0][0])[i]);
}

void launch_bin(const void* table, const uint4* el_a, const uint4* el_b, int64_t n, int items, uint64_t* bdesc, int nb,
                WsHdr* hdr, uint32_t cap, uint2* inst, uint32_t* hist, const TilePasses& tp, uint32_t* desc0,
                uint32_t desc0_words, hipStream_t s) {
  if (nb <= 0) return;  // the prologue left count = 0, overflow = 0
  if (items == kScanItemsLarge)
    hipLaunchKernelGGL(k_emit<kScanItemsLarge>, dim3(nb), dim3(kScanBlock), 0, s, table, el_a, el_b, n, (uint32_t)nb,
                       bdesc, hdr, cap, inst, hist, tp, desc0, desc0_words);
  else
    hipLaunchKernelGGL(k_emit<kScanItemsSmall>, dim3(nb), dim3(kScanBlock), 0, s, table, el_a, el_b, n, (uint32_t)nb,
                       bdesc, hdr, cap, inst, hist, tp, desc0, desc0_words);
}

}  // namespace gmr
