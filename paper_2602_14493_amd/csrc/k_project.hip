// Conversion (Sec. 2.2) fused with the EWA projection (Sec. 2.1), one thread per face.
//
// A face is converted once, in double precision, and projected into every view of its mesh.  Per
// face-view it writes, view-major (coalesced across consecutive faces):
//   rec[fv]  3 x float4 = 48 B  {u_hi, v_hi, u_lo, v_lo}  mean as float pairs (u = u_hi + u_lo)
//                              {k l11, k l12, k l22, x-rect}  scaled Cholesky factor of the conic
//                              {r, g, b, y-rect}              Eq. 16 colour; rects pack lo | hi << 16
//   el[fv]   uint4 = 16 B      {float32 depth bits, fv, first tile, nx | ny << 16}: the element the
//                              depth passes of the radix sort move (culled: nx = ny = 0); with
//                              raster-block masks, the spare bits of the last two words hold the
//                              rectangle's block columns and rows in its first and last tiles
// and adds each element's four 8-bit depth digits to the sort's histograms (LDS, then one global
// atomic per bin and workgroup), and the range of the visible keys' high 16 bits to the workspace
// header (per-thread, then one atomic pair per wavefront).
// The mean stays in double until it is split into two floats: a float32 pixel coordinate near
// x = 1920 carries ~1e-4 px of rounding, which alone would move alpha by ~1e-4.
#include "gmr_common.h"
#include "gmr_launch.h"
#include "gmr_sh.h"

namespace gmr {

// One-workgroup list build for small batches: at most kSmallThreads * kSmallPer face-views and
// kSmallInst instances, keys (tile | depth | face-view) with the face-view in kSmallFvBits bits.
constexpr int kSmallThreads = 1024, kSmallPer = 4, kSmallInst = 8192, kSmallFvBits = 14;

// SHD > 0: view-dependent colour of degree SHD (colours hold (SHD + 1)^2 coefficients per
// channel and vertex); SHD = 0: Eq. 16.
template <int SHD>
__device__ inline void project_face(const TableHdr* th, const void* __restrict__ table, const float* __restrict__ verts,
                                    const int32_t* __restrict__ faces, const float* __restrict__ colors, const KOpts& o,
                                    float4* __restrict__ rec, uint4* __restrict__ el, uint32_t* s_h,
                                    uint32_t& kmin, uint32_t& kmax, float4* __restrict__ dfv_zero, int64_t f,
                                    int u, int lpf) {
  const int32_t* mfo = table_i32(table, th->mesh_face_off);
  const int32_t* mvo = table_i32(table, th->mesh_view_off);
  const int32_t* mvs = table_i32(table, th->mesh_views_off);
  const ViewDev* views = table_views(table);
  const int m = find_mesh(mfo, th->num_meshes, (int32_t)f);
  const int tw = th->tile_w, tht = th->tile_h;

  const int32_t i0 = faces[3 * f], i1 = faces[3 * f + 1], i2 = faces[3 * f + 2];
  double vi[3], vj[3], vk[3];
  for (int a = 0; a < 3; ++a) {
    vi[a] = verts[3 * (int64_t)i0 + a];
    vj[a] = verts[3 * (int64_t)i1 + a];
    vk[a] = verts[3 * (int64_t)i2 + a];
  }
  FaceGeo g;
  const bool ok = face_convert(vi, vj, vk, o.cov_mode, g);
  float col[3];
  float coef[sh_count<SHD>()][3];
  if constexpr (SHD == 0) {
    for (int a = 0; a < 3; ++a)
      col[a] = (float)(((double)colors[3 * (int64_t)i0 + a] + (double)colors[3 * (int64_t)i1 + a] +
                        (double)colors[3 * (int64_t)i2 + a]) * (1.0 / 3.0));
  } else {
    face_coefs<SHD>(colors, i0, i1, i2, coef);
  }
  const double kscale = kRasterScale;

  for (int k = mvo[m] + u; k < mvo[m + 1]; k += lpf) {
    const ViewDev& V = views[mvs[k]];
    const int64_t fv = V.fv_offset + (f - V.face_begin);
    uint4 e = make_uint4(0xffffffffu, (uint32_t)fv, 0u, 0u);
    ProjGeo q;
    if (ok && view_project(V, g.mu, g.S, (double)o.dilation, q)) {
      const double rx = 3.0 * sqrt(q.sxx), ry = 3.0 * sqrt(q.syy);
      double x0 = ceil(q.u - rx - 0.5), x1 = floor(q.u + rx - 0.5);
      double y0 = ceil(q.v - ry - 0.5), y1 = floor(q.v + ry - 0.5);
      x0 = fmax(x0, 0.0); x1 = fmin(x1, (double)(V.W - 1));
      y0 = fmax(y0, 0.0); y1 = fmin(y1, (double)(V.H - 1));
      if (x0 <= x1 && y0 <= y1) {
        const int ix0 = (int)x0, ix1 = (int)x1, iy0 = (int)y0, iy1 = (int)y1;
        const int tx0 = ix0 / tw, tx1 = ix1 / tw, ty0 = iy0 / tht, ty1 = iy1 / tht;
        const int nx = tx1 - tx0 + 1, ny = ty1 - ty0 + 1;
        if constexpr (SHD > 0) {  // colour in this view
          double cc[3];
          view_centre(V.R, V.t, cc);
          const double px = g.mu[0] - cc[0], py = g.mu[1] - cc[1], pz = g.mu[2] - cc[2];
          const double ir = 1.0 / sqrt(px * px + py * py + pz * pz);
          double Y[sh_count<SHD>()];
          sh_basis<SHD>(px * ir, py * ir, pz * ir, Y);
          for (int a = 0; a < 3; ++a) {
            double raw = 0.0;
#pragma unroll
            for (int k = 0; k < sh_count<SHD>(); ++k) raw += (double)coef[k][a] * Y[k];
            col[a] = (float)fmax(raw, 0.0);
          }
        }
        const float uh = (float)q.u, vh = (float)q.v;
        const float ul = (float)(q.u - (double)uh), vl = (float)(q.v - (double)vh);
        // conic = L^T L, L = [[l11, l12], [0, l22]]; l22 = sqrt(det conic) / l11 = 1 / (l11 sqrt(det))
        const double l11 = sqrt(q.a);
        const double l12 = q.b / l11;
        const double l22 = 1.0 / (l11 * sqrt(q.det));
        float4* r = rec + kRecF4 * fv;
        r[0] = make_float4(uh, vh, ul, vl);
        r[1] = make_float4((float)(kscale * l11), (float)(kscale * l12), (float)(kscale * l22),
                           u2f((uint32_t)ix0 | ((uint32_t)ix1 << 16)));
        r[2] = make_float4(col[0], col[1], col[2], u2f((uint32_t)iy0 | ((uint32_t)iy1 << 16)));
        uint32_t ez = (uint32_t)(V.tile_base + ty0 * V.tiles_x + tx0), ew = (uint32_t)nx | ((uint32_t)ny << 16);
        if (th->bm_shift1 > 0) {  // the rectangle's block columns / rows in its first and last tiles
          const int bh = tht / th->sub_y;
          ez |= ((uint32_t)((ix1 - tx1 * tw) / kSub) << 26) | ((uint32_t)((iy1 - ty1 * tht) / bh) << 29);
          ew |= ((uint32_t)((ix0 - tx0 * tw) / kSub) << 13) | ((uint32_t)((iy0 - ty0 * tht) / bh) << 29);
        }
        e = make_uint4(f2u((float)q.p[2]), (uint32_t)fv, ez, ew);
        kmin = min(kmin, e.x >> 16);
        kmax = max(kmax, e.x >> 16);
      }
    }
    el[fv] = e;
    if (s_h) {  // the sort's digit histograms (the one-workgroup build below needs none)
#pragma unroll
      for (int p = 0; p < kDepthPasses; ++p) {
        const uint32_t dg = (e.x >> (8 * p)) & 255u;
        if (p < 2) {  // low digits: spread over the bins
          atomicAdd(&s_h[p * 256 + dg], 1u);
        } else {
          // high digits: neighbouring faces share them, and same-address LDS atomics serialise --
          // the lanes holding the first active lane's digit add once, with their count
          const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
          const uint64_t same = __ballot(dg == d0);
          if (dg != d0) atomicAdd(&s_h[p * 256 + dg], 1u);
          else if ((__lane_id() & (kWave - 1)) == (uint32_t)__builtin_ctzll(same))
            atomicAdd(&s_h[p * 256 + d0], (uint32_t)__popcll(same));
        }
      }
    }
    if (dfv_zero) {
      dfv_zero[2 * fv] = make_float4(0.f, 0.f, 0.f, 0.f);
      dfv_zero[2 * fv + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

// LPF lanes per face (1, or 8 with 1024-thread workgroups): lane u of a face's group converts the
// face and projects it into views u, u + LPF, ... of its mesh -- small batches then run LPF times as
// many wavefronts, each with a shorter FP64 chain, while a workgroup still covers 256 face-views'
// worth of histogram flushes per 256 threads.
template <int SHD, int LPF>
__global__ __launch_bounds__(256 * (LPF > 1 ? 4 : 1)) void k_project(const void* __restrict__ table, const float* __restrict__ verts,
                                                 const int32_t* __restrict__ faces, const float* __restrict__ colors,
                                                 KOpts o, float4* __restrict__ rec, uint4* __restrict__ el,
                                                 uint32_t* __restrict__ hist, WsHdr* __restrict__ hdr,
                                                 float4* __restrict__ dfv_zero) {
  __shared__ uint32_t s_h[kDepthPasses * 256];
  __shared__ uint32_t s_kmin[1024 / kWave], s_kmax[1024 / kWave];
  for (int i = threadIdx.x; i < kDepthPasses * 256; i += blockDim.x) s_h[i] = 0u;
  __syncthreads();
  const TableHdr* th = static_cast<const TableHdr*>(table);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t f = t / LPF;
  const int u = (int)(t - f * LPF);
  uint32_t kmin = 0xffffffffu, kmax = 0u;  // high 16 key bits of this thread's visible face-views
  if (f < th->faces_total)
    project_face<SHD>(th, table, verts, faces, colors, o, rec, el, s_h, kmin, kmax, dfv_zero, f, u, LPF);
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, d, kWave));
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, d, kWave));
  }
  // one atomic pair per workgroup, into copy b mod kKeyCopies: same-address atomics serialise, and
  // one pair per wavefront on a single address had set the projection's time
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_kmin[threadIdx.x / kWave] = kmin;
    s_kmax[threadIdx.x / kWave] = kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) {
      kmin = min(kmin, s_kmin[w]);
      kmax = max(kmax, s_kmax[w]);
    }
    if (kmin <= kmax) {
      atomicMin(&hdr->key_hi_min[blockIdx.x % kKeyCopies], kmin);
      atomicMax(&hdr->key_hi_max[blockIdx.x % kKeyCopies], kmax);
    }
  }
  for (int i = threadIdx.x; i < kDepthPasses * 256; i += blockDim.x)
    if (s_h[i]) atomicAdd(&hist[(blockIdx.x % kHistCopies) * kHistWords + (i >> 8) * kHistStride + (i & 255)], s_h[i]);
}

// Clears the per-build counters, every histogram row, the first depth pass's descriptors and the
// emission's block descriptors, sets the instance capacity (count 0 until the emission) and
// records where the raster kernels' per-item statistics live.
__global__ __launch_bounds__(256) void k_prologue(WsHdr* hdr, uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ desc0, int64_t desc0_words,
                                                  uint32_t* __restrict__ ranges, int64_t ranges_words,
                                                  uint64_t* __restrict__ bdesc, int64_t bdesc_n, uint32_t cap,
                                                  StatsInfo si) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t; i < desc0_words; i += stride) desc0[i] = 0u;
  for (int64_t i = t; i < ranges_words; i += stride) ranges[i] = 0u;  // empty tiles keep [0, 0)
  for (int64_t i = t; i < bdesc_n; i += stride) bdesc[i] = 0ull;
  for (int64_t i = t; i < kHistCopies * kHistWords; i += stride) hist[i] = 0u;
  if (t == 0) {
    for (int p = 0; p < kMaxPasses; ++p) hdr->part_ctr[p] = 0u;
    hdr->emit_ctr = 0u;
    hdr->count = 0u;  // the emission's last block overwrites both
    hdr->overflow = 0u;
    hdr->capacity = cap;
    hdr->stats_items = si.items;
    hdr->bwd_stats = si.bwd;
    hdr->stats_fwd_off = si.fwd_off;
    hdr->stats_bwd_off = si.bwd_off;
    hdr->red_ticket = 0u;
    if (si.bwd) {
      hdr->loss = 0.f;
      hdr->loss_sil = 0.f;
    }
    for (int c = 0; c < kKeyCopies; ++c) {
      hdr->key_hi_min[c] = 0xffffffffu;
      hdr->key_hi_max[c] = 0u;
    }
  }
}

// One-workgroup list build for small batches (every face-view and instance fits the workgroup's
// LDS): the same projection, then the instances' (tile | depth | face-view) keys -- tile id in the
// top kSmallTileBits bits, the float32 depth bits, the face-view in the low kSmallFvBits bits --
// sorted in LDS by a bitonic network, and the tile ranges.  Sorting that key orders the instances
// by (tile, depth, face-view), the order the radix sort of the large path produces, so the lists
// are identical; one launch replaces the prologue, the projection, the depth passes, the emission,
// the tile passes and the ranges, whose launch latencies dominate a small batch.  More instances
// than cap: the overflow flag is set (count = the true total) and no list is written.
__global__ __launch_bounds__(kSmallThreads) void k_build_small(const void* __restrict__ table,
                                                               const float* __restrict__ verts,
                                                               const int32_t* __restrict__ faces,
                                                               const float* __restrict__ colors, KOpts o,
                                                               float4* __restrict__ rec, uint4* __restrict__ el,
                                                               WsHdr* __restrict__ hdr, float4* __restrict__ dfv_zero,
                                                               uint32_t* __restrict__ ranges, int64_t ranges_words,
                                                               uint32_t* __restrict__ keys_out,
                                                               uint32_t* __restrict__ vals_out, uint32_t cap,
                                                               StatsInfo si) {
  __shared__ uint64_t s_key[kSmallInst];
  __shared__ uint32_t s_wsum[kSmallThreads / kWave];
  const TableHdr* th = static_cast<const TableHdr*>(table);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int64_t nfv = th->fv_total;
  for (int64_t i = tid; i < ranges_words; i += kSmallThreads) ranges[i] = 0u;  // empty tiles keep [0, 0)
  if (tid == 0) {
    hdr->capacity = cap;
    hdr->stats_items = si.items;
    hdr->bwd_stats = si.bwd;
    hdr->stats_fwd_off = si.fwd_off;
    hdr->stats_bwd_off = si.bwd_off;
    hdr->red_ticket = 0u;
    if (si.bwd) {
      hdr->loss = 0.f;
      hdr->loss_sil = 0.f;
    }
  }
  // 1. projection: records to the workspace, elements {depth bits, fv, first tile, nx | ny << 16}
  {
    uint32_t kmin = 0xffffffffu, kmax = 0u;
    for (int64_t f = tid; f < th->faces_total; f += kSmallThreads)
      project_face<0>(th, table, verts, faces, colors, o, rec, el, nullptr, kmin, kmax, dfv_zero, f, 0, 1);
  }
  __syncthreads();  // the elements (global, written by this workgroup) are visible to it
  // 2. instance offsets: thread t owns face-views [t * kSmallPer, (t + 1) * kSmallPer)
  uint4 e[kSmallPer];
  uint32_t cnt = 0;
#pragma unroll
  for (int i = 0; i < kSmallPer; ++i) {
    const int64_t fv = (int64_t)tid * kSmallPer + i;
    e[i] = fv < nfv ? el[fv] : make_uint4(0xffffffffu, 0u, 0u, 0u);
    cnt += el_nx(e[i].w) * el_ny(e[i].w);
  }
  uint32_t inc = cnt;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, kWave);
    if (lane >= d) inc += y;
  }
  if (lane == kWave - 1) s_wsum[w] = inc;
  __syncthreads();
  uint32_t base = inc - cnt, total = 0;
  for (int k = 0; k < kSmallThreads / kWave; ++k) {
    if (k < w) base += s_wsum[k];
    total += s_wsum[k];
  }
  if (tid == 0) {
    hdr->count = total;
    hdr->overflow = total > cap ? 1u : 0u;
    hdr->peak_count = max(hdr->peak_count, total);
  }
  if (total > cap) return;  // uniform: the host grows the capacity and builds again
  // 3. keys
  const ViewDev* views = table_views(table);
  const int bsh = th->bm_shift1 - 1;  // key bit of the raster-block masks (< 0: none)
#pragma unroll
  for (int i = 0; i < kSmallPer; ++i) {
    const uint32_t nx = el_nx(e[i].w), ny = el_ny(e[i].w);
    if (nx * ny == 0u) continue;
    const uint32_t fv = e[i].y;
    const uint32_t tiles_x = (uint32_t)views[find_view_by_fv(views, th->num_views, (int64_t)fv)].tiles_x;
    const uint32_t tile0 = bsh >= 0 ? e[i].z & kElTileMask : e[i].z;
    const uint64_t low = ((uint64_t)e[i].x << kSmallFvBits) | fv;
    for (uint32_t ty = 0; ty < ny; ++ty)
      for (uint32_t tx = 0; tx < nx; ++tx)
        s_key[base++] = ((uint64_t)(tile0 + ty * tiles_x + tx) << (32 + kSmallFvBits)) | low;
  }
  uint32_t n2 = 64;  // the network's width: the next power of two >= total
  while (n2 < total) n2 <<= 1;
  for (uint32_t i = total + tid; i < n2; i += kSmallThreads) s_key[i] = ~0ull;
  __syncthreads();
  // 4. bitonic sort of s_key[0, n2): thread t compares pairs t, t + T, ... (T = kSmallThreads).  A
  // stage of distance j <= 64 keeps every wavefront inside its own 128-key runs (keys 128 (w + 16 r)
  // onwards), so two such stages in a row need only the wavefront in step; any stage that crosses
  // runs, or is followed by one that does, ends with a workgroup barrier
  for (uint32_t k = 2; k <= n2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < n2 / 2; i += kSmallThreads) {
        const uint32_t lo = ((i & ~(j - 1u)) << 1) | (i & (j - 1u)), hi = lo + j;
        const uint64_t a = s_key[lo], b = s_key[hi];
        if ((a > b) == ((lo & k) == 0u)) {
          s_key[lo] = b;
          s_key[hi] = a;
        }
      }
      const uint32_t next_j = j > 1u ? j >> 1 : k;  // the next stage's distance (k: the next round's first)
      if (j > (uint32_t)kWave || next_j > (uint32_t)kWave) __syncthreads();
      else wave_lds_sync();
    }
  }
  __syncthreads();
  // 5. keys (with the raster-block masks, from the record's pixel rectangle), values, tile ranges
  for (uint32_t i = tid; i < total; i += kSmallThreads) {
    const uint64_t key = s_key[i];
    const uint32_t tile = (uint32_t)(key >> (32 + kSmallFvBits));
    const uint32_t fv = (uint32_t)key & ((1u << kSmallFvBits) - 1u);
    uint32_t kout = tile;
    if (bsh >= 0) {
      const ViewDev& V = views[find_view_by_tile(views, th->num_views, (int32_t)tile)];
      const int lt = (int)tile - V.tile_base, tyi = lt / V.tiles_x, txi = lt - tyi * V.tiles_x;
      const uint32_t rx = f2u(rec[kRecF4 * (size_t)fv + 1].w), ry = f2u(rec[kRecF4 * (size_t)fv + 2].w);
      kout |= rect_block_mask((int)(rx & 0xffffu), (int)(rx >> 16), (int)(ry & 0xffffu), (int)(ry >> 16),
                              txi * th->tile_w, tyi * th->tile_h, th->tile_w, th->tile_h, th->sub_x, th->sub_y)
              << bsh;
    }
    keys_out[i] = kout;
    vals_out[i] = fv;
    if (i == 0 || (uint32_t)(s_key[i - 1] >> (32 + kSmallFvBits)) != tile) ranges[2 * (size_t)tile] = i;
    if (i + 1 == total || (uint32_t)(s_key[i + 1] >> (32 + kSmallFvBits)) != tile) ranges[2 * (size_t)tile + 1] = i + 1;
  }
}

bool small_build_fits(int64_t fv_total, int64_t tiles_total, int64_t capacity, int sh_degree) {
  return sh_degree == 0 && fv_total <= (int64_t)kSmallThreads * kSmallPer && fv_total < (1ll << kSmallFvBits) &&
         tiles_total <= (1ll << (32 - kSmallFvBits)) && capacity <= kSmallInst;
}

void launch_build_small(const void* table, const float* verts, const int32_t* faces, const float* colors,
                        const KOpts& o, float4* rec, uint4* el, WsHdr* hdr, float4* dfv_zero, uint32_t* ranges,
                        int64_t ranges_words, uint32_t* keys, uint32_t* vals, uint32_t cap, const StatsInfo& si,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_build_small, dim3(1), dim3(kSmallThreads), 0, s, table, verts, faces, colors, o, rec, el, hdr,
                     dfv_zero, ranges, ranges_words, keys, vals, cap, si);
}

void launch_project(const void* table, int64_t faces_total, const float* verts, const int32_t* faces,
                    const float* colors, const KOpts& o, float4* rec, uint4* el, uint32_t* hist, float4* dfv_zero,
                    WsHdr* hdr, uint32_t* desc0, int64_t desc0_words, uint32_t* ranges, int64_t ranges_words,
                    uint64_t* bdesc, int64_t bdesc_n, uint32_t cap, const StatsInfo& si, int max_views,
                    hipStream_t s) {
  int64_t pb = (std::max(std::max(desc0_words, ranges_words), bdesc_n) + 255) / 256;
  pb = pb < 1 ? 1 : (pb > 4096 ? 4096 : pb);
  hipLaunchKernelGGL(k_prologue, dim3((unsigned)pb), dim3(256), 0, s, hdr, hist, desc0, desc0_words, ranges,
                     ranges_words, bdesc, bdesc_n, cap, si);
  if (faces_total <= 0) return;
  // 8 lanes per face when the faces alone would leave most of the GPU idle (fewer than 256 per CU)
  if (o.sh_degree == 0 && max_views > 1 && faces_total < 256 * 256) {
    const int64_t nb = (faces_total * 8 + 1023) / 1024;
    hipLaunchKernelGGL((k_project<0, 8>), dim3((unsigned)nb), dim3(1024), 0, s, table, verts, faces, colors, o, rec, el,
                       hist, hdr, dfv_zero);
    return;
  }
  const int bs = 256;
  const int64_t nb = (faces_total + bs - 1) / bs;
#define GMR_PROJECT(D)                                                                                        \
  hipLaunchKernelGGL((k_project<D, 1>), dim3((unsigned)nb), dim3(bs), 0, s, table, verts, faces, colors, o, rec, el, \
                     hist, hdr, dfv_zero)
  switch (o.sh_degree) {
    case 1: GMR_PROJECT(1); break;
    case 2: GMR_PROJECT(2); break;
    case 3: GMR_PROJECT(3); break;
    default: GMR_PROJECT(0); break;
  }
#undef GMR_PROJECT
}

}  // namespace gmr
