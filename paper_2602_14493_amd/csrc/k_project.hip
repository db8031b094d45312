// Conversion (Sec. 2.2) fused with the EWA projection (Sec. 2.1), one thread per face.
//
// A face is converted once, in double precision, and projected into every view of its mesh.  Per
// face-view it writes, view-major (coalesced across consecutive faces):
//   rec[fv]  3 x float4 = 48 B  {u_hi, v_hi, u_lo, v_lo}  mean as float pairs (u = u_hi + u_lo)
//                              {k l11, k l12, k l22, x-rect}  scaled Cholesky factor of the conic
//                              {r, g, b, y-rect}              Eq. 16 colour; rects pack lo | hi << 16
//   el[fv]   uint4 = 16 B      {float32 depth bits, fv, first tile, nx | ny << 16}: the element the
//                              depth passes of the radix sort move (culled: nx = ny = 0)
// and adds each element's four 8-bit depth digits to the sort's histograms (LDS, then one global
// atomic per bin and workgroup), and the range of the visible keys' high 16 bits to the workspace
// header (per-thread, then one atomic pair per wavefront).
// The mean stays in double until it is split into two floats: a float32 pixel coordinate near
// x = 1920 carries ~1e-4 px of rounding, which alone would move alpha by ~1e-4.
#include "gmr_common.h"
#include "gmr_launch.h"
#include "gmr_sh.h"

namespace gmr {

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
        e = make_uint4(f2u((float)q.p[2]), (uint32_t)fv, (uint32_t)(V.tile_base + ty0 * V.tiles_x + tx0),
                       (uint32_t)nx | ((uint32_t)ny << 16));
        kmin = min(kmin, e.x >> 16);
        kmax = max(kmax, e.x >> 16);
      }
    }
    el[fv] = e;
#pragma unroll
    for (int p = 0; p < kDepthPasses; ++p) atomicAdd(&s_h[p * 256 + ((e.x >> (8 * p)) & 255u)], 1u);
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
    hdr->bwd_stats = 0u;
    hdr->stats_fwd_off = si.fwd_off;
    hdr->stats_bwd_off = si.bwd_off;
    hdr->red_ticket = 0u;
    for (int c = 0; c < kKeyCopies; ++c) {
      hdr->key_hi_min[c] = 0xffffffffu;
      hdr->key_hi_max[c] = 0u;
    }
  }
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
