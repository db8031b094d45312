// The reconstruction step around the renderer (Sec. 3.1, Loss Functions and Implementation
// Details): edge-length and Laplacian-smoothing regularisers on the mesh and the VectorAdam update
// of the vertices.  (The silhouette term is fused into the rasteriser's backward.)
//
// Readings (the paper names the terms without formulas or weights):
//   edge length  w_e / E * sum over unique edges of (|v_i - v_j| - l0)^2
//   Laplacian    w_l / V * sum over vertices of |(1/deg i) sum_{j ~ i} v_j - v_i|   (uniform weights)
//   VectorAdam   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) |g|^2 (one second moment per vertex);
//                p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
//
// Gradients are formed without atomics: one kernel writes each edge's gradient vector and each
// vertex's normalised Laplacian, and a gather over the vertex -> incident-edge CSR adds them to
// the vertex gradient in a fixed order, so the result is deterministic (vertices of more than 32
// edges are summed by their wavefront in a fixed tree order).  The loss values are
// per-block partial sums reduced by one block in block order (deterministic as well).
#include "gmr_common.h"
#include "gmr_launch.h"

namespace gmr {

namespace {

__device__ inline float3 ld3(const float* p, int64_t i) { return make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }

// Block sum in a fixed order, written by thread 0 to *dst.
__device__ inline void block_sum_store(double x, double* dst) {
  __shared__ double s_w[256 / kWave];
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += s_w[i];
    *dst = t;
  }
}

// Vertices with more incident edges than this (UV-sphere poles have hundreds) are summed by their
// whole wavefront: lane l takes entries l, l + 64, ..., then a fixed-order tree sum, so no lane
// serialises a long run of dependent loads while the rest of the wavefront waits.
constexpr int32_t kCoopDegree = 32;

__device__ inline float wave_sum_f(float x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

}  // namespace

// Per edge e = (i, j): ge[e] = 2 (len - l0) / len * d * w / E with d = v_i - v_j; loss += (len - l0)^2 w / E.
__global__ __launch_bounds__(256) void k_edge_terms(const float* __restrict__ verts, const int32_t* __restrict__ edges,
                                                    int64_t E, float l0, float scale, float4* __restrict__ ge,
                                                    double* __restrict__ part) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (e < E) {
    const float3 a = ld3(verts, edges[2 * e]), b = ld3(verts, edges[2 * e + 1]);
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const float len = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    const float r = len - l0;
    const float c = len > 0.f ? 2.f * r / len * scale : 0.f;
    ge[e] = make_float4(c * dx, c * dy, c * dz, 0.f);
    l = r * r * scale;
  }
  block_sum_store((double)l, &part[blockIdx.x]);
}

// Per vertex i: lap = mean of the neighbours - v_i; lu[i] = {lap / |lap| * w / V, 1 / deg i};
// loss += |lap| w / V.  Neighbours are the other ends of the incident edges (CSR entry = edge << 1 | side).
__global__ __launch_bounds__(256) void k_lap_terms(const float* __restrict__ verts, const int32_t* __restrict__ edges,
                                                   const int32_t* __restrict__ voff, const int32_t* __restrict__ vent,
                                                   int64_t V, float scale, float4* __restrict__ lu,
                                                   double* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  int32_t b = 0, n = 0;
  if (i < V) {
    b = voff[i];
    n = voff[i + 1] - b;
  }
  const bool coop = n > kCoopDegree;
  float sx = 0.f, sy = 0.f, sz = 0.f;
  if (i < V && !coop) {
    for (int32_t k = 0; k < n; ++k) {
      const int32_t t = vent[b + k];
      const float3 q = ld3(verts, edges[2 * (t >> 1) + (1 - (t & 1))]);
      sx += q.x; sy += q.y; sz += q.z;
    }
  }
  for (uint64_t m = __ballot(coop); m; m &= m - 1) {  // high-degree vertices of this wavefront
    const int o = __builtin_ctzll(m);
    const int32_t bb = __shfl(b, o, kWave), nn = __shfl(n, o, kWave);
    float px = 0.f, py = 0.f, pz = 0.f;
    for (int32_t k = lane; k < nn; k += kWave) {
      const int32_t t = vent[bb + k];
      const float3 q = ld3(verts, edges[2 * (t >> 1) + (1 - (t & 1))]);
      px += q.x; py += q.y; pz += q.z;
    }
    px = wave_sum_f(px); py = wave_sum_f(py); pz = wave_sum_f(pz);
    if (lane == o) { sx = px; sy = py; sz = pz; }
  }
  float l = 0.f;
  if (i < V) {
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (n > 0) {
      const float inv = 1.f / (float)n;
      const float3 v = ld3(verts, i);
      const float lx = fmaf(sx, inv, -v.x), ly = fmaf(sy, inv, -v.y), lz = fmaf(sz, inv, -v.z);
      const float nrm = sqrtf(fmaf(lx, lx, fmaf(ly, ly, lz * lz)));
      const float c = nrm > 0.f ? scale / nrm : 0.f;
      out = make_float4(c * lx, c * ly, c * lz, inv);
      l = nrm * scale;
    }
    lu[i] = out;
  }
  block_sum_store((double)l, &part[blockIdx.x]);
}

// losses[0] = sum of the edge blocks' partials, losses[1] = that of the Laplacian blocks (block
// order; a term that was skipped reads as 0).  One block.
__global__ __launch_bounds__(256) void k_reg_losses(const double* __restrict__ part_e, int ne,
                                                    const double* __restrict__ part_l, int nl,
                                                    float* __restrict__ losses) {
  __shared__ double s_w[2][256 / kWave];
  for (int t = 0; t < 2; ++t) {
    const double* p = t ? part_l : part_e;
    const int n = t ? nl : ne;
    double x = 0.0;
    for (int i = (int)threadIdx.x; i < n; i += 256) x += p[i];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s_w[t][threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double x = 0.0;
    for (int i = 0; i < 256 / kWave; ++i) x += s_w[threadIdx.x][i];
    losses[threadIdx.x] = (float)x;
  }
}

// Per vertex k: grad[k] += sum over incident edges of (+/-) ge + sum over neighbours i of lu_i / deg i - lu_k.
__global__ __launch_bounds__(256) void k_reg_gather(const int32_t* __restrict__ edges, const int32_t* __restrict__ voff,
                                                    const int32_t* __restrict__ vent, int64_t V,
                                                    const float4* __restrict__ ge, const float4* __restrict__ lu,
                                                    float* __restrict__ grad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  int32_t b = 0, n = 0;
  if (k < V) {
    b = voff[k];
    n = voff[k + 1] - b;
  }
  // incident-edge terms of entries j0, j0 + step, ... < n of the CSR row at b
  auto add_row = [&](int32_t bb, int32_t j0, int32_t nn, int32_t step, float& gx, float& gy, float& gz) {
    for (int32_t j = j0; j < nn; j += step) {
      const int32_t t = vent[bb + j];
      const int32_t e = t >> 1;
      if (ge) {
        const float4 g = ge[e];
        const float sg = (t & 1) ? -1.f : 1.f;  // side 0 = first end of the edge
        gx = fmaf(sg, g.x, gx); gy = fmaf(sg, g.y, gy); gz = fmaf(sg, g.z, gz);
      }
      if (lu) {
        const float4 q = lu[edges[2 * e + (1 - (t & 1))]];
        gx = fmaf(q.x, q.w, gx); gy = fmaf(q.y, q.w, gy); gz = fmaf(q.z, q.w, gz);
      }
    }
  };
  const bool coop = n > kCoopDegree;
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if (k < V) {
    const float4 own = lu ? lu[k] : make_float4(0.f, 0.f, 0.f, 0.f);
    gx = -own.x; gy = -own.y; gz = -own.z;
    if (!coop) add_row(b, 0, n, 1, gx, gy, gz);
  }
  for (uint64_t m = __ballot(coop); m; m &= m - 1) {  // high-degree vertices of this wavefront
    const int o = __builtin_ctzll(m);
    const int32_t bb = __shfl(b, o, kWave), nn = __shfl(n, o, kWave);
    float px = 0.f, py = 0.f, pz = 0.f;
    add_row(bb, lane, nn, kWave, px, py, pz);
    px = wave_sum_f(px); py = wave_sum_f(py); pz = wave_sum_f(pz);
    if (lane == o) { gx += px; gy += py; gz += pz; }
  }
  if (k < V) {
    grad[3 * k] += gx;
    grad[3 * k + 1] += gy;
    grad[3 * k + 2] += gz;
  }
}

// VectorAdam on V 3-vectors; t = *step + 1 (advanced by k_adam_tick after the update).
__global__ __launch_bounds__(256) void k_vector_adam(float* __restrict__ p, const float* __restrict__ g,
                                                     float* __restrict__ m, float* __restrict__ v, int64_t V, float lr,
                                                     float b1, float b2, float eps, const int32_t* __restrict__ step) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const float t = (float)(*step + 1);
  const float gx = g[3 * i], gy = g[3 * i + 1], gz = g[3 * i + 2];
  const float mx = fmaf(b1, m[3 * i], (1.f - b1) * gx);
  const float my = fmaf(b1, m[3 * i + 1], (1.f - b1) * gy);
  const float mz = fmaf(b1, m[3 * i + 2], (1.f - b1) * gz);
  const float vv = fmaf(b2, v[i], (1.f - b2) * fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
  m[3 * i] = mx; m[3 * i + 1] = my; m[3 * i + 2] = mz;
  v[i] = vv;
  const float c1 = 1.f / (1.f - powf(b1, t)), c2 = 1.f / (1.f - powf(b2, t));
  const float den = sqrtf(vv * c2) + eps;
  const float s = lr * c1 / den;
  p[3 * i] -= s * mx;
  p[3 * i + 1] -= s * my;
  p[3 * i + 2] -= s * mz;
}

void launch_regularizers(const float* verts, int64_t V, const int32_t* edges, int64_t E, const int32_t* voff,
                         const int32_t* vent, float l0, float w_edge, float w_lap, float4* ge, float4* lu,
                         double* part, float* losses, float* grad, hipStream_t s) {
  const bool do_e = w_edge != 0.f && E > 0, do_l = w_lap != 0.f && V > 0;
  const int be = do_e ? (int)((E + 255) / 256) : 0, bl = do_l ? (int)((V + 255) / 256) : 0;
  if (do_e)
    hipLaunchKernelGGL(k_edge_terms, dim3((unsigned)be), dim3(256), 0, s, verts, edges, E, l0, w_edge / (float)E, ge,
                       part);
  if (do_l)
    hipLaunchKernelGGL(k_lap_terms, dim3((unsigned)bl), dim3(256), 0, s, verts, edges, voff, vent, V,
                       w_lap / (float)V, lu, part + be);
  hipLaunchKernelGGL(k_reg_losses, dim3(1), dim3(256), 0, s, part, be, part + be, bl, losses);
  if ((do_e || do_l) && V > 0)
    hipLaunchKernelGGL(k_reg_gather, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, edges, voff, vent, V,
                       do_e ? ge : nullptr, do_l ? lu : nullptr, grad);
}

void launch_vector_adam(float* p, const float* g, float* m, float* v, int64_t V, float lr, float b1, float b2, float eps,
                        int32_t* step, hipStream_t s) {
  if (V > 0)
    hipLaunchKernelGGL(k_vector_adam, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, p, g, m, v, V, lr, b1, b2,
                       eps, step);
  launch_adam_tick(step, s);
}

}  // namespace gmr
