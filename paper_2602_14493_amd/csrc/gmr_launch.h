// Host-side launchers of the kernels (one per stage); implemented next to their kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gmr_common.h"

namespace gmr {

void launch_project(const void* table, int64_t faces_total, const float* verts, const int32_t* faces,
                    const float* colors, const KOpts& o, float4* rec, uint4* bin, uint32_t* cnt, float4* dfv_zero,
                    hipStream_t s);

void launch_bin(const uint32_t* cnt, const uint4* bin, int64_t n, uint32_t* bsum, uint64_t* boff, int nb, WsHdr* hdr,
                uint32_t* hist, int hist_n, uint32_t cap, uint32_t passes, uint64_t* keys, uint32_t* vals,
                hipStream_t s);

void launch_sort_hist(const uint64_t* keys0, const WsHdr* hdr, uint32_t* hist, uint32_t* dig, uint32_t* desc0,
                      int64_t parts_max, int passes, int hist_blocks, hipStream_t s);
void launch_sort_pass(uint64_t* keys0, uint32_t* vals0, uint64_t* keys1, uint32_t* vals1, WsHdr* hdr, const uint32_t* dig,
                      uint32_t* desc0, uint32_t* desc1, int64_t parts_max, int p, hipStream_t s);
void launch_tile_ranges(const uint64_t* sorted_keys, const WsHdr* hdr, uint32_t* ranges, int64_t tiles_total,
                        int blocks, hipStream_t s);

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t s);
void launch_fill_f32(float* p, int64_t n, float val, hipStream_t s);

void launch_raster_fwd(const void* table, int items, int persistent_blocks, const uint32_t* ranges, const uint32_t* vals,
                       const float4* rec, const KOpts& o, float* out_rgb, float* out_alpha, float* saved_T,
                       uint32_t* saved_n, WsHdr* hdr, hipStream_t s);

void launch_raster_bwd(const void* table, int items, int persistent_blocks, const uint32_t* ranges, const uint32_t* vals,
                       const float4* rec, const KOpts& o, const float* saved_T, const uint32_t* saved_n,
                       const float* d_rgb, const float* d_alpha, const float* rgb, const float* target, float l2_grad_scale,
                       float l2_loss_scale, float* dfv, WsHdr* hdr, hipStream_t s);

void launch_face_bwd(const void* table, int64_t faces_total, const float* verts, const int32_t* faces, const KOpts& o,
                     const float4* dfv, float4* fgrad, hipStream_t s);

void launch_vertex_gather(const int32_t* off, const int32_t* ent, const float* fgrad, int64_t nv, float* dV, float* dC,
                          hipStream_t s);

void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t* step, hipStream_t s);

}  // namespace gmr
