// Host-side launchers of the kernels (one per stage); implemented next to their kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gmr_common.h"

namespace gmr {

// Clears the per-build counters, histograms, first depth-pass descriptors and the emission's
// block descriptors, then converts and projects every face into every view of its mesh.
void launch_project(const void* table, int64_t faces_total, const float* verts, const int32_t* faces,
                    const float* colors, const KOpts& o, float4* rec, uint4* el, uint32_t* hist, float4* dfv_zero,
                    WsHdr* hdr, uint32_t* desc0, int64_t desc0_words, uint32_t* ranges, int64_t ranges_words,
                    uint64_t* bdesc, int64_t bdesc_n, uint32_t cap, const StatsInfo& si, int max_views,
                    hipStream_t s);

// One-workgroup list build (small batches; see small_build_fits): projection, keys, sort, ranges.
bool small_build_fits(int64_t fv_total, int64_t tiles_total, int64_t capacity, int sh_degree);
void launch_build_small(const void* table, const float* verts, const int32_t* faces, const float* colors,
                        const KOpts& o, float4* rec, uint4* el, WsHdr* hdr, float4* dfv_zero, uint32_t* ranges,
                        int64_t ranges_words, uint32_t* keys, uint32_t* vals, uint32_t cap, const StatsInfo& si,
                        hipStream_t s);

// One-pass scan of tiles-touched and emission of the instances (nb blocks of kScanBlock * items
// face-views); writes the instance count and overflow flag.
void launch_bin(const void* table, const uint4* el_a, const uint4* el_b, int64_t n, int items, uint64_t* bdesc, int nb,
                WsHdr* hdr, uint32_t cap, uint2* inst, uint32_t* hist, const TilePasses& tp, uint32_t* desc0,
                uint32_t desc0_words, hipStream_t s);

void launch_sort_fv_pass(const uint4* in, uint4* out, uint32_t n, const uint32_t* hist, uint32_t* desc_cur,
                         uint32_t* desc_next, uint32_t next_words, uint32_t* ticket, int pass, const WsHdr* hdr,
                         int items, hipStream_t s);
void launch_sort_inst_pass(const uint2* in, uint2* out, uint32_t* out_k, uint32_t* out_v, const uint32_t* n_dev,
                           uint32_t cap, const uint32_t* hist, uint32_t* desc_cur, uint32_t* desc_next,
                           uint32_t next_words, uint32_t* ticket, int shift, uint32_t mask, int items, hipStream_t s);
void launch_tile_ranges(const uint32_t* sorted_keys, uint32_t tile_mask, const WsHdr* hdr, uint32_t* ranges, int blocks,
                        hipStream_t s);

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t s);
void launch_fill_f32(float* p, int64_t n, float val, hipStream_t s);
// zeroes the backward counters of hdr and dfv[0, n)
void launch_bwd_prologue(WsHdr* hdr, float* dfv, int64_t n, hipStream_t s);

// The fused-loss backward's fixed-order sum of the per-item loss slots: into hdr->loss / loss_sil
// and, when out is given, out[0..n_out).  part holds kLossReduceBlocks (a, b) partials.
struct LossRed {
  const float4* stats;
  int items;
  unsigned long long* part;
  WsHdr* hdr;
  float* out;
  int n_out;
  int nb;  // blocks taking part (set by the launchers)
};
void launch_loss_reduce(const LossRed& r, hipStream_t s);

void launch_raster_fwd(const void* table, int items, int persistent_blocks, int px, bool lane_lists, const uint32_t* ranges,
                       const uint32_t* vals, const uint32_t* keys,
                       const float4* rec, const KOpts& o, float* out_rgb, float* out_alpha, float* saved_T,
                       uint32_t* saved_n, uint32_t* blk, unsigned long long* stats, hipStream_t s);

// One step's compositing for the fused colour loss, with the silhouette term when mask is given
// (one pixel per lane, plain grid): per wavefront the forward of its block (image, alpha, saved
// state, forward statistics), then that block's adjoint (face-view sums into dfv, backward
// statistics).
void launch_raster_step(const void* table, int items, bool lane_lists, const uint32_t* ranges, const uint32_t* vals,
                        const uint32_t* keys, const float4* rec, const KOpts& o, float* out_rgb, float* out_alpha, float* saved_T,
                        uint32_t* saved_n, uint32_t* blk, unsigned long long* stats_fwd, const float* target,
                        float l2_grad_scale,
                        float l2_loss_scale, const float* mask, float sil_scale, float* dfv, float4* stats_bwd,
                        hipStream_t s);
void launch_raster_bwd(const void* table, int items, int persistent_blocks, int px, const uint32_t* ranges, const uint32_t* vals,
                       const uint32_t* keys, const float4* rec, const KOpts& o, const float* saved_T, const uint32_t* saved_n,
                       const uint32_t* blk, const float* d_rgb, const float* d_alpha, const float* rgb, const float* target, float l2_grad_scale,
                       float l2_loss_scale, const float* mask, float sil_scale, float* dfv, float4* stats,
                       hipStream_t s);

void launch_face_bwd(const void* table, int64_t faces_total, const float* verts, const int32_t* faces,
                     const float* colors, const KOpts& o, const float4* dfv, float4* fgrad, float* fsh, int max_views,
                     hipStream_t s);

// With red != NULL the gather's first blocks also perform the loss sum (one launch fewer).
void launch_vertex_gather(const int32_t* off, const int32_t* ent, const float* fgrad, const float* fsh, int sh_degree,
                          int64_t nv, float* dV, float* dC, const LossRed* red, hipStream_t s);

void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int32_t* step, hipStream_t s);
void launch_adam_tick(int32_t* step, hipStream_t s);
void launch_regularizers(const float* verts, int64_t V, const int32_t* edges, int64_t E, const int32_t* voff,
                         const int32_t* vent, float l0, float w_edge, float w_lap, float4* ge, float4* lu,
                         double* part, float* losses, float* grad, hipStream_t s);
void launch_vector_adam(float* p, const float* g, float* m, float* v, int64_t V, float lr, float b1, float b2, float eps,
                        int32_t* step, hipStream_t s);

}  // namespace gmr
