/* gmr.h -- C ABI of the MI355X (gfx950) Gaussian Mesh Renderer hot path (libgmr.so).
 *
 * The renderer turns every triangle of a mesh into one planar 3D Gaussian (Liu & Okura,
 * "Gaussian Mesh Renderer for Lightweight Differentiable Rendering", Sec. 2.2: local facet frame,
 * closed-form second moments Eq. 6-9, area-matched covariance Eq. 12-13 or the embedded form
 * Eq. 15, opacity 1 and the vertex-average colour Eq. 16), splats it with the 3DGS rasteriser the
 * paper adopts (Sec. 2.1: EWA projection, tile binning on a (tile | depth) key, front-to-back
 * alpha compositing) and back-propagates image gradients to vertex positions and colours.
 *
 * Conventions shared by every entry point
 *  - Pointers named *_dev are DEVICE pointers owned by the caller; pointers named *_host are host
 *    pointers owned by the caller.  No entry point keeps a pointer after it returns.
 *  - No entry point allocates or frees device memory, or synchronises the stream, except
 *    gmr_read_counters (which synchronises) -- so fwd/bwd/adam may be captured in a hipGraph.
 *  - Work is enqueued on `stream`.  Argument errors are detected on the host BEFORE anything is
 *    enqueued and return a status; nothing is thrown across the ABI.  gmr_last_error() returns a
 *    thread-local description of the last failure.
 *  - Indices are int32 (vertices, faces, face-views and pixels of one batch < 2^31; instances
 *    < 2^30).  Image sides are <= 32767.
 *  - Colours are linear RGB floats; images are float32 [pixels][3], pixels of all views back to
 *    back, each view row-major.  Pixel (i, j) has its centre at (i + 0.5, j + 0.5).
 *  - Cameras are pinholes with OpenCV axes (+x right, +y down, +z forward): p = R x + t,
 *    u = fx p.x / p.z + cx, v = fy p.y / p.z + cy.
 */
#ifndef GMR_H
#define GMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gmr_status {
  GMR_OK = 0,
  GMR_ERR_INVALID_ARG = 1,   /* a size, pointer or option is out of range                       */
  GMR_ERR_WORKSPACE = 2,     /* the workspace / saved buffer is smaller than required            */
  GMR_ERR_CAPACITY = 3,      /* instance count exceeded the workspace's capacity (see counters)  */
  GMR_ERR_UNSUPPORTED = 4,   /* valid request the library does not support                       */
  GMR_ERR_HIP = 5            /* a HIP runtime call failed                                        */
} gmr_status;

/* Pinhole camera (world -> camera p = R x + t, R row-major).  near_plane/far_plane cull
 * Gaussians whose centre depth p.z is outside (near_plane, far_plane). */
typedef struct gmr_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float near_plane, far_plane;
} gmr_camera;

/* Renderer options.  gmr_default_options() fills the defaults given in brackets. */
typedef struct gmr_options {
  int32_t cov_mode;          /* [0] 0: area-matched covariance (Eq. 13); 1: embedded Sigma2D (Eq. 15);
                                2: the "3DGS-based" baseline of Sec. 3.1 (Baselines): frame from the
                                normal and the first edge, diagonal scales kappa Sigma2D_xx, _yy, s_z */
  float dilation;            /* [0.3] screen-space low-pass added to the 2D covariance, px^2      */
  float alpha_min;           /* [1/255] Gaussians with alpha below it are skipped at a pixel       */
  float alpha_max;           /* [0.99] alpha clamp (keeps 1 - alpha >= 0.01)                      */
  float t_eps;               /* [1e-4] compositing stops before transmittance would fall below it */
  float bg[3];               /* [0,0,0] background colour                                         */
  int32_t tile_w, tile_h;    /* [16,16] binning tile in pixels: multiples of 8 in [8, 64]          */
  int32_t raster_mode;       /* [0] 0: one workgroup per 4 work items; 1: persistent grid (4
                                workgroups per CU striding over the work items)                    */
  int32_t px_per_lane;       /* [1] pixels per lane in the rasteriser: 1, 2 or 4 (a wavefront then
                                covers an 8 x 8*px_per_lane block); tile_h % (8*px_per_lane) == 0   */
  int32_t lane_lists;        /* [1] 1: the forward compositing walks per-lane lists -- each lane visits
                                only the Gaussians whose pixel rectangle holds its pixel (lists
                                built per staged batch with a 64 x 64 bit transpose) -- instead of
                                every Gaussian meeting its block.  Images and saved states are
                                bit-identical either way; the backward is unaffected.              */
  int32_t sh_degree;         /* [0] view-dependent colour, the extension named with Sec. 2.2's colour
                                assignment: 0 = one colour per vertex (Eq. 16); 1..3 = colors_dev
                                holds K = (sh_degree+1)^2 coefficients per channel, [V][K][3]
                                (coefficient 0 is the colour itself), a face takes their mean and its
                                colour in a view is max(0, c_0 + sum_k c_k Y_k(d)), d the unit
                                direction from the camera centre to the face's mean, Y_k the real
                                spherical harmonics (3DGS sign convention); d_colors_dev has the
                                same layout                                                          */
  int32_t composited_lists;  /* [2046] per 8 x 8 raster block, how many list positions of the Gaussians
                                some pixel of the block composited the forward records in the saved
                                state (0 to 8190): the backward then visits only those, and a block
                                with more (or in a tile whose list exceeds 65536 entries) walks its
                                tile's whole list.  The saved state takes 4 (1 + ceil(
                                composited_lists / 2)) bytes per block beyond its 8 bytes per pixel
                                (4 KB at the default); 0 records none.  Results are the same for
                                every value.                                                       */
  int64_t instance_capacity; /* [0] (Gaussian, tile) instances the workspace holds; must be > 0
                                when sizing a workspace or rendering                               */
} gmr_options;

/* A batch: M meshes stored back to back (face indices are GLOBAL into the flat vertex array and
 * the faces of mesh m reference only its vertices), and NV views, each bound to one mesh.
 * All arrays are HOST arrays.  Global Gaussian id of face f of the flat face array is f. */
typedef struct gmr_batch {
  int32_t num_meshes;
  int32_t num_views;
  const int64_t* vert_offsets_host;  /* [num_meshes + 1], vert_offsets[0] = 0                  */
  const int64_t* face_offsets_host;  /* [num_meshes + 1], face_offsets[0] = 0                  */
  const int32_t* view_mesh_host;     /* [num_views] mesh of each view                          */
  const gmr_camera* cams_host;       /* [num_views]                                            */
} gmr_batch;

/* Counters the device keeps in the workspace (read back with gmr_read_counters). */
typedef struct gmr_counters {
  int64_t instances;   /* (Gaussian, tile) instances the last pass generated                  */
  int64_t capacity;    /* capacity of the workspace                                           */
  int32_t overflow;    /* 1 if instances > capacity (outputs of that pass are incomplete)    */
  int32_t overflow_any;/* 1 if any list build since the previous read overflowed             */
  int64_t pairs_fwd;   /* (pixel, Gaussian) pairs the last forward evaluated: pixel inside the
                          Gaussian's 3-sigma rectangle and (with a margin) its 1/255 ellipse,
                          up to the pixel's transmittance stop                                */
  int64_t pairs_bwd;   /* pairs the last backward differentiated (composited ones)           */
  float loss;          /* colour loss of the last fused backward (L2 or reconstruction)       */
  float loss_sil;      /* silhouette loss of the last gmr_render_bwd_recon (0 otherwise)      */
  int64_t peak_instances; /* largest instance count of any list build since the previous read
                             (e.g. over the replays of a captured optimisation loop)          */
} gmr_counters;

typedef struct gmr_ctx* gmr_handle;

/* ---------------------------------------------------------------------------------------------
 * Library / context
 * ------------------------------------------------------------------------------------------- */

/* Returns the default options (Sec. 2.2 constants are compiled in; see gmr_options). */
gmr_options gmr_default_options(void);

/* Creates a context bound to HIP device `device` (queries its CU count for persistent launches).
 * Errors: GMR_ERR_INVALID_ARG (null out / bad device), GMR_ERR_HIP. */
gmr_status gmr_create(gmr_handle* out, int device);
gmr_status gmr_destroy(gmr_handle h);

const char* gmr_status_string(gmr_status s);
const char* gmr_last_error(void);

/* ---------------------------------------------------------------------------------------------
 * Sizing.  All pure host functions.
 * ------------------------------------------------------------------------------------------- */

/* Bytes of the device view table for this batch + options (see gmr_view_table_fill). */
gmr_status gmr_view_table_size(const gmr_batch* batch, const gmr_options* opt, size_t* bytes);

/* Writes the view table (per-view camera, offsets, tile grid; per-mesh face ranges and view
 * lists) into a HOST buffer; the caller copies it to device memory and passes that device copy as
 * `table_dev` to the render calls, together with the SAME batch and options.  The table is
 * immutable across calls, so a captured graph may keep using it. */
gmr_status gmr_view_table_fill(const gmr_batch* batch, const gmr_options* opt, void* host_dst, size_t bytes);

/* Workspace bytes for one forward+backward of this batch at opt->instance_capacity.  The
 * workspace holds the per face-view projected records, the instance keys/values (double
 * buffered), the sort state, the tile ranges and the backward's gradient accumulators.
 * `saved_bytes` is the state render_fwd leaves for render_bwd: 8 bytes per pixel, then
 * 4 (1 + ceil(opt->composited_lists / 2)) bytes per 8 x 8 raster block when composited_lists > 0
 * (the block's composited list, below).
 * The workspace needs no initialisation, except that zeroing its first 256 bytes once after
 * allocation arms the peak instance counter gmr_read_counters reports. */
gmr_status gmr_workspace_size(const gmr_batch* batch, const gmr_options* opt, size_t* ws_bytes, size_t* saved_bytes);

/* CSR of (vertex -> face*3 + corner), entries ascending per vertex: the deterministic gather the
 * backward uses to sum per-corner gradients into vertices.  Host-side; build once per topology.
 * faces_host [num_faces][3] global indices; off_host [num_verts + 1]; ent_host [3 num_faces].
 * Errors: GMR_ERR_INVALID_ARG for an index outside [0, num_verts). */
gmr_status gmr_build_adjacency(const int32_t* faces_host, int64_t num_faces, int64_t num_verts,
                               int32_t* off_host, int32_t* ent_host);

/* ---------------------------------------------------------------------------------------------
 * Forward / backward
 * ------------------------------------------------------------------------------------------- */

/* Forward pass of every view of the batch: per-face conversion (Sec. 2.2) fused with EWA
 * projection per view, instance emission, (tile | depth) radix sort, tile ranges, and per-tile
 * front-to-back compositing.
 *   verts_dev  [V][3] f32, faces_dev [F][3] i32 (global), colors_dev [V][3] f32 ([V][K][3] with sh_degree)
 *   out_rgb_dev   [P][3] f32  composite + T_final * bg
 *   out_alpha_dev [P]    f32  1 - T_final (may be NULL)
 *   saved_dev     saved_bytes: per pixel T_final and the list position after the last
 *                 composited Gaussian; per raster block a uint32 count of the tile-list entries
 *                 some pixel of the block composited, then their positions in the tile's list as
 *                 uint16, ascending (the first opt->composited_lists; a larger count, or
 *                 0xffffffff for a tile list too long for 16-bit positions, makes the backward
 *                 walk the block's whole list) -- input of
 *                 gmr_render_bwd
 *   ws_dev/ws_bytes  workspace of gmr_workspace_size; after the call it holds the sorted
 *                 lists, which gmr_render_bwd may reuse (recompute_lists = 0).
 * If the instance count exceeds the capacity, writes are clamped, the overflow counter is set and
 * the image is incomplete; the call still returns GMR_OK (the count is only known on the device):
 * check gmr_read_counters and re-run with a larger capacity. */
gmr_status gmr_render_fwd(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table_dev,
                          const float* verts_dev, const int32_t* faces_dev, const float* colors_dev,
                          float* out_rgb_dev, float* out_alpha_dev, void* saved_dev,
                          void* ws_dev, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gmr_render_fwd with the workspace taken from a static
 * device array of GMR_NOALLOC_WORKSPACE_BYTES that the library holds on every GPU it runs on until
 * the process ends.  The call allocates and frees nothing, synchronises nothing and is capturable.
 * Arguments as gmr_render_fwd, without ws_dev / ws_bytes, plus
 *   counters_dev  [2] uint32 (may be NULL): {instance count, overflow flag} of this call's list
 *                 build, copied on the stream (gmr_read_counters cannot see the static workspace).
 * Errors (returned before anything is enqueued): GMR_ERR_WORKSPACE when the batch's workspace
 * (gmr_workspace_size for these options) exceeds GMR_NOALLOC_WORKSPACE_BYTES -- lower
 * instance_capacity or use gmr_render_fwd; the other errors of gmr_render_fwd.
 * Every call on one GPU shares that GPU's array, which keeps the last call's contents (each call
 * clears what it needs): calls that overlap on one GPU (several streams or threads) race, and the
 * lists a call leaves there cannot be handed to gmr_render_bwd -- its backward rebuilds them
 * (recompute_lists = 1) in a caller workspace. */
#define GMR_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
gmr_status gmr_render_fwd_noalloc(gmr_handle h, const gmr_batch* batch, const gmr_options* opt,
                                  const void* table_dev, const float* verts_dev, const int32_t* faces_dev,
                                  const float* colors_dev, float* out_rgb_dev, float* out_alpha_dev,
                                  void* saved_dev, uint32_t* counters_dev, void* stream);

/* Backward pass: reverse-order adjoint of the compositing per pixel, chained through the EWA
 * projection and the conversion to vertex positions and colours.
 *   d_rgb_dev   [P][3] f32  dL/d rgb;  d_alpha_dev [P] f32 dL/d alpha (may be NULL)
 *   saved_dev   as written by gmr_render_fwd for the same inputs
 *   adj_off_dev [V + 1], adj_ent_dev [3F]  from gmr_build_adjacency (device copies)
 *   recompute_lists  0: ws_dev still holds the forward's lists (same inputs, untouched);
 *                    1: rebuild them (bit-identical to the forward's) inside ws_dev.
 *   d_verts_dev [V][3], d_colors_dev (colors_dev's layout)  OVERWRITTEN with the gradients.
 * Culled faces (degenerate, behind the camera, off-screen) receive zero gradient. */
gmr_status gmr_render_bwd(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table_dev,
                          const float* verts_dev, const int32_t* faces_dev, const float* colors_dev,
                          const float* d_rgb_dev, const float* d_alpha_dev, const void* saved_dev,
                          const int32_t* adj_off_dev, const int32_t* adj_ent_dev, int32_t recompute_lists,
                          float* d_verts_dev, float* d_colors_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Same as gmr_render_bwd for the colour loss of Sec. 3.1 (mean squared error over every channel
 * of every pixel of every view, times loss_weight): dL/d rgb = loss_weight * 2 (rgb - target) / (3P)
 * is formed inside the backward kernel from out_rgb_dev (the forward's output) and target_dev.
 * If loss_dev is not NULL, the loss value (f32) is written there. */
gmr_status gmr_render_bwd_l2(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table_dev,
                             const float* verts_dev, const int32_t* faces_dev, const float* colors_dev,
                             const float* rgb_dev, const float* target_dev, float loss_weight,
                             const void* saved_dev, const int32_t* adj_off_dev, const int32_t* adj_ent_dev,
                             int32_t recompute_lists, float* d_verts_dev, float* d_colors_dev, float* loss_dev,
                             void* ws_dev, size_t ws_bytes, void* stream);

/* One training step's rendering for the colour loss of Sec. 3.1, fused: gmr_render_fwd followed by
 * gmr_render_bwd_l2 with one list build instead of the forward's and the backward's (the sorted
 * lists live only inside this call, as with recompute_lists = 1, so nothing is saved for a later
 * backward).  The compositing of Sec. 2.1 and its reverse-order adjoint run in one launch: each
 * 8 x 8 pixel block composites its pixels and then differentiates them, since a pixel's L2
 * upstream gradient needs only its own colour (px_per_lane 1 and the plain grid schedule; other
 * options run the two compositing launches in turn after the one build).
 * Writes out_rgb_dev, out_alpha_dev (may be NULL) and saved_dev as gmr_render_fwd does (bit for
 * bit), and d_verts_dev, d_colors_dev and loss_dev (may be NULL) as gmr_render_bwd_l2 does (equal up
 * to the order of the float atomics that sum each face-view's gradient).  Errors as those calls. */
gmr_status gmr_render_step_l2(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table_dev,
                              const float* verts_dev, const int32_t* faces_dev, const float* colors_dev,
                              const float* target_dev, float loss_weight, float* out_rgb_dev, float* out_alpha_dev,
                              void* saved_dev, const int32_t* adj_off_dev, const int32_t* adj_ent_dev,
                              float* d_verts_dev, float* d_colors_dev, float* loss_dev, void* ws_dev,
                              size_t ws_bytes, void* stream);

/* The reconstruction objective's image terms (Sec. 3.1, Loss Functions): gmr_render_bwd_l2's colour
 * loss (weight color_weight) plus the silhouette loss, color_weight * MSE(rgb, target) +
 * sil_weight * mean over every pixel of every view of -(s log a + (1 - s) log(1 - a)), with
 * a = 1 - T_final clamped to [1e-6, 1 - 1e-6] (the clamp is part of the loss: zero derivative
 * where it is active) and s = mask_dev [P] f32 (a binary silhouette; any value in [0, 1] is
 * accepted).  dL/d alpha is formed inside the backward kernel from the saved T_final.
 * losses_dev (may be NULL) receives two f32: the colour loss and the silhouette loss, each with
 * its weight applied.  Other arguments and errors as gmr_render_bwd_l2; rgb_dev, target_dev and
 * mask_dev must not be NULL. */
gmr_status gmr_render_bwd_recon(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table_dev,
                                const float* verts_dev, const int32_t* faces_dev, const float* colors_dev,
                                const float* rgb_dev, const float* target_dev, float color_weight,
                                const float* mask_dev, float sil_weight, const void* saved_dev,
                                const int32_t* adj_off_dev, const int32_t* adj_ent_dev, int32_t recompute_lists,
                                float* d_verts_dev, float* d_colors_dev, float* losses_dev, void* ws_dev,
                                size_t ws_bytes, void* stream);

/* gmr_render_step_l2 for the reconstruction objective's image terms: gmr_render_fwd followed by
 * gmr_render_bwd_recon (colour loss with weight color_weight plus the silhouette loss against
 * mask_dev with weight sil_weight, Sec. 3.1) from one list build, the compositing and its adjoint in
 * one launch.  losses_dev (may be NULL) receives the two weighted losses.  Outputs and errors as
 * gmr_render_step_l2; mask_dev must not be NULL. */
gmr_status gmr_render_step_recon(gmr_handle h, const gmr_batch* batch, const gmr_options* opt, const void* table_dev,
                                 const float* verts_dev, const int32_t* faces_dev, const float* colors_dev,
                                 const float* target_dev, float color_weight, const float* mask_dev, float sil_weight,
                                 float* out_rgb_dev, float* out_alpha_dev, void* saved_dev,
                                 const int32_t* adj_off_dev, const int32_t* adj_ent_dev, float* d_verts_dev,
                                 float* d_colors_dev, float* losses_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Where the forward's tile lists live inside a workspace laid out for (batch, opt): byte offsets
 * of the tile ranges (uint32 [tiles][2] = start, end into the sorted instances), the sorted
 * instance values (uint32 [instance_capacity] face-view indices, sorted by (tile, float32 depth,
 * face-view)), the projected records (float32 [face-views][12]) and the sorted instance keys
 * (uint32 [instance_capacity]: the global tile id in the low b bits, b = ceil(log2(total tiles));
 * when b <= 26 and the tile's (tile_w / 8) * (tile_h / (8 px_per_lane)) raster blocks fit in the
 * 32 - b bits above, those bits hold the mask of the blocks that the instance's pixel rectangle
 * meets, block (sx, sy) of 8 x (8 px_per_lane) pixels at bit b + sy * (tile_w / 8) + sx).  Tiles of view v are numbered from the sum of the
 * earlier views' tile counts, row-major.  Face-views of view v are numbered from the sum of the
 * earlier views' face counts, in face order.  Pure host arithmetic; the contents are valid after
 * gmr_render_fwd (or a recomputing gmr_render_bwd). */
gmr_status gmr_workspace_view(const gmr_batch* batch, const gmr_options* opt, size_t* ranges_off, size_t* vals_off,
                              size_t* rec_off, size_t* keys_off);

/* Reads the workspace's device counters (synchronises `stream`).  Not capturable.
 * peak_instances / overflow_any cover every list build since the previous read (the read restarts
 * them); they are meaningful from the first read on only if the caller zeroed the workspace's
 * first 256 bytes after allocating it (the other counters need no initialisation). */
gmr_status gmr_read_counters(const void* ws_dev, size_t ws_bytes, gmr_counters* out_host, void* stream);

/* ---------------------------------------------------------------------------------------------
 * Stage timing (tracing).  While enabled, every stage of gmr_render_fwd / gmr_render_bwd* on this
 * handle is bracketed by a HIP event pair on the call's stream.  For eager calls only: do not
 * enable it around graph capture.
 * ------------------------------------------------------------------------------------------- */

/* Turns stage timing on (enable = 1) or off and discards what was recorded. */
gmr_status gmr_profile_enable(gmr_handle h, int32_t enable);

/* Waits for the recorded events and returns, per stage, its name (names: max_stages x 32 chars),
 * the summed milliseconds and the number of timed launch groups; then discards the records.
 * Stages: project, scan_emit, sort_fv_pass (the depth passes over face-views), sort_pass (the
 * instance passes), tile_ranges, raster_fwd, fill, raster_bwd, face_bwd, vertex_gather (with the
 * fused-loss backwards' fixed-order loss sum), build_small (the one-launch list build of small
 * batches, in place of the first five), raster_step (gmr_render_step_l2's compositing and adjoint in
 * one launch).  max_stages must be >= 12. */
gmr_status gmr_profile_read(gmr_handle h, int32_t max_stages, char* names, float* ms_total, int32_t* launches,
                            int32_t* n_stages);

/* ---------------------------------------------------------------------------------------------
 * Optimiser step (the configuration's Adam on vertex positions)
 * ------------------------------------------------------------------------------------------- */

/* One Adam step on n floats: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), with t = ++(*step_dev) read and
 * incremented on the device (so a captured graph advances it on every replay).
 * step_dev: one int32 on the device, 0 before the first step. */
gmr_status gmr_adam_step(float* param_dev, const float* grad_dev, float* m_dev, float* v_dev, int64_t n,
                         float lr, float beta1, float beta2, float eps, int32_t* step_dev, void* stream);

/* ---------------------------------------------------------------------------------------------
 * Mesh regularisers and VectorAdam (Sec. 3.1, Implementation Details and Loss Functions): the
 * rest of the reconstruction step around the renderer.  The paper names the edge-length and
 * Laplacian-smoothing terms without formulas; the forms used are
 *   edge     edge_weight / E * sum over unique edges (i, j) of (|v_i - v_j| - target_length)^2
 *   Laplacian lap_weight / V * sum over vertices of |(1/deg i) sum over neighbours j of v_j - v_i|
 * (uniform weights; neighbours share an edge; an isolated vertex contributes 0).
 * ------------------------------------------------------------------------------------------- */

/* Number of unique undirected edges of a triangle list (host).  faces_host [num_faces][3] global
 * indices.  Errors: GMR_ERR_INVALID_ARG for an index outside [0, num_verts). */
gmr_status gmr_mesh_graph_size(const int32_t* faces_host, int64_t num_faces, int64_t num_verts, int64_t* num_edges);

/* Edge list and vertex -> incident-edge CSR (host): edges_host [num_edges][2] = (i, j), i < j,
 * sorted lexicographically (degenerate face corners i == j are skipped); vedge_off_host
 * [num_verts + 1]; vedge_ent_host [2 num_edges], entry = edge << 1 | side (side 0: the vertex is
 * the edge's first end), ascending per vertex.  num_edges must be gmr_mesh_graph_size's value.
 * Build once per topology and copy to the device for gmr_regularizers. */
gmr_status gmr_build_mesh_graph(const int32_t* faces_host, int64_t num_faces, int64_t num_verts, int64_t num_edges,
                                int32_t* edges_host, int32_t* vedge_off_host, int32_t* vedge_ent_host);

/* Device scratch bytes gmr_regularizers needs (16 B per edge and per vertex, plus 8 B per 256 of
 * each for the loss partials). */
gmr_status gmr_regularizers_scratch_size(int64_t num_verts, int64_t num_edges, size_t* bytes);

/* Adds the gradients of the two regularisers to d_verts_dev [V][3] (accumulates: call it after the
 * render backward has written its gradient) and writes their values, weights applied, to
 * losses_dev [2] f32 (edge, Laplacian).  Deterministic (no atomics; fixed summation order).  A weight
 * of 0 skips its term.  Stream-ordered and capturable (no allocation, no memset node). */
gmr_status gmr_regularizers(const float* verts_dev, int64_t num_verts, const int32_t* edges_dev, int64_t num_edges,
                            const int32_t* vedge_off_dev, const int32_t* vedge_ent_dev, float target_length,
                            float edge_weight, float lap_weight, void* scratch_dev, size_t scratch_bytes,
                            float* losses_dev, float* d_verts_dev, void* stream);

/* One VectorAdam step on num_verts 3-vectors (one second moment per vertex, on the squared norm
 * of its gradient, so a rotation of the gradients rotates the update):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) |g|^2;  p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * with t = ++(*step_dev) as in gmr_adam_step.  param/grad/m [V][3] f32, v [V] f32. */
gmr_status gmr_vector_adam_step(float* param_dev, const float* grad_dev, float* m_dev, float* v_dev,
                                int64_t num_verts, float lr, float beta1, float beta2, float eps, int32_t* step_dev,
                                void* stream);

/* ---------------------------------------------------------------------------------------------
 * Autotuning (tile shape and raster mode).  Allocates its own scratch and synchronises: call it
 * outside graph capture.
 * ------------------------------------------------------------------------------------------- */

/* Times forward + L2 backward for each candidate tile shape, block shape, raster mode and forward
 * list walk on the given inputs (iters timed steps each, after one warm-up step), times the three
 * fastest once more and writes the options with the best of their two timings to best_out
 * (instance_capacity set with 25% headroom over the measured count).  recompute = 1 times the
 * backward with the tile lists rebuilt (as gmr_render_bwd_l2 with recompute = 1 runs it: the list
 * building then counts twice per step); 0 reuses the forward's lists.  Results are cached in the
 * handle per (image sizes, face count, views, cov_mode, sh_degree, recompute); a cached entry is
 * returned without timing.  ms_out (may be NULL) receives the best time per forward+backward.
 * Returns GMR_ERR_INVALID_ARG for a NULL pointer, iters < 1 or recompute not 0 / 1. */
gmr_status gmr_autotune(gmr_handle h, const gmr_batch* batch, const gmr_options* base,
                        const float* verts_dev, const int32_t* faces_dev, const float* colors_dev,
                        const float* target_dev, const int32_t* adj_off_dev, const int32_t* adj_ent_dev,
                        int32_t iters, int32_t recompute, gmr_options* best_out, float* ms_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GMR_H */
