/*
 * trips.h -- C ABI of the MI355X trilinear point-splatting library (libtrips.so).
 *
 * The library renders the differentiable trilinear point splatting of TRIPS
 * (Franke, Rueckert, Fink, Stamminger, "TRIPS: Trilinear Point Splatting for
 * Real-Time Radiance Field Rendering", 2024): the render function of Eq. 1 without
 * the environment map, I = Phi(C, R, t, x, s_w, tau, alpha), whose output is a
 * feature image pyramid, and its backward pass.
 *
 * Conventions for every entry point:
 *  - Pointers to point data, outputs, `saved` and `workspace` are DEVICE pointers;
 *    `*_host` arguments and the config / camera / tuning structs are HOST memory.
 *  - The caller owns and allocates all memory.  The library never allocates device
 *    memory, never synchronises the stream, and never throws across the ABI.
 *  - Every argument is validated on the host before anything is launched; a call
 *    that returns an error launched nothing.  HIP launch failures return
 *    TRIPS_ERR_HIP and the HIP error code is kept for trips_last_hip_error().
 *  - All work is enqueued on `stream` in order; results are ready when the stream is.
 *    Part of a forward or backward call (the kernels of the tiles with few entries) runs on
 *    a second stream of the device that the library creates once, with the default
 *    priority, forked from `stream` and joined back into it within the call; captured into
 *    a graph, the two become branches of it.
 *  - Up to TRIPS_MAX_VIEWS views of arbitrary, different resolutions are rendered by
 *    one call ("batched views"); every point is read once per call and projected
 *    into every view.  Gradients are summed over the views of a call.
 */
#ifndef TRIPS_H
#define TRIPS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRIPS_MAX_VIEWS 16
#define TRIPS_MAX_LAYERS 12
#define TRIPS_KEEP 16 /* list clamp of Sec. 3.2: the 16 front-most fragments are blended */

typedef enum {
  TRIPS_OK = 0,
  TRIPS_ERR_INVALID_ARG = -1, /* null pointer, bad size, bad camera or config */
  TRIPS_ERR_WORKSPACE = -2,   /* workspace or saved buffer smaller than required */
  TRIPS_ERR_CAPACITY = -3,    /* problem exceeds 32-bit fragment indexing */
  TRIPS_ERR_HIP = -4,         /* a HIP call failed; see trips_last_hip_error() */
  TRIPS_ERR_UNSUPPORTED = -5  /* valid but not built: max_list != 16, desc_dim not 4 or 8,
                                 or too many tiles in one view */
} trips_status;

/* Pinhole camera (Sec. 3.1, Eq. 2), OpenCV axes (x right, y down, z forward).
   World to camera: X_c = R * X_w + t, R row-major.  Screen: x = fx * X_c / Z_c + cx,
   y = fy * Y_c / Z_c + cy, depth Z_c, screen size s = fx * s_w / Z_c.
   Points with Z_c <= znear (znear > 0) or non-finite x, y, s are culled. */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height; /* layer 0 resolution; layer L is ceil(width/2^L) x ceil(height/2^L) */
  float znear;
} trips_camera;

/* Renderer hyper-parameters (Sec. 3.1-3.2).
   include_coarser (0 or 1; zero-initialised configs leave it off): coarser-layer inclusion
   of Sec. 3.6.  The list blended at texel (i, j) of layer L then holds, besides the
   texel's own fragments, the fragments of texel (i >> k, j >> k) of every coarser layer
   L + k, each with its own gamma; the union is ordered by depth, point index, then layer
   (finer first; a point written to two layers can appear twice) and clamped to
   TRIPS_KEEP.  Gradients flow to every fragment through every list that keeps it.  It
   adds 196 B per texel of every tile to `saved` and two tables of 16 (1 + D) floats per
   texel of every tile to the backward part of `workspace`. */
typedef struct {
  int32_t num_layers; /* pyramid layers n, 1..TRIPS_MAX_LAYERS; texel size of layer L is 2^L */
  int32_t max_list;   /* must be TRIPS_KEEP (16) */
  float eps;          /* minimum layer weight for points smaller than a pixel (0.25) */
  int32_t desc_dim;   /* descriptor channels D: 4 or 8 */
  int32_t include_coarser;
} trips_config;

/* Point cloud, structure of arrays, all float32 device arrays of length n; desc is
   row-major [n][desc_dim].  size_w is the world-space size s_w; opacity is alpha. */
typedef struct {
  const float *x, *y, *z;
  const float *size_w;
  const float *opacity;
  const float *desc;
  int64_t n;
} trips_points;

/* Launch-shape choices (all optional: pass NULL, or 0 in a field, for the defaults).
   tile_w is the width in texels of a screen tile (16x16 by default; tiles always hold
   256 texels: 8x32, 16x16, 32x8, 64x4).  points_per_block is the number of points one
   binning workgroup histograms (256..65535, default 4096).  item_entries is the number of
   tile entries one sort/blend workgroup consumes before handing over to a merge
   (256..65536; default 8192 for up to one point per pixel of the largest view, doubled for
   each doubling of that density, up to 32768). */
typedef struct {
  int32_t tile_w;
  int32_t points_per_block;
  int32_t item_entries;
} trips_tuning;

/* Optional arguments of trips_forward, trips_backward and trips_plan_create (pass NULL, or
   NULL fields, for none; each call takes the fields of its direction).  Device pointers in
   pyramid order (P texels of all views and layers, the pyramid's order), [P][D] arrays
   row-major per texel and 16-byte aligned.
   - background [P][D] (forward and backward): composited behind each texel's kept
     fragments with the transmittance they leave, C += T_K * background, T_K =
     prod_m (1 - gamma_m) over the kept list.  This is where the environment map E of Eq. 1
     enters; the caller samples it per texel.
   - alpha_out [P] (forward output): the coverage 1 - T_K of every texel.
   - grad_alpha [P] (backward input): upstream gradient of alpha_out.
   - grad_background [P][D] (backward output): T_K * grad_pyramid.
   - grad_camera [views][16] (backward output): per view dL/dR (9, row-major, for
     X_c = R X_w + t), dL/dt (3), dL/dfx, dL/dfy, dL/dcx, dL/dcy. */
typedef struct {
  const float* background;
  float* alpha_out;
  const float* grad_alpha;
  float* grad_background;
  float* grad_camera;
} trips_extras;

/* Host only.  Layer sizes of one view's image pyramid (Sec. 3.1: layer L has texels of
   2^L pixels; for sizes not divisible by 2^L the layer is rounded up, W_L = ceil(W / 2^L)):
   dims_host[2L] = W_L, dims_host[2L+1] = H_L, and offsets_host[L] = first texel of layer L
   in the concatenated pyramid of that view, offsets_host[num_layers] = total texels.
   Either output may be NULL.  Errors: INVALID_ARG for a null struct, a layer count outside
   1..TRIPS_MAX_LAYERS or a view size outside 1..65536. */
trips_status trips_layer_layout(const trips_camera* cam_host, const trips_config* cfg_host,
                                int32_t* dims_host, int64_t* offsets_host);

/* Host only.  Bytes of the `workspace` (scratch, any call) and `saved` (written by the
   forward pass, read by backward and export) buffers for `views` cameras and n points.
   `saved` holds what Sec. 3.6 keeps from the forward pass for the backward pass: the
   sorted per-texel lists (here clamped to the 16 kept fragments, Sec. 3.2) and their
   lengths, plus the tile entries; every capacity is a worst case, so no call needs to
   read a count back to the host.  Both buffers must be 256-byte aligned.  Errors as
   trips_forward's argument checks (INVALID_ARG, UNSUPPORTED, CAPACITY). */
trips_status trips_buffer_sizes(const trips_config* cfg_host, const trips_camera* cams_host,
                                int32_t views, int64_t n, const trips_tuning* tuning_host,
                                size_t* workspace_bytes, size_t* saved_bytes);

/* Forward render (Eq. 1-7).  pyramid_out: float32, for each view in order, each layer
   in order, row-major [H_L][W_L][D]; overwritten.  `saved` receives the per-texel list
   lengths, the kept fragments (<= 16 per texel, front to back) and the tile entries,
   which trips_backward and trips_export_fragments read.  extras_host (may be NULL):
   background (composited) and alpha_out (written), see trips_extras. */
trips_status trips_forward(const trips_config* cfg_host, const trips_points* pts_host,
                           const trips_camera* cams_host, int32_t views,
                           const trips_tuning* tuning_host, float* pyramid_out, void* saved,
                           size_t saved_bytes, void* workspace, size_t workspace_bytes,
                           const trips_extras* extras_host, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): trips_forward with the same arguments
   minus the workspace.  The forward scratch (the part of trips_buffer_sizes' workspace a
   forward call uses) is taken from a device array inside the library of
   TRIPS_STATIC_SCRATCH_MB MiB, one per GPU the library runs on, held until the process
   ends; problems whose forward scratch is larger return TRIPS_ERR_WORKSPACE (the headline
   view, 2M points at 1920x1080 with 8 layers, needs about 220 MB).  No allocation of any
   kind is made.  Every call on one GPU uses that GPU's one array: calls that overlap on a
   device (different streams, or host threads without ordering) race and give undefined
   results; calls ordered on one stream are safe.  `saved` is the caller's, as for
   trips_forward, and trips_backward / trips_export_fragments read it as usual (the
   backward still takes a caller workspace). */
#define TRIPS_STATIC_SCRATCH_MB 256
trips_status trips_forward_noalloc(const trips_config* cfg_host, const trips_points* pts_host,
                                   const trips_camera* cams_host, int32_t views,
                                   const trips_tuning* tuning_host, float* pyramid_out,
                                   void* saved, size_t saved_bytes,
                                   const trips_extras* extras_host, hipStream_t stream);

/* The pipeline is differentiable end to end (Sec. 1 and 3: point positions, sizes,
   descriptors and opacities are optimised by gradient descent); this is the renderer's
   part of that, the adjoint of Eq. 6-7 through Eq. 2-5.
   Backward of sum(grad_pyramid * pyramid) for the forward call that filled `saved`
   (same points, cameras, config and tuning).  grad_pyramid has the pyramid layout.
   All six gradient outputs are device float32 arrays ([n], desc [n][D]) and are
   OVERWRITTEN (culled points get 0).  The per-texel blend state is recomputed from the
   kept fragments, not stored.  Sort order, culling and the 16-element clamp are
   piecewise constant and carry no gradient.  extras_host (may be NULL): the background
   the forward call used, grad_alpha (adds sum(grad_alpha * alpha_out) to the loss), and
   the outputs grad_background and grad_camera, see trips_extras. */
trips_status trips_backward(const trips_config* cfg_host, const trips_points* pts_host,
                            const trips_camera* cams_host, int32_t views,
                            const trips_tuning* tuning_host, const float* grad_pyramid,
                            const void* saved, size_t saved_bytes, void* workspace,
                            size_t workspace_bytes, float* grad_x, float* grad_y, float* grad_z,
                            float* grad_size_w, float* grad_opacity, float* grad_desc,
                            const trips_extras* extras_host, hipStream_t stream);

/* Parity export of the fragment lists of the forward call that filled `saved`.
   counts: int32 [P] untruncated number of each texel's own fragments; ids: int32 [P][16]
   the point indices of the blended list front to back (depth ascending, ties by index;
   with include_coarser, the list with the coarser layers' fragments), -1 padded.  P =
   texels of all views and layers in pyramid order. */
trips_status trips_export_fragments(const trips_config* cfg_host, const trips_camera* cams_host,
                                    int32_t views, const trips_tuning* tuning_host,
                                    const void* saved, size_t saved_bytes, int32_t* counts,
                                    int32_t* ids, hipStream_t stream);

/* Statistics of the forward call that filled `saved`, copied to host memory after a
   stream synchronisation: stats_host[0] = tile entries, [1] = work items (tile pieces of
   at most item_entries entries, and tiles of at most 256 entries, which are rendered whole;
   with include_coarser only empty tiles are rendered whole),
   [2] = tiles (bins), [3] = (point, view) pairs that wrote at least one fragment.
   For tests and reports; not needed for rendering. */
trips_status trips_forward_stats(const trips_config* cfg_host, const trips_camera* cams_host,
                                 int32_t views, const trips_tuning* tuning_host, const void* saved,
                                 size_t saved_bytes, int64_t* stats_host, hipStream_t stream);

/* Per-tile statistics of the forward call that filled `saved`, for reports: after a stream
   synchronisation, entries_host[b] = tile entries of tile b and kept_host[b] = kept
   fragments of its texels (sum of min(list length, 16)), for every tile b in bin order
   (views, then layers, then tile rows).  Both host arrays hold stats_host[2] elements. */
trips_status trips_tile_stats(const trips_config* cfg_host, const trips_camera* cams_host,
                              int32_t views, const trips_tuning* tuning_host, const void* saved,
                              size_t saved_bytes, uint32_t* entries_host, uint32_t* kept_host,
                              hipStream_t stream);

const char* trips_status_string(trips_status status);
int32_t trips_last_hip_error(void);

/* Kernel timing for reports (host side only, per calling thread).  While enabled, every
   kernel that trips_forward, trips_backward and trips_export_fragments launch outside a
   graph capture is bracketed by two HIP events recorded on its launch stream.
   trips_timing_read waits for those events and returns, per stage, the summed
   milliseconds and the number of launches since the last read (or enable), then resets.
   Stage k is named by trips_stage_name(k), k < TRIPS_NUM_STAGES.  The events are host
   objects owned by the library; no device memory is allocated. */
#define TRIPS_NUM_STAGES 14
trips_status trips_timing_enable(int32_t enable);
trips_status trips_timing_read(float* ms_host /*[TRIPS_NUM_STAGES]*/,
                               int32_t* launches_host /*[TRIPS_NUM_STAGES]*/);
const char* trips_stage_name(int32_t stage);

/* Autotuner.  Times forward + backward for each of the ncand launch shapes (one warm-up,
   then `reps` timed repetitions, HIP events on `stream`, which is synchronised) and
   returns the fastest in *best and every mean time in ms_host[ncand] (milliseconds).
   All candidates are validated first; the buffers must be large enough for every one of
   them (trips_buffer_sizes per candidate, take the maximum).  The outputs hold the result
   of the last candidate timed. */
trips_status trips_autotune(const trips_config* cfg_host, const trips_points* pts_host,
                            const trips_camera* cams_host, int32_t views,
                            const trips_tuning* candidates_host, int32_t ncand, int32_t reps,
                            float* pyramid_out, void* saved, size_t saved_bytes, void* workspace,
                            size_t workspace_bytes, const float* grad_pyramid, float* grad_x,
                            float* grad_y, float* grad_z, float* grad_size_w,
                            float* grad_opacity, float* grad_desc, trips_tuning* best_host,
                            float* ms_host, hipStream_t stream);

/* ---------------------------------------------------------------------------------
   Plan: the batched multi-view form captured once in a HIP graph and replayed.
   Buffers are bound at creation; every launch replays the forward and/or backward
   kernels for all views.  The plan owns only host objects (the graphs); all device
   memory still comes from the caller.  trips_plan_create captures on `stream`, which
   must be a created stream (not the null stream) with no capture in progress;
   grad_pyramid may be NULL for a forward-only plan.  The optional arguments (extras_host,
   may be NULL) are bound at creation too.  Launches may use any stream. */
typedef struct trips_plan trips_plan;

trips_status trips_plan_create(const trips_config* cfg_host, const trips_points* pts_host,
                               const trips_camera* cams_host, int32_t views,
                               const trips_tuning* tuning_host, float* pyramid_out, void* saved,
                               size_t saved_bytes, void* workspace, size_t workspace_bytes,
                               const float* grad_pyramid, float* grad_x, float* grad_y,
                               float* grad_z, float* grad_size_w, float* grad_opacity,
                               float* grad_desc, const trips_extras* extras_host,
                               hipStream_t stream, trips_plan** plan_out);
/* which: 1 = forward, 2 = backward, 3 = both (in that order). */
trips_status trips_plan_launch(trips_plan* plan, int32_t which, hipStream_t stream);
void trips_plan_destroy(trips_plan* plan);

/* ---------------------------------------------------------------------------------
   Reconstruction network (Sec. 3.3, Fig. conv): the feature pyramid of one view becomes one
   full-resolution image.  One block per layer, coarsest first; block L reads its layer's D
   feature channels and, below the coarsest layer, the bilinear doubling of block L+1's
   output (texel k of layer L+1 centred where texels 2k and 2k+1 of layer L meet, edge
   texels repeated, cropped to layer L); it is one gated 3x3 convolution (zero padding,
   2 x TRIPS_DEC_FEATURES outputs: ELU of the first half times the logistic sigmoid of the
   second half) plus, below the coarsest layer, the doubled input features (the
   self-bypass).  The finest block's features go through a 1x1 convolution to out_dim
   channels.  Binary16 operands, float32 accumulation: the layer features, the doubled
   features and every block output are rounded to binary16 (nearest even) where they are
   stored. */
#define TRIPS_DEC_FEATURES 32

typedef struct {
  int32_t num_layers;    /* n, 1..TRIPS_MAX_LAYERS (the pyramid's layers) */
  int32_t desc_dim;      /* D, the pyramid's channels: 4 or 8 */
  int32_t out_dim;       /* output channels, 1..8 (3 for RGB) */
  int32_t width, height; /* layer 0 resolution; layer L is ceil(width/2^L) x ceil(height/2^L) */
} trips_decoder_config;

/* Network weights, device pointers.  kernel[L]: binary16 bit patterns, [3][3][C_in][64]
   row-major (tap row, tap column, input channel, output), C_in = D for the coarsest layer and
   D + 32 otherwise (the layer's channels first, then the doubled features); outputs 0..31
   are the feature half, 32..63 the gate half.  bias[L]: float32 [64].  out_weight: float32
   [32][out_dim]; out_bias: float32 [out_dim]. */
typedef struct {
  const uint16_t* kernel[TRIPS_MAX_LAYERS];
  const float* bias[TRIPS_MAX_LAYERS];
  const float* out_weight;
  const float* out_bias;
} trips_decoder_weights;

/* Host only.  Bytes of the packed weights (trips_decoder_pack) and of the workspace of
   trips_decoder_forward (the block outputs of layers 1..n-1, binary16); both buffers
   256-byte aligned. */
trips_status trips_decoder_sizes(const trips_decoder_config* cfg_host, size_t* packed_bytes,
                                 size_t* workspace_bytes);

/* Rewrites the weights into the matrix-core operand order the convolution reads (once per
   set of weights; enqueued on `stream`).  `packed` is caller-owned device memory. */
trips_status trips_decoder_pack(const trips_decoder_config* cfg_host,
                                const trips_decoder_weights* weights_host, void* packed,
                                size_t packed_bytes, hipStream_t stream);

/* The whole network.  pyramid: float32, layers in order, each row-major [H_L][W_L][D] (the
   layout trips_forward writes for one view), 16-byte aligned.  image: float32
   [height][width][out_dim], overwritten. */
trips_status trips_decoder_forward(const trips_decoder_config* cfg_host, const void* packed,
                                   size_t packed_bytes, const float* pyramid, float* image,
                                   void* workspace, size_t workspace_bytes, hipStream_t stream);

/* One block, for tests and callers that schedule the layers themselves.  features: float32
   [H_L][W_L][D] of layer `layer`; coarse: binary16 [H_{L+1}][W_{L+1}][32], block L+1's
   output (ignored, may be NULL, for the coarsest layer).  Exactly one of `out` (binary16
   [H_L][W_L][32], the block's output) and `image` (float32 [H_L][W_L][out_dim], the output
   layer applied to the block's output) is non-NULL.  16-byte aligned. */
trips_status trips_decoder_block(const trips_decoder_config* cfg_host, const void* packed,
                                 size_t packed_bytes, int32_t layer, const float* features,
                                 const uint16_t* coarse, uint16_t* out, float* image,
                                 hipStream_t stream);

/* HIP error code of the last decoder call that returned TRIPS_ERR_HIP. */
int32_t trips_decoder_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TRIPS_H */
