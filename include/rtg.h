/*
 * rtg.h -- C ABI of the masked differentiable Gaussian rasterizer for
 * MI355X (gfx950): the mapping hot path of RTG-SLAM (Peng et al., SIGGRAPH
 * 2024, arXiv 2404.19706).
 *
 * The problem statement the calls follow (Sec. 3.1 "Image rendering" and
 * supplementary Sec. B of the paper): given a set of 3D Gaussians
 * (position p, scale s, rotation q, opacity alpha, colour c), a camera with
 * intrinsics K and one or more poses T_g in SE(3), and the pixels that need
 * rendering, produce
 *   - the colour image C by front-to-back alpha blending (Eq. 1, 2),
 *   - the transmission image T (Eq. 3),
 *   - the depth image D from the first Gaussian along each ray whose
 *     per-pixel opacity exceeds e^-0.5, intersected as a disc (Eq. 4) with
 *     the 60 degree fallback to the centre depth and -1 with no hit (Eq. 5),
 *   - the index image I (the hit Gaussian, Sec. 3.1),
 * and the gradients of a loss on C and D with respect to the parameters of
 * the unstable Gaussians (Sec. 3.2 "Gaussian optimization"; Eq. 7-8).
 *
 * Conventions (all frames of one call share the intrinsics and image size):
 *   - Gaussians are structure-of-arrays float32 in device memory:
 *     pos[N][3] (metres), scale[N][3] (metres, activated), rot[N][4] raw
 *     quaternion (w, x, y, z), used unnormalised through
 *     R = I + (2/|q|^2) M(q); opacity[N] in (0, 1]; color[N][3];
 *     unstable[N] uint8 (non-zero = unstable: receives gradients).
 *   - poses: device float64 [F][12]: camera-to-world rotation R_g
 *     row-major, then the camera centre t_g.  The camera looks along +z,
 *     x right, y down; pixel (x, y) has centre (x + 0.5, y + 0.5).
 *   - images are dense float32/int32 [F][H][W] (colour [F][H][W][3]);
 *     masks are uint8 [F][H][W], non-zero = render this pixel.  Only masked
 *     pixels are written; the caller pre-fills the rest.
 *
 * Ownership and errors: the caller owns every buffer, including the
 * workspace sized by rtg_plan_workspace_bytes.  The library never
 * allocates device memory and never synchronises; every call only enqueues
 * kernels on `stream` (a hipStream_t passed as void*, NULL = default
 * stream), so the sequence project -> bin -> render -> backward can be
 * captured in a HIP graph.  Host-side argument errors return RTG_E_INVALID
 * before anything is enqueued; launch failures return RTG_E_HIP.  A pair
 * capacity overflow is detected on the device: nothing is rendered and
 * rtg_read_status reports RTG_E_CAPACITY.  Calls that share one workspace
 * must be ordered on one stream.
 */
#ifndef RTG_H
#define RTG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTG_MAX_FRAMES 32

typedef enum rtg_status {
    RTG_OK = 0,
    RTG_E_INVALID = -1,     /* bad argument (checked on the host)            */
    RTG_E_CAPACITY = -2,    /* more (Gaussian, tile) pairs than max_pairs    */
    RTG_E_HIP = -3,         /* a HIP runtime call or kernel launch failed    */
    RTG_E_UNSUPPORTED = -4, /* no usable gfx950 device, or a call the plan's
                               configuration does not support             */
    RTG_E_DEVICE = -5,      /* a device error flag was set (reserved: no
                               current kernel sets one)                      */
    RTG_E_TOO_LARGE = -6    /* the plan's workspace does not fit the fixed
                               scratch of rtg_forward_static                 */
} rtg_status;

/* Size of the fixed device scratch that rtg_forward_static uses as its
 * workspace (one copy per device, held until the process ends). */
#define RTG_STATIC_SCRATCH_BYTES (64ull << 20)

typedef struct rtg_config {
    int32_t tile_w, tile_h;   /* tile shape: 8x8, 16x16 or 32x8 (supp. B)    */
    float cutoff2;            /* rho^2: a pixel sees Gaussian i iff its
                                 squared Mahalanobis distance d^2 <= rho^2
                                 (default 9, i.e. 3 sigma)                   */
    float dilation;           /* added to both diagonal entries of the 2D
                                 covariance (default 0: Eq. 2 as written)    */
    float z_near;             /* Gaussians with camera z <= z_near are culled
                                 (default 0.2 m)                             */
    float t_eps;              /* colour compositing of a pixel stops once its
                                 transmission falls below t_eps (the depth
                                 search continues to the first hit); the
                                 dropped colour is below t_eps * max c       */
    int32_t items_per_pop;    /* work distribution of the compositing
                                 kernels: 0 = static round-robin over the
                                 persistent waves, k >= 1 = dequeue k items
                                 at a time from an atomic queue head         */
    int32_t tile_filter50;    /* 1: drop the masked pixels of every fixed
                                 16x16 block in which fewer than half of the
                                 in-image pixels are masked (supp. B)        */
    int32_t sort_cap;         /* per-tile sorts of more than sort_cap pairs
                                 use the global-memory path (0 = 4096)       */
    int32_t stage_cap;        /* pairs each of the binning's staging regions
                                 holds (0 = 4 * max_pairs / regions, the
                                 most that fits; larger values are
                                 rejected).  The counting pass stages every
                                 pair it finds, so the pairs are enumerated
                                 once; a block whose region overflows
                                 enumerates its pairs again (same lists,
                                 slower)                                     */
    int32_t sh_degree;        /* colour parameters (Sec. 3.1): 0 = RGB
                                 colour [N][3] (default); D = 1..3 =
                                 spherical-harmonic coefficients
                                 [N][(D+1)^2][3] of the orthonormal real
                                 basis (index l^2 + l + m), the colour of
                                 Gaussian i in frame f being sum_k SH_k
                                 Y_k(d) at the unit direction d from the
                                 camera centre to the Gaussian (no offset,
                                 no clamp).  Every `color` / `d_color_param`
                                 argument then has that shape.               */
    int32_t depth_mode;       /* 0 = the depth of Eq. 4-5 (default); 1 =
                                 alpha-blended depth sum_i z_i f_i T_i (z_i
                                 the camera depth of Gaussian i's centre;
                                 -1 where no Gaussian blends) of the paper's
                                 depth-rendering ablation.  The index map
                                 keeps the first-hit rule of Eq. 5 in both
                                 modes; the backward and the L1 depth loss
                                 follow the mode.                            */
    int32_t straggler_lanes;  /* forward compositing of a pack of pixels:
                                 once at most this many of its pixels are
                                 still compositing (or searching their
                                 depth hit) and at least straggler_rest
                                 list entries remain, each such pixel walks
                                 the rest of the list alone, one entry per
                                 lane.  Same operations in the same order,
                                 so the same outputs; only the speed on
                                 long lists changes.  0 = off; default 8,
                                 at most 32                                  */
    int32_t straggler_rest;   /* see straggler_lanes (default 128, >= 1)     */
    int32_t static_share;     /* with items_per_pop >= 1: the first
                                 static_share percent of the work items
                                 (longest lists first; whole rounds) go
                                 round robin as with items_per_pop = 0,
                                 the rest come from the queue (default 0:
                                 all from the queue; 0..100)                 */
    int32_t fwd_items_per_pop; /* the forward compositing kernel's own
                                  items_per_pop (-1, the default: the same
                                  as items_per_pop; -1..1024).  The two
                                  kernels' costs per item differ, so their
                                  best chunk sizes can too.                  */
    int32_t fwd_static_share; /* the forward's own static_share (-1, the
                                 default: the same as static_share;
                                 -1..100)                                    */
} rtg_config;

typedef struct rtg_intrinsics {
    double fx, fy, cx, cy;    /* pinhole K (Sec. 3.1)                        */
    int32_t width, height;    /* image size in pixels                        */
} rtg_intrinsics;

typedef struct rtg_plan rtg_plan;   /* opaque host-side description of one
                                       problem size; holds no device memory */

/* Fill cfg with the defaults listed above. */
void rtg_config_default(rtg_config* cfg);

/* Create a plan for N < 2^30 Gaussians, F frames (1..RTG_MAX_FRAMES) of
 * the given intrinsics, and at most max_pairs (Gaussian, tile) pairs per
 * call (< 2^31).  The plan only fixes sizes and the workspace layout; it
 * touches no device.  Returns RTG_E_INVALID for unsupported tile shapes,
 * sizes or F * N >= 2^32. */
rtg_status rtg_plan_create(const rtg_config* cfg, const rtg_intrinsics* intr, int64_t n_gaussians,
                           int32_t frames, int64_t max_pairs, rtg_plan** out);
void rtg_plan_destroy(rtg_plan* plan);

/* Bytes of device workspace one plan needs (256-byte aligned base). */
size_t rtg_plan_workspace_bytes(const rtg_plan* plan);

/* Step a1 -- projection of every Gaussian into every frame (Sec. 3.1,
 * Eq. 2): camera-frame centre, splatted 2D Gaussian, depth key, surfel
 * normal, depth-test threshold and conservative pixel rectangle.  Also
 * resets the workspace counters.  Reads the Gaussian arrays and poses;
 * writes only the workspace. */
rtg_status rtg_project(const rtg_plan* plan, void* ws, const float* pos, const float* scale,
                       const float* rot, const float* opacity, const float* color,
                       const uint8_t* unstable, const double* poses, void* stream);

/* Step a2 helper (supp. B) -- M_unstable: writes mask_out[F][H][W] = 1 on
 * every pixel covered (d^2 <= rho^2) by a projected unstable Gaussian, 0
 * elsewhere; equal to {T_unstable < 1}.  Requires rtg_project first. */
rtg_status rtg_unstable_mask(const rtg_plan* plan, void* ws, uint8_t* mask_out, void* stream);

/* Steps a2-a4 -- tile binning (supp. B): active tiles and masked-pixel
 * lists from mask[F][H][W], one (Gaussian, tile) pair per projected
 * Gaussian and active tile of its rectangle, sorted per tile by (depth,
 * index).  The mask is read only during this call.  For plans of at
 * least 16384 (frame, tile)s part of the sorting runs on a side stream of
 * the current device that the library creates at its first such call
 * outside stream capture (default priority, kept until the process ends)
 * and joins back to `stream` with events before returning:
 * work enqueued on `stream` afterwards sees the finished lists.  Under graph
 * capture the fork and join become graph branches (serial launches when the
 * first call on a device is a captured one). */
rtg_status rtg_bin(const rtg_plan* plan, void* ws, const uint8_t* mask, void* stream);

/* Step a5 -- forward rasterization of the masked pixels (Eq. 1-5): colour
 * [F][H][W][3], depth, transmission [F][H][W] float32 and index [F][H][W]
 * int32 (Gaussian index of the depth hit, -1 with no hit; depth is then
 * -1).  All four outputs are required.  Also records, per masked pixel, the
 * last Gaussian that changed its colour (read by rtg_backward). */
rtg_status rtg_render(const rtg_plan* plan, void* ws, float* color, float* depth, float* trans,
                      int32_t* index, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): steps a1-a5 as
 * rtg_project + rtg_bin + rtg_render, with the workspace taken from a fixed
 * device array of RTG_STATIC_SCRATCH_BYTES inside the library instead of a
 * caller buffer.  The call allocates nothing (no hipMalloc, no library
 * allocation); the array's device address is looked up on the first call on
 * each device.  Arguments as rtg_project (Gaussians, poses), rtg_bin (mask)
 * and rtg_render (out_color, out_depth, out_trans, out_index: only masked
 * pixels are written).  status_out (device int32, may be NULL) receives,
 * on the stream, RTG_OK or RTG_E_CAPACITY when the plan's pair capacity
 * overflowed (nothing is rendered then).  Returns RTG_E_TOO_LARGE, before
 * anything is enqueued, when rtg_plan_workspace_bytes(plan) exceeds
 * RTG_STATIC_SCRATCH_BYTES (choose a smaller max_pairs, fewer Gaussians,
 * frames or pixels), RTG_E_INVALID for null arguments.  Every call on a
 * device shares that device's array and overwrites what the last call left
 * there: calls on one device that overlap in time (on different streams or
 * host threads without ordering) race; order them on one stream. */
rtg_status rtg_forward_static(const rtg_plan* plan, const float* pos, const float* scale, const float* rot,
                              const float* opacity, const float* color, const uint8_t* unstable,
                              const double* poses, const uint8_t* mask, float* out_color, float* out_depth,
                              float* out_trans, int32_t* out_index, int32_t* status_out, void* stream);

/* Steps a7-a8 -- backward pass.  d_color [F][H][W][3] and d_depth
 * [F][H][W] are dL/dC and dL/dD (read at masked pixels only); color,
 * depth, trans, index are the outputs of rtg_render on this workspace.
 * Writes the gradient rows of every unstable Gaussian (summed over frames;
 * zero rows for unstable Gaussians seen in no frame): d_pos[N][3],
 * d_scale[N][3], d_rot[N][4], d_opacity[N], d_color_param[N][3] (with
 * sh_degree D > 0: [N][(D+1)^2][3], and d_pos includes the view-direction
 * term of the SH colour).  Rows of stable Gaussians are not touched.  The
 * Gaussian arrays and poses must be those given to rtg_project; `color` (the
 * colour parameters) is read only with sh_degree > 0 and may be NULL
 * otherwise. */
rtg_status rtg_backward(const rtg_plan* plan, void* ws, const float* pos, const float* scale,
                        const float* rot, const float* opacity, const float* color,
                        const uint8_t* unstable, const double* poses, const float* out_depth,
                        const float* out_trans, const int32_t* out_index, const float* d_color,
                        const float* d_depth, float* d_pos, float* d_scale, float* d_rot,
                        float* d_opacity, float* d_color_param, void* stream);

/* The two halves of rtg_backward, for callers that schedule them apart:
 * step a7 accumulates per-frame camera-space gradients of the unstable
 * Gaussians in the workspace (colour path back to front, depth path on the
 * hit Gaussian); step a8 turns them into parameter gradients (same
 * arguments and output semantics as rtg_backward). */
rtg_status rtg_backward_raster(const rtg_plan* plan, void* ws, const float* out_depth, const float* out_trans,
                               const int32_t* out_index, const float* d_color, const float* d_depth,
                               void* stream);
rtg_status rtg_backward_project(const rtg_plan* plan, void* ws, const float* pos, const float* scale,
                                const float* rot, const float* color, const uint8_t* unstable,
                                const double* poses, float* d_pos, float* d_scale, float* d_rot,
                                float* d_opacity, float* d_color_param, void* stream);

/* Step a6 (Eq. 7-8) -- L1 colour + L1 depth loss over the rendered pixels
 * M (after the optional tile filter), w_c/(3|M|) sum|C - C*| +
 * w_d/|M_D| sum_{M_D} |D - D*| with M_D = {u in M : D != -1, D* > 0}.
 * Writes d_color / d_depth at the pixels of M (other pixels untouched) and
 * loss_out[0] (device float) = the loss.  Uses the pixel lists of rtg_bin. */
rtg_status rtg_loss_l1(const rtg_plan* plan, void* ws, const float* color, const float* depth,
                       const float* color_gt, const float* depth_gt, float w_c, float w_d,
                       float* d_color, float* d_depth, float* loss_out, void* stream);

/* Steps a6-a8 fused for the L1 loss of Eq. 7-8 (the loss rtg_loss_l1
 * computes, without upstream arrays and without the loss kernels):
 * rtg_backward_raster_l1 runs step a7 with the upstream formed per pixel at
 * unit scale, sign(C - C*) per channel and sign(D - D*) on M_D (0 elsewhere),
 * and leaves per-wave sums of |C - C*|, |D - D*| and |M_D| in the workspace;
 * rtg_backward_project_l1 then runs step a8 with the colour-path gradients
 * scaled by w_c/(3|M|) and the depth-path ones by w_d/|M_D| (both paths are
 * linear in their upstream) and writes loss_out[0] (device float) = the
 * loss; it reads the sums of the last rtg_backward_raster_l1 on this
 * workspace, so the two are called as a pair (the plain
 * rtg_backward_raster leaves no sums; after it use rtg_backward_project).
 * Gradients and loss match rtg_loss_l1 + rtg_backward_raster +
 * rtg_backward_project up to float summation order.  out_color, out_depth,
 * out_trans, out_index: the outputs of rtg_render on this workspace;
 * color_gt [F][H][W][3], depth_gt [F][H][W]: the targets; other arguments
 * and errors as rtg_backward_raster / rtg_backward_project (RTG_E_INVALID
 * also for a null loss_out).  With depth_mode 1 the two paths share the
 * footprint and opacity gradients, so rtg_backward_raster_l1 returns
 * RTG_E_UNSUPPORTED there: use rtg_loss_l1 + rtg_backward_raster +
 * rtg_backward_project. */
rtg_status rtg_backward_raster_l1(const rtg_plan* plan, void* ws, const float* out_color,
                                  const float* out_depth, const float* out_trans, const int32_t* out_index,
                                  const float* color_gt, const float* depth_gt, void* stream);
rtg_status rtg_backward_project_l1(const rtg_plan* plan, void* ws, const float* pos, const float* scale,
                                   const float* rot, const float* color, const uint8_t* unstable,
                                   const double* poses, float w_c, float w_d, float* d_pos, float* d_scale,
                                   float* d_rot, float* d_opacity, float* d_color_param, float* loss_out,
                                   void* stream);

/* Step a10 -- Adam on the rows of unstable Gaussians (Sec. 3.2; learning
 * rates of the implementation details, one per parameter group, opacity
 * fixed).  Positions, raw quaternions and colour parameters take the
 * textbook update; the scale takes it on log(scale) (scale is multiplied by
 * exp of the step).  lr_color is the rate of RGB colours, or of the band-0
 * SH coefficients, and lr_sh_rest that of SH bands 1..D (the paper uses
 * 0.05 lr_color); a zero rate leaves its group unchanged (e.g. no position
 * updates in the global optimisation).  m, v: device float32 [N][10 + 3K]
 * moments (pos 3, scale 3, rot 4, colour parameters 3K; K = 1 for RGB,
 * (D+1)^2 for SH), zero-initialised by the caller; step: device int32
 * counter incremented by this call before use (bias correction uses the
 * incremented value). */
rtg_status rtg_adam(const rtg_plan* plan, float* pos, float* scale, float* rot, float* color,
                    const uint8_t* unstable, const float* d_pos, const float* d_scale,
                    const float* d_rot, const float* d_color, float* m, float* v, int32_t* step,
                    float lr_pos, float lr_scale, float lr_rot, float lr_color, float lr_sh_rest,
                    float beta1, float beta2, float eps, void* stream);

/* ---- Gaussian adding and state management (Sec. 3.2) ----------------------
 * The steps either side of the optimisation, on one frame's images: the
 * render of the frame by the current Gaussians (colour [H][W][3], depth,
 * transmission [H][W] float32, index [H][W] int32, as written by
 * rtg_render with every pixel masked) and the input frame (colour
 * [H][W][3], depth [H][W] float32; depth <= 0 = invalid).  Per-Gaussian
 * state: unstable uint8[N], eta (confidence count), err (error count) and
 * tstamp (frame of creation or of the last stable -> unstable change)
 * int32[N].  All pointers are device pointers except the parameter
 * structs; calls enqueue on `stream` and never synchronise. */
typedef struct rtg_adding_params {
    float delta_T;            /* Eq. 6: transmission above it -> M_s (0.5)  */
    float delta_d;            /* Eq. 6: |D_render - D| above it -> M_s (0.1 m) */
    float delta_c;            /* Eq. 6: per-channel mean |C_render - C| above
                                 it -> M_c (0.1)                             */
    float rate;               /* fraction of M_s / M_c pixels sampled (0.05) */
    float alpha_opaque;       /* opacity of discs added on M_s (0.99)        */
    float alpha_transparent;  /* opacity of discs added on M_c (0.1)         */
    float r_transparent;      /* radius cap of transparent discs (0.01 m)    */
    float thickness;          /* thin-axis / in-plane scale ratio (0.1)      */
    int32_t delta_eta;        /* unstable -> stable when eta > it (100)      */
    int32_t delta_e;          /* stable -> unstable when err > it (5; the
                                 paper gives no value)                       */
    int32_t delta_t;          /* unstable for more than it frames ->
                                 removed (200; the paper gives no value)    */
    int32_t sh_degree;        /* colour rows written for new Gaussians: 0 =
                                 RGB [3]; D = SH [(D+1)^2][3] with the
                                 band-0 coefficient c / Y_00 (so the colour
                                 is the pixel's from every direction) and
                                 the higher bands zero (0)                   */
} rtg_adding_params;

void rtg_adding_params_default(rtg_adding_params* prm);

/* Bytes of device workspace rtg_add_gaussians needs for an image of the
 * given size (256-byte aligned base); 0 for invalid intrinsics. */
size_t rtg_adding_workspace_bytes(const rtg_intrinsics* intr);

/* Gaussian adding of Sec. 3.2 (Eq. 6) for one frame with camera-to-world
 * pose `pose` (device float64 [12], as rtg_project).  Per pixel with valid
 * input depth: M_s = {T > delta_T or |D_r - D| > delta_d}, M_c = {summed
 * channel |C_r - C| > 3 delta_c, not M_s} (decisions in binary32 as
 * written).  A pixel of M_s or M_c is sampled when rand[H][W] (uniform in
 * [0, 1), supplied by the caller) is below `rate`; a sampled M_s pixel adds
 * an opaque disc, a sampled M_c pixel adds a transparent one when its
 * depth-hit Gaussian (index_r) is stable, and neither is added without a
 * normal (the cross product of the vertex differences to the right and
 * lower neighbours; none on the last row / column or next to invalid
 * depth).  The new Gaussians go to rows n_cur, n_cur + 1, ... in raster
 * order of their pixels, while rows < capacity remain: position = the
 * pixel's vertex in the world, colour = the input colour, scales
 * (r, r, thickness r) with r = sqrt(1 / (pi rate)) D / ((fx + fy) / 2)
 * (transparent: at most r_transparent), rotation taking the thin axis to
 * the normal (unit quaternion), unstable = 1, eta = err = 0,
 * tstamp = frame_k.  counts[2] (device int64) receives the rows added and
 * the pixels that qualified; mask_out[H][W] (may be NULL) the Eq. 6 mask
 * (1 M_s, 2 M_c, 0 none).  ws: rtg_adding_workspace_bytes bytes.
 * RTG_E_INVALID for null arguments, capacity < n_cur or >= 2^30. */
rtg_status rtg_add_gaussians(const rtg_intrinsics* intr, const rtg_adding_params* prm, const double* pose,
                             const float* color_in, const float* depth_in, const float* color_r,
                             const float* depth_r, const float* trans_r, const int32_t* index_r,
                             const float* rand, int32_t frame_k, int64_t n_cur, int64_t capacity, float* pos,
                             float* scale, float* rot, float* opacity, float* color, uint8_t* unstable,
                             int32_t* eta, int32_t* err, int32_t* tstamp, uint8_t* mask_out, int64_t* counts,
                             void* ws, size_t ws_bytes, void* stream);

/* Confidence count of Sec. 3.2: eta + 1 for every unstable Gaussian whose
 * colour gradient row d_color[N][row_width] of the step is non-zero (its
 * colour was updated); row_width = 3 for RGB colours, 3 (D+1)^2 for SH
 * coefficients of degree D (1..48). */
rtg_status rtg_confidence_count(int64_t n, int32_t row_width, const uint8_t* unstable, const float* d_color,
                                int32_t* eta, void* stream);

/* State management of Sec. 3.2 for frame frame_k, from the render by the
 * optimised Gaussians and the input frame: every stable Gaussian that the
 * index map names at a pixel with valid input depth and a colour error
 * (as Eq. 6) or a depth error (hit pixels) gets err + 1 (once per call);
 * then a stable Gaussian with err > delta_e becomes unstable (err = eta = 0,
 * tstamp = frame_k), an unstable one with eta > delta_eta becomes stable,
 * and an unstable one with frame_k - tstamp > delta_t is marked for removal
 * (keep[i] = 0; else 1).  flag_ws: n bytes of device scratch.  Removal
 * itself is rtg_compact_rows over the per-Gaussian arrays. */
rtg_status rtg_state_update(const rtg_intrinsics* intr, const rtg_adding_params* prm, const float* color_in,
                            const float* depth_in, const float* color_r, const float* depth_r,
                            const int32_t* index_r, int32_t frame_k, int64_t n, uint8_t* unstable,
                            int32_t* eta, int32_t* err, int32_t* tstamp, uint8_t* keep, uint8_t* flag_ws,
                            void* stream);

/* Bytes of device workspace rtg_compact_rows needs for n rows. */
size_t rtg_compact_workspace_bytes(int64_t n);

/* Stable compaction (the removal of Sec. 3.2 "State management"): copies
 * the rows i with keep[i] != 0, in order, of n_arrays (<= 16) device arrays
 * src[k] (row_bytes[k] bytes per row, 1..4096) to dst[k] (distinct from
 * src[k]); n_out (device int64) receives the kept count.  The pointer
 * arrays src, dst and row_bytes are host memory.  n < 2^31. */
rtg_status rtg_compact_rows(int64_t n, const uint8_t* keep, int32_t n_arrays, void* const* src, void* const* dst,
                            const int32_t* row_bytes, int64_t* n_out, void* ws, size_t ws_bytes, void* stream);

/* ---- The mapping iteration around the backward (Sec. 3.2) -----------------
 * Device pointers except where stated; calls enqueue on `stream` and never
 * synchronise. */

/* The regulariser L_reg of Eq. 8 ("Gaussian optimization"): an L2 pull of
 * every transparent Gaussian's position, activated scale and raw
 * quaternion to the values it was added with (pos0 [N][3], scale0 [N][3],
 * rot0 [N][4]): L_reg = sum over transparent[i] != 0 of |p - p0|^2 +
 * |s - s0|^2 + |q - q0|^2.  Adds w_reg L_reg (binary64, one atomic add per
 * workgroup, so the order of the partial sums varies) to loss_out[0]
 * (device double, zeroed by the caller), and the gradient
 * 2 w_reg (x - x0) to the rows d_pos, d_scale, d_rot of the unstable
 * transparent Gaussians (stable rows are not touched).  The paper uses
 * w_reg = 1000.  n < 2^31. */
rtg_status rtg_reg_l2(int64_t n, float w_reg, const uint8_t* transparent, const uint8_t* unstable,
                      const float* pos, const float* scale, const float* rot, const float* pos0,
                      const float* scale0, const float* rot0, float* d_pos, float* d_scale, float* d_rot,
                      double* loss_out, void* stream);

/* Eq. 9: fuses a window's optimised Gaussians G' (pos, scale, rot, color,
 * updated in place) with their values before the window G_prev: per
 * Gaussian w = (eta_cur - eta_prev) / eta_cur as a binary32 division of the
 * confidence counts (w = 1 when eta_cur = 0), and every value becomes
 * fl32(fl32((1 - w) G_prev) + fl32(w G')).  color_width: colour values per
 * row (3 for RGB, 3 (D+1)^2 for SH; 1..48).  The counts keep eta_cur.
 * n < 2^31. */
rtg_status rtg_fuse(int64_t n, int32_t color_width, const int32_t* eta_prev, const int32_t* eta_cur,
                    const float* pos_prev, const float* scale_prev, const float* rot_prev, const float* color_prev,
                    float* pos, float* scale, float* rot, float* color, void* stream);

/* Pixel selection of the global optimisation ("Keyframes and global
 * optimization": the pixels with the top 40 % colour errors of each
 * keyframe): with the colour error e = (|dC0| + |dC1|) + |dC2| in binary32
 * of the render color_r against the input color_in ([F][H][W][3]) and
 * k = floor(frac H W) (binary64 product), mask_out[F][H][W] = 1 on the
 * pixels whose error is at least the k-th largest of their frame (ties at
 * that value all selected; none when k = 0), else 0.  frac in [0, 1].
 * ws: rtg_select_workspace_bytes bytes (256-byte aligned). */
size_t rtg_select_workspace_bytes(int32_t frames, int32_t height, int32_t width);
rtg_status rtg_select_top_error(int32_t frames, int32_t height, int32_t width, double frac,
                                const float* color_r, const float* color_in, uint8_t* mask_out, void* ws,
                                size_t ws_bytes, void* stream);

/* ---- Frame-to-model tracking (Sec. 3.2 "Camera tracking", Eq. 10) -------- */

/* Normal map of the last rtg_render on ws (Sec. 3.1): per rendered pixel the
 * hit Gaussian's binary32 camera-frame normal (its smallest-scale axis),
 * turned to face the camera (flipped when its dot product with the pixel's
 * ray direction ((x + 0.5 - cx) / fx, (y + 0.5 - cy) / fy, 1) is positive);
 * 0 on rendered pixels without a hit; other pixels untouched.
 * normal_out [F][H][W][3]. */
rtg_status rtg_render_normals(const rtg_plan* plan, void* ws, float* normal_out, void* stream);

typedef struct rtg_icp_params {
    int32_t levels;           /* pyramid levels, 1..3 (3)                    */
    int32_t iters[3];         /* iterations per level, finest first
                                 (10, 5, 4); levels run coarse to fine        */
    double dist;              /* pairs farther apart are dropped (0.1 m)     */
    double sin_angle;         /* pairs whose normals differ by more than this
                                 angle's sine are dropped (sin 20 deg)       */
} rtg_icp_params;

void rtg_icp_params_default(rtg_icp_params* prm);

/* Device workspace of rtg_icp for one image size (256-byte aligned base);
 * 0 for invalid arguments. */
size_t rtg_icp_workspace_bytes(const rtg_intrinsics* intr, int32_t levels);

/* Multi-level projective point-to-plane ICP (Eq. 10, as KinectFusion) of
 * the input depth frame depth_in [H][W] (<= 0 invalid) against the model's
 * rendered depth_model [H][W] (-1 or <= 0: no surface) and normals
 * normal_model [H][W][3] (camera frame of pose_model, e.g. from
 * rtg_render_normals), starting from pose_init; writes the refined
 * camera-to-world pose of the input frame to pose_out (device double[12],
 * rotation row-major then centre; may equal pose_init).  Level l has
 * floor(W / 2^l) x floor(H / 2^l) pixels and intrinsics divided by 2^l;
 * its depths are the mean of the valid depths of each 2 x 2 block, its
 * model normals those of each block's first valid pixel.  Per iteration:
 * input vertices V and normals (cross product of the forward differences)
 * under the estimate T, projected into the model camera; a pair (p, q, n)
 * is kept when the model pixel has depth and normal, |p - q| <= dist and
 * the normals' angle is within sin_angle; residual r = (p - q) . n,
 * Jacobian [p x n, n] for the update T <- exp(xi) T; the normal equations
 * are summed in binary64 in a fixed order and solved by Cholesky (no
 * update with fewer than 6 pairs or a non-positive pivot).  trace_out
 * (device double[total iterations][48], or NULL): per iteration the pose it
 * used (12), sum r^2, the pair count, A's upper triangle (21, row-major) and
 * b (6).  All on `stream`, no host synchronisation. */
rtg_status rtg_icp(const rtg_intrinsics* intr, const rtg_icp_params* prm, const float* depth_in,
                   const float* depth_model, const float* normal_model, const double* pose_model,
                   const double* pose_init, double* pose_out, double* trace_out, void* ws, size_t ws_bytes,
                   void* stream);

/* Device counters of the calls on ws since the last rtg_project, copied to
 * the host: enqueues a one-workgroup reduction of the per-wave work
 * counters and a 128-byte header copy, then synchronises `stream` (the one
 * synchronising call of the library; it allocates nothing); counts_out
 * holds 11 values:
 * [0] pairs K, [1] masked pixels, [2] work items, [3] overflow flag,
 * [4] tiles sorted on the global path, [5] device error flags,
 * [6] list entries the pixels tested before finishing (forward),
 * [7] Gaussians blended into colours, [8] list entries walked back
 * (backward), [9] (pixel, Gaussian) gradient contributions, [10] binning
 * blocks whose pair staging overflowed (their pairs were enumerated
 * twice; see stage_cap).  Counters [6]-[9] describe the last rtg_render /
 * rtg_backward call, [10] the last rtg_bin.  Returns RTG_E_CAPACITY
 * when the pair capacity overflowed (RTG_E_DEVICE is reserved). */
rtg_status rtg_read_status(const rtg_plan* plan, void* ws, int64_t* counts_out, void* stream);

/* Byte offsets of the workspace arrays (for inspection in tests):
 * out[0] projected records (64 B per frame-major slot f*N+i: mu.x, mu.y,
 * Q.xx, 2 Q.xy, Q.yy, alpha, tau, colour, index word, centre residual,
 * n^c, h), [1] depth
 * keys (float32 per slot), [2] pixel rectangles (int16 x0,x1,y0,y1 per
 * slot), [3] visibility bits (uint32 per Gaussian), [4] per-tile pair
 * range ends, [5] per-tile pair range starts (both 0 for tiles without
 * pairs), [6] sorted pairs (uint32 slot ids),
 * [7] per-tile masked-pixel counts, [8] camera-space gradient
 * accumulators (16 float32 per slot), [9] header.  Returns the count
 * written (<= n). */
int32_t rtg_plan_layout(const rtg_plan* plan, int64_t* out, int32_t n);

const char* rtg_status_string(rtg_status s);
const char* rtg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RTG_H */
