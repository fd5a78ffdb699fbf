/*
 * splat.h -- C ABI of the MI355X (gfx950) differentiable splatting library.
 *
 * The library renders LiDAR-anchored 3-D Gaussians into many camera views and
 * back-propagates an image-space loss gradient to the Gaussian parameters, to
 * the camera->LiDAR extrinsic correction and to the per-camera time offset, as
 * the calibration method of 3DGS-Calib (arXiv 2403.11577) requires.
 *
 * Call order of one calibration step (every call is asynchronous on `stream`):
 *   splat_pose_interp_fwd -> splat_project -> splat_bin_sort -> splat_render_fwd
 *   (loss gradient by the caller) -> splat_render_bwd -> splat_project_bwd
 *   -> splat_pose_interp_bwd
 *
 * Memory.  Every pointer argument that is not a `const splat_plan *` or a
 * `const splat_gaussians *` / `const splat_settings *` (host structs) is a
 * DEVICE pointer owned by the caller.  The library never allocates, frees,
 * copies to the host or synchronises, so a whole step can be captured in a HIP
 * graph.  Intermediate per-step state lives in one caller-allocated device
 * workspace `ws` whose size and internal layout `splat_plan_make` computes.
 *
 * Errors.  Arguments are checked on the host before anything is launched;
 * a bad argument returns a negative code, launches nothing, and leaves a text
 * message for splat_last_error() (thread local).  Data-dependent conditions
 * found on the device are OR-ed into the status word at ws + plan->off_status:
 *   SPLAT_ST_CAPACITY  slot or instance capacity exceeded (outputs undefined;
 *                      grow the capacities and run again),
 *   SPLAT_ST_NONFINITE a Gaussian with a non-finite parameter (culled),
 *   SPLAT_ST_DEGENERATE a Gaussian with |q| < 1e-12 (culled),
 *   SPLAT_ST_EXTRAPOLATED a camera time outside the trajectory (informational),
 *   SPLAT_ST_RANGE     a point outside the voxel grid (voxel downsampling; the
 *                      point was clamped into the grid),
 *   SPLAT_ST_SEQUENCE  splat_bin_sort on a projection made for the other bin
 *                      sort (plan->slot_sort changed in between): nothing was
 *                      binned, every tile list is empty; project again.
 * The library never clears the status word; the caller zeroes it when it wants.
 *
 * Threading.  Re-entrant; no global mutable state except the thread-local
 * error text.  Calls that share a workspace must be ordered on one stream.
 */
#ifndef SPLAT_H
#define SPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define SPLAT_API __attribute__((visibility("default")))
#else
#define SPLAT_API
#endif

#define SPLAT_OK 0
#define SPLAT_EINVAL (-1)       /* invalid argument: nothing launched */
#define SPLAT_EUNSUPPORTED (-2) /* valid but unsupported (e.g. key wider than 64 bits) */
#define SPLAT_ELAUNCH (-3)      /* the HIP runtime refused a launch */

#define SPLAT_ST_CAPACITY 1u
#define SPLAT_ST_NONFINITE 2u
#define SPLAT_ST_DEGENERATE 4u
#define SPLAT_ST_EXTRAPOLATED 8u
#define SPLAT_ST_RANGE 16u
#define SPLAT_ST_SEQUENCE 32u

/*
 * Renderer constants.  The paper fixes none of them (it defers the splatting
 * function to EWA splatting and the loss to the original 3DGS work); these are
 * the library's readings, identical to the reference renderer's defaults:
 *   near_z 0.2 m, far_z 256 m   depth window on the FP32 depth key (culls)
 *   eps2d 0.3 px^2               screen-space low-pass added to the 2-D covariance
 *   alpha_min 1/255, alpha_max 0.99, t_min 1e-4   compositing thresholds
 *   guard 0.15                   Jacobian guard band, fraction of the image size
 *   bg                           background colour
 *   pad_px 0.1, pad_rel 1e-4     footprint padding (absolute px, relative)
 * Launch shape (results do not depend on it):
 *   tile_w x tile_h in {8x8, 16x16, 16x32, 32x16}; batch = Gaussians per LDS
 *   batch in [16, 256], multiple of 16; persistent = 1 runs the render kernels
 *   as persistent workgroups over a cost-ordered (view, tile) queue, 0 launches
 *   one workgroup per (view, tile).
 */
typedef struct splat_settings {
    double near_z, far_z, eps2d, alpha_min, alpha_max, t_min, guard;
    double bg[3];
    double pad_px, pad_rel;
    int32_t tile_w, tile_h, batch, persistent;
    int32_t roi_y0;     /* first image row of the region of interest; rows above are not rendered */
    int32_t split_len;  /* instances per work item of the render adjoint (0: 1024; else a power of
                           two in [64, 2^24]); a tile list at least this long is split into chunks of
                           this length that are walked in parallel                                 */
    int32_t split_fwd;  /* 1: the forward also composites the chunks after the first of every split
                           list in parallel, each from T = 1, and joins them per pixel (exact up to
                           rounding; a chunk in which a pixel could reach t_min is walked in order).
                           Pays off when few pixels saturate; 0 (default): one walk per list */
    int32_t reserved0;
} splat_settings;

/* Gaussian parameters: device SoA planes of length n (float32).
 * mean[3][n] world position (fixed LiDAR points, Sec. III-B), quat[4][n]
 * rotation (w,x,y,z; normalised inside), scale[3][n] (> 0), opacity[n] in (0,1)
 * (activated), color[3][n] view-independent RGB (Sec. III-B). */
typedef struct splat_gaussians {
    const float *mean, *quat, *scale, *opacity, *color;
    int64_t n;
} splat_gaussians;

/* Workspace layout for one (settings, views, Gaussians, image, capacity) shape.
 * All off_* are byte offsets into the workspace; every region is 256-byte
 * aligned.  Filled by splat_plan_make; treat as read-only. */
typedef struct splat_plan {
    splat_settings s;
    int32_t n_views, width, height;
    int32_t tiles_x, tiles_y, tiles_per_view;
    int32_t depth_bits, tile_bits;   /* sort key = (view*T + tile) << depth_bits | depth */
    int32_t n_blocks_proj;           /* project workgroups (256 Gaussians each, 4 waves) */
    int32_t n_sort_blocks;           /* radix-sort partitions */
    int64_t n_gauss, slot_cap, inst_cap;
    size_t ws_bytes;
    size_t off_status;      /* u32                                                      */
    size_t off_counts;      /* u32[8]: 0 slots, 1 instances, 2 work counter, 3 split lists, 4 chunks
                               of the split lists, 5 render-adjoint items, 6 the bin sort the
                               last projection prepared for, 7 runs of 64 depth-sorted slots  */
    size_t off_view_off;    /* u32[V+1] first slot of every view                          */
    size_t off_blockcnt;    /* u32[V*n_blocks_proj*4+1] visible count per (view, wave), scanned in place to slot offsets */
    size_t off_rec;         /* float4[3][slot_cap]: (mx,my,lx,ly) (a,b,c,o) (r,g,b,depth) */
    size_t off_meta;        /* int2[slot_cap]: (Gaussian id, view); see splat_slot_meta  */
    size_t off_rect;        /* u16x4[slot_cap]: tile rect (x0,x1,y0,y1) inclusive (slot_sort 0) */
    size_t off_ntiles;      /* u32[slot_cap+1]: tiles per slot, scanned to offsets (slot_sort 0) */
    size_t off_keys;        /* u64[2][inst_cap] (the sort's last passes keep u32 keys, see key_shift) */
    size_t off_vals;        /* u32[2][inst_cap]                                          */
    size_t off_ranges;      /* u32x2[V*T]: [start,end) of every (view, tile) list         */
    size_t off_queue;       /* u32[V*T]: (view, tile) work items, most expensive first    */
    size_t off_hist;        /* u32[2^radix_bits*n_sort_blocks + 129] radix / queue histograms */
    size_t off_scan;        /* u32[scan partials]                                        */
    size_t off_grad2d;      /* float[slot_cap][9]: moments of dL/dpower over the pixel offsets
                               (x, y, xx, xy, yy, 1), then dL/d(r,g,b)                      */
    size_t off_visbits;     /* u64[V*n_blocks_proj*4]: visible (view, Gaussian) bit masks  */
    size_t off_dwpart;      /* f64[V][n_blocks_proj][4][12] per-wave W2C gradient partials (written for the
                               waves with a visible Gaussian in the view), then f64[V][32][12] stage sums */
    size_t off_cam;         /* per view f64[8] + f32[20]: camera constants of the projection, then
                               float32 copies of the view matrix and of those constants        */
    int32_t sorted_buf;     /* which of the two key/value buffers holds the sorted result */
    int32_t radix_bits;     /* digit width of the LSD radix sort (passes = ceil(key bits / radix_bits)) */
    int32_t split_len;      /* instances per render-adjoint work item (the settings' value or 1024)   */
    int32_t key_shift;      /* >= 0: the sorted keys are u32 (key >> key_shift), in the first half of
                               the sorted key buffer; -1: u64 keys                                      */
    int64_t chk_cap;        /* checkpoint slots (an upper bound of what the tile lists can need)     */
    int64_t bq_cap;         /* render-adjoint work items (upper bound)                               */
    size_t off_bqueue;      /* uint4[bq_cap]: adjoint items (view-tile, chunk, first checkpoint slot or
                               0xFFFFFFFF, 0): the chunks of the split lists, then the other tiles,
                               both in work-queue order                                              */
    size_t off_bqoff;       /* u32[V*T+1]: chunk count per split queue position, scanned to offsets */
    size_t off_chk;         /* float4[chk_cap][tile_w*tile_h]: per-pixel (T, C) of a split list: its
                               first slot holds the final state, slot c the state where chunk c starts */
    size_t off_chklast;     /* i32[chk_cap][tile_w*tile_h]: last blended instance of chunk c composited
                               on its own (split_fwd)                                                   */
    size_t off_bmask;       /* u8[inst_cap]: per instance, bit k set when the forward blended it into a
                               pixel of 8x8 sub-block k of its tile; the adjoint skips the others      */
    size_t off_dkey;        /* u32[slot_cap]: depth field of each slot's sort key,
                               bits(depth32) - bits(near_z) (a compact copy for the emission; with
                               slot_sort, the slot sort's input keys, overwritten by it)             */
    int32_t slot_sort;      /* 1: the slots are sorted by their depth field first, carrying a packed
                               payload; the instances are emitted in that order with u32 keys
                               view*T + tile and sorted on the tile bits only (the same order as the
                               64-bit sort: stable sorts, ties in depth keep the slot order).  Chosen
                               when the payload fits 64 bits; 0: one 64-bit key per instance.        */
    int32_t pack_bits[3];   /* slot_sort: widths b0, b1, b2 of the payload fields: slot | first tile
                               << b0 | (w - 1) << (b0 + tile_bits) | (h - 1) << (b0 + tile_bits + b1),
                               the tile rect being w x h tiles from its first tile (view*T + tile) */
    size_t off_spay;        /* u64[2][slot_cap]: packed payloads of the slot sort (slot_sort)        */
    size_t off_skeys;       /* u32[slot_cap]: the slot sort's second key buffer (slot_sort)          */
    size_t off_soff;        /* u32[ceil(slot_cap/64)+1]: instances of every run of 64 slots in depth
                               order, scanned to the runs' first instance (slot_sort)               */
    size_t off_l1part;      /* f64[V*T + ceil(V*T / 4096)]: splat_render_fwd_l1's partial sums of
                               |C - target|, one per (view, tile), then one per group of 4096 of
                               them; summed in this fixed order                                    */
} splat_plan;

/* Fill `s` with the default settings listed above (16x16 tiles, batch 64,
 * persistent). */
SPLAT_API void splat_default_settings(splat_settings *s);

/*
 * Compute the workspace layout.  n_views >= 1, n_gauss >= 0, width and height
 * in [1, 16384], slot_cap >= 1 (visible (view, Gaussian) pairs, at most
 * n_views*n_gauss is ever needed), inst_cap >= 1 ((Gaussian, tile) pairs);
 * both capacities below 2^31.  Returns SPLAT_EUNSUPPORTED when the sort key
 * (tile bits + depth bits) would exceed 64 bits.
 */
SPLAT_API int splat_plan_make(const splat_settings *s, int32_t n_views, int64_t n_gauss, int32_t width,
                    int32_t height, int64_t slot_cap, int64_t inst_cap, splat_plan *plan);

/*
 * Camera poses (paper Sec. III-A, Eq. 1 and Eq. 2).  The LiDAR trajectory is
 * the piecewise interpolation of K >= 2 timestamped poses: linear in the
 * translation and SLERP in the rotation (shortest arc); the camera pose of view
 * v at camera time t_v is T_L(t_v + delta_c) * T_c with the camera->LiDAR
 * extrinsic T_c = (R0_c Exp(phi_c), t0_c + rho_c), and the output is its
 * inverse (world->camera).  Segments are left-closed; times before the first
 * or after the last knot extrapolate the end segment and set
 * SPLAT_ST_EXTRAPOLATED.
 *   knot_t[K] (strictly increasing, seconds), knot_q[K][4] (w,x,y,z, LiDAR->
 *   world), knot_p[K][3]; R0[C][9] row-major, t0[C][3]; xi[C][6] = (rho, phi);
 *   delta[C] seconds; view_cam[V] in [0,C); view_t[V] seconds.
 *   Output w2c[V][12] float64, row-major [W | w] with x_cam = W x_world + w.
 * Monotonicity of knot_t and the range of view_cam are the caller's contract:
 * the library does not read device data on the host, so it cannot check them
 * (the Python binding checks both once, when a scene is copied to the device).
 */
SPLAT_API int splat_pose_interp_fwd(int32_t K, const double *knot_t, const double *knot_q,
                          const double *knot_p, int32_t C, const double *R0, const double *t0,
                          const double *xi, const double *delta, int32_t V,
                          const int32_t *view_cam, const double *view_t, double *w2c,
                          uint32_t *status, void *stream);

/*
 * Adjoint of splat_pose_interp_fwd (end of Sec. III-B: the photometric loss
 * reaches the extrinsic and the time offset through the input pose, i.e.
 * through Eq. 2, Eq. 1 and the interpolation of Sec. III-A).
 * Given dL/dw2c[V][12] (float64) it ADDS
 * dL/dxi[C][6] and dL/ddelta[C] (float64, caller zeroes).  The rotation part
 * uses the right Jacobian of SO(3); d/ddelta goes through the interpolation
 * (translation velocity of the segment and its angular velocity).  Views of
 * one camera are summed in view order (deterministic).
 */
SPLAT_API int splat_pose_interp_bwd(int32_t K, const double *knot_t, const double *knot_q,
                          const double *knot_p, int32_t C, const double *R0, const double *t0,
                          const double *xi, const double *delta, int32_t V,
                          const int32_t *view_cam, const double *view_t, const double *dw2c,
                          double *dxi, double *ddelta, void *stream);

/*
 * Projection (paper Eq. 2 and Eq. 3 folded into W Sigma W^T, then EWA):
 * for every (view, Gaussian) the float32 depth key depth32 =
 * fma(W20, x, fma(W21, y, fma(W22, z, w2))) on float32-rounded row 2 of w2c;
 * cull when depth32 <= near_z or > far_z, opacity < alpha_min, |q| < 1e-12, a
 * non-finite parameter, or an empty on-screen footprint; otherwise (in float64)
 * the camera-frame covariance, the perspective Jacobian with the guard band,
 * the 2-D covariance + eps2d, its inverse (conic), the pixel mean and the
 * opacity-aware footprint (alpha >= alpha_min inside an axis-aligned box of
 * half-widths sqrt(2 ln(o/alpha_min) Sigma2_ii), padded).  Visible pairs are
 * compacted per view in Gaussian order into slots.
 *   g: Gaussians (device planes); w2c[V][12] float64 (device);
 *   intr[V][4] float64 (fx, fy, cx, cy) per view (device).
 * Writes counts, view_off, rec, the depth fields and, for the bin sort the
 * plan selects, the slot payloads (plan->slot_sort = 1) or meta and the tile
 * rects and counts (0) in the workspace.
 */
SPLAT_API int splat_project(const splat_plan *plan, void *ws, const splat_gaussians *g, const double *w2c,
                  const double *intr, void *stream);

/*
 * The (Gaussian id, view) of every slot of the last splat_project on this
 * workspace, written to meta (int2[slot_cap] at plan->off_meta), for callers
 * that map slots back to Gaussians (checks, statistics).  The paper has no
 * passage for it: slots are this library's compaction of the visible pairs
 * of the projection (Sec. III-B).  The projection stores meta itself only
 * for plan->slot_sort = 0, whose binning reads it.  Reads the visibility
 * words and slot offsets the projection left, so call it after that
 * splat_project and before the next one.
 */
SPLAT_API int splat_slot_meta(const splat_plan *plan, void *ws, void *stream);

/*
 * Tile binning (the paper has no passage for it: it is how Phi of Eq. 5 finds
 * the Gaussians of a tile in depth order).  Every tile list ends up in
 * (depth32, Gaussian id) order, value = slot:
 *  - plan->slot_sort = 1: the slots are sorted by bits(depth32) - bits(near_z)
 *    (stable LSD radix sort, so equal depths keep the slot order, which is
 *    (view, Gaussian id)), one instance per (slot, covered tile) is emitted in
 *    that order with key view*T + tile, and a stable radix sort on the tile bits
 *    finishes the lists;
 *  - plan->slot_sort = 0: the instances are emitted in (view, Gaussian, tile
 *    row-major) order with key ((view*T + tile) << depth_bits) | (bits(depth32)
 *    - bits(near_z)) and sorted on all key bits.
 * Writes the sorted values, per-(view, tile) ranges and the cost-ordered work
 * queue in the workspace; plan->sorted_buf names the buffer that holds the
 * sorted result (it is a function of the plan only).  With slot_sort = 0 the
 * per-slot tile counts written by splat_project are turned into instance
 * offsets in place; with slot_sort = 1 the slot sort consumes the depth fields.
 * Either way, call this exactly once after each splat_project, with the same
 * slot_sort as that projection (otherwise nothing is binned and
 * SPLAT_ST_SEQUENCE is set).  When the instances exceed inst_cap, the longest
 * prefix of whole slots in emission order is kept and SPLAT_ST_CAPACITY is set.
 */
SPLAT_API int splat_bin_sort(const splat_plan *plan, void *ws, void *stream);

/*
 * Forward compositing (the splatting function Phi of Eq. 5): every pixel
 * (sampled at its centre, +0.5) walks its tile list front to back, alpha =
 * min(alpha_max, o exp(-d^T Q d / 2)), skips alpha < alpha_min, stops before a
 * blend that would take T below t_min, and accumulates C += c alpha T.
 * Outputs (device, float32/int32): img[V][3][H][W] = C + T bg,
 * T_final[V][H][W], last_pos[V][H][W] = instance index of the last blended
 * Gaussian (into the sorted value buffer) or -1.  Also records, for
 * splat_render_bwd, the checkpoints of the split lists it starts its chunks
 * from and which 8x8 sub-blocks of its tile each instance was blended into,
 * and clears the slots' gradient sums that splat_render_bwd adds into.
 * With settings.split_fwd the chunks after the first of each split list are
 * composited in parallel from T = 1 and joined per pixel (C += T C_chunk,
 * T *= T_chunk); a chunk in which some pixel of the tile could reach t_min
 * (T T_chunk below t_min with a relative margin covering the rounding) is
 * walked in order instead, so the stop decisions are the sequential ones.
 */
SPLAT_API int splat_render_fwd(const splat_plan *plan, void *ws, float *img, float *T_final,
                     int32_t *last_pos, void *stream);

/*
 * splat_render_fwd and, in the same launch, splat_l1_loss_grad of the image it
 * renders (paper Eq. 4, the L1 term; the rows [plan->s.roi_y0, H)): img,
 * T_final and last_pos as splat_render_fwd writes them, dL_dimg = weight *
 * sign(img - target)/N inside the region of interest (0 above it and where
 * mask is set; N = V*3*(H - roi_y0)*W) and *loss += weight * sum |img -
 * target|/N (float64, caller zeroes it; NULL to skip), exactly as
 * splat_l1_loss_grad computes them (dL_dimg bit for bit; the loss summed in
 * another order).  target and dL_dimg are [V][3][H][W] float32, mask (nullable)
 * uint8 [V][H][W].  The forward is bound by its instructions, so the extra
 * per-pixel reads and writes cost it little.
 */
SPLAT_API int splat_render_fwd_l1(const splat_plan *plan, void *ws, float *img, float *T_final, int32_t *last_pos,
                                  const float *target, const uint8_t *mask, double weight, float *dL_dimg,
                                  double *loss, void *stream);

/*
 * Backward compositing: the adjoint of Phi (Eq. 5) that carries the loss
 * gradient back to the 2-D Gaussians (end of Sec. III-B).  Every pixel walks
 * its list in reverse from last_pos, recovering T by division and the suffix
 * colour sum, and accumulates d(loss)/d(mean2d, conic, opacity, colour) of
 * every slot with wave-reduced atomics into the workspace gradient buffer,
 * which splat_render_fwd cleared: call it once per forward (a second call adds
 * to the first).  dL_dimg[V][3][H][W], T_final and last_pos are the caller's
 * (last two from splat_render_fwd).  The chunks of a split list are walked in
 * parallel, each from the checkpoint splat_render_fwd recorded, and a Gaussian
 * is evaluated only in the sub-blocks the forward blended it into: call it
 * after splat_render_fwd of the same splat_bin_sort.
 */
SPLAT_API int splat_render_bwd(const splat_plan *plan, void *ws, const float *dL_dimg, const float *T_final,
                     const int32_t *last_pos, void *stream);

/*
 * Adjoint of splat_project (end of Sec. III-B: gradients to the Gaussian
 * parameters and, through Eq. 3 and Eq. 2, to the camera pose): from the slot
 * gradients it ADDS d(loss)/d quat,
 * scale, opacity, colour and (if dmean != NULL) mean of every Gaussian
 * (float32 device planes of the parameter shapes; the caller zeroes them), and
 * ADDS d(loss)/d w2c[V][12] (float64, reduced in float64 in a fixed order, so
 * the result is deterministic; caller zeroes).  The adjoint runs in float64.
 * g, w2c and intr must be the ones given to splat_project.
 */
SPLAT_API int splat_project_bwd(const splat_plan *plan, void *ws, const splat_gaussians *g,
                      const double *w2c, const double *intr, float *dquat, float *dscale,
                      float *dopacity, float *dcolor, float *dmean, double *dw2c, void *stream);

/*
 * The L1 term of the photometric loss (paper Eq. 4) over the region of interest
 * (rows [roi_y0, H); Sec. III-C computes the losses on the bottom part of the
 * image), scaled by weight ((1 - lambda_1) in Eq. 4, 1 for the L1 loss alone):
 * with N = V*3*(H - roi_y0)*W, dL_dimg = weight * sign(img - target)/N inside the
 * region (sign(0) = 0) and 0 above it (dL_dimg is overwritten), and *loss +=
 * weight * sum |img - target|/N (float64, caller zeroes it; NULL to skip).  img,
 * target, dL_dimg are [V][3][H][W] float32 device arrays; mask (nullable) is
 * uint8 [V][H][W] and removes the pixels where it is non-zero from the sum (N is
 * unchanged).  0 <= roi_y0 < H.
 */
SPLAT_API int splat_l1_loss_grad(const float *img, const float *target, const uint8_t *mask, int32_t n_views,
                                 int32_t width, int32_t height, int32_t roi_y0, double weight, float *dL_dimg,
                                 double *loss, void *stream);

/*
 * The D-SSIM term of Eq. (4) (the structural-similarity loss of the original 3DGS
 * work): SSIM with an 11x11 Gaussian window (sigma 1.5), zero padding, per
 * channel, C1 = 0.01^2, C2 = 0.03^2, of the images cropped to the rows
 * [roi_y0, H).  ADDS weight * d(1 - mean SSIM)/d img to dL_dimg (rows >= roi_y0)
 * and weight * (1 - mean SSIM) to *loss (float64, nullable).  img, target and
 * dL_dimg are [V][3][H][W] float32 device arrays; ws is device scratch of at least
 * splat_dssim_workspace_size() bytes (three float maps of the cropped images),
 * owned by the caller.
 */
SPLAT_API size_t splat_dssim_workspace_size(int32_t n_views, int32_t width, int32_t height, int32_t roi_y0);
SPLAT_API int splat_dssim_loss_grad(const float *img, const float *target, int32_t n_views, int32_t width,
                                    int32_t height, int32_t roi_y0, double weight, void *ws, size_t ws_bytes,
                                    float *dL_dimg, double *loss, void *stream);

/*
 * splat_dssim_loss_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments and results without ws.  The three gradient maps live in a fixed
 * array inside the library that holds SPLAT_DSSIM_NOALLOC_MAX_PX pixel-channels,
 * i.e. 3 * n_views * (height - roi_y0) * width must not exceed it (192 MiB of
 * device memory, reserved on every GPU the library runs on until the process
 * ends); a larger input returns SPLAT_EINVAL and launches nothing.  The call
 * allocates nothing and calls no allocating routine; the array's device address
 * is looked up once per device, on the first call with that device current.
 * Every call on one GPU uses that GPU's one array, so calls that overlap on one
 * GPU (other streams, other threads) race and give undefined results; calls
 * ordered on one stream are safe.  Nothing of the array needs clearing: each call
 * writes every entry it reads.
 */
#define SPLAT_DSSIM_NOALLOC_MAX_PX (1 << 24)
SPLAT_API int splat_dssim_loss_grad_noalloc(const float *img, const float *target, int32_t n_views, int32_t width,
                                            int32_t height, int32_t roi_y0, double weight, float *dL_dimg,
                                            double *loss, void *stream);

/*
 * Instrumented variants of splat_render_fwd / splat_render_bwd: identical
 * outputs, plus pair counters ADDED into stats (uint64 device array, caller
 * zeroes, 8 entries): [0] forward evaluated (pixel, Gaussian) pairs, [1] forward
 * blended pairs, [2] backward evaluated pairs, [3] backward contributing pairs,
 * [4] backward wave-reduced atomic groups (9 atomics each), [5] forward
 * (Gaussian, 8x8 sub-block) evaluations of a wave (the exponent computed for its
 * 64 pixels), [6] those of them that went on to blend, [7] backward (Gaussian,
 * 8x8 sub-block) evaluations of a wave.  Used to turn kernel durations into
 * achieved work; slower than the plain calls.
 */
SPLAT_API int splat_render_fwd_stats(const splat_plan *plan, void *ws, float *img, float *T_final,
                                     int32_t *last_pos, uint64_t *stats, void *stream);
SPLAT_API int splat_render_bwd_stats(const splat_plan *plan, void *ws, const float *dL_dimg,
                                     const float *T_final, const int32_t *last_pos, uint64_t *stats,
                                     void *stream);

/*
 * The scale regulariser of Sec. III-C: lambda * sum_g ||s_g - mean(s_g)||_1 over
 * the three axes of every Gaussian (it keeps the axes of a Gaussian from drifting
 * far apart).  scale[3][n] float32 device plane (activated scales); ADDS
 * lambda * (sign(s - m) - mean of the three signs) to dscale[3][n] and the loss
 * to *loss (float64, nullable).  The mean and the signs are taken in float64.
 */
SPLAT_API int splat_scale_reg(const float *scale, int64_t n, double lambda, float *dscale, double *loss,
                              void *stream);

/*
 * Gaussian parameters from a neural field, F(X|Theta) of Sec. III-C (the model of
 * Instant-NGP with four heads).  Per Gaussian: the LiDAR position is normalised
 * into [0,1]^3 by the box [lo, hi] and clamped; level l (resolution
 * N_l = floor(n_min * b^l), b = exp(ln(n_max / n_min) / (levels - 1))) blends the
 * 8 vertices of the position's cell trilinearly, each vertex being the row
 * v0 + (N_l+1)(v1 + (N_l+1) v2) of the level's table when (N_l+1)^3 <= T, else
 * the row (v0 * 1) ^ (v1 * 2654435761) ^ (v2 * 805459861) mod T (32-bit
 * unsigned); the 2 * levels features go through an MLP 2L -> 64 -> 64 -> 11 with
 * ReLU, and the heads give colour = sigmoid(o[0:3]), opacity = sigmoid(o[3]),
 * scale = scale_max * sigmoid(o[4:7]) (below the voxel size, Sec. III-C) and
 * quaternion = o[7:11] + (1, 0, 0, 0).
 * Layout (float32 device arrays): tables[levels][T][2], w1[64][2*levels],
 * b1[64], w2[64][64], b2[64], w3[11][64], b3[11] (row-major, out x in).
 * Limits: 1 <= levels <= 16, feat = 2, hidden = 64, 4 <= log2_table <= 24,
 * 1 <= n_min <= n_max, hi > lo on every axis, scale_max > 0.
 */
typedef struct splat_ngp {
    int32_t levels, feat, log2_table, n_min, n_max, hidden;
    double scale_max;
    double lo[3], hi[3];
    const float *tables;
    const float *w1, *b1, *w2, *b2, *w3, *b3;
} splat_ngp;

/* Writes quat[4][n], scale[3][n], opacity[n], color[3][n] (the splat_gaussians
 * planes) for the n positions mean[3][n]. */
SPLAT_API int splat_ngp_fwd(const splat_ngp *m, const float *mean, int64_t n, float *quat, float *scale,
                            float *opacity, float *color, void *stream);

/* Device scratch of splat_ngp_bwd and splat_ngp_bwd_indexed for n Gaussians
 * (per-Gaussian activations and deltas, 1392 bytes each, encoding gradients,
 * 128 bytes each, the weight-gradient partials and the index reduction's
 * carries). */
SPLAT_API size_t splat_ngp_workspace_size(int64_t n);

/* Adjoint of splat_ngp_fwd: from d(loss)/d(quat, scale, opacity, color) it ADDS
 * the gradients of the tables (float atomics; order-dependent rounding) and of
 * the weights and biases (fixed-order sums).  ws is caller-owned scratch of at
 * least splat_ngp_workspace_size(n) bytes. */
SPLAT_API int splat_ngp_bwd(const splat_ngp *m, const float *mean, int64_t n, const float *dquat,
                            const float *dscale, const float *dopacity, const float *dcolor, void *ws,
                            size_t ws_bytes, float *dtables, float *dw1, float *db1, float *dw2, float *db2,
                            float *dw3, float *db3, void *stream);

/*
 * Voxel downsampling of the accumulated LiDAR cloud (Sec. III-C: one point per
 * voxel, run per stage of the coarse-to-fine schedule).  Point i (pts[3][n],
 * float32 device planes x, y, z) lies in the voxel
 *   v_d = floor((pts[d][i] - lo[d]) / voxel),  d = x, y, z  (float64 arithmetic),
 * and of every occupied voxel the point with the lowest index is kept.  keep
 * (device, >= n int32) receives the kept indices in Z-curve (Morton) order of
 * their voxels (bit b of v_x, v_y, v_z is bit 3b, 3b+1, 3b+2 of the code) and
 * *n_keep (device u32) their number.  Each v_d must lie in
 * [0, 2^21): choose lo at or below the cloud's minimum and voxel large enough;
 * a point outside (or a NaN coordinate) is clamped into the grid and
 * SPLAT_ST_RANGE is OR-ed into *status (device u32).  ws is caller-owned scratch
 * of at least splat_voxel_workspace_size(n) bytes.  Deterministic.  n = 0 only
 * zeroes *n_keep.
 */
SPLAT_API size_t splat_voxel_workspace_size(int64_t n);
SPLAT_API int splat_voxel_downsample(const float *pts, int64_t n, const double lo[3], double voxel, void *ws,
                                     size_t ws_bytes, int32_t *keep, uint32_t *n_keep, uint32_t *status,
                                     void *stream);

/*
 * Table adjoint through an inverse index.  While the Gaussian positions stay
 * fixed (a stage of the coarse-to-fine schedule, Sec. III-C), the table rows
 * every position looks up, and the trilinear weights, do not change; the index
 * lists, per level, every (Gaussian, weight) pair grouped by table row.
 * splat_ngp_bwd_indexed then forms each row's gradient as one fixed-order
 * float64 sum instead of float atomics: same result as splat_ngp_bwd up to
 * rounding, reproducible bit for bit, and no contention.
 * The index depends on mean, n and the model's levels, log2_table, n_min,
 * n_max, lo and hi (not on the tables or weights); rebuild it when any of these
 * change.  index is caller-owned device memory of splat_ngp_index_size(m, n)
 * bytes (about 64 * levels bytes per Gaussian); the build needs a scratch ws of
 * splat_ngp_index_workspace_size(m, n) bytes (about 224 * levels bytes per
 * Gaussian).  n <= 2^24.  Sizes return 0 for invalid arguments.
 */
SPLAT_API size_t splat_ngp_index_size(const splat_ngp *m, int64_t n);
SPLAT_API size_t splat_ngp_index_workspace_size(const splat_ngp *m, int64_t n);
SPLAT_API int splat_ngp_index_build(const splat_ngp *m, const float *mean, int64_t n, void *index,
                                    size_t index_bytes, void *ws, size_t ws_bytes, void *stream);

/* splat_ngp_bwd with the table gradients formed through an index built by
 * splat_ngp_index_build for the same mean, n and grid (see above).  ADDS to
 * every gradient array; ws as for splat_ngp_bwd. */
SPLAT_API int splat_ngp_bwd_indexed(const splat_ngp *m, const float *mean, int64_t n, const void *index,
                                    size_t index_bytes, const float *dquat, const float *dscale,
                                    const float *dopacity, const float *dcolor, void *ws, size_t ws_bytes,
                                    float *dtables, float *dw1, float *db1, float *dw2, float *db2, float *dw3,
                                    float *db3, void *stream);

/* Training pair.  splat_ngp_fwd_train is splat_ngp_fwd that also keeps in ws
 * (splat_ngp_workspace_size(n) bytes) what the adjoint needs: per Gaussian the
 * encoding, both hidden layers, the outputs before the heads and the ReLU
 * masks.  splat_ngp_bwd_saved is splat_ngp_bwd_indexed computed from those
 * values instead of evaluating the field again (the positions are not read);
 * it is valid only while ws, the tables and the weights are those of the last
 * splat_ngp_fwd_train call on this ws, and it overwrites the deltas in ws (the
 * forward values stay, so it may be called again). */
SPLAT_API int splat_ngp_fwd_train(const splat_ngp *m, const float *mean, int64_t n, float *quat, float *scale,
                                  float *opacity, float *color, void *ws, size_t ws_bytes, void *stream);
SPLAT_API int splat_ngp_bwd_saved(const splat_ngp *m, int64_t n, const void *index, size_t index_bytes,
                                  const float *dquat, const float *dscale, const float *dopacity,
                                  const float *dcolor, void *ws, size_t ws_bytes, float *dtables, float *dw1,
                                  float *db1, float *dw2, float *db2, float *dw3, float *db3, void *stream);

/* Text of the last synchronous error on this thread ("" if none). */
SPLAT_API const char *splat_last_error(void);

/* Library version string. */
SPLAT_API const char *splat_version(void);

/*
 * The optimiser step of the per-Gaussian parameters in the calibration loop:
 * Adam, the optimiser the paper trains with (Sec. IV-B), over up to
 * SPLAT_ADAM_MAX_GROUPS parameter arrays in one launch, fused with the
 * activation the render applies to each.  Per element of a group (float32
 * device arrays of n values; the value array holds act(param), what the render
 * read this step; act = identity uses param itself and value may be NULL):
 *   g = grad * act'(param)          sigmoid: value (1 - value); exp: value; identity: 1
 *   t = *step + 1,  m = b1 m + (1 - b1) g,  s = b2 s + (1 - b2) g^2
 *   param -= lr / (1 - b1^t) * m / (sqrt(s) / sqrt(1 - b2^t) + eps)
 *   value = act(param),  grad = 0   (ready for the next step's adjoint, which adds)
 * and then *step += 1 (a float32 device scalar shared by the groups).  lr is a
 * device scalar per group, so a captured graph replays with the caller's current
 * rates.  exp_avg and exp_avg_sq start at zero (the caller's).
 */
#define SPLAT_ADAM_MAX_GROUPS 8
#define SPLAT_ACT_IDENTITY 0
#define SPLAT_ACT_SIGMOID 1
#define SPLAT_ACT_EXP 2
typedef struct splat_adam_group {
    float *param;        /* raw parameter, updated in place            */
    float *exp_avg;      /* first moment                               */
    float *exp_avg_sq;   /* second moment                              */
    float *grad;         /* d(loss)/d(value), zeroed after the update  */
    float *value;        /* act(param), rewritten (NULL for identity)   */
    const float *lr;     /* device scalar learning rate                */
    int64_t n;
    int32_t act;         /* SPLAT_ACT_*                                */
    int32_t reserved;
} splat_adam_group;

SPLAT_API int splat_adam_step(const splat_adam_group *groups, int32_t n_groups, double beta1, double beta2,
                              double eps, float *step, void *stream);

/* sizeof of the ABI structs, for bindings to check their mirrors:
 * which = 0 splat_settings, 1 splat_gaussians, 2 splat_plan, 3 splat_ngp,
 * 4 splat_adam_group; else 0. */
SPLAT_API size_t splat_struct_size(int32_t which);

#ifdef __cplusplus
}
#endif
#endif /* SPLAT_H */
