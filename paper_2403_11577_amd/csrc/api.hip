// api.hip -- the C ABI of the splatting library: host-side argument checks, the
// workspace plan, and dispatch to the kernels.  Nothing here allocates device
// memory or synchronises; every check happens before the first launch.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>

#include "common.hpp"

namespace splat {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int launch_status(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: HIP launch failed: %s", what, hipGetErrorString(e));
        return SPLAT_ELAUNCH;
    }
    return SPLAT_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int bit_length(uint64_t x) {
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// Where the sorted instances end up: the buffer (0 or 1) after the last pass, and key_shift >= 0
// when the sorted keys are u32 (key >> key_shift).  The 64-bit instance sort narrows its keys to
// 32 bits from the first pass whose remaining digits fit 32 bits above a shift inside the depth
// field; the slot-first sort's instance keys are the tile field itself (key >> depth_bits).
static void sort_fields(const splat_plan &p, int slot_sort, int32_t *sorted_buf, int32_t *key_shift) {
    if (slot_sort) {
        *sorted_buf = ((p.tile_bits + kRadixBits - 1) / kRadixBits) & 1;
        *key_shift = p.depth_bits;
        return;
    }
    int bits = p.depth_bits + p.tile_bits;
    int passes = (bits + kRadixBits - 1) / kRadixBits;
    *sorted_buf = passes & 1;
    *key_shift = -1;
    for (int ps = 0; ps + 1 < passes; ++ps) {
        int s1 = kRadixBits * (ps + 1);
        if (s1 <= p.depth_bits && bits - s1 <= 32) {
            *key_shift = s1;
            break;
        }
    }
}

static uint32_t fbits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static bool tile_supported(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 32) || (tw == 32 && th == 16);
}

static int check_settings(const splat_settings *s) {
    if (!s) { set_error("settings is NULL"); return SPLAT_EINVAL; }
    if (!(s->near_z > 0.0) || !(s->far_z > s->near_z) || !std::isfinite(s->far_z)) {
        set_error("need 0 < near_z < far_z < inf (got %g, %g)", s->near_z, s->far_z); return SPLAT_EINVAL;
    }
    if (!(s->alpha_min > 0.0 && s->alpha_min < 1.0) || !(s->alpha_max > s->alpha_min && s->alpha_max < 1.0)) {
        set_error("need 0 < alpha_min < alpha_max < 1 (got %g, %g)", s->alpha_min, s->alpha_max); return SPLAT_EINVAL;
    }
    if (!(s->t_min > 0.0 && s->t_min < 1.0)) { set_error("need 0 < t_min < 1 (got %g)", s->t_min); return SPLAT_EINVAL; }
    if (!(s->eps2d >= 0.0) || !(s->guard >= 0.0) || !(s->pad_px >= 0.0) || !(s->pad_rel >= 0.0)) {
        set_error("eps2d, guard, pad_px and pad_rel must be >= 0"); return SPLAT_EINVAL;
    }
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(s->bg[i])) { set_error("background must be finite"); return SPLAT_EINVAL; }
    if (!tile_supported(s->tile_w, s->tile_h)) {
        set_error("unsupported tile %dx%d (8x8, 16x16, 16x32, 32x16)", s->tile_w, s->tile_h); return SPLAT_EINVAL;
    }
    if (s->batch != 32 && s->batch != 64 && s->batch != 128 && s->batch != 256) {
        set_error("batch must be 32, 64, 128 or 256 (got %d)", s->batch); return SPLAT_EINVAL;
    }
    if (s->persistent != 0 && s->persistent != 1) { set_error("persistent must be 0 or 1"); return SPLAT_EINVAL; }
    if (s->roi_y0 < 0) { set_error("roi_y0 must be >= 0 (got %d)", s->roi_y0); return SPLAT_EINVAL; }
    if (s->split_len != 0 && (s->split_len < 64 || s->split_len > (1 << 24) || (s->split_len & (s->split_len - 1)))) {
        set_error("split_len must be 0 or a power of two in [64, 2^24] (got %d)", s->split_len); return SPLAT_EINVAL;
    }
    if (s->split_fwd != 0 && s->split_fwd != 1) { set_error("split_fwd must be 0 or 1"); return SPLAT_EINVAL; }
    return SPLAT_OK;
}

static int check_plan(const splat_plan *p, const void *ws, const char *who) {
    if (!p) { set_error("%s: plan is NULL", who); return SPLAT_EINVAL; }
    if (!ws) { set_error("%s: workspace is NULL", who); return SPLAT_EINVAL; }
    if (p->n_views < 1 || p->ws_bytes == 0 || p->tiles_per_view < 1 || check_settings(&p->s)) {
        set_error("%s: plan is not initialised by splat_plan_make", who); return SPLAT_EINVAL;
    }
    // the chunking of long lists assumes whole 64-instance batches and capacities that cover the
    // tiles (a changed split_len needs a new plan: the checkpoint capacity depends on it)
    const int64_t ntiles = (int64_t)p->n_views * p->tiles_per_view;
    if (p->split_len < 64 || p->split_len > (1 << 24) || (p->split_len & (p->split_len - 1)) ||
        p->chk_cap != 2 * ((p->inst_cap + p->split_len - 1) / p->split_len) + 1 || p->bq_cap != ntiles + p->chk_cap) {
        set_error("%s: plan's split fields are inconsistent (make a new plan instead of editing them)", who);
        return SPLAT_EINVAL;
    }
    // the slot-first sort may be switched off (the 64-bit instance sort needs nothing extra), with
    // sorted_buf and key_shift set to match; it may not be switched on where the payload does not fit
    int32_t sb = 0, ks = 0;
    bool fits = p->pack_bits[0] >= (p->slot_cap > 1 ? bit_length((uint64_t)(p->slot_cap - 1)) : 1) &&
                p->pack_bits[1] >= bit_length((uint64_t)(p->tiles_x - 1)) &&
                p->pack_bits[2] >= bit_length((uint64_t)(p->tiles_y - 1)) &&
                p->pack_bits[0] + p->tile_bits + p->pack_bits[1] + p->pack_bits[2] <= 64;
    if (p->slot_sort == 0 || p->slot_sort == 1) sort_fields(*p, p->slot_sort, &sb, &ks);
    if ((p->slot_sort != 0 && p->slot_sort != 1) || (p->slot_sort == 1 && !fits) || p->sorted_buf != sb ||
        p->key_shift != ks) {
        set_error("%s: plan's sort fields are inconsistent (slot_sort %d, sorted_buf %d, key_shift %d)", who,
                  p->slot_sort, p->sorted_buf, p->key_shift);
        return SPLAT_EINVAL;
    }
    return SPLAT_OK;
}

static int check_gauss(const splat_gaussians *g, const splat_plan *p, const char *who) {
    if (!g) { set_error("%s: gaussians is NULL", who); return SPLAT_EINVAL; }
    if (g->n != p->n_gauss) {
        set_error("%s: %lld Gaussians but the plan was made for %lld", who, (long long)g->n, (long long)p->n_gauss);
        return SPLAT_EINVAL;
    }
    if (g->n > 0 && (!g->mean || !g->quat || !g->scale || !g->opacity || !g->color)) {
        set_error("%s: a Gaussian parameter plane is NULL", who); return SPLAT_EINVAL;
    }
    return SPLAT_OK;
}

static int check_pose_args(int32_t K, const double *kt, const double *kq, const double *kp, int32_t C,
                           const double *R0, const double *t0, const double *xi, const double *delta,
                           int32_t V, const int32_t *vcam, const double *vt, const char *who) {
    if (K < 2) { set_error("%s: need at least 2 trajectory knots (got %d)", who, K); return SPLAT_EINVAL; }
    if (C < 1 || V < 1) { set_error("%s: need C >= 1 and V >= 1 (got %d, %d)", who, C, V); return SPLAT_EINVAL; }
    if (!kt || !kq || !kp || !R0 || !t0 || !xi || !delta || !vcam || !vt) {
        set_error("%s: NULL pointer argument", who); return SPLAT_EINVAL;
    }
    return SPLAT_OK;
}

}  // namespace splat

using namespace splat;

extern "C" {

const char *splat_last_error(void) { return g_err; }

const char *splat_version(void) { return "splat-gfx950 0.1"; }

size_t splat_struct_size(int32_t which) {
    switch (which) {
        case 0: return sizeof(splat_settings);
        case 1: return sizeof(splat_gaussians);
        case 2: return sizeof(splat_plan);
        case 3: return sizeof(splat_ngp);
        case 4: return sizeof(splat_adam_group);
        default: return 0;
    }
}

void splat_default_settings(splat_settings *s) {
    if (!s) return;
    s->near_z = 0.2;
    s->far_z = 256.0;
    s->eps2d = 0.3;
    s->alpha_min = 1.0 / 255.0;
    s->alpha_max = 0.99;
    s->t_min = 1e-4;
    s->guard = 0.15;
    s->bg[0] = s->bg[1] = s->bg[2] = 0.0;
    s->pad_px = 0.1;
    s->pad_rel = 1e-4;
    s->tile_w = 16;
    s->tile_h = 16;
    s->batch = 64;
    s->persistent = 1;
    s->roi_y0 = 0;
    s->split_len = 0;
    s->split_fwd = 0;
    s->reserved0 = 0;
}

int splat_plan_make(const splat_settings *s, int32_t n_views, int64_t n_gauss, int32_t width, int32_t height,
                    int64_t slot_cap, int64_t inst_cap, splat_plan *plan) {
    g_err[0] = 0;
    if (!plan) { set_error("plan is NULL"); return SPLAT_EINVAL; }
    int rc = check_settings(s);
    if (rc) return rc;
    if (n_views < 1 || n_views > 1023) { set_error("n_views must be in [1, 1023] (got %d)", n_views); return SPLAT_EINVAL; }
    if (n_gauss < 0 || n_gauss >= ((int64_t)1 << 31)) { set_error("n_gauss must be in [0, 2^31)"); return SPLAT_EINVAL; }
    if (width < 1 || height < 1 || width > 16384 || height > 16384) {
        set_error("image size %dx%d outside [1, 16384]", width, height); return SPLAT_EINVAL;
    }
    if (s->roi_y0 >= height) { set_error("roi_y0 %d must be below the image height %d", s->roi_y0, height); return SPLAT_EINVAL; }
    if (slot_cap < 1 || slot_cap >= ((int64_t)1 << 31) || inst_cap < 1 || inst_cap >= ((int64_t)1 << 31)) {
        set_error("capacities must be in [1, 2^31) (got %lld, %lld)", (long long)slot_cap, (long long)inst_cap);
        return SPLAT_EINVAL;
    }
    splat_plan p;
    memset(&p, 0, sizeof p);
    p.s = *s;
    p.n_views = n_views;
    p.width = width;
    p.height = height;
    p.tiles_x = (width + s->tile_w - 1) / s->tile_w;
    p.tiles_y = (height + s->tile_h - 1) / s->tile_h;
    p.tiles_per_view = p.tiles_x * p.tiles_y;
    if (p.tiles_x > 65535 || p.tiles_y > 65535) { set_error("too many tiles"); return SPLAT_EUNSUPPORTED; }
    uint32_t nb = fbits((float)s->near_z), fb = fbits((float)s->far_z);
    if (!(fb > nb)) { set_error("far_z and near_z round to the same float"); return SPLAT_EINVAL; }
    p.depth_bits = bit_length(fb - nb);
    uint64_t ntiles_all = (uint64_t)n_views * (uint64_t)p.tiles_per_view;
    p.tile_bits = ntiles_all > 1 ? bit_length(ntiles_all - 1) : 1;
    if (p.depth_bits + p.tile_bits > 64) {
        set_error("sort key needs %d + %d bits > 64", p.tile_bits, p.depth_bits); return SPLAT_EUNSUPPORTED;
    }
    if (ntiles_all >= ((uint64_t)1 << 31)) { set_error("too many (view, tile) items"); return SPLAT_EUNSUPPORTED; }
    p.n_blocks_proj = (int32_t)((n_gauss + 255) / 256);
    if (p.n_blocks_proj < 1) p.n_blocks_proj = 1;
    int64_t nsb = (inst_cap + 8191) / 8192;
    p.n_sort_blocks = (int32_t)(nsb < 1 ? 1 : (nsb > 2048 ? 2048 : nsb));
    p.n_gauss = n_gauss;
    p.slot_cap = slot_cap;
    p.inst_cap = inst_cap;
    p.radix_bits = kRadixBits;
    // the slot-first sort packs (slot, first tile, rect width - 1, rect height - 1) into 64 bits
    p.pack_bits[0] = slot_cap > 1 ? bit_length((uint64_t)(slot_cap - 1)) : 1;
    p.pack_bits[1] = bit_length((uint64_t)(p.tiles_x - 1));
    p.pack_bits[2] = bit_length((uint64_t)(p.tiles_y - 1));
    p.slot_sort = p.pack_bits[0] + p.tile_bits + p.pack_bits[1] + p.pack_bits[2] <= 64 ? 1 : 0;
    sort_fields(p, p.slot_sort, &p.sorted_buf, &p.key_shift);

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + (bytes ? bytes : 1));
        return o;
    };
    int64_t nproj = (int64_t)n_views * p.n_blocks_proj * 4 + 1;
    size_t nparts = scan_partials(slot_cap + 1);
    size_t np2 = scan_partials(nproj);
    size_t np3 = scan_partials((int64_t)kRadixDigits * p.n_sort_blocks);
    if (np2 > nparts) nparts = np2;
    if (np3 > nparts) nparts = np3;
    size_t np4 = scan_partials((int64_t)n_views * p.tiles_per_view + 1);
    if (np4 > nparts) nparts = np4;
    p.off_status = take(4);
    p.off_counts = take(8 * 4);
    p.off_view_off = take((size_t)(n_views + 1) * 4);
    p.off_blockcnt = take((size_t)nproj * 4);
    p.off_rec = take((size_t)slot_cap * 48);
    p.off_meta = take((size_t)slot_cap * 8);
    p.off_rect = take((size_t)slot_cap * 8);
    p.off_ntiles = take((size_t)(slot_cap + 1) * 4);
    p.off_keys = take((size_t)inst_cap * 16);
    p.off_vals = take((size_t)inst_cap * 8);
    p.off_ranges = take((size_t)ntiles_all * 8);
    p.off_queue = take((size_t)ntiles_all * 4);
    p.off_hist = take(((size_t)kRadixDigits * p.n_sort_blocks + 1 + 128) * 4);
    p.off_scan = take(nparts * 4);
    p.off_grad2d = take((size_t)slot_cap * 36);
    p.off_visbits = take((size_t)n_views * p.n_blocks_proj * 4 * 8);
    p.off_dwpart = take((size_t)n_views * (p.n_blocks_proj * 4 + kDw2cStages) * 12 * 8);  // + the stage sums
    p.off_cam = take((size_t)n_views * kCamBytes);
    // render-adjoint work items: a list of L >= split_len instances becomes ceil(L / split_len) <=
    // 2 L / split_len chunks, so the split lists need fewer than 2 inst_cap / split_len chunks
    p.split_len = s->split_len ? s->split_len : 1024;
    p.chk_cap = 2 * ((inst_cap + p.split_len - 1) / p.split_len) + 1;
    p.bq_cap = (int64_t)ntiles_all + p.chk_cap;
    p.off_bqueue = take((size_t)p.bq_cap * 16);
    p.off_bqoff = take(((size_t)ntiles_all + 1) * 4);
    p.off_chk = take((size_t)p.chk_cap * (size_t)(s->tile_w * s->tile_h) * 16);
    p.off_chklast = take((size_t)p.chk_cap * (size_t)(s->tile_w * s->tile_h) * 4);
    p.off_bmask = take((size_t)inst_cap);
    p.off_dkey = take((size_t)slot_cap * 4);
    p.off_spay = take(p.slot_sort ? (size_t)slot_cap * 16 : 0);
    p.off_skeys = take(p.slot_sort ? (size_t)slot_cap * 4 : 0);
    p.off_soff = take(p.slot_sort ? (size_t)((slot_cap + 63) / 64 + 1) * 4 : 0);
    p.off_l1part = take(((size_t)ntiles_all + (ntiles_all + kL1Span - 1) / kL1Span) * 8);
    p.ws_bytes = off;
    *plan = p;
    return SPLAT_OK;
}

int splat_pose_interp_fwd(int32_t K, const double *knot_t, const double *knot_q, const double *knot_p, int32_t C,
                          const double *R0, const double *t0, const double *xi, const double *delta, int32_t V,
                          const int32_t *view_cam, const double *view_t, double *w2c, uint32_t *status,
                          void *stream) {
    g_err[0] = 0;
    int rc = check_pose_args(K, knot_t, knot_q, knot_p, C, R0, t0, xi, delta, V, view_cam, view_t, "pose_interp_fwd");
    if (rc) return rc;
    if (!w2c) { set_error("pose_interp_fwd: w2c is NULL"); return SPLAT_EINVAL; }
    return launch_pose_fwd(K, knot_t, knot_q, knot_p, C, R0, t0, xi, delta, V, view_cam, view_t, w2c, status,
                           (hipStream_t)stream);
}

int splat_pose_interp_bwd(int32_t K, const double *knot_t, const double *knot_q, const double *knot_p, int32_t C,
                          const double *R0, const double *t0, const double *xi, const double *delta, int32_t V,
                          const int32_t *view_cam, const double *view_t, const double *dw2c, double *dxi,
                          double *ddelta, void *stream) {
    g_err[0] = 0;
    int rc = check_pose_args(K, knot_t, knot_q, knot_p, C, R0, t0, xi, delta, V, view_cam, view_t, "pose_interp_bwd");
    if (rc) return rc;
    if (!dw2c || !dxi || !ddelta) { set_error("pose_interp_bwd: NULL gradient pointer"); return SPLAT_EINVAL; }
    return launch_pose_bwd(K, knot_t, knot_q, knot_p, C, R0, t0, xi, delta, V, view_cam, view_t, dw2c, dxi, ddelta,
                           (hipStream_t)stream);
}

int splat_project(const splat_plan *plan, void *ws, const splat_gaussians *g, const double *w2c, const double *intr,
                  void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "project");
    if (rc) return rc;
    if ((rc = check_gauss(g, plan, "project"))) return rc;
    if (!w2c || !intr) { set_error("project: w2c or intr is NULL"); return SPLAT_EINVAL; }
    return launch_project(*plan, ws, *g, w2c, intr, (hipStream_t)stream);
}

int splat_slot_meta(const splat_plan *plan, void *ws, void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "slot_meta");
    if (rc) return rc;
    return launch_slot_meta(*plan, ws, (hipStream_t)stream);
}

int splat_bin_sort(const splat_plan *plan, void *ws, void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "bin_sort");
    if (rc) return rc;
    return launch_bin_sort(*plan, ws, (hipStream_t)stream);
}

int splat_render_fwd(const splat_plan *plan, void *ws, float *img, float *T_final, int32_t *last_pos, void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "render_fwd");
    if (rc) return rc;
    if (!img || !T_final || !last_pos) { set_error("render_fwd: NULL output"); return SPLAT_EINVAL; }
    return launch_render_fwd(*plan, ws, img, T_final, last_pos, nullptr, (hipStream_t)stream);
}

int splat_render_fwd_l1(const splat_plan *plan, void *ws, float *img, float *T_final, int32_t *last_pos,
                        const float *target, const uint8_t *mask, double weight, float *dL_dimg, double *loss,
                        void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "render_fwd_l1");
    if (rc) return rc;
    if (!img || !T_final || !last_pos || !target || !dL_dimg) {
        set_error("render_fwd_l1: NULL argument"); return SPLAT_EINVAL;
    }
    if (plan->s.roi_y0 >= plan->height) {
        set_error("render_fwd_l1: roi_y0 %d leaves no rows of %d", plan->s.roi_y0, plan->height); return SPLAT_EINVAL;
    }
    if (!std::isfinite(weight)) { set_error("render_fwd_l1: weight must be finite"); return SPLAT_EINVAL; }
    const double inv_n = weight / (3.0 * (double)plan->n_views * (double)plan->width *
                                   (double)(plan->height - plan->s.roi_y0));
    const L1Fuse l1{target, mask, dL_dimg, loss, inv_n};
    return launch_render_fwd(*plan, ws, img, T_final, last_pos, nullptr, (hipStream_t)stream, &l1);
}

int splat_render_fwd_stats(const splat_plan *plan, void *ws, float *img, float *T_final, int32_t *last_pos,
                           uint64_t *stats, void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "render_fwd_stats");
    if (rc) return rc;
    if (!img || !T_final || !last_pos || !stats) { set_error("render_fwd_stats: NULL argument"); return SPLAT_EINVAL; }
    return launch_render_fwd(*plan, ws, img, T_final, last_pos, stats, (hipStream_t)stream);
}

int splat_l1_loss_grad(const float *img, const float *target, const uint8_t *mask, int32_t n_views, int32_t width,
                       int32_t height, int32_t roi_y0, double weight, float *dL_dimg, double *loss, void *stream) {
    g_err[0] = 0;
    if (!img || !target || !dL_dimg) { set_error("l1_loss_grad: NULL argument"); return SPLAT_EINVAL; }
    if (n_views < 1 || width < 1 || height < 1) { set_error("l1_loss_grad: bad shape"); return SPLAT_EINVAL; }
    if (roi_y0 < 0 || roi_y0 >= height) { set_error("l1_loss_grad: roi_y0 %d outside [0, %d)", roi_y0, height); return SPLAT_EINVAL; }
    if (!std::isfinite(weight)) { set_error("l1_loss_grad: weight must be finite"); return SPLAT_EINVAL; }
    double inv_n = weight / (3.0 * (double)n_views * (double)width * (double)(height - roi_y0));
    return launch_l1(img, target, mask, n_views, width, height, roi_y0, inv_n, dL_dimg, loss, (hipStream_t)stream);
}

size_t splat_dssim_workspace_size(int32_t n_views, int32_t width, int32_t height, int32_t roi_y0) {
    if (n_views < 1 || width < 1 || height < 1 || roi_y0 < 0 || roi_y0 >= height) return 0;
    return dssim_ws_bytes(n_views, width, height, roi_y0);
}

int splat_dssim_loss_grad(const float *img, const float *target, int32_t n_views, int32_t width, int32_t height,
                          int32_t roi_y0, double weight, void *ws, size_t ws_bytes, float *dL_dimg, double *loss,
                          void *stream) {
    g_err[0] = 0;
    if (!img || !target || !dL_dimg || !ws) { set_error("dssim_loss_grad: NULL argument"); return SPLAT_EINVAL; }
    if (n_views < 1 || n_views > 21845 || width < 1 || height < 1) { set_error("dssim_loss_grad: bad shape"); return SPLAT_EINVAL; }
    if (roi_y0 < 0 || roi_y0 >= height) { set_error("dssim_loss_grad: roi_y0 %d outside [0, %d)", roi_y0, height); return SPLAT_EINVAL; }
    if (!std::isfinite(weight)) { set_error("dssim_loss_grad: weight must be finite"); return SPLAT_EINVAL; }
    size_t need = dssim_ws_bytes(n_views, width, height, roi_y0);
    if (ws_bytes < need) {
        set_error("dssim_loss_grad: workspace of %zu bytes, %zu needed", ws_bytes, need); return SPLAT_EINVAL;
    }
    return launch_dssim(img, target, n_views, width, height, roi_y0, weight, ws, dL_dimg, loss, (hipStream_t)stream);
}

int splat_dssim_loss_grad_noalloc(const float *img, const float *target, int32_t n_views, int32_t width,
                                  int32_t height, int32_t roi_y0, double weight, float *dL_dimg, double *loss,
                                  void *stream) {
    g_err[0] = 0;
    if (!img || !target || !dL_dimg) { set_error("dssim_loss_grad_noalloc: NULL argument"); return SPLAT_EINVAL; }
    if (n_views < 1 || width < 1 || height < 1) { set_error("dssim_loss_grad_noalloc: bad shape"); return SPLAT_EINVAL; }
    if (roi_y0 < 0 || roi_y0 >= height) {
        set_error("dssim_loss_grad_noalloc: roi_y0 %d outside [0, %d)", roi_y0, height); return SPLAT_EINVAL;
    }
    if (!std::isfinite(weight)) { set_error("dssim_loss_grad_noalloc: weight must be finite"); return SPLAT_EINVAL; }
    const int64_t px = 3 * (int64_t)n_views * (int64_t)(height - roi_y0) * (int64_t)width;
    if (px > (int64_t)SPLAT_DSSIM_NOALLOC_MAX_PX) {
        set_error("dssim_loss_grad_noalloc: %lld pixel-channels exceed the maximum of %lld "
                  "(use splat_dssim_loss_grad with a workspace)", (long long)px, (long long)SPLAT_DSSIM_NOALLOC_MAX_PX);
        return SPLAT_EINVAL;
    }
    float *G = nullptr;
    int rc = dssim_scratch(&G);
    if (rc) return rc;
    return launch_dssim(img, target, n_views, width, height, roi_y0, weight, G, dL_dimg, loss, (hipStream_t)stream);
}

int splat_scale_reg(const float *scale, int64_t n, double lambda, float *dscale, double *loss, void *stream) {
    g_err[0] = 0;
    if (n < 0) { set_error("scale_reg: n must be >= 0"); return SPLAT_EINVAL; }
    if (n == 0) return SPLAT_OK;
    if (!scale || !dscale) { set_error("scale_reg: NULL argument"); return SPLAT_EINVAL; }
    if (!std::isfinite(lambda)) { set_error("scale_reg: lambda must be finite"); return SPLAT_EINVAL; }
    return launch_scale_reg(scale, n, lambda, dscale, loss, (hipStream_t)stream);
}

int splat_adam_step(const splat_adam_group *groups, int32_t n_groups, double beta1, double beta2, double eps,
                    float *step, void *stream) {
    g_err[0] = 0;
    if (!groups || !step) { set_error("adam_step: NULL argument"); return SPLAT_EINVAL; }
    if (n_groups < 1 || n_groups > SPLAT_ADAM_MAX_GROUPS) {
        set_error("adam_step: n_groups must be in [1, %d] (got %d)", SPLAT_ADAM_MAX_GROUPS, n_groups);
        return SPLAT_EINVAL;
    }
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.0) || !std::isfinite(eps)) {
        set_error("adam_step: need 0 <= beta1, beta2 < 1 and 0 <= eps < inf"); return SPLAT_EINVAL;
    }
    for (int i = 0; i < n_groups; ++i) {
        const splat_adam_group &g = groups[i];
        if (g.n < 0 || g.n >= ((int64_t)1 << 40)) { set_error("adam_step: group %d has n = %lld", i, (long long)g.n); return SPLAT_EINVAL; }
        if (g.act < SPLAT_ACT_IDENTITY || g.act > SPLAT_ACT_EXP) {
            set_error("adam_step: group %d has an unknown activation %d", i, g.act); return SPLAT_EINVAL;
        }
        if (g.n > 0 && (!g.param || !g.exp_avg || !g.exp_avg_sq || !g.grad || !g.lr ||
                        (g.act != SPLAT_ACT_IDENTITY && !g.value))) {
            set_error("adam_step: group %d has a NULL array", i); return SPLAT_EINVAL;
        }
    }
    return launch_adam(groups, n_groups, beta1, beta2, eps, step, (hipStream_t)stream);
}

int splat_render_bwd(const splat_plan *plan, void *ws, const float *dL_dimg, const float *T_final,
                     const int32_t *last_pos, void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "render_bwd");
    if (rc) return rc;
    if (!dL_dimg || !T_final || !last_pos) { set_error("render_bwd: NULL input"); return SPLAT_EINVAL; }
    return launch_render_bwd(*plan, ws, dL_dimg, T_final, last_pos, nullptr, (hipStream_t)stream);
}

int splat_render_bwd_stats(const splat_plan *plan, void *ws, const float *dL_dimg, const float *T_final,
                           const int32_t *last_pos, uint64_t *stats, void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "render_bwd_stats");
    if (rc) return rc;
    if (!dL_dimg || !T_final || !last_pos || !stats) { set_error("render_bwd_stats: NULL argument"); return SPLAT_EINVAL; }
    return launch_render_bwd(*plan, ws, dL_dimg, T_final, last_pos, stats, (hipStream_t)stream);
}

int splat_project_bwd(const splat_plan *plan, void *ws, const splat_gaussians *g, const double *w2c,
                      const double *intr, float *dquat, float *dscale, float *dopacity, float *dcolor, float *dmean,
                      double *dw2c, void *stream) {
    g_err[0] = 0;
    int rc = check_plan(plan, ws, "project_bwd");
    if (rc) return rc;
    if ((rc = check_gauss(g, plan, "project_bwd"))) return rc;
    if (!w2c || !intr || !dquat || !dscale || !dopacity || !dcolor || !dw2c) {
        set_error("project_bwd: NULL argument"); return SPLAT_EINVAL;
    }
    return launch_project_bwd(*plan, ws, *g, w2c, intr, dquat, dscale, dopacity, dcolor, dmean, dw2c,
                              (hipStream_t)stream);
}


static int check_ngp(const splat_ngp *m, const char *who) {
    if (!m) { set_error("%s: model is NULL", who); return SPLAT_EINVAL; }
    if (m->levels < 1 || m->levels > 16 || m->feat != 2 || m->hidden != 64) {
        set_error("%s: need 1 <= levels <= 16, feat = 2, hidden = 64 (got %d, %d, %d)", who, m->levels, m->feat,
                  m->hidden);
        return SPLAT_EUNSUPPORTED;
    }
    if (m->log2_table < 4 || m->log2_table > 24) { set_error("%s: log2_table outside [4, 24]", who); return SPLAT_EINVAL; }
    if (m->n_min < 1 || m->n_max < m->n_min) { set_error("%s: need 1 <= n_min <= n_max", who); return SPLAT_EINVAL; }
    for (int d = 0; d < 3; ++d)
        if (!(m->hi[d] > m->lo[d]) || !std::isfinite(m->lo[d]) || !std::isfinite(m->hi[d])) {
            set_error("%s: the box needs finite hi > lo on every axis", who); return SPLAT_EINVAL;
        }
    if (!(m->scale_max > 0.0)) { set_error("%s: scale_max must be > 0", who); return SPLAT_EINVAL; }
    if (!m->tables || !m->w1 || !m->b1 || !m->w2 || !m->b2 || !m->w3 || !m->b3) {
        set_error("%s: NULL model array", who); return SPLAT_EINVAL;
    }
    return SPLAT_OK;
}

int splat_ngp_fwd(const splat_ngp *m, const float *mean, int64_t n, float *quat, float *scale, float *opacity,
                  float *color, void *stream) {
    g_err[0] = 0;
    int rc = check_ngp(m, "ngp_fwd");
    if (rc) return rc;
    if (n < 0 || n >= ((int64_t)1 << 31)) { set_error("ngp_fwd: n outside [0, 2^31)"); return SPLAT_EINVAL; }
    if (n == 0) return SPLAT_OK;
    if (!mean || !quat || !scale || !opacity || !color) { set_error("ngp_fwd: NULL argument"); return SPLAT_EINVAL; }
    return launch_ngp_fwd(*m, mean, n, quat, scale, opacity, color, (hipStream_t)stream);
}

size_t splat_ngp_workspace_size(int64_t n) { return n < 0 ? 0 : ngp_ws_bytes(n); }

int splat_ngp_bwd(const splat_ngp *m, const float *mean, int64_t n, const float *dquat, const float *dscale,
                  const float *dopacity, const float *dcolor, void *ws, size_t ws_bytes, float *dtables, float *dw1,
                  float *db1, float *dw2, float *db2, float *dw3, float *db3, void *stream) {
    g_err[0] = 0;
    int rc = check_ngp(m, "ngp_bwd");
    if (rc) return rc;
    if (n < 0 || n >= ((int64_t)1 << 31)) { set_error("ngp_bwd: n outside [0, 2^31)"); return SPLAT_EINVAL; }
    if (n == 0) return SPLAT_OK;
    if (!mean || !dquat || !dscale || !dopacity || !dcolor || !ws || !dtables || !dw1 || !db1 || !dw2 || !db2 ||
        !dw3 || !db3) {
        set_error("ngp_bwd: NULL argument"); return SPLAT_EINVAL;
    }
    size_t need = ngp_ws_bytes(n);
    if (ws_bytes < need) { set_error("ngp_bwd: workspace of %zu bytes, %zu needed", ws_bytes, need); return SPLAT_EINVAL; }
    return launch_ngp_bwd(*m, mean, n, dquat, dscale, dopacity, dcolor, ws, dtables, dw1, db1, dw2, db2, dw3, db3,
                          (hipStream_t)stream);
}

static int check_ngp_index(const splat_ngp *m, int64_t n, const char *who) {
    int rc = check_ngp(m, who);
    if (rc) return rc;
    if (n < 0 || n > ((int64_t)1 << 24)) { set_error("%s: n outside [0, 2^24]", who); return SPLAT_EINVAL; }
    return SPLAT_OK;
}

size_t splat_ngp_index_size(const splat_ngp *m, int64_t n) {
    g_err[0] = 0;
    return check_ngp_index(m, n, "ngp_index_size") ? 0 : ngp_index_bytes(*m, n);
}

size_t splat_ngp_index_workspace_size(const splat_ngp *m, int64_t n) {
    g_err[0] = 0;
    return check_ngp_index(m, n, "ngp_index_workspace_size") ? 0 : ngp_index_ws_bytes(*m, n);
}

int splat_ngp_index_build(const splat_ngp *m, const float *mean, int64_t n, void *index, size_t index_bytes,
                          void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    int rc = check_ngp_index(m, n, "ngp_index_build");
    if (rc) return rc;
    if (n == 0) return SPLAT_OK;
    if (!mean || !index || !ws) { set_error("ngp_index_build: NULL argument"); return SPLAT_EINVAL; }
    size_t ni = ngp_index_bytes(*m, n), nw = ngp_index_ws_bytes(*m, n);
    if (index_bytes < ni) { set_error("ngp_index_build: index of %zu bytes, %zu needed", index_bytes, ni); return SPLAT_EINVAL; }
    if (ws_bytes < nw) { set_error("ngp_index_build: workspace of %zu bytes, %zu needed", ws_bytes, nw); return SPLAT_EINVAL; }
    return launch_ngp_index_build(*m, mean, n, index, ws, (hipStream_t)stream);
}

int splat_ngp_bwd_indexed(const splat_ngp *m, const float *mean, int64_t n, const void *index, size_t index_bytes,
                          const float *dquat, const float *dscale, const float *dopacity, const float *dcolor,
                          void *ws, size_t ws_bytes, float *dtables, float *dw1, float *db1, float *dw2, float *db2,
                          float *dw3, float *db3, void *stream) {
    g_err[0] = 0;
    int rc = check_ngp_index(m, n, "ngp_bwd_indexed");
    if (rc) return rc;
    if (n == 0) return SPLAT_OK;
    if (!mean || !index || !dquat || !dscale || !dopacity || !dcolor || !ws || !dtables || !dw1 || !db1 || !dw2 ||
        !db2 || !dw3 || !db3) {
        set_error("ngp_bwd_indexed: NULL argument"); return SPLAT_EINVAL;
    }
    size_t ni = ngp_index_bytes(*m, n), nw = ngp_ws_bytes(n);
    if (index_bytes < ni) { set_error("ngp_bwd_indexed: index of %zu bytes, %zu needed", index_bytes, ni); return SPLAT_EINVAL; }
    if (ws_bytes < nw) { set_error("ngp_bwd_indexed: workspace of %zu bytes, %zu needed", ws_bytes, nw); return SPLAT_EINVAL; }
    return launch_ngp_bwd_indexed(*m, mean, n, index, dquat, dscale, dopacity, dcolor, ws, dtables, dw1, db1, dw2,
                                  db2, dw3, db3, (hipStream_t)stream);
}

int splat_ngp_fwd_train(const splat_ngp *m, const float *mean, int64_t n, float *quat, float *scale,
                        float *opacity, float *color, void *ws, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    int rc = check_ngp(m, "ngp_fwd_train");
    if (rc) return rc;
    if (n < 0 || n >= ((int64_t)1 << 31)) { set_error("ngp_fwd_train: n outside [0, 2^31)"); return SPLAT_EINVAL; }
    if (n == 0) return SPLAT_OK;
    if (!mean || !quat || !scale || !opacity || !color || !ws) {
        set_error("ngp_fwd_train: NULL argument"); return SPLAT_EINVAL;
    }
    size_t need = ngp_ws_bytes(n);
    if (ws_bytes < need) { set_error("ngp_fwd_train: workspace of %zu bytes, %zu needed", ws_bytes, need); return SPLAT_EINVAL; }
    return launch_ngp_fwd_train(*m, mean, n, quat, scale, opacity, color, ws, (hipStream_t)stream);
}

int splat_ngp_bwd_saved(const splat_ngp *m, int64_t n, const void *index, size_t index_bytes, const float *dquat,
                        const float *dscale, const float *dopacity, const float *dcolor, void *ws, size_t ws_bytes,
                        float *dtables, float *dw1, float *db1, float *dw2, float *db2, float *dw3, float *db3,
                        void *stream) {
    g_err[0] = 0;
    int rc = check_ngp_index(m, n, "ngp_bwd_saved");
    if (rc) return rc;
    if (n == 0) return SPLAT_OK;
    if (!index || !dquat || !dscale || !dopacity || !dcolor || !ws || !dtables || !dw1 || !db1 || !dw2 || !db2 ||
        !dw3 || !db3) {
        set_error("ngp_bwd_saved: NULL argument"); return SPLAT_EINVAL;
    }
    size_t ni = ngp_index_bytes(*m, n), nw = ngp_ws_bytes(n);
    if (index_bytes < ni) { set_error("ngp_bwd_saved: index of %zu bytes, %zu needed", index_bytes, ni); return SPLAT_EINVAL; }
    if (ws_bytes < nw) { set_error("ngp_bwd_saved: workspace of %zu bytes, %zu needed", ws_bytes, nw); return SPLAT_EINVAL; }
    return launch_ngp_bwd_saved(*m, n, index, dquat, dscale, dopacity, dcolor, ws, dtables, dw1, db1, dw2, db2, dw3,
                                db3, (hipStream_t)stream);
}

size_t splat_voxel_workspace_size(int64_t n) { return n < 0 ? 0 : voxel_ws_bytes(n); }

int splat_voxel_downsample(const float *pts, int64_t n, const double *lo, double voxel, void *ws, size_t ws_bytes,
                           int32_t *keep, uint32_t *n_keep, uint32_t *status, void *stream) {
    g_err[0] = 0;
    if (n < 0 || n >= ((int64_t)1 << 31)) { set_error("voxel_downsample: n outside [0, 2^31)"); return SPLAT_EINVAL; }
    if (!lo || !n_keep) { set_error("voxel_downsample: NULL argument"); return SPLAT_EINVAL; }
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(lo[d])) { set_error("voxel_downsample: lo must be finite"); return SPLAT_EINVAL; }
    if (!(voxel > 0.0) || !std::isfinite(voxel)) {
        set_error("voxel_downsample: voxel size must be finite and > 0"); return SPLAT_EINVAL;
    }
    if (n == 0) return launch_fill_u32(n_keep, 0u, 1, (hipStream_t)stream);
    if (!pts || !ws || !keep || !status) { set_error("voxel_downsample: NULL argument"); return SPLAT_EINVAL; }
    size_t need = voxel_ws_bytes(n);
    if (ws_bytes < need) {
        set_error("voxel_downsample: workspace of %zu bytes, %zu needed", ws_bytes, need); return SPLAT_EINVAL;
    }
    return launch_voxel_downsample(pts, n, lo, voxel, ws, keep, n_keep, status, (hipStream_t)stream);
}

}  // extern "C"
