// C ABI of libkfvol (declared in include/kf.h): argument validation, per-frame constants,
// work decomposition, launch and graph management.  No arithmetic of the integration
// itself happens here beyond the per-frame constants of Eq. 3 and Eq. 5, which are
// composed in double precision and rounded once to single precision.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kf.h"
#include "kf_device.h"
#include "kf_launch.h"

struct kf_volume {
    kf_volume_desc desc;
    kf_volume_buffers bufs;
};

namespace {

thread_local char g_err[512] = "";

kf_status fail(kf_status s, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

kf_status hip_fail(hipError_t e, const char* what)
{
    return fail(KF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define KF_HIP(call, what)                         \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Workspaces come from the device's default stream-ordered pool.  Its default release
// threshold of 0 hands freed memory back at every synchronisation, so each call would map
// its workspace afresh; the library raises the threshold once per device so that freed
// workspaces stay in the pool for the next call (the pool grows to the largest workspace
// used and keeps it until the process ends).
hipError_t workspace_alloc(void** p, size_t bytes, hipStream_t stream)
{
    static std::mutex mu;
    static bool kept[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) {
        std::lock_guard<std::mutex> lock(mu);
        if (!kept[dev]) {
            hipMemPool_t pool;
            if ((e = hipDeviceGetDefaultMemPool(&pool, dev)) != hipSuccess) return e;
            uint64_t threshold = UINT64_MAX;
            if ((e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold)) != hipSuccess)
                return e;
            kept[dev] = true;
        }
    }
    return hipMallocAsync(p, bytes, stream);
}

// ------------------------------------------------------------------------- validation

bool finite_all(const double* p, int n)
{
    for (int q = 0; q < n; ++q)
        if (!isfinite(p[q])) return false;
    return true;
}

kf_status check_K(const double* K, const char* name)
{
    if (!K) return fail(KF_E_ARG, "%s is NULL", name);
    if (!finite_all(K, 9)) return fail(KF_E_ARG, "%s has a non-finite entry", name);
    if (K[1] != 0.0 || K[3] != 0.0 || K[6] != 0.0 || K[7] != 0.0 || K[8] != 1.0)
        return fail(KF_E_ARG, "%s must be [[fx,0,cx],[0,fy,cy],[0,0,1]]", name);
    if (!(K[0] > 0.0) || !(K[4] > 0.0)) return fail(KF_E_ARG, "%s focal lengths must be > 0", name);
    return KF_OK;
}

kf_status check_rigid(const double* T, const char* name)
{
    if (!T) return fail(KF_E_ARG, "%s is NULL", name);
    if (!finite_all(T, 16)) return fail(KF_E_ARG, "%s has a non-finite entry", name);
    if (T[12] != 0.0 || T[13] != 0.0 || T[14] != 0.0 || T[15] != 1.0)
        return fail(KF_E_ARG, "%s last row must be (0,0,0,1)", name);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += T[4 * k + r] * T[4 * k + c];
            if (fabs(s - (r == c ? 1.0 : 0.0)) > 1e-6)
                return fail(KF_E_ARG, "%s rotation is not orthonormal", name);
        }
    return KF_OK;
}

kf_status check_desc(const kf_volume_desc* d)
{
    if (!d) return fail(KF_E_ARG, "volume description is NULL");
    for (int a = 0; a < 3; ++a) {
        if (d->geom_dim[a] < 1 || d->colour_dim[a] < 1)
            return fail(KF_E_SHAPE, "volume dimensions must be >= 1");
        if (d->geom_dim[a] > 65536 || d->colour_dim[a] > 65536)
            return fail(KF_E_RANGE, "volume dimension above 65536");
        if (!isfinite(d->origin[a]) || !isfinite(d->extent[a]) || !(d->extent[a] > 0.0))
            return fail(KF_E_ARG, "origin must be finite and extent > 0");
    }
    const double ng = (double)d->geom_dim[0] * d->geom_dim[1] * d->geom_dim[2];
    const double nc = (double)d->colour_dim[0] * d->colour_dim[1] * d->colour_dim[2];
    if (ng > 2147483647.0 || nc > 2147483647.0)
        return fail(KF_E_RANGE, "a volume holds more than 2^31-1 voxels");
    if ((double)d->geom_dim[0] * d->geom_dim[1] >= 67108864.0 ||
        (double)d->colour_dim[0] * d->colour_dim[1] >= 67108864.0)
        return fail(KF_E_RANGE, "a z slice holds 2^26 voxels or more");
    if (!isfinite(d->colour_band) || !(d->colour_band > 0.0))
        return fail(KF_E_ARG, "colour_band must be finite and > 0");
    if (!isfinite(d->colour_gate) || d->colour_gate < 0.0)
        return fail(KF_E_ARG, "colour_gate must be finite and >= 0");
    if (d->hd_sampling != KF_HD_BILINEAR && d->hd_sampling != KF_HD_NEAREST)
        return fail(KF_E_ARG, "hd_sampling must be KF_HD_BILINEAR or KF_HD_NEAREST");
    return KF_OK;
}

kf_status check_images(const float* depth, int32_t dw, int32_t dh, const void* rgb,
                       int32_t fmt, int32_t cw, int32_t ch)
{
    if (dw < 1 || dh < 1) return fail(KF_E_SHAPE, "depth image must be at least 1x1");
    if (cw < 2 || ch < 2) return fail(KF_E_SHAPE, "HD image must be at least 2x2");
    // the 16-byte pixel map of a depth image is read through a buffer resource whose
    // byte offsets stay below 2^31 - 16 (the out-of-image marker)
    if (dw > 65535 || dh > 65535 || (double)dw * dh * 16.0 >= 2147483632.0 ||
        (double)cw * ch * 3.0 > 2147483647.0)
        return fail(KF_E_RANGE, "image too large");
    if (fmt != KF_RGB8 && fmt != KF_RGBF32) return fail(KF_E_ARG, "unknown pixel format");
    if (!depth || !rgb) return fail(KF_E_ARG, "image pointer is NULL");
    return KF_OK;
}

kf_status check_scalars(double trunc_m, double w_max)
{
    if (!isfinite(trunc_m) || !(trunc_m > 0.0)) return fail(KF_E_ARG, "trunc_m must be finite and > 0");
    if (!isfinite(w_max) || !(w_max >= 1.0)) return fail(KF_E_ARG, "w_max must be finite and >= 1");
    return KF_OK;
}

kf_status check_volume(const kf_volume* v)
{
    if (!v) return fail(KF_E_ARG, "volume handle is NULL");
    return KF_OK;
}

// ------------------------------------------------------------------ per-frame constants

// Voxel index -> R (origin + (idx + 1/2) s) + t as A idx + b, A = R diag(s); double.
void fold(const double R[9], const double t[3], const double origin[3], const double s[3],
          double A[9], double b[3])
{
    const double c0 = origin[0] + 0.5 * s[0];
    const double c1 = origin[1] + 0.5 * s[1];
    const double c2 = origin[2] + 0.5 * s[2];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) A[3 * r + c] = R[3 * r + c] * s[c];
        b[r] = ((R[3 * r + 0] * c0 + R[3 * r + 1] * c1) + R[3 * r + 2] * c2) + t[r];
    }
}

void frame_consts(const kf_volume_desc& vd, const double* K_d, const double* K_rgb,
                  const double* T_rd, const double* T_wc, double trunc_m, double w_max,
                  const float* depth, int32_t dw, int32_t dh, const void* rgb, int32_t cw,
                  int32_t ch, kf::FrameConsts* out)
{
    // (R_n, t_n) of Eq. 5: world -> current depth camera, the inverse of the pose.
    double Rcw[9], tcw[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) Rcw[3 * r + c] = T_wc[4 * c + r];
        tcw[r] = -((T_wc[0 * 4 + r] * T_wc[3] + T_wc[1 * 4 + r] * T_wc[7]) + T_wc[2 * 4 + r] * T_wc[11]);
    }
    // Eq. 3 composed with Eq. 5: world -> HD camera.
    double Rhw[9], thw[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            Rhw[3 * r + c] = (T_rd[4 * r + 0] * Rcw[0 + c] + T_rd[4 * r + 1] * Rcw[3 + c])
                             + T_rd[4 * r + 2] * Rcw[6 + c];
        thw[r] = ((T_rd[4 * r + 0] * tcw[0] + T_rd[4 * r + 1] * tcw[1]) + T_rd[4 * r + 2] * tcw[2])
                 + T_rd[4 * r + 3];
    }
    double sg[3], sc[3];
    for (int a = 0; a < 3; ++a) {
        sg[a] = vd.extent[a] / (double)vd.geom_dim[a];
        sc[a] = vd.extent[a] / (double)vd.colour_dim[a];
    }
    double Ag[9], bg[3], Ac[9], bc[3], Ah[9], bh[3];
    fold(Rcw, tcw, vd.origin, sg, Ag, bg);
    fold(Rcw, tcw, vd.origin, sc, Ac, bc);
    fold(Rhw, thw, vd.origin, sc, Ah, bh);
    for (int q = 0; q < 9; ++q) {
        out->Ag[q] = (float)Ag[q];
        out->Ac[q] = (float)Ac[q];
        out->Ah[q] = (float)Ah[q];
    }
    for (int q = 0; q < 3; ++q) {
        out->bg[q] = (float)bg[q];
        out->bc[q] = (float)bc[q];
        out->bh[q] = (float)bh[q];
    }
    out->fx = (float)K_d[0];
    out->fy = (float)K_d[4];
    out->cx = (float)K_d[2];
    out->cy = (float)K_d[5];
    out->inv_fx = (float)(1.0 / K_d[0]);
    out->inv_fy = (float)(1.0 / K_d[4]);
    out->fxr = (float)K_rgb[0];
    out->fyr = (float)K_rgb[4];
    out->cxr = (float)K_rgb[2];
    out->cyr = (float)K_rgb[5];
    out->trunc = (float)trunc_m;
    out->inv_trunc = (float)(1.0 / trunc_m);
    out->w_max = (float)w_max;
    out->sigma2 = (float)(vd.colour_band * vd.colour_band);
    out->gate = (float)vd.colour_gate;
    out->sigma = (float)vd.colour_band;
    out->wm1 = (float)(dw - 1);
    out->hm1 = (float)(dh - 1);
    // the last pixel a sample may start from: the cell's top-left (bilinear) or the pixel
    const bool nearest = vd.hd_sampling == KF_HD_NEAREST;
    out->hd_nearest = nearest ? 1 : 0;
    out->hd_xmax = (float)(nearest ? cw - 1 : cw - 2);
    out->hd_ymax = (float)(nearest ? ch - 1 : ch - 2);
    out->dw = dw;
    out->dh = dh;
    out->cw = cw;
    out->ch = ch;
    out->depth = depth;
    out->rgb = rgb;
    // the depth pyramid: 2x2-pixel tiles, halved until one tile covers the image
    out->pyr = nullptr;
    out->pyr_w0 = (dw + (1 << kf::PYR_SHIFT) - 1) >> kf::PYR_SHIFT;
    out->pyr_h0 = (dh + (1 << kf::PYR_SHIFT) - 1) >> kf::PYR_SHIFT;
    int32_t levels = 1, w = out->pyr_w0, h = out->pyr_h0;
    while (w > 1 || h > 1) {
        w = (w + 1) / 2;
        h = (h + 1) / 2;
        ++levels;
    }
    out->pyr_levels = levels;
}

// float2 entries of a frame's depth pyramid.
size_t pyramid_entries(const kf::FrameConsts& c)
{
    int32_t w, h, off;
    kf::pyr_level_dims(c.pyr_w0, c.pyr_h0, c.pyr_levels, &w, &h, &off);
    return (size_t)off;
}

uint32_t ceil_div(int32_t a, int32_t b) { return (uint32_t)((a + b - 1) / b); }

// Scene table entry of a volume for bricks of shapes BRICK_SHAPES[kind][shape[kind]].
void scene_dev(const kf_volume* v, int32_t fmt, const int shape[2], kf::SceneDev* s)
{
    memset(s, 0, sizeof *s);
    s->tsdf = v->bufs.tsdf;
    s->wg = v->bufs.w_geom;
    s->r = v->bufs.r;
    s->g = v->bufs.g;
    s->b = v->bufs.b;
    s->wc = v->bufs.w_col;
    for (int a = 0; a < 3; ++a) {
        s->gdim[a] = v->desc.geom_dim[a];
        s->cdim[a] = v->desc.colour_dim[a];
    }
    const kf::BrickShape& gs = kf::BRICK_SHAPES[kf::KIND_GEOM][shape[kf::KIND_GEOM]];
    const kf::BrickShape& cs = kf::BRICK_SHAPES[kf::KIND_COLOUR][shape[kf::KIND_COLOUR]];
    s->gshape[0] = gs.bx;
    s->gshape[1] = gs.by;
    s->gshape[2] = gs.bz;
    s->cshape[0] = cs.bx;
    s->cshape[1] = cs.by;
    s->cshape[2] = cs.bz;
    for (int a = 0; a < 3; ++a) {
        s->gbricks[a] = (int32_t)ceil_div(s->gdim[a], s->gshape[a]);
        s->cbricks[a] = (int32_t)ceil_div(s->cdim[a], s->cshape[a]);
    }
    s->geom_items = (uint32_t)s->gbricks[0] * (uint32_t)s->gbricks[1] * (uint32_t)s->gbricks[2];
    s->colour_items = (uint32_t)s->cbricks[0] * (uint32_t)s->cbricks[1] * (uint32_t)s->cbricks[2];
    for (int a = 0; a < 3; ++a) {
        s->gchunks[a] = (int32_t)ceil_div(s->gbricks[a], kf::CHUNK);
        s->cchunks[a] = (int32_t)ceil_div(s->cbricks[a], kf::CHUNK);
    }
    s->geom_chunks = (uint32_t)s->gchunks[0] * (uint32_t)s->gchunks[1] * (uint32_t)s->gchunks[2];
    s->colour_chunks = (uint32_t)s->cchunks[0] * (uint32_t)s->cchunks[1] * (uint32_t)s->cchunks[2];
    s->fmt = fmt;
}

// KF_DISABLE_CULL=1 in the environment makes every brick live in every frame (the
// results are identical; only the work grows).
bool cull_disabled()
{
    const char* v = getenv("KF_DISABLE_CULL");
    return v && v[0] == '1';
}

kf_status check_frame_args(kf_volume* vol, const float* depth, int32_t dw, int32_t dh,
                           const void* rgb, kf_pixfmt fmt, int32_t cw, int32_t ch,
                           const double* K_d, const double* K_rgb, const double* T_rd,
                           const double* T_wc, double trunc_m, double w_max)
{
    kf_status s;
    if ((s = check_volume(vol)) != KF_OK) return s;
    if ((s = check_images(depth, dw, dh, rgb, fmt, cw, ch)) != KF_OK) return s;
    if ((s = check_K(K_d, "K_d")) != KF_OK) return s;
    if ((s = check_K(K_rgb, "K_rgb")) != KF_OK) return s;
    if ((s = check_rigid(T_rd, "T_rgb_from_d")) != KF_OK) return s;
    if ((s = check_rigid(T_wc, "T_world_from_cam")) != KF_OK) return s;
    return check_scalars(trunc_m, w_max);
}

// --------------------------------------------------------------- pinned staging buffer

// A ring of pinned buffers: a slot is reused once the copy that last read it has run, so
// the host can run a few calls ahead of the device.
struct StagingSlot {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};
constexpr int kStagingSlots = 8;
struct Staging {
    std::mutex mu;
    StagingSlot slot[kStagingSlots];
    int next = 0;
};
Staging g_stage;

// Copy `bytes` from host memory `src` to device `dst` on `stream` through a pinned slot.
kf_status staged_copy(void* dst, const void* src, size_t bytes, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(g_stage.mu);
    StagingSlot& s = g_stage.slot[g_stage.next];
    g_stage.next = (g_stage.next + 1) % kStagingSlots;
    if (s.pending) {
        KF_HIP(hipEventSynchronize(s.ev), "hipEventSynchronize");
        s.pending = false;
    }
    if (!s.ev) KF_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming), "hipEventCreate");
    if (bytes > s.cap) {
        if (s.host) KF_HIP(hipHostFree(s.host), "hipHostFree");
        s.host = nullptr;
        s.cap = 0;
        const size_t cap = bytes < 65536 ? 65536 : bytes * 2;
        KF_HIP(hipHostMalloc(&s.host, cap, hipHostMallocDefault), "hipHostMalloc");
        s.cap = cap;
    }
    memcpy(s.host, src, bytes);
    KF_HIP(hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, stream), "hipMemcpyAsync");
    KF_HIP(hipEventRecord(s.ev, stream), "hipEventRecord");
    s.pending = true;
    return KF_OK;
}

// -------------------------------------------------------------------- batch planning

struct BatchPlan {
    std::vector<kf::FrameConsts> frames;            // every frame of every scene
    std::vector<std::vector<kf::SceneDev>> passes;  // scenes with frames in each pass
    std::vector<uint32_t> pass_items;
    std::vector<uint32_t> pass_chunks;
};

// Frames a pass can hold: one bit per frame in a brick's 64-bit live mask.
constexpr int32_t kMaxFramesPerPass = 64;
// Counters of a pass: live entries of the heavy and light lists of each kind, then the
// queue head of each kind.
constexpr size_t kPassCounters = 6;

// The default brick shapes (entry 0 of each kind).
const int kDefaultShapes[2] = {0, 0};

kf_status plan_batch(const kf_scene* scenes, int32_t n_scenes, int32_t K, const int shape[2],
                     BatchPlan* plan)
{
    if (!scenes && n_scenes > 0) return fail(KF_E_ARG, "scenes is NULL");
    if (n_scenes < 0) return fail(KF_E_ARG, "n_scenes < 0");
    if (K < 1) return fail(KF_E_ARG, "frames_per_pass must be >= 1");
    if (K > kMaxFramesPerPass) K = kMaxFramesPerPass;
    std::vector<int32_t> first(n_scenes);
    int32_t max_frames = 0;
    for (int s = 0; s < n_scenes; ++s) {
        const kf_scene& sc = scenes[s];
        kf_status st;
        if ((st = check_volume(sc.vol)) != KF_OK) return st;
        for (int t = 0; t < s; ++t)
            if (scenes[t].vol == sc.vol) return fail(KF_E_ARG, "a volume appears twice in one batch");
        if (sc.n_frames < 0) return fail(KF_E_ARG, "n_frames < 0");
        if (sc.n_frames == 0) { first[s] = (int32_t)plan->frames.size(); continue; }
        if ((st = check_images(sc.depth, sc.dw, sc.dh, sc.rgb, sc.fmt, sc.cw, sc.ch)) != KF_OK) return st;
        if ((st = check_K(sc.K_d, "K_d")) != KF_OK) return st;
        if ((st = check_K(sc.K_rgb, "K_rgb")) != KF_OK) return st;
        if ((st = check_rigid(sc.T_rgb_from_d, "T_rgb_from_d")) != KF_OK) return st;
        if (!sc.T_world_from_cam) return fail(KF_E_ARG, "T_world_from_cam is NULL");
        for (int f = 0; f < sc.n_frames; ++f)
            if ((st = check_rigid(sc.T_world_from_cam + 16 * (size_t)f, "T_world_from_cam")) != KF_OK) return st;
        if ((st = check_scalars(sc.trunc_m, sc.w_max)) != KF_OK) return st;
        first[s] = (int32_t)plan->frames.size();
        const size_t dpix = (size_t)sc.dw * sc.dh;
        const size_t cbytes = (size_t)sc.cw * sc.ch * 3 * (sc.fmt == KF_RGB8 ? 1 : 4);
        for (int f = 0; f < sc.n_frames; ++f) {
            kf::FrameConsts fc;
            frame_consts(sc.vol->desc, sc.K_d, sc.K_rgb, sc.T_rgb_from_d,
                         sc.T_world_from_cam + 16 * (size_t)f, sc.trunc_m, sc.w_max,
                         sc.depth + dpix * f, sc.dw, sc.dh,
                         (const uint8_t*)sc.rgb + cbytes * f, sc.cw, sc.ch, &fc);
            plan->frames.push_back(fc);
        }
        if (sc.n_frames > max_frames) max_frames = sc.n_frames;
    }
    if ((double)plan->frames.size() > 1e7) return fail(KF_E_RANGE, "too many frames in one batch");
    for (int32_t f0 = 0; f0 < max_frames; f0 += K) {
        std::vector<kf::SceneDev> pass;
        uint64_t items = 0, chunks = 0;
        for (int s = 0; s < n_scenes; ++s) {
            const int32_t nf = scenes[s].n_frames - f0;
            if (nf <= 0) continue;
            kf::SceneDev d;
            scene_dev(scenes[s].vol, scenes[s].fmt, shape, &d);
            d.frame_begin = first[s] + f0;
            d.n_frames = nf < K ? nf : K;
            d.item_begin = (uint32_t)items;
            d.chunk_begin = (uint32_t)chunks;
            items += (uint64_t)d.geom_items + d.colour_items;
            chunks += (uint64_t)d.geom_chunks + d.colour_chunks;
            if (items > 2147483647ull) return fail(KF_E_RANGE, "too many work items in one pass");
            pass.push_back(d);
        }
        plan->passes.push_back(pass);
        plan->pass_items.push_back((uint32_t)items);
        plan->pass_chunks.push_back((uint32_t)chunks);
    }
    return KF_OK;
}

// Device image of a plan:
//   [frame table][scene table of each pass][kPassCounters counters per pass][two live
//   buffers (passes alternate), each a heavy and a light list][pyramids][pixel maps]
struct DeviceTables {
    std::vector<unsigned char> host;
    size_t frames_off = 0, counters_off = 0, live_off = 0, live_entries = 0, pyr_off = 0, bytes = 0;
    std::vector<size_t> pass_off, frame_pyr_off, frame_pmap_off;
    int32_t max_tiles0 = 0, max_pixels = 0;
};

void layout_tables(const BatchPlan& p, DeviceTables* t)
{
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    size_t off = 0;
    t->frames_off = off;
    off = align(off + p.frames.size() * sizeof(kf::FrameConsts));
    for (const auto& pass : p.passes) {
        t->pass_off.push_back(off);
        off = align(off + pass.size() * sizeof(kf::SceneDev));
    }
    t->counters_off = off;
    off = align(off + kPassCounters * (p.passes.size() + 1) * sizeof(uint32_t));
    uint32_t max_items = 0;
    for (uint32_t n : p.pass_items) max_items = n > max_items ? n : max_items;
    t->live_off = off;
    t->live_entries = 2 * (size_t)max_items;   // one buffer: heavy list, light list
    off = align(off + 2 * t->live_entries * sizeof(uint4));   // two buffers, passes alternate
    t->pyr_off = off;
    for (const auto& fc : p.frames) {
        t->frame_pyr_off.push_back(off);
        off += pyramid_entries(fc) * sizeof(float2);
        const int32_t tiles = fc.pyr_w0 * fc.pyr_h0;
        t->max_tiles0 = tiles > t->max_tiles0 ? tiles : t->max_tiles0;
    }
    off = align(off);
    for (const auto& fc : p.frames) {
        t->frame_pmap_off.push_back(off);
        off = align(off + (size_t)fc.dw * fc.dh * sizeof(float4));
        const int32_t pixels = fc.dw * fc.dh;
        t->max_pixels = pixels > t->max_pixels ? pixels : t->max_pixels;
    }
    t->bytes = align(off);
}

// Fill the host image for device base address `dev` (the frames point at their pyramids).
void fill_tables(const BatchPlan& p, unsigned char* dev, DeviceTables* t)
{
    // the tables and counters; the live lists, pyramids and pixel maps are written on
    // the device (the counters are cleared there too)
    t->host.assign(t->live_off, 0);
    std::vector<kf::FrameConsts> frames = p.frames;
    for (size_t f = 0; f < frames.size(); ++f) {
        frames[f].pyr = (float2*)(dev + t->frame_pyr_off[f]);
        frames[f].pmap = (float4*)(dev + t->frame_pmap_off[f]);
    }
    if (!frames.empty())
        memcpy(t->host.data() + t->frames_off, frames.data(), frames.size() * sizeof(kf::FrameConsts));
    for (size_t q = 0; q < p.passes.size(); ++q)
        if (!p.passes[q].empty())
            memcpy(t->host.data() + t->pass_off[q], p.passes[q].data(), p.passes[q].size() * sizeof(kf::SceneDev));
}

// Resident blocks of the geometry ([0]) and colour ([1]) persistent launches.
kf_status resident_grid(int mode, const int shape[2], uint32_t grid[2])
{
    int device = 0;
    KF_HIP(hipGetDevice(&device), "hipGetDevice");
    KF_HIP(kf::persistent_grid(mode, kf::KIND_GEOM, shape[0], device, &grid[0]), "occupancy query");
    KF_HIP(kf::persistent_grid(mode, kf::KIND_COLOUR, shape[1], device, &grid[1]), "occupancy query");
    return KF_OK;
}

// Caller events recorded around the integration launch of each pass (may be empty).
struct PassEvents {
    void* const* start = nullptr;
    void* const* mid = nullptr;       // may be NULL
    void* const* end = nullptr;
    int32_t n = 0;
};

// A side stream per device on which the culling of pass p + 1 runs while pass p
// integrates (the cull reads only frame data; the two live buffers alternate), with the
// events that order the two streams.  Enqueueing on it is serialised per device.
struct CullSide {
    std::mutex mu;
    hipStream_t stream = nullptr;
    hipEvent_t ev[6] = {};   // start, cull done (2), integration done (2), end
};
CullSide g_side[64];

kf_status cull_side(int device, CullSide** out)
{
    if (device < 0 || device >= 64) return fail(KF_E_UNSUPPORTED, "device index above 63");
    CullSide& c = g_side[device];
    if (!c.stream) KF_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking), "hipStreamCreate");
    for (hipEvent_t& e : c.ev)
        if (!e) KF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    *out = &c;
    return KF_OK;
}

// Enqueue the pyramids, pixel maps and passes of a plan whose tables live at `dev`;
// `grid`: blocks of the geometry and colour persistent launches (resident_grid).  With
// `side` (its mutex held by the caller) the culling runs one pass ahead on the side stream
// (the first pass's beside the pixel maps); without it everything runs on `stream` in order.
kf_status enqueue_passes(const BatchPlan& p, const DeviceTables& t, unsigned char* dev, int mode,
                         const int shape[2], unsigned long long* counters, const uint32_t grid[2],
                         hipStream_t stream, const PassEvents& ev = PassEvents(),
                         CullSide* side = nullptr)
{
    const kf::FrameConsts* frames = (const kf::FrameConsts*)(dev + t.frames_off);
    KF_HIP(kf::launch_pyramids(frames, (int32_t)p.frames.size(), t.max_tiles0, stream), "pyramid launch");
    uint32_t* cnt = (uint32_t*)(dev + t.counters_off);
    KF_HIP(kf::launch_fill_u32(cnt, kPassCounters * (p.passes.size() + 1), 0u, stream), "counter reset");
    uint4* live = (uint4*)(dev + t.live_off);
    const int disable = cull_disabled() ? 1 : 0;
    std::vector<size_t> run;   // passes with work
    for (size_t q = 0; q < p.passes.size(); ++q)
        if (p.pass_items[q] != 0) run.push_back(q);
    auto cull_args = [&](size_t r) {
        const size_t q = run[r];
        kf::CullArgs c;
        memset(&c, 0, sizeof c);
        c.scenes = (const kf::SceneDev*)(dev + t.pass_off[q]);
        c.frames = frames;
        c.n_scenes = (int32_t)p.passes[q].size();
        c.n_items = p.pass_items[q];
        c.n_chunks = p.pass_chunks[q];
        c.disable = disable;
        c.max_frames = 0;
        for (const kf::SceneDev& d : p.passes[q]) c.max_frames = d.n_frames > c.max_frames ? d.n_frames : c.max_frames;
        c.live = live + (r % 2) * t.live_entries;
        c.n_live = cnt + kPassCounters * q;
        return c;
    };
    hipStream_t cs = side ? side->stream : stream;
    if (side && !run.empty()) {
        // the first cull needs the pyramids and the cleared counters, not the pixel maps:
        // it runs beside them
        KF_HIP(hipEventRecord(side->ev[0], stream), "hipEventRecord");
        KF_HIP(hipStreamWaitEvent(cs, side->ev[0], 0), "hipStreamWaitEvent");
    }
    KF_HIP(kf::launch_pixel_maps(frames, (int32_t)p.frames.size(), t.max_pixels, stream),
           "pixel map launch");
    for (size_t r = 0; r < run.size(); ++r) {
        const size_t q = run[r];
        if (!side) {
            KF_HIP(kf::launch_cull(cull_args(r), stream), "cull launch");
        } else {
            if (r == 0) {
                KF_HIP(kf::launch_cull(cull_args(0), cs), "cull launch");
                KF_HIP(hipEventRecord(side->ev[1], cs), "hipEventRecord");
            }
            if (r + 1 < run.size()) {
                // the next pass's buffer was last read by pass r - 1
                if (r >= 1) KF_HIP(hipStreamWaitEvent(cs, side->ev[3 + (r - 1) % 2], 0), "hipStreamWaitEvent");
                KF_HIP(kf::launch_cull(cull_args(r + 1), cs), "cull launch");
                KF_HIP(hipEventRecord(side->ev[1 + (r + 1) % 2], cs), "hipEventRecord");
            }
            KF_HIP(hipStreamWaitEvent(stream, side->ev[1 + r % 2], 0), "hipStreamWaitEvent");
        }
        kf::IntegrateArgs a;
        memset(&a, 0, sizeof a);
        a.scenes = (const kf::SceneDev*)(dev + t.pass_off[q]);
        a.frames = frames;
        a.n_scenes = (int32_t)p.passes[q].size();
        a.live = live + (r % 2) * t.live_entries;
        a.cap = p.pass_items[q];
        a.n_live = cnt + kPassCounters * q;
        a.queue = cnt + kPassCounters * q + 4;
        a.counters = counters;
        const bool timed = (int32_t)q < ev.n;
        if (timed) KF_HIP(hipEventRecord((hipEvent_t)ev.start[q], stream), "hipEventRecord");
        KF_HIP(kf::launch_integrate(mode, kf::KIND_GEOM, shape[0], a, grid[0], stream), "integrate launch");
        if (timed && ev.mid) KF_HIP(hipEventRecord((hipEvent_t)ev.mid[q], stream), "hipEventRecord");
        KF_HIP(kf::launch_integrate(mode, kf::KIND_COLOUR, shape[1], a, grid[1], stream), "integrate launch");
        if (timed) KF_HIP(hipEventRecord((hipEvent_t)ev.end[q], stream), "hipEventRecord");
        if (side) KF_HIP(hipEventRecord(side->ev[3 + r % 2], stream), "hipEventRecord");
    }
    if (side && !run.empty()) {
        // the caller's stream continues only after the side stream's last work
        KF_HIP(hipEventRecord(side->ev[5], cs), "hipEventRecord");
        KF_HIP(hipStreamWaitEvent(stream, side->ev[5], 0), "hipStreamWaitEvent");
    }
    return KF_OK;
}

// ------------------------------------------------------------------------ graph cache

struct GraphEntry {
    std::string key;
    int device = 0;
    unsigned char* dev = nullptr;
    size_t bytes = 0;
    hipGraphExec_t exec = nullptr;
};

// Recorded batches, most recently used first.  Each entry owns its graph and the workspace
// the graph's kernels use (tables, live lists, pyramids and pixel maps of every frame), so
// the cache is bounded by entries and by workspace bytes; the least recently used entries
// go first (the newest is always kept).
struct GraphCache {
    std::mutex mu;
    std::list<GraphEntry> lru;
    size_t bytes = 0;
    hipStream_t capture[64] = {};
};
GraphCache g_graphs;
constexpr size_t kMaxGraphs = 64;
constexpr size_t kMaxGraphBytes = size_t(4) << 30;

std::string batch_key(const kf_scene* scenes, int32_t n_scenes, int32_t K, const int shape[2],
                      int device)
{
    std::string k;
    auto put = [&k](const void* p, size_t n) { k.append((const char*)p, n); };
    put(&device, sizeof device);
    put(shape, 2 * sizeof(int));
    put(&n_scenes, sizeof n_scenes);
    put(&K, sizeof K);
    for (int s = 0; s < n_scenes; ++s) {
        const kf_scene& sc = scenes[s];
        put(&sc.vol->desc, sizeof sc.vol->desc);
        put(&sc.vol->bufs, sizeof sc.vol->bufs);
        put(&sc.n_frames, sizeof sc.n_frames);
        put(&sc.depth, sizeof sc.depth);
        put(&sc.rgb, sizeof sc.rgb);
        put(&sc.fmt, sizeof sc.fmt);
        put(&sc.dw, 4 * sizeof(int32_t));
        if (sc.n_frames > 0) {
            put(sc.K_d, 9 * sizeof(double));
            put(sc.K_rgb, 9 * sizeof(double));
            put(sc.T_rgb_from_d, 16 * sizeof(double));
            put(sc.T_world_from_cam, 16 * sizeof(double) * (size_t)sc.n_frames);
        }
        put(&sc.trunc_m, sizeof sc.trunc_m);
        put(&sc.w_max, sizeof sc.w_max);
    }
    return k;
}

// Destroys an entry's graph and frees its workspace (hipFree waits for the device, so a
// replay still in flight finishes first).
void drop_entry(GraphEntry& e)
{
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.dev) (void)hipFree(e.dev);
    e.exec = nullptr;
    e.dev = nullptr;
}

kf_status run_graph(const kf_scene* scenes, int32_t n_scenes, int32_t K, const int shape[2],
                    hipStream_t stream)
{
    int device = 0;
    KF_HIP(hipGetDevice(&device), "hipGetDevice");
    if (device < 0 || device >= 64) return fail(KF_E_UNSUPPORTED, "device index above 63");
    const std::string key = batch_key(scenes, n_scenes, K, shape, device);
    std::lock_guard<std::mutex> lock(g_graphs.mu);
    for (auto it = g_graphs.lru.begin(); it != g_graphs.lru.end(); ++it) {
        if (it->key == key) {
            g_graphs.lru.splice(g_graphs.lru.begin(), g_graphs.lru, it);
            KF_HIP(hipGraphLaunch(it->exec, stream), "hipGraphLaunch");
            return KF_OK;
        }
    }
    BatchPlan plan;
    kf_status st = plan_batch(scenes, n_scenes, K, shape, &plan);
    if (st != KF_OK) return st;
    DeviceTables t;
    layout_tables(plan, &t);
    GraphEntry e;
    e.key = key;
    e.device = device;
    e.bytes = t.bytes;
    KF_HIP(hipMalloc(&e.dev, t.bytes), "hipMalloc");
    fill_tables(plan, e.dev, &t);
    hipError_t he = hipMemcpy(e.dev, t.host.data(), t.host.size(), hipMemcpyHostToDevice);
    if (he != hipSuccess) { drop_entry(e); return hip_fail(he, "hipMemcpy"); }
    uint32_t grid[2] = {0, 0};
    if ((st = resident_grid(kf::MODE_INTEGRATE, shape, grid)) != KF_OK) { drop_entry(e); return st; }
    hipStream_t& cs = g_graphs.capture[device];
    if (!cs) {
        he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (he != hipSuccess) { drop_entry(e); return hip_fail(he, "hipStreamCreate"); }
    }
    CullSide* side = nullptr;
    if ((st = cull_side(device, &side)) != KF_OK) { drop_entry(e); return st; }
    std::lock_guard<std::mutex> side_lock(side->mu);
    he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) { drop_entry(e); return hip_fail(he, "hipStreamBeginCapture"); }
    st = enqueue_passes(plan, t, e.dev, kf::MODE_INTEGRATE, shape, nullptr, grid, cs, PassEvents(), side);
    hipGraph_t graph = nullptr;
    he = hipStreamEndCapture(cs, &graph);
    if (st != KF_OK) { if (graph) (void)hipGraphDestroy(graph); drop_entry(e); return st; }
    if (he != hipSuccess) { drop_entry(e); return hip_fail(he, "hipStreamEndCapture"); }
    he = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (he != hipSuccess) { drop_entry(e); return hip_fail(he, "hipGraphInstantiate"); }
    he = hipGraphLaunch(e.exec, stream);
    if (he != hipSuccess) { drop_entry(e); return hip_fail(he, "hipGraphLaunch"); }
    g_graphs.lru.push_front(e);
    g_graphs.bytes += e.bytes;
    while (g_graphs.lru.size() > 1 &&
           (g_graphs.lru.size() > kMaxGraphs || g_graphs.bytes > kMaxGraphBytes)) {
        g_graphs.bytes -= g_graphs.lru.back().bytes;
        drop_entry(g_graphs.lru.back());
        g_graphs.lru.pop_back();
    }
    return KF_OK;
}

kf_status run_batch(const kf_scene* scenes, int32_t n_scenes, int32_t K, int mode,
                    const int shape[2], unsigned long long* counters, hipStream_t stream,
                    const PassEvents& ev = PassEvents())
{
    BatchPlan plan;
    kf_status st = plan_batch(scenes, n_scenes, K, shape, &plan);
    if (st != KF_OK) return st;
    if (plan.passes.empty()) return KF_OK;
    if (ev.n > 0 && (size_t)ev.n < plan.passes.size())
        return fail(KF_E_ARG, "n_events (%d) is below the number of passes (%zu)", (int)ev.n,
                    plan.passes.size());
    DeviceTables t;
    layout_tables(plan, &t);
    uint32_t grid[2] = {0, 0};
    if ((st = resident_grid(mode, shape, grid)) != KF_OK) return st;
    unsigned char* dev = nullptr;
    KF_HIP(workspace_alloc((void**)&dev, t.bytes, stream), "hipMallocAsync");
    fill_tables(plan, dev, &t);
    st = staged_copy(dev, t.host.data(), t.host.size(), stream);
    if (st == KF_OK) {
        int device = 0;
        CullSide* side = nullptr;
        if (hipGetDevice(&device) != hipSuccess) st = fail(KF_E_DEVICE, "hipGetDevice failed");
        else st = cull_side(device, &side);
        if (st == KF_OK) {
            std::lock_guard<std::mutex> side_lock(side->mu);
            st = enqueue_passes(plan, t, dev, mode, shape, counters, grid, stream, ev, side);
        }
    }
    hipError_t he = hipFreeAsync(dev, stream);
    if (st != KF_OK) return st;
    if (he != hipSuccess) return hip_fail(he, "hipFreeAsync");
    return KF_OK;
}

// ------------------------------------------------------------ allocation-free workspace

// Workspace of kf_integrate_batch_noalloc: a file-scope device array, one copy per GPU that
// loads the library, held until the process ends.  On the host the array's name is only a
// stand-in for the device symbol, never a device address: each GPU's copy is looked up
// once per device with hipGetSymbolAddress (scratch_base) and that address is what the
// launches receive.  Calls that overlap on one GPU share the array and race.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchBases {
    std::mutex mu;
    unsigned char* ptr[64] = {};
};
ScratchBases g_scratch;

// Device address of the current device's scratch array (looked up on its first use).
kf_status scratch_base(unsigned char** out)
{
    int device = 0;
    KF_HIP(hipGetDevice(&device), "hipGetDevice");
    if (device < 0 || device >= 64) return fail(KF_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch.mu);
    if (!g_scratch.ptr[device]) {
        void* p = nullptr;
        KF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(KF_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch.ptr[device] = (unsigned char*)p;
    }
    *out = g_scratch.ptr[device];
    return KF_OK;
}

// Host bytes carried to device memory by value in a kernel's arguments: no staging buffer,
// no copy from host memory that must outlive the call (a captured launch keeps its
// arguments).
constexpr uint32_t kUploadWords = 960;
struct UploadChunk {
    uint32_t* dst;
    uint32_t words;
    uint32_t data[kUploadWords];
};

__global__ __launch_bounds__(256) void upload_kernel(UploadChunk c)
{
    for (uint32_t t = threadIdx.x; t < c.words; t += 256) c.dst[t] = c.data[t];
}

// Copy `bytes` (a multiple of 4) from host `src` to device `dst` in kernel arguments.
kf_status upload(unsigned char* dst, const unsigned char* src, size_t bytes, hipStream_t stream)
{
    UploadChunk c;
    for (size_t off = 0; off < bytes; off += 4 * (size_t)kUploadWords) {
        const size_t n = bytes - off < 4 * (size_t)kUploadWords ? bytes - off : 4 * (size_t)kUploadWords;
        c.dst = (uint32_t*)(dst + off);
        c.words = (uint32_t)(n / 4);
        memcpy(c.data, src + off, n);
        hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, stream, c);
        KF_HIP(hipGetLastError(), "upload launch");
    }
    return KF_OK;
}

kf_status run_batch_noalloc(const kf_scene* scenes, int32_t n_scenes, int32_t K, hipStream_t stream)
{
    BatchPlan plan;
    kf_status st = plan_batch(scenes, n_scenes, K, kDefaultShapes, &plan);
    if (st != KF_OK) return st;
    if (plan.passes.empty()) return KF_OK;
    DeviceTables t;
    layout_tables(plan, &t);
    if (t.bytes > kScratchBytes)
        return fail(KF_E_RANGE, "the batch needs %zu bytes of workspace; the allocation-free "
                                "entry point holds %zu (fewer frames per call or smaller volumes)",
                    t.bytes, kScratchBytes);
    uint32_t grid[2] = {0, 0};
    if ((st = resident_grid(kf::MODE_INTEGRATE, kDefaultShapes, grid)) != KF_OK) return st;
    unsigned char* dev = nullptr;
    if ((st = scratch_base(&dev)) != KF_OK) return st;
    fill_tables(plan, dev, &t);
    if ((st = upload(dev, t.host.data(), t.host.size(), stream)) != KF_OK) return st;
    return enqueue_passes(plan, t, dev, kf::MODE_INTEGRATE, kDefaultShapes, nullptr, grid, stream);
}

}  // namespace

// =========================================================================== C ABI

extern "C" {

const char* kf_status_str(kf_status s)
{
    switch (s) {
    case KF_OK: return "ok";
    case KF_E_ARG: return "invalid argument";
    case KF_E_SHAPE: return "invalid or unsupported shape";
    case KF_E_RANGE: return "size out of range";
    case KF_E_DEVICE: return "device error";
    case KF_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* kf_last_error(void) { return g_err; }

kf_status kf_volume_buffer_bytes(const kf_volume_desc* desc, size_t out_bytes[6])
{
    kf_status s = check_desc(desc);
    if (s != KF_OK) return s;
    if (!out_bytes) return fail(KF_E_ARG, "out_bytes is NULL");
    const size_t ng = (size_t)desc->geom_dim[0] * desc->geom_dim[1] * desc->geom_dim[2];
    const size_t nc = (size_t)desc->colour_dim[0] * desc->colour_dim[1] * desc->colour_dim[2];
    for (int q = 0; q < 6; ++q) out_bytes[q] = (q < 2 ? ng : nc) * sizeof(float);
    return KF_OK;
}

kf_status kf_volume_create(const kf_volume_desc* desc, const kf_volume_buffers* bufs,
                           kf_volume** out)
{
    kf_status s = check_desc(desc);
    if (s != KF_OK) return s;
    if (!bufs || !out) return fail(KF_E_ARG, "buffers or output handle is NULL");
    if (!bufs->tsdf || !bufs->w_geom || !bufs->r || !bufs->g || !bufs->b || !bufs->w_col)
        return fail(KF_E_ARG, "a volume buffer is NULL");
    kf_volume* v = new (std::nothrow) kf_volume;
    if (!v) return fail(KF_E_DEVICE, "out of host memory");
    v->desc = *desc;
    v->bufs = *bufs;
    *out = v;
    return KF_OK;
}

void kf_volume_destroy(kf_volume* vol) { delete vol; }

kf_status kf_volume_reset(kf_volume* vol, void* stream)
{
    kf_status s = check_volume(vol);
    if (s != KF_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const kf_volume_desc& d = vol->desc;
    const size_t ng = (size_t)d.geom_dim[0] * d.geom_dim[1] * d.geom_dim[2];
    const size_t nc = (size_t)d.colour_dim[0] * d.colour_dim[1] * d.colour_dim[2];
    float* arrays[6] = {vol->bufs.tsdf, vol->bufs.w_geom, vol->bufs.r, vol->bufs.g, vol->bufs.b, vol->bufs.w_col};
    for (int q = 0; q < 6; ++q)
        KF_HIP(kf::launch_fill_f32(arrays[q], q < 2 ? ng : nc, 0.0f, st), "volume reset");
    return KF_OK;
}

static kf_scene single_scene(kf_volume* vol, const float* depth, int32_t dw, int32_t dh,
                             const void* rgb, kf_pixfmt fmt, int32_t cw, int32_t ch,
                             const double* K_d, const double* K_rgb, const double* T_rd,
                             const double* T_wc, double trunc_m, double w_max)
{
    kf_scene sc;
    sc.vol = vol;
    sc.n_frames = 1;
    sc.depth = depth;
    sc.rgb = rgb;
    sc.fmt = fmt;
    sc.dw = dw;
    sc.dh = dh;
    sc.cw = cw;
    sc.ch = ch;
    sc.K_d = K_d;
    sc.K_rgb = K_rgb;
    sc.T_rgb_from_d = T_rd;
    sc.T_world_from_cam = T_wc;
    sc.trunc_m = trunc_m;
    sc.w_max = w_max;
    return sc;
}

kf_status kf_integrate(kf_volume* vol, const float* depth, int32_t dw, int32_t dh,
                       const void* rgb, kf_pixfmt fmt, int32_t cw, int32_t ch,
                       const double K_d[9], const double K_rgb[9],
                       const double T_rgb_from_d[16], const double T_world_from_cam[16],
                       double trunc_m, double w_max, void* stream)
{
    kf_status s = check_frame_args(vol, depth, dw, dh, rgb, fmt, cw, ch, K_d, K_rgb,
                                   T_rgb_from_d, T_world_from_cam, trunc_m, w_max);
    if (s != KF_OK) return s;
    const kf_scene sc = single_scene(vol, depth, dw, dh, rgb, fmt, cw, ch, K_d, K_rgb,
                                     T_rgb_from_d, T_world_from_cam, trunc_m, w_max);
    return run_batch(&sc, 1, 1, kf::MODE_INTEGRATE, kDefaultShapes, nullptr, (hipStream_t)stream);
}

kf_status kf_debug_status(kf_volume* vol, const float* depth, int32_t dw, int32_t dh,
                          const void* rgb, kf_pixfmt fmt, int32_t cw, int32_t ch,
                          const double K_d[9], const double K_rgb[9],
                          const double T_rgb_from_d[16], const double T_world_from_cam[16],
                          double trunc_m, double w_max, uint8_t* geom_status,
                          uint8_t* colour_status, void* stream)
{
    kf_status s = check_frame_args(vol, depth, dw, dh, rgb, fmt, cw, ch, K_d, K_rgb,
                                   T_rgb_from_d, T_world_from_cam, trunc_m, w_max);
    if (s != KF_OK) return s;
    if (!geom_status || !colour_status) return fail(KF_E_ARG, "status output is NULL");
    kf::StatusArgs a;
    memset(&a, 0, sizeof a);
    scene_dev(vol, fmt, kDefaultShapes, &a.scene);
    a.scene.n_frames = 1;
    frame_consts(vol->desc, K_d, K_rgb, T_rgb_from_d, T_world_from_cam, trunc_m, w_max, depth,
                 dw, dh, rgb, cw, ch, &a.frame);
    hipStream_t st = (hipStream_t)stream;
    // workspace: [frame constants][pixel map]
    const size_t map_off = (sizeof(kf::FrameConsts) + 255) / 256 * 256;
    unsigned char* ws = nullptr;
    KF_HIP(workspace_alloc((void**)&ws, map_off + (size_t)dw * dh * sizeof(float4), st), "hipMallocAsync");
    a.frame.pmap = (float4*)(ws + map_off);
    s = staged_copy(ws, &a.frame, sizeof a.frame, st);
    hipError_t e = hipSuccess;
    const char* what = nullptr;
    if (s == KF_OK) {
        if ((e = kf::launch_pixel_maps((const kf::FrameConsts*)ws, 1, dw * dh, st)) != hipSuccess)
            what = "pixel map launch";
        if (!what) {
            a.n_items = a.scene.geom_items;
            a.status = geom_status;
            if ((e = kf::launch_status(false, a, st)) != hipSuccess) what = "status launch";
        }
        if (!what) {
            a.n_items = a.scene.colour_items;
            a.status = colour_status;
            if ((e = kf::launch_status(true, a, st)) != hipSuccess) what = "status launch";
        }
        if (what) s = hip_fail(e, what);
    }
    const hipError_t fe = hipFreeAsync(ws, st);
    if (s != KF_OK) return s;
    if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
    return KF_OK;
}

kf_status kf_brick_shapes(int32_t kind, int32_t* shapes, int32_t capacity, int32_t* n_shapes)
{
    if (kind != kf::KIND_GEOM && kind != kf::KIND_COLOUR) return fail(KF_E_ARG, "kind must be 0 or 1");
    if (!n_shapes || capacity < 0 || (capacity > 0 && !shapes)) return fail(KF_E_ARG, "NULL pointer");
    *n_shapes = kf::N_BRICK_SHAPES;
    for (int q = 0; q < kf::N_BRICK_SHAPES && q < capacity; ++q) {
        shapes[3 * q + 0] = kf::BRICK_SHAPES[kind][q].bx;
        shapes[3 * q + 1] = kf::BRICK_SHAPES[kind][q].by;
        shapes[3 * q + 2] = kf::BRICK_SHAPES[kind][q].bz;
    }
    return KF_OK;
}

// Shape indices of kf_bricks (NULL: the defaults).
static kf_status resolve_bricks(const kf_bricks* b, int shape[2])
{
    shape[0] = shape[1] = 0;
    if (!b) return KF_OK;
    const int32_t* want[2] = {b->geom, b->colour};
    for (int kind = 0; kind < 2; ++kind) {
        int found = -1;
        for (int q = 0; q < kf::N_BRICK_SHAPES && found < 0; ++q) {
            const kf::BrickShape& s = kf::BRICK_SHAPES[kind][q];
            if (s.bx == want[kind][0] && s.by == want[kind][1] && s.bz == want[kind][2]) found = q;
        }
        if (found < 0)
            return fail(KF_E_UNSUPPORTED, "%s brick %d x %d x %d is not one of the compiled shapes (kf_brick_shapes)",
                        kind ? "colour" : "geometry", (int)want[kind][0], (int)want[kind][1], (int)want[kind][2]);
        shape[kind] = found;
    }
    return KF_OK;
}

kf_status kf_integrate_batch_bricks(const kf_scene* scenes, int32_t n_scenes, int32_t frames_per_pass,
                                    int32_t use_graph, const kf_bricks* bricks, void* stream)
{
    int shape[2];
    kf_status s = resolve_bricks(bricks, shape);
    if (s != KF_OK) return s;
    if (use_graph) {
        // validate before looking at the cache, so errors never depend on its state
        BatchPlan probe;
        s = plan_batch(scenes, n_scenes, frames_per_pass, shape, &probe);
        if (s != KF_OK) return s;
        if (probe.passes.empty()) return KF_OK;
        return run_graph(scenes, n_scenes, frames_per_pass, shape, (hipStream_t)stream);
    }
    return run_batch(scenes, n_scenes, frames_per_pass, kf::MODE_INTEGRATE, shape, nullptr,
                     (hipStream_t)stream);
}

kf_status kf_integrate_batch(const kf_scene* scenes, int32_t n_scenes, int32_t frames_per_pass,
                             int32_t use_graph, void* stream)
{
    return kf_integrate_batch_bricks(scenes, n_scenes, frames_per_pass, use_graph, nullptr, stream);
}

kf_status kf_release_graphs(int32_t* n_released, size_t* bytes_released)
{
    std::lock_guard<std::mutex> lock(g_graphs.mu);
    if (n_released) *n_released = (int32_t)g_graphs.lru.size();
    if (bytes_released) *bytes_released = g_graphs.bytes;
    int device = 0;
    KF_HIP(hipGetDevice(&device), "hipGetDevice");
    for (GraphEntry& e : g_graphs.lru) {
        // free each workspace on the device it was allocated on
        if (e.device != device) (void)hipSetDevice(e.device);
        drop_entry(e);
        if (e.device != device) (void)hipSetDevice(device);
    }
    g_graphs.lru.clear();
    g_graphs.bytes = 0;
    return KF_OK;
}

kf_status kf_integrate_batch_noalloc(const kf_scene* scenes, int32_t n_scenes,
                                     int32_t frames_per_pass, void* stream)
{
    return run_batch_noalloc(scenes, n_scenes, frames_per_pass, (hipStream_t)stream);
}

kf_status kf_integrate_batch_timed(const kf_scene* scenes, int32_t n_scenes,
                                   int32_t frames_per_pass, const kf_bricks* bricks,
                                   void* const* start_events, void* const* mid_events,
                                   void* const* end_events, int32_t n_events, void* stream)
{
    int shape[2];
    kf_status s = resolve_bricks(bricks, shape);
    if (s != KF_OK) return s;
    if (n_events < 1 || !start_events || !end_events) return fail(KF_E_ARG, "events missing");
    for (int32_t q = 0; q < n_events; ++q)
        if (!start_events[q] || !end_events[q] || (mid_events && !mid_events[q]))
            return fail(KF_E_ARG, "an event is NULL");
    PassEvents ev;
    ev.start = start_events;
    ev.mid = mid_events;
    ev.end = end_events;
    ev.n = n_events;
    return run_batch(scenes, n_scenes, frames_per_pass, kf::MODE_INTEGRATE, shape, nullptr,
                     (hipStream_t)stream, ev);
}

kf_status kf_integrate_batch_counted(const kf_scene* scenes, int32_t n_scenes,
                                     int32_t frames_per_pass, const kf_bricks* bricks,
                                     unsigned long long* counters, void* stream)
{
    int shape[2];
    kf_status s = resolve_bricks(bricks, shape);
    if (s != KF_OK) return s;
    if (!counters) return fail(KF_E_ARG, "counters is NULL");
    return run_batch(scenes, n_scenes, frames_per_pass, kf::MODE_COUNT, shape, counters,
                     (hipStream_t)stream);
}

namespace {

// One call of the adjoint kernels over n_frames <= 64 frames (arguments checked by the
// caller).  tail_in / tail_out / wc_out: see BackwardArgs (chunks of a longer scan).
kf_status backward_call(const kf_volume_desc* desc, const float* w_col0, int32_t n_frames,
                        const float* depth, const float* rgb_f32, int32_t dw, int32_t dh,
                        int32_t cw, int32_t ch, const double K_d[9], const double K_rgb[9],
                        const double T_rgb_from_d[16], const double* T_world_from_cam,
                        const float* grad_rgb_vol, const float* tail_in, float* tail_out,
                        float* wc_out, float* d_rgb, double* d_xi, double* d_pose, void* stream)
{
    kf_status s = KF_OK;
    hipStream_t st = (hipStream_t)stream;
    kf::BackwardArgs a;
    memset(&a, 0, sizeof a);
    for (int q = 0; q < 3; ++q) a.cdim[q] = desc->colour_dim[q];
    a.cbricks[0] = (int32_t)ceil_div(a.cdim[0], kf::CBX);
    a.cbricks[1] = (int32_t)ceil_div(a.cdim[1], kf::CBY);
    a.cbricks[2] = (int32_t)ceil_div(a.cdim[2], kf::ZS);
    a.n_items = n_frames > 0 ? (uint32_t)a.cbricks[0] * (uint32_t)a.cbricks[1] * (uint32_t)a.cbricks[2] : 0u;
    a.n_frames = n_frames;
    a.disable_cull = cull_disabled() ? 1 : 0;
    a.wc0 = w_col0;
    a.grad = grad_rgb_vol;
    a.tail_in = tail_in;
    a.tail_out = tail_out;
    a.wc_out = wc_out;
    a.d_rgb = d_rgb;
    // workspace: [frames][n_live, queue][live list][partials][pyramids][pixel maps]
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    std::vector<kf::FrameConsts> fc((size_t)(n_frames > 0 ? n_frames : 1));
    memset(fc.data(), 0, fc.size() * sizeof(kf::FrameConsts));
    const size_t dpix = (size_t)dw * dh, cvals = (size_t)cw * ch * 3;
    for (int f = 0; f < n_frames; ++f)
        frame_consts(*desc, K_d, K_rgb, T_rgb_from_d, T_world_from_cam + 16 * (size_t)f, 1.0, 1.0,
                     depth + dpix * f, dw, dh, rgb_f32 + cvals * f, cw, ch, &fc[f]);
    const size_t frames_off = 0;
    const size_t counters_off = align(frames_off + fc.size() * sizeof(kf::FrameConsts));
    const size_t live_off = align(counters_off + 2 * sizeof(uint32_t));
    const size_t partials_off = align(live_off + (size_t)a.n_items * sizeof(uint4));
    // per-brick partials, then the block sums of the first reduction stage
    const size_t pose_t_off = align(partials_off + ((size_t)a.n_items + kf::XI_BLOCKS) * 6 * sizeof(double));
    // depth-pose adjoint: per-frame T_hd_from_world, then per-brick per-frame partials,
    // the first-stage block sums and the per-frame sums
    const bool pose = d_pose != nullptr && n_frames > 0;
    const size_t width = (size_t)n_frames * 6;
    const size_t pose_p_off = align(pose_t_off + (pose ? (size_t)n_frames * 12 * sizeof(double) : 0));
    // image-gradient records, their segments and (frame, tile) bins: records for half an
    // update per HD pixel and frame (a brick that finds the buffer full scatters with
    // atomics instead), one segment per live brick and frame, four bins per segment
    a.tiles_x = (int32_t)ceil_div(cw, kf::BWD_TILE_W);
    a.tiles_y = (int32_t)ceil_div(ch, kf::BWD_TILE_H);
    // a record holds its cell's x and y in 16 bits each
    const bool binned = n_frames > 0 && !wc_out && cw <= 65536 && ch <= 65536;
    uint64_t rec_cap = binned ? (uint64_t)n_frames * (uint64_t)cw * (uint64_t)ch / 2 : 0;
    if (binned && rec_cap < (1u << 20)) rec_cap = 1u << 20;
    if (rec_cap > 0x7FFFFFFFull) rec_cap = 0x7FFFFFFFull;
    if (const char* ev = getenv("KF_BWD_RECORDS")) rec_cap = binned ? strtoull(ev, nullptr, 10) : 0;
    if (rec_cap > 0x7FFFFFFFull) rec_cap = 0x7FFFFFFFull;
    a.rec_cap = (uint32_t)rec_cap;
    a.seg_cap = binned ? (uint32_t)n_frames * a.n_items : 0u;
    const size_t n_bins = binned ? (size_t)n_frames * (size_t)a.tiles_x * (size_t)a.tiles_y : 0;
    const size_t rec_off = align(pose_p_off + (pose ? ((size_t)a.n_items + kf::XI_BLOCKS + 1) * width * sizeof(double) : 0));
    const size_t recn_off = align(rec_off + (size_t)a.rec_cap * 6 * sizeof(float));
    const size_t seg_off = align(recn_off + 2 * sizeof(unsigned long long));
    const size_t bins_off = align(seg_off + (size_t)a.seg_cap * sizeof(uint4));
    const size_t fill_off = align(bins_off + (n_bins + 1) * sizeof(uint32_t));
    const size_t bsegs_off = align(fill_off + n_bins * sizeof(uint32_t));
    const size_t pyr_off = align(bsegs_off + 4 * (size_t)a.seg_cap * sizeof(uint32_t));
    size_t off = pyr_off;
    int32_t max_tiles0 = 0;
    std::vector<size_t> pyr(fc.size(), 0);
    for (int f = 0; f < n_frames; ++f) {
        pyr[f] = off;
        off += pyramid_entries(fc[f]) * sizeof(float2);
        const int32_t tiles = fc[f].pyr_w0 * fc[f].pyr_h0;
        max_tiles0 = tiles > max_tiles0 ? tiles : max_tiles0;
    }
    off = align(off);
    std::vector<size_t> pmap(fc.size(), 0);
    for (int f = 0; f < n_frames; ++f) {
        pmap[f] = off;
        off = align(off + dpix * sizeof(float4));
    }
    const size_t bytes = align(off);
    unsigned char* ws = nullptr;
    KF_HIP(workspace_alloc((void**)&ws, bytes, st), "hipMallocAsync");
    for (int f = 0; f < n_frames; ++f) {
        fc[f].pyr = (float2*)(ws + pyr[f]);
        fc[f].pmap = (float4*)(ws + pmap[f]);
    }
    a.frames = (const kf::FrameConsts*)(ws + frames_off);
    a.n_live = (uint32_t*)(ws + counters_off);
    a.queue = a.n_live + 1;
    a.live = (uint4*)(ws + live_off);
    a.partials = (double*)(ws + partials_off);
    a.records = (float*)(ws + rec_off);
    a.rec_next = (unsigned long long*)(ws + recn_off);
    a.segs = (uint4*)(ws + seg_off);
    a.seg_next = (uint32_t*)(ws + recn_off + sizeof(unsigned long long));
    a.bin_count = (uint32_t*)(ws + bins_off);
    a.bin_fill = (uint32_t*)(ws + fill_off);
    a.bin_segs = (uint32_t*)(ws + bsegs_off);
    std::vector<double> pose_t;
    if (pose) {
        // T_hd_from_world = T_rgb_from_d T_world_from_cam^-1 of each frame, in double
        pose_t.resize((size_t)n_frames * 12);
        for (int f = 0; f < n_frames; ++f) {
            const double* Tw = T_world_from_cam + 16 * (size_t)f;
            double Rcw[9], tcw[3];
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c) Rcw[3 * r + c] = Tw[4 * c + r];
                tcw[r] = -(Tw[r] * Tw[3] + Tw[4 + r] * Tw[7] + Tw[8 + r] * Tw[11]);
            }
            double* out = pose_t.data() + 12 * (size_t)f;
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c)
                    out[3 * r + c] = T_rgb_from_d[4 * r] * Rcw[c] + T_rgb_from_d[4 * r + 1] * Rcw[3 + c] +
                                     T_rgb_from_d[4 * r + 2] * Rcw[6 + c];
                out[9 + r] = T_rgb_from_d[4 * r] * tcw[0] + T_rgb_from_d[4 * r + 1] * tcw[1] +
                             T_rgb_from_d[4 * r + 2] * tcw[2] + T_rgb_from_d[4 * r + 3];
            }
        }
        a.pose_adjoint = (const double*)(ws + pose_t_off);
        a.pose_partials = (double*)(ws + pose_p_off);
    }
    s = staged_copy(ws + frames_off, fc.data(), fc.size() * sizeof(kf::FrameConsts), st);
    if (s == KF_OK && pose) s = staged_copy(ws + pose_t_off, pose_t.data(), pose_t.size() * sizeof(double), st);
    hipError_t e = hipSuccess;
    const char* what = nullptr;
    if (s == KF_OK && n_frames > 0) {
        if (d_rgb && (e = kf::launch_fill_f32(d_rgb, cvals * (size_t)n_frames, 0.0f, st)) != hipSuccess)
            what = "gradient reset";
        else if ((e = kf::launch_fill_u32((uint32_t*)(ws + counters_off), 2, 0u, st)) != hipSuccess) what = "counter reset";
        else if ((e = kf::launch_fill_u32((uint32_t*)(ws + recn_off), 4, 0u, st)) != hipSuccess) what = "record counter reset";
        else if (n_bins > 0 && (e = kf::launch_fill_u32((uint32_t*)(ws + bins_off), n_bins + 1, 0u, st)) != hipSuccess)
            what = "bin reset";
        else if (n_bins > 0 && (e = kf::launch_fill_u32((uint32_t*)(ws + fill_off), n_bins, 0u, st)) != hipSuccess)
            what = "bin reset";
        else if ((e = kf::launch_fill_u32((uint32_t*)a.partials, (size_t)a.n_items * 12, 0u, st)) != hipSuccess)
            what = "partial reset";
        else if (pose && (e = kf::launch_fill_u32((uint32_t*)a.pose_partials, (size_t)a.n_items * width * 2, 0u,
                                                  st)) != hipSuccess)
            what = "pose partial reset";
        else if ((e = kf::launch_pyramids(a.frames, n_frames, max_tiles0, st)) != hipSuccess) what = "pyramid launch";
        else if ((e = kf::launch_pixel_maps(a.frames, n_frames, dw * dh, st)) != hipSuccess)
            what = "pixel map launch";
    }
    if (s == KF_OK && !what) {
        int device = 0;
        if ((e = hipGetDevice(&device)) != hipSuccess) what = "hipGetDevice";
        else if ((e = kf::launch_backward(a, d_xi, pose ? d_pose : nullptr, device, st)) != hipSuccess)
            what = "backward launch";
    }
    if (s == KF_OK && what) s = hip_fail(e, what);
    hipError_t fe = hipFreeAsync(ws, st);
    if (s != KF_OK) return s;
    if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
    return KF_OK;
}

// Frames per adjoint call: 64 (the kernel's alpha history), or KF_BWD_CHUNK in [1, 64]
// from the environment (smaller chunks give the same gradients up to rounding).
int32_t backward_chunk_frames()
{
    const char* v = getenv("KF_BWD_CHUNK");
    const long n = v ? strtol(v, nullptr, 10) : 64;
    return n >= 1 && n <= 64 ? (int32_t)n : 64;
}

}  // namespace

kf_status kf_integrate_backward(const kf_volume_desc* desc, const float* w_col0,
                                int32_t n_frames, const float* depth, const float* rgb_f32,
                                int32_t dw, int32_t dh, int32_t cw, int32_t ch,
                                const double K_d[9], const double K_rgb[9],
                                const double T_rgb_from_d[16], const double* T_world_from_cam,
                                const float* grad_rgb_vol, float* d_rgb, double* d_xi,
                                double* d_pose, void* stream)
{
    kf_status s = check_desc(desc);
    if (s != KF_OK) return s;
    if (desc->hd_sampling != KF_HD_BILINEAR)
        return fail(KF_E_UNSUPPORTED, "the adjoint is defined for bilinear HD sampling");
    if (n_frames < 0) return fail(KF_E_ARG, "n_frames < 0");
    if (!grad_rgb_vol || !d_xi || (n_frames > 0 && !d_rgb))
        return fail(KF_E_ARG, "gradient pointer is NULL");
    if (n_frames > 0) {
        if ((s = check_images(depth, dw, dh, rgb_f32, KF_RGBF32, cw, ch)) != KF_OK) return s;
        if ((s = check_K(K_d, "K_d")) != KF_OK) return s;
        if ((s = check_K(K_rgb, "K_rgb")) != KF_OK) return s;
        if ((s = check_rigid(T_rgb_from_d, "T_rgb_from_d")) != KF_OK) return s;
        if (!T_world_from_cam) return fail(KF_E_ARG, "T_world_from_cam is NULL");
        for (int f = 0; f < n_frames; ++f)
            if ((s = check_rigid(T_world_from_cam + 16 * (size_t)f, "T_world_from_cam")) != KF_OK) return s;
    }
    const int32_t chunk = backward_chunk_frames();
    if (n_frames <= chunk)
        return backward_call(desc, w_col0, n_frames, depth, rgb_f32, dw, dh, cw, ch, K_d, K_rgb,
                             T_rgb_from_d, T_world_from_cam, grad_rgb_vol, nullptr, nullptr, nullptr,
                             d_rgb, d_xi, d_pose, stream);
    // Longer scans in chunks of `chunk` frames.  C_N depends on a chunk's samples through
    // that chunk's alphas and the product of (1 - alpha) over every later frame, so: a
    // forward sweep stores the colour weights at the start of every chunk (the replay's
    // own weight recurrence, bit-identical to the forward integration's); then the chunks
    // from the last, each with the gradient at its end (grad times the running product of
    // (1 - alpha) over the later chunks, updated in place by each call); d_xi is the sum of
    // the chunks' in chunk order.
    hipStream_t st = (hipStream_t)stream;
    const int32_t n_chunks = (n_frames + chunk - 1) / chunk;
    const size_t nvox = (size_t)desc->colour_dim[0] * desc->colour_dim[1] * desc->colour_dim[2];
    const size_t dpix = (size_t)dw * dh, cvals = (size_t)cw * ch * 3;
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t ckpt_off = 0;
    const size_t tail_off = align(ckpt_off + (size_t)(n_chunks - 1) * nvox * sizeof(float));
    const size_t xi_off = align(tail_off + nvox * sizeof(float));
    unsigned char* ws = nullptr;
    KF_HIP(workspace_alloc((void**)&ws, align(xi_off + (size_t)n_chunks * 6 * sizeof(double)), st),
           "hipMallocAsync");
    float* ckpt = (float*)(ws + ckpt_off);
    float* tail = (float*)(ws + tail_off);
    double* xi_rows = (double*)(ws + xi_off);
    hipError_t e = hipSuccess;
    for (int32_t c = 0; s == KF_OK && c + 1 < n_chunks; ++c) {
        const size_t f0 = (size_t)c * chunk;
        const float* w_in = c == 0 ? w_col0 : ckpt + (size_t)(c - 1) * nvox;
        float* w_out = ckpt + (size_t)c * nvox;
        e = w_in ? hipMemcpyAsync(w_out, w_in, nvox * sizeof(float), hipMemcpyDeviceToDevice, st)
                 : kf::launch_fill_f32(w_out, nvox, 0.0f, st);
        if (e != hipSuccess) {
            s = hip_fail(e, "checkpoint copy");
            break;
        }
        s = backward_call(desc, w_in, chunk, depth + dpix * f0, rgb_f32 + cvals * f0, dw, dh, cw, ch,
                          K_d, K_rgb, T_rgb_from_d, T_world_from_cam + 16 * f0, grad_rgb_vol,
                          nullptr, nullptr, w_out, nullptr, xi_rows + 6 * (size_t)c, nullptr, stream);
    }
    if (s == KF_OK && (e = kf::launch_fill_f32(tail, nvox, 1.0f, st)) != hipSuccess)
        s = hip_fail(e, "tail reset");
    for (int32_t c = n_chunks - 1; s == KF_OK && c >= 0; --c) {
        const size_t f0 = (size_t)c * chunk;
        const int32_t nf = (int32_t)((size_t)n_frames - f0 < (size_t)chunk ? (size_t)n_frames - f0 : (size_t)chunk);
        const float* w_in = c == 0 ? w_col0 : ckpt + (size_t)(c - 1) * nvox;
        s = backward_call(desc, w_in, nf, depth + dpix * f0, rgb_f32 + cvals * f0, dw, dh, cw, ch,
                          K_d, K_rgb, T_rgb_from_d, T_world_from_cam + 16 * f0, grad_rgb_vol, tail,
                          c > 0 ? tail : nullptr, nullptr, d_rgb + cvals * f0, xi_rows + 6 * (size_t)c,
                          d_pose ? d_pose + 6 * f0 : nullptr, stream);
    }
    if (s == KF_OK && (e = kf::launch_sum_rows(xi_rows, (uint32_t)n_chunks, 6u, d_xi, st)) != hipSuccess)
        s = hip_fail(e, "d_xi sum");
    const hipError_t fe = hipFreeAsync(ws, st);
    if (s != KF_OK) return s;
    if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
    return KF_OK;
}

kf_status kf_raycast(kf_volume* vol, int32_t width, int32_t height, const double K[9],
                     const double T_world_from_cam[16], double step_m, float* depth,
                     float* vertex, float* normal, float* rgb, void* stream)
{
    kf_status s;
    if ((s = check_volume(vol)) != KF_OK) return s;
    if ((s = check_K(K, "K")) != KF_OK) return s;
    if ((s = check_rigid(T_world_from_cam, "T_world_from_cam")) != KF_OK) return s;
    if (!isfinite(step_m) || !(step_m > 0.0)) return fail(KF_E_ARG, "step_m must be finite and > 0");
    if (width < 1 || height < 1) return fail(KF_E_SHAPE, "image must be at least 1x1");
    if ((double)width * height * 3.0 > 2147483647.0) return fail(KF_E_RANGE, "image too large");
    if (!depth) return fail(KF_E_ARG, "depth output is NULL");
    const kf_volume_desc& d = vol->desc;
    for (int k = 0; k < 3; ++k)
        if (d.geom_dim[k] < 2 || d.colour_dim[k] < 2)
            return fail(KF_E_SHAPE, "ray casting needs at least 2 voxels per axis");
    // per-camera constants in double, each rounded once
    const double fx = K[0], fy = K[4], cx = K[2], cy = K[5];
    double R[9], t[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R[3 * r + c] = T_world_from_cam[4 * r + c];
        t[r] = T_world_from_cam[4 * r + 3];
    }
    kf::RaycastArgs a;
    memset(&a, 0, sizeof a);
    for (int k = 0; k < 3; ++k) {
        const double sg = d.extent[k] / d.geom_dim[k];
        const double sc = d.extent[k] / d.colour_dim[k];
        // world direction of pixel (x, y) at unit camera depth
        const double ru = R[3 * k + 0] / fx, rv = R[3 * k + 1] / fy;
        const double r0 = (R[3 * k + 2] - R[3 * k + 0] * cx / fx) - R[3 * k + 1] * cy / fy;
        a.Ru[k] = (float)ru;
        a.Rv[k] = (float)rv;
        a.R0[k] = (float)r0;
        a.tw[k] = (float)t[k];
        // index coordinates put voxel i's centre at i: (p - origin) / s - 1/2
        a.a[k] = (float)((t[k] - d.origin[k]) / sg - 0.5);
        a.Bu[k] = (float)(ru / sg);
        a.Bv[k] = (float)(rv / sg);
        a.B0[k] = (float)(r0 / sg);
        a.ac[k] = (float)((t[k] - d.origin[k]) / sc - 0.5);
        a.Bcu[k] = (float)(ru / sc);
        a.Bcv[k] = (float)(rv / sc);
        a.Bc0[k] = (float)(r0 / sc);
        a.inv_s[k] = (float)(1.0 / sg);
        a.gmax[k] = (float)(d.geom_dim[k] - 1);
        a.cmax[k] = (float)(d.colour_dim[k] - 1);
        a.gdim[k] = d.geom_dim[k];
        a.cdim[k] = d.colour_dim[k];
    }
    a.delta = (float)step_m;
    a.width = width;
    a.height = height;
    a.tsdf = vol->bufs.tsdf;
    a.wg = vol->bufs.w_geom;
    a.r = vol->bufs.r;
    a.g = vol->bufs.g;
    a.b = vol->bufs.b;
    a.wc = vol->bufs.w_col;
    a.depth = depth;
    a.vertex = vertex;
    a.normal = normal;
    a.rgb = rgb;
    KF_HIP(kf::launch_raycast(a, (hipStream_t)stream), "ray cast launch");
    return KF_OK;
}

kf_status kf_mesh_extract(kf_volume* vol, float* vertices, int64_t vertex_capacity,
                          int32_t* triangles, int64_t triangle_capacity, int64_t counts[2],
                          void* stream)
{
    kf_status s;
    if ((s = check_volume(vol)) != KF_OK) return s;
    if (!counts) return fail(KF_E_ARG, "counts is NULL");
    counts[0] = counts[1] = 0;
    if (vertex_capacity < 0 || triangle_capacity < 0) return fail(KF_E_ARG, "negative capacity");
    if ((vertices == nullptr) != (triangles == nullptr))
        return fail(KF_E_ARG, "give both outputs or neither");
    const kf_volume_desc& d = vol->desc;
    const int64_t n = (int64_t)d.geom_dim[0] * d.geom_dim[1] * d.geom_dim[2];
    // at most 3 vertices and 5 triangles per voxel, counted in 32 bits
    if (5 * n > 2147483647LL) return fail(KF_E_RANGE, "volume too large for mesh extraction");
    if (d.geom_dim[0] < 2 || d.geom_dim[1] < 2 || d.geom_dim[2] < 2) return KF_OK;   // no cubes
    const hipStream_t st = (hipStream_t)stream;
    kf::MeshArgs a;
    memset(&a, 0, sizeof a);
    for (int k = 0; k < 3; ++k) {
        a.dim[k] = d.geom_dim[k];
        const double sz = d.extent[k] / d.geom_dim[k];
        a.s[k] = (float)sz;
        a.c[k] = (float)(d.origin[k] + 0.5 * sz);     // world centre of voxel 0
    }
    a.n_voxels = (uint32_t)n;
    a.n_blocks = (uint32_t)((n + 4095) / 4096);
    a.tsdf = vol->bufs.tsdf;
    a.wg = vol->bufs.w_geom;
    // workspace: per-voxel vertex/triangle info, first-vertex indices, block sums, totals
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t info_off = 0;
    const size_t cfg_off = align(info_off + (size_t)n);
    const size_t voff_off = align(cfg_off + (size_t)n);
    const size_t sums_off = align(voff_off + (size_t)n * sizeof(uint32_t));
    const size_t tot_off = align(sums_off + (size_t)a.n_blocks * 2 * sizeof(uint32_t));
    const size_t bytes = align(tot_off + 2 * sizeof(uint32_t));
    unsigned char* ws = nullptr;
    KF_HIP(workspace_alloc((void**)&ws, bytes, st), "hipMallocAsync");
    a.info = ws + info_off;
    a.cfg = ws + cfg_off;
    a.voff = (uint32_t*)(ws + voff_off);
    a.block_sums = (uint32_t*)(ws + sums_off);
    a.totals = (uint32_t*)(ws + tot_off);
    // with outputs, every kernel is enqueued at once (writes past the capacities are
    // dropped on the device) and the counts are read at the end; without, only the count
    // kernels run
    const bool emit = vertices != nullptr;
    a.vertices = vertices;
    a.triangles = triangles;
    a.vcap = (uint32_t)(vertex_capacity < 4294967295LL ? vertex_capacity : 4294967295LL);
    a.tcap = (uint32_t)(triangle_capacity < 4294967295LL ? triangle_capacity : 4294967295LL);
    uint32_t totals[2] = {0, 0};
    hipError_t e = kf::launch_mesh_count(a, st);
    const char* what = e != hipSuccess ? "mesh count launch" : nullptr;
    if (!what && emit && (e = kf::launch_mesh_emit(a, st)) != hipSuccess) what = "mesh emit launch";
    if (!what && (e = hipMemcpyAsync(totals, a.totals, sizeof totals, hipMemcpyDeviceToHost, st)) != hipSuccess)
        what = "mesh count copy";
    const hipError_t fe = hipFreeAsync(ws, st);
    if (!what && (e = hipStreamSynchronize(st)) != hipSuccess) what = "mesh synchronisation";
    if (what) return hip_fail(e, what);
    if (fe != hipSuccess) return hip_fail(fe, "hipFreeAsync");
    counts[0] = totals[0];
    counts[1] = totals[1];
    if (emit && (counts[0] > vertex_capacity || counts[1] > triangle_capacity))
        return fail(KF_E_RANGE, "mesh of %lld vertices and %lld triangles exceeds the capacities",
                    (long long)counts[0], (long long)counts[1]);
    return KF_OK;
}

kf_status kf_mesh_decimate(const float* vertices, int64_t n_vertices, const int32_t* triangles,
                           int64_t n_triangles, double rate, float* out_vertices,
                           int64_t* out_n_vertices, int32_t* out_triangles,
                           int64_t* out_n_triangles)
{
    if (!out_n_vertices || !out_n_triangles) return fail(KF_E_ARG, "count outputs are NULL");
    *out_n_vertices = *out_n_triangles = 0;
    if (n_vertices < 0 || n_triangles < 0) return fail(KF_E_ARG, "negative mesh size");
    if (n_vertices > 2147483647LL || n_triangles > 2147483647LL / 3)
        return fail(KF_E_RANGE, "mesh too large for int32 indices");
    if ((n_vertices > 0 && !vertices) || (n_triangles > 0 && !triangles))
        return fail(KF_E_ARG, "input mesh is NULL");
    if (!out_vertices || !out_triangles) return fail(KF_E_ARG, "output mesh is NULL");
    if (!isfinite(rate) || rate < 0.0 || rate > 1.0) return fail(KF_E_ARG, "rate must lie in [0, 1]");
    for (int64_t t = 0; t < n_triangles; ++t) {
        const int32_t* q = triangles + 3 * t;
        for (int k = 0; k < 3; ++k)
            if (q[k] < 0 || q[k] >= n_vertices)
                return fail(KF_E_ARG, "triangle %lld: vertex index out of range", (long long)t);
        if (q[0] == q[1] || q[1] == q[2] || q[0] == q[2])
            return fail(KF_E_ARG, "triangle %lld repeats a vertex", (long long)t);
    }
    for (int64_t q = 0; q < 3 * n_vertices; ++q)
        if (!isfinite(vertices[q])) return fail(KF_E_ARG, "vertex %lld is not finite", (long long)(q / 3));
    kf::decimate_mesh(vertices, n_vertices, triangles, n_triangles, rate, out_vertices,
                      out_n_vertices, out_triangles, out_n_triangles);
    return KF_OK;
}

// ------------------------------------------------------------------- se(3) helpers

// Power series of a square matrix A (n x n, row-major): sum_k coeff[k] A^k, k < terms.
static void matrix_series(const double* A, int n, const double* coeff, int terms, double* out)
{
    double P[36], Q[36];
    for (int i = 0; i < n * n; ++i) {
        P[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
        out[i] = 0.0;
    }
    for (int k = 0; k < terms; ++k) {
        for (int i = 0; i < n * n; ++i) out[i] += coeff[k] * P[i];
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                double acc = 0.0;
                for (int m = 0; m < n; ++m) acc += P[r * n + m] * A[m * n + c];
                Q[r * n + c] = acc;
            }
        memcpy(P, Q, sizeof(double) * (size_t)(n * n));
    }
}

static bool xi_valid(const double* xi)
{
    if (!xi || !finite_all(xi, 6)) return false;
    const double th2 = xi[3] * xi[3] + xi[4] * xi[4] + xi[5] * xi[5];
    return th2 <= 100.0;   // |phi| <= 10 rad: the 40-term series converges to rounding
}

static void hat3(const double* w, double* M, int ld, int r0, int c0)
{
    M[(r0 + 0) * ld + c0 + 1] = -w[2];
    M[(r0 + 0) * ld + c0 + 2] = w[1];
    M[(r0 + 1) * ld + c0 + 0] = w[2];
    M[(r0 + 1) * ld + c0 + 2] = -w[0];
    M[(r0 + 2) * ld + c0 + 0] = -w[1];
    M[(r0 + 2) * ld + c0 + 1] = w[0];
}

constexpr int kSeriesTerms = 40;

kf_status kf_se3_compose(const double xi[6], const double T_in[16], double T_out[16])
{
    if (!xi_valid(xi)) return fail(KF_E_ARG, "xi must be finite with |phi| <= 10");
    kf_status s = check_rigid(T_in, "T_in");
    if (s != KF_OK) return s;
    if (!T_out) return fail(KF_E_ARG, "T_out is NULL");
    // exp of the twist [[phi^, rho], [0, 0]]
    double A[16] = {0}, E[16], coeff[kSeriesTerms];
    hat3(xi + 3, A, 4, 0, 0);
    for (int r = 0; r < 3; ++r) A[r * 4 + 3] = xi[r];
    coeff[0] = 1.0;
    for (int k = 1; k < kSeriesTerms; ++k) coeff[k] = coeff[k - 1] / k;
    matrix_series(A, 4, coeff, kSeriesTerms, E);
    double out[16];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int m = 0; m < 4; ++m) acc += E[r * 4 + m] * T_in[m * 4 + c];
            out[r * 4 + c] = acc;
        }
    out[12] = out[13] = out[14] = 0.0;
    out[15] = 1.0;
    memcpy(T_out, out, sizeof out);
    return KF_OK;
}

kf_status kf_se3_pullback(const double xi[6], const double d_eps[6], double d_xi[6])
{
    if (!xi_valid(xi)) return fail(KF_E_ARG, "xi must be finite with |phi| <= 10");
    if (!d_eps || !d_xi) return fail(KF_E_ARG, "NULL gradient");
    // left Jacobian J = sum_k ad^k / (k+1)!, ad = [[phi^, rho^], [0, phi^]]; d_xi = J^T d_eps
    double ad[36] = {0}, J[36], coeff[kSeriesTerms];
    hat3(xi + 3, ad, 6, 0, 0);
    hat3(xi, ad, 6, 0, 3);
    hat3(xi + 3, ad, 6, 3, 3);
    coeff[0] = 1.0;
    for (int k = 1; k < kSeriesTerms; ++k) coeff[k] = coeff[k - 1] / (k + 1);
    matrix_series(ad, 6, coeff, kSeriesTerms, J);
    double out[6];
    for (int c = 0; c < 6; ++c) {
        double acc = 0.0;
        for (int r = 0; r < 6; ++r) acc += J[r * 6 + c] * d_eps[r];
        out[c] = acc;
    }
    memcpy(d_xi, out, sizeof out);
    return KF_OK;
}

kf_status kf_texture_layout(int32_t n_tri, const float* tri, double size_pixel,
                            int32_t atlas_height, int32_t* rects, int32_t* atlas_width)
{
    if (n_tri < 0) return fail(KF_E_ARG, "n_tri must be >= 0");
    if (!atlas_width || (n_tri > 0 && (!tri || !rects))) return fail(KF_E_ARG, "NULL pointer");
    if (!isfinite(size_pixel) || !(size_pixel > 0.0))
        return fail(KF_E_ARG, "size_pixel must be finite and > 0");
    if (atlas_height < 2) return fail(KF_E_SHAPE, "atlas_height must be >= 2");
    int64_t x = 0, y = 0, column_w = 0;
    for (int32_t n = 0; n < n_tri; ++n) {
        const float* V = tri + 9 * (size_t)n;
        // squared lengths of V1V2 and V1V3, summed x, y, z in double
        double l12 = 0.0, l13 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double a = (double)V[3 + k] - (double)V[k];
            const double b = (double)V[6 + k] - (double)V[k];
            l12 += a * a;
            l13 += b * b;
        }
        // Eq. 11-12: a whole number of texels, rounded up, at least 2 per side
        const double wd = ceil(sqrt(l12) / size_pixel);
        const double hd = ceil(sqrt(l13) / size_pixel);
        if (!(wd <= 65535.0) || !(hd <= 65535.0))
            return fail(KF_E_RANGE, "triangle %d: map wider or taller than 65535 texels", (int)n);
        const int64_t w = wd < 2.0 ? 2 : (int64_t)wd;
        const int64_t h = hd < 2.0 ? 2 : (int64_t)hd;
        if (h > atlas_height)
            return fail(KF_E_RANGE, "triangle %d: map of %lld rows exceeds the atlas height",
                        (int)n, (long long)h);
        // column-wise from the top left: the next map goes below the previous one, or at the
        // top of a new column right of the widest map of this one when it does not fit
        if (y + h > atlas_height) {
            x += column_w;
            y = 0;
            column_w = 0;
        }
        if (x + w > 2147483647LL) return fail(KF_E_RANGE, "atlas wider than 2^31 - 1 texels");
        rects[4 * (size_t)n + 0] = (int32_t)x;
        rects[4 * (size_t)n + 1] = (int32_t)y;
        rects[4 * (size_t)n + 2] = (int32_t)w;
        rects[4 * (size_t)n + 3] = (int32_t)h;
        y += h;
        column_w = w > column_w ? w : column_w;
    }
    *atlas_width = (int32_t)(x + column_w);
    return KF_OK;
}

kf_status kf_texture_generate(kf_volume* vol, int32_t n_tri, const float* tri,
                              const int32_t* rects, int32_t atlas_width, int32_t atlas_height,
                              float* atlas_rgb, uint8_t* atlas_rgb8, void* stream)
{
    kf_status s;
    if ((s = check_volume(vol)) != KF_OK) return s;
    if (n_tri < 0) return fail(KF_E_ARG, "n_tri must be >= 0");
    if (n_tri > 0 && (!tri || !rects)) return fail(KF_E_ARG, "NULL triangles or rects");
    if (!atlas_rgb && !atlas_rgb8) return fail(KF_E_ARG, "both atlas outputs are NULL");
    if (atlas_width < 0 || atlas_height < 0) return fail(KF_E_SHAPE, "negative atlas size");
    if ((double)atlas_width * atlas_height * 3.0 > 9007199254740992.0)
        return fail(KF_E_RANGE, "atlas too large");
    if (n_tri > 2147483647 / 9) return fail(KF_E_RANGE, "too many triangles");
    const kf_volume_desc& d = vol->desc;
    for (int k = 0; k < 3; ++k)
        if (d.colour_dim[k] < 2)
            return fail(KF_E_SHAPE, "texture lookup needs at least 2 colour voxels per axis");
    kf::TextureArgs a;
    memset(&a, 0, sizeof a);
    for (int k = 0; k < 3; ++k) {
        const double sc = d.extent[k] / d.colour_dim[k];
        // colour index of a world point p: p / s - (origin / s + 1/2), voxel i's centre at i
        a.inv_s[k] = (float)(1.0 / sc);
        a.off[k] = (float)(-d.origin[k] / sc - 0.5);
        a.cmax[k] = (float)(d.colour_dim[k] - 1);
        a.cdim[k] = d.colour_dim[k];
    }
    a.n_tri = n_tri;
    a.atlas_width = atlas_width;
    a.atlas_height = atlas_height;
    a.tri = tri;
    a.rects = rects;
    a.r = vol->bufs.r;
    a.g = vol->bufs.g;
    a.b = vol->bufs.b;
    a.wc = vol->bufs.w_col;
    a.atlas = atlas_rgb;
    a.atlas8 = atlas_rgb8;
    KF_HIP(kf::launch_texture(a, (hipStream_t)stream), "texture launch");
    return KF_OK;
}

}  // extern "C"
