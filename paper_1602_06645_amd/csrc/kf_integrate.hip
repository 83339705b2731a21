// Forward integration kernels for gfx950: TSDF geometry volume (Sec. III) and asymmetric
// colour volume (Sec. IV.B, Eq. 5-10, with the depth-to-HD mapping of Eq. 1-4).
//
// A pass applies up to 64 consecutive frames of every scan in the launch:
//   1. pyramid kernels: per frame, min/max of the valid depths over 2x2-pixel tiles and
//      their 2x2 reductions (built once per batch call for all frames);
//   2. cull kernel: one thread per (brick, frame) decides whether any voxel of the
//      brick can pass the depth tests (conservatively, from the brick's corners and the
//      pyramid) and appends (brick, frame mask) of the live bricks to a heavy or a light
//      list by the number of frames in the mask;
//   3. integrate kernels (one launch for geometry bricks, one for colour bricks):
//      persistent waves take live bricks from the lists, heavy ones first; each lane
//      keeps its column's voxels in registers for all frames of the pass, reads a
//      voxel's state only when a frame first needs it and writes it back only if it was
//      read.
// Culling never changes a result: a brick is dropped for a frame only if every voxel in
// it would have been rejected before touching its state.
//
// Arithmetic is IEEE single precision in a fixed order: explicit fmaf, correctly rounded
// division and square root, rintf for the nearest depth pixel, floorf for the HD cell.
// The library is compiled with -ffp-contract=off, so nothing else is fused.
#include <hip/hip_runtime.h>

#include <utility>

#include "kf_cull.h"
#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

namespace {

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

// One channel of an HD pixel as a value in [0,1] (8-bit input is scaled before any
// interpolation, so 8-bit and the equivalent float image give identical volumes).
template <int FMT>
__device__ __forceinline__ float hd_px(const void* rgb, int idx)
{
    if constexpr (FMT == FMT_RGB8)
        return (float)((const uint8_t*)rgb)[idx] * (float)(1.0 / 255.0);
    else
        return ((const float*)rgb)[idx];
}

// HD sample of channel ch (Eq. 9's HD(x_hd, y_hd)): bilinear between pixel centres at the
// cell whose top-left pixel's first channel is at `cell`, or (nearest) that pixel alone.
__device__ __forceinline__ float hd_sample(const void* rgb, int fmt, bool nearest, int cell, int row,
                                           int ch, float ax, float ay)
{
    if (nearest)
        return fmt == FMT_RGB8 ? hd_px<FMT_RGB8>(rgb, cell + ch) : hd_px<FMT_RGBF32>(rgb, cell + ch);
    float p00, p10, p01, p11;
    if (fmt == FMT_RGB8) {
        p00 = hd_px<FMT_RGB8>(rgb, cell + ch);
        p10 = hd_px<FMT_RGB8>(rgb, cell + 3 + ch);
        p01 = hd_px<FMT_RGB8>(rgb, cell + row + ch);
        p11 = hd_px<FMT_RGB8>(rgb, cell + row + 3 + ch);
    } else {
        p00 = hd_px<FMT_RGBF32>(rgb, cell + ch);
        p10 = hd_px<FMT_RGBF32>(rgb, cell + 3 + ch);
        p01 = hd_px<FMT_RGBF32>(rgb, cell + row + ch);
        p11 = hd_px<FMT_RGBF32>(rgb, cell + row + 3 + ch);
    }
    return lerp(lerp(p00, p10, ax), lerp(p01, p11, ax), ay);
}

// The three channels of the HD sample (hd_sample's values).  An 8-bit bilinear sample
// reads each of its two rows as one 4-byte and one 2-byte load: the six bytes of the cell's
// two pixels, at byte addresses (unaligned loads).
__device__ __forceinline__ void hd_sample3(const void* rgb, int fmt, bool nearest, int cell, int row,
                                           float ax, float ay, float* s)
{
    if (fmt == FMT_RGB8 && !nearest) {
        const uint8_t* p = (const uint8_t*)rgb + cell;
        uint32_t a0, a1;
        uint16_t b0, b1;
        __builtin_memcpy(&a0, p, 4);
        __builtin_memcpy(&b0, p + 4, 2);
        __builtin_memcpy(&a1, p + row, 4);
        __builtin_memcpy(&b1, p + row + 4, 2);
        const float k = (float)(1.0 / 255.0);
        auto px = [k](uint32_t w, int n) { return (float)((w >> (8 * n)) & 0xFFu) * k; };
        // channel ch of the left pixel is byte ch of the row, of the right pixel byte 3 + ch
        s[0] = lerp(lerp(px(a0, 0), px(a0, 3), ax), lerp(px(a1, 0), px(a1, 3), ax), ay);
        s[1] = lerp(lerp(px(a0, 1), px(b0, 0), ax), lerp(px(a1, 1), px(b1, 0), ax), ay);
        s[2] = lerp(lerp(px(a0, 2), px(b0, 1), ax), lerp(px(a1, 2), px(b1, 1), ax), ay);
        return;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) s[ch] = hd_sample(rgb, fmt, nearest, cell, row, ch, ax, ay);
}

struct Counts {
    unsigned long long g_upd = 0, g_touch = 0, c_eval = 0, c_read = 0, c_upd = 0, c_touch = 0;
    unsigned long long g_bricks = 0, c_bricks = 0;   // brick-frames (same in every lane)
};

// Voxel column of a lane in brick li of a volume with brick shape BX x BY x BZ.  The
// brick's z slab (BZ slices from k0) is wave-uniform: state arrays are read through a
// buffer resource based at the slab, with per-lane byte offsets off + kk * zstride.
struct Column {
    int i, j, k0, kn;
    size_t base, slice, slab;   // element index of (i, j, k0); elements per slice; of (0, 0, k0)
    uint32_t off, zstride, slab_bytes;
    bool active;
};

template <int BX, int BY, int BZ, class Dims>
__device__ __forceinline__ Column column(const Dims& dim, const Dims& bricks, uint32_t li)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const uint32_t bx = li % (uint32_t)bricks[0];
    const uint32_t rest = li / (uint32_t)bricks[0];
    const uint32_t by = rest % (uint32_t)bricks[1];
    const uint32_t bz = rest / (uint32_t)bricks[1];
    Column c;
    c.i = (int)bx * BX + lane % BX;
    c.j = (int)by * BY + lane / BX;
    c.k0 = (int)bz * BZ;
    c.kn = min(BZ, dim[2] - c.k0);
    c.active = c.i < dim[0] && c.j < dim[1];
    c.slice = (size_t)dim[0] * (size_t)dim[1];
    c.slab = (size_t)c.k0 * c.slice;
    c.base = c.slab + (size_t)c.j * (size_t)dim[0] + (size_t)c.i;
    c.off = ((uint32_t)c.j * (uint32_t)dim[0] + (uint32_t)c.i) * 4u;
    c.zstride = (uint32_t)c.slice * 4u;
    c.slab_bytes = (uint32_t)c.kn * c.zstride;
    return c;
}

// ------------------------------------------------------------------ image fetches

// Depth maps are read through a bounds-checked buffer resource: an offset past the image
// reads 0 (a hole), so a voxel outside the frustum needs no separate branch.
constexpr uint32_t kOutside = 0x7FFFFFF0u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ float load_f32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

__device__ __forceinline__ float4 load_f32x4(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
    float4 f;
    __builtin_memcpy(&f, &v, sizeof f);
    return f;
}

// Nearest depth pixel of camera point (X, Y, Z) (Eq. 6 with the perspective division):
// the pixel as floats, whether it lies inside the image, and its index (valid only when it
// does).
struct Pixel {
    float u, v;
    bool inside;
    uint32_t pix;   // v * width + u
};

// A uniform value copied into a VGPR once, so that an operation with another uniform
// operand (the VOP3 forms read at most one SGPR) does not re-copy it per voxel.
__device__ __forceinline__ float in_vgpr(float x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Frame constants of the projection held per lane for a frame's sweep.
struct ProjRegs {
    float cx, cy;
};

template <class C>
__device__ __forceinline__ ProjRegs proj_regs(const C& c)
{
    return {in_vgpr(c.cx), in_vgpr(c.cy)};
}

// EXACT: the caller has established recip_exact(Z) for the whole column, and zpos is
// whether its depths are positive (one sign for the column).
template <bool EXACT, class C>
__device__ __forceinline__ Pixel project(const C& c, const ProjRegs& pr, float X, float Y, float Z,
                                         bool zpos)
{
    Pixel p;
    const float iz = EXACT ? recip_newton(Z) : recip(Z);
    p.u = rintf(fmaf(c.fx, X * iz, pr.cx));
    p.v = rintf(fmaf(c.fy, Y * iz, pr.cy));
    const bool front = EXACT ? zpos : (Z > 0.0f);
    p.inside = front & (p.u >= 0.0f) & (p.u <= c.wm1) & (p.v >= 0.0f) & (p.v <= c.hm1);
    // the pixel's index, meaningful only when inside (then the pixel is below 2^24 and the
    // 24-bit multiply exact); callers select it with their own conditions
    p.pix = __umul24((uint32_t)(int)p.v, (uint32_t)c.dw) + (uint32_t)(int)p.u;
    return p;
}

// Buffer resource over the lane column's z slab of one state array (see Column).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(float* p, const Column& col)
{
    return image_rsrc(p + col.slab, col.slab_bytes);
}

// ------------------------------------------------------------------ geometry (Sec. III)

// Projective TSDF with running average for the frames of `mask` (bit f = frame f of the
// pass).  The column's state lives in registers for the whole pass: read from HBM when a
// frame first updates a voxel, written back at the end if it was read.  Per frame, the
// eight depth samples of the column are fetched before any of them is used.  MODE_STATUS
// writes the outcome code of the (single) frame instead.
template <int MODE, int BX, int BY, int BZ, class Scene, class FramePtr>
__device__ __forceinline__ void geom_brick(const Scene& sc, FramePtr frames, unsigned long long mask,
                                           uint32_t li, uint8_t* status, Counts& cnt)
{
    static_assert(BX * BY == WAVE && BZ <= MAX_BZ, "one lane per column, masks of 32 bits");
    const Column col = column<BX, BY, BZ>(sc.gdim, sc.gbricks, li);
    if (!col.active) return;
    const float fi = (float)col.i, fj = (float)col.j;
    float F[BZ], W[BZ];
    // The column's state is read whole at its first update of the pass and written back
    // whole at the end (a voxel that no frame updated gets its own value back).  Per-voxel
    // flags are one bool per voxel, held as lane masks in scalar registers, so testing them
    // costs no vector instruction.
    bool loaded = false;
    bool touched[BZ];   // counted only: voxels updated in the pass
#pragma unroll
    for (int kk = 0; kk < BZ; ++kk) {
        F[kk] = W[kk] = 0.0f;
        touched[kk] = false;
    }
    unsigned long long n_upd = 0;
    for (unsigned long long m = mask; m; m &= m - 1) {
        const auto& c = frames[__builtin_ctzll(m)];
        const __amdgpu_buffer_rsrc_t depth = image_rsrc(c.depth, (uint32_t)(c.dw * c.dh) * 4u);
        // Eq. 5 for this column; the z term is added per voxel.
        const float cX = fmaf(c.Ag[1], fj, fmaf(c.Ag[0], fi, c.bg[0]));
        const float cY = fmaf(c.Ag[4], fj, fmaf(c.Ag[3], fi, c.bg[1]));
        const float cZ = fmaf(c.Ag[7], fj, fmaf(c.Ag[6], fi, c.bg[2]));
        const ProjRegs pr = proj_regs(c);
        const float z_first = fmaf(c.Ag[8], (float)col.k0, cZ);
        const bool zpos = z_first > 0.0f;
        float sdf[BZ];
        bool upd[BZ];
        auto sweep = [&](auto exact) {
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) {
                const float fk = (float)(col.k0 + kk);
                const float Zc = fmaf(c.Ag[8], fk, cZ);
                const Pixel px = project<decltype(exact)::value>(c, pr, fmaf(c.Ag[2], fk, cX),
                                                                 fmaf(c.Ag[5], fk, cY), Zc, zpos);
                const bool in = px.inside & (kk < col.kn);
                const float d = load_f32(depth, in ? px.pix * 4u : kOutside);
                const bool valid = in & valid_depth(d);
                sdf[kk] = d - Zc;
                upd[kk] = valid & !(sdf[kk] < -c.trunc);
                if constexpr (MODE == MODE_STATUS) {
                    if (kk < col.kn)
                        status[col.base + (size_t)kk * col.slice] = (uint8_t)(!px.inside ? 0 : !valid ? 1 : upd[kk] ? 6 : 2);
                }
            }
        };
        // the per-voxel range test of the reciprocal, once per column and frame (a branch
        // every lane takes the same way unless a column reaches the camera plane)
        if (column_recip_exact(z_first, fmaf(c.Ag[8], (float)(col.k0 + BZ - 1), cZ)))
            sweep(std::true_type{});
        else
            sweep(std::false_type{});
        if constexpr (MODE != MODE_STATUS) {
            bool any = false;
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) any |= upd[kk];
            if (any & !loaded) {
                const __amdgpu_buffer_rsrc_t tr = slab_rsrc(sc.tsdf, col), wr = slab_rsrc(sc.wg, col);
#pragma unroll
                for (int kk = 0; kk < BZ; ++kk) {
                    const uint32_t o = col.off + (uint32_t)kk * col.zstride;   // past the slab: 0
                    F[kk] = load_f32(tr, o);
                    W[kk] = load_f32(wr, o);
                }
                loaded = true;
            }
            // the truncated distances, then the divisions of the voxels whose distance
            // changes, then the weights of all voxels without branches (in_vgpr keeps
            // min(W + 1, w_max) in that one block of code, next to its addition, where it
            // needs no quieting of its operands)
            float t[BZ];
            bool dv[BZ];
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) {
                t[kk] = fminf(1.0f, sdf[kk] * c.inv_trunc);
                // F + (t - F) / (W + 1) is F itself when t and F are the same float (then
                // t - F = +0), except for F = -0: skip the division in that case (free
                // space seen again, t = F = 1).
                const uint32_t tb = __builtin_bit_cast(uint32_t, t[kk]);
                const uint32_t fb = __builtin_bit_cast(uint32_t, F[kk]);
                dv[kk] = upd[kk] & ((tb != fb) | (fb == 0x80000000u));
                if constexpr (MODE == MODE_COUNT) {
                    n_upd += upd[kk] ? 1u : 0u;
                    touched[kk] |= upd[kk];
                }
            }
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk)
                if (dv[kk]) F[kk] = F[kk] + (t[kk] - F[kk]) / (W[kk] + 1.0f);
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) {
                const float wc = in_vgpr(fminf(W[kk] + 1.0f, c.w_max));
                W[kk] = upd[kk] ? wc : W[kk];
            }
        }
    }
    if constexpr (MODE != MODE_STATUS) {
        if (loaded) {
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) {
                if (kk < col.kn) {
                    sc.tsdf[col.base + (size_t)kk * col.slice] = F[kk];
                    sc.wg[col.base + (size_t)kk * col.slice] = W[kk];
                }
            }
        }
    }
    if constexpr (MODE == MODE_COUNT) {
        cnt.g_upd += n_upd;
#pragma unroll
        for (int kk = 0; kk < BZ; ++kk) cnt.g_touch += touched[kk] ? 1u : 0u;
    }
}

// --------------------------------------------------------------- colour (Sec. IV.B)

// HD pixel of a colour voxel centre (Eq. 3-5 composed into one affine map, then Eq. 4's
// division) and its bilinear cell (inside when the cell's four pixels are in the image),
// or the nearest pixel (inside when it is in the image).
struct HdCell {
    bool inside;
    int cell;        // index of the cell's top-left pixel's first channel
    float ax, ay;    // bilinear weights along x and y
};

template <class C>
__device__ __forceinline__ HdCell hd_cell(const C& c, float fi, float fj, float fk)
{
    const float qx = fmaf(c.Ah[2], fk, fmaf(c.Ah[1], fj, fmaf(c.Ah[0], fi, c.bh[0])));
    const float qy = fmaf(c.Ah[5], fk, fmaf(c.Ah[4], fj, fmaf(c.Ah[3], fi, c.bh[1])));
    const float qz = fmaf(c.Ah[8], fk, fmaf(c.Ah[7], fj, fmaf(c.Ah[6], fi, c.bh[2])));
    const float iqz = recip(qz);
    const float xh = fmaf(c.fxr, qx * iqz, c.cxr);
    const float yh = fmaf(c.fyr, qy * iqz, c.cyr);
    const float x0 = c.hd_nearest ? rintf(xh) : floorf(xh), y0 = c.hd_nearest ? rintf(yh) : floorf(yh);
    HdCell h;
    h.inside = (qz > 0.0f) & (x0 >= 0.0f) & (x0 <= c.hd_xmax) & (y0 >= 0.0f) & (y0 <= c.hd_ymax);
    h.ax = xh - x0;
    h.ay = yh - y0;
    h.cell = h.inside ? ((int)y0 * c.cw + (int)x0) * 3 : 0;
    return h;
}

// Sec. IV.B in the paper's order of tests, then Eq. 9 and Eq. 10, for the frames of mask.
// Per frame, in stages over the column's voxels so that the loads of a stage are in flight
// together: (1) frustum, depth and sigma tests, each voxel reading its pixel's map entry
// (depth, Eq. 7's P, Eq. 8's weight); (2)-(3) the voxels in the band whose pixel has a
// normal, and the gate against the running weight; (4) HD pixel, Eq. 9 and Eq. 10 for the
// gated voxels, shared out over the wave.  The column's colour state lives in registers
// for the whole pass.
template <int MODE, int BX, int BY, int BZ, class Scene, class FramePtr>
__device__ __forceinline__ void colour_brick(const Scene& sc, FramePtr frames, unsigned long long mask,
                                             uint32_t li, uint8_t* status, float4* slots, Counts& cnt)
{
    static_assert(BX * BY == WAVE && BZ <= MAX_BZ && BZ <= 64, "one lane per column, masks of 32 bits");
    const Column col = column<BX, BY, BZ>(sc.cdim, sc.cbricks, li);
    // a column outside the volume (a partial brick) stays with the wave, touching nothing:
    // its voxels never pass the first test, and its lane takes sampling jobs in stage 4
    const int lane = threadIdx.x & (WAVE - 1);
    const float fi = (float)col.i, fj = (float)col.j;
    float R[BZ], G[BZ], B[BZ], Wt[BZ];
    // The column's colour weights are read whole when a voxel of it first reaches the gate,
    // its colours when one first passes it; the column is written back whole if its colours
    // were read (a voxel that no frame updated gets its own values back).  Per-voxel flags
    // are one bool per voxel, held as lane masks in scalar registers.
    bool wl = false, cl = false;
    bool rd[BZ], tc[BZ];   // counted only: voxels whose weight was read / that were updated
#pragma unroll
    for (int kk = 0; kk < BZ; ++kk) {
        R[kk] = G[kk] = B[kk] = Wt[kk] = 0.0f;
        rd[kk] = tc[kk] = false;
    }
    unsigned long long n_eval = 0, n_upd = 0;
    for (unsigned long long m = mask; m; m &= m - 1) {
        const auto& c = frames[__builtin_ctzll(m)];
        const __amdgpu_buffer_rsrc_t pmap = image_rsrc(c.pmap, (uint32_t)(c.dw * c.dh) * 16u);
        const float cX = fmaf(c.Ac[1], fj, fmaf(c.Ac[0], fi, c.bc[0]));
        const float cY = fmaf(c.Ac[4], fj, fmaf(c.Ac[3], fi, c.bc[1]));
        const float cZ = fmaf(c.Ac[7], fj, fmaf(c.Ac[6], fi, c.bc[2]));
        const ProjRegs pr = proj_regs(c);
        const float z_first = fmaf(c.Ac[8], (float)col.k0, cZ);
        const bool zpos = z_first > 0.0f;
        int st[BZ];
        // (1) Eq. 5-7 and the distance test against sigma: the voxel's depth pixel gives its
        // depth, P (Eq. 7) and W from the frame's pixel map in one read; W is kept for the
        // voxels in the band.
        float wv[BZ];
        bool band[BZ];
        auto sweep = [&](auto exact) {
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) {
                const float fk = (float)(col.k0 + kk);
                const float Xc = fmaf(c.Ac[2], fk, cX);
                const float Yc = fmaf(c.Ac[5], fk, cY);
                const float Zc = fmaf(c.Ac[8], fk, cZ);
                const Pixel px = project<decltype(exact)::value>(c, pr, Xc, Yc, Zc, zpos);
                const bool in = px.inside & (kk < col.kn) & col.active;
                const float4 pm = load_f32x4(pmap, in ? px.pix * 16u : kOutside);
                const float d = pm.x;
                const bool valid = in & valid_depth(d);
                const float dx = Xc - pm.y, dy = Yc - pm.z, dz = Zc - d;
                const float dist2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const bool bd = valid & !(dist2 > c.sigma2);
                band[kk] = bd;
                wv[kk] = bd ? pm.w : 0.0f;
                if constexpr (MODE == MODE_STATUS) st[kk] = !px.inside ? 0 : !valid ? 1 : bd ? 3 : 2;
            }
        };
        // the per-voxel range test of the reciprocal, once per column and frame (a branch
        // every lane takes the same way unless a column reaches the camera plane)
        if (column_recip_exact(z_first, fmaf(c.Ac[8], (float)(col.k0 + BZ - 1), cZ)))
            sweep(std::true_type{});
        else
            sweep(std::false_type{});
        // (2)-(3) the voxels in the band whose pixel has a normal (W of the pixel map: the
        // Eq. 8 normal from the neighbours (u+1, v) and (u, v+1), dotted with the unit
        // viewing direction), the read of the column's colour weights when one of them first
        // reaches this point, and the gate against the running weight.
        bool gate[BZ], any_band = false, any_gate = false;
#pragma unroll
        for (int kk = 0; kk < BZ; ++kk) {
            gate[kk] = false;
            any_band |= band[kk];
        }
        if (any_band) {
            bool reach[BZ], any_reach = false;
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) {
                reach[kk] = band[kk] & (__builtin_bit_cast(uint32_t, wv[kk]) != kNoNormal);
                any_reach |= reach[kk];
            }
            if (any_reach & !wl) {
                const __amdgpu_buffer_rsrc_t wr = slab_rsrc(sc.wc, col);
#pragma unroll
                for (int kk = 0; kk < BZ; ++kk) Wt[kk] = load_f32(wr, col.off + (uint32_t)kk * col.zstride);
                wl = true;
            }
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) {
                const bool gk = reach[kk] & (wv[kk] > c.gate * Wt[kk]);
                gate[kk] = gk;
                any_gate |= gk;
                if constexpr (MODE == MODE_COUNT) {
                    n_eval += reach[kk] ? 1u : 0u;
                    rd[kk] |= reach[kk];
                }
                if constexpr (MODE == MODE_STATUS)
                    if (reach[kk]) st[kk] = gk ? 5 : 4;
            }
        }
        // (4) for every gated voxel of the wave: the HD pixel of its centre (Eq. 3-5), the
        // bilinear cell inside the image, the HD sample (Eq. 9's HD(x, y)) and
        // alpha = W / (W_c + W) (Eq. 10's update as a blend).  Gated voxels are few and
        // scattered over the wave's lanes, so they are numbered (z slice by z slice, lanes
        // in order) and handed out to the active lanes in turn through LDS: a lane computes
        // the sample of another lane's voxel, and the owner blends the result into its
        // registers.  Same operations on the same values as in the owner's lane.
        if (__ballot(any_gate)) {
            if constexpr (MODE != MODE_STATUS) {
                if (any_gate & !cl) {
                    const __amdgpu_buffer_rsrc_t rr = slab_rsrc(sc.r, col), gr = slab_rsrc(sc.g, col),
                                                 br = slab_rsrc(sc.b, col);
#pragma unroll
                    for (int kk = 0; kk < BZ; ++kk) {
                        const uint32_t o = col.off + (uint32_t)kk * col.zstride;
                        R[kk] = load_f32(rr, o);
                        G[kk] = load_f32(gr, o);
                        B[kk] = load_f32(br, o);
                    }
                    cl = true;
                }
            }
            const unsigned long long act = __ballot(1);
            const uint32_t n_act = (uint32_t)__builtin_popcountll(act);
            const uint32_t wrank = lane_rank(act);
            uint32_t total = 0;
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) total += (uint32_t)__builtin_popcountll(__ballot(gate[kk]));
            const int i0 = col.i - lane % BX, j0 = col.j - lane / BX;   // the brick's first column
            const int row = c.cw * 3;
            const bool nearest = c.hd_nearest != 0;
            bool upd[BZ];
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) upd[kk] = false;
            for (uint32_t r0 = 0; r0 < total; r0 += n_act) {
                // jobs r0 .. r0 + n_act - 1: each owner puts (voxel, W, W_c) into the slot
                // of the lane that takes the job
                uint32_t first = 0;
#pragma unroll
                for (int kk = 0; kk < BZ; ++kk) {
                    const bool gk = gate[kk];
                    const unsigned long long b = __ballot(gk);
                    const uint32_t q = first + lane_rank(b) - r0;
                    if (gk && q < n_act)
                        slots[q] = make_float4(__builtin_bit_cast(float, (uint32_t)(lane | kk << 6)), wv[kk],
                                               Wt[kk], 0.0f);
                    first += (uint32_t)__builtin_popcountll(b);
                }
                __builtin_amdgcn_wave_barrier();
                if (r0 + wrank < total) {
                    const float4 job = slots[wrank];
                    const uint32_t code = __builtin_bit_cast(uint32_t, job.x);
                    const int l = (int)(code & 63u), kk = (int)(code >> 6);
                    const HdCell h = hd_cell(c, (float)(i0 + l % BX), (float)(j0 + l / BX), (float)(col.k0 + kk));
                    float4 res = make_float4(-1.0f, 0.0f, 0.0f, 0.0f);   // alpha < 0: outside the image
                    if (h.inside) {
                        res.x = job.y / (job.z + job.y);
                        if constexpr (MODE != MODE_STATUS) {
                            float smp[3];
                            hd_sample3(c.rgb, sc.fmt, nearest, h.cell, row, h.ax, h.ay, smp);
                            res.y = smp[0];
                            res.z = smp[1];
                            res.w = smp[2];
                        }
                    }
                    slots[wrank] = res;
                }
                __builtin_amdgcn_wave_barrier();
                // each owner blends its results (Eq. 9 and Eq. 10 as running averages)
                first = 0;
#pragma unroll
                for (int kk = 0; kk < BZ; ++kk) {
                    const bool gk = gate[kk];
                    const unsigned long long b = __ballot(gk);
                    const uint32_t q = first + lane_rank(b) - r0;
                    if (gk && q < n_act) {
                        const float4 res = slots[q];
                        if (res.x >= 0.0f) {
                            if constexpr (MODE == MODE_STATUS) {
                                st[kk] = 6;
                            } else {
                                R[kk] = fmaf(res.x, res.y - R[kk], R[kk]);
                                G[kk] = fmaf(res.x, res.z - G[kk], G[kk]);
                                B[kk] = fmaf(res.x, res.w - B[kk], B[kk]);
                                Wt[kk] = fmaf(wv[kk], 1.0f - Wt[kk], Wt[kk]);
                            }
                            upd[kk] = true;
                        }
                    }
                    first += (uint32_t)__builtin_popcountll(b);
                }
                __builtin_amdgcn_wave_barrier();   // the slots are free for the next round
            }
            if constexpr (MODE == MODE_COUNT) {
#pragma unroll
                for (int kk = 0; kk < BZ; ++kk) {
                    n_upd += upd[kk] ? 1u : 0u;
                    tc[kk] |= upd[kk];
                }
            }
        }
        if constexpr (MODE == MODE_STATUS) {
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk)
                if (col.active && kk < col.kn) status[col.base + (size_t)kk * col.slice] = (uint8_t)st[kk];
        }
    }
    if constexpr (MODE != MODE_STATUS) {
        if (cl) {   // a column outside the volume never reads
#pragma unroll
            for (int kk = 0; kk < BZ; ++kk) {
                if (kk < col.kn) {
                    const size_t idx = col.base + (size_t)kk * col.slice;
                    sc.r[idx] = R[kk];
                    sc.g[idx] = G[kk];
                    sc.b[idx] = B[kk];
                    sc.wc[idx] = Wt[kk];
                }
            }
        }
    }
    if constexpr (MODE == MODE_COUNT) {
        cnt.c_eval += n_eval;
        cnt.c_upd += n_upd;
#pragma unroll
        for (int kk = 0; kk < BZ; ++kk) {
            cnt.c_read += rd[kk] ? 1u : 0u;
            cnt.c_touch += tc[kk] ? 1u : 0u;
        }
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

}  // namespace

// One wave per culling chunk (CHUNK^3 bricks of one kind), four chunks per block, each
// wave on its own: it tests the chunk's voxel box against the frames of the pass (one lane
// per frame), then its bricks (one lane per brick) against each frame the chunk passed in
// turn, the frame being wave-uniform there so that its constants come through scalar
// loads; a lane collects its brick's frame mask in a register.  Skipping the other frames
// is exact: the chunk test is conservative for every voxel of the chunk, as the brick test
// is for every voxel of the brick.  The wave then appends its bricks with a non-empty mask
// to the heavy or the light list in brick order, with one atomic per list (geometry from
// the front, colour from the back).
constexpr int CHUNK_BRICKS = CHUNK * CHUNK * CHUNK;
static_assert(CHUNK_BRICKS <= WAVE, "one lane per brick of a chunk");
constexpr int CULL_WAVES = BLOCK / WAVE;   // chunks per block

__global__ __launch_bounds__(BLOCK) void cull_kernel(CullArgs a)
{
    const uint32_t chunk = first_lane_u32(blockIdx.x * (uint32_t)CULL_WAVES + threadIdx.x / WAVE);
    if (chunk >= a.n_chunks) return;
    int s = 0;
    while (s + 1 < a.n_scenes && a.scenes[s + 1].chunk_begin <= chunk) ++s;
    const SceneDev& sc = a.scenes[s];
    uint32_t lc = chunk - sc.chunk_begin;
    const bool colour = lc >= sc.geom_chunks;
    if (colour) lc -= sc.geom_chunks;
    const int32_t* dim = colour ? sc.cdim : sc.gdim;
    const int32_t* nb = colour ? sc.cbricks : sc.gbricks;
    const int32_t* nc = colour ? sc.cchunks : sc.gchunks;
    const int32_t* shape = colour ? sc.cshape : sc.gshape;
    const int BX = shape[0], BY = shape[1], BZ = shape[2];
    const int bx0 = (int)(lc % (uint32_t)nc[0]) * CHUNK;
    const int by0 = (int)((lc / (uint32_t)nc[0]) % (uint32_t)nc[1]) * CHUNK;
    const int bz0 = (int)(lc / ((uint32_t)nc[0] * (uint32_t)nc[1])) * CHUNK;
    const int nbx = min(CHUNK, nb[0] - bx0), nby = min(CHUNK, nb[1] - by0), nbz = min(CHUNK, nb[2] - bz0);
    const FrameConsts* frames = a.frames + sc.frame_begin;
    const int lane = threadIdx.x & (WAVE - 1);
    bool chunk_live = false;
    if (lane < sc.n_frames) {
        const int i0 = bx0 * BX, i1 = min(dim[0], (bx0 + nbx) * BX) - 1;
        const int j0 = by0 * BY, j1 = min(dim[1], (by0 + nby) * BY) - 1;
        const int k0 = bz0 * BZ, k1 = min(dim[2], (bz0 + nbz) * BZ) - 1;
        chunk_live = a.disable || brick_live(frames[lane], colour, i0, i1, j0, j1, k0, k1);
    }
    const unsigned long long fm = __ballot(chunk_live);
    if (fm == 0ull) return;   // no brick of the chunk is live
    const uint32_t nbr = (uint32_t)(nbx * nby * nbz);
    const uint32_t q = (uint32_t)lane;
    const int bx = bx0 + (int)(q % (uint32_t)nbx), by = by0 + (int)((q / (uint32_t)nbx) % (uint32_t)nby);
    const int bz = bz0 + (int)(q / (uint32_t)(nbx * nby));
    unsigned long long mask = 0ull;
    {
        const int i0 = bx * BX, i1 = min(dim[0], i0 + BX) - 1;
        const int j0 = by * BY, j1 = min(dim[1], j0 + BY) - 1;
        const int k0 = bz * BZ, k1 = min(dim[2], k0 + BZ) - 1;
        const const_ptr<FrameConsts> cframes = as_const(frames);
        for (unsigned long long m = fm; m; m &= m - 1) {   // wave-uniform
            const int f = __builtin_ctzll(m);
            if (q < nbr && (a.disable || brick_live(cframes[f], colour, i0, i1, j0, j1, k0, k1)))
                mask |= 1ull << f;
        }
    }
    const unsigned long long has = __ballot(mask != 0ull);
    if (has == 0ull) return;
    // bricks live in at least half of the pass's frames go to the heavy list, which the
    // integration drains first (longest first shortens the launch's tail)
    const bool heavy = 2u * (uint32_t)__builtin_popcountll(mask) >= (uint32_t)a.max_frames;
    const unsigned long long hv = __ballot(mask != 0ull && heavy), lt = has & ~hv;
    const int kind = colour ? KIND_COLOUR : KIND_GEOM;
    uint32_t base_h = 0, base_l = 0;
    if (lane == 0) {
        if (hv) base_h = atomicAdd(a.n_live + kind, (uint32_t)__builtin_popcountll(hv));
        if (lt) base_l = atomicAdd(a.n_live + 2 + kind, (uint32_t)__builtin_popcountll(lt));
    }
    base_h = __shfl(base_h, 0, WAVE);
    base_l = __shfl(base_l, 0, WAVE);
    if (mask != 0ull) {
        const uint32_t li = (uint32_t)bx + (uint32_t)nb[0] * ((uint32_t)by + (uint32_t)nb[1] * (uint32_t)bz);
        const uint32_t item = sc.item_begin + (colour ? sc.geom_items : 0u) + li;
        const unsigned long long below = (1ull << lane) - 1ull;
        const bool h = (hv >> lane) & 1ull;
        const uint32_t pos = h ? base_h + (uint32_t)__builtin_popcountll(hv & below)
                               : base_l + (uint32_t)__builtin_popcountll(lt & below);
        uint4* list = a.live + (h ? 0u : a.n_items);
        list[colour ? a.n_items - 1u - pos : pos] = make_uint4(item, (uint32_t)mask, (uint32_t)(mask >> 32), 0u);
    }
}

// ------------------------------------------------------------------- depth pyramid

// Level 0: one lane per 2x2 tile of one frame (blockIdx.y = frame).
__global__ __launch_bounds__(BLOCK) void pyramid_base_kernel(const FrameConsts* frames)
{
    const FrameConsts& c = frames[blockIdx.y];
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= c.pyr_w0 * c.pyr_h0) return;
    const int tx = t % c.pyr_w0, ty = t / c.pyr_w0;
    float dmin = __builtin_huge_valf(), dmax = -__builtin_huge_valf();
    const int u0 = tx << PYR_SHIFT, v0 = ty << PYR_SHIFT;
    const int u1 = min(c.dw, u0 + (1 << PYR_SHIFT)), v1 = min(c.dh, v0 + (1 << PYR_SHIFT));
    for (int v = v0; v < v1; ++v)
        for (int u = u0; u < u1; ++u) {
            const float d = c.depth[v * c.dw + u];
            if (valid_depth(d)) {
                dmin = fminf(dmin, d);
                dmax = fmaxf(dmax, d);
            }
        }
    c.pyr[t] = make_float2(dmin, dmax);
}

// Levels 1.. : one block of 16 waves per frame, each level the 2x2 reduction of the
// previous one.
constexpr int PYR_UP_BLOCK = 1024;

__global__ __launch_bounds__(PYR_UP_BLOCK) void pyramid_up_kernel(const FrameConsts* frames)
{
    const FrameConsts& c = frames[blockIdx.x];
    int w = c.pyr_w0, h = c.pyr_h0, off = 0;
    for (int l = 1; l < c.pyr_levels; ++l) {
        const int nw = (w + 1) / 2, nh = (h + 1) / 2, noff = off + w * h;
        for (int t = threadIdx.x; t < nw * nh; t += PYR_UP_BLOCK) {
            const int tx = t % nw, ty = t / nw;
            float dmin = __builtin_huge_valf(), dmax = -__builtin_huge_valf();
            for (int y = 2 * ty; y < min(h, 2 * ty + 2); ++y)
                for (int x = 2 * tx; x < min(w, 2 * tx + 2); ++x) {
                    const float2 r = c.pyr[off + y * w + x];
                    dmin = fminf(dmin, r.x);
                    dmax = fmaxf(dmax, r.y);
                }
            c.pyr[noff + t] = make_float2(dmin, dmax);
        }
        __syncthreads();
        off = noff;
        w = nw;
        h = nh;
    }
}

// -------------------------------------------------------------------- pixel maps

// Per pixel of one frame (blockIdx.y = frame): its depth d, the x and y of its
// back-projection P = (((u - c_x) / f_x) d, ((v - c_y) / f_y) d, d) (Eq. 7) and the colour
// weight W (Sec. IV.B: Eq. 8 normal from the neighbours (u+1, v) and (u, v+1), dot the unit
// viewing direction from the camera to P).  They depend only on the depth pixel, so every
// colour voxel that looks it up shares them; the operations are those of the per-voxel
// definition, and one 16-byte read gives a voxel all of them.
__global__ __launch_bounds__(BLOCK) void pixel_map_kernel(const FrameConsts* frames)
{
    const FrameConsts& c = frames[blockIdx.y];
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    if (p >= c.dw * c.dh) return;
    const int x = p % c.dw, y = p / c.dw;
    float W = __builtin_bit_cast(float, kNoNormal);
    const float d = c.depth[p];
    const float u = (float)x, v = (float)y;
    const float Px = ((u - c.cx) * c.inv_fx) * d;
    const float Py = ((v - c.cy) * c.inv_fy) * d;
    if (valid_depth(d) && x + 1 < c.dw && y + 1 < c.dh) {
        const float d1 = c.depth[p + 1], d2 = c.depth[p + c.dw];
        const float P1x = ((u + 1.0f - c.cx) * c.inv_fx) * d1;
        const float P1y = ((v - c.cy) * c.inv_fy) * d1;
        const float P2x = ((u - c.cx) * c.inv_fx) * d2;
        const float P2y = ((v + 1.0f - c.cy) * c.inv_fy) * d2;
        const float e1x = P1x - Px, e1y = P1y - Py, e1z = d1 - d;
        const float e2x = P2x - Px, e2y = P2y - Py, e2z = d2 - d;
        const float Nx = fmaf(e1y, e2z, -(e1z * e2y));
        const float Ny = fmaf(e1z, e2x, -(e1x * e2z));
        const float Nz = fmaf(e1x, e2y, -(e1y * e2x));
        const float nn = fmaf(Nx, Nx, fmaf(Ny, Ny, Nz * Nz));
        if ((int)valid_depth(d1) & (int)valid_depth(d2) & (int)(nn > 0.0f)) {
            const float pp = fmaf(Px, Px, fmaf(Py, Py, d * d));
            const float dp = fmaf(Nx, Px, fmaf(Ny, Py, Nz * d));
            W = dp / sqrtf(nn * pp);
        }
    }
    c.pmap[p] = make_float4(d, Px, Py, W);
}

// ------------------------------------------------------------------------ integration

// Persistent waves: each takes (brick, frame mask) entries of one kind from the live list;
// bricks have shape BRICK_SHAPES[KIND][SHAPE].
template <int MODE, int KIND, int SHAPE>
__global__ __launch_bounds__(BLOCK) void integrate_kernel(IntegrateArgs a)
{
    constexpr BrickShape S = BRICK_SHAPES[KIND][SHAPE];
    const int lane = threadIdx.x & (WAVE - 1);
    __shared__ float4 s_slots[KIND == KIND_COLOUR ? BLOCK : 1];   // colour: sampling jobs
    Counts cnt;
    // the heavy list first, then the light one
    const uint32_t n_heavy = *as_const(a.n_live + KIND);
    const uint32_t n_live = n_heavy + *as_const(a.n_live + 2 + KIND);
    const const_ptr<SceneDev> scenes = as_const(a.scenes);
    for (;;) {
        const uint32_t e = wave_ticket(a.queue + KIND);
        if (e >= n_live) break;
        const bool light = e >= n_heavy;
        const uint32_t el = light ? e - n_heavy : e;
        const uint32_t pos = (KIND == KIND_COLOUR ? a.cap - 1u - el : el) + (light ? a.cap : 0u);
        const const_ptr<uint32_t> ent = as_const((const uint32_t*)a.live) + 4 * (size_t)pos;
        const uint32_t item = ent[0];
        const unsigned long long fmask = ent[1] | (unsigned long long)ent[2] << 32;
        int s = 0;
        while (s + 1 < a.n_scenes && scenes[s + 1].item_begin <= item) ++s;
        const auto& sc = scenes[s];
        const const_ptr<FrameConsts> frames = as_const(a.frames) + sc.frame_begin;
        const uint32_t li = item - sc.item_begin;
        if constexpr (KIND == KIND_GEOM) {
            geom_brick<MODE, S.bx, S.by, S.bz>(sc, frames, fmask, li, nullptr, cnt);
            if constexpr (MODE == MODE_COUNT) cnt.g_bricks += (unsigned)__builtin_popcountll(fmask);
        } else {
            colour_brick<MODE, S.bx, S.by, S.bz>(sc, frames, fmask, li - sc.geom_items, nullptr,
                                                 s_slots + (threadIdx.x & ~(WAVE - 1)), cnt);
            if constexpr (MODE == MODE_COUNT) cnt.c_bricks += (unsigned)__builtin_popcountll(fmask);
        }
    }
    if constexpr (MODE == MODE_COUNT) {
        // brick-frames in units of 512 voxels, whatever the brick's size
        constexpr unsigned long long vox = (unsigned long long)WAVE * S.bz;
        const unsigned long long v[8] = {wave_sum(cnt.g_upd), wave_sum(cnt.g_touch),
                                         wave_sum(cnt.c_eval), wave_sum(cnt.c_read),
                                         wave_sum(cnt.c_upd), wave_sum(cnt.c_touch),
                                         cnt.g_bricks * vox, cnt.c_bricks * vox};
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (v[q]) atomicAdd(a.counters + q, v[q]);
        }
    }
}

// Outcome codes of one frame for every brick of one kind (no culling, no update), with
// the default brick shapes.
template <bool COLOUR>
__global__ __launch_bounds__(BLOCK) void status_kernel(StatusArgs a)
{
    __shared__ float4 s_slots[COLOUR ? BLOCK : 1];   // colour: sampling jobs
    const uint32_t li = blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE;
    if (li >= a.n_items) return;
    Counts cnt;
    const FrameConsts* frames = &a.frame;
    constexpr BrickShape S = BRICK_SHAPES[COLOUR ? KIND_COLOUR : KIND_GEOM][0];
    if constexpr (COLOUR)
        colour_brick<MODE_STATUS, S.bx, S.by, S.bz>(a.scene, frames, 1u, li, a.status,
                                                    s_slots + (threadIdx.x & ~(WAVE - 1)), cnt);
    else
        geom_brick<MODE_STATUS, S.bx, S.by, S.bz>(a.scene, frames, 1u, li, a.status, cnt);
}

__global__ void fill_f32_kernel(float* p, size_t n, float v)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = v;
}

// The same for a 16-byte aligned array, four elements per store (the last n % 4 by the
// first thread).
__global__ void fill_f32x4_kernel(float4* p, size_t n, float v)
{
    const size_t n4 = n / 4, stride = (size_t)gridDim.x * blockDim.x;
    const float4 v4 = make_float4(v, v, v, v);
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) p[q] = v4;
    if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) ((float*)(p + n4))[threadIdx.x] = v;
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = v;
}

// ----------------------------------------------------------------------------- launchers

hipError_t launch_pyramids(const FrameConsts* frames_dev, int32_t n_frames, int32_t max_tiles0,
                           hipStream_t stream)
{
    if (n_frames <= 0) return hipSuccess;
    const unsigned bx = (unsigned)((max_tiles0 + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(pyramid_base_kernel, dim3(bx, (unsigned)n_frames), dim3(BLOCK), 0, stream,
                       frames_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pyramid_up_kernel, dim3((unsigned)n_frames), dim3(PYR_UP_BLOCK), 0, stream,
                       frames_dev);
    return hipGetLastError();
}

hipError_t launch_pixel_maps(const FrameConsts* frames_dev, int32_t n_frames, int32_t max_pixels,
                              hipStream_t stream)
{
    if (n_frames <= 0 || max_pixels <= 0) return hipSuccess;
    const unsigned bx = (unsigned)((max_pixels + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(pixel_map_kernel, dim3(bx, (unsigned)n_frames), dim3(BLOCK), 0, stream,
                       frames_dev);
    return hipGetLastError();
}

hipError_t launch_cull(const CullArgs& a, hipStream_t stream)
{
    if (a.n_chunks == 0) return hipSuccess;
    if (a.max_frames > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cull_kernel, dim3((a.n_chunks + CULL_WAVES - 1) / CULL_WAVES), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

// Launch and occupancy query of each integration kernel, by (mode, kind, shape).
template <int MODE, int KIND, int SHAPE>
static hipError_t launch_one(const IntegrateArgs& a, uint32_t grid, hipStream_t stream)
{
    hipLaunchKernelGGL((integrate_kernel<MODE, KIND, SHAPE>), dim3(grid), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

template <int MODE, int KIND, int SHAPE>
static hipError_t occupancy_one(int* per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, integrate_kernel<MODE, KIND, SHAPE>, BLOCK, 0);
}

struct IntegrateEntry {
    hipError_t (*launch)(const IntegrateArgs&, uint32_t, hipStream_t);
    hipError_t (*occupancy)(int*);
};

template <int MODE, int KIND, int... SH>
static const IntegrateEntry* entry_row(std::integer_sequence<int, SH...>)
{
    static const IntegrateEntry row[] = {{launch_one<MODE, KIND, SH>, occupancy_one<MODE, KIND, SH>}...};
    return row;
}

static const IntegrateEntry* integrate_entry(int mode, int kind, int shape)
{
    if (shape < 0 || shape >= N_BRICK_SHAPES) return nullptr;
    using Seq = std::make_integer_sequence<int, N_BRICK_SHAPES>;
    if (mode == MODE_INTEGRATE && kind == KIND_GEOM) return entry_row<MODE_INTEGRATE, KIND_GEOM>(Seq{}) + shape;
    if (mode == MODE_INTEGRATE && kind == KIND_COLOUR) return entry_row<MODE_INTEGRATE, KIND_COLOUR>(Seq{}) + shape;
    if (mode == MODE_COUNT && kind == KIND_GEOM) return entry_row<MODE_COUNT, KIND_GEOM>(Seq{}) + shape;
    if (mode == MODE_COUNT && kind == KIND_COLOUR) return entry_row<MODE_COUNT, KIND_COLOUR>(Seq{}) + shape;
    return nullptr;
}

hipError_t launch_integrate(int mode, int kind, int shape, const IntegrateArgs& a, uint32_t grid,
                            hipStream_t stream)
{
    if (grid == 0) return hipSuccess;
    const IntegrateEntry* e = integrate_entry(mode, kind, shape);
    return e ? e->launch(a, grid, stream) : hipErrorInvalidValue;
}

hipError_t launch_status(bool colour, const StatusArgs& a, hipStream_t stream)
{
    if (a.n_items == 0) return hipSuccess;
    const unsigned blocks = (a.n_items + (BLOCK / WAVE) - 1) / (BLOCK / WAVE);
    if (colour)
        hipLaunchKernelGGL(status_kernel<true>, dim3(blocks), dim3(BLOCK), 0, stream, a);
    else
        hipLaunchKernelGGL(status_kernel<false>, dim3(blocks), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

hipError_t persistent_grid(int mode, int kind, int shape, int device, uint32_t* blocks)
{
    int n_cu = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    const IntegrateEntry* k = integrate_entry(mode, kind, shape);
    if (!k) return hipErrorInvalidValue;
    if ((e = k->occupancy(&per_cu)) != hipSuccess) return e;
    *blocks = (uint32_t)(n_cu * (per_cu > 0 ? per_cu : 1));
    return hipSuccess;
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    if (((uintptr_t)p & 15u) == 0) {
        const size_t want = (n / 4 + 255) / 256;
        const unsigned blocks = (unsigned)(want < 1 ? 1 : want < 65536 ? want : 65536);
        hipLaunchKernelGGL(fill_f32x4_kernel, dim3(blocks), dim3(256), 0, stream, (float4*)p, n, v);
        return hipGetLastError();
    }
    const size_t want = (n + 255) / 256;
    const unsigned blocks = (unsigned)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(fill_f32_kernel, dim3(blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const size_t want = (n + 255) / 256;
    const unsigned blocks = (unsigned)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

}  // namespace kf
