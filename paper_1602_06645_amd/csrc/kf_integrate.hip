// Forward integration kernels for gfx950: TSDF geometry volume (Sec. III) and asymmetric
// colour volume (Sec. IV.B, Eq. 5-10, with the depth-to-HD mapping of Eq. 1-4).
//
// One kernel serves every forward entry point.  A work item is a brick of 64 x 4 columns
// by 8 voxels along z of one volume of one scan.  Each lane owns one column of the brick
// and keeps the state of its 8 voxels in registers while it applies every frame of the
// pass in order; a voxel's state is read only when a frame first needs it (lazily) and
// written back only if some frame updated it.  A wave64 covers 64 consecutive x voxels,
// so every state access is a coalesced 256-byte row per array.
//
// Arithmetic is IEEE single precision in a fixed order: explicit fmaf, correctly rounded
// division and square root, rintf for the nearest depth pixel, floorf for the HD cell.
// The library is compiled with -ffp-contract=off, so nothing else is fused.
#include <hip/hip_runtime.h>

#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

namespace {

__device__ __forceinline__ bool valid_depth(float d)
{
    return d > 0.0f && d < __builtin_huge_valf();
}

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

struct InlineFrames {
    const FrameConsts& c;
    __device__ __forceinline__ const FrameConsts& operator[](int) const { return c; }
};

// Per-launch tables are read-only for the whole launch: reading them through the
// constant address space lets the compiler use scalar loads and keep them in SGPRs.
template <class T>
using const_ptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ const_ptr<T> as_const(const T* p)
{
    return (const_ptr<T>)p;
}

struct TableFrames {
    const_ptr<FrameConsts> p;
    __device__ __forceinline__ const __attribute__((address_space(4))) FrameConsts&
    operator[](int f) const { return p[f]; }
};

struct Counts {
    unsigned long long g_upd = 0, g_touch = 0, c_eval = 0, c_read = 0, c_upd = 0, c_touch = 0;
};

// Each lane parks the state of its ZS voxels in its own slots of an LDS scratchpad
// (slot kk of lane t at [kk * BLOCK + t]); no other lane touches them, so no barrier is
// needed, and the z loop can stay rolled.
struct Scratch {
    float4* v;   // ZS * BLOCK entries
};

// Geometry brick: projective TSDF with running average (KinectFusion, Sec. III).
template <int MODE, class Scene, class Frames>
__device__ __forceinline__ void geom_brick(const IntegrateArgs& a, const Scene& sc,
                                           Frames frames, int nf, uint32_t li, Scratch lds,
                                           Counts& cnt)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int X = sc.gdim[0], Y = sc.gdim[1], Z = sc.gdim[2];
    const uint32_t tx = li % (uint32_t)sc.gtiles[0];
    const uint32_t rest = li / (uint32_t)sc.gtiles[0];
    const uint32_t ty = rest % (uint32_t)sc.gtiles[1];
    const uint32_t tz = rest / (uint32_t)sc.gtiles[1];
    const int i = (int)tx * TX + lane, j = (int)ty * TY + wave, k0 = (int)tz * ZS;
    if (i >= X || j >= Y) return;
    const int kn = min(ZS, Z - k0);
    const size_t slice = (size_t)X * (size_t)Y;
    const size_t base = ((size_t)k0 * (size_t)Y + (size_t)j) * (size_t)X + (size_t)i;
    const float fi = (float)i, fj = (float)j;
    float4* slot = lds.v + threadIdx.x;

    uint32_t loaded = 0;
    unsigned long long n_upd = 0;
    for (int f = 0; f < nf; ++f) {
        const auto& c = frames[f];
        // Eq. 5 for this column; the z term is added per voxel.
        const float cX = fmaf(c.Ag[1], fj, fmaf(c.Ag[0], fi, c.bg[0]));
        const float cY = fmaf(c.Ag[4], fj, fmaf(c.Ag[3], fi, c.bg[1]));
        const float cZ = fmaf(c.Ag[7], fj, fmaf(c.Ag[6], fi, c.bg[2]));
#pragma unroll 2
        for (int kk = 0; kk < kn; ++kk) {
            const float fk = (float)(k0 + kk);
            const float Xc = fmaf(c.Ag[2], fk, cX);
            const float Yc = fmaf(c.Ag[5], fk, cY);
            const float Zc = fmaf(c.Ag[8], fk, cZ);
            int st = 0;
            float sdf = 0.0f;
            if (Zc > 0.0f) {
                // Eq. 6 with the perspective division; nearest depth pixel.
                const float iz = 1.0f / Zc;
                const float u = rintf(fmaf(c.fx, Xc * iz, c.cx));
                const float v = rintf(fmaf(c.fy, Yc * iz, c.cy));
                if (u >= 0.0f && u <= c.wm1 && v >= 0.0f && v <= c.hm1) {
                    const float d = c.depth[(int)v * c.dw + (int)u];
                    st = 1;
                    if (valid_depth(d)) {
                        sdf = d - Zc;
                        st = (sdf < -c.trunc) ? 2 : 6;
                    }
                }
            }
            if constexpr (MODE == MODE_STATUS) {
                a.gstatus[base + (size_t)kk * slice] = (uint8_t)st;
            } else if (st == 6) {
                float2 s;
                if (!((loaded >> kk) & 1u)) {
                    s.x = sc.tsdf[base + (size_t)kk * slice];
                    s.y = sc.wg[base + (size_t)kk * slice];
                    loaded |= 1u << kk;
                } else {
                    const float4 t4 = slot[kk * BLOCK];
                    s.x = t4.x;
                    s.y = t4.y;
                }
                const float t = fminf(1.0f, sdf * c.inv_trunc);
                const float wn = s.y + 1.0f;
                s.x = s.x + (t - s.x) / wn;
                s.y = fminf(wn, c.w_max);
                slot[kk * BLOCK] = make_float4(s.x, s.y, 0.0f, 0.0f);
                ++n_upd;
            }
        }
    }
    if constexpr (MODE != MODE_STATUS) {
        for (int kk = 0; kk < kn; ++kk) {
            if ((loaded >> kk) & 1u) {
                const float4 t4 = slot[kk * BLOCK];
                sc.tsdf[base + (size_t)kk * slice] = t4.x;
                sc.wg[base + (size_t)kk * slice] = t4.y;
            }
        }
    }
    if constexpr (MODE == MODE_COUNT) {
        cnt.g_upd += n_upd;
        cnt.g_touch += (unsigned long long)__builtin_popcount(loaded);
    }
}

// Bilinear HD sample of channel ch at cell `cell` (index of the top-left pixel's first
// channel), Eq. 9's HD(x_hd, y_hd) read between pixel centres.
__device__ __forceinline__ float hd_sample(const void* rgb, int fmt, int cell, int row, int ch,
                                           float ax, float ay)
{
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

// Colour brick: Sec. IV.B in the paper's order of tests, then Eq. 9 and Eq. 10.
template <int MODE, class Scene, class Frames>
__device__ __forceinline__ void colour_brick(const IntegrateArgs& a, const Scene& sc,
                                             Frames frames, int nf, uint32_t li, Scratch lds,
                                             Counts& cnt)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int X = sc.cdim[0], Y = sc.cdim[1], Z = sc.cdim[2];
    const uint32_t tx = li % (uint32_t)sc.ctiles[0];
    const uint32_t rest = li / (uint32_t)sc.ctiles[0];
    const uint32_t ty = rest % (uint32_t)sc.ctiles[1];
    const uint32_t tz = rest / (uint32_t)sc.ctiles[1];
    const int i = (int)tx * TX + lane, j = (int)ty * TY + wave, k0 = (int)tz * ZS;
    if (i >= X || j >= Y) return;
    const int kn = min(ZS, Z - k0);
    const size_t slice = (size_t)X * (size_t)Y;
    const size_t base = ((size_t)k0 * (size_t)Y + (size_t)j) * (size_t)X + (size_t)i;
    const float fi = (float)i, fj = (float)j;
    float4* slot = lds.v + threadIdx.x;

    uint32_t wl = 0;   // colour weight read (slot .w valid)
    uint32_t cl = 0;   // colour read and updated (slot .xyz valid, store at the end)
    unsigned long long n_eval = 0, n_upd = 0;
    for (int f = 0; f < nf; ++f) {
        const auto& c = frames[f];
        const float cX = fmaf(c.Ac[1], fj, fmaf(c.Ac[0], fi, c.bc[0]));
        const float cY = fmaf(c.Ac[4], fj, fmaf(c.Ac[3], fi, c.bc[1]));
        const float cZ = fmaf(c.Ac[7], fj, fmaf(c.Ac[6], fi, c.bc[2]));
#pragma unroll 2
        for (int kk = 0; kk < kn; ++kk) {
            const float fk = (float)(k0 + kk);
            const float Xc = fmaf(c.Ac[2], fk, cX);
            const float Yc = fmaf(c.Ac[5], fk, cY);
            const float Zc = fmaf(c.Ac[8], fk, cZ);
            int st = 0;
            float w = 0.0f;
            if (Zc > 0.0f) {
                const float iz = 1.0f / Zc;
                const float u = rintf(fmaf(c.fx, Xc * iz, c.cx));
                const float v = rintf(fmaf(c.fy, Yc * iz, c.cy));
                if (u >= 0.0f && u <= c.wm1 && v >= 0.0f && v <= c.hm1) {
                    const int pix = (int)v * c.dw + (int)u;
                    const float d = c.depth[pix];
                    st = 1;
                    if (valid_depth(d)) {
                        // Eq. 7 at the integer pixel, then the distance test against sigma.
                        const float Px = ((u - c.cx) * c.inv_fx) * d;
                        const float Py = ((v - c.cy) * c.inv_fy) * d;
                        const float dx = Xc - Px, dy = Yc - Py, dz = Zc - d;
                        const float dist2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        st = 2;
                        if (!(dist2 > c.sigma2)) {
                            st = 3;
                            if (u + 1.0f <= c.wm1 && v + 1.0f <= c.hm1) {
                                const float d1 = c.depth[pix + 1];
                                const float d2 = c.depth[pix + c.dw];
                                if (valid_depth(d1) && valid_depth(d2)) {
                                    // Eq. 8 from the neighbours (u+1, v) and (u, v+1).
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
                                    if (nn > 0.0f) {
                                        // W: unit normal . unit viewing direction (camera -> P).
                                        const float pp = fmaf(Px, Px, fmaf(Py, Py, d * d));
                                        const float dp = fmaf(Nx, Px, fmaf(Ny, Py, Nz * d));
                                        w = dp / sqrtf(nn * pp);
                                        st = 4;
                                    }
                                }
                            }
                        }
                    }
                }
            }
            if (st >= 4) {
                const size_t idx = base + (size_t)kk * slice;
                float4 s = slot[kk * BLOCK];
                if (!((wl >> kk) & 1u)) {
                    s.w = sc.wc[idx];
                    wl |= 1u << kk;
                }
                ++n_eval;
                float ax = 0.0f, ay = 0.0f;
                int cell = 0;
                if (w > c.gate * s.w) {
                    // Eq. 3-5 on the voxel centre: HD pixel and bilinear cell.
                    st = 5;
                    const float qx = fmaf(c.Ah[2], fk, fmaf(c.Ah[1], fj, fmaf(c.Ah[0], fi, c.bh[0])));
                    const float qy = fmaf(c.Ah[5], fk, fmaf(c.Ah[4], fj, fmaf(c.Ah[3], fi, c.bh[1])));
                    const float qz = fmaf(c.Ah[8], fk, fmaf(c.Ah[7], fj, fmaf(c.Ah[6], fi, c.bh[2])));
                    if (qz > 0.0f) {
                        const float iqz = 1.0f / qz;
                        const float xh = fmaf(c.fxr, qx * iqz, c.cxr);
                        const float yh = fmaf(c.fyr, qy * iqz, c.cyr);
                        const float x0 = floorf(xh), y0 = floorf(yh);
                        if (x0 >= 0.0f && x0 <= c.cwm2 && y0 >= 0.0f && y0 <= c.chm2) {
                            st = 6;
                            ax = xh - x0;
                            ay = yh - y0;
                            cell = ((int)y0 * c.cw + (int)x0) * 3;
                        }
                    }
                }
                if constexpr (MODE != MODE_STATUS) {
                    if (st == 6) {
                        if (!((cl >> kk) & 1u)) {
                            s.x = sc.r[idx];
                            s.y = sc.g[idx];
                            s.z = sc.b[idx];
                            cl |= 1u << kk;
                        }
                        const int row = c.cw * 3;
                        const float s0 = hd_sample(c.rgb, sc.fmt, cell, row, 0, ax, ay);
                        const float s1 = hd_sample(c.rgb, sc.fmt, cell, row, 1, ax, ay);
                        const float s2 = hd_sample(c.rgb, sc.fmt, cell, row, 2, ax, ay);
                        const float alpha = w / (s.w + w);
                        s.x = fmaf(alpha, s0 - s.x, s.x);
                        s.y = fmaf(alpha, s1 - s.y, s.y);
                        s.z = fmaf(alpha, s2 - s.z, s.z);
                        s.w = fmaf(w, 1.0f - s.w, s.w);
                        ++n_upd;
                    }
                }
                slot[kk * BLOCK] = s;
            }
            if constexpr (MODE == MODE_STATUS)
                a.cstatus[base + (size_t)kk * slice] = (uint8_t)st;
        }
    }
    if constexpr (MODE != MODE_STATUS) {
        for (int kk = 0; kk < kn; ++kk) {
            if ((cl >> kk) & 1u) {
                const size_t idx = base + (size_t)kk * slice;
                const float4 s = slot[kk * BLOCK];
                sc.r[idx] = s.x;
                sc.g[idx] = s.y;
                sc.b[idx] = s.z;
                sc.wc[idx] = s.w;
            }
        }
    }
    if constexpr (MODE == MODE_COUNT) {
        cnt.c_eval += n_eval;
        cnt.c_read += (unsigned long long)__builtin_popcount(wl);
        cnt.c_upd += n_upd;
        cnt.c_touch += (unsigned long long)__builtin_popcount(cl);
    }
}

// KIND: which bricks a kernel instantiation handles.
enum Kind : int { KIND_BOTH = 0, KIND_GEOM = 1, KIND_COLOUR = 2 };

template <int MODE, int KIND, class Scene, class Frames>
__device__ __forceinline__ void run_brick(const IntegrateArgs& a, const Scene& sc,
                                          Frames frames, int nf, uint32_t li, Scratch lds,
                                          Counts& cnt)
{
    if constexpr (KIND == KIND_GEOM) {
        geom_brick<MODE>(a, sc, frames, nf, li, lds, cnt);
    } else if constexpr (KIND == KIND_COLOUR) {
        colour_brick<MODE>(a, sc, frames, nf, li, lds, cnt);
    } else {
        if (li < sc.geom_items)
            geom_brick<MODE>(a, sc, frames, nf, li, lds, cnt);
        else
            colour_brick<MODE>(a, sc, frames, nf, li - sc.geom_items, lds, cnt);
    }
}

// INLINE: one scene and one frame passed by value; the geometry and the colour bricks of
// the frame are then two launches (KIND_GEOM, KIND_COLOUR), item counted per kind.
template <int MODE, bool INLINE, int KIND>
__device__ __forceinline__ void run_item(const IntegrateArgs& a, uint32_t item, Scratch lds,
                                         Counts& cnt)
{
    if constexpr (INLINE) {
        run_brick<MODE, KIND>(a, a.scene0, InlineFrames{a.frame0}, 1, item, lds, cnt);
    } else {
        const const_ptr<SceneDev> scenes = as_const(a.scenes);
        int s = 0;
        while (s + 1 < a.n_scenes && scenes[s + 1].item_begin <= item) ++s;
        const auto& sc = scenes[s];
        run_brick<MODE, KIND_BOTH>(a, sc, TableFrames{as_const(a.frames) + sc.frame_begin},
                                   sc.n_frames, item - sc.item_begin, lds, cnt);
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

}  // namespace

template <int MODE, bool INLINE, int KIND>
__global__ __launch_bounds__(BLOCK) void integrate_kernel(IntegrateArgs a)
{
    __shared__ float4 s_state[ZS * BLOCK];
    __shared__ uint32_t s_item;
    Counts cnt;
    const Scratch lds{s_state};
    for (;;) {
        uint32_t item;
        if (a.queue) {
            // persistent launch: take the next brick from the shared queue
            if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1u);
            __syncthreads();
            // the item is the same for the whole block: keep it (and everything derived
            // from it, such as the frame constants) in scalar registers
            item = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
        } else {
            // grid launch: consecutive blocks go to different XCDs round-robin, so hand
            // each XCD a contiguous range of bricks (and of the image footprint) instead
            item = (blockIdx.x % 8u) * (gridDim.x / 8u) + blockIdx.x / 8u;
        }
        if (item >= a.n_items) break;
        run_item<MODE, INLINE, KIND>(a, item, lds, cnt);
        if (!a.queue) break;
    }
    if constexpr (MODE == MODE_COUNT) {
        const unsigned long long v[6] = {wave_sum(cnt.g_upd), wave_sum(cnt.g_touch),
                                         wave_sum(cnt.c_eval), wave_sum(cnt.c_read),
                                         wave_sum(cnt.c_upd), wave_sum(cnt.c_touch)};
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int q = 0; q < 6; ++q)
                if (v[q]) atomicAdd(a.counters + q, v[q]);
        }
    }
}

__global__ void fill_f32_kernel(float* p, size_t n, float v)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = v;
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = v;
}

// ----------------------------------------------------------------------------- launchers

static uint32_t pad8(uint32_t n) { return (n + 7u) / 8u * 8u; }


template <int MODE, bool INLINE, int KIND>
static void launch_one(const IntegrateArgs& a, uint32_t blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((integrate_kernel<MODE, INLINE, KIND>), dim3(blocks), dim3(BLOCK), 0,
                       stream, a);
}

hipError_t launch_integrate(int mode, bool inline_args, const IntegrateArgs& a, uint32_t grid,
                            hipStream_t stream)
{
    if (inline_args) {
        // one frame of one scene: geometry bricks, then colour bricks
        IntegrateArgs g = a, c = a;
        g.n_items = a.scene0.geom_items;
        c.n_items = a.scene0.colour_items;
        const uint32_t gb = pad8(g.n_items), cb = pad8(c.n_items);
        if (mode == MODE_INTEGRATE) {
            if (gb) launch_one<MODE_INTEGRATE, true, KIND_GEOM>(g, gb, stream);
            if (cb) launch_one<MODE_INTEGRATE, true, KIND_COLOUR>(c, cb, stream);
        } else if (mode == MODE_STATUS) {
            if (gb) launch_one<MODE_STATUS, true, KIND_GEOM>(g, gb, stream);
            if (cb) launch_one<MODE_STATUS, true, KIND_COLOUR>(c, cb, stream);
        } else {
            if (gb) launch_one<MODE_COUNT, true, KIND_GEOM>(g, gb, stream);
            if (cb) launch_one<MODE_COUNT, true, KIND_COLOUR>(c, cb, stream);
        }
        return hipGetLastError();
    }
    // table-driven launch, persistent when a.queue is set (grid blocks), else one block
    // per brick
    const uint32_t blocks = a.queue ? grid : pad8(a.n_items);
    if (blocks == 0) return hipSuccess;
    if (mode == MODE_INTEGRATE) launch_one<MODE_INTEGRATE, false, KIND_BOTH>(a, blocks, stream);
    else if (mode == MODE_COUNT) launch_one<MODE_COUNT, false, KIND_BOTH>(a, blocks, stream);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t persistent_grid(int mode, int device, uint32_t* blocks)
{
    int n_cu = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    if (mode == MODE_COUNT)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, integrate_kernel<MODE_COUNT, false, KIND_BOTH>, BLOCK, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, integrate_kernel<MODE_INTEGRATE, false, KIND_BOTH>, BLOCK, 0);
    if (e != hipSuccess) return e;
    *blocks = (uint32_t)(n_cu * (per_cu > 0 ? per_cu : 1));
    return hipSuccess;
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
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
