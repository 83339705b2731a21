// Ray casting of the geometry and colour volumes for gfx950: the rendering the method uses
// for live feedback and the predicted surface of tracking (abstract and Sec. III, after
// KinectFusion).  Per pixel, in single precision with a fixed operation order:
//   - the ray in geometry-index coordinates q(t) = a + t b(x, y), t the camera depth
//     (voxel i has its centre at index i), b affine in the pixel;
//   - samples at t = n delta (n >= 1) inside the slab where q lies in [0, dim - 1] on every
//     axis (at most 2^20 samples, none beyond 2^23 steps); a sample is valid iff the 8
//     corner geometry weights of its trilinear cell (min(floor(q), dim - 2)) are positive;
//   - the TSDF by trilinear interpolation, x, then y, then z, each a lerp fma(f, b - a, a);
//   - the hit: the first two consecutive valid samples with F > 0 then F < 0 (a surface
//     seen from its front), refined linearly: t* = t_prev + delta F_prev / (F_prev - F);
//   - outputs: depth t*, the world point, the normal (central differences of the trilinear
//     TSDF one index step away, scaled to world units, normalised; zero when a difference
//     sample is invalid or the gradient vanishes) and the trilinear colour (zero unless
//     the 8 corner colour weights are positive).  A miss writes zeros.
// One thread per pixel; each wave renders an 8 x 8 tile so that its rays gather from
// neighbouring voxels.
#include <hip/hip_runtime.h>

#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

namespace {

__device__ __forceinline__ float rc_lerp(float a, float b, float f) { return fmaf(f, b - a, a); }

// Trilinear interpolation of N fields of a volume with dims d at index point q; false
// when q leaves [0, qmax] or a corner weight is not positive.
template <int N>
__device__ __forceinline__ bool trilinear(const int32_t* d, const float* qmax, const float* w,
                                          const float* const* fields, const float* q, float* out)
{
    int i[3];
    float f[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (!(q[k] >= 0.0f && q[k] <= qmax[k])) return false;
        const int c = min((int)floorf(q[k]), d[k] - 2);
        i[k] = c;
        f[k] = q[k] - (float)c;
    }
    const size_t X = (size_t)d[0], XY = (size_t)d[0] * (size_t)d[1];
    const size_t base = (size_t)i[0] + X * (size_t)i[1] + XY * (size_t)i[2];
    const size_t off[8] = {0, 1, X, X + 1, XY, XY + 1, XY + X, XY + X + 1};
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 8; ++c) ok &= w[base + off[c]] > 0.0f;
    if (!ok) return false;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const float* F = fields[m];
        const float c00 = rc_lerp(F[base + off[0]], F[base + off[1]], f[0]);
        const float c10 = rc_lerp(F[base + off[2]], F[base + off[3]], f[0]);
        const float c01 = rc_lerp(F[base + off[4]], F[base + off[5]], f[0]);
        const float c11 = rc_lerp(F[base + off[6]], F[base + off[7]], f[0]);
        out[m] = rc_lerp(rc_lerp(c00, c10, f[1]), rc_lerp(c01, c11, f[1]), f[2]);
    }
    return true;
}

}  // namespace

__global__ __launch_bounds__(BLOCK) void raycast_kernel(RaycastArgs a)
{
    // block: 16 x 16 pixels; wave w: the 8 x 8 quadrant (w & 1, w >> 1)
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int x = (int)blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
    const int y = (int)blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
    if (x >= a.width || y >= a.height) return;
    const size_t pix = (size_t)y * (size_t)a.width + (size_t)x;
    const float u = (float)x, v = (float)y;
    float bq[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) bq[k] = fmaf(a.Bv[k], v, fmaf(a.Bu[k], u, a.B0[k]));
    float t_in = -__builtin_huge_valf(), t_out = __builtin_huge_valf();
    bool miss = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (bq[k] != 0.0f) {
            const float ta = (0.0f - a.a[k]) / bq[k];
            const float tb = (a.gmax[k] - a.a[k]) / bq[k];
            t_in = fmaxf(t_in, fminf(ta, tb));
            t_out = fminf(t_out, fmaxf(ta, tb));
        } else if (!(a.a[k] >= 0.0f && a.a[k] <= a.gmax[k])) {
            miss = true;
        }
    }
    const float n0 = fmaxf(ceilf(t_in / a.delta), 1.0f);
    const float n1 = fminf(floorf(t_out / a.delta), n0 + 1048575.0f);
    miss |= !(n0 <= n1) || !(n0 <= 8388608.0f);
    float t_hit = 0.0f;
    bool hit = false;
    if (!miss) {
        const float* fields[1] = {a.tsdf};
        bool prev_valid = false;
        float prev_F = 0.0f, prev_t = 0.0f;
        for (int n = (int)n0; n <= (int)n1; ++n) {
            const float t = (float)n * a.delta;
            float q[3], F = 0.0f;
#pragma unroll
            for (int k = 0; k < 3; ++k) q[k] = fmaf(t, bq[k], a.a[k]);
            const bool valid = trilinear<1>(a.gdim, a.gmax, a.wg, fields, q, &F);
            if (valid && prev_valid && prev_F > 0.0f && F < 0.0f) {
                t_hit = fmaf(a.delta, prev_F / (prev_F - F), prev_t);
                hit = true;
                break;
            }
            prev_valid = valid;
            prev_F = F;
            prev_t = t;
        }
    }
    float vert[3] = {0, 0, 0}, nrm[3] = {0, 0, 0}, col[3] = {0, 0, 0};
    if (hit) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            vert[k] = fmaf(t_hit, fmaf(a.Rv[k], v, fmaf(a.Ru[k], u, a.R0[k])), a.tw[k]);
        float qh[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) qh[k] = fmaf(t_hit, bq[k], a.a[k]);
        if (a.normal) {
            const float* fields[1] = {a.tsdf};
            float grad[3];
            bool ok = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float qp[3] = {qh[0], qh[1], qh[2]}, qm[3] = {qh[0], qh[1], qh[2]};
                qp[k] = qh[k] + 1.0f;
                qm[k] = qh[k] - 1.0f;
                float Fp = 0.0f, Fm = 0.0f;
                if (ok) ok = trilinear<1>(a.gdim, a.gmax, a.wg, fields, qp, &Fp) &&
                             trilinear<1>(a.gdim, a.gmax, a.wg, fields, qm, &Fm);
                grad[k] = (Fp - Fm) * a.inv_s[k];
            }
            if (ok) {
                const float gg = fmaf(grad[0], grad[0], fmaf(grad[1], grad[1], grad[2] * grad[2]));
                if (gg > 0.0f) {
                    const float len = sqrtf(gg);
#pragma unroll
                    for (int k = 0; k < 3; ++k) nrm[k] = grad[k] / len;
                }
            }
        }
        if (a.rgb) {
            float qc[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float bc = fmaf(a.Bcv[k], v, fmaf(a.Bcu[k], u, a.Bc0[k]));
                qc[k] = fmaf(t_hit, bc, a.ac[k]);
            }
            const float* cf[3] = {a.r, a.g, a.b};
            float c3[3];
            if (trilinear<3>(a.cdim, a.cmax, a.wc, cf, qc, c3))
#pragma unroll
                for (int k = 0; k < 3; ++k) col[k] = c3[k];
        }
    }
    a.depth[pix] = hit ? t_hit : 0.0f;
    if (a.vertex)
#pragma unroll
        for (int k = 0; k < 3; ++k) a.vertex[3 * pix + k] = vert[k];
    if (a.normal)
#pragma unroll
        for (int k = 0; k < 3; ++k) a.normal[3 * pix + k] = nrm[k];
    if (a.rgb)
#pragma unroll
        for (int k = 0; k < 3; ++k) a.rgb[3 * pix + k] = col[k];
}

hipError_t launch_raycast(const RaycastArgs& a, hipStream_t stream)
{
    if (a.width <= 0 || a.height <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.width + 15) / 16), (unsigned)((a.height + 15) / 16));
    hipLaunchKernelGGL(raycast_kernel, grid, dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

}  // namespace kf
