// Adjoint of the colour-volume integration for gfx950.
//
// Eq. 9 in incremental form is C_n = (1 - alpha_n) C_{n-1} + alpha_n s_n, with
// alpha_n = W / (W_pre + W) in frames that update the voxel and 0 otherwise; Eq. 10 and
// every test of Sec. IV.B use only depth maps and poses, so the alpha_n do not depend on
// the HD images.  For L = sum_v g_v . C_N(v):
//   dL/ds_n = g_v beta_n,  beta_n = alpha_n prod_{m>n} (1 - alpha_m),
// s_n is the bilinear HD sample at the projection (Eq. 2-4) of the voxel centre, so the
// image gradient is g beta_n times the four bilinear weights, and the extrinsic gradient
// chains the sample's spatial derivative through the pinhole projection and the se(3)
// left perturbation dq/d(rho, phi) = [I | -[q]x].
//
// One lane per voxel column of a 64 x 4 x 8 brick (the forward's bricks).  Each voxel
// first replays the forward decisions of all frames (the same single-precision sequence
// as the forward kernel, so the same frames update it) and records alpha_n in LDS; a
// reverse sweep then scatters the image gradient with float atomics and accumulates the
// extrinsic gradient in double.  Per-block extrinsic partials are summed in a fixed order
// by a second kernel, so d_xi is deterministic.
#include <hip/hip_runtime.h>

#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

constexpr int BWD_MAX_FRAMES = 64;

namespace {

__device__ __forceinline__ bool bvalid(float d) { return d > 0.0f && d < __builtin_huge_valf(); }

// Forward decision of one colour voxel for one frame; returns the weight W (> 0) if the
// frame updates the voxel given the current weight, 0 otherwise.  Same operation
// sequence as the forward kernel.
__device__ __forceinline__ float colour_weight(const FrameConsts& c, float fi, float fj,
                                               float fk, float Wc)
{
    const float Xc = fmaf(c.Ac[2], fk, fmaf(c.Ac[1], fj, fmaf(c.Ac[0], fi, c.bc[0])));
    const float Yc = fmaf(c.Ac[5], fk, fmaf(c.Ac[4], fj, fmaf(c.Ac[3], fi, c.bc[1])));
    const float Zc = fmaf(c.Ac[8], fk, fmaf(c.Ac[7], fj, fmaf(c.Ac[6], fi, c.bc[2])));
    if (!(Zc > 0.0f)) return 0.0f;
    const float iz = 1.0f / Zc;
    const float u = rintf(fmaf(c.fx, Xc * iz, c.cx));
    const float v = rintf(fmaf(c.fy, Yc * iz, c.cy));
    if (!(u >= 0.0f && u <= c.wm1 && v >= 0.0f && v <= c.hm1)) return 0.0f;
    const int pix = (int)v * c.dw + (int)u;
    const float d = c.depth[pix];
    if (!bvalid(d)) return 0.0f;
    const float Px = ((u - c.cx) * c.inv_fx) * d;
    const float Py = ((v - c.cy) * c.inv_fy) * d;
    const float dx = Xc - Px, dy = Yc - Py, dz = Zc - d;
    if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) > c.sigma2) return 0.0f;
    if (!(u + 1.0f <= c.wm1 && v + 1.0f <= c.hm1)) return 0.0f;
    const float d1 = c.depth[pix + 1];
    const float d2 = c.depth[pix + c.dw];
    if (!bvalid(d1) || !bvalid(d2)) return 0.0f;
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
    if (!(nn > 0.0f)) return 0.0f;
    const float pp = fmaf(Px, Px, fmaf(Py, Py, d * d));
    const float dp = fmaf(Nx, Px, fmaf(Ny, Py, Nz * d));
    const float w = dp / sqrtf(nn * pp);
    if (!(w > c.gate * Wc)) return 0.0f;
    const float qx = fmaf(c.Ah[2], fk, fmaf(c.Ah[1], fj, fmaf(c.Ah[0], fi, c.bh[0])));
    const float qy = fmaf(c.Ah[5], fk, fmaf(c.Ah[4], fj, fmaf(c.Ah[3], fi, c.bh[1])));
    const float qz = fmaf(c.Ah[8], fk, fmaf(c.Ah[7], fj, fmaf(c.Ah[6], fi, c.bh[2])));
    if (!(qz > 0.0f)) return 0.0f;
    const float iqz = 1.0f / qz;
    const float x0 = floorf(fmaf(c.fxr, qx * iqz, c.cxr));
    const float y0 = floorf(fmaf(c.fyr, qy * iqz, c.cyr));
    if (!(x0 >= 0.0f && x0 <= c.cwm2 && y0 >= 0.0f && y0 <= c.chm2)) return 0.0f;
    return w;
}

__device__ __forceinline__ double wave_sum_d(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

}  // namespace

__global__ __launch_bounds__(BLOCK) void backward_kernel(BackwardArgs a)
{
    extern __shared__ float s_alpha[];   // [n_frames][BLOCK]
    __shared__ double s_xi[BLOCK / 64][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t li = blockIdx.x;
    const int X = a.cdim[0], Y = a.cdim[1], Z = a.cdim[2];
    const uint32_t tx = li % (uint32_t)a.ctiles[0];
    const uint32_t rest = li / (uint32_t)a.ctiles[0];
    const uint32_t ty = rest % (uint32_t)a.ctiles[1];
    const uint32_t tz = rest / (uint32_t)a.ctiles[1];
    const int i = (int)tx * BWD_TX + lane, j = (int)ty * BWD_TY + wave, k0 = (int)tz * ZS;
    const size_t nvox = (size_t)X * (size_t)Y * (size_t)Z;
    double xi[6] = {0, 0, 0, 0, 0, 0};
    float* hist = s_alpha + threadIdx.x;

    if (i < X && j < Y) {
        const float fi = (float)i, fj = (float)j;
        const int kn = min(ZS, Z - k0);
        for (int kk = 0; kk < kn; ++kk) {
            const int k = k0 + kk;
            const float fk = (float)k;
            const size_t idx = ((size_t)k * (size_t)Y + (size_t)j) * (size_t)X + (size_t)i;
            const float g0 = a.grad[idx], g1 = a.grad[nvox + idx], g2 = a.grad[2 * nvox + idx];
            if (g0 == 0.0f && g1 == 0.0f && g2 == 0.0f) continue;
            // forward replay: alpha_n of every frame
            float Wc = a.wc0 ? a.wc0[idx] : 0.0f;
            int any = 0;
            for (int f = 0; f < a.n_frames; ++f) {
                const float w = colour_weight(a.frames[f], fi, fj, fk, Wc);
                float alpha = 0.0f;
                if (w > 0.0f) {
                    alpha = w / (Wc + w);
                    Wc = fmaf(w, 1.0f - Wc, Wc);
                    any = 1;
                }
                hist[f * BLOCK] = alpha;
            }
            if (!any) continue;
            // reverse sweep
            float tail = 1.0f;
            for (int f = a.n_frames - 1; f >= 0; --f) {
                const float alpha = hist[f * BLOCK];
                if (alpha == 0.0f) continue;
                const float beta = alpha * tail;
                tail *= 1.0f - alpha;
                const FrameConsts& c = a.frames[f];
                const float qx = fmaf(c.Ah[2], fk, fmaf(c.Ah[1], fj, fmaf(c.Ah[0], fi, c.bh[0])));
                const float qy = fmaf(c.Ah[5], fk, fmaf(c.Ah[4], fj, fmaf(c.Ah[3], fi, c.bh[1])));
                const float qz = fmaf(c.Ah[8], fk, fmaf(c.Ah[7], fj, fmaf(c.Ah[6], fi, c.bh[2])));
                const float iqz = 1.0f / qz;
                const float xh = fmaf(c.fxr, qx * iqz, c.cxr);
                const float yh = fmaf(c.fyr, qy * iqz, c.cyr);
                const float x0 = floorf(xh), y0 = floorf(yh);
                const float ax = xh - x0, ay = yh - y0;
                const int cell = ((int)y0 * c.cw + (int)x0) * 3;
                const int row = c.cw * 3;
                const float* img = (const float*)c.rgb;
                float* dimg = a.d_rgb + (size_t)f * (size_t)c.cw * (size_t)c.ch * 3;
                const float w00 = (1.0f - ax) * (1.0f - ay), w10 = ax * (1.0f - ay);
                const float w01 = (1.0f - ax) * ay, w11 = ax * ay;
                const float gv[3] = {g0, g1, g2};
                float gx = 0.0f, gy = 0.0f;   // sum_ch g beta ds/dx, ds/dy
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float gb = gv[ch] * beta;
                    if (gb == 0.0f) continue;
                    unsafeAtomicAdd(dimg + cell + ch, gb * w00);
                    unsafeAtomicAdd(dimg + cell + 3 + ch, gb * w10);
                    unsafeAtomicAdd(dimg + cell + row + ch, gb * w01);
                    unsafeAtomicAdd(dimg + cell + row + 3 + ch, gb * w11);
                    const float p00 = img[cell + ch], p10 = img[cell + 3 + ch];
                    const float p01 = img[cell + row + ch], p11 = img[cell + row + 3 + ch];
                    gx = fmaf(gb, (1.0f - ay) * (p10 - p00) + ay * (p11 - p01), gx);
                    gy = fmaf(gb, (1.0f - ax) * (p01 - p00) + ax * (p11 - p10), gy);
                }
                // pinhole Jacobian of Eq. 4 after the division by z
                const double dqx = (double)gx * c.fxr * iqz;
                const double dqy = (double)gy * c.fyr * iqz;
                const double dqz = -((double)gx * c.fxr * qx + (double)gy * c.fyr * qy) * iqz * iqz;
                xi[0] += dqx;
                xi[1] += dqy;
                xi[2] += dqz;
                xi[3] += (double)qy * dqz - (double)qz * dqy;
                xi[4] += (double)qz * dqx - (double)qx * dqz;
                xi[5] += (double)qx * dqy - (double)qy * dqx;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double s = wave_sum_d(xi[q]);
        if (lane == 0) s_xi[wave][q] = s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) s += s_xi[w][threadIdx.x];
        a.partials[(size_t)blockIdx.x * 6 + threadIdx.x] = s;
    }
}

// Sum the per-block partials in a fixed order: lane t of component q adds blocks
// t, t+256, ...; then a fixed tree over the 256 lanes.
__global__ __launch_bounds__(256) void reduce_xi_kernel(const double* partials, uint32_t n, double* out)
{
    __shared__ double s[256];
    for (int q = 0; q < 6; ++q) {
        double acc = 0.0;
        for (uint32_t b = threadIdx.x; b < n; b += 256) acc += partials[(size_t)b * 6 + q];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = s[0];
        __syncthreads();
    }
}

uint32_t backward_blocks(const BackwardArgs& a) { return a.n_items; }

hipError_t launch_backward(const BackwardArgs& a, double* d_xi, hipStream_t stream)
{
    if (a.n_frames > BWD_MAX_FRAMES) return hipErrorInvalidValue;
    const size_t lds = (size_t)(a.n_frames > 0 ? a.n_frames : 1) * BLOCK * sizeof(float);
    static bool lds_raised = false;
    if (!lds_raised) {
        const hipError_t e = hipFuncSetAttribute((const void*)backward_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)(BWD_MAX_FRAMES * BLOCK * sizeof(float)));
        if (e != hipSuccess) return e;
        lds_raised = true;
    }
    if (a.n_items > 0) {
        hipLaunchKernelGGL(backward_kernel, dim3(a.n_items), dim3(BLOCK), lds, stream, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(reduce_xi_kernel, dim3(1), dim3(256), 0, stream, a.partials, a.n_items, d_xi);
    return hipGetLastError();
}

}  // namespace kf
