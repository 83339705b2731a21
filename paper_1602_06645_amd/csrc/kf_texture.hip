// Per-polygon texture maps from the colour volume for gfx950 (Sec. IV.C, Eq. 13-14 and
// the colour-volume lookup).  Texel (i, j) of the w x h map of triangle (V1, V2, V3), placed
// at (x, y) in the atlas, is the world point V1 + i (V2 - V1)/(w - 1) + j (V3 - V1)/(h - 1)
// (i then j, each an fma) coloured by trilinear interpolation of the colour volume, in
// single precision with a fixed operation order:
//   - colour-index coordinates q = fma(p, 1/s, -origin/s - 1/2) per axis (voxel i's centre
//     at index i); the cell min(floor(q), dim - 2), fractions q - cell;
//   - x, then y, then z lerps fma(f, b - a, a);
//   - zero unless q lies in [0, dim - 1] and the 8 corner colour weights are positive;
//   - the 8-bit texel rint(255 min(max(c, 0), 1)).
// Every texel of the map is written, also those of its lower-right half that the mesh does
// not show.  One workgroup per triangle (its constants are uniform); the map is cut into
// 8 x 8 blocks of texels, one per wave pass, so that a gather instruction touches a small
// neighbourhood of voxels and a store writes 8 runs of 8 neighbouring texels; the waves of
// the workgroup take the blocks in turn.
#include <hip/hip_runtime.h>

#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

namespace {

constexpr int TX_WAVES = 4;   // waves per workgroup

__device__ __forceinline__ float tx_lerp(float a, float b, float f) { return fmaf(f, b - a, a); }

__global__ __launch_bounds__(64 * TX_WAVES) void texture_kernel(TextureArgs a)
{
    const int32_t n = (int32_t)blockIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int32_t* rc = a.rects + 4 * (size_t)n;
    const int32_t x0 = rc[0], y0 = rc[1], w = rc[2], h = rc[3];
    // a map outside the atlas (or narrower than 2 texels) is not written
    if (x0 < 0 || y0 < 0 || w < 2 || h < 2 || w > a.atlas_width - x0 || h > a.atlas_height - y0)
        return;
    const float* V = a.tri + 9 * (size_t)n;
    float v1[3], s1[3], s2[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v1[k] = V[k];
        s1[k] = (V[3 + k] - V[k]) / (float)(w - 1);   // Eq. 13
        s2[k] = (V[6 + k] - V[k]) / (float)(h - 1);   // Eq. 14
    }
    const uint32_t X = (uint32_t)a.cdim[0], XY = (uint32_t)a.cdim[0] * (uint32_t)a.cdim[1];
    const int bw = (w + 7) >> 3, bh = (h + 7) >> 3;
    for (int blk = wave; blk < bw * bh; blk += TX_WAVES) {
        const int by = blk / bw;
        const int i = ((blk - by * bw) << 3) + (lane & 7);
        const int j = (by << 3) + (lane >> 3);
        if (i >= w || j >= h) continue;
        float q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float p = fmaf((float)j, s2[k], fmaf((float)i, s1[k], v1[k]));
            q[k] = fmaf(p, a.inv_s[k], a.off[k]);
        }
        float c[3] = {0.0f, 0.0f, 0.0f};
        bool ok = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) ok &= q[k] >= 0.0f && q[k] <= a.cmax[k];
        if (ok) {
            int ci[3];
            float f[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ci[k] = min((int)floorf(q[k]), a.cdim[k] - 2);
                f[k] = q[k] - (float)ci[k];
            }
            // the volume holds fewer than 2^31 voxels: 32-bit indices
            const uint32_t base = (uint32_t)ci[0] + X * (uint32_t)ci[1] + XY * (uint32_t)ci[2];
            const uint32_t off[8] = {0u, 1u, X, X + 1u, XY, XY + 1u, XY + X, XY + X + 1u};
#pragma unroll
            for (int k = 0; k < 8; ++k) ok &= a.wc[base + off[k]] > 0.0f;
            if (ok) {
                const float* F[3] = {a.r, a.g, a.b};
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const float* G = F[m];
                    const float c00 = tx_lerp(G[base + off[0]], G[base + off[1]], f[0]);
                    const float c10 = tx_lerp(G[base + off[2]], G[base + off[3]], f[0]);
                    const float c01 = tx_lerp(G[base + off[4]], G[base + off[5]], f[0]);
                    const float c11 = tx_lerp(G[base + off[6]], G[base + off[7]], f[0]);
                    c[m] = tx_lerp(tx_lerp(c00, c10, f[1]), tx_lerp(c01, c11, f[1]), f[2]);
                }
            }
        }
        const size_t t = ((size_t)(y0 + j) * (size_t)a.atlas_width + (size_t)(x0 + i)) * 3;
        if (a.atlas) {
#pragma unroll
            for (int m = 0; m < 3; ++m) a.atlas[t + m] = c[m];
        }
        if (a.atlas8) {
#pragma unroll
            for (int m = 0; m < 3; ++m)
                a.atlas8[t + m] = (uint8_t)rintf(fminf(fmaxf(c[m], 0.0f), 1.0f) * 255.0f);
        }
    }
}

}  // namespace

hipError_t launch_texture(const TextureArgs& a, hipStream_t stream)
{
    if (a.n_tri <= 0) return hipSuccess;
    hipLaunchKernelGGL(texture_kernel, dim3((uint32_t)a.n_tri), dim3(64 * TX_WAVES), 0, stream, a);
    return hipGetLastError();
}

}  // namespace kf
