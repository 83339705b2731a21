// Per-polygon texture maps from the colour volume for gfx950 (Sec. IV.D, Eq. 13-14 and
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
// not show.
//
// One workgroup of 4 waves per triangle (its constants are uniform); the map is cut into
// 8 x 8 blocks of texels, one block per wave pass, the waves taking the blocks in turn.
// Neighbouring texels (texels are usually smaller than colour voxels) share most of their
// trilinear corners, so a wave first stages the voxels its block spans in LDS: the box of
// voxels between the cells of the block's four corner texels, up to 8 voxels along x and
// 48 rows in y and z, for the four fields (colour weight, R, G, B), loaded row by row;
// each lane then reads its 8 corners of each field from LDS.  A lane whose cell falls
// outside the box (rounding at the box's edge) and every lane of a block whose box is
// larger gather their corners from global memory in x-pairs.  Both routes read the same
// voxel values, so the arithmetic and the result are the same.
#include <hip/hip_runtime.h>

#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

namespace {

constexpr int TX_WAVES = 4;    // waves per workgroup (one triangle)
constexpr int TX_ROWS = 48;    // LDS rows (y, z) of 8 voxels per field and wave

__device__ __forceinline__ float tx_lerp(float a, float b, float f) { return fmaf(f, b - a, a); }

// Two neighbouring voxels along x (4-byte aligned 8-byte load).
__device__ __forceinline__ float2 load_pair(const float* p)
{
    float2 v;
    __builtin_memcpy(&v, p, 8);
    return v;
}

// Orders the wave's LDS writes before its later reads (and reads before later writes).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * TX_WAVES) void texture_kernel(TextureArgs a)
{
    __shared__ float lds[TX_WAVES][4][TX_ROWS * 8];
    const int32_t n = (int32_t)blockIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    float* box = &lds[wave][0][0];
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
    // the volume holds fewer than 2^31 voxels: 32-bit indices
    const uint32_t X = (uint32_t)a.cdim[0], XY = (uint32_t)a.cdim[0] * (uint32_t)a.cdim[1];
    const float* fields[4] = {a.wc, a.r, a.g, a.b};
    const int bw = (w + 7) >> 3, bh = (h + 7) >> 3;
    for (int blk = wave; blk < bw * bh; blk += TX_WAVES) {
        const int by = blk / bw;
        const int bi = (blk - by * bw) << 3, bj = by << 3;
        const int i = bi + (lane & 7);
        const int j = bj + (lane >> 3);
        // the voxel box between the cells of the block's corner texels (every lane computes
        // the same values)
        const int ie = min(bi + 7, w - 1), je = min(bj + 7, h - 1);
        int lo[3], nb[3];
        bool fits = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float qa = fmaf(fmaf((float)bj, s2[k], fmaf((float)bi, s1[k], v1[k])), a.inv_s[k], a.off[k]);
            const float qb = fmaf(fmaf((float)bj, s2[k], fmaf((float)ie, s1[k], v1[k])), a.inv_s[k], a.off[k]);
            const float qc = fmaf(fmaf((float)je, s2[k], fmaf((float)bi, s1[k], v1[k])), a.inv_s[k], a.off[k]);
            const float qd = fmaf(fmaf((float)je, s2[k], fmaf((float)ie, s1[k], v1[k])), a.inv_s[k], a.off[k]);
            const float qlo = fminf(fminf(qa, qb), fminf(qc, qd));
            const float qhi = fmaxf(fmaxf(qa, qb), fmaxf(qc, qd));
            fits &= qlo > -1e30f && qhi < 1e30f;            // finite (NaN fails both)
            const float l = fminf(fmaxf(floorf(qlo), 0.0f), a.cmax[k]);
            const float u = fminf(fmaxf(floorf(qhi) + 1.0f, -1.0f), a.cmax[k]);
            lo[k] = (int)l;
            nb[k] = (int)u - lo[k] + 1;
        }
        fits &= nb[0] >= 2 && nb[1] >= 2 && nb[2] >= 2 && nb[0] <= 8 && nb[1] * nb[2] <= TX_ROWS;
        fits = __builtin_amdgcn_readfirstlane((int)fits) != 0;
        wave_sync();                                        // the previous block's reads are done
        if (fits) {
            // rows (y, z) of the box, 8 lanes per row, one voxel per lane
            const int ny = nb[1], rows = nb[1] * nb[2];
            // (row + 1/2) / ny is at least 1/(2 ny) from an integer: the approximate
            // reciprocal (1 ulp) cannot move it across one
            const float rny = __builtin_amdgcn_rcpf((float)ny);
            const int x = lane & 7;
            for (int row = lane >> 3; row < rows; row += 8) {
                if (x < nb[0]) {
                    const int rz = (int)(((float)row + 0.5f) * rny);
                    const int ry = row - rz * ny;
                    const uint32_t g = (uint32_t)(lo[0] + x) + X * (uint32_t)(lo[1] + ry) +
                                       XY * (uint32_t)(lo[2] + rz);
#pragma unroll
                    for (int f = 0; f < 4; ++f) box[f * TX_ROWS * 8 + row * 8 + x] = fields[f][g];
                }
            }
            wave_sync();
        }
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
            bool in_box = fits;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ci[k] = min((int)floorf(q[k]), a.cdim[k] - 2);
                f[k] = q[k] - (float)ci[k];
                in_box &= ci[k] >= lo[k] && ci[k] + 2 <= lo[k] + nb[k];
            }
            // v[field][corner], corners x fastest: (0,0,0), (1,0,0), (0,1,0), ... (1,1,1)
            float v[4][8];
            if (in_box) {
                const int sb = (ci[0] - lo[0]) + 8 * ((ci[1] - lo[1]) + nb[1] * (ci[2] - lo[2]));
                const int so[4] = {0, 8, 8 * nb[1], 8 * nb[1] + 8};
#pragma unroll
                for (int fl = 0; fl < 4; ++fl)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        v[fl][2 * k] = box[fl * TX_ROWS * 8 + sb + so[k]];
                        v[fl][2 * k + 1] = box[fl * TX_ROWS * 8 + sb + so[k] + 1];
                    }
            } else {
                const uint32_t base = (uint32_t)ci[0] + X * (uint32_t)ci[1] + XY * (uint32_t)ci[2];
                const uint32_t off[4] = {0u, X, XY, XY + X};
#pragma unroll
                for (int fl = 0; fl < 4; ++fl)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float2 t = load_pair(fields[fl] + base + off[k]);
                        v[fl][2 * k] = t.x;
                        v[fl][2 * k + 1] = t.y;
                    }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) ok &= v[0][k] > 0.0f;
            if (ok) {
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const float* t = v[m + 1];
                    const float c00 = tx_lerp(t[0], t[1], f[0]);
                    const float c10 = tx_lerp(t[2], t[3], f[0]);
                    const float c01 = tx_lerp(t[4], t[5], f[0]);
                    const float c11 = tx_lerp(t[6], t[7], f[0]);
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
