// Conservative brick culling shared by the forward and the adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "kf_device.h"

namespace kf {

// A depth pixel is a measurement iff it is positive and finite.
__device__ __forceinline__ bool valid_depth(float d)
{
    return d > 0.0f && d < __builtin_huge_valf();
}

// --------------------------------------------------------------------------- culling

// Valid-depth (min, max) over pixels [u0,u1] x [v0,v1] (inclusive, inside the image),
// read from the finest pyramid level on which the box spans at most 4 x 4 tiles.  The
// tiles cover the box, so the range contains every depth inside it.  A tile holds the
// (min, max) of its valid depths, which are positive, or (+inf, -inf) when it has none:
// no NaN, so the bit patterns order as signed integers exactly as the floats do, and the
// integer min and max need no quieting of their operands.
template <class C>
__device__ inline float2 depth_range(const C& c, int u0, int u1, int v0, int v1)
{
    int w = c.pyr_w0, h = c.pyr_h0, off = 0, s = PYR_SHIFT;
    for (int l = 0; l < c.pyr_levels; ++l) {
        const int tx0 = u0 >> s, tx1 = u1 >> s, ty0 = v0 >> s, ty1 = v1 >> s;
        if ((tx1 - tx0 <= 3 && ty1 - ty0 <= 3) || l == c.pyr_levels - 1) {
            int32_t lo = 0x7F800000, hi = (int32_t)0xFF800000;   // +inf, -inf
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    const float2 r = c.pyr[off + ty * w + tx];
                    lo = min(lo, __builtin_bit_cast(int32_t, r.x));
                    hi = max(hi, __builtin_bit_cast(int32_t, r.y));
                }
            return make_float2(__builtin_bit_cast(float, lo), __builtin_bit_cast(float, hi));
        }
        off += w * h;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
        ++s;
    }
    return make_float2(__builtin_huge_valf(), -__builtin_huge_valf());
}

// Can any voxel of the index box [i0,i1] x [j0,j1] x [k0,k1] pass the depth tests of this
// frame?  Its voxel centres form a parallelepiped (Eq. 5 is affine in the index), so
// their depths lie between the corners' and, when all corners are in front of the
// camera, their projections lie in the corners' bounding box; a voxel's pixel is the
// nearest integer to its projection, so the pixels lie in [ceil(min - 1/2), floor(max +
// 1/2)], taken with 1/16 pixel to spare plus the rounding of the coordinates: the corners
// are the first corner plus the box's edge vectors (additions), the voxels' own
// coordinates are rounded too, and the projection uses the hardware reciprocal (within 1
// ulp), all within 1e-6 of the coordinates' magnitude, which the margin converts to
// pixels at the nearest corner; a box with a corner within 5 cm of the camera plane (or
// behind it) takes the whole image.  A colour voxel needs a depth within sigma of its own z
// (|p - P| >= |z - d|); a geometry voxel needs a depth no more than trunc in front of it.
// 1 mm of slack covers the single-precision rounding of z and d.
template <class C>
__device__ inline bool brick_live(const C& c, bool colour, int i0, int i1, int j0, int j1, int k0,
                                  int k1)
{
    const auto* A = colour ? c.Ac : c.Ag;
    const auto* b = colour ? c.bc : c.bg;
    const float fi = (float)i0, fj = (float)j0, fk = (float)k0;
    const float di = (float)(i1 - i0), dj = (float)(j1 - j0), dk = (float)(k1 - k0);
    // corner q = first corner + (q & 1) di e_i + (q & 2) dj e_j + (q & 4) dk e_k, per coordinate
    float P[3][8];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        P[a][0] = fmaf(A[3 * a + 2], fk, fmaf(A[3 * a + 1], fj, fmaf(A[3 * a], fi, b[a])));
        P[a][1] = P[a][0] + A[3 * a] * di;
        const float ej = A[3 * a + 1] * dj, ek = A[3 * a + 2] * dk;
        P[a][2] = P[a][0] + ej;
        P[a][3] = P[a][1] + ej;
#pragma unroll
        for (int q = 4; q < 8; ++q) P[a][q] = P[a][q - 4] + ek;
    }
    float zmin = __builtin_huge_valf(), zmax = -__builtin_huge_valf();
    float xmin = __builtin_huge_valf(), xmax = -__builtin_huge_valf();
    float ymin = __builtin_huge_valf(), ymax = -__builtin_huge_valf();
    float amax = 0.0f;   // largest |X|, |Y| among the corners
    bool near = false;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float Z = P[2][q];
        zmin = fminf(zmin, Z);
        zmax = fmaxf(zmax, Z);
        near |= !(Z > 0.05f);
        amax = fmaxf(amax, fmaxf(fabsf(P[0][q]), fabsf(P[1][q])));
        const float rz = __builtin_amdgcn_rcpf(Z);
        const float x = P[0][q] * rz, y = P[1][q] * rz;   // X / Z, Y / Z
        xmin = fminf(xmin, x);
        xmax = fmaxf(xmax, x);
        ymin = fminf(ymin, y);
        ymax = fmaxf(ymax, y);
    }
    if (!(zmax > -1e-4f)) return false;                  // entirely behind the camera
    int u0 = 0, u1 = c.dw - 1, v0 = 0, v1 = c.dh - 1;
    if (!near) {
        // to pixels (f > 0 keeps the order), with the margin for the coordinates' rounding
        // (1e-6 of their magnitude, about 8 ulps) at the nearest corner
        const float rel = 1e-6f * amax * __builtin_amdgcn_rcpf(zmin);   // the ratio to 1 ulp
        const float mx = 0.5625f + rel * c.fx;
        const float my = 0.5625f + rel * c.fy;
        const float fu0 = ceilf(fmaf(c.fx, xmin, c.cx) - mx), fu1 = floorf(fmaf(c.fx, xmax, c.cx) + mx);
        const float fv0 = ceilf(fmaf(c.fy, ymin, c.cy) - my), fv1 = floorf(fmaf(c.fy, ymax, c.cy) + my);
        if (fu1 < 0.0f || fu0 > c.wm1 || fv1 < 0.0f || fv0 > c.hm1) return false;
        u0 = (int)fmaxf(fu0, 0.0f);
        u1 = (int)fminf(fu1, c.wm1);
        v0 = (int)fmaxf(fv0, 0.0f);
        v1 = (int)fminf(fv1, c.hm1);
    }
    const float2 r = depth_range(c, u0, u1, v0, v1);
    if (!(r.x <= r.y)) return false;                      // no measurement in the footprint
    const float slack = 1e-3f;
    if (colour) return r.x <= zmax + c.sigma + slack && r.y >= zmin - c.sigma - slack;
    return zmin <= r.y + c.trunc + slack;
}


}  // namespace kf
