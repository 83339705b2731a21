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
// tiles cover the box, so the range contains every depth inside it.
template <class C>
__device__ inline float2 depth_range(const C& c, int u0, int u1, int v0, int v1)
{
    int w = c.pyr_w0, h = c.pyr_h0, off = 0, s = PYR_SHIFT;
    for (int l = 0; l < c.pyr_levels; ++l) {
        const int tx0 = u0 >> s, tx1 = u1 >> s, ty0 = v0 >> s, ty1 = v1 >> s;
        if ((tx1 - tx0 <= 3 && ty1 - ty0 <= 3) || l == c.pyr_levels - 1) {
            float dmin = __builtin_huge_valf(), dmax = -__builtin_huge_valf();
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    const float2 r = c.pyr[off + ty * w + tx];
                    dmin = fminf(dmin, r.x);
                    dmax = fmaxf(dmax, r.y);
                }
            return make_float2(dmin, dmax);
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
// 1/2)], taken with 1/16 pixel to spare for the rounding of the voxel and corner
// coordinates and the hardware reciprocal (together below 1e-3 pixel at image
// coordinates up to a few thousand).  A colour voxel needs a depth within sigma of
// its own z (|p - P| >= |z - d|); a geometry voxel needs a depth no more than trunc in
// front of it.  1 mm of slack covers the single-precision rounding of z and d.
template <class C>
__device__ inline bool brick_live(const C& c, bool colour, int i0, int i1, int j0, int j1, int k0,
                                  int k1)
{
    const auto* A = colour ? c.Ac : c.Ag;
    const auto* b = colour ? c.bc : c.bg;
    float zmin = __builtin_huge_valf(), zmax = -__builtin_huge_valf();
    float xmin = __builtin_huge_valf(), xmax = -__builtin_huge_valf();
    float ymin = __builtin_huge_valf(), ymax = -__builtin_huge_valf();
    bool near = false;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float fi = (float)((q & 1) ? i1 : i0);
        const float fj = (float)((q & 2) ? j1 : j0);
        const float fk = (float)((q & 4) ? k1 : k0);
        const float X = fmaf(A[2], fk, fmaf(A[1], fj, fmaf(A[0], fi, b[0])));
        const float Y = fmaf(A[5], fk, fmaf(A[4], fj, fmaf(A[3], fi, b[1])));
        const float Z = fmaf(A[8], fk, fmaf(A[7], fj, fmaf(A[6], fi, b[2])));
        zmin = fminf(zmin, Z);
        zmax = fmaxf(zmax, Z);
        if (Z > 1e-3f) {
            // hardware reciprocal (within 1 ulp): its error, ~1e-7 of the pixel coordinate,
            // is far inside the one-pixel widening of the box below
            const float rz = __builtin_amdgcn_rcpf(Z);
            const float x = c.fx * (X * rz) + c.cx, y = c.fy * (Y * rz) + c.cy;
            xmin = fminf(xmin, x);
            xmax = fmaxf(xmax, x);
            ymin = fminf(ymin, y);
            ymax = fmaxf(ymax, y);
        } else {
            near = true;
        }
    }
    if (!(zmax > -1e-4f)) return false;                  // entirely behind the camera
    int u0 = 0, u1 = c.dw - 1, v0 = 0, v1 = c.dh - 1;
    if (!near) {
        const float fu0 = ceilf(xmin - 0.5625f), fu1 = floorf(xmax + 0.5625f);
        const float fv0 = ceilf(ymin - 0.5625f), fv1 = floorf(ymax + 0.5625f);
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
