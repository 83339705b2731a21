// Data shared by the host launchers and the gfx950 kernels of libkfvol.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace kf {

// A brick is the work of one wave64 in the forward integration: 64 voxel columns (bx x by)
// of bz voxels along z.  Each lane owns one column and keeps the state of its bz voxels
// for every frame of a pass.  The integration kernels are compiled for a few shapes per
// kind (BRICK_SHAPES); results do not depend on the shape, only the work does: longer
// columns share the per-column part of Eq. 5 among more voxels and hold more state per
// lane, smaller bricks are culled more finely.  Shape 0 of each kind is the default:
// geometry 16 x 4 x 8 (64-byte rows of each state array), colour 8 x 8 x 8 (compact, so
// most bricks are far from the observed surface in a given frame and skipped whole).
struct BrickShape {
    int32_t bx, by, bz;
};
constexpr int N_BRICK_SHAPES = 5;
constexpr BrickShape BRICK_SHAPES[2][N_BRICK_SHAPES] = {
    {{16, 4, 8}, {16, 4, 16}, {32, 2, 8}, {8, 8, 8}, {16, 4, 4}},   // geometry
    {{8, 8, 8}, {8, 8, 4}, {16, 4, 4}, {16, 4, 8}, {8, 8, 16}},     // colour
};
constexpr int MAX_BZ = 16;
// The adjoint's colour bricks (its own launch and culling): 8 x 8 x 8.
constexpr int CBX = 8, CBY = 8, ZS = 8;
constexpr int WAVE = 64;
constexpr int BLOCK = 256;              // four waves that work independently
constexpr int PYR_SHIFT = 1;            // level-0 tiles of the depth pyramid: 2 x 2 pixels
constexpr int XI_BLOCKS = 256;          // first-stage blocks of the adjoint's dxi reduction
constexpr int CHUNK = 4;                // culling chunks: CHUNK^3 bricks of one kind

// Everything one frame contributes to the per-voxel arithmetic, rounded once from the
// double-precision values computed on the host.
struct FrameConsts {
    float Ag[9], bg[3];   // geometry voxel index -> depth camera (Eq. 5, voxel size folded in)
    float Ac[9], bc[3];   // colour voxel index   -> depth camera
    float Ah[9], bh[3];   // colour voxel index   -> HD camera (Eq. 3 composed with Eq. 5)
    float fx, fy, cx, cy, inv_fx, inv_fy;  // K_c and the diagonal of K_c^-1
    float fxr, fyr, cxr, cyr;              // K_hd
    float trunc, inv_trunc, w_max, sigma2, gate, sigma;
    float wm1, hm1;       // depth image W-1, H-1 (exact in float)
    float hd_xmax, hd_ymax;  // largest first pixel of an HD sample: CW-2, CH-2 (bilinear)
                             // or CW-1, CH-1 (nearest pixel)
    int32_t dw, dh, cw, ch;
    const float* depth;   // [dh][dw]
    const void* rgb;      // [ch][cw][3], uint8 or float
    float2* pyr;          // min/max depth pyramid of this frame, levels back to back
    float4* pmap;         // [dh][dw] per depth pixel: its depth, the x and y of its
                          // back-projection P (Eq. 7) and the colour weight W (Eq. 8
                          // normal and the viewing ray) or kNoNormal
    int32_t pyr_w0, pyr_h0, pyr_levels;
    int32_t hd_nearest;   // 1: Eq. 9 reads the nearest HD pixel; 0: the bilinear sample
};

// Weight-map entry of a pixel without a normal (no depth at the pixel or a neighbour, a
// neighbour outside the image, or a zero cross product): a signalling-NaN pattern, which
// no arithmetic result can take, so that every computed weight (NaN included) stays
// distinguishable from it.
constexpr uint32_t kNoNormal = 0x7F800001u;

enum PixFmt : int32_t { FMT_RGB8 = 0, FMT_RGBF32 = 1 };

// One volume (scan) of a launch.
struct SceneDev {
    float *tsdf, *wg, *r, *g, *b, *wc;
    int32_t gdim[3], cdim[3];
    int32_t gshape[3], cshape[3];     // brick shapes (voxels per axis) of the pass
    int32_t gbricks[3], cbricks[3];   // bricks per axis
    uint32_t item_begin;              // first global brick index of this scene in the pass
    uint32_t geom_items;              // geometry bricks; colour bricks follow them
    uint32_t colour_items;
    int32_t gchunks[3], cchunks[3];   // culling chunks per axis
    uint32_t chunk_begin;             // first global chunk index of this scene in the pass
    uint32_t geom_chunks;             // geometry chunks; colour chunks follow them
    uint32_t colour_chunks;
    int32_t frame_begin;              // first entry of the frame table used by this pass
    int32_t n_frames;                 // frames of this scene in this pass (<= 64)
    int32_t fmt;                      // PixFmt
};

enum Mode : int32_t { MODE_INTEGRATE = 0, MODE_STATUS = 1, MODE_COUNT = 2 };
// Geometry and colour bricks are integrated by separate launches (their register needs
// differ, and so does the occupancy each can reach).
enum Kind : int32_t { KIND_GEOM = 0, KIND_COLOUR = 1 };

struct IntegrateArgs {
    const SceneDev* scenes;           // table of n_scenes
    const FrameConsts* frames;        // frame table
    int32_t n_scenes;
    const uint4* live;                // (brick, frame mask low, frame mask high, 0): a
                                      // heavy list [cap] and a light list [cap], each
                                      // with geometry entries from the front and colour
                                      // entries from the back
    uint32_t cap;                     // entries `live` can hold (bricks of the pass)
    const uint32_t* n_live;           // [list][KIND]: entries of each list and kind
    uint32_t* queue;                  // [KIND]: next entry to take
    unsigned long long* counters;     // MODE_COUNT: uint64[8]
};

// Single-frame status dump (no culling, no update): one scene and frame by value.
struct StatusArgs {
    SceneDev scene;
    FrameConsts frame;
    uint32_t n_items;                 // bricks of one kind
    uint8_t* status;
};

struct CullArgs {
    const SceneDev* scenes;
    const FrameConsts* frames;
    int32_t n_scenes;
    uint32_t n_items;                 // bricks of all scenes of the pass
    uint32_t n_chunks;                // culling chunks of all scenes of the pass
    int32_t disable;                  // 1: every brick is live in every frame
    int32_t max_frames;               // frames of the pass's longest scene (<= 64)
    uint4* live;                      // 2 x n_items entries (see IntegrateArgs)
    uint32_t* n_live;                 // [list][KIND]
};

// The adjoint over up to 64 frames: colour bricks culled like the forward's, then
// persistent waves over the live list.
struct BackwardArgs {
    int32_t cdim[3];
    int32_t cbricks[3];
    uint32_t n_items;                 // colour bricks
    int32_t n_frames;                 // <= 64
    int32_t disable_cull;             // 1: every brick is live in every frame
    const FrameConsts* frames;        // [n_frames], with their depth pyramids
    const float* wc0;                 // initial colour weights or NULL
    const float* grad;                // [3][Nc]
    // chunks of a longer scan (the frames of the call are one chunk of it):
    const float* tail_in;             // NULL, or [Nc] prod (1 - alpha) over the later chunks'
                                      // frames; the gradient of C at the chunk's end is
                                      // grad * tail_in
    float* tail_out;                  // NULL, or [Nc] tail_in times this chunk's prod
                                      // (1 - alpha) (may be tail_in; voxels with a zero
                                      // gradient are left as they are)
    float* wc_out;                    // non-NULL: advance only, the colour weights after the
                                      // call's frames into wc_out (voxels of live bricks; the
                                      // others must hold wc0 already), no adjoint
    float* d_rgb;                     // [n][ch][cw][3]
    double* partials;                 // [n_items][6] (zero for bricks never live), then
                                      // [XI_BLOCKS][6] block sums of the reduction
    uint4* live;                      // (brick, frame mask low, frame mask high, 0)
    uint32_t* n_live;
    uint32_t* queue;
    double* pose_partials;            // NULL, or [n_items][n_frames][6] per-frame extrinsic
                                      // partials (zero for bricks never live), then
                                      // [XI_BLOCKS][n_frames][6] block sums and the
                                      // [n_frames][6] sums
    const double* pose_adjoint;       // [n_frames][12]: R (row-major) and t of each frame's
                                      // T_hd_from_world, for d_pose = -Ad^T (frame partial)
    // image-gradient records and their (frame, HD tile) bins (see kf_backward.hip)
    float* records;                   // [rec_cap][6]: cell x | y << 16 (bits), ax, ay, g beta (3)
    unsigned long long* rec_next;     // records reserved so far (may pass rec_cap)
    uint32_t rec_cap;                 // 0: every update is scattered with atomics
    uint4* segs;                      // [seg_cap] (first record, count, frame | spans, tiles)
    uint32_t* seg_next;
    uint32_t seg_cap;                 // n_frames * n_items: a brick has one segment per frame
    int32_t tiles_x, tiles_y;         // BWD_TILE_W x BWD_TILE_H tiles of the HD image
    uint32_t* bin_count;              // [n_frames * tiles + 1] segments per (frame, tile), then
                                      // their exclusive prefix sum
    uint32_t* bin_fill;               // [n_frames * tiles]
    uint32_t* bin_segs;               // [4 * seg_cap] segment of each bin entry
};

// Tiles of the HD image over which the adjoint adds its image-gradient records.
constexpr int BWD_TILE_W = 64, BWD_TILE_H = 32;

// 1.0f / z, correctly rounded, in fewer instructions than the IEEE division: the hardware
// reciprocal refined by one Newton step with an FMA residual, r + r (1 - z r), equals the
// IEEE quotient for every normal z with |z| <= 2^125; zero, subnormal, larger, infinite
// and NaN z take the IEEE division (a branch no lane takes for the camera depths of a
// scene).  The equality is checked over all 2^32 inputs by the test suite on gfx950.
__device__ __forceinline__ bool recip_exact(float z)
{
    const uint32_t mag = __builtin_bit_cast(uint32_t, z) & 0x7FFFFFFFu;
    return mag - 0x00800000u <= 0x7E000000u - 0x00800000u;
}

// The Newton-refined reciprocal alone: equal to 1.0f / z where recip_exact(z).
__device__ __forceinline__ float recip_newton(float z)
{
    const float r = __builtin_amdgcn_rcpf(z);
    return fmaf(fmaf(-z, r, 1.0f), r, r);
}

__device__ __forceinline__ float recip(float z)
{
    float q = recip_newton(z);
    if (__builtin_expect(!recip_exact(z), 0)) q = 1.0f / z;
    return q;
}

// A column's camera depths Z(k) = fma(a, k, c) are monotone in k (the fma of an exact
// product and sum is rounded monotonically), so if its first and last voxels' depths have
// one sign and lie where recip_newton is exact, so do all of them.
__device__ __forceinline__ bool column_recip_exact(float z_first, float z_last)
{
    const bool a = recip_exact(z_first), b = recip_exact(z_last);
    return a & b & ((z_first > 0.0f) == (z_last > 0.0f));
}

// The first active lane's value of a 32-bit unsigned quantity.  The builtin takes and
// returns a signed int: widening its result directly would sign-extend bit 31.
__device__ __forceinline__ uint32_t first_lane_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Rank of this lane among the set lanes of `ballot` below it.
__device__ __forceinline__ uint32_t lane_rank(unsigned long long ballot)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

// Per-launch tables are read-only for the whole launch: reading them through the
// constant address space lets the compiler use scalar loads and keep them in SGPRs (a
// kernel that also writes global memory otherwise gets vector loads, since the compiler
// cannot prove that its writes leave the table alone).
template <class T>
using const_ptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ const_ptr<T> as_const(const T* p)
{
    return (const_ptr<T>)p;
}

// Next entry of a work queue for the whole wave (one ticket per wave).  Every active lane
// takes part in the atomic (the first active lane adds 1, the others 0) and the first
// lane's result is broadcast, so the ticket is never defined under lane-dependent
// control flow.  (With a ticket taken inside `if (lane == 0)` the compiler may thread the
// loop into per-lane paths on which the other lanes never see a new ticket.)
__device__ __forceinline__ uint32_t wave_ticket(uint32_t* queue)
{
    const uint64_t ex = __builtin_amdgcn_read_exec();
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(ex >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)ex, 0u));
    return first_lane_u32(atomicAdd(queue, rank == 0 ? 1u : 0u));
}

// Ray casting of one camera through a volume (see kf_raycast.hip), rounded once from the
// double-precision constants the host computes.
struct RaycastArgs {
    float a[3], Bu[3], Bv[3], B0[3];     // geometry-index ray q = a + t (Bu x + Bv y + B0)
    float ac[3], Bcu[3], Bcv[3], Bc0[3]; // colour-index ray
    float Ru[3], Rv[3], R0[3], tw[3];    // world ray p = tw + t (Ru x + Rv y + R0)
    float inv_s[3];                      // 1 / geometry voxel size
    float gmax[3], cmax[3];              // dim - 1
    float delta;                         // sample spacing (camera depth, metres)
    int32_t gdim[3], cdim[3];
    int32_t width, height;
    const float *tsdf, *wg, *r, *g, *b, *wc;
    float* depth;                        // [height][width]
    float *vertex, *normal, *rgb;        // [height][width][3] each, or NULL
};

struct TextureArgs {
    float inv_s[3];                      // 1 / colour voxel size per axis
    float off[3];                        // -origin / s - 1/2: colour index of a world point
    float cmax[3];                       // colour dim - 1
    int32_t cdim[3];
    int32_t n_tri;
    int32_t atlas_width, atlas_height;
    const float* tri;                    // [n_tri][3][3] world vertices V1, V2, V3
    const int32_t* rects;                // [n_tri][4]: x, y, w, h of each map in the atlas
    const float *r, *g, *b, *wc;
    float* atlas;                        // [atlas_height][atlas_width][3], or NULL
    uint8_t* atlas8;                     // [atlas_height][atlas_width][3], or NULL
};

struct MeshArgs {
    int32_t dim[3];                      // geometry voxels per axis
    uint32_t n_voxels, n_blocks;         // n_blocks = ceil(n_voxels / 4096)
    float s[3], c[3];                    // voxel size; world centre of voxel 0
    const float *tsdf, *wg;
    uint8_t* info;                       // [n_voxels] vertex axes | triangle count << 3
    uint8_t* cfg;                        // [n_voxels] inside corners (cubes with triangles only)
    uint32_t* voff;                      // [n_voxels] first vertex index (vertex owners only)
    uint32_t* block_sums;                // [n_blocks][2] vertices, triangles (then offsets)
    uint32_t* totals;                    // [2]
    float* vertices;                     // [vcap][3]: slots at or past vcap are not written
    int32_t* triangles;                  // [tcap][3]
    uint32_t vcap, tcap;
};

// Tiles of level l of a pyramid whose level 0 has w0 x h0 tiles.
__host__ __device__ inline void pyr_level_dims(int32_t w0, int32_t h0, int32_t l, int32_t* w,
                                               int32_t* h, int32_t* offset)
{
    int32_t ww = w0, hh = h0, off = 0;
    for (int32_t q = 0; q < l; ++q) {
        off += ww * hh;
        ww = (ww + 1) / 2;
        hh = (hh + 1) / 2;
    }
    *w = ww;
    *h = hh;
    *offset = off;
}

}  // namespace kf
