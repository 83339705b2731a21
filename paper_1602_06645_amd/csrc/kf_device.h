// Data shared by the host launchers and the gfx950 kernels of libkfvol.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace kf {

// A work item is a brick of TX x TY columns and ZS voxels along z.  One workgroup of
// TX*TY = 256 lanes (four wave64s, one x-row of 64 voxels each) handles it; every lane
// keeps the state of its ZS voxels in registers for all frames of a pass.
constexpr int TX = 64;
constexpr int TY = 4;
constexpr int ZS = 8;
constexpr int BLOCK = TX * TY;

// Everything one frame contributes to the per-voxel arithmetic, rounded once from the
// double-precision values computed on the host.
struct FrameConsts {
    float Ag[9], bg[3];   // geometry voxel index -> depth camera (Eq. 5, voxel size folded in)
    float Ac[9], bc[3];   // colour voxel index   -> depth camera
    float Ah[9], bh[3];   // colour voxel index   -> HD camera (Eq. 3 composed with Eq. 5)
    float fx, fy, cx, cy, inv_fx, inv_fy;  // K_c and the diagonal of K_c^-1
    float fxr, fyr, cxr, cyr;              // K_hd
    float trunc, inv_trunc, w_max, sigma2, gate;
    float wm1, hm1;       // depth image W-1, H-1 (exact in float)
    float cwm2, chm2;     // HD image CW-2, CH-2
    int32_t dw, dh, cw, ch;
    const float* depth;   // [dh][dw]
    const void* rgb;      // [ch][cw][3], uint8 or float
};

enum PixFmt : int32_t { FMT_RGB8 = 0, FMT_RGBF32 = 1 };

// One volume (scan) of a launch.
struct SceneDev {
    float *tsdf, *wg, *r, *g, *b, *wc;
    int32_t gdim[3], cdim[3];
    int32_t gtiles[3], ctiles[3];   // bricks per axis
    uint32_t item_begin;            // first global work item of this scene
    uint32_t geom_items;            // geometry bricks; colour bricks follow them
    uint32_t colour_items;
    int32_t frame_begin;            // first entry of the frame table used by this pass
    int32_t n_frames;               // frames of this scene in this pass (may be 0)
    int32_t fmt;                    // PixFmt
};

enum Mode : int32_t { MODE_INTEGRATE = 0, MODE_STATUS = 1, MODE_COUNT = 2 };

struct IntegrateArgs {
    const SceneDev* scenes;         // table of n_scenes (batch launches)
    const FrameConsts* frames;      // frame table (batch launches)
    int32_t n_scenes;
    uint32_t n_items;
    uint32_t* queue;                // persistent launch: shared item counter; NULL: grid launch
    unsigned long long* counters;   // MODE_COUNT: uint64[6]
    uint8_t* gstatus;               // MODE_STATUS outputs
    uint8_t* cstatus;
    SceneDev scene0;                // single-scene launches: the scene ...
    FrameConsts frame0;             // ... and its single frame, passed by value
};

struct BackwardArgs {
    int32_t cdim[3];
    int32_t ctiles[3];
    uint32_t n_items;
    int32_t n_frames;
    const FrameConsts* frames;      // [n_frames]
    const float* wc0;               // initial colour weights or NULL
    const float* grad;              // [3][Nc]
    float* d_rgb;                   // [n][ch][cw][3]
    double* partials;               // [gridDim][6]
};

}  // namespace kf
