// Host-side launchers of the libkfvol kernels (defined next to the kernels).
#pragma once
#include <hip/hip_runtime.h>

#include "kf_device.h"

namespace kf {

// Depth min/max pyramids of frames_dev[0 .. n_frames); max_tiles0: the largest level-0
// tile count among them.
hipError_t launch_pyramids(const FrameConsts* frames_dev, int32_t n_frames, int32_t max_tiles0,
                           hipStream_t stream);
// Pixel maps (FrameConsts::pmap) of frames_dev[0 .. n_frames); max_pixels: the largest
// depth image among them.
hipError_t launch_pixel_maps(const FrameConsts* frames_dev, int32_t n_frames, int32_t max_pixels,
                              hipStream_t stream);
// One lane per (brick, frame) of the pass: append (brick, live-frame mask) entries.
hipError_t launch_cull(const CullArgs& a, hipStream_t stream);
// Persistent integration over the live entries of one kind (mode: MODE_INTEGRATE or
// MODE_COUNT; kind: KIND_GEOM or KIND_COLOUR; shape: index into BRICK_SHAPES[kind], the
// shape the pass's scene tables were planned with).
hipError_t launch_integrate(int mode, int kind, int shape, const IntegrateArgs& a, uint32_t grid,
                            hipStream_t stream);
// Status codes of one frame for every brick of one kind.
hipError_t launch_status(bool colour, const StatusArgs& a, hipStream_t stream);
// Blocks that stay resident at once on `device` for a persistent launch of (mode, kind).
hipError_t persistent_grid(int mode, int kind, int shape, int device, uint32_t* blocks);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t stream);

// Ray cast one camera (see kf_raycast.hip).
hipError_t launch_raycast(const RaycastArgs& a, hipStream_t stream);

// Texel colours of every triangle's texture map (see kf_texture.hip).
hipError_t launch_texture(const TextureArgs& a, hipStream_t stream);

// Marching cubes (see kf_mesh.hip): classify, count and scan (totals at a.totals), then
// write vertices and triangles (needs the outputs of the count step).
hipError_t launch_mesh_count(const MeshArgs& a, hipStream_t stream);
hipError_t launch_mesh_emit(const MeshArgs& a, hipStream_t stream);

// Quadric-error decimation of a valid mesh on the host (kf_decimate.cpp; the C ABI entry
// kf_mesh_decimate checks the arguments): writes the kept vertices and triangles (at most the
// input counts) and their numbers.
void decimate_mesh(const float* vertices, int64_t n_vertices, const int32_t* triangles,
                   int64_t n_triangles, double rate, float* out_vertices, int64_t* out_n_vertices,
                   int32_t* out_triangles, int64_t* out_n_triangles);

// Adjoint: cull the colour bricks, integrate the live ones backwards (persistent grid),
// then sum the per-brick extrinsic partials in a fixed order into d_xi.
hipError_t launch_backward(const BackwardArgs& a, double* d_xi, double* d_pose, int device,
                           hipStream_t stream);

// Column sums of a [n_rows][width] double array, rows added in order (one block).
hipError_t launch_sum_rows(const double* rows, uint32_t n_rows, uint32_t width, double* out,
                           hipStream_t stream);

}  // namespace kf
