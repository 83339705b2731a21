// Host-side launchers of the libkfvol kernels (defined next to the kernels).
#pragma once
#include <hip/hip_runtime.h>

#include "kf_device.h"

namespace kf {

// mode: Mode; inline_args: single scene and single frame passed by value in `a`.
// grid: number of blocks of a persistent launch (a.queue != NULL); ignored otherwise.
hipError_t launch_integrate(int mode, bool inline_args, const IntegrateArgs& a, uint32_t grid,
                            hipStream_t stream);
// Blocks that stay resident at once on `device` for a persistent launch of `mode`.
hipError_t persistent_grid(int mode, int device, uint32_t* blocks);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t stream);

// Backward: one block per colour brick; partials holds 6 doubles per block.
uint32_t backward_blocks(const BackwardArgs& a);
hipError_t launch_backward(const BackwardArgs& a, double* d_xi, hipStream_t stream);

}  // namespace kf
