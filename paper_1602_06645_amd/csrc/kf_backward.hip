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
// The colour bricks of the forward (8 x 8 x 8, one wave each) are culled frame by frame
// exactly like the forward's (a culled frame cannot update any voxel of the brick, so
// its alpha is 0).  Persistent waves take the live bricks; each voxel replays the forward
// decisions of its live frames (the same single-precision sequence as the forward, so the
// same frames update it), keeps alpha_n in an LDS history private to the lane, and a
// reverse sweep scatters the image gradient with float atomics and accumulates the
// extrinsic gradient in double.  Each brick writes its own extrinsic partial; a last
// kernel sums them in a fixed order, so d_xi is deterministic.
#include <hip/hip_runtime.h>

#include "kf_cull.h"
#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

constexpr int BWD_MAX_FRAMES = 64;

namespace {

// Image reads of the replay go through bounds-checked buffer resources: an offset past
// the image reads 0, so a voxel outside the frustum needs no branch around its reads.
constexpr uint32_t kOffImage = 0x7FFFFFF0u;

__device__ __forceinline__ float image_load(const void* p, uint32_t bytes, uint32_t byte_off)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// The forward decision of one colour voxel for one frame, split so that several frames'
// image reads can be in flight together: weight_fetch projects the voxel centre into the
// depth camera (Eq. 5-6) and reads its depth and weight-map entries; weight_test applies
// every test of Sec. IV.B except the gate (which needs the running weight) and returns the
// weight-map W if they all pass, else 0.  Same single-precision operations as the forward.
struct WeightFetch {
    float Xc, Yc, Zc, u, v, d, w;
    bool in;
};

template <class C>
__device__ __forceinline__ WeightFetch weight_fetch(const C& c, float fi, float fj, float fk)
{
    WeightFetch r;
    r.Xc = fmaf(c.Ac[2], fk, fmaf(c.Ac[1], fj, fmaf(c.Ac[0], fi, c.bc[0])));
    r.Yc = fmaf(c.Ac[5], fk, fmaf(c.Ac[4], fj, fmaf(c.Ac[3], fi, c.bc[1])));
    r.Zc = fmaf(c.Ac[8], fk, fmaf(c.Ac[7], fj, fmaf(c.Ac[6], fi, c.bc[2])));
    const float iz = recip(r.Zc);
    r.u = rintf(fmaf(c.fx, r.Xc * iz, c.cx));
    r.v = rintf(fmaf(c.fy, r.Yc * iz, c.cy));
    r.in = (r.Zc > 0.0f) & (r.u >= 0.0f) & (r.u <= c.wm1) & (r.v >= 0.0f) & (r.v <= c.hm1);
    const uint32_t off = r.in ? ((uint32_t)(int)r.v * (uint32_t)c.dw + (uint32_t)(int)r.u) * 4u : kOffImage;
    const uint32_t bytes = (uint32_t)(c.dw * c.dh) * 4u;
    r.d = image_load(c.depth, bytes, off);
    r.w = image_load(c.wmap, bytes, off);
    return r;
}

template <class C>
__device__ __forceinline__ float weight_test(const C& c, const WeightFetch& r, float fi, float fj,
                                             float fk)
{
    const float Px = ((r.u - c.cx) * c.inv_fx) * r.d;
    const float Py = ((r.v - c.cy) * c.inv_fy) * r.d;
    const float dx = r.Xc - Px, dy = r.Yc - Py, dz = r.Zc - r.d;
    const bool valid = valid_depth(r.d);
    const bool band = r.in & valid & !(fmaf(dx, dx, fmaf(dy, dy, dz * dz)) > c.sigma2) &
                      (__builtin_bit_cast(uint32_t, r.w) != kNoNormal);
    const float qx = fmaf(c.Ah[2], fk, fmaf(c.Ah[1], fj, fmaf(c.Ah[0], fi, c.bh[0])));
    const float qy = fmaf(c.Ah[5], fk, fmaf(c.Ah[4], fj, fmaf(c.Ah[3], fi, c.bh[1])));
    const float qz = fmaf(c.Ah[8], fk, fmaf(c.Ah[7], fj, fmaf(c.Ah[6], fi, c.bh[2])));
    const float iqz = recip(qz);
    const float x0 = floorf(fmaf(c.fxr, qx * iqz, c.cxr));
    const float y0 = floorf(fmaf(c.fyr, qy * iqz, c.cyr));
    const bool hd = (qz > 0.0f) & (x0 >= 0.0f) & (x0 <= c.hd_xmax) & (y0 >= 0.0f) & (y0 <= c.hd_ymax);
    return (band & hd) ? r.w : 0.0f;
}

__device__ __forceinline__ double wave_sum_d(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

}  // namespace

// One block per culling chunk of CHUNK^3 colour bricks: the first wave tests the chunk's
// voxel box against the frames (one lane per frame); the chunk's bricks are then tested,
// four at a time (one wave per brick), only for the frames the chunk passed (exact, the
// chunk test being conservative for every voxel in it), a ballot giving each brick's live
// frames.  The live entries are gathered in LDS and appended with one atomic per block.
constexpr int BWD_CHUNK_BRICKS = CHUNK * CHUNK * CHUNK;

__global__ __launch_bounds__(BLOCK) void backward_cull_kernel(BackwardArgs a)
{
    __shared__ uint4 s_ent[BWD_CHUNK_BRICKS];
    __shared__ uint32_t s_n, s_base;
    __shared__ unsigned long long s_cmask;
    const int cc[3] = {(a.cbricks[0] + CHUNK - 1) / CHUNK, (a.cbricks[1] + CHUNK - 1) / CHUNK,
                       (a.cbricks[2] + CHUNK - 1) / CHUNK};
    const uint32_t lc = blockIdx.x;
    const int bx0 = (int)(lc % (uint32_t)cc[0]) * CHUNK;
    const int by0 = (int)((lc / (uint32_t)cc[0]) % (uint32_t)cc[1]) * CHUNK;
    const int bz0 = (int)(lc / ((uint32_t)cc[0] * (uint32_t)cc[1])) * CHUNK;
    const int nbx = min(CHUNK, a.cbricks[0] - bx0), nby = min(CHUNK, a.cbricks[1] - by0);
    const int nbz = min(CHUNK, a.cbricks[2] - bz0);
    const int f = (int)(threadIdx.x % WAVE);
    if (threadIdx.x < WAVE) {
        bool live = false;
        if (f < a.n_frames) {
            const int i0 = bx0 * CBX, i1 = min(a.cdim[0], (bx0 + nbx) * CBX) - 1;
            const int j0 = by0 * CBY, j1 = min(a.cdim[1], (by0 + nby) * CBY) - 1;
            const int k0 = bz0 * ZS, k1 = min(a.cdim[2], (bz0 + nbz) * ZS) - 1;
            live = a.disable_cull || brick_live(a.frames[f], true, i0, i1, j0, j1, k0, k1);
        }
        const unsigned long long m = __ballot(live);
        if (threadIdx.x == 0) {
            s_cmask = m;
            s_n = 0;
        }
    }
    __syncthreads();
    const unsigned long long cmask = s_cmask;
    if (cmask == 0) return;   // the whole block
    const int nbr = nbx * nby * nbz;
    for (int r = 0; r < BWD_CHUNK_BRICKS / (BLOCK / WAVE); ++r) {
        const int q = r * (BLOCK / WAVE) + (int)(threadIdx.x / WAVE);
        bool live = false;
        uint32_t li = 0;
        if (q < nbr) {
            const int bx = bx0 + q % nbx, by = by0 + (q / nbx) % nby, bz = bz0 + q / (nbx * nby);
            li = (uint32_t)bx + (uint32_t)a.cbricks[0] * ((uint32_t)by + (uint32_t)a.cbricks[1] * (uint32_t)bz);
            if ((cmask >> f) & 1ull) {
                const int i0 = bx * CBX, i1 = min(a.cdim[0], i0 + CBX) - 1;
                const int j0 = by * CBY, j1 = min(a.cdim[1], j0 + CBY) - 1;
                const int k0 = bz * ZS, k1 = min(a.cdim[2], k0 + ZS) - 1;
                live = a.disable_cull || brick_live(a.frames[f], true, i0, i1, j0, j1, k0, k1);
            }
        }
        const unsigned long long mask = __ballot(live);
        if (f == 0 && mask != 0)
            s_ent[atomicAdd(&s_n, 1u)] = make_uint4(li, (uint32_t)mask, (uint32_t)(mask >> 32), 0u);
    }
    __syncthreads();
    if (threadIdx.x == 0) s_base = s_n ? atomicAdd(a.n_live, s_n) : 0u;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < s_n; e += BLOCK) a.live[s_base + e] = s_ent[e];
}

// HIST: LDS floats per lane for the alpha history (at least the frames of the call).
// POSE: also the per-frame extrinsic partials of each brick (for the depth-pose adjoint),
// summed per frame in the wave's LDS and written as one row per brick.
template <int HIST, bool POSE>
__global__ __launch_bounds__(BLOCK) void backward_kernel(BackwardArgs a)
{
    __shared__ float s_alpha[BLOCK * HIST];   // lane t of wave w: [w][f][t]
    __shared__ double s_pose[POSE ? (BLOCK / WAVE) * HIST * 6 : 1];
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    float* hist = s_alpha + wave * WAVE * HIST + lane;
    double* facc = s_pose + (POSE ? wave * HIST * 6 : 0);
    const size_t nvox = (size_t)a.cdim[0] * (size_t)a.cdim[1] * (size_t)a.cdim[2];
    const uint32_t n_live = *a.n_live;
    const const_ptr<FrameConsts> frames = as_const(a.frames);
    for (;;) {
        const uint32_t e = wave_ticket(a.queue);
        if (e >= n_live) break;
        const uint4 ent = a.live[e];
        const uint32_t li = first_lane_u32(ent.x);
        const unsigned long long mask = ((unsigned long long)first_lane_u32(ent.z) << 32) |
                                        (unsigned long long)first_lane_u32(ent.y);
        const int bx = (int)(li % (uint32_t)a.cbricks[0]);
        const int by = (int)((li / (uint32_t)a.cbricks[0]) % (uint32_t)a.cbricks[1]);
        const int bz = (int)(li / ((uint32_t)a.cbricks[0] * (uint32_t)a.cbricks[1]));
        const int i = bx * CBX + lane % CBX, j = by * CBY + lane / CBX, k0 = bz * ZS;
        double xi[6] = {0, 0, 0, 0, 0, 0};
        if constexpr (POSE) {
            for (int q = lane; q < a.n_frames * 6; q += WAVE) facc[q] = 0.0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (i < a.cdim[0] && j < a.cdim[1]) {
            const float fi = (float)i, fj = (float)j;
            const int kn = min(ZS, a.cdim[2] - k0);
            for (int kk = 0; kk < kn; ++kk) {
                const int k = k0 + kk;
                const float fk = (float)k;
                const size_t idx = ((size_t)k * (size_t)a.cdim[1] + (size_t)j) * (size_t)a.cdim[0] + (size_t)i;
                const float g0 = a.grad[idx], g1 = a.grad[nvox + idx], g2 = a.grad[2 * nvox + idx];
                if (g0 == 0.0f && g1 == 0.0f && g2 == 0.0f) continue;
                // forward replay over the live frames, by rank among them: first the
                // weight-independent tests, four frames at a time with their image reads
                // in flight together (W or 0 into the history) ...
                int r = 0;
                for (unsigned long long m = mask; m;) {
                    int fr[4];
                    bool ok[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        ok[q] = m != 0ull;
                        fr[q] = ok[q] ? __builtin_ctzll(m) : fr[0];
                        m &= m - 1;
                    }
                    WeightFetch wf[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) wf[q] = weight_fetch(frames[fr[q]], fi, fj, fk);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (ok[q]) hist[(r + q) * WAVE] = weight_test(frames[fr[q]], wf[q], fi, fj, fk);
                    r += 4;
                }
                // ... then the gate against the running weight and alpha_n
                float Wc = a.wc0 ? a.wc0[idx] : 0.0f;
                int any = 0;
                r = 0;
                for (unsigned long long m = mask; m; m &= m - 1, ++r) {
                    const float w = hist[r * WAVE];
                    float alpha = 0.0f;
                    if (w > 0.0f && w > frames[__builtin_ctzll(m)].gate * Wc) {
                        alpha = w / (Wc + w);
                        Wc = fmaf(w, 1.0f - Wc, Wc);
                        any = 1;
                    }
                    hist[r * WAVE] = alpha;
                }
                if (!any) continue;
                // reverse sweep
                float tail = 1.0f;
                for (unsigned long long m = mask; m; m &= ~(1ull << (63 - __builtin_clzll(m)))) {
                    const int f = 63 - __builtin_clzll(m);
                    --r;
                    const float alpha = hist[r * WAVE];
                    if (alpha == 0.0f) continue;
                    const float beta = alpha * tail;
                    tail *= 1.0f - alpha;
                    const auto& c = frames[f];
                    const float qx = fmaf(c.Ah[2], fk, fmaf(c.Ah[1], fj, fmaf(c.Ah[0], fi, c.bh[0])));
                    const float qy = fmaf(c.Ah[5], fk, fmaf(c.Ah[4], fj, fmaf(c.Ah[3], fi, c.bh[1])));
                    const float qz = fmaf(c.Ah[8], fk, fmaf(c.Ah[7], fj, fmaf(c.Ah[6], fi, c.bh[2])));
                    const float iqz = recip(qz);
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
                    if constexpr (POSE) {
                        double* fa = facc + f * 6;
                        atomicAdd(fa + 0, dqx);
                        atomicAdd(fa + 1, dqy);
                        atomicAdd(fa + 2, dqz);
                        atomicAdd(fa + 3, (double)qy * dqz - (double)qz * dqy);
                        atomicAdd(fa + 4, (double)qz * dqx - (double)qx * dqz);
                        atomicAdd(fa + 5, (double)qx * dqy - (double)qy * dqx);
                    }
                }
            }
        }
        // the brick's extrinsic partial (a fixed butterfly order: deterministic)
        const double s0 = wave_sum_d(xi[0]), s1 = wave_sum_d(xi[1]), s2 = wave_sum_d(xi[2]);
        const double s3 = wave_sum_d(xi[3]), s4 = wave_sum_d(xi[4]), s5 = wave_sum_d(xi[5]);
        // every lane stores component lane % 6 (the values are the same in every lane), so
        // nothing in the loop depends on the lane index
        const int q = lane % 6;
        const double sq = q == 0 ? s0 : q == 1 ? s1 : q == 2 ? s2 : q == 3 ? s3 : q == 4 ? s4 : s5;
        a.partials[(size_t)li * 6 + q] = sq;
        if constexpr (POSE) {
            // the brick's per-frame partials, one row per brick (indexed by the brick, so the
            // reduction order does not depend on scheduling)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            double* row = a.pose_partials + (size_t)li * (size_t)a.n_frames * 6;
            for (int c = lane; c < a.n_frames * 6; c += WAVE) row[c] = facc[c];
        }
    }
}

// Column sums of a [n_rows][width] double array over rows [b * span, (b + 1) * span) for
// block b: thread t adds columns t, t + 256, ... row by row in order (deterministic).
__global__ __launch_bounds__(256) void reduce_rows_kernel(const double* rows, uint32_t n_rows,
                                                          uint32_t width, uint32_t span, double* out)
{
    const uint32_t r0 = blockIdx.x * span, r1 = min(n_rows, r0 + span);
    for (uint32_t c = threadIdx.x; c < width; c += 256) {
        double acc = 0.0;
        for (uint32_t r = r0; r < r1; ++r) acc += rows[(size_t)r * width + c];
        out[(size_t)blockIdx.x * width + c] = acc;
    }
}

// d_pose[f] = -Ad(T_f)^T x_f for the frame's extrinsic partial x_f = (x_rho, x_phi) and
// T_f = T_hd_from_world = (R, t): rho part -R^T x_rho, phi part R^T (t x x_rho - x_phi).
__global__ __launch_bounds__(64) void pose_adjoint_kernel(const double* x, const double* T,
                                                          int32_t n_frames, double* d_pose)
{
    const int f = (int)(blockIdx.x * 64 + threadIdx.x);
    if (f >= n_frames) return;
    const double* R = T + 12 * (size_t)f;
    const double* t = R + 9;
    const double* xr = x + 6 * (size_t)f;
    const double* xp = xr + 3;
    const double c[3] = {t[1] * xr[2] - t[2] * xr[1] - xp[0], t[2] * xr[0] - t[0] * xr[2] - xp[1],
                         t[0] * xr[1] - t[1] * xr[0] - xp[2]};
    for (int m = 0; m < 3; ++m) {
        d_pose[6 * (size_t)f + m] = -(R[m] * xr[0] + R[3 + m] * xr[1] + R[6 + m] * xr[2]);
        d_pose[6 * (size_t)f + 3 + m] = R[m] * c[0] + R[3 + m] * c[1] + R[6 + m] * c[2];
    }
}

// Sum the per-brick partials in a fixed order, in two launches: block b of the first adds
// the partials of bricks [b * span, (b + 1) * span) (lane t takes bricks t, t + 256, ...
// of the range, then a fixed tree over the 256 lanes); the second adds the block sums the
// same way.  The result does not depend on scheduling.

__global__ __launch_bounds__(256) void reduce_xi_kernel(const double* partials, uint32_t n,
                                                        uint32_t span, double* out)
{
    __shared__ double s[6][256];
    const uint32_t b0 = blockIdx.x * span;
    const uint32_t b1 = min(n, b0 + span);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += 256)
        for (int q = 0; q < 6; ++q) acc[q] += partials[(size_t)b * 6 + q];
    for (int q = 0; q < 6; ++q) s[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int q = 0; q < 6; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[(size_t)blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

template <int HIST, bool POSE>
static hipError_t launch_backward_hist(const BackwardArgs& a, int device, hipStream_t stream)
{
    int n_cu = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, backward_kernel<HIST, POSE>, BLOCK, 0);
    if (e != hipSuccess) return e;
    const unsigned grid = (unsigned)(n_cu * (per_cu > 0 ? per_cu : 1));
    hipLaunchKernelGGL((backward_kernel<HIST, POSE>), dim3(grid), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_backward(const BackwardArgs& a, double* d_xi, double* d_pose, int device,
                           hipStream_t stream)
{
    const bool pose = d_pose != nullptr && a.pose_partials != nullptr;
    if (a.n_frames > BWD_MAX_FRAMES) return hipErrorInvalidValue;
    if (a.n_items > 0) {
        const uint32_t chunks = (uint32_t)((a.cbricks[0] + CHUNK - 1) / CHUNK) *
                                (uint32_t)((a.cbricks[1] + CHUNK - 1) / CHUNK) *
                                (uint32_t)((a.cbricks[2] + CHUNK - 1) / CHUNK);
        hipLaunchKernelGGL(backward_cull_kernel, dim3(chunks), dim3(BLOCK), 0, stream, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (pose)
            e = a.n_frames <= 32 ? launch_backward_hist<32, true>(a, device, stream)
                                 : launch_backward_hist<64, true>(a, device, stream);
        else
            e = a.n_frames <= 32 ? launch_backward_hist<32, false>(a, device, stream)
                                 : launch_backward_hist<64, false>(a, device, stream);
        if (e != hipSuccess) return e;
    }
    if (pose && a.n_frames > 0) {
        // per-frame column sums over the bricks (two fixed-order stages), then the adjoint map
        const uint32_t width = (uint32_t)a.n_frames * 6;
        double* stage = a.pose_partials + (size_t)a.n_items * width;
        double* sums = stage + (size_t)XI_BLOCKS * width;
        const uint32_t span = (a.n_items + XI_BLOCKS - 1) / XI_BLOCKS;
        hipLaunchKernelGGL(reduce_rows_kernel, dim3(XI_BLOCKS), dim3(256), 0, stream,
                           (const double*)a.pose_partials, a.n_items, width, span > 0 ? span : 1u, stage);
        hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(256), 0, stream, (const double*)stage,
                           (uint32_t)XI_BLOCKS, width, (uint32_t)XI_BLOCKS, sums);
        hipLaunchKernelGGL(pose_adjoint_kernel, dim3((a.n_frames + 63) / 64), dim3(64), 0, stream,
                           (const double*)sums, a.pose_adjoint, a.n_frames, d_pose);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // stage 1 writes XI_BLOCKS block sums after the partials (a.partials holds room for them)
    double* block_sums = a.partials + (size_t)a.n_items * 6;
    const uint32_t span = (a.n_items + XI_BLOCKS - 1) / XI_BLOCKS;
    hipLaunchKernelGGL(reduce_xi_kernel, dim3(XI_BLOCKS), dim3(256), 0, stream, a.partials,
                       a.n_items, span > 0 ? span : 1u, block_sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_xi_kernel, dim3(1), dim3(256), 0, stream, (const double*)block_sums,
                       (uint32_t)XI_BLOCKS, (uint32_t)XI_BLOCKS, d_xi);
    return hipGetLastError();
}

}  // namespace kf
