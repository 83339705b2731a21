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
// The colour bricks of the forward (8 x 8 x 8) are culled frame by frame exactly like the
// forward's (a culled frame cannot update any voxel of the brick, so its alpha is 0).  A
// persistent workgroup of 512 threads takes one live brick at a time, one voxel per
// thread: each voxel replays the forward decisions of its live frames (the same
// single-precision sequence as the forward, so the same frames update it) and keeps
// alpha_n in LDS; the brick then sweeps the frames backwards together.  Each update's
// image gradient is written as a record (pixel, bilinear fractions, g beta) into the
// brick's segment for that frame; a segment lists the HD tiles its cells can touch
// (from the brick's projected corners).  Three small launches sort the segments by
// (frame, tile), and one workgroup per (frame, tile) adds its records in LDS and adds
// the tile into the image gradient: no global atomics per update.  A brick whose records
// do not fit the record buffer, or whose footprint in a frame is larger than 2 x 2 tiles
// (or crosses the HD camera plane), scatters that frame's updates with float atomics
// instead (same values, another order of addition).  The extrinsic gradient is summed
// per brick in double and the bricks' partials in a fixed order (deterministic d_xi).
#include <hip/hip_runtime.h>

#include "kf_cull.h"
#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

constexpr int BWD_MAX_FRAMES = 64;
constexpr int BWD_BLOCK = CBX * CBY * ZS;      // one colour brick, one voxel per thread
constexpr int BWD_WAVES = BWD_BLOCK / WAVE;    // one wave per z slice of the brick
static_assert(BWD_WAVES == ZS && CBX * CBY == WAVE, "a wave is one z slice of a brick");

namespace {

// Image reads of the replay go through bounds-checked buffer resources: an offset past
// the image reads 0, so a voxel outside the frustum needs no branch around its reads.
constexpr uint32_t kOffImage = 0x7FFFFFF0u;

__device__ __forceinline__ float4 image_load4(const void* p, uint32_t bytes, uint32_t byte_off)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
    float4 f;
    __builtin_memcpy(&f, &v, sizeof f);
    return f;
}

// The forward decision of one colour voxel for one frame, split so that several frames'
// image reads can be in flight together: weight_fetch projects the voxel centre into the
// depth camera (Eq. 5-6) and reads its pixel-map entry (depth, P of Eq. 7, W); weight_test applies
// every test of Sec. IV.B except the gate (which needs the running weight) and returns the
// weight-map W if they all pass, else 0.  Same single-precision operations as the forward.
struct WeightFetch {
    float Xc, Yc, Zc, d, Px, Py, w;
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
    const float u = rintf(fmaf(c.fx, r.Xc * iz, c.cx));
    const float v = rintf(fmaf(c.fy, r.Yc * iz, c.cy));
    r.in = (r.Zc > 0.0f) & (u >= 0.0f) & (u <= c.wm1) & (v >= 0.0f) & (v <= c.hm1);
    const uint32_t off = r.in ? ((uint32_t)(int)v * (uint32_t)c.dw + (uint32_t)(int)u) * 16u : kOffImage;
    const float4 pm = image_load4(c.pmap, (uint32_t)(c.dw * c.dh) * 16u, off);
    r.d = pm.x;
    r.Px = pm.y;
    r.Py = pm.z;
    r.w = pm.w;
    return r;
}

template <class C>
__device__ __forceinline__ float weight_test(const C& c, const WeightFetch& r, float fi, float fj,
                                             float fk)
{
    const float dx = r.Xc - r.Px, dy = r.Yc - r.Py, dz = r.Zc - r.d;
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

// HD tiles that the bilinear cells of a brick's voxels can touch in one frame: the
// brick's box lies in front of the HD camera and its image lies inside the hull of its
// 8 projected corners (projected in double, widened by a pixel for the single-precision
// rounding of the per-voxel projection, and by the cell's second pixel), clamped to the
// image.  Returns the first tile on each axis (t[0] = x, t[1] = y) and whether the range
// spans a second tile (t[2] = x, t[3] = y); false when a corner is not in front of the
// camera, the range spans more than 2 tiles on an axis, or no pixel of the image (the
// frame's updates are then scattered directly).
__device__ inline bool brick_tiles(const FrameConsts& c, int i0, int i1, int j0, int j1, int k0,
                                   int k1, int* t)
{
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int q = 0; q < 8; ++q) {
        const double fi = (q & 1) ? i1 : i0, fj = (q & 2) ? j1 : j0, fk = (q & 4) ? k1 : k0;
        const double qx = (double)c.Ah[0] * fi + (double)c.Ah[1] * fj + (double)c.Ah[2] * fk + c.bh[0];
        const double qy = (double)c.Ah[3] * fi + (double)c.Ah[4] * fj + (double)c.Ah[5] * fk + c.bh[1];
        const double qz = (double)c.Ah[6] * fi + (double)c.Ah[7] * fj + (double)c.Ah[8] * fk + c.bh[2];
        if (!(qz > 1e-6)) return false;
        const double x = (double)c.fxr * qx / qz + c.cxr, y = (double)c.fyr * qy / qz + c.cyr;
        xmin = fmin(xmin, x);
        xmax = fmax(xmax, x);
        ymin = fmin(ymin, y);
        ymax = fmax(ymax, y);
    }
    const double lo_x = fmax(floor(xmin) - 1.0, 0.0), hi_x = fmin(floor(xmax) + 2.0, (double)(c.cw - 1));
    const double lo_y = fmax(floor(ymin) - 1.0, 0.0), hi_y = fmin(floor(ymax) + 2.0, (double)(c.ch - 1));
    if (!(lo_x <= hi_x) || !(lo_y <= hi_y)) return false;
    const int tx0 = (int)lo_x / BWD_TILE_W, tx1 = (int)hi_x / BWD_TILE_W;
    const int ty0 = (int)lo_y / BWD_TILE_H, ty1 = (int)hi_y / BWD_TILE_H;
    t[0] = tx0;
    t[1] = ty0;
    t[2] = tx1 - tx0;
    t[3] = ty1 - ty0;
    return tx1 - tx0 <= 1 && ty1 - ty0 <= 1;
}

// A segment (uint4): first record, record count, frame | x span << 8 | y span << 9, and
// first tile x | first tile y << 16.
__device__ __forceinline__ void segment_tiles(uint4 sg, int* f, int* tx0, int* tx1, int* ty0, int* ty1)
{
    *f = (int)(sg.z & 0xFFu);
    *tx0 = (int)(sg.w & 0xFFFFu);
    *ty0 = (int)(sg.w >> 16);
    *tx1 = *tx0 + (int)((sg.z >> 8) & 1u);
    *ty1 = *ty0 + (int)((sg.z >> 9) & 1u);
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

// HIST: frames of the alpha history (at least the frames of the call).
// POSE: also the per-frame extrinsic partials of each brick (for the depth-pose adjoint),
// summed per frame in LDS and written as one row per brick.
template <int HIST, bool POSE>
__global__ __launch_bounds__(BWD_BLOCK) void backward_kernel(BackwardArgs a)
{
    __shared__ float s_alpha[HIST * BWD_BLOCK];         // [rank][thread]
    __shared__ uint32_t s_wcnt[BWD_WAVES][HIST];        // records per wave and rank, then
                                                        // the wave's offset in the segment
    __shared__ uint32_t s_seg[HIST];                    // first record of each rank's segment
    __shared__ uint32_t s_cnt[HIST];                    // records of each rank's segment
    __shared__ int32_t s_tiles[HIST][4];                // tiles of each rank's segment (brick_tiles)
    __shared__ double s_xi[BWD_WAVES][6];
    __shared__ double s_pose[POSE ? HIST * 6 : 1];      // [frame][6]
    __shared__ double s_pw[POSE ? 2 : 1][BWD_WAVES][6]; // per-wave sums of one frame (two
                                                        // frames alternate)
    __shared__ uint32_t s_ticket;
    __shared__ unsigned long long s_direct;             // ranks scattered with atomics

    const int t = threadIdx.x, lane = t & (WAVE - 1), wave = t / WAVE;
    float* hist = s_alpha + t;
    const size_t nvox = (size_t)a.cdim[0] * (size_t)a.cdim[1] * (size_t)a.cdim[2];
    const uint32_t n_live = *a.n_live;
    const const_ptr<FrameConsts> frames = as_const(a.frames);
    for (;;) {
        if (t == 0) s_ticket = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t e = first_lane_u32(s_ticket);
        if (e >= n_live) break;
        const uint4 ent = a.live[e];
        const uint32_t li = first_lane_u32(ent.x);
        const unsigned long long mask = ((unsigned long long)first_lane_u32(ent.z) << 32) |
                                        (unsigned long long)first_lane_u32(ent.y);
        const int n_r = __builtin_popcountll(mask);
        const int bx = (int)(li % (uint32_t)a.cbricks[0]);
        const int by = (int)((li / (uint32_t)a.cbricks[0]) % (uint32_t)a.cbricks[1]);
        const int bz = (int)(li / ((uint32_t)a.cbricks[0] * (uint32_t)a.cbricks[1]));
        const int i = bx * CBX + lane % CBX, j = by * CBY + lane / CBX, k = bz * ZS + wave;
        const bool inside = i < a.cdim[0] && j < a.cdim[1] && k < a.cdim[2];
        const float fi = (float)i, fj = (float)j, fk = (float)k;
        const size_t idx = ((size_t)k * (size_t)a.cdim[1] + (size_t)j) * (size_t)a.cdim[0] + (size_t)i;
        float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, tail0 = 1.0f;
        if (inside && !a.wc_out) {
            g0 = a.grad[idx];
            g1 = a.grad[nvox + idx];
            g2 = a.grad[2 * nvox + idx];
            if (a.tail_in) {
                tail0 = a.tail_in[idx];
                g0 *= tail0;
                g1 *= tail0;
                g2 *= tail0;
            }
        }
        // the frames' tile ranges (one thread per rank), and a clear per-frame pose table
        if (t < n_r) {
            unsigned long long m = mask;
            for (int q = 0; q < t; ++q) m &= m - 1;
            const int f = __builtin_ctzll(m);
            const int i0 = bx * CBX, i1 = min(a.cdim[0], i0 + CBX) - 1;
            const int j0 = by * CBY, j1 = min(a.cdim[1], j0 + CBY) - 1;
            const int k0 = bz * ZS, k1 = min(a.cdim[2], k0 + ZS) - 1;
            int tr[4] = {0, 0, 0, 0};
            const bool binned = a.rec_cap > 0 && brick_tiles(a.frames[f], i0, i1, j0, j1, k0, k1, tr);
            for (int q = 0; q < 4; ++q) s_tiles[t][q] = tr[q];
            s_cnt[t] = binned ? 0u : 0xFFFFFFFFu;   // marks a direct rank until the counts
        }
        if constexpr (POSE)
            for (int q = t; q < a.n_frames * 6; q += BWD_BLOCK) s_pose[q] = 0.0;
        // forward replay over the live frames, by rank among them: first the
        // weight-independent tests, four frames at a time with their image reads in flight
        // together (W or 0 into the history) ...
        const bool active = inside && (a.wc_out || g0 != 0.0f || g1 != 0.0f || g2 != 0.0f);
        unsigned long long upd = 0;   // bit r: rank r updates this voxel
        if (active) {
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
                    if (ok[q]) hist[(r + q) * BWD_BLOCK] = weight_test(frames[fr[q]], wf[q], fi, fj, fk);
                r += 4;
            }
            // ... then the gate against the running weight and alpha_n
            float Wc = a.wc0 ? a.wc0[idx] : 0.0f;
            r = 0;
            for (unsigned long long m = mask; m; m &= m - 1, ++r) {
                const float w = hist[r * BWD_BLOCK];
                float alpha = 0.0f;
                if (w > 0.0f && w > frames[__builtin_ctzll(m)].gate * Wc) {
                    alpha = w / (Wc + w);
                    Wc = fmaf(w, 1.0f - Wc, Wc);
                    upd |= 1ull << r;
                }
                hist[r * BWD_BLOCK] = alpha;
            }
            if (a.wc_out) a.wc_out[idx] = Wc;
        }
        if (a.wc_out) {
            __syncthreads();   // every thread has read the ticket
            continue;
        }
        __syncthreads();   // s_tiles, s_cnt (direct marks) and s_pose are set
        // records per wave and rank (direct ranks have none)
        for (int r = 0; r < n_r; ++r) {
            const unsigned long long b = __ballot((upd >> r) & 1ull);
            if (lane == 0) s_wcnt[wave][r] = s_cnt[r] == 0xFFFFFFFFu ? 0u : (uint32_t)__builtin_popcountll(b);
        }
        __syncthreads();
        // segments: per rank the waves' offsets and the count (wave 0, one lane per rank),
        // then one reservation for the brick's records
        if (wave == 0) {
            uint32_t cnt = 0;
            const bool direct = lane < n_r && s_cnt[lane] == 0xFFFFFFFFu;
            if (lane < n_r) {
                for (int w = 0; w < BWD_WAVES; ++w) {
                    const uint32_t c = s_wcnt[w][lane];
                    s_wcnt[w][lane] = cnt;
                    cnt += c;
                }
            }
            uint32_t incl = cnt;
#pragma unroll
            for (int off = 1; off < WAVE; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, WAVE);
                if (lane >= off) incl += y;
            }
            const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
            unsigned long long base = 0;
            if (lane == 0 && total > 0) base = atomicAdd(a.rec_next, (unsigned long long)total);
            base = __shfl(base, 0, WAVE);
            const bool fits = base + total <= (unsigned long long)a.rec_cap;
            if (lane < n_r) {
                s_seg[lane] = (uint32_t)base + incl - cnt;
                s_cnt[lane] = cnt;
            }
            const unsigned long long dm = __ballot(lane < n_r && (direct || !fits));
            if (lane == 0) s_direct = dm;
        }
        __syncthreads();
        const unsigned long long direct = s_direct;
        // reverse sweep over the ranks, all voxels of the brick together
        double xi[6] = {0, 0, 0, 0, 0, 0};
        float tail = 1.0f;
        unsigned long long m = mask;
        for (int r = n_r - 1; r >= 0; --r) {
            const int f = 63 - __builtin_clzll(m);
            m &= ~(1ull << f);
            const bool u = (upd >> r) & 1ull;
            const unsigned long long bal = __ballot(u);
            double pf[6] = {0, 0, 0, 0, 0, 0};   // this update's extrinsic terms (POSE)
            if (u) {
                const float alpha = hist[r * BWD_BLOCK];
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
                const int pix = (int)y0 * c.cw + (int)x0;
                const int cell = pix * 3;
                const int row = c.cw * 3;
                const float* img = (const float*)c.rgb;
                const float gb0 = g0 * beta, gb1 = g1 * beta, gb2 = g2 * beta;
                if ((direct >> r) & 1ull) {
                    float* dimg = a.d_rgb + (size_t)f * (size_t)c.cw * (size_t)c.ch * 3;
                    const float w00 = (1.0f - ax) * (1.0f - ay), w10 = ax * (1.0f - ay);
                    const float w01 = (1.0f - ax) * ay, w11 = ax * ay;
                    const float gv[3] = {gb0, gb1, gb2};
                    for (int ch = 0; ch < 3; ++ch) {
                        if (gv[ch] == 0.0f) continue;
                        unsafeAtomicAdd(dimg + cell + ch, gv[ch] * w00);
                        unsafeAtomicAdd(dimg + cell + 3 + ch, gv[ch] * w10);
                        unsafeAtomicAdd(dimg + cell + row + ch, gv[ch] * w01);
                        unsafeAtomicAdd(dimg + cell + row + 3 + ch, gv[ch] * w11);
                    }
                } else {
                    const size_t pos = (size_t)s_seg[r] + s_wcnt[wave][r] + lane_rank(bal);
                    float2* rec = (float2*)(a.records + pos * 6);
                    rec[0] = make_float2(__builtin_bit_cast(float, (uint32_t)(int)x0 | (uint32_t)(int)y0 << 16), ax);
                    rec[1] = make_float2(ay, gb0);
                    rec[2] = make_float2(gb1, gb2);
                }
                const float gvals[3] = {gb0, gb1, gb2};
                float gx = 0.0f, gy = 0.0f;   // sum_ch g beta ds/dx, ds/dy
                for (int ch = 0; ch < 3; ++ch) {
                    const float gb = gvals[ch];
                    if (gb == 0.0f) continue;
                    const float p00 = img[cell + ch], p10 = img[cell + 3 + ch];
                    const float p01 = img[cell + row + ch], p11 = img[cell + row + 3 + ch];
                    gx = fmaf(gb, (1.0f - ay) * (p10 - p00) + ay * (p11 - p01), gx);
                    gy = fmaf(gb, (1.0f - ax) * (p01 - p00) + ax * (p11 - p10), gy);
                }
                // pinhole Jacobian of Eq. 4 after the division by z
                const double dqx = (double)gx * c.fxr * iqz;
                const double dqy = (double)gy * c.fyr * iqz;
                const double dqz = -((double)gx * c.fxr * qx + (double)gy * c.fyr * qy) * iqz * iqz;
                const double p3 = (double)qy * dqz - (double)qz * dqy;
                const double p4 = (double)qz * dqx - (double)qx * dqz;
                const double p5 = (double)qx * dqy - (double)qy * dqx;
                xi[0] += dqx;
                xi[1] += dqy;
                xi[2] += dqz;
                xi[3] += p3;
                xi[4] += p4;
                xi[5] += p5;
                pf[0] = dqx;
                pf[1] = dqy;
                pf[2] = dqz;
                pf[3] = p3;
                pf[4] = p4;
                pf[5] = p5;
            }
            if constexpr (POSE) {
                // the frame's terms summed over the brick in a fixed order: a butterfly per
                // wave, then the waves in order (deterministic); the per-wave sums of
                // consecutive frames alternate between two tables, one barrier per frame
                double (*pw)[6] = s_pw[r & 1];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    const double sum = bal ? wave_sum_d(pf[q]) : 0.0;
                    if (lane == q) pw[wave][q] = sum;
                }
                __syncthreads();
                if (t < 6) {
                    double acc = 0.0;
                    for (int w = 0; w < BWD_WAVES; ++w) acc += pw[w][t];
                    s_pose[f * 6 + t] = acc;
                }
            }
        }
        if (a.tail_out && active) a.tail_out[idx] = tail0 * tail;
        // the brick's extrinsic partial: per wave a fixed butterfly, then the waves in order
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const double s = wave_sum_d(xi[q]);
            if (lane == q) s_xi[wave][q] = s;
        }
        __syncthreads();   // s_xi, s_pose complete; the history is free again
        if (t < 6) {
            double acc = 0.0;
            for (int w = 0; w < BWD_WAVES; ++w) acc += s_xi[w][t];
            a.partials[(size_t)li * 6 + t] = acc;
        }
        if constexpr (POSE) {
            // the brick's per-frame partials, one row per brick (indexed by the brick, so the
            // reduction order does not depend on scheduling)
            double* prow = a.pose_partials + (size_t)li * (size_t)a.n_frames * 6;
            for (int q = t; q < a.n_frames * 6; q += BWD_BLOCK) prow[q] = s_pose[q];
        }
        // the segments of the binned ranks, and their (frame, tile) counts
        if (t < n_r && !((direct >> t) & 1ull) && s_cnt[t] > 0) {
            unsigned long long mm = mask;
            for (int q = 0; q < t; ++q) mm &= mm - 1;
            const int f = __builtin_ctzll(mm);
            const uint4 sg = make_uint4(s_seg[t], s_cnt[t],
                                        (uint32_t)f | (uint32_t)s_tiles[t][2] << 8 | (uint32_t)s_tiles[t][3] << 9,
                                        (uint32_t)s_tiles[t][0] | (uint32_t)s_tiles[t][1] << 16);
            const uint32_t slot = atomicAdd(a.seg_next, 1u);
            a.segs[slot] = sg;
            const uint32_t n_tiles = (uint32_t)(a.tiles_x * a.tiles_y);
            for (int ty = s_tiles[t][1]; ty <= s_tiles[t][1] + s_tiles[t][3]; ++ty)
                for (int tx = s_tiles[t][0]; tx <= s_tiles[t][0] + s_tiles[t][2]; ++tx)
                    atomicAdd(a.bin_count + (size_t)f * n_tiles + (uint32_t)(ty * a.tiles_x + tx), 1u);
        }
        __syncthreads();   // LDS tables are reused by the next brick
    }
}

// Exclusive prefix sum of n counts in place (one block of 1024 threads; n + 1 entries, the
// last receiving the total).
__global__ __launch_bounds__(1024) void bin_scan_kernel(uint32_t* counts, uint32_t n)
{
    __shared__ uint32_t s[1024];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t b0 = min(n, t * per), b1 = min(n, b0 + per);
    uint32_t sum = 0;
    for (uint32_t q = b0; q < b1; ++q) sum += counts[q];
    s[t] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t y = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += y;
        __syncthreads();
    }
    uint32_t run = s[t] - sum;
    for (uint32_t q = b0; q < b1; ++q) {
        const uint32_t c = counts[q];
        counts[q] = run;
        run += c;
    }
    if (t == 1023) counts[n] = s[1023];
}

// Each segment's index into every (frame, tile) bin its range covers.
__global__ __launch_bounds__(256) void bin_fill_kernel(BackwardArgs a)
{
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= *a.seg_next) return;
    int f, tx0, tx1, ty0, ty1;
    segment_tiles(a.segs[s], &f, &tx0, &tx1, &ty0, &ty1);
    const uint32_t n_tiles = (uint32_t)(a.tiles_x * a.tiles_y);
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            const size_t bin = (size_t)f * n_tiles + (uint32_t)(ty * a.tiles_x + tx);
            const uint32_t p = atomicAdd(a.bin_fill + bin, 1u);
            a.bin_segs[a.bin_count[bin] + p] = s;
        }
}

// One block per (tile, frame): the records of the segments binned there, added in LDS
// over the tile's pixels (a record adds g beta times its four bilinear weights to the
// pixels of its cell that lie in the tile), then added to the image gradient.  Each wave
// takes whole segments in turn, its lanes reading consecutive records.
constexpr int IMG_BLOCK = 256;

__global__ __launch_bounds__(IMG_BLOCK) void backward_image_kernel(BackwardArgs a)
{
    __shared__ float s_acc[BWD_TILE_W * BWD_TILE_H * 3];
    const uint32_t n_tiles = (uint32_t)(a.tiles_x * a.tiles_y);
    const uint32_t tile = blockIdx.x, f = blockIdx.y;
    const size_t bin = (size_t)f * n_tiles + tile;
    const uint32_t b0 = a.bin_count[bin], b1 = a.bin_count[bin + 1];
    if (b0 == b1) return;   // the whole block
    const int t = threadIdx.x, lane = t & (WAVE - 1);
    const FrameConsts& c = a.frames[f];
    const int tx0 = (int)(tile % (uint32_t)a.tiles_x) * BWD_TILE_W;
    const int ty0 = (int)(tile / (uint32_t)a.tiles_x) * BWD_TILE_H;
    for (int q = t; q < BWD_TILE_W * BWD_TILE_H * 3; q += IMG_BLOCK) s_acc[q] = 0.0f;
    __syncthreads();
    for (uint32_t s = b0 + (uint32_t)(t / WAVE); s < b1; s += IMG_BLOCK / WAVE) {
        const uint4 sg = a.segs[first_lane_u32(a.bin_segs[s])];
        const uint32_t first = first_lane_u32(sg.x), cnt = first_lane_u32(sg.y);
        for (uint32_t r = (uint32_t)lane; r < cnt; r += WAVE) {
            const float2* rec = (const float2*)(a.records + ((size_t)first + r) * 6);
            const float2 r0 = rec[0], r1 = rec[1], r2 = rec[2];
            const uint32_t cell = __builtin_bit_cast(uint32_t, r0.x);   // x | y << 16
            const float ax = r0.y, ay = r1.x;
            const float gv[3] = {r1.y, r2.x, r2.y};
            const int x0 = (int)(cell & 0xFFFFu), y0 = (int)(cell >> 16);
            const float w[4] = {(1.0f - ax) * (1.0f - ay), ax * (1.0f - ay), (1.0f - ax) * ay, ax * ay};
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int lx = x0 + (p & 1) - tx0, ly = y0 + (p >> 1) - ty0;
                if (lx < 0 || lx >= BWD_TILE_W || ly < 0 || ly >= BWD_TILE_H) continue;
                float* acc = s_acc + (ly * BWD_TILE_W + lx) * 3;
                for (int ch = 0; ch < 3; ++ch)
                    if (gv[ch] != 0.0f) atomicAdd(acc + ch, gv[ch] * w[p]);
            }
        }
    }
    __syncthreads();
    float* dimg = a.d_rgb + (size_t)f * (size_t)c.cw * (size_t)c.ch * 3;
    for (int q = t; q < BWD_TILE_W * BWD_TILE_H * 3; q += IMG_BLOCK) {
        const float v = s_acc[q];
        if (v == 0.0f) continue;
        const int p = q / 3, ch = q - 3 * p;
        const int x = tx0 + p % BWD_TILE_W, y = ty0 + p / BWD_TILE_W;
        if (x < c.cw && y < c.ch) {
            float* d = dimg + ((size_t)y * (size_t)c.cw + (size_t)x) * 3 + ch;
            *d += v;
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

hipError_t launch_sum_rows(const double* rows, uint32_t n_rows, uint32_t width, double* out,
                           hipStream_t stream)
{
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(256), 0, stream, rows, n_rows, width,
                       n_rows, out);
    return hipGetLastError();
}

template <int HIST, bool POSE>
static hipError_t launch_backward_hist(const BackwardArgs& a, int device, hipStream_t stream)
{
    int n_cu = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, backward_kernel<HIST, POSE>, BWD_BLOCK, 0);
    if (e != hipSuccess) return e;
    const unsigned grid = (unsigned)(n_cu * (per_cu > 0 ? per_cu : 1));
    hipLaunchKernelGGL((backward_kernel<HIST, POSE>), dim3(grid), dim3(BWD_BLOCK), 0, stream, a);
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
        if (a.seg_cap > 0) {
            // sort the segments by (frame, tile) and add each tile's records
            const uint32_t n_bins = (uint32_t)a.n_frames * (uint32_t)(a.tiles_x * a.tiles_y);
            hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(1024), 0, stream, a.bin_count, n_bins);
            hipLaunchKernelGGL(bin_fill_kernel, dim3((a.seg_cap + 255) / 256), dim3(256), 0, stream, a);
            hipLaunchKernelGGL(backward_image_kernel,
                               dim3((unsigned)(a.tiles_x * a.tiles_y), (unsigned)a.n_frames),
                               dim3(IMG_BLOCK), 0, stream, a);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
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
