// Marching cubes of the geometry volume for gfx950: the triangle mesh extracted from the
// integrated TSDF (Sec. III, after KinectFusion), which the method decimates and textures
// per polygon (Sec. IV.C).  The mesh is defined by:
//   - a voxel is observed iff its weight is > 0, inside iff F < 0 (+0 and -0 are outside);
//   - cubes are the 2x2x2 voxel groups with lower corner u in [0, dim - 2]^3; only cubes
//     with 8 observed voxels ("complete") make triangles;
//   - one vertex per grid edge (u, u + e_a) with observed ends on opposite sides that
//     belongs to a complete cube, at index position u + t e_a, t = F(u) / (F(u) - F(u +
//     e_a)), world p = fma(q, s, origin + s/2); vertices numbered by (linear u, axis);
//   - per cube: on each face, walking its corners counter-clockwise seen from outside the
//     cube, a step from an outside to an inside corner starts a segment that ends at the
//     next step from an inside to an outside corner; the segments close into loops; loops
//     in order of their smallest edge id, each walked from that edge and fanned from its
//     first vertex whose edge shares no face with a non-neighbouring vertex's edge;
//     triangles face towards positive F; cubes in linear order.
// The per-configuration triangles are generated at compile time from that rule
// (build_table).  Extraction is a stream compaction over voxels: classify the cubes,
// count each voxel's vertices and triangles, scan the counts (per block, then over the
// blocks), then write vertices and triangles at their scanned offsets.
#include <hip/hip_runtime.h>

#include "kf_device.h"
#include "kf_launch.h"

namespace kf {

namespace {

// ------------------------------------------------------------------ the cube table

struct McTable {
    uint8_t count[256];        // triangles per configuration (at most 5)
    uint8_t edge[256][15];     // their corners as cube edge ids
};

// Id of the edge from corner c (whose bit `axis` is clear) along `axis`: 4 axis + the
// corner's two other coordinates, the lower axis as bit 0.
constexpr int edge_from(int c, int axis)
{
    const int lo = axis == 0 ? (c >> 1) & 1 : c & 1;
    const int hi = axis == 2 ? (c >> 1) & 1 : (c >> 2) & 1;
    return 4 * axis + lo + 2 * hi;
}

// The two faces an edge lies on, as bits 2 axis + side.
constexpr unsigned edge_faces(int e)
{
    const int axis = e >> 2, lo = e & 1, hi = (e >> 1) & 1;
    const int pa = axis == 0 ? 1 : 0, qa = axis == 2 ? 1 : 2;   // the other axes, ascending
    return (1u << (2 * pa + lo)) | (1u << (2 * qa + hi));
}

constexpr McTable build_table()
{
    McTable t{};
    // the four corners of each face counter-clockwise about its outward normal, found by
    // the sign of the cross product of the corners' offsets from the face centre
    int ring[6][4] = {};
    for (int axis = 0; axis < 3; ++axis)
        for (int side = 0; side < 2; ++side) {
            const int p = (axis + 1) % 3, q = (axis + 2) % 3;       // e_p x e_q = e_axis
            const int sgn = side ? 1 : -1;
            int cur = side << axis;                                  // lowest corner of the face
            for (int i = 0; i < 4; ++i) {
                ring[2 * axis + side][i] = cur;
                for (int nb = 0; nb < 8; ++nb) {
                    if (((nb >> axis) & 1) != side) continue;
                    const int diff = nb ^ cur;
                    if (diff != (1 << p) && diff != (1 << q)) continue;   // not adjacent
                    const int dcp = 2 * ((cur >> p) & 1) - 1, dcq = 2 * ((cur >> q) & 1) - 1;
                    const int dnp = 2 * ((nb >> p) & 1) - 1, dnq = 2 * ((nb >> q) & 1) - 1;
                    if (sgn * (dcp * dnq - dcq * dnp) > 0) {
                        cur = nb;
                        break;
                    }
                }
            }
        }
    for (int cfg = 0; cfg < 256; ++cfg) {
        int next[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
        for (int f = 0; f < 6; ++f)
            for (int i = 0; i < 4; ++i) {
                const int a = ring[f][i], b = ring[f][(i + 1) & 3];
                if (((cfg >> a) & 1) || !((cfg >> b) & 1)) continue;     // outside -> inside
                for (int j = 1; j < 4; ++j) {
                    const int c = ring[f][(i + j) & 3], d = ring[f][(i + j + 1) & 3];
                    if (((cfg >> c) & 1) && !((cfg >> d) & 1)) {         // inside -> outside
                        const int ax_ab = (a ^ b) == 1 ? 0 : (a ^ b) == 2 ? 1 : 2;
                        const int ax_cd = (c ^ d) == 1 ? 0 : (c ^ d) == 2 ? 1 : 2;
                        next[edge_from(a < b ? a : b, ax_ab)] = edge_from(c < d ? c : d, ax_cd);
                        break;
                    }
                }
            }
        int n = 0;
        bool used[12] = {};
        for (int start = 0; start < 12; ++start) {
            if (next[start] < 0 || used[start]) continue;
            int loop[12] = {}, len = 0;
            for (int e = start; e >= 0 && !used[e]; e = next[e]) {
                used[e] = true;
                loop[len++] = e;
            }
            int centre = 0;
            for (int c = 0; c < len; ++c) {
                bool clean = true;
                for (int k = 2; k + 1 < len; ++k)
                    if (edge_faces(loop[c]) & edge_faces(loop[(c + k) % len])) clean = false;
                if (clean) {
                    centre = c;
                    break;
                }
            }
            for (int k = 1; k + 1 < len && n < 5; ++k, ++n) {
                t.edge[cfg][3 * n + 0] = (uint8_t)loop[centre];
                t.edge[cfg][3 * n + 1] = (uint8_t)loop[(centre + k) % len];
                t.edge[cfg][3 * n + 2] = (uint8_t)loop[(centre + k + 1) % len];
            }
        }
        t.count[cfg] = (uint8_t)n;
    }
    return t;
}

__constant__ McTable kMc = build_table();

constexpr int MC_BLOCK = 256;

// Per voxel (cube with lower corner u): bit 8 = complete, bits 0-7 = inside corners.
__global__ __launch_bounds__(MC_BLOCK) void mc_classify_kernel(MeshArgs a)
{
    const uint32_t v = blockIdx.x * MC_BLOCK + threadIdx.x;
    if (v >= a.n_voxels) return;
    const uint32_t X = (uint32_t)a.dim[0], Y = (uint32_t)a.dim[1], Z = (uint32_t)a.dim[2];
    const uint32_t x = v % X, y = (v / X) % Y, z = v / (X * Y);
    uint16_t info = 0;
    if (x + 1 < X && y + 1 < Y && z + 1 < Z) {
        bool complete = true;
        uint32_t cfg = 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t i = v + (c & 1) + ((c >> 1) & 1) * X + ((c >> 2) & 1) * X * Y;
            complete &= a.wg[i] > 0.0f;
            cfg |= (a.tsdf[i] < 0.0f ? 1u : 0u) << c;
        }
        info = complete ? (uint16_t)(0x100u | cfg) : 0;
    }
    a.cube[v] = info;
}

// Per voxel: bits 0-2 = axes whose edge from the voxel carries a vertex, bits 3-5 = the
// voxel's cube's triangle count; per block: the sums of vertices and triangles.
__global__ __launch_bounds__(MC_BLOCK) void mc_count_kernel(MeshArgs a)
{
    __shared__ uint32_t red[2][MC_BLOCK / 64];
    const uint32_t v = blockIdx.x * MC_BLOCK + threadIdx.x;
    uint32_t nv = 0, nt = 0;
    if (v < a.n_voxels) {
        const uint32_t X = (uint32_t)a.dim[0], Y = (uint32_t)a.dim[1], Z = (uint32_t)a.dim[2];
        const uint32_t xyz[3] = {v % X, (v / X) % Y, v / (X * Y)};
        const uint32_t dims[3] = {X, Y, Z};
        const uint32_t step[3] = {1u, X, X * Y};
        const uint16_t own = a.cube[v];
        nt = (own & 0x100u) ? kMc.count[own & 0xFFu] : 0u;
        const float f0 = a.tsdf[v];
        const bool obs0 = a.wg[v] > 0.0f;
        uint32_t mask = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (!obs0 || xyz[ax] + 1 >= dims[ax]) continue;
            const uint32_t w = v + step[ax];
            if (!(a.wg[w] > 0.0f) || ((f0 < 0.0f) == (a.tsdf[w] < 0.0f))) continue;
            // the four cubes holding the edge have lower corners v - db e_b - dc e_c
            const int b = (ax + 1) % 3, c = (ax + 2) % 3;
            bool used = false;
#pragma unroll
            for (int db = 0; db < 2; ++db)
#pragma unroll
                for (int dc = 0; dc < 2; ++dc) {
                    if ((db && xyz[b] == 0) || (dc && xyz[c] == 0)) continue;
                    used |= (a.cube[v - db * step[b] - dc * step[c]] & 0x100u) != 0;
                }
            if (used) mask |= 1u << ax;
        }
        nv = (uint32_t)__builtin_popcount(mask);
        a.info[v] = (uint8_t)(mask | (nt << 3));
    }
    // block sums
    for (int o = 32; o > 0; o >>= 1) {
        nv += __shfl_xor(nv, o);
        nt += __shfl_xor(nt, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = nv;
        red[1][threadIdx.x >> 6] = nt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sv = 0, st = 0;
        for (int w = 0; w < MC_BLOCK / 64; ++w) {
            sv += red[0][w];
            st += red[1][w];
        }
        a.block_sums[2 * blockIdx.x] = sv;
        a.block_sums[2 * blockIdx.x + 1] = st;
    }
}

// One workgroup: exclusive scan of the per-block sums (in place) and the totals.
__global__ __launch_bounds__(1024) void mc_scan_blocks_kernel(MeshArgs a)
{
    __shared__ uint32_t part[2][1024];
    const uint32_t nb = a.n_blocks, per = (nb + 1023) / 1024;
    const uint32_t b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    uint32_t sv = 0, st = 0;
    for (uint32_t b = b0; b < b1; ++b) {
        sv += a.block_sums[2 * b];
        st += a.block_sums[2 * b + 1];
    }
    part[0][threadIdx.x] = sv;
    part[1][threadIdx.x] = st;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 1024 partial sums
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t pv = threadIdx.x >= (unsigned)o ? part[0][threadIdx.x - o] : 0u;
        const uint32_t pt = threadIdx.x >= (unsigned)o ? part[1][threadIdx.x - o] : 0u;
        __syncthreads();
        part[0][threadIdx.x] += pv;
        part[1][threadIdx.x] += pt;
        __syncthreads();
    }
    uint32_t ov = part[0][threadIdx.x] - sv, ot = part[1][threadIdx.x] - st;
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t cv = a.block_sums[2 * b], ct = a.block_sums[2 * b + 1];
        a.block_sums[2 * b] = ov;
        a.block_sums[2 * b + 1] = ot;
        ov += cv;
        ot += ct;
    }
    if (threadIdx.x == 1023) {
        a.totals[0] = part[0][1023];
        a.totals[1] = part[1][1023];
    }
}

// Exclusive prefix of `val` over the workgroup (in voxel order) plus the block offset.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t val, uint32_t* lds)
{
    lds[threadIdx.x] = val;
    __syncthreads();
    for (int o = 1; o < MC_BLOCK; o <<= 1) {
        const uint32_t p = threadIdx.x >= (unsigned)o ? lds[threadIdx.x - o] : 0u;
        __syncthreads();
        lds[threadIdx.x] += p;
        __syncthreads();
    }
    const uint32_t incl = lds[threadIdx.x];
    __syncthreads();
    return incl - val;
}

// Vertices: positions at their scanned slots, and each voxel's first vertex index.
__global__ __launch_bounds__(MC_BLOCK) void mc_vertices_kernel(MeshArgs a)
{
    __shared__ uint32_t lds[MC_BLOCK];
    const uint32_t v = blockIdx.x * MC_BLOCK + threadIdx.x;
    const uint32_t mask = v < a.n_voxels ? (a.info[v] & 7u) : 0u;
    const uint32_t first = a.block_sums[2 * blockIdx.x] +
                           block_exclusive((uint32_t)__builtin_popcount(mask), lds);
    if (v >= a.n_voxels) return;
    a.voff[v] = first;
    if (!mask) return;
    const uint32_t X = (uint32_t)a.dim[0], Y = (uint32_t)a.dim[1];
    const uint32_t xyz[3] = {v % X, (v / X) % Y, v / (X * Y)};
    const uint32_t step[3] = {1u, X, X * Y};
    const float f0 = a.tsdf[v];
    uint32_t slot = first;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (!((mask >> ax) & 1)) continue;
        const float t = f0 / (f0 - a.tsdf[v + step[ax]]);
        float* out = a.vertices + 3 * (size_t)slot;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float q = k == ax ? (float)xyz[k] + t : (float)xyz[k];
            out[k] = fmaf(q, a.s[k], a.c[k]);
        }
        ++slot;
    }
}

// Triangles at their scanned slots, corners as vertex indices.
__global__ __launch_bounds__(MC_BLOCK) void mc_triangles_kernel(MeshArgs a)
{
    __shared__ uint32_t lds[MC_BLOCK];
    const uint32_t v = blockIdx.x * MC_BLOCK + threadIdx.x;
    const uint32_t nt = v < a.n_voxels ? (uint32_t)(a.info[v] >> 3) : 0u;
    const uint32_t first = a.block_sums[2 * blockIdx.x + 1] + block_exclusive(nt, lds);
    if (v >= a.n_voxels || nt == 0) return;
    const uint32_t X = (uint32_t)a.dim[0], Y = (uint32_t)a.dim[1];
    const uint32_t cfg = a.cube[v] & 0xFFu;
    for (uint32_t i = 0; i < nt; ++i) {
        int32_t* out = a.triangles + 3 * (size_t)(first + i);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int e = kMc.edge[cfg][3 * i + k];
            const int ax = e >> 2, lo = e & 1, hi = (e >> 1) & 1;
            // the edge's lower end: the cube corner offset by (lo, hi) on the other axes
            const uint32_t ox = ax == 0 ? 0u : (uint32_t)lo;
            const uint32_t oy = ax == 0 ? (uint32_t)lo : ax == 1 ? 0u : (uint32_t)hi;
            const uint32_t oz = ax == 2 ? 0u : (uint32_t)hi;
            const uint32_t owner = v + ox + oy * X + oz * X * Y;
            const uint32_t below = a.info[owner] & ((1u << ax) - 1u);
            out[k] = (int32_t)(a.voff[owner] + (uint32_t)__builtin_popcount(below));
        }
    }
}

}  // namespace

hipError_t launch_mesh_count(const MeshArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(mc_classify_kernel, dim3(a.n_blocks), dim3(MC_BLOCK), 0, stream, a);
    hipLaunchKernelGGL(mc_count_kernel, dim3(a.n_blocks), dim3(MC_BLOCK), 0, stream, a);
    hipLaunchKernelGGL(mc_scan_blocks_kernel, dim3(1), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_mesh_emit(const MeshArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(mc_vertices_kernel, dim3(a.n_blocks), dim3(MC_BLOCK), 0, stream, a);
    hipLaunchKernelGGL(mc_triangles_kernel, dim3(a.n_blocks), dim3(MC_BLOCK), 0, stream, a);
    return hipGetLastError();
}

}  // namespace kf
