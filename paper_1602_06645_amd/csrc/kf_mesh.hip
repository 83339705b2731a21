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
// (build_table).  Extraction is a stream compaction over voxels: classify the cubes and
// count each voxel's vertices and triangles (tiles in LDS), sum the counts per linear
// block, scan the block sums, then write vertices and triangles at their scanned offsets.
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

// Classification works on tiles of 32 x 8 x 8 voxels staged in LDS with a one-voxel
// halo; compaction works on linear blocks of 4096 voxels (16 per thread), so that the
// vertex and triangle order follows the linear voxel index.
constexpr int TX = 32, TY = 8, TZ = 8;
constexpr int BX = TX + 2, BY = TY + 2, BZ = TZ + 2;     // voxels: tile - 1 .. tile end + 1
constexpr int CX = TX + 1, CY = TY + 1, CZ = TZ + 1;     // cubes: lower corners tile - 1 .. tile end
constexpr int MC_THREADS = 256;
constexpr int LB = 4096, PER = LB / MC_THREADS;          // linear block, voxels per thread
static_assert(MC_THREADS == 256, "one thread per cube configuration when tables are staged");

// Per voxel of a tile: info = (axes whose edge from the voxel carries a vertex) |
// (triangles of the cube at the voxel) << 3.
__global__ __launch_bounds__(MC_THREADS) void mc_classify_kernel(MeshArgs a)
{
    // voxel codes: bit 0 observed, bit 1 inside; cube codes: bit 7 complete | triangles
    __shared__ uint8_t code[BZ * BY * BX];
    __shared__ uint8_t cube[CZ * CY * CX];
    __shared__ uint8_t count[256];                 // triangles per configuration
    count[threadIdx.x] = kMc.count[threadIdx.x];
    const int X = a.dim[0], Y = a.dim[1], Z = a.dim[2];
    const int ntx = (X + TX - 1) / TX, nty = (Y + TY - 1) / TY;
    const int t = (int)blockIdx.x;
    const int ox = (t % ntx) * TX - 1, oy = ((t / ntx) % nty) * TY - 1, oz = (t / (ntx * nty)) * TZ - 1;
    // the voxel box (voxels outside the volume are unobserved); every load of the thread is
    // issued before the first is used
    constexpr int NBOX = BX * BY * BZ, ITER = (NBOX + MC_THREADS - 1) / MC_THREADS;
    float fv[ITER], wv[ITER];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int i = (int)threadIdx.x + it * MC_THREADS;
        const int gx = ox + i % BX, gy = oy + (i / BX) % BY, gz = oz + i / (BX * BY);
        fv[it] = 0.0f;
        wv[it] = 0.0f;
        if (i < NBOX && gx >= 0 && gx < X && gy >= 0 && gy < Y && gz >= 0 && gz < Z) {
            const uint32_t v = (uint32_t)gx + (uint32_t)X * ((uint32_t)gy + (uint32_t)Y * (uint32_t)gz);
            fv[it] = a.tsdf[v];
            wv[it] = a.wg[v];
        }
    }
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int i = (int)threadIdx.x + it * MC_THREADS;
        if (i < NBOX) code[i] = (uint8_t)((wv[it] > 0.0f ? 1u : 0u) | (fv[it] < 0.0f ? 2u : 0u));
    }
    __syncthreads();
    // the cubes (one reaching outside the volume has an unobserved corner)
    for (int i = (int)threadIdx.x; i < CX * CY * CZ; i += MC_THREADS) {
        const int cx = i % CX, cy = (i / CX) % CY, cz = i / (CX * CY);
        const int b0 = cx + BX * (cy + BY * cz);
        uint32_t all = 1u, cfg = 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t k = code[b0 + (c & 1) + ((c >> 1) & 1) * BX + ((c >> 2) & 1) * BX * BY];
            all &= k;
            cfg |= ((k >> 1) & 1u) << c;
        }
        cube[i] = all ? (uint8_t)(0x80u | count[cfg]) : (uint8_t)0;
    }
    __syncthreads();
    // each thread: one (x, y) of the tile, all 8 z
    const int x = (int)threadIdx.x % TX, y = (int)threadIdx.x / TX;
    const int gx = ox + 1 + x, gy = oy + 1 + y;
    if (gx >= X || gy >= Y) return;
    const int bstep[3] = {1, BX, BX * BY}, cstep[3] = {1, CX, CX * CY};
    for (int z = 0; z < TZ; ++z) {
        const int gz = oz + 1 + z;
        if (gz >= Z) break;
        const int b = (x + 1) + BX * ((y + 1) + BY * (z + 1));
        const int c = (x + 1) + CX * ((y + 1) + CY * (z + 1));   // the cube at this voxel
        uint32_t info = (uint32_t)(cube[c] & 0x7Fu) << 3;
        const uint32_t vg = (uint32_t)gx + (uint32_t)X * ((uint32_t)gy + (uint32_t)Y * (uint32_t)gz);
        if (info) {
            // the configuration of a cube with triangles, for the triangle pass
            uint32_t cfg = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                cfg |= ((code[b + (k & 1) + ((k >> 1) & 1) * BX + ((k >> 2) & 1) * BX * BY] >> 1) & 1u) << k;
            a.cfg[vg] = (uint8_t)cfg;
        }
        const uint32_t k0 = code[b];
        if (k0 & 1u) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const uint32_t k1 = code[b + bstep[ax]];
                if (!(k1 & 1u) || ((k0 ^ k1) & 2u) == 0) continue;
                // the four cubes holding the edge: lower corners v - db e_p - dc e_q
                const int p = (ax + 1) % 3, q = (ax + 2) % 3;
                const uint32_t used = cube[c] | cube[c - cstep[p]] | cube[c - cstep[q]] |
                                      cube[c - cstep[p] - cstep[q]];
                if (used & 0x80u) info |= 1u << ax;
            }
        }
        a.info[vg] = (uint8_t)info;
    }
}

__device__ __forceinline__ uint32_t vertices_of(uint32_t info) { return (uint32_t)__builtin_popcount(info & 7u); }
__device__ __forceinline__ uint32_t triangles_of(uint32_t info) { return info >> 3; }

// The 16 info bytes of this thread's voxels in linear block b (zero past the volume).
__device__ __forceinline__ void load_run(const MeshArgs& a, uint32_t b, uint8_t* run)
{
    const uint32_t v0 = b * LB + threadIdx.x * PER;
    if (v0 + PER <= a.n_voxels) {
        uint4 w;
        __builtin_memcpy(&w, a.info + v0, 16);
        __builtin_memcpy(run, &w, 16);
    } else {
#pragma unroll
        for (int k = 0; k < PER; ++k) run[k] = v0 + k < a.n_voxels ? a.info[v0 + k] : 0;
    }
}

// Inclusive scan over the workgroup of one value per thread (thread order).
__device__ __forceinline__ uint32_t block_inclusive(uint32_t x, uint32_t* lds)
{
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += lds[w];
    __syncthreads();
    return base + x;
}

// Per linear block: total vertices and triangles.
__global__ __launch_bounds__(MC_THREADS) void mc_block_sums_kernel(MeshArgs a)
{
    __shared__ uint32_t lds[MC_THREADS / 64];
    uint8_t run[PER];
    load_run(a, blockIdx.x, run);
    uint32_t nv = 0, nt = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        nv += vertices_of(run[k]);
        nt += triangles_of(run[k]);
    }
    // pack both sums (each below 2^16 per block: 3 and 5 per voxel, 4096 voxels)
    const uint32_t tot = block_inclusive(nv | (nt << 16), lds);
    if (threadIdx.x == MC_THREADS - 1) {
        a.block_sums[2 * blockIdx.x] = tot & 0xFFFFu;
        a.block_sums[2 * blockIdx.x + 1] = tot >> 16;
    }
}

// One workgroup: exclusive scan of the block sums in place, and the totals.
__global__ __launch_bounds__(1024) void mc_scan_blocks_kernel(MeshArgs a)
{
    __shared__ uint32_t lds[2][1024 / 64];
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    uint32_t carry_v = 0, carry_t = 0;
    for (uint32_t base = 0; base < a.n_blocks; base += 1024) {
        const uint32_t b = base + threadIdx.x;
        uint32_t v = b < a.n_blocks ? a.block_sums[2 * b] : 0u;
        uint32_t t = b < a.n_blocks ? a.block_sums[2 * b + 1] : 0u;
        uint32_t iv = v, it = t;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t yv = __shfl_up(iv, o), yt = __shfl_up(it, o);
            if (lane >= o) {
                iv += yv;
                it += yt;
            }
        }
        if (lane == 63) {
            lds[0][wave] = iv;
            lds[1][wave] = it;
        }
        __syncthreads();
        uint32_t pv = carry_v, pt = carry_t;
        for (int w = 0; w < wave; ++w) {
            pv += lds[0][w];
            pt += lds[1][w];
        }
        uint32_t sum_v = 0, sum_t = 0;
        for (int w = 0; w < 1024 / 64; ++w) {
            sum_v += lds[0][w];
            sum_t += lds[1][w];
        }
        __syncthreads();
        if (b < a.n_blocks) {
            a.block_sums[2 * b] = pv + iv - v;
            a.block_sums[2 * b + 1] = pt + it - t;
        }
        carry_v += sum_v;
        carry_t += sum_t;
    }
    if (threadIdx.x == 0) {
        a.totals[0] = carry_v;
        a.totals[1] = carry_t;
    }
}

// The voxels of this thread's run that have outputs (count(info) > 0), gathered for the
// workgroup in voxel order: list[i] = (voxel offset in the block) | (first output slot
// relative to the block's first, << 12).  Returns the list length.
template <class Count>
__device__ __forceinline__ uint32_t gather_active(const uint8_t* run, Count count, uint32_t* list,
                                                  uint32_t* lds)
{
    uint32_t n = 0, m = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t c = count(run[k]);
        n += c;
        m += c ? 1u : 0u;
    }
    // both prefixes in one scan (outputs below 2^15, active voxels below 2^13 per block)
    const uint32_t incl = block_inclusive(n | (m << 16), lds);
    uint32_t slot = (incl & 0xFFFFu) - n;
    uint32_t pos = (incl >> 16) - m;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t c = count(run[k]);
        if (c) {
            list[pos++] = (threadIdx.x * PER + k) | (slot << 12);
            slot += c;
        }
    }
    if (threadIdx.x == MC_THREADS - 1) lds[0] = incl >> 16;
    __syncthreads();
    return lds[0];
}

// Vertices at their scanned slots (those below the capacity); each vertex-owning voxel's
// first vertex index.
__global__ __launch_bounds__(MC_THREADS) void mc_vertices_kernel(MeshArgs a)
{
    __shared__ uint32_t lds[MC_THREADS / 64];
    __shared__ uint32_t list[LB];
    uint8_t run[PER];
    load_run(a, blockIdx.x, run);
    const uint32_t n_active = gather_active(run, [](uint32_t i) { return vertices_of(i); }, list, lds);
    const uint32_t base = a.block_sums[2 * blockIdx.x];
    const uint32_t X = (uint32_t)a.dim[0], Y = (uint32_t)a.dim[1];
    const uint32_t step[3] = {1u, X, X * Y};
    for (uint32_t e = threadIdx.x; e < n_active; e += MC_THREADS) {
        const uint32_t v = blockIdx.x * LB + (list[e] & 0xFFFu);
        uint32_t slot = base + (list[e] >> 12);
        const uint32_t mask = a.info[v] & 7u;
        a.voff[v] = slot;
        const uint32_t xyz[3] = {v % X, (v / X) % Y, v / (X * Y)};
        const float f0 = a.tsdf[v];
        for (int ax = 0; ax < 3; ++ax) {
            if (!((mask >> ax) & 1)) continue;
            if (slot < a.vcap) {
                const float t = f0 / (f0 - a.tsdf[v + step[ax]]);
                float* out = a.vertices + 3 * (size_t)slot;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float q = j == ax ? (float)xyz[j] + t : (float)xyz[j];
                    out[j] = fmaf(q, a.s[j], a.c[j]);
                }
            }
            ++slot;
        }
    }
}

// Triangles at their scanned slots (those below the capacity), corners as vertex indices.
__global__ __launch_bounds__(MC_THREADS) void mc_triangles_kernel(MeshArgs a)
{
    __shared__ uint32_t lds[MC_THREADS / 64];
    __shared__ uint32_t list[LB];
    __shared__ uint8_t table[256 * 15];            // the cube table's triangle edges
    for (int i = (int)threadIdx.x; i < 256 * 15; i += MC_THREADS) table[i] = kMc.edge[i / 15][i % 15];
    uint8_t run[PER];
    load_run(a, blockIdx.x, run);
    const uint32_t n_active = gather_active(run, [](uint32_t i) { return triangles_of(i); }, list, lds);
    const uint32_t base = a.block_sums[2 * blockIdx.x + 1];
    const uint32_t X = (uint32_t)a.dim[0], XY = (uint32_t)a.dim[0] * (uint32_t)a.dim[1];
    for (uint32_t e = threadIdx.x; e < n_active; e += MC_THREADS) {
        const uint32_t v = blockIdx.x * LB + (list[e] & 0xFFFu);
        uint32_t slot = base + (list[e] >> 12);
        const uint32_t nt = triangles_of(a.info[v]);
        const uint32_t cfg = a.cfg[v];
        for (uint32_t i = 0; i < nt; ++i, ++slot) {
            if (slot >= a.tcap) continue;
            int32_t* out = a.triangles + 3 * (size_t)slot;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int ed = table[15 * cfg + 3 * i + j];
                const int ax = ed >> 2, lo = ed & 1, hi = (ed >> 1) & 1;
                // the edge's lower end: the cube corner offset by (lo, hi) on the other axes
                const uint32_t ox = ax == 0 ? 0u : (uint32_t)lo;
                const uint32_t oy = ax == 0 ? (uint32_t)lo : ax == 1 ? 0u : (uint32_t)hi;
                const uint32_t oz = ax == 2 ? 0u : (uint32_t)hi;
                const uint32_t owner = v + ox + oy * X + oz * XY;
                const uint32_t below = a.info[owner] & ((1u << ax) - 1u);
                out[j] = (int32_t)(a.voff[owner] + (uint32_t)__builtin_popcount(below));
            }
        }
    }
}

}  // namespace

hipError_t launch_mesh_count(const MeshArgs& a, hipStream_t stream)
{
    const uint32_t tiles = (uint32_t)(((a.dim[0] + TX - 1) / TX) * ((a.dim[1] + TY - 1) / TY) *
                                      ((a.dim[2] + TZ - 1) / TZ));
    hipLaunchKernelGGL(mc_classify_kernel, dim3(tiles), dim3(MC_THREADS), 0, stream, a);
    hipLaunchKernelGGL(mc_block_sums_kernel, dim3(a.n_blocks), dim3(MC_THREADS), 0, stream, a);
    hipLaunchKernelGGL(mc_scan_blocks_kernel, dim3(1), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_mesh_emit(const MeshArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(mc_vertices_kernel, dim3(a.n_blocks), dim3(MC_THREADS), 0, stream, a);
    hipLaunchKernelGGL(mc_triangles_kernel, dim3(a.n_blocks), dim3(MC_THREADS), 0, stream, a);
    return hipGetLastError();
}

}  // namespace kf
