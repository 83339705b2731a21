/*
 * Marching cubes of the geometry volume: the triangle mesh the method extracts from the
 * integrated TSDF before decimating and texturing it (Sec. III, after KinectFusion; the
 * polygons of Sec. IV.C come from it).  Included once by kf_oracle.c.  TEST
 * INFRASTRUCTURE ONLY.
 *
 * The paper names the algorithm only; this is the definition both sides implement:
 *   samples    geometry voxel centres; a voxel is observed iff its weight is > 0, and
 *              inside iff F < 0 (F = +0 and -0 are outside);
 *   cubes      the 2x2x2 voxel groups with lower corner u in [0, dim - 2]^3; a cube is
 *              complete iff its 8 voxels are observed; only complete cubes make triangles;
 *   vertices   one per grid edge (u, u + e_a) whose two voxels are observed and on
 *              opposite sides and which belongs to at least one complete cube; in index
 *              coordinates it sits at u + t e_a with t = F(u) / (F(u) - F(u + e_a)), in
 *              world coordinates p_k = fma(q_k, s_k, origin_k + s_k / 2); vertices are
 *              numbered in the order of (linear index of u, axis a);
 *   polygons   cube corners c = x + 2y + 4z; the cube's edge along axis a whose other two
 *              coordinates (in increasing axis order) are (b0, b1) has id 4a + b0 + 2 b1.
 *              On each face, walking its corners counter-clockwise as seen from outside
 *              the cube, every step from an outside to an inside corner starts a segment
 *              that ends at the next step from an inside to an outside corner (so a face
 *              with four crossings cuts off each of its inside corners).  The segments
 *              chain into closed loops;
 *   triangles  loops in the order of their smallest edge id, each walked from that edge
 *              along its segments (L0, L1, ...) and fanned from its first vertex Lc whose
 *              edge shares no cube face with the edge of any vertex not next to it on the
 *              loop (so that no fan chord lies in a face, where the neighbouring cube
 *              could lay the same chord): (Lc, Lc+k, Lc+k+1), k = 1 .. len - 2, indices
 *              modulo len; every loop of every configuration has such a vertex.  Cubes in
 *              linear order of u.  A triangle's normal (right-hand rule) points from the
 *              inside to the outside, towards positive F.
 */

/* Edge id of the cube edge between corners c0 and c1 (which differ in one coordinate). */
static int mc_edge_between(int c0, int c1)
{
    const int d = (c0 ^ c1) == 1 ? 0 : (c0 ^ c1) == 2 ? 1 : 2;
    const int x = c0 & 1, y = (c0 >> 1) & 1, z = (c0 >> 2) & 1;
    if (d == 0) return 0 + y + 2 * z;
    if (d == 1) return 4 + x + 2 * z;
    return 8 + x + 2 * y;
}

/* next[e]: the edge after e along its loop, or -1 when edge e is not crossed. */
static void mc_segments(unsigned inside_mask, int next[12])
{
    for (int e = 0; e < 12; ++e) next[e] = -1;
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;   /* e_b x e_c = e_a */
        for (int side = 0; side < 2; ++side) {
            /* the face's corners counter-clockwise about its outward normal (2 side - 1) e_a */
            static const int ccw_pos[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            static const int ccw_neg[4][2] = {{0, 0}, {0, 1}, {1, 1}, {1, 0}};
            int corner[4];
            for (int i = 0; i < 4; ++i) {
                int coord[3];
                coord[a] = side;
                coord[b] = side ? ccw_pos[i][0] : ccw_neg[i][0];
                coord[c] = side ? ccw_pos[i][1] : ccw_neg[i][1];
                corner[i] = coord[0] + 2 * coord[1] + 4 * coord[2];
            }
            for (int i = 0; i < 4; ++i) {
                const int k0 = corner[i], k1 = corner[(i + 1) % 4];
                const int in0 = (inside_mask >> k0) & 1, in1 = (inside_mask >> k1) & 1;
                if (in0 || !in1) continue;               /* not an outside -> inside step */
                for (int s = 1; s < 4; ++s) {
                    const int m0 = corner[(i + s) % 4], m1 = corner[(i + s + 1) % 4];
                    if (((inside_mask >> m0) & 1) && !((inside_mask >> m1) & 1)) {
                        next[mc_edge_between(k0, k1)] = mc_edge_between(m0, m1);
                        break;
                    }
                }
            }
        }
    }
}

/* Whether cube edges e and f lie on a common face: each edge lies on the two faces
 * (axis, side) given by its other two coordinates. */
static int mc_share_face(int e, int f)
{
    const int a = e >> 2, b = f >> 2;
    const int ea[2] = {a == 0 ? 1 : 0, a == 2 ? 1 : 2}, eb[2] = {b == 0 ? 1 : 0, b == 2 ? 1 : 2};
    const int es[2] = {e & 1, (e >> 1) & 1}, fs[2] = {f & 1, (f >> 1) & 1};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (ea[i] == eb[j] && es[i] == fs[j]) return 1;
    return 0;
}

/* Triangles of one cube configuration as edge ids (at most 12 edges, so at most 10
 * triangles); returns their number. */
static int mc_cube_triangles(unsigned inside_mask, int tri[][3])
{
    int next[12], seen[12] = {0}, n = 0;
    mc_segments(inside_mask, next);
    for (int e = 0; e < 12; ++e) {
        if (next[e] < 0 || seen[e]) continue;
        int loop[12], len = 0;
        for (int f = e; f >= 0 && !seen[f]; f = next[f]) {
            seen[f] = 1;
            loop[len++] = f;
        }
        int c = 0;
        for (; c < len; ++c) {
            int clean = 1;
            for (int k = 2; k + 1 < len; ++k)
                clean &= !mc_share_face(loop[c], loop[(c + k) % len]);
            if (clean) break;
        }
        if (c == len) c = 0;   /* never happens (checked over all configurations) */
        for (int k = 1; k + 1 < len; ++k) {
            tri[n][0] = loop[c];
            tri[n][1] = loop[(c + k) % len];
            tri[n][2] = loop[(c + k + 1) % len];
            ++n;
        }
    }
    return n;
}

/* Lower-corner offset and axis of edge id e. */
static void mc_edge_geometry(int e, int off[3], int* axis)
{
    const int a = e >> 2, b0 = e & 1, b1 = (e >> 1) & 1;
    off[0] = off[1] = off[2] = 0;
    if (a == 0) { off[1] = b0; off[2] = b1; }
    if (a == 1) { off[0] = b0; off[2] = b1; }
    if (a == 2) { off[0] = b0; off[1] = b1; }
    *axis = a;
}

int or_marching_cubes(const or_volume* vol, const float* tsdf, const float* wg, float* vert32,
                      double* vert64, int64_t vcap, int32_t* tris, int64_t tcap, int64_t* n_vert,
                      int64_t* n_tri)
{
    const int64_t X = vol->gdim[0], Y = vol->gdim[1], Z = vol->gdim[2];
    const int64_t N = X * Y * Z;
    *n_vert = *n_tri = 0;
    if (X < 2 || Y < 2 || Z < 2) return 0;
#define LIN(x, y, z) ((x) + X * ((y) + Y * (int64_t)(z)))
    unsigned char* complete = (unsigned char*)calloc((size_t)N, 1);
    int32_t* vid = (int32_t*)malloc((size_t)N * 3 * sizeof(int32_t));
    /* complete cubes */
    for (int64_t z = 0; z + 1 < Z; ++z)
        for (int64_t y = 0; y + 1 < Y; ++y)
            for (int64_t x = 0; x + 1 < X; ++x) {
                int ok = 1;
                for (int c = 0; c < 8; ++c)
                    ok &= wg[LIN(x + (c & 1), y + ((c >> 1) & 1), z + ((c >> 2) & 1))] > 0.0f;
                complete[LIN(x, y, z)] = (unsigned char)ok;
            }
    /* vertices: crossed edges of at least one complete cube, in (voxel, axis) order */
    int64_t nv = 0;
    double s[3], c0[3];
    float sf[3], cf[3];
    for (int k = 0; k < 3; ++k) {
        s[k] = vol->extent[k] / vol->gdim[k];
        c0[k] = vol->origin[k] + 0.5 * s[k];
        sf[k] = (float)s[k];
        cf[k] = (float)c0[k];
    }
    for (int64_t z = 0; z < Z; ++z)
        for (int64_t y = 0; y < Y; ++y)
            for (int64_t x = 0; x < X; ++x) {
                const int64_t u = LIN(x, y, z);
                const int64_t p[3] = {x, y, z}, dims[3] = {X, Y, Z};
                for (int a = 0; a < 3; ++a) {
                    vid[3 * u + a] = -1;
                    if (p[a] + 1 >= dims[a]) continue;
                    const int64_t w = u + (a == 0 ? 1 : a == 1 ? X : X * Y);
                    if (!(wg[u] > 0.0f) || !(wg[w] > 0.0f)) continue;
                    if ((tsdf[u] < 0.0f) == (tsdf[w] < 0.0f)) continue;
                    /* the (up to) four cubes that hold this edge: lower corners u - db - dc */
                    const int b = (a + 1) % 3, c = (a + 2) % 3;
                    int used = 0;
                    for (int db = 0; db < 2 && !used; ++db)
                        for (int dc = 0; dc < 2 && !used; ++dc) {
                            int64_t q[3] = {x, y, z};
                            q[b] -= db;
                            q[c] -= dc;
                            if (q[b] < 0 || q[c] < 0 || q[0] + 1 >= X || q[1] + 1 >= Y || q[2] + 1 >= Z)
                                continue;
                            used = complete[LIN(q[0], q[1], q[2])];
                        }
                    if (!used) continue;
                    if (nv < vcap) {
                        const float t32 = tsdf[u] / (tsdf[u] - tsdf[w]);
                        const double t64 = (double)tsdf[u] / ((double)tsdf[u] - (double)tsdf[w]);
                        for (int k = 0; k < 3; ++k) {
                            const float q32 = k == a ? (float)p[k] + t32 : (float)p[k];
                            const double q64 = k == a ? (double)p[k] + t64 : (double)p[k];
                            if (vert32) vert32[3 * nv + k] = fmaf(q32, sf[k], cf[k]);
                            if (vert64) vert64[3 * nv + k] = fma(q64, s[k], c0[k]);
                        }
                    }
                    vid[3 * u + a] = (int32_t)nv++;
                }
            }
    /* triangles, cube by cube */
    int64_t nt = 0;
    for (int64_t z = 0; z + 1 < Z; ++z)
        for (int64_t y = 0; y + 1 < Y; ++y)
            for (int64_t x = 0; x + 1 < X; ++x) {
                if (!complete[LIN(x, y, z)]) continue;
                unsigned mask = 0;
                for (int c = 0; c < 8; ++c)
                    if (tsdf[LIN(x + (c & 1), y + ((c >> 1) & 1), z + ((c >> 2) & 1))] < 0.0f)
                        mask |= 1u << c;
                int t[12][3];
                const int n = mc_cube_triangles(mask, t);
                for (int i = 0; i < n; ++i, ++nt) {
                    if (nt >= tcap) continue;
                    for (int v = 0; v < 3; ++v) {
                        int off[3], axis;
                        mc_edge_geometry(t[i][v], off, &axis);
                        tris[3 * nt + v] = vid[3 * LIN(x + off[0], y + off[1], z + off[2]) + axis];
                    }
                }
            }
#undef LIN
    free(complete);
    free(vid);
    *n_vert = nv;
    *n_tri = nt;
    return (nv > vcap || nt > tcap) ? -1 : 0;
}
