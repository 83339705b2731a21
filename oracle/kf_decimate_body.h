/* Quadric-error mesh decimation (Sec. IV.C: the dense marching-cubes mesh is simplified by
 * the quadric-based decimation of Garland and Heckbert down to a reduction rate, the
 * fraction of the polygons that remain).  Plain reference: every step takes the cheapest
 * edge by a linear scan over all edges.  Included by kf_oracle.c.
 *
 * The method, as read here:
 *   - each triangle's plane (unit normal u, offset d = -u.v0) gives the fundamental
 *     quadric K = [u d][u d]^T (the squared distance to the plane); a vertex's quadric is
 *     the sum of its triangles' (in triangle order), then, for every boundary edge (used
 *     by one triangle) in triangle order and edge slot order, the quadric of the plane
 *     through the edge perpendicular to its triangle, weighted by 1000, added to both
 *     ends;
 *   - an edge (a, b), a < b, would be contracted to the minimiser of v^T (Q_a + Q_b) v
 *     when the 3x3 part of the quadric is well conditioned (|det| > 1e-10 trace^3), else
 *     to the cheapest of a, b and their midpoint; its cost is the quadric at that point;
 *   - repeatedly, the edge of least (cost, a, b) that is not blocked is tested: it may be
 *     contracted when the common neighbours of a and b are exactly the opposite vertices
 *     of its triangles, the two ends are not both on the boundary unless the edge is, it
 *     is not the edge of a tetrahedron (both {a, c, d} and {b, c, d} present), and no
 *     remaining triangle of a or b turns over (its normal's dot product with the old one
 *     stays positive).  A failing edge is blocked; contracting (a, b) moves a to the
 *     point, adds b's quadric to a's, removes the triangles of the edge, gives b's other
 *     triangles to a, recomputes the costs of a's edges and unblocks every edge at a or at
 *     a neighbour of a;
 *   - it stops when at most round(rate * triangles) triangles remain (or no edge can be
 *     contracted); the output keeps the surviving triangles in input order (orientation
 *     unchanged) and the vertices they use in input order, as float.
 * All arithmetic in double, in the order written.  No blocking, heap or reordering beyond
 * that: the product's implementation must give the same mesh.
 */
#define DEC_BOUNDARY_WEIGHT 1000.0
#define DEC_DET_EPS 1e-10

typedef struct {
    int32_t* v;
    int32_t n, cap;
} dec_list;

static void dec_push(dec_list* l, int32_t x)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 8;
        l->v = (int32_t*)realloc(l->v, (size_t)l->cap * sizeof(int32_t));
    }
    l->v[l->n++] = x;
}

static void dec_remove(dec_list* l, int32_t x)
{
    for (int32_t i = 0; i < l->n; ++i)
        if (l->v[i] == x) {
            memmove(l->v + i, l->v + i + 1, (size_t)(l->n - i - 1) * sizeof(int32_t));
            --l->n;
            return;
        }
}

typedef struct {
    int32_t a, b;        /* a < b */
    int alive, blocked;
    double cost, p[3];
} dec_edge;

typedef struct {
    int64_t nv, nt;
    double (*pos)[3];
    double (*Q)[10];
    int32_t (*tri)[3];
    char* tri_alive;
    char* v_alive;
    dec_list* vt;        /* triangles of each vertex */
    dec_edge* e;
    int64_t ne, ecap;
    int64_t* hkey;       /* open-addressing table: edge key -> index */
    int64_t* hval;
    int64_t hcap;
    int64_t live_tri;
} dec_mesh;

static int64_t dec_key(int32_t a, int32_t b) { return ((int64_t)a << 32) | (uint32_t)b; }

static uint64_t dec_hash(int64_t k)
{
    uint64_t x = (uint64_t)k;
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    return x;
}

static int64_t dec_find(dec_mesh* m, int32_t a, int32_t b)
{
    const int64_t k = dec_key(a, b);
    for (uint64_t h = dec_hash(k) & (uint64_t)(m->hcap - 1);; h = (h + 1) & (uint64_t)(m->hcap - 1)) {
        if (m->hkey[h] == -1) return -1;
        if (m->hkey[h] == k) return m->hval[h];
    }
}

static void dec_insert_key(dec_mesh* m, int64_t k, int64_t idx)
{
    for (uint64_t h = dec_hash(k) & (uint64_t)(m->hcap - 1);; h = (h + 1) & (uint64_t)(m->hcap - 1))
        if (m->hkey[h] == -1 || m->hkey[h] == k) {
            m->hkey[h] = k;
            m->hval[h] = idx;
            return;
        }
}

/* Quadric of the plane (u, d) with weight w, added to q. */
static void dec_add_plane(double* q, const double u[3], double d, double w)
{
    q[0] += w * (u[0] * u[0]);
    q[1] += w * (u[0] * u[1]);
    q[2] += w * (u[0] * u[2]);
    q[3] += w * (u[0] * d);
    q[4] += w * (u[1] * u[1]);
    q[5] += w * (u[1] * u[2]);
    q[6] += w * (u[1] * d);
    q[7] += w * (u[2] * u[2]);
    q[8] += w * (u[2] * d);
    q[9] += w * (d * d);
}

static double dec_eval(const double* q, const double* v)
{
    const double x = v[0], y = v[1], z = v[2];
    return q[0] * x * x + 2.0 * q[1] * x * y + 2.0 * q[2] * x * z + 2.0 * q[3] * x
           + q[4] * y * y + 2.0 * q[5] * y * z + 2.0 * q[6] * y + q[7] * z * z
           + 2.0 * q[8] * z + q[9];
}

static void dec_cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* Unnormalised normal of a triangle whose vertex slot `slot` sits at `p` instead. */
static void dec_tri_normal(const dec_mesh* m, int64_t t, int slot, const double* p, double n[3])
{
    const double* v[3];
    for (int k = 0; k < 3; ++k) v[k] = (k == slot && p) ? p : m->pos[m->tri[t][k]];
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = v[1][k] - v[0][k];
        e2[k] = v[2][k] - v[0][k];
    }
    dec_cross(e1, e2, n);
}

/* Contraction point and cost of edge (a, b). */
static void dec_edge_cost(const dec_mesh* m, dec_edge* e)
{
    double q[10];
    for (int k = 0; k < 10; ++k) q[k] = m->Q[e->a][k] + m->Q[e->b][k];
    const double det = q[0] * (q[4] * q[7] - q[5] * q[5]) - q[1] * (q[1] * q[7] - q[5] * q[2])
                       + q[2] * (q[1] * q[5] - q[4] * q[2]);
    const double tr = q[0] + q[4] + q[7];
    if (tr > 0.0 && fabs(det) > DEC_DET_EPS * tr * tr * tr) {
        /* v = -A^-1 (q3, q6, q8) through the adjugate of the symmetric A */
        const double i00 = q[4] * q[7] - q[5] * q[5], i01 = q[2] * q[5] - q[1] * q[7];
        const double i02 = q[1] * q[5] - q[2] * q[4], i11 = q[0] * q[7] - q[2] * q[2];
        const double i12 = q[1] * q[2] - q[0] * q[5], i22 = q[0] * q[4] - q[1] * q[1];
        e->p[0] = -(i00 * q[3] + i01 * q[6] + i02 * q[8]) / det;
        e->p[1] = -(i01 * q[3] + i11 * q[6] + i12 * q[8]) / det;
        e->p[2] = -(i02 * q[3] + i12 * q[6] + i22 * q[8]) / det;
        e->cost = dec_eval(q, e->p);
    } else {
        const double* pa = m->pos[e->a];
        const double* pb = m->pos[e->b];
        const double mid[3] = {(pa[0] + pb[0]) * 0.5, (pa[1] + pb[1]) * 0.5, (pa[2] + pb[2]) * 0.5};
        const double* cand[3] = {pa, pb, mid};
        double best = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double cst = dec_eval(q, cand[c]);
            if (c == 0 || cst < best) {
                best = cst;
                memcpy(e->p, cand[c], sizeof e->p);
            }
        }
        e->cost = best;
    }
    if (isnan(e->cost)) e->cost = INFINITY;
}

static int64_t dec_add_edge(dec_mesh* m, int32_t x, int32_t y)
{
    const int32_t a = x < y ? x : y, b = x < y ? y : x;
    int64_t i = dec_find(m, a, b);
    if (i >= 0 && m->e[i].alive) return i;
    if (i < 0) {
        if (m->ne == m->ecap) {
            m->ecap = m->ecap ? 2 * m->ecap : 1024;
            m->e = (dec_edge*)realloc(m->e, (size_t)m->ecap * sizeof(dec_edge));
        }
        i = m->ne++;
        dec_insert_key(m, dec_key(a, b), i);
    }
    dec_edge* e = &m->e[i];
    e->a = a;
    e->b = b;
    e->alive = 1;
    e->blocked = 0;
    dec_edge_cost(m, e);
    return i;
}

static int dec_tri_has(const dec_mesh* m, int64_t t, int32_t x)
{
    return m->tri[t][0] == x || m->tri[t][1] == x || m->tri[t][2] == x;
}

/* Triangles (live) containing both x and y. */
static int dec_shared(const dec_mesh* m, int32_t x, int32_t y, int64_t* out, int max)
{
    int n = 0;
    const dec_list* l = &m->vt[x];
    for (int32_t i = 0; i < l->n; ++i)
        if (dec_tri_has(m, l->v[i], y)) {
            if (n < max) out[n] = l->v[i];
            ++n;
        }
    return n;
}

static int dec_is_boundary_edge(const dec_mesh* m, int32_t x, int32_t y)
{
    int64_t t[4];
    return dec_shared(m, x, y, t, 4) == 1;
}

static int dec_is_boundary_vertex(const dec_mesh* m, int32_t x)
{
    const dec_list* l = &m->vt[x];
    for (int32_t i = 0; i < l->n; ++i)
        for (int k = 0; k < 3; ++k) {
            const int32_t y = m->tri[l->v[i]][k];
            if (y != x && dec_is_boundary_edge(m, x, y)) return 1;
        }
    return 0;
}

/* Vertex neighbours of x (each once), into l (cleared first). */
static void dec_neighbours(const dec_mesh* m, int32_t x, dec_list* out)
{
    out->n = 0;
    const dec_list* l = &m->vt[x];
    for (int32_t i = 0; i < l->n; ++i)
        for (int k = 0; k < 3; ++k) {
            const int32_t y = m->tri[l->v[i]][k];
            if (y == x) continue;
            int seen = 0;
            for (int32_t j = 0; j < out->n && !seen; ++j) seen = out->v[j] == y;
            if (!seen) dec_push(out, y);
        }
}

static int dec_has_triangle(const dec_mesh* m, int32_t x, int32_t y, int32_t z)
{
    const dec_list* l = &m->vt[x];
    for (int32_t i = 0; i < l->n; ++i)
        if (dec_tri_has(m, l->v[i], y) && dec_tri_has(m, l->v[i], z)) return 1;
    return 0;
}

static int dec_valid(const dec_mesh* m, const dec_edge* e)
{
    const int32_t a = e->a, b = e->b;
    int64_t shared[3];
    const int ns = dec_shared(m, a, b, shared, 3);
    if (ns < 1 || ns > 2) return 0;
    dec_list na = {0, 0, 0}, nb = {0, 0, 0};
    dec_neighbours(m, a, &na);
    dec_neighbours(m, b, &nb);
    int common = 0;
    for (int32_t i = 0; i < na.n; ++i)
        for (int32_t j = 0; j < nb.n; ++j) common += na.v[i] == nb.v[j];
    free(na.v);
    free(nb.v);
    if (common != ns) return 0;
    if (ns == 2) {
        int32_t opp[2];
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < 3; ++k) {
                const int32_t y = m->tri[shared[s]][k];
                if (y != a && y != b) opp[s] = y;
            }
        if (dec_has_triangle(m, a, opp[0], opp[1]) && dec_has_triangle(m, b, opp[0], opp[1])) return 0;
        if (dec_is_boundary_vertex(m, a) && dec_is_boundary_vertex(m, b)) return 0;
    }
    for (int side = 0; side < 2; ++side) {
        const int32_t x = side ? b : a, other = side ? a : b;
        const dec_list* l = &m->vt[x];
        for (int32_t i = 0; i < l->n; ++i) {
            const int64_t t = l->v[i];
            if (dec_tri_has(m, t, other)) continue;
            int slot = 0;
            while (m->tri[t][slot] != x) ++slot;
            double n0[3], n1[3];
            dec_tri_normal(m, t, -1, NULL, n0);
            dec_tri_normal(m, t, slot, e->p, n1);
            if (!(n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2] > 0.0)) return 0;
        }
    }
    return 1;
}

/* Decimate; writes the kept vertices (float [n][3]) and triangles (int32 [n][3]) and
 * returns their counts.  Outputs may be NULL to count only.  Returns -1 on a bad index. */
int64_t or_decimate(const float* vin, int64_t nv, const int32_t* tin, int64_t nt, double rate,
                    float* vout, int64_t* nv_out, int32_t* tout, int64_t* nt_out)
{
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* q = tin + 3 * t;
        for (int k = 0; k < 3; ++k)
            if (q[k] < 0 || q[k] >= nv) return -1;
        if (q[0] == q[1] || q[1] == q[2] || q[0] == q[2]) return -1;
    }
    dec_mesh m;
    memset(&m, 0, sizeof m);
    m.nv = nv;
    m.nt = nt;
    m.pos = (double(*)[3])calloc((size_t)(nv ? nv : 1), sizeof *m.pos);
    m.Q = (double(*)[10])calloc((size_t)(nv ? nv : 1), sizeof *m.Q);
    m.tri = (int32_t(*)[3])calloc((size_t)(nt ? nt : 1), sizeof *m.tri);
    m.tri_alive = (char*)calloc((size_t)(nt ? nt : 1), 1);
    m.v_alive = (char*)calloc((size_t)(nv ? nv : 1), 1);
    m.vt = (dec_list*)calloc((size_t)(nv ? nv : 1), sizeof(dec_list));
    m.hcap = 1024;
    while (m.hcap < 8 * (nt + 16)) m.hcap *= 2;
    m.hkey = (int64_t*)malloc((size_t)m.hcap * sizeof(int64_t));
    m.hval = (int64_t*)malloc((size_t)m.hcap * sizeof(int64_t));
    for (int64_t h = 0; h < m.hcap; ++h) m.hkey[h] = -1;
    for (int64_t v = 0; v < nv; ++v) {
        for (int k = 0; k < 3; ++k) m.pos[v][k] = (double)vin[3 * v + k];
        m.v_alive[v] = 1;
    }
    for (int64_t t = 0; t < nt; ++t) {
        for (int k = 0; k < 3; ++k) {
            m.tri[t][k] = tin[3 * t + k];
            dec_push(&m.vt[m.tri[t][k]], (int32_t)t);
        }
        m.tri_alive[t] = 1;
    }
    m.live_tri = nt;
    /* triangle quadrics, in triangle order */
    for (int64_t t = 0; t < nt; ++t) {
        double n[3];
        dec_tri_normal(&m, t, -1, NULL, n);
        const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(len > 0.0)) continue;
        const double u[3] = {n[0] / len, n[1] / len, n[2] / len};
        const double* p0 = m.pos[m.tri[t][0]];
        const double d = -(u[0] * p0[0] + u[1] * p0[1] + u[2] * p0[2]);
        for (int k = 0; k < 3; ++k) dec_add_plane(m.Q[m.tri[t][k]], u, d, 1.0);
    }
    /* boundary constraint planes, in triangle and edge-slot order */
    for (int64_t t = 0; t < nt; ++t) {
        double n[3];
        dec_tri_normal(&m, t, -1, NULL, n);
        const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(len > 0.0)) continue;
        const double u[3] = {n[0] / len, n[1] / len, n[2] / len};
        for (int k = 0; k < 3; ++k) {
            const int32_t x = m.tri[t][k], y = m.tri[t][(k + 1) % 3];
            if (!dec_is_boundary_edge(&m, x, y)) continue;
            const double ed[3] = {m.pos[y][0] - m.pos[x][0], m.pos[y][1] - m.pos[x][1],
                                  m.pos[y][2] - m.pos[x][2]};
            double c[3];
            dec_cross(ed, u, c);
            const double cl = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            if (!(cl > 0.0)) continue;
            const double w[3] = {c[0] / cl, c[1] / cl, c[2] / cl};
            const double d = -(w[0] * m.pos[x][0] + w[1] * m.pos[x][1] + w[2] * m.pos[x][2]);
            const double wt = DEC_BOUNDARY_WEIGHT;
            dec_add_plane(m.Q[x], w, d, wt);
            dec_add_plane(m.Q[y], w, d, wt);
        }
    }
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) dec_add_edge(&m, m.tri[t][k], m.tri[t][(k + 1) % 3]);
    const int64_t target = (int64_t)floor(rate * (double)nt + 0.5);
    dec_list nbs = {0, 0, 0}, nas = {0, 0, 0}, nns = {0, 0, 0};
    while (m.live_tri > target) {
        int64_t best = -1;
        for (int64_t i = 0; i < m.ne; ++i) {
            const dec_edge* e = &m.e[i];
            if (!e->alive || e->blocked) continue;
            if (best < 0) { best = i; continue; }
            const dec_edge* f = &m.e[best];
            if (e->cost < f->cost || (e->cost == f->cost && (e->a < f->a || (e->a == f->a && e->b < f->b))))
                best = i;
        }
        if (best < 0) break;
        dec_edge* e = &m.e[best];
        if (!dec_valid(&m, e)) {
            e->blocked = 1;
            continue;
        }
        const int32_t a = e->a, b = e->b;
        double p[3];
        memcpy(p, e->p, sizeof p);
        /* every edge at b dies (the edge itself included) */
        dec_neighbours(&m, b, &nbs);
        for (int32_t j = 0; j < nbs.n; ++j) {
            const int32_t y = nbs.v[j];
            const int64_t i = dec_find(&m, y < b ? y : b, y < b ? b : y);
            if (i >= 0) m.e[i].alive = 0;
        }
        /* the triangles of the edge go; b's other triangles become a's */
        int64_t shared[3];
        const int ns = dec_shared(&m, a, b, shared, 3);
        for (int s = 0; s < ns; ++s) {
            const int64_t t = shared[s];
            m.tri_alive[t] = 0;
            --m.live_tri;
            for (int k = 0; k < 3; ++k) dec_remove(&m.vt[m.tri[t][k]], (int32_t)t);
        }
        for (int32_t i = 0; i < m.vt[b].n; ++i) {
            const int64_t t = m.vt[b].v[i];
            for (int k = 0; k < 3; ++k)
                if (m.tri[t][k] == b) m.tri[t][k] = a;
            dec_push(&m.vt[a], (int32_t)t);
        }
        m.vt[b].n = 0;
        m.v_alive[b] = 0;
        memcpy(m.pos[a], p, sizeof p);
        for (int k = 0; k < 10; ++k) m.Q[a][k] = m.Q[a][k] + m.Q[b][k];
        /* a's edges (new costs), then every edge at a neighbour of a unblocked */
        dec_neighbours(&m, a, &nas);
        for (int32_t j = 0; j < nas.n; ++j) {
            const int32_t x = nas.v[j] < a ? nas.v[j] : a, y = nas.v[j] < a ? a : nas.v[j];
            const int64_t i = dec_find(&m, x, y);
            if (i >= 0 && m.e[i].alive) {
                m.e[i].blocked = 0;
                dec_edge_cost(&m, &m.e[i]);
            } else {
                dec_add_edge(&m, x, y);
            }
        }
        for (int32_t j = 0; j < nas.n; ++j) {
            const int32_t w = nas.v[j];
            dec_neighbours(&m, w, &nns);
            for (int32_t q = 0; q < nns.n; ++q) {
                const int32_t x = nns.v[q] < w ? nns.v[q] : w, y = nns.v[q] < w ? w : nns.v[q];
                const int64_t i = dec_find(&m, x, y);
                if (i >= 0 && m.e[i].alive) m.e[i].blocked = 0;
            }
        }
    }
    free(nbs.v);
    free(nas.v);
    free(nns.v);
    /* output: surviving triangles in order, the vertices they use in order */
    int64_t* remap = (int64_t*)malloc((size_t)(nv ? nv : 1) * sizeof(int64_t));
    for (int64_t v = 0; v < nv; ++v) remap[v] = -1;
    for (int64_t t = 0; t < nt; ++t)
        if (m.tri_alive[t])
            for (int k = 0; k < 3; ++k) remap[m.tri[t][k]] = 0;
    int64_t kv = 0, kt = 0;
    for (int64_t v = 0; v < nv; ++v)
        if (remap[v] == 0) {
            remap[v] = kv;
            if (vout)
                for (int k = 0; k < 3; ++k) vout[3 * kv + k] = (float)m.pos[v][k];
            ++kv;
        }
    for (int64_t t = 0; t < nt; ++t)
        if (m.tri_alive[t]) {
            if (tout)
                for (int k = 0; k < 3; ++k) tout[3 * kt + k] = (int32_t)remap[m.tri[t][k]];
            ++kt;
        }
    *nv_out = kv;
    *nt_out = kt;
    free(remap);
    for (int64_t v = 0; v < nv; ++v) free(m.vt[v].v);
    free(m.vt);
    free(m.pos);
    free(m.Q);
    free(m.tri);
    free(m.tri_alive);
    free(m.v_alive);
    free(m.e);
    free(m.hkey);
    free(m.hval);
    return kt;
}
