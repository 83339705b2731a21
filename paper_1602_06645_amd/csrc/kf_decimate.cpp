// Quadric-error decimation of a triangle mesh (Sec. IV.C: the dense marching-cubes model is
// simplified with the quadric-based decimation of Garland and Heckbert to a reduction
// rate, the fraction of the polygons kept).  Host code: a sequential greedy edge collapse
// with a priority queue (the GPU extracts the mesh, kf_mesh_extract; this simplifies it).
//
// Each triangle's plane (unit normal u, offset d) contributes its fundamental quadric
// [u d][u d]^T (the squared distance to the plane) to the quadric of its vertices; each
// boundary edge (used by one triangle) adds, to both ends, the quadric of the plane through
// it perpendicular to its triangle with weight 1000, so that open borders keep their place.  An edge (a, b), a < b, contracts
// to the minimiser of v^T (Q_a + Q_b) v (when its 3x3 part is well conditioned, else the
// cheapest of a, b and their midpoint) at the quadric's value there.  The cheapest edge
// (ties by a, then b) that is not blocked is contracted when the common neighbours of a and
// b are exactly the opposite vertices of its triangles, both ends are on the boundary only
// if the edge is, it is not an edge of a tetrahedron, and no other triangle of a or b turns
// over; an edge that fails is blocked until a contraction next to it (a's new edges get new
// costs; the edges at a and at its neighbours are unblocked).  Collapses continue until at
// most round(rate * triangles) remain or no edge can go.  Every choice depends only on
// these definitions (not on the order of containers), in double precision, so the result
// is reproducible.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <queue>
#include <unordered_map>
#include <vector>

#include "kf_launch.h"

namespace {

constexpr double kBoundaryWeight = 1000.0;
constexpr double kDetEps = 1e-10;

struct Edge {
    int32_t a, b;
    bool alive, blocked;
    uint32_t version;
    double cost, p[3];
};

struct Item {
    double cost;
    int32_t a, b;
    uint32_t edge, version;
};

// std::priority_queue keeps the largest on top: order by (cost, a, b) reversed.
struct Later {
    bool operator()(const Item& x, const Item& y) const
    {
        if (x.cost != y.cost) return x.cost > y.cost;
        if (x.a != y.a) return x.a > y.a;
        return x.b > y.b;
    }
};

struct Mesh {
    std::vector<double> pos;          // [nv][3]
    std::vector<double> Q;            // [nv][10]
    std::vector<int32_t> tri;         // [nt][3]
    std::vector<char> tri_alive;
    std::vector<std::vector<int32_t>> vt;   // live triangles of each vertex
    std::vector<Edge> edges;
    std::unordered_map<int64_t, uint32_t> index;
    std::priority_queue<Item, std::vector<Item>, Later> heap;
    int64_t live_tri = 0;

    static int64_t key(int32_t a, int32_t b) { return ((int64_t)a << 32) | (uint32_t)b; }
    const double* P(int32_t v) const { return &pos[3 * (size_t)v]; }
    bool has(int64_t t, int32_t x) const
    {
        const int32_t* q = &tri[3 * (size_t)t];
        return q[0] == x || q[1] == x || q[2] == x;
    }

    void push(uint32_t i)
    {
        const Edge& e = edges[i];
        heap.push(Item{e.cost, e.a, e.b, i, e.version});
    }

    static void add_plane(double* q, const double u[3], double d, double w)
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

    static double eval(const double* q, const double* v)
    {
        const double x = v[0], y = v[1], z = v[2];
        return q[0] * x * x + 2.0 * q[1] * x * y + 2.0 * q[2] * x * z + 2.0 * q[3] * x
               + q[4] * y * y + 2.0 * q[5] * y * z + 2.0 * q[6] * y + q[7] * z * z
               + 2.0 * q[8] * z + q[9];
    }

    static void cross(const double a[3], const double b[3], double out[3])
    {
        out[0] = a[1] * b[2] - a[2] * b[1];
        out[1] = a[2] * b[0] - a[0] * b[2];
        out[2] = a[0] * b[1] - a[1] * b[0];
    }

    // Unnormalised normal of triangle t, with vertex slot `slot` moved to p (slot < 0: none).
    void normal(int64_t t, int slot, const double* p, double n[3]) const
    {
        const double* v[3];
        for (int k = 0; k < 3; ++k) v[k] = (k == slot) ? p : P(tri[3 * (size_t)t + k]);
        double e1[3], e2[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = v[1][k] - v[0][k];
            e2[k] = v[2][k] - v[0][k];
        }
        cross(e1, e2, n);
    }

    void cost(Edge& e) const
    {
        double q[10];
        for (int k = 0; k < 10; ++k) q[k] = Q[10 * (size_t)e.a + k] + Q[10 * (size_t)e.b + k];
        const double det = q[0] * (q[4] * q[7] - q[5] * q[5]) - q[1] * (q[1] * q[7] - q[5] * q[2])
                           + q[2] * (q[1] * q[5] - q[4] * q[2]);
        const double tr = q[0] + q[4] + q[7];
        if (tr > 0.0 && fabs(det) > kDetEps * tr * tr * tr) {
            const double i00 = q[4] * q[7] - q[5] * q[5], i01 = q[2] * q[5] - q[1] * q[7];
            const double i02 = q[1] * q[5] - q[2] * q[4], i11 = q[0] * q[7] - q[2] * q[2];
            const double i12 = q[1] * q[2] - q[0] * q[5], i22 = q[0] * q[4] - q[1] * q[1];
            e.p[0] = -(i00 * q[3] + i01 * q[6] + i02 * q[8]) / det;
            e.p[1] = -(i01 * q[3] + i11 * q[6] + i12 * q[8]) / det;
            e.p[2] = -(i02 * q[3] + i12 * q[6] + i22 * q[8]) / det;
            e.cost = eval(q, e.p);
        } else {
            const double* pa = P(e.a);
            const double* pb = P(e.b);
            const double mid[3] = {(pa[0] + pb[0]) * 0.5, (pa[1] + pb[1]) * 0.5, (pa[2] + pb[2]) * 0.5};
            const double* cand[3] = {pa, pb, mid};
            double best = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double v = eval(q, cand[c]);
                if (c == 0 || v < best) {
                    best = v;
                    memcpy(e.p, cand[c], sizeof e.p);
                }
            }
            e.cost = best;
        }
        if (isnan(e.cost)) e.cost = INFINITY;
    }

    // Edge (x, y) made live (a new record, or a dead one revived) with its cost, queued.
    void add_edge(int32_t x, int32_t y)
    {
        const int32_t a = std::min(x, y), b = std::max(x, y);
        auto it = index.find(key(a, b));
        uint32_t i;
        if (it == index.end()) {
            i = (uint32_t)edges.size();
            edges.push_back(Edge{a, b, false, false, 0, 0.0, {0, 0, 0}});
            index.emplace(key(a, b), i);
        } else {
            i = it->second;
            if (edges[i].alive) return;
        }
        Edge& e = edges[i];
        e.alive = true;
        e.blocked = false;
        ++e.version;
        cost(e);
        push(i);
    }

    Edge* find(int32_t x, int32_t y)
    {
        auto it = index.find(key(std::min(x, y), std::max(x, y)));
        return it == index.end() ? nullptr : &edges[it->second];
    }

    int shared(int32_t x, int32_t y, int64_t* out, int max) const
    {
        int n = 0;
        for (int32_t t : vt[x])
            if (has(t, y)) {
                if (n < max) out[n] = t;
                ++n;
            }
        return n;
    }

    bool boundary_edge(int32_t x, int32_t y) const
    {
        int64_t t[2];
        return shared(x, y, t, 2) == 1;
    }

    bool boundary_vertex(int32_t x) const
    {
        for (int32_t t : vt[x])
            for (int k = 0; k < 3; ++k) {
                const int32_t y = tri[3 * (size_t)t + k];
                if (y != x && boundary_edge(x, y)) return true;
            }
        return false;
    }

    void neighbours(int32_t x, std::vector<int32_t>& out) const
    {
        out.clear();
        for (int32_t t : vt[x])
            for (int k = 0; k < 3; ++k) {
                const int32_t y = tri[3 * (size_t)t + k];
                if (y != x && std::find(out.begin(), out.end(), y) == out.end()) out.push_back(y);
            }
    }

    bool has_triangle(int32_t x, int32_t y, int32_t z) const
    {
        for (int32_t t : vt[x])
            if (has(t, y) && has(t, z)) return true;
        return false;
    }

    bool valid(const Edge& e, std::vector<int32_t>& na, std::vector<int32_t>& nb) const
    {
        const int32_t a = e.a, b = e.b;
        int64_t sh[3];
        const int ns = shared(a, b, sh, 3);
        if (ns < 1 || ns > 2) return false;
        neighbours(a, na);
        neighbours(b, nb);
        int common = 0;
        for (int32_t x : na) common += (int)std::count(nb.begin(), nb.end(), x);
        if (common != ns) return false;
        if (ns == 2) {
            int32_t opp[2];
            for (int s = 0; s < 2; ++s)
                for (int k = 0; k < 3; ++k) {
                    const int32_t y = tri[3 * (size_t)sh[s] + k];
                    if (y != a && y != b) opp[s] = y;
                }
            if (has_triangle(a, opp[0], opp[1]) && has_triangle(b, opp[0], opp[1])) return false;
            if (boundary_vertex(a) && boundary_vertex(b)) return false;
        }
        for (int side = 0; side < 2; ++side) {
            const int32_t x = side ? b : a, other = side ? a : b;
            for (int32_t t : vt[x]) {
                if (has(t, other)) continue;
                int slot = 0;
                while (tri[3 * (size_t)t + slot] != x) ++slot;
                double n0[3], n1[3];
                normal(t, -1, nullptr, n0);
                normal(t, slot, e.p, n1);
                if (!(n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2] > 0.0)) return false;
            }
        }
        return true;
    }
};

}  // namespace

namespace kf {

// Decimate a valid mesh (indices in range, no triangle repeating a vertex, finite vertices,
// rate in [0, 1]; kf_mesh_decimate checks them): writes the kept vertices and triangles
// (at most the input counts) and their numbers.
void decimate_mesh(const float* vertices, int64_t n_vertices, const int32_t* triangles,
                   int64_t n_triangles, double rate, float* out_vertices, int64_t* out_n_vertices,
                   int32_t* out_triangles, int64_t* out_n_triangles)
{
    Mesh m;
    const size_t nv = (size_t)n_vertices, nt = (size_t)n_triangles;
    m.pos.resize(3 * nv);
    m.Q.assign(10 * nv, 0.0);
    m.tri.assign(triangles, triangles + 3 * nt);
    m.tri_alive.assign(nt, 1);
    m.vt.resize(nv);
    for (size_t q = 0; q < 3 * nv; ++q) m.pos[q] = (double)vertices[q];
    for (size_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) m.vt[m.tri[3 * t + k]].push_back((int32_t)t);
    m.live_tri = (int64_t)nt;
    // triangle quadrics in triangle order, then the boundary planes in (triangle, slot) order
    for (size_t t = 0; t < nt; ++t) {
        double n[3];
        m.normal((int64_t)t, -1, nullptr, n);
        const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(len > 0.0)) continue;
        const double u[3] = {n[0] / len, n[1] / len, n[2] / len};
        const double* p0 = m.P(m.tri[3 * t]);
        const double d = -(u[0] * p0[0] + u[1] * p0[1] + u[2] * p0[2]);
        for (int k = 0; k < 3; ++k) Mesh::add_plane(&m.Q[10 * (size_t)m.tri[3 * t + k]], u, d, 1.0);
    }
    for (size_t t = 0; t < nt; ++t) {
        double n[3];
        m.normal((int64_t)t, -1, nullptr, n);
        const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(len > 0.0)) continue;
        const double u[3] = {n[0] / len, n[1] / len, n[2] / len};
        for (int k = 0; k < 3; ++k) {
            const int32_t x = m.tri[3 * t + k], y = m.tri[3 * t + (k + 1) % 3];
            if (!m.boundary_edge(x, y)) continue;
            const double* px = m.P(x);
            const double* py = m.P(y);
            const double ed[3] = {py[0] - px[0], py[1] - px[1], py[2] - px[2]};
            double c[3];
            Mesh::cross(ed, u, c);
            const double cl = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            if (!(cl > 0.0)) continue;
            const double w[3] = {c[0] / cl, c[1] / cl, c[2] / cl};
            const double d = -(w[0] * px[0] + w[1] * px[1] + w[2] * px[2]);
            const double wt = kBoundaryWeight;
            Mesh::add_plane(&m.Q[10 * (size_t)x], w, d, wt);
            Mesh::add_plane(&m.Q[10 * (size_t)y], w, d, wt);
        }
    }
    m.edges.reserve(3 * nt / 2 + 16);
    m.index.reserve(3 * nt + 16);
    for (size_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) m.add_edge(m.tri[3 * t + k], m.tri[3 * t + (k + 1) % 3]);

    const int64_t target = (int64_t)floor(rate * (double)n_triangles + 0.5);
    std::vector<int32_t> na, nb, nn;
    while (m.live_tri > target && !m.heap.empty()) {
        const Item it = m.heap.top();
        m.heap.pop();
        Edge& top = m.edges[it.edge];
        if (!top.alive || top.blocked || top.version != it.version) continue;   // stale
        if (!m.valid(top, na, nb)) {
            top.blocked = true;
            ++top.version;
            continue;
        }
        const int32_t a = top.a, b = top.b;
        double p[3];
        memcpy(p, top.p, sizeof p);
        // every edge at b dies (this one included)
        m.neighbours(b, nb);
        for (int32_t y : nb)
            if (Edge* e = m.find(y, b)) {
                e->alive = false;
                ++e->version;
            }
        // the triangles of the edge go; b's other triangles become a's
        int64_t sh[3];
        const int ns = m.shared(a, b, sh, 3);
        for (int s = 0; s < ns; ++s) {
            const int64_t t = sh[s];
            m.tri_alive[t] = 0;
            --m.live_tri;
            for (int k = 0; k < 3; ++k) {
                auto& l = m.vt[m.tri[3 * (size_t)t + k]];
                l.erase(std::find(l.begin(), l.end(), (int32_t)t));
            }
        }
        for (int32_t t : m.vt[b]) {
            for (int k = 0; k < 3; ++k)
                if (m.tri[3 * (size_t)t + k] == b) m.tri[3 * (size_t)t + k] = a;
            m.vt[a].push_back(t);
        }
        m.vt[b].clear();
        memcpy(&m.pos[3 * (size_t)a], p, sizeof p);
        for (int k = 0; k < 10; ++k) m.Q[10 * (size_t)a + k] = m.Q[10 * (size_t)a + k] + m.Q[10 * (size_t)b + k];
        // a's edges get new costs; the edges at a's neighbours are unblocked
        m.neighbours(a, na);
        for (int32_t x : na) {
            Edge* e = m.find(x, a);
            if (e && e->alive) {
                e->blocked = false;
                ++e->version;
                m.cost(*e);
                m.push((uint32_t)(e - m.edges.data()));
            } else {
                m.add_edge(x, a);
            }
        }
        for (int32_t w : na) {
            m.neighbours(w, nn);
            for (int32_t y : nn) {
                Edge* e = m.find(y, w);
                if (e && e->alive && e->blocked) {
                    e->blocked = false;
                    ++e->version;
                    m.push((uint32_t)(e - m.edges.data()));
                }
            }
        }
    }
    // surviving triangles in input order, the vertices they use in input order
    std::vector<int64_t> remap(nv, -1);
    for (size_t t = 0; t < nt; ++t)
        if (m.tri_alive[t])
            for (int k = 0; k < 3; ++k) remap[m.tri[3 * t + k]] = 0;
    int64_t kv = 0, kt = 0;
    for (size_t v = 0; v < nv; ++v)
        if (remap[v] == 0) {
            remap[v] = kv;
            for (int k = 0; k < 3; ++k) out_vertices[3 * kv + k] = (float)m.pos[3 * v + k];
            ++kv;
        }
    for (size_t t = 0; t < nt; ++t)
        if (m.tri_alive[t]) {
            for (int k = 0; k < 3; ++k) out_triangles[3 * kt + k] = (int32_t)remap[m.tri[3 * t + k]];
            ++kt;
        }
    *out_n_vertices = kv;
    *out_n_triangles = kt;
}

}  // namespace kf
