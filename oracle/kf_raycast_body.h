/*
 * Ray casting of the geometry and colour volumes, written once and included twice by
 * kf_oracle.c: REAL = float (the parity precision) and REAL = double (the
 * precision of the closed-form and brute-force checks).  TEST INFRASTRUCTURE ONLY.
 *
 * The method renders the volumes it integrates for live feedback and obtains the
 * predicted surface for tracking by ray tracing the TSDF (abstract; Sec. III, after
 * KinectFusion).  The paper gives no formulas, so the steps below are the readings of
 * this implementation (listed with the other readings in the design notes):
 *
 *   ray       pixel (x, y) -> camera point (t (x - cx)/fx, t (y - cy)/fy, t): t is the
 *             camera depth.  In continuous geometry-index coordinates (voxel i has its
 *             centre at index i) the ray is q(t) = a + t b(x, y), b affine in (x, y).
 *   samples   t_n = n * delta for integer n >= 1, restricted to the slab where every
 *             coordinate of q lies in [0, dim - 1] (so that the 8 trilinear corners
 *             exist; at most 2^20 samples, none beyond 2^23 steps); a sample is valid iff
 *             q is inside that box and the 8 corner geometry weights are positive.
 *   TSDF      trilinear interpolation, x first, then y, then z, each step a lerp
 *             fma(f, b - a, a); the cell is min(floor(q), dim - 2).
 *   hit       the first pair of consecutive valid samples with F_{n-1} > 0 > F_n (the
 *             surface seen from its front); t* = t_{n-1} + delta F_{n-1} / (F_{n-1} - F_n).
 *   outputs   depth t*; the world point of the ray at t*; the normal: the gradient of the
 *             trilinear TSDF by central differences one index step away on each axis,
 *             scaled to world units and normalised (zero when a difference sample is
 *             invalid or the gradient is zero); the colour: trilinear interpolation of
 *             the colour volume at the hit (zero unless its 8 corner colour weights are
 *             positive).  A miss writes zeros.
 *
 * Required macros: REAL, SFX, FMA, SQRT, FLOOR, CEIL, FMIN, FMAX.
 */

#define RC_CAT2(a, b) a##b
#define RC_CAT(a, b) RC_CAT2(a, b)
#define RC_FN(name) RC_CAT(name, SFX)

typedef struct {
    REAL a[3], Bu[3], Bv[3], B0[3];     /* geometry index space: q = a + t (Bu x + Bv y + B0) */
    REAL ac[3], Bcu[3], Bcv[3], Bc0[3]; /* colour index space                             */
    REAL Ru[3], Rv[3], R0[3], tw[3];    /* world: p = tw + t (Ru x + Rv y + R0)           */
    REAL inv_s[3];                      /* 1 / geometry voxel size per axis               */
    REAL gmax[3], cmax[3];              /* dim - 1 per axis                               */
    REAL delta;
} RC_CAT(or_rc_, SFX);

static void RC_FN(rc_round_)(const or_rc64* in, RC_CAT(or_rc_, SFX)* out)
{
    for (int k = 0; k < 3; ++k) {
        out->a[k] = (REAL)in->a[k];
        out->Bu[k] = (REAL)in->Bu[k];
        out->Bv[k] = (REAL)in->Bv[k];
        out->B0[k] = (REAL)in->B0[k];
        out->ac[k] = (REAL)in->ac[k];
        out->Bcu[k] = (REAL)in->Bcu[k];
        out->Bcv[k] = (REAL)in->Bcv[k];
        out->Bc0[k] = (REAL)in->Bc0[k];
        out->Ru[k] = (REAL)in->Ru[k];
        out->Rv[k] = (REAL)in->Rv[k];
        out->R0[k] = (REAL)in->R0[k];
        out->tw[k] = (REAL)in->tw[k];
        out->inv_s[k] = (REAL)in->inv_s[k];
        out->gmax[k] = (REAL)in->gmax[k];
        out->cmax[k] = (REAL)in->cmax[k];
    }
    out->delta = (REAL)in->delta;
}

static REAL RC_FN(rc_lerp_)(REAL a, REAL b, REAL f) { return FMA(f, b - a, a); }

/* Trilinear interpolation of up to three fields of a volume of dims d at index point q.
 * Returns 1 iff q lies in [0, max] on every axis and the 8 corner weights are > 0. */
static int RC_FN(rc_trilinear_)(const int32_t* d, const REAL* qmax, const float* w,
                                const float* const* fields, int n_fields, const REAL* q,
                                REAL* out)
{
    int i[3];
    REAL f[3];
    for (int k = 0; k < 3; ++k) {
        if (!(q[k] >= (REAL)0 && q[k] <= qmax[k])) return 0;
        int c = (int)FLOOR(q[k]);
        if (c > d[k] - 2) c = d[k] - 2;
        i[k] = c;
        f[k] = q[k] - (REAL)c;
    }
    const size_t X = (size_t)d[0], XY = (size_t)d[0] * (size_t)d[1];
    const size_t base = (size_t)i[0] + X * (size_t)i[1] + XY * (size_t)i[2];
    const size_t off[8] = {0, 1, X, X + 1, XY, XY + 1, XY + X, XY + X + 1};
    for (int c = 0; c < 8; ++c)
        if (!(w[base + off[c]] > 0.0f)) return 0;
    for (int m = 0; m < n_fields; ++m) {
        const float* F = fields[m];
        const REAL c00 = RC_FN(rc_lerp_)((REAL)F[base + off[0]], (REAL)F[base + off[1]], f[0]);
        const REAL c10 = RC_FN(rc_lerp_)((REAL)F[base + off[2]], (REAL)F[base + off[3]], f[0]);
        const REAL c01 = RC_FN(rc_lerp_)((REAL)F[base + off[4]], (REAL)F[base + off[5]], f[0]);
        const REAL c11 = RC_FN(rc_lerp_)((REAL)F[base + off[6]], (REAL)F[base + off[7]], f[0]);
        const REAL c0 = RC_FN(rc_lerp_)(c00, c10, f[1]);
        const REAL c1 = RC_FN(rc_lerp_)(c01, c11, f[1]);
        out[m] = RC_FN(rc_lerp_)(c0, c1, f[2]);
    }
    return 1;
}

/* One pixel.  Writes depth, vertex[3], normal[3], colour[3]. */
static void RC_FN(rc_pixel_)(const or_volume* vol, const RC_CAT(or_rc_, SFX)* c,
                             const float* tsdf, const float* wg, const float* r,
                             const float* g, const float* b, const float* wc, int x, int y,
                             float* depth, float* vertex, float* normal, float* colour)
{
    *depth = 0.0f;
    for (int k = 0; k < 3; ++k) vertex[k] = normal[k] = colour[k] = 0.0f;
    const REAL u = (REAL)x, v = (REAL)y;
    REAL bq[3];
    for (int k = 0; k < 3; ++k) bq[k] = FMA(c->Bv[k], v, FMA(c->Bu[k], u, c->B0[k]));
    /* the slab of the ray inside [0, dim - 1] on every axis */
    REAL t_in = (REAL)-INFINITY, t_out = (REAL)INFINITY;
    for (int k = 0; k < 3; ++k) {
        if (bq[k] != (REAL)0) {
            const REAL ta = ((REAL)0 - c->a[k]) / bq[k];
            const REAL tb = (c->gmax[k] - c->a[k]) / bq[k];
            t_in = FMAX(t_in, FMIN(ta, tb));
            t_out = FMIN(t_out, FMAX(ta, tb));
        } else if (!(c->a[k] >= (REAL)0 && c->a[k] <= c->gmax[k])) {
            return;
        }
    }
    /* sample indices n0..n1; a ray whose first sample lies beyond 2^23 steps misses, and
     * at most 2^20 samples are taken (both keep n exact in single precision) */
    const REAL n0 = FMAX(CEIL(t_in / c->delta), (REAL)1);
    const REAL n1 = FMIN(FLOOR(t_out / c->delta), n0 + (REAL)1048575);
    if (!(n0 <= n1) || !(n0 <= (REAL)8388608)) return;
    const float* fields[3] = {tsdf, NULL, NULL};
    int prev_valid = 0;
    REAL prev_F = 0, prev_t = 0, t_hit = 0;
    int hit = 0;
    for (int64_t n = (int64_t)n0; n <= (int64_t)n1; ++n) {
        const REAL t = (REAL)n * c->delta;
        REAL q[3], F = 0;
        for (int k = 0; k < 3; ++k) q[k] = FMA(t, bq[k], c->a[k]);
        const int valid = RC_FN(rc_trilinear_)(vol->gdim, c->gmax, wg, fields, 1, q, &F);
        if (valid && prev_valid && prev_F > (REAL)0 && F < (REAL)0) {
            t_hit = FMA(c->delta, prev_F / (prev_F - F), prev_t);
            hit = 1;
            break;
        }
        prev_valid = valid;
        prev_F = F;
        prev_t = t;
    }
    if (!hit) return;
    *depth = (float)t_hit;
    for (int k = 0; k < 3; ++k)
        vertex[k] = (float)FMA(t_hit, FMA(c->Rv[k], v, FMA(c->Ru[k], u, c->R0[k])), c->tw[k]);
    /* normal: central differences of the trilinear TSDF one index step away */
    REAL qh[3];
    for (int k = 0; k < 3; ++k) qh[k] = FMA(t_hit, bq[k], c->a[k]);
    REAL grad[3];
    int ok = 1;
    for (int k = 0; k < 3 && ok; ++k) {
        REAL qp[3] = {qh[0], qh[1], qh[2]}, qm[3] = {qh[0], qh[1], qh[2]};
        qp[k] = qh[k] + (REAL)1;
        qm[k] = qh[k] - (REAL)1;
        REAL Fp, Fm;
        ok = RC_FN(rc_trilinear_)(vol->gdim, c->gmax, wg, fields, 1, qp, &Fp) &&
             RC_FN(rc_trilinear_)(vol->gdim, c->gmax, wg, fields, 1, qm, &Fm);
        if (ok) grad[k] = (Fp - Fm) * c->inv_s[k];
    }
    if (ok) {
        const REAL gg = FMA(grad[0], grad[0], FMA(grad[1], grad[1], grad[2] * grad[2]));
        if (gg > (REAL)0) {
            const REAL len = SQRT(gg);
            for (int k = 0; k < 3; ++k) normal[k] = (float)(grad[k] / len);
        }
    }
    /* colour: trilinear interpolation of the colour volume at the hit */
    REAL qc[3];
    for (int k = 0; k < 3; ++k) {
        const REAL bc = FMA(c->Bcv[k], v, FMA(c->Bcu[k], u, c->Bc0[k]));
        qc[k] = FMA(t_hit, bc, c->ac[k]);
    }
    const float* cf[3] = {r, g, b};
    REAL col[3];
    if (RC_FN(rc_trilinear_)(vol->cdim, c->cmax, wc, cf, 3, qc, col))
        for (int k = 0; k < 3; ++k) colour[k] = (float)col[k];
}

static void RC_FN(raycast_)(const or_volume* vol, const or_rc64* c64, const float* tsdf,
                            const float* wg, const float* r, const float* g, const float* b,
                            const float* wc, int width, const int32_t* pixels, int64_t n_pix,
                            float* depth, float* vertex, float* normal, float* colour)
{
    RC_CAT(or_rc_, SFX) c;
    RC_FN(rc_round_)(c64, &c);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < n_pix; ++p) {
        const int32_t pix = pixels[p];
        RC_FN(rc_pixel_)(vol, &c, tsdf, wg, r, g, b, wc, pix % width, pix / width, depth + p,
                         vertex + 3 * p, normal + 3 * p, colour + 3 * p);
    }
}

#undef RC_CAT2
#undef RC_CAT
#undef RC_FN
