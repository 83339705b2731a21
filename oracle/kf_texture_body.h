/*
 * Per-polygon texture maps (Sec. IV.D, Eq. 13-14 and the colour-volume lookup), written
 * once and included twice by kf_oracle.c (REAL = float, the parity precision; REAL =
 * double).  TEST INFRASTRUCTURE ONLY.
 *
 * Texel (i, j) of a map of w x h texels for triangle (V1, V2, V3): the step vectors of
 * Eq. 13-14 are (V2 - V1) / (w - 1) and (V3 - V1) / (h - 1); the texel's world point is
 * V1 + i step_1 + j step_2 (i then j, each an fma); its colour is the trilinear
 * interpolation of the colour volume at that point, in colour-index coordinates
 * q = p / s - (origin / s + 1/2) per axis (voxel i's centre at index i), x then y then z,
 * each a lerp fma(f, b - a, a), with the cell min(floor(q), dim - 2); zero unless q lies
 * in [0, dim - 1] and the 8 corner colour weights are positive.  The 8-bit texel is
 * rint(255 min(max(c, 0), 1)).
 *
 * Required macros: REAL, SFX, FMA, FLOOR, FMIN, FMAX, RINT.
 */

#define TX_CAT2(a, b) a##b
#define TX_CAT(a, b) TX_CAT2(a, b)
#define TX_FN(name) TX_CAT(name, SFX)

static REAL TX_FN(tx_lerp_)(REAL a, REAL b, REAL f) { return FMA(f, b - a, a); }

static int TX_FN(tx_colour_)(const int32_t* d, const REAL* qmax, const float* w,
                             const float* const* fields, const REAL* q, REAL* out)
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
    for (int m = 0; m < 3; ++m) {
        const float* F = fields[m];
        const REAL c00 = TX_FN(tx_lerp_)((REAL)F[base + off[0]], (REAL)F[base + off[1]], f[0]);
        const REAL c10 = TX_FN(tx_lerp_)((REAL)F[base + off[2]], (REAL)F[base + off[3]], f[0]);
        const REAL c01 = TX_FN(tx_lerp_)((REAL)F[base + off[4]], (REAL)F[base + off[5]], f[0]);
        const REAL c11 = TX_FN(tx_lerp_)((REAL)F[base + off[6]], (REAL)F[base + off[7]], f[0]);
        out[m] = TX_FN(tx_lerp_)(TX_FN(tx_lerp_)(c00, c10, f[1]), TX_FN(tx_lerp_)(c01, c11, f[1]), f[2]);
    }
    return 1;
}

static void TX_FN(texture_)(const or_volume* vol, const float* r, const float* g,
                            const float* b, const float* wc, int32_t n_tri, const float* tri,
                            const int32_t* rects, int32_t atlas_width, float* atlas,
                            uint8_t* atlas8)
{
    REAL inv_s[3], off[3], qmax[3];
    for (int k = 0; k < 3; ++k) {
        const double s = vol->extent[k] / vol->cdim[k];
        inv_s[k] = (REAL)(1.0 / s);
        off[k] = (REAL)(-vol->origin[k] / s - 0.5);
        qmax[k] = (REAL)(vol->cdim[k] - 1);
    }
    const float* fields[3] = {r, g, b};
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t n = 0; n < n_tri; ++n) {
        const float* V = tri + 9 * (size_t)n;
        const int32_t x0 = rects[4 * n], y0 = rects[4 * n + 1], w = rects[4 * n + 2], h = rects[4 * n + 3];
        REAL s1[3], s2[3];
        for (int k = 0; k < 3; ++k) {
            s1[k] = ((REAL)V[3 + k] - (REAL)V[k]) / (REAL)(w - 1);   /* Eq. 13 */
            s2[k] = ((REAL)V[6 + k] - (REAL)V[k]) / (REAL)(h - 1);   /* Eq. 14 */
        }
        for (int32_t j = 0; j < h; ++j)
            for (int32_t i = 0; i < w; ++i) {
                REAL q[3], c[3] = {0, 0, 0};
                for (int k = 0; k < 3; ++k) {
                    const REAL p = FMA((REAL)j, s2[k], FMA((REAL)i, s1[k], (REAL)V[k]));
                    q[k] = FMA(p, inv_s[k], off[k]);
                }
                if (!TX_FN(tx_colour_)(vol->cdim, qmax, wc, fields, q, c)) c[0] = c[1] = c[2] = 0;
                const size_t t = ((size_t)(y0 + j) * (size_t)atlas_width + (size_t)(x0 + i)) * 3;
                for (int m = 0; m < 3; ++m) {
                    atlas[t + m] = (float)c[m];
                    if (atlas8)
                        atlas8[t + m] = (uint8_t)RINT(FMIN(FMAX(c[m], (REAL)0), (REAL)1) * (REAL)255);
                }
            }
    }
}

#undef TX_CAT2
#undef TX_CAT
#undef TX_FN
