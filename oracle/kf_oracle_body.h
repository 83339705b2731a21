/*
 * Per-voxel steps of the oracle, written once and included twice by kf_oracle.c:
 * with REAL = float (the parity precision) and REAL = double (the precision of the
 * finite-difference and adjoint checks).  TEST INFRASTRUCTURE ONLY (see kf_oracle.c).
 *
 * Every step follows the paper, "Creating Simplified 3D Models with High Quality
 * Textures", Sec. IV.B (colour volume integration, Eq. 5-10) with the depth-to-HD
 * mapping of Sec. IV.A (Eq. 1-4), and Sec. III for the TSDF geometry volume the method
 * inherits from KinectFusion.  The order of every floating-point operation is fixed,
 * so that the FP32 instance is the exact reference for masks and weights.
 *
 * Required macros: REAL, SFX (name suffix), FMA, SQRT, RINT, FLOOR, FMIN.
 */

#define OR_CAT2(a, b) a##b
#define OR_CAT(a, b) OR_CAT2(a, b)
#define OR_FN(name) OR_CAT(name, SFX)
#define OR_T(name) OR_CAT(name, SFX)

/* Per-frame constants.  Built in double on the host, then rounded once to REAL. */
typedef struct {
    REAL Ag[9], bg[3];   /* geometry voxel index -> depth-camera coordinates (Eq. 5)  */
    REAL Ac[9], bc[3];   /* colour voxel index   -> depth-camera coordinates (Eq. 5)  */
    REAL Ah[9], bh[3];   /* colour voxel index   -> HD-camera coordinates (Eq. 5 + 3) */
    REAL fx, fy, cx, cy, inv_fx, inv_fy;  /* K_c and the diagonal of K_c^-1 (Eq. 6, 7) */
    REAL fxr, fyr, cxr, cyr;               /* K_hd (Eq. 4)                            */
    REAL trunc, inv_trunc, w_max, sigma2, gate;
    int hd_nearest;                        /* nearest-pixel HD sampling (else bilinear) */
} OR_T(or_fc_);

static void OR_FN(round_consts_)(const or_fc64* in, OR_T(or_fc_)* out)
{
    for (int q = 0; q < 9; ++q) {
        out->Ag[q] = (REAL)in->Ag[q];
        out->Ac[q] = (REAL)in->Ac[q];
        out->Ah[q] = (REAL)in->Ah[q];
    }
    for (int q = 0; q < 3; ++q) {
        out->bg[q] = (REAL)in->bg[q];
        out->bc[q] = (REAL)in->bc[q];
        out->bh[q] = (REAL)in->bh[q];
    }
    out->fx = (REAL)in->fx; out->fy = (REAL)in->fy;
    out->cx = (REAL)in->cx; out->cy = (REAL)in->cy;
    out->inv_fx = (REAL)in->inv_fx; out->inv_fy = (REAL)in->inv_fy;
    out->fxr = (REAL)in->fxr; out->fyr = (REAL)in->fyr;
    out->cxr = (REAL)in->cxr; out->cyr = (REAL)in->cyr;
    out->trunc = (REAL)in->trunc; out->inv_trunc = (REAL)in->inv_trunc;
    out->w_max = (REAL)in->w_max; out->sigma2 = (REAL)in->sigma2;
    out->gate = (REAL)in->gate;
    out->hd_nearest = in->hd_nearest != 0.0;
}

/* A depth pixel is a measurement iff it is a positive finite number; zero marks a
 * hole (Sec. IV.B: only a non-zero D_n is used). */
static int OR_FN(valid_depth_)(REAL d)
{
    return d > (REAL)0 && d < (REAL)INFINITY;
}

/* Eq. 5 for voxel (i,j,k): R_n (s*(i,j,k) + o + s/2) + t_n folded into A, b.  The
 * innermost term is the x index, then y, then z. */
static void OR_FN(affine_)(const REAL* A, const REAL* b, int i, int j, int k, REAL* p)
{
    REAL fi = (REAL)i, fj = (REAL)j, fk = (REAL)k;
    for (int r = 0; r < 3; ++r)
        p[r] = FMA(A[3 * r + 2], fk, FMA(A[3 * r + 1], fj, FMA(A[3 * r + 0], fi, b[r])));
}

/* Eq. 6 plus the frustum test: project p with K_c, divide by z, round to the nearest
 * pixel (ties to even).  Returns 0 when the voxel is outside the depth frustum. */
static int OR_FN(project_depth_)(const OR_T(or_fc_)* c, const REAL* p, int W, int H,
                                 REAL* u, REAL* v)
{
    if (!(p[2] > (REAL)0)) return 0;
    REAL iz = (REAL)1 / p[2];
    REAL x = FMA(c->fx, p[0] * iz, c->cx);
    REAL y = FMA(c->fy, p[1] * iz, c->cy);
    *u = RINT(x);
    *v = RINT(y);
    return *u >= (REAL)0 && *u <= (REAL)(W - 1) && *v >= (REAL)0 && *v <= (REAL)(H - 1);
}

/* TSDF update of one geometry voxel for one frame (Sec. III; projective signed
 * distance, truncated to +1 in front of the surface, not updated far behind it).
 * When apply is 0 the state is left untouched and only the status is returned. */
static int OR_FN(geom_voxel_)(const OR_T(or_fc_)* c, const float* D, int W, int H,
                              int i, int j, int k, REAL* F, REAL* Wg, int apply)
{
    REAL p[3], u, v;
    OR_FN(affine_)(c->Ag, c->bg, i, j, k, p);
    if (!OR_FN(project_depth_)(c, p, W, H, &u, &v)) return OR_ST_FRUSTUM;
    REAL d = (REAL)D[(size_t)(int)v * (size_t)W + (size_t)(int)u];
    if (!OR_FN(valid_depth_)(d)) return OR_ST_NODEPTH;
    REAL sdf = d - p[2];
    if (sdf < -c->trunc) return OR_ST_BAND;
    if (!apply) return OR_ST_UPDATED;
    REAL t = FMIN((REAL)1, sdf * c->inv_trunc);
    REAL wn = *Wg + (REAL)1;
    *F = *F + (t - *F) / wn;
    *Wg = FMIN(wn, c->w_max);
    return OR_ST_UPDATED;
}

/* One HD colour channel value as a REAL in [0,1]. */
static REAL OR_FN(hd_px_)(const uint8_t* rgb8, const float* rgbf, size_t idx)
{
    if (rgb8) return (REAL)rgb8[idx] * (REAL)(1.0 / 255.0);
    return (REAL)rgbf[idx];
}

static REAL OR_FN(lerp_)(REAL a, REAL b, REAL t) { return FMA(t, b - a, a); }

/* Eq. 7 at an integer depth pixel: D * K_c^-1 (u, v, 1). */
static void OR_FN(backproject_)(const OR_T(or_fc_)* c, REAL u, REAL v, REAL d, REAL* P)
{
    P[0] = ((u - c->cx) * c->inv_fx) * d;
    P[1] = ((v - c->cy) * c->inv_fy) * d;
    P[2] = d;
}

/* Everything the colour update of one voxel in one frame decides before touching the
 * state, plus where it samples the HD image.  Filled by colour_eval_. */
typedef struct {
    int status;       /* OR_ST_* (OR_ST_UPDATED when every test passes)         */
    int u, v;         /* nearest depth pixel (valid from OR_ST_NODEPTH on)       */
    REAL w;           /* normal-times-view weight W (Sec. IV.B, Eq. 8)           */
    REAL q[3];        /* voxel centre in HD camera coordinates (Eq. 5 then 3)    */
    REAL xh, yh;      /* HD image coordinates (Eq. 4 with perspective division) */
    int x0, y0;       /* top-left pixel of the bilinear cell, or the nearest pixel */
    REAL ax, ay;      /* bilinear fractions                                      */
    int nearest;      /* sample the single pixel (x0, y0)                        */
} OR_T(or_ceval_);

/* Colour-volume tests of Sec. IV.B in the paper's order: frustum, depth, distance
 * sigma, normal, gate against the current weight, then the HD pixel (Eq. 1-4). */
static void OR_FN(colour_eval_)(const OR_T(or_fc_)* c, const float* D, int W, int H,
                                int CW, int CH, int i, int j, int k, REAL Wc,
                                OR_T(or_ceval_)* e)
{
    REAL p[3], u, v, P[3], P1[3], P2[3];
    e->status = OR_ST_FRUSTUM;
    OR_FN(affine_)(c->Ac, c->bc, i, j, k, p);
    if (!OR_FN(project_depth_)(c, p, W, H, &u, &v)) return;
    size_t iu = (size_t)(int)u, iv = (size_t)(int)v;
    e->u = (int)u;
    e->v = (int)v;
    REAL d = (REAL)D[iv * (size_t)W + iu];
    e->status = OR_ST_NODEPTH;
    if (!OR_FN(valid_depth_)(d)) return;
    /* Eq. 7, then the Euclidean distance test against sigma. */
    OR_FN(backproject_)(c, u, v, d, P);
    REAL dx = p[0] - P[0], dy = p[1] - P[1], dz = p[2] - P[2];
    REAL dist2 = FMA(dx, dx, FMA(dy, dy, dz * dz));
    e->status = OR_ST_BAND;
    if (dist2 > c->sigma2) return;
    /* Eq. 8: neighbours (u+1, v) and (u, v+1) must exist and hold depth. */
    e->status = OR_ST_NORMAL;
    if (!(u + (REAL)1 <= (REAL)(W - 1) && v + (REAL)1 <= (REAL)(H - 1))) return;
    REAL d1 = (REAL)D[iv * (size_t)W + iu + 1];
    REAL d2 = (REAL)D[(iv + 1) * (size_t)W + iu];
    if (!OR_FN(valid_depth_)(d1) || !OR_FN(valid_depth_)(d2)) return;
    OR_FN(backproject_)(c, u + (REAL)1, v, d1, P1);
    OR_FN(backproject_)(c, u, v + (REAL)1, d2, P2);
    REAL e1x = P1[0] - P[0], e1y = P1[1] - P[1], e1z = P1[2] - P[2];
    REAL e2x = P2[0] - P[0], e2y = P2[1] - P[1], e2z = P2[2] - P[2];
    REAL Nx = FMA(e1y, e2z, -(e1z * e2y));
    REAL Ny = FMA(e1z, e2x, -(e1x * e2z));
    REAL Nz = FMA(e1x, e2y, -(e1y * e2x));
    REAL nn = FMA(Nx, Nx, FMA(Ny, Ny, Nz * Nz));
    if (!(nn > (REAL)0)) return;
    /* W = <N/|N|, P/|P|>: the viewing direction runs from the camera centre to P. */
    REAL pp = FMA(P[0], P[0], FMA(P[1], P[1], P[2] * P[2]));
    REAL dp = FMA(Nx, P[0], FMA(Ny, P[1], Nz * P[2]));
    e->w = dp / SQRT(nn * pp);
    e->status = OR_ST_GATE;
    if (!(e->w > c->gate * Wc)) return;
    /* Eq. 2-4 applied to the voxel centre, composed with Eq. 5. */
    e->status = OR_ST_HD;
    OR_FN(affine_)(c->Ah, c->bh, i, j, k, e->q);
    if (!(e->q[2] > (REAL)0)) return;
    REAL iqz = (REAL)1 / e->q[2];
    e->xh = FMA(c->fxr, e->q[0] * iqz, c->cxr);
    e->yh = FMA(c->fyr, e->q[1] * iqz, c->cyr);
    e->nearest = c->hd_nearest;
    if (c->hd_nearest) {
        /* the pixel whose centre is nearest (ties to even), inside the image */
        REAL rx = RINT(e->xh), ry = RINT(e->yh);
        if (!(rx >= (REAL)0 && rx <= (REAL)(CW - 1) && ry >= (REAL)0 && ry <= (REAL)(CH - 1)))
            return;
        e->x0 = (int)rx;
        e->y0 = (int)ry;
        e->ax = e->ay = (REAL)0;
        e->status = OR_ST_UPDATED;
        return;
    }
    REAL fx0 = FLOOR(e->xh), fy0 = FLOOR(e->yh);
    if (!(fx0 >= (REAL)0 && fx0 <= (REAL)(CW - 2) && fy0 >= (REAL)0 && fy0 <= (REAL)(CH - 2)))
        return;
    e->x0 = (int)fx0;
    e->y0 = (int)fy0;
    e->ax = e->xh - fx0;
    e->ay = e->yh - fy0;
    e->status = OR_ST_UPDATED;
}

/* Bilinear HD sample of one channel at the cell found by colour_eval_. */
static REAL OR_FN(hd_sample_)(const OR_T(or_ceval_)* e, const uint8_t* rgb8,
                              const float* rgbf, int CW, int ch)
{
    size_t r0 = (size_t)e->y0 * (size_t)CW, r1 = r0 + (size_t)CW;
    if (e->nearest) return OR_FN(hd_px_)(rgb8, rgbf, (r0 + (size_t)e->x0) * 3 + (size_t)ch);
    REAL p00 = OR_FN(hd_px_)(rgb8, rgbf, (r0 + (size_t)e->x0) * 3 + (size_t)ch);
    REAL p10 = OR_FN(hd_px_)(rgb8, rgbf, (r0 + (size_t)e->x0 + 1) * 3 + (size_t)ch);
    REAL p01 = OR_FN(hd_px_)(rgb8, rgbf, (r1 + (size_t)e->x0) * 3 + (size_t)ch);
    REAL p11 = OR_FN(hd_px_)(rgb8, rgbf, (r1 + (size_t)e->x0 + 1) * 3 + (size_t)ch);
    return OR_FN(lerp_)(OR_FN(lerp_)(p00, p10, e->ax), OR_FN(lerp_)(p01, p11, e->ax), e->ay);
}

/* Eq. 9 (as C + alpha (HD - C), alpha = W / (W_pre + W)) and Eq. 10. */
static void OR_FN(colour_apply_)(const OR_T(or_ceval_)* e, const uint8_t* rgb8,
                                 const float* rgbf, int CW, REAL* C3, REAL* Wc)
{
    REAL alpha = e->w / (*Wc + e->w);
    for (int ch = 0; ch < 3; ++ch) {
        REAL s = OR_FN(hd_sample_)(e, rgb8, rgbf, CW, ch);
        C3[ch] = FMA(alpha, s - C3[ch], C3[ch]);
    }
    *Wc = FMA(e->w, (REAL)1 - *Wc, *Wc);
}

/* Integrate frames [0, n_frames) into the voxels of z-slabs [gz0,gz1) (geometry) and
 * [cz0,cz1) (colour).  State arrays hold only those slabs (voxel (0,0,z0) first).
 * Frames are applied to each voxel in order; voxels are independent.  Optional
 * outputs: the status of the last frame per voxel, and byte-accounting counters for
 * passes of frames_per_pass frames (see kf_oracle.h). */
static void OR_FN(integrate_)(const or_volume* vol, const or_frames* fr, const or_fc64* fc64,
                              REAL* tsdf, REAL* wg, REAL* cr, REAL* cg, REAL* cb, REAL* wc,
                              int gz0, int gz1, int cz0, int cz1, int frames_per_pass,
                              int apply, uint8_t* gstatus, uint8_t* cstatus,
                              int64_t* counters)
{
    int n = fr->n_frames;
    OR_T(or_fc_)* fc = (OR_T(or_fc_)*)malloc(sizeof(OR_T(or_fc_)) * (size_t)(n > 0 ? n : 1));
    for (int f = 0; f < n; ++f) OR_FN(round_consts_)(&fc64[f], &fc[f]);
    int K = frames_per_pass > 0 ? frames_per_pass : 1;
    size_t dpix = (size_t)fr->dw * (size_t)fr->dh, cpix = (size_t)fr->cw * (size_t)fr->ch * 3;
    int64_t g_upd = 0, g_touch = 0, c_eval = 0, c_read = 0, c_upd = 0, c_touch = 0;

    int GX = vol->gdim[0], GY = vol->gdim[1];
    #pragma omp parallel for schedule(static) reduction(+:g_upd,g_touch)
    for (int k = gz0; k < gz1; ++k) {
        for (int j = 0; j < GY; ++j) {
            for (int i = 0; i < GX; ++i) {
                size_t idx = ((size_t)(k - gz0) * (size_t)GY + (size_t)j) * (size_t)GX + (size_t)i;
                REAL F = tsdf[idx], Wg = wg[idx];
                int touched = 0, st = OR_ST_FRUSTUM;
                for (int f = 0; f < n; ++f) {
                    if (f % K == 0) { g_touch += touched; touched = 0; }
                    st = OR_FN(geom_voxel_)(&fc[f], fr->depth + (size_t)f * dpix, fr->dw, fr->dh,
                                            i, j, k, &F, &Wg, apply);
                    if (st == OR_ST_UPDATED) { ++g_upd; touched = 1; }
                }
                g_touch += touched;
                if (apply) { tsdf[idx] = F; wg[idx] = Wg; }
                if (gstatus) gstatus[idx] = (uint8_t)st;
            }
        }
    }

    int CX = vol->cdim[0], CY = vol->cdim[1];
    #pragma omp parallel for schedule(static) reduction(+:c_eval,c_read,c_upd,c_touch)
    for (int k = cz0; k < cz1; ++k) {
        for (int j = 0; j < CY; ++j) {
            for (int i = 0; i < CX; ++i) {
                size_t idx = ((size_t)(k - cz0) * (size_t)CY + (size_t)j) * (size_t)CX + (size_t)i;
                REAL C3[3] = {cr[idx], cg[idx], cb[idx]}, W = wc[idx];
                int read = 0, touched = 0, st = OR_ST_FRUSTUM;
                for (int f = 0; f < n; ++f) {
                    if (f % K == 0) { c_read += read; c_touch += touched; read = touched = 0; }
                    OR_T(or_ceval_) e;
                    const uint8_t* rgb8 = fr->rgb8 ? fr->rgb8 + (size_t)f * cpix : NULL;
                    const float* rgbf = fr->rgbf ? fr->rgbf + (size_t)f * cpix : NULL;
                    OR_FN(colour_eval_)(&fc[f], fr->depth + (size_t)f * dpix, fr->dw, fr->dh,
                                        fr->cw, fr->ch, i, j, k, W, &e);
                    st = e.status;
                    if (st >= OR_ST_GATE) { ++c_eval; read = 1; }
                    if (st == OR_ST_UPDATED) {
                        ++c_upd; touched = 1;
                        if (apply) OR_FN(colour_apply_)(&e, rgb8, rgbf, fr->cw, C3, &W);
                    }
                }
                c_read += read;
                c_touch += touched;
                if (apply) { cr[idx] = C3[0]; cg[idx] = C3[1]; cb[idx] = C3[2]; wc[idx] = W; }
                if (cstatus) cstatus[idx] = (uint8_t)st;
            }
        }
    }
    if (counters) {
        counters[0] += g_upd;  counters[1] += g_touch;
        counters[2] += c_eval; counters[3] += c_read;
        counters[4] += c_upd;  counters[5] += c_touch;
    }
    free(fc);
}

#undef OR_FN
#undef OR_T
#undef OR_CAT
#undef OR_CAT2
