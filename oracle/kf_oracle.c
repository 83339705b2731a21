/*
 * Oracle for the volumetric integration of arXiv 1602.06645 (Sec. III, Sec. IV.A-B), the
 * ray casting of its volumes and the per-polygon texture maps of Sec. IV.D (Eq. 11-14).
 *
 * TEST INFRASTRUCTURE ONLY: a plain CPU implementation used by the tests, the smoke
 * check and the benchmark's CPU-baseline leg.  The product library never links or calls
 * it.  Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math), so that
 * every multiply, add, fma, division and square root is the IEEE operation written.
 *
 * The FP32 instance is the parity reference: its masks and weights are exact targets.
 * The FP64 instance and the adjoint serve the finite-difference and closed-form checks.
 */
#include "kf_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

int or_num_threads(void) { return omp_get_max_threads(); }

/* Threads of the OpenMP loops from now on (timing on a given number of cores). */
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* ---- per-frame constants, double precision (Eq. 3 and Eq. 5 folded into affine maps) */

/* 4x4 row-major rigid transform -> R (3x3) and t (3). */
static void split_rt(const double* T, double* R, double* t)
{
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R[3 * r + c] = T[4 * r + c];
        t[r] = T[4 * r + 3];
    }
}

/* Voxel index (i,j,k) -> R (origin + (idx + 1/2) s) + t, as A idx + b with A = R diag(s). */
static void fold_voxel_map(const double* R, const double* t, const double* origin,
                           const double* s, double* A, double* b)
{
    double c0 = origin[0] + 0.5 * s[0];
    double c1 = origin[1] + 0.5 * s[1];
    double c2 = origin[2] + 0.5 * s[2];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) A[3 * r + c] = R[3 * r + c] * s[c];
        b[r] = ((R[3 * r + 0] * c0 + R[3 * r + 1] * c1) + R[3 * r + 2] * c2) + t[r];
    }
}

void or_frame_consts(const or_volume* vol, const or_frames* fr, int frame, or_fc64* out)
{
    double Rwc[9], twc[3], Rcw[9], tcw[3];
    split_rt(fr->T_world_from_cam + 16 * (size_t)frame, Rwc, twc);
    /* (R_n, t_n) of Eq. 5 maps world (first-frame) coordinates into the current depth
     * camera: the inverse of the camera pose. */
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) Rcw[3 * r + c] = Rwc[3 * c + r];
        tcw[r] = -((Rwc[0 + r] * twc[0] + Rwc[3 + r] * twc[1]) + Rwc[6 + r] * twc[2]);
    }
    /* Eq. 3: HD camera coordinates = R_calib * depth camera coordinates + t_calib. */
    double Rrd[9], trd[3], Rhw[9], thw[3];
    split_rt(fr->T_rgb_from_d, Rrd, trd);
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            Rhw[3 * r + c] = (Rrd[3 * r + 0] * Rcw[0 + c] + Rrd[3 * r + 1] * Rcw[3 + c])
                             + Rrd[3 * r + 2] * Rcw[6 + c];
        thw[r] = ((Rrd[3 * r + 0] * tcw[0] + Rrd[3 * r + 1] * tcw[1]) + Rrd[3 * r + 2] * tcw[2])
                 + trd[r];
    }
    double sg[3], sc[3];
    for (int a = 0; a < 3; ++a) {
        sg[a] = vol->extent[a] / (double)vol->gdim[a];
        sc[a] = vol->extent[a] / (double)vol->cdim[a];
    }
    fold_voxel_map(Rcw, tcw, vol->origin, sg, out->Ag, out->bg);
    fold_voxel_map(Rcw, tcw, vol->origin, sc, out->Ac, out->bc);
    fold_voxel_map(Rhw, thw, vol->origin, sc, out->Ah, out->bh);
    out->fx = fr->K_d[0];
    out->fy = fr->K_d[4];
    out->cx = fr->K_d[2];
    out->cy = fr->K_d[5];
    out->inv_fx = 1.0 / fr->K_d[0];
    out->inv_fy = 1.0 / fr->K_d[4];
    out->fxr = fr->K_rgb[0];
    out->fyr = fr->K_rgb[4];
    out->cxr = fr->K_rgb[2];
    out->cyr = fr->K_rgb[5];
    out->trunc = fr->trunc;
    out->inv_trunc = 1.0 / fr->trunc;
    out->w_max = fr->w_max;
    out->sigma2 = vol->sigma * vol->sigma;
    out->gate = vol->gate;
    out->hd_nearest = vol->hd_nearest ? 1.0 : 0.0;
}

static or_fc64* all_consts(const or_volume* vol, const or_frames* fr)
{
    int n = fr->n_frames > 0 ? fr->n_frames : 1;
    or_fc64* fc = (or_fc64*)calloc((size_t)n, sizeof(or_fc64));
    for (int f = 0; f < fr->n_frames; ++f) or_frame_consts(vol, fr, f, &fc[f]);
    return fc;
}

/* ---- the per-voxel steps, instantiated in single and double precision */

#define REAL float
#define SFX _f32
#define FMA fmaf
#define SQRT sqrtf
#define RINT rintf
#define FLOOR floorf
#define FMIN fminf
#include "kf_oracle_body.h"
#undef REAL
#undef SFX
#undef FMA
#undef SQRT
#undef RINT
#undef FLOOR
#undef FMIN

#define REAL double
#define SFX _f64
#define FMA fma
#define SQRT sqrt
#define RINT rint
#define FLOOR floor
#define FMIN fmin
#include "kf_oracle_body.h"
#undef REAL
#undef SFX
#undef FMA
#undef SQRT
#undef RINT
#undef FLOOR
#undef FMIN

void or_integrate_f32(const or_volume* vol, const or_frames* fr, float* tsdf, float* wg,
                      float* r, float* g, float* b, float* wc, int gz0, int gz1, int cz0,
                      int cz1, int frames_per_pass, int apply, uint8_t* gstatus,
                      uint8_t* cstatus, int64_t* counters)
{
    or_fc64* fc = all_consts(vol, fr);
    integrate__f32(vol, fr, fc, tsdf, wg, r, g, b, wc, gz0, gz1, cz0, cz1, frames_per_pass,
                   apply, gstatus, cstatus, counters);
    free(fc);
}

void or_integrate_f64(const or_volume* vol, const or_frames* fr, double* tsdf, double* wg,
                      double* r, double* g, double* b, double* wc, int gz0, int gz1, int cz0,
                      int cz1, int frames_per_pass, int apply, uint8_t* gstatus,
                      uint8_t* cstatus, int64_t* counters)
{
    or_fc64* fc = all_consts(vol, fr);
    integrate__f64(vol, fr, fc, tsdf, wg, r, g, b, wc, gz0, gz1, cz0, cz1, frames_per_pass,
                   apply, gstatus, cstatus, counters);
    free(fc);
}

/* ---- adjoint of the colour update (FP64)
 *
 * Eq. 9 is C_n = (1 - alpha_n) C_{n-1} + alpha_n s_n with alpha_n = W / (W_pre + W) in
 * frames that update the voxel (0 otherwise), and Eq. 10 makes the weights independent
 * of the HD image.  Hence C_N = sum_n beta_n s_n + prod_n (1 - alpha_n) C_0 with
 * beta_n = alpha_n prod_{m>n} (1 - alpha_m); s_n is the bilinear HD sample at the
 * projection (Eq. 2-4) of the voxel centre, which depends on T_rgb_from_d = (R_calib,
 * t_calib).  The weights depend on T_rgb_from_d only through the HD bounds test.
 */
/* FP64 values of one colour update whose integer decisions (depth pixel (u,v), bilinear
 * cell (x0,y0)) were taken elsewhere: the weight W of Eq. 8 and the HD-camera point q
 * with its image coordinates (Eq. 2-5). */
static void colour_values_f64(const or_fc__f64* c, const float* D, int W, int u, int v,
                              int i, int j, int k, or_ceval__f64* e)
{
    double P[3], P1[3], P2[3];
    size_t pix = (size_t)v * (size_t)W + (size_t)u;
    backproject__f64(c, (double)u, (double)v, (double)D[pix], P);
    backproject__f64(c, (double)u + 1.0, (double)v, (double)D[pix + 1], P1);
    backproject__f64(c, (double)u, (double)v + 1.0, (double)D[pix + (size_t)W], P2);
    double e1[3] = {P1[0] - P[0], P1[1] - P[1], P1[2] - P[2]};
    double e2[3] = {P2[0] - P[0], P2[1] - P[1], P2[2] - P[2]};
    double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                   e1[0] * e2[1] - e1[1] * e2[0]};
    double nn = N[0] * N[0] + N[1] * N[1] + N[2] * N[2];
    double pp = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
    e->w = (N[0] * P[0] + N[1] * P[1] + N[2] * P[2]) / sqrt(nn * pp);
    affine__f64(c->Ah, c->bh, i, j, k, e->q);
    e->xh = c->fxr * (e->q[0] / e->q[2]) + c->cxr;
    e->yh = c->fyr * (e->q[1] / e->q[2]) + c->cyr;
    e->ax = e->xh - (double)e->x0;
    e->ay = e->yh - (double)e->y0;
}

void or_backward_f64(const or_volume* vol, const or_frames* fr, const double* wc0,
                     const double* g, int cz0, int cz1, int decide_f32, double* d_rgb,
                     double* d_xi, double* d_pose)
{
    if (vol->hd_nearest) return;
    /* world -> HD camera rotation of each frame, R_rd R_wc^T, for the pose gradient */
    double* Rqw = (double*)calloc((size_t)(fr->n_frames > 0 ? fr->n_frames : 1) * 9, sizeof(double));
    for (int f = 0; f < fr->n_frames; ++f) {
        const double* Tw = fr->T_world_from_cam + 16 * (size_t)f;
        const double* Td = fr->T_rgb_from_d;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int m = 0; m < 3; ++m) acc += Td[4 * r + m] * Tw[4 * c + m];   /* R_wc^T[m][c] */
                Rqw[9 * f + 3 * r + c] = acc;
            }
    }
    if (d_pose) memset(d_pose, 0, sizeof(double) * 6 * (size_t)(fr->n_frames > 0 ? fr->n_frames : 0));
    double cs[3];
    for (int q = 0; q < 3; ++q) cs[q] = vol->extent[q] / vol->cdim[q];
    int n = fr->n_frames;
    or_fc64* fc64 = all_consts(vol, fr);
    or_fc__f64* fc = (or_fc__f64*)malloc(sizeof(or_fc__f64) * (size_t)(n > 0 ? n : 1));
    or_fc__f32* fc32 = (or_fc__f32*)malloc(sizeof(or_fc__f32) * (size_t)(n > 0 ? n : 1));
    for (int f = 0; f < n; ++f) {
        round_consts__f64(&fc64[f], &fc[f]);
        round_consts__f32(&fc64[f], &fc32[f]);
    }
    size_t dpix = (size_t)fr->dw * (size_t)fr->dh;
    size_t cpix = (size_t)fr->cw * (size_t)fr->ch * 3;
    memset(d_rgb, 0, sizeof(double) * cpix * (size_t)(n > 0 ? n : 0));
    double xi0 = 0, xi1 = 0, xi2 = 0, xi3 = 0, xi4 = 0, xi5 = 0;
    int CX = vol->cdim[0], CY = vol->cdim[1];
    size_t nslab = (size_t)CX * (size_t)CY * (size_t)(cz1 - cz0);

    #pragma omp parallel reduction(+:xi0,xi1,xi2,xi3,xi4,xi5)
    {
        or_ceval__f64* ev = (or_ceval__f64*)malloc(sizeof(or_ceval__f64) * (size_t)(n > 0 ? n : 1));
        double* alpha = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        #pragma omp for schedule(static)
        for (int k = cz0; k < cz1; ++k) {
            for (int j = 0; j < CY; ++j) {
                for (int i = 0; i < CX; ++i) {
                    size_t idx = ((size_t)(k - cz0) * (size_t)CY + (size_t)j) * (size_t)CX + (size_t)i;
                    double gv[3] = {g[idx], g[nslab + idx], g[2 * nslab + idx]};
                    if (gv[0] == 0.0 && gv[1] == 0.0 && gv[2] == 0.0) continue;
                    /* forward replay: which frames update the voxel, and alpha_n */
                    double W = wc0 ? wc0[idx] : 0.0;
                    float W32 = (float)W;
                    for (int f = 0; f < n; ++f) {
                        const float* Df = fr->depth + (size_t)f * dpix;
                        if (decide_f32) {
                            /* the decisions of the single-precision forward */
                            or_ceval__f32 e32;
                            colour_eval__f32(&fc32[f], Df, fr->dw, fr->dh, fr->cw, fr->ch, i, j, k,
                                             W32, &e32);
                            ev[f].status = e32.status;
                            if (e32.status == OR_ST_UPDATED) {
                                W32 = fmaf(e32.w, 1.0f - W32, W32);
                                ev[f].x0 = e32.x0;
                                ev[f].y0 = e32.y0;
                                colour_values_f64(&fc[f], Df, fr->dw, e32.u, e32.v, i, j, k, &ev[f]);
                            }
                        } else {
                            colour_eval__f64(&fc[f], Df, fr->dw, fr->dh, fr->cw, fr->ch, i, j, k,
                                             W, &ev[f]);
                        }
                        alpha[f] = 0.0;
                        if (ev[f].status == OR_ST_UPDATED) {
                            alpha[f] = ev[f].w / (W + ev[f].w);
                            W = fma(ev[f].w, 1.0 - W, W);
                        }
                    }
                    /* reverse sweep: beta_n = alpha_n prod_{m>n} (1 - alpha_m) */
                    double tail = 1.0;
                    for (int f = n - 1; f >= 0; --f) {
                        if (ev[f].status != OR_ST_UPDATED) continue;
                        double beta = alpha[f] * tail;
                        tail *= 1.0 - alpha[f];
                        const or_ceval__f64* e = &ev[f];
                        const float* img = fr->rgbf + (size_t)f * cpix;
                        double* dimg = d_rgb + (size_t)f * cpix;
                        double ax = e->ax, ay = e->ay;
                        double wts[4] = {(1 - ax) * (1 - ay), ax * (1 - ay), (1 - ax) * ay, ax * ay};
                        size_t px[4];
                        px[0] = ((size_t)e->y0 * (size_t)fr->cw + (size_t)e->x0) * 3;
                        px[1] = px[0] + 3;
                        px[2] = px[0] + (size_t)fr->cw * 3;
                        px[3] = px[2] + 3;
                        double iqz = 1.0 / e->q[2];
                        double a[3] = {0, 0, 0};
                        for (int ch = 0; ch < 3; ++ch) {
                            double gb = gv[ch] * beta;
                            if (gb == 0.0) continue;
                            for (int q = 0; q < 4; ++q) {
                                #pragma omp atomic
                                dimg[px[q] + (size_t)ch] += gb * wts[q];
                            }
                            double p00 = img[px[0] + ch], p10 = img[px[1] + ch];
                            double p01 = img[px[2] + ch], p11 = img[px[3] + ch];
                            double dsx = (1 - ay) * (p10 - p00) + ay * (p11 - p01);
                            double dsy = (1 - ax) * (p01 - p00) + ax * (p11 - p10);
                            /* chain through the pinhole projection (Eq. 4 / z) */
                            a[0] += gb * dsx * fc[f].fxr * iqz;
                            a[1] += gb * dsy * fc[f].fyr * iqz;
                            a[2] += -gb * (dsx * fc[f].fxr * e->q[0] + dsy * fc[f].fyr * e->q[1])
                                    * iqz * iqz;
                        }
                        /* dq/d(rho, phi) = [I | -[q]x]  =>  d(phi) += q x a */
                        xi0 += a[0];
                        xi1 += a[1];
                        xi2 += a[2];
                        xi3 += e->q[1] * a[2] - e->q[2] * a[1];
                        xi4 += e->q[2] * a[0] - e->q[0] * a[2];
                        xi5 += e->q[0] * a[1] - e->q[1] * a[0];
                        if (d_pose) {
                            /* T_world_from_cam <- exp(xi) T_world_from_cam moves the voxel's
                             * camera point by -R_cw (rho + phi x p_w), so dq = -R_qw (rho +
                             * phi x p_w): with b = R_qw^T a, dL/drho = -b, dL/dphi = b x p_w */
                            const double* R = Rqw + 9 * (size_t)f;
                            double b[3], pw[3];
                            for (int m = 0; m < 3; ++m)
                                b[m] = R[m] * a[0] + R[3 + m] * a[1] + R[6 + m] * a[2];
                            pw[0] = vol->origin[0] + ((double)i + 0.5) * cs[0];
                            pw[1] = vol->origin[1] + ((double)j + 0.5) * cs[1];
                            pw[2] = vol->origin[2] + ((double)k + 0.5) * cs[2];
                            double* dp = d_pose + 6 * (size_t)f;
                            const double v6[6] = {-b[0], -b[1], -b[2], b[1] * pw[2] - b[2] * pw[1],
                                                  b[2] * pw[0] - b[0] * pw[2], b[0] * pw[1] - b[1] * pw[0]};
                            for (int m = 0; m < 6; ++m) {
                                #pragma omp atomic
                                dp[m] += v6[m];
                            }
                        }
                    }
                }
            }
        }
        free(ev);
        free(alpha);
    }
    d_xi[0] = xi0; d_xi[1] = xi1; d_xi[2] = xi2;
    d_xi[3] = xi3; d_xi[4] = xi4; d_xi[5] = xi5;
    free(fc);
    free(fc32);
    free(fc64);
    free(Rqw);
}

/* ---- ray casting (see kf_raycast_body.h for the steps) */

void or_raycast_consts(const or_volume* vol, const double* K, const double* T_world_from_cam,
                       double delta, or_rc64* out)
{
    const double fx = K[0], fy = K[4], cx = K[2], cy = K[5];
    double R[9], t[3];
    split_rt(T_world_from_cam, R, t);
    for (int k = 0; k < 3; ++k) {
        const double s = vol->extent[k] / vol->gdim[k];
        const double sc = vol->extent[k] / vol->cdim[k];
        /* world direction of pixel (x, y) at unit depth: R ((x - cx)/fx, (y - cy)/fy, 1) */
        const double ru = R[3 * k + 0] / fx, rv = R[3 * k + 1] / fy;
        const double r0 = (R[3 * k + 2] - R[3 * k + 0] * cx / fx) - R[3 * k + 1] * cy / fy;
        out->Ru[k] = ru;
        out->Rv[k] = rv;
        out->R0[k] = r0;
        out->tw[k] = t[k];
        /* index coordinates: (p - origin) / s - 1/2 puts voxel i's centre at i */
        out->a[k] = (t[k] - vol->origin[k]) / s - 0.5;
        out->Bu[k] = ru / s;
        out->Bv[k] = rv / s;
        out->B0[k] = r0 / s;
        out->ac[k] = (t[k] - vol->origin[k]) / sc - 0.5;
        out->Bcu[k] = ru / sc;
        out->Bcv[k] = rv / sc;
        out->Bc0[k] = r0 / sc;
        out->inv_s[k] = 1.0 / s;
        out->gmax[k] = (double)(vol->gdim[k] - 1);
        out->cmax[k] = (double)(vol->cdim[k] - 1);
    }
    out->delta = delta;
}

#define REAL float
#define SFX _f32
#define FMA fmaf
#define SQRT sqrtf
#define FLOOR floorf
#define CEIL ceilf
#define FMIN fminf
#define FMAX fmaxf
#include "kf_raycast_body.h"
#undef REAL
#undef SFX
#undef FMA
#undef SQRT
#undef FLOOR
#undef CEIL
#undef FMIN
#undef FMAX

#define REAL double
#define SFX _f64
#define FMA fma
#define SQRT sqrt
#define FLOOR floor
#define CEIL ceil
#define FMIN fmin
#define FMAX fmax
#include "kf_raycast_body.h"
#undef REAL
#undef SFX
#undef FMA
#undef SQRT
#undef FLOOR
#undef CEIL
#undef FMIN
#undef FMAX

void or_raycast_f32(const or_volume* vol, const float* tsdf, const float* wg, const float* r,
                    const float* g, const float* b, const float* wc, const double* K,
                    const double* T_world_from_cam, double delta, int width,
                    const int32_t* pixels, int64_t n_pix, float* depth, float* vertex,
                    float* normal, float* colour)
{
    or_rc64 c;
    or_raycast_consts(vol, K, T_world_from_cam, delta, &c);
    raycast__f32(vol, &c, tsdf, wg, r, g, b, wc, width, pixels, n_pix, depth, vertex, normal,
                 colour);
}

void or_raycast_f64(const or_volume* vol, const float* tsdf, const float* wg, const float* r,
                    const float* g, const float* b, const float* wc, const double* K,
                    const double* T_world_from_cam, double delta, int width,
                    const int32_t* pixels, int64_t n_pix, float* depth, float* vertex,
                    float* normal, float* colour)
{
    or_rc64 c;
    or_raycast_consts(vol, K, T_world_from_cam, delta, &c);
    raycast__f64(vol, &c, tsdf, wg, r, g, b, wc, width, pixels, n_pix, depth, vertex, normal,
                 colour);
}

/* ---- per-polygon texture maps and their atlas (see kf_texture_body.h) */

int32_t or_texture_layout(int32_t n_tri, const float* tri, double size_pixel,
                          int32_t atlas_height, int32_t* rects)
{
    int32_t col_x = 0, col_w = 0, y = 0;
    for (int32_t n = 0; n < n_tri; ++n) {
        const float* V = tri + 9 * (size_t)n;
        double d12 = 0.0, d13 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double e1 = (double)V[3 + k] - (double)V[k];
            const double e2 = (double)V[6 + k] - (double)V[k];
            d12 += e1 * e1;
            d13 += e2 * e2;
        }
        /* Eq. 11-12, rounded up to whole texels, at least 2 (Eq. 13-14 divide by w-1, h-1) */
        const double wf = ceil(sqrt(d12) / size_pixel), hf = ceil(sqrt(d13) / size_pixel);
        if (!(wf <= 65535.0) || !(hf <= 65535.0)) return -1;
        const int32_t w = wf < 2.0 ? 2 : (int32_t)wf;
        const int32_t h = hf < 2.0 ? 2 : (int32_t)hf;
        if (h > atlas_height) return -1;
        if (y + h > atlas_height) {   /* the column is full: start the next one */
            col_x += col_w;
            col_w = 0;
            y = 0;
        }
        rects[4 * n] = col_x;
        rects[4 * n + 1] = y;
        rects[4 * n + 2] = w;
        rects[4 * n + 3] = h;
        y += h;
        if (w > col_w) col_w = w;
    }
    return col_x + col_w;
}

#define REAL float
#define SFX _f32
#define FMA fmaf
#define FLOOR floorf
#define FMIN fminf
#define FMAX fmaxf
#define RINT rintf
#include "kf_texture_body.h"
#undef REAL
#undef SFX
#undef FMA
#undef FLOOR
#undef FMIN
#undef FMAX
#undef RINT

#define REAL double
#define SFX _f64
#define FMA fma
#define FLOOR floor
#define FMIN fmin
#define FMAX fmax
#define RINT rint
#include "kf_texture_body.h"
#undef REAL
#undef SFX
#undef FMA
#undef FLOOR
#undef FMIN
#undef FMAX
#undef RINT

void or_texture_generate_f32(const or_volume* vol, const float* r, const float* g,
                             const float* b, const float* wc, int32_t n_tri, const float* tri,
                             const int32_t* rects, int32_t atlas_width, float* atlas,
                             uint8_t* atlas8)
{
    texture__f32(vol, r, g, b, wc, n_tri, tri, rects, atlas_width, atlas, atlas8);
}

void or_texture_generate_f64(const or_volume* vol, const float* r, const float* g,
                             const float* b, const float* wc, int32_t n_tri, const float* tri,
                             const int32_t* rects, int32_t atlas_width, float* atlas,
                             uint8_t* atlas8)
{
    texture__f64(vol, r, g, b, wc, n_tri, tri, rects, atlas_width, atlas, atlas8);
}

/* ---- marching cubes of the geometry volume (see kf_mesh_body.h) */
#include "kf_mesh_body.h"

int or_mc_cube_triangles(unsigned inside_mask, int32_t* tri_edges)
{
    int t[12][3];
    const int n = mc_cube_triangles(inside_mask, t);
    for (int i = 0; i < n; ++i)
        for (int v = 0; v < 3; ++v) tri_edges[3 * i + v] = t[i][v];
    return n;
}

/* ---- quadric-error decimation of a triangle mesh (see kf_decimate_body.h) */
#include "kf_decimate_body.h"
