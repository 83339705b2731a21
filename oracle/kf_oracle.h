/*
 * Oracle for the per-frame volumetric integration of "Creating Simplified 3D Models
 * with High Quality Textures" (arXiv 1602.06645): the TSDF geometry volume of Sec. III
 * and the asymmetric colour volume of Sec. IV.B (Eq. 5-10) with the depth-to-HD-RGB
 * mapping of Sec. IV.A (Eq. 1-4), plus the adjoint of the colour update; ray casting of
 * the two volumes (Sec. III rendering); the per-polygon texture maps of Sec. IV.D
 * (Eq. 11-14) and their column-wise atlas; marching cubes and the quadric-error decimation
 * of the mesh (Sec. IV.C).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow CPU implementation that the test
 * suite, the smoke check and the benchmark's CPU-baseline leg compare the GPU library
 * against.  Nothing in the product library links, includes or calls it, and it shares
 * no code with the GPU path.
 *
 * Conventions (all arrays host memory, row-major):
 *   - volumes are dense, x fastest: index = x + X*(y + Y*z); voxel centres sit at
 *     origin + (i + 1/2) * extent/dim on each axis; geometry and colour volumes share
 *     origin and extent and differ in dimension (Sec. IV.B, asymmetric volume);
 *   - depth is float metres [n][H][W], 0 (or any non-positive / non-finite value) marks
 *     a hole; RGB is [n][CH][CW][3], either uint8 or float in [0,1];
 *   - K matrices are 3x3 with zero skew; poses are 4x4 rigid transforms:
 *     T_world_from_cam per frame, T_rgb_from_d = (R_calib | t_calib) of Eq. 3.
 */
#ifndef KF_ORACLE_H
#define KF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Per-voxel outcome of one frame, in the order the tests are made. */
enum {
    OR_ST_FRUSTUM = 0,  /* behind the camera or projects outside the depth image    */
    OR_ST_NODEPTH = 1,  /* the depth pixel is a hole                                */
    OR_ST_BAND = 2,     /* geometry: farther than trunc behind the surface;
                           colour: farther than sigma from the back-projected point */
    OR_ST_NORMAL = 3,   /* colour: no normal (neighbour missing or degenerate)       */
    OR_ST_GATE = 4,     /* colour: W does not exceed gate * W_pre                   */
    OR_ST_HD = 5,       /* colour: the HD sample falls outside the HD image         */
    OR_ST_UPDATED = 6
};

typedef struct {
    int32_t gdim[3], cdim[3];
    double origin[3], extent[3];
    double sigma;  /* colour distance threshold in metres (paper: 20 mm) */
    double gate;   /* colour weight gate factor (paper: 0.8)             */
    int32_t hd_nearest;  /* 1: the HD pixel nearest the projection; 0: bilinear */
} or_volume;

typedef struct {
    int32_t n_frames, dw, dh, cw, ch;
    const float* depth;            /* [n][dh][dw]                           */
    const uint8_t* rgb8;           /* [n][ch][cw][3] or NULL                */
    const float* rgbf;             /* [n][ch][cw][3] or NULL                */
    const double* K_d;             /* [9]                                   */
    const double* K_rgb;           /* [9]                                   */
    const double* T_rgb_from_d;    /* [16]                                  */
    const double* T_world_from_cam;/* [n][16]                               */
    double trunc, w_max;
} or_frames;

/* The per-frame constants in double, before rounding (exposed for tests). */
typedef struct {
    double Ag[9], bg[3], Ac[9], bc[3], Ah[9], bh[3];
    double fx, fy, cx, cy, inv_fx, inv_fy;
    double fxr, fyr, cxr, cyr;
    double trunc, inv_trunc, w_max, sigma2, gate;
    double hd_nearest;   /* 1.0 for nearest-pixel HD sampling, 0.0 for bilinear */
} or_fc64;

void or_frame_consts(const or_volume* vol, const or_frames* fr, int frame, or_fc64* out);

/* Threads the OpenMP loops of this library use. */
int or_num_threads(void);
void or_set_num_threads(int n);

/*
 * Forward integration in FP32 (or_integrate_f32) or FP64 (or_integrate_f64).
 * State arrays cover geometry z-slabs [gz0,gz1) and colour z-slabs [cz0,cz1) only.
 * apply = 0 leaves the state untouched (status-only).  gstatus/cstatus (optional)
 * receive the OR_ST_* code of the last frame for each voxel.  counters (optional,
 * int64[6], accumulated):
 *   [0] geometry updates (voxel-frames)
 *   [1] geometry voxels updated at least once per pass of frames_per_pass frames
 *   [2] colour voxel-frames reaching the gate (the colour weight is read)
 *   [3] colour voxels reaching the gate at least once per pass
 *   [4] colour updates (voxel-frames)
 *   [5] colour voxels updated at least once per pass
 */
void or_integrate_f32(const or_volume* vol, const or_frames* fr, float* tsdf, float* wg,
                      float* r, float* g, float* b, float* wc, int gz0, int gz1, int cz0,
                      int cz1, int frames_per_pass, int apply, uint8_t* gstatus,
                      uint8_t* cstatus, int64_t* counters);
void or_integrate_f64(const or_volume* vol, const or_frames* fr, double* tsdf, double* wg,
                      double* r, double* g, double* b, double* wc, int gz0, int gz1, int cz0,
                      int cz1, int frames_per_pass, int apply, uint8_t* gstatus,
                      uint8_t* cstatus, int64_t* counters);

/*
 * Adjoint of the colour volume after all frames, in FP64, for the functional
 * L = sum_v sum_ch g[ch][v] * C_N(v)_ch over colour z-slabs [cz0,cz1) (g covers those
 * slabs only).  Starts from colour weights wc0 (NULL = zero).  Requires fr->rgbf.
 * Writes dL/dRGB into d_rgb ([n][ch][cw][3], overwritten) and dL/dxi into d_xi[6],
 * xi = (rho, phi) a left perturbation T_rgb_from_d <- exp(xi^) T_rgb_from_d at xi = 0.
 * decide_f32 = 0: every step in FP64 (the adjoint of the FP64 forward).
 * decide_f32 = 1: the integer decisions (depth pixel, the tests of Sec. IV.B, the
 * bilinear cell) are those of the FP32 forward; the values stay FP64.
 * d_pose (NULL to skip): [n][6], dL/dxi_n for the depth-camera poses, xi_n = (rho, phi) a
 * left perturbation in world coordinates T_world_from_cam[n] <- exp(xi_n^) T_world_from_cam[n]
 * at xi_n = 0, with the integer decisions held (the derivative wherever no decision
 * changes): only the HD sample position of each update moves with the pose.
 * Defined for bilinear HD sampling only (vol->hd_nearest == 0); otherwise nothing is
 * written.
 */
void or_backward_f64(const or_volume* vol, const or_frames* fr, const double* wc0,
                     const double* g, int cz0, int cz1, int decide_f32, double* d_rgb,
                     double* d_xi, double* d_pose);

/*
 * Ray casting of the volumes (the rendering the method uses for live feedback and the
 * predicted surface of tracking; abstract and Sec. III).  The constants of one camera,
 * in double before rounding: geometry- and colour-index rays q = a + t (Bu x + Bv y + B0),
 * the world ray p = tw + t (Ru x + Rv y + R0) (t = camera depth), 1 / voxel size, dim - 1
 * and the sample spacing delta (metres of camera depth).
 */
typedef struct {
    double a[3], Bu[3], Bv[3], B0[3];
    double ac[3], Bcu[3], Bcv[3], Bc0[3];
    double Ru[3], Rv[3], R0[3], tw[3];
    double inv_s[3], gmax[3], cmax[3];
    double delta;
} or_rc64;

void or_raycast_consts(const or_volume* vol, const double* K, const double* T_world_from_cam,
                       double delta, or_rc64* out);

/*
 * Ray cast the pixels pixels[0..n_pix) (index y * width + x) of a camera with intrinsics K
 * and pose T_world_from_cam through the whole volume (tsdf, wg over gdim; r, g, b, wc over
 * cdim).  Per pixel p: depth[p] (0 = miss), vertex[3p..3p+2] (world), normal[3p..] and
 * colour[3p..] (zeros when missing).  Steps in kf_raycast_body.h.
 */
void or_raycast_f32(const or_volume* vol, const float* tsdf, const float* wg, const float* r,
                    const float* g, const float* b, const float* wc, const double* K,
                    const double* T_world_from_cam, double delta, int width,
                    const int32_t* pixels, int64_t n_pix, float* depth, float* vertex,
                    float* normal, float* colour);
void or_raycast_f64(const or_volume* vol, const float* tsdf, const float* wg, const float* r,
                    const float* g, const float* b, const float* wc, const double* K,
                    const double* T_world_from_cam, double delta, int width,
                    const int32_t* pixels, int64_t n_pix, float* depth, float* vertex,
                    float* normal, float* colour);

/*
 * Per-polygon texture maps and their atlas (Sec. IV.D, Eq. 11-14 and the merging scheme).
 * tri: [n][3][3] world vertices (V1, V2, V3) of each triangle.  Layout (double, host):
 * w = max(2, ceil(|V1V2| / size_pixel)), h = max(2, ceil(|V1V3| / size_pixel)); the maps
 * are placed down a column of an atlas of atlas_height texels, top to bottom, and a new
 * column starts to the right (at the widest map of the previous column) when the next map
 * does not fit below.  rects[4n..4n+3] = (x, y, w, h); returns the atlas width, or -1 when a
 * map is taller than the atlas or a size exceeds 65535.
 */
int32_t or_texture_layout(int32_t n_tri, const float* tri, double size_pixel,
                          int32_t atlas_height, int32_t* rects);

/*
 * Texel colours: texel (i, j) of triangle n (i < w towards V2, j < h towards V3) is the
 * world point V1 + i (V2 - V1)/(w - 1) + j (V3 - V1)/(h - 1) (Eq. 13-14), coloured by
 * trilinear interpolation of the colour volume (zero unless the 8 corner colour weights are
 * positive).  Writes atlas[(y + j) * atlas_width + x + i][3] (float) and, if atlas8 is not
 * NULL, rint(255 * min(max(c, 0), 1)) as bytes; other texels are untouched.
 */
void or_texture_generate_f32(const or_volume* vol, const float* r, const float* g,
                             const float* b, const float* wc, int32_t n_tri, const float* tri,
                             const int32_t* rects, int32_t atlas_width, float* atlas,
                             uint8_t* atlas8);
void or_texture_generate_f64(const or_volume* vol, const float* r, const float* g,
                             const float* b, const float* wc, int32_t n_tri, const float* tri,
                             const int32_t* rects, int32_t atlas_width, float* atlas,
                             uint8_t* atlas8);

/*
 * Marching cubes of the geometry volume (the mesh extraction of Sec. III, after
 * KinectFusion; the definition is in kf_mesh_body.h).  tsdf, wg: [Z][Y][X] floats (host).
 * Writes up to vcap vertices (world, [n][3]: vert32 in FP32 with the canonical operation
 * order, vert64 in FP64; either may be NULL) and up to tcap triangles ([n][3] vertex
 * indices); *n_vert and *n_tri receive the full counts.  Returns -1 when they exceed the
 * capacities (call with zero capacities to size the outputs), else 0.
 */
int or_marching_cubes(const or_volume* vol, const float* tsdf, const float* wg, float* vert32,
                      double* vert64, int64_t vcap, int32_t* tris, int64_t tcap, int64_t* n_vert,
                      int64_t* n_tri);

/* Triangles (as cube edge ids, [n][3]) of one cube whose inside corners are the set bits of
 * inside_mask (corner c = x + 2y + 4z); returns n. */
int or_mc_cube_triangles(unsigned inside_mask, int32_t* tri_edges);

/*
 * Quadric-error decimation (Sec. IV.C, the reduction rate of Fig. 3; the definition is in
 * kf_decimate_body.h): vin [nv][3], tin [nt][3] (CCW) in; writes the kept vertices (vout,
 * at most nv) and triangles (tout, at most nt; either output may be NULL) and their counts.
 * Returns the triangle count, or -1 for an index out of range or a triangle repeating a
 * vertex.
 */
int64_t or_decimate(const float* vin, int64_t nv, const int32_t* tin, int64_t nt, double rate,
                    float* vout, int64_t* nv_out, int32_t* tout, int64_t* nt_out);

#ifdef __cplusplus
}
#endif
#endif
