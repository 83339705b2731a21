/*
 * libkfvol: per-frame volumetric integration for RGB-D scanning with an HD colour
 * camera, on AMD Instinct MI355X (gfx950).
 *
 * Implements the integration step of "Creating Simplified 3D Models with High Quality
 * Textures" (arXiv 1602.06645):
 *   - the TSDF geometry volume the method inherits from KinectFusion (Sec. III): every
 *     voxel is projected into the depth map and its truncated signed distance and weight
 *     are updated by running average;
 *   - the asymmetric colour volume of Sec. IV.B (Eq. 5-10): a volume over the same cube
 *     with more voxels per axis; every colour voxel near the observed surface is weighted
 *     by the cosine between the surface normal (Eq. 8) and the viewing ray, gated against
 *     its previous weight, and blended with the HD image sample found through the
 *     depth-to-HD calibration of Sec. IV.A (Eq. 1-4).
 *
 * Arithmetic: every decision is taken in IEEE single precision with a fixed sequence of
 * operations (fused multiply-adds where written, correctly rounded division and square
 * root, round-half-to-even pixel rounding), so masks and weights are reproducible
 * bit for bit on any IEEE machine.
 *
 * Memory: every image and volume pointer below is a DEVICE pointer owned by the caller;
 * it must stay valid until the work enqueued on `stream` has completed.  Matrices and
 * poses are HOST arrays of doubles, row-major, read during the call.  `stream` is a
 * hipStream_t (NULL = the null stream).  All calls are asynchronous unless stated
 * otherwise: argument errors are returned before anything is enqueued; launch errors
 * return KF_E_DEVICE; faults inside kernels surface at the caller's synchronisation.
 * A volume handle may be used by one stream at a time.  Per voxel, frames are applied in
 * call order and, within a batch, in array order.
 */
#ifndef KF_H
#define KF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KF_OK = 0,
    KF_E_ARG = 1,          /* NULL pointer, non-finite or out-of-domain parameter        */
    KF_E_SHAPE = 2,        /* inconsistent or unsupported sizes                          */
    KF_E_RANGE = 3,        /* sizes beyond what the library indexes (e.g. > 2^31 voxels) */
    KF_E_DEVICE = 4,       /* a HIP call failed; see kf_last_error()                     */
    KF_E_UNSUPPORTED = 5   /* valid request the library does not implement              */
} kf_status;

typedef enum {
    KF_RGB8 = 0,   /* uint8 HWC, value / 255 is the colour in [0,1]          */
    KF_RGBF32 = 1  /* float32 HWC, colour in [0,1] (any finite value works)  */
} kf_pixfmt;

/* How the colour update reads the HD image at the projection (x_hd, y_hd) of a colour
 * voxel centre (Eq. 9).  Bilinear: between the four surrounding pixel centres (both must
 * lie in the image: 0 <= floor(x_hd) <= CW-2, likewise y); the adjoint is defined for it.
 * Nearest: the pixel whose centre is nearest (rint, ties to even), inside the image
 * (0 <= rint(x_hd) <= CW-1, likewise y); the adjoint returns KF_E_UNSUPPORTED for it. */
typedef enum {
    KF_HD_BILINEAR = 0,
    KF_HD_NEAREST = 1
} kf_hd_sampling;

/* Volume description.  Both volumes cover the same axis-aligned box (Sec. IV.B: the
 * colour volume has a higher dimension but the same size); voxel (i,j,k) has its centre
 * at origin + (i+1/2, j+1/2, k+1/2) * extent / dim; storage is x fastest.  Limits
 * (KF_E_RANGE beyond them): at most 65536 voxels per axis, 2^31-1 per volume and fewer
 * than 2^26 per z slice (dim x * dim y). */
typedef struct {
    int32_t geom_dim[3];    /* geometry voxels per axis (x, y, z), each >= 1             */
    int32_t colour_dim[3];  /* colour voxels per axis, each >= 1                          */
    double origin[3];       /* world coordinates of the box's minimum corner (metres)    */
    double extent[3];       /* box size (metres), each > 0                                */
    double colour_band;     /* sigma: max distance from the measured surface point (m);
                               the paper uses 20 mm (Sec. IV.B)                           */
    double colour_gate;     /* update only if W > colour_gate * W_pre; paper: 0.8         */
    int32_t hd_sampling;    /* kf_hd_sampling: how Eq. 9 reads HD(x_hd, y_hd)             */
} kf_volume_desc;

/* Six caller-owned device arrays of float32 (structure of arrays):
 * tsdf, w_geom: geometry volume, prod(geom_dim) each;
 * r, g, b, w_col: colour volume, prod(colour_dim) each.  A fresh volume is all zeros. */
typedef struct {
    float *tsdf, *w_geom, *r, *g, *b, *w_col;
} kf_volume_buffers;

typedef struct kf_volume kf_volume;

/* Bytes of each of the six arrays (host-only, no device work). */
kf_status kf_volume_buffer_bytes(const kf_volume_desc* desc, size_t out_bytes[6]);

/* Validate `desc` and borrow `bufs` (not copied, not freed).  Host-only. */
kf_status kf_volume_create(const kf_volume_desc* desc, const kf_volume_buffers* bufs,
                           kf_volume** out);

/* Zero all six arrays on `stream` (by a fill kernel, safe inside stream capture). */
kf_status kf_volume_reset(kf_volume* vol, void* stream);

/* Release the handle (the arrays stay with the caller). */
void kf_volume_destroy(kf_volume* vol);

/*
 * Integrate one frame (Sec. III and Sec. IV.B).
 *   depth: [dh][dw] float32 metres; 0, negative, NaN or infinite = no measurement;
 *          dw, dh <= 65535 and dw * dh < 2^27 - 1 (KF_E_RANGE otherwise).
 *   rgb:   [ch][cw][3] in `fmt`; cw, ch >= 2; cw * ch * 3 < 2^31.
 *   K_d, K_rgb: 3x3 intrinsics (K_c, K_hd of Eq. 1-4), zero skew, last row (0,0,1),
 *          positive focal lengths.
 *   T_rgb_from_d: 4x4 rigid transform (R_calib, t_calib) of Eq. 3.
 *   T_world_from_cam: 4x4 rigid pose of the depth camera; Eq. 5 uses its inverse.
 *   trunc_m: truncation distance in metres (> 0); w_max: cap of the geometry weight (>= 1).
 * Rigid transforms must have last row (0,0,0,1) and |R^T R - I| <= 1e-6.
 */
kf_status kf_integrate(kf_volume* vol, const float* depth, int32_t dw, int32_t dh,
                       const void* rgb, kf_pixfmt fmt, int32_t cw, int32_t ch,
                       const double K_d[9], const double K_rgb[9],
                       const double T_rgb_from_d[16], const double T_world_from_cam[16],
                       double trunc_m, double w_max, void* stream);

/* One scan for kf_integrate_batch: n_frames frames stored back to back. */
typedef struct {
    kf_volume* vol;
    int32_t n_frames;
    const float* depth;              /* device, [n][dh][dw]                          */
    const void* rgb;                 /* device, [n][ch][cw][3]                       */
    kf_pixfmt fmt;
    int32_t dw, dh, cw, ch;
    const double* K_d;               /* host [9]                                     */
    const double* K_rgb;             /* host [9]                                     */
    const double* T_rgb_from_d;      /* host [16]                                    */
    const double* T_world_from_cam;  /* host [n][16]                                 */
    double trunc_m, w_max;
} kf_scene;

/* Voxels per brick (x, y, z) of the forward integration's work items, per volume kind.
 * A brick is the work of one wavefront: x * y == 64 voxel columns of z voxels.  The
 * result never depends on the shapes (each voxel sees the same operations in the same
 * frame order); the time does: longer columns share the per-column part of Eq. 5 among
 * more voxels, smaller bricks are culled more finely.  Only the shapes listed by
 * kf_brick_shapes are compiled. */
typedef struct {
    int32_t geom[3];     /* default 16 x 4 x 8 */
    int32_t colour[3];   /* default 8 x 8 x 8  */
} kf_bricks;

/* The brick shapes compiled for kind 0 (geometry) or 1 (colour): writes up to `capacity`
 * triples (x, y, z) to `shapes` (host int32 [capacity][3]), the first being the default,
 * and their number to *n_shapes.  Host-only. */
kf_status kf_brick_shapes(int32_t kind, int32_t* shapes, int32_t capacity, int32_t* n_shapes);

/*
 * Integrate several independent scans (different volumes, sizes and frame counts).
 * Each voxel keeps its state on chip for frames_per_pass (K, 1 <= K; values above 64 act
 * as 64) consecutive frames of its scan, so a voxel's state is read and written at most
 * once per pass instead of once per frame; all scans advance together, one pass at a
 * time: a culling launch lists the (scan, brick) work items that can be updated in some
 * frame of the pass, and two persistent launches (geometry bricks, then colour bricks)
 * take them from queues.  The result
 * equals integrating each scan frame by frame with kf_integrate.  use_graph != 0 records
 * the passes into a HIP graph the first time a given batch (same pointers, sizes and
 * matrices) is seen and replays it afterwards.  The volumes of the batch must be distinct.
 */
kf_status kf_integrate_batch(const kf_scene* scenes, int32_t n_scenes,
                             int32_t frames_per_pass, int32_t use_graph, void* stream);

/* Destroy every graph recorded by kf_integrate_batch(..., use_graph != 0, ...) and free the
 * workspaces they own (waits for the device).  The cache keeps at most 64 graphs and 4 GiB
 * of workspace on its own, dropping the least recently used; this empties it, e.g. before
 * the volumes or images it refers to are freed for good.  *n_released and *bytes_released
 * (either may be NULL) receive what was dropped. */
kf_status kf_release_graphs(int32_t* n_released, size_t* bytes_released);

/* kf_integrate_batch with the bricks of the given shapes (NULL: the defaults); a shape not
 * listed by kf_brick_shapes is KF_E_UNSUPPORTED.  Same result for every shape. */
kf_status kf_integrate_batch_bricks(const kf_scene* scenes, int32_t n_scenes,
                                    int32_t frames_per_pass, int32_t use_graph,
                                    const kf_bricks* bricks, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): kf_integrate_batch without a graph, with the
 * same arguments and the same result, whose workspace (frame constants, per-pass tables,
 * queue counters, live lists, depth pyramids and pixel maps) lives in a fixed
 * 256 MiB device array inside the library instead of the stream-ordered allocator.  Calls
 * nothing that allocates device or pinned host memory: the tables reach the device in
 * kernel arguments, the counters are cleared by a kernel.  The array exists once per GPU
 * (held until the process ends) and every call on that GPU uses it, so calls that overlap
 * on one GPU (other streams, other threads) race and must be serialised by the caller; a
 * call's workspace is re-initialised by the call itself.  KF_E_RANGE if the batch needs
 * more than 256 MiB of workspace: about 32 bytes per brick of the largest pass's volumes
 * (a brick is 16 x 4 x 8 geometry or 8 x 8 x 8 colour voxels) plus about 5 MB per
 * 640 x 480 depth frame of the batch (a 256^3 / 512^3 pair of volumes takes 9.4 MB plus
 * its frames, a 512^3 / 1024^3 pair 75 MB plus its frames).  Other errors as
 * kf_integrate_batch.
 */
kf_status kf_integrate_batch_noalloc(const kf_scene* scenes, int32_t n_scenes,
                                     int32_t frames_per_pass, void* stream);

/*
 * kf_integrate_batch_bricks (without a graph) that also records start_events[q] and
 * end_events[q] (hipEvent_t handles created by the caller) on `stream` immediately before
 * the geometry and after the colour integration launch of pass q, for q < n_events, and,
 * when mid_events is not NULL, mid_events[q] between the two launches; n_events must be
 * at least the number of passes.  For measuring the integration kernels alone.
 */
kf_status kf_integrate_batch_timed(const kf_scene* scenes, int32_t n_scenes,
                                   int32_t frames_per_pass, const kf_bricks* bricks,
                                   void* const* start_events, void* const* mid_events,
                                   void* const* end_events, int32_t n_events, void* stream);

/*
 * Byte accounting for kf_integrate_batch_bricks with the same arguments: performs the
 * same integration and adds into counters (device, uint64[8], not cleared):
 *   [0] geometry voxel updates        [1] geometry voxels updated at least once per pass
 *   [2] colour voxel-frames reaching the weight gate
 *   [3] colour voxels reaching the gate at least once per pass
 *   [4] colour voxel updates          [5] colour voxels updated at least once per pass
 *   [6] geometry voxel-frames processed  [7] colour voxel-frames processed
 *       (the voxels of the live bricks of each frame; the rest were culled as unable to
 *       pass the depth tests; [0]-[5] do not depend on the brick shapes, [6]-[7] do)
 * Slower than kf_integrate_batch; for measurement only.
 */
kf_status kf_integrate_batch_counted(const kf_scene* scenes, int32_t n_scenes,
                                     int32_t frames_per_pass, const kf_bricks* bricks,
                                     unsigned long long* counters, void* stream);

/*
 * Per-voxel outcome of one frame against the volume's current state, without updating
 * it (same kernel as kf_integrate).  Codes: 0 outside the depth frustum, 1 no depth,
 * 2 outside the band (geometry: more than trunc behind the surface; colour: more than
 * colour_band from the back-projected depth pixel), 3 no normal, 4 weight gate failed,
 * 5 HD sample outside the HD image, 6 updated.  geom_status / colour_status: device
 * uint8 arrays of prod(geom_dim) / prod(colour_dim) elements.
 */
kf_status kf_debug_status(kf_volume* vol, const float* depth, int32_t dw, int32_t dh,
                          const void* rgb, kf_pixfmt fmt, int32_t cw, int32_t ch,
                          const double K_d[9], const double K_rgb[9],
                          const double T_rgb_from_d[16], const double T_world_from_cam[16],
                          double trunc_m, double w_max, uint8_t* geom_status,
                          uint8_t* colour_status, void* stream);

/*
 * Adjoint of the colour volume with respect to the HD images and the RGB extrinsic
 * (Eq. 9-10 with Eq. 2-4 differentiated through bilinear sampling and projection).
 * For L = sum_v sum_c grad_rgb_vol[c][v] * C_N(v)_c, where C_N is the colour volume
 * after integrating the n_frames frames (float32 images in [0,1]) starting from colour
 * weights w_col0 (device, prod(colour_dim) floats, or NULL for zeros), writes
 *   d_rgb: device float32 [n][ch][cw][3], overwritten with dL/dRGB;
 *   d_xi:  device float64 [6], overwritten with dL/dxi, xi = (rho, phi) the se(3) left
 *          perturbation T_rgb_from_d <- exp(xi^) T_rgb_from_d at xi = 0;
 *   d_pose: device float64 [n][6] or NULL, overwritten with dL/dxi_n for the depth-camera
 *          poses, xi_n the left perturbation in world coordinates T_world_from_cam[n] <-
 *          exp(xi_n^) T_world_from_cam[n] at xi_n = 0.  The depth pixel, the tests of
 *          Sec. IV.B and the bilinear cell are held (the derivative wherever none of them
 *          changes); the pose then moves only where each update samples the HD image, and
 *          d_pose[n] = -Ad(T_hd_from_world[n])^T of frame n's extrinsic contribution.
 * The per-frame blending weights are recomputed from the depth maps (nothing from the
 * forward is stored).  Any number of frames: the kernels replay at most 64 per launch
 * sequence, so a longer scan is taken in chunks of 64 (KF_BWD_CHUNK in the environment, 1
 * to 64, sets another size): a first sweep stores the colour weights at the start of
 * every chunk (prod(colour_dim) floats per chunk after the first), then the chunks are
 * replayed from the last with the gradient carried across chunk boundaries.  The geometry volume and the colour weights do not depend on the
 * HD images or the extrinsic (except where a sample leaves the HD image), so they have no
 * adjoint here.  Uses a workspace allocated on `stream` with the stream-ordered allocator.
 */
kf_status kf_integrate_backward(const kf_volume_desc* desc, const float* w_col0,
                                int32_t n_frames, const float* depth, const float* rgb_f32,
                                int32_t dw, int32_t dh, int32_t cw, int32_t ch,
                                const double K_d[9], const double K_rgb[9],
                                const double T_rgb_from_d[16], const double* T_world_from_cam,
                                const float* grad_rgb_vol, float* d_rgb,
                                double* d_xi, double* d_pose, void* stream);

/*
 * se(3) helpers for the extrinsic of the adjoint (host-only, double precision):
 *   kf_se3_compose:  T_out = exp(xi^) T_in, xi = (rho, phi) (translation, rotation), the
 *                    left perturbation kf_integrate_backward differentiates (T_in rigid);
 *   kf_se3_pullback: d_xi = J_l(xi)^T d_eps, the gradient with respect to xi of a function
 *                    of exp(xi^) T when d_eps is its gradient for a left perturbation at
 *                    exp(xi^) T (J_l the left Jacobian of SE(3)).
 * Both sum the exponential series (40 terms); |phi| must not exceed 10 (KF_E_ARG).
 */
kf_status kf_se3_compose(const double xi[6], const double T_in[16], double T_out[16]);
kf_status kf_se3_pullback(const double xi[6], const double d_eps[6], double d_xi[6]);

/*
 * Ray cast the volumes from a camera (the rendering the method uses for live feedback and
 * the predicted surface of tracking: abstract and Sec. III).  For pixel (x, y) of a
 * width x height image with intrinsics K (zero skew, positive focal lengths) and pose
 * T_world_from_cam (rigid), the ray is sampled every step_m metres of camera depth inside
 * the volume; the first two consecutive observed samples (all 8 trilinear corner weights
 * positive) whose trilinear TSDF goes from positive to negative give the surface, refined
 * linearly between them.  Writes, per pixel (device arrays, caller-owned):
 *   depth:  [height][width] float32, camera depth of the surface, 0 for no surface;
 *   vertex: [height][width][3] world point (or NULL to skip);
 *   normal: [height][width][3] unit normal from central differences of the trilinear TSDF
 *           (or NULL), zero where a difference sample is unobserved;
 *   rgb:    [height][width][3] trilinear colour of the colour volume at the surface (or
 *           NULL), zero unless its 8 corner colour weights are positive.
 * Both volumes need at least 2 voxels per axis (KF_E_SHAPE); step_m must be finite and
 * positive; at most 2^20 samples are taken per ray.  Asynchronous on `stream`.
 */
kf_status kf_raycast(kf_volume* vol, int32_t width, int32_t height, const double K[9],
                     const double T_world_from_cam[16], double step_m, float* depth,
                     float* vertex, float* normal, float* rgb, void* stream);

/*
 * Marching cubes of the geometry volume: the triangle mesh of the zero level of the TSDF
 * (Sec. III, after KinectFusion; the mesh the method decimates and textures per polygon).
 * Cubes are the 2x2x2 groups of voxel centres; only cubes whose 8 voxels are observed
 * (weight > 0) make triangles; a voxel is inside iff its TSDF is < 0.  Writes, when both
 * output pointers are given and large enough (device arrays, caller-owned):
 *   vertices:  float32 [n_vertices][3], world coordinates: one vertex per crossed grid
 *              edge of a complete cube, linearly interpolated along the edge; ordered by
 *              (linear index of the edge's lower voxel, axis x, y, z);
 *   triangles: int32 [n_triangles][3] vertex indices, ordered by cube (linear index of its
 *              lower corner), counter-clockwise seen from the positive-TSDF side.
 * counts (host int64 [2]) receives (n_vertices, n_triangles).  Call with both outputs
 * NULL to size them (KF_OK, only the counts); giving one output without the other is
 * KF_E_ARG.  When the counts exceed the capacities the call returns KF_E_RANGE and the
 * outputs hold an incomplete mesh (nothing is written past the capacities).  Returns after
 * synchronising `stream` (the counts are read at the end, the outputs are complete).  The
 * volume needs fewer than 2^31 / 5 voxels (KF_E_RANGE).  Uses a workspace of about 6
 * bytes per voxel from the stream-ordered allocator.
 */
kf_status kf_mesh_extract(kf_volume* vol, float* vertices, int64_t vertex_capacity,
                          int32_t* triangles, int64_t triangle_capacity, int64_t counts[2],
                          void* stream);

/*
 * Quadric-error decimation of a triangle mesh (Sec. IV.C: the dense marching-cubes model
 * is simplified by quadric-based decimation to a reduction rate, the fraction of its
 * polygons that remain; Fig. 3).  Host-only and synchronous: every pointer is HOST memory.
 *   vertices:  float32 [n_vertices][3]; triangles: int32 [n_triangles][3] vertex indices,
 *              counter-clockwise seen from outside (kf_mesh_extract's output, copied to
 *              the host), each triangle with three distinct vertices;
 *   rate:      in [0, 1]; edges are contracted until at most round(rate * n_triangles)
 *              triangles remain (or no edge can be contracted without breaking the
 *              surface);
 *   out_vertices, out_triangles: room for n_vertices and n_triangles entries; receive the
 *              kept vertices (in input order) and triangles (in input order, re-indexed,
 *              orientation kept); *out_n_vertices, *out_n_triangles their counts.
 * The squared distances to the planes of a vertex's triangles make its quadric error;
 * open borders add planes perpendicular to their triangles (weight 1000) so they stay in
 * place.  The cheapest edge (ties by its vertex indices) is
 * contracted to the point minimising the summed quadric when the contraction keeps the
 * surface manifold and turns no triangle over.  Deterministic (double precision).
 * KF_E_ARG for bad indices, non-finite vertices or a rate outside [0, 1].
 */
kf_status kf_mesh_decimate(const float* vertices, int64_t n_vertices, const int32_t* triangles,
                           int64_t n_triangles, double rate, float* out_vertices,
                           int64_t* out_n_vertices, int32_t* out_triangles,
                           int64_t* out_n_triangles);

/*
 * Texture-map sizes and their place in an atlas image (Sec. IV.D: Eq. 11-12 and the
 * merging of the maps into one image).  Host-only, no device work.
 *   tri:   host float32 [n_tri][3][3], the world vertices (V1, V2, V3) of each triangle;
 *          V1 maps to the map's top-left texel, V2 to its top-right, V3 to its bottom-left.
 *   size_pixel: the size of one texel on the model, metres (finite, > 0).
 *   rects: host int32 [n_tri][4], written: (x, y, w, h) of each map in the atlas, with
 *          w = max(2, ceil(|V1V2| / size_pixel)) and h = max(2, ceil(|V1V3| / size_pixel))
 *          (lengths in double from the float vertices).
 * Maps are placed column-wise from the top-left corner: each below the previous one; when
 * a map does not fit in the atlas_height rows that remain, a new column starts at the top,
 * right of the widest map of the previous column.  *atlas_width receives the width the
 * columns reach (0 for no triangles).  KF_E_RANGE if a map is taller than the atlas or
 * wider or taller than 65535 texels (rects then holds the maps placed so far).
 */
kf_status kf_texture_layout(int32_t n_tri, const float* tri, double size_pixel,
                            int32_t atlas_height, int32_t* rects, int32_t* atlas_width);

/*
 * Texel colours of every triangle's texture map from the colour volume (Sec. IV.D,
 * Eq. 13-14).  Texel (i, j) of the w x h map of triangle n (i < w, j < h) is the world
 * point V1 + i (V2 - V1) / (w - 1) + j (V3 - V1) / (h - 1), coloured by trilinear
 * interpolation of the colour volume (zero unless the point lies between the first and
 * last voxel centres on every axis and the 8 corner colour weights are positive).
 *   tri:   device float32 [n_tri][3][3] world vertices (as for kf_texture_layout);
 *   rects: device int32 [n_tri][4] (x, y, w, h); a rect that leaves the atlas or has w or h
 *          below 2 is skipped (kf_texture_layout never makes one);
 *   atlas_rgb:  device float32 [atlas_height][atlas_width][3], or NULL;
 *   atlas_rgb8: device uint8 [atlas_height][atlas_width][3] = rint(255 clamp(c, 0, 1)),
 *          or NULL (not both NULL).
 * Only the texels of the maps are written; the rest of the atlas keeps its contents.  The
 * colour volume needs at least 2 voxels per axis (KF_E_SHAPE).  Asynchronous on `stream`.
 */
kf_status kf_texture_generate(kf_volume* vol, int32_t n_tri, const float* tri,
                              const int32_t* rects, int32_t atlas_width, int32_t atlas_height,
                              float* atlas_rgb, uint8_t* atlas_rgb8, void* stream);

/* Message for a status code (static string). */
const char* kf_status_str(kf_status s);

/* Message of the last failing call on this thread ("" if none). */
const char* kf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KF_H */
