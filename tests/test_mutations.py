"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutant is a copy of the oracle's C source with one plausible mistake (a wrong sign,
a swapped index, a dropped term, a wrong rounding rule, a transposed operand).  The
copy is compiled into a temporary library and the pin suites are run against it in a
subprocess; every mutant must make them fail.  This is how the pins are shown to pin
the oracle rather than merely agree with it.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")
BODY, MAIN, RC, TX = "kf_oracle_body.h", "kf_oracle.c", "kf_raycast_body.h", "kf_texture_body.h"
MC = "kf_mesh_body.h"
DEC = "kf_decimate_body.h"

# (name, file, original text, mutated text)
MUTANTS = [
    ("cx_for_x_uses_cy", BODY, "REAL x = FMA(c->fx, p[0] * iz, c->cx);", "REAL x = FMA(c->fx, p[0] * iz, c->cy);"),
    ("fy_for_y_uses_fx", BODY, "REAL y = FMA(c->fy, p[1] * iz, c->cy);", "REAL y = FMA(c->fx, p[1] * iz, c->cy);"),
    ("round_by_floor", BODY, "*u = RINT(x);", "*u = FLOOR(x);"),
    ("frustum_off_by_one", BODY, "*u <= (REAL)(W - 1)", "*u <= (REAL)W"),
    ("affine_drops_z_column", BODY, "FMA(A[3 * r + 2], fk, FMA(", "(0 * fk) + (FMA("),
    ("trunc_sign", BODY, "if (sdf < -c->trunc) return OR_ST_BAND;", "if (sdf < c->trunc) return OR_ST_BAND;"),
    ("tsdf_no_clamp", BODY, "REAL t = FMIN((REAL)1, sdf * c->inv_trunc);", "REAL t = sdf * c->inv_trunc;"),
    ("tsdf_wrong_average", BODY, "*F = *F + (t - *F) / wn;", "*F = *F + (t - *F) / *Wg;"),
    ("no_weight_cap", BODY, "*Wg = FMIN(wn, c->w_max);", "*Wg = wn;"),
    ("backproject_y_uses_fx", BODY, "P[1] = ((v - c->cy) * c->inv_fy) * d;", "P[1] = ((v - c->cy) * c->inv_fx) * d;"),
    ("sigma_not_squared", BODY, "if (dist2 > c->sigma2) return;", "if (dist2 > c->sigma2 * c->sigma2 * 4) return;"),
    ("normal_operands_swapped", BODY, "REAL Nz = FMA(e1x, e2y, -(e1y * e2x));", "REAL Nz = FMA(e1y, e2x, -(e1x * e2y));"),
    ("normal_neighbour_v_instead_of_u", BODY, "REAL d1 = (REAL)D[iv * (size_t)W + iu + 1];", "REAL d1 = (REAL)D[(iv + 1) * (size_t)W + iu];"),
    ("weight_not_normalised", BODY, "e->w = dp / SQRT(nn * pp);", "e->w = dp / SQRT(pp);"),
    ("gate_without_factor", BODY, "if (!(e->w > c->gate * Wc)) return;", "if (!(e->w > Wc)) return;"),
    ("hd_ignores_extrinsic", BODY, "OR_FN(affine_)(c->Ah, c->bh, i, j, k, e->q);", "OR_FN(affine_)(c->Ac, c->bc, i, j, k, e->q);"),
    ("hd_uses_depth_intrinsics", BODY, "e->xh = FMA(c->fxr, e->q[0] * iqz, c->cxr);", "e->xh = FMA(c->fx, e->q[0] * iqz, c->cx);"),
    ("bilinear_wrong_fraction", BODY, "OR_FN(lerp_)(p00, p10, e->ax), OR_FN(lerp_)(p01, p11, e->ax), e->ay);", "OR_FN(lerp_)(p00, p10, e->ay), OR_FN(lerp_)(p01, p11, e->ax), e->ay);"),
    ("colour_alpha_wrong", BODY, "REAL alpha = e->w / (*Wc + e->w);", "REAL alpha = e->w / ((REAL)1 + e->w);"),
    ("eq10_dropped_factor", BODY, "*Wc = FMA(e->w, (REAL)1 - *Wc, *Wc);", "*Wc = *Wc + e->w;"),
    ("rgb8_scale_wrong", BODY, "(REAL)rgb8[idx] * (REAL)(1.0 / 255.0)", "(REAL)rgb8[idx] * (REAL)(1.0 / 256.0)"),
    ("pose_not_inverted", MAIN, "for (int c = 0; c < 3; ++c) Rcw[3 * r + c] = Rwc[3 * c + r];", "for (int c = 0; c < 3; ++c) Rcw[3 * r + c] = Rwc[3 * r + c];"),
    ("translation_sign", MAIN, "tcw[r] = -((Rwc[0 + r] * twc[0]", "tcw[r] = +((Rwc[0 + r] * twc[0]"),
    ("no_half_voxel_offset", MAIN, "double c0 = origin[0] + 0.5 * s[0];", "double c0 = origin[0];"),
    ("extrinsic_composed_backwards", MAIN, "thw[r] = ((Rrd[3 * r + 0] * tcw[0] + Rrd[3 * r + 1] * tcw[1]) + Rrd[3 * r + 2] * tcw[2])\n                 + trd[r];", "thw[r] = tcw[r] + trd[r];"),
    ("adjoint_beta_without_tail", MAIN, "double beta = alpha[f] * tail;", "double beta = alpha[f];"),
    ("adjoint_dsy_wrong", MAIN, "double dsy = (1 - ax) * (p01 - p00) + ax * (p11 - p10);", "double dsy = (1 - ay) * (p01 - p00) + ay * (p11 - p10);"),
    ("adjoint_rotation_sign", MAIN, "xi4 += e->q[2] * a[0] - e->q[0] * a[2];", "xi4 += e->q[0] * a[2] - e->q[2] * a[0];"),
    ("adjoint_projection_z_term", MAIN, "a[2] += -gb * (dsx * fc[f].fxr * e->q[0] + dsy * fc[f].fyr * e->q[1])", "a[2] += -gb * (dsx * fc[f].fxr * e->q[0])"),
    # ray casting
    ("raycast_trilinear_y_uses_x_fraction", RC, "const REAL c0 = RC_FN(rc_lerp_)(c00, c10, f[1]);", "const REAL c0 = RC_FN(rc_lerp_)(c00, c10, f[0]);"),
    ("raycast_corner_y_z_swapped", RC, "{0, 1, X, X + 1, XY, XY + 1, XY + X, XY + X + 1}", "{0, 1, XY, XY + 1, X, X + 1, XY + X, XY + X + 1}"),
    ("raycast_back_face_crossing", RC, "prev_F > (REAL)0 && F < (REAL)0", "prev_F < (REAL)0 && F > (REAL)0"),
    ("raycast_refinement_wrong_sample", RC, "prev_F / (prev_F - F)", "F / (prev_F - F)"),
    ("raycast_weights_ignored", RC, "if (!(w[base + off[c]] > 0.0f)) return 0;", ""),
    ("raycast_colour_in_geometry_index", RC, "qc[k] = FMA(t_hit, bc, c->ac[k]);", "qc[k] = FMA(t_hit, bc, c->a[k]);"),
    ("raycast_normal_not_scaled", RC, "grad[k] = (Fp - Fm) * c->inv_s[k];", "grad[k] = (Fp - Fm);"),
    ("raycast_no_half_voxel", MAIN, "out->a[k] = (t[k] - vol->origin[k]) / s - 0.5;", "out->a[k] = (t[k] - vol->origin[k]) / s;"),
    ("raycast_ray_y_uses_fx", MAIN, "const double ru = R[3 * k + 0] / fx, rv = R[3 * k + 1] / fy;", "const double ru = R[3 * k + 0] / fx, rv = R[3 * k + 1] / fx;"),
    ("raycast_vertex_drops_translation", RC, "c->R0[k])), c->tw[k]);", "c->R0[k])), (REAL)0);"),
    ("texture_step_divides_by_w", TX, "/ (REAL)(w - 1);   /* Eq. 13 */", "/ (REAL)w;   /* Eq. 13 */"),
    ("texture_steps_swapped", TX, "FMA((REAL)j, s2[k], FMA((REAL)i, s1[k]", "FMA((REAL)i, s2[k], FMA((REAL)j, s1[k]"),
    ("texture_no_half_voxel", TX, "off[k] = (REAL)(-vol->origin[k] / s - 0.5);", "off[k] = (REAL)(-vol->origin[k] / s);"),
    ("texture_weights_ignored", TX, "if (!(w[base + off[c]] > 0.0f)) return 0;", ""),
    ("texture_corner_y_z_swapped", TX, "{0, 1, X, X + 1, XY, XY + 1, XY + X, XY + X + 1}", "{0, 1, XY, XY + 1, X, X + 1, XY + X, XY + X + 1}"),
    ("texture_lerp_y_uses_x_fraction", TX, "TX_FN(tx_lerp_)(c00, c10, f[1])", "TX_FN(tx_lerp_)(c00, c10, f[0])"),
    ("texture_byte_round_half_up", TX, "RINT(FMIN(FMAX(c[m], (REAL)0), (REAL)1) * (REAL)255)", "FLOOR(FMIN(FMAX(c[m], (REAL)0), (REAL)1) * (REAL)255 + (REAL)0.5)"),
    ("texture_byte_no_upper_clamp", TX, "RINT(FMIN(FMAX(c[m], (REAL)0), (REAL)1) * (REAL)255)", "RINT(FMIN(FMAX(c[m], (REAL)0), (REAL)2) * (REAL)127)"),
    ("texture_size_rounds_down", MAIN, "const double wf = ceil(sqrt(d12) / size_pixel)", "const double wf = floor(sqrt(d12) / size_pixel)"),
    ("texture_height_from_first_edge", MAIN, "const double e2 = (double)V[6 + k] - (double)V[k];", "const double e2 = (double)V[3 + k] - (double)V[k];"),
    ("texture_layout_breaks_column_early", MAIN, "if (y + h > atlas_height) {", "if (y + h >= atlas_height) {"),
    ("texture_layout_column_width_last_map", MAIN, "if (w > col_w) col_w = w;", "col_w = w;"),
    ("nearest_rounds_down", BODY, "REAL rx = RINT(e->xh), ry = RINT(e->yh);", "REAL rx = FLOOR(e->xh), ry = FLOOR(e->yh);"),
    ("nearest_bilinear_bounds", BODY, "rx <= (REAL)(CW - 1) && ry >= (REAL)0 && ry <= (REAL)(CH - 1)", "rx <= (REAL)(CW - 2) && ry >= (REAL)0 && ry <= (REAL)(CH - 2)"),
    ("nearest_ignored", MAIN, "out->hd_nearest = vol->hd_nearest ? 1.0 : 0.0;", "out->hd_nearest = 0.0;"),
    ("pose_rho_sign", MAIN, "const double v6[6] = {-b[0], -b[1], -b[2],", "const double v6[6] = {b[0], b[1], b[2],"),
    ("pose_rotation_transposed", MAIN, "b[m] = R[m] * a[0] + R[3 + m] * a[1] + R[6 + m] * a[2];", "b[m] = R[3 * m] * a[0] + R[3 * m + 1] * a[1] + R[3 * m + 2] * a[2];"),
    ("pose_no_half_voxel", MAIN, "pw[0] = vol->origin[0] + ((double)i + 0.5) * cs[0];", "pw[0] = vol->origin[0] + (double)i * cs[0];"),
    ("mesh_zero_counts_inside", MC, "if (tsdf[LIN(x + (c & 1), y + ((c >> 1) & 1), z + ((c >> 2) & 1))] < 0.0f)", "if (tsdf[LIN(x + (c & 1), y + ((c >> 1) & 1), z + ((c >> 2) & 1))] <= 0.0f)"),
    ("mesh_interpolation_from_far_end", MC, "const double t64 = (double)tsdf[u] / ((double)tsdf[u] - (double)tsdf[w]);", "const double t64 = (double)tsdf[w] / ((double)tsdf[w] - (double)tsdf[u]);"),
    ("mesh_no_half_voxel", MC, "c0[k] = vol->origin[k] + 0.5 * s[k];", "c0[k] = vol->origin[k];"),
    ("mesh_fan_reversed", MC, "tri[n][1] = loop[(c + k) % len];\n            tri[n][2] = loop[(c + k + 1) % len];", "tri[n][1] = loop[(c + k + 1) % len];\n            tri[n][2] = loop[(c + k) % len];"),
    ("mesh_faces_walked_clockwise", MC, "coord[b] = side ? ccw_pos[i][0] : ccw_neg[i][0];\n                coord[c] = side ? ccw_pos[i][1] : ccw_neg[i][1];", "coord[b] = side ? ccw_neg[i][0] : ccw_pos[i][0];\n                coord[c] = side ? ccw_neg[i][1] : ccw_pos[i][1];"),
    ("mesh_weights_ignored", MC, "ok &= wg[LIN(x + (c & 1), y + ((c >> 1) & 1), z + ((c >> 2) & 1))] > 0.0f;", "ok &= 1;"),
    ("mesh_unused_vertices_kept", MC, "if (!used) continue;", ""),
    ("mesh_edge_id_axes_swapped", MC, "if (d == 0) return 0 + y + 2 * z;", "if (d == 0) return 0 + z + 2 * y;"),
    ("mesh_fan_from_loop_start", MC, "for (; c < len; ++c) {", "for (; c < 0; ++c) {"),
    ("mesh_last_cube_column_dropped", MC, "for (int64_t x = 0; x + 1 < X; ++x) {", "for (int64_t x = 0; x + 2 < X; ++x) {"),
    # quadric-error decimation
    ("decimate_no_boundary_planes", DEC, "const double wt = DEC_BOUNDARY_WEIGHT;", "const double wt = 0.0;"),
    ("decimate_no_link_condition", DEC, "    if (common != ns) return 0;\n", ""),
    ("decimate_no_flip_test", DEC, "if (!(n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2] > 0.0)) return 0;", ""),
    ("decimate_midpoint_only", DEC, "if (tr > 0.0 && fabs(det) > DEC_DET_EPS * tr * tr * tr) {", "if (0) {"),
    ("decimate_target_truncated", DEC, "floor(rate * (double)nt + 0.5)", "floor(rate * (double)nt)"),
    ("decimate_quadrics_not_merged", DEC, "m.Q[a][k] = m.Q[a][k] + m.Q[b][k];", "m.Q[a][k] = m.Q[a][k];"),
    ("decimate_cost_drops_cross_term", DEC, "+ 2.0 * q[1] * x * y", "+ 0.0 * q[1] * x * y"),
]

PIN_FILES = [os.path.join(HERE, n) for n in (
    "test_oracle_pins.py", "test_nearest_pins.py", "test_raycast_pins.py", "test_texture_pins.py",
    "test_mesh_pins.py", "test_backward_pins.py")]     # slowest last (each run stops at a failure)
# A mistake in a body that only one operation includes runs that operation's pins; a
# mistake in the shared source or the integration body runs them all.
PINS_FOR = {RC: [os.path.join(HERE, "test_raycast_pins.py")],
            TX: [os.path.join(HERE, "test_texture_pins.py")],
            MC: [os.path.join(HERE, "test_mesh_pins.py")],
            DEC: [os.path.join(HERE, "test_decimate_pins.py")]}


def _run_mutant(m, workdir):
    name, fname, old, new = m
    src = os.path.join(workdir, name)
    os.makedirs(src)
    for f in (BODY, MAIN, RC, TX, MC, DEC, "kf_oracle.h"):
        shutil.copy(os.path.join(ORACLE, f), src)
    path = os.path.join(src, fname)
    text = open(path).read()
    assert text.count(old) >= 1, f"mutant {name}: pattern not found"
    open(path, "w").write(text.replace(old, new, 1))
    lib = os.path.join(src, "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11",
                           "-shared", "-fPIC", "-o", lib, os.path.join(src, MAIN), "-lm"])
    env = dict(os.environ, KF_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS_FOR.get(fname, PIN_FILES)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    return name, r.returncode


def test_every_planted_mistake_is_caught():
    names = [m[0] for m in MUTANTS]
    assert len(set(names)) == len(names)
    # control: an unmodified copy built and run the same way must pass every pin
    control = ("control_unmodified", BODY, "static REAL OR_FN(lerp_)", "static REAL OR_FN(lerp_)")
    with tempfile.TemporaryDirectory() as tmp:
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda m: _run_mutant(m, tmp), [control] + MUTANTS))
    assert results[0] == ("control_unmodified", 0), "the unmodified oracle copy fails its pins"
    results = results[1:]
    survivors = [n for n, rc in results if rc == 0]
    errors = [(n, rc) for n, rc in results if rc not in (0, 1)]
    assert not errors, f"pin suite crashed (not a clean failure) for {errors}"
    assert not survivors, f"planted mistakes not caught by any pin: {survivors}"
