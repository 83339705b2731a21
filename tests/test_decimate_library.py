"""The library's quadric-error decimation (kf_mesh_decimate: host code with a priority
queue) against the oracle's (a linear scan for the cheapest edge at every step), mesh for
mesh and bit for bit, on the scanned scene's marching-cubes mesh, a sphere, a cube, a
planar grid and a rough terrain at several rates; and its argument checks.  CPU only."""
import ctypes as C

import numpy as np

from paper_1602_06645_amd import _lib as L
from test_decimate_pins import cube, grid, sphere_mesh


def _decimate_lib(V, T, rate):
    lib = L.load()
    V = np.ascontiguousarray(V, np.float32)
    T = np.ascontiguousarray(T, np.int32)
    ov = np.zeros((max(len(V), 1), 3), np.float32)
    ot = np.zeros((max(len(T), 1), 3), np.int32)
    nv, nt = C.c_int64(), C.c_int64()
    L.check(lib.kf_mesh_decimate(V.ctypes.data, len(V), T.ctypes.data, len(T), float(rate),
                                 ov.ctypes.data, C.byref(nv), ot.ctypes.data, C.byref(nt)))
    return ov[:nv.value], ot[:nt.value]


def _cases(oracle):
    from kf_synth import configs
    spec, fr = configs.tiny()
    st = oracle.State(spec, np.float32)
    oracle.integrate(spec, fr.numpy(), st)
    scan = oracle.marching_cubes(spec, st.tsdf, st.wg, "f32")
    return [("scan", scan, (0.5, 0.1, 0.02)), ("sphere", sphere_mesh(oracle), (0.3, 0.05)),
            ("cube", cube(6), (12 / 432, 0.5)), ("grid", grid(20), (0.2, 0.02)),
            ("terrain", grid(18, jitter=0.02, seed=5), (0.25, 0.03))]


def test_library_equals_oracle(oracle):
    for name, (V, T), rates in _cases(oracle):
        for rate in rates:
            v0, t0 = oracle.decimate(V, T, rate)
            v1, t1 = _decimate_lib(V, T, rate)
            assert v0.shape == v1.shape and t0.shape == t1.shape, (name, rate, t0.shape, t1.shape)
            assert np.array_equal(v0.view(np.uint32), v1.view(np.uint32)), (name, rate)
            assert np.array_equal(t0, t1), (name, rate)


def test_rate_one_and_zero_and_empty(oracle):
    V, T = grid(6)
    v, t = _decimate_lib(V, T, 1.0)
    assert np.array_equal(v, V) and np.array_equal(t, T)
    v, t = _decimate_lib(V, T, 0.0)
    v0, t0 = oracle.decimate(V, T, 0.0)
    assert np.array_equal(t, t0) and len(t) < len(T)
    v, t = _decimate_lib(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), 0.5)
    assert len(v) == 0 and len(t) == 0


def test_library_rejects_bad_meshes():
    lib = L.load()
    V, T = grid(3)
    ov = np.zeros_like(V)
    ot = np.zeros_like(T)
    nv, nt = C.c_int64(), C.c_int64()

    def call(v, t, rate):
        return lib.kf_mesh_decimate(v.ctypes.data, len(v), t.ctypes.data, len(t), rate,
                                    ov.ctypes.data, C.byref(nv), ot.ctypes.data, C.byref(nt))
    assert call(V, T, 1.5) == L.KF_E_ARG
    assert call(V, T, float("nan")) == L.KF_E_ARG
    bad = T.copy()
    bad[2, 1] = len(V)
    assert call(V, bad, 0.5) == L.KF_E_ARG
    bad = T.copy()
    bad[1, 2] = bad[1, 0]
    assert call(V, bad, 0.5) == L.KF_E_ARG
    Vn = V.copy()
    Vn[3, 1] = np.nan
    assert call(Vn, T, 0.5) == L.KF_E_ARG
    assert lib.kf_mesh_decimate(V.ctypes.data, len(V), T.ctypes.data, len(T), 0.5, None,
                                C.byref(nv), ot.ctypes.data, C.byref(nt)) == L.KF_E_ARG
