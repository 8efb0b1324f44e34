"""Remap set-up on the host (no GPU): the library's located triangles and
weights against the oracle's brute-force location, and argument errors."""
import ctypes

import numpy as np
import pytest

import paper_1908_07038_amd as pa
from oracle.mesh import build_mesh
from oracle import remap as R


@pytest.mark.parametrize("src,dst", [("O32", "F8"), ("O16", "O16"), ("O12", "F30"), ("O8", "O3"),
                                     ("O24", "F24"), ("O4", "F1"), ("O20", "O9"), ("O1", "F1"), ("O1", "O1"),
                                     ("O2", "F40")])
def test_remap_tables_match_the_oracle(src, dst):
    """Target positions equal the oracle's; every chosen triangle is a mesh
    triangle containing the point; interpolated values agree with the
    oracle's to rounding (on-edge and on-node points may pick a different
    one of the triangles that contain them, with the same value)."""
    M = pa.Mesh(src, device=-1)
    r = pa.Remap(M, dst)
    e = r.export()
    m = build_mesh(int(src[1:]))
    tg = R.TargetGrid(dst)
    assert r.npoints == tg.npoints and r.nfallback == 0
    np.testing.assert_allclose(e["xyz"], tg.xyz, rtol=0, atol=2e-16)
    # a mesh triangle, in its stored rotation
    tris = {tuple(t) for t in m.tris.tolist()}
    assert all(tuple(t) in tris for t in e["nodes"].tolist())
    # containment: every triple product >= -1e-14 (R.DET_TOL)
    xyz = m.grid.xyz
    a, b, c = (xyz[e["nodes"][:, j]] for j in range(3))
    dd = R.triple_products(a, b, c, tg.xyz)
    assert (dd.sum(axis=1) > 0).all() and (dd.min(axis=1) >= -R.DET_TOL).all()
    _, nodes, w = R.locate(xyz, m.tris, tg.xyz)
    f = np.random.default_rng(11).standard_normal((m.grid.nnodes, 3))
    got = R.apply(e["nodes"].astype(np.int64), e["weights"], f)
    np.testing.assert_allclose(got, R.apply(nodes, w, f), rtol=0, atol=1e-12)
    np.testing.assert_allclose(e["weights"].sum(axis=1), 1.0, rtol=0, atol=1e-13)


def test_remap_errors_are_status_codes():
    L = pa.lib()
    M = pa.Mesh("O4", device=-1)
    h = ctypes.c_void_p()
    for bad in [b"X8", b"F0", b"F", b"O-1", b"", b"Fx"]:
        assert L.atlas_remap_build(M.handle, bad, ctypes.byref(h)) == -1
    assert L.atlas_remap_build(None, b"F2", ctypes.byref(h)) == -1
    assert L.atlas_remap_build(M.handle, None, ctypes.byref(h)) == -1
    assert L.atlas_remap_build(M.handle, b"F2", None) == -1
    assert L.atlas_remap_sizes(None, None, None) == -1
    assert L.atlas_remap_export(None, None, None, None) == -1
    L.atlas_remap_free(None)
    r = pa.Remap(M, " f2 ")
    assert r.npoints == 4 * 8
    buf = (ctypes.c_double * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    # a host-only mesh runs no kernel
    assert L.atlas_remap_apply(r.handle, 0, 1, p, p, None) == -4
    assert L.atlas_remap_apply(None, 0, 1, p, p, None) == -1
