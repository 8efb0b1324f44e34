"""C ABI checks that need no GPU: every declared symbol is exported, the host
mesh builder matches the oracle bit for bit on connectivity and positions and
to rounding on geometry, and argument errors come back as status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1908_07038_amd as pa
from _oracle_cache import mesh_and_dual

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(atlas_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20, names
    L = ctypes.CDLL(pa.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    # and the binding declares a signature for each
    assert set(names) <= set(pa._SIGS), set(names) - set(pa._SIGS)


def test_version():
    assert pa.version().startswith("atlas-nabla")


@pytest.mark.parametrize("N", [1, 2, 4, 32, 128])
def test_host_mesh_matches_oracle(N):
    M = pa.Mesh(f"O{N}", device=-1)
    m, g = mesh_and_dual(N)
    assert (M.nnodes, M.nedges, M.ntris, M.npole_edges) == (m.nnodes, m.nedges, m.ntris, 34)
    assert M.max_slots == m.degree.max()
    c = M.export_connectivity()
    np.testing.assert_array_equal(c["tris"], m.tris)
    np.testing.assert_array_equal(c["edges"], m.edges)
    np.testing.assert_array_equal(c["csr_off"], m.off)
    np.testing.assert_array_equal(c["nbr"], m.nbr)
    np.testing.assert_array_equal(c["eid"], m.eid)
    np.testing.assert_array_equal(c["sgn"], m.sgn)
    np.testing.assert_array_equal(c["rev"], m.rev)
    np.testing.assert_array_equal(c["is_pole"].astype(bool), m.is_pole)
    gr = M.export_grid()
    np.testing.assert_array_equal(gr["row_size"], m.grid.row_size)
    np.testing.assert_array_equal(gr["row_off"], m.grid.row_off)
    # positions: bit for bit (they enter every dual quantity through differences)
    np.testing.assert_array_equal(gr["colat"], m.grid.theta)
    np.testing.assert_array_equal(gr["xyz"], m.grid.xyz)
    np.testing.assert_array_equal(gr["lonlat"][:, 0], m.grid.lon)
    ge = M.export_geometry()
    rel = np.linalg.norm(ge["S"] - g.S, axis=1) / np.linalg.norm(g.S, axis=1)
    assert rel.max() < 2e-15
    np.testing.assert_allclose(ge["V"], g.V, rtol=2e-15, atol=0)
    np.testing.assert_array_equal(ge["basis"][:, 0], g.east)
    np.testing.assert_array_equal(ge["basis"][:, 1], g.north)
    np.testing.assert_allclose(ge["C"], g.C, rtol=0, atol=1e-13 * np.abs(g.C).max())
    M.close()


def test_errors_are_status_codes():
    L = pa.lib()
    h = ctypes.c_void_p()
    for bad in [b"F8", b"O0", b"", b"O-3", b"Oxx", b"N32"]:
        assert L.atlas_mesh_build(bad, 6371220.0, -1, ctypes.byref(h)) == -1
        assert L.atlas_last_error()
    assert L.atlas_mesh_build(b"O4", -1.0, -1, ctypes.byref(h)) == -1
    assert L.atlas_mesh_build(b"O4", 1.0, -1, None) == -1
    assert L.atlas_mesh_build(None, 1.0, -1, ctypes.byref(h)) == -1
    assert L.atlas_mesh_build(b"O4", 1.0, -7, ctypes.byref(h)) == -4
    assert L.atlas_mesh_sizes(None, None, None, None, None, None, None) == -1
    L.atlas_mesh_free(None)
    # operators on a host-only mesh or a NULL mesh
    M = pa.Mesh("O4", device=-1)
    buf = (ctypes.c_double * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.atlas_nabla_gradient(M.handle, 0, 1, p, p, None) == -4
    assert L.atlas_nabla_gradient(None, 0, 1, p, p, None) == -1
    assert L.atlas_nabla_conservation(M.handle, 0, 1, p, p, p, None) == -4
    assert L.atlas_batch_create(M.handle, 1, None, 0, 1, None, ctypes.byref(h)) == -4
    assert L.atlas_batch_run(None, None) == -1
    assert L.atlas_nabla_set_tune(M.handle, 9, 1, None) == -5
    assert L.atlas_nabla_set_tune(M.handle, 0, 3, None) == -1    # not a single op bit
    bad = pa.TuneShape(waves_per_block=3)
    assert L.atlas_nabla_set_tune(M.handle, 0, 1, ctypes.byref(bad)) == -1
    assert L.atlas_nabla_set_tune(M.handle, 0, 1, None) == 0


def test_no_device_is_reported():
    if pa.device_count() > 0:
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert pa.lib().atlas_mesh_build(b"O4", 1.0, 0, ctypes.byref(h)) == -4
    n = ctypes.c_int(5)
    assert pa.lib().atlas_device_count(ctypes.byref(n)) == -4 and n.value == 0
    with pytest.raises(pa.AtlasError) as e:
        pa.Mesh("O4", device=0)
    assert e.value.code == -4


def test_describe_resolves_the_default_paths():
    """The launch a call would make, without a device: per-operator default
    paths for FP32/FP64 columns of more than 32 levels, the row-window walk
    or the gather otherwise, and an explicit shape overriding the default."""
    M = pa.Mesh("O8", device=-1)
    # 137 levels: two whole 64-level slices per step, the 9-level remainder
    # in the packed tail pass; 160 levels: three slices (remainder of 32)
    cases = [(pa.OP_GRADIENT, pa.F32, 137, "k_tile<float, 0, 2>"),
             (pa.OP_DIVERGENCE_ADJOINT, pa.F32, 137, "k_tile<float, 3, 2>"),
             (pa.OP_DIVERGENCE, pa.F32, 137, "k_tile<float, 1, 2>"),
             (pa.OP_LAPLACIAN, pa.F32, 137, "k_tile<float, 4, 2>"),
             (pa.OP_LAPLACIAN, pa.F32, 160, "k_tile<float, 4, 2>"),
             (pa.OP_LAPLACIAN, pa.F32, 170, "k_tile<float, 4, 3>"),
             (pa.OP_GRADIENT, pa.F64, 137, "k_tile<double, 0, 2>"),
             # two level chunks of 69 and 68 levels: one whole slice each
             (pa.OP_DIVERGENCE, pa.F64, 137, "k_tile<double, 1, 1>"),
             (pa.OP_LAPLACIAN, pa.F64, 137, "k_tile<double, 4, 2>"),
             (pa.OP_GRADIENT, pa.BF16, 137, "k_tile<unsigned short, 0, 2>"),
             (pa.OP_LAPLACIAN, pa.BF16, 137, "k_tile<unsigned short, 4, 2>"),
             (pa.OP_GRADIENT, pa.F32, 19, "k_op<float, 0, 1>")]
    for op, dt, L, name in cases:
        shape, kernel = pa.describe(M, op, dt, L)
        assert kernel == name, (op, dt, L, kernel)
        assert shape["lds_tiles"] in (1, 2, 3)
    pa.set_tune(M, pa.OP_GRADIENT, pa.F32, dict(lds_tiles=2))
    assert pa.describe(M, pa.OP_GRADIENT, pa.F32, 137)[1] == "k_win<float, 0, 3>"
    pa.set_tune(M, pa.OP_GRADIENT, pa.F32, dict(lds_tiles=2, row_window=2, lanes_per_node=16, slices_per_iter=2))
    assert pa.describe(M, pa.OP_GRADIENT, pa.F32, 137)[1] == "k_op<float, 0, 2>"
    pa.set_tune(M, pa.OP_GRADIENT, pa.F32, None)
    with pytest.raises(pa.AtlasError):
        pa.describe(M, pa.OP_GRADIENT, pa.F32, 0)


def test_describe_names_the_one_pass_kernels():
    """The one-pass calls run the fused tile kernels (operator 7: gradient and
    Laplacian; 8: the divergence with the curl or the gradient adjoint) on
    their own default shapes, and their two operators one after the other
    when the shape is not the one-tile form."""
    M = pa.Mesh("O8", device=-1)
    cases = [(pa.OP_GRADIENT_LAPLACIAN, pa.F32, 137, "k_tile<float, 7, 2>"),
             (pa.OP_DIVERGENCE_CURL, pa.F32, 137, "k_tile<float, 8, 2>"),
             (pa.OP_DIVERGENCE_GRADIENT_ADJOINT, pa.F32, 137, "k_tile<float, 8, 2>"),
             # FP64: one slice per step for the gradient and Laplacian; the
             # divergence pairs on whole columns (160 KiB tiles), two slices
             (pa.OP_GRADIENT_LAPLACIAN, pa.F64, 137, "k_tile<double, 7, 1>"),
             (pa.OP_DIVERGENCE_GRADIENT_ADJOINT, pa.F64, 137, "k_tile<double, 8, 2>"),
             (pa.OP_DIVERGENCE_GRADIENT_ADJOINT, pa.BF16, 137, "k_tile<unsigned short, 8, 2>"),
             (pa.OP_DIVERGENCE_GRADIENT_ADJOINT, pa.F32, 19, "two calls")]
    for op, dt, L, name in cases:
        assert pa.describe(M, op, dt, L)[1] == name, (op, dt, L)
    shape = pa.describe(M, pa.OP_DIVERGENCE_GRADIENT_ADJOINT, pa.F32, 137)[0]
    assert (shape["tile_kb"], shape["waves_per_block"]) == (80, 16)
    shape = pa.describe(M, pa.OP_DIVERGENCE_GRADIENT_ADJOINT, pa.F64, 137)[0]
    assert (shape["tile_kb"], shape["waves_per_block"]) == (160, 8)
    # BF16 1-ring operators: 16-wave workgroups (80 KiB for vector input,
    # 64 KiB for scalar input); the single divergence keeps its own shape
    for op, kb in ((pa.OP_DIVERGENCE, 80), (pa.OP_GRADIENT_ADJOINT, 80), (pa.OP_GRADIENT, 64),
                   (pa.OP_DIVERGENCE_ADJOINT, 64)):
        shape = pa.describe(M, op, pa.BF16, 137)[0]
        assert (shape["tile_kb"], shape["waves_per_block"]) == (kb, 16), op
    shape = pa.describe(M, pa.OP_DIVERGENCE, pa.F32, 137)[0]
    assert (shape["tile_kb"], shape["waves_per_block"]) == (64, 8)
    # the pairs read the divergence's shape entry
    pa.set_tune(M, pa.OP_DIVERGENCE, pa.F32, dict(lds_tiles=2))
    assert pa.describe(M, pa.OP_DIVERGENCE_GRADIENT_ADJOINT, pa.F32, 137)[1] == "two calls"
    pa.set_tune(M, pa.OP_DIVERGENCE, pa.F32, None)
    with pytest.raises(pa.AtlasError):
        pa.describe(M, pa.OP_GRADIENT_LAPLACIAN | pa.OP_DIVERGENCE_CURL, pa.F32, 137)


def test_tuning_cache_applies_shapes(tmp_path):
    """A JSON cache of tuned shapes is read back and set on the mesh."""
    from paper_1908_07038_amd import tuning
    M = pa.Mesh("O8", device=-1)
    path = str(tmp_path / "tune.json")
    cache = {tuning.cache_key(M, "gradient", "float32", 137): {"shape": {"lds_tiles": 2, "row_window": 1}, "ms": 1.0},
             tuning.cache_key(M, "laplacian", "float64", 91): {"shape": {"lds_tiles": 2}, "ms": 2.0}}
    tuning.save_cache(path, cache)
    back = tuning.load_cache(path)
    assert back == cache
    applied = tuning.apply_cache(M, back, 137)
    assert applied == ["O8/gradient/float32/137"]
    assert pa.describe(M, pa.OP_GRADIENT, pa.F32, 137)[1] == "k_win<float, 0, 3>"
    assert pa.describe(M, pa.OP_LAPLACIAN, pa.F64, 137)[1].startswith("k_tile<")
    assert tuning.apply_cache(M, back, 91, ops=["laplacian"]) == ["O8/laplacian/float64/91"]
    assert pa.describe(M, pa.OP_LAPLACIAN, pa.F64, 91)[1] == "k_op<double, 4, 3>"
    assert tuning.load_cache(str(tmp_path / "missing.json")) == {}
