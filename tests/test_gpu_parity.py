"""GPU parity: the HIP kernels (through the C ABI) against the FP64 oracle.

Bars: normwise relative L2 ||gpu - oracle|| / ||oracle|| and element-wise
max |gpu - oracle| / max |oracle|, both under the tolerance, the element-wise
one also per level and on the polar rows and the nodes of degree 5 and 7
separately (tests/_parity.py):
  FP64: <= 1e-12.
  FP32: <= 1e-5 against the oracle applied to the FP32-rounded input (the
    kernel's own error), and <= 1e-5 normwise against the oracle applied to
    the FP64 input (total error, the input rounding included: a Laplacian of
    a field with a large level offset amplifies that rounding to ~1e-5 at
    single nodes, so the total error is bounded normwise only).
  BF16 storage: <= 4e-3 against the oracle applied to the bf16-rounded input
    (each output is rounded once to bfloat16, whose half-ulp is at most 2^-8
    of the value; FP32 arithmetic adds ~1e-6).  The total error against the
    FP64 input is printed, not bounded here.
Sizes span several workgroups, ragged level tails (nlev not a multiple of 64)
and every launch form: several nodes per wave (nlev <= 32) and one node per
wave (nlev > 32).
"""
import numpy as np
import pytest
import torch

import paper_1908_07038_amd as pa
import workloads as W
from oracle import nabla
from _oracle_cache import mesh_and_dual, coords
from _parity import check, special_groups

pytestmark = pytest.mark.gpu

R = 6371220.0
DEV = torch.device("cuda", 0)
TOL = {torch.float64: 1e-12, torch.float32: 1e-5, torch.bfloat16: 4e-3}
_MESHES = {}


def gpu_mesh(N):
    if N not in _MESHES:
        _MESHES[N] = pa.Mesh(f"O{N}", radius=R, device=0)
    return _MESHES[N]


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


OPS = {
    "gradient": (1, pa.gradient, nabla.gradient),
    "divergence": (2, pa.divergence, nabla.divergence),
    "laplacian": (1, pa.laplacian, nabla.laplacian),
    "gradient_adjoint": (2, pa.gradient_adjoint, nabla.gradient_adjoint),
    "divergence_adjoint": (1, pa.divergence_adjoint, nabla.divergence_adjoint),
    "curl": (2, pa.curl, nabla.curl),
    "curl_adjoint": (1, pa.curl_adjoint, nabla.curl_adjoint),
}


def _input(N, L, comps, seed):
    m, _ = mesh_and_dual(N)
    if comps == 1:
        # smooth content with a level-wise scale plus a little noise
        s = W.sh_field(coords(m), min(12, 2 * N), seed)
        return W.scaled_levels(s, L, 0.1) + W.normal((m.nnodes, L), seed + 1, 1e-3)
    return W.normal((m.nnodes, L, 2), seed)


def _run(name, N, L, dtype, seed=11):
    comps, gpu_fn, ora_fn = OPS[name]
    m, g = mesh_and_dual(N)
    x = _input(N, L, comps, seed)
    xt = torch.from_numpy(x).to(DEV).to(dtype)
    y = gpu_fn(gpu_mesh(N), xt)
    torch.cuda.synchronize()
    xin = xt.double().cpu().numpy() if dtype != torch.float64 else x
    ref = ora_fn(m, g, xin)
    return y.double().cpu().numpy(), ref, x, m, g


CASES = [(4, 1), (4, 3), (32, 10), (32, 19), (32, 33), (32, 64), (32, 137), (1, 5), (2, 70)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
@pytest.mark.parametrize("name", list(OPS))
@pytest.mark.parametrize("N,L", CASES)
def test_parity(name, N, L, dtype):
    print(f"case {name} O{N} x {L} {dtype}", flush=True)
    y, ref, x, m, g = _run(name, N, L, dtype)
    err, emax = check(y, ref, TOL[dtype], (name, N, L, str(dtype)), per_level=True, groups=special_groups(m))
    print(f"  rel L2 {err:.2e} max {emax:.2e}")
    if dtype != torch.float64:
        total = rel(y, OPS[name][2](m, g, x))
        print(f"  kernel-only {err:.2e} total {total:.2e}")
        if dtype == torch.float32:
            assert total <= TOL[dtype], (name, N, L, "total", total)


TILE_CODES = {torch.float64: pa.F64, torch.float32: pa.F32}
OP_BITS = {"gradient": pa.OP_GRADIENT, "divergence": pa.OP_DIVERGENCE, "laplacian": pa.OP_LAPLACIAN,
           "gradient_adjoint": pa.OP_GRADIENT_ADJOINT, "divergence_adjoint": pa.OP_DIVERGENCE_ADJOINT,
           "curl": pa.OP_CURL, "curl_adjoint": pa.OP_CURL_ADJOINT}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(OPS))
@pytest.mark.parametrize("form", [1, 3], ids=["persistent", "one_tile"])
@pytest.mark.parametrize("N,L,kb", [(32, 137, 0), (32, 33, 8), (2, 70, 64), (32, 200, 16), (8, 96, 0),
                                    (8, 65, 0), (8, 40, 0)])
def test_parity_lds_tiles(name, N, L, kb, form, dtype):
    """The LDS tile paths against the oracle: whole columns and level chunks,
    remainders past the whole 64-level slices of 1 (65), 6 (70), 8 (200), 9
    (137) and 32 (96) levels, which the one-tile form evaluates in its packed
    tail pass, and columns of 33 and 40 levels (one partial slice)."""
    print(f"case tiles {name} O{N} x {L} kb {kb} form {form} {dtype}", flush=True)
    M = gpu_mesh(N)
    pa.set_tune(M, OP_BITS[name], TILE_CODES[dtype], dict(lds_tiles=form, tile_kb=kb))
    try:
        y, ref, _, m, _ = _run(name, N, L, dtype)
    finally:
        pa.set_tune(M, OP_BITS[name], TILE_CODES[dtype], None)
    check(y, ref, TOL[dtype], (name, N, L, kb, form, str(dtype)), per_level=True, groups=special_groups(m))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_config_o32(dtype):
    """O32 x 10: SH sum to degree 10 with scale 1 + 0.1 k; grad, div(grad f), lap."""
    M = gpu_mesh(32)
    m, g = mesh_and_dual(32)
    f = W.workload_o32(coords(m))
    ft = torch.from_numpy(f).to(DEV).to(dtype)
    gr = pa.gradient(M, ft)
    dv = pa.divergence(M, gr)
    lp = pa.laplacian(M, ft)
    torch.cuda.synchronize()
    og = nabla.gradient(m, g, f)
    od = nabla.divergence(m, g, og)
    ol = nabla.laplacian(m, g, f)
    fk = ft.double().cpu().numpy()                 # the input as the kernel sees it
    ogk = nabla.gradient(m, g, fk)
    kern = {"gradient": ogk, "divergence": nabla.divergence(m, g, ogk), "laplacian": nabla.laplacian(m, g, fk)}
    for what, y, r in [("gradient", gr, og), ("divergence", dv, od), ("laplacian", lp, ol)]:
        yy = y.double().cpu().numpy()
        check(yy, kern[what], TOL[dtype], what, per_level=True, groups=special_groups(m))
        assert rel(yy, r) <= TOL[dtype], (what, "total", rel(yy, r))
    # the fused and two-pass Laplacian agree with div(grad f) computed on the GPU
    np.testing.assert_allclose(lp.double().cpu().numpy(), dv.double().cpu().numpy(),
                               rtol=0, atol=TOL[dtype] * np.abs(ol).max() * 10)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_two_pass_laplacian(dtype):
    M = gpu_mesh(32)
    m, g = mesh_and_dual(32)
    f = _input(32, 137, 1, 5)
    ft = torch.from_numpy(f).to(DEV).to(dtype)
    ws = torch.empty((M.nnodes, 137, 2), dtype=dtype, device=DEV)
    l2 = pa.laplacian(M, ft, workspace=ws)
    gr = pa.gradient(M, ft)
    torch.cuda.synchronize()
    assert torch.equal(ws, gr)               # the workspace holds the gradient
    yy = l2.double().cpu().numpy()
    check(yy, nabla.laplacian(m, g, ft.double().cpu().numpy()), TOL[dtype], "two-pass laplacian",
          per_level=True, groups=special_groups(m))
    assert rel(yy, nabla.laplacian(m, g, f)) <= TOL[dtype]


def test_conservation_sums():
    M = gpu_mesh(32)
    m, g = mesh_and_dual(32)
    uv = W.normal((m.nnodes, 37, 2), 3)
    d = pa.divergence(M, torch.from_numpy(uv).to(DEV))
    s, a = pa.conservation(M, d)
    torch.cuda.synchronize()
    os_, oa = nabla.conservation(m, g, d.cpu().numpy())
    s, a = s.cpu().numpy(), a.cpu().numpy()
    assert np.all(np.abs(s - os_) <= 1e-13 * oa)
    np.testing.assert_allclose(a, oa, rtol=1e-13)
    assert np.all(np.abs(s) <= 1e-13 * a)            # discrete Gauss theorem
    # FP32 and BF16 inputs accumulate in FP64 too
    for dt in (torch.float32, torch.bfloat16):
        d2 = d.to(dt)
        s2, a2 = pa.conservation(M, d2)
        os2, oa2 = nabla.conservation(m, g, d2.double().cpu().numpy())
        assert np.all(np.abs(s2.cpu().numpy() - os2) <= 1e-13 * oa2)
        np.testing.assert_allclose(a2.cpu().numpy(), oa2, rtol=1e-13)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
def test_deterministic_reruns(dtype):
    M = gpu_mesh(32)
    x = torch.from_numpy(_input(32, 137, 1, 9)).to(DEV).to(dtype)
    w = torch.from_numpy(_input(32, 137, 2, 10)).to(DEV).to(dtype)
    for fn, inp in [(pa.gradient, x), (pa.divergence, w), (pa.laplacian, x),
                    (pa.gradient_adjoint, w), (pa.divergence_adjoint, x)]:
        a = fn(M, inp)
        b = fn(M, inp)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


def test_gradient_of_constant_is_zero():
    M = gpu_mesh(32)
    for dt in (torch.float64, torch.float32, torch.bfloat16):
        f = torch.full((M.nnodes, 65), 3.25, dtype=dt, device=DEV)
        assert torch.count_nonzero(pa.gradient(M, f)).item() == 0
        assert torch.count_nonzero(pa.laplacian(M, f)).item() == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_dot_product_identities(dtype):
    M = gpu_mesh(32)
    V, L = M.nnodes, 91
    x = torch.from_numpy(W.normal((V, L), 1)).to(DEV).to(dtype)
    y = torch.from_numpy(W.normal((V, L, 2), 2)).to(DEV).to(dtype)
    # scale of the rounding: ||G x|| ||y|| (Cauchy-Schwarz), not the
    # cancelling sum itself
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    gx = pa.gradient(M, x).double()
    lhs = (gx * y.double()).sum().item()
    rhs = (x.double() * pa.gradient_adjoint(M, y).double()).sum().item()
    assert abs(lhs - rhs) <= tol * (gx.norm() * y.double().norm()).item()
    dy = pa.divergence(M, y).double()
    lhs = (dy * x.double()).sum().item()
    rhs = (y.double() * pa.divergence_adjoint(M, x).double()).sum().item()
    assert abs(lhs - rhs) <= tol * (dy.norm() * x.double().norm()).item()
    cy = pa.curl(M, y).double()
    lhs = (cy * x.double()).sum().item()
    rhs = (y.double() * pa.curl_adjoint(M, x).double()).sum().item()
    assert abs(lhs - rhs) <= tol * (cy.norm() * x.double().norm()).item()


def test_autograd_gradcheck():
    M = gpu_mesh(4)
    f = torch.from_numpy(W.normal((M.nnodes, 2), 4)).to(DEV).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: pa.grad(M, t), (f,), eps=1e-6, atol=1e-7)
    uv = torch.from_numpy(W.normal((M.nnodes, 2, 2), 5)).to(DEV).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: pa.div(M, t), (uv,), eps=1e-6, atol=1e-7)
    assert torch.autograd.gradcheck(lambda t: pa.lap(M, t), (f,), eps=1e-6, atol=1e-6)
    assert torch.autograd.gradcheck(lambda t: pa.rot(M, t), (uv,), eps=1e-6, atol=1e-7)
    # the one-pass pairs: both outputs, and each alone (the other's cotangent absent)
    assert torch.autograd.gradcheck(lambda t: pa.grad_lap(M, t), (f,), eps=1e-6, atol=1e-6)
    assert torch.autograd.gradcheck(lambda t: pa.grad_lap(M, t)[1], (f,), eps=1e-6, atol=1e-6)
    assert torch.autograd.gradcheck(lambda t: pa.div_rot(M, t), (uv,), eps=1e-6, atol=1e-7)
    assert torch.autograd.gradcheck(lambda t: pa.div_rot(M, t)[0], (uv,), eps=1e-6, atol=1e-7)
    assert torch.autograd.gradcheck(lambda t: pa.div_gradt(M, t), (uv,), eps=1e-6, atol=1e-7)
    assert torch.autograd.gradcheck(lambda t: pa.div_gradt(M, t)[1], (uv,), eps=1e-6, atol=1e-7)


def test_curl_of_solid_body_rotation():
    """GPU curl of the rotation about the polar axis against 2 sin(lat)/R
    (FP64; the same bound the oracle meets at O64)."""
    import math
    M = gpu_mesh(32)
    m, g = mesh_and_dual(32)
    gr = m.grid
    uv = np.zeros((m.nnodes, 1, 2))
    uv[:, 0, 0] = gr.coslat            # u = R cos(lat) * (1 / R)
    z = pa.curl(M, torch.from_numpy(uv).to(DEV)).cpu().numpy()[:, 0]
    ex = 2.0 * gr.sinlat / R
    assert math.sqrt(np.sum(g.V * (z - ex) ** 2) / np.sum(g.V * ex ** 2)) < 1e-2
    np.testing.assert_allclose(z, nabla.curl(m, g, uv)[:, 0], rtol=0, atol=1e-12 * np.abs(ex).max())


def test_argument_errors():
    M = gpu_mesh(4)
    f = torch.zeros((M.nnodes, 4), dtype=torch.float32, device=DEV)
    g = torch.zeros((M.nnodes, 4, 2), dtype=torch.float32, device=DEV)
    L = pa.lib()
    assert L.atlas_nabla_gradient(M.handle, 1, 0, f.data_ptr(), g.data_ptr(), None) == -6
    assert L.atlas_nabla_gradient(M.handle, 7, 4, f.data_ptr(), g.data_ptr(), None) == -5
    assert L.atlas_nabla_gradient(M.handle, 1, 4, None, g.data_ptr(), None) == -1
    assert L.atlas_nabla_gradient(M.handle, 1, 4, f.data_ptr() + 2, g.data_ptr(), None) == -1
    assert L.atlas_nabla_gradient(M.handle, 1, 4, f.data_ptr(), g.data_ptr() + 4, None) == -1
    assert L.atlas_nabla_gradient(M.handle, 1, 4, g.data_ptr(), g.data_ptr(), None) == -1   # overlap
    with pytest.raises(ValueError):
        pa.gradient(M, g)
    # caller-given outputs and workspaces must match the input
    with pytest.raises(ValueError):
        pa.laplacian(M, f, out=torch.empty((M.nnodes, 4), dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        pa.laplacian(M, f, workspace=torch.empty((M.nnodes, 3, 2), dtype=torch.float32, device=DEV))
    with pytest.raises(ValueError):
        pa.gradient(M, f, out=torch.empty((M.nnodes, 4, 3), dtype=torch.float32, device=DEV))
    torch.cuda.synchronize()


SHAPES = [dict(lanes_per_node=p, slices_per_iter=u, waves_per_block=w, nodes_per_wave=n, xcd_remap=x,
               band_rows=h, run_nodes=r, nt_stores=nt, row_window=rw)
          for (p, u, w, n, x, h, r, nt, rw) in [(16, 1, 1, 1, 2, 1, 1, 1, 2), (16, 3, 4, 2, 1, 0, 0, 2, 2),
                                                (32, 2, 2, 4, 1, 7, 3, 1, 2), (64, 3, 4, 8, 2, 64, 64, 2, 2),
                                                (64, 1, 1, 3, 1, 1000, 5, 1, 2), (32, 3, 4, 1, 2, 2, 1000, 2, 2),
                                                (0, 1, 1, 1, 2, 1, 1, 1, 1), (0, 3, 4, 2, 1, 0, 0, 2, 1),
                                                (0, 2, 2, 4, 1, 7, 3, 1, 1), (0, 3, 4, 8, 2, 64, 64, 2, 0),
                                                (0, 1, 1, 3, 1, 1000, 5, 1, 1), (0, 2, 4, 1, 2, 2, 1000, 2, 1)]]
# LDS tiles (FP32/FP64 only; other dtypes ignore the switch): budgets that
# force whole columns, level chunks and tiny tiles, every wave count
SHAPES += [dict(lds_tiles=3, tile_kb=kb, waves_per_block=w, slices_per_iter=u, band_rows=h, run_nodes=r,
                xcd_remap=x, nt_stores=nt)
           for (kb, w, u, h, r, x, nt) in [(0, 4, 0, 0, 0, 0, 0), (64, 2, 3, 32, 16, 1, 2), (8, 1, 1, 1, 1, 2, 1),
                                           (24, 4, 2, 4, 8, 1, 1), (16, 2, 3, 1000, 1000, 2, 2),
                                           (40, 1, 2, 7, 3, 1, 2), (160, 16, 0, 4, 8, 1, 0),
                                           (48, 16, 3, 3, 8, 2, 0)]]
# persistent double-buffered tiles: wave splits, workgroups per CU, lanes per node
SHAPES += [dict(lds_tiles=1, tile_kb=kb, tile_waves=c, producer_waves=pw, tile_wgs_per_cu=g, lanes_per_node=p,
                slices_per_iter=u, band_rows=h, run_nodes=r, xcd_remap=x, nt_stores=nt)
           for (kb, c, pw, g, p, u, h, r, x, nt) in [(0, 0, 0, 0, 0, 0, 0, 0, 0, 0), (64, 7, 1, 1, 64, 3, 32, 16, 1, 2),
                                                     (8, 1, 1, 4, 16, 1, 1, 1, 2, 1), (24, 4, 4, 3, 32, 2, 4, 8, 1, 1),
                                                     (16, 2, 2, 4, 0, 3, 1000, 1000, 2, 2),
                                                     (40, 6, 2, 2, 16, 2, 7, 3, 1, 2),
                                                     (64, 12, 4, 1, 32, 3, 5, 8, 1, 0)]]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
def test_launch_shape_invariance(dtype):
    """Every tunable launch shape gives the same values (up to the sign of
    zero) as the default one: the per-element slot order never changes."""
    M = gpu_mesh(32)
    codes = {torch.float64: pa.F64, torch.float32: pa.F32, torch.bfloat16: pa.BF16}
    for L in (137, 96, 91, 65, 40, 19):
        x = torch.from_numpy(_input(32, L, 1, 21)).to(DEV).to(dtype)
        w = torch.from_numpy(_input(32, L, 2, 22)).to(DEV).to(dtype)
        cases = [(pa.OP_GRADIENT, pa.gradient, x), (pa.OP_DIVERGENCE, pa.divergence, w),
                 (pa.OP_LAPLACIAN, pa.laplacian, x), (pa.OP_GRADIENT_ADJOINT, pa.gradient_adjoint, w),
                 (pa.OP_DIVERGENCE_ADJOINT, pa.divergence_adjoint, x), (pa.OP_CURL, pa.curl, w),
                 (pa.OP_CURL_ADJOINT, pa.curl_adjoint, x)]
        for op, fn, inp in cases:
            ref = fn(M, inp)
            for sh in SHAPES:
                if dtype == torch.float64 and sh.get("tile_waves", 0) + sh.get("producer_waves", 0) > 8:
                    continue   # FP64 persistent tiles take at most 8 waves
                pa.set_tune(M, op, codes[dtype], sh)
                y = fn(M, inp)
                torch.cuda.synchronize()
                assert torch.equal(y, ref), (op, L, sh)
            pa.set_tune(M, op, codes[dtype], None)


def test_tuner_returns_a_valid_shape():
    M = gpu_mesh(32)
    x = torch.from_numpy(_input(32, 137, 1, 23)).to(DEV).float()
    y = torch.empty((M.nnodes, 137, 2), dtype=torch.float32, device=DEV)
    shape, ms = pa.tune(M, pa.OP_GRADIENT, x, y, reps=2)
    assert ms > 0 and shape["waves_per_block"] in (1, 2, 4)
    # the tuner leaves the output of its last candidate, identical to any shape's
    pa.set_tune(M, pa.OP_GRADIENT, pa.F32, shape)
    tuned = pa.gradient(M, x)
    pa.set_tune(M, pa.OP_GRADIENT, pa.F32, None)
    ref = pa.gradient(M, x)
    torch.cuda.synchronize()
    assert torch.equal(tuned, ref) and torch.equal(y, ref)


def test_bf16_unaligned_field_falls_back():
    """BF16 tiles copy whole dwords: a field that starts 2 bytes into a dword
    takes the row-window walk and still gives the same bits."""
    M = gpu_mesh(32)
    L = 137
    x = torch.from_numpy(_input(32, L, 1, 31)).to(DEV).to(torch.bfloat16)
    ref = pa.gradient(M, x)
    lap_ref = pa.laplacian(M, x)
    buf = torch.empty(M.nnodes * L + 1, dtype=torch.bfloat16, device=DEV)
    xu = buf[1:].view(M.nnodes, L)
    xu.copy_(x)
    assert xu.data_ptr() % 4 == 2
    torch.cuda.synchronize()
    assert torch.equal(pa.gradient(M, xu), ref)
    assert torch.equal(pa.laplacian(M, xu), lap_ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
def test_gradient_laplacian_in_one_pass(dtype):
    """The fused pass gives the two operators' values (up to the sign of
    zero) at every level count -- whole 64-level slices, packed remainders,
    level chunks, columns of at most 32 levels (the two calls one after the
    other) -- and on every Laplacian launch shape it runs with; against the
    oracle through the separate calls' parity."""
    M = gpu_mesh(32)
    codes = {torch.float64: pa.F64, torch.float32: pa.F32, torch.bfloat16: pa.BF16}
    shapes = [None, dict(lds_tiles=3, tile_kb=16), dict(lds_tiles=3, tile_levels=50, waves_per_block=4),
              dict(lds_tiles=3, tile_kb=24, slices_per_iter=1, band_rows=2), dict(lds_tiles=2)]
    for L in (137, 96, 70, 40, 19, 1):
        print(f"case gradient_laplacian L {L} {dtype}", flush=True)
        x = torch.from_numpy(_input(32, L, 1, 31)).to(DEV).to(dtype)
        for sh in shapes:
            pa.set_tune(M, pa.OP_LAPLACIAN, codes[dtype], sh)
            try:
                g, lp = pa.gradient_laplacian(M, x)
                g0 = pa.gradient(M, x)
                l0 = pa.laplacian(M, x)
                torch.cuda.synchronize()
            finally:
                pa.set_tune(M, pa.OP_LAPLACIAN, codes[dtype], None)
            assert torch.equal(g + 0.0, g0 + 0.0), (L, sh)
            assert torch.equal(lp + 0.0, l0 + 0.0), (L, sh)
    # outputs given; overlapping outputs are refused
    x = torch.from_numpy(_input(32, 137, 1, 32)).to(DEV).to(dtype)
    g = torch.empty((M.nnodes, 137, 2), dtype=dtype, device=DEV)
    lp = torch.empty((M.nnodes, 137), dtype=dtype, device=DEV)
    assert pa.gradient_laplacian(M, x, g, lp)[0] is g
    with pytest.raises(pa.AtlasError):
        pa.gradient_laplacian(M, x, g, g.view(-1)[:M.nnodes * 137].view(M.nnodes, 137))


def _divergence_pair_case(dtype, fused, second, name):
    """The divergence and a second operator of one vector field in one pass
    give the two calls' values (up to the sign of zero) at every level count
    and on the divergence launch shapes it runs with."""
    M = gpu_mesh(32)
    codes = {torch.float64: pa.F64, torch.float32: pa.F32, torch.bfloat16: pa.BF16}
    shapes = [None, dict(lds_tiles=3, tile_kb=16), dict(lds_tiles=3, tile_levels=50, waves_per_block=4),
              dict(lds_tiles=3, tile_kb=24, slices_per_iter=1, band_rows=2), dict(lds_tiles=2)]
    for L in (137, 96, 70, 40, 19, 1):
        print(f"case {name} L {L} {dtype}", flush=True)
        uv = torch.from_numpy(_input(32, L, 2, 33)).to(DEV).to(dtype)
        for sh in shapes:
            pa.set_tune(M, pa.OP_DIVERGENCE, codes[dtype], sh)
            try:
                d, z = fused(M, uv)
                d0 = pa.divergence(M, uv)
                z0 = second(M, uv)
                torch.cuda.synchronize()
            finally:
                pa.set_tune(M, pa.OP_DIVERGENCE, codes[dtype], None)
            assert torch.equal(d + 0.0, d0 + 0.0), (L, sh)
            assert torch.equal(z + 0.0, z0 + 0.0), (L, sh)
    uv = torch.from_numpy(_input(32, 137, 2, 34)).to(DEV).to(dtype)
    d = torch.empty((M.nnodes, 137), dtype=dtype, device=DEV)
    with pytest.raises(pa.AtlasError):
        fused(M, uv, d, d)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
def test_divergence_curl_in_one_pass(dtype):
    """Divergence and curl of one vector field in one pass equal the two calls."""
    _divergence_pair_case(dtype, pa.divergence_curl, pa.curl, "divergence_curl")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
def test_divergence_gradient_adjoint_in_one_pass(dtype):
    """Divergence and gradient adjoint of one vector field in one pass equal
    the two calls (whose parity with the oracle is tested above)."""
    _divergence_pair_case(dtype, pa.divergence_gradient_adjoint, pa.gradient_adjoint,
                          "divergence_gradient_adjoint")
