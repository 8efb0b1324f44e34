"""GPU parity of grid-to-grid remapping (Section 4.3, Figures 4-6): the HIP
kernel (through the C ABI) against the oracle's brute-force location and
FP64 interpolation.

Cases: the paper's O32 -> F8, an identity remap (O16 -> O16, every point on
a node), a finer target (O12 -> F30), a target sharing the source's
latitudes (O24 -> F24, points on edges and nodes) and a reduced target
(O20 -> O9); levels 1, 10 (several points per wave), 33, 64, 65 and 137
(one point per wave, ragged slices); the transpose also at 300 levels (a
column in several blocks of levels).  Bars as for the operators: FP64 1e-12,
FP32 1e-5 (total, against the FP64 input), BF16 4e-3 (against the oracle on
the bf16-rounded input), normwise and element-wise (also per level)."""
import functools

import numpy as np
import pytest
import torch

import paper_1908_07038_amd as pa
import workloads as W
from oracle import remap as R
from _oracle_cache import mesh_and_dual, coords
from _parity import check

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
TOL = {torch.float64: 1e-12, torch.float32: 1e-5, torch.bfloat16: 4e-3}
_MESHES = {}


def gpu_mesh(N):
    if N not in _MESHES:
        _MESHES[N] = pa.Mesh(f"O{N}", device=0)
    return _MESHES[N]


@functools.lru_cache(maxsize=None)
def oracle_remap(src, dst):
    m, _ = mesh_and_dual(int(src[1:]))
    _, nodes, w = R.locate(m.grid.xyz, m.tris, R.TargetGrid(dst).xyz)
    return nodes, w


@functools.lru_cache(maxsize=None)
def gpu_remap(src, dst):
    return pa.Remap(gpu_mesh(int(src[1:])), dst)


def _input(N, L, seed):
    m, _ = mesh_and_dual(N)
    s = W.sh_field(coords(m), min(12, 2 * N), seed)
    return W.scaled_levels(s, L, 0.1) + W.normal((m.nnodes, L), seed + 1, 1e-3)


CASES = [("O32", "F8"), ("O16", "O16"), ("O12", "F30"), ("O24", "F24"), ("O20", "O9"), ("O1", "F6")]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
@pytest.mark.parametrize("L", [1, 10, 33, 64, 65, 137])
@pytest.mark.parametrize("src,dst", CASES)
def test_remap_parity(src, dst, L, dtype):
    print(f"case remap {src}->{dst} L {L} {dtype}", flush=True)
    r = gpu_remap(src, dst)
    x = _input(int(src[1:]), L, 40 + L)
    xt = torch.from_numpy(x).to(DEV).to(dtype)
    y = r(xt)
    torch.cuda.synchronize()
    assert y.shape == (r.npoints, L) and y.dtype == dtype
    nodes, w = oracle_remap(src, dst)
    xin = xt.double().cpu().numpy() if dtype == torch.bfloat16 else x
    ref = R.apply(nodes, w, xin)
    check(y.double().cpu().numpy(), ref, TOL[dtype], ("remap", src, dst, L, str(dtype)), per_level=True)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_remap_reproduces_constants_and_is_deterministic(dtype):
    r = gpu_remap("O32", "F8")
    M = gpu_mesh(32)
    c = torch.full((M.nnodes, 70), 2.5, dtype=dtype, device=DEV)
    y = r(c)
    tol = 1e-15 if dtype == torch.float64 else 1e-6
    assert torch.allclose(y, torch.full_like(y, 2.5), rtol=0, atol=2.5 * tol)
    x = torch.from_numpy(_input(32, 70, 5)).to(DEV).to(dtype)
    assert torch.equal(r(x), r(x))
    # out= is written in place, on the current stream
    out = torch.empty((r.npoints, 70), dtype=dtype, device=DEV)
    assert r(x, out=out) is out and torch.equal(out, r(x))


def test_remap_argument_errors():
    r = gpu_remap("O32", "F8")
    M = gpu_mesh(32)
    x = torch.zeros((M.nnodes, 4), dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError):
        r(x, out=torch.empty((r.npoints, 5), dtype=torch.float32, device=DEV))
    with pytest.raises(ValueError):
        r(torch.zeros((M.nnodes + 1, 4), dtype=torch.float32, device=DEV))
    with pytest.raises(ValueError):
        r(x.t().contiguous().t())
    with pytest.raises(TypeError):
        r(x.to(torch.float16))
    # dst overlapping src is refused by the library
    big = torch.zeros((M.nnodes + r.npoints, 4), dtype=torch.float32, device=DEV)
    with pytest.raises(pa.AtlasError) as e:
        r(big[:M.nnodes], out=big[M.nnodes - 1:M.nnodes - 1 + r.npoints])
    assert e.value.code == -1


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
@pytest.mark.parametrize("L", [1, 10, 33, 65, 137, 300])
@pytest.mark.parametrize("src,dst", [("O32", "F8"), ("O12", "F30"), ("O24", "F24")])
def test_remap_adjoint_parity(src, dst, L, dtype):
    """The transpose kernel against the oracle's scatter, and (FP64) the
    dot-product identity <R x, y> = <x, R^T y>."""
    print(f"case remap adjoint {src}->{dst} L {L} {dtype}", flush=True)
    r = gpu_remap(src, dst)
    y = torch.from_numpy(np.random.default_rng(7 + L).standard_normal((r.npoints, L))).to(DEV).to(dtype)
    fb = r.adjoint(y)
    torch.cuda.synchronize()
    nodes, w = oracle_remap(src, dst)
    ref = R.apply_adjoint(nodes, w, y.double().cpu().numpy(), r.mesh.nnodes)
    check(fb.double().cpu().numpy(), ref, TOL[dtype], ("remap adjoint", src, dst, L, str(dtype)), per_level=True)
    if dtype == torch.float64:
        x = torch.from_numpy(_input(int(src[1:]), L, 60 + L)).to(DEV)
        rx = r(x)
        lhs = float((rx * y).sum())
        rhs = float((x * fb).sum())
        assert abs(lhs - rhs) <= 1e-13 * float(rx.norm() * y.norm()), (lhs, rhs)


def test_remap_autograd_gradcheck():
    M = gpu_mesh(4)
    r = pa.Remap(M, "F2")
    f = torch.from_numpy(np.random.default_rng(3).standard_normal((M.nnodes, 3))).to(DEV).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: pa.remap(r, t), (f,), eps=1e-6, atol=1e-8)
