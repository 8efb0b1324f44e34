"""The allocation-free conservation call against atlas_nabla_conservation.

Both run the same partial-sum and final kernels in the same order, so the
per-level sums must agree bit for bit; the allocation-free call keeps its
partials in the library's static per-GPU array.  Two calls in a row, the
second on a smaller input, check that nothing left in the array by the first
call leaks into the second; the FP64 oracle pins the values themselves.
"""
import numpy as np
import pytest
import torch

import paper_1908_07038_amd as pa
import workloads as W
from oracle import nabla
from tests._oracle_cache import mesh_and_dual

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _both(M, d):
    s0, a0 = pa.conservation(M, d)
    nlev = d.shape[1]
    s1 = torch.full((nlev,), float("nan"), dtype=torch.float64, device=DEV)
    a1 = torch.full((nlev,), float("nan"), dtype=torch.float64, device=DEV)
    pa.conservation_noalloc(M, d, s1, a1)
    torch.cuda.synchronize()
    return s0.cpu().numpy(), a0.cpu().numpy(), s1.cpu().numpy(), a1.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
def test_noalloc_conservation_matches_allocating_call(dtype):
    # first call: O32 x 137 levels (33 partial-sum blocks x 137 levels);
    # second: O16 x 19 levels, fewer blocks and levels, reading only what it writes
    for N, nlev, seed in ((32, 137, 41), (16, 19, 42)):
        M = pa.Mesh(f"O{N}", radius=6371220.0, device=0)
        m, g = mesh_and_dual(N)
        uv = torch.from_numpy(W.normal((M.nnodes, nlev, 2), seed)).to(DEV)
        d = pa.divergence(M, uv).to(dtype)
        s0, a0, s1, a1 = _both(M, d)
        print(f"O{N} x {nlev} {dtype}: max |sum| {np.abs(s1).max():.3e}, abs {a1.max():.3e}", flush=True)
        assert np.array_equal(s0, s1) and np.array_equal(a0, a1)
        os_, oa = nabla.conservation(m, g, d.double().cpu().numpy())
        assert np.all(np.abs(s1 - os_) <= 1e-13 * oa)
        np.testing.assert_allclose(a1, oa, rtol=1e-13)


def test_noalloc_conservation_full_size_levels_and_limit():
    # O320 (4096 partial-sum blocks): 137 levels fit the static array, 257 do not
    M = pa.Mesh("O320", radius=6371220.0, device=0)
    f = torch.from_numpy(W.normal((M.nnodes, 137), 43)).to(DEV).float()
    d = pa.divergence(M, pa.gradient(M, f))
    s0, a0, s1, a1 = _both(M, d)
    assert np.array_equal(s0, s1) and np.array_equal(a0, a1)
    big = torch.zeros((M.nnodes, 257), dtype=torch.float32, device=DEV)
    s = torch.empty(257, dtype=torch.float64, device=DEV)
    a = torch.empty(257, dtype=torch.float64, device=DEV)
    with pytest.raises(pa.AtlasError, match="at most 256 levels"):
        pa.conservation_noalloc(M, big, s, a)
    # the allocating call still takes it
    pa.conservation(M, big)
    torch.cuda.synchronize()


def test_noalloc_conservation_replays_in_a_graph():
    """Captured into a HIP graph (code under capture is what the call is for)
    and replayed three times, with eager calls on the same static array and
    synchronisations between the replays: every replay equals the eager
    result bit for bit."""
    M = pa.Mesh("O32", radius=6371220.0, device=0)
    nlev = 64
    d = pa.divergence(M, torch.from_numpy(W.normal((M.nnodes, nlev, 2), 44)).to(DEV))
    other = pa.divergence(M, torch.from_numpy(W.normal((M.nnodes, 91, 2), 45)).to(DEV)).float()
    s = torch.empty(nlev, dtype=torch.float64, device=DEV)
    a = torch.empty(nlev, dtype=torch.float64, device=DEV)
    pa.conservation_noalloc(M, d, s, a)        # eager: also sets up the array's address on this GPU
    torch.cuda.synchronize()
    s_ref, a_ref = s.clone(), a.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pa.conservation_noalloc(M, d, s, a)
    so = torch.empty(91, dtype=torch.float64, device=DEV)
    ao = torch.empty(91, dtype=torch.float64, device=DEV)
    for _ in range(3):
        s.fill_(float("nan"))
        a.fill_(float("nan"))
        pa.conservation_noalloc(M, other, so, ao)   # other contents in the shared array
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(s, s_ref) and torch.equal(a, a_ref)
