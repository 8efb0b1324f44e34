"""The benchmark's step captured into a HIP graph: once every tiling and
record table a call needs has been built by an eager call, the single-field
calls launch kernels only (no allocation, no copy, no memset), so the whole
step - gradient and Laplacian in one pass, divergence and gradient adjoint
in one pass, the divergence adjoint and the allocation-free conservation
sums, curl and the remap with its transpose - records into one graph.  The
graph is replayed three times, with eager calls on other fields and
synchronisations between the replays, and every replay must equal the eager
results bit for bit."""
import pytest
import torch

import paper_1908_07038_amd as pa
import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16], ids=["f64", "f32", "bf16"])
def test_step_replays_in_a_graph(dtype):
    M = pa.Mesh("O32", radius=6371220.0, device=0)
    r = pa.Remap(M, "F16")
    V, L = M.nnodes, 137
    f = torch.from_numpy(W.normal((V, L), 51)).to(DEV).to(dtype)
    g = torch.empty((V, L, 2), dtype=dtype, device=DEV)
    lp = torch.empty((V, L), dtype=dtype, device=DEV)
    d = torch.empty((V, L), dtype=dtype, device=DEV)
    fT = torch.empty((V, L), dtype=dtype, device=DEV)
    gT = torch.empty((V, L, 2), dtype=dtype, device=DEV)
    z = torch.empty((V, L), dtype=dtype, device=DEV)
    y = torch.empty((r.npoints, L), dtype=dtype, device=DEV)
    yT = torch.empty((V, L), dtype=dtype, device=DEV)
    s = torch.empty(L, dtype=torch.float64, device=DEV)
    a = torch.empty(L, dtype=torch.float64, device=DEV)
    outs = (g, lp, d, fT, gT, z, y, yT, s, a)

    def step():
        pa.gradient_laplacian(M, f, g, lp)
        pa.divergence_gradient_adjoint(M, g, d, fT)
        pa.divergence_adjoint(M, d, out=gT)
        pa.curl(M, g, out=z)
        pa.conservation_noalloc(M, d, s, a)
        r(f, out=y)
        r.adjoint(y, out=yT)

    step()                       # eager: builds the tilings and records
    torch.cuda.synchronize()
    ref = [t.clone() for t in outs]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    other = torch.from_numpy(W.normal((V, 91), 52)).to(DEV).to(dtype)
    for _ in range(3):
        for t in outs:
            t.fill_(float("nan"))
        # eager calls on another field (other tilings, the shared sums array)
        og, ol = pa.gradient_laplacian(M, other)
        pa.conservation_noalloc(M, pa.divergence(M, og), torch.empty(91, dtype=torch.float64, device=DEV),
                                torch.empty(91, dtype=torch.float64, device=DEV))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for t, e in zip(outs, ref):
            assert torch.equal(bits(t), bits(e))


def bits(t):
    """The tensor's bit patterns (so NaNs and signed zeros compare exactly)."""
    return t.view({8: torch.int64, 4: torch.int32, 2: torch.int16}[t.element_size()])
