"""Full-size workloads on the GPU, in the launch configuration the benchmark
times, checked against the oracle on sampled outputs and by identities that
hold at any size.

* O640 and O1280 meshes: connectivity and indexing bit for bit, geometry to
  rounding, against the oracle's mesh.
* Remap O1280 x 137 -> F640 and its transpose (FP64, FP32, BF16; the
  transpose also at 164 levels in FP64, an input over 4 GiB) at sampled
  target points / source nodes against the oracle's location.
* O1280 x 137 (FP64, FP32, BF16 storage): every operator (and the curl) at ~700 sampled
  nodes (random, polar rows, nodes of degree 5 and 7, row starts, equator).
* O320 x 137 (FP64, FP32): SH sum to degree 64 with scale 1 + 0.1 k plus
  N(0, 1e-3) noise; gradient, divergence and Laplacian against the oracle at
  sampled nodes, the FP32 error against FP64 reported.
* O640 x 137 adjoints (FP64, FP32): autograd backward of sum(w * grad f) and
  of sum(w' * div uv), dot-product tests, central differences on 100 seeded
  node-level entries, sampled oracle values of the adjoints.
* O640 batched: 64 tracers with level counts drawn from {1, 19, 60, 91, 137},
  run as the batched plan (default form: one persistent launch per operator
  over every tracer's tiles) replayed as a HIP graph, bitwise equal to the
  single-field calls and sampled against the oracle.
Bars as in test_gpu_parity (FP64 1e-12, FP32 1e-5 total, BF16 4e-3 kernel),
normwise and element-wise, the element-wise bar also per level and on the
special node groups (tests/_parity.py).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1908_07038_amd as pa
import workloads as W
from oracle import nabla
from _parity import check, special_groups

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

DEV = torch.device("cuda", 0)
R = 6371220.0
_CACHE = {}


def oracle_mesh(N):
    if N not in _CACHE:
        m = oracle.build_mesh(N)
        _CACHE[N] = (m, oracle.build_dual(m, R))
    return _CACHE[N]


def sample_nodes(m, count, seed):
    g = m.grid
    rng = np.random.default_rng(seed)
    special = [np.arange(g.row_off[0], g.row_off[2]),                      # polar rows
               np.arange(g.row_off[g.nrows - 2], g.row_off[g.nrows]),
               np.nonzero(m.degree != 6)[0],                              # degree 5 and 7
               g.row_off[:-1][::max(1, g.nrows // 64)],                   # row starts
               g.row_off[g.N - 1] + np.arange(0, g.row_size[g.N - 1], 97),
               rng.choice(m.nnodes, count, replace=False)]
    return np.unique(np.concatenate(special)).astype(np.int64)


def rows(t, idx):
    """Rows idx of a device tensor as an FP64 numpy array (input data)."""
    return t[torch.from_numpy(np.asarray(idx)).to(t.device)].double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_o1280_sampled_parity():
    print("O1280 x 137: building meshes", flush=True)
    M = pa.Mesh("O1280", radius=R, device=0)
    m, g = oracle_mesh(1280)
    L = 137
    co = M.coords()
    s, trend = W.workload_o1280(co, nlev=L, device=DEV)
    tr = torch.from_numpy(trend).to(DEV)
    f64 = (s[:, None] + tr[None, :]).contiguous()
    su = W.sh_field(co, 128, 1013, device=DEV)
    sv = W.sh_field(co, 128, 1023, device=DEV)
    uv64 = torch.stack([su[:, None] + tr[None, :], sv[:, None] - tr[None, :]], dim=2).contiguous()
    del s, su, sv
    nodes = sample_nodes(m, 600, 77)
    groups = special_groups(m, nodes)
    ops = [("gradient", pa.gradient, nabla.gradient_at, "f"),
           ("divergence", pa.divergence, nabla.divergence_at, "uv"),
           ("laplacian", pa.laplacian, nabla.laplacian_at, "f"),
           ("gradient_adjoint", pa.gradient_adjoint, nabla.gradient_adjoint_at, "uv"),
           ("divergence_adjoint", pa.divergence_adjoint, nabla.divergence_adjoint_at, "f"),
           ("curl", pa.curl, nabla.curl_at, "uv")]
    refs = {}
    for name, _, ora, inp in ops:
        src = f64 if inp == "f" else uv64
        n_, refs[name] = ora(m, g, lambda idx, src=src: rows(src, idx), nodes)
        assert np.array_equal(n_, nodes)
    for dt, tol in [(torch.float64, 1e-12), (torch.float32, 1e-5), (torch.bfloat16, 4e-3)]:
        f = f64.to(dt)
        uv = uv64.to(dt)
        for name, fn, ora, inp in ops:
            x = f if inp == "f" else uv
            y = fn(M, x)
            torch.cuda.synchronize()
            got = rows(y, nodes)
            if dt != torch.float64:
                # the kernel's own error: the oracle on the rounded input
                _, ref = ora(m, g, lambda idx, x=x: rows(x, idx), nodes)
                total = rel(got, refs[name])
                if dt == torch.float32:
                    assert total <= tol, (name, "total", total)   # total error: normwise bar
            else:
                ref = refs[name]
                total = rel(got, ref)
            err, emax = check(got, ref, tol, (name, str(dt)), per_level=True, groups=groups)
            print(f"  {name} {dt}: rel L2 {err:.3e} max {emax:.3e} (total vs FP64 input {total:.3e})", flush=True)
            del y
        del f, uv
        torch.cuda.empty_cache()
    # the one-pass pairs equal the separate calls at full size, every dtype
    for dt in (torch.float64, torch.float32, torch.bfloat16):
        f = f64.to(dt)
        uv = uv64.to(dt)
        g, lp = pa.gradient_laplacian(M, f)
        assert torch.equal(g + 0.0, pa.gradient(M, f) + 0.0)
        assert torch.equal(lp + 0.0, pa.laplacian(M, f) + 0.0)
        del g, lp
        d, z = pa.divergence_curl(M, uv)
        assert torch.equal(d + 0.0, pa.divergence(M, uv) + 0.0)
        assert torch.equal(z + 0.0, pa.curl(M, uv) + 0.0)
        d, fb = pa.divergence_gradient_adjoint(M, uv, d, z)
        assert torch.equal(d + 0.0, pa.divergence(M, uv) + 0.0)
        assert torch.equal(fb + 0.0, pa.gradient_adjoint(M, uv) + 0.0)
        del d, z, fb, f, uv
        torch.cuda.empty_cache()
    print("  one-pass pairs equal to the separate calls", flush=True)
    # invariants at full size
    f = f64.float()
    gc = pa.gradient(M, torch.full_like(f, 2.5))
    assert torch.count_nonzero(gc).item() == 0
    d = pa.divergence(M, uv64.float())
    cs, ca = pa.conservation(M, d)
    assert (cs.abs() / ca).max().item() < 1e-6
    d64 = pa.divergence(M, uv64)
    cs, ca = pa.conservation(M, d64)
    assert (cs.abs() / ca).max().item() < 1e-13


@pytest.mark.parametrize("N", [640, 1280])
def test_full_size_mesh_matches_oracle(N):
    """Connectivity and indexing of the benchmarked meshes bit for bit (32-bit
    slot offsets and counting sorts at 6.6M nodes), node positions bit for
    bit, dual geometry to rounding."""
    print(f"O{N}: mesh against the oracle", flush=True)
    M = pa.Mesh(f"O{N}", radius=R, device=0)
    m, g = oracle_mesh(N)
    assert (M.nnodes, M.nedges, M.ntris, M.npole_edges) == (m.nnodes, m.nedges, m.ntris, 34)
    c = M.export_connectivity()
    for key, ref in [("tris", m.tris), ("edges", m.edges), ("csr_off", m.off), ("nbr", m.nbr), ("eid", m.eid),
                     ("sgn", m.sgn), ("rev", m.rev)]:
        assert np.array_equal(c[key], ref), key
        del c[key]
    assert np.array_equal(c["is_pole"].astype(bool), m.is_pole)
    gr = M.export_grid()
    assert np.array_equal(gr["row_size"], m.grid.row_size) and np.array_equal(gr["row_off"], m.grid.row_off)
    assert np.array_equal(gr["colat"], m.grid.theta)
    assert np.array_equal(gr["xyz"], m.grid.xyz)
    del gr
    ge = M.export_geometry()
    relS = np.linalg.norm(ge["S"] - g.S, axis=1) / np.linalg.norm(g.S, axis=1)
    assert relS.max() < 2e-15, relS.max()
    assert np.max(np.abs(ge["V"] - g.V) / g.V) < 2e-15
    print(f"  bit-exact; S rel {relS.max():.1e}", flush=True)
    M.close()


def test_o320_config():
    """O320 x 137 (421,120 nodes): f = s64 (1 + 0.1 k) + N(0, 1e-3) noise in
    FP64 and FP32; gradient, divergence of the gradient and Laplacian against
    the oracle at ~1,500 sampled nodes; the FP32 error against FP64 reported
    (and bounded at 1e-5 normwise and element-wise)."""
    print("O320 x 137: building", flush=True)
    M = pa.Mesh("O320", radius=R, device=0)
    m, g = oracle_mesh(320)
    assert M.nnodes == 421120
    L = 137
    f64 = torch.from_numpy(W.workload_o320(M.coords(), nlev=L)).to(DEV)
    nodes = sample_nodes(m, 1200, 80)
    groups = special_groups(m, nodes)
    get_f = lambda idx: rows(f64, idx)   # noqa: E731
    _, rg = nabla.gradient_at(m, g, get_f, nodes)
    _, rl = nabla.laplacian_at(m, g, get_f, nodes)   # the oracle's Laplacian is div(grad f)
    rd = rl
    got = {}
    for dt, tol in [(torch.float64, 1e-12), (torch.float32, 1e-5)]:
        f = f64.to(dt)
        gr = pa.gradient(M, f)
        dv = pa.divergence(M, gr)
        lp = pa.laplacian(M, f)
        torch.cuda.synchronize()
        if dt == torch.float32:
            # the kernel's own error: the oracle on the FP32-rounded input
            get_k = lambda idx, f=f: rows(f, idx)   # noqa: E731
            _, kg = nabla.gradient_at(m, g, get_k, nodes)
            _, kl = nabla.laplacian_at(m, g, get_k, nodes)
            kern = {"gradient": kg, "divergence of gradient": kl, "laplacian": kl}
        for name, y, ref in [("gradient", gr, rg), ("divergence of gradient", dv, rd), ("laplacian", lp, rl)]:
            a = rows(y, nodes)
            total = rel(a, ref)
            assert total <= tol, (name, str(dt), total)
            err, emax = check(a, kern[name] if dt == torch.float32 else ref, tol, (name, str(dt)),
                              per_level=True, groups=groups)
            got[(name, dt)] = y.double()
            print(f"  {name} {dt}: vs oracle rel L2 {err:.3e} max {emax:.3e} (total {total:.3e})", flush=True)
        del f
    # FP32 against FP64 over every node and level (the total FP32 error:
    # normwise bar; the element-wise figure is reported)
    for name in ("gradient", "divergence of gradient", "laplacian"):
        a, b = got[(name, torch.float32)], got[(name, torch.float64)]
        e2 = ((a - b).norm() / b.norm()).item()
        emax = ((a - b).abs().max() / b.abs().max()).item()
        print(f"  {name} FP32 vs FP64 (all {M.nnodes} x {L}): rel L2 {e2:.3e} max {emax:.3e}", flush=True)
        assert e2 <= 1e-5, (name, e2, emax)


def test_o1280_to_f640_remap_sampled():
    """Remap O1280 x 137 -> F640 (the benchmarked configuration) at ~400
    sampled target points (random, polar rows, equator, row starts) against
    the oracle's location restricted to nearby triangles; constants are
    reproduced everywhere."""
    from oracle import remap as Rm
    print("O1280 -> F640 remap: building", flush=True)
    M = pa.Mesh("O1280", radius=R, device=0)
    m, _ = oracle_mesh(1280)
    r = pa.Remap(M, "F640")
    assert r.npoints == 1280 * 2560 and r.nfallback == 0
    tg = Rm.TargetGrid("F640")
    rng = np.random.default_rng(91)
    n = 2560
    pts = np.unique(np.concatenate([rng.choice(r.npoints, 300, replace=False), np.arange(0, 2 * n, 37),
                                    r.npoints - 1 - np.arange(0, 2 * n, 41), 639 * n + np.arange(0, 2 * n, 53),
                                    np.arange(0, r.npoints, 97 * n + 13)])).astype(np.int64)
    _, nodes, w = Rm.locate_near(m.grid.xyz, m.tris, tg.xyz[pts], math.cos(0.01))
    L = 137
    co = M.coords()
    s, trend = W.workload_o1280(co, nlev=L, device=DEV)
    f64 = (s[:, None] + torch.from_numpy(trend).to(DEV)[None, :]).contiguous()
    del s
    for dt, tol in [(torch.float64, 1e-12), (torch.float32, 1e-5), (torch.bfloat16, 4e-3)]:
        x = f64.to(dt)
        y = r(x)
        torch.cuda.synchronize()
        got = rows(y, pts)
        ref = np.zeros_like(got)
        for j in range(3):
            ref += w[:, j:j + 1] * rows(x, nodes[:, j])
        err, emax = check(got, ref, tol, ("remap", str(dt)), per_level=True)
        print(f"  remap {dt}: rel L2 {err:.3e} max {emax:.3e}", flush=True)
        del x, y
    ones = r(torch.ones((M.nnodes, 3), dtype=torch.float32, device=DEV))
    assert (ones - 1).abs().max().item() < 1e-6


_REMAP = {}


def o1280_f640():
    """(GPU mesh, GPU remap) O1280 -> F640, built once per session."""
    if not _REMAP:
        M = pa.Mesh("O1280", radius=R, device=0)
        _REMAP["r"] = (M, pa.Remap(M, "F640"))
    return _REMAP["r"]


def located_near(xyz, tris, first, targets, centre, rt, rtri):
    """The oracle's location of the targets within angle rt of centre,
    among the triangles whose first node is within rtri of it: (target
    indices, nodes [n][3], weights [n][3])."""
    from oracle import remap as Rm
    t = np.nonzero(targets @ centre >= math.cos(rt))[0]
    cand = np.nonzero(first @ centre >= math.cos(rtri))[0]
    _, nodes, w = Rm.locate(xyz, tris[cand], targets[t])
    return t, nodes, w


@pytest.mark.parametrize("dtype,L", [(torch.float64, 137), (torch.float32, 137), (torch.bfloat16, 137),
                                     (torch.float64, 164)], ids=["f64", "f32", "bf16", "f64-164"])
def test_o1280_to_f640_remap_adjoint_sampled(dtype, L):
    """Transpose of the O1280 -> F640 remap at ~160 sampled source nodes
    (random, the two rows next to each pole, whose nodes take the most
    target points, nodes of degree 5 and 7, the zero meridian) against the
    oracle's location of every target point near each node: a target point
    uses a node only if it lies in one of the node's triangles, within one
    edge (at most 0.13 degrees on this mesh) of it, so the targets within
    0.3 degrees (0.45 degrees of a pole for the polar rows) are all of them.
    FP64 at 164 levels has an input over 4 GiB (the 64-bit addressing form).
    Also the dot-product identity <R x, y> = <x, R^T y> over all nodes."""
    from oracle import remap as Rm
    print(f"O1280 <- F640 remap adjoint {dtype} L {L}", flush=True)
    M, r = o1280_f640()
    m, _ = oracle_mesh(1280)
    g = m.grid
    xyz, tris = g.xyz, m.tris
    first = xyz[tris[:, 0]]
    tg = Rm.TargetGrid("F640")
    rng = np.random.default_rng(117 + L)
    # every fifth node of the two rows next to each pole (44 nodes a pole)
    polar = np.concatenate([np.arange(0, 44, 5), g.row_off[g.nrows - 2] + np.arange(0, 44, 5)])
    other = np.unique(np.concatenate([rng.choice(M.nnodes, 100, replace=False), np.nonzero(m.degree != 6)[0],
                                      g.row_off[np.arange(3, g.nrows - 3, 211)]]))
    other = np.setdiff1d(other, polar)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(1170 + L)
    y = torch.randn((r.npoints, L), generator=gen, device=DEV, dtype=torch.float64).to(dtype)
    fb = r.adjoint(y)
    torch.cuda.synchronize()
    idx = np.concatenate([polar, other])
    got = rows(fb, idx)
    ref = np.zeros_like(got)
    rad = math.radians
    # the polar rows from one location per pole, the other nodes one by one
    for i, n in enumerate(idx):
        if i == 0 or i == polar.size // 2:
            centre = np.array([0.0, 0.0, 1.0 if i == 0 else -1.0])
            t, nodes, w = located_near(xyz, tris, first, tg.xyz, centre, rad(0.45), rad(0.8))
            yt = rows(y, t)
        elif i >= polar.size:
            t, nodes, w = located_near(xyz, tris, first, tg.xyz, xyz[n], rad(0.3), rad(0.5))
            yt = rows(y, t)
        tr, slot = np.nonzero(nodes == n)
        ref[i] = (w[tr, slot][:, None] * yt[tr]).sum(axis=0)
    tol = {torch.float64: 1e-12, torch.float32: 1e-5, torch.bfloat16: 4e-3}[dtype]
    err, emax = check(got, ref, tol, ("remap adjoint", str(dtype), L), per_level=True,
                      groups={"polar rows": np.arange(polar.size)})
    print(f"  remap adjoint {dtype} L {L}: rel L2 {err:.3e} max {emax:.3e}", flush=True)
    if dtype == torch.float64:
        gen.manual_seed(1180 + L)
        x = torch.randn((M.nnodes, L), generator=gen, device=DEV, dtype=torch.float64)
        rx = r(x)
        lhs = float((rx * y).sum())
        rhs = float((x * fb).sum())
        assert abs(lhs - rhs) <= 1e-13 * float(rx.norm() * y.norm()), (lhs, rhs)
        del x, rx
    del y, fb


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_o640_adjoints(dtype):
    print(f"O640 x 137 adjoints {dtype}", flush=True)
    M = pa.Mesh("O640", radius=R, device=0)
    m, g = oracle_mesh(640)
    V, L = M.nnodes, 137
    co = M.coords()
    s = W.sh_field(co, 64, 1004, device=DEV)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(1004)
    f = (s[:, None] * (1.0 + 0.1 * torch.arange(L, device=DEV, dtype=torch.float64))[None, :]
         + 1e-3 * torch.randn((V, L), generator=gen, device=DEV, dtype=torch.float64)).to(dtype)
    gen.manual_seed(1014)
    w = torch.randn((V, L, 2), generator=gen, device=DEV, dtype=torch.float64).to(dtype)
    fr = f.clone().requires_grad_(True)
    loss = (w * pa.grad(M, fr)).sum()
    loss.backward()
    fbar = fr.grad
    assert torch.equal(fbar, pa.gradient_adjoint(M, w))
    # divergence: backward of sum(w' * div uv)
    gen.manual_seed(1044)
    uv = torch.randn((V, L, 2), generator=gen, device=DEV, dtype=torch.float64).to(dtype).requires_grad_(True)
    gen.manual_seed(1054)
    wd = torch.randn((V, L), generator=gen, device=DEV, dtype=torch.float64).to(dtype)
    (wd * pa.div(M, uv)).sum().backward()
    assert torch.equal(uv.grad, pa.divergence_adjoint(M, wd))
    # oracle values of both adjoints at sampled nodes
    nodes = sample_nodes(m, 400, 78)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    _, ref = nabla.gradient_adjoint_at(m, g, lambda idx: rows(w, idx), nodes)
    groups = special_groups(m, nodes)
    check(rows(fbar, nodes), ref, tol, "gradient adjoint", per_level=True, groups=groups)
    _, ref = nabla.divergence_adjoint_at(m, g, lambda idx: rows(wd, idx), nodes)
    check(rows(uv.grad, nodes), ref, tol, "divergence adjoint", per_level=True, groups=groups)
    # dot-product tests on random x, y
    gen.manual_seed(1024)
    x = torch.randn((V, L), generator=gen, device=DEV, dtype=torch.float64).to(dtype)
    y = torch.randn((V, L, 2), generator=gen, device=DEV, dtype=torch.float64).to(dtype)
    # <G x, y> = <x, G^T y> up to rounding, measured against ||G x|| ||y||
    # (Cauchy-Schwarz): the sums cancel heavily, so |<G x, y>| itself is no
    # scale for the rounding of ~10^8 products
    dtol = 1e-13 if dtype == torch.float64 else 1e-5
    gx = pa.gradient(M, x).double()
    lhs = (gx * y.double()).sum().item()
    rhs = (x.double() * pa.gradient_adjoint(M, y).double()).sum().item()
    scale = (gx.norm() * y.double().norm()).item()
    assert abs(lhs - rhs) <= dtol * scale, (lhs, rhs, scale)
    dy = pa.divergence(M, y).double()
    lhs = (dy * x.double()).sum().item()
    rhs = (y.double() * pa.divergence_adjoint(M, x).double()).sum().item()
    scale = (dy.norm() * x.double().norm()).item()
    assert abs(lhs - rhs) <= dtol * scale, (lhs, rhs, scale)
    # central differences of the linear loss on 100 seeded entries: only the
    # stencil of the entry changes, so the difference of the two outputs is
    # exactly zero elsewhere and the FP64 sum has no cancellation
    entries = W.fd_entries(V, L, 100, 1034)
    fd_tol = 1e-9 if dtype == torch.float64 else 1e-4
    wd64 = w.double()
    for i, k in entries:
        fik = f[i, k].item()
        eps = (1e-3 if dtype == torch.float64 else 0.5) * max(1.0, abs(fik))
        fp, fm = f.clone(), f.clone()
        fp[i, k] += eps
        fm[i, k] -= eps
        h = (fp[i, k].double() - fm[i, k].double()).item()    # the step actually taken
        diff = (pa.gradient(M, fp).double() - pa.gradient(M, fm).double())
        fd = (wd64 * diff).sum().item() / h
        an = fbar[i, k].double().item()
        assert abs(fd - an) <= fd_tol * max(abs(an), 1e-30) + 1e-30, (i, k, fd, an)


def test_o640_batched_config():
    print("O640 batched, 64 tracers", flush=True)
    M = pa.Mesh("O640", radius=R, device=0)
    m, g = oracle_mesh(640)
    V = M.nnodes
    levels = [int(x) for x in W.batch_levels(64, 1005)]
    need = sum(levels) * V * 4 * 7 + (1 << 31)
    free, _ = torch.cuda.mem_get_info(DEV)
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free")
    co = M.coords()
    tracers = []
    for t, L in enumerate(levels):
        s = W.tracer_surface(co, t, device=DEV)
        scale = 1.0 + torch.arange(L, device=DEV, dtype=torch.float64) / L
        f = (s[:, None] * scale[None, :]).float().contiguous()
        gbuf = torch.empty((V, L, 2), device=DEV)
        d = torch.empty((V, L), device=DEV)
        fT = torch.empty((V, L), device=DEV)
        gT = torch.empty((V, L, 2), device=DEV)
        tracers.append({"gradient": (f, gbuf), "divergence": (gbuf, d), "gradient_adjoint": (gbuf, fT),
                        "divergence_adjoint": (d, gT)})
    plan = pa.Batch(M, tracers)
    for rep in range(2):
        for tr in tracers:
            for n in ("divergence", "gradient_adjoint", "divergence_adjoint"):
                tr[n][1].fill_(float("nan"))
        plan.graph_launch()
        torch.cuda.synchronize()
    # bitwise against the single-field chain
    for tr in tracers:
        f = tr["gradient"][0]
        g1 = pa.gradient(M, f)
        d1 = pa.divergence(M, g1)
        assert torch.equal(tr["gradient"][1], g1)
        assert torch.equal(tr["divergence"][1], d1)
        assert torch.equal(tr["gradient_adjoint"][1], pa.gradient_adjoint(M, g1))
        assert torch.equal(tr["divergence_adjoint"][1], pa.divergence_adjoint(M, d1))
        del g1, d1
    # oracle at sampled nodes for a tracer of each level count (FP64 chain)
    nodes = sample_nodes(m, 150, 79)
    seen = set()
    for t, L in enumerate(levels):
        if L in seen:
            continue
        seen.add(L)
        tr = tracers[t]
        get_f = lambda idx, x=tr["gradient"][0]: rows(x, idx)   # noqa: E731
        _, rg = nabla.gradient_at(m, g, get_f, nodes)
        _, rl = nabla.laplacian_at(m, g, get_f, nodes)
        groups = special_groups(m, nodes)
        check(rows(tr["gradient"][1], nodes), rg, 1e-5, ("gradient", L), per_level=True, groups=groups)
        check(rows(tr["divergence"][1], nodes), rl, 1e-5, ("divergence", L), per_level=True, groups=groups)
        # adjoints of the chain: grad^T(grad f) and div^T(div grad f)
        ring_nodes, ring_eids = nabla._incident(m, nodes)
        ring = np.unique(np.concatenate([ring_nodes, m.edges[ring_eids].ravel()]))
        ring, g_ring = nabla.gradient_at(m, g, get_f, ring)
        lut = np.full(m.nnodes, -1)
        lut[ring] = np.arange(ring.size)
        _, rgt = nabla.gradient_adjoint_at(m, g, lambda idx: g_ring[lut[idx]], nodes)
        check(rows(tr["gradient_adjoint"][1], nodes), rgt, 1e-5, ("gradient adjoint", L), per_level=True,
              groups=groups)
        ring, l_ring = nabla.laplacian_at(m, g, get_f, ring)
        _, rdt = nabla.divergence_adjoint_at(m, g, lambda idx: l_ring[lut[idx]], nodes)
        check(rows(tr["divergence_adjoint"][1], nodes), rdt, 1e-5, ("divergence adjoint", L), per_level=True,
              groups=groups)
    assert math.isfinite(float(tracers[0]["divergence_adjoint"][1].abs().max()))
