"""Benchmark of the median-dual Nabla hot path on one MI355X.

Workload: O1280 octahedral mesh (6,599,680 nodes, 19,799,034 edges), 137
levels, FP32 fields; input = seeded spherical-harmonic sum to degree 256 plus a
level-wise linear trend (synthetic; the paper measures nothing and names no
dataset).  One step = gradient f -> g and fused Laplacian f -> l (one pass
over f: the library's gradient_laplacian call), divergence g -> d, gradient
adjoint g -> fT, divergence adjoint d -> gT, and the FP64 conservation sums of
d, all on one stream with inputs resident in HBM.  The gradient and the
Laplacian are also timed as separate calls (reported per operator, not in
the step).

value = edge-level updates per second = 6 E L / t_step (gradient, divergence
and both adjoints count one sweep over the edges each, the Laplacian two).
The same step is also timed in FP64 and with BF16 storage.

Per-kernel durations come from HIP events recorded on the launch stream around
every operator call inside the timed region; achieved bandwidth divides each
kernel's algorithmic bytes (fields read once and written once, plus the
minimal FP64 geometry of 104 bytes per node) by that duration.

A second, separate measurement (not in value): the O640 64-tracer batched
plan replayed as a HIP graph, against the same work as single-field calls.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-cpu] [--skip-batched]
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
GEOM_BYTES_PER_NODE = 104  # S_e (24 B) + two int32 ends (8 B) per edge x 3 edges, + V_i (8 B)
METRIC = "edge-level updates/s and % HBM peak, Nabla grad+div+lap O1280×137, FP32 vs FP64"
UNIT = "edge-level updates/s"
# the step: gradient and Laplacian of f in one pass, divergence and gradient
# adjoint of that gradient in one pass, divergence adjoint of the divergence,
# conservation sums of the divergence
OPS = ["gradient_laplacian", "divergence_gradient_adjoint", "divergence_adjoint", "conservation"]
SEPARATE = ["gradient", "laplacian", "divergence", "gradient_adjoint"]   # timed alone as well (not in the step)
# (elements read, elements written) per node-level, and edge sweeps
OP_ELEMS = {"gradient": (1, 2), "divergence": (2, 1), "laplacian": (1, 1), "gradient_laplacian": (1, 3),
            "gradient_adjoint": (2, 1), "divergence_adjoint": (1, 2), "conservation": (1, 0),
            "divergence_gradient_adjoint": (2, 2)}
OP_SWEEPS = {"gradient": 1, "divergence": 1, "laplacian": 2, "gradient_laplacian": 3, "gradient_adjoint": 1,
             "divergence_adjoint": 1, "conservation": 0, "divergence_gradient_adjoint": 2}
CONSERVATION_KERNELS = "k_cons_partial + k_cons_final"


def kernel_names(pa, mesh, dtype_code, L):
    """Kernel each operator runs with the mesh's current (default) shapes."""
    bits = {"gradient": pa.OP_GRADIENT, "divergence": pa.OP_DIVERGENCE, "laplacian": pa.OP_LAPLACIAN,
            "gradient_adjoint": pa.OP_GRADIENT_ADJOINT, "divergence_adjoint": pa.OP_DIVERGENCE_ADJOINT}
    names = {op: pa.describe(mesh, b, dtype_code, L)[1] for op, b in bits.items()}
    names["conservation"] = CONSERVATION_KERNELS
    # the one-pass calls: their kernel, or "two calls" when the shape is not the one-tile form
    names["gradient_laplacian"] = pa.describe(mesh, pa.OP_GRADIENT_LAPLACIAN, dtype_code, L)[1]
    names["divergence_gradient_adjoint"] = pa.describe(mesh, pa.OP_DIVERGENCE_GRADIENT_ADJOINT, dtype_code, L)[1]
    return names


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def alg_bytes(op, V, L, esize):
    r, w = OP_ELEMS[op]
    geom = GEOM_BYTES_PER_NODE * V if op != "conservation" else 8 * V
    return (r + w) * esize * V * L + geom


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "launch.hpp"):
        with open(os.path.join(ROOT, "paper_1908_07038_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(op, dtype_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash()
    for line in open(path):
        p = line.split()
        if len(p) >= 5 and not line.startswith("#") and p[0] == src and p[1] == op and p[2] == dtype_name:
            return float(p[3]) + float(p[4])
    return None


def sample_nodes(mesh, count, seed):
    """Nodes where the outputs are checked against the FP64 oracle (sorted
    unique): the two polar rows at each pole, every node of degree 5 or 7,
    row starts, a run of the equatorial row and `count` random nodes, from
    the mesh's exported grid and connectivity."""
    import numpy as np

    gr = mesh.export_grid()
    deg = np.diff(mesh.export_connectivity()["csr_off"])
    ro, rs = gr["row_off"], gr["row_size"]
    R = rs.size
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([
        np.arange(ro[0], ro[2]), np.arange(ro[R - 2], ro[R]), np.nonzero(deg != 6)[0],
        ro[:-1][::max(1, R // 64)], ro[R // 2 - 1] + np.arange(0, rs[R // 2 - 1], 97),
        rng.choice(mesh.nnodes, count, replace=False)])).astype(np.int64)


def run_gpu(args):
    import torch

    import paper_1908_07038_amd as pa
    import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    mesh = pa.Mesh(args.grid, radius=6371220.0, device=0)
    V, E, L = mesh.nnodes, mesh.nedges, args.levels
    log(f"mesh {args.grid}: V={V} E={E} built+uploaded in {time.time() - t0:.1f}s")
    t0 = time.time()
    s, trend = W.workload_o1280(mesh.coords(), nlev=L, device=dev)
    f64 = (s[:, None] + torch.from_numpy(trend).to(dev)[None, :]).contiguous()
    torch.cuda.synchronize()
    log(f"input generated in {time.time() - t0:.1f}s")

    results = {}
    # sample nodes for the error against the FP64 oracle, and the input rows
    # on their three-ring (what the oracle's chains at those nodes read)
    sample = sample_nodes(mesh, 600, 1234)
    sample_t = torch.from_numpy(sample).to(dev)
    samples = {"nodes": sample, "surface": s.cpu().numpy(), "trend": trend}
    for dname, dtype, esize in (("f64", torch.float64, 8), ("f32", torch.float32, 4), ("bf16", torch.bfloat16, 2)):
        f = f64.to(dtype)
        g = torch.empty((V, L, 2), dtype=dtype, device=dev)
        d = torch.empty((V, L), dtype=dtype, device=dev)
        lp = torch.empty((V, L), dtype=dtype, device=dev)
        fT = torch.empty((V, L), dtype=dtype, device=dev)
        gT = torch.empty((V, L, 2), dtype=dtype, device=dev)
        calls = {
            "gradient_laplacian": lambda: pa.gradient_laplacian(mesh, f, g, lp),
            "gradient": lambda: pa.gradient(mesh, f, out=g),
            "divergence": lambda: pa.divergence(mesh, g, out=d),
            "laplacian": lambda: pa.laplacian(mesh, f, out=lp),
            "gradient_adjoint": lambda: pa.gradient_adjoint(mesh, g, out=fT),
            "divergence_gradient_adjoint": lambda: pa.divergence_gradient_adjoint(mesh, g, d, fT),
            "divergence_adjoint": lambda: pa.divergence_adjoint(mesh, d, out=gT),
            "conservation": lambda: pa.conservation(mesh, d),
        }
        for _ in range(args.warmup):
            for op in OPS:
                calls[op]()
        torch.cuda.synchronize()
        ev = {op: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)] for op in OPS}
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(args.steps):
            for op in OPS:
                a, b = ev[op][k]
                a.record()
                calls[op]()
                b.record()
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t_start) / args.steps
        per_op = {}
        for op in OPS:
            ms = sum(a.elapsed_time(b) for a, b in ev[op]) / args.steps
            by = alg_bytes(op, V, L, esize)
            per_op[op] = {"ms": round(ms, 4), "alg_GB": round(by / 1e9, 3),
                          "GB_s": round(by / (ms * 1e-3) / 1e9, 1),
                          "hbm_frac": round(by / (ms * 1e-3) / HBM_PEAK, 3)}
            if OP_SWEEPS[op]:
                per_op[op]["edge_updates_s"] = float(f"{OP_SWEEPS[op] * E * L / (ms * 1e-3):.4g}")
        # the gradient, the Laplacian, the divergence and the gradient adjoint
        # as separate calls (not in value)
        for op in SEPARATE:
            calls[op]()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.steps):
                calls[op]()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / args.steps
            by = alg_bytes(op, V, L, esize)
            per_op[op] = {"ms": round(ms, 4), "alg_GB": round(by / 1e9, 3), "GB_s": round(by / (ms * 1e-3) / 1e9, 1),
                          "hbm_frac": round(by / (ms * 1e-3) / HBM_PEAK, 3),
                          "edge_updates_s": float(f"{OP_SWEEPS[op] * E * L / (ms * 1e-3):.4g}"), "in_step": False}
        calls["gradient_laplacian"]()
        # the curl and its adjoint, timed apart from the step (not in value)
        zt = torch.empty((V, L), dtype=dtype, device=dev)
        ut = torch.empty((V, L, 2), dtype=dtype, device=dev)
        extra = {}
        dd = torch.empty((V, L), dtype=dtype, device=dev)
        for name, fn in (("curl", lambda: pa.curl(mesh, g, out=zt)),
                         ("curl_adjoint", lambda: pa.curl_adjoint(mesh, d, out=ut)),
                         ("divergence_curl", lambda: pa.divergence_curl(mesh, g, dd, zt))):
            fn()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / args.steps
            nel = 4 if name == "divergence_curl" else 3   # elements read + written per node-level
            by = nel * esize * V * L + GEOM_BYTES_PER_NODE * V
            sweeps_x = 2 if name == "divergence_curl" else 1
            extra[name] = {"ms": round(ms, 4), "GB_s": round(by / (ms * 1e-3) / 1e9, 1),
                           "hbm_frac": round(by / (ms * 1e-3) / HBM_PEAK, 3),
                           "edge_updates_s": float(f"{sweeps_x * E * L / (ms * 1e-3):.4g}")}
        del zt, ut, dd
        cs, ca = calls["conservation"]()
        cons = float((cs.abs() / ca).max().item())
        outs = {"gradient": g, "divergence": d, "laplacian": lp, "gradient_adjoint": fT,
                "divergence_adjoint": gT}
        # rows at the sample nodes, compared with the FP64 oracle in the CPU leg
        for k, v in outs.items():
            samples[f"{dname}:{k}"] = v[sample_t].double().cpu().numpy()
        sweeps = sum(OP_SWEEPS[op] for op in OPS)
        codes = {"f64": pa.F64, "f32": pa.F32, "bf16": pa.BF16}
        for op, name in kernel_names(pa, mesh, codes[dname], L).items():
            per_op[op]["kernel"] = name
        results[dname] = {"ms_per_step": round(t_step * 1e3, 4),
                          "edge_updates_s": float(f"{sweeps * E * L / t_step:.4g}"),
                          "per_op": per_op, "curl_ops": extra, "conservation_max_rel": cons}
        log(f"{dname}: {t_step * 1e3:.3f} ms/step, " +
            ", ".join(f"{op} {per_op[op]['ms']:.3f}ms {per_op[op]['hbm_frac'] * 100:.0f}%" for op in OPS))
        del f, g, d, lp, fT, gT, outs
        torch.cuda.empty_cache()
    if not args.skip_remap:
        results["remap"] = run_remap(args, pa, mesh, f64)
    del f64
    torch.cuda.empty_cache()
    return mesh, results, samples


def run_remap(args, pa, mesh, f64):
    """Remap of the benchmark field to the regular Gaussian grid of half the
    resolution (O1280 -> F640 by default): HIP-event time per call, and
    algorithmic bytes = the source columns the tables reference (each read
    once) + the target columns written + the tables (16 B of node indices and
    4 weights of the dtype's weight type per target point)."""
    import numpy as np
    import torch

    N = int(args.grid[1:])
    target = f"F{max(1, N // 2)}"
    t0 = time.time()
    r = pa.Remap(mesh, target)
    log(f"remap {args.grid} -> {target}: {r.npoints} points located in {time.time() - t0:.1f}s "
        f"({r.nfallback} by exhaustive search)")
    nsrc = int(np.unique(r.export()["nodes"]).size)
    V, L, P = mesh.nnodes, args.levels, r.npoints
    out = {"target": target, "npoints": P, "source_columns_read": nsrc}
    for dname, dtype, esize in (("f64", torch.float64, 8), ("f32", torch.float32, 4), ("bf16", torch.bfloat16, 2)):
        x = f64.to(dtype)
        y = torch.empty((P, L), dtype=dtype, device=x.device)
        for _ in range(max(1, args.warmup)):
            r(x, out=y)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.steps):
            r(x, out=y)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        by = (nsrc + P) * L * esize + P * (16 + 4 * (8 if dname == "f64" else 4))
        out[dname] = {"ms": round(ms, 4), "alg_GB": round(by / 1e9, 3), "GB_s": round(by / (ms * 1e-3) / 1e9, 1),
                      "hbm_frac": round(by / (ms * 1e-3) / HBM_PEAK, 3),
                      "point_levels_s": float(f"{P * L / (ms * 1e-3):.4g}")}
        # the transpose (target field -> source nodes): reads the target
        # columns once, writes every source column, plus its tables
        fb = torch.empty((V, L), dtype=dtype, device=x.device)
        r.adjoint(y, out=fb)
        a.record()
        for _ in range(args.steps):
            r.adjoint(y, out=fb)
        b.record()
        torch.cuda.synchronize()
        ms_t = a.elapsed_time(b) / args.steps
        by_t = (P + V) * L * esize + 8 * V + 3 * P * (4 + (8 if dname == "f64" else 4))
        out[dname]["adjoint"] = {"ms": round(ms_t, 4), "GB_s": round(by_t / (ms_t * 1e-3) / 1e9, 1),
                                 "hbm_frac": round(by_t / (ms_t * 1e-3) / HBM_PEAK, 3)}
        log(f"remap {dname}: {ms:.3f} ms, {out[dname]['GB_s']:.0f} GB/s algorithmic; "
            f"adjoint {ms_t:.3f} ms, {out[dname]['adjoint']['GB_s']:.0f} GB/s")
        del x, y, fb
    r.close()
    return out


def run_batched(args):
    """O640, 64 tracers with level counts drawn from {1, 19, 60, 91, 137}:
    gradient, divergence and both adjoints of every tracer in one persistent
    launch per operator, replayed as a HIP graph; against the same chain as
    single-field calls (default shapes) one tracer at a time."""
    import torch

    import paper_1908_07038_amd as pa
    import workloads as W

    dev = torch.device("cuda", 0)
    t0 = time.time()
    mesh = pa.Mesh("O640", radius=6371220.0, device=0)
    V, E = mesh.nnodes, mesh.nedges
    levels = [int(x) for x in W.batch_levels(64, 1005)]
    need = sum(levels) * V * 4 * 7 + (4 << 30)
    free, _ = torch.cuda.mem_get_info(dev)
    if free < need:
        log(f"batched: skipped, needs {need / 1e9:.0f} GB, {free / 1e9:.0f} GB free")
        return None
    co = mesh.coords()
    tracers = []
    for t, L in enumerate(levels):
        s = W.tracer_surface(co, t, device=dev)
        scale = 1.0 + torch.arange(L, device=dev, dtype=torch.float64) / L
        f = (s[:, None] * scale[None, :]).float().contiguous()
        g = torch.empty((V, L, 2), device=dev)
        d = torch.empty((V, L), device=dev)
        fT = torch.empty((V, L), device=dev)
        gT = torch.empty((V, L, 2), device=dev)
        tracers.append({"gradient": (f, g), "divergence": (g, d), "gradient_adjoint": (g, fT),
                        "divergence_adjoint": (d, gT)})
    torch.cuda.synchronize()
    log(f"batched: O640 mesh and 64 tracer fields (sum of levels {sum(levels)}) in {time.time() - t0:.1f}s")
    reps = max(2, min(args.steps, 5))
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_graph(plan):
        plan.graph_launch()
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            plan.graph_launch()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # the tracers' field launches replayed as a graph, the persistent plan at
    # its default shape, then the persistent plan after the autotuner
    fields = pa.Batch(mesh, tracers, tune={"batch_mode": 2})
    t_fields = time_graph(fields)
    fields.close()
    plan = pa.Batch(mesh, tracers)
    t_default = time_graph(plan)
    t0 = time.time()
    shapes, tune_ms = plan.tune(reps=2)
    tuned = {op: {k: sh[k] for k in ("batch_mode", "tile_kb", "batch_claim", "waves_per_block")}
             for op, sh in shapes.items()}
    log(f"batched: tuned in {time.time() - t0:.1f}s ({tune_ms:.2f} ms): {tuned}")
    t_graph = time_graph(plan)

    def single_field():
        for tr in tracers:
            pa.gradient(mesh, tr["gradient"][0], out=tr["gradient"][1])
            # the divergence and gradient adjoint of g in one pass, as the plan runs them
            pa.divergence_gradient_adjoint(mesh, tr["divergence"][0], tr["divergence"][1], tr["gradient_adjoint"][1])
            pa.divergence_adjoint(mesh, tr["divergence_adjoint"][0], out=tr["divergence_adjoint"][1])

    single_field()   # builds the one-pass calls' tilings and records outside the timed loop
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        single_field()
    b.record()
    torch.cuda.synchronize()
    t_single = a.elapsed_time(b) / reps
    sl = sum(levels)
    # gradient (1 + 2 elements), divergence and gradient adjoint of g in one
    # pass (2 read, 1 + 1 written), divergence adjoint (1 + 2): 10 FP32
    # elements per node-level, and the geometry once per pass
    by = 10 * 4 * V * sl + 3 * GEOM_BYTES_PER_NODE * V * len(levels)
    out = {"workload": "O640, 64 tracers, levels from {1,19,60,91,137} (seed 1005), FP32: grad, div, "
                       "grad adjoint, div adjoint (div and grad adjoint of the same field as one pass), "
                       "one persistent launch per operator, graph-replayed, autotuned",
           "sum_levels": sl, "graph_ms": round(t_graph, 3),
           "edge_updates_s": float(f"{4 * E * sl / (t_graph * 1e-3):.4g}"),
           "alg_GB_s": round(by / (t_graph * 1e-3) / 1e9, 1),
           "hbm_frac": round(by / (t_graph * 1e-3) / HBM_PEAK, 4),
           "tuned_shapes": tuned,
           "default_shape_graph_ms": round(t_default, 3),
           "field_launch_graph_ms": round(t_fields, 3),
           "single_field_ms": round(t_single, 3),
           "speedup_over_single_field": round(t_single / t_graph, 3)}
    log(f"batched: persistent graph {t_graph:.2f} ms (default shape {t_default:.2f}), field-launch graph "
        f"{t_fields:.2f} ms, single-field calls {t_single:.2f} ms")
    del tracers, plan
    torch.cuda.empty_cache()
    return out


POOL_MAX = 16   # worker processes at most: the host's CPU share per GPU


def host_description():
    """CPU model, usable cores and RAM of this host."""
    model, ram = "unknown", None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "cores_available": len(os.sched_getaffinity(0)), "ram_GiB": ram}


_LEG = {}   # oracle mesh and input of the CPU leg, shared with forked workers


def _oracle_step(k0, k1):
    """One full step of the FP64 oracle on levels [k0, k1) of the workload."""
    from oracle import nabla
    m, geo, s, trend = _LEG["mesh"], _LEG["geo"], _LEG["surface"], _LEG["trend"]
    f = s[:, None] + trend[None, k0:k1]
    g = nabla.gradient(m, geo, f)
    d = nabla.divergence(m, geo, g)
    nabla.laplacian(m, geo, f)
    nabla.gradient_adjoint(m, geo, g)
    nabla.divergence_adjoint(m, geo, d)
    nabla.conservation(m, geo, d)


def _pool_worker(block):
    t0 = time.perf_counter()
    _oracle_step(*block)
    return time.perf_counter() - t0


def cpu_leg(path):
    """The oracle side of the benchmark, run in a child process that never
    touches the GPU: (1) the FP64 oracle at the sampled nodes, from the same
    input, against the GPU outputs of every dtype; (2) the oracle's time for
    one full step on a bounded level sample, in one process and in a pool of
    processes over level blocks (levels are independent)."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    from oracle import nabla

    z = np.load(path, allow_pickle=False)
    grid, nlev_sample = str(z["grid"]), int(z["nlev_sample"])
    s, trend, nodes = z["surface"], z["trend"], z["nodes"]
    L = trend.size
    t0 = time.time()
    m = oracle.build_mesh(grid)
    geo = oracle.build_dual(m)
    log(f"oracle mesh {grid} built in {time.time() - t0:.1f}s")
    _LEG.update(mesh=m, geo=geo, surface=s, trend=trend)

    # (1) errors at the sampled nodes against the FP64 chains of the step:
    # gradient G f, Laplacian, divergence of the gradient D G f (= the
    # Laplacian), gradient adjoint G^T G f, divergence adjoint D^T D G f
    def get_f(idx):
        return s[idx][:, None] + trend[None, :]
    ref = {}
    _, ref["gradient"] = nabla.gradient_at(m, geo, get_f, nodes)
    _, ref["laplacian"] = nabla.laplacian_at(m, geo, get_f, nodes)
    ref["divergence"] = ref["laplacian"]
    ring_nodes, ring_eids = nabla._incident(m, nodes)
    ring = np.unique(np.concatenate([ring_nodes, m.edges[ring_eids].ravel()]))
    lut = np.full(m.nnodes, -1)
    lut[ring] = np.arange(ring.size)
    _, g_ring = nabla.gradient_at(m, geo, get_f, ring)
    _, ref["gradient_adjoint"] = nabla.gradient_adjoint_at(m, geo, lambda idx: g_ring[lut[idx]], nodes)
    _, l_ring = nabla.laplacian_at(m, geo, get_f, ring)
    _, ref["divergence_adjoint"] = nabla.divergence_adjoint_at(m, geo, lambda idx: l_ring[lut[idx]], nodes)
    errors = {}
    for key in z.files:
        if ":" not in key:
            continue
        dname, op = key.split(":")
        a, r = z[key], ref[op]
        errors.setdefault(dname, {})[op] = {
            "rel_l2": float(f"{np.linalg.norm(a - r) / np.linalg.norm(r):.3g}"),
            "max_rel": float(f"{np.abs(a - r).max() / np.abs(r).max():.3g}")}
    log("errors vs the FP64 oracle at sampled nodes: " +
        "; ".join(f"{d} " + ", ".join(f"{o} {v['rel_l2']:.2g}" for o, v in e.items()) for d, e in errors.items()))

    # (2) timing: one process on levels 0..nlev_sample-1, then one worker per
    # core (at most POOL_MAX), each on its own block of nlev_sample levels
    E = m.nedges
    t0 = time.perf_counter()
    _oracle_step(0, nlev_sample)
    t1 = time.perf_counter() - t0
    log(f"oracle step on {nlev_sample} levels, one process: {t1:.1f}s")
    nw = max(1, min(POOL_MAX, len(os.sched_getaffinity(0)), L // nlev_sample))
    blocks = [(w * nlev_sample, (w + 1) * nlev_sample) for w in range(nw)]
    with mp.get_context("fork").Pool(nw) as pool:
        t0 = time.perf_counter()
        pool.map(_pool_worker, blocks, chunksize=1)
        tp = time.perf_counter() - t0
    log(f"oracle step on {nw} x {nlev_sample} levels, {nw} processes: {tp:.1f}s")
    host = host_description()
    single = float(f"{6 * E * nlev_sample / t1:.4g}")
    pooled = float(f"{6 * E * nw * nlev_sample / tp:.4g}")
    base = {"value": pooled, "unit": UNIT, "cores": nw, "kind": "oracle",
            "sample": f"one full step (grad, div, lap, both adjoints, conservation) of the FP64 NumPy oracle on "
                      f"the {grid} mesh; {nw} processes (fork pool) over level blocks of {nlev_sample} levels "
                      f"(levels 0..{nw * nlev_sample - 1} of the {L}-level workload), wall time; NumPy's "
                      f"scatter is single-threaded, so one process uses one core",
            "seconds": round(tp, 2),
            "single_process": {"value": single, "cores": 1, "levels": nlev_sample, "seconds": round(t1, 2)},
            "host": host}
    return {"cpu_baseline": base, "errors_vs_oracle": errors, "sample_nodes": int(nodes.size)}


def run_cpu_baseline(args, samples):
    """Runs cpu_leg in a child process (a fresh interpreter that never
    initialises the GPU, so it may fork its worker pool) on the input surface
    and the sampled GPU outputs handed over in a temporary .npz."""
    import subprocess
    import tempfile

    import numpy as np

    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "leg.npz")
        np.savez(path, grid=np.array(args.grid), nlev_sample=np.array(args.cpu_levels), **samples)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", path],
                           stdout=subprocess.PIPE, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"the oracle leg failed with status {r.returncode}")
    return json.loads(r.stdout.strip().splitlines()[-1])


# Kernel instances of one bench dtype: (op name in hbm_traffic.txt, kernel
# operator number in the k_tile<type, op, U> template, or a kernel name prefix).
PROFILE_STATS_CMD = ("cd /tmp && export TMPDIR=/tmp && cd <repo> && rocprofv3 --kernel-trace --stats -d <out>/stats "
                     "-o bench -- python3 bench.py --steps 5 --warmup 2 --skip-cpu")
PROFILE_PMC_CMD = ("cd /tmp && export TMPDIR=/tmp && cd <repo> && rocprofv3 --pmc COUNTER --kernel-trace -d <out>/COUNTER "
                   "-o run -- python3 bench.py --steps 2 --warmup 1 --skip-cpu --skip-batched --calibrate-copy")
TRAFFIC_KERNELS = [("gradient_laplacian", "k_tile<{t}, 7,"), ("divergence", "k_tile<{t}, 1,"),
                   ("gradient_adjoint", "k_tile<{t}, 2,"), ("divergence_adjoint", "k_tile<{t}, 3,"),
                   ("divergence_gradient_adjoint", "k_tile<{t}, 8,"),
                   ("gradient", "k_tile<{t}, 0,"), ("laplacian", "k_tile<{t}, 4,"),
                   ("divergence_curl", "k_tile<{t}, 8,"), ("remap_f640", "k_remap<{t},"),
                   ("remap_adjoint_f640", "k_remap_adj<{t},")]
TYPE_OF = {"f64": "double", "f32": "float", "bf16": "unsigned short"}


def _dispatches(db, counter=None):
    """(short kernel name, duration ns or counter value) per dispatch of a
    rocprofv3 database."""
    import re
    import sqlite3
    c = sqlite3.connect(db)
    short = lambda n: re.sub(r"^void ", "", re.sub(r"atlasnabla::\(anonymous namespace\)::", "", n))  # noqa: E731
    if counter is None:
        return [(short(n), e - s) for n, s, e in c.execute("select name, start, end from kernels")]
    return [(short(n), v) for n, v in
            c.execute("select kernel_name, value from counters_collection where counter_name = ?", (counter,))]


def summarize_profiles(stats_db, fetch_db, write_db, stats_cmd, pmc_cmd):
    """Writes profiles/bench_o1280x137_kernel_stats.md (kernel times) and
    profiles/hbm_traffic.txt (HBM bytes per launch: the FETCH_SIZE and
    WRITE_SIZE averages per kernel, in KiB, scaled so that the plain 4 GiB
    device copy of --calibrate-copy reads 4 GiB fetched and written)."""
    import collections
    src = kernel_source_hash()
    times = collections.defaultdict(list)
    for n, d in _dispatches(stats_db):
        times[n].append(d / 1e6)
    total = sum(sum(v) for v in times.values())
    rows = sorted(times.items(), key=lambda kv: -sum(kv[1]))
    with open(os.path.join(ROOT, "profiles", "bench_o1280x137_kernel_stats.md"), "w") as fh:
        fh.write("# Kernel time summary: bench O1280 x 137 (FP64, FP32, BF16 steps, remap, O640 batched)\n\n")
        fh.write("Command (from the repository root, on one MI355X):\n\n```\n" + stats_cmd + "\n```\n\n")
        fh.write(f"Kernel source hash (bench.kernel_source_hash): `{src}`.  The k_tile_batched rows include the "
                 "autotuner's candidate shapes.\n\n")
        fh.write("| kernel | calls | average ms | min ms | max ms | share % |\n|---|---|---|---|---|---|\n")
        for n, v in rows:
            if sum(v) / total < 0.002:
                continue
            fh.write(f"| `{n[:90]}` | {len(v)} | {sum(v) / len(v):.4f} | {min(v):.4f} | {max(v):.4f} | "
                     f"{100 * sum(v) / total:.2f} |\n")
    per, cal = {}, {}
    for key, db in (("fetch", fetch_db), ("write", write_db)):
        acc = collections.defaultdict(list)
        for n, v in _dispatches(db, "FETCH_SIZE" if key == "fetch" else "WRITE_SIZE"):
            acc[n].append(v)
        per[key] = {n: sum(v) / len(v) for n, v in acc.items()}
        # the calibration copy is the largest copyBuffer dispatch (4 GiB)
        big = max(v for n, vs in acc.items() if n.startswith("__amd_rocclr_copyBuffer") for v in vs)
        cal[key] = 4 * 2 ** 30 / (big * 1024)
    cal_f, cal_w = cal["fetch"], cal["write"]
    lines = ["# HBM traffic per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged per",
             "# kernel), each scaled by what the same counter reads for a plain 4 GiB device copy (torch copy_ ->",
             f"# __amd_rocclr_copyBuffer): FETCH x{cal_f:.3f}, WRITE x{cal_w:.3f}.",
             "# Workload: bench.py O1280 x 137.  Commands (repository root, one MI355X):",
             "#   " + pmc_cmd.replace("COUNTER", "FETCH_SIZE"), "#   " + pmc_cmd.replace("COUNTER", "WRITE_SIZE"),
             "# Rows are valid only for the kernel source hash in column 1 (bench.py ignores others).",
             "# hash op dtype fetch_bytes write_bytes"]
    for dname, ty in TYPE_OF.items():
        for op, pat in TRAFFIC_KERNELS:
            pre = pat.format(t=ty)
            names = [n for n in per["fetch"] if n.startswith(pre)]
            if not names:
                continue
            n = max(names, key=lambda x: per["fetch"][x])   # the instance the bench times
            if n not in per["write"]:
                continue
            lines.append(f"{src} {op} {dname} {per['fetch'][n] * 1024 * cal_f:.0f} {per['write'][n] * 1024 * cal_w:.0f}")
        cons = [n for n in per["fetch"] if n.startswith(f"k_cons_partial<{ty},")]
        if cons:
            f_ = sum(per["fetch"][n] for n in cons[:1]) * 1024 * cal_f
            w_ = sum(per["write"].get(n, 0.0) for n in cons[:1]) * 1024 * cal_w
            lines.append(f"{src} conservation {dname} {f_:.0f} {w_:.0f}")
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", default="O1280")
    ap.add_argument("--levels", type=int, default=137)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--cpu-levels", type=int, default=2)
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-remap", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 4 GiB device copy (reference for rocprofv3 byte counters)")
    ap.add_argument("--cpu-leg", metavar="NPZ", help=argparse.SUPPRESS)   # the oracle child process
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("STATS_DB", "FETCH_DB", "WRITE_DB"),
                    help="write profiles/ summaries from rocprofv3 databases of this benchmark (no GPU needed)")
    args = ap.parse_args()
    if args.cpu_leg:
        print(json.dumps(cpu_leg(args.cpu_leg)))
        return
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles, PROFILE_STATS_CMD, PROFILE_PMC_CMD)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X and has no "
              "multi-GPU path (levels and tracers would shard with no communication). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        import torch
        a = torch.ones(1 << 30, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    mesh, res, samples = run_gpu(args)
    V, E, L = mesh.nnodes, mesh.nedges, args.levels
    f32 = res["f32"]
    dom = max((op for op in OPS), key=lambda op: f32["per_op"][op]["ms"])
    dms = f32["per_op"][dom]["ms"]
    dbytes = alg_bytes(dom, V, L, 4)
    traffic = measured_traffic(dom, "f32")
    roof = {"bound": "hbm", "kernel": f32["per_op"][dom]["kernel"], "op": dom,
            "achieved": round(dbytes / (dms * 1e-3) / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": round(dbytes / (dms * 1e-3) / HBM_PEAK, 4),
            "alg_bytes_per_launch": dbytes,
            "traffic": traffic}
    batched = None if args.skip_batched else run_batched(args)
    cpu, errors, nsample = None, None, None
    if not args.skip_cpu:
        leg = run_cpu_baseline(args, samples)
        cpu, errors, nsample = leg["cpu_baseline"], leg["errors_vs_oracle"], leg["sample_nodes"]
    out = {
        "metric": METRIC, "value": f32["edge_updates_s"], "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded SH degree 256 + level trend)",
        "config": {"workload": f"{args.grid} x {L} levels, FP32 fields, FP64 geometry: grad, div, fused lap, "
                               "grad adjoint, div adjoint, FP64 conservation (grad and lap of f in one pass, div "
                               "and grad adjoint of that gradient in one pass)", "nnodes": V, "nedges": E,
                   "nlev": L, "edge_updates_per_step": 6 * E * L},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64": {"ms_per_step": res["f64"]["ms_per_step"], "edge_updates_s": res["f64"]["edge_updates_s"]},
        "bf16": {"ms_per_step": res["bf16"]["ms_per_step"], "edge_updates_s": res["bf16"]["edge_updates_s"]},
        "f32_speedup_over_f64": round(res["f64"]["ms_per_step"] / f32["ms_per_step"], 3),
        "errors_vs_fp64_oracle": None if errors is None else {
            "sample": f"{nsample} nodes (polar rows, degree 5/7, row starts, equator, random) x {L} levels; "
                      "FP64 oracle chains from the same FP64 input (divergence of the gradient and the "
                      "adjoints of the step's chain); FP32 and BF16 include the rounding of the input",
            **errors},
        "batched_o640": batched,
        "remap": res.get("remap"),
        "detail": {k: v for k, v in res.items() if k != "remap"},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
