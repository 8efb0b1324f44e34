"""Batched multi-tracer plans over tracers with uneven level counts, in both
forms (the default one persistent launch per operator over every tracer's
(tile, level chunk) items, and the tracers' field launches), eager and
replayed as a HIP graph, must give the same bits as the single-field calls."""
import pytest
import torch

import paper_1908_07038_amd as pa
from _oracle_cache import mesh_and_dual
from oracle import nabla
from _parity import check, special_groups

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
SINGLE = {"gradient": pa.gradient, "divergence": pa.divergence,
          "gradient_adjoint": pa.gradient_adjoint, "divergence_adjoint": pa.divergence_adjoint}
COMPS = {"gradient": (1, 2), "divergence": (2, 1), "gradient_adjoint": (2, 1), "divergence_adjoint": (1, 2)}


def _tracers(mesh, levels, dtype, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    tracers = []
    for L in levels:
        tr = {}
        for name, (ci, co) in COMPS.items():
            x = torch.randn((mesh.nnodes, L) + ((2,) if ci == 2 else ()), generator=g, device=DEV,
                            dtype=torch.float64).to(dtype)
            y = torch.full((mesh.nnodes, L) + ((2,) if co == 2 else ()), float("nan"), device=DEV, dtype=dtype)
            tr[name] = (x, y)
        tracers.append(tr)
    return tracers


def _check_against_single(mesh, tracers):
    for tr in tracers:
        for name, (x, y) in tr.items():
            ref = SINGLE[name](mesh, x)
            torch.cuda.synchronize()
            assert torch.equal(y, ref), (name, x.shape)


MODES = {"persistent": None, "fields": {"batch_mode": 2},
         "persistent_shaped": {"batch_mode": 1, "waves_per_block": 16, "band_rows": 6, "tile_levels": 64,
                               "tile_wgs_per_cu": 2, "batch_claim": 1},
         "persistent_claim8": {"batch_claim": 8, "tile_kb": 80, "slices_per_iter": 1}}


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batched_equals_single(dtype, mode):
    M = pa.Mesh("O32", device=0)
    levels = [1, 19, 60, 91, 137, 137, 5, 33, 2, 64]
    tracers = _tracers(M, levels, dtype, 1)
    plan = pa.Batch(M, tracers, tune=MODES[mode])
    plan.run()
    torch.cuda.synchronize()
    _check_against_single(M, tracers)


@pytest.mark.parametrize("levels", [[1, 5, 19], [137], [2, 33, 1]], ids=["short", "one", "mixed"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batched_edge_plans(dtype, levels):
    # plans of short columns only (tiles cut for 32 levels or fewer), a single
    # tracer, and a short mix: persistent form and graph replay, bitwise
    M = pa.Mesh("O16", device=0)
    tracers = _tracers(M, levels, dtype, 5)
    plan = pa.Batch(M, tracers)
    for launch in (plan.run, plan.graph_launch, plan.graph_launch):
        for tr in tracers:
            for _, (x, y) in tr.items():
                y.fill_(float("nan"))
        torch.cuda.synchronize()
        launch()
        torch.cuda.synchronize()
        _check_against_single(M, tracers)


@pytest.mark.parametrize("mode", list(MODES))
def test_graph_replays_equal_eager(mode):
    M = pa.Mesh("O32", device=0)
    levels = [137, 1, 60, 19, 91]
    tracers = _tracers(M, levels, torch.float32, 2)
    plan = pa.Batch(M, tracers, tune=MODES[mode])
    for rep in range(3):
        for tr in tracers:                       # eager work between replays
            for _, (x, y) in tr.items():
                y.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.graph_launch()
        torch.cuda.synchronize()
        _check_against_single(M, tracers)
        # change an input in place: the replay must see the new values
        tracers[0]["gradient"][0].mul_(2.0)


def _shared_tracers(mesh, levels, seed, dtype=torch.float32):
    """Tracers whose divergence and gradient adjoint take the same vector
    field (the plan runs them as one pass), the rest as in _tracers."""
    tracers = _tracers(mesh, levels, dtype, seed)
    for tr in tracers:
        tr["gradient_adjoint"] = (tr["divergence"][0], tr["gradient_adjoint"][1])
    return tracers


@pytest.mark.parametrize("mode", ["persistent", "persistent_shaped", "persistent_claim8", "fields"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_batched_divergence_gradient_adjoint_pairs(dtype, mode):
    # plans whose divergence and gradient adjoint read the same fields: one
    # persistent launch for both (FP64: on shapes of at most 8 waves, so the
    # 16-wave shape runs two launches), or the field launches; eager and
    # replayed, bitwise the single-field calls
    M = pa.Mesh("O32", device=0)
    tracers = _shared_tracers(M, [1, 19, 60, 91, 137, 137, 5, 33, 2, 64], 11, dtype)
    plan = pa.Batch(M, tracers, tune=MODES[mode])
    for launch in (plan.run, plan.graph_launch, plan.graph_launch):
        for tr in tracers:
            for _, (x, y) in tr.items():
                y.fill_(float("nan"))
        torch.cuda.synchronize()
        launch()
        torch.cuda.synchronize()
        _check_against_single(M, tracers)


def test_batched_pairs_after_tune():
    # the autotuner times the divergence and the gradient adjoint one at a
    # time and leaves the plan re-planned with the pair: still bitwise
    M = pa.Mesh("O16", device=0)
    tracers = _shared_tracers(M, [137, 19, 1, 60], 12)
    plan = pa.Batch(M, tracers)
    shapes, ms = plan.tune(reps=1)
    assert ms > 0 and set(shapes) == set(COMPS)
    for launch in (plan.run, plan.graph_launch, plan.graph_launch):
        for tr in tracers:
            for _, (x, y) in tr.items():
                y.fill_(float("nan"))
        torch.cuda.synchronize()
        launch()
        torch.cuda.synchronize()
        _check_against_single(M, tracers)


def test_batch_tune_keeps_results():
    M = pa.Mesh("O16", device=0)
    tracers = _tracers(M, [137, 19, 1], torch.float32, 3)
    plan = pa.Batch(M, tracers)
    shapes, ms = plan.tune(reps=1)
    assert ms > 0
    assert set(shapes) == set(COMPS)
    assert all(sh["batch_mode"] in (1, 2) for sh in shapes.values())
    for launch in (plan.run, plan.graph_launch, plan.graph_launch):
        for tr in tracers:
            for _, (x, y) in tr.items():
                y.fill_(float("nan"))
        torch.cuda.synchronize()
        launch()
        torch.cuda.synchronize()
        _check_against_single(M, tracers)


@pytest.mark.parametrize("mode", list(MODES))
def test_batched_against_oracle(mode):
    M = pa.Mesh("O8", device=0)
    m, g = mesh_and_dual(8)
    levels = [3, 40, 1]
    tracers = _tracers(M, levels, torch.float64, 4)
    pa.Batch(M, tracers, tune=MODES[mode]).run()
    torch.cuda.synchronize()
    ora = {"gradient": nabla.gradient, "divergence": nabla.divergence,
           "gradient_adjoint": nabla.gradient_adjoint, "divergence_adjoint": nabla.divergence_adjoint}
    for tr in tracers:
        for name, (x, y) in tr.items():
            ref = ora[name](m, g, x.cpu().numpy())
            check(y.cpu().numpy(), ref, 1e-12, (name, x.shape), per_level=True, groups=special_groups(m))


def test_batch_argument_errors():
    M = pa.Mesh("O4", device=0)
    x = torch.zeros((M.nnodes, 3), device=DEV)
    y = torch.zeros((M.nnodes, 3, 2), device=DEV)
    with pytest.raises(ValueError):
        pa.Batch(M, [])
    with pytest.raises(ValueError):
        pa.Batch(M, [{"gradient": (x, y)}, {"divergence": (y, x)}])
    with pytest.raises(pa.AtlasError) as e:
        pa.Batch(M, [{"gradient": (x, y)}], tune={"waves_per_block": 3})
    assert e.value.code == -1
    # bf16 plans are refused
    xb, yb = x.bfloat16(), y.bfloat16()
    with pytest.raises(ValueError):
        pa.Batch(M, [{"gradient": (xb, yb)}])
