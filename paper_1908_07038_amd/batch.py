"""Batched multi-tracer plans over many fields with different level counts.

By default each operator is one persistent launch over every tracer: the
workgroups of each XCD walk that XCD's share of the (tracer, tile, level
chunk) items on the LDS tiles of the single-field one-tile form, with the
same arithmetic per output element, so results equal the single-field calls
bit for bit.  ``tune={"batch_mode": 2}`` runs the tracers' single-field
launches instead.  Either form can be replayed as a HIP graph."""

import ctypes

from . import (F32, F64, OP_DIVERGENCE, OP_DIVERGENCE_ADJOINT, OP_GRADIENT, OP_GRADIENT_ADJOINT,
               TracerDesc, TuneShape, _check, _dtype_code, _field, _like, _stream, lib)

_OPS = {"gradient": OP_GRADIENT, "divergence": OP_DIVERGENCE,
        "gradient_adjoint": OP_GRADIENT_ADJOINT, "divergence_adjoint": OP_DIVERGENCE_ADJOINT}
_BIT = {OP_GRADIENT: 0, OP_DIVERGENCE: 1, OP_GRADIENT_ADJOINT: 2, OP_DIVERGENCE_ADJOINT: 3}
_COMPS = {OP_GRADIENT: (1, 2), OP_DIVERGENCE: (2, 1), OP_GRADIENT_ADJOINT: (2, 1),
          OP_DIVERGENCE_ADJOINT: (1, 2)}


class Batch:
    """Plan over ``tracers``: a list of dicts {op name: (input, output)}.

    Every tracer must give tensors for the same set of operators.  The plan
    keeps references to the tensors; their storage must stay alive and in
    place while the plan is used.
    """

    def __init__(self, mesh, tracers, tune=None):
        if not tracers:
            raise ValueError("need at least one tracer")
        names = set(tracers[0])
        if not names or not names <= set(_OPS):
            raise ValueError(f"operators must be among {sorted(_OPS)}")
        mask = 0
        for n in names:
            mask |= _OPS[n]
        self.mesh = mesh
        self.mask = mask
        self._keep = []
        dtype = None
        levels = []
        for t, tr in enumerate(tracers):
            if set(tr) != names:
                raise ValueError("all tracers must use the same operators")
            nlev = None
            for n, (x, y) in tr.items():
                ci, co = _COMPS[_OPS[n]]
                # contiguous device tensors [nnodes][nlev], or [nnodes][nlev][2]
                # for vector fields, one level count per tracer
                lx = _field(mesh, x, ci, f"tracer {t} {n} input")
                nlev = lx if nlev is None else nlev
                _like(mesh, y, co, nlev, x.dtype, f"tracer {t} {n} output")
                if lx != nlev:
                    raise ValueError(f"tracer {t}: all fields need the same level count")
                dtype = _dtype_code(x) if dtype is None else dtype
                if _dtype_code(x) != dtype:
                    raise ValueError("one dtype per plan")
            levels.append(nlev)
        if dtype not in (F32, F64):
            raise ValueError("batched plans take float32 or float64 fields")
        descs = (TracerDesc * len(tracers))()
        for t, tr in enumerate(tracers):
            descs[t].nlev = levels[t]
            for n, (x, y) in tr.items():
                b = _BIT[_OPS[n]]
                descs[t].in_[b] = x.data_ptr()
                descs[t].out[b] = y.data_ptr()
                self._keep += [x, y]
        self.dtype = dtype
        self.device_tensor = tracers[0][next(iter(names))][0]
        ts = TuneShape(**tune) if tune else None
        h = ctypes.c_void_p()
        _check(lib().atlas_batch_create(mesh.handle, dtype, descs, len(tracers), mask,
                                        ctypes.byref(ts) if ts is not None else None, ctypes.byref(h)))
        self._h = h

    def run(self):
        """Enqueue the plan on the current stream: one persistent launch per
        operator (or the field launches with ``batch_mode`` 2)."""
        _check(lib().atlas_batch_run(self._h, _stream(self.device_tensor)))

    def graph_launch(self):
        """Replay the plan as a HIP graph on the current stream (captured once)."""
        _check(lib().atlas_batch_graph_launch(self._h, _stream(self.device_tensor)))

    def tune(self, reps=3):
        """Time the field form and persistent shapes of each operator on the
        plan's own fields (overwriting its outputs); keeps each operator's
        fastest shape in the plan.  Returns ({operator name: shape dict},
        ms per run of the whole plan)."""
        best = (TuneShape * 4)()
        ms = ctypes.c_float()
        _check(lib().atlas_batch_tune(self._h, reps, _stream(self.device_tensor), best, ctypes.byref(ms)))
        shapes = {n: best[_BIT[b]].as_dict() for n, b in _OPS.items() if self.mask & b}
        return shapes, ms.value

    def close(self):
        if getattr(self, "_h", None):
            lib().atlas_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
