"""Autotuning with a JSON cache of launch shapes.

The cache maps "<grid>/<operator>/<dtype>/<levels>" to the shape the tuner
(atlas_nabla_tune) found fastest on this device, so a later process applies
the shapes without timing again.  Shapes depend on the device; keep one cache
file per device model.
"""

import json
import os

from . import BF16, F32, F64, OP_CURL, OP_CURL_ADJOINT, OP_DIVERGENCE, OP_DIVERGENCE_ADJOINT, OP_GRADIENT, \
    OP_GRADIENT_ADJOINT, OP_LAPLACIAN, set_tune, tune

OPERATORS = {"gradient": (OP_GRADIENT, 1, 2), "divergence": (OP_DIVERGENCE, 2, 1),
             "laplacian": (OP_LAPLACIAN, 1, 1), "gradient_adjoint": (OP_GRADIENT_ADJOINT, 2, 1),
             "divergence_adjoint": (OP_DIVERGENCE_ADJOINT, 1, 2), "curl": (OP_CURL, 2, 1),
             "curl_adjoint": (OP_CURL_ADJOINT, 1, 2)}
DTYPES = {"float64": F64, "float32": F32, "bfloat16": BF16}


def cache_key(mesh, op_name, dtype_name, nlev):
    return f"{mesh.grid}/{op_name}/{dtype_name}/{int(nlev)}"


def load_cache(path):
    """The cache as a dict (empty if the file does not exist)."""
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        data = json.load(fh)
    if not isinstance(data, dict):
        raise ValueError(f"{path}: not a tuning cache")
    return data


def save_cache(path, cache):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply_cache(mesh, cache, nlev, ops=None, dtypes=None):
    """Set the cached shapes of (ops x dtypes) at nlev levels on the mesh;
    returns the keys applied."""
    applied = []
    for op_name in ops or OPERATORS:
        bit = OPERATORS[op_name][0]
        for dtype_name in dtypes or DTYPES:
            key = cache_key(mesh, op_name, dtype_name, nlev)
            if key in cache:
                set_tune(mesh, bit, DTYPES[dtype_name], cache[key]["shape"])
                applied.append(key)
    return applied


def autotune(mesh, nlev, ops=None, dtypes=("float32",), cache_path=None, reps=5):
    """Tune (ops x dtypes) at nlev levels on the mesh's device, reusing and
    extending the cache at cache_path; the chosen shapes are set on the mesh.
    Returns {key: milliseconds per launch (None if taken from the cache)}."""
    import torch

    cache = load_cache(cache_path)
    dev = torch.device("cuda", mesh.device)
    result = {}
    for op_name in ops or OPERATORS:
        bit, ci, co = OPERATORS[op_name]
        for dtype_name in dtypes:
            key = cache_key(mesh, op_name, dtype_name, nlev)
            if key in cache:
                set_tune(mesh, bit, DTYPES[dtype_name], cache[key]["shape"])
                result[key] = None
                continue
            dt = getattr(torch, dtype_name)
            x = torch.randn((mesh.nnodes, nlev) + ((2,) if ci == 2 else ()), device=dev).to(dt)
            y = torch.empty((mesh.nnodes, nlev) + ((2,) if co == 2 else ()), device=dev, dtype=dt)
            shape, ms = tune(mesh, bit, x, y, reps=reps)
            set_tune(mesh, bit, DTYPES[dtype_name], shape)
            cache[key] = {"shape": shape, "ms": ms}
            result[key] = ms
            del x, y
    if cache_path:
        save_cache(cache_path, cache)
    return result
