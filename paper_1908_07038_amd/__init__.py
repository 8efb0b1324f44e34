"""MI355X (gfx950) median-dual Nabla operators on octahedral reduced Gaussian
meshes.

Thin Python binding of ``libatlas_nabla.so`` (C ABI in
``include/atlas_nabla.h``).  Every step of every operator runs in the HIP
kernels of that library; this module only marshals arguments: it turns torch
tensors into device pointers, the current torch stream into a ``hipStream_t``
and status codes into exceptions.  PyTorch provides device memory and streams.

Workflow, after the Grid -> Mesh -> FunctionSpace -> Field sequence of the
Atlas report (Section 2.3, Figure 2)::

    mesh = Mesh("O1280", radius=6371220.0, device=0)
    fs = NodeColumns(mesh, levels=137)
    f = fs.create_field(torch.float32)            # [nnodes][137]
    g = gradient(mesh, f)                         # [nnodes][137][2]
    lap = laplacian(mesh, f)
"""

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libatlas_nabla.so")

F64, F32, BF16 = 0, 1, 2
OP_GRADIENT, OP_DIVERGENCE, OP_GRADIENT_ADJOINT, OP_DIVERGENCE_ADJOINT, OP_LAPLACIAN = 1, 2, 4, 8, 16
OP_CURL, OP_CURL_ADJOINT = 32, 64
# the one-pass calls, for describe() only
OP_GRADIENT_LAPLACIAN, OP_DIVERGENCE_CURL, OP_DIVERGENCE_GRADIENT_ADJOINT = 1 << 16, 1 << 17, 1 << 18
STATUS = {0: "ATLAS_OK", -1: "ATLAS_EINVAL", -2: "ATLAS_ENOMEM", -3: "ATLAS_EHIP",
          -4: "ATLAS_ENODEV", -5: "ATLAS_EDTYPE", -6: "ATLAS_ESHAPE"}


class AtlasError(RuntimeError):
    """A non-OK status from the C ABI."""

    def __init__(self, code, message):
        self.code = code
        super().__init__(f"{STATUS.get(code, code)}: {message}")


class TuneShape(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("nodes_per_wave", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("lanes_per_node", ctypes.c_int32), ("slices_per_iter", ctypes.c_int32),
                ("band_rows", ctypes.c_int32), ("run_nodes", ctypes.c_int32),
                ("nt_stores", ctypes.c_int32), ("row_window", ctypes.c_int32),
                ("lds_tiles", ctypes.c_int32), ("tile_kb", ctypes.c_int32),
                ("tile_waves", ctypes.c_int32), ("producer_waves", ctypes.c_int32),
                ("tile_wgs_per_cu", ctypes.c_int32), ("tile_levels", ctypes.c_int32),
                ("batch_mode", ctypes.c_int32), ("batch_claim", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class TracerDesc(ctypes.Structure):
    _fields_ = [("nlev", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("in_", ctypes.c_void_p * 4), ("out", ctypes.c_void_p * 4)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64P = ctypes.POINTER(ctypes.c_int64)
_SIGS = {
    "atlas_version": (ctypes.c_char_p, []),
    "atlas_last_error": (ctypes.c_char_p, []),
    "atlas_device_count": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int)]),
    "atlas_mesh_build": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_P)]),
    "atlas_mesh_free": (None, [_P]),
    "atlas_mesh_sizes": (ctypes.c_int, [_P, _I64P, _I64P, _I64P, _I64P, ctypes.POINTER(_I32),
                                        ctypes.POINTER(_I32)]),
    "atlas_mesh_export_grid": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "atlas_mesh_export_connectivity": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "atlas_mesh_export_geometry": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "atlas_nabla_gradient": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P]),
    "atlas_nabla_divergence": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P]),
    "atlas_nabla_laplacian": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P, _P]),
    "atlas_nabla_gradient_adjoint": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P]),
    "atlas_nabla_divergence_adjoint": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P]),
    "atlas_nabla_conservation": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P, _P]),
    "atlas_nabla_conservation_noalloc": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P, _P]),
    "atlas_nabla_gradient_laplacian": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P, _P]),
    "atlas_nabla_divergence_curl": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P, _P]),
    "atlas_nabla_divergence_gradient_adjoint": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P, _P]),
    "atlas_nabla_curl": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P]),
    "atlas_nabla_curl_adjoint": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P]),
    "atlas_batch_create": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(TracerDesc), _I32,
                                          ctypes.c_uint32, ctypes.POINTER(TuneShape), ctypes.POINTER(_P)]),
    "atlas_batch_run": (ctypes.c_int, [_P, _P]),
    "atlas_batch_graph_launch": (ctypes.c_int, [_P, _P]),
    "atlas_batch_free": (None, [_P]),
    "atlas_batch_tune": (ctypes.c_int, [_P, _I32, _P, ctypes.POINTER(TuneShape),
                                        ctypes.POINTER(ctypes.c_float)]),
    "atlas_nabla_tune": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_uint32, _I32, _P, _P, _I32, _P,
                                        ctypes.POINTER(TuneShape), ctypes.POINTER(ctypes.c_float)]),
    "atlas_nabla_set_tune": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(TuneShape)]),
    "atlas_nabla_describe": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_uint32, _I32, ctypes.POINTER(TuneShape),
                                            ctypes.c_char_p, _I32]),
    "atlas_remap_build": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.POINTER(_P)]),
    "atlas_remap_free": (None, [_P]),
    "atlas_remap_sizes": (ctypes.c_int, [_P, _I64P, _I64P]),
    "atlas_remap_export": (ctypes.c_int, [_P, _P, _P, _P]),
    "atlas_remap_apply": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P]),
    "atlas_remap_apply_adjoint": (ctypes.c_int, [_P, ctypes.c_int, _I32, _P, _P, _P]),
}


def lib():
    """Load libatlas_nabla.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1908_07038_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise AtlasError(code, lib().atlas_last_error().decode())


def version():
    return lib().atlas_version().decode()


def device_count():
    n = ctypes.c_int(0)
    code = lib().atlas_device_count(ctypes.byref(n))
    return n.value if code == 0 else 0


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Mesh:
    """Median-dual mesh of an octahedral grid "O<N>" (see atlas_mesh_build).

    ``device`` is a HIP device ordinal, or -1 for a host-only mesh whose
    connectivity and geometry can be exported but which runs no operator.
    """

    def __init__(self, grid, radius=6371220.0, device=0):
        self.grid = grid
        self.radius = float(radius)
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(lib().atlas_mesh_build(grid.encode(), self.radius, self.device, ctypes.byref(h)))
        self._h = h
        v, e, t, p = (ctypes.c_int64() for _ in range(4))
        ms, nr = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().atlas_mesh_sizes(h, *(ctypes.byref(x) for x in (v, e, t, p, ms, nr))))
        self.nnodes, self.nedges, self.ntris = v.value, e.value, t.value
        self.npole_edges, self.max_slots, self.nrows = p.value, ms.value, nr.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().atlas_mesh_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- host exports (numpy) -------------------------------------------------
    def export_grid(self):
        V, R = self.nnodes, self.nrows
        out = dict(row_size=np.empty(R, np.int32), row_off=np.empty(R + 1, np.int64),
                   colat=np.empty(R, np.float64), lonlat=np.empty((V, 2), np.float64),
                   xyz=np.empty((V, 3), np.float64))
        _check(lib().atlas_mesh_export_grid(self._h, *(_np_ptr(out[k]) for k in
                                                       ("row_size", "row_off", "colat", "lonlat", "xyz"))))
        return out

    def export_connectivity(self):
        V, E, T = self.nnodes, self.nedges, self.ntris
        out = dict(tris=np.empty((T, 3), np.int32), edges=np.empty((E, 2), np.int32),
                   csr_off=np.empty(V + 1, np.int64), nbr=np.empty(2 * E, np.int32),
                   eid=np.empty(2 * E, np.int32), sgn=np.empty(2 * E, np.int8),
                   rev=np.empty(2 * E, np.int8), is_pole=np.empty(E, np.uint8))
        keys = ("tris", "edges", "csr_off", "nbr", "eid", "sgn", "rev", "is_pole")
        _check(lib().atlas_mesh_export_connectivity(self._h, *(_np_ptr(out[k]) for k in keys)))
        return out

    def export_geometry(self):
        V, E = self.nnodes, self.nedges
        out = dict(S=np.empty((E, 3)), V=np.empty(V), basis=np.empty((V, 2, 3)), C=np.empty((V, 3)))
        _check(lib().atlas_mesh_export_geometry(self._h, *(_np_ptr(out[k]) for k in ("S", "V", "basis", "C"))))
        return out

    def coords(self):
        """(lon, sin(lat), cos(lat)) of every node, for input generators."""
        g = self.export_grid()
        sl = np.cos(g["colat"])[np.repeat(np.arange(self.nrows), g["row_size"])]
        cl = np.sin(g["colat"])[np.repeat(np.arange(self.nrows), g["row_size"])]
        return g["lonlat"][:, 0].copy(), sl, cl


class NodeColumns:
    """Function space of node columns: fields [nnodes][levels](, 2)."""

    def __init__(self, mesh, levels):
        self.mesh = mesh
        self.levels = int(levels)

    def create_field(self, dtype, variables=1, fill=None):
        import torch
        shape = (self.mesh.nnodes, self.levels) + ((2,) if variables == 2 else ())
        dev = torch.device("cuda", self.mesh.device)
        t = torch.empty(shape, dtype=dtype, device=dev)
        if fill is not None:
            t.fill_(fill)
        return t


# ---- torch marshalling ------------------------------------------------------

def _dtype_code(t):
    import torch
    codes = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
    if t.dtype not in codes:
        raise TypeError(f"unsupported dtype {t.dtype} (float64, float32, bfloat16)")
    return codes[t.dtype]


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _field(mesh, t, comps, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    want = 3 if comps == 2 else 2
    if t.dim() != want or t.shape[0] != mesh.nnodes or (comps == 2 and t.shape[2] != 2):
        raise ValueError(f"{name} must have shape [nnodes][nlev]" + ("[2]" if comps == 2 else ""))
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.shape[1]


def _like(mesh, t, comps, nlev, dtype, name):
    """Checks a caller-given output or workspace: a contiguous device tensor
    [nnodes][nlev] (or [nnodes][nlev][2]) of the input's dtype.  The kernels
    write nnodes * nlev (* 2) elements through it, so a smaller or narrower
    buffer is refused here."""
    if _field(mesh, t, comps, name) != nlev or t.dtype != dtype:
        raise ValueError(f"{name} must be [nnodes][{nlev}]" + ("[2]" if comps == 2 else "") + f" of {dtype}")
    return t


def _apply(fn, mesh, x, in_comps, out_comps, out):
    import torch
    nlev = _field(mesh, x, in_comps, "input")
    shape = (mesh.nnodes, nlev) + ((2,) if out_comps == 2 else ())
    if out is None:
        out = torch.empty(shape, dtype=x.dtype, device=x.device)
    else:
        _like(mesh, out, out_comps, nlev, x.dtype, "out")
    _check(fn(mesh.handle, _dtype_code(x), nlev, ctypes.c_void_p(x.data_ptr()),
              ctypes.c_void_p(out.data_ptr()), _stream(x)))
    return out


def gradient(mesh, f, out=None):
    """[V][L] -> [V][L][2] (east, north)."""
    return _apply(lib().atlas_nabla_gradient, mesh, f, 1, 2, out)


def divergence(mesh, uv, out=None):
    """[V][L][2] -> [V][L]."""
    return _apply(lib().atlas_nabla_divergence, mesh, uv, 2, 1, out)


def gradient_adjoint(mesh, w, out=None):
    """[V][L][2] -> [V][L], exact transpose of :func:`gradient`."""
    return _apply(lib().atlas_nabla_gradient_adjoint, mesh, w, 2, 1, out)


def divergence_adjoint(mesh, d, out=None):
    """[V][L] -> [V][L][2], exact transpose of :func:`divergence`."""
    return _apply(lib().atlas_nabla_divergence_adjoint, mesh, d, 1, 2, out)


def curl(mesh, uv, out=None):
    """[V][L][2] -> [V][L]: vertical vorticity (circulation per unit area)."""
    return _apply(lib().atlas_nabla_curl, mesh, uv, 2, 1, out)


def curl_adjoint(mesh, z, out=None):
    """[V][L] -> [V][L][2], exact transpose of :func:`curl`."""
    return _apply(lib().atlas_nabla_curl_adjoint, mesh, z, 1, 2, out)


def laplacian(mesh, f, out=None, workspace=None):
    """div(grad f): fused two-ring pass, or two passes through ``workspace``
    ([V][L][2], same dtype) when given."""
    import torch
    nlev = _field(mesh, f, 1, "f")
    if workspace is not None:
        _like(mesh, workspace, 2, nlev, f.dtype, "workspace")
    if out is None:
        out = torch.empty_like(f)
    else:
        _like(mesh, out, 1, nlev, f.dtype, "out")
    ws = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    _check(lib().atlas_nabla_laplacian(mesh.handle, _dtype_code(f), nlev, ctypes.c_void_p(f.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), ws, _stream(f)))
    return out


class Remap:
    """Remapping of node fields of ``mesh`` to the points of a target grid
    ("F<M>" or "O<M>") by linear interpolation over the source triangles in
    3-D on the sphere (see atlas_remap_build).  Keep ``mesh`` alive while the
    remap is used (the object holds a reference to it)."""

    def __init__(self, mesh, target):
        self.mesh = mesh
        self.target = target
        h = ctypes.c_void_p()
        _check(lib().atlas_remap_build(mesh.handle, target.encode(), ctypes.byref(h)))
        self._h = h
        n, f = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().atlas_remap_sizes(h, ctypes.byref(n), ctypes.byref(f)))
        self.npoints, self.nfallback = n.value, f.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().atlas_remap_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export(self):
        """Host tables: nodes int32 [P][3], weights FP64 [P][3], xyz [P][3]."""
        P = self.npoints
        out = dict(nodes=np.empty((P, 3), np.int32), weights=np.empty((P, 3), np.float64),
                   xyz=np.empty((P, 3), np.float64))
        _check(lib().atlas_remap_export(self._h, *(_np_ptr(out[k]) for k in ("nodes", "weights", "xyz"))))
        return out

    def __call__(self, f, out=None):
        """[V][L] source field -> [P][L] target field (same dtype)."""
        import torch
        nlev = _field(self.mesh, f, 1, "f")
        if out is None:
            out = torch.empty((self.npoints, nlev), dtype=f.dtype, device=f.device)
        elif (not out.is_cuda or out.dtype != f.dtype or tuple(out.shape) != (self.npoints, nlev)
              or not out.is_contiguous()):
            raise ValueError("out must be a contiguous device tensor [npoints][nlev] of the input dtype")
        _check(lib().atlas_remap_apply(self._h, _dtype_code(f), nlev, ctypes.c_void_p(f.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream(f)))
        return out

    def adjoint(self, ybar, out=None):
        """[P][L] -> [V][L]: exact transpose of the remap."""
        import torch
        if (not ybar.is_cuda or ybar.dim() != 2 or ybar.shape[0] != self.npoints or not ybar.is_contiguous()):
            raise ValueError("ybar must be a contiguous device tensor [npoints][nlev]")
        nlev = ybar.shape[1]
        if out is None:
            out = torch.empty((self.mesh.nnodes, nlev), dtype=ybar.dtype, device=ybar.device)
        else:
            _like(self.mesh, out, 1, nlev, ybar.dtype, "out")
        _check(lib().atlas_remap_apply_adjoint(self._h, _dtype_code(ybar), nlev, ctypes.c_void_p(ybar.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), _stream(ybar)))
        return out


def gradient_laplacian(mesh, f, out_grad=None, out_lap=None):
    """(gradient(f), laplacian(f)) in one pass over f (same values as the two
    calls, up to the sign of zero)."""
    import torch
    nlev = _field(mesh, f, 1, "f")
    if out_grad is not None:
        _like(mesh, out_grad, 2, nlev, f.dtype, "out_grad")
    if out_lap is not None:
        _like(mesh, out_lap, 1, nlev, f.dtype, "out_lap")
    if out_grad is None:
        out_grad = torch.empty((mesh.nnodes, nlev, 2), dtype=f.dtype, device=f.device)
    if out_lap is None:
        out_lap = torch.empty_like(f)
    _check(lib().atlas_nabla_gradient_laplacian(mesh.handle, _dtype_code(f), nlev, ctypes.c_void_p(f.data_ptr()),
                                                ctypes.c_void_p(out_grad.data_ptr()),
                                                ctypes.c_void_p(out_lap.data_ptr()), _stream(f)))
    return out_grad, out_lap


def divergence_curl(mesh, uv, out_div=None, out_curl=None):
    """(divergence(uv), curl(uv)) in one pass over uv (same values as the two
    calls, up to the sign of zero)."""
    import torch
    nlev = _field(mesh, uv, 2, "uv")
    if out_div is not None:
        _like(mesh, out_div, 1, nlev, uv.dtype, "out_div")
    if out_curl is not None:
        _like(mesh, out_curl, 1, nlev, uv.dtype, "out_curl")
    if out_div is None:
        out_div = torch.empty((mesh.nnodes, nlev), dtype=uv.dtype, device=uv.device)
    if out_curl is None:
        out_curl = torch.empty((mesh.nnodes, nlev), dtype=uv.dtype, device=uv.device)
    _check(lib().atlas_nabla_divergence_curl(mesh.handle, _dtype_code(uv), nlev, ctypes.c_void_p(uv.data_ptr()),
                                             ctypes.c_void_p(out_div.data_ptr()),
                                             ctypes.c_void_p(out_curl.data_ptr()), _stream(uv)))
    return out_div, out_curl


def divergence_gradient_adjoint(mesh, uv, out_div=None, out_fbar=None):
    """(divergence(uv), gradient_adjoint(uv)) in one pass over uv (same values
    as the two calls, up to the sign of zero)."""
    import torch
    nlev = _field(mesh, uv, 2, "uv")
    if out_div is not None:
        _like(mesh, out_div, 1, nlev, uv.dtype, "out_div")
    if out_fbar is not None:
        _like(mesh, out_fbar, 1, nlev, uv.dtype, "out_fbar")
    if out_div is None:
        out_div = torch.empty((mesh.nnodes, nlev), dtype=uv.dtype, device=uv.device)
    if out_fbar is None:
        out_fbar = torch.empty((mesh.nnodes, nlev), dtype=uv.dtype, device=uv.device)
    _check(lib().atlas_nabla_divergence_gradient_adjoint(mesh.handle, _dtype_code(uv), nlev,
                                                         ctypes.c_void_p(uv.data_ptr()),
                                                         ctypes.c_void_p(out_div.data_ptr()),
                                                         ctypes.c_void_p(out_fbar.data_ptr()), _stream(uv)))
    return out_div, out_fbar


def conservation(mesh, div):
    """Per-level FP64 (sum V_i div_ik, sum |V_i div_ik|) as device tensors."""
    import torch
    nlev = _field(mesh, div, 1, "div")
    s = torch.empty(nlev, dtype=torch.float64, device=div.device)
    a = torch.empty(nlev, dtype=torch.float64, device=div.device)
    _check(lib().atlas_nabla_conservation(mesh.handle, _dtype_code(div), nlev, ctypes.c_void_p(div.data_ptr()),
                                          ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                                          _stream(div)))
    return s, a


def conservation_noalloc(mesh, div, out_sum, out_abs):
    """conservation() into caller-given FP64 [nlev] device tensors; the library
    allocates nothing (its partial sums live in a static per-GPU array, so
    calls that overlap on one GPU race)."""
    import torch
    nlev = _field(mesh, div, 1, "div")
    for t, name in ((out_sum, "out_sum"), (out_abs, "out_abs")):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.device == div.device
                and tuple(t.shape) == (nlev,) and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape ({nlev},) on {div.device}")
    _check(lib().atlas_nabla_conservation_noalloc(mesh.handle, _dtype_code(div), nlev,
                                                  ctypes.c_void_p(div.data_ptr()),
                                                  ctypes.c_void_p(out_sum.data_ptr()),
                                                  ctypes.c_void_p(out_abs.data_ptr()), _stream(div)))
    return out_sum, out_abs


def tune(mesh, op, x, out, reps=10):
    """Time launch shapes of one operator on (x, out); returns (shape dict, ms)."""
    best = TuneShape()
    ms = ctypes.c_float()
    nlev = x.shape[1]
    _check(lib().atlas_nabla_tune(mesh.handle, _dtype_code(x), op, nlev, ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), reps, _stream(x), ctypes.byref(best),
                                  ctypes.byref(ms)))
    return best.as_dict(), ms.value


def describe(mesh, op, dtype_code, nlev):
    """(resolved shape dict, kernel name) of a single-field call of op (an OP_*
    bit, or OP_GRADIENT_LAPLACIAN, OP_DIVERGENCE_CURL,
    OP_DIVERGENCE_GRADIENT_ADJOINT for the one-pass calls)."""
    sh = TuneShape()
    buf = ctypes.create_string_buffer(128)
    _check(lib().atlas_nabla_describe(mesh.handle, dtype_code, op, nlev, ctypes.byref(sh), buf, 128))
    return sh.as_dict(), buf.value.decode()


def set_tune(mesh, op, dtype_code, shape=None):
    """Fix the launch shape of (op, dtype) on this mesh; None restores the default."""
    if shape is None:
        _check(lib().atlas_nabla_set_tune(mesh.handle, dtype_code, op, None))
    else:
        ts = TuneShape(**shape)
        _check(lib().atlas_nabla_set_tune(mesh.handle, dtype_code, op, ctypes.byref(ts)))


from .autograd import (Gradient, Divergence, Laplacian, Curl, GradientLaplacian, DivergenceCurl,  # noqa: E402,F401
                       DivergenceGradientAdjoint, RemapFunction, grad, div, lap, rot, grad_lap, div_rot, div_gradt,
                       remap)
from .batch import Batch  # noqa: E402,F401
