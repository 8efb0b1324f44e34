"""Argument checks of the Python binding that need no GPU: every caller-given
output or workspace is refused before any device pointer reaches the library
when its dtype, level count, vector width or layout does not match the input
(the kernels write nnodes * nlev (* 2) elements through it).  Device tensors
are stood in for by objects that raise if their address is ever taken."""
import pytest
import torch

import paper_1908_07038_amd as pa


class DeviceTensorStub:
    """Shape, dtype and layout of a device tensor; no storage."""

    is_cuda = True

    def __init__(self, shape, dtype=torch.float32, contiguous=True):
        self.shape = tuple(shape)
        self.dtype = dtype
        self._contiguous = contiguous

    def dim(self):
        return len(self.shape)

    def is_contiguous(self):
        return self._contiguous

    def data_ptr(self):
        raise AssertionError("a checked-out argument reached the library")


@pytest.fixture(scope="module")
def mesh():
    M = pa.Mesh("O4", device=-1)
    yield M
    M.close()


def test_outputs_and_workspace_are_checked(mesh):
    V = mesh.nnodes
    f = DeviceTensorStub((V, 5))
    uv = DeviceTensorStub((V, 5, 2))
    bad_out_scalar = [DeviceTensorStub((V, 4)), DeviceTensorStub((V, 5), torch.float64),
                      DeviceTensorStub((V, 5), contiguous=False), DeviceTensorStub((V + 1, 5)),
                      DeviceTensorStub((V, 5, 2))]
    bad_out_vector = [DeviceTensorStub((V, 4, 2)), DeviceTensorStub((V, 5, 2), torch.bfloat16),
                      DeviceTensorStub((V, 5, 3)), DeviceTensorStub((V, 5)),
                      DeviceTensorStub((V, 5, 2), contiguous=False)]
    for bad in bad_out_scalar:
        with pytest.raises(ValueError):
            pa.laplacian(mesh, f, out=bad)
        with pytest.raises(ValueError):
            pa.divergence(mesh, uv, out=bad)
        with pytest.raises(ValueError):
            pa.gradient_adjoint(mesh, uv, out=bad)
        with pytest.raises(ValueError):
            pa.curl(mesh, uv, out=bad)
        with pytest.raises(ValueError):
            pa.divergence_curl(mesh, uv, out_div=bad)
        with pytest.raises(ValueError):
            pa.divergence_gradient_adjoint(mesh, uv, out_fbar=bad)
        with pytest.raises(ValueError):
            pa.gradient_laplacian(mesh, f, out_lap=bad)
    for bad in bad_out_vector:
        with pytest.raises(ValueError):
            pa.gradient(mesh, f, out=bad)
        with pytest.raises(ValueError):
            pa.divergence_adjoint(mesh, f, out=bad)
        with pytest.raises(ValueError):
            pa.laplacian(mesh, f, workspace=bad)
        with pytest.raises(ValueError):
            pa.gradient_laplacian(mesh, f, out_grad=bad)


def test_inputs_are_checked(mesh):
    V = mesh.nnodes
    for bad in [DeviceTensorStub((V + 1, 5)), DeviceTensorStub((V, 5), contiguous=False),
                DeviceTensorStub((V, 5, 2))]:
        with pytest.raises(ValueError):
            pa.gradient(mesh, bad)
    for bad in [DeviceTensorStub((V, 5, 3)), DeviceTensorStub((V, 5)), DeviceTensorStub((V, 5, 1))]:
        with pytest.raises(ValueError):
            pa.divergence(mesh, bad)


def test_batch_fields_are_checked(mesh):
    V = mesh.nnodes
    f = DeviceTensorStub((V, 3))
    good_vec = DeviceTensorStub((V, 3, 2))
    for tracer in [{"gradient": (f, DeviceTensorStub((V, 3, 3)))},          # vector width
                   {"divergence": (DeviceTensorStub((V, 3, 4)), f)},
                   {"gradient": (f, DeviceTensorStub((V, 2, 2)))},          # level count
                   {"gradient": (f, DeviceTensorStub((V, 3, 2), torch.float64))},
                   {"gradient": (f, good_vec), "divergence": (good_vec, DeviceTensorStub((V, 4)))},
                   {"gradient": (DeviceTensorStub((V, 3), contiguous=False), good_vec)}]:
        with pytest.raises(ValueError):
            pa.Batch(mesh, [tracer])
