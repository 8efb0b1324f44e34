"""Plain FP64 CPU oracle for the median-dual Nabla operators.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import anything from this package.  The HIP library never calls it and shares
no code with it: the two meet only through seeded inputs from ``workloads``.

What it computes (the paper names the operators in its description of Atlas,
Section 2.3, and the octahedral "O" grids in Section 4.3 and Figure 4; the
grid, mesh and dual definitions it defers to other documents are restated
here in the readings listed in each module):

* ``grid``  -- Gaussian colatitudes and the octahedral reduced Gaussian grid.
* ``mesh``  -- triangulation between latitude rows with polar caps, unique
  edges, node-to-edge CSR with signs and reverse slots.
* ``dual``  -- the median dual on the sphere: dual normals S_e, dual volumes
  V_i, local (east, north) basis, closure vectors C_i.
* ``nabla`` -- gradient, divergence, Laplacian and the exact adjoints of
  gradient and divergence, applied as edge loops with scatter, plus the
  FP64 conservation sums.
* ``remap`` -- target grids (regular "F" and octahedral "O" Gaussian grids)
  and the linear interpolation of a field over the source triangles in 3-D
  on the sphere (Section 4.3, Figures 4-6), with brute-force point location.
* ``capstudy`` -- alternative treatments of the poles for the accuracy study
  only: pole-node fans on the spherical dual, and the dual taken in the
  longitude-latitude plane with pole strips and antipodal pole edges.

Everything is FP64 NumPy, vectorised where a loop would be too slow for the
large grids; no blocking or reordering beyond what each formula states.
"""

from .grid import OGrid, gaussian_colatitudes, parse_grid_name  # noqa: F401
from .mesh import OMesh, build_mesh  # noqa: F401
from .dual import DualGeometry, build_dual  # noqa: F401
from . import nabla  # noqa: F401
from . import remap  # noqa: F401
from . import capstudy  # noqa: F401
