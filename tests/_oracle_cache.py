"""Memoised oracle meshes for the tests (the oracle is test infrastructure)."""
import functools

import oracle

R_EARTH = 6371220.0


@functools.lru_cache(maxsize=None)
def mesh_and_dual(N, radius=R_EARTH):
    m = oracle.build_mesh(N)
    return m, oracle.build_dual(m, radius)


def coords(mesh):
    g = mesh.grid
    return (g.lon, g.sinlat, g.coslat)
