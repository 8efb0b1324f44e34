"""Pins of the remapping oracle (linear interpolation over the source
triangles in 3-D on the sphere; Section 4.3, Figures 4-6)."""
import math

import numpy as np
import pytest

from oracle.grid import OGrid, gaussian_colatitudes
from oracle.mesh import build_mesh
from oracle import remap as R


def _src(N):
    m = build_mesh(N)
    return m.grid.xyz, m.tris


def test_weights_of_the_octant_triangle_by_hand():
    # the triangle through the three axis points lies in the plane x+y+z = 1;
    # the ray through (2,1,1) meets it at (2,1,1)/4 = 1/2 a + 1/4 b + 1/4 c
    a, b, c = np.eye(3)
    for p, want in [((1.0, 1.0, 1.0), (1 / 3, 1 / 3, 1 / 3)), ((2.0, 1.0, 1.0), (0.5, 0.25, 0.25)),
                    ((0.0, 1.0, 3.0), (0.0, 0.25, 0.75)), ((1.0, 0.0, 0.0), (1.0, 0.0, 0.0))]:
        p = np.array(p) / np.linalg.norm(p)
        w, d = R.triangle_weights(a, b, c, p)
        np.testing.assert_allclose(w, want, rtol=0, atol=1e-15)
        assert d > 0
    # the antipodal cone: all triple products negative, D < 0
    w, d = R.triangle_weights(a, b, c, -np.ones(3) / math.sqrt(3))
    assert d < 0


def test_target_f_grid_structure():
    # F8: 16 Gaussian latitudes (the roots of P_16), 32 longitudes each
    g = R.TargetGrid("F8")
    assert g.npoints == 16 * 32
    np.testing.assert_allclose(np.cos(g.theta), np.polynomial.legendre.leggauss(16)[0][::-1], atol=4e-15)
    np.testing.assert_allclose(np.linalg.norm(g.xyz, axis=1), 1.0, atol=1e-15)
    lon = np.arctan2(g.xyz[:, 1], g.xyz[:, 0]) % (2 * math.pi)
    np.testing.assert_allclose(np.sort(lon[:32]), 2 * math.pi * np.arange(32) / 32, atol=1e-14)
    o = R.TargetGrid("O8")
    np.testing.assert_array_equal(o.xyz, OGrid(8).xyz)
    for bad in ("X8", "F0", "F", "O-2"):
        with pytest.raises(ValueError):
            R.TargetGrid(bad)


@pytest.mark.parametrize("N", [4, 12])
def test_identity_remap_reproduces_the_field(N):
    # target = source grid: every point is a node, so the remap is the
    # identity (the zero weights are rounding of triple products of a node
    # with itself, ~eps, divided by D ~ h^2)
    xyz, tris = _src(N)
    _, nodes, w = R.locate(xyz, tris, xyz)
    f = np.random.default_rng(3).standard_normal((xyz.shape[0], 5))
    np.testing.assert_allclose(R.apply(nodes, w, f), f, rtol=0, atol=1e-13)
    assert (nodes == np.arange(xyz.shape[0])[:, None]).any(axis=1).all()


@pytest.mark.parametrize("src,dst", [("O16", "F8"), ("O32", "F8"), ("O12", "O7")])
def test_linear_field_is_exact_at_the_ray_plane_intersection(src, dst):
    # f(X) = g.X + h at the nodes; the linear interpolant equals g.q + h at
    # q = t p, t = (a.n)/(p.n) with n the triangle's normal (ray-plane
    # intersection, computed here without the weights)
    xyz, tris = _src(int(src[1:]))
    p = R.TargetGrid(dst).xyz
    tri, nodes, w = R.locate(xyz, tris, p)
    a, b, c = (xyz[nodes[:, j]] for j in range(3))
    n = np.cross(b - a, c - a)
    t = np.einsum("ij,ij->i", a, n) / np.einsum("ij,ij->i", p, n)
    q = t[:, None] * p
    g = np.array([[0.3, -1.2, 0.7], [1.0, 0.5, -0.25]])
    h = np.array([2.0, -0.5])
    f = xyz @ g.T + h
    np.testing.assert_allclose(R.apply(nodes, w, f), q @ g.T + h, rtol=0, atol=1e-13)
    # the chosen triangle contains the point and the weights sum to one
    assert (w >= -1e-12).all()
    np.testing.assert_allclose(w.sum(axis=1), 1.0, atol=1e-14)
    assert (t > 0).all() and (t <= 1 + 1e-15).all()


def test_located_triangle_brute_force_uniqueness():
    # no other triangle contains a point strictly inside the chosen one
    xyz, tris = _src(8)
    p = R.TargetGrid("F5").xyz
    tri, nodes, w = R.locate(xyz, tris, p)
    a, b, c = (xyz[tris[:, j]] for j in range(3))
    for i in np.nonzero(w.min(axis=1) > 1e-9)[0]:
        dd = R.triple_products(a, b, c, p[i])
        inside = np.nonzero((dd.sum(axis=1) > 0) & (dd.min(axis=1) >= -R.DET_TOL))[0]
        assert inside.tolist() == [tri[i]]


def test_second_order_convergence_of_a_smooth_field():
    # remap of a smooth field to F8 from finer and finer O-grids: the error
    # against the exact values at the target points falls as h^2 (rates
    # 1.71, 1.98 from O32 to O128; the coarsest grids are pre-asymptotic)
    p = R.TargetGrid("F8").xyz

    def field(x):
        lat = np.arcsin(np.clip(x[:, 2], -1, 1))
        lon = np.arctan2(x[:, 1], x[:, 0])
        return np.cos(lat) ** 2 * np.sin(2 * lon) + 0.5 * np.sin(lat)

    errs = []
    for N in (32, 64, 128):
        xyz, tris = _src(N)
        _, nodes, w = R.locate(xyz, tris, p)
        errs.append(np.abs(R.apply(nodes, w, field(xyz)) - field(p)).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (rates > 1.6).all() and rates[-1] > 1.9, (errs, rates)


def test_locate_near_matches_locate():
    xyz, tris = _src(12)
    p = R.TargetGrid("F6").xyz[::7]
    t0, n0, w0 = R.locate(xyz, tris, p)
    t1, n1, w1 = R.locate_near(xyz, tris, p, math.cos(0.5))
    np.testing.assert_array_equal(t0, t1)
    np.testing.assert_array_equal(w0, w1)


def test_adjoint_is_the_dense_transpose():
    # the interpolation as a dense P x V matrix, assembled entry by entry
    xyz, tris = _src(6)
    p = R.TargetGrid("F3").xyz
    _, nodes, w = R.locate(xyz, tris, p)
    A = np.zeros((p.shape[0], xyz.shape[0]))
    for t in range(p.shape[0]):
        for j in range(3):
            A[t, nodes[t, j]] += w[t, j]
    rng = np.random.default_rng(5)
    x = rng.standard_normal((xyz.shape[0], 4))
    y = rng.standard_normal((p.shape[0], 4))
    np.testing.assert_allclose(R.apply(nodes, w, x), A @ x, rtol=0, atol=1e-14)
    np.testing.assert_allclose(R.apply_adjoint(nodes, w, y, xyz.shape[0]), A.T @ y, rtol=0, atol=1e-14)

