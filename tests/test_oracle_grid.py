"""Pins of the oracle's O-grid: Gaussian colatitudes and row structure."""
import math
import os

import numpy as np
import pytest
import scipy.special

import oracle
from oracle.grid import gaussian_colatitudes, OGrid, parse_grid_name

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [2, 4, 8, 20, 64, 128, 512])
def test_colatitudes_match_numpy_gauss_legendre(n):
    # library routine: Gauss-Legendre nodes are the roots of P_n
    x_np, _ = np.polynomial.legendre.leggauss(n)
    theta = gaussian_colatitudes(n)
    assert np.all(np.diff(theta) > 0)
    np.testing.assert_allclose(np.cos(theta), x_np[::-1], rtol=0, atol=4e-15)


@pytest.mark.parametrize("n", [64, 640])
def test_colatitudes_match_scipy_roots(n):
    x_sp, _ = scipy.special.roots_legendre(n)
    theta = gaussian_colatitudes(n)
    np.testing.assert_allclose(np.cos(theta), x_sp[::-1], rtol=0, atol=4e-15)


@pytest.mark.parametrize("n", [64, 2560])
def test_colatitudes_are_roots(n):
    theta = gaussian_colatitudes(n)
    x = np.cos(theta)
    p = scipy.special.eval_legendre(n, x)
    # |P_n| near a root is |P_n'| * |dx|; P_n' ~ n / sin(theta)^(3/2)
    slope = np.abs(scipy.special.eval_legendre(n - 1, x) - x * p) * n / np.sin(theta) ** 2
    assert np.max(np.abs(p) / slope) < 1e-14
    # symmetric about the equator
    np.testing.assert_allclose(theta + theta[::-1], math.pi, rtol=0, atol=1e-15)


def test_printed_node_counts():
    rows = [l.split(maxsplit=2) for l in open(os.path.join(GOLDEN, "node_counts.txt"))
            if l.strip() and not l.startswith("#")]
    for N, V, _ in rows:
        N, V = int(N), int(V)
        g = OGrid(N)
        assert g.nnodes == V == 4 * N * N + 36 * N


def test_row_rule():
    g = OGrid(32)
    # latitude i from the pole (1-based) holds 4 i + 16 points
    for k in range(32):
        assert g.row_size[k] == 4 * (k + 1) + 16
        assert g.row_size[63 - k] == g.row_size[k]
    assert g.row_size[0] == 20 and g.row_size[31] == 4 * 32 + 16
    # positions are unit vectors; longitudes equispaced from 0
    np.testing.assert_allclose(np.linalg.norm(g.xyz, axis=1), 1.0, atol=2e-16)
    r = 5
    lon = g.lon[g.row_off[r]:g.row_off[r + 1]]
    np.testing.assert_allclose(np.diff(lon), 2 * math.pi / g.row_size[r], rtol=1e-13)
    assert lon[0] == 0.0


def test_grid_names():
    assert parse_grid_name("O32") == 32
    assert parse_grid_name("o1280") == 1280
    for bad in ["F8", "O0", "N32", "O", "32"]:
        with pytest.raises(ValueError):
            parse_grid_name(bad)
    assert oracle.OGrid("O4").nnodes == 208
