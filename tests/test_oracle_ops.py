"""Pins of the oracle's dual geometry and Nabla operators.

Each check is fixed by something other than the oracle's own formulas:
an independent cell-by-cell construction on a tiny mesh, closed-form
derivatives, eigenfunctions of the Laplace-Beltrami operator, exact
invariants of the discrete scheme and algebraic identities of adjoints.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import nabla
from oracle.dual import solid_angle
from _oracle_cache import mesh_and_dual, coords

R = 6371220.0


# ---------------------------------------------------------------- geometry

@pytest.mark.parametrize("N", [1, 4, 32, 64])
def test_dual_volumes_tile_sphere(N):
    m, g = mesh_and_dual(N)
    assert np.all(g.V > 0)
    np.testing.assert_allclose(g.V.sum(), 4 * math.pi * R * R, rtol=4e-16)


@pytest.mark.parametrize("N", [4, 32])
def test_dual_normals_point_from_a_to_b(N):
    m, g = mesh_and_dual(N)
    X = m.grid.xyz
    d = X[m.edges[:, 1]] - X[m.edges[:, 0]]
    assert np.all(np.einsum("ec,ec->e", g.S, d) > 0)
    # S_e is tangent at the edge midpoint and shorter than the two arcs
    tang = np.abs(np.einsum("ec,ec->e", g.S, g.m)) / np.linalg.norm(g.S, axis=1)
    assert tang.max() < 0.2


def test_closure_is_nearly_radial():
    for N, bound in [(16, 0.05), (64, 0.015)]:
        m, g = mesh_and_dual(N)
        X = m.grid.xyz
        rad = np.einsum("vc,vc->v", g.C, X)
        tang = np.linalg.norm(g.C - rad[:, None] * X, axis=1)
        # the outward conormal integrates to (2/R) x area along the normal:
        # C_i ~ -2 V_i / R X_i  (inward-pointing closure of the sum)
        np.testing.assert_allclose(np.abs(rad) * R / (2 * g.V), 1.0, rtol=0.1)
        assert np.max(tang / np.linalg.norm(g.C, axis=1)) < bound


# ------------------------------------------- independent cell construction

def _ring_walk_operators(m, R):
    """Dense gradient, divergence and curl matrices built cell by cell.

    For every node the median cell boundary is walked counter-clockwise
    (seen from outside) through its triangles T = (i, j, k):
    arc m_ij -> c_T carries the face value of edge ij, arc c_T -> m_ik that
    of edge ik.  An arc p -> q walked counter-clockwise has outward conormal
    R * angle(p, q) * unit(q x p).  Cell areas are taken with the other
    diagonal of each quadrilateral (X_i, m_ij, c_T, m_ik) than the oracle.
    """
    X = m.grid.xyz
    V = m.nnodes
    mid = lambda i, j: (X[i] + X[j]) / np.linalg.norm(X[i] + X[j])  # noqa: E731
    G = np.zeros((V, 3, V))
    D = np.zeros((V, V, 3))
    K = np.zeros((V, V, 3))
    area = np.zeros(V)
    east = np.stack([-m.grid.sinlon, m.grid.coslon, 0 * m.grid.lon], 1)
    north = np.stack([-m.grid.sinlat * m.grid.coslon, -m.grid.sinlat * m.grid.sinlon,
                      m.grid.coslat], 1)
    for t in m.tris:
        c = X[t].sum(0)
        c /= np.linalg.norm(c)
        for r in range(3):
            i, j, k = t[r], t[(r + 1) % 3], t[(r + 2) % 3]
            mij, mik = mid(i, j), mid(i, k)
            area[i] += (solid_angle(X[i][None], mij[None], mik[None])[0] +
                        solid_angle(mij[None], c[None], mik[None])[0])
            for (p, q, nb, mf) in [(mij, c, j, mij), (c, mik, k, mik)]:
                w = np.cross(q, p)
                ang = math.atan2(np.linalg.norm(w), p @ q)
                nu = R * ang * w / np.linalg.norm(w)
                # face value 0.5 (f_i + f_nb); closure subtracts f_i nu
                G[i, :, i] += 0.5 * nu - nu
                G[i, :, nb] += 0.5 * nu
                D[i, i, :] += 0.5 * nu
                D[i, nb, :] += 0.5 * nu
                # circulation: the arc's conormal turned about its face's
                # midpoint direction
                tau = np.cross(mf, nu)
                K[i, i, :] += 0.5 * tau
                K[i, nb, :] += 0.5 * tau
    vol = R * R * area
    Gm = np.zeros((V, 2, V))
    Gm[:, 0, :] = np.einsum("vcx,vc->vx", G, east) / vol[:, None]
    Gm[:, 1, :] = np.einsum("vcx,vc->vx", G, north) / vol[:, None]
    Dm = np.zeros((V, V, 2))
    Dm[:, :, 0] = np.einsum("vxc,xc->vx", D, east) / vol[:, None]
    Dm[:, :, 1] = np.einsum("vxc,xc->vx", D, north) / vol[:, None]
    Km = np.zeros((V, V, 2))
    Km[:, :, 0] = np.einsum("vxc,xc->vx", K, east) / vol[:, None]
    Km[:, :, 1] = np.einsum("vxc,xc->vx", K, north) / vol[:, None]
    return Gm, Dm, vol, Km


@pytest.fixture(scope="module")
def o4_brute():
    m, g = mesh_and_dual(4)
    return m, g, _ring_walk_operators(m, R)


def test_o4_volumes_brute_force(o4_brute):
    m, g, (_, _, vol, _) = o4_brute
    np.testing.assert_allclose(g.V, vol, rtol=1e-13)


def test_o4_gradient_brute_force(o4_brute):
    m, g, (Gm, _, _, _) = o4_brute
    V = m.nnodes
    eye = np.eye(V)
    G = nabla.gradient(m, g, eye)                       # [V][V][2]
    scale = np.abs(Gm).max()
    np.testing.assert_allclose(G[:, :, 0], Gm[:, 0, :], rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(G[:, :, 1], Gm[:, 1, :], rtol=0, atol=1e-13 * scale)
    Gs = nabla.gradient_sum_form(m, g, eye)
    np.testing.assert_allclose(Gs, G, rtol=0, atol=1e-13 * scale)


def test_o4_divergence_brute_force(o4_brute):
    m, g, (_, Dm, _, _) = o4_brute
    V = m.nnodes
    scale = np.abs(Dm).max()
    for comp in range(2):
        uv = np.zeros((V, V, 2))
        uv[np.arange(V), np.arange(V), comp] = 1.0     # column j: unit at node j
        D = nabla.divergence(m, g, uv)                  # [V][V]
        np.testing.assert_allclose(D, Dm[:, :, comp], rtol=0, atol=1e-13 * scale)


def test_o4_adjoints_are_dense_transposes(o4_brute):
    m, g, (Gm, Dm, _, Km) = o4_brute
    V = m.nnodes
    # G as a (2V x V) matrix, rows (node, comp)
    Gmat = Gm.transpose(0, 1, 2).reshape(2 * V, V)
    w = np.zeros((V, 2 * V, 2))
    for r in range(2 * V):
        w[r // 2, r, r % 2] = 1.0
    GT = nabla.gradient_adjoint(m, g, w)                # [V][2V]
    np.testing.assert_allclose(GT, Gmat.T, rtol=0, atol=1e-13 * np.abs(Gmat).max())
    DT = nabla.divergence_adjoint(m, g, np.eye(V))      # [V][V][2]
    # (D^T e_i)_(j, c) = D[i, (j, c)]
    np.testing.assert_allclose(DT, Dm.transpose(1, 0, 2), rtol=0,
                               atol=1e-13 * np.abs(Dm).max())
    KT = nabla.curl_adjoint(m, g, np.eye(V))
    np.testing.assert_allclose(KT, Km.transpose(1, 0, 2), rtol=0, atol=1e-13 * np.abs(Km).max())


def test_o4_curl_brute_force(o4_brute):
    m, g, (_, _, _, Km) = o4_brute
    V = m.nnodes
    scale = np.abs(Km).max()
    for comp in range(2):
        uv = np.zeros((V, V, 2))
        uv[np.arange(V), np.arange(V), comp] = 1.0
        K = nabla.curl(m, g, uv)
        np.testing.assert_allclose(K, Km[:, :, comp], rtol=0, atol=1e-13 * scale)


# ------------------------------------------------------------ invariants

@pytest.mark.parametrize("N", [4, 32])
def test_gradient_of_constant_vanishes(N):
    m, g = mesh_and_dual(N)
    f = np.full((m.nnodes, 3), 7.25)
    f[:, 1] = -1e6
    assert np.abs(nabla.gradient(m, g, f)).max() == 0.0
    gs = nabla.gradient_sum_form(m, g, f)
    assert np.abs(gs).max() * R / 1e6 < 1e-12


@pytest.mark.parametrize("N", [4, 32])
def test_conservation(N):
    m, g = mesh_and_dual(N)
    uv = W.normal((m.nnodes, 5, 2), 7)
    d = nabla.divergence(m, g, uv)
    s, a = nabla.conservation(m, g, d)
    assert np.all(np.abs(s) <= 1e-14 * a)
    # div(grad const) = 0
    lap = nabla.laplacian(m, g, np.ones((m.nnodes, 1)))
    assert np.abs(lap).max() == 0.0


# ------------------------------------------------------------ closed forms

def _l2(err, vol):
    return math.sqrt(np.sum(vol * err ** 2) / np.sum(vol))


def test_gradient_closed_forms_converge():
    errs = {}
    for N in [16, 32, 64]:
        m, g = mesh_and_dual(N)
        gr = m.grid
        # f = sin(lat): grad = (0, cos(lat)/R)
        G1 = nabla.gradient(m, g, gr.sinlat[:, None])[:, 0, :]
        e1 = np.sqrt(G1[:, 0] ** 2 + (G1[:, 1] - gr.coslat / R) ** 2) * R
        # f = cos(lat) cos(lon): grad = (-sin(lon), -sin(lat) cos(lon)) / R
        f2 = gr.coslat * gr.coslon
        G2 = nabla.gradient(m, g, f2[:, None])[:, 0, :]
        e2 = np.hypot(G2[:, 0] + gr.sinlon / R, G2[:, 1] + gr.sinlat * gr.coslon / R) * R
        errs[N] = (_l2(e1, g.V), _l2(e2, g.V), e2.max())
    assert errs[16][1] < 5e-3 and errs[64][1] < 6e-4
    for a, b in [(16, 32), (32, 64)]:
        for q in range(2):
            order = math.log2(errs[a][q] / errs[b][q])
            assert order > 1.2, (a, b, q, order)
        assert math.log2(errs[a][2] / errs[b][2]) > 0.9     # L-inf first order


def _masked(m):
    """Exclude 3 rows at each pole and +-2 columns around the quadrant
    meridians (where the triangulation has its exact longitude ties)."""
    g = m.grid
    row_ok = (g.node_row >= 3) & (g.node_row < g.nrows - 3)
    q = g.row_size[g.node_row] // 4
    dist = np.minimum(g.node_j % q, q - g.node_j % q)
    return row_ok & (dist > 2)


def test_laplacian_of_spherical_harmonics_converges():
    res = {}
    for N in [32, 64, 128]:
        m, g = mesh_and_dual(N)
        co = coords(m)
        row = []
        for (l, mm) in [(4, 0), (6, 2)]:
            y = W.real_sh(l, mm, co)
            lap = nabla.laplacian(m, g, y[:, None])[:, 0]
            ex = -l * (l + 1) / R ** 2 * y
            glob = math.sqrt(np.sum(g.V * (lap - ex) ** 2) / np.sum(g.V * ex ** 2))
            k = _masked(m)
            mask = math.sqrt(np.sum(g.V[k] * (lap - ex)[k] ** 2) / np.sum(g.V[k] * ex[k] ** 2))
            row.append((glob, mask))
        res[N] = row
    for q in range(2):
        # global L2 converges (about first order, limited by the caps)
        assert res[128][q][0] < res[64][q][0] < res[32][q][0]
        # second order away from the caps and quadrant meridians
        o1 = math.log2(res[32][q][1] / res[64][q][1])
        o2 = math.log2(res[64][q][1] / res[128][q][1])
        assert o1 > 1.7 and o2 > 1.7, (q, o1, o2)
    assert res[128][0][0] < 6e-3


def _rotation_field(gr, axis):
    """Solid-body rotation U = axis x r (unit angular speed, R = radius) as
    (east, north) components: its vertical vorticity is 2 axis . r_hat."""
    rhat = np.stack([gr.coslat * gr.coslon, gr.coslat * gr.sinlon, gr.sinlat], 1)
    east = np.stack([-gr.sinlon, gr.coslon, 0 * gr.lon], 1)
    north = np.stack([-gr.sinlat * gr.coslon, -gr.sinlat * gr.sinlon, gr.coslat], 1)
    U = R * np.cross(np.asarray(axis, dtype=float)[None, :], rhat)
    uv = np.stack([np.sum(U * east, 1), np.sum(U * north, 1)], 1)[:, None, :]
    return uv, 2.0 * rhat @ np.asarray(axis, dtype=float)


def test_curl_of_solid_body_rotation_converges():
    """Rotation about the polar axis (u = R cos(lat), v = 0) and about the x
    axis: curl = 2 axis . r_hat.  Measured orders from O16 to O64: L-inf 1.0;
    L2 away from the caps and quadrant meridians 2.1 (polar axis) and 1.4-1.5
    (x axis, whose flow crosses the zipper rows)."""
    res = {}
    for N in [16, 32, 64]:
        m, g = mesh_and_dual(N)
        k = _masked(m)
        row = []
        for axis in [(0, 0, 1), (1, 0, 0)]:
            uv, ex = _rotation_field(m.grid, axis)
            z = nabla.curl(m, g, uv)[:, 0]
            err = z - ex
            row.append((math.sqrt(np.sum(g.V[k] * err[k] ** 2) / np.sum(g.V[k] * ex[k] ** 2)),
                        np.abs(err).max() / 2.0))
        res[N] = row
    for q, l2_order in [(0, 1.9), (1, 1.3)]:
        assert res[64][q][0] < 1e-3, res[64][q]
        for a, b in [(16, 32), (32, 64)]:
            assert math.log2(res[a][q][0] / res[b][q][0]) > l2_order, (q, a, b, res)
            assert math.log2(res[a][q][1] / res[b][q][1]) > 0.9, (q, a, b, res)


@pytest.mark.parametrize("N", [4, 32])
def test_curl_circulation_sums_to_zero(N):
    """Each dual face is shared by two cells with opposite orientation, so
    the area-weighted curl sums to zero over the closed sphere."""
    m, g = mesh_and_dual(N)
    uv = W.normal((m.nnodes, 4, 2), 17)
    z = nabla.curl(m, g, uv)
    prod = g.V[:, None] * z
    assert np.all(np.abs(prod.sum(0)) <= 1e-14 * np.abs(prod).sum(0))


def test_curl_of_gradient_converges_to_zero():
    """curl(grad f) of a smooth f vanishes in the limit (not exactly on the
    discrete dual): it shrinks with resolution relative to |grad f| / R."""
    res = {}
    for N in [16, 32, 64]:
        m, g = mesh_and_dual(N)
        f = W.real_sh(3, 1, coords(m))[:, None]
        gr_ = nabla.gradient(m, g, f)
        z = nabla.curl(m, g, gr_)[:, 0]
        k = _masked(m)
        res[N] = math.sqrt(np.sum(g.V[k] * z[k] ** 2) / np.sum(g.V[k])) * R / np.abs(gr_).max()
    assert res[64] < res[32] < res[16], res


def test_curl_at_equals_full_scatter():
    m, g = mesh_and_dual(16)
    uv = W.normal((m.nnodes, 3, 2), 19)
    nodes = np.array([0, 5, 17, 100, m.nnodes // 2, m.nnodes - 1])
    idx, z = nabla.curl_at(m, g, lambda i: uv[i], nodes)
    full = nabla.curl(m, g, uv)
    np.testing.assert_allclose(z, full[idx], rtol=0, atol=1e-15 * np.abs(full).max())


def test_spherical_harmonics_are_orthonormal():
    m, g = mesh_and_dual(64)
    co = coords(m)
    ys = [W.real_sh(l, mm, co) for (l, mm) in [(0, 0), (3, -2), (3, 2), (5, 1)]]
    Gram = np.array([[np.sum(g.V * a * b) / R ** 2 for b in ys] for a in ys])
    np.testing.assert_allclose(Gram, np.eye(4), atol=2e-3)


# -------------------------------------------------------------- adjoints

@pytest.mark.parametrize("N", [4, 32])
def test_dot_product_tests(N):
    m, g = mesh_and_dual(N)
    V, L = m.nnodes, 3
    x = W.normal((V, L), 11)
    y = W.normal((V, L, 2), 12)
    lhs = np.sum(nabla.gradient(m, g, x) * y)
    rhs = np.sum(x * nabla.gradient_adjoint(m, g, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    cy = nabla.curl(m, g, y)
    lhs = np.sum(cy * x)
    rhs = np.sum(y * nabla.curl_adjoint(m, g, x))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(cy) * np.linalg.norm(x)
    lhs = np.sum(nabla.divergence(m, g, y) * x)
    rhs = np.sum(y * nabla.divergence_adjoint(m, g, x))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_finite_differences_of_linear_loss():
    m, g = mesh_and_dual(8)
    V, L = m.nnodes, 4
    f = W.normal((V, L), 21)
    w = W.normal((V, L, 2), 22)
    grad_f = nabla.gradient_adjoint(m, g, w)
    for (i, k) in W.fd_entries(V, L, count=10, seed=23):
        eps = 1e-3 * max(1.0, abs(f[i, k]))
        fp, fm = f.copy(), f.copy()
        fp[i, k] += eps
        fm[i, k] -= eps
        fd = (np.sum(w * nabla.gradient(m, g, fp)) - np.sum(w * nabla.gradient(m, g, fm))) / (2 * eps)
        assert abs(fd - grad_f[i, k]) <= 1e-7 * max(1.0, abs(grad_f[i, k]))


# -------------------------------------------------------------- symmetry

def test_gradient_rotation_equivariance():
    m, g = mesh_and_dual(16)
    gr = m.grid
    shift = gr.row_size[gr.node_row] // 4
    P = gr.row_off[gr.node_row] + (gr.node_j + shift) % gr.row_size[gr.node_row]
    f = W.sh_field(coords(m), 8, 3)[:, None]
    frot = np.empty_like(f)
    frot[P] = f                                 # rotated field: value moves with its node
    G = nabla.gradient(m, g, f)
    Grot = nabla.gradient(m, g, frot)
    inner = (gr.node_row >= 3) & (gr.node_row < gr.nrows - 3)
    scale = np.abs(G).max()
    np.testing.assert_allclose(Grot[P[inner]], G[inner], rtol=0, atol=1e-12 * scale)


def test_gradient_mirror_equivariance():
    m, g = mesh_and_dual(16)
    gr = m.grid
    P = gr.row_off[gr.nrows - 1 - gr.node_row] + gr.node_j
    f = W.sh_field(coords(m), 8, 4)[:, None]
    fm = np.empty_like(f)
    fm[P] = f
    G = nabla.gradient(m, g, f)
    Gm = nabla.gradient(m, g, fm)
    far = np.abs(gr.node_row - (gr.N - 0.5)) > 3
    scale = np.abs(G).max()
    np.testing.assert_allclose(Gm[P[far], :, 0], G[far, :, 0], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(Gm[P[far], :, 1], -G[far, :, 1], rtol=0, atol=1e-12 * scale)


# -------------------------------------------------------------- sampled

def test_sampled_evaluation_matches_full():
    m, g = mesh_and_dual(16)
    V, L = m.nnodes, 3
    f = W.normal((V, L), 31)
    uv = W.normal((V, L, 2), 32)
    nodes = np.array([0, 5, 19, 20, 700, V - 1])
    get_f = lambda idx: f[idx]      # noqa: E731
    get_uv = lambda idx: uv[idx]    # noqa: E731
    n, G = nabla.gradient_at(m, g, get_f, nodes)
    np.testing.assert_allclose(G, nabla.gradient(m, g, f)[n], rtol=1e-13, atol=0)
    n, D = nabla.divergence_at(m, g, get_uv, nodes)
    np.testing.assert_allclose(D, nabla.divergence(m, g, uv)[n], rtol=1e-12, atol=1e-25)
    n, Lp = nabla.laplacian_at(m, g, get_f, nodes)
    full = nabla.laplacian(m, g, f)
    np.testing.assert_allclose(Lp, full[n], rtol=0, atol=1e-13 * np.abs(full).max())
    n, A = nabla.gradient_adjoint_at(m, g, get_uv, nodes)
    full = nabla.gradient_adjoint(m, g, uv)
    np.testing.assert_allclose(A, full[n], rtol=0, atol=1e-13 * np.abs(full).max())
    n, B = nabla.divergence_adjoint_at(m, g, get_f, nodes)
    full = nabla.divergence_adjoint(m, g, f)
    np.testing.assert_allclose(B, full[n], rtol=0, atol=1e-13 * np.abs(full).max())
