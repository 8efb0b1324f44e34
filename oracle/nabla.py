"""Nabla operators on node-column fields (oracle; test infrastructure only).

The paper lists gradient, divergence, curl and Laplacian among the operations
the library offers (Section 2.3) without formulas; the edge-based median-dual
finite-volume form used here is:

* gradient:   G_i = (1/V_i) [ sum_{e at i} sign(i,e) 0.5 (f_a + f_b) S_e
                              - f_i C_i ],
  grad_i = (east_i . G_i, north_i . G_i).  The closure term -f_i C_i makes
  the gradient of a constant vanish on the curved surface.  Per edge the two
  terms combine exactly into d_e = 0.5 (f_b - f_a) S_e added to both G_a and
  G_b; that is how :func:`gradient` evaluates it (no cancellation of large
  offsets), while :func:`gradient_sum_form` keeps the literal sum.
* divergence: div_i = (1/V_i) sum_{e at i} sign(i,e) 0.5 (U_a + U_b) . S_e,
  with U_j = u_j east_j + v_j north_j.
* Laplacian:  lap = div(grad f).
* curl:       curl_i = (1/V_i) sum_{e at i} sign(i,e) 0.5 (U_a + U_b) . T_e with
  T_e = m_e x S_e, m_e the unit edge midpoint: the dual face conormal turned
  by a right angle about the local vertical, so the sum is the circulation of
  U around the cell, counter-clockwise seen from outside (Stokes), divided by
  the cell area -- the vertical component of the vorticity.  The paper names
  curl next to gradient and divergence (Section 2.3); this is the same
  edge-based form with the tangential instead of the normal face flux.
* adjoints: the exact transposes of gradient, divergence and curl for the plain
  Euclidean inner product over every (node, level, component) entry,
  evaluated as transposed edge scatters.
* conservation: per level, sum_i V_i div_ik and sum_i |V_i div_ik| in FP64
  (exactly rounded sums, ``math.fsum``).

Layout: fields are ``[node][level]`` (scalars) and ``[node][level][2]``
(vectors with (east, north) innermost).  Each operator is an edge loop
written with ``np.bincount`` as the scatter; levels are independent and are
processed in blocks only to bound memory.
"""

import math

import numpy as np

LEVEL_BLOCK = 16


def _blocks(L, lb=LEVEL_BLOCK):
    for k0 in range(0, L, lb):
        yield k0, min(L, k0 + lb)


def _scatter(idx, vals, nbins):
    """out[idx[e], k] += vals[e, k] for a 2-D block of values."""
    M, Lb = vals.shape
    flat = (idx[:, None] * Lb + np.arange(Lb)[None, :]).ravel()
    return np.bincount(flat, weights=vals.ravel(), minlength=nbins * Lb).reshape(nbins, Lb)


def _check_scalar(mesh, f):
    f = np.asarray(f, dtype=np.float64)
    if f.ndim != 2 or f.shape[0] != mesh.nnodes:
        raise ValueError("scalar field must be [nnodes][nlev]")
    return f


def _check_vector(mesh, uv):
    uv = np.asarray(uv, dtype=np.float64)
    if uv.ndim != 3 or uv.shape[0] != mesh.nnodes or uv.shape[2] != 2:
        raise ValueError("vector field must be [nnodes][nlev][2]")
    return uv


def gradient(mesh, geom, f):
    """grad f: [V][L] -> [V][L][2] (east, north), units of f per metre."""
    f = _check_scalar(mesh, f)
    V, L = f.shape
    a, b = mesh.edges[:, 0], mesh.edges[:, 1]
    out = np.empty((V, L, 2))
    for k0, k1 in _blocks(L):
        d = 0.5 * (f[b, k0:k1] - f[a, k0:k1])            # [E, Lb]
        G = np.empty((V, k1 - k0, 3))
        for c in range(3):
            flux = d * geom.S[:, c][:, None]
            G[:, :, c] = _scatter(a, flux, V) + _scatter(b, flux, V)
        G /= geom.V[:, None, None]
        out[:, k0:k1, 0] = np.einsum("vkc,vc->vk", G, geom.east)
        out[:, k0:k1, 1] = np.einsum("vkc,vc->vk", G, geom.north)
    return out


def gradient_sum_form(mesh, geom, f):
    """The gradient with the literal face-average sum and closure term."""
    f = _check_scalar(mesh, f)
    V, L = f.shape
    fa = f[mesh.edges[:, 0]]
    fb = f[mesh.edges[:, 1]]
    face = 0.5 * (fa + fb)                                  # [E, L]
    G = np.zeros((V, L, 3))
    for c in range(3):
        vals = mesh.sgn[:, None] * face[mesh.eid] * geom.S[mesh.eid, c][:, None]
        G[:, :, c] = _scatter(mesh.slot_node, vals, V)
        G[:, :, c] -= f * geom.C[:, c][:, None]
    G /= geom.V[:, None, None]
    return np.stack([np.einsum("vkc,vc->vk", G, geom.east),
                     np.einsum("vkc,vc->vk", G, geom.north)], axis=2)


def _to_cartesian(geom, uv, nodes=None):
    e = geom.east if nodes is None else geom.east[nodes]
    n = geom.north if nodes is None else geom.north[nodes]
    return uv[..., 0:1] * e[:, None, :] + uv[..., 1:2] * n[:, None, :]


def divergence(mesh, geom, uv):
    """div (u, v): [V][L][2] -> [V][L], per metre."""
    uv = _check_vector(mesh, uv)
    V, L, _ = uv.shape
    a, b = mesh.edges[:, 0], mesh.edges[:, 1]
    out = np.empty((V, L))
    for k0, k1 in _blocks(L):
        U = _to_cartesian(geom, uv[:, k0:k1])              # [V, Lb, 3]
        flux = 0.5 * np.einsum("ekc,ec->ek", U[a] + U[b], geom.S)
        out[:, k0:k1] = (_scatter(a, flux, V) - _scatter(b, flux, V)) / geom.V[:, None]
    return out


def face_tangents(geom):
    """T_e = m_e x S_e: [E][3]."""
    return np.cross(geom.m, geom.S)


def curl(mesh, geom, uv):
    """curl (u, v): [V][L][2] -> [V][L], per metre (vertical vorticity)."""
    uv = _check_vector(mesh, uv)
    V, L, _ = uv.shape
    a, b = mesh.edges[:, 0], mesh.edges[:, 1]
    T = face_tangents(geom)
    out = np.empty((V, L))
    for k0, k1 in _blocks(L):
        U = _to_cartesian(geom, uv[:, k0:k1])              # [V, Lb, 3]
        flux = 0.5 * np.einsum("ekc,ec->ek", U[a] + U[b], T)
        out[:, k0:k1] = (_scatter(a, flux, V) - _scatter(b, flux, V)) / geom.V[:, None]
    return out


def curl_adjoint(mesh, geom, z):
    """Transpose of :func:`curl`: [V][L] -> [V][L][2] (as the divergence
    adjoint, with T_e in place of S_e)."""
    z = _check_scalar(mesh, z)
    V, L = z.shape
    a, b = mesh.edges[:, 0], mesh.edges[:, 1]
    T = face_tangents(geom)
    out = np.empty((V, L, 2))
    for k0, k1 in _blocks(L):
        q = z[:, k0:k1] / geom.V[:, None]
        h = 0.5 * (q[a] - q[b])                              # [E, Lb]
        H = np.empty((V, k1 - k0, 3))
        for c in range(3):
            vals = h * T[:, c][:, None]
            H[:, :, c] = _scatter(a, vals, V) + _scatter(b, vals, V)
        out[:, k0:k1, 0] = np.einsum("vkc,vc->vk", H, geom.east)
        out[:, k0:k1, 1] = np.einsum("vkc,vc->vk", H, geom.north)
    return out


def laplacian(mesh, geom, f):
    """lap f = div(grad f): [V][L] -> [V][L], per square metre."""
    return divergence(mesh, geom, gradient(mesh, geom, f))


def gradient_adjoint(mesh, geom, w):
    """Transpose of :func:`gradient`: [V][L][2] -> [V][L].

    <w, grad f> = sum_e 0.5 (f_b - f_a) (W_a + W_b) . S_e with
    W_i = (wx_i east_i + wy_i north_i) / V_i, so the edge term
    g_e = 0.5 (W_a + W_b) . S_e goes to +b and -a.
    """
    w = _check_vector(mesh, w)
    V, L, _ = w.shape
    a, b = mesh.edges[:, 0], mesh.edges[:, 1]
    out = np.empty((V, L))
    for k0, k1 in _blocks(L):
        W = _to_cartesian(geom, w[:, k0:k1]) / geom.V[:, None, None]
        g = 0.5 * np.einsum("ekc,ec->ek", W[a] + W[b], geom.S)
        out[:, k0:k1] = _scatter(b, g, V) - _scatter(a, g, V)
    return out


def divergence_adjoint(mesh, geom, d):
    """Transpose of :func:`divergence`: [V][L] -> [V][L][2].

    <d, div U> = sum_e 0.5 (U_a + U_b) . S_e (q_a - q_b) with q = d / V, so
    node j receives sum_{e at j} 0.5 (q_a - q_b) S_e, projected on its basis.
    """
    d = _check_scalar(mesh, d)
    V, L = d.shape
    a, b = mesh.edges[:, 0], mesh.edges[:, 1]
    out = np.empty((V, L, 2))
    for k0, k1 in _blocks(L):
        q = d[:, k0:k1] / geom.V[:, None]
        h = 0.5 * (q[a] - q[b])                              # [E, Lb]
        H = np.empty((V, k1 - k0, 3))
        for c in range(3):
            vals = h * geom.S[:, c][:, None]
            H[:, :, c] = _scatter(a, vals, V) + _scatter(b, vals, V)
        out[:, k0:k1, 0] = np.einsum("vkc,vc->vk", H, geom.east)
        out[:, k0:k1, 1] = np.einsum("vkc,vc->vk", H, geom.north)
    return out


def conservation(mesh, geom, div):
    """Per level: (sum_i V_i div_ik, sum_i |V_i div_ik|), exactly rounded."""
    div = _check_scalar(mesh, div)
    prod = geom.V[:, None] * div
    s = np.array([math.fsum(prod[:, k]) for k in range(div.shape[1])])
    a = np.array([math.fsum(np.abs(prod[:, k])) for k in range(div.shape[1])])
    return s, a


# ---------------------------------------------------------------------------
# Sampled evaluation: the same edge scatters restricted to the edges incident
# to a set of nodes.  Used where the full grid is too large to evaluate
# everywhere; ``get`` returns field rows for an index array.


def _incident(mesh, nodes):
    nodes = np.unique(np.asarray(nodes, dtype=np.int64))
    starts = mesh.off[nodes]
    counts = mesh.off[nodes + 1] - starts
    slots = np.repeat(starts, counts) + (np.arange(counts.sum()) -
                                         np.repeat(np.cumsum(counts) - counts, counts))
    return nodes, np.unique(mesh.eid[slots])


def _local_scatter(lut, idx, vals, n):
    keep = lut[idx] >= 0
    return _scatter(lut[idx[keep]], vals[keep], n)


def _lut(mesh, nodes):
    lut = np.full(mesh.nnodes, -1, dtype=np.int64)
    lut[nodes] = np.arange(nodes.size)
    return lut


def gradient_at(mesh, geom, get, nodes):
    """gradient at the sorted unique ``nodes``: returns (nodes, [n][L][2])."""
    nodes, eids = _incident(mesh, nodes)
    lut = _lut(mesh, nodes)
    a, b = mesh.edges[eids, 0], mesh.edges[eids, 1]
    d = 0.5 * (get(b) - get(a))
    n, L = nodes.size, d.shape[1]
    G = np.empty((n, L, 3))
    for c in range(3):
        flux = d * geom.S[eids, c][:, None]
        G[:, :, c] = _local_scatter(lut, a, flux, n) + _local_scatter(lut, b, flux, n)
    G /= geom.V[nodes][:, None, None]
    out = np.stack([np.einsum("vkc,vc->vk", G, geom.east[nodes]),
                    np.einsum("vkc,vc->vk", G, geom.north[nodes])], axis=2)
    return nodes, out


def divergence_at(mesh, geom, get, nodes):
    """divergence at ``nodes``; ``get`` returns [m][L][2] rows."""
    nodes, eids = _incident(mesh, nodes)
    lut = _lut(mesh, nodes)
    a, b = mesh.edges[eids, 0], mesh.edges[eids, 1]
    Ua = _to_cartesian(geom, get(a), a)
    Ub = _to_cartesian(geom, get(b), b)
    flux = 0.5 * np.einsum("ekc,ec->ek", Ua + Ub, geom.S[eids])
    n = nodes.size
    out = (_local_scatter(lut, a, flux, n) - _local_scatter(lut, b, flux, n))
    return nodes, out / geom.V[nodes][:, None]


def curl_at(mesh, geom, get, nodes):
    """curl at ``nodes``; ``get`` returns [m][L][2] rows."""
    nodes, eids = _incident(mesh, nodes)
    lut = _lut(mesh, nodes)
    a, b = mesh.edges[eids, 0], mesh.edges[eids, 1]
    Ua = _to_cartesian(geom, get(a), a)
    Ub = _to_cartesian(geom, get(b), b)
    T = np.cross(geom.m[eids], geom.S[eids])
    flux = 0.5 * np.einsum("ekc,ec->ek", Ua + Ub, T)
    n = nodes.size
    out = (_local_scatter(lut, a, flux, n) - _local_scatter(lut, b, flux, n))
    return nodes, out / geom.V[nodes][:, None]


def laplacian_at(mesh, geom, get, nodes):
    """div(grad f) at ``nodes`` from the gradient on their one-ring."""
    nodes, eids = _incident(mesh, nodes)
    ring = np.unique(np.concatenate([nodes, mesh.edges[eids].ravel()]))
    ring, g = gradient_at(mesh, geom, get, ring)
    lut = _lut(mesh, ring)
    return divergence_at(mesh, geom, lambda idx: g[lut[idx]], nodes)


def gradient_adjoint_at(mesh, geom, get, nodes):
    nodes, eids = _incident(mesh, nodes)
    lut = _lut(mesh, nodes)
    a, b = mesh.edges[eids, 0], mesh.edges[eids, 1]
    Wa = _to_cartesian(geom, get(a), a) / geom.V[a][:, None, None]
    Wb = _to_cartesian(geom, get(b), b) / geom.V[b][:, None, None]
    g = 0.5 * np.einsum("ekc,ec->ek", Wa + Wb, geom.S[eids])
    n = nodes.size
    return nodes, _local_scatter(lut, b, g, n) - _local_scatter(lut, a, g, n)


def divergence_adjoint_at(mesh, geom, get, nodes):
    nodes, eids = _incident(mesh, nodes)
    lut = _lut(mesh, nodes)
    a, b = mesh.edges[eids, 0], mesh.edges[eids, 1]
    h = 0.5 * (get(a) / geom.V[a][:, None] - get(b) / geom.V[b][:, None])
    n, L = nodes.size, h.shape[1]
    H = np.empty((n, L, 3))
    for c in range(3):
        vals = h * geom.S[eids, c][:, None]
        H[:, :, c] = _local_scatter(lut, a, vals, n) + _local_scatter(lut, b, vals, n)
    out = np.stack([np.einsum("vkc,vc->vk", H, geom.east[nodes]),
                    np.einsum("vkc,vc->vk", H, geom.north[nodes])], axis=2)
    return nodes, out
