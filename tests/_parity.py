"""Parity bars shared by the GPU tests.

Every comparison of a GPU result a with the oracle's b asserts two bars:

* normwise:     ||a - b||_2 / ||b||_2 <= tol
* element-wise: max |a - b| <= tol * max |b|

and, where asked, the element-wise bar again
* per level (axis 1 of a [node][level](, 2) array: each level's largest error
  against that level's largest value), and
* per group of nodes (polar rows, nodes of degree 5 and 7, ...), each group's
  largest error against the group's own largest value,
so that a local error on a few special nodes cannot hide under the norm of
the whole field.
"""
import numpy as np


def special_groups(m, idx=None):
    """Node groups of an oracle mesh where the stencil is not the regular
    one: the two rows next to each pole (ladder caps, explicit pole edges)
    and the nodes of degree 5 or 7.  With idx (sampled node indices), the
    positions within idx of the group members."""
    g = m.grid
    polar = np.concatenate([np.arange(g.row_off[0], g.row_off[min(2, g.nrows)]),
                            np.arange(g.row_off[max(g.nrows - 2, 0)], g.row_off[g.nrows])])
    odd = np.nonzero(m.degree != 6)[0]
    groups = {"polar rows": np.unique(polar), "degree 5/7": odd}
    if idx is not None:
        idx = np.asarray(idx)
        groups = {k: np.nonzero(np.isin(idx, v))[0] for k, v in groups.items()}
    return {k: v for k, v in groups.items() if v.size}


def errors(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.abs(a - b)
    return (float(np.linalg.norm(a - b) / np.linalg.norm(b)), float(d.max() / np.abs(b).max()))


def check(a, b, tol, what="", per_level=False, groups=None):
    """Asserts the normwise and element-wise bars (see the module docstring);
    returns (normwise, element-wise) relative errors of the whole array."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    assert np.all(np.isfinite(a)), (what, "non-finite GPU values")
    l2, mx = errors(a, b)
    assert l2 <= tol, (what, "normwise", l2, tol)
    assert mx <= tol, (what, "element-wise", mx, tol)
    d = np.abs(a - b)
    if per_level and a.ndim >= 2:
        ax = tuple(i for i in range(a.ndim) if i != 1)
        err_k = d.max(axis=ax)
        ref_k = np.abs(b).max(axis=ax)
        bad = np.nonzero(err_k > tol * ref_k)[0]
        assert bad.size == 0, (what, "per level", bad[:8].tolist(), (err_k[bad] / ref_k[bad])[:8].tolist())
    for name, rows in (groups or {}).items():
        e = float(d[rows].max())
        r = float(np.abs(b[rows]).max())
        assert e <= tol * r, (what, name, e / r if r else e, tol)
    return l2, mx
