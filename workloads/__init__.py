"""Seeded synthetic inputs shared by the tests, the oracle and the benchmark.

This module holds no arithmetic of the Nabla method: it turns node
coordinates (handed in by the caller, from whichever mesh it built) and seeds
into field values.  The HIP library and the oracle never import each other;
both are fed arrays made here.

* Real spherical harmonics, orthonormal on the unit sphere, no Condon-Shortley
  phase: Y_l^0 = P_l0(sin lat), Y_l^m = sqrt(2) P_lm(sin lat) cos(m lon) and
  Y_l^-m = sqrt(2) P_lm(sin lat) sin(m lon) for m > 0, where P_lm are the
  fully normalised associated Legendre functions (standard forward-column
  recurrences).  Coefficients come in the order l = 0..lmax, m = -l..l from
  ``numpy.random.default_rng(seed).standard_normal``.
* Level structure, noise and tracer recipes for the five workloads
  (O32 x 10, O320 x 137, O1280 x 137, O640 x 137 adjoint, O640 batched).
  The paper measures nothing and names no dataset; these synthetic fields
  stand in for model data of the stated spectral content.
"""

import math

import numpy as np

BATCH_LEVEL_CHOICES = (1, 19, 60, 91, 137)


def sh_coefficients(lmax, seed):
    """(lmax+1)^2 N(0,1) coefficients, index l*l + (m + l)."""
    return np.random.default_rng(seed).standard_normal((lmax + 1) ** 2)


def _row_coefficients(coeffs, lmax, x, u):
    """Per-latitude Fourier coefficients A_m, B_m (m = 0..lmax).

    f(lon) = sum_m A_m cos(m lon) + B_m sin(m lon) on a latitude circle with
    sin(lat) = x, cos(lat) = u.
    """
    nx = x.size
    A = np.zeros((lmax + 1, nx))
    B = np.zeros((lmax + 1, nx))
    pmm = np.full(nx, 1.0 / math.sqrt(4.0 * math.pi))
    for m in range(lmax + 1):
        if m > 0:
            pmm = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * u * pmm
        w = 1.0 if m == 0 else math.sqrt(2.0)
        p_lm2 = None
        p_lm1 = pmm
        for l in range(m, lmax + 1):
            if l == m:
                p = pmm
            elif l == m + 1:
                p = math.sqrt(2.0 * m + 3.0) * x * pmm
            else:
                a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
                bb = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
                p = a * (x * p_lm1 - bb * p_lm2)
            if l > m:
                p_lm2, p_lm1 = p_lm1, p
            A[m] += coeffs[l * l + l + m] * w * p
            if m > 0:
                B[m] += coeffs[l * l + l - m] * w * p
    return A, B


def sh_synthesis(coeffs, lmax, lon, sinlat, coslat, chunk=1 << 21, device=None):
    """Evaluate sum c_lm Y_l^m at points given by lon, sin(lat), cos(lat).

    The per-latitude Legendre stage runs in NumPy; the per-point sum over m
    (Horner in exp(i lon)) runs in NumPy, or with torch on ``device`` when
    given (then a float64 torch tensor on that device is returned).
    """
    lon = np.asarray(lon, dtype=np.float64)
    xs, inv = np.unique(np.asarray(sinlat, dtype=np.float64), return_inverse=True)
    # one cos(lat) per distinct latitude
    us = np.zeros_like(xs)
    us[inv] = np.asarray(coslat, dtype=np.float64)
    A, B = _row_coefficients(coeffs, lmax, xs, us)
    Cm = (A - 1j * B)                       # [lmax+1, nrows]
    if device is not None:
        import torch
        Ct = torch.from_numpy(Cm).to(device)
        lt = torch.from_numpy(lon).to(device)
        it = torch.from_numpy(inv.astype(np.int64)).to(device)
        z = torch.polar(torch.ones_like(lt), lt)
        acc = Ct[lmax][it].clone()
        for m in range(lmax - 1, -1, -1):
            acc.mul_(z)
            acc.add_(Ct[m][it])
        return acc.real.contiguous()
    out = np.empty(lon.size)
    for s0 in range(0, lon.size, chunk):
        s1 = min(lon.size, s0 + chunk)
        z = np.exp(1j * lon[s0:s1])
        r = inv[s0:s1]
        acc = Cm[lmax][r].copy()
        for m in range(lmax - 1, -1, -1):
            acc *= z
            acc += Cm[m][r]
        out[s0:s1] = acc.real
    return out


def sh_field(coords, lmax, seed, device=None):
    """Seeded SH sum up to degree lmax at coords = (lon, sinlat, coslat)."""
    return sh_synthesis(sh_coefficients(lmax, seed), lmax, *coords, device=device)


def real_sh(l, m, coords):
    """A single real orthonormal harmonic Y_l^m (m may be negative)."""
    c = np.zeros((l + 1) ** 2)
    c[l * l + l + m] = 1.0
    return sh_synthesis(c, l, *coords)


# --- workload recipes -------------------------------------------------------

def scaled_levels(s, nlev, step):
    """f[i, k] = s[i] * (1 + step * k)."""
    return s[:, None] * (1.0 + step * np.arange(nlev, dtype=np.float64))[None, :]


def workload_o32(coords, nlev=10, seed=1001):
    """SH sum up to degree 10, per-level scale 1 + 0.1 k."""
    return scaled_levels(sh_field(coords, 10, seed), nlev, 0.1)


def workload_o320(coords, nlev=137, seed=1002, noise_seed=1012, sigma=1e-3):
    """SH sum up to degree 64, scale 1 + 0.1 k, plus iid N(0, sigma) noise."""
    f = scaled_levels(sh_field(coords, 64, seed), nlev, 0.1)
    f += sigma * np.random.default_rng(noise_seed).standard_normal(f.shape)
    return f


def workload_o1280(coords, nlev=137, seed=1003, lmax=256, device=None):
    """SH sum up to degree 256 plus a level-wise linear trend rms(s) k/(L-1).

    Returns (s, trend): f[i, k] = s[i] + trend[k].  With ``device`` the surface
    s is a float64 torch tensor on that device."""
    s = sh_field(coords, lmax, seed, device=device)
    rms = math.sqrt(float((s * s).mean()))
    trend = rms * np.arange(nlev, dtype=np.float64) / max(1, nlev - 1)
    return s, trend


def normal(shape, seed, sigma=1.0):
    return sigma * np.random.default_rng(seed).standard_normal(shape)


def batch_levels(ntracers=64, seed=1005):
    """Tracer level counts drawn uniformly from {1, 19, 60, 91, 137}."""
    return np.random.default_rng(seed).choice(np.array(BATCH_LEVEL_CHOICES), ntracers)


def tracer_surface(coords, t, lmax=128, base_seed=2000, device=None):
    """Surface pattern of tracer t (degree <= 128, seed base + t)."""
    return sh_field(coords, lmax, base_seed + t, device=device)


def tracer_field(s, nlev):
    """Tracer levels: s[i] * (1 + k / L_t)."""
    return scaled_levels(s, nlev, 1.0 / nlev)


def fd_entries(nnodes, nlev, count=100, seed=1034):
    """Distinct (node, level) entries drawn without replacement."""
    flat = np.random.default_rng(seed).choice(nnodes * nlev, size=count, replace=False)
    return np.stack([flat // nlev, flat % nlev], axis=1)
