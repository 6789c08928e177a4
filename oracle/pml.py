"""SC-PML profiles and the diagonal tensors of eq. (9) (oracle, FP64).

Profiles (Sec. III, plane-wave and sphere examples): along each axis u the
attenuation is sigma_u = sigma_max * (d_u / L_u)^p and the stretch is
kappa_u = 1 + (kappa_max - 1) * (d_u / L_u)^p, where d_u >= 0 is the distance
from the interface plane into the layer (zero inside the computation domain).
Here the interface is an axis-aligned box [lo, hi]; p = 0 means a step
(ratio^0 = 1 inside the layer, 0 outside).

Tensor entries, eq. (9), normalised units eps0 = 1, with (u, v, w) the cyclic
permutations (x, y, z), (y, z, x), (z, x, y):

    a_uu = kappa_v kappa_w / kappa_u
    b_uu = (sigma_v kappa_w + sigma_w kappa_v - a_uu sigma_u) / kappa_u
    c_uu = sigma_v sigma_w - b_uu sigma_u
    d_uu = sigma_u / kappa_u
    kappa_uu = kappa_u

Parity: pinned by tests/test_oracle_pml.py against the frequency-domain
stretching of eqs. (3)-(4): for every omega,
j omega a + b + (c / kappa_u) / (j omega + d) = j omega s_v s_w / s_u.
"""
from __future__ import annotations

import numpy as np

CYCLIC = ((0, 1, 2), (1, 2, 0), (2, 0, 1))  # (u, v, w)


def profile_ratio(x: np.ndarray, lo, hi, L, p: float) -> np.ndarray:
    """(d_u / L_u)^p per axis for points x [..., 3] -> [..., 3]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    d = np.maximum(0.0, np.maximum(x - hi, lo - x))
    ratio = d / L
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(d > 0.0, ratio ** p, 0.0)
    return out


def sigma_kappa(x: np.ndarray, pml: dict):
    """sigma_u and kappa_u at points x [..., 3]; pml keys lo, hi, L, sigma_max, order, kappa_max."""
    q = profile_ratio(x, pml["lo"], pml["hi"], pml["L"], pml["order"])
    smax = np.asarray(pml["sigma_max"], dtype=np.float64)
    sigma = smax * q
    kappa = 1.0 + (float(pml.get("kappa_max", 1.0)) - 1.0) * q
    return sigma, kappa


def tensors(sigma: np.ndarray, kappa: np.ndarray):
    """Eq. (9): returns a, b, c, d, kappa, each [..., 3] (diagonal entry u in last axis)."""
    a = np.empty_like(sigma)
    b = np.empty_like(sigma)
    c = np.empty_like(sigma)
    d = np.empty_like(sigma)
    for (u, v, w) in CYCLIC:
        su, sv, sw = sigma[..., u], sigma[..., v], sigma[..., w]
        ku, kv, kw = kappa[..., u], kappa[..., v], kappa[..., w]
        a[..., u] = kv * kw / ku
        b[..., u] = (sv * kw + sw * kv - a[..., u] * su) / ku
        c[..., u] = sv * sw - b[..., u] * su
        d[..., u] = su / ku
    return a, b, c, d, kappa.copy()
