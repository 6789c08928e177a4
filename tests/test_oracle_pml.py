"""Pins of the SC-PML profiles and of eq. (9) (CPU).

The tensor entries of eq. (9) are checked against the frequency-domain
coordinate stretching of eqs. (3)-(4): the auxiliary-variable system
d/dt (a f) = ... - b f - c P,  d/dt P = kappa_u^{-1} f - d P
has the frequency response j w a + b + (c / kappa_u) / (j w + d), which must
equal j w s_v s_w / s_u with s_u = kappa_u + sigma_u / (j w).
"""
import numpy as np

from oracle.pml import CYCLIC, profile_ratio, sigma_kappa, tensors


def test_tensors_match_coordinate_stretching():
    rng = np.random.default_rng(7)
    sigma = rng.uniform(0, 50, size=(200, 3))
    sigma[:40, 1:] = 0.0  # single-axis layers
    kappa = rng.uniform(1, 3, size=(200, 3))
    a, b, c, d, kap = tensors(sigma, kappa)
    for w in (0.3, 1.0, 7.5, 120.0):
        jw = 1j * w
        s = kappa + sigma / jw
        for (u, v, ww) in CYCLIC:
            lhs = jw * a[:, u] + b[:, u] + (c[:, u] / kap[:, u]) / (jw + d[:, u])
            rhs = jw * s[:, v] * s[:, ww] / s[:, u]
            scale = np.abs(jw * a[:, u]) + np.abs(b[:, u]) + np.abs(c[:, u] / kap[:, u] / (jw + d[:, u]))
            assert np.max(np.abs(lhs - rhs) / scale) < 1e-14


def test_kappa_one_special_case():
    sigma = np.array([[1.0, 2.0, 3.0]])
    a, b, c, d, kap = tensors(sigma, np.ones_like(sigma))
    assert np.allclose(a, 1.0)
    assert np.allclose(b, [[2 + 3 - 1, 3 + 1 - 2, 1 + 2 - 3]])
    assert np.allclose(c, [[2 * 3 - 4 * 1, 3 * 1 - 2 * 2, 1 * 2 - 0 * 3]])
    assert np.allclose(d, sigma)


def test_profile_shape():
    pml = {"lo": [-1.0] * 3, "hi": [1.0] * 3, "L": [0.5] * 3, "sigma_max": [30.0] * 3, "order": 3.0, "kappa_max": 2.0}
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [1.25, 0.0, 0.0], [1.5, -1.5, 0.2]])
    s, k = sigma_kappa(x, pml)
    assert np.all(s[0] == 0) and np.all(k[0] == 1)
    assert np.all(s[1] == 0)
    assert abs(s[2, 0] - 30.0 * 0.5 ** 3) < 1e-14
    assert abs(s[3, 0] - 30.0) < 1e-14 and abs(s[3, 1] - 30.0) < 1e-14 and s[3, 2] == 0
    assert abs(k[3, 0] - 2.0) < 1e-14
    # order 0 is a step
    r = profile_ratio(x, pml["lo"], pml["hi"], pml["L"], 0.0)
    assert r[0, 0] == 0 and r[2, 0] == 1.0
