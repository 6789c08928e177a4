"""Element-constant PML coefficients, the paper's "EC-paved" configuration (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. III, configuration (i): sigma_u and kappa_u are constant inside each PML
element, sampled at the element's node that lies farthest beyond the PML
interface along +-u.  With a constant weight alpha the weighted mass matrix of
eq. (15) is alpha M_k, so eqs. (10)-(13) reduce to pointwise updates of the
nodal values:

    d/dt f_u = (R_u - b_u f_u - c_u P_u) / a_u
    d/dt P_u = f_u / kappa_u - d_u P_u

with a, b, c, d the eq. (9) entries at the element's constant sigma, kappa
and R the vacuum right-hand side (curl, lifted flux, source).  Elements are
classified as PML exactly as in the weight-adjusted scheme (a nonzero sigma
or kappa != 1 at a cubature point), so both schemes carry auxiliary fields on
the same elements.

Parity: pinned by tests/test_oracle_ec.py: the sampled values against the
profile at the element's vertices (the farthest node of a straight-sided
element along an axis is a vertex), the update against the weight-adjusted
operator fed with the same constants at every cubature point (exact there,
since P_q V_q = I for a rule of degree 2N), and zero conductivity against the
vacuum operator.
"""
from __future__ import annotations

import numpy as np

from .pml import profile_ratio, tensors
from .rhs import Operator


def ec_samples(x_nodes: np.ndarray, pml: dict):
    """sigma_u, kappa_u [K, 3] at the node of each element farthest beyond the interface along u.

    x_nodes [K, Np, 3]; the distance beyond the interface along u is max(0, x_u - hi_u, lo_u - x_u).
    """
    lo = np.asarray(pml["lo"], dtype=np.float64)
    hi = np.asarray(pml["hi"], dtype=np.float64)
    dist = np.maximum(0.0, np.maximum(x_nodes - hi, lo - x_nodes))  # [K, Np, 3]
    far = np.argmax(dist, axis=1)                                   # [K, 3] node index per axis
    K = x_nodes.shape[0]
    xs = np.empty((K, 3))
    for u in range(3):
        xs[:, u] = x_nodes[np.arange(K), far[:, u], u]
    # the profile of axis u depends on the u coordinate only, so column u of xs gives sigma_u
    ratio = profile_ratio(xs, pml["lo"], pml["hi"], pml["L"], pml["order"])
    sigma = np.asarray(pml["sigma_max"], dtype=np.float64) * ratio
    kappa = 1.0 + (float(pml.get("kappa_max", 1.0)) - 1.0) * ratio
    return sigma, kappa


class ECOperator(Operator):
    """Right-hand side with element-constant coefficients on the PML elements."""

    def __init__(self, mesh, ref, pml, alpha=1.0, source=None):
        super().__init__(mesh, ref, pml, alpha=alpha, source=source)
        sig, kap = ec_samples(mesh.x[self.pml_elems], pml)
        self.ec_sigma, self.ec_kappa = sig, kap
        self.ec_a, self.ec_b, self.ec_c, self.ec_d, self.ec_kap = tensors(sig, kap)  # [K_pml, 3]

    def pml_update(self, f, P, R, p):
        a = self.ec_a[p][:, :, None]
        b = self.ec_b[p][:, :, None]
        c = self.ec_c[p][:, :, None]
        d = self.ec_d[p][:, :, None]
        kap = self.ec_kap[p][:, :, None]
        df = (R - b * f - c * P) / a
        dP = f / kap - d * P
        return df, dP
