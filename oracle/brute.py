"""Direct stored-mass-matrix scheme, eqs. (10)-(15) (oracle, FP64).

This is the paper's "SV-paved" implementation (Sec. I, Sec. II-A before
eq. (18), Table I): every PML element stores, per Cartesian component u, the
five weighted mass matrices of eq. (15),

    M_k^{alpha,u}(i, j) = int_{Omega_k} alpha_uu(x) l_i l_j dx,  alpha in {a, b, c, d, 1/kappa},

and advances

    d/dt f_u = (M_k^{a,u})^{-1} [ M_k R_{f,u} - M_k^{b,u} f_u - M_k^{c,u} P_u ]
    d/dt P_u = M_k^{-1} ( M_k^{1/kappa,u} f_u - M_k^{d,u} P_u )

(eqs. (10)-(13) with the strong-form reading of the curl operator).  The
integrals use a conical-product rule of high degree on the exact profile; the
matrices are solved densely per element.  It differs from eqs. (26)-(29) only
through the weight-adjusted approximation of eq. (18) and the cubature of
eq. (19), which is what the tests measure.

Parity: this is itself a definition (the exact-mass scheme); it is pinned by
the same curl-operator tests as oracle.rhs and by its agreement with the WAA
scheme where the WAA is exact (element-constant weights, polynomial profiles
of low degree).
"""
from __future__ import annotations

import numpy as np

from .pml import sigma_kappa, tensors
from .refel import collapsed_rule_tet
from .rhs import Operator


class BruteOperator(Operator):
    """rule: optional (rst [nr, 3], w [nr]) on the reference tetrahedron for the weighted mass matrices
    (an input like the cubature rule of the weight-adjusted scheme; default: the conical product rule with
    quad_points points per direction).  elements: optional subset of element indices; the stored matrices
    are then formed for the PML elements of that subset only, and rhs(..., el) accepts only elements
    whose PML terms are stored."""

    def __init__(self, mesh, ref, pml, alpha=1.0, source=None, quad_points: int = 9, elements=None, rule=None):
        super().__init__(mesh, ref, pml, alpha=alpha, source=source)
        if rule is None:
            xr, wr = collapsed_rule_tet(quad_points)
        else:
            xr, wr = np.asarray(rule[0], dtype=np.float64), np.asarray(rule[1], dtype=np.float64)
        L = ref.lagrange(xr)  # [nr, Np]
        pe = self.pml_elems if elements is None else np.intersect1d(self.pml_elems, np.asarray(elements))
        self.brute_index = np.full(len(self.pml_elems), -1)
        self.brute_index[np.searchsorted(self.pml_elems, pe)] = np.arange(len(pe))
        xp = mesh.v[pe][:, None, 0, :] + np.einsum("kij,nj->kni", mesh.Jm[pe], xr + 1.0)  # [Kp, nr, 3]
        sigma, kappa = sigma_kappa(xp, pml)
        a, b, c, d, kap = tensors(sigma, kappa)
        J = mesh.J[pe]

        def mass(alpha):  # alpha [Kp, nr, 3] -> [Kp, 3, Np, Np]
            return J[:, None, None, None] * np.einsum("qi,kqu,q,qj->kuij", L, alpha, wr, L)

        self.Ma = mass(a)
        self.Mb = mass(b)
        self.Mc = mass(c)
        self.Md = mass(d)
        self.Mik = mass(1.0 / kap)
        self.Mk = J[:, None, None] * ref.M[None]

    def pml_update(self, f, P, R, p):
        p = self.brute_index[p]
        if np.any(p < 0):
            raise ValueError("the stored matrices of these PML elements were not formed")
        Mk = self.Mk[p][:, None]  # [k, 1, Np, Np]
        rhs_f = np.einsum("kuij,kuj->kui", np.broadcast_to(Mk, self.Ma[p].shape), R) \
            - np.einsum("kuij,kuj->kui", self.Mb[p], f) - np.einsum("kuij,kuj->kui", self.Mc[p], P)
        df = np.linalg.solve(self.Ma[p], rhs_f[..., None])[..., 0]
        rhs_P = np.einsum("kuij,kuj->kui", self.Mik[p], f) - np.einsum("kuij,kuj->kui", self.Md[p], P)
        dP = np.linalg.solve(np.broadcast_to(Mk, self.Ma[p].shape), rhs_P[..., None])[..., 0]
        return df, dP
