"""Semi-discrete right-hand side of the weight-adjusted SC-PML DGTD system (oracle, FP64).

State layout: q [K, 12, N_p] with components
Ex Ey Ez Hx Hy Hz PEx PEy PEz PHx PHy PHz (user element order, library node
order).  Auxiliary fields exist only in PML elements; their rows are zero and
stay zero elsewhere (the paper stores "12 x N_p in the PML", Sec. II-A).

Curl operator with flux, eqs. (15)-(17), for eps = mu = 1 (vacuum), in the
strong nodal form obtained by applying M_k^{-1} to the curl operator C_k
(reading of the bracket in eqs. (26)-(27): C_k there stands for
M_k^{-1} C_k):

    R_E =  curl H + LIFT( Fscale * 1/2 ( -n x [H] + alpha n x (n x [E]) ) ) - J
    R_H = -curl E + LIFT( Fscale * 1/2 (  n x [E] + alpha n x (n x [H]) ) )

with jumps [u] = u^- - u^+ (interior minus exterior trace).  The paper leaves
the flux open (text after eq. (15)); alpha = 1 is the upwind flux, alpha = 0
the central flux.  A wall face with no neighbour is a perfect electric
conductor: E^+ = -E^-, H^+ = H^-.

Outside the PML the right-hand side is (R_E, R_H).  Inside, per Cartesian
component u and field f in {E, H} with auxiliary field P^f, eqs. (26)-(29):

    d/dt f_u   = - P_q a_u^{-1} V_q [ P_q ( b_u V_q f_u + c_u V_q P_u ) - R_{f,u} ]
    d/dt P_u   =   P_q ( kappa_u^{-1} V_q f_u - d_u V_q P_u )

where a_u, b_u, c_u, d_u, kappa_u are diagonal matrices of the eq. (9)
entries at the cubature points of the element.  An element belongs to the
PML when sigma or kappa differ from vacuum at any of its cubature points.

Parity: pinned by tests/test_oracle_rhs.py (energy decay with upwind flux,
energy conservation with central flux, PEC cavity eigenmode convergence,
uniform-sigma exponential decay, local PML operator, agreement with the direct
stored-mass scheme of oracle.brute).
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh
from .pml import sigma_kappa, tensors
from .refel import RefElement


def cross(a, b):
    """Cross product along axis 1 of arrays shaped [k, 3, ...]."""
    return np.stack([a[:, 1] * b[:, 2] - a[:, 2] * b[:, 1],
                     a[:, 2] * b[:, 0] - a[:, 0] * b[:, 2],
                     a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]], axis=1)


def dipole(src: dict, x: np.ndarray, t: float) -> np.ndarray:
    """Gaussian-modulated dipole current J(x, t) at points x [..., 3] -> [..., 3].

    J = amplitude * sin(2 pi f0 (t - t0)) exp(-((t - t0)/tau)^2)
        * exp(-|x - center|^2 / width^2) * direction
    """
    g = src["amplitude"] * np.sin(2.0 * np.pi * src["f0"] * (t - src["t0"])) * \
        np.exp(-((t - src["t0"]) / src["tau"]) ** 2)
    r2 = np.sum((x - np.asarray(src["center"])) ** 2, axis=-1)
    s = np.exp(-r2 / src["width"] ** 2)
    return g * s[..., None] * np.asarray(src["direction"], dtype=np.float64)


class Operator:
    """Right-hand side of eqs. (26)-(29) on a mesh with a PML profile."""

    def __init__(self, mesh: Mesh, ref: RefElement, pml: dict | None, alpha: float = 1.0,
                 source: dict | None = None, sigma_q: np.ndarray | None = None):
        self.mesh, self.ref = mesh, ref
        self.alpha = float(alpha)
        self.source = source
        K = mesh.K
        self.xq = mesh.map_points(ref.rq)  # physical cubature points [K, Nq, 3]
        if sigma_q is not None:
            sigma = np.asarray(sigma_q, dtype=np.float64)
            kappa = np.ones_like(sigma)
        elif pml is not None:
            sigma, kappa = sigma_kappa(self.xq, pml)
        else:
            sigma = np.zeros((K, ref.Nq, 3))
            kappa = np.ones_like(sigma)
        self.sigma, self.kappa = sigma, kappa
        self.is_pml = np.any(sigma != 0.0, axis=(1, 2)) | np.any(kappa != 1.0, axis=(1, 2))
        self.pml_elems = np.nonzero(self.is_pml)[0]
        a, b, c, d, kap = tensors(sigma[self.pml_elems], kappa[self.pml_elems])
        # [K_pml, Nq, 3]
        self.a, self.b, self.c, self.d, self.kap = a, b, c, d, kap

    # ---- curl operator with numerical flux (eqs. (15)-(17)) ----
    def curl_flux(self, q: np.ndarray, t: float, el: np.ndarray):
        m, ref = self.mesh, self.ref
        Np, Nfp = ref.Np, ref.Nfp
        U = q[el, 0:6]  # [k, 6, Np]
        dr = np.einsum("ij,kcj->kci", ref.Dr, U)
        ds = np.einsum("ij,kcj->kci", ref.Ds, U)
        dt = np.einsum("ij,kcj->kci", ref.Dt, U)

        def grad(axis):
            rr = (m.rx, m.ry, m.rz)[axis][el][:, None, None]
            ss = (m.sx, m.sy, m.sz)[axis][el][:, None, None]
            tt = (m.tx, m.ty, m.tz)[axis][el][:, None, None]
            return rr * dr + ss * ds + tt * dt

        gx, gy, gz = grad(0), grad(1), grad(2)  # [k, 6, Np]
        # curl of E (comps 0..2) and H (comps 3..5)
        curlE = np.stack([gy[:, 2] - gz[:, 1], gz[:, 0] - gx[:, 2], gx[:, 1] - gy[:, 0]], axis=1)
        curlH = np.stack([gy[:, 5] - gz[:, 4], gz[:, 3] - gx[:, 5], gx[:, 4] - gy[:, 3]], axis=1)

        # Traces at the 4 N_fp face nodes.
        fm = np.stack(ref.fmask)  # [4, Nfp]
        minus = U[:, :, fm]  # [k, 6, 4, Nfp]
        Q6 = q[:, 0:6].transpose(1, 0, 2).reshape(6, -1)  # [6, K*Np]
        plus = Q6[:, m.vmapP[el]].transpose(1, 0, 2, 3)  # [k, 6, 4, Nfp]
        bnd = m.boundary[el][:, None, :, None]  # PEC walls
        plusE = np.where(bnd, -minus[:, 0:3], plus[:, 0:3])
        plusH = np.where(bnd, minus[:, 3:6], plus[:, 3:6])
        dE = minus[:, 0:3] - plusE
        dH = minus[:, 3:6] - plusH
        n = m.nrm[el].transpose(0, 2, 1)[:, :, :, None]  # [k, 3, 4, 1]
        ndE = np.sum(n * dE, axis=1, keepdims=True)
        ndH = np.sum(n * dH, axis=1, keepdims=True)
        fluxE = 0.5 * (-cross(n, dH) + self.alpha * (n * ndE - dE))
        fluxH = 0.5 * (cross(n, dE) + self.alpha * (n * ndH - dH))
        Fs = m.Fscale[el][:, None, :, None]
        k = len(el)
        liftE = np.einsum("ij,kcj->kci", ref.LIFT, (Fs * fluxE).reshape(k, 3, 4 * Nfp))
        liftH = np.einsum("ij,kcj->kci", ref.LIFT, (Fs * fluxH).reshape(k, 3, 4 * Nfp))
        RE = curlH + liftE
        RH = -curlE + liftH
        if self.source is not None:
            RE = RE - dipole(self.source, m.x[el], t).transpose(0, 2, 1)
        return RE, RH

    # ---- full right-hand side, eqs. (26)-(29) ----
    def rhs(self, q: np.ndarray, t: float, el: np.ndarray | None = None) -> np.ndarray:
        """d q / dt for elements el (default: all) -> [len(el), 12, N_p]."""
        if el is None:
            el = np.arange(self.mesh.K)
        el = np.asarray(el)
        RE, RH = self.curl_flux(q, t, el)
        out = np.zeros((len(el), 12, self.ref.Np))
        out[:, 0:3] = RE
        out[:, 3:6] = RH
        # PML elements among el.
        pos = np.searchsorted(self.pml_elems, el)
        pos = np.minimum(pos, max(len(self.pml_elems) - 1, 0))
        inpml = (len(self.pml_elems) > 0) & (self.pml_elems[pos] == el) if len(self.pml_elems) else np.zeros(len(el), bool)
        if np.any(inpml):
            sel = np.nonzero(inpml)[0]
            p = pos[sel]
            ek = el[sel]
            for fld, R in ((0, RE[sel]), (3, RH[sel])):
                f = q[ek, fld:fld + 3]          # [k, 3, Np]
                P = q[ek, 6 + fld:9 + fld]      # [k, 3, Np]
                df, dP = self.pml_update(f, P, R, p)
                out[sel, fld:fld + 3] = df
                out[sel, 6 + fld:9 + fld] = dP
        return out

    def pml_update(self, f, P, R, p):
        """Eqs. (26)-(29) for one field f (E or H) on PML elements with indices p into pml_elems."""
        ref = self.ref
        Vq, Pq = ref.Vq, ref.Pq
        a = self.a[p].transpose(0, 2, 1)    # [k, 3, Nq]
        b = self.b[p].transpose(0, 2, 1)
        c = self.c[p].transpose(0, 2, 1)
        d = self.d[p].transpose(0, 2, 1)
        kap = self.kap[p].transpose(0, 2, 1)
        Vf = np.einsum("qj,kcj->kcq", Vq, f)
        VP = np.einsum("qj,kcj->kcq", Vq, P)
        inner = np.einsum("iq,kcq->kci", Pq, b * Vf + c * VP) - R
        df = -np.einsum("iq,kcq->kci", Pq, (1.0 / a) * np.einsum("qj,kcj->kcq", Vq, inner))
        dP = np.einsum("iq,kcq->kci", Pq, (1.0 / kap) * Vf - d * VP)
        return df, dP
