"""Discrete adjoint of the weight-adjusted SC-PML DGTD scheme and the gradient
of a shell-energy loss with respect to the PML conductivity (oracle, FP64).

Test infrastructure: only tests/, __graft_entry__.smoke() and bench.py's CPU
baseline use this package.

Everything here is the exact adjoint of the discrete scheme in oracle.rhs and
oracle.lserk, written in the energy inner product

    <x, y>_M = sum_k J_k sum_c x_{k,c}^T M y_{k,c}      (M_k = J_k M, all 12 components)

so that an adjoint variable is M-weighted (x_hat = M_J^{-1} x_bar).

Operator.  The right-hand side is affine in the fields, q' = L q + s(t).  Its
M-adjoint L* = M_J^{-1} L^T M_J is, per element:

* vacuum part: with the central flux M_J L is skew-symmetric and the upwind
  penalty (the alpha terms) symmetric (integration by parts is exact on affine
  elements), so the vacuum operator's adjoint is the same operator with alpha
  replaced by -alpha, negated;
* PML part (eqs. (26)-(29)): with P_q g V_q = M^{-1} M_g (eqs. (19)-(21)),
      z_u      = P_q a_u^{-1} V_q y_{f,u}                  (interior: z = y_f)
      (L* y)_f = -L_vac(-alpha) z - P_q b_u V_q z_u + P_q kappa_u^{-1} V_q y_{P,u}
      (L* y)_P = -P_q c_u V_q z_u - P_q d_u V_q y_{P,u}
  where L_vac acts on z with the neighbours' z traces.

Time stepping.  For the 2N-storage scheme res <- A_i res + dt F(q), q <- q + B_i res,
the adjoint runs the stages backwards with y <- A_{i+1} y + B_i q_hat (A_6 = 0) and
q_hat <- q_hat + dt L* y; the parameter gradient gathers dt <y, dF/dtheta>_M
at the forward stage input of stage i.

Loss.  J = sum_{n=1..nsteps} dt E_shell(q_n) with the shell energy in
cubature form, E_shell = 1/2 sum_k J_k sum_q w_q chi(x_{k,q}) sum_{c<6} (V_q q_{k,c})_q^2,
chi the indicator of the shell between an outer and an inner box.  Its
M-weighted gradient is P_q (chi V_q q_c) for the six E,H components.

Gradient with respect to sigma at the cubature points of the PML elements
(kappa held at one, a_u = 1): per node and axis a,
    dJ/dsigma_a += dt J_k w_q sum_{f,u} [ -(V_q z_u)(db_u/dsigma_a V_q f_u + dc_u/dsigma_a V_q P_u)
                                          -(V_q y_{P,u}) dd_u/dsigma_a V_q P_u ].
The profile parameters follow by the chain rule through
sigma_a = sigma_max_a (d_a / L_a)^p with the outer wall fixed and the
interface moving with L_a.

Parity: pinned by tests/test_oracle_adjoint.py (dot-product identities for
L* and for a whole step, the central-flux skew case L* = -L, finite
differences of the eq. (9) derivatives, and central finite differences of the
loss for per-node sigma and for the profile parameters).
"""
from __future__ import annotations

import copy

import numpy as np

from . import lserk
from .pml import CYCLIC, profile_ratio
from .rhs import Operator


def inner_m(op: Operator, x: np.ndarray, y: np.ndarray) -> float:
    """<x, y>_M over all elements and components."""
    return float(np.sum(op.mesh.J * np.einsum("kci,ij,kcj->k", x, op.ref.M, y)))


def tensor_derivatives(sigma: np.ndarray, kappa: np.ndarray):
    """Derivatives of the eq. (9) entries with respect to sigma_a.

    Returns db, dc, dd shaped [..., 3 (u), 3 (a)]: d b_uu / d sigma_a etc.
    (a_uu and kappa_uu do not depend on sigma).
    """
    shape = sigma.shape[:-1] + (3, 3)
    db, dc, dd = np.zeros(shape), np.zeros(shape), np.zeros(shape)
    for (u, v, w) in CYCLIC:
        su, sv, sw = sigma[..., u], sigma[..., v], sigma[..., w]
        ku, kv, kw = kappa[..., u], kappa[..., v], kappa[..., w]
        a = kv * kw / ku
        b = (sv * kw + sw * kv - a * su) / ku
        # b_u = (sigma_v kappa_w + sigma_w kappa_v - a sigma_u) / kappa_u
        db[..., u, u] = -a / ku
        db[..., u, v] = kw / ku
        db[..., u, w] = kv / ku
        # c_u = sigma_v sigma_w - b_u sigma_u
        dc[..., u, u] = -db[..., u, u] * su - b
        dc[..., u, v] = sw - db[..., u, v] * su
        dc[..., u, w] = sv - db[..., u, w] * su
        # d_u = sigma_u / kappa_u
        dd[..., u, u] = 1.0 / ku
    return db, dc, dd


def shell_indicator(x: np.ndarray, shell: dict) -> np.ndarray:
    """1 at points inside the outer box [outer_lo, outer_hi] and not strictly inside
    the inner box (inner_lo, inner_hi); x [..., 3]."""
    olo, ohi = np.asarray(shell["outer_lo"], float), np.asarray(shell["outer_hi"], float)
    ilo, ihi = np.asarray(shell["inner_lo"], float), np.asarray(shell["inner_hi"], float)
    in_outer = np.all((x >= olo) & (x <= ohi), axis=-1)
    in_inner = np.all((x > ilo) & (x < ihi), axis=-1)
    return (in_outer & ~in_inner).astype(np.float64)


class Adjoint:
    """M-adjoint of the right-hand side of an oracle Operator (kappa = 1)."""

    def __init__(self, op: Operator):
        if np.any(op.kappa != 1.0):
            raise ValueError("the adjoint is written for kappa = 1")
        self.op = op
        self.neg = copy.copy(op)  # same mesh and tensors, flux parameter negated, no source
        self.neg.alpha = -op.alpha
        self.neg.source = None
        self.all = np.arange(op.mesh.K)

    def _waa(self, y, p):
        """P_q a^{-1} V_q y for fields y [k, 3, Np] of PML elements p."""
        ref = self.op.ref
        a = self.op.a[p].transpose(0, 2, 1)
        return np.einsum("iq,kcq->kci", ref.Pq, (1.0 / a) * np.einsum("qj,kcj->kcq", ref.Vq, y))

    def z_fields(self, y: np.ndarray) -> np.ndarray:
        """z = P_q a^{-1} V_q y_f on PML elements, y_f elsewhere -> [K, 6, Np]."""
        op = self.op
        z = y[:, 0:6].copy()
        pe = op.pml_elems
        if len(pe):
            p = np.arange(len(pe))
            for f in (0, 3):
                z[pe, f:f + 3] = self._waa(y[pe, f:f + 3], p)
        return z

    def apply(self, y: np.ndarray) -> np.ndarray:
        """L* y for y [K, 12, Np]."""
        op, ref = self.op, self.op.ref
        z = self.z_fields(y)
        zq = np.zeros_like(y)
        zq[:, 0:6] = z
        RE, RH = self.neg.curl_flux(zq, 0.0, self.all)
        out = np.zeros_like(y)
        out[:, 0:3] = -RE
        out[:, 3:6] = -RH
        pe = op.pml_elems
        if len(pe):
            b = op.b.transpose(0, 2, 1)
            c = op.c.transpose(0, 2, 1)
            d = op.d.transpose(0, 2, 1)
            kap = op.kap.transpose(0, 2, 1)
            for f in (0, 3):
                VZ = np.einsum("qj,kcj->kcq", ref.Vq, z[pe, f:f + 3])
                VY = np.einsum("qj,kcj->kcq", ref.Vq, y[pe, 6 + f:9 + f])
                out[pe, f:f + 3] += np.einsum("iq,kcq->kci", ref.Pq, -b * VZ + VY / kap)
                out[pe, 6 + f:9 + f] = np.einsum("iq,kcq->kci", ref.Pq, -c * VZ - d * VY)
        return out

    def sigma_terms(self, y: np.ndarray, q: np.ndarray) -> np.ndarray:
        """<y, d(L q)/d sigma>_M per PML element, cubature node and axis -> [K_pml, Nq, 3]."""
        op, ref = self.op, self.op.ref
        pe = op.pml_elems
        out = np.zeros((len(pe), ref.Nq, 3))
        if not len(pe):
            return out
        db, dc, dd = tensor_derivatives(op.sigma[pe], op.kappa[pe])  # [k, Nq, u, a]
        z = self.z_fields(y)
        for f in (0, 3):
            VZ = np.einsum("qj,kcj->kqc", ref.Vq, z[pe, f:f + 3])          # [k, Nq, u]
            VY = np.einsum("qj,kcj->kqc", ref.Vq, y[pe, 6 + f:9 + f])
            VF = np.einsum("qj,kcj->kqc", ref.Vq, q[pe, f:f + 3])
            VP = np.einsum("qj,kcj->kqc", ref.Vq, q[pe, 6 + f:9 + f])
            out += -np.einsum("kqu,kqua->kqa", VZ * VF, db) \
                   - np.einsum("kqu,kqua->kqa", VZ * VP, dc) \
                   - np.einsum("kqu,kqua->kqa", VY * VP, dd)
        return out * (op.mesh.J[pe, None, None] * ref.wq[None, :, None])


def shell_weights(op: Operator, shell: dict) -> np.ndarray:
    """chi(x_{k,q}) [K, Nq]."""
    return shell_indicator(op.xq, shell)


def shell_energy(op: Operator, chi: np.ndarray, q: np.ndarray) -> float:
    ref = op.ref
    V = np.einsum("qj,kcj->kcq", ref.Vq, q[:, 0:6])
    return 0.5 * float(np.sum(op.mesh.J[:, None] * ref.wq[None, :] * chi * np.sum(V * V, axis=1)))


def shell_gradient(op: Operator, chi: np.ndarray, q: np.ndarray) -> np.ndarray:
    """M-weighted gradient of shell_energy: P_q (chi V_q q_c) for c < 6."""
    ref = op.ref
    g = np.zeros_like(q)
    V = np.einsum("qj,kcj->kcq", ref.Vq, q[:, 0:6])
    g[:, 0:6] = np.einsum("iq,kcq->kci", ref.Pq, chi[:, None, :] * V)
    return g


def forward_stages(op: Operator, q: np.ndarray, t: float, dt: float):
    """One LSERK4 step; returns (q_next, [stage inputs q^(0..4)])."""
    stages = []
    res = None
    q = q.copy()
    for i in range(5):
        stages.append(q.copy())
        k = op.rhs(q, t + lserk.C[i] * dt)
        res = dt * k if res is None else lserk.A[i] * res + dt * k
        q = q + lserk.B[i] * res
    return q, stages


def adjoint_step(adj: Adjoint, qhat: np.ndarray, stages, dt: float, grad: np.ndarray | None = None) -> np.ndarray:
    """Reverse one LSERK4 step: returns the adjoint at the step's start; adds the
    sigma gradient of the step into grad [K_pml, Nq, 3] when given."""
    y = np.zeros_like(qhat)
    for i in range(4, -1, -1):
        a_next = lserk.A[i + 1] if i + 1 < 5 else 0.0
        y = a_next * y + lserk.B[i] * qhat
        if grad is not None:
            grad += dt * adj.sigma_terms(y, stages[i])
        qhat = qhat + dt * adj.apply(y)
    return qhat


def loss(op: Operator, q0: np.ndarray, t0: float, dt: float, nsteps: int, shell: dict) -> float:
    """J = sum_{n=1..nsteps} dt E_shell(q_n)."""
    chi = shell_weights(op, shell)
    q, t, out = q0.copy(), t0, 0.0
    for _ in range(nsteps):
        q = lserk.step(op.rhs, q, t, dt)
        t += dt
        out += dt * shell_energy(op, chi, q)
    return out


def loss_and_gradient(op: Operator, q0: np.ndarray, t0: float, dt: float, nsteps: int, shell: dict):
    """Loss J, dJ/dsigma at the PML cubature nodes [K_pml, Nq, 3] (order of op.pml_elems),
    and the M-weighted adjoint of the initial state."""
    adj = Adjoint(op)
    chi = shell_weights(op, shell)
    q, t = q0.copy(), t0
    steps = []
    loss = 0.0
    for _ in range(nsteps):
        q_next, stages = forward_stages(op, q, t, dt)
        steps.append(stages)
        q, t = q_next, t + dt
        loss += dt * shell_energy(op, chi, q)
    grad = np.zeros((len(op.pml_elems), op.ref.Nq, 3))
    qhat = np.zeros_like(q0)
    for n in range(nsteps - 1, -1, -1):
        q_after = steps[n + 1][0] if n + 1 < nsteps else q
        qhat = qhat + dt * shell_gradient(op, chi, q_after)
        qhat = adjoint_step(adj, qhat, steps[n], dt, grad)
    return loss, grad, qhat


def profile_derivatives(xq: np.ndarray, pml: dict):
    """d sigma_a / d theta at points xq [..., 3] for theta = (sigma_max_xyz, L_xyz, p).

    The outer wall stays fixed (at hi + L and lo - L) while L moves the interface.
    Returns [..., 3 (a), 7]."""
    lo, hi = np.asarray(pml["lo"], float), np.asarray(pml["hi"], float)
    L = np.asarray(pml["L"], float)
    p = float(pml["order"])
    smax = np.asarray(pml["sigma_max"], float)
    d = np.maximum(0.0, np.maximum(xq - hi, lo - xq))
    r = d / L
    inside = d > 0.0
    out = np.zeros(xq.shape[:-1] + (3, 7))
    with np.errstate(divide="ignore", invalid="ignore"):
        rp = np.where(inside, r ** p, 0.0)
        rp1 = np.where(inside, r ** (p - 1.0), 0.0)
        lnr = np.where(inside, np.log(np.where(inside, r, 1.0)), 0.0)
    for a in range(3):
        out[..., a, a] = rp[..., a]                                                    # d/d sigma_max_a
        out[..., a, 3 + a] = smax[a] * p * rp1[..., a] * (1.0 - r[..., a]) / L[a]      # d/d L_a
        out[..., a, 6] = smax[a] * rp[..., a] * lnr[..., a]                            # d/d p
    return out


def profile_gradient(op: Operator, pml: dict, grad_sigma: np.ndarray) -> np.ndarray:
    """dJ/d(sigma_max_xyz, L_xyz, p) from dJ/dsigma at the PML nodes."""
    dsig = profile_derivatives(op.xq[op.pml_elems], pml)  # [k, Nq, 3, 7]
    return np.einsum("kqa,kqat->t", grad_sigma, dsig)


def moved_interface(pml: dict, L_new) -> dict:
    """Profile with layer thickness L_new and the outer wall kept in place."""
    out = dict(pml)
    L_old = np.asarray(pml["L"], float)
    L_new = np.asarray(L_new, float)
    out["lo"] = list(np.asarray(pml["lo"], float) + (L_new - L_old))
    out["hi"] = list(np.asarray(pml["hi"], float) - (L_new - L_old))
    out["L"] = list(L_new)
    return out


__all__ = ["Adjoint", "inner_m", "tensor_derivatives", "shell_indicator", "shell_weights", "shell_energy",
           "shell_gradient", "forward_stages", "adjoint_step", "loss", "loss_and_gradient", "profile_derivatives",
           "profile_gradient", "moved_interface", "profile_ratio"]
