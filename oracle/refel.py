"""Reference tetrahedron operators for the nodal DG method (oracle, FP64).

Follows Sec. II-A: fields are expanded in Lagrange polynomials l_i on N_p
interpolation nodes (text before eq. (10)); the reference mass matrix M of
eq. (14) scaled by the element Jacobian gives M_k (text after eq. (17)); the
interpolation matrix V_q = V_I V^{-1} maps nodal values to cubature points and
P_q = M^{-1} V_q^T W (eqs. (20)-(21)).

Construction used here (deliberately plain): the polynomial space P_N is
spanned by products of Legendre polynomials P_a(r) P_b(s) P_c(t) with
a+b+c <= N.  With G the generalized Vandermonde matrix of that basis at the
nodes, the Lagrange functions evaluated at any points X are Psi(X) G^{-1}.
Mass and face-mass matrices are integrals of products of Lagrange functions,
evaluated with a collapsed Gauss-Jacobi (conical product) rule that is exact
for the polynomial degree involved.  V_q and P_q do not depend on which basis
spans P_N, so this matches eqs. (20)-(21) exactly in exact arithmetic.

Conventions fixed as data (shared with the library only through documentation):
* reference tetrahedron vertices v0=(-1,-1,-1), v1=(1,-1,-1), v2=(-1,1,-1),
  v3=(-1,-1,1); faces f0: t=-1, f1: s=-1, f2: r+s+t=-1, f3: r=-1;
* nodes: equispaced lattice r=-1+2a/N, s=-1+2b/N, t=-1+2c/N, a+b+c<=N,
  ordered with c outermost, then b, then a innermost;
* face nodes: the nodes lying on the face, in increasing node index;
* face integrals use a reference measure of total area 2 per face, so the
  physical surface Jacobian is sJ = (face area)/2.

Parity: pinned (orthonormality-free checks: exact differentiation of
monomials, mass matrix integrates monomials exactly, LIFT reproduces face
integrals, P_q V_q = I) by tests/test_oracle_refel.py.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import roots_jacobi

REF_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
# Local vertex triples of the four faces (f0: t=-1, f1: s=-1, f2: r+s+t=-1, f3: r=-1).
FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))


def n_nodes(N: int) -> int:
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_face_nodes(N: int) -> int:
    return (N + 1) * (N + 2) // 2


def equispaced_nodes(N: int) -> np.ndarray:
    """Equispaced lattice nodes [N_p, 3] in (r, s, t), c outer, b middle, a inner."""
    pts = []
    for c in range(N + 1):
        for b in range(N + 1 - c):
            for a in range(N + 1 - b - c):
                pts.append([-1.0 + 2.0 * a / N, -1.0 + 2.0 * b / N, -1.0 + 2.0 * c / N])
    return np.asarray(pts)


def face_masks(nodes: np.ndarray, tol: float = 1e-12):
    r, s, t = nodes[:, 0], nodes[:, 1], nodes[:, 2]
    conds = [np.abs(t + 1.0) < tol, np.abs(s + 1.0) < tol, np.abs(r + s + t + 1.0) < tol, np.abs(r + 1.0) < tol]
    return [np.nonzero(c)[0] for c in conds]


def _exponents(N: int):
    return [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]


def _leg(n: int, x: np.ndarray, deriv: int = 0) -> np.ndarray:
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    if deriv:
        coef = npleg.legder(coef, deriv)
    return npleg.legval(x, coef)


def psi(N: int, X: np.ndarray, d: int | None = None) -> np.ndarray:
    """Legendre-product basis [len(X), N_p] at points X; d=0,1,2 gives d/dr, d/ds, d/dt."""
    cols = []
    for (a, b, c) in _exponents(N):
        fa = _leg(a, X[:, 0], 1 if d == 0 else 0)
        fb = _leg(b, X[:, 1], 1 if d == 1 else 0)
        fc = _leg(c, X[:, 2], 1 if d == 2 else 0)
        cols.append(fa * fb * fc)
    return np.stack(cols, axis=1)


def collapsed_rule_tet(n: int):
    """Conical-product rule on the reference tet, n points per direction, exact to degree 2n-1.

    Unit simplex x = u, y = v(1-u), z = w(1-u)(1-v) with Jacobian (1-u)^2 (1-v);
    u uses Gauss-Jacobi weight (1-u)^2, v weight (1-v), w Gauss-Legendre.
    Mapped to the reference tet by (r,s,t) = -1 + 2 (x,y,z) (volume factor 8).
    """
    xu, wu = roots_jacobi(n, 2.0, 0.0)
    xv, wv = roots_jacobi(n, 1.0, 0.0)
    xw, ww = roots_jacobi(n, 0.0, 0.0)
    u, v, w = (xu + 1) / 2, (xv + 1) / 2, (xw + 1) / 2
    wu, wv, ww = wu / 8.0, wv / 4.0, ww / 2.0
    U, V, W = np.meshgrid(u, v, w, indexing="ij")
    WU, WV, WW = np.meshgrid(wu, wv, ww, indexing="ij")
    x = U
    y = V * (1 - U)
    z = W * (1 - U) * (1 - V)
    pts = -1.0 + 2.0 * np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    wts = 8.0 * (WU * WV * WW).ravel()
    return pts, wts


def collapsed_rule_tri(n: int):
    """Rule on the unit triangle {x,y>=0, x+y<=1}, exact to degree 2n-1 (area 1/2)."""
    xu, wu = roots_jacobi(n, 1.0, 0.0)
    xv, wv = roots_jacobi(n, 0.0, 0.0)
    u, v = (xu + 1) / 2, (xv + 1) / 2
    wu, wv = wu / 4.0, wv / 2.0
    U, V = np.meshgrid(u, v, indexing="ij")
    WU, WV = np.meshgrid(wu, wv, indexing="ij")
    return np.stack([U.ravel(), (V * (1 - U)).ravel()], axis=1), (WU * WV).ravel()


class RefElement:
    """All reference operators for order N and a cubature rule (rq [N_q,3], wq [N_q])."""

    def __init__(self, N: int, rq: np.ndarray | None = None, wq: np.ndarray | None = None):
        if N < 1:
            raise ValueError("N must be >= 1")
        self.N = N
        self.Np = n_nodes(N)
        self.Nfp = n_face_nodes(N)
        self.nodes = equispaced_nodes(N)
        self.fmask = face_masks(self.nodes)
        assert all(len(f) == self.Nfp for f in self.fmask)
        self.G = psi(N, self.nodes)
        self.Ginv = np.linalg.inv(self.G)
        # Lagrange derivative matrices (D_u)_{ij} = d l_j / du at node i.
        self.Dr = psi(N, self.nodes, 0) @ self.Ginv
        self.Ds = psi(N, self.nodes, 1) @ self.Ginv
        self.Dt = psi(N, self.nodes, 2) @ self.Ginv
        # Mass matrix, eq. (14) on the reference element.
        xr, wr = collapsed_rule_tet(N + 1)
        L = self.lagrange(xr)
        self.M = L.T @ (wr[:, None] * L)
        self.Minv = np.linalg.inv(self.M)
        # Face mass matrices (eq. (17) split per face) and LIFT = M^{-1} F.
        xt, wt = collapsed_rule_tri(N + 1)
        self.LIFT = np.zeros((self.Np, 4 * self.Nfp))
        self.Sface = []
        for f, (ia, ib, ic) in enumerate(FACE_VERTS):
            A, B, C = REF_VERTS[ia], REF_VERTS[ib], REF_VERTS[ic]
            X = A[None, :] + xt[:, :1] * (B - A)[None, :] + xt[:, 1:2] * (C - A)[None, :]
            Lf = self.lagrange(X)
            Sf = 4.0 * (Lf.T @ (wt[:, None] * Lf))  # reference face measure has area 2
            self.Sface.append(Sf)
            self.LIFT[:, f * self.Nfp:(f + 1) * self.Nfp] = self.Minv @ Sf[:, self.fmask[f]]
        self.Nq = 0
        if rq is not None:
            self.set_cubature(rq, wq)

    def lagrange(self, X: np.ndarray) -> np.ndarray:
        """Values of the N_p Lagrange functions at points X [n,3] -> [n, N_p]."""
        return psi(self.N, np.atleast_2d(X)) @ self.Ginv

    def set_cubature(self, rq: np.ndarray, wq: np.ndarray) -> None:
        """V_q = V_I V^{-1} (eq. (20)) and P_q = M^{-1} V_q^T W (eq. (21))."""
        self.rq = np.asarray(rq, dtype=np.float64)
        self.wq = np.asarray(wq, dtype=np.float64)
        self.Nq = len(self.wq)
        self.Vq = self.lagrange(self.rq)
        self.Pq = self.Minv @ self.Vq.T @ np.diag(self.wq)
