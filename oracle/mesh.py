"""Affine tetrahedral geometry and face connectivity (oracle, FP64).

Sec. II-A, text after eq. (17): for straight-sided (linear) elements the local
mass matrix is the reference one scaled by the constant Jacobian J_k, and the
curl operator of eqs. (15)-(17) couples element k only to its face
neighbours k'.

Construction used here:
* the affine map is x = v0 + [v1-v0, v2-v0, v3-v0] (r+1, s+1, t+1)/2, so the
  Jacobian matrix columns are (v_i - v0)/2 and J_k = det of that matrix
  (= volume / (4/3));
* metric terms (r_x ... t_z) are the rows of the inverse Jacobian matrix;
* the outward unit normal of a face is the normalised cross product of two
  physical face edges, flipped to point away from the opposite vertex; the
  surface Jacobian is sJ = (face area)/2 and Fscale = sJ / J_k;
* faces are matched through their sorted global vertex triples; face nodes
  are matched by physical coordinates relative to the face centroid; a face
  with no partner is a perfect electric conductor (PEC) wall;
* periodic meshes: an optional vertex identification vertex_id [nv] names, for
  every vertex, the vertex it stands for; faces are matched on identified
  triples, so a face on the upper side of a periodic box meets its image on
  the lower side (its nodes differ by the period, which the centroid-relative
  node matching ignores).

Negatively oriented input tetrahedra have their last two vertices swapped.

Parity: pinned by tests/test_oracle_mesh.py (volumes, closed-surface normal
sums, involutive neighbour maps, matched node coordinates).
"""
from __future__ import annotations

import numpy as np

from .refel import FACE_VERTS, RefElement

OPPOSITE = (3, 2, 0, 1)  # local vertex not on face f


class Mesh:
    def __init__(self, vxyz: np.ndarray, etov: np.ndarray, ref: RefElement, vertex_id=None):
        vxyz = np.asarray(vxyz, dtype=np.float64)
        etov = np.array(etov, dtype=np.int64, copy=True)
        self.vertex_id = np.arange(len(vxyz)) if vertex_id is None else np.asarray(vertex_id, dtype=np.int64)
        K = etov.shape[0]
        if K == 0:
            raise ValueError("empty mesh")
        v = vxyz[etov]
        det6 = np.einsum("ki,ki->k", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))
        neg = det6 < 0
        etov[neg, 2], etov[neg, 3] = etov[neg, 3].copy(), etov[neg, 2].copy()
        self.etov = etov
        self.vxyz = vxyz
        self.K = K
        self.ref = ref
        v = vxyz[etov]  # [K, 4, 3]
        self.v = v

        # Jacobian matrix columns x_r, x_s, x_t.
        Jm = np.stack([(v[:, 1] - v[:, 0]) / 2, (v[:, 2] - v[:, 0]) / 2, (v[:, 3] - v[:, 0]) / 2], axis=2)
        self.Jm = Jm
        self.J = np.linalg.det(Jm)
        if np.any(self.J <= 0):
            raise ValueError("degenerate tetrahedron")
        self.Jinv = np.linalg.inv(Jm)  # rows: grad r, grad s, grad t
        self.rx, self.ry, self.rz = self.Jinv[:, 0, 0], self.Jinv[:, 0, 1], self.Jinv[:, 0, 2]
        self.sx, self.sy, self.sz = self.Jinv[:, 1, 0], self.Jinv[:, 1, 1], self.Jinv[:, 1, 2]
        self.tx, self.ty, self.tz = self.Jinv[:, 2, 0], self.Jinv[:, 2, 1], self.Jinv[:, 2, 2]

        # Physical node coordinates [K, N_p, 3].
        self.x = self.map_points(ref.nodes)

        # Faces: outward unit normals and surface Jacobians.
        self.nrm = np.zeros((K, 4, 3))
        self.sJ = np.zeros((K, 4))
        for f, (a, b, c) in enumerate(FACE_VERTS):
            e1 = v[:, b] - v[:, a]
            e2 = v[:, c] - v[:, a]
            cr = np.cross(e1, e2)
            area = 0.5 * np.linalg.norm(cr, axis=1)
            n = cr / (2.0 * area[:, None])
            away = v[:, a] - v[:, OPPOSITE[f]]
            sign = np.sign(np.einsum("ki,ki->k", n, away))
            self.nrm[:, f] = n * sign[:, None]
            self.sJ[:, f] = area / 2.0
        self.Fscale = self.sJ / self.J[:, None]

        self._connect()

    def map_points(self, rst: np.ndarray) -> np.ndarray:
        """Physical coordinates [K, n, 3] of reference points rst [n, 3]."""
        return self.v[:, None, 0, :] + np.einsum("kij,nj->kni", self.Jm, np.asarray(rst) + 1.0)

    def _connect(self):
        K, ref = self.K, self.ref
        Nfp = ref.Nfp
        faces = {}
        self.EToE = np.tile(np.arange(K)[:, None], (1, 4))
        self.EToF = np.tile(np.arange(4)[None, :], (K, 1))
        ids = self.vertex_id[self.etov]
        if np.any([len(set(row)) < 4 for row in ids]):
            raise ValueError("the vertex identification collapses an element")
        for k in range(K):
            for f, tri in enumerate(FACE_VERTS):
                key = tuple(sorted(ids[k, list(tri)]))
                faces.setdefault(key, []).append((k, f))
        for key, lst in faces.items():
            if len(lst) > 2:
                raise ValueError("non-manifold face")
            if len(lst) == 2:
                (k1, f1), (k2, f2) = lst
                self.EToE[k1, f1], self.EToF[k1, f1] = k2, f2
                self.EToE[k2, f2], self.EToF[k2, f2] = k1, f1
        self.boundary = self.EToE == np.arange(K)[:, None]

        # vmapM / vmapP as flat (k * N_p + node) indices, shape [K, 4, N_fp].
        Np = ref.Np
        fm = np.stack(ref.fmask)  # [4, Nfp]
        self.vmapM = np.arange(K)[:, None, None] * Np + fm[None, :, :]
        self.vmapP = self.vmapM.copy()
        hmin = np.min(self.sJ) ** 0.5
        tol = 1e-8 * hmin
        for k in range(K):
            for f in range(4):
                if self.boundary[k, f]:
                    continue
                k2, f2 = self.EToE[k, f], self.EToF[k, f]
                xm = self.x[k, fm[f]]
                xp = self.x[k2, fm[f2]]
                xm = xm - xm.mean(axis=0)
                xp = xp - xp.mean(axis=0)
                d = np.linalg.norm(xm[:, None, :] - xp[None, :, :], axis=2)
                idx = np.argmin(d, axis=1)
                if np.max(d[np.arange(Nfp), idx]) > tol:
                    raise ValueError("face nodes do not match")
                self.vmapP[k, f] = k2 * Np + fm[f2][idx]
