"""Seeded synthetic tetrahedral meshes (inputs only: no DG or PML arithmetic here).

A box ``[lo, hi]^3`` is cut into ``n^3`` sub-cubes and every sub-cube into six
tetrahedra that all share the cube diagonal from its (0,0,0) corner to its
(1,1,1) corner (the Kuhn / Freudenthal split).  The split is the same in every
cube, so neighbouring cubes meet in matching triangles and the mesh is
conforming.  Optionally every vertex that is not on the outer boundary is moved
by a uniform random offset of at most ``perturb * h`` per coordinate, drawn from
``numpy.random.default_rng(seed)``, so that element faces no longer line up with
an absorbing-layer interface.

Vertex order inside every tetrahedron is chosen so that
``det[v1-v0, v2-v0, v3-v0] > 0`` (positive orientation).

``kuhn_grid`` does the same for a box with its own number of cubes per axis and
can return a periodic vertex identification: along a periodic axis the vertices
of the upper face are identified with those of the lower face (the split is
translation invariant, so the two faces carry the same triangles).
"""
from __future__ import annotations

import itertools

import numpy as np

# The six Kuhn simplices of the unit cube: a path 000 -> e_a -> e_a+e_b -> 111
# for every permutation (a, b, c) of the three axes.
_PERMS = list(itertools.permutations(range(3)))


def kuhn_grid(n, lo, hi, perturb: float = 0.0, seed: int = 0, periodic=(False, False, False)):
    """Return ``(vxyz, etov, vertex_id)`` for an ``nx ny nz x 6`` tetrahedral mesh of the box ``[lo, hi]``.

    n, lo, hi : three cube counts and the box corners.
    perturb : maximum displacement of the vertices off the box surface, as a fraction of each axis' cube
              edge (per coordinate, uniform, ``default_rng(seed)``).
    periodic : per axis; the vertex identification ``vertex_id [nv]`` maps every vertex to the vertex it
              stands for (itself, or its image on the lower face of a periodic axis).  A periodic axis needs
              at least 3 cubes (with 2, a triangle across the diagonal of two periodic axes would be identified
              with a different triangle).
    """
    n = [int(x) for x in n]
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if min(n) < 1:
        raise ValueError("every cube count must be >= 1")
    if any(p and m < 3 for p, m in zip(periodic, n)):
        raise ValueError("a periodic axis needs at least 3 cubes")
    h = (hi - lo) / np.asarray(n)
    ii, jj, kk = np.meshgrid(np.arange(n[0] + 1), np.arange(n[1] + 1), np.arange(n[2] + 1), indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    vxyz = lo + h * ijk.astype(np.float64)

    def vid(i, j, k):
        return (i * (n[1] + 1) + j) * (n[2] + 1) + k

    tets = []
    for i in range(n[0]):
        for j in range(n[1]):
            for k in range(n[2]):
                base = np.array([i, j, k])
                for p in _PERMS:
                    c = base.copy()
                    path = [vid(*c)]
                    for ax in p:
                        c = c.copy()
                        c[ax] += 1
                        path.append(vid(*c))
                    tets.append(path)
    etov = np.asarray(tets, dtype=np.int64)

    if perturb > 0.0:
        rng = np.random.default_rng(seed)
        interior = np.all((ijk > 0) & (ijk < np.asarray(n)), axis=1)
        disp = rng.uniform(-perturb, perturb, size=vxyz.shape) * h
        vxyz = vxyz + disp * interior[:, None]

    img = ijk.copy()
    for ax in range(3):
        if periodic[ax]:
            img[img[:, ax] == n[ax], ax] = 0
    vertex_id = vid(img[:, 0], img[:, 1], img[:, 2]).astype(np.int32)
    etov = orient_positive(vxyz, etov)
    return vxyz, etov.astype(np.int32), vertex_id


def kuhn_box(n: int, lo: float = -1.0, hi: float = 1.0, perturb: float = 0.0, seed: int = 0):
    """Return ``(vxyz, etov)`` for an ``n^3 x 6`` tetrahedral mesh of ``[lo, hi]^3``.

    vxyz : float64 array ``[(n+1)^3, 3]`` of vertex coordinates.
    etov : int32 array ``[6 n^3, 4]`` of vertex indices per tetrahedron,
           positively oriented.
    perturb : maximum interior-vertex displacement as a fraction of the
           cube edge ``h = (hi - lo) / n`` (0 gives the regular mesh).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = (hi - lo) / n
    g = np.arange(n + 1)
    ii, jj, kk = np.meshgrid(g, g, g, indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    vxyz = lo + h * ijk.astype(np.float64)

    def vid(i, j, k):
        return (i * (n + 1) + j) * (n + 1) + k

    tets = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                base = np.array([i, j, k])
                for p in _PERMS:
                    c = base.copy()
                    path = [vid(*c)]
                    for ax in p:
                        c = c.copy()
                        c[ax] += 1
                        path.append(vid(*c))
                    tets.append(path)
    etov = np.asarray(tets, dtype=np.int64)

    if perturb > 0.0:
        rng = np.random.default_rng(seed)
        interior = np.all((ijk > 0) & (ijk < n), axis=1)
        disp = rng.uniform(-perturb * h, perturb * h, size=vxyz.shape)
        vxyz = vxyz + disp * interior[:, None]

    etov = orient_positive(vxyz, etov)
    return vxyz, etov.astype(np.int32)


def orient_positive(vxyz: np.ndarray, etov: np.ndarray) -> np.ndarray:
    """Swap the last two vertices of every negatively oriented tetrahedron."""
    etov = np.array(etov, dtype=np.int64, copy=True)
    v = vxyz[etov]
    det = np.einsum("ki,ki->k", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))
    neg = det < 0
    etov[neg, 2], etov[neg, 3] = etov[neg, 3].copy(), etov[neg, 2].copy()
    return etov
