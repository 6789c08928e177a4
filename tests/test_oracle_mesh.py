"""Pins of the oracle's geometry and connectivity (CPU)."""
import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.refel import FACE_VERTS, RefElement
from paper_2006_02551_amd import inputs


@pytest.fixture(scope="module", params=[(2, 0.0), (3, 0.1)])
def mesh(request, rules):
    n, pert = request.param
    vx, ev = inputs.kuhn_box(n, -1.0, 1.0, pert, seed=1)
    ref = RefElement(3, *rules(6))
    return Mesh(vx, ev, ref)


def test_volumes(mesh):
    assert np.all(mesh.J > 0)
    assert abs(np.sum(mesh.J) * 4.0 / 3.0 - 8.0) < 1e-12


def test_closed_surface_and_outward(mesh):
    # sum_f area_f n_f = 0 for a closed surface; area = 2 sJ
    s = np.einsum("kf,kfi->ki", 2.0 * mesh.sJ, mesh.nrm)
    assert np.max(np.abs(s)) < 1e-13
    assert np.allclose(np.linalg.norm(mesh.nrm, axis=2), 1.0)
    cen = mesh.v.mean(axis=1)
    for f, tri in enumerate(FACE_VERTS):
        fc = mesh.v[:, list(tri)].mean(axis=1)
        assert np.all(np.einsum("ki,ki->k", mesh.nrm[:, f], fc - cen) > 0)


def test_neighbour_maps(mesh):
    K = mesh.K
    k2 = mesh.EToE
    f2 = mesh.EToF
    back = k2[k2, f2]
    assert np.array_equal(back, np.tile(np.arange(K)[:, None], (1, 4)))
    # opposite normals on shared faces
    inner = ~mesh.boundary
    assert np.allclose(mesh.nrm[inner], -mesh.nrm[k2[inner], f2[inner]], atol=1e-13)
    # matched face node coordinates, involutive node map
    X = mesh.x.reshape(-1, 3)
    assert np.max(np.abs(X[mesh.vmapP] - X[mesh.vmapM])) < 1e-12
    flatP = mesh.vmapP.reshape(-1)
    flatM = mesh.vmapM.reshape(-1)
    pos = {int(m): i for i, m in enumerate(flatM)}  # node -> one occurrence is enough for an involution check per face
    for k in range(K):
        for f in range(4):
            if mesh.boundary[k, f]:
                continue
            kk, ff = k2[k, f], f2[k, f]
            assert set(mesh.vmapP[kk, ff]) == set(mesh.vmapM[k, f])
    assert len(pos) > 0 and len(flatP) == len(flatM)


def test_boundary_count(mesh):
    n = round((mesh.K / 6) ** (1 / 3))
    assert np.sum(mesh.boundary) == 12 * n * n


def _column(rules, N=3, n=(3, 3, 10), hi=(0.3, 0.3, 1.0), periodic=(True, True, True), perturb=0.0):
    vx, ev, vid = inputs.kuhn_grid(n, [0.0] * 3, hi, perturb, seed=2, periodic=periodic)
    ref = RefElement(N, *rules(2 * N))
    return Mesh(vx, ev, ref, vertex_id=vid), ref


def test_periodic_connectivity(rules):
    mesh, ref = _column(rules, periodic=(True, True, False), perturb=0.15)
    K = mesh.K
    back = mesh.EToE[mesh.EToE, mesh.EToF]
    assert np.array_equal(back, np.tile(np.arange(K)[:, None], (1, 4)))
    # boundary faces remain only on the two z ends: 2 x (3 x 3 squares x 2 triangles)
    assert int(mesh.boundary.sum()) == 36
    bn = mesh.nrm[mesh.boundary]
    assert np.allclose(np.abs(bn[:, 2]), 1.0)
    # matched face nodes coincide up to a whole period along x or y
    xm = mesh.x.reshape(-1, 3)[mesh.vmapM]
    xp = mesh.x.reshape(-1, 3)[mesh.vmapP]
    d = xp - xm
    per = np.array([0.3, 0.3, 0.0])
    for ax in range(3):
        r = d[..., ax] / per[ax] if per[ax] else d[..., ax]
        if per[ax]:
            assert np.max(np.abs(r - np.round(r))) < 1e-12
        else:
            assert np.max(np.abs(r)) < 1e-12
    assert np.any(np.abs(d[..., 0]) > 0.1) and np.any(np.abs(d[..., 1]) > 0.1)
    # opposite normals across every interior face, periodic ones included
    inner = ~mesh.boundary
    assert np.allclose(mesh.nrm[inner], -mesh.nrm[mesh.EToE, mesh.EToF][inner])
    with pytest.raises(ValueError):
        vx, ev, vid = inputs.kuhn_grid((3, 2, 2), [0.0] * 3, [1.0] * 3, periodic=(True, False, False))
        vid[vid == vid[1]] = vid[0]  # an identification that merges two vertices of one element
        Mesh(vx, ev, RefElement(1, *rules(2)), vertex_id=vid)


def test_periodic_plane_wave_and_conservation(rules):
    # A plane wave E_x = H_y = sin(2 pi (z - t)) in a fully periodic box travels exactly (up to the
    # discretisation error, which falls with N); with the central flux the discrete energy is conserved.
    from oracle import lserk
    from oracle.readout import energy
    from oracle.rhs import Operator
    errs = []
    for N in (2, 3):
        mesh, ref = _column(rules, N=N)
        z = mesh.x[..., 2]
        q = np.zeros((mesh.K, 12, ref.Np))
        q[:, 0] = np.sin(2 * np.pi * z)
        q[:, 4] = np.sin(2 * np.pi * z)
        op = Operator(mesh, ref, None, alpha=1.0)
        dt = 0.5 / ((N + 1) ** 2 * np.max(mesh.Fscale))
        nsteps = int(np.ceil(0.25 / dt))
        dt = 0.25 / nsteps
        for i in range(nsteps):
            q = lserk.step(op.rhs, q, i * dt, dt)
        exact = np.sin(2 * np.pi * (z - 0.25))
        errs.append(np.max(np.abs(q[:, 0] - exact)) + np.max(np.abs(q[:, 4] - exact)))
        # translation invariance: the mesh and the data repeat every cube along x and y, so does the solution
        cen = mesh.v.mean(axis=1)
        for shift in ((0.1, 0.0), (0.0, 0.1)):
            tgt = cen.copy()
            tgt[:, 0] = np.mod(tgt[:, 0] + shift[0], 0.3)
            tgt[:, 1] = np.mod(tgt[:, 1] + shift[1], 0.3)
            d = np.linalg.norm(cen[None, :, :] - tgt[:, None, :], axis=2)
            img = np.argmin(d, axis=1)
            assert np.max(d[np.arange(mesh.K), img]) < 1e-12
            assert np.max(np.abs(q[img] - q)) < 1e-12
    assert errs[0] < 5e-2 and errs[1] < errs[0] / 8, errs  # 2.2e-2 and 1.5e-3 at h = 0.1
    mesh, ref = _column(rules, N=2, perturb=0.1)
    rng = np.random.default_rng(3)
    q = np.zeros((mesh.K, 12, ref.Np))
    q[:, :6] = rng.standard_normal((mesh.K, 6, ref.Np))
    op = Operator(mesh, ref, None, alpha=0.0)
    e0 = energy(mesh, ref, q)
    dt = 0.2 / (9 * np.max(mesh.Fscale))
    for i in range(20):
        q = lserk.step(op.rhs, q, i * dt, dt)
    # LSERK4 dissipates a skew operator only at order dt^5 ... ||dt L||^6
    assert abs(energy(mesh, ref, q) - e0) < 1e-6 * e0
