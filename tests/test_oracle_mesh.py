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
