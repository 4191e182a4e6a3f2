"""Pins of the oracle's mesh quantities: Jacobians, connectivity, normals, face maps."""
import numpy as np
import pytest

import dginputs
from oracle import mesh as Mm
from oracle import refelem as R


@pytest.fixture(scope="module")
def jittered():
    v, e = dginputs.kuhn_cube(3, jitter=0.15, permute=True)
    return Mm.Mesh(v, e, R.ref_element(3))


@pytest.mark.parametrize("n", [1, 2, 4])
def test_kuhn_cube_counts_and_volume(n):
    v, e = dginputs.kuhn_cube(n)
    m = Mm.Mesh(v, e, R.ref_element(1))
    assert m.K == 6 * n ** 3
    # reference volume 4/3 times J sums to the unit cube
    assert abs(np.sum(m.J) * 4.0 / 3.0 - 1.0) < 1e-13
    nb = int(np.sum(m.boundary))
    assert nb == 12 * n * n
    assert (4 * m.K - nb) % 2 == 0


def test_jittered_volume_and_positive_jacobian(jittered):
    assert np.all(jittered.J > 0)
    assert abs(np.sum(jittered.J) * 4.0 / 3.0 - 1.0) < 1e-13


def test_connectivity_is_an_involution(jittered):
    m = jittered
    k = np.arange(m.K)[:, None].repeat(4, 1)
    f = np.arange(4)[None, :].repeat(m.K, 0)
    assert np.array_equal(m.EToE[m.EToE, m.EToF], k)
    assert np.array_equal(m.EToF[m.EToE, m.EToF], f)


def test_normals_are_outward_unit_and_opposite(jittered):
    m = jittered
    v = m.vxyz[m.etov]
    cent = v.mean(axis=1)
    for f, (a, b, c) in enumerate(R.FACE_VERTS):
        fc = (v[:, a] + v[:, b] + v[:, c]) / 3.0
        assert np.all(np.sum((fc - cent) * m.n[:, f], axis=1) > 0)
        # sJ is physical area over the area (2) of the in-face reference triangle
        area = 0.5 * np.linalg.norm(np.cross(v[:, b] - v[:, a], v[:, c] - v[:, a]), axis=1)
        assert np.max(np.abs(m.sJ[:, f] * 2.0 - area) / area) < 1e-13
    assert np.allclose(np.linalg.norm(m.n, axis=2), 1.0, atol=1e-15)
    inter = ~m.boundary
    kk, ff = np.nonzero(inter)
    assert np.max(np.abs(m.n[kk, ff] + m.n[m.EToE[kk, ff], m.EToF[kk, ff]])) < 1e-13


def test_geometric_factors_invert_the_affine_map(jittered):
    m = jittered
    v = m.vxyz[m.etov]
    A = np.stack([(v[:, 1] - v[:, 0]) / 2, (v[:, 2] - v[:, 0]) / 2, (v[:, 3] - v[:, 0]) / 2], axis=2)
    assert np.max(np.abs(np.einsum("kij,kjl->kil", m.G, A) - np.eye(3))) < 1e-12
    # the physical nodes of the reference vertices are the element vertices
    ref = m.ref
    for lv, rv in enumerate(R.REF_VERTS):
        idx = np.nonzero(np.linalg.norm(ref.rst - rv, axis=1) < 1e-14)[0][0]
        assert np.max(np.abs(m.x[:, :, idx].T - v[:, lv])) < 1e-15


def test_face_maps_match_coordinates_and_are_involutive(jittered):
    m = jittered
    Np = m.ref.Np
    flatx = m.x.reshape(3, -1)
    assert np.max(np.abs(flatx[:, m.vmapM] - flatx[:, m.vmapP])) < 1e-13
    inter = ~m.boundary
    vM, vP = m.vmapM[inter].ravel(), m.vmapP[inter].ravel()
    back = np.empty(m.K * Np, dtype=np.int64)
    back[vM] = vP
    # P(P(node)) = node on interior face nodes (a face node may sit on several faces of one
    # element, so compare coordinates of the round trip per face slot instead of ids)
    assert np.max(np.abs(flatx[:, back[vP]] - flatx[:, vM])) < 1e-13
    # boundary nodes lie on the cube walls
    bx = flatx[:, m.vmapM[m.boundary].ravel()]
    on_wall = np.min(np.stack([np.abs(bx), np.abs(bx - 1.0)]), axis=0).min(axis=0)
    assert np.max(on_wall) < 1e-14


def test_orientation_fix_and_nonconforming_error():
    v, e = dginputs.kuhn_cube(1)
    bad = e.copy()
    bad[:, [2, 3]] = bad[:, [3, 2]]
    fixed = Mm.orient(v, bad)
    vv = v[fixed]
    det = np.linalg.det(np.stack([vv[:, 1] - vv[:, 0], vv[:, 2] - vv[:, 0], vv[:, 3] - vv[:, 0]], axis=2))
    assert np.all(det > 0)
    with pytest.raises(Mm.MeshError):
        Mm.connect(np.concatenate([e, e[:1]]))
