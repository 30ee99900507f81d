"""The seeded input generator: meshes of low-dip faults and concatenated batches.
(Geometry and bookkeeping only; the generator holds none of the method's arithmetic.)"""
import math

import numpy as np
import pytest

from paper_2410_17133_amd import inputs as I


def tet_volumes(xyz, tets):
    X = xyz[tets]
    return np.einsum("ij,ij->i", np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), X[:, 3] - X[:, 0]) / 6.0


def test_dip_of_45_degrees_is_rejected():
    """At exactly 45 degrees the plane passes through two box edges (zero-width cells)."""
    with pytest.raises(ValueError):
        I.make_instance(I.cube_config(8, dip_deg=45.0))


@pytest.mark.parametrize("dip", [30.0, 35.0, 44.0, 46.0, 60.0, 90.0])
def test_fault_dip_orientation_and_volume(dip):
    n = 8
    inst = I.make_instance(I.cube_config(n, dip_deg=dip))
    m = inst.mesh
    V = tet_volumes(m.xyz, m.tets)
    assert np.all(V > 0)
    assert V.sum() == pytest.approx(1.0, rel=1e-12)          # the unit cube, no gaps or overlaps
    # every interface triangle lies in one plane whose dip (angle to the horizontal) is the requested one
    X = m.xyz[m.coh[:, 3:]]
    nrm = np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    assert np.allclose(nrm, nrm[0], atol=1e-12)
    assert math.degrees(math.acos(abs(nrm[0, 2]))) == pytest.approx(dip, abs=1e-9)
    # + and - copies coincide, and the normal points from the - block to the + block
    assert np.allclose(m.xyz[m.coh[:, :3]], m.xyz[m.coh[:, 3:]])
    plus = np.zeros(m.n_nodes, bool)
    plus[m.pairs[:, 1]] = True
    on_plane = np.zeros(m.n_nodes, bool)
    on_plane[m.pairs.reshape(-1)] = True
    side = (m.xyz[m.tets].mean(1) - m.xyz[m.coh[0, 3]]) @ nrm[0]
    touching = on_plane[m.tets].any(1)
    uses_plus = plus[m.tets].any(1)
    assert touching.sum() > 0
    np.testing.assert_array_equal(uses_plus[touching], side[touching] > 0)
    # the interface covers the whole fault plane: area = 1 / sin(angle to the cube face it crosses)
    area = 0.5 * np.linalg.norm(np.cross(X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]), axis=1).sum()
    s = math.sin(math.radians(dip)) if dip >= 45 else math.cos(math.radians(dip))
    assert area == pytest.approx(1.0 / s, rel=1e-12)


def test_concatenated_batch_keeps_each_instance():
    insts = [I.make_instance(c, seed=i) for i, c in
             enumerate([I.cube_config(4), I.cube_config(6, dip_deg=35, heterogeneous=True), I.cube_config(4, 70)])]
    B = I.concat_instances(insts)
    assert list(B.node_off) == [0] + list(np.cumsum([i.n_nodes for i in insts]))
    for g, inst in enumerate(insts):
        lo, hi = B.node_off[g], B.node_off[g + 1]
        tl, th = B.tet_off[g], B.tet_off[g + 1]
        cl, ch = B.coh_off[g], B.coh_off[g + 1]
        assert np.all(B.group[lo:hi] == g)
        np.testing.assert_array_equal(B.xyz[lo:hi], inst.mesh.xyz)
        np.testing.assert_array_equal(B.tets[tl:th] - lo, inst.mesh.tets)
        np.testing.assert_array_equal(B.coh[cl:ch] - lo, inst.mesh.coh)
        np.testing.assert_array_equal(B.E[tl:th], inst.E)
        np.testing.assert_array_equal(B.source[lo:hi], inst.source)
        np.testing.assert_array_equal(B.dir_u[3 * lo:3 * hi], inst.dir_u)
        # no element reaches into another instance
        assert B.tets[tl:th].min() >= lo and B.tets[tl:th].max() < hi


def test_batched_configs_are_seeded_and_uneven():
    a, b = I.batched_configs(48), I.batched_configs(48)
    assert [c.name for c in a] == [c.name for c in b]
    ns = np.array([c.n for c in a])
    dips = np.array([c.dip_deg for c in a])
    assert np.all(ns % 2 == 0) and ns.min() >= 16 and ns.max() <= 48 and len(set(ns)) > 5
    assert dips.min() >= 30 and dips.max() <= 90 and (dips < 45).any() and (dips > 45).any()
    # penalties follow each instance's element size
    for c in a:
        assert c.params.k_n == pytest.approx(1e3 * 10e9 * c.n) and c.params.k_s == pytest.approx(0.1 * c.params.k_n)
