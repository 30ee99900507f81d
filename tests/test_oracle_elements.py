"""Pins of the oracle's element routines and return map against facts fixed by
the mathematics: closed forms on the unit right tetrahedron, continuum energy
identities computed through an independent (tensor, not Voigt) route, null
spaces, an independent quadrature rule, and textbook friction responses.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

UNIT = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)


def random_tet(seed):
    r = np.random.default_rng(seed)
    while True:
        X = r.uniform(-1, 1, (4, 3))
        v = np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)) / 6
        if abs(v) > 0.05:
            return X


def test_unit_tet_gradients():
    V, g = O.tet_grad(UNIT)
    assert V == pytest.approx(1 / 6, abs=1e-15)
    np.testing.assert_allclose(g, [[-1, -1, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]], atol=1e-15)


def test_unit_tet_stiffness_hand_values():
    # nu = 0: lambda = 0, G = E/2; entries derived by hand from eps:C:eps
    K = O.tet_stiffness(UNIT, 1.0, 0.0)
    assert K[0, 0] == pytest.approx(1 / 3)      # g0x^2 (2G) + G (g0y^2 + g0z^2) = 2, times V
    assert K[0, 3] == pytest.approx(-1 / 6)     # node0 x / node1 x
    assert K[0, 4] == pytest.approx(-1 / 12)    # node0 x / node1 y: G g0y g1x V
    assert K[3, 3] == pytest.approx(1 / 6)      # node1 x / node1 x: 2G * 1 * V
    assert K[4, 4] == pytest.approx(1 / 12)     # node1 y / node1 y: G * 1 * V
    assert K[3, 7] == pytest.approx(0.0, abs=1e-15)


def _energy_tensor(Hgrad, E, nu, V):
    eps = 0.5 * (Hgrad + Hgrad.T)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))
    sig = lam * np.trace(eps) * np.eye(3) + 2 * G * eps
    return 0.5 * V * np.sum(sig * eps)


@pytest.mark.parametrize("seed", range(5))
def test_stiffness_energy_linear_field(seed):
    X = random_tet(seed)
    E, nu = 7.3e9, 0.27
    K = O.tet_stiffness(X, E, nu)
    H = np.random.default_rng(100 + seed).standard_normal((3, 3))
    u = (X @ H.T).reshape(-1)                   # u(x) = H x at the nodes
    V = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1))) / 6
    assert 0.5 * u @ K @ u == pytest.approx(_energy_tensor(H, E, nu, V), rel=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_stiffness_null_space_and_rank(seed):
    X = random_tet(seed)
    K = O.tet_stiffness(X, 3e9, 0.3)
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-6 * np.abs(K).max())
    modes = []
    for c in range(3):
        t = np.zeros((4, 3))
        t[:, c] = 1
        modes.append(t.reshape(-1))
    for W in ([[0, -1, 0], [1, 0, 0], [0, 0, 0]], [[0, 0, 1], [0, 0, 0], [-1, 0, 0]], [[0, 0, 0], [0, 0, -1], [0, 1, 0]]):
        modes.append((X @ np.array(W, float).T).reshape(-1))
    for m in modes:
        assert np.abs(K @ m).max() <= 1e-9 * np.abs(K).max() * np.abs(m).max()
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev > 1e-9 * ev.max()) == 6
    assert ev.min() > -1e-9 * ev.max()


@pytest.mark.parametrize("seed", range(3))
def test_coupling_is_divergence(seed):
    # u^T A_e p = alpha * int div(u) p, for linear u and linear p
    X = random_tet(seed)
    A = O.tet_coupling(X, 0.8)
    r = np.random.default_rng(seed)
    H = r.standard_normal((3, 3))
    c0, gp = r.standard_normal(), r.standard_normal(3)
    u = (X @ H.T).reshape(-1)
    p = c0 + X @ gp
    V = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1))) / 6
    int_p = V * (c0 + X.mean(0) @ gp)           # linear p: integral = V * value at centroid
    assert u @ A @ p == pytest.approx(0.8 * np.trace(H) * int_p, rel=1e-12)


# degree-2 four-point rule on the tetrahedron (exact for quadratics)
_A, _B = 0.5854101966249685, 0.1381966011250105


def test_flow_element_against_independent_quadrature():
    X = random_tet(7)
    V = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1))) / 6
    S, Cm = O.tet_flow(X, 2.5, 1 / 3.0)
    r = np.random.default_rng(1)
    c0, gp = r.standard_normal(), r.standard_normal(3)
    p = c0 + X @ gp
    # conductivity: (k/mu) int |grad p|^2
    assert p @ Cm @ p == pytest.approx(2.5 * V * gp @ gp, rel=1e-12)
    assert np.abs(Cm @ np.ones(4)).max() < 1e-12 * np.abs(Cm).max()
    # storage: (1/M) int p^2 by a quadrature rule that does not use the mass formula
    pts = []
    for k in range(4):
        bary = np.full(4, _B)
        bary[k] = _A
        pts.append(bary @ X)
    quad = sum(V / 4 * (c0 + q @ gp) ** 2 for q in pts)
    assert p @ S @ p == pytest.approx(quad / 3.0, rel=1e-12)
    assert np.ones(4) @ S @ np.ones(4) == pytest.approx(V / 3.0, rel=1e-13)


def test_triangle_geometry_and_flow():
    from paper_2410_17133_amd.inputs import Params
    X = np.array([[0.5, 0.0, 0.0], [0.5, 2.0, 0.0], [0.5, 2.0, 1.0]])  # normal +x, area 1
    A, n, t1, t2, gG = O.tri_geom(X)
    assert A == pytest.approx(1.0)
    np.testing.assert_allclose(n, [1, 0, 0], atol=1e-15)
    np.testing.assert_allclose(t1, [0, 0, 1], atol=1e-15)
    np.testing.assert_allclose(t2, np.cross(n, t1), atol=1e-15)
    prm = Params(k_par=3e-12, k_perp=5e-12, w0=2e-3, M_F=0.4e6, mu=1e-3)
    S, Cm = O.tri_flow(X, prm)
    one = np.ones(6)
    # both lips at unit pressure: <p> = 1, [[p]] = 0
    assert one @ S @ one == pytest.approx(prm.w0 / prm.M_F * A, rel=1e-13)
    assert np.abs(Cm @ one).max() < 1e-9 * np.abs(Cm).max()
    # unit jump: <p> = 1/2 and [[p]] = 1
    j = np.r_[np.ones(3), np.zeros(3)]
    assert j @ S @ j == pytest.approx(prm.w0 / prm.M_F * A / 4, rel=1e-13)
    assert j @ Cm @ j == pytest.approx(prm.k_perp / (prm.mu * prm.w0) * A, rel=1e-13)
    # linear in-plane pressure on both lips: longitudinal term only
    gp = np.array([0.0, 0.7, -1.3])
    pl = np.r_[X @ gp, X @ gp]
    assert pl @ Cm @ pl == pytest.approx(prm.w0 * prm.k_par / prm.mu * A * gp @ gp, rel=1e-12)


def test_dipping_triangle_tangent():
    c = 1 / math.tan(math.radians(60))
    X = np.array([[0.0, 0.0, 0.0], [0.0, 1.0, 0.0], [c, 1.0, 1.0]])
    A, n, t1, t2, _ = O.tri_geom(X)
    assert abs(n @ t1) < 1e-15 and t1[2] > 0 and abs(t1[1]) < 1e-15
    np.testing.assert_allclose(np.cross(n, t1), t2, atol=1e-15)


# ------------------------------------------------------------ return map
KN, KS, F = 8e13, 8e12, 0.6
T0 = np.array([20e6, 6.6e6, 0.0])


def _rm(d, die=(0.0, 0.0), t0=T0):
    return O.return_map(np.asarray(d, float), np.asarray(die, float), t0, KN, KS, F)


def test_return_map_initial_state_is_initial_traction():
    trac, die, flag, D, _ = _rm([0, 0, 0])
    np.testing.assert_allclose(trac, T0, rtol=1e-15)
    assert flag == 0 and np.all(die == 0)


def test_monotone_shear_textbook():
    # fixed t'_n: shear traction = min(k_s delta_s_total, f t'_n)
    for ds in np.linspace(0, 2e-6, 41):
        trac, die, flag, D, _ = _rm([0, ds, 0])
        expect = min(KS * (T0[1] / KS + ds), F * T0[0])
        assert trac[1] == pytest.approx(expect, rel=1e-12)
        assert trac[0] == pytest.approx(T0[0], rel=1e-15)
        if KS * (T0[1] / KS + ds) > F * T0[0]:
            assert flag == 1
            assert die[0] == pytest.approx((KS * (T0[1] / KS + ds) - F * T0[0]) / KS, rel=1e-10)


@pytest.mark.parametrize("seed", range(20))
def test_kkt_after_projection(seed):
    r = np.random.default_rng(seed)
    d = r.normal(0, 2e-6, 3)
    die_n = r.normal(0, 1e-6, 2)
    trac, die, flag, D, nt = _rm(d, die_n)
    dl = np.linalg.norm(die - die_n) * KS
    ts = np.hypot(trac[1], trac[2])
    Fv = ts - F * trac[0]
    assert trac[0] >= 0 and dl >= 0
    assert Fv <= 1e-12 * max(1.0, F * trac[0], nt)
    if flag == 1:
        assert ts == pytest.approx(F * trac[0], rel=1e-12)
        # flow rule: increment parallel to the final shear traction
        inc = die - die_n
        assert abs(inc[0] * trac[2] - inc[1] * trac[1]) <= 1e-9 * np.linalg.norm(inc) * ts
    if flag == 0:
        assert np.all(die == die_n)
    assert dl * Fv <= 1e-9 * max(1.0, dl * F * trac[0])


def test_open_gives_zero_traction():
    trac, die, flag, D, _ = _rm([T0[0] / KN + 1e-7, 3e-6, 1e-6])
    assert flag == 2
    np.testing.assert_array_equal(trac, [0, 0, 0])
    assert np.all(D == 0)


def test_unloading_recovers_elastic_slip_only():
    trac1, die1, flag1, _, _ = _rm([0, 3e-6, 0])
    assert flag1 == 1
    # reverse a little: elastic unloading from the slipped state, inelastic slip kept
    back = 1e-7
    trac2, die2, flag2, _, _ = _rm([0, 3e-6 - back, 0], die1)
    assert flag2 == 0
    np.testing.assert_array_equal(die2, die1)
    assert trac2[1] == pytest.approx(trac1[1] - KS * back, rel=1e-9)


@pytest.mark.parametrize("case", ["stick", "slip", "contact_only_open"])
def test_tangent_against_finite_differences(case):
    d = {"stick": [1e-8, 1e-8, 2e-8], "slip": [2e-8, 4e-6, 1.5e-6], "contact_only_open": [T0[0] / KN + 1e-7, 0, 0]}[case]
    d = np.array(d)
    die_n = np.zeros(2)

    def force(dd):
        tr, _, _, _, _ = _rm(dd, die_n)
        return np.array([-tr[0], tr[1], tr[2]])   # components of T along (n, t1, t2)

    _, _, flag, D, _ = _rm(d, die_n)
    h = 1e-12
    J = np.stack([(force(d + h * e) - force(d - h * e)) / (2 * h) for e in np.eye(3)], 1)
    if flag == 1:
        trac, _, _, _, _ = _rm(d, die_n)
        tau = trac[1:] / np.hypot(trac[1], trac[2])
        # slip: t_s = f t'_n tau with t'_n = -k_n delta_nt, so d t_s / d delta_n = -f k_n tau;
        # the symmetric Newton tangent omits exactly this column
        nonsym = np.zeros((3, 3))
        nonsym[1:, 0] = -F * KN * tau
        np.testing.assert_allclose(J, D + nonsym, rtol=1e-5, atol=1e-5 * KN)
    else:
        np.testing.assert_allclose(J, D, rtol=1e-6, atol=1e-6 * KN)
