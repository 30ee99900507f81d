"""Oracle adjoint through a time loop: the inelastic slip carried from step to step
(the return map of Sec. 2.2.1) is differentiated point by point, pinned against
central differences of the return map itself, and the reverse sweep over several
steps is pinned against central differences of the oracle's own time loop."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_17133_amd import inputs as I

TIGHT = dict(tol_newton=1e-13, max_newton=80, tol_outer=1e-13, tol_inner=1e-14)


def slip_instance():
    """4^3 cube, 2e-3 m^3/s injection: slip starts in the second step and spreads, and
    part of the fault opens in the fourth."""
    return I.make_instance(dataclasses.replace(I.cube_config(4), Q=2e-3))


def slip_objective(inst, U, uplift):
    """sum over fault pairs of |tangential jump|^2 + squared uplift, and its gradient in U."""
    m = inst.mesh
    X = m.xyz[m.coh[0, 3:]]
    n = np.cross(X[1] - X[0], X[2] - X[0])
    n /= np.linalg.norm(n)
    U3 = U.reshape(-1, 3)
    jump = U3[m.pairs[:, 1]] - U3[m.pairs[:, 0]]
    slip = jump - np.outer(jump @ n, n)
    g = np.zeros_like(U3)
    np.add.at(g, m.pairs[:, 1], 2 * slip)
    np.add.at(g, m.pairs[:, 0], -2 * slip)
    g[uplift, 2] += 2 * U3[uplift, 2]
    return np.sum(slip * slip) + np.sum(U3[uplift, 2] ** 2), g.reshape(-1)


@pytest.fixture(scope="module")
def loop3():
    inst = slip_instance()
    P = O.Problem(inst)
    ck = P.trajectory(4, **TIGHT)
    flags = [P.cohesive(U, die_prev)[2] for U, Pp, die_prev, die in ck]
    return inst, P, ck, flags


def test_loop_carries_slip(loop3):
    inst, P, ck, flags = loop3
    nslip = [int((f == 1).sum()) for f in flags]
    nopen = [int((f == 2).sum()) for f in flags]
    assert nslip[0] == 0 and min(nslip[1:]) > 0 and nopen[-1] > 0
    size = [np.abs(c[3]).max() for c in ck]
    assert size[0] == 0 and all(b > a for a, b in zip(size[1:], size[2:]))   # the slip grows over the loop


def test_slip_state_adjoint_against_return_map_differences(loop3):
    """gU . v and a_old . w equal the central differences of a.die_new(U, die_old)
    (and of -lam.f_coh) at a state with stick, slip and open points."""
    inst, P, ck, flags = loop3
    U, Pp, die_prev, die = ck[-1]
    r = np.random.default_rng(4)
    # push part of the fault open and part into slip: a state with every branch present
    U2 = U + r.normal(0.0, 3e-7, U.size) * (1 - inst.dir_u)
    t, d_new, flag, f = P.cohesive(U2, die_prev)
    assert all((flag == k).sum() > 0 for k in (0, 1, 2))
    a_new = r.standard_normal((P.nq, 2))
    lam = r.standard_normal(3 * P.N) * (1 - inst.dir_u)
    gU, a_old = P.slip_adjoint(U2, die_prev, a_new, lam)
    gU0, a_old0 = P.slip_adjoint(U2, die_prev, a_new)
    np.testing.assert_array_equal(gU, gU0)                  # lam only enters a_old
    v = r.standard_normal(U.size) * (1 - inst.dir_u)
    h = 1e-13
    dp = P.cohesive(U2 + h * v, die_prev)[1]
    dm = P.cohesive(U2 - h * v, die_prev)[1]
    fd = np.sum(a_new * (dp - dm)) / (2 * h)
    assert abs(fd - gU @ v) <= 1e-5 * abs(fd)
    w = r.standard_normal((P.nq, 2))
    hw = 1e-12
    (_, dp, _, fp), (_, dm, _, fm) = P.cohesive(U2, die_prev + hw * w), P.cohesive(U2, die_prev - hw * w)
    fd = (np.sum(a_new * (dp - dm)) - lam @ (fp - fm)) / (2 * hw)
    assert abs(fd - np.sum(a_old * w)) <= 1e-5 * abs(fd)


@pytest.mark.slow
def test_loop_gradient_matches_central_differences(loop3):
    """dJ/d(ln k, ln E) of J = sum over the 4 steps of the slip-and-uplift objective, by
    the reverse sweep, against central differences of the whole 4-step loop."""
    inst, P, ck, flags = loop3
    uplift = I.uplift_nodes(inst, 8)
    dE, dk = P.trajectory_gradient(ck, lambda n, U, Pp: (slip_objective(inst, U, uplift)[1], np.zeros(P.N)))
    grad = np.r_[dk, dE * inst.E]                      # w.r.t. (ln k, ln E)
    ne = inst.E.size
    D = I.fd_directions(2 * ne, count=2, seed=1)

    def J(x):
        inst2 = dataclasses.replace(inst, logk=inst.logk + x[:ne], E=inst.E * np.exp(x[ne:]))
        P2 = O.Problem(inst2)
        return sum(slip_objective(inst, U, uplift)[0] for U, _, _, _ in P2.trajectory(4, **TIGHT))
    eps = 1e-5
    for d in D:
        fd = (J(eps * d) - J(-eps * d)) / (2 * eps)
        assert abs(fd - grad @ d) <= 1e-5 * abs(fd), (fd, grad @ d)
    # the slip-state terms matter: without them the sweep misses the finite differences
    dE0, dk0 = P.trajectory_gradient(ck, lambda n, U, Pp: (slip_objective(inst, U, uplift)[1], np.zeros(P.N)),
                                     slip_state=False)
    g0 = np.r_[dk0, dE0 * inst.E]
    assert abs(g0 @ D[0] - grad @ D[0]) > 1e-3 * abs(grad @ D[0])
