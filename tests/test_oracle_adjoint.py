"""Pins of the oracle adjoint: the transposed exact Jacobian solved densely, and
central finite differences of the oracle's own converged step (the definition
of the gradient)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_17133_amd import inputs as I

TIGHT = dict(tol_newton=1e-13, max_newton=80, tol_outer=1e-13, tol_inner=1e-14)


def objective(inst, U, uplift):
    """J = sum over fault pairs of |tangential jump|^2 + sum of squared vertical uplift; and dJ/dU."""
    m = inst.mesh
    U3 = U.reshape(-1, 3)
    X = m.xyz[m.coh[0, 3:]]
    n = np.cross(X[1] - X[0], X[2] - X[0])
    n /= np.linalg.norm(n)            # planar fault: one normal
    jump = U3[m.pairs[:, 1]] - U3[m.pairs[:, 0]]
    slip = jump - np.outer(jump @ n, n)
    J = np.sum(slip * slip) + np.sum(U3[uplift, 2] ** 2)
    g = np.zeros_like(U3)
    np.add.at(g, m.pairs[:, 1], 2 * slip)
    np.add.at(g, m.pairs[:, 0], -2 * slip)
    g[uplift, 2] += 2 * U3[uplift, 2]
    return J, g.reshape(-1)


def forward(inst, E=None, logk=None):
    import dataclasses
    inst2 = dataclasses.replace(inst, E=inst.E if E is None else E, logk=inst.logk if logk is None else logk)
    P = O.Problem(inst2)
    U, Pp, die = np.zeros(3 * P.N), np.zeros(P.N), np.zeros((P.nq, 2))
    trac, flag, info, st = P.step(U, Pp, die, **TIGHT)
    assert st == 0, info
    return P, U, Pp, flag


def small_slip_instance():
    """4^3 cube with a stronger injection (4e-3 m^3/s) so that the converged step has slip points."""
    import dataclasses
    return I.make_instance(dataclasses.replace(I.cube_config(4), Q=4e-3))


@pytest.fixture(scope="module")
def converged():
    inst = small_slip_instance()
    P, U, Pp, flag = forward(inst)
    assert (flag == 1).sum() > 0          # slip points present: the non-symmetric term matters
    uplift = I.uplift_nodes(inst, 8)
    P.cohesive(U, np.zeros((P.nq, 2)))    # tangent and point states at the converged state
    return inst, P, U, Pp, uplift


def test_adjoint_equals_dense_transposed_exact_jacobian(converged):
    inst, P, U, Pp, uplift = converged
    J, gu = objective(inst, U, uplift)
    gp = np.zeros(P.N)
    lu, lp, st, stats = P.adjoint(gu, gp)
    assert st == 0 and stats[0] >= 2
    K = P.scipy(O.K_TANGENT).toarray()
    Nt = np.stack([P.apply_NT(e) for e in np.eye(3 * P.N)], 1)     # N^T as a dense matrix
    A = np.stack([P.apply_Apu(e) for e in np.eye(P.N)], 1)
    A22 = P.scipy(O.A22).toarray()
    JT = np.block([[K + Nt, A], [-A.T, A22]])                       # transposed exact Jacobian
    free = np.r_[1 - inst.dir_u, 1 - inst.dir_p].astype(bool)
    rhs = np.r_[gu * (1 - inst.dir_u), gp]
    lam = np.zeros(4 * P.N)
    lam[free] = np.linalg.solve(JT[np.ix_(free, free)], rhs[free])
    assert np.linalg.norm(lu - lam[:3 * P.N]) <= 1e-8 * np.linalg.norm(lam[:3 * P.N])
    assert np.linalg.norm(lp - lam[3 * P.N:]) <= 1e-8 * np.linalg.norm(lam[3 * P.N:])


def test_nonsymmetric_part_is_the_exact_tangent_defect(converged):
    """K_t + N equals central differences of the interface force (slip points included)."""
    inst, P, U, Pp, uplift = converged
    die = np.zeros((P.nq, 2))
    free = 1.0 - inst.dir_u
    v = np.random.default_rng(3).standard_normal(3 * P.N) * free
    P.cohesive(U, die)
    Kt = P.scipy(O.K_TANGENT)
    Kb = P.scipy(O.K_BULK)
    Nv = P.apply_NT(np.zeros(3 * P.N))
    assert np.all(Nv == 0)
    # N v from N^T by duality: e_i . N v = (N^T e_i) . v, only for the interface rows
    rows = np.unique(np.r_[3 * inst.mesh.coh.reshape(-1), 3 * inst.mesh.coh.reshape(-1) + 1, 3 * inst.mesh.coh.reshape(-1) + 2])
    Nv = np.zeros(3 * P.N)
    for i in rows:
        e = np.zeros(3 * P.N)
        e[i] = 1
        Nv[i] = P.apply_NT(e) @ v
    h = 1e-13
    fp = P.cohesive(U + h * v, die)[3]
    fm = P.cohesive(U - h * v, die)[3]
    P.cohesive(U, die)
    fd = (fp - fm) / (2 * h)
    np.testing.assert_allclose((Kt - Kb) @ v + Nv, fd, rtol=0, atol=1e-5 * np.abs(fd).max())


@pytest.mark.slow
def test_adjoint_gradient_matches_central_differences(converged):
    inst, P, U, Pp, uplift = converged
    J0, gu = objective(inst, U, uplift)
    lu, lp, st, stats = P.adjoint(gu, np.zeros(P.N))
    dE, dk = P.sensitivity(U, Pp, lu, lp)
    grad_lnE = dE * inst.E                   # dJ/dln E = E dJ/dE
    ne = inst.E.size
    D = I.fd_directions(2 * ne, count=3)
    # a 1e-5 step keeps the difference well above the tolerance floor of the two
    # forward solves; the truncation error is O(eps^2)
    eps = 1e-5
    for d in D:
        dlk, dlE = d[:ne], d[ne:]
        Jp = objective(inst, forward(inst, E=inst.E * np.exp(eps * dlE), logk=inst.logk + eps * dlk)[1], uplift)[0]
        Jm = objective(inst, forward(inst, E=inst.E * np.exp(-eps * dlE), logk=inst.logk - eps * dlk)[1], uplift)[0]
        fd = (Jp - Jm) / (2 * eps)
        ad = dk @ dlk + grad_lnE @ dlE
        assert abs(fd - ad) <= 1e-5 * abs(ad), (fd, ad)


def test_forward_slip_term_is_the_exact_tangent_defect(converged):
    """N v (forward product) completes the symmetric tangent to central differences of the
    interface force, and is the transpose of N^T (x.(N v) = (N^T x).v)."""
    inst, P, U, Pp, uplift = converged
    die = np.zeros((P.nq, 2))
    free = 1.0 - inst.dir_u
    r = np.random.default_rng(5)
    v = r.standard_normal(3 * P.N) * free
    x = r.standard_normal(3 * P.N) * free
    P.cohesive(U, die)
    Kt, Kb = P.scipy(O.K_TANGENT), P.scipy(O.K_BULK)
    Nv = P.apply_N(v)
    assert np.abs(Nv).max() > 0
    assert abs(x @ Nv - P.apply_NT(x) @ v) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(Nv)
    h = 1e-13
    fd = (P.cohesive(U + h * v, die)[3] - P.cohesive(U - h * v, die)[3]) / (2 * h)
    P.cohesive(U, die)
    np.testing.assert_allclose((Kt - Kb) @ v + Nv, fd, rtol=0, atol=1e-5 * np.abs(fd).max())
    # without it the symmetric tangent misses the force change along the slip direction
    assert np.abs((Kt - Kb) @ v - fd).max() > 1e-3 * np.abs(fd).max()


def test_bicgstab_solves_the_exact_tangent(converged):
    """BiCGStab on K_t + N: its solution against a dense solve of the exact tangent, its
    residual with independent products, and fewer iterations than point-Jacobi CG takes
    on the symmetric part."""
    inst, P, U, Pp, uplift = converged
    P.cohesive(U, np.zeros((P.nq, 2)))
    free = (1.0 - inst.dir_u).astype(bool)
    b = np.random.default_rng(6).standard_normal(3 * P.N) * free
    x, st, it, rr = P.bicgstab_exact(b, tol=1e-12)
    assert st == 0 and rr <= 1e-12
    K = P.scipy(O.K_TANGENT).toarray()
    Nd = np.stack([P.apply_N(e) for e in np.eye(3 * P.N)], 1)
    A = K + Nd
    assert np.linalg.norm(b - A @ x) <= 1e-11 * np.linalg.norm(b)
    xd = np.zeros(3 * P.N)
    xd[free] = np.linalg.solve(A[np.ix_(free, free)], b[free])
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    # the symmetric tangent's solution is a different one
    xs, s2, it2, _ = P.pcg(O.K_TANGENT, b, tol=1e-12)
    assert np.linalg.norm(xs - xd) > 1e-6 * np.linalg.norm(xd)
    print(f"[bicgstab] {it} iterations (2 products each); point-Jacobi CG on K_t {it2}")
    # zero right-hand side
    x0, st0, it0, _ = P.bicgstab_exact(np.zeros(3 * P.N))
    assert st0 == 0 and it0 == 0 and not x0.any()
