"""The oracle's Chebyshev polynomial preconditioner over block Jacobi (Saad,
Iterative Methods for Sparse Linear Systems, Sec. 12.3) and the Lanczos estimate
of its interval (Sec. 6.7.3), pinned to things other than themselves:

* the polynomial against its closed form on the generalized eigenvectors of
  (K, M) on a small mesh (dense eigensolver, Chebyshev T_m from numpy);
* the Ritz values against the dense spectrum (interlacing; the top one converged);
* degree 1 against block-Jacobi PCG (a scaled preconditioner gives the same iterates);
* the probe vector against the published SplitMix64 outputs."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from paper_2410_17133_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def _problem(n, dip=60):
    inst = I.make_instance(I.cube_config(n, dip_deg=dip, heterogeneous=True))
    P = O.Problem(inst)
    P.cohesive(np.zeros(3 * P.N), np.zeros((P.nq, 2)))
    return inst, P


def _dense_M(inst, K):
    """Block-diagonal M built from K itself: every node's 3x3 diagonal block, the
    6x6 block of each pair of lips' nodes that face each other."""
    N = K.shape[0] // 3
    partner = -np.ones(N, dtype=np.int64)
    for t in np.asarray(inst.mesh.coh).reshape(-1, 6):
        for a in range(3):
            u, v = int(t[a]), int(t[3 + a])
            partner[u] = v if partner[u] in (-1, v) else -2
            partner[v] = u if partner[v] in (-1, u) else -2
    M = np.zeros_like(K)
    for u in range(N):
        v = partner[u]
        idx = np.r_[3 * u:3 * u + 3, 3 * v:3 * v + 3] if v >= 0 and partner[v] == u else np.arange(3 * u, 3 * u + 3)
        M[np.ix_(idx, idx)] = K[np.ix_(idx, idx)]
    return M


def _cheb_T(m, x):
    return np.polynomial.chebyshev.chebval(x, [0] * m + [1])


@pytest.fixture(scope="module")
def small():
    inst, P = _problem(4)
    K = P.scipy(O.K_TANGENT).toarray()
    M = _dense_M(inst, K)
    lam, V = sla.eigh(K, M)          # K V = M V diag(lam), V^T M V = I
    return inst, P, K, M, lam, V


def test_probe_vector_is_splitmix64():
    ref = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            i, h = line.split()
            ref.append((int(i), int(h, 16)))
    inst, P = _problem(2)
    v = P.probe_vector()
    for i, z in ref:
        want = 0.0 if inst.dir_u[i] else (z >> 11) * 2.0 ** -53 - 0.5
        assert v[i] == want
    assert np.all(v[inst.dir_u.astype(bool)] == 0) and np.all(np.abs(v) < 0.5)


@pytest.mark.parametrize("degree", [1, 2, 3, 5])
def test_chebyshev_apply_matches_the_spectral_closed_form(small, degree):
    inst, P, K, M, lam, V = small
    lo, hi = 0.05 * lam[-1], 1.1 * lam[-1]
    r = np.random.default_rng(degree).standard_normal(K.shape[0])
    z = P.cheb_apply(r, degree, lo, hi)
    # p(t) = (1 - T_m((hi+lo-2t)/(hi-lo)) / T_m((hi+lo)/(hi-lo))) / t on the eigenvalues of M^-1 K
    sig = (hi + lo) / (hi - lo)
    p = (1.0 - _cheb_T(degree, (hi + lo - 2 * lam) / (hi - lo)) / _cheb_T(degree, sig)) / lam
    z_ref = V @ (p * (V.T @ r))
    assert np.linalg.norm(z - z_ref) <= 1e-10 * np.linalg.norm(z_ref)
    # the residual polynomial is bounded by 1/T_m(sigma) on [lo, hi]
    inside = (lam >= lo) & (lam <= hi)
    assert np.all(np.abs(1 - lam[inside] * p[inside]) <= 1.0 / _cheb_T(degree, sig) * (1 + 1e-9))


def test_lanczos_ritz_values_interlace_and_converge(small):
    inst, P, K, M, lam, V = small
    a, b = P.bj_lanczos(60)
    theta = O.ritz_values(a, b)
    assert theta[0] >= lam[0] * (1 - 1e-9) and theta[-1] <= lam[-1] * (1 + 1e-9)
    assert abs(theta[-1] - lam[-1]) <= 1e-9 * lam[-1]
    a10, b10 = P.bj_lanczos(10)
    np.testing.assert_allclose(a10, a[:10], rtol=1e-12)   # the first steps do not depend on the count
    t10 = O.ritz_values(a10, b10)
    assert lam[0] * (1 - 1e-9) <= t10[0] and t10[-1] <= lam[-1] * (1 + 1e-9)
    lo, hi = P.cheb_bounds(60, 1.1, 300)
    assert hi == pytest.approx(1.1 * lam[-1], rel=1e-9) and lo == pytest.approx(hi / 300, rel=1e-14)


def test_lanczos_matrix_of_plain_cg_is_the_projected_operator():
    """Without a preconditioner the Lanczos matrix of the CG coefficients equals
    Q^T A Q for the normalised residuals Q (the textbook identity, checked on a
    dense SPD matrix with numpy's own CG loop)."""
    rng = np.random.default_rng(3)
    G = rng.standard_normal((40, 40))
    A = G @ G.T + 40 * np.eye(40)
    r = rng.standard_normal(40)
    p, rho = r.copy(), r @ r
    al, be, Q = [], [], [r / np.sqrt(rho)]
    for _ in range(12):
        q = A @ p
        alpha = rho / (p @ q)
        r = r - alpha * q
        rho2 = r @ r
        al.append(alpha), be.append(rho2 / rho)
        p = r + be[-1] * p
        rho = rho2
        Q.append(r / np.sqrt(rho))
    Q = np.array(Q[:12]).T
    T = O.lanczos_matrix(np.array(al), np.array(be))
    # residuals alternate in sign relative to the Lanczos vectors: compare |T|
    np.testing.assert_allclose(np.abs(T), np.abs(Q.T @ A @ Q), rtol=1e-8, atol=1e-8 * np.abs(T).max())


def test_degree_one_is_block_jacobi_pcg():
    inst, P = _problem(8)
    b = np.random.default_rng(2).standard_normal(3 * P.N) * (1 - inst.dir_u)
    x1, s1, it1, r1 = P.pcg_block(b, tol=1e-11)
    x2, s2, it2, r2 = P.pcg_cheb(b, 1, 0.01, 2.7, tol=1e-11)
    # same iterates up to rounding (the 1/theta scale and the threaded dot products): the stop test may
    # fall one iteration either way
    assert s1 == 0 and s2 == 0 and abs(it1 - it2) <= 1
    assert np.linalg.norm(x2 - x1) <= 1e-9 * np.linalg.norm(x1)


def test_chebyshev_pcg_solves_in_fewer_iterations():
    inst, P = _problem(12)
    b = np.random.default_rng(1).standard_normal(3 * P.N) * (1 - inst.dir_u)
    x1, s1, it1, _ = P.pcg_block(b, tol=1e-12)
    lo, hi = P.cheb_bounds(40, 1.1, 300)
    for deg in (2, 4):
        x2, s2, it2, _ = P.pcg_cheb(b, deg, lo, hi, tol=1e-12)
        assert s2 == 0
        assert np.linalg.norm(b - P.spmv(O.K_TANGENT, x2)) <= 1e-11 * np.linalg.norm(b)
        assert np.linalg.norm(x2 - x1) <= 1e-9 * np.linalg.norm(x1)
        print(f"[chebyshev] degree {deg}: {it2} iterations ({deg * it2} products), block Jacobi {it1}")
        # products stay within 20 % of block-Jacobi CG while the iterations drop about deg-fold
        assert it2 <= 1.2 * it1 / deg and deg * it2 >= 0.9 * it1


def test_zero_right_hand_side():
    inst, P = _problem(4)
    x, s, it, rr = P.pcg_cheb(np.zeros(3 * P.N), 3, 0.01, 3.0)
    assert s == 0 and it == 0 and not x.any()
