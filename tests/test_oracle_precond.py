"""The oracle's block-Jacobi preconditioned CG on K (nodal 3x3 blocks, 6x6 blocks
over the two lips' nodes at each interface point): its small inverses, its
solution against point-Jacobi CG on the same system, and the drop in iterations
the fault-pair blocks give on the penalty-stiffened interface."""
import ctypes as C

import numpy as np

from oracle import oracle as O
from paper_2410_17133_amd import inputs as I


def test_gauss_jordan_inverse():
    r = np.random.default_rng(0)
    for n in (3, 6):
        G = r.standard_normal((n, n))
        M = G @ G.T + n * np.eye(n)
        M[[0, 2]] = M[[2, 0]]                          # a row swap forces pivoting
        inv, ok = np.zeros(n * n), C.c_int()
        O.lib().or_gj_inverse(n, np.ascontiguousarray(M.reshape(-1)).copy(), inv, C.byref(ok))
        assert ok.value == 1
        np.testing.assert_allclose(inv.reshape(n, n) @ M, np.eye(n), atol=1e-12)
    inv, ok = np.zeros(9), C.c_int()
    O.lib().or_gj_inverse(3, np.zeros(9), inv, C.byref(ok))
    assert ok.value == 0


def test_block_jacobi_cg_solves_the_same_system_in_fewer_iterations():
    inst = I.make_instance(I.cube_config(12, dip_deg=60, heterogeneous=True))
    P = O.Problem(inst)
    P.cohesive(np.zeros(3 * P.N), np.zeros((P.nq, 2)))
    b = np.random.default_rng(1).standard_normal(3 * P.N) * (1 - inst.dir_u)
    x1, s1, it1, r1 = P.pcg(O.K_TANGENT, b, tol=1e-12)
    x2, s2, it2, r2 = P.pcg_block(b, tol=1e-12)
    assert s1 == 0 and s2 == 0
    assert np.linalg.norm(b - P.spmv(O.K_TANGENT, x2)) <= 1e-11 * np.linalg.norm(b)
    assert np.linalg.norm(x2 - x1) <= 1e-9 * np.linalg.norm(x1)
    print(f"[block Jacobi] point {it1} iterations, block {it2}")
    assert it2 < 0.5 * it1
