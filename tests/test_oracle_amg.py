"""Pins of the oracle's smoothed-aggregation AMG preconditioner of K_t (the
third stage of the stronger preconditioner): its Galerkin coarse operators equal
the triple products of the exported prolongators, the smoothed prolongator still
reproduces the rigid-body modes of a free body exactly, the V-cycle is symmetric
and contracts the error, and AMG-PCG reaches the direct solution in a small
fraction of the block-Jacobi iterations."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_2410_17133_amd import inputs as I

from test_oracle_system import box_instance


def faulted(n=10):
    inst = I.make_instance(I.cube_config(n, dip_deg=60, heterogeneous=True))
    P = O.Problem(inst)
    P.cohesive(np.zeros(3 * P.N), np.zeros((P.nq, 2)))
    hi0 = P.cheb_bounds(40, 1.1, 300)[1]
    return inst, P, hi0


def test_galerkin_coarse_operators_equal_triple_products():
    inst, P, hi0 = faulted(10)
    A0 = P.scipy(O.K_TANGENT)
    assert abs(P.amg_export(hi0, 0, 0) - A0).max() == 0.0          # level 0 is K_t itself
    for l in range(2):   # coarsening down to 8 nodes: three levels
        A, Pl, Ac = (P.amg_export(hi0, l, 0, coarse_nodes=8), P.amg_export(hi0, l, 1, coarse_nodes=8),
                     P.amg_export(hi0, l + 1, 0, coarse_nodes=8))
        ref = (Pl.T @ A @ Pl).tocsr()
        err = abs(Ac - ref).max() / abs(ref).max()
        print(f"level {l}: {A.shape[0]} -> {Ac.shape[0]} unknowns, Galerkin error {err:.1e}")
        assert err < 1e-13
        assert abs(Ac - Ac.T).max() <= 1e-13 * abs(Ac).max()


def test_smoothed_prolongator_reproduces_rigid_modes_of_a_free_body():
    """On a cube with no restraint, K has the six rigid-body modes in its null space;
    each is a combination of every aggregate's tentative modes, and (I - w D^-1 K)
    leaves it unchanged, so it lies in the range of the smoothed P exactly, and its
    coarse representation is in the null space of the coarse operator."""
    inst = box_instance(6, 6, 6)
    P = O.Problem(inst)
    P.cohesive(np.zeros(3 * P.N), np.zeros((0, 2)))
    hi0 = P.cheb_bounds(40, 1.1, 300)[1]
    P0, A1 = P.amg_export(hi0, 0, 1), P.amg_export(hi0, 1, 0)
    x = inst.mesh.xyz - 0.5
    K = P.scipy(O.K_TANGENT)
    for k in range(6):
        v = np.zeros((P.N, 3))
        if k < 3:
            v[:, k] = 1.0
        else:
            e = np.zeros(3)
            e[k - 3] = 1.0
            v = np.cross(e, x)
        v = v.reshape(-1)
        assert np.linalg.norm(K @ v) <= 1e-9 * abs(K).max() * np.linalg.norm(v)
        y = spla.lsqr(P0, v, atol=1e-15, btol=1e-15, iter_lim=20000)[0]
        assert np.linalg.norm(P0 @ y - v) <= 1e-9 * np.linalg.norm(v)
        assert np.linalg.norm(A1 @ y) <= 1e-8 * abs(A1).max() * np.linalg.norm(y)


def test_vcycle_is_symmetric_and_contracts():
    inst, P, hi0 = faulted(12)
    r = np.random.default_rng(3)
    free = 1.0 - inst.dir_u
    u, v = r.standard_normal(3 * P.N) * free, r.standard_normal(3 * P.N) * free
    Bu, Bv = P.amg_apply(u, hi0), P.amg_apply(v, hi0)
    assert abs(u @ Bv - v @ Bu) <= 1e-12 * abs(u @ Bv)
    assert u @ Bu > 0 and v @ Bv > 0
    # the V-cycle as a stationary iteration x <- x + B (b - K x): A-norm error factor
    K = P.scipy(O.K_TANGENT)
    xs = r.standard_normal(3 * P.N) * free
    b = K @ xs
    x = np.zeros_like(b)
    errs = []
    for _ in range(8):
        x = x + P.amg_apply(b - K @ x, hi0)
        e = x - xs
        errs.append(np.sqrt(e @ (K @ e)))
    factors = np.array(errs[1:]) / np.array(errs[:-1])
    print(f"V-cycle error factors {np.round(factors, 3)}")
    assert factors.max() < 0.7           # a stationary V-cycle converges by itself (CG accelerates it)


@pytest.mark.parametrize("n", [8, 16])
def test_amg_pcg_reaches_the_direct_solution_in_few_iterations(n):
    inst, P, hi0 = faulted(n)
    b = np.random.default_rng(4).standard_normal(3 * P.N) * (1 - inst.dir_u)
    x, st, it, rr, levels, nodes = P.pcg_amg(b, hi0, tol=1e-12)
    xd = spla.spsolve(P.scipy(O.K_TANGENT).tocsc(), b)
    _, _, itb, _ = P.pcg_block(b, tol=1e-12)
    print(f"{n}^3: AMG-PCG {it} iterations ({levels} levels, nodes {list(nodes)}), block Jacobi {itb}")
    assert st == 0 and levels >= 2
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert it * 5 < itb
