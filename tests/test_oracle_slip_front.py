"""Pins of the oracle's chain from fracture pressure to fault slip, with the
Sec. 4.2 workload (injection into a frictional fault, Table 1 materials):

* a uniform fracture pressure p lowers the effective normal traction of every
  interface point by exactly p (equilibrium of the free block on the far side of
  the fault), and the Coulomb return map then slips every point once
  tau0 > f (sigma0 - p): this fixes the sign and size of the pressure load on
  the lips and of t'_n in the yield function;
* a constant-rate injection makes the slip front R(t) and the diffusion front
  L(t) = sqrt(4 alpha_f t) grow self-similarly, R = lambda L with lambda fixed
  by the fault-stress parameter T, both in proportion to sqrt(t), with R > L
  for a critically stressed fault (T << 1) and R < L for a marginally
  pressurized one (T = 4) (Sec. 4.2).  The values of lambda(T) and the slip
  profiles are not printed in the paper and are not asserted.

The workload is the paper's turned so that the fault is a vertical grid plane
(nu = 0, isotropic: the turn changes nothing), on graded boxes far smaller
than the paper's 40 m box; the final times keep both fronts well inside it.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2410_17133_amd import inputs as I

B = I.SLIP_BENCHMARK
QP = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])


def qp_radius(inst):
    """Distance of every interface quadrature point (3 t + q) from the injection node."""
    m = inst.mesh
    xq = np.einsum("qa,fad->fqd", QP, m.xyz[m.coh[:, :3]]).reshape(-1, 3)
    return np.linalg.norm(xq - m.xyz[inst.centre_pair[0]], axis=1)


def diffusion_front(inst, t):
    """L(t) = sqrt(4 alpha_f t), alpha_f = k_par M_F / mu: the radius of the Theis
    pressure E1(r^2 / L^2) of a constant-rate injection into the fault."""
    p = inst.params
    return math.sqrt(4 * p.k_par * p.M_F / p.mu * t)


def fault_stress_parameter(tau0):
    """T = (1 - tau0 / (f sigma0')) / (dp* / sigma0'), dp* = Q mu / (4 pi w k_par) (Sec. 4.2)."""
    dps = B["Q"] * B["mu"] / (4 * math.pi * B["wk_par"])
    return (1 - tau0 / (B["friction"] * B["sigma0"])) / (dps / B["sigma0"])


def test_uniform_fault_pressure_lowers_the_effective_normal_traction_by_p():
    inst = I.slip_benchmark_instance(B["tau0_MP"], h=0.25, n_fine=4, n_grade=3, nx_grade=3)
    m = inst.mesh
    P = O.Problem(inst)
    U0, die0 = np.zeros(3 * P.N), np.zeros((P.nq, 2))
    P.cohesive(U0, die0)                                   # stick tangent at the initial state
    p_fault = np.zeros(P.N)
    p_fault[m.pairs.reshape(-1)] = 1.0                     # unit pressure on both lips, zero in the rock
    U1, st, _, _ = P.pcg(O.K_TANGENT, P.apply_Apu(p_fault), tol=1e-14)
    assert st == 0
    # the - side is clamped, the + block is held by the interface alone: it moves
    # away rigidly by p / k_n and carries no stress
    plus = m.pairs[:, 1]
    gap = U1[3 * plus]                                    # normal (x) displacement of the + lip
    np.testing.assert_allclose(gap, 1.0 / B["k_n"], rtol=1e-8)
    sigma0, f, tau0 = B["sigma0"], B["friction"], B["tau0_MP"]
    p_crit = sigma0 - tau0 / f                            # tau0 = f (sigma0 - p)
    for p in (0.5 * p_crit, 0.999 * p_crit, 1.001 * p_crit, 2 * p_crit):
        trac, _, flag, _ = P.cohesive(p * U1, die0)
        np.testing.assert_allclose(trac[:, 0], sigma0 - p, rtol=1e-10)
        slipping = p > p_crit
        assert np.all(flag == (1 if slipping else 0))
        ts = np.hypot(trac[:, 1], trac[:, 2])
        np.testing.assert_allclose(ts, f * (sigma0 - p) if slipping else tau0, rtol=1e-10)


def run_fronts(inst, steps, measure_from, tol_newton=1e-8):
    """Time loop of the oracle's implicit steps from rest; returns (t, L, R, h_front)
    per measured step, R the radius of the outermost point with inelastic slip."""
    P = O.Problem(inst)
    rq = qp_radius(inst)
    U, Pp, die = np.zeros(3 * P.N), np.zeros(P.N), np.zeros((P.nq, 2))
    out = []
    for s in range(1, steps + 1):
        _, flag, info, st = P.step(U, Pp, die, tol_newton=tol_newton, tol_outer=1e-10, tol_inner=1e-12)
        assert st == 0
        assert not np.any(flag == 2)                      # the fault stays closed
        if s >= measure_from:
            t = s * inst.params.dt
            slipped = np.linalg.norm(die, axis=1) > 0
            R = rq[slipped].max() if slipped.any() else 0.0
            print(f"t {t:8.1f}  L {diffusion_front(inst, t):.4f}  R {R:.4f}  newton {int(info[0])}", flush=True)
            out.append((t, diffusion_front(inst, t), R))
    return np.array(out)


def check_self_similar(fronts, h):
    """R = lambda L to within one cell of the fault mesh at every measured time,
    and R grows as t^beta with beta = 1/2 to within 0.1 (least squares)."""
    t, L, R = fronts.T
    assert np.all(R > 0)
    lam = float(R @ L / (L @ L))
    assert np.all(np.abs(R - lam * L) <= h), (R, lam * L)
    beta = np.polyfit(np.log(t), np.log(R), 1)[0]
    assert abs(beta - 0.5) <= 0.1, beta
    assert t[-1] / t[0] >= 4                               # the fronts double over the measured times
    return lam


@pytest.mark.slow
def test_slip_front_critically_stressed_runs_ahead_of_the_pressure():
    """tau0 = 47.999 MPa (T = 0.0235 << 1): the rupture front is several times
    the diffusion front from the first step on.  h = 0.1 m cells over the central
    1.6 m of the fault; the front reaches about 0.57 m at t = 16 s (L = 0.12 m)."""
    assert fault_stress_parameter(B["tau0_CS"]) < 0.05
    inst = I.slip_benchmark_instance(B["tau0_CS"], h=0.1, n_fine=16, n_grade=6, nx_grade=7, dt=4.0)
    fronts = run_fronts(inst, steps=4, measure_from=1)
    lam = check_self_similar(fronts, h=0.1)
    assert lam > 2 and np.all(fronts[:, 2] > fronts[:, 1])


@pytest.mark.slow
def test_slip_front_marginally_pressurized_stays_inside_the_pressure():
    """tau0 = 47.830 MPa (T = 4): the rupture stays well inside the pressurized
    region.  h = 0.05 m cells over the central 0.8 m of the fault, graded out to
    a 17.8 m wide box; L reaches 2.5 m at t = 6960 s."""
    assert fault_stress_parameter(B["tau0_MP"]) == pytest.approx(4.0, rel=2e-3)
    inst = I.slip_benchmark_instance(B["tau0_MP"], h=0.05, n_fine=16, n_grade=10, nx_grade=7, dt=870.0)
    fronts = run_fronts(inst, steps=8, measure_from=2)
    lam = check_self_similar(fronts, h=0.05)
    assert lam < 0.5 and np.all(fronts[:, 2] < fronts[:, 1])
