"""Cryer's problem (Sec. 4.1): the centre pressure of a poroelastic sphere under a
suddenly applied, then constant, uniform surface compression, drained at its
surface.  The paper cites the closed form without printing it; it is derived
here from the radially symmetric Biot equations.

With u radial, equilibrium makes (lambda + 2G) e - alpha p = f(t) uniform (e the
volumetric strain); the surface traction fixes f from the mean pressure
pbar = (3/R^3) int r^2 p dr, and the fluid balance d(alpha e + p/M)/dt = (k/mu) lap p
becomes, with S = 1/M + alpha^2/(lambda + 2G), c = k/(mu S) and
beta = 4 G alpha^2 / (3 K (lambda + 2G) S),

    dp/dt = c lap p - beta dpbar/dt,   p(R, t) = 0,   p(r, 0+) = p0 = alpha M F / (K + alpha^2 M).

In Laplace space (q^2 = s R^2 / c) the centre pressure is
    P_c(s) = (p0/s) [1 - N(q)/D(q)],   N = 1 - beta h(q)/(1 + beta),   D = sinh(q)/q - beta h(q)/(1 + beta),
    h(q) = 3 (q cosh q - sinh q) / q^3,
whose poles q = i xi_n, (1 - eta xi^2) tan xi = xi with eta = (1 + beta)/(3 beta), give
    p_c(t) / p0 = sum_n -2 N(i xi_n) / (xi_n dD/dxi(xi_n)) exp(-xi_n^2 c t / R^2).
`radial_reference` integrates the same radial equation by finite volumes and
implicit Euler: an independent route to the same curve.

Test helper, not part of the library."""
import math

import numpy as np
import scipy.linalg
from scipy.optimize import brentq


def elastic_constants(E, nu, alpha, M):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    G = E / (2 * (1 + nu))
    K = lam + 2 * G / 3
    S = 1 / M + alpha ** 2 / (lam + 2 * G)
    beta = 4 * G * alpha ** 2 / (3 * K * (lam + 2 * G) * S)
    return lam, G, K, S, beta


def _g(x):
    return 3 * (math.sin(x) - x * math.cos(x)) / x ** 3


def roots(beta, count):
    """The first `count` positive roots of sin(xi)/xi = beta/(1+beta) * 3 (sin xi - xi cos xi)/xi^3."""
    D = lambda x: math.sin(x) / x - beta / (1 + beta) * _g(x)
    out, x, f0, step = [], 1e-3, None, 0.01
    f0 = D(x)
    while len(out) < count:
        x1 = x + step
        f1 = D(x1)
        if f0 * f1 < 0:
            out.append(brentq(D, x, x1, xtol=1e-15))
        x, f0 = x1, f1
    return np.array(out), D


def centre_pressure(beta, tau, terms=400):
    """p_c / p0 at dimensionless times tau = c t / R^2 (the residue series)."""
    tau = np.asarray(tau, dtype=float)
    xi, D = roots(beta, terms)
    out = np.zeros_like(tau)
    for x in xi:
        N = 1 - beta * _g(x) / (1 + beta)
        h = 1e-7 * x
        dD = (D(x + h) - D(x - h)) / (2 * h)
        out += -2 * N / (x * dD) * np.exp(-x * x * tau)
    return out


def radial_reference(beta, tau_end, nr=200, nt=4000):
    """(tau, p_c/p0) of the radial equation dp/dtau = lap p - beta dpbar/dtau on the
    unit ball by finite volumes (nr cells) and implicit Euler (nt steps)."""
    r = np.linspace(0.0, 1.0, nr + 1)
    dr = r[1] - r[0]
    n = nr
    w = np.zeros(n)
    L = np.zeros((n, n))
    for i in range(n):
        rm, rp = max(r[i] - dr / 2, 0.0), r[i] + dr / 2
        w[i] = rp ** 3 - rm ** 3                   # 3 int r^2 dr over the control volume
        vol = w[i] / 3
        if i + 1 < n:
            L[i, i + 1] += rp ** 2 / dr / vol
        L[i, i] -= rp ** 2 / dr / vol              # node n (p = 0) closes the last flux
        if i > 0:
            L[i, i - 1] += rm ** 2 / dr / vol
            L[i, i] -= rm ** 2 / dr / vol
    dt = tau_end / nt
    A = np.eye(n) / dt - L + beta * np.outer(np.ones(n), w) / dt
    lu = scipy.linalg.lu_factor(A)
    p = np.ones(n)
    ts, pc = [0.0], [1.0]
    for k in range(nt):
        p = scipy.linalg.lu_solve(lu, p / dt + beta * (w @ p) / dt)
        ts.append((k + 1) * dt)
        pc.append(p[0])
    return np.array(ts), np.array(pc)
