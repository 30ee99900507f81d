"""Seeded synthetic inputs: structured Kuhn-tetrahedron meshes with a conforming
zero-thickness fault, per-element heterogeneity, boundary masks and sources.

This module is input generation only. It holds none of the solver's arithmetic
(no element matrices, no return map, no solves); both the CPU oracle and the
HIP library consume the arrays it produces.

Mesh conventions (the library header states the same ones):
  * nodes are numbered node-major; a displacement vector is [u0x,u0y,u0z,u1x,...]
  * every hexahedron of an nx*ny*nz grid is cut into 6 tetrahedra along its
    (0,0,0)->(1,1,1) diagonal (Kuhn split), all positively oriented; the split
    is conforming, so the fault plane is a union of tetrahedron faces
  * the fault is the grid plane i = i_f; its (ny+1)(nz+1) nodes are duplicated
    over the whole plane (the paper duplicates the full fault plane, Sec. 4.2);
    tetrahedra on the + side (x beyond the plane) use the copies
  * cohesive elements are 6-node triangle pairs [+a,+b,+c,-a,-b,-c]; the vertex
    order (a,b,c) makes (x_b-x_a) x (x_c-x_a) point from the - side to the + side
  * a dipping fault uses a column-shift map of the grid: node (i,j,k) keeps its
    topology and gets x = x_f(z) i/i_f on the - side and
    x_f + (Lx-x_f)(i-i_f)/(nx-i_f) on the + side, x_f(z) = x_mid + (z-z_mid)cot(dip)
  * below 45 degrees that plane would leave the cube through its top and bottom,
    so the fault is the grid plane k = n/2 with the z-layers shifted instead,
    z_f(x) = z_mid + (x-x_mid) tan(dip) (built as the (90-dip) mesh with x and z
    exchanged)
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

# Sub-stream numbers of the master seed (one independent stream per draw).
STREAM_LOGK = 1
STREAM_E = 2
STREAM_UPLIFT = 3
STREAM_FD = 4
STREAM_INJECTION = 5
STREAM_INSTANCES = 6

STATE_STICK = 0
STATE_SLIP = 1
STATE_OPEN = 2


def rng(seed: int, stream: int) -> np.random.Generator:
    """Independent PCG64 stream `stream` of master seed `seed`."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy=seed, spawn_key=(stream,))))


@dataclass(frozen=True)
class Params:
    """Scalar material, fluid, fault and time-step data (SI units)."""
    nu: float = 0.25             # Poisson ratio
    alpha: float = 1.0           # Biot coefficient
    biot_M: float = 22.7e9       # Biot modulus M [Pa]
    mu: float = 0.89e-3          # fluid viscosity [Pa s]
    k_par: float = 1e-12         # longitudinal fault permeability [m^2]
    k_perp: float = 1e-12        # transverse fault permeability [m^2]
    w0: float = 1e-3             # default hydraulic aperture [m]
    M_F: float = 0.2e6           # fracture Biot modulus [Pa]
    k_n: float = 8e13            # normal contact penalty [Pa/m]
    k_s: float = 8e12            # shear penalty [Pa/m]
    friction: float = 0.6        # Coulomb friction coefficient
    dt: float = 1.0              # time step [s]

    def as_tuple(self):
        return tuple(getattr(self, f.name) for f in dataclasses.fields(self))


@dataclass(frozen=True)
class Config:
    """One workload. Every reading of an unstated paper quantity is a named field."""
    name: str
    n: int                        # hexes per edge of the unit cube
    dip_deg: float = 90.0         # fault dip; 90 = vertical plane x = 0.5
    fault: bool = True
    heterogeneous: bool = False   # seeded log-normal k and uniform E per tet
    E0: float = 10e9              # nominal Young modulus [Pa]
    E_range: tuple = (5e9, 30e9)  # uniform E range when heterogeneous
    lnk_mean: float = math.log(1e-15)
    lnk_sigma: float = 1.0
    kn_factor: float = 1e3        # k_n = kn_factor * E0 / h
    ks_ratio: float = 0.1         # k_s = ks_ratio * k_n
    tn0: float = 20e6             # initial effective normal traction [Pa]
    stress_ratio: float = 0.55    # initial shear / (f * tn0)
    Q: float = 1e-3               # injection rate at the fault centre [m^3/s]
    n_steps: int = 1
    params: Params = field(default_factory=Params)


def config(idx: int) -> Config:
    """The five synthetic workloads, numbered 1..5."""
    p = Params()
    if idx == 1:
        n = 8
        return Config("cube8_vertical_fault", n, 90.0, params=_scaled(p, n, 1e3, 0.1, 10e9))
    if idx in (2, 4):
        n = 64
        return Config("cube64_dip60_hetero", n, 60.0, heterogeneous=True, n_steps=20 if idx == 2 else 1,
                      params=_scaled(p, n, 1e3, 0.1, 10e9))
    if idx == 3:
        n = 128
        return Config("cube128_dip60_hetero", n, 60.0, heterogeneous=True,
                      params=_scaled(p, n, 1e3, 0.1, 10e9))
    if idx == 5:
        n = 64
        return Config("cube64_dip60_hetero_batched", n, 60.0, heterogeneous=True,
                      params=_scaled(p, n, 1e3, 0.1, 10e9))
    raise ValueError(idx)


def cube_config(n: int, dip_deg: float = 90.0, heterogeneous: bool = False, name: str | None = None) -> Config:
    """A config-1-like cube at any resolution n (penalties rescaled with h = 1/n)."""
    p = _scaled(Params(), n, 1e3, 0.1, 10e9)
    return Config(name or f"cube{n}", n, dip_deg, heterogeneous=heterogeneous, params=p)


def _scaled(p: Params, n: int, kn_factor: float, ks_ratio: float, E0: float) -> Params:
    h = 1.0 / n
    kn = kn_factor * E0 / h
    return dataclasses.replace(p, k_n=kn, k_s=ks_ratio * kn)


@dataclass
class Mesh:
    nx: int
    ny: int
    nz: int
    xyz: np.ndarray        # f64 [N,3]
    tets: np.ndarray       # i32 [E,4]
    coh: np.ndarray        # i32 [F,6]
    pairs: np.ndarray      # i32 [P,2] (- node, + node)
    grid: np.ndarray       # i32 [N,3] (i,j,k) grid index of each node
    n_orig: int            # nodes before duplication

    @property
    def n_nodes(self):
        return self.xyz.shape[0]


def _node_id(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def make_mesh(nx: int, ny: int, nz: int, L=(1.0, 1.0, 1.0), fault_i: int | None = None,
              dip_deg: float = 90.0, lines=None) -> Mesh:
    """Structured Kuhn mesh of the box [0,Lx]x[0,Ly]x[0,Lz], optionally cut by a
    fault on the grid plane i = fault_i.  `lines` = (xs, ys, zs), increasing
    grid-line positions (nx+1, ny+1, nz+1 values), replaces the uniform spacing
    (a graded tensor-product grid; vertical faults only)."""
    Lx, Ly, Lz = L
    n_orig = (nx + 1) * (ny + 1) * (nz + 1)
    gi, gj, gk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    # node id = i + (nx+1)(j + (ny+1)k): transpose so that i varies fastest
    gi = gi.transpose(2, 1, 0).reshape(-1)
    gj = gj.transpose(2, 1, 0).reshape(-1)
    gk = gk.transpose(2, 1, 0).reshape(-1)
    grid = np.stack([gi, gj, gk], axis=1).astype(np.int32)

    # hex corners, hex index h = i + nx (j + ny k)
    hi, hj, hk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    hi = hi.transpose(2, 1, 0).reshape(-1)
    hj = hj.transpose(2, 1, 0).reshape(-1)
    hk = hk.transpose(2, 1, 0).reshape(-1)
    n_hex = hi.size
    perms = [((0, 1, 2), False), ((0, 2, 1), True), ((1, 0, 2), True),
             ((1, 2, 0), False), ((2, 0, 1), False), ((2, 1, 0), True)]
    tet_vi = np.empty((n_hex, 6, 4), dtype=np.int64)
    tet_vj = np.empty_like(tet_vi)
    tet_vk = np.empty_like(tet_vi)
    for t, (perm, odd) in enumerate(perms):
        off = np.zeros((4, 3), dtype=np.int64)
        off[1, perm[0]] = 1
        off[2] = off[1]
        off[2, perm[1]] = 1
        off[3] = 1
        if odd:
            off[[2, 3]] = off[[3, 2]]
        for v in range(4):
            tet_vi[:, t, v] = hi + off[v, 0]
            tet_vj[:, t, v] = hj + off[v, 1]
            tet_vk[:, t, v] = hk + off[v, 2]
    tets = _node_id(tet_vi, tet_vj, tet_vk, nx, ny)

    n_plane = (ny + 1) * (nz + 1)
    coh = np.zeros((0, 6), dtype=np.int32)
    pairs = np.zeros((0, 2), dtype=np.int32)
    if fault_i is not None:
        assert 0 < fault_i < nx
        plus_side = (hi >= fault_i)[:, None, None] & (tet_vi == fault_i)
        copy_id = n_orig + tet_vj + (ny + 1) * tet_vk
        tets = np.where(plus_side, copy_id, tets)
        cj, ck = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
        cj = cj.T.reshape(-1)
        ck = ck.T.reshape(-1)
        # two triangles per plane cell, both ordered so the normal points -x -> +x
        tri_j = np.stack([np.stack([cj, cj + 1, cj + 1], 1), np.stack([cj, cj + 1, cj], 1)], 1).reshape(-1, 3)
        tri_k = np.stack([np.stack([ck, ck, ck + 1], 1), np.stack([ck, ck + 1, ck + 1], 1)], 1).reshape(-1, 3)
        minus = _node_id(fault_i, tri_j, tri_k, nx, ny)
        plus = n_orig + tri_j + (ny + 1) * tri_k
        coh = np.concatenate([plus, minus], axis=1).astype(np.int32)
        pj, pk = np.meshgrid(np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
        pj = pj.T.reshape(-1)
        pk = pk.T.reshape(-1)
        pairs = np.stack([_node_id(fault_i, pj, pk, nx, ny), n_orig + pj + (ny + 1) * pk], 1).astype(np.int32)
        grid = np.concatenate([grid, np.stack([np.full(n_plane, fault_i), pj, pk], 1).astype(np.int32)])

    if lines is not None:
        xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in lines)
        if (xs.size, ys.size, zs.size) != (nx + 1, ny + 1, nz + 1) or abs(dip_deg - 90.0) > 1e-12:
            raise ValueError("grid lines need nx+1, ny+1, nz+1 positions and a vertical fault")
        if min(np.diff(xs).min(), np.diff(ys).min(), np.diff(zs).min()) <= 0:
            raise ValueError("grid lines must increase")
        xyz = np.stack([xs[grid[:, 0]], ys[grid[:, 1]], zs[grid[:, 2]]], axis=1)
        return Mesh(nx, ny, nz, np.ascontiguousarray(xyz), np.ascontiguousarray(tets.reshape(-1, 4), dtype=np.int32),
                    coh, pairs, grid, n_orig)

    # coordinates, with the column-shift map for a dipping fault
    fi = grid[:, 0].astype(np.float64)
    z = grid[:, 2] * (Lz / nz)
    y = grid[:, 1] * (Ly / ny)
    if fault_i is not None and abs(dip_deg - 90.0) > 1e-12:
        x_mid = fault_i * Lx / nx
        xf = x_mid + (z - 0.5 * Lz) / math.tan(math.radians(dip_deg))
        if not (np.all(xf > 0) and np.all(xf < Lx)):
            raise ValueError(f"a fault dipping {dip_deg} degrees leaves the box through its side faces")
        x = np.where(fi <= fault_i, xf * fi / fault_i, xf + (Lx - xf) * (fi - fault_i) / (nx - fault_i))
    else:
        x = fi * (Lx / nx)
    xyz = np.stack([x, y, z], axis=1)
    return Mesh(nx, ny, nz, np.ascontiguousarray(xyz, dtype=np.float64),
                np.ascontiguousarray(tets.reshape(-1, 4), dtype=np.int32), coh, pairs, grid, n_orig)


@dataclass
class Instance:
    """Everything one solve needs, as flat numpy arrays."""
    cfg: Config
    mesh: Mesh
    params: Params
    E: np.ndarray            # f64 [E]   Young modulus per tet
    logk: np.ndarray         # f64 [E]   ln(matrix permeability) per tet
    dir_u: np.ndarray        # u8 [3N]   1 = displacement DOF held at zero
    dir_p: np.ndarray        # u8 [N]    1 = pressure DOF held at zero
    source: np.ndarray       # f64 [N]   volumetric source per node [m^3/s]
    load: np.ndarray         # f64 [3N]  external nodal force increment [N]
    t0: np.ndarray           # f64 [F*3,3] initial effective traction per qp (t'_n, t'_s1, t'_s2)
    centre_pair: tuple = (0, 0)

    @property
    def n_nodes(self):
        return self.mesh.n_nodes


def swap_xz(mesh: Mesh) -> Mesh:
    """The mesh mirrored through the plane x = z (coordinates and grid indices
    exchanged), with tetrahedra and interface triangles re-oriented."""
    xyz = np.ascontiguousarray(mesh.xyz[:, [2, 1, 0]])
    tets = np.ascontiguousarray(mesh.tets[:, [0, 1, 3, 2]])
    coh = np.ascontiguousarray(mesh.coh[:, [0, 2, 1, 3, 5, 4]]) if mesh.coh.size else mesh.coh
    grid = np.ascontiguousarray(mesh.grid[:, [2, 1, 0]])
    return Mesh(mesh.nz, mesh.ny, mesh.nx, xyz, tets, coh, mesh.pairs, grid, mesh.n_orig)


def make_instance(cfg: Config, seed: int = 0) -> Instance:
    n = cfg.n
    if cfg.fault and cfg.dip_deg < 45.0:
        mesh = swap_xz(make_mesh(n, n, n, fault_i=n // 2, dip_deg=90.0 - cfg.dip_deg))
    else:
        mesh = make_mesh(n, n, n, fault_i=n // 2 if cfg.fault else None, dip_deg=cfg.dip_deg)
    ne = mesh.tets.shape[0]
    if cfg.heterogeneous:
        logk = rng(seed, STREAM_LOGK).normal(cfg.lnk_mean, cfg.lnk_sigma, size=ne)
        E = rng(seed, STREAM_E).uniform(cfg.E_range[0], cfg.E_range[1], size=ne)
    else:
        logk = np.full(ne, cfg.lnk_mean)
        E = np.full(ne, cfg.E0)
    N = mesh.n_nodes
    dir_u = np.zeros(3 * N, dtype=np.uint8)
    bottom = np.nonzero(mesh.grid[:, 2] == 0)[0]
    for c in range(3):
        dir_u[3 * bottom + c] = 1
    dir_p = np.zeros(N, dtype=np.uint8)
    source = np.zeros(N, dtype=np.float64)
    centre = (0, 0)
    t0 = np.zeros((mesh.coh.shape[0] * 3, 3), dtype=np.float64)
    if cfg.fault:
        c = n // 2
        pid = c + (n + 1) * c          # plane node (j,k) = (n/2, n/2)
        centre = (int(mesh.pairs[pid, 0]), int(mesh.pairs[pid, 1]))
        source[centre[0]] += 0.5 * cfg.Q
        source[centre[1]] += 0.5 * cfg.Q
        t0[:, 0] = cfg.tn0
        t0[:, 1] = cfg.stress_ratio * cfg.params.friction * cfg.tn0
    return Instance(cfg, mesh, cfg.params, np.ascontiguousarray(E), np.ascontiguousarray(logk),
                    dir_u, dir_p, source, np.zeros(3 * N), t0, centre)


def uplift_nodes(inst: Instance, count: int = 32, seed: int = 0) -> np.ndarray:
    """Seeded top-surface nodes whose vertical displacement enters the adjoint objective."""
    top = np.nonzero(inst.mesh.grid[:, 2] == inst.mesh.nz)[0]
    top = top[top < inst.mesh.n_orig]
    return np.sort(rng(seed, STREAM_UPLIFT).choice(top, size=count, replace=False)).astype(np.int32)


def fd_directions(n_params: int, count: int = 20, seed: int = 0, unit: bool = True) -> np.ndarray:
    """Random directions for finite-difference gradient checks: independent standard
    normal components, normalised to unit length unless unit is False (then a step h
    moves every parameter by about h)."""
    d = rng(seed, STREAM_FD).standard_normal((count, n_params))
    return d / np.linalg.norm(d, axis=1, keepdims=True) if unit else d


def injection_scenarios(inst: Instance, count: int = 32, seed: int = 0):
    """Seeded interior fault pairs and log-uniform rates in [1e-4, 1e-2] m^3/s."""
    g = rng(seed, STREAM_INJECTION)
    m = inst.mesh
    pg = m.grid[m.pairs[:, 0]]
    interior = np.nonzero((pg[:, 1] > 0) & (pg[:, 1] < m.ny) & (pg[:, 2] > 0) & (pg[:, 2] < m.nz))[0]
    sel = g.choice(interior, size=count, replace=False)
    rates = np.exp(g.uniform(math.log(1e-4), math.log(1e-2), size=count))
    return m.pairs[sel], rates


def source_matrix(inst: Instance, pairs: np.ndarray, rates: np.ndarray) -> np.ndarray:
    """[count, N] source vectors, each rate split equally over its node pair."""
    S = np.zeros((len(rates), inst.n_nodes))
    for c, ((a, b), q) in enumerate(zip(pairs, rates)):
        S[c, a] += 0.5 * q
        S[c, b] += 0.5 * q
    return S


def batched_configs(count: int = 48, seed: int = 0, n_range=(16, 48), dip_range=(30.0, 90.0)):
    """Seeded uneven instances: n ~ U{n_range}, dip ~ U[dip_range], heterogeneous."""
    g = rng(seed, STREAM_INSTANCES)
    ns = g.integers(n_range[0] // 2, n_range[1] // 2 + 1, size=count) * 2     # even n: the fault sits at n/2
    dips = g.uniform(dip_range[0], dip_range[1], size=count)
    return [cube_config(int(n), dip_deg=float(d), heterogeneous=True, name=f"batch{i}_n{n}_dip{d:.1f}")
            for i, (n, d) in enumerate(zip(ns, dips))]


@dataclass
class Batch:
    """Several instances concatenated into one disjoint mesh; group[node] = instance."""
    instances: list
    xyz: np.ndarray
    tets: np.ndarray
    coh: np.ndarray
    group: np.ndarray
    dir_u: np.ndarray
    dir_p: np.ndarray
    E: np.ndarray
    logk: np.ndarray
    source: np.ndarray
    t0: np.ndarray
    node_off: np.ndarray
    tet_off: np.ndarray
    coh_off: np.ndarray


def concat_instances(instances) -> Batch:
    node_off = np.cumsum([0] + [i.n_nodes for i in instances])
    tet_off = np.cumsum([0] + [i.mesh.tets.shape[0] for i in instances])
    coh_off = np.cumsum([0] + [i.mesh.coh.shape[0] for i in instances])
    cat = lambda xs: np.ascontiguousarray(np.concatenate(xs))
    return Batch(
        instances,
        cat([i.mesh.xyz for i in instances]),
        cat([i.mesh.tets + o for i, o in zip(instances, node_off)]).astype(np.int32),
        cat([i.mesh.coh + o for i, o in zip(instances, node_off)]).astype(np.int32),
        cat([np.full(i.n_nodes, g, np.int32) for g, i in enumerate(instances)]),
        cat([i.dir_u for i in instances]), cat([i.dir_p for i in instances]),
        cat([i.E for i in instances]), cat([i.logk for i in instances]),
        cat([i.source for i in instances]), cat([i.t0 for i in instances]),
        node_off, tet_off, coh_off)


# ------------------------------------------------------------ injection into a frictional fault (Sec. 4.2)
SLIP_BENCHMARK = dict(
    E=60e9, nu=0.0, alpha=0.0, biot_M=1e14, mu=0.89e-3, friction=0.6,   # Table 1 (M = 1e5 GPa, k_M = 0)
    k_n=6e12, k_s=6e11,            # Table 1 normal / shear stiffness, printed in GPa, read as Pa/m
    wk_par=1e-15, M_F=0.2e6,       # Table 1 transmissibility w k_par [m^3], fracture Biot modulus [Pa]
    sigma0=80e6, Q=1e-6,           # Sec. 4.2 normal load [Pa], injection 0.06 L/min [m^3/s]
    tau0_CS=47.999e6, tau0_MP=47.830e6)


def graded_lines(h: float, n_fine: int, n_grade: int, ratio: float, centre: float = 0.0) -> np.ndarray:
    """Grid-line positions symmetric about `centre`: n_fine cells of width h
    (n_fine even) around it, then n_grade cells on each side, each `ratio`
    times wider than the one before."""
    assert n_fine % 2 == 0
    w = [h] * (n_fine // 2) + [h * ratio ** (k + 1) for k in range(n_grade)]
    half = np.concatenate([[0.0], np.cumsum(w)])
    return np.concatenate([centre - half[:0:-1], centre + half])


def slip_benchmark_instance(tau0: float, h: float = 0.1, n_fine: int = 16, n_grade: int = 6, ratio: float = 1.5,
                            nx_fine: int = 2, nx_grade: int = 7, dt: float = 1.0, k_perp: float = 1e-11,
                            w0: float = 1e-3) -> Instance:
    """The injection-into-a-frictional-fault workload of Sec. 4.2 on a graded box.

    The paper's horizontal fault with shear along x is turned so that the fault is
    the vertical grid plane through the box centre (normal +x) and the initial
    shear acts along t1 (+z); with nu = 0 and isotropic elasticity the turn
    changes nothing.  Cells are h wide over the central n_fine x n_fine patch of
    the fault and grow by `ratio` outwards; across the fault the first nx_fine/2
    cells on each side are h wide.  Table 1 materials: impermeable matrix
    (ln k = ln 1e-30) with alpha = 0 and a stiff Biot modulus, fault flow only
    (w0 k_par = 1e-15 m^3 with w0 = 1 mm, k_perp = 1e-11 m^2 so that the two lips'
    pressures move together), penalties k_n, k_s, friction 0.6.  Initial
    tractions t'_n0 = sigma0 = 80 MPa and t'_s0 = tau0 along t1; injection
    Q = 0.06 L/min split over the centre node pair.  The face x = 0 (parallel to
    the fault, on its - side) is clamped: it removes the rigid-body modes of the
    increment problem, as the paper's restraints on its bottom face do."""
    b = SLIP_BENCHMARK
    xs = graded_lines(h, nx_fine, nx_grade, ratio)
    ys = graded_lines(h, n_fine, n_grade, ratio)
    xs, ys = xs - xs[0], ys - ys[0]
    nx, ny = xs.size - 1, ys.size - 1
    mesh = make_mesh(nx, ny, ny, (xs[-1], ys[-1], ys[-1]), fault_i=nx // 2, lines=(xs, ys, ys))
    prm = Params(nu=b["nu"], alpha=b["alpha"], biot_M=b["biot_M"], mu=b["mu"], k_par=b["wk_par"] / w0,
                 k_perp=k_perp, w0=w0, M_F=b["M_F"], k_n=b["k_n"], k_s=b["k_s"], friction=b["friction"], dt=dt)
    cfg = Config(f"slip_benchmark_tau{tau0 / 1e6:.3f}", ny, 90.0, E0=b["E"], tn0=b["sigma0"],
                 stress_ratio=tau0 / (b["friction"] * b["sigma0"]), Q=b["Q"], params=prm)
    ne, N = mesh.tets.shape[0], mesh.n_nodes
    dir_u = np.zeros(3 * N, dtype=np.uint8)
    face = np.nonzero(mesh.grid[:, 0] == 0)[0]
    for c in range(3):
        dir_u[3 * face + c] = 1
    pid = ny // 2 + (ny + 1) * (ny // 2)
    centre = (int(mesh.pairs[pid, 0]), int(mesh.pairs[pid, 1]))
    source = np.zeros(N)
    source[list(centre)] = 0.5 * b["Q"]
    t0 = np.zeros((mesh.coh.shape[0] * 3, 3))
    t0[:, 0] = b["sigma0"]
    t0[:, 1] = tau0
    return Instance(cfg, mesh, prm, np.full(ne, b["E"]), np.full(ne, math.log(1e-30)), dir_u,
                    np.zeros(N, dtype=np.uint8), source, np.zeros(3 * N), t0, centre)


# ------------------------------------------------------------ Cryer's sphere (Sec. 4.1)
def sphere_octant_mesh(n: int, R: float = 1.0) -> Mesh:
    """One octant (x, y, z >= 0) of a ball of radius R: the structured Kuhn mesh of
    the unit cube with grid node v = (i, j, k) / n moved to R max(v) v / |v|, so
    that every cube shell max(v) = m becomes the sphere of radius R m and the
    three faces max(v) = 1 the spherical surface."""
    m = make_mesh(n, n, n)
    v = m.grid.astype(np.float64) / n
    norm = np.linalg.norm(v, axis=1)
    scale = np.where(norm > 0, v.max(axis=1) / np.where(norm > 0, norm, 1.0), 0.0)
    m.xyz = np.ascontiguousarray(R * v * scale[:, None])
    return m


def sphere_surface_triangles(mesh: Mesh) -> np.ndarray:
    """[T, 3] node triples of the tetrahedron faces on the spherical surface
    (all three nodes on the shell max(i, j, k) = n), ordered so that the right-hand
    normal points out of the ball."""
    n = mesh.nx
    shell = mesh.grid.max(axis=1) == n
    tris = []
    for t in mesh.tets:
        for drop in range(4):
            f = np.delete(t, drop)
            if shell[f].all():
                a, b, c = mesh.xyz[f]
                if np.dot(np.cross(b - a, c - a), a - mesh.xyz[t[drop]]) < 0:
                    f = f[[0, 2, 1]]
                tris.append(f)
    return np.array(tris, dtype=np.int64)


def cryer_instance(n: int, R: float = 1.0, F: float = 1e6, E: float = 10e9, nu: float = 0.25, alpha: float = 1.0,
                   biot_M: float = 22.7e9, k: float = 1e-15, mu: float = 0.89e-3, dt: float = 1.0) -> Instance:
    """Cryer's problem of Sec. 4.1 on one octant of the sphere: a saturated
    poroelastic ball, drained (p = 0) on its surface, loaded at t = 0+ by a
    uniform compressive surface pressure F held constant.  The three symmetry
    planes x = 0, y = 0, z = 0 carry no normal displacement and no flux.  No
    fault.  The load is the consistent nodal force of the pressure F on the
    surface triangles (F area / 3 per vertex, along the inward normal), the total
    external force change F_u of every step."""
    mesh = sphere_octant_mesh(n, R)
    N, ne = mesh.n_nodes, mesh.tets.shape[0]
    prm = Params(nu=nu, alpha=alpha, biot_M=biot_M, mu=mu, dt=dt)
    cfg = Config(f"cryer_octant{n}", n, fault=False, E0=E, lnk_mean=math.log(k), Q=0.0, params=prm)
    dir_u = np.zeros(3 * N, dtype=np.uint8)
    for c in range(3):
        dir_u[3 * np.nonzero(mesh.grid[:, c] == 0)[0] + c] = 1
    dir_p = (mesh.grid.max(axis=1) == n).astype(np.uint8)
    load = np.zeros((N, 3))
    for f in sphere_surface_triangles(mesh):
        a, b, c = mesh.xyz[f]
        an = 0.5 * np.cross(b - a, c - a)          # area times outward unit normal
        for v in f:
            load[v] -= F * an / 3.0
    return Instance(cfg, mesh, prm, np.full(ne, E), np.full(ne, math.log(k)), dir_u, dir_p, np.zeros(N),
                    np.ascontiguousarray(load.reshape(-1)), np.zeros((0, 3)), (0, 0))
