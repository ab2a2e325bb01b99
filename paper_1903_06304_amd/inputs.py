"""Seeded synthetic inputs: logically structured quadrilateral meshes (periodic, or with
boundary faces), their geometry nodes and grid velocities, and initial primitive fields
(p, u, v, T).

This module is shared by the CPU oracle tests, the GPU tests and the benchmark.
It holds no arithmetic of the discretisation itself: it only places mesh nodes,
evaluates analytic maps and analytic initial fields, and draws random numbers.

Conventions (also those of the C ABI):
  * element e = ix + nx*iy on an nx-by-ny logically structured mesh, periodic in a
    direction unless that direction's two sides carry boundary codes;
  * a boundary face has a negative neighbour entry: BC_FARFIELD (-1), BC_SLIP_WALL
    (-2), BC_NOSLIP_WALL (-3) (adiabatic); its nbr_face entry is -1;
  * local faces 0: xi=-1, 1: xi=+1, 2: eta=-1, 3: eta=+1; face point k runs
    along the face (eta index on faces 0/1, xi index on faces 2/3);
  * geometry nodes: Gauss-Lobatto tensor grid of degree pg, node (a, b) at index
    a + (pg+1)*b, a along xi; arrays [2][E][(pg+1)^2] (x then y);
  * solution points: Gauss-Legendre tensor grid, point (i, j) at index i + n*j;
  * state arrays [4][E][Np], variables (p, u, v, T).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

GAMMA = 1.4
PRANDTL = 0.72

BC_FARFIELD = -1
BC_SLIP_WALL = -2
BC_NOSLIP_WALL = -3


def gl_points(n: int) -> np.ndarray:
    """n Gauss-Legendre points on [-1, 1] (where the unknowns live)."""
    return np.polynomial.legendre.leggauss(n)[0]


def gll_points(n: int) -> np.ndarray:
    """n Gauss-Lobatto points on [-1, 1] (geometry node positions)."""
    if n < 2:
        raise ValueError("need at least 2 Gauss-Lobatto points")
    if n == 2:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots().real
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


# --------------------------------------------------------------------------
# mesh maps: (xr, yr, t) -> (x, y, u_g, v_g), xr/yr the undeformed coordinates
# --------------------------------------------------------------------------
MapFn = Callable[[np.ndarray, np.ndarray, float], tuple]


def map_affine(xr, yr, t):
    z = np.zeros_like(xr)
    return xr.copy(), yr.copy(), z, z.copy()


def map_curved(amp: float = 0.1) -> MapFn:
    """Static curved map x = xi + a sin(xi) sin(eta), y = eta + a sin(xi) sin(eta)."""
    def f(xr, yr, t):
        d = amp * np.sin(xr) * np.sin(yr)
        z = np.zeros_like(xr)
        return xr + d, yr + d, z, z.copy()
    return f


def map_deforming(amp: float = 0.05, scale: float = 1.0) -> MapFn:
    """Deforming map x = xr + s*a sin(pi xr/s) sin(pi yr/s) sin(2 pi t) (same for y).

    scale=1 is periodic on [0,2]^2; scale=pi on [0, 2 pi]^2.
    """
    def f(xr, yr, t):
        shape = np.sin(np.pi * xr / scale) * np.sin(np.pi * yr / scale)
        d = scale * amp * shape * np.sin(2.0 * np.pi * t)
        vel = scale * amp * shape * 2.0 * np.pi * np.cos(2.0 * np.pi * t)
        return xr + d, yr + d, vel, vel.copy()
    return f


def map_annulus(r0: float = 0.5, r1: float = 50.0) -> MapFn:
    """O-grid around a cylinder of radius r0 out to radius r1, for a reference domain
    [0, 1]^2: the angle runs clockwise with xr (periodic in xr, positive Jacobian), the
    radius grows geometrically with yr (eta = -1 sides of the first row on the cylinder,
    eta = +1 sides of the last row on the outer circle)."""
    def f(xr, yr, t):
        th = -2.0 * np.pi * xr
        r = r0 * (r1 / r0) ** yr
        z = np.zeros_like(xr)
        return r * np.cos(th), r * np.sin(th), z, z.copy()
    return f


def map_vortex_motion(a: float = 1.0, fn: float = 1.0, fx: float = 0.1, fy: float = 0.1) -> MapFn:
    """Prescribed sinusoidal grid motion of the isentropic-vortex case (paper Sec. 4.3)."""
    def f(xr, yr, t):
        shape = np.sin(2 * np.pi * fx * xr) * np.sin(2 * np.pi * fy * yr)
        d = a * np.sin(2 * np.pi * fn * t) * shape
        vel = a * 2 * np.pi * fn * np.cos(2 * np.pi * fn * t) * shape
        return xr + d, yr + d, vel, vel.copy()
    return f


@dataclasses.dataclass
class Mesh:
    nx: int
    ny: int
    p: int
    domain: tuple = (0.0, 1.0, 0.0, 1.0)
    mapping: MapFn = map_affine
    moving: bool = False
    pg: Optional[int] = None
    # boundary codes of the sides (xi = -1, xi = +1, eta = -1, eta = +1) of the logical
    # rectangle; 0 on both sides of a direction makes it periodic
    bc: tuple = (0, 0, 0, 0)

    def __post_init__(self):
        if self.pg is None:
            self.pg = self.p
        self.pg = max(1, self.pg)
        b = tuple(int(x) for x in self.bc)
        if len(b) != 4 or any(x not in (0, BC_FARFIELD, BC_SLIP_WALL, BC_NOSLIP_WALL) for x in b):
            raise ValueError(f"boundary codes must be 0 or -1..-3: {self.bc}")
        if (b[0] == 0) != (b[1] == 0) or (b[2] == 0) != (b[3] == 0):
            raise ValueError("a direction is either periodic on both sides or bounded on both")
        self.bc = b

    @property
    def n(self):
        return self.p + 1

    @property
    def Np(self):
        return self.n * self.n

    @property
    def E(self):
        return self.nx * self.ny

    @property
    def ng(self):
        return (self.pg + 1) ** 2

    def connectivity(self):
        """Face table (nbr[E,4] int32, nbr_face[E,4] int32, flip[E,4] int8); boundary faces
        carry their (negative) code in nbr and -1 in nbr_face."""
        nx, ny = self.nx, self.ny
        e = np.arange(nx * ny)
        ix, iy = e % nx, e // nx
        nbr = np.stack([
            (ix - 1) % nx + nx * iy,
            (ix + 1) % nx + nx * iy,
            ix + nx * ((iy - 1) % ny),
            ix + nx * ((iy + 1) % ny),
        ], axis=1).astype(np.int32)
        nbr_face = np.tile(np.array([1, 0, 3, 2], np.int32), (nx * ny, 1))
        edge = [ix == 0, ix == nx - 1, iy == 0, iy == ny - 1]
        for f in range(4):
            if self.bc[f]:
                nbr[edge[f], f] = self.bc[f]
                nbr_face[edge[f], f] = -1
        flip = np.zeros((nx * ny, 4), np.int8)
        return nbr, nbr_face, flip

    def _ref_coords(self, r1d: np.ndarray):
        """Undeformed coordinates of a tensor grid r1d x r1d in every element: [E][m*m]."""
        x0, x1, y0, y1 = self.domain
        hx, hy = (x1 - x0) / self.nx, (y1 - y0) / self.ny
        e = np.arange(self.E)
        ix, iy = e % self.nx, e // self.nx
        m = len(r1d)
        a = np.tile(r1d, m)              # index a + m*b -> xi = r1d[a]
        b = np.repeat(r1d, m)
        xr = x0 + hx * (ix[:, None] + 0.5 * (a[None, :] + 1.0))
        yr = y0 + hy * (iy[:, None] + 0.5 * (b[None, :] + 1.0))
        return xr, yr

    def nodes(self, t: float = 0.0):
        """Geometry nodes [2][E][(pg+1)^2] and node velocities (None if static)."""
        xr, yr = self._ref_coords(gll_points(self.pg + 1))
        x, y, ug, vg = self.mapping(xr, yr, t)
        xg = np.ascontiguousarray(np.stack([x, y]))
        vgs = np.ascontiguousarray(np.stack([ug, vg])) if self.moving else None
        return xg, vgs

    def solution_points(self, t: float = 0.0):
        """Physical coordinates of the solution points from the analytic map: [2][E][Np]."""
        xr, yr = self._ref_coords(gl_points(self.n))
        x, y, _, _ = self.mapping(xr, yr, t)
        return np.stack([x, y])


def _local_rotation(m: int, k: int):
    """Index map of a tensor grid of m x m points when an element's local frame turns by k
    quarter turns: new index (a', b') -> old index (a, b), as an array over a' + m b'."""
    ap, bp = np.meshgrid(np.arange(m), np.arange(m), indexing="xy")
    ap, bp = ap.reshape(-1), bp.reshape(-1)
    a, b = ap, bp
    for _ in range(k % 4):
        # one quarter turn: xi = -eta', eta = xi'
        a, b = m - 1 - b, a
    return a + m * b


def _face_map(k: int):
    """For each new local face F of an element turned by k quarter turns: the old face it
    is and whether its points run in the opposite order ((old face, reversed) pairs)."""
    m = 3
    perm = _local_rotation(m, k)
    out = []
    for F in range(4):
        new = [(0, j) if F == 0 else (m - 1, j) if F == 1 else (j, 0) if F == 2 else (j, m - 1) for j in range(m)]
        old = [(perm[a + m * b] % m, perm[a + m * b] // m) for a, b in new]
        for f in range(4):
            on = [(a == 0) if f == 0 else (a == m - 1) if f == 1 else (b == 0) if f == 2 else (b == m - 1)
                  for a, b in old]
            if all(on):
                along = [b if f < 2 else a for a, b in old]
                out.append((f, along[0] > along[-1]))
                break
    return out


def renumber_elements(nbr, nbr_face, flip, rot):
    """The same mesh with element e's local frame turned by rot[e] quarter turns: the face
    table (nbr, nbr_face, flip) of the new numbering, and a function that carries arrays
    [k][E][m*m] of the old numbering (geometry nodes, states) to the new one.  Exercises
    neighbour faces other than the opposite one and reversed face-point order."""
    E = nbr.shape[0]
    rot = np.asarray(rot, dtype=np.int64) % 4
    maps = [_face_map(k) for k in range(4)]
    inv = [{f: F for F, (f, _) in enumerate(mp)} for mp in maps]
    nb2 = np.empty_like(nbr)
    nf2 = np.empty_like(nbr_face)
    fl2 = np.zeros_like(flip)
    for e in range(E):
        for F in range(4):
            f, rev = maps[rot[e]][F]
            m = nbr[e, f]
            if m < 0:
                nb2[e, F], nf2[e, F] = m, -1
                continue
            G = inv[rot[m]][nbr_face[e, f]]
            nb2[e, F], nf2[e, F] = m, G
            fl2[e, F] = int(flip[e, f]) ^ int(rev) ^ int(maps[rot[m]][G][1])

    def carry(arr):
        arr = np.asarray(arr)
        npts = arr.shape[-1]
        mm = int(round(math.sqrt(npts)))
        out = np.empty_like(arr)
        for e in range(E):
            out[..., e, :] = arr[..., e, _local_rotation(mm, rot[e])]
        return out

    return nb2, nf2, fl2, carry


# --------------------------------------------------------------------------
# physical parameters
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Params:
    order: int
    n_elem: int
    mach_ref: float
    reynolds: float = 1.0
    viscous: bool = False
    moving: bool = False
    kappa: float = 1.0
    mach_inf: Optional[float] = None
    gamma: float = GAMMA
    prandtl: float = PRANDTL
    mu: float = 1.0
    geom_order: Optional[int] = None

    def __post_init__(self):
        if self.mach_inf is None:
            self.mach_inf = self.mach_ref
        if self.geom_order is None:
            self.geom_order = self.order

    @property
    def gas_constant(self):
        return 1.0 / (self.gamma * self.mach_ref ** 2)

    @property
    def cp(self):
        return 1.0 / ((self.gamma - 1.0) * self.mach_ref ** 2)


# --------------------------------------------------------------------------
# initial fields (analytic / seeded random); all return q[4][E][Np]
# --------------------------------------------------------------------------
def uniform_flow(mesh: Mesh, prm: Params, u=math.sqrt(0.5), v=math.sqrt(0.5), rho=1.0, T=1.0):
    q = np.empty((4, mesh.E, mesh.Np))
    q[0] = rho * prm.gas_constant * T
    q[1], q[2], q[3] = u, v, T
    return q


def isentropic_vortex(mesh: Mesh, prm: Params, t=0.0, alpha=5.0, phi=0.5, center=(5.0, 5.0),
                      vinf=(math.sqrt(0.5), math.sqrt(0.5)), xy=None):
    """Isentropic vortex (paper Eq. VP_Solution) in the non-dimensionalisation of Sec. 2.1, Eq. (comp_ns).

    T_inf = rho_inf = 1, |v_inf| = 1, r the Euclidean distance to the (advected)
    centre; the temperature dip is written with Cp so that it holds for R = 1/(gamma Ma^2);
    rho = T^(1/(gamma-1)) (isentropic), p = rho R T. The nearest periodic image
    of the centre is used.
    """
    if xy is None:
        xy = mesh.solution_points(t)
    x, y = xy
    x0, x1, y0, y1 = mesh.domain
    Lx, Ly = x1 - x0, y1 - y0
    cx = center[0] + vinf[0] * t
    cy = center[1] + vinf[1] * t
    dx = (x - cx + 0.5 * Lx) % Lx - 0.5 * Lx
    dy = (y - cy + 0.5 * Ly) % Ly - 0.5 * Ly
    r2 = dx * dx + dy * dy
    ex = np.exp(phi * (1.0 - r2))
    du = -alpha / (2 * np.pi) * dy * ex
    dv = alpha / (2 * np.pi) * dx * ex
    dT = -alpha ** 2 / (16.0 * phi * np.pi ** 2 * prm.cp) * ex * ex
    T = 1.0 + dT
    rho = T ** (1.0 / (prm.gamma - 1.0))
    q = np.empty((4,) + x.shape)
    q[0] = rho * prm.gas_constant * T
    q[1] = vinf[0] + du
    q[2] = vinf[1] + dv
    q[3] = T
    return q


def taylor_green(mesh: Mesh, prm: Params, xy=None):
    """Taylor-Green field: u = sin x cos y, v = -cos x sin y, p = p_inf + (cos2x + cos2y)/4, T = 1."""
    if xy is None:
        xy = mesh.solution_points()
    x, y = xy
    q = np.empty((4,) + x.shape)
    q[0] = prm.gas_constant + 0.25 * (np.cos(2 * x) + np.cos(2 * y))
    q[1] = np.sin(x) * np.cos(y)
    q[2] = -np.cos(x) * np.sin(y)
    q[3] = 1.0
    return q


def _fourier_modes(kmax: int):
    ks = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
          if (kx, ky) != (0, 0)]
    return np.array(ks, dtype=float)


def _mode_sum(x, y, x0, y0, Lx, Ly, ks, coef, kmax):
    """sum_k Re(coef_k exp(i (2 pi kx (x - x0)/Lx + 2 pi ky (y - y0)/Ly))), evaluated with
    the separable factors exp(i 2 pi kx x / Lx) and exp(i 2 pi ky y / Ly)."""
    n = 2 * kmax + 1
    C = np.zeros((n, n), dtype=complex)
    for (kx, ky), c in zip(ks.astype(int), coef):
        C[kx + kmax, ky + kmax] += c
    ex = np.exp(1j * 2 * np.pi * np.outer(np.arange(-kmax, kmax + 1), (x - x0).ravel() / Lx))
    ey = np.exp(1j * 2 * np.pi * np.outer(np.arange(-kmax, kmax + 1), (y - y0).ravel() / Ly))
    return np.real(np.sum(ex * (C @ ey), axis=0)).reshape(x.shape)


def random_scalar_field(mesh: Mesh, rng: np.random.Generator, kmax: int = 4, xy=None):
    """Unit-RMS smooth periodic random field sum_k a_k cos(k.x + phase_k), |k|_inf <= kmax."""
    if xy is None:
        xy = mesh.solution_points()
    x, y = xy
    x0, x1, y0, y1 = mesh.domain
    ks = _fourier_modes(kmax)
    amp = rng.standard_normal(len(ks)) / np.maximum(1.0, np.hypot(ks[:, 0], ks[:, 1]))
    ph = rng.uniform(0, 2 * np.pi, len(ks))
    f = _mode_sum(x, y, x0, y0, x1 - x0, y1 - y0, ks, amp * np.exp(1j * ph), kmax)
    return f / np.sqrt(np.mean(f * f))


def random_solenoidal_velocity(mesh: Mesh, rng: np.random.Generator, rms: float, kmax: int = 4, xy=None):
    """Smooth periodic divergence-free velocity from a random stream function.

    psi = sum_k (a_k/|k|^2) sin(k.x + phase_k), a_k ~ N(0,1); (u, v) = (psi_y, -psi_x),
    scaled to the given RMS speed.
    """
    if xy is None:
        xy = mesh.solution_points()
    x, y = xy
    x0, x1, y0, y1 = mesh.domain
    Lx, Ly = x1 - x0, y1 - y0
    ks = _fourier_modes(kmax)
    a = rng.standard_normal(len(ks))
    ph = rng.uniform(0, 2 * np.pi, len(ks))
    base = a / (ks[:, 0] ** 2 + ks[:, 1] ** 2) * np.exp(1j * ph)
    u = _mode_sum(x, y, x0, y0, Lx, Ly, ks, base * (2 * np.pi * ks[:, 1] / Ly), kmax)
    v = -_mode_sum(x, y, x0, y0, Lx, Ly, ks, base * (2 * np.pi * ks[:, 0] / Lx), kmax)
    scale = rms / np.sqrt(np.mean(u * u + v * v) / 2.0 + 1e-300)
    return u * scale, v * scale


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Case:
    name: str
    mesh: Mesh
    prm: Params
    q: np.ndarray
    q_nm1: Optional[np.ndarray] = None
    dt: float = 0.01
    t: float = 0.0
    krylov: int = 30
    extra: dict = dataclasses.field(default_factory=dict)

    def connectivity(self):
        return self.mesh.connectivity()

    def nodes(self, t=None):
        return self.mesh.nodes(self.t if t is None else t)


def config_c1(nx: int = 8, p: int = 2) -> Case:
    """Euler p=2, 8x8 affine periodic on [0,10]^2, isentropic vortex, Ma=0.1, kappa=0."""
    mesh = Mesh(nx, nx, p, (0.0, 10.0, 0.0, 10.0))
    prm = Params(order=p, n_elem=mesh.E, mach_ref=0.1, viscous=False, kappa=0.0)
    dt = 0.01
    q = isentropic_vortex(mesh, prm, t=0.0)
    q_nm1 = isentropic_vortex(mesh, prm, t=-dt)
    return Case("c1_euler_vortex_p2_8x8", mesh, prm, q, q_nm1, dt=dt, krylov=20)


def config_c2(nx: int = 64, p: int = 3, mach: float = 0.05) -> Case:
    """NS p=3, 64x64 curved static mesh on [0,2pi]^2, Taylor-Green, Ma=0.05, Re=100."""
    mesh = Mesh(nx, nx, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi), map_curved(0.1))
    prm = Params(order=p, n_elem=mesh.E, mach_ref=mach, reynolds=100.0, viscous=True, kappa=1.0)
    q = taylor_green(mesh, prm)
    return Case(f"c2_ns_taylor_green_p{p}_{nx}x{nx}_curved", mesh, prm, q)


def config_c3(nx: int = 128, p: int = 3, perturbed: bool = True, seed: int = 3) -> Case:
    """NS p=3, 128x128 deforming mesh on [0,2]^2, free stream Ma=0.01, Re=100 (+ perturbation)."""
    mesh = Mesh(nx, nx, p, (0.0, 2.0, 0.0, 2.0), map_deforming(0.05, 1.0), moving=True)
    prm = Params(order=p, n_elem=mesh.E, mach_ref=0.01, reynolds=100.0, viscous=True,
                 moving=True, kappa=1.0)
    q = uniform_flow(mesh, prm)
    if perturbed:
        rng = np.random.default_rng(seed)
        du, dv = random_solenoidal_velocity(mesh, rng, rms=1e-3)
        q[1] += du
        q[2] += dv
    return Case(f"c3_ns_deforming_p{p}_{nx}x{nx}", mesh, prm, q, None, dt=0.01)


def config_c4(nx: int = 256, p: int = 3, seed: int = 4, mach: float = 0.05) -> Case:
    """NS 256x256 affine on [0,2pi]^2, Ma=0.05, Re=1000, smooth seeded random fields."""
    mesh = Mesh(nx, nx, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi))
    prm = Params(order=p, n_elem=mesh.E, mach_ref=mach, reynolds=1000.0, viscous=True, kappa=1.0)
    rng = np.random.default_rng(seed)
    u, v = random_solenoidal_velocity(mesh, rng, rms=1.0)
    phip = random_scalar_field(mesh, rng)
    phiT = random_scalar_field(mesh, rng)
    q = np.empty((4, mesh.E, mesh.Np))
    q[0] = prm.gas_constant + 0.1 * phip
    q[1], q[2] = u, v
    q[3] = 1.0 + 0.1 * prm.gamma * mach ** 2 * phiT
    return Case(f"c4_ns_random_p{p}_{nx}x{nx}", mesh, prm, q, None, dt=0.01)


def config_c5_specs(n_cases: int = 48, seed: int = 190306304):
    """Per-case draws (N, p, Ma, Re, deforming) of the batched workload."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_cases):
        N = 16 * int(rng.integers(1, 13))
        p = int(rng.integers(2, 5))
        ma = 10 ** rng.uniform(-2, math.log10(0.3))
        re = 10 ** rng.uniform(2, math.log10(5000))
        specs.append(dict(N=N, p=p, mach=ma, re=re, deforming=bool(i % 2)))
    return specs


def config_c5_case(i: int, spec: dict, scale: float = 1.0) -> Case:
    """Case i of the batched workload (optionally with the mesh size scaled down)."""
    N = max(2, int(round(spec["N"] * scale)))
    p = spec["p"]
    deforming = spec["deforming"]
    dom = (0.0, 2 * np.pi, 0.0, 2 * np.pi)
    mapping = map_deforming(0.05, np.pi) if deforming else map_affine
    mesh = Mesh(N, N, p, dom, mapping, moving=deforming)
    prm = Params(order=p, n_elem=mesh.E, mach_ref=spec["mach"], reynolds=spec["re"],
                 viscous=True, moving=deforming, kappa=1.0)
    rng = np.random.default_rng(100 + i)
    u, v = random_solenoidal_velocity(mesh, rng, rms=1.0)
    phip = random_scalar_field(mesh, rng)
    phiT = random_scalar_field(mesh, rng)
    q = np.empty((4, mesh.E, mesh.Np))
    q[0] = prm.gas_constant + 0.1 * phip
    q[1], q[2] = u, v
    q[3] = 1.0 + 0.1 * prm.gamma * spec["mach"] ** 2 * phiT
    return Case(f"c5_case{i}_p{p}_{N}x{N}", mesh, prm, q, None, dt=0.01)
