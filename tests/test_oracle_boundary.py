"""Pins of the oracle's boundary faces (Sec. "Boundary Conditions": far field through the
approximate Riemann solver with the free-stream state, slip walls, adiabatic no-slip walls).

Each pin ties a boundary face to something fixed elsewhere, not to the formula it uses:

* far field == an interior face whose neighbour element holds the uniform free stream
  (a periodic mesh with one extra column at q^inf), inviscid and viscous;
* slip wall == a mirror plane: on a mesh mirrored across the wall, with the mirrored
  state, the interior faces on the mirror line give the same residual (affine, curved
  and moving meshes; inviscid and viscous, which pins the mirrored gradients);
* no-slip adiabatic wall: a fluid at rest is steady; a closed box conserves mass for any
  state; with the fluid at rest and any temperature field the box also conserves energy
  (no heat flux through the walls);
* a closed box in rigid translation with its fluid is steady (moving wall states);
* no-slip wall, exact solutions: plane Poiseuille (walls at rest) and plane Couette (the
  upper wall moving with the mesh) profiles give the exact pointwise residual of the
  Navier-Stokes equations at p = 3, where every flux is a polynomial of degree <= p.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_1903_06304_amd import inputs as I

FAR, SLIP, WALL = I.BC_FARFIELD, I.BC_SLIP_WALL, I.BC_NOSLIP_WALL


def random_state(mesh, prm, seed, amp_u=0.3, xy=None):
    rng = np.random.default_rng(seed)
    q = I.uniform_flow(mesh, prm, u=0.4, v=-0.2)
    f = [I.random_scalar_field(mesh, rng, kmax=2, xy=xy) for _ in range(4)]
    q[0] *= 1 + 0.05 * f[0]
    q[1] += amp_u * f[1]
    q[2] += amp_u * f[2]
    q[3] *= 1 + 0.03 * f[3]
    return q


def scale(R):
    return np.max(np.abs(R), axis=(1, 2)) + 1e-300


def wavy_map(amp, Lx, Ly, moving=False):
    """Map symmetric under y -> -y and periodic in x (period Lx) and y (period 2 Ly):
    x' = x + amp s(x) cos(pi y/Ly), y' = y + amp s(x) sin(pi y/Ly), s = sin(2 pi x/Lx);
    moving: the displacement times (1 + sin(2 pi t))."""
    def f(xr, yr, t):
        s = np.sin(2 * np.pi * xr / Lx)
        dx, dy = amp * s * np.cos(np.pi * yr / Ly), amp * s * np.sin(np.pi * yr / Ly)
        a, da = (1 + np.sin(2 * np.pi * t), 2 * np.pi * np.cos(2 * np.pi * t)) if moving else (1.0, 0.0)
        return xr + a * dx, yr + a * dy, da * dx, da * dy
    return f


@pytest.mark.parametrize("p,viscous", [(2, False), (2, True), (3, True)])
def test_far_field_is_a_free_stream_neighbour(p, viscous):
    nx, ny, h = 5, 4, 0.7
    prm = I.Params(order=p, n_elem=0, mach_ref=0.1, reynolds=20.0, viscous=viscous, kappa=1.0)
    mf = I.Mesh(nx - 1, ny, p, (0.0, (nx - 1) * h, 0.0, ny * h), bc=(FAR, FAR, 0, 0))
    mp = I.Mesh(nx, ny, p, (0.0, nx * h, 0.0, ny * h))
    prm.n_elem = mf.E
    qf = random_state(mf, prm, 11)
    qinf = np.array([prm.gas_constant * 1.02, 0.35, 0.1, 0.98])
    qp = np.empty((4, mp.E, mp.Np))
    for e in range(mp.E):
        ix, iy = e % nx, e // nx
        qp[:, e] = qinf[:, None] if ix == nx - 1 else qf[:, ix + (nx - 1) * iy]
    of = Oracle(prm, mf)
    of.set_farfield(qinf)
    Rf = of.residual(qf)
    prm.n_elem = mp.E
    Rp = Oracle(prm, mp).residual(qp)
    keep = [ix + nx * iy for iy in range(ny) for ix in range(nx - 1)]
    d = np.max(np.abs(Rf - Rp[:, keep]), axis=(1, 2))
    assert np.all(d <= 1e-12 * scale(Rf)), (d, scale(Rf))
    # the boundary is felt: a different free stream changes the boundary elements
    of.set_farfield(qinf * np.array([1.0, 1.5, 1.0, 1.0]))
    assert np.max(np.abs(of.residual(qf) - Rf)) > 1e-3 * np.max(scale(Rf))


def mirrored(q_half, nx, nh, n):
    """State of the full mesh (2 nh rows) from the upper half: upper rows copy it, lower
    rows hold its mirror image (v negated, eta reversed)."""
    Np = n * n
    qf = np.empty((4, nx * 2 * nh, Np))
    jrev = np.array([i + n * (n - 1 - j) for j in range(n) for i in range(n)])
    sgn = np.array([1.0, 1.0, -1.0, 1.0])[:, None]
    for iyh in range(nh):
        for ix in range(nx):
            src = q_half[:, ix + nx * iyh]
            qf[:, ix + nx * (nh + iyh)] = src
            qf[:, ix + nx * (nh - 1 - iyh)] = sgn * src[:, jrev]
    return qf


@pytest.mark.parametrize("p,viscous,amp,moving", [
    (2, False, 0.0, False), (3, True, 0.0, False), (2, True, 0.08, False), (3, True, 0.08, True)])
def test_slip_wall_is_a_mirror_plane(p, viscous, amp, moving):
    nx, nh, Lx, Ly = 4, 3, 2.0, 1.0
    n = p + 1
    mp = wavy_map(amp, Lx, Ly, moving)
    half = I.Mesh(nx, nh, p, (0.0, Lx, 0.0, Ly), mp, moving=moving, bc=(0, 0, SLIP, SLIP))
    full = I.Mesh(nx, 2 * nh, p, (0.0, Lx, -Ly, Ly), mp, moving=moving)
    prm = I.Params(order=p, n_elem=half.E, mach_ref=0.1, reynolds=30.0, viscous=viscous, kappa=1.0,
                   moving=moving)
    t = 0.13
    qh = random_state(half, prm, 5, xy=half.solution_points(t))
    Rh = Oracle(prm, half, *half.nodes(t)).residual(qh)
    prm.n_elem = full.E
    Rf = Oracle(prm, full, *full.nodes(t)).residual(mirrored(qh, nx, nh, n))
    upper = np.arange(nx * nh, 2 * nx * nh)
    d = np.max(np.abs(Rh - Rf[:, upper]), axis=(1, 2))
    assert np.all(d <= 1e-11 * scale(Rh)), (d, scale(Rh))
    # and the full residual is itself mirror-symmetric
    Rm = mirrored(Rh, nx, nh, n)
    assert np.all(np.max(np.abs(Rm - Rf), axis=(1, 2)) <= 1e-11 * scale(Rh))


@pytest.mark.parametrize("kind", [SLIP, WALL])
def test_wall_rest_state_is_steady(kind):
    p = 3
    mesh = I.Mesh(4, 3, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1), bc=(kind,) * 4)
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=10.0, viscous=True, kappa=1.0)
    q = I.uniform_flow(mesh, prm, u=0.0, v=0.0)
    R = Oracle(prm, mesh).residual(q)
    assert np.max(np.abs(R)) <= 1e-10 * prm.gas_constant, np.max(np.abs(R))


def test_slip_channel_uniform_flow_is_steady():
    p = 3
    mesh = I.Mesh(4, 3, p, (0.0, 2.0, 0.0, 1.0), bc=(0, 0, SLIP, SLIP))
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=10.0, viscous=True, kappa=1.0)
    q = I.uniform_flow(mesh, prm, u=0.7, v=0.0)
    R = Oracle(prm, mesh).residual(q)
    assert np.max(np.abs(R)) <= 1e-10 * prm.gas_constant, np.max(np.abs(R))


def integrals(o, R, p):
    g = o.geometry()
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    W = np.outer(w, w).reshape(-1) * g["jac"]
    return np.einsum("es,ves->v", W, R), np.einsum("es,ves->v", W, np.abs(R))


@pytest.mark.parametrize("kind,p", [(SLIP, 2), (WALL, 2), (WALL, 3)])
def test_closed_box_conserves_mass(kind, p):
    mesh = I.Mesh(4, 3, p, (0.0, 2.0, 0.0, 1.5), bc=(kind,) * 4)
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.2, reynolds=50.0, viscous=True, kappa=1.0)
    q = random_state(mesh, prm, 3 + p)
    o = Oracle(prm, mesh)
    tot, mag = integrals(o, o.residual(q), p)
    assert abs(tot[0]) <= 1e-13 * mag[0], (tot, mag)


@pytest.mark.parametrize("p", [2, 3])
def test_adiabatic_box_at_rest_conserves_energy(p):
    mesh = I.Mesh(4, 3, p, (0.0, 2.0, 0.0, 1.5), bc=(WALL,) * 4)
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.2, reynolds=5.0, viscous=True, kappa=1.0)
    rng = np.random.default_rng(p)
    q = I.uniform_flow(mesh, prm, u=0.0, v=0.0)
    q[3] *= 1 + 0.1 * I.random_scalar_field(mesh, rng, kmax=2)
    o = Oracle(prm, mesh)
    tot, mag = integrals(o, o.residual(q), p)
    assert abs(tot[0]) <= 1e-13 * mag[0] and abs(tot[3]) <= 1e-13 * mag[3], (tot, mag)
    assert mag[3] > 0.0


def test_noslip_poiseuille_profile_is_exact():
    """u = U y (H - y), v = 0, p and T uniform between walls at rest: the exact residual is
    R = (0, mu/Re u'', 0, mu/Re (u'^2 + u u'')) (momentum from the shear stress, energy from
    its work), reproduced to rounding at p = 3."""
    p, H, U = 3, 1.0, 0.3
    mesh = I.Mesh(3, 4, p, (0.0, 2.0, 0.0, H), bc=(0, 0, WALL, WALL))
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.1, reynolds=7.0, viscous=True, kappa=1.0)
    _, y = mesh.solution_points()
    q = I.uniform_flow(mesh, prm, u=0.0, v=0.0)
    q[1] = U * y * (H - y)
    R = Oracle(prm, mesh).residual(q)
    up, upp = U * (H - 2 * y), -2.0 * U
    k = prm.mu / prm.reynolds
    ex = np.stack([0 * y, k * upp + 0 * y, 0 * y, k * (up * up + q[1] * upp)])
    assert np.max(np.abs(R - ex)) <= 1e-9 * prm.gas_constant, np.max(np.abs(R - ex), axis=(1, 2))


def test_noslip_couette_with_moving_wall_is_exact():
    """u = U y/H between a wall at rest (y = 0) and a wall moving with speed U (y = H),
    the mesh sheared with grid velocity U y/H: the exact residual is (0, 0, 0, mu/Re U^2/H^2)
    (viscous heating), which needs the moving wall's velocity in the wall state."""
    p, H, U = 3, 1.0, 0.25

    def shear(xr, yr, t):
        return xr + U * t * yr / H, yr.copy(), U * yr / H, np.zeros_like(yr)
    mesh = I.Mesh(3, 4, p, (0.0, 2.0, 0.0, H), shear, moving=True, bc=(0, 0, WALL, WALL))
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.1, reynolds=7.0, viscous=True, kappa=1.0, moving=True)
    _, y = mesh.solution_points()
    q = I.uniform_flow(mesh, prm, u=0.0, v=0.0)
    q[1] = U * y / H
    R = Oracle(prm, mesh, *mesh.nodes(0.0)).residual(q)
    ex = np.zeros_like(R)
    ex[3] = prm.mu / prm.reynolds * U * U / (H * H)
    assert np.max(np.abs(R - ex)) <= 1e-9 * prm.gas_constant, np.max(np.abs(R - ex), axis=(1, 2))


@pytest.mark.parametrize("kind", [SLIP, WALL])
def test_translating_closed_box_carries_its_fluid(kind):
    """A curved closed box in rigid translation with velocity W, filled with fluid moving at
    W: nothing changes in the box frame, so R = 0; the walls' state must take the wall
    velocity into account (normal and tangential)."""
    p, W = 3, (0.3, -0.2)
    base = I.map_curved(0.1)

    def translate(xr, yr, t):
        x, y, _, _ = base(xr, yr, t)
        return x + W[0] * t, y + W[1] * t, np.full_like(x, W[0]), np.full_like(y, W[1])
    mesh = I.Mesh(4, 3, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi), translate, moving=True, bc=(kind,) * 4)
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=10.0, viscous=True, kappa=1.0, moving=True)
    q = I.uniform_flow(mesh, prm, u=W[0], v=W[1])
    R = Oracle(prm, mesh, *mesh.nodes(0.4)).residual(q)
    assert np.max(np.abs(R)) <= 1e-10 * prm.gas_constant, np.max(np.abs(R))
