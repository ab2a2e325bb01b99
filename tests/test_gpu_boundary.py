"""GPU parity on meshes with boundary faces (paper Sec. "Boundary Conditions": far field
through the Riemann solver with the free stream, slip walls, adiabatic no-slip walls)
against the FP64 CPU oracle, whose boundary faces are pinned by the CPU tests.

Cases (several tiles each, ragged last tile): an O-grid around a cylinder with P4 curved
elements (no-slip wall inside, far field outside), a curved box with all three kinds, a
slip channel (inviscid), a translating box with moving walls, a P1 annulus (inviscid).
Bars as for periodic meshes: R per row <= 1e-12 S_c; JVP, VJP, Newton operator <= 1e-12
normwise; blocks <= 1e-12 of their largest entry; BDF2 and steady states 1e-8 relative.
The GPU path is also held to the invariants that pin the oracle's boundary faces, with no
oracle in the loop: a slip wall is a mirror plane (curved and moving meshes), a far-field
face is a neighbour holding the free stream, plane Poiseuille flow gives the exact residual,
and a closed adiabatic box at rest conserves mass and energy.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_1903_06304_amd import inputs as I  # noqa: E402

from helpers import flux_scale, residual_parity, normwise_rel, row_errors  # noqa: E402

pytestmark = pytest.mark.gpu

FAR, SLIP, WALL = I.BC_FARFIELD, I.BC_SLIP_WALL, I.BC_NOSLIP_WALL


def _translating(W=(0.3, -0.2)):
    base = I.map_curved(0.1)

    def f(xr, yr, t):
        x, y, _, _ = base(xr, yr, t)
        return x + W[0] * t, y + W[1] * t, np.full_like(x, W[0]), np.full_like(y, W[1])
    return f


def _state(mesh, prm, t, amp=0.2):
    """Uniform flow (u, v) = (1, 0) plus smooth perturbations of every variable."""
    x, y = mesh.solution_points(t)
    q = I.uniform_flow(mesh, prm, u=1.0, v=0.0)
    q[0] *= 1 + 0.02 * np.sin(0.7 * x + 0.3) * np.cos(0.5 * y)
    q[1] += amp * np.cos(0.6 * x - 0.4 * y)
    q[2] += amp * np.sin(0.5 * x + 0.8 * y + 0.2)
    q[3] *= 1 + 0.01 * np.cos(0.4 * x + 0.9 * y)
    return q


def bc_cases():
    out = []
    m = I.Mesh(10, 4, 4, (0.0, 1.0, 0.0, 1.0), I.map_annulus(0.5, 8.0), bc=(0, 0, WALL, FAR))
    out.append(("cylinder_p4_ns", m, dict(viscous=True, reynolds=40.0), 0.0))
    m = I.Mesh(5, 4, 3, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1), bc=(FAR, FAR, WALL, SLIP))
    out.append(("box_mixed_p3_ns", m, dict(viscous=True, reynolds=50.0), 0.0))
    m = I.Mesh(6, 3, 2, (0.0, 2.0, 0.0, 1.0), bc=(0, 0, SLIP, SLIP))
    out.append(("channel_slip_p2_euler", m, dict(viscous=False), 0.0))
    m = I.Mesh(4, 5, 3, (0.0, 2 * np.pi, 0.0, 2 * np.pi), _translating(), moving=True,
               bc=(SLIP, SLIP, WALL, WALL))
    out.append(("translating_box_p3_ns_moving", m, dict(viscous=True, reynolds=30.0, moving=True), 0.4))
    m = I.Mesh(8, 3, 1, (0.0, 1.0, 0.0, 1.0), I.map_annulus(0.5, 4.0), bc=(0, 0, SLIP, FAR))
    out.append(("annulus_p1_euler", m, dict(viscous=False), 0.0))
    return out


CASES = bc_cases()


def _setup(case):
    from paper_1903_06304_amd import lmfr
    name, mesh, kw, t = case
    prm = I.Params(order=mesh.p, n_elem=mesh.E, mach_ref=0.05, kappa=1.0, **kw)
    qinf = np.array([prm.gas_constant, 1.0, 0.0, 1.0])
    xg, vg = mesh.nodes(t)
    o = Oracle(prm, mesh, xg, vg)
    o.set_farfield(qinf)
    nbr, nbf, flip = mesh.connectivity()
    g = lmfr.Context(prm, nbr, nbf, flip)
    g.set_geometry(xg, vg)
    g.set_farfield(qinf)
    return prm, o, g, _state(mesh, prm, t)


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


IDS = [c[0] for c in CASES]


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_residual_parity(case):
    print(f"[boundary] residual {case[0]} E={case[1].E}", flush=True)
    prm, o, g, q = _setup(case)
    # no element with a boundary face takes the affine kernels
    nbr = case[1].connectivity()[0]
    assert g.affine_elements() <= int(np.sum(np.all(nbr >= 0, axis=1)))
    R = g.residual(_dev(q)).cpu().numpy()
    Ro = o.residual(q)
    err_s = residual_parity(o.geometry(), prm, q, R, Ro)
    assert np.all(err_s <= 1e-12), err_s


def test_channel_interior_row_is_affine():
    prm, o, g, q = _setup(CASES[2])
    assert g.affine_elements() == 6


def test_farfield_must_be_set():
    from paper_1903_06304_amd import lmfr
    name, mesh, kw, t = CASES[0]
    prm = I.Params(order=mesh.p, n_elem=mesh.E, mach_ref=0.05, kappa=1.0, **kw)
    g = lmfr.Context(prm, *mesh.connectivity())
    g.set_geometry(*mesh.nodes(0.0))
    q = _dev(_state(mesh, prm, 0.0))
    with pytest.raises(RuntimeError, match="fr_set_farfield"):
        g.residual(q)
    with pytest.raises(RuntimeError):
        g.set_farfield([1.0, 0.0, 0.0, -1.0])
    g.set_farfield([prm.gas_constant, 1.0, 0.0, 1.0])
    R1 = g.residual(q)
    # the far-field state is read at every call
    g.set_farfield([prm.gas_constant, 0.5, 0.1, 1.0])
    R2 = g.residual(q)
    assert not torch.equal(R1, R2)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_jvp_and_vjp_parity(case):
    print(f"[boundary] jvp/vjp {case[0]}", flush=True)
    prm, o, g, q = _setup(case)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(q.shape)
    w = rng.standard_normal(q.shape)
    Jv, R = g.jvp(_dev(q), _dev(v), want_residual=True)
    Jv = Jv.cpu().numpy()
    errj = normwise_rel(Jv, o.jvp(q, v))
    JTw = g.vjp(_dev(q), _dev(w)).cpu().numpy()
    errv = normwise_rel(JTw, o.vjp_dofs(q, w, np.arange(q.size)).reshape(q.shape))
    print("  jvp", errj, "vjp", errv, flush=True)
    assert np.all(errj <= 1e-12), errj
    assert np.all(errv <= 1e-12), errv
    lhs, rhs = np.dot(w.ravel(), Jv.ravel()), np.dot(JTw.ravel(), v.ravel())
    assert abs(lhs - rhs) <= 1e-12 * np.abs(w.ravel() * Jv.ravel()).sum()


@pytest.mark.parametrize("packs", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_blocks_and_operator_parity(case, packs):
    print(f"[boundary] blocks {case[0]} packs={packs}", flush=True)
    prm, o, g, q = _setup(case)
    g.set_option("keep_blocks", 1)
    g.set_option("operator_packs", packs)
    ct, idt = 150.0, 0.37
    g.block_jacobi_factor(_dev(q), ct, idt, "fp64")
    B = g.get_blocks().cpu().numpy()
    Bo = o.blocks(q, ct, idt)
    err = np.max(np.abs(B - Bo)) / np.max(np.abs(Bo))
    print("  blocks", err, flush=True)
    assert err <= 1e-12, err
    # Newton operator (dual numbers, or tangents over the packs)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(q.shape)
    Av = g.bdf_operator(_dev(q), _dev(v), ct, idt).cpu().numpy()
    B0 = o.blocks(q, 0.0, 0.0)
    ref = -o.jvp(q, v)
    for e in range(o.E):
        ref[:, e, :] += ((Bo[e] - B0[e]) @ v[:, e, :].reshape(-1)).reshape(4, o.Np)
    erra = normwise_rel(Av, ref)
    assert np.all(erra <= 1e-12), erra


def test_bdf2_step_parity_cylinder():
    prm, o, g, q = _setup(CASES[0])
    dt = 0.05
    kw = dict(tol_pseudo=1e-10, tol_res=1e-10, krylov=30, max_lin_it=400, max_newton=20)
    qo, sto = o.bdf2_step(q, q, dt, **kw)
    qg = _dev(q)
    st = g.bdf2_step(qg, _dev(q), dt, **kw)
    torch.cuda.synchronize()
    print("[boundary] bdf2 cylinder", st, {k: v for k, v in sto.items() if k != "hist"}, flush=True)
    assert st["converged"] == 1 and sto["converged"] == 1
    diff = np.max(np.abs(qg.cpu().numpy() - qo), axis=(1, 2))
    chg = np.max(np.abs(qo - q), axis=(1, 2))
    assert np.all(diff <= 1e-8 * chg + 1e-12 * np.max(np.abs(qo), axis=(1, 2))), diff / chg


@pytest.mark.parametrize("precond", [0, 1])
def test_steady_first_steps_parity_box(precond):
    prm, o, g, q = _setup(CASES[1])
    g.set_option("preconditioner", precond)
    kw = dict(tol_pseudo=1e-30, tol_res=1e-12, krylov=60, max_lin_it=2000, max_steps=4, dtau0=0.05, dtau_min=0.05)
    qg = _dev(q)
    st = g.steady_solve(qg, **kw)
    torch.cuda.synchronize()
    qo, sto = o.steady_solve(q, precond=precond, **kw)
    print(f"[boundary] steady GPU {st} oracle { {k: v for k, v in sto.items() if k != 'hist'} }", flush=True)
    assert st["steps"] == sto["steps"] == 4
    diff = np.max(np.abs(qg.cpu().numpy() - qo), axis=(1, 2))
    chg = np.max(np.abs(qo - q), axis=(1, 2))
    assert np.all(diff <= 1e-8 * chg + 1e-12 * np.max(np.abs(qo), axis=(1, 2))), diff / chg


def test_batch_of_boundary_and_periodic_cases_matches_singles():
    """A batch mixing meshes with and without boundary faces runs each case with the same
    kernel variant as a context alone: residuals bitwise equal."""
    from paper_1903_06304_amd import lmfr
    ctxs, qs = [], []
    for case in (CASES[0], CASES[1], CASES[3]):
        prm, o, g, q = _setup(case)
        ctxs.append(g)
        qs.append(_dev(q))
    mesh = I.Mesh(5, 3, 3, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1))
    prm = I.Params(order=3, n_elem=mesh.E, mach_ref=0.05, reynolds=50.0, viscous=True, kappa=1.0)
    g = lmfr.Context(prm, *mesh.connectivity())
    g.set_geometry(*mesh.nodes(0.0))
    ctxs.append(g)
    qs.append(_dev(_state(mesh, prm, 0.0)))
    singles = [c.residual(x) for c, x in zip(ctxs, qs)]
    b = lmfr.Batch(ctxs)
    Rb = b.unpack(b.residual(b.pack(qs)))
    torch.cuda.synchronize()
    for k, (a, r) in enumerate(zip(singles, Rb)):
        assert torch.equal(a, r), k


def test_cylinder_full_size_parity():
    """The benchmark's boundary workload at full size (256 x 256 P4 O-grid, 65,536 elements,
    potential flow past the cylinder), in the launch shape the autotuner picks: residual and
    JVP, every row."""
    from paper_1903_06304_amd import lmfr
    mesh = I.Mesh(256, 256, 4, (0.0, 1.0, 0.0, 1.0), I.map_annulus(0.5, 50.0), bc=(0, 0, WALL, FAR))
    prm = I.Params(order=4, n_elem=mesh.E, mach_ref=0.05, reynolds=40.0, viscous=True, kappa=1.0)
    print(f"[boundary] full-size cylinder E={mesh.E}", flush=True)
    x, y = mesh.solution_points()
    r4 = (x * x + y * y) ** 2
    q = I.uniform_flow(mesh, prm, u=1.0, v=0.0)
    q[1] = 1.0 - 0.25 * (x * x - y * y) / r4
    q[2] = -0.5 * x * y / r4
    qinf = [prm.gas_constant, 1.0, 0.0, 1.0]
    o = Oracle(prm, mesh)
    o.set_farfield(qinf)
    g = lmfr.Context(prm, *mesh.connectivity())
    g.set_geometry(*mesh.nodes(0.0))
    g.set_farfield(qinf)
    g.autotune(None)
    R = g.residual(_dev(q)).cpu().numpy()
    Ro = o.residual(q)
    err_s = residual_parity(o.geometry(), prm, q, R, Ro)
    assert np.all(err_s <= 1e-12), err_s
    v = np.random.default_rng(8).standard_normal(q.shape)
    errj = normwise_rel(g.jvp(_dev(q), _dev(v)).cpu().numpy(), o.jvp(q, v))
    print("  jvp", errj, flush=True)
    assert np.all(errj <= 1e-12), errj


# ---- the oracle's boundary pins, evaluated with the GPU library (independent of the oracle)
def _gpu_residual(prm, mesh, q, t=0.0, qinf=None):
    from paper_1903_06304_amd import lmfr
    g = lmfr.Context(prm, *mesh.connectivity())
    g.set_geometry(*mesh.nodes(t))
    if qinf is not None:
        g.set_farfield(qinf)
    return g.residual(_dev(q)).cpu().numpy()


def _wavy(amp, Lx, Ly, moving):
    def f(xr, yr, t):
        s = np.sin(2 * np.pi * xr / Lx)
        dx, dy = amp * s * np.cos(np.pi * yr / Ly), amp * s * np.sin(np.pi * yr / Ly)
        a, da = (1 + np.sin(2 * np.pi * t), 2 * np.pi * np.cos(2 * np.pi * t)) if moving else (1.0, 0.0)
        return xr + a * dx, yr + a * dy, da * dx, da * dy
    return f


@pytest.mark.parametrize("p,moving", [(3, False), (4, True)])
def test_gpu_slip_wall_is_a_mirror_plane(p, moving):
    """Curved (and moving) mesh mirrored across y = 0: the half domain with slip walls at
    y = 0 and y = Ly gives the residual of the full periodic domain's upper half."""
    nx, nh, Lx, Ly, t = 6, 5, 2.0, 1.0, 0.13
    n = p + 1
    mp = _wavy(0.08, Lx, Ly, moving)
    half = I.Mesh(nx, nh, p, (0.0, Lx, 0.0, Ly), mp, moving=moving, bc=(0, 0, SLIP, SLIP))
    full = I.Mesh(nx, 2 * nh, p, (0.0, Lx, -Ly, Ly), mp, moving=moving)
    prm = I.Params(order=p, n_elem=half.E, mach_ref=0.1, reynolds=30.0, viscous=True, kappa=1.0, moving=moving)
    qh = _state(half, prm, t)
    Rh = _gpu_residual(prm, half, qh, t)
    Np = n * n
    qf = np.empty((4, full.E, Np))
    jrev = np.array([i + n * (n - 1 - j) for j in range(n) for i in range(n)])
    sgn = np.array([1.0, 1.0, -1.0, 1.0])[:, None]
    for iyh in range(nh):
        for ix in range(nx):
            src = qh[:, ix + nx * iyh]
            qf[:, ix + nx * (nh + iyh)] = src
            qf[:, ix + nx * (nh - 1 - iyh)] = sgn * src[:, jrev]
    prm.n_elem = full.E
    Rf = _gpu_residual(prm, full, qf, t)
    upper = np.arange(nx * nh, 2 * nx * nh)
    d = np.max(np.abs(Rh - Rf[:, upper]), axis=(1, 2))
    s = np.max(np.abs(Rh), axis=(1, 2))
    assert np.all(d <= 1e-11 * s), (d, s)


def test_gpu_far_field_is_a_free_stream_neighbour():
    p, nx, ny, h = 3, 6, 5, 0.7
    prm = I.Params(order=p, n_elem=(nx - 1) * ny, mach_ref=0.1, reynolds=20.0, viscous=True, kappa=1.0)
    mf = I.Mesh(nx - 1, ny, p, (0.0, (nx - 1) * h, 0.0, ny * h), bc=(FAR, FAR, 0, 0))
    mpm = I.Mesh(nx, ny, p, (0.0, nx * h, 0.0, ny * h))
    qf = _state(mf, prm, 0.0)
    qinf = np.array([prm.gas_constant * 1.02, 0.35, 0.1, 0.98])
    qp = np.empty((4, mpm.E, mpm.Np))
    for e in range(mpm.E):
        ix, iy = e % nx, e // nx
        qp[:, e] = qinf[:, None] if ix == nx - 1 else qf[:, ix + (nx - 1) * iy]
    Rf = _gpu_residual(prm, mf, qf, qinf=qinf)
    prm.n_elem = mpm.E
    Rp = _gpu_residual(prm, mpm, qp)
    keep = [ix + nx * iy for iy in range(ny) for ix in range(nx - 1)]
    d = np.max(np.abs(Rf - Rp[:, keep]), axis=(1, 2))
    assert np.all(d <= 1e-12 * np.max(np.abs(Rf), axis=(1, 2))), d


def test_gpu_noslip_poiseuille_and_closed_box():
    """Plane Poiseuille between walls at rest: the exact NS residual at p = 3; a closed
    adiabatic box with the fluid at rest and any temperature field conserves mass and energy."""
    p, H, U = 3, 1.0, 0.3
    mesh = I.Mesh(4, 5, p, (0.0, 2.0, 0.0, H), bc=(0, 0, WALL, WALL))
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.1, reynolds=7.0, viscous=True, kappa=1.0)
    _, y = mesh.solution_points()
    q = I.uniform_flow(mesh, prm, u=0.0, v=0.0)
    q[1] = U * y * (H - y)
    R = _gpu_residual(prm, mesh, q)
    up, upp, k = U * (H - 2 * y), -2.0 * U, prm.mu / prm.reynolds
    ex = np.stack([0 * y, k * upp + 0 * y, 0 * y, k * (up * up + q[1] * upp)])
    assert np.max(np.abs(R - ex)) <= 1e-9 * prm.gas_constant, np.max(np.abs(R - ex), axis=(1, 2))
    box = I.Mesh(5, 4, p, (0.0, 2.0, 0.0, 1.5), bc=(WALL,) * 4)
    prm = I.Params(order=p, n_elem=box.E, mach_ref=0.2, reynolds=5.0, viscous=True, kappa=1.0)
    x, y = box.solution_points()
    q = I.uniform_flow(box, prm, u=0.0, v=0.0)
    q[3] *= 1 + 0.1 * np.cos(2.0 * x + 0.5) * np.sin(3.0 * y + 0.2)
    R = _gpu_residual(prm, box, q)
    o = Oracle(prm, box)      # geometry (|J|) only
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    W = np.outer(w, w).reshape(-1)[None, :] * o.geometry()["jac"]
    tot = np.einsum("es,ves->v", W, R)
    mag = np.einsum("es,ves->v", W, np.abs(R))
    assert abs(tot[0]) <= 1e-13 * mag[0] and abs(tot[3]) <= 1e-13 * mag[3], (tot, mag)
