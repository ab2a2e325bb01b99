"""The paper's isentropic-vortex verification on a deforming mesh (Sec. 4.3), at its own
configuration, on the GPU path.

Periodic [-10, 10]^2, free stream (sqrt(2)/2, sqrt(2)/2) at Ma = 0.05, vortex strength 5 with
phi = 1/2 centred at the origin (Eq. VP_Solution), prescribed motion x, y = x_r, y_r +
a sin(2 pi f_n t) sin(2 pi f_x x_r) sin(2 pi f_y y_r) with a = 1, f_n = 1, f_x = f_y = 0.1;
Euler, BDF2 dual-time steps with GMRES tol_res 1e-6 and at most 100 iterations, Newton as far
as it goes within 100 pseudo-time steps (to the round-off floor of the residual).
  * temporal study: fifth order (p = 4) on 96 x 96, dt = T_n/100 ... T_n/800 to T_n/4;
    BDF2 order 2 from successive differences;
  * spatial study: 12^2 ... 96^2 at dt = 1e-4, against the exact advected vortex at the
    moving solution points; the paper reports orders close to k + 1/2.  The paper gives no
    final time for this study; the test runs 500 steps (t = 0.05), in which the mesh moves by
    a third of its largest displacement.
Reading: the paper sets the global cut-off kappa = 0, which leaves U_r = 0 wherever the
flow velocity equals the grid velocity (|v_g| reaches 2 pi a = 6.3 here, against |v| of
about 1): the preconditioner is then singular.  The tests take kappa = 1 (U_r >= Ma c).
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1903_06304_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

DOM = (-10.0, 10.0, -10.0, 10.0)
TN = 1.0   # period of the mesh motion, 1 / f_n
T_SPATIAL = 0.05


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _exact(mesh, prm, t):
    return I.isentropic_vortex(mesh, prm, t=t, center=(0.0, 0.0), xy=mesh.solution_points(t))


def _floor(g, q):
    """Ten times the change of the mass-row norm of R under a one-ulp perturbation of q: the
    Newton iteration stops there (it cannot go lower)."""
    gen = torch.Generator(device=q.device).manual_seed(3)
    r = torch.rand(q.shape, generator=gen, device=q.device, dtype=torch.float64) * 2.0 - 1.0
    d = g.residual(q * (1.0 + 2.0 ** -52 * r)) - g.residual(q)
    return 10.0 * float(torch.linalg.vector_norm(d[0]))


def march(p, N, dt, T):
    from paper_1903_06304_amd import lmfr
    mesh = I.Mesh(N, N, p, DOM, I.map_vortex_motion(1.0, 1.0, 0.1, 0.1), moving=True)
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, viscous=False, moving=True, kappa=1.0)
    g = lmfr.Context(prm, *mesh.connectivity())
    g.reserve(30, "fp64")
    g.set_geometry(*mesh.nodes(0.0))
    q = _dev(_exact(mesh, prm, 0.0))
    qm1 = _dev(_exact(mesh, prm, -dt))
    floor = _floor(g, q)
    nsteps = int(round(T / dt))
    its = 0
    for n in range(nsteps):
        g.set_geometry(*mesh.nodes((n + 1) * dt))
        qn = q.clone()
        st = g.bdf2_step(q, qm1, dt, tol_pseudo=1e-12, tol_res=1e-6, krylov=30, max_lin_it=100, max_newton=100,
                         tol_abs=floor, check=False)
        assert st["rc"] in (0, -5), (p, N, dt, n, st)
        assert st["converged"] == 1, (p, N, dt, n, st)
        its += st["gmres_its"]
        qm1 = qn
    torch.cuda.synchronize()
    return mesh, prm, q.cpu().numpy(), its


def _l2(a, b, var):
    return float(np.sqrt(np.mean((a[var] - b[var]) ** 2)))


def test_paper_vortex_bdf2_temporal_order():
    """p = 4 on 96 x 96, dt = T_n/100, /200, /400, /800 to T_n/4."""
    t0 = time.perf_counter()
    sols = []
    for k in (100, 200, 400, 800):
        mesh, prm, q, its = march(4, 96, TN / k, TN / 4)
        sols.append(q)
        print(f"[vortex-paper] dt = T_n/{k}: {int(round(k / 4))} steps, {its} GMRES iterations, "
              f"{time.perf_counter() - t0:.1f} s", flush=True)
    for var, name in ((0, "p"), (1, "u")):
        d = [_l2(sols[k], sols[k + 1], var) for k in range(3)]
        orders = [np.log2(d[k] / d[k + 1]) for k in range(2)]
        print(f"[vortex-paper] temporal, {name}: successive differences {d}, orders {orders}", flush=True)
        assert min(orders) >= 1.9, (name, d, orders)
    ex = _exact(mesh, prm, TN / 4)
    print(f"[vortex-paper] dt = T_n/800 against the exact vortex: p {_l2(sols[-1], ex, 0):.3e}, "
          f"u {_l2(sols[-1], ex, 1):.3e}", flush=True)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_paper_vortex_spatial_order(p):
    """12^2, 24^2, 48^2, 96^2 at dt = 1e-4; errors of p and u against the exact vortex."""
    Ns = (12, 24, 48, 96)
    T = T_SPATIAL
    errs = {0: [], 1: []}
    t0 = time.perf_counter()
    for N in Ns:
        mesh, prm, q, its = march(p, N, 1e-4, T)
        ex = _exact(mesh, prm, T)
        for var in (0, 1):
            errs[var].append(_l2(q, ex, var))
        print(f"[vortex-paper] p={p} N={N}: errors p {errs[0][-1]:.3e} u {errs[1][-1]:.3e}, {its} GMRES, "
              f"{time.perf_counter() - t0:.1f} s", flush=True)
    for var, name in ((0, "p"), (1, "u")):
        orders = [np.log(errs[var][k] / errs[var][k + 1]) / np.log(2.0) for k in range(3)]
        print(f"[vortex-paper] spatial p={p}, {name}: orders {orders} (k + 1/2 = {p + 0.5})", flush=True)
        assert orders[-1] >= p + 0.5 - 0.2 or orders[-2] >= p + 0.5 - 0.2, (name, errs[var], orders)
