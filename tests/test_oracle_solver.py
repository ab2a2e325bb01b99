"""Pins of the oracle's linear algebra and dual-time step.

* Partial-pivot LU vs scipy.linalg.lu_factor (same pivots, same factors).
* Restarted right-preconditioned GMRES vs numpy.linalg.solve.
* BDF2 step (Sec. 3.2, Eq. unsteady_pre_discretized_3): free stream on a deforming
  mesh stays unchanged (implicit GCL); the converged iterate satisfies the BDF2
  equation; temporal order 2 on the isentropic vortex (paper Sec. 4.3 reports
  the optimal BDF2 rate).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_1903_06304_amd import inputs as I


@pytest.mark.parametrize("n", [1, 5, 36, 64])
def test_lu_matches_scipy(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    LU, piv, rc = O.lu_factor(A)
    assert rc == 0
    LU_s, piv_s = sla.lu_factor(A)
    assert np.array_equal(piv, piv_s)
    assert np.allclose(LU, LU_s, rtol=1e-12, atol=1e-12)
    b = rng.standard_normal(n)
    x = O.lu_solve(LU, piv, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


def test_lu_singular_reports():
    A = np.ones((4, 4))
    _, _, rc = O.lu_factor(A)
    assert rc != 0


@pytest.mark.parametrize("m", [200, 15])
def test_gmres_matches_solve(m):
    rng = np.random.default_rng(3)
    n = 200
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, its, rel = O.gmres_dense(A, b, m=m, tol=1e-12, max_it=2000)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert rel <= 1e-12
    # right preconditioning by an exact inverse converges in one iteration
    x2, its2, _ = O.gmres_dense(A, b, m=m, tol=1e-12, max_it=50, Pinv=np.linalg.inv(A))
    assert its2 <= 2 and np.linalg.norm(x2 - xs) <= 1e-10 * np.linalg.norm(xs)


def test_bdf2_free_stream_deforming():
    c = I.config_c3(nx=4, p=2, perturbed=False)
    o = Oracle(c.prm, c.mesh, *c.mesh.nodes(0.05))
    q = c.q
    q1, st = o.bdf2_step(q, q, dt=0.01, krylov=10, tol_abs=1e-9 * c.prm.gas_constant)
    assert st["converged"] == 1
    assert np.max(np.abs(q1 - q) / np.abs(q).max(axis=(1, 2))[:, None, None]) < 1e-13


def _vortex_run(N, p, dt, t_end, mach=0.1):
    mesh = I.Mesh(N, N, p, (0.0, 10.0, 0.0, 10.0))
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=mach, kappa=0.0)
    o = Oracle(prm, mesh)
    # BDF1 start (q^{n-1} absent): its O(dt^2) local error keeps the global order 2, while an
    # exact q(-dt) would be inconsistent with the discrete dynamics at O(dt)
    q_nm1 = None
    q = I.isentropic_vortex(mesh, prm, t=0.0)
    nsteps = int(round(t_end / dt))
    for _ in range(nsteps):
        q_new, st = o.bdf2_step(q, q_nm1, dt=dt, tol_pseudo=1e-10, tol_res=1e-10, krylov=30, tol_abs=2e-12,
                                max_lin_it=200, max_newton=20)
        assert st["converged"] == 1, st
        q_nm1, q = q, q_new
    return q


def test_bdf2_converged_state_satisfies_equation():
    c = I.config_c1(nx=4)
    o = Oracle(c.prm, c.mesh)
    q1, st = o.bdf2_step(c.q, c.q_nm1, dt=c.dt, tol_pseudo=1e-10, tol_res=1e-8, krylov=20)
    assert st["converged"] == 1 and st["newton_its"] >= 1
    # plug the converged state into the BDF2 residual built from R and q^c
    def qc(q):
        p, u, v, T = q
        rho = p / (c.prm.gas_constant * T)
        return np.stack([rho, rho * u, rho * v, p / (c.prm.gamma - 1) + 0.5 * rho * (u * u + v * v)])
    b = -(1.5 * qc(q1) - 2 * qc(c.q) + 0.5 * qc(c.q_nm1)) / c.dt + o.residual(q1)
    b0 = -(1.5 * qc(c.q) - 2 * qc(c.q) + 0.5 * qc(c.q_nm1)) / c.dt + o.residual(c.q)
    assert np.linalg.norm(b[0]) <= 1e-9 * np.linalg.norm(b0[0])


@pytest.mark.slow
def test_bdf2_temporal_order():
    # The preconditioned Rusanov dissipation scales pressure modes by Theta/rho_p ~ 1/Ma^2,
    # which makes the semi-discrete system stiff; the step sizes are chosen inside the
    # asymptotic range (lambda_max dt < 1).
    N, p, T_end = 4, 2, 0.1
    ref = _vortex_run(N, p, T_end / 256, T_end)
    errs = []
    for k in (8, 16, 32):
        q = _vortex_run(N, p, T_end / k, T_end)
        errs.append(np.sqrt(np.mean((q[1] - ref[1]) ** 2)))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all(rates > 1.6) and rates[-1] > 1.85 and np.all(rates < 2.3), (errs, rates)
