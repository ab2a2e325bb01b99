"""Pins of the oracle's 1-D operators and pointwise physics against facts the paper
and the mathematics fix (not against the oracle itself).

* Gauss-Legendre points/weights vs numpy's Golub-Welsch routine.
* D and the face interpolation are exact on polynomials of degree <= p.
* Radau corrections (Sec. 3.1): g_L = right Radau, g_R = left Radau polynomial,
  built here with numpy's Legendre series; end values 1/0; the identity
  g_L'(xi_i) = -l_i(-1)/w_i that makes FR equal to nodal DG.
* M = dq^c/dq^p (Eq. jacobian) vs a complex-step derivative of q^c.
* Gamma = M when eps = 1 (Eq. theta with U_r = c); beta = 1/c^2.
* Eigenvalues of Gamma^-1 A_n,mov (Eqs. eigenvalues, eigenvalues_para, Sec. 2.3)
  vs a numerical eigen-solve.
* Common flux: consistency, conservation symmetry, viscous special cases.
"""
import numpy as np
import numpy.polynomial.legendre as L
import pytest

from oracle import oracle as O
from paper_1903_06304_amd import inputs as I


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_gauss_legendre(p):
    op = O.operators(p)
    x, w = np.polynomial.legendre.leggauss(p + 1)
    assert np.allclose(op["xi"], x, atol=1e-14, rtol=0)
    assert np.allclose(op["w"], w, atol=1e-14, rtol=0)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_derivative_and_interpolation_exact(p):
    op = O.operators(p)
    xi = op["xi"]
    for deg in range(p + 1):
        c = np.zeros(deg + 1); c[-1] = 1.0
        poly = np.polynomial.Polynomial(c)
        vals = poly(xi)
        assert np.allclose(op["D"] @ vals, poly.deriv()(xi), atol=1e-12)
        assert abs(op["lamL"] @ vals - poly(-1.0)) < 1e-13
        assert abs(op["lamR"] @ vals - poly(1.0)) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_radau_corrections(p):
    op = O.operators(p)
    xi, w = op["xi"], op["w"]
    # right Radau polynomial of degree p+1 (vanishes at +1) and left one (vanishes at -1)
    PL = L.Legendre.basis(p + 1) - L.Legendre.basis(p)
    gL = PL * (0.5 * (-1) ** (p + 1))
    gR = (L.Legendre.basis(p + 1) + L.Legendre.basis(p)) * 0.5
    assert abs(gL(-1.0) - 1.0) < 1e-14 and abs(gL(1.0)) < 1e-14
    assert abs(gR(1.0) - 1.0) < 1e-14 and abs(gR(-1.0)) < 1e-14
    assert np.allclose(op["gamL"], gL.deriv()(xi), atol=1e-12)
    assert np.allclose(op["gamR"], gR.deriv()(xi), atol=1e-12)
    # FR with Radau corrections == nodal DG: g_L'(xi_i) = -l_i(-1)/w_i, g_R'(xi_i) = l_i(1)/w_i
    assert np.allclose(op["gamL"], -op["lamL"] / w, atol=1e-12)
    assert np.allclose(op["gamR"], op["lamR"] / w, atol=1e-12)
    # slope at the end point (p+1)^2/2, used by the face-local BR2 lifting
    assert abs(gL.deriv()(-1.0) + 0.5 * (p + 1) ** 2) < 1e-11


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_gauss_lobatto(n):
    op = O.operators(1, n - 1)
    assert np.allclose(op["gll"], I.gll_points(n), atol=1e-14)


def _ctx(mach=0.05, kappa=1.0, viscous=True, moving=False, re=100.0):
    mesh = I.Mesh(2, 2, 1, (0, 1, 0, 1))
    prm = I.Params(order=1, n_elem=4, mach_ref=mach, reynolds=re, viscous=viscous,
                   moving=moving, kappa=kappa)
    return O.Oracle(prm, mesh), prm


def _random_state(rng, prm):
    return np.array([prm.gas_constant * (1 + 0.1 * rng.standard_normal()),
                     rng.standard_normal(), rng.standard_normal(), 1 + 0.05 * rng.standard_normal()])


def test_M_is_dqc_dqp():
    o, prm = _ctx()
    rng = np.random.default_rng(0)
    for _ in range(5):
        q = _random_state(rng, prm)
        M = o.point(q)["M"]
        h = 1e-30
        Mcs = np.zeros((4, 4))
        for k in range(4):
            z = q.astype(complex); z[k] += 1j * h
            Mcs[:, k] = o.cons_complex(z).imag / h
        assert np.allclose(M, Mcs, rtol=1e-13, atol=1e-13 * np.abs(M).max())


def test_gamma_equals_M_at_eps_one_and_beta():
    # kappa*Ma_inf >= 1 forces eps = 1, i.e. U_r = c, where Theta = rho_p.
    o, prm = _ctx(kappa=30.0)
    rng = np.random.default_rng(1)
    q = _random_state(rng, prm)
    d = o.point(q)
    assert np.allclose(d["Gamma"], d["M"], rtol=1e-12, atol=1e-14)
    # beta = rho_p + rho_T/(rho Cp) = 1/c^2 for an ideal gas; with eps = 1, alpha = 0 and the
    # largest eigenvalue is |u_n| + c.
    c = np.sqrt(prm.gamma * prm.gas_constant * q[3])
    assert abs(d["lam"] - (abs(q[1]) + c)) < 1e-12 * c


def _A_n(o, q, nx, ny, ug, vg):
    """d f_n / d q^p of the oracle's moving-mesh inviscid normal flux, central differences."""
    A = np.zeros((4, 4))
    for k in range(4):
        h = 1e-6 * max(1.0, abs(q[k]))
        qp, qm = q.copy(), q.copy(); qp[k] += h; qm[k] -= h
        A[:, k] = (o.point(qp, nx, ny, ug, vg)["fn"] - o.point(qm, nx, ny, ug, vg)["fn"]) / (2 * h)
    return A


@pytest.mark.parametrize("mach,kappa", [(0.05, 1.0), (0.01, 1.0), (0.3, 1.0), (0.1, 0.0)])
def test_preconditioned_eigenvalues(mach, kappa):
    o, prm = _ctx(mach=mach, kappa=kappa, moving=True)
    rng = np.random.default_rng(2)
    for _ in range(4):
        q = _random_state(rng, prm)
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = np.cos(th), np.sin(th)
        ug, vg = 0.3 * rng.standard_normal(2)
        d = o.point(q, nx, ny, ug, vg)
        A = _A_n(o, q, nx, ny, ug, vg)
        ev = np.linalg.eigvals(np.linalg.solve(d["Gamma"], A))
        # closed form: u_n (twice), u_n' +- c' with u_n = (v - v_g).n
        c = np.sqrt(prm.gamma * prm.gas_constant * q[3])
        un = (q[1] - ug) * nx + (q[2] - vg) * ny
        Ma = np.hypot(q[1] - ug, q[2] - vg) / c
        eps = min(1.0, max(kappa * prm.mach_inf, Ma))
        Ur = eps * c
        alpha = (1 - Ur ** 2 / c ** 2) / 2
        unp = un * (1 - alpha)
        cp = np.sqrt(alpha ** 2 * un ** 2 + Ur ** 2)
        expect = np.sort([un, un, unp + cp, unp - cp])
        got = np.sort(ev.real)
        assert np.allclose(got, expect, rtol=1e-6, atol=1e-6 * cp)
        assert np.max(np.abs(ev.imag)) < 1e-6 * cp
        assert abs(d["lam"] - np.max(np.abs(expect))) < 1e-12 * cp


def test_common_flux_consistency_and_symmetry():
    o, prm = _ctx(moving=True)
    rng = np.random.default_rng(3)
    for _ in range(5):
        q = _random_state(rng, prm)
        gx, gy = rng.standard_normal(4), rng.standard_normal(4)
        th = rng.uniform(0, 2 * np.pi); nx, ny = np.cos(th), np.sin(th)
        ug, vg = 0.2 * rng.standard_normal(2)
        # consistency: equal states and gradients give the physical normal flux
        fn, qcom = o.common_flux(q, q, gx, gy, gx, gy, nx, ny, 1.3, 0.7, 0.9, ug, vg)
        f, g = o.phys_flux(q, gx, gy)
        qc = o.point(q)["qc"]
        expect = f * nx + g * ny - (ug * nx + vg * ny) * qc
        assert np.allclose(fn, expect, rtol=1e-13, atol=1e-13 * np.abs(expect).max())
        assert np.allclose(qcom, q)
        # conservation: swapping sides and flipping the normal negates the flux
        q2 = _random_state(rng, prm)
        gx2, gy2 = rng.standard_normal(4), rng.standard_normal(4)
        a, _ = o.common_flux(q, q2, gx, gy, gx2, gy2, nx, ny, 1.3, 0.7, 0.9, ug, vg)
        b, _ = o.common_flux(q2, q, gx2, gy2, gx, gy, -nx, -ny, 1.3, 0.9, 0.7, ug, vg)
        assert np.allclose(a, -b, rtol=1e-13, atol=1e-12 * np.abs(a).max())


def test_viscous_flux_special_cases():
    o, prm = _ctx(re=10.0)
    q = np.array([prm.gas_constant, 0.3, -0.2, 1.1])
    z = np.zeros(4)
    f0, g0 = o.phys_flux(q, z, z)
    # rigid rotation u = -w y, v = w x: no viscous stress
    w = 0.7
    gx = np.array([0, 0, w, 0.0]); gy = np.array([0, -w, 0, 0.0])
    f, g = o.phys_flux(q, gx, gy)
    assert np.allclose(f, f0, atol=1e-13) and np.allclose(g, g0, atol=1e-13)
    # uniform dilatation u = a x, v = a y: tau_xx = tau_yy = (2/3) mu a, tau_xy = 0 (Stokes)
    a = 0.5
    f, g = o.phys_flux(q, np.array([0, a, 0, 0.0]), np.array([0, 0, a, 0.0]))
    tau = 2.0 / 3.0 * prm.mu * a / prm.reynolds
    assert np.allclose(f0 - f, [0, tau, 0, q[1] * tau], atol=1e-13)
    assert np.allclose(g0 - g, [0, 0, tau, q[2] * tau], atol=1e-13)
    # Fourier heat flux: k = mu Cp / Pr
    f, g = o.phys_flux(q, np.array([0, 0, 0, 2.0]), z)
    assert np.allclose(f0 - f, [0, 0, 0, prm.mu * prm.cp / prm.prandtl * 2.0 / prm.reynolds], rtol=1e-13)


def _cons(prm, q):
    """q^c = (rho, rho u, rho v, E) of the Sec. 2.1 non-dimensionalisation, written out."""
    rho = q[0] / (prm.gas_constant * q[3])
    E = q[0] / (prm.gamma - 1.0) + 0.5 * rho * (q[1] ** 2 + q[2] ** 2)
    return np.array([rho, rho * q[1], rho * q[2], E])


def _inviscid_ctx(mach, kappa, moving=True):
    return _ctx(mach=mach, kappa=kappa, viscous=False, moving=moving)


def test_rusanov_dissipation_at_eps_one_is_scalar_jump_of_conserved_state():
    """Eq. (Rosanov) at eps = 1 (kappa Ma_inf >= 1): Gamma~ = M at the averaged state and
    |lambda|max = |u_n| + c (alpha = 0), so the dissipation is -1/2 (|u_n| + c) times the
    jump of the conserved state up to O(delta^3): M at the midpoint integrates dq^c/dq^p
    along the jump with a midpoint-rule error.  The relative deviation therefore falls
    4x when the jump halves.  A dissipation with the wrong sign (relative deviation 2) or a
    coefficient 1 instead of 1/2 (deviation 1) fails at once."""
    o, prm = _inviscid_ctx(0.05, 30.0)
    rng = np.random.default_rng(11)
    z = np.zeros(4)
    for _ in range(6):
        q = _random_state(rng, prm)
        d = np.array([0.05 * q[0], 0.3, 0.3, 0.02 * q[3]]) * rng.choice([-1.0, 1.0], 4)
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = np.cos(th), np.sin(th)
        ug, vg = 0.2 * rng.standard_normal(2)
        c = np.sqrt(prm.gamma * prm.gas_constant * q[3])
        lam = abs((q[1] - ug) * nx + (q[2] - vg) * ny) + c
        rel = []
        for s in (1.0, 0.5):
            qL, qR = q - 0.5 * s * d, q + 0.5 * s * d
            fn, _ = o.common_flux(qL, qR, z, z, z, z, nx, ny, 1.0, 1.0, 1.0, ug, vg)
            avg = 0.5 * (o.point(qL, nx, ny, ug, vg)["fn"] + o.point(qR, nx, ny, ug, vg)["fn"])
            expect = -0.5 * lam * (_cons(prm, qR) - _cons(prm, qL))
            rel.append(np.linalg.norm((fn - avg) - expect) / np.linalg.norm(expect))
        assert rel[0] < 5e-3, rel
        assert 3.5 < rel[0] / rel[1] < 4.5, rel


@pytest.mark.parametrize("mach,kappa,moving", [(0.05, 1.0, True), (0.01, 1.0, False), (0.2, 0.0, True)])
def test_rusanov_dissipation_below_eps_one(mach, kappa, moving):
    """Eq. (Rosanov) with eps < 1: f^com = (f_n(q+) + f_n(q-))/2 - |lambda|max Gamma~ (q+ - q-)/2,
    Gamma~ at the averaged primitive state (pinned: Gamma = M at eps = 1 and the eigenvalues of
    Gamma^-1 A_n against the closed form) and |lambda|max = |u_n'| + c' from the closed form of
    Eqs. (eigenvalues_para), (eps_move) at the same state (pinned against an eigen-solve).  The
    jumps are O(1), so the identity is exact, not asymptotic.  The acoustic |u_n| + c in place
    of |u_n'| + c' (about 1/Ma times larger), Gamma~ at one side's state, a flipped sign or a
    coefficient 1 each fail."""
    o, prm = _inviscid_ctx(mach, kappa, moving)
    rng = np.random.default_rng(12)
    z = np.zeros(4)
    for _ in range(6):
        qL, qR = _random_state(rng, prm), _random_state(rng, prm)
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = np.cos(th), np.sin(th)
        ug, vg = (0.2 * rng.standard_normal(2)) if moving else (0.0, 0.0)
        qb = 0.5 * (qL + qR)
        c = np.sqrt(prm.gamma * prm.gas_constant * qb[3])
        un = (qb[1] - ug) * nx + (qb[2] - vg) * ny
        eps = min(1.0, max(kappa * prm.mach_inf, np.hypot(qb[1] - ug, qb[2] - vg) / c))
        Ur = eps * c
        alpha = 0.5 * (1.0 - Ur ** 2 / c ** 2)
        lam = abs(un * (1 - alpha)) + np.sqrt(alpha ** 2 * un ** 2 + Ur ** 2)
        G = o.point(qb, nx, ny, ug, vg)["Gamma"]
        avg = 0.5 * (o.point(qL, nx, ny, ug, vg)["fn"] + o.point(qR, nx, ny, ug, vg)["fn"])
        expect = avg - 0.5 * lam * (G @ (qR - qL))
        fn, _ = o.common_flux(qL, qR, z, z, z, z, nx, ny, 1.0, 1.0, 1.0, ug, vg)
        scale = np.abs(avg) + 0.5 * lam * (np.abs(G) @ np.abs(qR - qL))
        assert np.all(np.abs(fn - expect) <= 1e-13 * scale), (fn - expect) / scale
        # the dissipation is not negligible next to the average: a wrong term shows
        assert np.linalg.norm(fn - avg) > 1e-3 * np.linalg.norm(avg)
