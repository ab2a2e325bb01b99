"""Pins of the oracle's derivatives.

* Complex-step JVP (Im R(q + i h v)/h) vs central finite differences (eps = 1e-7).
* Dense complex-step Jacobian times v vs the JVP.
* Adjoint identity <w, J v> = <J^T w, v>, with J^T w from per-DOF local re-evaluation.
* Element blocks (seeded on one element, neighbours frozen) = diagonal blocks of the
  dense Jacobian, also on a mesh where an element is its own neighbour; the time
  terms Gamma/dtau + c_t M are added pointwise (Eq. unsteady_pre_discretized_3).
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_1903_06304_amd import inputs as I


def _case(kind, nx=3, ny=3, p=2):
    if kind == "euler":
        mesh = I.Mesh(nx, ny, p, (0.0, 10.0, 0.0, 10.0))
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.1, kappa=0.0)
        q = I.isentropic_vortex(mesh, prm)
        t = 0.0
    elif kind == "ns_curved":
        mesh = I.Mesh(nx, ny, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1))
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, kappa=1.0)
        q = I.taylor_green(mesh, prm)
        # Taylor-Green's odd symmetry puts the averaged normal velocity exactly at the kink
        # of |lambda|max on the x = 0, pi faces; a small offset moves the state off it.
        q[1] += 0.05
        q[2] -= 0.03
        t = 0.0
    else:
        mesh = I.Mesh(nx, ny, p, (0.0, 2.0, 0.0, 2.0), I.map_deforming(0.05), moving=True)
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True,
                       moving=True, kappa=1.0)
        rng = np.random.default_rng(7)
        q = I.uniform_flow(mesh, prm)
        du, dv = I.random_solenoidal_velocity(mesh, rng, rms=0.3)
        q[1] += du; q[2] += dv
        t = 0.11
    return Oracle(prm, mesh, *mesh.nodes(t)), q


@pytest.mark.parametrize("kind", ["euler", "ns_curved", "ns_deforming"])
def test_jvp_vs_central_fd(kind):
    o, q = _case(kind)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(q.shape)
    Jv = o.jvp(q, v)
    eps = 1e-7
    fd = (o.residual(q + eps * v) - o.residual(q - eps * v)) / (2 * eps)
    for r in range(4):
        err = np.linalg.norm(Jv[r] - fd[r]) / np.linalg.norm(Jv[r])
        assert err < 1e-6, (kind, r, err)


@pytest.mark.parametrize("kind", ["euler", "ns_deforming"])
def test_dense_jacobian_and_adjoint(kind):
    o, q = _case(kind)
    rng = np.random.default_rng(1)
    v, w = rng.standard_normal(q.shape), rng.standard_normal(q.shape)
    J = o.dense_jacobian(q)
    Jv = o.jvp(q, v)
    assert np.allclose(J @ v.ravel(), Jv.ravel(), rtol=0, atol=1e-12 * np.abs(Jv).max())
    JTw = o.vjp_dofs(q, w, np.arange(q.size))
    assert np.allclose(JTw, J.T @ w.ravel(), rtol=0, atol=1e-12 * np.abs(JTw).max())
    lhs, rhs = np.dot(w.ravel(), Jv.ravel()), np.dot(JTw, v.ravel())
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(w.ravel() * Jv.ravel()).sum())


@pytest.mark.parametrize("nx,ny", [(3, 3), (1, 3), (2, 3)])
def test_blocks_are_diagonal_of_jacobian(nx, ny):
    o, q = _case("ns_curved", nx=nx, ny=ny, p=1)
    J = o.dense_jacobian(q)
    E, Np = o.E, o.Np
    nb = 4 * Np
    B = o.blocks(q, 0.0, 0.0)
    idx = lambda e: np.array([v * E * Np + e * Np + s for v in range(4) for s in range(Np)])
    for e in range(E):
        ii = idx(e)
        assert np.allclose(B[e], -J[np.ix_(ii, ii)], rtol=0, atol=1e-12 * np.abs(J).max())
    # time terms: + c_t M + Gamma/dtau at each solution point
    ct, idt = 150.0, 0.3
    B2 = o.blocks(q, ct, idt, elements=[E - 1])
    e = E - 1
    D = B2[0] - B[e]
    g = o.geometry()
    for s in range(Np):
        d = o.point(q[:, e, s], ug=g["ug"][e, s], vg=g["vg"][e, s])
        rows = [v * Np + s for v in range(4)]
        assert np.allclose(D[np.ix_(rows, rows)], ct * d["M"] + idt * d["Gamma"], rtol=1e-12, atol=1e-9)
    off = D.copy()
    for s in range(Np):
        rows = [v * Np + s for v in range(4)]
        off[np.ix_(rows, rows)] = 0
    assert np.abs(off).max() <= 1e-10
