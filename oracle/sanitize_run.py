"""Runs the oracle's entry points on small meshes, for the sanitizer build (test infrastructure:
tests/test_oracle_sanitizers.py starts it with the oracle built under AddressSanitizer and
UndefinedBehaviorSanitizer named by LMFR_ORACLE_LIB).  Every kind of element and face is
visited: affine, curved and deforming maps; periodic, far-field, slip-wall and no-slip faces;
flipped connectivity; Euler and Navier-Stokes; orders 1-4."""
import os
import sys

import numpy as np

# the repository root replaces this folder on the path (this folder holds oracle.py)
sys.path[0] = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

from oracle.oracle import Oracle, gmres_dense, lu_factor, lu_solve, operators  # noqa: E402
from paper_1903_06304_amd import inputs as I  # noqa: E402


def state(mesh, prm, seed, xy=None):
    rng = np.random.default_rng(seed)
    q = I.uniform_flow(mesh, prm, u=0.3, v=-0.2)
    f = [I.random_scalar_field(mesh, rng, kmax=2, xy=xy) for _ in range(4)]
    q[0] *= 1 + 0.05 * f[0]
    q[1] += 0.2 * f[1]
    q[2] += 0.2 * f[2]
    q[3] *= 1 + 0.03 * f[3]
    return q


def cases():
    F, S, W = I.BC_FARFIELD, I.BC_SLIP_WALL, I.BC_NOSLIP_WALL
    yield "affine p1 euler periodic", I.Mesh(3, 2, 1), dict(viscous=False)
    yield "curved p3 ns periodic", I.Mesh(3, 3, 3, (0.0, 2.0, 0.0, 2.0), I.map_curved(0.1)), dict(viscous=True)
    yield "deforming p2 ns", I.Mesh(3, 3, 2, (0.0, 2.0, 0.0, 2.0), I.map_deforming(0.05, 1.0), moving=True), \
        dict(viscous=True, moving=True)
    yield "walls p2 ns", I.Mesh(3, 3, 2, (0.0, 1.5, 0.0, 1.5), bc=(F, F, W, S)), dict(viscous=True)
    yield "far field p4 ns", I.Mesh(2, 2, 4, (0.0, 1.0, 0.0, 1.0), I.map_curved(0.05), bc=(F, F, F, F)), \
        dict(viscous=True)


class Renumbered:
    """A mesh whose elements' local frames are turned by seeded quarter turns: faces meet arbitrary
    neighbour faces, half of them with reversed point order."""

    def __init__(self, mesh, seed=7):
        nbr, nbf, flip = mesh.connectivity()
        rot = np.random.default_rng(seed).integers(0, 4, mesh.E)
        self.E, self.p, self.bc = mesh.E, mesh.p, mesh.bc
        self._conn = I.renumber_elements(nbr, nbf, flip, rot)
        self.carry = self._conn[3]

    def connectivity(self):
        return self._conn[:3]


def main():
    for p in (1, 2, 3, 4):
        operators(p)
    A = np.eye(6) * 4 + np.random.default_rng(0).standard_normal((6, 6))
    LU, piv, _ = lu_factor(A)
    lu_solve(LU, piv, np.ones(6))
    gmres_dense(A, np.ones(6), m=4)
    for name, mesh, kw in cases():
        prm = I.Params(order=mesh.p, n_elem=mesh.E, mach_ref=0.1, reynolds=50.0, kappa=1.0, **kw)
        o = Oracle(prm, mesh, t=0.1)
        o.geometry()
        if mesh.bc is not None and any(mesh.bc):
            o.set_farfield(I.uniform_flow(mesh, prm, u=0.3, v=0.0)[:, 0, 0])
        q = state(mesh, prm, 1)
        v = state(mesh, prm, 2) - q
        o.residual(q)
        o.count_residual(q)
        o.jvp(q, v)
        o.vjp_dofs(q, v, [0, o.N // 2, o.N - 1])
        o.blocks(q, 1.0, 10.0)
        o.precond_apply(q, v, 1.0, 10.0, precond=1)
        o.bdf2_step(q, None, 1e-2, krylov=10, max_lin_it=20, max_newton=2)
        o.steady_solve(q, krylov=10, max_lin_it=20, max_steps=2)
        print("ran", name, flush=True)
    # flipped and rotated connectivity
    mesh = I.Mesh(3, 3, 2, (0.0, 2.0, 0.0, 2.0), I.map_curved(0.1))
    prm = I.Params(order=2, n_elem=mesh.E, mach_ref=0.1, reynolds=50.0, viscous=True, kappa=1.0)
    rn = Renumbered(mesh)
    xg, _ = mesh.nodes(0.0)
    o = Oracle(prm, rn, rn.carry(xg), None)
    q = rn.carry(state(mesh, prm, 1))
    o.residual(q)
    o.jvp(q, rn.carry(state(mesh, prm, 2)) - q)
    o.blocks(q, 1.0, 10.0)
    print("ran renumbered p2 ns", flush=True)
    print("ok", flush=True)


if __name__ == "__main__":
    main()
