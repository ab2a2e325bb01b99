"""Mixed-precision preconditioner against the FP64 oracle, and the allocation-free hot path.

Bars (written here, derived in the design notes):
  * converged state of a BDF2 step with FP32 or BF16 blocks (block Jacobi, symmetric or
    forward block Gauss-Seidel) against the oracle's FP64 step: per variable, max |q_gpu - q_oracle| <=
    1e-5 x the variable's range over the field (the stated mixed-precision bar); FP64 blocks
    1e-8.  The preconditioner does not change the solution of the Newton system, so the gap
    is the Newton and GMRES tolerances times the conditioning, not the storage precision.
  * stored inverse: exactly representable in the storage precision; against the inverse of
    the oracle's blocks within the storage rounding plus the factorisation's own error;
  * apply: z = (stored inverse) r with FP64 accumulation, 1e-12 relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_1903_06304_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _ctx(prm, mesh, t=0.0):
    from paper_1903_06304_amd import lmfr
    g = lmfr.Context(prm, *mesh.connectivity())
    g.set_geometry(*mesh.nodes(t))
    return g


def _mixed_cases():
    c4 = I.config_c4(nx=8, p=3)
    c4p4 = I.config_c4(nx=6, p=4)
    curved = I.Mesh(6, 5, 4, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1))
    prm = I.Params(order=4, n_elem=curved.E, mach_ref=0.05, reynolds=1000.0, viscous=True, kappa=1.0)
    rng = np.random.default_rng(14)
    q = I.uniform_flow(curved, prm)
    du, dv = I.random_solenoidal_velocity(curved, rng, rms=1.0)
    q[1] += du
    q[2] += dv
    return [("c4_8x8_p3", c4.prm, c4.mesh, c4.q), ("c4_6x6_p4", c4p4.prm, c4p4.mesh, c4p4.q),
            ("curved_6x5_p4", prm, curved, q)]


_CASES = _mixed_cases()
_ORACLE_STEPS = {}


def _oracle_steps(name, prm, mesh, q0):
    """The oracle's BDF1 start-up step q0 -> q1 and its FP64 BDF2 step (q1, q0) -> q2."""
    if name not in _ORACLE_STEPS:
        o = Oracle(prm, mesh)
        kw = dict(tol_pseudo=1e-8, tol_res=1e-6, krylov=30, max_lin_it=300, max_newton=30)
        q1, s1 = o.bdf2_step(q0, None, 0.01, **kw)
        q2, s2 = o.bdf2_step(q1, q0, 0.01, **kw)
        assert s1["converged"] == 1 and s2["converged"] == 1
        _ORACLE_STEPS[name] = (q1, q2, s2)
    return _ORACLE_STEPS[name]


@pytest.mark.parametrize("precond", [0, 1, 2], ids=["block_jacobi", "gauss_seidel", "forward_gauss_seidel"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("case", _CASES, ids=[c[0] for c in _CASES])
def test_step_converged_state_matches_fp64_oracle(case, prec, precond):
    """One BDF2 step (Sec. 3.2, Eq. unsteady_pre_discretized_3; dt = 0.01, GMRES(30),
    tol_res 1e-6, Newton to Res_m/Res_0 <= 1e-8) from the oracle's start-up state, with the
    preconditioner blocks stored in `prec`, against the oracle's FP64 step."""
    name, prm, mesh, q0 = case
    q1, q2o, so = _oracle_steps(name, prm, mesh, q0)
    g = _ctx(prm, mesh)
    g.set_option("preconditioner", precond)
    q = _dev(q1)
    st = g.bdf2_step(q, _dev(q0), 0.01, tol_pseudo=1e-8, tol_res=1e-6, krylov=30, max_lin_it=300,
                     max_newton=30, prec=prec)
    torch.cuda.synchronize()
    q2 = q.cpu().numpy()
    rng_ = np.max(q2o, axis=(1, 2)) - np.min(q2o, axis=(1, 2))
    gap = np.max(np.abs(q2 - q2o), axis=(1, 2)) / rng_
    chg = np.max(np.abs(q2o - q1), axis=(1, 2))
    print(f"[mixed] {name} {prec} precond={precond} gpu {st} oracle newton {so['newton_its']} gmres "
          f"{so['gmres_its']}: gap / range {np.array2string(gap, precision=2)}, gap / step change "
          f"{np.array2string(np.max(np.abs(q2 - q2o), axis=(1, 2)) / chg, precision=2)}", flush=True)
    assert st["converged"] == 1
    assert np.all(gap <= (1e-8 if prec == "fp64" else 1e-5)), gap


def _storage_exact(x, prec):
    """x (float64) holds values exactly representable in the storage precision."""
    if prec == "fp64":
        return True
    if prec == "fp32":
        return np.array_equal(x.astype(np.float32).astype(np.float64), x)
    bits = x.astype(np.float32).view(np.uint32)
    return np.array_equal(x.astype(np.float32).astype(np.float64), x) and not np.any(bits & 0xFFFF)


@pytest.mark.parametrize("nx,ny,p", [(3, 3, 2), (4, 3, 3), (3, 2, 4)])
def test_stored_inverse_and_apply(nx, ny, p):
    """Per stored precision: the stored inverse is representable in it, lies within its
    rounding (plus the factorisation error, bounded by the block's condition number) of the
    inverse of the oracle's blocks, and the apply multiplies by exactly that inverse."""
    mesh = I.Mesh(nx, ny, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1))
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, kappa=1.0)
    q = I.taylor_green(mesh, prm)
    q[1] += 0.05
    q[2] -= 0.03
    o = Oracle(prm, mesh)
    ct, idt = 150.0, 1e-3
    Bo = o.blocks(q, ct, idt)
    inv_ex = np.linalg.inv(Bo)
    cond = np.array([np.linalg.cond(b) for b in Bo])
    g = _ctx(prm, mesh)
    r = np.random.default_rng(9).standard_normal(q.shape)
    E, Np = mesh.E, (p + 1) ** 2
    unit = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -8}   # half an ulp, relative
    for prec in ("fp64", "fp32", "bf16"):
        g.block_jacobi_factor(_dev(q), ct, idt, prec)
        X = g.get_inverse().cpu().numpy()
        z = g.block_jacobi_apply(_dev(r)).cpu().numpy()
        assert _storage_exact(X, prec), prec
        zref = np.einsum("eij,ej->ei", X, r.transpose(1, 0, 2).reshape(E, -1)).reshape(E, 4, Np).transpose(1, 0, 2)
        rel_apply = np.linalg.norm(z - zref) / np.linalg.norm(zref)
        # elementwise: storage rounding of each entry, plus a normwise factorisation error of
        # one unit of the arithmetic precision times the condition number (measured: a few
        # hundredths of that)
        arith = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
        dev = np.abs(X - inv_ex)
        bound = unit[prec] * np.abs(inv_ex) + (arith * cond)[:, None, None] * np.max(np.abs(inv_ex), axis=(1, 2),
                                                                                            keepdims=True)
        worst = np.max(dev / bound)
        print(f"[mixed] inverse {prec} p={p}: cond max {cond.max():.2e}, max |X - inv| / bound {worst:.2e}, "
              f"apply rel {rel_apply:.2e}", flush=True)
        assert worst <= 1.0, (prec, worst)
        assert rel_apply <= 1e-12, (prec, rel_apply)


def test_reserve_then_hot_path_allocates_nothing():
    """After fr_reserve, factor, apply, Newton operator and BDF2 steps (block Jacobi and Gauss-
    Seidel, every stored precision, graph replay off) leave the device's free memory as it was."""
    from paper_1903_06304_amd import lmfr
    c = I.config_c4(nx=8, p=3)
    g = _ctx(c.prm, c.mesh)
    g.set_option("graph", 0)
    g.reserve(30, "fp64")
    q = _dev(c.q)
    qs = q.clone()
    qm = q.clone()
    r = _dev(np.random.default_rng(1).standard_normal(c.q.shape))
    z = torch.empty_like(r)
    L = lmfr.load_library()
    torch.cuda.synchronize()
    free0, res0 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
    for precond in (0, 1, 2):
        g.set_option("preconditioner", precond)
        for prec in ("fp64", "fp32", "bf16"):
            g.block_jacobi_factor(q, 150.0, 0.0, prec)
            lmfr._check(L.fr_block_jacobi_apply(g.h, lmfr._ptr(r), lmfr._ptr(z), lmfr._stream()))
            lmfr._check(L.fr_bdf_operator(g.h, lmfr._ptr(q), lmfr._ptr(r), 150.0, 0.0, lmfr._ptr(z), lmfr._stream()))
            qs.copy_(q)
            st = g.bdf2_step(qs, None, 0.01, krylov=30, max_lin_it=300, prec=prec)
            assert st["converged"] == 1, st
            st = g.bdf2_step(qs, qm, 0.01, krylov=20, max_lin_it=300, prec=prec)
            assert st["converged"] == 1, st
    torch.cuda.synchronize()
    free1, res1 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
    print(f"[alloc] free device memory before {free0}, after {free1}; torch's reserve {res0} -> {res1}", flush=True)
    assert (free0 - free1) - (res1 - res0) == 0, (free0, free1, res0, res1)
