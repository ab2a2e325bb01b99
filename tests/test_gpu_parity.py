"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

Bars (written here, derived in the design notes):
  * R: per row, max |R_gpu - R_oracle| <= 1e-12 * max(S_c, S_d): S_c the flux scale, S_d the
    scale of the operands of the preconditioned Rusanov dissipation (tests/helpers.py); every
    test also prints the error over S_c alone;
  * JVP / BDF operator: per-row normwise relative error <= 1e-12;
  * element blocks: max abs error <= 1e-12 * max |block|;
  * block apply (every stored precision): within a bound derived from the storage rounding and
    the factorisation error of the stored inverse;
  * BDF2 step (FP64 blocks): converged states agree to 1e-8 relative per variable.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.oracle import Oracle  # noqa: E402
from paper_1903_06304_amd import inputs as I  # noqa: E402

from helpers import (affine_metric_noise, flux_scale, normwise_rel, residual_parity, row_errors,  # noqa: E402
                     small_cases)

pytestmark = pytest.mark.gpu


def _lmfr():
    from paper_1903_06304_amd import lmfr
    return lmfr


def _pair(prm, mesh, t=0.0):
    lmfr = _lmfr()
    xg, vg = mesh.nodes(t)
    o = Oracle(prm, mesh, xg, vg)
    nbr, nbf, flip = mesh.connectivity()
    g = lmfr.Context(prm, nbr, nbf, flip)
    g.set_geometry(xg, vg)
    return o, g


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


CASES = small_cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_residual_parity(case):
    name, prm, mesh, q, t = case
    print(f"[parity] residual {name} E={mesh.E}", flush=True)
    o, g = _pair(prm, mesh, t)
    # which elements take the constant-metric form of the neighbour gradient trace
    n_aff = g.affine_elements()
    if "halfaffine" in name:
        assert n_aff == mesh.E // 2, n_aff
    elif "affine" in name:
        assert n_aff == mesh.E, n_aff
    elif "curved" in name:
        assert n_aff == 0, n_aff
    R = g.residual(_dev(q)).cpu().numpy()
    Ro = o.residual(q)
    err_s = residual_parity(o.geometry(), prm, q, R, Ro)
    assert np.all(err_s <= 1e-12), (name, err_s)
    if "random" in name:
        # R is as large as its terms here, so a plain relative bar is meaningful
        assert np.all(normwise_rel(R, Ro) <= 1e-12), normwise_rel(R, Ro)


def test_residual_parity_c2_full():
    c = I.config_c2()
    print(f"[parity] residual C2 full E={c.mesh.E}", flush=True)
    o, g = _pair(c.prm, c.mesh)
    R = g.residual(_dev(c.q)).cpu().numpy()
    Ro = o.residual(c.q)
    err_s = residual_parity(o.geometry(), c.prm, c.q, R, Ro)
    assert np.all(err_s <= 1e-12), err_s
    print("  plain rel", normwise_rel(R, Ro), flush=True)


@pytest.mark.parametrize("p", [3, 4])
def test_residual_and_jvp_parity_c4_full(p):
    """The 256x256 affine workload at full size (p = 3: the headline residual; p = 4: the
    100 x 100-block steps), every row."""
    c = I.config_c4(p=p)
    print(f"[parity] residual + jvp C4 full p={p} E={c.mesh.E}", flush=True)
    o, g = _pair(c.prm, c.mesh)
    assert g.affine_elements() == c.mesh.E
    R = g.residual(_dev(c.q)).cpu().numpy()
    Ro = o.residual(c.q)
    err_s = residual_parity(o.geometry(), c.prm, c.q, R, Ro)
    assert np.all(err_s <= 1e-12), err_s
    v = np.random.default_rng(8).standard_normal(c.q.shape)
    Jv = g.jvp(_dev(c.q), _dev(v)).cpu().numpy()
    errj = normwise_rel(Jv, o.jvp(c.q, v))
    print("  jvp", errj, flush=True)
    assert np.all(errj <= 1e-12), errj


def test_residual_deterministic_and_free_stream():
    c = I.config_c3(nx=16, perturbed=False)
    o, g = _pair(c.prm, c.mesh, 0.07)
    q = _dev(c.q)
    R1 = g.residual(q)
    R2 = g.residual(q)
    assert torch.equal(R1, R2)
    S = flux_scale(o.geometry(), c.prm, c.q)
    assert np.all(np.max(np.abs(R1.cpu().numpy()).reshape(4, -1), axis=1) <= 1e-13 * S)


def _offset_tg(c):
    # Taylor-Green's odd symmetry puts averaged normal velocities exactly at the kink of
    # |lambda|max; derivative parity uses a state moved off it.
    q = c.q.copy()
    q[1] += 0.05
    q[2] -= 0.03
    return q


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_jvp_parity(case):
    name, prm, mesh, q, t = case
    print(f"[parity] jvp {name}", flush=True)
    if "curved" in name:
        q = q.copy(); q[1] += 0.05; q[2] -= 0.03
    o, g = _pair(prm, mesh, t)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(q.shape)
    Jv, R = g.jvp(_dev(q), _dev(v), want_residual=True)
    Jo = o.jvp(q, v)
    assert np.all(normwise_rel(Jv.cpu().numpy(), Jo) <= 1e-12), normwise_rel(Jv.cpu().numpy(), Jo)
    err_s = residual_parity(o.geometry(), prm, q, R.cpu().numpy(), o.residual(q), name)
    assert np.all(err_s <= 1e-12), err_s
    # without R the kernels carry only the tangent from the point fluxes on; the same bits at
    # both workgroup widths of the dual-number kernels (at 128 lanes an element of p = 2 or 4
    # spans two wavefronts), for the JVP and for the Newton operator
    Jt = g.jvp(_dev(q), _dev(v))
    A64 = g.bdf_operator(_dev(q), _dev(v), 150.0, 0.37)
    g.set_option("tile_lanes", 128)
    Jt128 = g.jvp(_dev(q), _dev(v))
    A128 = g.bdf_operator(_dev(q), _dev(v), 150.0, 0.37)
    torch.cuda.synchronize()
    err_t = normwise_rel(Jt.cpu().numpy(), Jo)
    print(f"  tangent-only jvp {err_t}", flush=True)
    assert np.all(err_t <= 1e-12), err_t
    assert torch.equal(Jt, Jt128)
    assert torch.equal(A64, A128)


def test_jvp_parity_c2_full():
    c = I.config_c2()
    q = _offset_tg(c)
    o, g = _pair(c.prm, c.mesh)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(q.shape)
    Jv = g.jvp(_dev(q), _dev(v)).cpu().numpy()
    Jo = o.jvp(q, v)
    err = normwise_rel(Jv, Jo)
    print("[parity] jvp C2 full", err, flush=True)
    assert np.all(err <= 1e-12), err


def test_bdf_operator_parity():
    c = I.config_c3(nx=4, p=2)
    o, g = _pair(c.prm, c.mesh, 0.05)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(c.q.shape)
    ct, idt = 150.0, 0.37
    Av = g.bdf_operator(_dev(c.q), _dev(v), ct, idt).cpu().numpy()
    # oracle: time terms from its blocks' diagonal point matrices, J v by complex step
    B0 = o.blocks(c.q, 0.0, 0.0)
    Bt = o.blocks(c.q, ct, idt)
    E, Np = o.E, o.Np
    ref = -o.jvp(c.q, v)
    for e in range(E):
        T = Bt[e] - B0[e]
        ve = v[:, e, :].reshape(-1)
        ref[:, e, :] += (T @ ve).reshape(4, Np)
    err = normwise_rel(Av, ref)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("packs", [0, 1])
@pytest.mark.parametrize("nx,ny,p,kind", [(3, 3, 2, "curved"), (1, 3, 1, "curved"), (2, 3, 2, "deforming"),
                                          (4, 3, 3, "curved"), (3, 2, 4, "curved"), (5, 3, 3, "affine"),
                                          (3, 4, 4, "affine")])
def test_blocks_parity(nx, ny, p, kind, packs):
    """Blocks from dual-number columns (packs = 0) and from tangent-only columns over the
    linearisation packs (packs = 1, the BDF2 step's path; on affine meshes every column of a
    block in one launch)."""
    print(f"[parity] blocks {nx}x{ny} p={p} {kind} packs={packs}", flush=True)
    if kind in ("curved", "affine"):
        mesh = I.Mesh(nx, ny, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi),
                      I.map_curved(0.1) if kind == "curved" else I.map_affine)
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, kappa=1.0)
        q = I.taylor_green(mesh, prm); q[1] += 0.05; q[2] -= 0.03
        t = 0.0
    else:
        mesh = I.Mesh(nx, ny, p, (0.0, 2.0, 0.0, 2.0), I.map_deforming(0.05), moving=True)
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, moving=True,
                       kappa=1.0)
        q = I.uniform_flow(mesh, prm)
        rng = np.random.default_rng(5)
        du, dv = I.random_solenoidal_velocity(mesh, rng, rms=0.2)
        q[1] += du; q[2] += dv
        t = 0.1
    o, g = _pair(prm, mesh, t)
    g.set_option("keep_blocks", 1)
    g.set_option("operator_packs", packs)
    ct, idt = 150.0, 1e-3
    g.block_jacobi_factor(_dev(q), ct, idt, "fp64")
    B = g.get_blocks().cpu().numpy()
    Bo = o.blocks(q, ct, idt)
    err = np.max(np.abs(B - Bo)) / np.max(np.abs(Bo))
    assert err <= 1e-12, err
    # apply in each precision vs a dense solve with the oracle's blocks
    rng = np.random.default_rng(9)
    r = rng.standard_normal(q.shape)
    E, Np = mesh.E, (p + 1) ** 2
    zref = np.zeros_like(r)
    for e in range(E):
        zref[:, e, :] = np.linalg.solve(Bo[e], r[:, e, :].reshape(-1)).reshape(4, Np)
    # bar per precision, from the arithmetic: the stored inverse is X~ = X + dX, X = B^-1, with
    # |dX| within half an ulp of storage, u_s |X|, plus the factorisation error, at most one unit
    # u_a of the factoring precision times cond(B) ||X||_2 in norm; the apply is z~ = X~ r in
    # FP64 (test_stored_inverse_and_apply checks both parts entry by entry), so per element
    # ||z~ - z|| <= u_s || |X| |r| || + u_a cond(B) ||X||_2 ||r||
    Xo = np.linalg.inv(Bo)
    cond = np.array([np.linalg.cond(b) for b in Bo])
    rE = r.transpose(1, 0, 2).reshape(E, -1)
    n2 = np.linalg.norm(Xo, ord=2, axis=(1, 2))
    unit = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -8}
    for prec in ("fp64", "fp32", "bf16"):
        arith = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
        b_e = unit[prec] * np.linalg.norm(np.einsum("eij,ej->ei", np.abs(Xo), np.abs(rE)), axis=1) \
            + arith * cond * n2 * np.linalg.norm(rE, axis=1)
        bar = np.sqrt(np.sum(b_e ** 2)) + 1e-12 * np.linalg.norm(zref)
        g.block_jacobi_factor(_dev(q), ct, idt, prec)
        z = g.block_jacobi_apply(_dev(r)).cpu().numpy()
        err = np.linalg.norm(z - zref)
        print(f"  apply {prec}: rel {err / np.linalg.norm(zref):.2e}, error / derived bar {err / bar:.2e}", flush=True)
        assert err <= bar, (prec, err, bar)


@pytest.mark.parametrize("gram_schmidt", [1, 2])
def test_bdf2_step_parity_c1(gram_schmidt):
    """C1 as stated: 8x8 p=2 vortex, dt = 0.01, GMRES(20)."""
    c = I.config_c1()
    o, g = _pair(c.prm, c.mesh)
    g.set_option("gram_schmidt", gram_schmidt)
    kw = dict(tol_pseudo=1e-10, tol_res=1e-9, krylov=20, max_lin_it=200, max_newton=20)
    qo, sto = o.bdf2_step(c.q, c.q_nm1, c.dt, **kw)
    qg = _dev(c.q)
    st = g.bdf2_step(qg, _dev(c.q_nm1), c.dt, **kw)
    torch.cuda.synchronize()
    print("[parity] bdf2 c1", st, sto, flush=True)
    assert st["converged"] == 1 and sto["converged"] == 1
    qg = qg.cpu().numpy()
    scale = np.max(np.abs(qo), axis=(1, 2))
    assert np.all(row_errors(qg, qo) <= 1e-8 * scale), row_errors(qg, qo) / scale


@pytest.mark.parametrize("graph", [1, 0])
def test_fused_gram_schmidt_equals_separate_passes(graph):
    """With two Gram-Schmidt passes the first pass's update and the second pass's dot products
    run in one read of the basis (up to 32 vectors, 8- / 16- / 32-wide variants); the step
    equals the one with separate update and dot kernels bit for bit.  GMRES(40) also runs
    Arnoldi steps past 32 vectors, where the separate kernels take over."""
    from paper_1903_06304_amd import lmfr
    c = I.config_c1()
    kw = dict(tol_pseudo=1e-10, tol_res=1e-12, krylov=40, max_lin_it=120, max_newton=3)
    out = {}
    for fused in (1, 0):
        g = lmfr.Context(c.prm, *c.mesh.connectivity())
        g.set_geometry(*c.mesh.nodes())
        g.set_option("gram_schmidt", 2)
        g.set_option("graph", graph)
        g.set_option("fused_gram_schmidt", fused)
        q = _dev(c.q)
        st = g.bdf2_step(q, _dev(c.q_nm1), c.dt, check=False, **kw)
        torch.cuda.synchronize()
        out[fused] = (q.cpu().numpy(), st)
    print("[parity] fused / separate Gram-Schmidt", out[1][1], out[0][1], flush=True)
    assert out[1][1]["gmres_its"] == out[0][1]["gmres_its"] and out[1][1]["gmres_its"] > 32
    assert np.array_equal(out[1][0], out[0][0])


def test_bdf2_step_deforming_free_stream():
    c = I.config_c3(nx=6, p=2, perturbed=False)
    o, g = _pair(c.prm, c.mesh, 0.05)
    q = _dev(c.q)
    st = g.bdf2_step(q, q.clone(), 0.01, krylov=10, tol_abs=1e-9 * c.prm.gas_constant)
    torch.cuda.synchronize()
    assert st["converged"] == 1
    d = (q.cpu().numpy() - c.q) / np.max(np.abs(c.q), axis=(1, 2))[:, None, None]
    assert np.max(np.abs(d)) < 1e-13


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_vjp_parity(case):
    """J^T w against the oracle's per-DOF complex-step adjoint, plus the adjoint identity."""
    name, prm, mesh, q, t = case
    print(f"[parity] vjp {name}", flush=True)
    if "curved" in name:
        q = q.copy(); q[1] += 0.05; q[2] -= 0.03
    o, g = _pair(prm, mesh, t)
    rng = np.random.default_rng(4)
    w = rng.standard_normal(q.shape)
    v = rng.standard_normal(q.shape)
    JTw = g.vjp(_dev(q), _dev(w)).cpu().numpy()
    ref = o.vjp_dofs(q, w, np.arange(q.size)).reshape(q.shape)
    err = normwise_rel(JTw, ref)
    assert np.all(err <= 1e-12), err
    Jv = g.jvp(_dev(q), _dev(v)).cpu().numpy()
    lhs, rhs = np.dot(w.ravel(), Jv.ravel()), np.dot(JTw.ravel(), v.ravel())
    assert abs(lhs - rhs) <= 1e-12 * np.abs(w.ravel() * Jv.ravel()).sum()


@pytest.mark.parametrize("p", [3, 4])
def test_vjp_parity_c4_sampled(p):
    """The 256x256 affine workload at full size (the benchmark's VJP): J^T w at sampled DOFs
    against the oracle's per-DOF complex-step adjoint.  This mesh takes the adjoint's affine
    path (neighbour traces from neighbour states, 7-word face adjoints); the samples include
    every DOF of a few elements at the mesh's periodic seams and at workgroup boundaries."""
    c = I.config_c4(p=p)
    o, g = _pair(c.prm, c.mesh)
    assert g.affine_elements() == c.mesh.E
    rng = np.random.default_rng(60 + p)
    w = rng.standard_normal(c.q.shape)
    JTw = g.vjp(_dev(c.q), _dev(w)).cpu().numpy()
    E, Np = c.mesh.E, (p + 1) ** 2
    els = np.unique(np.concatenate([[0, 255, 256, E - 256, E - 1], rng.choice(E, 6, replace=False),
                                    np.arange(7, 10)]))
    grid = np.stack(np.meshgrid(np.arange(4), els, np.arange(Np), indexing="ij"), -1).reshape(-1, 3)
    dofs = np.concatenate([np.ravel_multi_index(grid.T, (4, E, Np)), rng.choice(c.q.size, 300, replace=False)])
    ref = o.vjp_dofs(c.q, w, dofs)
    got = JTw.ravel()[dofs]
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    # the GPU takes one metric value per affine element where the oracle keeps the per-point
    # values; they differ by the rounding of the node coordinates (delta), as in residual_parity
    delta = affine_metric_noise(o.geometry())
    print(f"[parity] vjp C4 p={p} sampled ({dofs.size} DOFs) {err:.2e}, affine metric noise {delta:.1e}", flush=True)
    assert err / (1.0 + 2.0 * delta / 1e-12) <= 1e-12, (err, delta)


def test_vjp_parity_c2_sampled():
    c = I.config_c2()
    q = _offset_tg(c)
    o, g = _pair(c.prm, c.mesh)
    rng = np.random.default_rng(6)
    w = rng.standard_normal(q.shape)
    JTw = g.vjp(_dev(q), _dev(w)).cpu().numpy().ravel()
    dofs = rng.choice(q.size, 400, replace=False)
    ref = o.vjp_dofs(q, w, dofs)
    err = np.max(np.abs(JTw[dofs] - ref)) / np.max(np.abs(ref))
    print("[parity] vjp C2 sampled", err, flush=True)
    assert err <= 1e-12, err
    # autograd: backward of the FRResidual function is the VJP
    from paper_1903_06304_amd import lmfr
    qt = _dev(q).requires_grad_(True)
    R = lmfr.residual(qt, g)
    R.backward(_dev(w))
    assert torch.equal(qt.grad.reshape(-1).cpu(), torch.tensor(JTw))


def test_bdf2_graph_replay_matches_eager():
    """The captured GMRES cycle, replayed over several Newton/BDF2 steps with eager work and
    synchronisations in between, reproduces the uncaptured launches bit for bit."""
    c = I.config_c1(nx=4)
    results = {}
    for use_graph in (0, 1):
        o, g = _pair(c.prm, c.mesh)
        g.set_option("graph", use_graph)
        q = _dev(c.q)
        qm1 = _dev(c.q_nm1)
        hist = []
        for step in range(3):
            qn = q.clone()
            st = g.bdf2_step(q, qm1, c.dt, tol_pseudo=1e-10, tol_res=1e-9, krylov=8, max_lin_it=200)
            torch.cuda.synchronize()
            assert st["converged"] == 1, st
            R = g.residual(q)        # eager work between replays
            torch.cuda.synchronize()
            hist.append((q.clone(), st["gmres_its"], R.clone()))
            qm1 = qn
        results[use_graph] = hist
    for (qa, ia, Ra), (qb, ib, Rb) in zip(results[0], results[1]):
        assert ia == ib
        assert torch.equal(qa, qb)
        assert torch.equal(Ra, Rb)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_bdf_operator_packs_bitwise(case):
    """The Newton operator applied on tangents from stored linearisation packs (the form used
    inside GMRES) reproduces the dual-number operator to rounding: the two kernels form the
    same sums in the same order, and differ only where the compiler contracts a different
    product into a fused multiply-add (a few ulp)."""
    name, prm, mesh, q, t = case
    if "curved" in name:
        q = q.copy(); q[1] += 0.05; q[2] -= 0.03
    _, g = _pair(prm, mesh, t)
    rng = np.random.default_rng(21)
    v = _dev(rng.standard_normal(q.shape))
    qd = _dev(q)
    A0 = g.bdf_operator(qd, v, 150.0, 0.37)
    g.set_option("operator_packs", 1)
    A1 = g.bdf_operator(qd, v, 150.0, 0.37)
    torch.cuda.synchronize()
    err = normwise_rel(A1.cpu().numpy(), A0.cpu().numpy())
    assert np.all(err <= 1e-14), (name, err)


@pytest.mark.parametrize("precond", [0, 1])
def test_context_recovers_after_non_finite_step(precond):
    """A step from a non-finite state (reported as FR_ENONFINITE) leaves nothing behind in the
    context's solver buffers, chunk padding included: the next steps on the same context equal
    those on a fresh context bit for bit."""
    lmfr = _lmfr()
    c = I.config_c1(nx=8)
    kw = dict(tol_pseudo=1e-10, tol_res=1e-9, krylov=20, max_lin_it=200, max_newton=20)

    def ctx():
        g = lmfr.Context(c.prm, *c.mesh.connectivity())
        g.set_geometry(*c.mesh.nodes(0.0))
        g.set_option("preconditioner", precond)
        return g

    used = ctx()
    bad = c.q.copy()
    bad[3, 5, 2] = np.nan
    st = used.bdf2_step(_dev(bad), _dev(c.q_nm1), c.dt, check=False, **kw)
    torch.cuda.synchronize()
    print("[parity] non-finite step", st, flush=True)
    assert st["rc"] == lmfr.FR_ENONFINITE and st["converged"] == 0
    out = {}
    for name, g_ in (("used", used), ("fresh", ctx())):
        q = _dev(c.q)
        out[name] = (q, g_.bdf2_step(q, _dev(c.q_nm1), c.dt, **kw))
    torch.cuda.synchronize()
    print("[parity] after it", out["used"][1], "fresh", out["fresh"][1], flush=True)
    assert out["used"][1]["converged"] == 1
    assert out["used"][1]["gmres_its"] == out["fresh"][1]["gmres_its"]
    assert torch.equal(out["used"][0], out["fresh"][0])


def _renumbered(name):
    """A mesh whose elements' local frames are turned by seeded quarter turns: faces meet
    arbitrary faces of their neighbours, half of them with reversed point order."""
    if name == "affine":
        mesh = I.Mesh(6, 5, 3, (0.0, 2 * np.pi, 0.0, 2 * np.pi))
        prm = I.Params(order=3, n_elem=mesh.E, mach_ref=0.2, reynolds=50.0, viscous=True, kappa=1.0)
        t = 0.0
    elif name == "curved":
        mesh = I.Mesh(5, 6, 4, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1))
        prm = I.Params(order=4, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, kappa=1.0)
        t = 0.0
    elif name == "deforming":
        mesh = I.Mesh(6, 4, 2, (0.0, 2.0, 0.0, 2.0), I.map_deforming(0.05), moving=True)
        prm = I.Params(order=2, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, moving=True, kappa=1.0)
        t = 0.13
    else:
        mesh = I.Mesh(5, 4, 2, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1),
                      bc=(I.BC_FARFIELD, I.BC_FARFIELD, I.BC_NOSLIP_WALL, I.BC_SLIP_WALL))
        prm = I.Params(order=2, n_elem=mesh.E, mach_ref=0.1, reynolds=50.0, viscous=True, kappa=1.0)
        t = 0.0
    rng = np.random.default_rng(31)
    q = I.uniform_flow(mesh, prm)
    q[0] *= 1 + 0.05 * rng.standard_normal(q[0].shape)
    q[1] += 0.3 * rng.standard_normal(q[1].shape)
    q[2] += 0.3 * rng.standard_normal(q[2].shape)
    q[3] *= 1 + 0.03 * rng.standard_normal(q[3].shape)
    rot = rng.integers(0, 4, mesh.E)
    rot[0], rot[1] = 1, 2
    nb2, nf2, fl2, carry = I.renumber_elements(*mesh.connectivity(), rot)
    xg, vg = mesh.nodes(t)
    return prm, mesh, (nb2, nf2, fl2), carry(xg), None if vg is None else carry(vg), carry(q)


@pytest.mark.parametrize("name", ["affine", "curved", "deforming", "boundary"])
def test_renumbered_mesh_parity(name):
    """Faces that meet a neighbour face other than the opposite one, and reversed face-point
    order (the h_nbr_face and h_flip tables of fr_create): R, JVP, VJP, blocks and the Newton
    operator against the oracle on the same tables."""
    lmfr = _lmfr()
    prm, mesh, conn, xg, vg, q = _renumbered(name)
    print(f"[parity] renumbered {name} E={mesh.E} flips={int(np.sum(conn[2]))}", flush=True)

    class M:
        E = mesh.E

        def connectivity(self):
            return conn

    o = Oracle(prm, M(), xg, vg)
    g = lmfr.Context(prm, *conn)
    g.set_geometry(xg, vg)
    if name == "boundary":
        qinf = [prm.gas_constant, 0.9, 0.1, 1.0]
        o.set_farfield(qinf)
        g.set_farfield(qinf)
    if name == "affine":
        assert g.affine_elements() == mesh.E
    R = g.residual(_dev(q)).cpu().numpy()
    Ro = o.residual(q)
    err_s = residual_parity(o.geometry(), prm, q, R, Ro, name)
    assert np.all(err_s <= 1e-12), err_s
    assert np.all(normwise_rel(R, Ro) <= 1e-12), normwise_rel(R, Ro)
    rng = np.random.default_rng(5)
    v, w = rng.standard_normal(q.shape), rng.standard_normal(q.shape)
    errj = normwise_rel(g.jvp(_dev(q), _dev(v)).cpu().numpy(), o.jvp(q, v))
    errv = normwise_rel(g.vjp(_dev(q), _dev(w)).cpu().numpy(), o.vjp_dofs(q, w, np.arange(q.size)).reshape(q.shape))
    print("  jvp", errj, "vjp", errv, flush=True)
    assert np.all(errj <= 1e-12) and np.all(errv <= 1e-12), (errj, errv)
    g.set_option("keep_blocks", 1)
    for packs in (0, 1):
        g.set_option("operator_packs", packs)
        g.block_jacobi_factor(_dev(q), 150.0, 1e-3, "fp64")
        B = g.get_blocks().cpu().numpy()
        Bo = o.blocks(q, 150.0, 1e-3)
        errb = np.max(np.abs(B - Bo)) / np.max(np.abs(Bo))
        Av = g.bdf_operator(_dev(q), _dev(v), 150.0, 1e-3).cpu().numpy()
        B0 = o.blocks(q, 0.0, 0.0)
        ref = -o.jvp(q, v)
        for e in range(mesh.E):
            ref[:, e, :] += ((Bo[e] - B0[e]) @ v[:, e, :].reshape(-1)).reshape(4, -1)
        erra = normwise_rel(Av, ref)
        print(f"  packs={packs} blocks {errb:.2e} operator {erra}", flush=True)
        assert errb <= 1e-12 and np.all(erra <= 1e-12), (errb, erra)


def test_forward_mode_through_frresidual():
    """torch.func.jvp and torch.autograd.forward_ad through FRResidual give fr_jvp bit for bit,
    and the primal output is fr_residual."""
    lmfr = _lmfr()
    c = I.config_c2(nx=6)
    q = _offset_tg(c)
    _, g = _pair(c.prm, c.mesh)
    qd = _dev(q)
    v = _dev(np.random.default_rng(12).standard_normal(q.shape))
    Jv_ref = g.jvp(qd, v)
    R_ref = g.residual(qd)
    R1, Jv1 = torch.func.jvp(lambda x: lmfr.residual(x, g), (qd,), (v,))
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        dual = fwAD.make_dual(qd, v)
        out = lmfr.residual(dual, g)
        R2, Jv2 = fwAD.unpack_dual(out)
    torch.cuda.synchronize()
    assert torch.equal(R1, R_ref) and torch.equal(R2, R_ref)
    assert torch.equal(Jv1, Jv_ref) and torch.equal(Jv2, Jv_ref)
