"""Resume from a checkpoint on the GPU path: a BDF2 march on a moving mesh (paper Sec. 3.2,
Sec. 4.3's prescribed motion) stopped after two steps, written to a file, read into a fresh
context and continued, gives the same states bit for bit as the march that did not stop."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1903_06304_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

DOM = (-10.0, 10.0, -10.0, 10.0)


def _setup(p=2, N=6):
    from paper_1903_06304_amd import lmfr
    mesh = I.Mesh(N, N, p, DOM, I.map_vortex_motion(1.0, 1.0, 0.1, 0.1), moving=True)
    prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, viscous=False, moving=True, kappa=1.0)
    g = lmfr.Context(prm, *mesh.connectivity())
    return mesh, prm, g


def _step(g, mesh, q, qm1, t_new, dt, prec):
    g.set_geometry(*mesh.nodes(t_new))
    st = g.bdf2_step(q, qm1, dt, tol_pseudo=1e-10, tol_res=1e-6, krylov=20, max_lin_it=100, max_newton=30,
                     prec=prec, check=False)
    assert st["rc"] in (0, -5) and st["converged"] == 1, st
    return st


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_resume_from_checkpoint_equals_continuous_march(tmp_path, prec):
    from paper_1903_06304_amd import lmfr
    dt, nsteps = 0.02, 3
    mesh, prm, g = _setup()
    q0 = torch.tensor(I.isentropic_vortex(mesh, prm, t=0.0, center=(0.0, 0.0), xy=mesh.solution_points(0.0)),
                      device="cuda")
    # continuous: BDF1 start, then BDF2
    q, qm1 = q0.clone(), None
    states = []
    for n in range(nsteps):
        qn = q.clone()
        _step(g, mesh, q, qm1, (n + 1) * dt, dt, prec)
        qm1 = qn
        states.append(q.clone())
    # stopped after two steps, written, read into a fresh context, continued
    q, qm1 = q0.clone(), None
    for n in range(2):
        qn = q.clone()
        _step(g, mesh, q, qm1, (n + 1) * dt, dt, prec)
        qm1 = qn
    lmfr.save_checkpoint(tmp_path / "s.safetensors", q, qm1, 2 * dt, dt, step=2)
    del g
    torch.cuda.synchronize()
    _, _, g2 = _setup()
    ck = lmfr.load_checkpoint(tmp_path / "s.safetensors")
    assert ck["step"] == 2 and ck["t"] == 2 * dt and ck["dt"] == dt
    assert torch.equal(ck["q"], states[1])   # the saved state is step 2's
    q2 = ck["q"].clone()
    _step(g2, mesh, q2, ck["q_nm1"], (ck["step"] + 1) * ck["dt"], ck["dt"], prec)   # the same time value
    torch.cuda.synchronize()
    assert torch.equal(q2, states[2]), float((q2 - states[2]).abs().max())
