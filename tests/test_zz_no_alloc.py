"""fr_vjp_noalloc (the allocation-free variant of fr_vjp) through the C ABI: the same values
as fr_vjp, bit for bit, on two calls in a row (the second on a smaller mesh), no change of
the device's free memory, and sizes above the scratch maximum rejected."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1903_06304_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


def _case(nx, ny, p, kind, seed):
    if kind in ("curved", "affine"):
        # affine static meshes take the adjoint's path without the trace buffer
        mesh = I.Mesh(nx, ny, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi),
                      I.map_curved(0.1) if kind == "curved" else I.map_affine)
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, kappa=1.0)
        t = 0.0
    else:
        mesh = I.Mesh(nx, ny, p, (0.0, 2.0, 0.0, 2.0), I.map_deforming(0.05), moving=True)
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, moving=True, kappa=1.0)
        t = 0.1
    rng = np.random.default_rng(seed)
    q = I.uniform_flow(mesh, prm)
    du, dv = I.random_solenoidal_velocity(mesh, rng, rms=0.3)
    q[1] += du
    q[2] += dv
    return prm, mesh, t, q, rng.standard_normal(q.shape)


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def test_vjp_noalloc_matches_vjp():
    from paper_1903_06304_amd import lmfr
    L = lmfr.load_library()
    # each later mesh is smaller than the first
    cases = [_case(64, 48, 3, "curved", 1), _case(9, 7, 2, "deforming", 2), _case(20, 16, 3, "affine", 3)]
    ctxs, args = [], []
    for prm, mesh, t, q, w in cases:
        g = lmfr.Context(prm, *mesh.connectivity())
        g.set_geometry(*mesh.nodes(t))
        if mesh.mapping is I.map_affine:
            assert g.affine_elements() == mesh.E
        qd, wd = _dev(q), _dev(w)
        ctxs.append(g)
        args.append((qd, wd, torch.empty_like(qd), torch.empty_like(qd)))
    # fr_vjp on both meshes first: the runtime loads the library's code (and with it each
    # device's copy of the scratch array) when the kernels first run
    for g, (qd, wd, ref, out) in zip(ctxs, args):
        lmfr._check(L.fr_vjp(g.h, lmfr._ptr(qd), lmfr._ptr(wd), lmfr._ptr(ref), lmfr._stream()))
    torch.cuda.synchronize()
    free0, res0 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
    for g, (qd, wd, ref, out) in zip(ctxs, args):
        print(f"[noalloc] E={g.E} Np={g.Np}", flush=True)
        lmfr._check(L.fr_vjp_noalloc(g.h, lmfr._ptr(qd), lmfr._ptr(wd), lmfr._ptr(out), lmfr._stream()))
    torch.cuda.synchronize()
    free1, res1 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
    print(f"[noalloc] free device memory {free0} -> {free1}, torch's reserve {res0} -> {res1}", flush=True)
    assert free1 == free0 and res1 == res0, (free0, free1, res0, res1)
    for g, (qd, wd, ref, out) in zip(ctxs, args):
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), (out - ref).abs().max().item()
    # the first context again, after the smaller one left its values in the shared array
    g, (qd, wd, ref, out) = ctxs[0], args[0]
    out.zero_()
    lmfr._check(L.fr_vjp_noalloc(g.h, lmfr._ptr(qd), lmfr._ptr(wd), lmfr._ptr(out), lmfr._stream()))
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_vjp_noalloc_rejects_meshes_above_the_maximum():
    from paper_1903_06304_amd import lmfr
    L = lmfr.load_library()
    mesh = I.Mesh(128, 128, 3, (0.0, 2 * np.pi, 0.0, 2 * np.pi))
    prm = I.Params(order=3, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, kappa=1.0)
    g = lmfr.Context(prm, *mesh.connectivity())
    g.set_geometry(*mesh.nodes(0.0))
    q = _dev(I.uniform_flow(mesh, prm))
    out = torch.empty_like(q)
    rc = L.fr_vjp_noalloc(g.h, lmfr._ptr(q), lmfr._ptr(q), lmfr._ptr(out), lmfr._stream())
    assert rc == lmfr.FR_EINVAL
    assert b"maximum" in L.fr_last_error()
