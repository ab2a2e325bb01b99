"""Shared test helpers: scales for residual parity and case construction."""
import numpy as np

from paper_1903_06304_amd import inputs as I


def flux_scale(geo, prm, q, parts=False):
    """Per-row scale of the terms summed into row c of R, for residual parity.

    Round-off in R is proportional to the magnitudes of the summed terms, not to R (a plain
    relative error is ill-posed at low Mach number).  Two scales, both multiplied by the
    largest metric norm max |grad xi| through which every term enters R:
      * S_c: the largest |f_c| + |g_c| + |v_g| |q^c_c| over the solution points, the
        inviscid fluxes and the grid-velocity term;
      * S_d: the largest |lambda|max (|Gamma~| |q^p|)_c, the size of the two operands whose
        difference the preconditioned Rusanov dissipation of Eq. (Rosanov) takes.  Its
        |lambda|max is the preconditioned |u_n'| + c' of Eqs. (eigenvalues_para), (eps_move),
        bounded over normal directions by |u_n| <= |v - v_g|.  At low Mach number its pressure
        part Theta |p| exceeds S_c in the mass row.
    Returns max(S_c, S_d) per row, or (S_c, S_d) with parts=True."""
    p, u, v, T = q
    Rg, Cp = prm.gas_constant, prm.cp
    rho = p / (Rg * T)
    E = p / (prm.gamma - 1) + 0.5 * rho * (u * u + v * v)
    f = np.stack([rho * u, rho * u * u + p, rho * u * v, (E + p) * u])
    g = np.stack([rho * v, rho * u * v, rho * v * v + p, (E + p) * v])
    qc = np.stack([rho, rho * u, rho * v, E])
    vg = np.hypot(geo["ug"], geo["vg"])
    c = np.sqrt(prm.gamma * Rg * T)
    w = np.hypot(u - geo["ug"], v - geo["vg"])
    eps = np.minimum(1.0, np.maximum(prm.kappa * prm.mach_inf, w / c))
    Ur = eps * c
    alpha = 0.5 * (1.0 - eps ** 2)
    lam = (1.0 - alpha) * w + np.sqrt(alpha ** 2 * w ** 2 + Ur ** 2)
    theta = 1.0 / Ur ** 2 + 1.0 / (Cp * T)
    h = Cp * T + 0.5 * (u * u + v * v)
    rT = rho / T
    # |Gamma~| |q^p| row by row (Eq. preconditioning with Theta of Eq. theta)
    gq = np.stack([theta * np.abs(p) + rT * T,
                   np.abs(u) * (theta * np.abs(p) + rT * T) + rho * np.abs(u),
                   np.abs(v) * (theta * np.abs(p) + rT * T) + rho * np.abs(v),
                   (theta * h + 1.0) * np.abs(p) + rho * (u * u + v * v) + (rT * h + rho * Cp) * T])
    gm = np.max(np.sqrt(np.maximum(geo["xix"] ** 2 + geo["xiy"] ** 2, geo["etx"] ** 2 + geo["ety"] ** 2)))
    S_c = np.max(np.abs(f) + np.abs(g) + vg * np.abs(qc), axis=(1, 2)) * gm
    S_d = np.max(lam * gq, axis=(1, 2)) * gm
    if parts:
        return S_c, S_d
    return np.maximum(S_c, S_d)


def row_errors(a, b):
    """Per-row max abs difference of two [4][E][Np] arrays."""
    return np.max(np.abs(np.asarray(a) - np.asarray(b)).reshape(4, -1), axis=1)


def normwise_rel(a, b):
    """Per-row ||a - b|| / ||b||."""
    a = np.asarray(a).reshape(4, -1)
    b = np.asarray(b).reshape(4, -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def map_half_curved(amp):
    """Identity for x in [0, pi], the curved map for x in [pi, 2 pi] (continuous at both ends):
    on a mesh with an even number of columns half of the elements are affine."""
    def f(xr, yr, t):
        d = amp * np.minimum(np.sin(xr), 0.0) * np.sin(yr)
        z = np.zeros_like(xr)
        return xr + d, yr + d, z, z.copy()
    return f


def small_cases():
    """Small meshes of every kind, sized so several workgroups and a ragged tail occur."""
    out = []
    c1 = I.config_c1(nx=8)
    out.append(("c1_euler_p2_8x8", c1.prm, c1.mesh, c1.q, 0.0))
    for p in (1, 2, 3, 4):
        mesh = I.Mesh(7, 5, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1))
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.05, reynolds=100.0, viscous=True, kappa=1.0)
        q = I.taylor_green(mesh, prm)
        out.append((f"ns_curved_p{p}_7x5", prm, mesh, q, 0.0))
    for p in (2, 3):
        mesh = I.Mesh(6, 9, p, (0.0, 2.0, 0.0, 2.0), I.map_deforming(0.05), moving=True)
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.01, reynolds=100.0, viscous=True,
                       moving=True, kappa=1.0)
        q = I.uniform_flow(mesh, prm)
        rng = np.random.default_rng(3)
        du, dv = I.random_solenoidal_velocity(mesh, rng, rms=1e-3)
        q[1] += du
        q[2] += dv
        out.append((f"ns_deforming_p{p}_6x9", prm, mesh, q, 0.13))
    mesh = I.Mesh(5, 4, 3, (0.0, 2 * np.pi, 0.0, 2 * np.pi), I.map_curved(0.1))
    prm = I.Params(order=3, n_elem=mesh.E, mach_ref=0.3, reynolds=50.0, viscous=True, kappa=1.0)
    out.append(("ns_curved_p3_ma0.3", prm, mesh, I.taylor_green(mesh, prm), 0.0))
    for p in (1, 2, 3, 4):
        # randomised states: O(1) jumps between elements and temperature variation, so every
        # term (dissipation, BR2, heat flux) is exercised and R is as large as its terms
        mov = p % 2 == 0
        mapping = I.map_deforming(0.05, np.pi) if mov else I.map_curved(0.1)
        mesh = I.Mesh(5, 6, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi), mapping, moving=mov)
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.2, reynolds=50.0, viscous=True, moving=mov,
                       kappa=1.0)
        rng = np.random.default_rng(40 + p)
        q = I.uniform_flow(mesh, prm)
        q[0] *= 1 + 0.05 * rng.standard_normal(q[0].shape)
        q[1] += 0.3 * rng.standard_normal(q[1].shape)
        q[2] += 0.3 * rng.standard_normal(q[2].shape)
        q[3] *= 1 + 0.03 * rng.standard_normal(q[3].shape)
        out.append((f"ns_random_p{p}", prm, mesh, q, 0.21 if mov else 0.0))
    for p in (1, 2, 3, 4):
        # affine elements (the kind of the 256x256 workload): an affine neighbour's gradient
        # trace is formed from its traces; the half-curved mesh puts both forms side by side
        half = p == 3
        mapping = map_half_curved(0.1) if half else I.map_affine
        mesh = I.Mesh(6, 5, p, (0.0, 2 * np.pi, 0.0, 2 * np.pi), mapping)
        prm = I.Params(order=p, n_elem=mesh.E, mach_ref=0.2, reynolds=50.0, viscous=True, kappa=1.0)
        rng = np.random.default_rng(50 + p)
        q = I.uniform_flow(mesh, prm)
        q[0] *= 1 + 0.05 * rng.standard_normal(q[0].shape)
        q[1] += 0.3 * rng.standard_normal(q[1].shape)
        q[2] += 0.3 * rng.standard_normal(q[2].shape)
        q[3] *= 1 + 0.03 * rng.standard_normal(q[3].shape)
        out.append((f"ns_random_{'halfaffine' if half else 'affine'}_p{p}", prm, mesh, q, 0.0))
    mesh = I.Mesh(5, 6, 2, (0.0, 10.0, 0.0, 10.0), I.map_vortex_motion(0.5, 1.0, 0.1, 0.1), moving=True)
    prm = I.Params(order=2, n_elem=mesh.E, mach_ref=0.1, moving=True, kappa=0.0)
    out.append(("euler_moving_p2", prm, mesh, I.isentropic_vortex(mesh, prm, xy=mesh.solution_points(0.1)), 0.1))
    return out


def affine_metric_noise(geo):
    """Largest variation of the metric terms over an element that counts as affine.

    An element is affine when every metric term is constant over it to 1e-10 of the metric
    scale (the affine reading of the design notes); the GPU then uses one value per element
    where the oracle keeps the per-point values, which differ by the rounding of the node
    coordinates (about 1e-12 relative on a 256 x 256 mesh of [0, 2 pi]^2).  Returns the
    largest such relative variation over the affine elements (0 if there are none)."""
    ms = max(np.max(np.abs(geo[k])) for k in ("xix", "xiy", "etx", "ety"))
    var = np.zeros(geo["xix"].shape[0])
    for k in ("xix", "xiy", "etx", "ety"):
        var = np.maximum(var, (geo[k].max(axis=1) - geo[k].min(axis=1)) / ms)
    j = geo["jac"]
    var = np.maximum(var, (j.max(axis=1) - j.min(axis=1)) / np.max(np.abs(j)))
    aff = var <= 1e-10
    return float(np.max(var[aff])) if np.any(aff) else 0.0


def residual_parity(geo, prm, q, R, Ro, tag=""):
    """Per-row max |R - Ro| over the parity scale max(S_c, S_d) of flux_scale, normalised so
    that the bar is 1e-12: the scale is multiplied by 1 + 2 delta / 1e-12, delta the metric
    noise of the affine elements (affine_metric_noise; negligible below 1e-13 except on the
    finest affine meshes).  Prints the raw error over S and over S_c alone (the flux-only
    scale), delta and the plain normwise relative error."""
    S_c, S_d = flux_scale(geo, prm, q, parts=True)
    err = row_errors(R, Ro)
    raw = err / np.maximum(S_c, S_d)
    delta = affine_metric_noise(geo)
    print(f"  {tag} err/S {np.array2string(raw, precision=2)}  err/S_c {np.array2string(err / S_c, precision=2)}"
          f"  affine metric noise {delta:.1e}  plain rel {np.array2string(normwise_rel(R, Ro), precision=2)}",
          flush=True)
    return raw / (1.0 + 2.0 * delta / 1e-12)
