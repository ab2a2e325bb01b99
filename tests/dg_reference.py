"""Independent nodal-DG weak-form reference for scalar advection-diffusion on an
affine periodic rectangle mesh (test utility; shares nothing with the oracle).

u_t + div(a u - nu sigma) = 0, sigma = grad u + sum_f r_f (global lifting), with
the BR2 face gradient {grad u + r_f}, an upwind advective flux and the averaged
face value. Lagrange basis on Gauss-Legendre points built from a Legendre
Vandermonde matrix; exact mass matrix; Gauss quadrature of the interpolated flux.
The flux reconstruction scheme with Radau corrections must reproduce this
(paper Sec. 3.1: Radau corrections recover nodal DG).
"""
import numpy as np
import numpy.polynomial.legendre as L


def _basis(p):
    n = p + 1
    xi, w = L.leggauss(n)
    V = L.legvander(xi, p)            # V[i,k] = P_k(xi_i)
    C = np.linalg.inv(V)              # l_a(x) = sum_k C[k,a] P_k(x)
    dV = np.stack([L.legval(xi, L.legder(np.eye(p + 1)[k])) if p > 0 else np.zeros(n)
                   for k in range(p + 1)], axis=1)
    D = dV @ C                        # D[i,a] = l_a'(xi_i)
    lm = L.legvander(np.array([-1.0]), p)[0] @ C
    lp = L.legvander(np.array([1.0]), p)[0] @ C
    return xi, w, D, lm, lp


def dg_residual(u, nx, ny, hx, hy, p, ax, ay, nu):
    """du/dt for nodal values u[E][Np] (element e = ix + nx*iy, node i + n*j)."""
    n = p + 1
    xi, w, D, lm, lp = _basis(p)
    U = u.reshape(ny, nx, n, n)               # [iy, ix, j, i]
    sx, sy = 2.0 / hx, 2.0 / hy
    Ux = sx * np.einsum("ia,yxja->yxji", D, U)
    Uy = sy * np.einsum("jb,yxbi->yxji", D, U)
    # traces: left/right faces indexed by j, bottom/top by i
    uL = np.einsum("a,yxja->yxj", lm, U); uR = np.einsum("a,yxja->yxj", lp, U)
    uB = np.einsum("b,yxbi->yxi", lm, U); uT = np.einsum("b,yxbi->yxi", lp, U)
    tr = lambda F, lam, ax_: np.einsum("a,yxja->yxj", lam, F) if ax_ == "x" else np.einsum("b,yxbi->yxi", lam, F)
    # neighbour values
    nb_R_of_left = np.roll(uR, 1, axis=1)      # right trace of left neighbour
    nb_L_of_right = np.roll(uL, -1, axis=1)
    nb_T_of_bottom = np.roll(uT, 1, axis=0)
    nb_B_of_top = np.roll(uB, -1, axis=0)
    hL = 0.5 * (uL + nb_R_of_left); hR = 0.5 * (uR + nb_L_of_right)
    hB = 0.5 * (uB + nb_T_of_bottom); hT = 0.5 * (uT + nb_B_of_top)
    # local liftings (mass-matrix solve of the face integral), x/y components
    # r_left[ab] = M^-1 int_f phi_ab (uhat-u) n dS, n = (-1, 0)
    dl, dr, db, dt = hL - uL, hR - uR, hB - uB, hT - uT
    rLx = -sx * np.einsum("a,yxj->yxja", lm / w, dl)
    rRx = sx * np.einsum("a,yxj->yxja", lp / w, dr)
    rBy = -sy * np.einsum("b,yxi->yxbi", lm / w, db)
    rTy = sy * np.einsum("b,yxi->yxbi", lp / w, dt)
    Sx = Ux + rLx + rRx
    Sy = Uy + rBy + rTy
    # face gradients: trace of grad u plus the own local lifting of that face (normal comp.)
    gL = tr(Ux, lm, "x") + tr(rLx, lm, "x")
    gR = tr(Ux, lp, "x") + tr(rRx, lp, "x")
    gB = tr(Uy, lm, "y") + tr(rBy, lm, "y")
    gT = tr(Uy, lp, "y") + tr(rTy, lp, "y")
    # common normal-gradient component along +x on vertical faces, +y on horizontal faces
    # (the tangential parts do not enter sigma_hat . n on an axis-aligned face)
    # right face of element shared with left face of its right neighbour
    sR = 0.5 * (gR + np.roll(gL, -1, axis=1))
    sL = 0.5 * (gL + np.roll(gR, 1, axis=1))
    sT = 0.5 * (gT + np.roll(gB, -1, axis=0))
    sB = 0.5 * (gB + np.roll(gT, 1, axis=0))

    def upwind(an, um, up):
        return 0.5 * an * (um + up) - 0.5 * abs(an) * (up - um)

    fR = upwind(ax, uR, nb_L_of_right) - nu * sR          # outward n = +x
    fL = upwind(-ax, uL, nb_R_of_left) + nu * sL          # outward n = -x
    fT = upwind(ay, uT, nb_B_of_top) - nu * sT
    fB = upwind(-ay, uB, nb_T_of_bottom) + nu * sB
    Fx = ax * U - nu * Sx
    Fy = ay * U - nu * Sy
    # weak form: M du/dt = int grad(phi).F - int_dK phi F^.n
    vol = 0.5 * hy * np.einsum("j,i,ia,yxji->yxja", w, w, D, Fx) \
        + 0.5 * hx * np.einsum("i,j,jb,yxji->yxbi", w, w, D, Fy)
    bnd = 0.5 * hy * (np.einsum("a,j,yxj->yxja", lm, w, fL) + np.einsum("a,j,yxj->yxja", lp, w, fR)) \
        + 0.5 * hx * (np.einsum("b,i,yxi->yxbi", lm, w, fB) + np.einsum("b,i,yxi->yxbi", lp, w, fT))
    M = 0.25 * hx * hy * np.outer(w, w)            # [j, i]
    return ((vol - bnd) / M).reshape(ny * nx, n * n)
