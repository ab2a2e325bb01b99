// Pointwise physics of the preconditioned FR/CPR residual (device + host inline),
// templated on the scalar type (double or Dual<K>).
//
//  - non-dimensional Navier-Stokes fluxes, paper Sec. 2.1 Eqs. (convection),
//    (diffusion), (shear_stress); total flux f = f_inv - f_vis
//  - M = dq^c/dq^p and the Weiss-Smith matrix Gamma (rho_p -> Theta),
//    Sec. 2.2 Eqs. (jacobian), (preconditioning), (theta); both applied in the
//    compact row form  r0 = a dp + rho_T dT,  r1 = u r0 + rho du,  r2 = v r0 + rho dv,
//    r3 = h r0 - dp + rho (u du + v dv) + rho Cp dT  with a = rho_p (M) or Theta (Gamma)
//  - reference velocity U_r = eps c, eps = min(1, max(kappa Ma_inf, Ma)), Ma from
//    v - v_g, Eqs. (eps_nonmove), (eps_move)
//  - preconditioned Rusanov flux, Eq. (Rosanov), with |lambda|max = |u_n'| + c' of
//    Eqs. (eigenvalues), (eigenvalues_para) (alpha = (1 - eps^2)/2 because
//    beta U_r^2 = eps^2 for an ideal gas), moving-face normal flux of Sec. 3.1
//  - BR2 common gradient (Sec. 3.1) with the face-local Radau lifting evaluated at
//    the face: r = ((p+1)^2/2)(|S|/|J|_f)(q^com - q) n_out on each side.
//  - boundary faces (Sec. "Boundary Conditions"): the state and uncorrected gradient
//    beyond the face, formed from the own trace and fed to the same common flux.
#pragma once
#include "fr_scalar.hpp"

#define FR_DEV __device__ __forceinline__

struct PhysConst {
    double gam, Rg, Cp, inv_gm1, gRg, inv_Cp, inv_Rg;
    double mu_re, kc_re;      // mu/Re, (mu Cp/Pr)/Re
    double eps_min;           // kappa * Ma_inf
    double br2;               // (p+1)^2 / 2
};

// q^c = (rho, rho u, rho v, E), E = p/(gamma-1) + rho |v|^2 / 2, rho = p/(R T)
template <class T>
FR_DEV void fr_cons(const PhysConst& c, const T* q, T* qc) {
    T rho = q[0] * c.inv_Rg * rcp(q[3]);
    qc[0] = rho;
    qc[1] = rho * q[1];
    qc[2] = rho * q[2];
    qc[3] = q[0] * c.inv_gm1 + 0.5 * rho * (q[1] * q[1] + q[2] * q[2]);
}

// Total physical flux (f, g) = (f_inv - f_vis, g_inv - g_vis) and q^c at a point.
// gu, gv, gT: (d/dx, d/dy) of u, v, T.
template <class T, bool VISC>
FR_DEV void fr_point_flux(const PhysConst& c, const T* q, const T* gu, const T* gv, const T* gT,
                         T* f, T* g, T* qc) {
    fr_cons(c, q, qc);
    const T& p = q[0]; const T& u = q[1]; const T& v = q[2];
    T Ep = qc[3] + p;
    f[0] = qc[1];
    f[1] = qc[1] * u + p;
    f[2] = qc[1] * v;
    f[3] = Ep * u;
    g[0] = qc[2];
    g[1] = qc[2] * u;
    g[2] = qc[2] * v + p;
    g[3] = Ep * v;
    if (VISC) {
        // tau/Re with mu constant; heat flux k grad T / Re
        T div = gu[0] + gv[1];
        T txx = c.mu_re * (2.0 * gu[0] - (2.0 / 3.0) * div);
        T tyy = c.mu_re * (2.0 * gv[1] - (2.0 / 3.0) * div);
        T txy = c.mu_re * (gu[1] + gv[0]);
        f[1] = f[1] - txx;
        f[2] = f[2] - txy;
        f[3] = f[3] - (u * txx + v * txy + c.kc_re * gT[0]);
        g[1] = g[1] - txy;
        g[2] = g[2] - tyy;
        g[3] = g[3] - (u * txy + v * tyy + c.kc_re * gT[1]);
    }
}

// eps of the preconditioner from the velocity relative to the grid and the sound speed
template <class T>
FR_DEV T fr_eps(const PhysConst& c, const T& urel, const T& vrel, const T& cs) {
    T Ma = ssqrt(urel * urel + vrel * vrel) * rcp(cs);
    return smin(cst<T>(1.0), smax(cst<T>(c.eps_min), Ma));
}

// out = (a-row matrix) * dq with a = rho_p (M) or Theta (Gamma); state q.
template <class T, class V>
FR_DEV void fr_gm_apply(const PhysConst& c, const T& a, const T& rho, const T& rhoT, const T& h,
                       const T* q, const V* dq, V* out) {
    V r0 = a * dq[0] + rhoT * dq[3];
    out[0] = r0;
    out[1] = q[1] * r0 + rho * dq[1];
    out[2] = q[2] * r0 + rho * dq[2];
    out[3] = h * r0 - dq[0] + rho * (q[1] * dq[1] + q[2] * dq[2]) + (rho * c.Cp) * dq[3];
}

// Time-term operator at a solution point: out = inv_dtau Gamma(q) x + c_time M(q) x.
template <class T, class V>
FR_DEV void fr_time_apply(const PhysConst& c, const T* q, double ug, double vg, double inv_dtau,
                         double c_time, const V* x, V* out) {
    T iT = rcp(q[3]);
    T rho = q[0] * c.inv_Rg * iT;
    T rhoT = -rho * iT;
    T rhop = c.inv_Rg * iT;
    T cs = ssqrt(c.gRg * q[3]);
    T eps = fr_eps(c, q[1] - ug, q[2] - vg, cs);
    T Ur = eps * cs;
    T theta = rcp(Ur * Ur) + c.inv_Cp * iT;
    T h = c.Cp * q[3] + 0.5 * (q[1] * q[1] + q[2] * q[2]);
    V a[4], b[4];
    fr_gm_apply(c, theta, rho, rhoT, h, q, x, a);
    fr_gm_apply(c, rhop, rho, rhoT, h, q, x, b);
    for (int r = 0; r < 4; ++r) out[r] = inv_dtau * a[r] + c_time * b[r];
}

// Normal inviscid flux through a moving face: f n_x + g n_y - (v_g . n) q^c
template <class T>
FR_DEV void fr_normal_flux(const PhysConst& c, const T* q, double nx, double ny, double vgn, T* fn) {
    T qc[4];
    fr_cons(c, q, qc);
    T un = q[1] * nx + q[2] * ny;
    T unr = un - vgn;
    fn[0] = qc[0] * unr;
    fn[1] = qc[1] * unr + q[0] * nx;
    fn[2] = qc[2] * unr + q[0] * ny;
    fn[3] = qc[3] * unr + q[0] * un;
}

// Common normal flux at one face point, normal n = outward normal of the own ('-') side.
// Inviscid part: qm, qp are the primitive states of the own side and of the neighbour;
// returns fn (preconditioned Rusanov flux for n) and dq = q^+ - q^-.
template <class T>
FR_DEV void fr_common_inviscid(const PhysConst& c, const T* qm, const T* qp, double nx, double ny,
                               double ug, double vg, T* fn, T* dq) {
    const double vgn = ug * nx + vg * ny;
    T fL[4], fR[4];
    fr_normal_flux(c, qm, nx, ny, vgn, fL);
    fr_normal_flux(c, qp, nx, ny, vgn, fR);
    T qb[4];
    for (int r = 0; r < 4; ++r) {
        qb[r] = 0.5 * (qm[r] + qp[r]);
        dq[r] = qp[r] - qm[r];
        fn[r] = 0.5 * (fL[r] + fR[r]);
    }
    T iT = rcp(qb[3]);
    T rho = qb[0] * c.inv_Rg * iT;
    T cs = ssqrt(c.gRg * qb[3]);
    T ur = qb[1] - ug, vr = qb[2] - vg;
    T eps = fr_eps(c, ur, vr, cs);
    T Ur = eps * cs;
    T Ur2 = Ur * Ur;
    T theta = rcp(Ur2) + c.inv_Cp * iT;
    T rhoT = -rho * iT;
    T h = c.Cp * qb[3] + 0.5 * (qb[1] * qb[1] + qb[2] * qb[2]);
    T gd[4];
    fr_gm_apply(c, theta, rho, rhoT, h, qb, dq, gd);
    T un = ur * nx + vr * ny;
    T alpha = 0.5 * (1.0 - eps * eps);
    T unp = un * (1.0 - alpha);
    T cp = ssqrt(alpha * alpha * un * un + Ur2);
    T lam = sabs(unp) + cp;
    T hl = 0.5 * lam;
    for (int r = 0; r < 4; ++r) fn[r] = fn[r] - hl * gd[r];
}

// Viscous part (subtracted from fn): f_vis(q^com, grad q^com) . n with the BR2 common
// gradient grad q^com = (g^- + g^+)/2 + cc (q^+ - q^-) n  (cc = (p+1)^2/8 |S| (1/|J|^- + 1/|J|^+),
// the face-local Radau liftings of both sides evaluated at the face);
// gm, gp: uncorrected gradient traces (ux, uy, vx, vy, Tx, Ty); qcu, qcv: q^com velocity.
// Returns dqh = q^com - q^- for (u, v, T).
template <class T>
FR_DEV void fr_common_viscous(const PhysConst& c, const T* dq, const T& qcu, const T& qcv, const T* gm,
                              const T* gp, double nx, double ny, double cc, T* fn, T* dqh) {
    T ux = 0.5 * (gm[0] + gp[0]) + (cc * nx) * dq[1];
    T uy = 0.5 * (gm[1] + gp[1]) + (cc * ny) * dq[1];
    T vx = 0.5 * (gm[2] + gp[2]) + (cc * nx) * dq[2];
    T vy = 0.5 * (gm[3] + gp[3]) + (cc * ny) * dq[2];
    T Tn = 0.5 * ((gm[4] + gp[4]) * nx + (gm[5] + gp[5]) * ny) + cc * dq[3];
    T div = ux + vy;
    T txx = c.mu_re * (2.0 * ux - (2.0 / 3.0) * div);
    T tyy = c.mu_re * (2.0 * vy - (2.0 / 3.0) * div);
    T txy = c.mu_re * (uy + vx);
    T tnx = txx * nx + txy * ny;
    T tny = txy * nx + tyy * ny;
    fn[1] = fn[1] - tnx;
    fn[2] = fn[2] - tny;
    fn[3] = fn[3] - (qcu * tnx + qcv * tny + c.kc_re * Tn);
    dqh[0] = 0.5 * dq[1];
    dqh[1] = 0.5 * dq[2];
    dqh[2] = 0.5 * dq[3];
}

// ---- boundary faces.  Kinds: 1 far field, 2 slip wall, 3 adiabatic no-slip wall.
// n: unit outward normal of the own side; (wx, wy): grid velocity at the face point.
//  far field:  q^+ = q^inf (uniform: zero gradient);
//  slip wall:  mirror image across the wall, velocity relative to the wall:
//              v^+ = v - 2 ((v - w).n) n, p and T unchanged, gradients mirrored;
//  no-slip:    v^+ = 2 w - v, p and T unchanged, velocity gradient unchanged,
//              temperature gradient mirrored (its average has no normal part).
// The mirror of a gradient g is g - 2 (g.n) n; that of the velocity gradient
// G (G[a][b] = d u_a / d x_b) is Rm G Rm with Rm = I - 2 n n^T.
// qinf (4 doubles) is read whatever the kind, so it must always be readable (every context
// holds one); the far-field values are then selected like the other kinds' values, which keeps
// the compiler from turning the selection into a load through a stack copy of the candidates.
template <class T>
FR_DEV void fr_bc_state(int kind, const double* qinf, const T* qm, double nx, double ny, double wx, double wy,
                        T* qp) {
    const double qi0 = qinf[0], qi1 = qinf[1], qi2 = qinf[2], qi3 = qinf[3];
    const bool far = kind == 1, slip = kind == 2;
    const T urn = (qm[1] - wx) * nx + (qm[2] - wy) * ny;
    const T s1 = qm[1] - (2.0 * nx) * urn, s2 = qm[2] - (2.0 * ny) * urn;   // slip
    const T w1 = 2.0 * wx - qm[1], w2 = 2.0 * wy - qm[2];                   // no-slip
    qp[0] = far ? cst<T>(qi0) : qm[0];
    qp[1] = far ? cst<T>(qi1) : slip ? s1 : w1;
    qp[2] = far ? cst<T>(qi2) : slip ? s2 : w2;
    qp[3] = far ? cst<T>(qi3) : qm[3];
}

// The same map on a tangent (its linear part; the wall velocity and q^inf drop out).
// It is symmetric, so it also maps an adjoint of q^+ to the adjoint of q^-.
template <class T>
FR_DEV void fr_bc_state_lin(int kind, const T* dm, double nx, double ny, T* dp) {
    const T un = dm[1] * nx + dm[2] * ny;
    const bool far = kind == 1;
    const T zero = cst<T>(0.0);
    dp[0] = far ? zero : dm[0];
    dp[3] = far ? zero : dm[3];
    dp[1] = far ? zero : kind == 2 ? dm[1] - (2.0 * nx) * un : -dm[1];
    dp[2] = far ? zero : kind == 2 ? dm[2] - (2.0 * ny) * un : -dm[2];
}

// Uncorrected gradient beyond the face from the own trace gm = (ux, uy, vx, vy, Tx, Ty).
// Linear and symmetric (self-adjoint): it also maps tangents and adjoints.
template <class T>
FR_DEV void fr_bc_grad(int kind, const T* gm, double nx, double ny, T* gp) {
    const bool far = kind == 1, slip = kind == 2;
    const T zero = cst<T>(0.0);
    const T tn = gm[4] * nx + gm[5] * ny;
    gp[4] = far ? zero : gm[4] - (2.0 * nx) * tn;
    gp[5] = far ? zero : gm[5] - (2.0 * ny) * tn;
    // slip: Rm G Rm = G - 2 n (n^T G) - 2 (G n) n^T + 4 (n^T G n) n n^T
    const T a0 = nx * gm[0] + ny * gm[2], a1 = nx * gm[1] + ny * gm[3];   // n^T G
    const T b0 = gm[0] * nx + gm[1] * ny, b1 = gm[2] * nx + gm[3] * ny;   // G n
    const T s4 = 4.0 * (a0 * nx + a1 * ny);
    const T m0 = gm[0] - (2.0 * nx) * a0 - (2.0 * nx) * b0 + (nx * nx) * s4;
    const T m1 = gm[1] - (2.0 * nx) * a1 - (2.0 * ny) * b0 + (nx * ny) * s4;
    const T m2 = gm[2] - (2.0 * ny) * a0 - (2.0 * nx) * b1 + (ny * nx) * s4;
    const T m3 = gm[3] - (2.0 * ny) * a1 - (2.0 * ny) * b1 + (ny * ny) * s4;
    gp[0] = far ? zero : slip ? m0 : gm[0];
    gp[1] = far ? zero : slip ? m1 : gm[1];
    gp[2] = far ? zero : slip ? m2 : gm[2];
    gp[3] = far ? zero : slip ? m3 : gm[3];
}
