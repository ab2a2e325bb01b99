// Vector-Jacobian products J^T w of the FR/CPR residual (reverse / adjoint mode).
//
// Gather formulation, three kernels, no atomics (bitwise deterministic):
//   1. value traces of every element (k_traces of the forward path); static meshes whose
//      elements are all affine skip it: the element kernel forms the neighbour traces
//      itself from the neighbour's line of states through each face point, with the
//      neighbour's constant metrics, as the affine residual kernel does;
//   2. k_vjp_elem: for each element e, recompute the forward stages in LDS and run
//      them backwards with the adjoint seed w_e: Radau lift and chain-rule divergence
//      (transposed), point fluxes (hand-derived adjoint), corrected gradient, the
//      preconditioned Rusanov + BR2 common flux (hand-derived adjoint), traces and the
//      uncorrected gradient (transposed).  The adjoint with respect to q_e is written
//      to the output; the adjoint with respect to each neighbour trace that e used is
//      written to a per-side buffer;
//   3. k_vjp_gather: each element collects, from its neighbours' side buffers, the
//      adjoint of its own traces and applies the trace / gradient transposes.
// Non-smooth points follow the forward convention: eps = Ma only when
// eps_min < Ma < 1, d|x|/dx = +1 at x = 0.
#include "fr_internal.hpp"

#include <mutex>

namespace {

template <int P>
struct Sz {
    static constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = (Np > NF ? Np : NF);
    static constexpr int EPB = (128 / NT) > 0 ? 128 / NT : 1;
    static constexpr int threads = EPB * NT;
};

__device__ __forceinline__ int line_pt(int n, int f, int k, int a) { return f < 2 ? a + n * k : k + n * a; }

// tile of workgroup b of a grid of 8 * per workgroups: workgroups go to the 8 XCDs round robin
// (b % 8), so XCD x takes the contiguous tiles x * per .. x * per + per - 1 and the face
// neighbours of a tile (the next tile, the next row of tiles) mostly share its L2
__device__ __forceinline__ int xcd_tile(int per) {
    return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

// ---------------------------------------------------------------- pointwise adjoints
// adjoint of the total flux (f, g) and q^c at a point w.r.t. q and the corrected gradient
template <bool VISC>
__device__ void point_flux_rev(const PhysConst& c, const double* q, const double* G, const double* af,
                               const double* ag, const double* aqc, double* aq, double* aG) {
    const double p = q[0], u = q[1], v = q[2], T = q[3];
    const double iT = 1.0 / T;   // one division; the quotients below multiply by it
    const double rho = p * c.inv_Rg * iT;
    const double ru = rho * u, rv = rho * v, k2 = u * u + v * v;
    const double E = p * c.inv_gm1 + 0.5 * rho * k2;
    const double Ep = E + p;
    double txx = 0, tyy = 0, txy = 0;
    if (VISC) {
        const double div = G[0] + G[3];
        txx = c.mu_re * (2.0 * G[0] - (2.0 / 3.0) * div);
        tyy = c.mu_re * (2.0 * G[3] - (2.0 / 3.0) * div);
        txy = c.mu_re * (G[1] + G[2]);
    }
    double a_ru = 0, a_rv = 0, a_u = 0, a_v = 0, a_p = 0, a_Ep = 0, a_E = 0, a_rho = 0, a_T = 0;
    double a_txx = 0, a_tyy = 0, a_txy = 0, a_Tx = 0, a_Ty = 0;
    a_ru += af[0];
    a_ru += af[1] * u; a_u += af[1] * ru; a_p += af[1];
    a_ru += af[2] * v; a_v += af[2] * ru;
    a_Ep += af[3] * u; a_u += af[3] * Ep;
    a_rv += ag[0];
    a_rv += ag[1] * u; a_u += ag[1] * rv;
    a_rv += ag[2] * v; a_v += ag[2] * rv; a_p += ag[2];
    a_Ep += ag[3] * v; a_v += ag[3] * Ep;
    if (VISC) {
        a_txx -= af[1]; a_txy -= af[2];
        a_u -= af[3] * txx; a_txx -= af[3] * u; a_v -= af[3] * txy; a_txy -= af[3] * v; a_Tx -= af[3] * c.kc_re;
        a_txy -= ag[1]; a_tyy -= ag[2];
        a_u -= ag[3] * txy; a_txy -= ag[3] * u; a_v -= ag[3] * tyy; a_tyy -= ag[3] * v; a_Ty -= ag[3] * c.kc_re;
    }
    a_rho += aqc[0]; a_ru += aqc[1]; a_rv += aqc[2]; a_E += aqc[3];
    a_E += a_Ep; a_p += a_Ep;
    a_p += a_E * c.inv_gm1; a_rho += a_E * 0.5 * k2;
    const double a_k2 = a_E * 0.5 * rho;
    a_u += 2.0 * u * a_k2; a_v += 2.0 * v * a_k2;
    a_rho += a_ru * u; a_u += a_ru * rho;
    a_rho += a_rv * v; a_v += a_rv * rho;
    a_p += a_rho * c.inv_Rg * iT; a_T -= a_rho * rho * iT;
    aq[0] = a_p; aq[1] = a_u; aq[2] = a_v; aq[3] = a_T;
    if (VISC) {
        // txx = mu_re (4/3 ux - 2/3 vy), tyy = mu_re (4/3 vy - 2/3 ux), txy = mu_re (uy + vx)
        aG[0] = c.mu_re * ((4.0 / 3.0) * a_txx - (2.0 / 3.0) * a_tyy);
        aG[3] = c.mu_re * ((4.0 / 3.0) * a_tyy - (2.0 / 3.0) * a_txx);
        aG[1] = c.mu_re * a_txy;
        aG[2] = c.mu_re * a_txy;
        aG[4] = a_Tx;
        aG[5] = a_Ty;
    }
}

// adjoint of the moving-face normal inviscid flux f n_x + g n_y - vgn q^c; accumulates into aq
__device__ void normal_flux_rev(const PhysConst& c, const double* q, double nx, double ny, double vgn,
                                const double* a, double* aq) {
    const double p = q[0], u = q[1], v = q[2], T = q[3];
    const double iT = 1.0 / T;
    const double rho = p * c.inv_Rg * iT;
    const double ru = rho * u, rv = rho * v;
    const double E = p * c.inv_gm1 + 0.5 * rho * (u * u + v * v);
    const double un = u * nx + v * ny, unr = un - vgn;
    double a_rho = a[0] * unr;
    double a_unr = a[0] * rho + a[1] * ru + a[2] * rv + a[3] * E;
    double a_ru = a[1] * unr, a_rv = a[2] * unr, a_E = a[3] * unr;
    double a_p = a[1] * nx + a[2] * ny + a[3] * un;
    double a_un = a[3] * p + a_unr;
    double a_u = a_un * nx, a_v = a_un * ny, a_T = 0.0;
    a_p += a_E * c.inv_gm1; a_rho += a_E * 0.5 * (u * u + v * v); a_u += a_E * rho * u; a_v += a_E * rho * v;
    a_rho += a_ru * u; a_u += a_ru * rho;
    a_rho += a_rv * v; a_v += a_rv * rho;
    a_p += a_rho * c.inv_Rg * iT; a_T -= a_rho * rho * iT;
    aq[0] += a_p; aq[1] += a_u; aq[2] += a_v; aq[3] += a_T;
}

// The adjoint of the BR2 common gradient's viscous flux with respect to either side's
// gradient trace, (u_x, u_y, v_x, v_y, T_x, T_y), from three face values: the adjoints of the
// normal stress components t_n = tau . n (a_tnx, a_tny) and of the heat-flux scale (a_T, with
// a_(T_x, T_y) = a_T n).  Each side's gradient trace enters the common gradient with weight 1/2.
__device__ __forceinline__ void grad_trace_adjoint(const PhysConst& c, double a_tnx, double a_tny, double a_T,
                                                   double nx, double ny, double* ag) {
    const double a_txx = a_tnx * nx, a_txy = a_tnx * ny + a_tny * nx, a_tyy = a_tny * ny;
    ag[0] = 0.5 * (c.mu_re * ((4.0 / 3.0) * a_txx - (2.0 / 3.0) * a_tyy));
    ag[1] = 0.5 * (c.mu_re * a_txy);
    ag[2] = 0.5 * (c.mu_re * a_txy);
    ag[3] = 0.5 * (c.mu_re * ((4.0 / 3.0) * a_tyy - (2.0 / 3.0) * a_txx));
    ag[4] = 0.5 * (a_T * nx);
    ag[5] = 0.5 * (a_T * ny);
}

// adjoint of the common flux (fr_common_flux): seeds afn[4] on fn and adqh[3] on dqh;
// outputs the adjoints of qm, qp (4 each) and gm, gp (6 each), and (ag3, when not null)
// the three face values that determine gm's and gp's adjoints (grad_trace_adjoint)
template <bool VISC>
__device__ void common_flux_rev(const PhysConst& c, const double* qm, const double* qp, const double* gm,
                                const double* gp, double nx, double ny, double cc,
                                double ug, double vg, const double* afn, const double* adqh, double* aqm,
                                double* aqp, double* agm, double* agp, double* ag3 = nullptr) {
    const double vgn = ug * nx + vg * ny;
    double qb[4], dq[4];
    for (int r = 0; r < 4; ++r) { qb[r] = 0.5 * (qm[r] + qp[r]); dq[r] = qp[r] - qm[r]; }
    // reciprocals taken once: T, c, U_r^2 (and |v - v_g|, c' below)
    const double iT = 1.0 / qb[3];
    const double rho = qb[0] * c.inv_Rg * iT;
    const double cs = sqrt(c.gRg * qb[3]);
    const double ics = 1.0 / cs;
    const double ur = qb[1] - ug, vr = qb[2] - vg;
    const double mg = sqrt(ur * ur + vr * vr);
    const double Ma = mg * ics;
    // eps = min(1, max(eps_min, Ma)) with the forward tie rules
    double eps;
    bool ma_branch = false;
    {
        const double t = (c.eps_min >= Ma) ? c.eps_min : Ma;
        const bool took_ma = !(c.eps_min >= Ma);
        eps = (1.0 <= t) ? 1.0 : t;
        ma_branch = took_ma && !(1.0 <= t);
    }
    const double Ur = eps * cs, Ur2 = Ur * Ur;
    const double iUr2 = 1.0 / Ur2;
    const double theta = iUr2 + c.inv_Cp * iT;
    const double rhoT = -rho * iT;
    const double h = c.Cp * qb[3] + 0.5 * (qb[1] * qb[1] + qb[2] * qb[2]);
    const double r0 = theta * dq[0] + rhoT * dq[3];
    double gd[4];
    gd[0] = r0;
    gd[1] = qb[1] * r0 + rho * dq[1];
    gd[2] = qb[2] * r0 + rho * dq[2];
    gd[3] = h * r0 - dq[0] + rho * (qb[1] * dq[1] + qb[2] * dq[2]) + (rho * c.Cp) * dq[3];
    const double un = ur * nx + vr * ny;
    const double alpha = 0.5 * (1.0 - eps * eps);
    const double unp = un * (1.0 - alpha);
    const double cp = sqrt(alpha * alpha * un * un + Ur2);
    const double lam = (unp >= 0.0 ? unp : -unp) + cp;

    double a_qb[4] = {0, 0, 0, 0}, a_dq[4] = {0, 0, 0, 0};
    for (int r = 0; r < 6; ++r) { agm[r] = 0.0; agp[r] = 0.0; }
    if (VISC) {
        const double ux = 0.5 * (gm[0] + gp[0]) + (cc * nx) * dq[1];
        const double uy = 0.5 * (gm[1] + gp[1]) + (cc * ny) * dq[1];
        const double vx = 0.5 * (gm[2] + gp[2]) + (cc * nx) * dq[2];
        const double vy = 0.5 * (gm[3] + gp[3]) + (cc * ny) * dq[2];
        const double div = ux + vy;
        const double txx = c.mu_re * (2.0 * ux - (2.0 / 3.0) * div);
        const double tyy = c.mu_re * (2.0 * vy - (2.0 / 3.0) * div);
        const double txy = c.mu_re * (uy + vx);
        const double tnx = txx * nx + txy * ny, tny = txy * nx + tyy * ny;
        const double a_tnx = -afn[1] - afn[3] * qb[1];
        const double a_tny = -afn[2] - afn[3] * qb[2];
        a_qb[1] -= afn[3] * tnx;
        a_qb[2] -= afn[3] * tny;
        const double a_Tx = -afn[3] * c.kc_re * nx, a_Ty = -afn[3] * c.kc_re * ny;
        const double a_txx = a_tnx * nx, a_txy = a_tnx * ny + a_tny * nx, a_tyy = a_tny * ny;
        const double a_ux = c.mu_re * ((4.0 / 3.0) * a_txx - (2.0 / 3.0) * a_tyy);
        const double a_vy = c.mu_re * ((4.0 / 3.0) * a_tyy - (2.0 / 3.0) * a_txx);
        const double a_uy = c.mu_re * a_txy, a_vx = c.mu_re * a_txy;
        const double ag6[6] = {a_ux, a_uy, a_vx, a_vy, a_Tx, a_Ty};
        for (int r = 0; r < 6; ++r) { agm[r] = 0.5 * ag6[r]; agp[r] = 0.5 * ag6[r]; }
        if (ag3) { ag3[0] = a_tnx; ag3[1] = a_tny; ag3[2] = -afn[3] * c.kc_re; }
        a_dq[1] += cc * (nx * a_ux + ny * a_uy);
        a_dq[2] += cc * (nx * a_vx + ny * a_vy);
        a_dq[3] += cc * (nx * a_Tx + ny * a_Ty);
        a_dq[1] += 0.5 * adqh[0];
        a_dq[2] += 0.5 * adqh[1];
        a_dq[3] += 0.5 * adqh[2];
    }
    // inviscid: fn = (fL + fR)/2 - lam gd / 2
    double a_fL[4], a_gd[4];
    double a_lam = 0.0;
    for (int r = 0; r < 4; ++r) {
        a_fL[r] = 0.5 * afn[r];
        a_gd[r] = -0.5 * lam * afn[r];
        a_lam -= 0.5 * afn[r] * gd[r];
    }
    const double a_unp = a_lam * (unp >= 0.0 ? 1.0 : -1.0);
    const double a_cp = a_lam;
    const double a_X = a_cp * (0.5 / cp);
    double a_alpha = a_X * 2.0 * alpha * un * un;
    double a_un = a_X * 2.0 * alpha * alpha * un;
    double a_Ur2 = a_X;
    a_un += a_unp * (1.0 - alpha);
    a_alpha -= a_unp * un;
    double a_eps = -a_alpha * eps;
    double a_ur = a_un * nx, a_vr = a_un * ny;
    // gd = Gamma~(qb) dq
    double a_r0 = a_gd[0];
    double a_rho = 0.0, a_h = 0.0;
    a_qb[1] += a_gd[1] * r0; a_r0 += a_gd[1] * qb[1]; a_rho += a_gd[1] * dq[1]; a_dq[1] += a_gd[1] * rho;
    a_qb[2] += a_gd[2] * r0; a_r0 += a_gd[2] * qb[2]; a_rho += a_gd[2] * dq[2]; a_dq[2] += a_gd[2] * rho;
    a_h += a_gd[3] * r0; a_r0 += a_gd[3] * h; a_dq[0] -= a_gd[3];
    a_rho += a_gd[3] * (qb[1] * dq[1] + qb[2] * dq[2] + c.Cp * dq[3]);
    a_qb[1] += a_gd[3] * rho * dq[1]; a_dq[1] += a_gd[3] * rho * qb[1];
    a_qb[2] += a_gd[3] * rho * dq[2]; a_dq[2] += a_gd[3] * rho * qb[2];
    a_dq[3] += a_gd[3] * rho * c.Cp;
    const double a_theta = a_r0 * dq[0];
    a_dq[0] += a_r0 * theta;
    const double a_rhoT = a_r0 * dq[3];
    a_dq[3] += a_r0 * rhoT;
    a_qb[3] += a_h * c.Cp; a_qb[1] += a_h * qb[1]; a_qb[2] += a_h * qb[2];
    a_rho -= a_rhoT * iT;
    a_qb[3] += a_rhoT * rho * iT * iT;   // d(-rho/T)/dT = rho/T^2
    a_Ur2 -= a_theta * iUr2 * iUr2;
    a_qb[3] -= a_theta * c.inv_Cp * iT * iT;
    const double a_Ur = 2.0 * Ur * a_Ur2;
    a_eps += a_Ur * cs;
    double a_cs = a_Ur * eps;
    if (ma_branch) {
        const double a_Ma = a_eps;
        const double a_mg = a_Ma * ics;
        a_cs -= a_Ma * Ma * ics;
        const double img = 1.0 / mg;   // Ma > eps_min >= 0 on this branch, so mg > 0
        a_ur += a_mg * ur * img;
        a_vr += a_mg * vr * img;
    }
    a_qb[1] += a_ur;
    a_qb[2] += a_vr;
    a_qb[3] += a_cs * c.gRg * (0.5 * ics);
    a_qb[0] += a_rho * c.inv_Rg * iT;
    a_qb[3] -= a_rho * rho * iT;
    for (int r = 0; r < 4; ++r) {
        aqm[r] = 0.5 * a_qb[r] - a_dq[r];
        aqp[r] = 0.5 * a_qb[r] + a_dq[r];
    }
    normal_flux_rev(c, qm, nx, ny, vgn, a_fL, aqm);
    normal_flux_rev(c, qp, nx, ny, vgn, a_fL, aqp);   // a_fR == a_fL
}

// ---------------------------------------------------------------- kernel 2: element reverse sweep
template <int P, bool VISC, bool MOV, bool BC, bool AFF = false>
__global__ void __launch_bounds__((Sz<P>::threads))
k_vjp_elem(int E, const double* __restrict__ q, const double* __restrict__ w, const double* __restrict__ tr,
           double* __restrict__ out, double* __restrict__ aside, OpTab op_in, PhysConst pc, Geo g) {
    static_assert(!AFF || (!MOV && !BC), "neighbour traces from states: static meshes without boundary faces");
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT, EPB = Sz<P>::EPB;
    constexpr int NTV = VISC ? 10 : 4;
    constexpr int NG = MOV ? NGSP : G_IJ + 1;   // static meshes have no grid velocity
    __shared__ double s_q[EPB][4][Np];
    // scratch fields at solution points: the adjoint seed times each metric term (20; moving
    // meshes add the 4 grid-velocity products); affine elements store the seed alone (4 fields,
    // the metric terms being element constants), so 6 fields cover the other phases
    constexpr int NA = AFF ? 6 : (MOV ? 24 : 20);
    __shared__ double s_a[EPB][NA][Np];
    __shared__ double s_f[EPB][NF][10];      // per flux point scratch
    __shared__ double s_S[EPB][NF][4];       // Sx, Sy, S.vg, scale sg|S|
    __shared__ OpTab sop;                    // operator tables (lane-dependent indexing in LDS)
    for (int t = threadIdx.x; t < (int)(sizeof(OpTab) / sizeof(double)); t += blockDim.x)
        reinterpret_cast<double*>(&sop)[t] = reinterpret_cast<const double*>(&op_in)[t];
    const OpTab& op = sop;
    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    const int e = xcd_tile(gridDim.x / 8) * EPB + el;
    const bool act = e < E;
    const bool isS = act && lt < Np, isF = act && lt < NF;
    const size_t EN = (size_t)E * Np, FE = (size_t)E * NF;
    const int i = lt % n, j = lt / n;
    double qs[4] = {0, 0, 0, 0}, G[6] = {0, 0, 0, 0, 0, 0}, geo[NGSP];
    #pragma unroll
    for (int c = 0; c < NGSP; ++c) geo[c] = 0.0;
    // ---- forward: load, uncorrected gradient
    if (isS) {
        const size_t id = (size_t)e * Np + lt;
        #pragma unroll
        for (int v = 0; v < 4; ++v) { qs[v] = q[v * EN + id]; s_q[el][v][lt] = qs[v]; }
    }
    if (AFF ? act : isS) {
        // affine: every lane, face lanes past Np included, holds the element's constant metrics
        const size_t id = (size_t)e * Np + lt % Np;
        #pragma unroll
        for (int c = 0; c < NG; ++c) geo[c] = g.sp[c * EN + id];
    }
    __syncthreads();
    if (VISC && isS) {
        #pragma unroll
        for (int c = 0; c < 3; ++c) {
            double dxi = 0, deta = 0;
            for (int b = 0; b < n; ++b) {
                dxi += op.D[i * n + b] * s_q[el][c + 1][b + n * j];
                deta += op.D[j * n + b] * s_q[el][c + 1][i + n * b];
            }
            G[2 * c] = geo[G_XIX] * dxi + geo[G_ETX] * deta;
            G[2 * c + 1] = geo[G_XIY] * dxi + geo[G_ETY] * deta;
            s_a[el][2 * c][lt] = G[2 * c];
            s_a[el][2 * c + 1][lt] = G[2 * c + 1];
        }
    }
    __syncthreads();
    // ---- forward: traces and the common solution (dqh) at flux points
    double qm[4], qp[4], gm[6], gp[6];
    double nx = 0, ny = 0, cc = 0, ugf = 0, vgf = 0, sc = 0;
    int f = 0, k = 0, bck = 0;
    if (isF) {
        f = lt / n; k = lt % n;
        const double* lam = (f == 0 || f == 2) ? op.lamL : op.lamR;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double sacc = 0;
            for (int a = 0; a < n; ++a) sacc += lam[a] * s_q[el][v][line_pt(n, f, k, a)];
            qm[v] = sacc;
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            double sacc = 0;
            if (VISC)
                for (int a = 0; a < n; ++a) sacc += lam[a] * s_a[el][c][line_pt(n, f, k, a)];
            gm[c] = sacc;
        }
        const int pk = g.nbr[e * 4 + f];
        const int nb = pk >> 3, nf = (pk >> 1) & 3, k2 = (pk & 1) ? n - 1 - k : k;
        if (AFF) {
            // the neighbour's line through this face point: its trace and face-normal
            // derivative; the neighbour traces of (u, v, T) go to slots 4..6 of their
            // own face point for the tangential derivative below
            const double* lamn = (nf == 0 || nf == 2) ? op.lamL : op.lamR;
            const double* dlamn = (nf == 0 || nf == 2) ? op.dlamL : op.dlamR;
            const size_t nbase = (size_t)nb * Np;
#pragma unroll
            for (int c = 0; c < 6; ++c) gp[c] = 0.0;
            double ln[4][n];
#pragma unroll
            for (int b = 0; b < n; ++b) {
                const int sp = line_pt(n, nf, k2, b);
#pragma unroll
                for (int v = 0; v < 4; ++v) ln[v][b] = q[v * EN + nbase + sp];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double sacc = 0;
                for (int b = 0; b < n; ++b) sacc += lamn[b] * ln[v][b];
                qp[v] = sacc;
            }
            if (VISC) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double sacc = 0;
                    for (int b = 0; b < n; ++b) sacc += dlamn[b] * ln[c + 1][b];
                    gp[2 * c] = sacc;   // face-normal derivative for now
                    s_f[el][f * n + k2][4 + c] = qp[c + 1];
                }
            }
        } else {
            const double* src = tr + ((size_t)(nb * 4 + nf) * NTV) * n;
#pragma unroll
            for (int v = 0; v < 4; ++v) qp[v] = src[(size_t)v * n + k2];
#pragma unroll
            for (int c = 0; c < 6; ++c) gp[c] = VISC ? src[(size_t)(4 + c) * n + k2] : 0.0;
        }
        const size_t sid = (size_t)e * NF + lt;
        nx = g.fp[F_NX * FE + sid]; ny = g.fp[F_NY * FE + sid];
        sc = g.fp[F_SC * FE + sid]; cc = g.fp[F_CC * FE + sid];
        ugf = MOV ? g.fp[F_UG * FE + sid] : 0.0;
        vgf = MOV ? g.fp[F_VG * FE + sid] : 0.0;
        // a boundary face: the state beyond it comes from the own trace
        bck = BC ? (g.bc[e] >> (2 * f)) & 3 : 0;
        if (BC && bck) {
            fr_bc_state<double>(bck, g.qinf, qm, nx, ny, ugf, vgf, qp);
            if (VISC) fr_bc_grad<double>(bck, gm, nx, ny, gp);
        }
        s_S[el][lt][0] = sc * nx; s_S[el][lt][1] = sc * ny;
        s_S[el][lt][2] = MOV ? sc * (ugf * nx + vgf * ny) : 0.0;
        s_S[el][lt][3] = sc;
        if (VISC) for (int c = 0; c < 3; ++c) s_f[el][lt][c] = 0.5 * (qp[c + 1] - qm[c + 1]);   // dqh
    }
    if (AFF && VISC) {
        // neighbour gradient trace: the tangential derivative is the 1-D derivative of the
        // neighbour traces along the face; the chain rule takes the neighbour's constant metrics
        __syncthreads();
        if (isF) {
            const int pk = g.nbr[e * 4 + f];
            const int nb = pk >> 3, nf = (pk >> 1) & 3, k2 = (pk & 1) ? n - 1 - k : k;
            const size_t gid = (size_t)nb * Np;
            const double mxix = g.sp[G_XIX * EN + gid], mxiy = g.sp[G_XIY * EN + gid];
            const double metx = g.sp[G_ETX * EN + gid], mety = g.sp[G_ETY * EN + gid];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double dtan = 0;
                for (int m = 0; m < n; ++m) dtan += op.D[k2 * n + m] * s_f[el][f * n + m][4 + c];
                const double dnor = gp[2 * c];
                const double dxi = nf < 2 ? dnor : dtan, deta = nf < 2 ? dtan : dnor;
                gp[2 * c] = mxix * dxi + metx * deta;
                gp[2 * c + 1] = mxiy * dxi + mety * deta;
            }
        }
    }
    __syncthreads();
    // ---- forward: corrected gradient; reverse: volume seeds
    double rho_w[4] = {0, 0, 0, 0};
    const int fp0 = 0 * n + j, fp1 = 1 * n + j, fp2 = 2 * n + i, fp3 = 3 * n + i;
    if (isS) {
        const double gLi = op.gamL[i], gRi = op.gamR[i], gLj = op.gamL[j], gRj = op.gamR[j];
        if (VISC) {
            #pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double cx = s_S[el][fp0][0] * gLi * s_f[el][fp0][c] + s_S[el][fp1][0] * gRi * s_f[el][fp1][c]
                                + s_S[el][fp2][0] * gLj * s_f[el][fp2][c] + s_S[el][fp3][0] * gRj * s_f[el][fp3][c];
                const double cy = s_S[el][fp0][1] * gLi * s_f[el][fp0][c] + s_S[el][fp1][1] * gRi * s_f[el][fp1][c]
                                + s_S[el][fp2][1] * gLj * s_f[el][fp2][c] + s_S[el][fp3][1] * gRj * s_f[el][fp3][c];
                G[2 * c] += geo[G_IJ] * cx;
                G[2 * c + 1] += geo[G_IJ] * cy;
            }
        }
        const size_t id = (size_t)e * Np + lt;
        #pragma unroll
        for (int v = 0; v < 4; ++v) rho_w[v] = -w[v * EN + id];
    }
    __syncthreads();   // gradient fields in s_a are dead from here
    // store per point: rho*xix, rho*etx, rho*xiy, rho*ety (+ rho*axi, rho*aet), rho*ij
    if constexpr (AFF) {
        if (isS) {
            #pragma unroll
            for (int v = 0; v < 4; ++v) s_a[el][v][lt] = rho_w[v];
        }
    } else if (isS) {
        const double axi = MOV ? geo[G_UG] * geo[G_XIX] + geo[G_VG] * geo[G_XIY] : 0.0;
        const double aet = MOV ? geo[G_UG] * geo[G_ETX] + geo[G_VG] * geo[G_ETY] : 0.0;
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
            s_a[el][0 + v][lt] = rho_w[v] * geo[G_XIX];
            s_a[el][4 + v][lt] = rho_w[v] * geo[G_ETX];
            s_a[el][8 + v][lt] = rho_w[v] * geo[G_XIY];
            s_a[el][12 + v][lt] = rho_w[v] * geo[G_ETY];
            s_a[el][16 + v][lt] = rho_w[v] * geo[G_IJ];
            if constexpr (MOV) {
                s_a[el][20 + v][lt] = rho_w[v] * axi;   // combined below with aet via a second pass
            }
        }
    }
    __syncthreads();
    // flux points: adjoint of F^num - F^loc from the lift
    double aDF[4] = {0, 0, 0, 0};
    if (isF) {
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
            double sacc = 0;
            for (int b = 0; b < n; ++b) {
                const int s = line_pt(n, f, k, b);
                const double gm_ = (f == 0 || f == 2) ? op.gamL[b] : op.gamR[b];
                sacc += gm_ * s_a[el][AFF ? v : 16 + v][s];
            }
            aDF[v] = AFF ? geo[G_IJ] * sacc : sacc;
        }
    }
    // solution points: adjoints of f, g (and q^c) from the divergence terms
    double af[4] = {0, 0, 0, 0}, ag[4] = {0, 0, 0, 0}, aqc[4] = {0, 0, 0, 0};
    if (isS) {
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
            double s1 = 0, s2 = 0, s3 = 0;
            if constexpr (AFF) {
                // the transposed reference derivatives of the seed, then the constant metrics
                for (int b = 0; b < n; ++b) {
                    s1 += op.D[b * n + i] * s_a[el][v][b + n * j];
                    s2 += op.D[b * n + j] * s_a[el][v][i + n * b];
                }
                af[v] = geo[G_XIX] * s1 + geo[G_ETX] * s2;
                ag[v] = geo[G_XIY] * s1 + geo[G_ETY] * s2;
            } else {
                for (int b = 0; b < n; ++b) {
                    const double Dxi = op.D[b * n + i], Det = op.D[b * n + j];   // D^T
                    s1 += Dxi * s_a[el][0 + v][b + n * j] + Det * s_a[el][4 + v][i + n * b];
                    s2 += Dxi * s_a[el][8 + v][b + n * j] + Det * s_a[el][12 + v][i + n * b];
                    if constexpr (MOV) s3 += Dxi * s_a[el][20 + v][b + n * j];
                }
                af[v] = s1; ag[v] = s2; aqc[v] = -s3;
            }
        }
    }
    __syncthreads();
    if constexpr (MOV) {
        if (isS) {
            const double aet = geo[G_UG] * geo[G_ETX] + geo[G_VG] * geo[G_ETY];
            #pragma unroll
            for (int v = 0; v < 4; ++v) s_a[el][20 + v][lt] = rho_w[v] * aet;
        }
    }
    if (isF) {
        // store -aDF (adjoint of F^loc) for the solution-point gather
        #pragma unroll
        for (int v = 0; v < 4; ++v) s_f[el][lt][3 + v] = -aDF[v];   // slots 3..6
    }
    __syncthreads();
    if (isS) {
        if constexpr (MOV) {
            #pragma unroll
            for (int v = 0; v < 4; ++v) {
                double s3 = 0;
                for (int b = 0; b < n; ++b) s3 += op.D[b * n + j] * s_a[el][20 + v][i + n * b];
                aqc[v] -= s3;
            }
        }
        // F^loc(fp) = sum_b lam_b [Sx f + Sy g - Svg q^c](line b): gather over the 4 lines through s
        const int fps[4] = {fp0, fp1, fp2, fp3};
        const double lams[4] = {op.lamL[i], op.lamR[i], op.lamL[j], op.lamR[j]};
        #pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int fp = fps[t];
            const double l = lams[t];
            #pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double aF = s_f[el][fp][3 + v];
                af[v] += l * s_S[el][fp][0] * aF;
                ag[v] += l * s_S[el][fp][1] * aF;
                if (MOV) aqc[v] -= l * s_S[el][fp][2] * aF;
            }
        }
    }
    __syncthreads();
    // point-flux adjoint -> aq(s), aGc(s); store ij*aGc for the dqh adjoint
    double aq[4] = {0, 0, 0, 0}, aG[6] = {0, 0, 0, 0, 0, 0};
    if (isS) {
        point_flux_rev<VISC>(pc, qs, G, af, ag, aqc, aq, aG);
        if (VISC)
            #pragma unroll
            for (int c = 0; c < 6; ++c) s_a[el][c][lt] = geo[G_IJ] * aG[c];
    }
    __syncthreads();
    // flux points: adjoint of dqh, then the common-flux adjoint
    if (isF) {
        double adqh[3] = {0, 0, 0};
        if (VISC) {
            const double Sx = s_S[el][lt][0], Sy = s_S[el][lt][1];
            for (int b = 0; b < n; ++b) {
                const int s = line_pt(n, f, k, b);
                const double gm_ = (f == 0 || f == 2) ? op.gamL[b] : op.gamR[b];
                #pragma unroll
                for (int c = 0; c < 3; ++c)
                    adqh[c] += gm_ * (Sx * s_a[el][2 * c][s] + Sy * s_a[el][2 * c + 1][s]);
            }
        }
        double afn[4];
        #pragma unroll
        for (int v = 0; v < 4; ++v) afn[v] = sc * aDF[v];
        double aqm[4], aqp[4], agm[6], agp[6], ag3[3] = {0.0, 0.0, 0.0};
        common_flux_rev<VISC>(pc, qm, qp, gm, gp, nx, ny, cc, ugf, vgf, afn, adqh, aqm, aqp, agm, agp,
                              AFF ? ag3 : nullptr);
        if (BC && bck) {
            // q^+ and g^+ depend on the own traces through symmetric linear maps: their
            // adjoints go back to the own side, and nothing to a neighbour
            double t[6];
            fr_bc_state_lin<double>(bck, aqp, nx, ny, t);
            #pragma unroll
            for (int v = 0; v < 4; ++v) { aqm[v] += t[v]; aqp[v] = 0.0; }
            if (VISC) {
                fr_bc_grad<double>(bck, agp, nx, ny, t);
                #pragma unroll
                for (int c = 0; c < 6; ++c) { agm[c] += t[c]; agp[c] = 0.0; }
            }
        }
        if (AFF) {
            // the neighbour's gradient-trace adjoint travels as the three face values it is made
            // of; the neighbour rebuilds it with its own face normal (minus this side's)
            constexpr int NTA = VISC ? 7 : 4;
            double* dst = aside + ((size_t)(e * 4 + f) * NTA) * n;
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[(size_t)v * n + k] = aqp[v];
            if (VISC) for (int c = 0; c < 3; ++c) dst[(size_t)(4 + c) * n + k] = ag3[c];
        } else {
            double* dst = aside + ((size_t)(e * 4 + f) * NTV) * n;
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[(size_t)v * n + k] = aqp[v];
            if (VISC) for (int c = 0; c < 6; ++c) dst[(size_t)(4 + c) * n + k] = agp[c];
        }
        #pragma unroll
        for (int v = 0; v < 4; ++v) s_f[el][lt][v] = aqm[v];
        if (VISC) for (int c = 0; c < 6; ++c) s_f[el][lt][4 + c] = agm[c];
    }
    __syncthreads();
    // solution points: trace transposes, then the gradient transpose
    if (isS) {
        const int fps[4] = {fp0, fp1, fp2, fp3};
        const double lams[4] = {op.lamL[i], op.lamR[i], op.lamL[j], op.lamR[j]};
        #pragma unroll
        for (int t = 0; t < 4; ++t) {
            #pragma unroll
            for (int v = 0; v < 4; ++v) aq[v] += lams[t] * s_f[el][fps[t]][v];
            if (VISC) for (int c = 0; c < 6; ++c) aG[c] += lams[t] * s_f[el][fps[t]][4 + c];
        }
        if (VISC) {
            #pragma unroll
            for (int c = 0; c < 3; ++c) {
                s_a[el][c][lt] = geo[G_XIX] * aG[2 * c] + geo[G_XIY] * aG[2 * c + 1];       // a d_xi
                s_a[el][3 + c][lt] = geo[G_ETX] * aG[2 * c] + geo[G_ETY] * aG[2 * c + 1];   // a d_eta
            }
        }
    }
    __syncthreads();
    if (isS) {
        if (VISC) {
            #pragma unroll
            for (int c = 0; c < 3; ++c) {
                double sacc = 0;
                for (int b = 0; b < n; ++b)
                    sacc += op.D[b * n + i] * s_a[el][c][b + n * j] + op.D[b * n + j] * s_a[el][3 + c][i + n * b];
                aq[c + 1] += sacc;
            }
        }
        const size_t id = (size_t)e * Np + lt;
        #pragma unroll
        for (int v = 0; v < 4; ++v) out[v * EN + id] = aq[v];
    }
}

// ---------------------------------------------------------------- kernel 3: gather from neighbours
// AFF: static affine meshes without boundary faces; the side buffer holds the compressed face
// values (aqp, then a_tnx, a_tny, a_T), and the element's constant metrics are read once.
template <int P, bool VISC, bool AFF = false>
__global__ void __launch_bounds__((Sz<P>::threads))
k_vjp_gather(int E, const double* __restrict__ aside, double* __restrict__ out, OpTab op_in, PhysConst pc,
             Geo g) {
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT, EPB = Sz<P>::EPB;
    constexpr int NTV = VISC ? (AFF ? 7 : 10) : 4;
    __shared__ double s_f[EPB][NF][10];
    __shared__ double s_d[EPB][6][Np];
    __shared__ OpTab sop;
    for (int t = threadIdx.x; t < (int)(sizeof(OpTab) / sizeof(double)); t += blockDim.x)
        reinterpret_cast<double*>(&sop)[t] = reinterpret_cast<const double*>(&op_in)[t];
    const OpTab& op = sop;
    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    const int e = xcd_tile(gridDim.x / 8) * EPB + el;
    const bool act = e < E;
    const bool isS = act && lt < Np, isF = act && lt < NF;
    const size_t EN = (size_t)E * Np;
    const int i = lt % n, j = lt / n;
    if (isF) {
        const int f = lt / n, k = lt % n;
        const int pk = g.nbr[e * 4 + f];
        const int nb = pk >> 3, nf = (pk >> 1) & 3, k2 = (pk & 1) ? n - 1 - k : k;
        const double* src = aside + ((size_t)(nb * 4 + nf) * NTV) * n;
        if (AFF && VISC) {
#pragma unroll
            for (int v = 0; v < 4; ++v) s_f[el][lt][v] = src[(size_t)v * n + k2];
            const size_t sid = (size_t)e * NF + lt, FE = (size_t)E * NF;
            const double nx = -g.fp[F_NX * FE + sid], ny = -g.fp[F_NY * FE + sid];   // the neighbour's normal
            double ag[6];
            grad_trace_adjoint(pc, src[(size_t)4 * n + k2], src[(size_t)5 * n + k2], src[(size_t)6 * n + k2], nx, ny,
                               ag);
#pragma unroll
            for (int c = 0; c < 6; ++c) s_f[el][lt][4 + c] = ag[c];
        } else {
            for (int v = 0; v < NTV; ++v) s_f[el][lt][v] = src[(size_t)v * n + k2];
        }
    }
    __syncthreads();
    double aq[4] = {0, 0, 0, 0}, aG[6] = {0, 0, 0, 0, 0, 0};
    double geo[4] = {0, 0, 0, 0};
    if (isS) {
        const int fps[4] = {0 * n + j, 1 * n + j, 2 * n + i, 3 * n + i};
        const double lams[4] = {op.lamL[i], op.lamR[i], op.lamL[j], op.lamR[j]};
        for (int t = 0; t < 4; ++t) {
            for (int v = 0; v < 4; ++v) aq[v] += lams[t] * s_f[el][fps[t]][v];
            if (VISC) for (int c = 0; c < 6; ++c) aG[c] += lams[t] * s_f[el][fps[t]][4 + c];
        }
        if (VISC) {
            const size_t id = (size_t)e * Np + (AFF ? 0 : lt);   // affine: the element's constant metrics
            geo[0] = g.sp[G_XIX * EN + id]; geo[1] = g.sp[G_XIY * EN + id];
            geo[2] = g.sp[G_ETX * EN + id]; geo[3] = g.sp[G_ETY * EN + id];
            for (int c = 0; c < 3; ++c) {
                s_d[el][c][lt] = geo[0] * aG[2 * c] + geo[1] * aG[2 * c + 1];
                s_d[el][3 + c][lt] = geo[2] * aG[2 * c] + geo[3] * aG[2 * c + 1];
            }
        }
    }
    __syncthreads();
    if (isS) {
        if (VISC) {
            for (int c = 0; c < 3; ++c) {
                double sacc = 0;
                for (int b = 0; b < n; ++b)
                    sacc += op.D[b * n + i] * s_d[el][c][b + n * j] + op.D[b * n + j] * s_d[el][3 + c][i + n * b];
                aq[c + 1] += sacc;
            }
        }
        const size_t id = (size_t)e * Np + lt;
        for (int v = 0; v < 4; ++v) out[v * EN + id] += aq[v];
    }
}

template <int P, bool VISC, bool MOV>
fr_status run_vjp(fr_ctx c, const double* q, const double* w, double* out, const double* trace, double* aside,
                  hipStream_t s) {
    const Geo g = c->geo();
    // tiles of EPB elements, the grid rounded up to a multiple of 8 for the XCD-contiguous order
    const int grid = 8 * (((c->E + Sz<P>::EPB - 1) / Sz<P>::EPB + 7) / 8);
    if (!trace) {
        if constexpr (!MOV)
            hipLaunchKernelGGL((k_vjp_elem<P, VISC, false, false, true>), dim3(grid), dim3(Sz<P>::threads), 0, s,
                               c->E, q, w, nullptr, out, aside, c->op, c->pc, g);
    } else if (g.bc)
        hipLaunchKernelGGL((k_vjp_elem<P, VISC, MOV, true>), dim3(grid), dim3(Sz<P>::threads), 0, s, c->E, q, w,
                           trace, out, aside, c->op, c->pc, g);
    else
        hipLaunchKernelGGL((k_vjp_elem<P, VISC, MOV, false>), dim3(grid), dim3(Sz<P>::threads), 0, s, c->E, q, w,
                           trace, out, aside, c->op, c->pc, g);
    FR_HIP(hipGetLastError());
    if (!trace)
        hipLaunchKernelGGL((k_vjp_gather<P, VISC, true>), dim3(grid), dim3(Sz<P>::threads), 0, s, c->E, aside, out,
                           c->op, c->pc, g);
    else
        hipLaunchKernelGGL((k_vjp_gather<P, VISC>), dim3(grid), dim3(Sz<P>::threads), 0, s, c->E, aside, out, c->op,
                           c->pc, g);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

template <int P>
fr_status vjp_p(fr_ctx c, const double* q, const double* w, double* out, const double* tr, double* as,
                hipStream_t s) {
    const bool visc = c->prm.viscous != 0, mov = c->prm.moving != 0;
    if (visc) return mov ? run_vjp<P, true, true>(c, q, w, out, tr, as, s) : run_vjp<P, true, false>(c, q, w, out, tr, as, s);
    return mov ? run_vjp<P, false, true>(c, q, w, out, tr, as, s) : run_vjp<P, false, false>(c, q, w, out, tr, as, s);
}

// Traces, element adjoints and the neighbour gather with the given side buffers: trace
// and aside each hold E * 4 * 10 * (p+1) doubles.  Static meshes of affine elements without
// boundary faces need no trace buffer.
fr_status vjp_with(fr_ctx c, const double* q, const double* w, double* out, double* trace, double* aside,
                   hipStream_t s) {
    if (c->prm.moving == 0 && !c->d_bc && c->all_affine)
        trace = nullptr;
    else
        FR_TRY(launch_traces(c, q, trace, s));
    switch (c->p) {
        case 1: return vjp_p<1>(c, q, w, out, trace, aside, s);
        case 2: return vjp_p<2>(c, q, w, out, trace, aside, s);
        case 3: return vjp_p<3>(c, q, w, out, trace, aside, s);
        case 4: return vjp_p<4>(c, q, w, out, trace, aside, s);
    }
    fr_set_error("order outside 1..4");
    return FR_EUNSUPPORTED;
}

}  // namespace

fr_status launch_vjp(fr_ctx c, const double* q, const double* w, double* out, hipStream_t s) {
    return vjp_with(c, q, w, out, c->d_trace, c->d_vj, s);
}

// ----------------------------------------------------------------------------- allocation-free VJP
// The same three kernels with their two side buffers (face traces, face adjoints) in a
// file-scope device array instead of context memory, for callers that cannot allocate.
// Each device holds its own copy of the array until the process ends.  Host code never
// uses the array's name as an address: its device address is looked up once per device
// and kept in scratch_dev.  Calls that overlap on one device share the array and race.
static constexpr size_t VJP_SCRATCH_BYTES = size_t(32) << 20;
static __device__ __align__(256) double scratch[VJP_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mtx;
double* scratch_dev[MAX_DEVICES] = {};

fr_status scratch_address(int dev, double** out) {
    std::lock_guard<std::mutex> lock(scratch_mtx);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fr_set_error(std::string("fr_vjp_noalloc: hipGetSymbolAddress of the scratch array: ") +
                         hipGetErrorString(e));
            return FR_EHIP;
        }
        scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = scratch_dev[dev];
    return FR_OK;
}

}  // namespace

extern "C" fr_status fr_vjp_noalloc(fr_ctx c, const double* q, const double* w, double* JTw, void* stream) {
    if (!c) { fr_set_error("fr_vjp_noalloc: null context"); return FR_EINVAL; }
    if (const char* m = ctx_not_ready(c)) { fr_set_error(m); return FR_EINVAL; }
    if (!q || !w || !JTw) { fr_set_error("fr_vjp_noalloc: null argument"); return FR_EINVAL; }
    const size_t side = (size_t)c->E * 4 * 10 * c->n;   // doubles per side buffer
    if (2 * side * sizeof(double) > VJP_SCRATCH_BYTES) {
        fr_set_error("fr_vjp_noalloc: the mesh needs " + std::to_string(2 * side * sizeof(double)) +
                     " bytes of scratch, above the maximum of " + std::to_string(VJP_SCRATCH_BYTES) +
                     " (E * 4 * 10 * (p+1) * 16 bytes); use fr_vjp");
        return FR_EINVAL;
    }
    int dev = -1;
    FR_HIP(hipGetDevice(&dev));
    if (dev != c->device || dev < 0 || dev >= MAX_DEVICES) {
        fr_set_error("fr_vjp_noalloc: the current device is not the context's");
        return FR_EINVAL;
    }
    double* base = nullptr;
    FR_TRY(scratch_address(dev, &base));
    return vjp_with(c, q, w, JTw, base, base + side, (hipStream_t)stream);
}
