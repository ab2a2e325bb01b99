// Geometry kernels (metrics, face vectors, grid velocity), the trace kernel of the
// adjoint path, and the dispatch of the fused residual kernels (fr_fused.hpp) over the
// launch groups of a solver.
#include "fr_internal.hpp"

namespace {

template <int P>
struct Sz {
    static constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = (Np > NF ? Np : NF);
};

// elements per workgroup: 256 lanes for plain doubles, fewer for dual numbers (LDS)
template <int P, int W>
struct Blk {
    static constexpr int NT = Sz<P>::NT;
    static constexpr int lanes = (W == 1) ? 256 : (W == 2 ? 128 : 64);
    static constexpr int EPB = (lanes / NT) > 0 ? (lanes / NT) : 1;
    static constexpr int threads = EPB * NT;
};

__device__ __forceinline__ int line_pt(int n, int f, int k, int a) {
    return f < 2 ? a + n * k : k + n * a;
}

// ------------------------------------------------------------------ geometry
// Isoparametric map on Gauss-Lobatto nodes; derivatives along xi (Bx) and eta (By).
__device__ void map_derivs(const GeoTab& gt, const double* X, const double* Y, const double* U, const double* V,
                           const double* Bx, const double* dBx, const double* By, const double* dBy,
                           double& xr, double& xs, double& yr, double& ys, double& u, double& v) {
    const int m = gt.m;
    xr = xs = yr = ys = u = v = 0.0;
    for (int b = 0; b < m; ++b)
        for (int a = 0; a < m; ++a) {
            double Xv = X[a + m * b], Yv = Y[a + m * b];
            xr += Xv * dBx[a] * By[b];
            xs += Xv * Bx[a] * dBy[b];
            yr += Yv * dBx[a] * By[b];
            ys += Yv * Bx[a] * dBy[b];
            if (U) { u += U[a + m * b] * Bx[a] * By[b]; v += V[a + m * b] * Bx[a] * By[b]; }
        }
}

__global__ void k_geo_sp(int E, int n, GeoTab gt, const double* __restrict__ xg, const double* __restrict__ vg,
                         double* __restrict__ gsp) {
    const int Np = n * n;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)E * Np) return;
    const int e = (int)(t / Np), s = (int)(t % Np), i = s % n, j = s / n;
    const int m = gt.m;
    const size_t ng = (size_t)m * m;
    const double* X = xg + e * ng;
    const double* Y = xg + (size_t)E * ng + e * ng;
    const double* U = vg ? vg + e * ng : nullptr;
    const double* V = vg ? vg + (size_t)E * ng + e * ng : nullptr;
    double xr, xs, yr, ys, u, v;
    map_derivs(gt, X, Y, U, V, gt.Ls + i * m, gt.dLs + i * m, gt.Ls + j * m, gt.dLs + j * m, xr, xs, yr, ys, u, v);
    const double J = xr * ys - xs * yr;
    const double ij = 1.0 / J;
    const size_t EN = (size_t)E * Np;
    gsp[G_XIX * EN + t] = ys * ij;
    gsp[G_XIY * EN + t] = -xs * ij;
    gsp[G_ETX * EN + t] = -yr * ij;
    gsp[G_ETY * EN + t] = xr * ij;
    gsp[G_IJ * EN + t] = ij;
    gsp[G_UG * EN + t] = u;
    gsp[G_VG * EN + t] = v;
}

// element-oriented face vector (|J| grad xi on faces 0/1, |J| grad eta on 2/3), |J|, v_g
__device__ void face_eval(int E, int n, const GeoTab& gt, const double* xg, const double* vg, int e, int f, int k,
                          double& Sx, double& Sy, double& J, double& u, double& v) {
    const int m = gt.m;
    const size_t ng = (size_t)m * m;
    double d0[FR_MAXN], dm[FR_MAXN];
    for (int a = 0; a < m; ++a) { d0[a] = (a == 0) ? 1.0 : 0.0; dm[a] = (a == m - 1) ? 1.0 : 0.0; }
    const double *Bx, *dBx, *By, *dBy;
    if (f < 2) {
        Bx = (f == 0) ? d0 : dm; dBx = (f == 0) ? gt.dLm : gt.dLp;
        By = gt.Ls + k * m; dBy = gt.dLs + k * m;
    } else {
        Bx = gt.Ls + k * m; dBx = gt.dLs + k * m;
        By = (f == 2) ? d0 : dm; dBy = (f == 2) ? gt.dLm : gt.dLp;
    }
    const double* X = xg + e * ng;
    const double* Y = xg + (size_t)E * ng + e * ng;
    const double* U = vg ? vg + e * ng : nullptr;
    const double* V = vg ? vg + (size_t)E * ng + e * ng : nullptr;
    double xr, xs, yr, ys;
    map_derivs(gt, X, Y, U, V, Bx, dBx, By, dBy, xr, xs, yr, ys, u, v);
    if (f < 2) { Sx = ys; Sy = -xs; } else { Sx = -yr; Sy = xr; }
    J = xr * ys - xs * yr;
}

// 1 when every solution-point metric term of the element equals its first point's to 1e-10
// of the metric's scale (an affine element): its gradient traces then follow from its
// face traces.  The rounding of metrics computed from node coordinates grows with
// |x| / h (about 1e-12 on a 256 x 256 mesh of [0, 2 pi]^2); a map curved by less than
// 1e-10 of the element size is affine for every purpose of the discretisation.  An
// element with a boundary face is not flagged: the kernels of affine elements assume
// that every face has a neighbour element.
__global__ void k_affine(int E, int Np, const double* __restrict__ gsp, const int32_t* __restrict__ bc,
                         int32_t* __restrict__ aff) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    if (bc && bc[e] != 0) { aff[e] = 0; return; }
    const size_t EN = (size_t)E * Np;
    const double* m = gsp + (size_t)e * Np;
    double scale = 0.0;
    for (int c = G_XIX; c <= G_ETY; ++c) scale = fmax(scale, fabs(m[c * EN]));
    bool ok = true;
    for (int c = G_XIX; c <= G_IJ; ++c) {
        const double* mc = m + c * EN;
        const double tol = 1e-10 * (c == G_IJ ? fabs(mc[0]) : scale);
        for (int s = 1; s < Np; ++s) ok = ok && fabs(mc[s] - mc[0]) <= tol;
    }
    aff[e] = ok ? 1 : 0;
}

__global__ void k_geo_fp(int E, int n, GeoTab gt, double br2, const int32_t* __restrict__ nbr,
                         const double* __restrict__ xg, const double* __restrict__ vg, double* __restrict__ gfp) {
    const int NF = 4 * n;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)E * NF) return;
    const int e = (int)(t / NF), f = (int)((t / n) % 4), k = (int)(t % n);
    double Sx, Sy, J, u, v;
    face_eval(E, n, gt, xg, vg, e, f, k, Sx, Sy, J, u, v);
    const int pk = nbr[e * 4 + f];
    const int nb = pk >> 3, nf = (pk >> 1) & 3, k2 = (pk & 1) ? n - 1 - k : k;
    double Sx2, Sy2, J2, u2, v2;
    face_eval(E, n, gt, xg, vg, nb, nf, k2, Sx2, Sy2, J2, u2, v2);
    const double sg = (f & 1) ? 1.0 : -1.0;
    if (e * 4 + f > nb * 4 + nf) {
        // the owner (smaller side index) defines the face vector and grid velocity
        const double s2 = sg * ((nf & 1) ? 1.0 : -1.0);
        Sx = -s2 * Sx2; Sy = -s2 * Sy2; u = u2; v = v2;
    }
    const double Ox = sg * Sx, Oy = sg * Sy;
    const double Smag = sqrt(Ox * Ox + Oy * Oy);
    const size_t FE = (size_t)E * NF;
    gfp[F_NX * FE + t] = Ox / Smag;
    gfp[F_NY * FE + t] = Oy / Smag;
    gfp[F_SC * FE + t] = sg * Smag;
    gfp[F_CC * FE + t] = 0.25 * br2 * Smag * (1.0 / J + 1.0 / J2);
    gfp[F_UG * FE + t] = u;
    gfp[F_VG * FE + t] = v;
}

// ------------------------------------------------------------------ trace kernel
// Traces of q and of the uncorrected chain-rule gradient at the flux points of every
// element, trace[E][4][NTV][n] (NTV = 10 viscous, 4 inviscid); value-only, used by the
// adjoint path.
struct TrArgs {
    int E;
    const double* q;
    double* out;
};

template <int P, bool VISC>
__global__ void __launch_bounds__((Blk<P, 1>::threads))
k_traces(TrArgs a, OpTab op_in, Geo g) {
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT;
    constexpr int EPB = Blk<P, 1>::EPB, NTV = VISC ? 10 : 4;
    __shared__ OpTab op;   // operator tables (lane-dependent indexing in LDS)
    for (int t = threadIdx.x; t < (int)(sizeof(OpTab) / sizeof(double)); t += blockDim.x)
        reinterpret_cast<double*>(&op)[t] = reinterpret_cast<const double*>(&op_in)[t];
    __shared__ double s_q[EPB][4][Np];
    __shared__ double s_w[EPB][VISC ? 6 : 1][Np];
    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    const int e = blockIdx.x * EPB + el;
    const bool act = e < a.E;
    const size_t EN = (size_t)a.E * Np;
    const int i = lt % n, j = lt / n;
    if (act && lt < Np) {
        const size_t id = (size_t)e * Np + lt;
#pragma unroll
        for (int v = 0; v < 4; ++v) s_q[el][v][lt] = a.q[v * EN + id];
    }
    __syncthreads();
    if (VISC && act && lt < Np) {
        const size_t id = (size_t)e * Np + lt;
        const double xix = g.sp[G_XIX * EN + id], xiy = g.sp[G_XIY * EN + id];
        const double etx = g.sp[G_ETX * EN + id], ety = g.sp[G_ETY * EN + id];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double dxi = 0.0, deta = 0.0;
#pragma unroll
            for (int b = 0; b < n; ++b) {
                dxi += op.D[i * n + b] * s_q[el][c + 1][b + n * j];
                deta += op.D[j * n + b] * s_q[el][c + 1][i + n * b];
            }
            s_w[el][2 * c][lt] = xix * dxi + etx * deta;
            s_w[el][2 * c + 1][lt] = xiy * dxi + ety * deta;
        }
    }
    __syncthreads();
    if (act && lt < NF) {
        const int f = lt / n, k = lt % n;
        const double* lam = (f == 0 || f == 2) ? op.lamL : op.lamR;
        double* dst = a.out + ((size_t)(e * 4 + f) * NTV) * n;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < n; ++b) acc += lam[b] * s_q[el][v][line_pt(n, f, k, b)];
            dst[(size_t)v * n + k] = acc;
        }
        if (VISC) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int b = 0; b < n; ++b) acc += lam[b] * s_w[el][c][line_pt(n, f, k, b)];
                dst[(size_t)(4 + c) * n + k] = acc;
            }
        }
    }
}

template <int P, bool VISC>
fr_status run_traces(fr_ctx c, const TrArgs& a, hipStream_t s) {
    using B = Blk<P, 1>;
    const Geo g = c->geo();
    const int grid = (c->E + B::EPB - 1) / B::EPB;
    hipLaunchKernelGGL((k_traces<P, VISC>), dim3(grid), dim3(B::threads), 0, s, a, c->op, g);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

template <int P>
fr_status traces_p(fr_ctx c, const TrArgs& a, hipStream_t s) {
    return c->prm.viscous ? run_traces<P, true>(c, a, s) : run_traces<P, false>(c, a, s);
}

}  // namespace

fr_status launch_geometry(fr_ctx c, const double* xg, const double* vg, hipStream_t s) {
    const int bs = 256;
    size_t nsp = (size_t)c->E * c->Np, nfp = (size_t)c->E * 4 * c->n;
    hipLaunchKernelGGL(k_geo_sp, dim3((unsigned)((nsp + bs - 1) / bs)), dim3(bs), 0, s, c->E, c->n, c->gt, xg, vg, c->d_gsp);
    FR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_geo_fp, dim3((unsigned)((nfp + bs - 1) / bs)), dim3(bs), 0, s, c->E, c->n, c->gt, c->pc.br2,
                       c->d_nbr, xg, vg, c->d_gfp);
    FR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_affine, dim3((unsigned)((c->E + bs - 1) / bs)), dim3(bs), 0, s, c->E, c->Np, c->d_gsp,
                       c->d_bc, c->d_aff);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

// value traces of q into `trace`
fr_status launch_traces(fr_ctx c, const double* q, double* trace, hipStream_t s) {
    TrArgs a{c->E, q, trace};
    switch (c->p) {
        case 1: return traces_p<1>(c, a, s);
        case 2: return traces_p<2>(c, a, s);
        case 3: return traces_p<3>(c, a, s);
        case 4: return traces_p<4>(c, a, s);
    }
    fr_set_error("order outside 1..4");
    return FR_EUNSUPPORTED;
}

fr_status launch_fused(const Solver& sv, const Group& gr, int mode, const KArgs& a, const Tune& t, hipStream_t s) {
    switch (gr.p) {
        case 1: return launch_fused_p<1>(sv, gr, mode, a, t, s);
        case 2: return launch_fused_p<2>(sv, gr, mode, a, t, s);
        case 3: return launch_fused_p<3>(sv, gr, mode, a, t, s);
        case 4: return launch_fused_p<4>(sv, gr, mode, a, t, s);
    }
    fr_set_error("order outside 1..4");
    return FR_EUNSUPPORTED;
}

fr_status solver_fused(const Solver& sv, int mode, const KArgs& a, hipStream_t s) {
    for (const Group& gr : sv.groups) FR_TRY(launch_fused(sv, gr, mode, a, gr.tune[mode], s));
    return FR_OK;
}

std::vector<int> fused_tile_widths(int p) {
    const int n = p + 1, Np = n * n, NF = 4 * n, NT = Np > NF ? Np : NF;
    std::vector<int> w;
    for (int lanes : {64, 128, 256}) {
        const int epb = lanes / NT > 0 ? lanes / NT : 1;
        bool have = false;
        for (int x : w) have |= x == epb;
        if (!have) w.push_back(epb);
    }
    return w;
}
