// FR/CPR residual kernels for gfx950: geometry (metrics, face vectors, grid
// velocity), solution/gradient traces, and the fused per-element residual kernel
// that also produces exact JVPs, the BDF2 Newton operator and seeded columns of the
// element Jacobian blocks (forward tangents through Dual<K> scalars).
//
// Work mapping: one workgroup holds EPB elements; each element owns NT = max(Np, 4n)
// lanes, lane `lt` acting as solution point lt (lt < Np) and as flux point lt
// (lt < 4n, face lt/n, point lt%n).  Element data live in LDS between the stages:
//   1. load q (+ tangent)                       [solution points]
//   2. uncorrected chain-rule gradient          [solution points]
//   3. traces, neighbour traces, common flux    [flux points]  Eq. (Rosanov), BR2
//   4. corrected gradient, fluxes f, g, q^c     [solution points]
//   5. F^num - F^loc at the flux points         [flux points]  Eq. (norm_f_2)
//   6. chain-rule divergence, moving-mesh terms, Radau lift -> R   Eq. (cpr_ns)
// Accesses to state and metric arrays are coalesced ([var][E][Np] layouts).
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

// ------------------------------------------------------------------ state loads
template <class T> struct Seed;
template <> struct Seed<double> {
    __device__ static double load(const KArgs& a, unsigned gid, int, double*) { return a.q[gid]; }
};
template <int K> struct Seed<Dual<K>> {
    // JVP / AOP: tangent from a.v; block mode: unit seeds at columns seed0..seed0+K-1
    __device__ static Dual<K> load(const KArgs& a, unsigned gid, int col, double*) {
        Dual<K> r; r.v = a.q[gid];
        if (a.v) {
#pragma unroll
            for (int k = 0; k < K; ++k) r.d[k] = a.v[gid];
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) r.d[k] = (col == a.seed0 + k) ? 1.0 : 0.0;
        }
        return r;
    }
};

template <class T, class TN> struct Conv;
template <class T> struct Conv<T, T> { __device__ static T c(const T& x) { return x; } };
template <int K> struct Conv<Dual<K>, double> { __device__ static Dual<K> c(double x) { return mkconst<K>(x); } };

// traces of q and of the uncorrected gradient at face f, point k of the element in LDS
template <int P, bool VISC, class T>
__device__ __forceinline__ void own_trace(const OpTab& op, const T (*sq)[Sz<P>::Np], const T (*sw)[Sz<P>::Np],
                                          int f, int k, T* qm, T* gm) {
    constexpr int n = P + 1;
    const double* lam = (f == 0 || f == 2) ? op.lamL : op.lamR;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        T s = cst<T>(0.0);
#pragma unroll
        for (int a = 0; a < n; ++a) s = s + lam[a] * sq[v][line_pt(n, f, k, a)];
        qm[v] = s;
    }
    if (VISC) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            T s = cst<T>(0.0);
#pragma unroll
            for (int a = 0; a < n; ++a) s = s + lam[a] * sw[c][line_pt(n, f, k, a)];
            gm[c] = s;
        }
    }
}

// stage 1+2 shared by the trace and residual kernels: load q, uncorrected gradient
template <int P, bool VISC, int NGL, class T>
__device__ __forceinline__ void stage_load_grad(const KArgs& a, const OpTab& op, const Geo& g, int e, int lt, bool act,
                                                T (*sq)[Sz<P>::Np], T (*sw)[Sz<P>::Np], T* qs, T* gu, T* gv, T* gT,
                                                double* geo) {
    constexpr int n = P + 1, Np = n * n;
    const size_t EN = (size_t)a.E * Np;
    if (act && lt < Np) {
        const size_t id = (size_t)e * Np + lt;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            qs[v] = Seed<T>::load(a, v * EN + id, v * Np + lt, nullptr);
            sq[v][lt] = qs[v];
        }
#pragma unroll
        for (int c = 0; c < NGL; ++c) geo[c] = g.sp[c * EN + id];   // only the fields this kernel uses
    }
    __syncthreads();
    if (VISC && act && lt < Np) {
        const int i = lt % n, j = lt / n;
        T* gr[3] = {gu, gv, gT};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T dxi = cst<T>(0.0), deta = cst<T>(0.0);
#pragma unroll
            for (int b = 0; b < n; ++b) {
                dxi = dxi + op.D[i * n + b] * sq[c + 1][b + n * j];
                deta = deta + op.D[j * n + b] * sq[c + 1][i + n * b];
            }
            gr[c][0] = geo[G_XIX] * dxi + geo[G_ETX] * deta;
            gr[c][1] = geo[G_XIY] * dxi + geo[G_ETY] * deta;
            sw[2 * c][lt] = gr[c][0];
            sw[2 * c + 1][lt] = gr[c][1];
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ trace kernel
template <int P, bool VISC, class T>
__global__ void __launch_bounds__((Blk<P, Store<T>::W>::threads))
k_traces(KArgs a, OpTab op_in, Geo g) {
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT;
    __shared__ OpTab sop;   // operator tables (lane-dependent indexing in LDS)
    for (int t = threadIdx.x; t < (int)(sizeof(OpTab) / sizeof(double)); t += blockDim.x)
        reinterpret_cast<double*>(&sop)[t] = reinterpret_cast<const double*>(&op_in)[t];
    const OpTab& op = sop;
    constexpr int EPB = Blk<P, Store<T>::W>::EPB, W = Store<T>::W, NTV = VISC ? 10 : 4;
    __shared__ T s_q[EPB][4][Np];
    __shared__ T s_w[EPB][VISC ? 6 : 1][Np];
    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    const int e = blockIdx.x * EPB + el;
    const bool act = e < a.E;
    T qs[4], gu[2], gv[2], gT[2];
    double geo[NGSP];
    stage_load_grad<P, VISC, VISC ? 4 : 0, T>(a, op, g, e, lt, act, s_q[el], s_w[el], qs, gu, gv, gT, geo);
    if (act && lt < NF) {
        const int f = lt / n, k = lt % n;
        T qm[4], gm[6];
        own_trace<P, VISC, T>(op, s_q[el], s_w[el], f, k, qm, gm);
        double* dst = a.out + ((size_t)(e * 4 + f) * NTV) * n * W;
#pragma unroll
        for (int v = 0; v < 4; ++v) Store<T>::st(dst + ((size_t)v * n + k) * W, qm[v]);
        if (VISC) {
#pragma unroll
            for (int c = 0; c < 6; ++c) Store<T>::st(dst + ((size_t)(4 + c) * n + k) * W, gm[c]);
        }
    }
}

// ------------------------------------------------------------------ fused residual kernel
template <int MODE, int K> struct ModeT { using T = Dual<K>; };
template <int K> struct ModeT<MODE_R, K> { using T = double; };

// workgroup shape of the fused kernel: 128 lanes for doubles, 64 for dual numbers (LDS)
template <int P, int W>
struct FBlk {
    static constexpr int NT = Sz<P>::NT;
    static constexpr int lanes = (W == 1) ? 128 : 64;
    static constexpr int EPB = (lanes / NT) > 0 ? (lanes / NT) : 1;
    static constexpr int threads = EPB * NT;
};

// neighbour state with the tangent the mode asks for: JVP/AOP carry v; block mode
// seeds only when the neighbour is the element itself (periodic single-element rows)
template <class T> struct NbLoad;
template <> struct NbLoad<double> {
    __device__ static double load(const KArgs& a, unsigned gid, int, bool) { return a.q[gid]; }
};
template <int K> struct NbLoad<Dual<K>> {
    __device__ static Dual<K> load(const KArgs& a, unsigned gid, int col, bool self) {
        Dual<K> r; r.v = a.q[gid];
        if (a.v) {
#pragma unroll
            for (int k = 0; k < K; ++k) r.d[k] = a.v[gid];
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) r.d[k] = (self && col == a.seed0 + k) ? 1.0 : 0.0;
        }
        return r;
    }
};

// (q^- + q^+)/2 of one variable, recomputed from the own trace and the jump
template <class T, int NP>
__device__ __forceinline__ T am_avg(const T* sv, const double* lam, int f, int k, const T& jump, int n) {
    T acc = cst<T>(0.0);
    for (int b = 0; b < n; ++b) acc = acc + lam[b] * sv[line_pt(n, f, k, b)];
    return acc + 0.5 * jump;
}

// Single pass per element.  The states of the four face neighbours are staged in LDS
// (their reads are served mostly by L2: neighbours are processed by nearby workgroups)
// and their traces on the shared faces are recomputed here, so state, metrics and the
// result cross HBM once.
template <int P, bool VISC, bool MOV, int MODE, int K>
__global__ void __launch_bounds__((FBlk<P, Store<typename ModeT<MODE, K>::T>::W>::threads))
k_fused(KArgs a, OpTab op, PhysConst pc, Geo g) {
    using T = typename ModeT<MODE, K>::T;
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT;
    constexpr int EPB = FBlk<P, Store<T>::W>::EPB;
    constexpr int NW = MOV ? 12 : 8;
    static_assert(NW <= 16, "flux fields alias the neighbour staging area");
    __shared__ T s_q[EPB][4][Np];
    __shared__ T s_n[EPB][16][Np];      // neighbour states [face*4 + var]; later f, g (, q^c)
    __shared__ T s_g[EPB][VISC ? 6 : 1][Np];
    __shared__ T s_F[EPB][NF][4];       // F^num, then F^num - F^loc
    __shared__ T s_dq[EPB][NF][VISC ? 3 : 1];
    __shared__ double s_S[EPB][NF][3];  // element-oriented S, S . v_g
    __shared__ double s_D[n * n];       // operator tables (lane-dependent indexing goes to LDS)
    __shared__ double s_lam[2][n], s_gam[2][n];

    if (a.skip && *a.skip) return;   // uniform: a finished GMRES cycle replays as no-ops
    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) s_D[t] = op.D[t];
    if (threadIdx.x < n) {
        s_lam[0][threadIdx.x] = op.lamL[threadIdx.x]; s_lam[1][threadIdx.x] = op.lamR[threadIdx.x];
        s_gam[0][threadIdx.x] = op.gamL[threadIdx.x]; s_gam[1][threadIdx.x] = op.gamR[threadIdx.x];
    }
    const int e = blockIdx.x * EPB + el;
    const bool act = e < a.E;
    const int E = a.E;
    const unsigned EN = (unsigned)E * Np;   // state arrays hold < 2^31 entries (checked at creation)
    const int i = lt % n, j = lt / n;
    // ---- stage 1: own state and neighbour states into LDS
    if (act && lt < Np) {
        const unsigned id = (unsigned)e * Np + lt;
#pragma unroll
        for (int v = 0; v < 4; ++v) s_q[el][v][lt] = Seed<T>::load(a, v * EN + id, v * Np + lt, nullptr);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int nb = g.nbr[e * 4 + f] >> 3;
            const unsigned nid = (unsigned)nb * Np + lt;
#pragma unroll
            for (int v = 0; v < 4; ++v) s_n[el][f * 4 + v][lt] = NbLoad<T>::load(a, v * EN + nid, v * Np + lt, nb == e);
        }
    }
    __syncthreads();
    // ---- stage 2: own uncorrected gradient (kept in LDS only)
    if (VISC && act && lt < Np) {
        const unsigned id = (unsigned)e * Np + lt;
        const double xix = g.sp[G_XIX * EN + id], xiy = g.sp[G_XIY * EN + id];
        const double etx = g.sp[G_ETX * EN + id], ety = g.sp[G_ETY * EN + id];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T dxi = cst<T>(0.0), deta = cst<T>(0.0);
#pragma unroll
            for (int b = 0; b < n; ++b) {
                dxi = dxi + s_D[i * n + b] * s_q[el][c + 1][b + n * j];
                deta = deta + s_D[j * n + b] * s_q[el][c + 1][i + n * b];
            }
            s_g[el][2 * c][lt] = xix * dxi + etx * deta;
            s_g[el][2 * c + 1][lt] = xiy * dxi + ety * deta;
        }
    }
    __syncthreads();
    // ---- stage 3: own and neighbour traces, common flux at the flux points
    if (act && lt < NF) {
        const int f = lt / n, k = lt % n;
        const int pk = g.nbr[e * 4 + f];
        const int nb = pk >> 3, nf = (pk >> 1) & 3, k2 = (pk & 1) ? n - 1 - k : k;
        const double* lam = s_lam[f & 1];
        const double* lamn = s_lam[nf & 1];
        const unsigned FE = (unsigned)E * NF;
        const unsigned sid = (unsigned)e * NF + lt;
        const double nx = g.fp[F_NX * FE + sid], ny = g.fp[F_NY * FE + sid];
        const double sc = g.fp[F_SC * FE + sid];
        const double ugf = MOV ? g.fp[F_UG * FE + sid] : 0.0;
        const double vgf = MOV ? g.fp[F_VG * FE + sid] : 0.0;
        T fn[4], dq[4];
        {
            T qm[4], qp[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T am = cst<T>(0.0), ap = cst<T>(0.0);
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    am = am + lam[b] * s_q[el][v][line_pt(n, f, k, b)];
                    ap = ap + lamn[b] * s_n[el][f * 4 + v][line_pt(n, nf, k2, b)];
                }
                qm[v] = am;
                qp[v] = ap;
            }
            fr_common_inviscid<T>(pc, qm, qp, nx, ny, ugf, vgf, fn, dq);
        }
        if (VISC) {
            T gm[6], gp[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                T am = cst<T>(0.0);
#pragma unroll
                for (int b = 0; b < n; ++b) am = am + lam[b] * s_g[el][c][line_pt(n, f, k, b)];
                gm[c] = am;
                gp[c] = cst<T>(0.0);
            }
            // neighbour's uncorrected gradient along the line through its face point, traced
#pragma unroll
            for (int b = 0; b < n; ++b) {
                const int sp = line_pt(n, nf, k2, b);
                const int is = sp % n, js = sp / n;
                const unsigned gid = (unsigned)nb * Np + sp;
                const double xix = g.sp[G_XIX * EN + gid], xiy = g.sp[G_XIY * EN + gid];
                const double etx = g.sp[G_ETX * EN + gid], ety = g.sp[G_ETY * EN + gid];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T dxi = cst<T>(0.0), deta = cst<T>(0.0);
#pragma unroll
                    for (int m = 0; m < n; ++m) {
                        dxi = dxi + s_D[is * n + m] * s_n[el][f * 4 + c + 1][m + n * js];
                        deta = deta + s_D[js * n + m] * s_n[el][f * 4 + c + 1][is + n * m];
                    }
                    gp[2 * c] = gp[2 * c] + lamn[b] * (xix * dxi + etx * deta);
                    gp[2 * c + 1] = gp[2 * c + 1] + lamn[b] * (xiy * dxi + ety * deta);
                }
            }
            // q^com velocity = average of the two traces = q^- + dq/2
            const T qcu = am_avg<T, Np>(s_q[el][1], lam, f, k, dq[1], n);
            const T qcv = am_avg<T, Np>(s_q[el][2], lam, f, k, dq[2], n);
            T dqh[3];
            fr_common_viscous<T>(pc, dq, qcu, qcv, gm, gp, nx, ny, g.fp[F_CC * FE + sid], fn, dqh);
#pragma unroll
            for (int c = 0; c < 3; ++c) s_dq[el][lt][c] = dqh[c];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) s_F[el][lt][v] = sc * fn[v];
        s_S[el][lt][0] = sc * nx;                                  // element-oriented S
        s_S[el][lt][1] = sc * ny;
        s_S[el][lt][2] = MOV ? sc * (ugf * nx + vgf * ny) : 0.0;   // S . v_g
    }
    __syncthreads();

    // ---- stage 4: corrected gradient, pointwise fluxes (into the staging area)
    T (*s_w)[Np] = s_n[el];
    T qs[4];
    if (act && lt < Np) {
        const unsigned id = (unsigned)e * Np + lt;
        const double ij = g.sp[G_IJ * EN + id];
#pragma unroll
        for (int v = 0; v < 4; ++v) qs[v] = s_q[el][v][lt];
        T gu[2], gv[2], gT[2];
        if (VISC) {
#pragma unroll
            for (int d = 0; d < 2; ++d) { gu[d] = s_g[el][d][lt]; gv[d] = s_g[el][2 + d][lt]; gT[d] = s_g[el][4 + d][lt]; }
        }
        if (VISC) {
            const int fp0 = 0 * n + j, fp1 = 1 * n + j, fp2 = 2 * n + i, fp3 = 3 * n + i;
            const double gL_i = s_gam[0][i], gR_i = s_gam[1][i], gL_j = s_gam[0][j], gR_j = s_gam[1][j];
            T* gr[3] = {gu, gv, gT};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T cx = (s_S[el][fp0][0] * gL_i) * s_dq[el][fp0][c] + (s_S[el][fp1][0] * gR_i) * s_dq[el][fp1][c]
                     + (s_S[el][fp2][0] * gL_j) * s_dq[el][fp2][c] + (s_S[el][fp3][0] * gR_j) * s_dq[el][fp3][c];
                T cy = (s_S[el][fp0][1] * gL_i) * s_dq[el][fp0][c] + (s_S[el][fp1][1] * gR_i) * s_dq[el][fp1][c]
                     + (s_S[el][fp2][1] * gL_j) * s_dq[el][fp2][c] + (s_S[el][fp3][1] * gR_j) * s_dq[el][fp3][c];
                gr[c][0] = gr[c][0] + ij * cx;
                gr[c][1] = gr[c][1] + ij * cy;
            }
        }
        T fl[4], gl[4], qc[4];
        fr_point_flux<T, VISC>(pc, qs, gu, gv, gT, fl, gl, qc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            s_w[v][lt] = fl[v];
            s_w[4 + v][lt] = gl[v];
            if (MOV) s_w[8 + v][lt] = qc[v];
        }
    }
    __syncthreads();

    // ---- stage 5: F^num - F^loc, F^loc = S.(Pi f, Pi g) - (S.v_g) Pi q^c
    if (act && lt < NF) {
        const int f = lt / n, k = lt % n;
        const double* lam = s_lam[f & 1];
        const double Sx = s_S[el][lt][0], Sy = s_S[el][lt][1], Svg = s_S[el][lt][2];
#pragma unroll 1
        for (int v = 0; v < 4; ++v) {
            T acc = cst<T>(0.0);
#pragma unroll
            for (int b = 0; b < n; ++b) {
                const int sp = line_pt(n, f, k, b);
                T vv = Sx * s_w[v][sp] + Sy * s_w[4 + v][sp];
                if (MOV) vv = vv - Svg * s_w[8 + v][sp];
                acc = acc + lam[b] * vv;
            }
            s_F[el][lt][v] = s_F[el][lt][v] - acc;
        }
    }
    __syncthreads();

    // ---- stage 6: divergence + moving-mesh terms + Radau lift, one variable at a time
    if (act && lt < Np) {
        const unsigned id = (unsigned)e * Np + lt;
        double geo[NGSP] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < (MOV ? NGSP : G_UG); ++c) geo[c] = g.sp[c * EN + id];
        const double axi = MOV ? geo[G_UG] * geo[G_XIX] + geo[G_VG] * geo[G_XIY] : 0.0;
        const double aet = MOV ? geo[G_UG] * geo[G_ETX] + geo[G_VG] * geo[G_ETY] : 0.0;
        double tt[4] = {0.0, 0.0, 0.0, 0.0};   // time terms (Newton operator)
        if constexpr (MODE == MODE_AOP) {
            double qv[4], x[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) { qv[v] = qs[v].v; x[v] = qs[v].d[0]; }
            fr_time_apply<double, double>(pc, qv, geo[G_UG], geo[G_VG], a.inv_dtau, a.c_time, x, tt);
        }
#pragma unroll 1
        for (int v = 0; v < 4; ++v) {
            T dfx = cst<T>(0.0), dfe = cst<T>(0.0), dgx = cst<T>(0.0), dge = cst<T>(0.0);
            T dqx = cst<T>(0.0), dqe = cst<T>(0.0);
#pragma unroll
            for (int b = 0; b < n; ++b) {
                const double Dx = s_D[i * n + b], De = s_D[j * n + b];
                dfx = dfx + Dx * s_w[v][b + n * j];
                dgx = dgx + Dx * s_w[4 + v][b + n * j];
                dfe = dfe + De * s_w[v][i + n * b];
                dge = dge + De * s_w[4 + v][i + n * b];
                if (MOV) {
                    dqx = dqx + Dx * s_w[8 + v][b + n * j];
                    dqe = dqe + De * s_w[8 + v][i + n * b];
                }
            }
            T vol = geo[G_XIX] * dfx + geo[G_ETX] * dfe + geo[G_XIY] * dgx + geo[G_ETY] * dge;
            if (MOV) vol = vol - axi * dqx - aet * dqe;
            T cor = s_gam[0][i] * s_F[el][0 * n + j][v] + s_gam[1][i] * s_F[el][1 * n + j][v]
                  + s_gam[0][j] * s_F[el][2 * n + i][v] + s_gam[1][j] * s_F[el][3 * n + i][v];
            const T R = -(vol + geo[G_IJ] * cor);
            if constexpr (MODE == MODE_R) {
                a.out[v * EN + id] = val(R);
            } else if constexpr (MODE == MODE_JVP) {
                a.out[v * EN + id] = R.d[0];
                if (a.out2) a.out2[v * EN + id] = R.v;
            } else if constexpr (MODE == MODE_AOP) {
                const double ttv = (v == 0) ? tt[0] : (v == 1) ? tt[1] : (v == 2) ? tt[2] : tt[3];
                a.out[v * EN + id] = ttv - R.d[0];
            } else {
                // block columns seed0..seed0+K-1 of element e, column-major [E][nb][nb]
                constexpr int nbk = 4 * Np;
                double* blk = a.out + (size_t)e * nbk * nbk;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int col = a.seed0 + k;
                    if (col < nbk) blk[(size_t)col * nbk + v * Np + lt] = -R.d[k];
                }
            }
        }
        if constexpr (MODE == MODE_BLK) {
            // time terms on the diagonal point block of the seeded columns
            constexpr int nbk = 4 * Np;
            double* blk = a.out + (size_t)e * nbk * nbk;
            double qv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) qv[v] = qs[v].v;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int col = a.seed0 + k;
                if (col < nbk && col % Np == lt) {
                    double x[4] = {0.0, 0.0, 0.0, 0.0}, t4[4];
                    x[col / Np] = 1.0;
                    fr_time_apply<double, double>(pc, qv, geo[G_UG], geo[G_VG], a.inv_dtau, a.c_time, x, t4);
#pragma unroll
                    for (int v = 0; v < 4; ++v) blk[(size_t)col * nbk + v * Np + lt] += t4[v];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ dispatch
template <int P, bool VISC, class T>
fr_status run_traces(fr_ctx c, const KArgs& a, hipStream_t s) {
    using B = Blk<P, Store<T>::W>;
    Geo g{c->d_gsp, c->d_gfp, c->d_nbr};
    const int grid = (c->E + B::EPB - 1) / B::EPB;
    hipLaunchKernelGGL((k_traces<P, VISC, T>), dim3(grid), dim3(B::threads), 0, s, a, c->op, g);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

template <int P, bool VISC, bool MOV, int MODE, int K>
fr_status run_resid(fr_ctx c, const KArgs& a, hipStream_t s) {
    using T = typename ModeT<MODE, K>::T;
    using B = FBlk<P, Store<T>::W>;
    Geo g{c->d_gsp, c->d_gfp, c->d_nbr};
    const int grid = (c->E + B::EPB - 1) / B::EPB;
    hipLaunchKernelGGL((k_fused<P, VISC, MOV, MODE, K>), dim3(grid), dim3(B::threads), 0, s, a, c->op, c->pc, g);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

template <int P, bool VISC, bool MOV>
fr_status resid_mode(fr_ctx c, int mode, const KArgs& a, hipStream_t s) {
    switch (mode) {
        case MODE_R: return run_resid<P, VISC, MOV, MODE_R, 1>(c, a, s);
        case MODE_JVP: return run_resid<P, VISC, MOV, MODE_JVP, 1>(c, a, s);
        case MODE_AOP: return run_resid<P, VISC, MOV, MODE_AOP, 1>(c, a, s);
        case MODE_BLK: return run_resid<P, VISC, MOV, MODE_BLK, 1>(c, a, s);
    }
    fr_set_error("unknown residual mode");
    return FR_EINVAL;
}

template <int P>
fr_status resid_p(fr_ctx c, int mode, const KArgs& a, hipStream_t s) {
    const bool visc = c->prm.viscous != 0, mov = c->prm.moving != 0;
    if (visc) return mov ? resid_mode<P, true, true>(c, mode, a, s) : resid_mode<P, true, false>(c, mode, a, s);
    return mov ? resid_mode<P, false, true>(c, mode, a, s) : resid_mode<P, false, false>(c, mode, a, s);
}

template <int P>
fr_status traces_p(fr_ctx c, const KArgs& a, int lanes, hipStream_t s) {
    const bool visc = c->prm.viscous != 0;
    if (lanes == 0) return visc ? run_traces<P, true, double>(c, a, s) : run_traces<P, false, double>(c, a, s);
    return visc ? run_traces<P, true, Dual<1>>(c, a, s) : run_traces<P, false, Dual<1>>(c, a, s);
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
    return FR_OK;
}

// traces of q (lanes = 0) or of (q, v) as Dual<1> (lanes = 1) into `trace`
fr_status launch_traces(fr_ctx c, const double* q, const double* v, double* trace, int lanes, hipStream_t s) {
    KArgs a{};
    a.E = c->E; a.q = q; a.v = v; a.out = trace;
    switch (c->p) {
        case 1: return traces_p<1>(c, a, lanes, s);
        case 2: return traces_p<2>(c, a, lanes, s);
        case 3: return traces_p<3>(c, a, lanes, s);
        case 4: return traces_p<4>(c, a, lanes, s);
    }
    fr_set_error("order outside 1..4");
    return FR_EUNSUPPORTED;
}

fr_status launch_residual(fr_ctx c, int mode, const KArgs& a, hipStream_t s) {
    switch (c->p) {
        case 1: return resid_p<1>(c, mode, a, s);
        case 2: return resid_p<2>(c, mode, a, s);
        case 3: return resid_p<3>(c, mode, a, s);
        case 4: return resid_p<4>(c, mode, a, s);
    }
    fr_set_error("order outside 1..4");
    return FR_EUNSUPPORTED;
}
