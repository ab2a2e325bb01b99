// Fused per-element FR/CPR residual kernel for gfx950, shared by the per-order
// translation units (fr_fused_p1..p4.hip).  One kernel produces, by mode,
//   R      the residual (paper Eq. cpr_ns with the moving-mesh terms),
//   JVP    the exact forward tangent Jv (and optionally R),
//   AOP    the Newton operator  Av = inv_dtau Gamma v + c_time M v - Jv,
//   BLK    one seeded column of every element's diagonal block of that operator.
//
// Work mapping: a workgroup tile holds EPB elements of one case; each element owns
// NT = max(Np, 4n) lanes, lane `lt` acting as solution point lt (lt < Np) and as flux
// point lt (lt < 4n, face lt/n, point lt%n).  Element data live in LDS between the
// stages:
//   1. own state and the four neighbour states      [solution points]
//   2. uncorrected chain-rule gradient               [solution points]
//   3. own and neighbour traces, common flux         [flux points]  Eq. (Rosanov), BR2
//   4. corrected gradient, fluxes f, g, q^c          [solution points]
//   5. F^num - F^loc at the flux points              [flux points]  Eq. (norm_f_2)
//   6. chain-rule divergence, moving-mesh terms, Radau lift -> output
// The grid is persistent and XCD-aware: workgroup b runs on XCD b % 8 and walks the
// tiles of a contiguous eighth of the tile list, so an element and its face
// neighbours (whose states are re-read here) are mostly served by the same L2.
// Tiles of many cases (a batch) form one list; a tile finds its case by binary search
// over the group's tile prefix and reads the case's metrics, offsets and constants
// from its descriptor.
#pragma once
#include "fr_internal.hpp"

namespace fused {

template <int P>
struct Sz {
    static constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = (Np > NF ? Np : NF);
};

// elements per workgroup for a workgroup width of LANES
template <int P, int LANES>
struct Shape {
    static constexpr int NT = Sz<P>::NT;
    static constexpr int EPB = (LANES / NT) > 0 ? (LANES / NT) : 1;
    static constexpr int threads = EPB * NT;
};

__device__ __forceinline__ int line_pt(int n, int f, int k, int a) {
    return f < 2 ? a + n * k : k + n * a;
}


template <class T> __device__ __forceinline__ T ldo(const T* base, unsigned idx);

template <int MODE, int K> struct ModeT { using T = Dual<K>; };
template <int K> struct ModeT<MODE_R, K> { using T = double; };
template <int K> struct ModeT<MODE_PREP, K> { using T = double; };

// own state with the tangent the mode asks for: JVP/AOP carry v; block mode seeds the
// unit column seed0 (+k)
template <class T> struct Seed;
template <> struct Seed<double> {
    __device__ static double load(const KArgs& a, const double* q, const double*, unsigned gid, int) { return ldo(q, gid); }
};
template <int K> struct Seed<Dual<K>> {
    __device__ static Dual<K> load(const KArgs& a, const double* q, const double* v, unsigned gid, int col) {
        Dual<K> r; r.v = ldo(q, gid);
        if (v) {
#pragma unroll
            for (int k = 0; k < K; ++k) r.d[k] = ldo(v, gid);
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) r.d[k] = (col == a.seed0 + k) ? 1.0 : 0.0;
        }
        return r;
    }
};

// neighbour state: block mode seeds only when the neighbour is the element itself
// (periodic single-element rows)
template <class T> struct NbLoad;
template <> struct NbLoad<double> {
    __device__ static double load(const KArgs&, const double* q, const double*, unsigned gid, int, bool) { return ldo(q, gid); }
};
template <int K> struct NbLoad<Dual<K>> {
    __device__ static Dual<K> load(const KArgs& a, const double* q, const double* v, unsigned gid, int col, bool self) {
        Dual<K> r; r.v = ldo(q, gid);
        if (v) {
#pragma unroll
            for (int k = 0; k < K; ++k) r.d[k] = ldo(v, gid);
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) r.d[k] = (self && col == a.seed0 + k) ? 1.0 : 0.0;
        }
        return r;
    }
};

// (q^- + q^+)/2 of one variable, recomputed from the own trace and the jump
template <class T>
__device__ __forceinline__ T am_avg(const T* sv, const double* lam, int f, int k, const T& jump, int n) {
    T acc = cst<T>(0.0);
    for (int b = 0; b < n; ++b) acc = acc + lam[b] * sv[line_pt(n, f, k, b)];
    return acc + 0.5 * jump;
}

// Values that are uniform across the workgroup but loaded from memory that the kernel
// also writes to are moved to scalar registers explicitly (the compiler cannot prove
// that they are not clobbered between tiles, so it keeps them in vector registers).
__device__ __forceinline__ int rfl(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ unsigned long long rfl(unsigned long long x) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double rfl(double x) {
    return __longlong_as_double((long long)rfl((unsigned long long)__double_as_longlong(x)));
}
template <class T> __device__ __forceinline__ T* rfl(T* p) {
    return reinterpret_cast<T*>(rfl((unsigned long long)reinterpret_cast<uintptr_t>(p)));
}

// base[idx] for a workgroup-uniform base: the byte offset is formed in 32 bits, so the load
// takes the scalar-base + 32-bit vector-offset form instead of per-lane 64-bit address
// arithmetic.  Needs idx * sizeof(T) < 2^32; every per-field index of a case (solution or flux
// point, connectivity entry) satisfies it by the size limits that fr_create checks.  The base
// goes through rfl (both 32-bit halves), so that the compiler does not fold a uniform part of
// it (a field or variable offset) into the per-lane address.
template <class T> __device__ __forceinline__ T ldo(const T* base, unsigned idx) {
    const unsigned off = idx * (unsigned)sizeof(T);
    const char* b = reinterpret_cast<const char*>(rfl(base));
    return *(const __attribute__((address_space(1))) T*)(b + off);
}

// Read-only tables of a launch (case descriptors, case ids, tile prefixes: written once when
// the solver is set up) are read through the scalar cache: the address is uniform, and a
// pointer into the constant address space lets the compiler use scalar loads.
template <class T> __device__ __forceinline__ T sld(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}

// Loads through pointers read from a descriptor: the compiler cannot tell that they point
// to global memory and would emit flat loads, which also count against the LDS wait
// counter; a pointer into the global address space gives plain global loads.
template <class T> __device__ __forceinline__ T gld(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}


// the descriptor of a case, in scalar registers (read as 8-byte words)
__device__ __forceinline__ CaseDev load_case(const CaseDev* p) {
    static_assert(sizeof(CaseDev) % 8 == 0 && alignof(CaseDev) == 8, "descriptor read as 8-byte words");
    constexpr int W = sizeof(CaseDev) / 8;
    const unsigned long long* w = reinterpret_cast<const unsigned long long*>(p);
    unsigned long long buf[W];
#pragma unroll
    for (int i = 0; i < W; ++i) buf[i] = sld(w + i);
    CaseDev c;
    __builtin_memcpy(&c, buf, sizeof(CaseDev));
    return c;
}

// member of a group that owns tile t (binary search over the tile prefix), uniform
__device__ __forceinline__ int find_member(const GroupArgs& ga, int t) {
    int lo = 0, hi = ga.nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sld(ga.pfx + mid) <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// element of lane slot `el` of a tile of member lo (the tile's EPB consecutive elements), and
// whether the slot holds one.  In a Gauss-Seidel coupling pass (ga.csel set) the tiles run over
// the member's elements of one colour instead, taken from its colour-sorted element list.
__device__ __forceinline__ int tile_elem(const GroupArgs& ga, const Geo& g, int lo, int tile, int epb, int el, int E,
                                         bool& act) {
    const int idx = (tile - sld(ga.pfx + lo)) * epb + el;
    if (!ga.csel) { act = idx < E; return idx; }
    act = idx < sld(ga.csel + 2 * lo + 1);
    return act ? ldo(g.corder, (unsigned)(sld(ga.csel + 2 * lo) + idx)) : 0;
}

// first tile of the range walked by this workgroup, the end of that range and the
// stride: XCD-contiguous ranges (workgroup b runs on XCD b % 8), or plain round robin
__device__ __forceinline__ void tile_range(int ntiles, int xcd_order, int& t0, int& tend, int& stride) {
    if (xcd_order) {
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per = gridDim.x >> 3;
        const int t8 = (ntiles + 7) >> 3;
        t0 = xcd * t8 + slot;
        tend = min((xcd + 1) * t8, ntiles);
        stride = per;
    } else {
        t0 = blockIdx.x;
        tend = ntiles;
        stride = gridDim.x;
    }
}

// LDS padding (in scalars of type T) of the solution-point arrays: per field, per group
// of four fields (one face of neighbour states) and per element.  Chosen with a model of
// the kernel's main access patterns so that the lanes of a wave (several elements, the
// four faces of each) spread over the 32 banks; W = doubles per scalar.
template <int P, int W> struct LPad { static constexpr int F = 0, FACE = 2, E = 1; };
template <> struct LPad<1, 1> { static constexpr int F = 1, FACE = 1, E = 0; };
template <> struct LPad<1, 2> { static constexpr int F = 0, FACE = 1, E = 2; };
template <> struct LPad<2, 1> { static constexpr int F = 1, FACE = 1, E = 0; };
template <> struct LPad<2, 2> { static constexpr int F = 1, FACE = 3, E = 2; };
template <> struct LPad<3, 1> { static constexpr int F = 0, FACE = 2, E = 1; };
template <> struct LPad<3, 2> { static constexpr int F = 0, FACE = 2, E = 3; };
template <> struct LPad<4, 1> { static constexpr int F = 1, FACE = 1, E = 4; };
template <> struct LPad<4, 2> { static constexpr int F = 0, FACE = 1, E = 5; };

// Metric terms one lane uses: those of its solution point, of its flux point and of the
// neighbour across that face (the neighbour's constant metrics, used when it is affine).
// They are requested when a tile starts, next to the states, so that a tile waits on memory
// twice (the connectivity, then all that depends on it) rather than once per stage.  Lanes
// past Np (NF) read a valid point they do not use, which keeps the loads in one sequence.
struct LaneGeo {
    double xix, xiy, etx, ety, ij, ug, vg;   // solution point lt % Np
    double nx, ny, sc, cc, fug, fvg;         // flux point lt % NF
    double mxix, mxiy, metx, mety;           // neighbour across face (lt % NF) / n
    int nb, nf, k2, aff;                     // that neighbour, its face, the point index there
};

template <int P, bool VISC, bool MOV>
__device__ __forceinline__ void lane_geo_load(const Geo& g, int E, int e, int lt, int pk, LaneGeo& lg) {
    constexpr int n = P + 1, Np = n * n, NF = 4 * n;
    const unsigned EN = (unsigned)E * Np, FE = (unsigned)E * NF;
    const int ls = lt % Np, lf = lt % NF, f = lf / n, k = lf % n;
    const unsigned id = (unsigned)e * Np + ls, sid = (unsigned)e * NF + lf;
    lg.xix = ldo(g.sp + G_XIX * EN, id); lg.xiy = ldo(g.sp + G_XIY * EN, id);
    lg.etx = ldo(g.sp + G_ETX * EN, id); lg.ety = ldo(g.sp + G_ETY * EN, id);
    lg.ij = ldo(g.sp + G_IJ * EN, id);
    lg.ug = MOV ? ldo(g.sp + G_UG * EN, id) : 0.0;
    lg.vg = MOV ? ldo(g.sp + G_VG * EN, id) : 0.0;
    lg.nx = ldo(g.fp + F_NX * FE, sid); lg.ny = ldo(g.fp + F_NY * FE, sid); lg.sc = ldo(g.fp + F_SC * FE, sid);
    lg.cc = VISC ? ldo(g.fp + F_CC * FE, sid) : 0.0;
    lg.fug = MOV ? ldo(g.fp + F_UG * FE, sid) : 0.0;
    lg.fvg = MOV ? ldo(g.fp + F_VG * FE, sid) : 0.0;
    lg.nb = pk >> 3; lg.nf = (pk >> 1) & 3; lg.k2 = (pk & 1) ? n - 1 - k : k;
    lg.aff = 0; lg.mxix = lg.mxiy = lg.metx = lg.mety = 0.0;
    if (VISC) {
        const unsigned gid = (unsigned)lg.nb * Np;
        lg.aff = ldo(g.aff, (unsigned)lg.nb);
        lg.mxix = ldo(g.sp + G_XIX * EN, gid); lg.mxiy = ldo(g.sp + G_XIY * EN, gid);
        lg.metx = ldo(g.sp + G_ETX * EN, gid); lg.mety = ldo(g.sp + G_ETY * EN, gid);
    }
}

template <int P, bool VISC, bool MOV, int MODE, int K, int LANES, bool BC, bool TAN = false>
__global__ void __launch_bounds__((Shape<P, LANES>::threads))
k_fused(GroupArgs ga, KArgs a, OpTab op) {
    // TAN: only the tangent is wanted from the point fluxes on (a JVP without R, the Newton
    // operator); stages 4-6 then keep the tangent fluxes in LDS as plain doubles
    static_assert(!TAN || ((MODE == MODE_JVP || MODE == MODE_AOP) && K == 1), "tangent-only stages need one tangent");
    using T = typename ModeT<MODE, K>::T;
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT;
    constexpr int EPB = Shape<P, LANES>::EPB;
    constexpr int NW = MOV ? 12 : 8;
    static_assert(NW <= 16, "flux fields alias the neighbour staging area");
    using PD = LPad<P, Store<T>::W>;
    constexpr int FS = Np + PD::F;               // field stride
    constexpr int FACE = 4 * FS + PD::FACE;      // stride of a group of 4 fields
    constexpr int ESN = 4 * FACE + PD::E;        // element stride of the neighbour / flux area
    constexpr int ESQ = 4 * FS + PD::E;
    constexpr int NG = VISC ? 6 : 1;
    constexpr int ESG = NG * FS + PD::E;
    constexpr int ESF = 4 * NF + 1, ND = VISC ? 3 : 1, ESD = ND * NF + 1, ESS = 3 * NF + 1;
    __shared__ T s_q[EPB * ESQ];       // own state [el][var][point]
    __shared__ T s_n[EPB * ESN];       // neighbour states [el][face][var][point]; later f, g (, q^c)
    __shared__ T s_g[EPB * ESG];       // own uncorrected gradient [el][6][point]
    __shared__ T s_F[EPB * ESF];       // F^num, then F^num - F^loc  [el][var][flux point]
    __shared__ T s_dq[EPB * ESD];      // q^com - q^- of (u, v, T)  [el][3][flux point]
    __shared__ double s_S[EPB * ESS];  // element-oriented S, S . v_g  [el][3][flux point]
    auto QI = [](int el, int v, int sp) { return el * ESQ + v * FS + sp; };
    auto NI = [](int el, int fld, int sp) { return el * ESN + (fld >> 2) * FACE + (fld & 3) * FS + sp; };
    auto GI = [](int el, int c, int sp) { return el * ESG + c * FS + sp; };
    auto FI = [](int el, int v, int fp) { return el * ESF + v * NF + fp; };
    auto DI = [](int el, int c, int fp) { return el * ESD + c * NF + fp; };
    auto SI = [](int el, int c, int fp) { return el * ESS + c * NF + fp; };
    // tangent-only fluxes: each element's areas of s_n and s_F read as doubles
    constexpr int ESND = ESN * Store<T>::W, ESFD = ESF * Store<T>::W;
    auto FD = [](int el, int v, int fp) { return el * ESFD + v * NF + fp; };
    double* s_nd = reinterpret_cast<double*>(s_n);
    double* s_Fd = reinterpret_cast<double*>(s_F);
    __shared__ double s_D[n * n];       // operator tables (lane-dependent indexing goes to LDS)
    __shared__ double s_lam[2][n], s_gam[2][n], s_dlam[2][n];

    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) s_D[t] = op.D[t];
    if (threadIdx.x < n) {
        s_lam[0][threadIdx.x] = op.lamL[threadIdx.x]; s_lam[1][threadIdx.x] = op.lamR[threadIdx.x];
        s_gam[0][threadIdx.x] = op.gamL[threadIdx.x]; s_gam[1][threadIdx.x] = op.gamR[threadIdx.x];
        s_dlam[0][threadIdx.x] = op.dlamL[threadIdx.x]; s_dlam[1][threadIdx.x] = op.dlamR[threadIdx.x];
    }
    const int i = lt % n, j = lt / n;
    int tile, tend, tstride;
    tile_range(ga.ntiles, ga.xcd, tile, tend, tstride);
    for (; tile < tend; tile += tstride) {
        // ---- the tile's case (uniform across the workgroup)
        const int lo = find_member(ga, tile);
        const int cid = sld(ga.ids + lo);
        if (a.flags && rfl(a.flags[cid * GI_STRIDE + a.flag])) continue;
        const CaseDev cd = load_case(ga.cases + cid);
        const PhysConst& pc = cd.pc;
        const Geo g = cd.g;
        const int E = cd.E;
        const int e = (tile - sld(ga.pfx + lo)) * EPB + el;
        const bool act = e < E;
        const unsigned EN = (unsigned)E * Np;   // state arrays hold < 2^31 entries (checked at creation)
        const double* q = a.q + cd.off;
        const double* v = a.v ? a.v + cd.off : nullptr;
        __syncthreads();   // the previous tile's readers of s_n / s_F are done
        // ---- stage 1: own state and neighbour states into LDS; the lane's metric terms
        LaneGeo lg;
        int bck = 0;   // boundary kind of the lane's face (0: interior)
        if (act) {
            int pk4[4];
#pragma unroll
            for (int ff = 0; ff < 4; ++ff) pk4[ff] = ldo(g.nbr, (unsigned)(e * 4 + ff));
            if (BC && g.bc) bck = (gld(g.bc + e) >> (2 * ((lt % NF) / n))) & 3;
            const int ls = lt % Np;
            const unsigned id = (unsigned)e * Np + ls;
            T qo[4];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) qo[vv] = Seed<T>::load(a, q + vv * EN, v ? v + vv * EN : nullptr, id, vv * Np + ls);
            // the lane's own face entry is loaded on its own: selecting it from pk4 by the lane's
            // face makes the compiler index a stack copy of pk4 (scratch memory)
            lane_geo_load<P, VISC, MOV>(g, E, e, lt, ldo(g.nbr, (unsigned)(e * 4 + (lt % NF) / n)), lg);
            if (lt < Np) {
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) s_q[QI(el, vv, lt)] = qo[vv];
#pragma unroll
                for (int ff = 0; ff < 4; ++ff) {
                    const int nb = pk4[ff] >> 3;
                    const unsigned nid = (unsigned)nb * Np + lt;
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv)
                        s_n[NI(el, ff * 4 + vv, lt)] = NbLoad<T>::load(a, q + vv * EN, v ? v + vv * EN : nullptr, nid, vv * Np + lt, nb == e);
                }
            }
        }
        __syncthreads();
        // ---- stage 2: own uncorrected gradient (kept in LDS only)
        if (VISC && act && lt < Np) {
            const double xix = lg.xix, xiy = lg.xiy, etx = lg.etx, ety = lg.ety;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T dxi = cst<T>(0.0), deta = cst<T>(0.0);
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    dxi = dxi + s_D[i * n + b] * s_q[QI(el, c + 1, b + n * j)];
                    deta = deta + s_D[j * n + b] * s_q[QI(el, c + 1, i + n * b)];
                }
                s_g[GI(el, 2 * c, lt)] = xix * dxi + etx * deta;
                s_g[GI(el, 2 * c + 1, lt)] = xiy * dxi + ety * deta;
            }
        }
        __syncthreads();
        // ---- stage 3: own and neighbour traces, common flux at the flux points.  The
        // neighbour's gradient trace on an affine neighbour follows from its traces: the
        // face-normal derivative from its line of states with l'(+-1), the tangential one
        // from the traces along the face; the trace samples wait in the (still unused) s_F.
        const int f = (lt % NF) / n, k = lt % n;
        const int nb = lg.nb, nf = lg.nf, k2 = lg.k2;
        T qm[4], qp[4];
        if (act && lt < NF) {
            const double* lam = s_lam[f & 1];
            const double* lamn = s_lam[nf & 1];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                T am = cst<T>(0.0), ap = cst<T>(0.0);
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    am = am + lam[b] * s_q[QI(el, vv, line_pt(n, f, k, b))];
                    ap = ap + lamn[b] * s_n[NI(el, f * 4 + vv, line_pt(n, nf, k2, b))];
                }
                qm[vv] = am;
                qp[vv] = ap;
            }
            if (BC && bck) fr_bc_state<T>(bck, g.qinf, qm, lg.nx, lg.ny, lg.fug, lg.fvg, qp);
            if constexpr (MODE == MODE_PREP) {
                double* fpk = a.fpack + cd.fpoff + (size_t)e * NF + lt;
                const size_t fs = (size_t)E * NF;
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) { fpk[vv * fs] = qm[vv]; fpk[(4 + vv) * fs] = qp[vv]; }
            }
            if (VISC) {
#pragma unroll
                for (int c = 0; c < 3; ++c) s_F[FI(el, c, f * n + k2)] = qp[c + 1];
            }
        }
        if (VISC) __syncthreads();
        T fsc[4];   // S F^num, kept in registers until stage 5 writes F^num - F^loc
        if (act && lt < NF) {
            const double* lam = s_lam[f & 1];
            const double* lamn = s_lam[nf & 1];
            const double nx = lg.nx, ny = lg.ny, sc = lg.sc, ugf = lg.fug, vgf = lg.fvg;
            T fn[4], dq[4];
            fr_common_inviscid<T>(pc, qm, qp, nx, ny, ugf, vgf, fn, dq);
            if (VISC) {
                T gm[6], gp[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    T am = cst<T>(0.0);
#pragma unroll
                    for (int b = 0; b < n; ++b) am = am + lam[b] * s_g[GI(el, c, line_pt(n, f, k, b))];
                    gm[c] = am;
                    gp[c] = cst<T>(0.0);
                }
                if (lg.aff) {
                    // constant metrics: the trace of the chain-rule gradient is the chain rule
                    // applied to the traced reference derivatives
                    const double xix = lg.mxix, xiy = lg.mxiy, etx = lg.metx, ety = lg.mety;
                    const double* dlamn = s_dlam[nf & 1];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        T dnor = cst<T>(0.0), dtan = cst<T>(0.0);
#pragma unroll
                        for (int m = 0; m < n; ++m) {
                            dnor = dnor + dlamn[m] * s_n[NI(el, f * 4 + c + 1, line_pt(n, nf, k2, m))];
                            dtan = dtan + s_D[k2 * n + m] * s_F[FI(el, c, f * n + m)];
                        }
                        const T dxi = nf < 2 ? dnor : dtan, deta = nf < 2 ? dtan : dnor;
                        gp[2 * c] = xix * dxi + etx * deta;
                        gp[2 * c + 1] = xiy * dxi + ety * deta;
                    }
                } else {
                    // neighbour's uncorrected gradient along the line through its face point, traced
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        const int sp = line_pt(n, nf, k2, b);
                        const int is = sp % n, js = sp / n;
                        const unsigned gid = (unsigned)nb * Np + sp;
                        const double xix = ldo(g.sp + G_XIX * EN, gid), xiy = ldo(g.sp + G_XIY * EN, gid);
                        const double etx = ldo(g.sp + G_ETX * EN, gid), ety = ldo(g.sp + G_ETY * EN, gid);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            T dxi = cst<T>(0.0), deta = cst<T>(0.0);
#pragma unroll
                            for (int m = 0; m < n; ++m) {
                                dxi = dxi + s_D[is * n + m] * s_n[NI(el, f * 4 + c + 1, m + n * js)];
                                deta = deta + s_D[js * n + m] * s_n[NI(el, f * 4 + c + 1, is + n * m)];
                            }
                            gp[2 * c] = gp[2 * c] + lamn[b] * (xix * dxi + etx * deta);
                            gp[2 * c + 1] = gp[2 * c + 1] + lamn[b] * (xiy * dxi + ety * deta);
                        }
                    }
                }
                if (BC && bck) fr_bc_grad<T>(bck, gm, nx, ny, gp);
                if constexpr (MODE == MODE_PREP) {
                    double* fpk = a.fpack + cd.fpoff + (size_t)e * NF + lt;
                    const size_t fs = (size_t)E * NF;
#pragma unroll
                    for (int c = 0; c < 6; ++c) fpk[(8 + c) * fs] = gm[c] + gp[c];   // the common flux needs the sum only
                }
                // q^com velocity = average of the two traces = q^- + dq/2
                const T qcu = am_avg<T>(&s_q[QI(el, 1, 0)], lam, f, k, dq[1], n);
                const T qcv = am_avg<T>(&s_q[QI(el, 2, 0)], lam, f, k, dq[2], n);
                T dqh[3];
                fr_common_viscous<T>(pc, dq, qcu, qcv, gm, gp, nx, ny, lg.cc, fn, dqh);
#pragma unroll
                for (int c = 0; c < 3; ++c) s_dq[DI(el, c, lt)] = dqh[c];
            }
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) fsc[vv] = sc * fn[vv];
            s_S[SI(el, 0, lt)] = sc * nx;                                  // element-oriented S
            s_S[SI(el, 1, lt)] = sc * ny;
            s_S[SI(el, 2, lt)] = MOV ? sc * (ugf * nx + vgf * ny) : 0.0;   // S . v_g
        }
        __syncthreads();

        // ---- stage 4: corrected gradient, pointwise fluxes (into the staging area)
        auto WI = [&](int fld, int sp) { return NI(el, fld, sp); };   // fluxes alias the neighbour area
        auto WD = [&](int fld, int sp) { return el * ESND + (fld >> 2) * FACE + (fld & 3) * FS + sp; };
        T qs[4];
        if (act && lt < Np) {
            const double ij = lg.ij;
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) qs[vv] = s_q[QI(el, vv, lt)];
            T gu[2], gv[2], gT[2];
            if (VISC) {
#pragma unroll
                for (int d = 0; d < 2; ++d) { gu[d] = s_g[GI(el, d, lt)]; gv[d] = s_g[GI(el, 2 + d, lt)]; gT[d] = s_g[GI(el, 4 + d, lt)]; }
                const int fp0 = 0 * n + j, fp1 = 1 * n + j, fp2 = 2 * n + i, fp3 = 3 * n + i;
                const double gL_i = s_gam[0][i], gR_i = s_gam[1][i], gL_j = s_gam[0][j], gR_j = s_gam[1][j];
                T* gr[3] = {gu, gv, gT};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T cx = (s_S[SI(el, 0, fp0)] * gL_i) * s_dq[DI(el, c, fp0)] + (s_S[SI(el, 0, fp1)] * gR_i) * s_dq[DI(el, c, fp1)]
                         + (s_S[SI(el, 0, fp2)] * gL_j) * s_dq[DI(el, c, fp2)] + (s_S[SI(el, 0, fp3)] * gR_j) * s_dq[DI(el, c, fp3)];
                    T cy = (s_S[SI(el, 1, fp0)] * gL_i) * s_dq[DI(el, c, fp0)] + (s_S[SI(el, 1, fp1)] * gR_i) * s_dq[DI(el, c, fp1)]
                         + (s_S[SI(el, 1, fp2)] * gL_j) * s_dq[DI(el, c, fp2)] + (s_S[SI(el, 1, fp3)] * gR_j) * s_dq[DI(el, c, fp3)];
                    gr[c][0] = gr[c][0] + ij * cx;
                    gr[c][1] = gr[c][1] + ij * cy;
                }
            }
            if constexpr (MODE == MODE_PREP) {
                double* spk = a.spack + cd.spoff + (size_t)e * Np + lt;
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) spk[(size_t)vv * EN] = qs[vv];
                if (VISC) {
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        spk[(size_t)(4 + d) * EN] = gu[d];
                        spk[(size_t)(6 + d) * EN] = gv[d];
                        spk[(size_t)(8 + d) * EN] = gT[d];
                    }
                }
            }
            T fl[4], gl[4], qc[4];
            fr_point_flux<T, VISC>(pc, qs, gu, gv, gT, fl, gl, qc);
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                if constexpr (TAN) {
                    s_nd[WD(vv, lt)] = fl[vv].d[0];
                    s_nd[WD(4 + vv, lt)] = gl[vv].d[0];
                    if (MOV) s_nd[WD(8 + vv, lt)] = qc[vv].d[0];
                } else {
                    s_n[WI(vv, lt)] = fl[vv];
                    s_n[WI(4 + vv, lt)] = gl[vv];
                    if (MOV) s_n[WI(8 + vv, lt)] = qc[vv];
                }
            }
        }
        __syncthreads();

        // ---- stage 5: F^num - F^loc, F^loc = S.(Pi f, Pi g) - (S.v_g) Pi q^c
        if (act && lt < NF) {
            const double* lam = s_lam[f & 1];
            const double Sx = s_S[SI(el, 0, lt)], Sy = s_S[SI(el, 1, lt)], Svg = s_S[SI(el, 2, lt)];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                if constexpr (TAN) {
                    double acc = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        const int sp = line_pt(n, f, k, b);
                        double w = Sx * s_nd[WD(vv, sp)] + Sy * s_nd[WD(4 + vv, sp)];
                        if (MOV) w = w - Svg * s_nd[WD(8 + vv, sp)];
                        acc = acc + lam[b] * w;
                    }
                    s_Fd[FD(el, vv, lt)] = fsc[vv].d[0] - acc;
                } else {
                    T acc = cst<T>(0.0);
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        const int sp = line_pt(n, f, k, b);
                        T w = Sx * s_n[WI(vv, sp)] + Sy * s_n[WI(4 + vv, sp)];
                        if (MOV) w = w - Svg * s_n[WI(8 + vv, sp)];
                        acc = acc + lam[b] * w;
                    }
                    s_F[FI(el, vv, lt)] = fsc[vv] - acc;
                }
            }
        }
        __syncthreads();

        // ---- stage 6: divergence + moving-mesh terms + Radau lift, one variable at a time
        if (act && lt < Np) {
            const unsigned id = (unsigned)e * Np + lt;
            const double geo[NGSP] = {lg.xix, lg.xiy, lg.etx, lg.ety, lg.ij, lg.ug, lg.vg};
            const double axi = MOV ? geo[G_UG] * geo[G_XIX] + geo[G_VG] * geo[G_XIY] : 0.0;
            const double aet = MOV ? geo[G_UG] * geo[G_ETX] + geo[G_VG] * geo[G_ETY] : 0.0;
            double ct = a.c_time, idt = a.inv_dtau;
            if (a.cstep) { ct = rfl(a.cstep[cid].ct); idt = rfl(a.cstep[cid].idt); }
            double tt[4] = {0.0, 0.0, 0.0, 0.0};   // time terms (Newton operator)
            if constexpr (MODE == MODE_AOP) {
                double qv[4], x[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) { qv[vv] = qs[vv].v; x[vv] = qs[vv].d[0]; }
                fr_time_apply<double, double>(pc, qv, geo[G_UG], geo[G_VG], idt, ct, x, tt);
            }
            double* out = a.out + ((MODE == MODE_BLK) ? cd.boff : cd.off);
#pragma unroll 1
            for (int vv = 0; vv < 4; ++vv) {
                if constexpr (TAN) {
                    double dfx = 0.0, dfe = 0.0, dgx = 0.0, dge = 0.0, dqx = 0.0, dqe = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        const double Dx = s_D[i * n + b], De = s_D[j * n + b];
                        dfx = dfx + Dx * s_nd[WD(vv, b + n * j)];
                        dgx = dgx + Dx * s_nd[WD(4 + vv, b + n * j)];
                        dfe = dfe + De * s_nd[WD(vv, i + n * b)];
                        dge = dge + De * s_nd[WD(4 + vv, i + n * b)];
                        if (MOV) {
                            dqx = dqx + Dx * s_nd[WD(8 + vv, b + n * j)];
                            dqe = dqe + De * s_nd[WD(8 + vv, i + n * b)];
                        }
                    }
                    double vol = geo[G_XIX] * dfx + geo[G_ETX] * dfe + geo[G_XIY] * dgx + geo[G_ETY] * dge;
                    if (MOV) vol = vol - axi * dqx - aet * dqe;
                    const double cor = s_gam[0][i] * s_Fd[FD(el, vv, 0 * n + j)] + s_gam[1][i] * s_Fd[FD(el, vv, 1 * n + j)]
                                     + s_gam[0][j] * s_Fd[FD(el, vv, 2 * n + i)] + s_gam[1][j] * s_Fd[FD(el, vv, 3 * n + i)];
                    const double R = -(vol + geo[G_IJ] * cor);
                    if constexpr (MODE == MODE_AOP) {
                        const double ttv = (vv == 0) ? tt[0] : (vv == 1) ? tt[1] : (vv == 2) ? tt[2] : tt[3];
                        out[vv * EN + id] = ttv - R;
                    } else {
                        out[vv * EN + id] = R;
                    }
                    continue;
                }
                T dfx = cst<T>(0.0), dfe = cst<T>(0.0), dgx = cst<T>(0.0), dge = cst<T>(0.0);
                T dqx = cst<T>(0.0), dqe = cst<T>(0.0);
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    const double Dx = s_D[i * n + b], De = s_D[j * n + b];
                    dfx = dfx + Dx * s_n[WI(vv, b + n * j)];
                    dgx = dgx + Dx * s_n[WI(4 + vv, b + n * j)];
                    dfe = dfe + De * s_n[WI(vv, i + n * b)];
                    dge = dge + De * s_n[WI(4 + vv, i + n * b)];
                    if (MOV) {
                        dqx = dqx + Dx * s_n[WI(8 + vv, b + n * j)];
                        dqe = dqe + De * s_n[WI(8 + vv, i + n * b)];
                    }
                }
                T vol = geo[G_XIX] * dfx + geo[G_ETX] * dfe + geo[G_XIY] * dgx + geo[G_ETY] * dge;
                if (MOV) vol = vol - axi * dqx - aet * dqe;
                T cor = s_gam[0][i] * s_F[FI(el, vv, 0 * n + j)] + s_gam[1][i] * s_F[FI(el, vv, 1 * n + j)]
                      + s_gam[0][j] * s_F[FI(el, vv, 2 * n + i)] + s_gam[1][j] * s_F[FI(el, vv, 3 * n + i)];
                const T R = -(vol + geo[G_IJ] * cor);
                if constexpr (MODE == MODE_R || MODE == MODE_PREP) {
                    out[vv * EN + id] = val(R);
                } else if constexpr (MODE == MODE_JVP) {
                    out[vv * EN + id] = R.d[0];
                    if (a.out2) a.out2[cd.off + vv * EN + id] = R.v;
                } else if constexpr (MODE == MODE_AOP) {
                    const double ttv = (vv == 0) ? tt[0] : (vv == 1) ? tt[1] : (vv == 2) ? tt[2] : tt[3];
                    out[vv * EN + id] = ttv - R.d[0];
                } else {
                    // block columns seed0..seed0+K-1 of element e, column-major [E][nb][nb]
                    constexpr int nbk = 4 * Np;
                    double* blk = out + (size_t)e * nbk * nbk;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const int col = a.seed0 + k;
                        if (col < nbk) blk[(size_t)col * nbk + vv * Np + lt] = -R.d[k];
                    }
                }
            }
            if constexpr (MODE == MODE_BLK) {
                // time terms on the diagonal point block of the seeded columns
                constexpr int nbk = 4 * Np;
                double* blk = out + (size_t)e * nbk * nbk;
                double qv[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) qv[vv] = qs[vv].v;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const int col = a.seed0 + k;
                    if (col < nbk && col % Np == lt) {
                        double x[4] = {0.0, 0.0, 0.0, 0.0}, t4[4];
                        x[col / Np] = 1.0;
                        fr_time_apply<double, double>(pc, qv, geo[G_UG], geo[G_VG], idt, ct, x, t4);
#pragma unroll
                        for (int vv = 0; vv < 4; ++vv) blk[(size_t)col * nbk + vv * Np + lt] += t4[vv];
                    }
                }
            }
        }
    }
}

// The residual (and in MODE_PREP the linearisation packs) of static groups whose elements
// are all affine.  Same stages as k_fused, with what constant metrics allow:
//  * neighbour states are not staged in LDS: each face lane reads the neighbour's line
//    through its face point and forms the neighbour trace q+ and, for the gradient trace,
//    the face-normal derivative sum_b l_b'(+-1) q_b in registers; the tangential derivative
//    is the 1-D derivative of the neighbour traces along the face, exchanged through the
//    (not yet used) F^num area; the neighbour's gradient trace is then the chain rule with
//    its constant metrics;
//  * point fluxes are kept in contravariant form, F~ = xi_x f + xi_y g, G~ = eta_x f + eta_y g,
//    so the divergence is dF~/dxi + dG~/deta and S.(Pi f, Pi g) on a xi (eta) face is |J| Pi F~
//    (|J| Pi G~): half the LDS reads of the last two stages.
// Equal to k_fused's values up to rounding.
//  * TAN: only the tangent is wanted from the point fluxes on (a JVP without R, the Newton
//    operator): stages 4-6 keep the tangent fluxes in LDS as plain doubles, and the value
//    parts that only R would need are not computed.
template <int P, bool VISC, int MODE, int LANES, bool TAN = false>
__global__ void __launch_bounds__((Shape<P, LANES>::threads))
k_fused_aff(GroupArgs ga, KArgs a, OpTab op) {
    static_assert(MODE == MODE_R || MODE == MODE_PREP || MODE == MODE_JVP || MODE == MODE_AOP,
                  "residual, packs, JVP or Newton operator");
    static_assert(!TAN || MODE == MODE_JVP || MODE == MODE_AOP, "tangent-only stages need a tangent");
    using T = typename ModeT<MODE, 1>::T;
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT;
    constexpr int EPB = Shape<P, LANES>::EPB;
    using PD = LPad<P, Store<T>::W>;
    constexpr int FS = Np + PD::F;
    constexpr int ESQ = 4 * FS + PD::E;
    constexpr int ESW = 8 * FS + PD::E;      // own gradient (6 fields); later F~ of the 4 equations, then G~
    constexpr int ESF = 4 * NF + 1, ND = VISC ? 3 : 1, ESD = ND * NF + 1;
    // tangent-only fluxes: each element's areas of s_w and s_F read as doubles
    constexpr int ESWD = ESW * Store<T>::W, ESFD = ESF * Store<T>::W;
    // an element whose lanes span two wavefronts: the gradient reads of stage 4 and its
    // (differently placed) tangent flux writes are then separated by a barrier
    constexpr bool SPLIT = TAN && (64 % NT != 0) && EPB * NT > 64;
    __shared__ T s_q[EPB * ESQ];       // own state [el][var][point]
    __shared__ T s_w[EPB * ESW];       // own uncorrected gradient [el][6][point]; then F~, G~ [el][8][point]
    __shared__ T s_F[EPB * ESF];       // neighbour traces of (u, v, T) by neighbour point; then F^num - F^loc
    __shared__ T s_dq[EPB * ESD];      // q^com - q^- of (u, v, T)
    auto QI = [](int el, int v, int sp) { return el * ESQ + v * FS + sp; };
    auto WI = [](int el, int fld, int sp) { return el * ESW + fld * FS + sp; };
    // the gradient shares the flux area: in stage 4 a lane reads its own point's gradient
    // before it writes its own point's fluxes, and no lane reads another point's gradient there
    auto GI = [](int el, int c, int sp) { return el * ESW + c * FS + sp; };
    auto FI = [](int el, int v, int fp) { return el * ESF + v * NF + fp; };
    auto DI = [](int el, int c, int fp) { return el * ESD + c * NF + fp; };
    auto WD = [](int el, int fld, int sp) { return el * ESWD + fld * FS + sp; };
    auto FD = [](int el, int v, int fp) { return el * ESFD + v * NF + fp; };
    double* s_wd = reinterpret_cast<double*>(s_w);
    double* s_Fd = reinterpret_cast<double*>(s_F);
    __shared__ double s_D[n * n];
    __shared__ double s_lam[2][n], s_gam[2][n], s_dlam[2][n];

    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) s_D[t] = op.D[t];
    if (threadIdx.x < n) {
        s_lam[0][threadIdx.x] = op.lamL[threadIdx.x]; s_lam[1][threadIdx.x] = op.lamR[threadIdx.x];
        s_gam[0][threadIdx.x] = op.gamL[threadIdx.x]; s_gam[1][threadIdx.x] = op.gamR[threadIdx.x];
        s_dlam[0][threadIdx.x] = op.dlamL[threadIdx.x]; s_dlam[1][threadIdx.x] = op.dlamR[threadIdx.x];
    }
    const int i = lt % n, j = lt / n;
    const int f = (lt % NF) / n, k = lt % n;
    int tile, tend, tstride;
    tile_range(ga.ntiles, ga.xcd, tile, tend, tstride);
    // connectivity of the next tile of this workgroup, requested one tile ahead (persistent grids)
    int pkn = 0;
    int pkn_tile = -1;
    for (; tile < tend; tile += tstride) {
        const int lo = find_member(ga, tile);
        const int cid = sld(ga.ids + lo);
        if (a.flags && rfl(a.flags[cid * GI_STRIDE + a.flag])) continue;
        const CaseDev cd = load_case(ga.cases + cid);
        const PhysConst& pc = cd.pc;
        const Geo g = cd.g;
        const int E = cd.E;
        const int e = (tile - sld(ga.pfx + lo)) * EPB + el;
        const bool act = e < E;
        const unsigned EN = (unsigned)E * Np;
        const double* q = a.q + cd.off;
        const double* v = a.v ? a.v + cd.off : nullptr;
        __syncthreads();   // the previous tile's readers of LDS are done
        // ---- stage 1: own state into LDS; the lane's metric terms; the neighbour's line
        // through this face point: trace and face-normal derivative
        LaneGeo lg;
        T qp[4], dnor[3];
        const bool pre = pkn_tile == tile;
        if (act) {
            const int pk = pre ? pkn : ldo(g.nbr, (unsigned)(e * 4 + f));
            const int ls = lt % Np;
            const unsigned id = (unsigned)e * Np + ls;
            T qo[4];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) qo[vv] = Seed<T>::load(a, q + vv * EN, v ? v + vv * EN : nullptr, id, vv * Np + ls);
            lane_geo_load<P, VISC, false>(g, E, e, lt, pk, lg);
            if (lt < NF) {
                const unsigned nbase = (unsigned)lg.nb * Np;
                T ln[4][n];
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    const int sp = line_pt(n, lg.nf, lg.k2, b);
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv)
                        ln[vv][b] = NbLoad<T>::load(a, q + vv * EN, v ? v + vv * EN : nullptr, nbase + sp, vv * Np + sp, lg.nb == e);
                }
                const double* lamn = s_lam[lg.nf & 1];
                const double* dlamn = s_dlam[lg.nf & 1];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    T acc = cst<T>(0.0);
#pragma unroll
                    for (int b = 0; b < n; ++b) acc = acc + lamn[b] * ln[vv][b];
                    qp[vv] = acc;
                }
                if (VISC) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        T acc = cst<T>(0.0);
#pragma unroll
                        for (int b = 0; b < n; ++b) acc = acc + dlamn[b] * ln[c + 1][b];
                        dnor[c] = acc;
                        s_F[FI(el, c, f * n + lg.k2)] = qp[c + 1];
                    }
                }
            }
            if (lt < Np) {
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) s_q[QI(el, vv, lt)] = qo[vv];
            }
        }
        {
            const int tn = tile + tstride;
            const int pfx_hi = lo + 1 < ga.nmem ? sld(ga.pfx + lo + 1) : ga.ntiles;
            pkn_tile = (tn < tend && tn < pfx_hi) ? tn : -1;
            const int en = (tn - sld(ga.pfx + lo)) * EPB + el;
            if (pkn_tile >= 0 && en < E) {
                pkn = ldo(g.nbr, (unsigned)(en * 4 + f));
            }
        }
        __syncthreads();
        // ---- stage 2: own uncorrected gradient
        if (VISC && act && lt < Np) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T dxi = cst<T>(0.0), deta = cst<T>(0.0);
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    dxi = dxi + s_D[i * n + b] * s_q[QI(el, c + 1, b + n * j)];
                    deta = deta + s_D[j * n + b] * s_q[QI(el, c + 1, i + n * b)];
                }
                s_w[GI(el, 2 * c, lt)] = lg.xix * dxi + lg.etx * deta;
                s_w[GI(el, 2 * c + 1, lt)] = lg.xiy * dxi + lg.ety * deta;
            }
        }
        __syncthreads();
        // ---- stage 3: own traces, common flux at the flux points
        T fsc[4];
        if (act && lt < NF) {
            const double* lam = s_lam[f & 1];
            const double nx = lg.nx, ny = lg.ny, sc = lg.sc;
            T qm[4];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                T acc = cst<T>(0.0);
#pragma unroll
                for (int b = 0; b < n; ++b) acc = acc + lam[b] * s_q[QI(el, vv, line_pt(n, f, k, b))];
                qm[vv] = acc;
            }
            if constexpr (MODE == MODE_PREP) {
                double* fpk = a.fpack + cd.fpoff + (size_t)e * NF + lt;
                const size_t fs = (size_t)E * NF;
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) { fpk[vv * fs] = qm[vv]; fpk[(4 + vv) * fs] = qp[vv]; }
            }
            T fn[4], dq[4];
            fr_common_inviscid<T>(pc, qm, qp, nx, ny, 0.0, 0.0, fn, dq);
            if (VISC) {
                T gm[6], gp[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    T acc = cst<T>(0.0);
#pragma unroll
                    for (int b = 0; b < n; ++b) acc = acc + lam[b] * s_w[GI(el, c, line_pt(n, f, k, b))];
                    gm[c] = acc;
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T dtan = cst<T>(0.0);
#pragma unroll
                    for (int m = 0; m < n; ++m) dtan = dtan + s_D[lg.k2 * n + m] * s_F[FI(el, c, f * n + m)];
                    const T dxi = lg.nf < 2 ? dnor[c] : dtan, deta = lg.nf < 2 ? dtan : dnor[c];
                    gp[2 * c] = lg.mxix * dxi + lg.metx * deta;
                    gp[2 * c + 1] = lg.mxiy * dxi + lg.mety * deta;
                }
                if constexpr (MODE == MODE_PREP) {
                    double* fpk = a.fpack + cd.fpoff + (size_t)e * NF + lt;
                    const size_t fs = (size_t)E * NF;
#pragma unroll
                    for (int c = 0; c < 6; ++c) fpk[(8 + c) * fs] = gm[c] + gp[c];   // the common flux needs the sum only
                }
                const T qcu = qm[1] + 0.5 * dq[1];
                const T qcv = qm[2] + 0.5 * dq[2];
                T dqh[3];
                fr_common_viscous<T>(pc, dq, qcu, qcv, gm, gp, nx, ny, lg.cc, fn, dqh);
#pragma unroll
                for (int c = 0; c < 3; ++c) s_dq[DI(el, c, lt)] = dqh[c];
            }
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) fsc[vv] = sc * fn[vv];
        }
        __syncthreads();
        // ---- stage 4: corrected gradient, point fluxes in contravariant form
        const bool s4 = act && lt < Np;
        T qs[4], gu[2], gv[2], gT[2];
        if (s4) {
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) qs[vv] = s_q[QI(el, vv, lt)];
            if (VISC) {
#pragma unroll
                for (int d = 0; d < 2; ++d) { gu[d] = s_w[GI(el, d, lt)]; gv[d] = s_w[GI(el, 2 + d, lt)]; gT[d] = s_w[GI(el, 4 + d, lt)]; }
            }
        }
        if constexpr (SPLIT) __syncthreads();
        if (s4) {
            if (VISC) {
                // lift of q^com - q^- through the Radau slopes; on an affine element the face
                // vectors are |J| grad(xi) (faces 0, 1) and |J| grad(eta) (faces 2, 3), and |J| / |J| = 1
                const int fp0 = 0 * n + j, fp1 = 1 * n + j, fp2 = 2 * n + i, fp3 = 3 * n + i;
                const double gL_i = s_gam[0][i], gR_i = s_gam[1][i], gL_j = s_gam[0][j], gR_j = s_gam[1][j];
                T* gr[3] = {gu, gv, gT};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T lx = gL_i * s_dq[DI(el, c, fp0)] + gR_i * s_dq[DI(el, c, fp1)];
                    const T le = gL_j * s_dq[DI(el, c, fp2)] + gR_j * s_dq[DI(el, c, fp3)];
                    gr[c][0] = gr[c][0] + (lg.xix * lx + lg.etx * le);
                    gr[c][1] = gr[c][1] + (lg.xiy * lx + lg.ety * le);
                }
            }
            if constexpr (MODE == MODE_PREP) {
                double* spk = a.spack + cd.spoff + (size_t)e * Np + lt;
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) spk[(size_t)vv * EN] = qs[vv];
                if (VISC) {
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        spk[(size_t)(4 + d) * EN] = gu[d];
                        spk[(size_t)(6 + d) * EN] = gv[d];
                        spk[(size_t)(8 + d) * EN] = gT[d];
                    }
                }
            }
            T fl[4], gl[4], qc[4];
            fr_point_flux<T, VISC>(pc, qs, gu, gv, gT, fl, gl, qc);
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                if constexpr (TAN) {
                    s_wd[WD(el, vv, lt)] = lg.xix * fl[vv].d[0] + lg.xiy * gl[vv].d[0];
                    s_wd[WD(el, 4 + vv, lt)] = lg.etx * fl[vv].d[0] + lg.ety * gl[vv].d[0];
                } else {
                    s_w[WI(el, vv, lt)] = lg.xix * fl[vv] + lg.xiy * gl[vv];
                    s_w[WI(el, 4 + vv, lt)] = lg.etx * fl[vv] + lg.ety * gl[vv];
                }
            }
        }
        __syncthreads();
        // ---- stage 5: F^num - F^loc, F^loc = |J| Pi F~ (xi faces) or |J| Pi G~ (eta faces)
        if (act && lt < NF) {
            const double* lam = s_lam[f & 1];
            const double jac = 1.0 / lg.ij;
            const int base = f < 2 ? 0 : 4;
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                if constexpr (TAN) {
                    double acc = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b) acc = acc + lam[b] * s_wd[WD(el, base + vv, line_pt(n, f, k, b))];
                    s_Fd[FD(el, vv, lt)] = fsc[vv].d[0] - jac * acc;
                } else {
                    T acc = cst<T>(0.0);
#pragma unroll
                    for (int b = 0; b < n; ++b) acc = acc + lam[b] * s_w[WI(el, base + vv, line_pt(n, f, k, b))];
                    s_F[FI(el, vv, lt)] = fsc[vv] - jac * acc;
                }
            }
        }
        __syncthreads();
        // ---- stage 6: divergence dF~/dxi + dG~/deta, Radau lift
        if (act && lt < Np) {
            const unsigned id = (unsigned)e * Np + lt;
            double* out = a.out + cd.off;
            double tt[4] = {0.0, 0.0, 0.0, 0.0};   // time terms of the Newton operator
            if constexpr (MODE == MODE_AOP) {
                double ct = a.c_time, idt = a.inv_dtau;
                if (a.cstep) { ct = rfl(a.cstep[cid].ct); idt = rfl(a.cstep[cid].idt); }
                double qv[4], x[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) { const T w = s_q[QI(el, vv, lt)]; qv[vv] = w.v; x[vv] = w.d[0]; }
                fr_time_apply<double, double>(pc, qv, 0.0, 0.0, idt, ct, x, tt);
            }
#pragma unroll 1
            for (int vv = 0; vv < 4; ++vv) {
                if constexpr (TAN) {
                    double dF = 0.0, dG = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        dF = dF + s_D[i * n + b] * s_wd[WD(el, vv, b + n * j)];
                        dG = dG + s_D[j * n + b] * s_wd[WD(el, 4 + vv, i + n * b)];
                    }
                    const double cor = s_gam[0][i] * s_Fd[FD(el, vv, 0 * n + j)] + s_gam[1][i] * s_Fd[FD(el, vv, 1 * n + j)]
                                     + s_gam[0][j] * s_Fd[FD(el, vv, 2 * n + i)] + s_gam[1][j] * s_Fd[FD(el, vv, 3 * n + i)];
                    const double R = -(dF + dG + lg.ij * cor);
                    if constexpr (MODE == MODE_AOP) {
                        const double ttv = (vv == 0) ? tt[0] : (vv == 1) ? tt[1] : (vv == 2) ? tt[2] : tt[3];
                        out[vv * EN + id] = ttv - R;
                    } else {
                        out[vv * EN + id] = R;
                    }
                    continue;
                }
                T dF = cst<T>(0.0), dG = cst<T>(0.0);
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    dF = dF + s_D[i * n + b] * s_w[WI(el, vv, b + n * j)];
                    dG = dG + s_D[j * n + b] * s_w[WI(el, 4 + vv, i + n * b)];
                }
                const T cor = s_gam[0][i] * s_F[FI(el, vv, 0 * n + j)] + s_gam[1][i] * s_F[FI(el, vv, 1 * n + j)]
                            + s_gam[0][j] * s_F[FI(el, vv, 2 * n + i)] + s_gam[1][j] * s_F[FI(el, vv, 3 * n + i)];
                const T R = -(dF + dG + lg.ij * cor);
                if constexpr (MODE == MODE_JVP) {
                    out[vv * EN + id] = R.d[0];
                    if (a.out2) a.out2[cd.off + vv * EN + id] = R.v;
                } else if constexpr (MODE == MODE_AOP) {
                    const double ttv = (vv == 0) ? tt[0] : (vv == 1) ? tt[1] : (vv == 2) ? tt[2] : tt[3];
                    out[vv * EN + id] = ttv - R.d[0];
                } else {
                    out[vv * EN + id] = R;
                }
            }
        }
    }
}

// Newton operator Av = inv_dtau Gamma v + c_time M v - J v from the linearisation packs of
// the state (MODE_LIN).  Every stage that is linear in the state (gradients, traces,
// interpolation, divergence, lifting) acts on the tangent v alone, so LDS holds doubles;
// the nonlinear point functions (common flux, point flux) run on dual numbers whose
// values come from the packs.  The tangent arithmetic is the dual-number arithmetic of
// the other modes term by term (same sums in the same order); the result matches MODE_AOP
// to a few ulp, where the compiler contracts different products into fused multiply-adds.
template <int P, bool VISC, bool MOV, int LANES, bool BLK, bool BC, bool CS = false>
__global__ void __launch_bounds__((Shape<P, LANES>::threads))
k_lin(GroupArgs ga, KArgs a, OpTab op) {
    using D = Dual<1>;
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT;
    constexpr int EPB = Shape<P, LANES>::EPB;
    using PD = LPad<P, 1>;
    constexpr int FS = Np + PD::F, FACE = 4 * FS + PD::FACE, ESN = 4 * FACE + PD::E, ESQ = 4 * FS + PD::E;
    constexpr int NG = VISC ? 6 : 1;
    constexpr int ESG = NG * FS + PD::E;
    constexpr int ESF = 4 * NF + 1, ND = VISC ? 3 : 1, ESD = ND * NF + 1, ESS = 3 * NF + 1;
    __shared__ double s_q[EPB * ESQ];       // own tangent [el][var][point]
    __shared__ double s_n[EPB * ESN];       // neighbour tangents [el][face][var][point]; later f', g' (, q^c')
    __shared__ double s_g[EPB * ESG];       // own uncorrected gradient tangent
    __shared__ double s_F[EPB * ESF];       // F^num', then F^num' - F^loc'
    __shared__ double s_dq[EPB * ESD];      // (q^com - q^-)' of (u, v, T)
    __shared__ double s_S[EPB * ESS];       // element-oriented S, S . v_g
    auto QI = [](int el, int v, int sp) { return el * ESQ + v * FS + sp; };
    auto NI = [](int el, int fld, int sp) { return el * ESN + (fld >> 2) * FACE + (fld & 3) * FS + sp; };
    auto GI = [](int el, int c, int sp) { return el * ESG + c * FS + sp; };
    auto FI = [](int el, int v, int fp) { return el * ESF + v * NF + fp; };
    auto DI = [](int el, int c, int fp) { return el * ESD + c * NF + fp; };
    auto SI = [](int el, int c, int fp) { return el * ESS + c * NF + fp; };
    __shared__ double s_D[n * n];
    __shared__ double s_lam[2][n], s_gam[2][n], s_dlam[2][n];
    auto mk = [](double v, double d) { D r; r.v = v; r.d[0] = d; return r; };

    // a Gauss-Seidel coupling pass: the element's own tangent is zero, and so are its gradient,
    // its traces and its time terms, which are therefore not formed
    constexpr bool ZO = CS && !BLK;
    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) s_D[t] = op.D[t];
    if (threadIdx.x < n) {
        s_lam[0][threadIdx.x] = op.lamL[threadIdx.x]; s_lam[1][threadIdx.x] = op.lamR[threadIdx.x];
        s_gam[0][threadIdx.x] = op.gamL[threadIdx.x]; s_gam[1][threadIdx.x] = op.gamR[threadIdx.x];
        s_dlam[0][threadIdx.x] = op.dlamL[threadIdx.x]; s_dlam[1][threadIdx.x] = op.dlamR[threadIdx.x];
    }
    const int i = lt % n, j = lt / n;
    int tile, tend, tstride;
    tile_range(ga.ntiles, ga.xcd, tile, tend, tstride);
    for (; tile < tend; tile += tstride) {
        const int lo = find_member(ga, tile);
        const int cid = sld(ga.ids + lo);
        if (a.flags && rfl(a.flags[cid * GI_STRIDE + a.flag])) continue;
        const CaseDev cd = load_case(ga.cases + cid);
        const PhysConst& pc = cd.pc;
        const Geo g = cd.g;
        const int E = cd.E;
        bool act;
        const int e = tile_elem(ga, g, lo, tile, EPB, el, E, act);
        const unsigned EN = (unsigned)E * Np;
        const double* v = BLK ? nullptr : a.v + cd.off;
        const double* fpk = a.fpack + cd.fpoff;
        const double* spk = a.spack + cd.spoff;
        __syncthreads();
        // ---- stage 1: own and neighbour tangents (block columns: the unit seed of column
        // seed0 in the element itself, and in a neighbour only when it is the element)
        LaneGeo lg;
        int bck = 0;   // boundary kind of the lane's face (0: interior)
        if (act) {
            int pk4[4];
#pragma unroll
            for (int ff = 0; ff < 4; ++ff) pk4[ff] = ldo(g.nbr, (unsigned)(e * 4 + ff));
            if (BC && g.bc) bck = (gld(g.bc + e) >> (2 * ((lt % NF) / n))) & 3;
            const int ls = lt % Np;
            const unsigned id = (unsigned)e * Np + ls;
            // a Gauss-Seidel coupling pass takes v on elements of lower (higher) colours only, so
            // never on the element itself
            constexpr bool cs = CS && !BLK;
            double qo[4];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv)
                qo[vv] = BLK ? ((vv * Np + ls == a.seed0) ? 1.0 : 0.0) : (cs ? 0.0 : ldo(v + vv * EN, id));
            // the lane's own face entry is loaded on its own: selecting it from pk4 by the lane's
            // face makes the compiler index a stack copy of pk4 (scratch memory)
            lane_geo_load<P, VISC, MOV>(g, E, e, lt, ldo(g.nbr, (unsigned)(e * 4 + (lt % NF) / n)), lg);
            if (lt < Np) {
#pragma unroll
                for (int vv = 0; vv < 4; ++vv)
                    if (!ZO) s_q[QI(el, vv, lt)] = qo[vv];
#pragma unroll
                for (int ff = 0; ff < 4; ++ff) {
                    const int nb = pk4[ff] >> 3;
                    const unsigned nid = (unsigned)nb * Np + lt;
                    bool take = true;
                    if (cs) {
                        const int cn = ldo(g.color, (unsigned)nb);
                        take = a.cbelow ? cn < a.csweep - 1 : cn > a.csweep - 1;
                    }
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv)
                        s_n[NI(el, ff * 4 + vv, lt)] =
                            BLK ? ((nb == e && vv * Np + lt == a.seed0) ? 1.0 : 0.0) : (take ? ldo(v + vv * EN, nid) : 0.0);
                }
            }
        }
        __syncthreads();
        // ---- stage 2: uncorrected gradient tangent
        if (VISC && !ZO && act && lt < Np) {
            const double xix = lg.xix, xiy = lg.xiy, etx = lg.etx, ety = lg.ety;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double dxi = 0.0, deta = 0.0;
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    dxi = dxi + s_D[i * n + b] * s_q[QI(el, c + 1, b + n * j)];
                    deta = deta + s_D[j * n + b] * s_q[QI(el, c + 1, i + n * b)];
                }
                s_g[GI(el, 2 * c, lt)] = xix * dxi + etx * deta;
                s_g[GI(el, 2 * c + 1, lt)] = xiy * dxi + ety * deta;
            }
        }
        __syncthreads();
        // ---- stage 3: trace tangents, common flux on dual numbers (values from the face pack);
        // an affine neighbour's gradient trace from its traces, as in the residual kernel
        const int f = (lt % NF) / n, k = lt % n;
        const int nf = lg.nf, k2 = lg.k2;
        double qmt[4], qpt[4];
        if (act && lt < NF) {
            const double* lam = s_lam[f & 1];
            const double* lamn = s_lam[nf & 1];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                double am = 0.0, ap = 0.0;
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    if (!ZO) am = am + lam[b] * s_q[QI(el, vv, line_pt(n, f, k, b))];
                    ap = ap + lamn[b] * s_n[NI(el, f * 4 + vv, line_pt(n, nf, k2, b))];
                }
                qmt[vv] = am;
                qpt[vv] = ap;
            }
            if (BC && bck) fr_bc_state_lin<double>(bck, qmt, lg.nx, lg.ny, qpt);
            if (VISC) {
#pragma unroll
                for (int c = 0; c < 3; ++c) s_F[FI(el, c, f * n + k2)] = qpt[c + 1];
            }
        }
        if (VISC) __syncthreads();
        double fsc[4];   // tangent of S F^num, kept in registers until stage 5
        if (act && lt < NF) {
            const double* lam = s_lam[f & 1];
            const double* lamn = s_lam[nf & 1];
            const unsigned FE = (unsigned)E * NF;
            const unsigned sid = (unsigned)e * NF + lt;
            const double nx = lg.nx, ny = lg.ny, sc = lg.sc, ugf = lg.fug, vgf = lg.fvg;
            D fn[4], dq[4], qm[4], qp[4];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                qm[vv] = mk(ldo(fpk + (size_t)vv * FE, sid), qmt[vv]);
                qp[vv] = mk(ldo(fpk + (size_t)(4 + vv) * FE, sid), qpt[vv]);
            }
            fr_common_inviscid<D>(pc, qm, qp, nx, ny, ugf, vgf, fn, dq);
            if (VISC) {
                D gm[6], gp[6];
                double gmt[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    double am = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b)
                        if (!ZO) am = am + lam[b] * s_g[GI(el, c, line_pt(n, f, k, b))];
                    gm[c] = mk(ldo(fpk + (size_t)(8 + c) * FE, sid), am);
                    gmt[c] = am;
                }
                double gpt[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                if (lg.aff) {
                    const double xix = lg.mxix, xiy = lg.mxiy, etx = lg.metx, ety = lg.mety;
                    const double* dlamn = s_dlam[nf & 1];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        double dnor = 0.0, dtan = 0.0;
#pragma unroll
                        for (int m = 0; m < n; ++m) {
                            dnor = dnor + dlamn[m] * s_n[NI(el, f * 4 + c + 1, line_pt(n, nf, k2, m))];
                            dtan = dtan + s_D[k2 * n + m] * s_F[FI(el, c, f * n + m)];
                        }
                        const double dxi = nf < 2 ? dnor : dtan, deta = nf < 2 ? dtan : dnor;
                        gpt[2 * c] = xix * dxi + etx * deta;
                        gpt[2 * c + 1] = xiy * dxi + ety * deta;
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        const int sp = line_pt(n, nf, k2, b);
                        const int is = sp % n, js = sp / n;
                        const unsigned gid = (unsigned)lg.nb * Np + sp;
                        const double xix = ldo(g.sp + G_XIX * EN, gid), xiy = ldo(g.sp + G_XIY * EN, gid);
                        const double etx = ldo(g.sp + G_ETX * EN, gid), ety = ldo(g.sp + G_ETY * EN, gid);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            double dxi = 0.0, deta = 0.0;
#pragma unroll
                            for (int m = 0; m < n; ++m) {
                                dxi = dxi + s_D[is * n + m] * s_n[NI(el, f * 4 + c + 1, m + n * js)];
                                deta = deta + s_D[js * n + m] * s_n[NI(el, f * 4 + c + 1, is + n * m)];
                            }
                            gpt[2 * c] = gpt[2 * c] + lamn[b] * (xix * dxi + etx * deta);
                            gpt[2 * c + 1] = gpt[2 * c + 1] + lamn[b] * (xiy * dxi + ety * deta);
                        }
                    }
                }
                if (BC && bck) fr_bc_grad<double>(bck, gmt, nx, ny, gpt);
#pragma unroll
                for (int c = 0; c < 6; ++c) gp[c] = mk(0.0, gpt[c]);   // the pack holds g^- + g^+ in gm
                // q^com velocity = q^- + dq/2 (the own trace as formed above)
                const D qcu = qm[1] + 0.5 * dq[1];
                const D qcv = qm[2] + 0.5 * dq[2];
                D dqh[3];
                fr_common_viscous<D>(pc, dq, qcu, qcv, gm, gp, nx, ny, lg.cc, fn, dqh);
#pragma unroll
                for (int c = 0; c < 3; ++c) s_dq[DI(el, c, lt)] = dqh[c].d[0];
            }
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) fsc[vv] = (sc * fn[vv]).d[0];
            s_S[SI(el, 0, lt)] = sc * nx;
            s_S[SI(el, 1, lt)] = sc * ny;
            s_S[SI(el, 2, lt)] = MOV ? sc * (ugf * nx + vgf * ny) : 0.0;
        }
        __syncthreads();
        // ---- stage 4: corrected gradient tangent, point flux on dual numbers (values from the point pack)
        auto WI = [&](int fld, int sp) { return NI(el, fld, sp); };
        double qv[4];
        if (act && lt < Np) {
            const unsigned id = (unsigned)e * Np + lt;
            const double ij = lg.ij;
            D qs[4], gu[2], gv[2], gT[2];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                qv[vv] = ldo(spk + (size_t)vv * EN, id);
                qs[vv] = mk(qv[vv], ZO ? 0.0 : s_q[QI(el, vv, lt)]);
            }
            if (VISC) {
                double gt[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) gt[c] = ZO ? 0.0 : s_g[GI(el, c, lt)];
                const int fp0 = 0 * n + j, fp1 = 1 * n + j, fp2 = 2 * n + i, fp3 = 3 * n + i;
                const double gL_i = s_gam[0][i], gR_i = s_gam[1][i], gL_j = s_gam[0][j], gR_j = s_gam[1][j];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double cx = (s_S[SI(el, 0, fp0)] * gL_i) * s_dq[DI(el, c, fp0)] + (s_S[SI(el, 0, fp1)] * gR_i) * s_dq[DI(el, c, fp1)]
                                    + (s_S[SI(el, 0, fp2)] * gL_j) * s_dq[DI(el, c, fp2)] + (s_S[SI(el, 0, fp3)] * gR_j) * s_dq[DI(el, c, fp3)];
                    const double cy = (s_S[SI(el, 1, fp0)] * gL_i) * s_dq[DI(el, c, fp0)] + (s_S[SI(el, 1, fp1)] * gR_i) * s_dq[DI(el, c, fp1)]
                                    + (s_S[SI(el, 1, fp2)] * gL_j) * s_dq[DI(el, c, fp2)] + (s_S[SI(el, 1, fp3)] * gR_j) * s_dq[DI(el, c, fp3)];
                    gt[2 * c] = gt[2 * c] + ij * cx;
                    gt[2 * c + 1] = gt[2 * c + 1] + ij * cy;
                }
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    gu[d] = mk(ldo(spk + (size_t)(4 + d) * EN, id), gt[d]);
                    gv[d] = mk(ldo(spk + (size_t)(6 + d) * EN, id), gt[2 + d]);
                    gT[d] = mk(ldo(spk + (size_t)(8 + d) * EN, id), gt[4 + d]);
                }
            }
            D fl[4], gl[4], qc[4];
            fr_point_flux<D, VISC>(pc, qs, gu, gv, gT, fl, gl, qc);
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                s_n[WI(vv, lt)] = fl[vv].d[0];
                s_n[WI(4 + vv, lt)] = gl[vv].d[0];
                if (MOV) s_n[WI(8 + vv, lt)] = qc[vv].d[0];
            }
        }
        __syncthreads();
        // ---- stage 5: F^num' - F^loc'
        if (act && lt < NF) {
            const double* lam = s_lam[f & 1];
            const double Sx = s_S[SI(el, 0, lt)], Sy = s_S[SI(el, 1, lt)], Svg = s_S[SI(el, 2, lt)];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                double acc = 0.0;
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    const int sp = line_pt(n, f, k, b);
                    double w = Sx * s_n[WI(vv, sp)] + Sy * s_n[WI(4 + vv, sp)];
                    if (MOV) w = w - Svg * s_n[WI(8 + vv, sp)];
                    acc = acc + lam[b] * w;
                }
                s_F[FI(el, vv, lt)] = fsc[vv] - acc;
            }
        }
        __syncthreads();
        // ---- stage 6: divergence, moving-mesh terms, lift of the tangents; time terms
        if (act && lt < Np) {
            const unsigned id = (unsigned)e * Np + lt;
            const double geo[NGSP] = {lg.xix, lg.xiy, lg.etx, lg.ety, lg.ij, lg.ug, lg.vg};
            const double axi = MOV ? geo[G_UG] * geo[G_XIX] + geo[G_VG] * geo[G_XIY] : 0.0;
            const double aet = MOV ? geo[G_UG] * geo[G_ETX] + geo[G_VG] * geo[G_ETY] : 0.0;
            double ct = a.c_time, idt = a.inv_dtau;
            if (a.cstep) { ct = rfl(a.cstep[cid].ct); idt = rfl(a.cstep[cid].idt); }
            double tt[4], x[4];
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) x[vv] = ZO ? 0.0 : s_q[QI(el, vv, lt)];
            if constexpr (ZO) {
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) tt[vv] = 0.0;
            } else {
                fr_time_apply<double, double>(pc, qv, geo[G_UG], geo[G_VG], idt, ct, x, tt);
            }
            double* out = a.out + (BLK ? cd.boff + (size_t)e * (4 * Np) * (4 * Np) : cd.off);
#pragma unroll 1
            for (int vv = 0; vv < 4; ++vv) {
                double dfx = 0.0, dfe = 0.0, dgx = 0.0, dge = 0.0, dqx = 0.0, dqe = 0.0;
#pragma unroll
                for (int b = 0; b < n; ++b) {
                    const double Dx = s_D[i * n + b], De = s_D[j * n + b];
                    dfx = dfx + Dx * s_n[WI(vv, b + n * j)];
                    dgx = dgx + Dx * s_n[WI(4 + vv, b + n * j)];
                    dfe = dfe + De * s_n[WI(vv, i + n * b)];
                    dge = dge + De * s_n[WI(4 + vv, i + n * b)];
                    if (MOV) {
                        dqx = dqx + Dx * s_n[WI(8 + vv, b + n * j)];
                        dqe = dqe + De * s_n[WI(8 + vv, i + n * b)];
                    }
                }
                double vol = geo[G_XIX] * dfx + geo[G_ETX] * dfe + geo[G_XIY] * dgx + geo[G_ETY] * dge;
                if (MOV) vol = vol - axi * dqx - aet * dqe;
                const double cor = s_gam[0][i] * s_F[FI(el, vv, 0 * n + j)] + s_gam[1][i] * s_F[FI(el, vv, 1 * n + j)]
                                 + s_gam[0][j] * s_F[FI(el, vv, 2 * n + i)] + s_gam[1][j] * s_F[FI(el, vv, 3 * n + i)];
                const double Rd = -(vol + geo[G_IJ] * cor);
                const double ttv = (vv == 0) ? tt[0] : (vv == 1) ? tt[1] : (vv == 2) ? tt[2] : tt[3];
                if (BLK) {
                    // column seed0 of the element's block, column-major; the time terms are zero
                    // away from the seeded point, where ttv - Rd is exactly -Rd
                    out[(size_t)a.seed0 * (4 * Np) + vv * Np + lt] = ttv - Rd;
                } else {
                    out[vv * EN + id] = ttv - Rd;
                }
            }
        }
    }
}

// The Newton operator from the linearisation packs (as k_lin) for static groups whose elements
// are all affine, with the changes of k_fused_aff: neighbour tangent lines read into
// registers, the neighbour gradient trace from its traces, contravariant flux tangents, face
// vectors from the constant metrics.  BLK: one seeded block column per launch.
template <int P, bool VISC, int LANES, bool BLK, bool CS = false>
__global__ void __launch_bounds__((Shape<P, LANES>::threads))
k_lin_aff(GroupArgs ga, KArgs a, OpTab op) {
    using D = Dual<1>;
    constexpr int n = P + 1, Np = n * n, NF = 4 * n, NT = Sz<P>::NT;
    constexpr int EPB = Shape<P, LANES>::EPB;
    using PD = LPad<P, 1>;
    constexpr int FS = Np + PD::F;
    constexpr int ESQ = 4 * FS + PD::E;
    constexpr int ESW = 8 * FS + PD::E;
    constexpr int NG = VISC ? 6 : 1;
    constexpr int ESG = NG * FS + PD::E;
    constexpr int ESF = 4 * NF + 1, ND = VISC ? 3 : 1, ESD = ND * NF + 1;
    __shared__ double s_q[EPB * ESQ];       // own tangent [el][var][point]
    __shared__ double s_w[EPB * ESW];       // F~', G~' [el][8][point]
    __shared__ double s_g[EPB * ESG];       // own uncorrected gradient tangent
    __shared__ double s_F[EPB * ESF];       // neighbour trace tangents of (u, v, T); then F^num' - F^loc'
    __shared__ double s_dq[EPB * ESD];      // (q^com - q^-)' of (u, v, T)
    auto QI = [](int el, int v, int sp) { return el * ESQ + v * FS + sp; };
    auto WI = [](int el, int fld, int sp) { return el * ESW + fld * FS + sp; };
    auto GI = [](int el, int c, int sp) { return el * ESG + c * FS + sp; };
    auto FI = [](int el, int v, int fp) { return el * ESF + v * NF + fp; };
    auto DI = [](int el, int c, int fp) { return el * ESD + c * NF + fp; };
    __shared__ double s_D[n * n];
    __shared__ double s_lam[2][n], s_gam[2][n], s_dlam[2][n];
    auto mk = [](double v, double d) { D r; r.v = v; r.d[0] = d; return r; };

    // a Gauss-Seidel coupling pass: the element's own tangent is zero, and so are its gradient,
    // its traces and its time terms, which are therefore not formed
    constexpr bool ZO = CS && !BLK;
    const int el = threadIdx.x / NT, lt = threadIdx.x % NT;
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) s_D[t] = op.D[t];
    if (threadIdx.x < n) {
        s_lam[0][threadIdx.x] = op.lamL[threadIdx.x]; s_lam[1][threadIdx.x] = op.lamR[threadIdx.x];
        s_gam[0][threadIdx.x] = op.gamL[threadIdx.x]; s_gam[1][threadIdx.x] = op.gamR[threadIdx.x];
        s_dlam[0][threadIdx.x] = op.dlamL[threadIdx.x]; s_dlam[1][threadIdx.x] = op.dlamR[threadIdx.x];
    }
    const int i = lt % n, j = lt / n;
    const int f = (lt % NF) / n, k = lt % n;
    int tile, tend, tstride;
    tile_range(ga.ntiles, ga.xcd, tile, tend, tstride);
    int pkn = 0;   // connectivity of the next tile, requested one tile ahead
    int pkn_tile = -1;
    for (; tile < tend; tile += tstride) {
        const int lo = find_member(ga, tile);
        const int cid = sld(ga.ids + lo);
        if (a.flags && rfl(a.flags[cid * GI_STRIDE + a.flag])) continue;
        const CaseDev cd = load_case(ga.cases + cid);
        const PhysConst& pc = cd.pc;
        const Geo g = cd.g;
        const int E = cd.E;
        bool act;
        const int e = tile_elem(ga, g, lo, tile, EPB, el, E, act);
        const unsigned EN = (unsigned)E * Np;
        const double* v = BLK ? nullptr : a.v + cd.off;
        const double* fpk = a.fpack + cd.fpoff;
        const double* spk = a.spack + cd.spoff;
        __syncthreads();
        LaneGeo lg;
        const bool pre = pkn_tile == tile;
        // block columns: the connectivity, the metric terms and the packs once per tile, for
        // every column of the launch (a.ncols from seed0)
        double fpv[14], spv[10];
        if constexpr (BLK) {
            if (act) {
                lane_geo_load<P, VISC, false>(g, E, e, lt, pre ? pkn : ldo(g.nbr, (unsigned)(e * 4 + f)), lg);
                if (lt < NF) {
                    const unsigned FE = (unsigned)E * NF, sid = (unsigned)e * NF + lt;
#pragma unroll
                    for (int c = 0; c < (VISC ? 14 : 8); ++c) fpv[c] = ldo(fpk + (size_t)c * FE, sid);
                }
                if (lt < Np) {
                    const unsigned id = (unsigned)e * Np + lt;
#pragma unroll
                    for (int c = 0; c < (VISC ? 10 : 4); ++c) spv[c] = ldo(spk + (size_t)c * EN, id);
                }
            }
        }
        const int c0 = BLK ? a.seed0 : 0;
        const int c1 = BLK ? min(a.seed0 + max(a.ncols, 1), 4 * Np) : 1;
        for (int col = c0; col < c1; ++col) {
            if (col > c0) __syncthreads();   // the previous column's readers of LDS are done
            // ---- stage 1: own tangent; the neighbour's tangent line through this face point
            double qpt[4], dnort[3];
            if (act) {
                const int ls = lt % Np;
                const unsigned id = (unsigned)e * Np + ls;
                // a Gauss-Seidel coupling pass takes v on elements of lower (higher) colours only, so
                // never on the element itself
                constexpr bool cs = CS && !BLK;
                double qo[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv)
                    qo[vv] = BLK ? ((vv * Np + ls == col) ? 1.0 : 0.0) : (cs ? 0.0 : ldo(v + vv * EN, id));
                if constexpr (!BLK) lane_geo_load<P, VISC, false>(g, E, e, lt, pre ? pkn : ldo(g.nbr, (unsigned)(e * 4 + f)), lg);
                if (lt < NF) {
                    const unsigned nbase = (unsigned)lg.nb * Np;
                    bool take = true;
                    if (cs) {
                        const int cn = ldo(g.color, (unsigned)lg.nb);
                        take = a.cbelow ? cn < a.csweep - 1 : cn > a.csweep - 1;
                    }
                    double ln[4][n];
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        const int sp = line_pt(n, lg.nf, lg.k2, b);
#pragma unroll
                        for (int vv = 0; vv < 4; ++vv)
                            ln[vv][b] = BLK ? ((lg.nb == e && vv * Np + sp == col) ? 1.0 : 0.0)
                                            : (take ? ldo(v + vv * EN, nbase + sp) : 0.0);
                    }
                    const double* lamn = s_lam[lg.nf & 1];
                    const double* dlamn = s_dlam[lg.nf & 1];
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv) {
                        double acc = 0.0;
#pragma unroll
                        for (int b = 0; b < n; ++b) acc = acc + lamn[b] * ln[vv][b];
                        qpt[vv] = acc;
                    }
                    if (VISC) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            double acc = 0.0;
#pragma unroll
                            for (int b = 0; b < n; ++b) acc = acc + dlamn[b] * ln[c + 1][b];
                            dnort[c] = acc;
                            s_F[FI(el, c, f * n + lg.k2)] = qpt[c + 1];
                        }
                    }
                }
                if (lt < Np) {
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv)
                        if (!ZO) s_q[QI(el, vv, lt)] = qo[vv];
                }
            }
            if (col == c0) {
                const int tn = tile + tstride;
                const int pfx_hi = lo + 1 < ga.nmem ? sld(ga.pfx + lo + 1) : ga.ntiles;
                pkn_tile = (tn < tend && tn < pfx_hi) ? tn : -1;
                if (pkn_tile >= 0) {
                    bool actn;
                    const int en = tile_elem(ga, g, lo, tn, EPB, el, E, actn);
                    if (actn) pkn = ldo(g.nbr, (unsigned)(en * 4 + f));
                }
            }
            __syncthreads();
            // ---- stage 2: uncorrected gradient tangent
            if (VISC && !ZO && act && lt < Np) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double dxi = 0.0, deta = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        dxi = dxi + s_D[i * n + b] * s_q[QI(el, c + 1, b + n * j)];
                        deta = deta + s_D[j * n + b] * s_q[QI(el, c + 1, i + n * b)];
                    }
                    s_g[GI(el, 2 * c, lt)] = lg.xix * dxi + lg.etx * deta;
                    s_g[GI(el, 2 * c + 1, lt)] = lg.xiy * dxi + lg.ety * deta;
                }
            }
            __syncthreads();
            // ---- stage 3: common flux on dual numbers (values from the face pack)
            double fsc[4];
            if (act && lt < NF) {
                const double* lam = s_lam[f & 1];
                const unsigned FE = (unsigned)E * NF;
                const unsigned sid = (unsigned)e * NF + lt;
                const double nx = lg.nx, ny = lg.ny, sc = lg.sc;
                D fn[4], dq[4], qm[4], qp[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    double acc = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b)
                        if (!ZO) acc = acc + lam[b] * s_q[QI(el, vv, line_pt(n, f, k, b))];
                    qm[vv] = mk(BLK ? fpv[vv] : ldo(fpk + (size_t)vv * FE, sid), acc);
                    qp[vv] = mk(BLK ? fpv[4 + vv] : ldo(fpk + (size_t)(4 + vv) * FE, sid), qpt[vv]);
                }
                fr_common_inviscid<D>(pc, qm, qp, nx, ny, 0.0, 0.0, fn, dq);
                if (VISC) {
                    D gm[6], gp[6];
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        double acc = 0.0;
#pragma unroll
                        for (int b = 0; b < n; ++b)
                            if (!ZO) acc = acc + lam[b] * s_g[GI(el, c, line_pt(n, f, k, b))];
                        gm[c] = mk(BLK ? fpv[8 + c] : ldo(fpk + (size_t)(8 + c) * FE, sid), acc);
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        double dtan = 0.0;
#pragma unroll
                        for (int m = 0; m < n; ++m) dtan = dtan + s_D[lg.k2 * n + m] * s_F[FI(el, c, f * n + m)];
                        const double dxi = lg.nf < 2 ? dnort[c] : dtan, deta = lg.nf < 2 ? dtan : dnort[c];
                        gp[2 * c] = mk(0.0, lg.mxix * dxi + lg.metx * deta);   // the pack holds g^- + g^+ in gm
                        gp[2 * c + 1] = mk(0.0, lg.mxiy * dxi + lg.mety * deta);
                    }
                    const D qcu = qm[1] + 0.5 * dq[1];
                    const D qcv = qm[2] + 0.5 * dq[2];
                    D dqh[3];
                    fr_common_viscous<D>(pc, dq, qcu, qcv, gm, gp, nx, ny, lg.cc, fn, dqh);
#pragma unroll
                    for (int c = 0; c < 3; ++c) s_dq[DI(el, c, lt)] = dqh[c].d[0];
                }
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) fsc[vv] = (sc * fn[vv]).d[0];
            }
            __syncthreads();
            // ---- stage 4: corrected gradient tangent, point flux on dual numbers, contravariant tangents
            double qv[4];
            if (act && lt < Np) {
                const unsigned id = (unsigned)e * Np + lt;
                D qs[4], gu[2], gv[2], gT[2];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    qv[vv] = BLK ? spv[vv] : ldo(spk + (size_t)vv * EN, id);
                    qs[vv] = mk(qv[vv], ZO ? 0.0 : s_q[QI(el, vv, lt)]);
                }
                if (VISC) {
                    double gt[6];
#pragma unroll
                    for (int c = 0; c < 6; ++c) gt[c] = ZO ? 0.0 : s_g[GI(el, c, lt)];
                    const int fp0 = 0 * n + j, fp1 = 1 * n + j, fp2 = 2 * n + i, fp3 = 3 * n + i;
                    const double gL_i = s_gam[0][i], gR_i = s_gam[1][i], gL_j = s_gam[0][j], gR_j = s_gam[1][j];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double lx = gL_i * s_dq[DI(el, c, fp0)] + gR_i * s_dq[DI(el, c, fp1)];
                        const double le = gL_j * s_dq[DI(el, c, fp2)] + gR_j * s_dq[DI(el, c, fp3)];
                        gt[2 * c] = gt[2 * c] + (lg.xix * lx + lg.etx * le);
                        gt[2 * c + 1] = gt[2 * c + 1] + (lg.xiy * lx + lg.ety * le);
                    }
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        gu[d] = mk(BLK ? spv[4 + d] : ldo(spk + (size_t)(4 + d) * EN, id), gt[d]);
                        gv[d] = mk(BLK ? spv[6 + d] : ldo(spk + (size_t)(6 + d) * EN, id), gt[2 + d]);
                        gT[d] = mk(BLK ? spv[8 + d] : ldo(spk + (size_t)(8 + d) * EN, id), gt[4 + d]);
                    }
                }
                D fl[4], gl[4], qc[4];
                fr_point_flux<D, VISC>(pc, qs, gu, gv, gT, fl, gl, qc);
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    s_w[WI(el, vv, lt)] = lg.xix * fl[vv].d[0] + lg.xiy * gl[vv].d[0];
                    s_w[WI(el, 4 + vv, lt)] = lg.etx * fl[vv].d[0] + lg.ety * gl[vv].d[0];
                }
            }
            __syncthreads();
            // ---- stage 5: F^num' - F^loc'
            if (act && lt < NF) {
                const double* lam = s_lam[f & 1];
                const double jac = 1.0 / lg.ij;
                const int base = f < 2 ? 0 : 4;
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    double acc = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b) acc = acc + lam[b] * s_w[WI(el, base + vv, line_pt(n, f, k, b))];
                    s_F[FI(el, vv, lt)] = fsc[vv] - jac * acc;
                }
            }
            __syncthreads();
            // ---- stage 6: divergence and lift of the tangents; time terms
            if (act && lt < Np) {
                const unsigned id = (unsigned)e * Np + lt;
                double ct = a.c_time, idt = a.inv_dtau;
                if (a.cstep) { ct = rfl(a.cstep[cid].ct); idt = rfl(a.cstep[cid].idt); }
                double tt[4], x[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) x[vv] = ZO ? 0.0 : s_q[QI(el, vv, lt)];
                if constexpr (ZO) {
#pragma unroll
                    for (int vv = 0; vv < 4; ++vv) tt[vv] = 0.0;
                } else {
                    fr_time_apply<double, double>(pc, qv, 0.0, 0.0, idt, ct, x, tt);
                }
                double* out = a.out + (BLK ? cd.boff + (size_t)e * (4 * Np) * (4 * Np) : cd.off);
#pragma unroll 1
                for (int vv = 0; vv < 4; ++vv) {
                    double dF = 0.0, dG = 0.0;
#pragma unroll
                    for (int b = 0; b < n; ++b) {
                        dF = dF + s_D[i * n + b] * s_w[WI(el, vv, b + n * j)];
                        dG = dG + s_D[j * n + b] * s_w[WI(el, 4 + vv, i + n * b)];
                    }
                    const double cor = s_gam[0][i] * s_F[FI(el, vv, 0 * n + j)] + s_gam[1][i] * s_F[FI(el, vv, 1 * n + j)]
                                     + s_gam[0][j] * s_F[FI(el, vv, 2 * n + i)] + s_gam[1][j] * s_F[FI(el, vv, 3 * n + i)];
                    const double Rd = -(dF + dG + lg.ij * cor);
                    const double ttv = (vv == 0) ? tt[0] : (vv == 1) ? tt[1] : (vv == 2) ? tt[2] : tt[3];
                    if (BLK) {
                        out[(size_t)col * (4 * Np) + vv * Np + lt] = ttv - Rd;
                    } else {
                        out[vv * EN + id] = ttv - Rd;
                    }
                }
            }
        }   // columns
    }
}

// every element of every member case is affine (the geometry pass's flags, read back by
// fr_set_geometry)
inline bool group_affine(const Solver& sv, const Group& gr) {
    for (int id : gr.ids)
        if (!sv.cs[id]->all_affine) return false;
    return true;
}

// grid of a launch: one workgroup per tile by default, else the tuned persistent size;
// always a multiple of 8 (the XCD count) so every XCD walks an equal tile range
inline unsigned grid_of(int ntiles, int grid) {
    long long g = grid > 0 ? grid : ntiles;
    g = ((g + 7) / 8) * 8;
    if (g < 8) g = 8;
    return (unsigned)g;
}

template <int P, bool VISC, bool MOV, int MODE, int LANES>
fr_status run(const Solver& sv, const Group& gr, const KArgs& a, int grid, int xcd, hipStream_t s) {
    using SH = Shape<P, LANES>;
    GroupArgs ga;
    ga.cases = sv.d_cases;
    ga.ids = gr.d_ids;
    ga.pfx = gr.tile_pfx(SH::EPB);
    ga.nmem = (int)gr.ids.size();
    ga.ntiles = gr.ntiles(SH::EPB);
    ga.xcd = xcd;
    if (MODE == MODE_LIN && a.csweep > 0) {
        // a Gauss-Seidel coupling pass: only the rows of colour csweep - 1 are used
        const Group::ColorTiles* ct = gr.color_tiles(SH::EPB, a.csweep - 1);
        if (!ct) { fr_set_error("colour tiles missing for this workgroup shape"); return FR_EINVAL; }
        ga.pfx = ct->d_pfx;
        ga.ntiles = ct->ntiles;
        ga.csel = ct->d_csel;
    }
    if (!ga.pfx) { fr_set_error("tile prefix missing for this workgroup shape"); return FR_EINVAL; }
    if (ga.ntiles == 0) return FR_OK;
    const OpTab& op = sv.cs[gr.ids[0]]->op;
    if constexpr (MODE == MODE_LIN || MODE == MODE_LINBLK) {
        constexpr bool B = MODE == MODE_LINBLK;
        if (!a.fpack || !a.spack || (!B && !a.v)) { fr_set_error("linearised operator without packs"); return FR_EINVAL; }
        bool aff = false;
        // a Gauss-Seidel coupling pass: the variants that take v on lower or higher colours only
        const bool cs = !B && a.csweep > 0;
        if constexpr (!MOV) {
            aff = group_affine(sv, gr);
            if (aff) {
                if (cs)
                    hipLaunchKernelGGL((k_lin_aff<P, VISC, LANES, B, !B>), dim3(grid_of(ga.ntiles, grid)),
                                       dim3(SH::threads), 0, s, ga, a, op);
                else
                    hipLaunchKernelGGL((k_lin_aff<P, VISC, LANES, B>), dim3(grid_of(ga.ntiles, grid)),
                                       dim3(SH::threads), 0, s, ga, a, op);
            }
        }
        if (!aff) {
            if (gr.bnd) {
                if constexpr (LANES <= 128) {
                    if (cs)
                        hipLaunchKernelGGL((k_lin<P, VISC, MOV, LANES, B, true, !B>), dim3(grid_of(ga.ntiles, grid)),
                                           dim3(SH::threads), 0, s, ga, a, op);
                    else
                        hipLaunchKernelGGL((k_lin<P, VISC, MOV, LANES, B, true>), dim3(grid_of(ga.ntiles, grid)),
                                           dim3(SH::threads), 0, s, ga, a, op);
                }
            } else {
                if (cs)
                    hipLaunchKernelGGL((k_lin<P, VISC, MOV, LANES, B, false, !B>), dim3(grid_of(ga.ntiles, grid)),
                                       dim3(SH::threads), 0, s, ga, a, op);
                else
                    hipLaunchKernelGGL((k_lin<P, VISC, MOV, LANES, B, false>), dim3(grid_of(ga.ntiles, grid)),
                                       dim3(SH::threads), 0, s, ga, a, op);
            }
        }
    } else {
        if (MODE == MODE_PREP && (!a.fpack || !a.spack)) { fr_set_error("packs missing"); return FR_EINVAL; }
        bool aff = false;
        constexpr bool has_aff = !MOV && (MODE == MODE_R || MODE == MODE_PREP || MODE == MODE_JVP || MODE == MODE_AOP);
        if constexpr (has_aff) aff = group_affine(sv, gr);
        if constexpr (has_aff) {
            if (aff) {
                // the tangent-only form whenever R is not wanted as well
                if constexpr (MODE == MODE_JVP || MODE == MODE_AOP) {
                    if (MODE == MODE_AOP || !a.out2)
                        hipLaunchKernelGGL((k_fused_aff<P, VISC, MODE, LANES, true>), dim3(grid_of(ga.ntiles, grid)),
                                           dim3(SH::threads), 0, s, ga, a, op);
                    else
                        hipLaunchKernelGGL((k_fused_aff<P, VISC, MODE, LANES>), dim3(grid_of(ga.ntiles, grid)),
                                           dim3(SH::threads), 0, s, ga, a, op);
                } else {
                    hipLaunchKernelGGL((k_fused_aff<P, VISC, MODE, LANES>), dim3(grid_of(ga.ntiles, grid)),
                                       dim3(SH::threads), 0, s, ga, a, op);
                }
            }
        }
        if (!aff) {
            constexpr bool dual1 = MODE == MODE_JVP || MODE == MODE_AOP;
            const bool tan = dual1 && (MODE == MODE_AOP || !a.out2);
            if (gr.bnd) {
                if constexpr (LANES <= 128) {
                    if constexpr (dual1) {
                        if (tan)
                            hipLaunchKernelGGL((k_fused<P, VISC, MOV, MODE, 1, LANES, true, true>),
                                               dim3(grid_of(ga.ntiles, grid)), dim3(SH::threads), 0, s, ga, a, op);
                    }
                    if (!tan)
                        hipLaunchKernelGGL((k_fused<P, VISC, MOV, MODE, 1, LANES, true>), dim3(grid_of(ga.ntiles, grid)),
                                           dim3(SH::threads), 0, s, ga, a, op);
                }
            } else {
                if constexpr (dual1) {
                    if (tan)
                        hipLaunchKernelGGL((k_fused<P, VISC, MOV, MODE, 1, LANES, false, true>),
                                           dim3(grid_of(ga.ntiles, grid)), dim3(SH::threads), 0, s, ga, a, op);
                }
                if (!tan)
                    hipLaunchKernelGGL((k_fused<P, VISC, MOV, MODE, 1, LANES, false>), dim3(grid_of(ga.ntiles, grid)),
                                       dim3(SH::threads), 0, s, ga, a, op);
            }
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { fr_set_error(std::string("k_fused launch: ") + hipGetErrorString(e)); return FR_EHIP; }
    return FR_OK;
}

// workgroup widths built per mode: plain doubles 64/128/256 lanes, dual numbers 64/128
template <int P, bool VISC, bool MOV, int MODE>
fr_status run_lanes(const Solver& sv, const Group& gr, const KArgs& a, const Tune& t, hipStream_t s) {
    constexpr bool dual = MODE == MODE_JVP || MODE == MODE_AOP || MODE == MODE_BLK;
    int lanes = t.lanes > 0 ? t.lanes : (dual ? 64 : 128);
    if (gr.bnd && lanes > 128) lanes = 128;   // the boundary-face variants are built for 64 and 128 lanes
    switch (lanes) {
        case 64: return run<P, VISC, MOV, MODE, 64>(sv, gr, a, t.grid, t.xcd, s);
        case 128: return run<P, VISC, MOV, MODE, 128>(sv, gr, a, t.grid, t.xcd, s);
        case 256:
            if constexpr (MODE == MODE_R) return run<P, VISC, MOV, MODE, 256>(sv, gr, a, t.grid, t.xcd, s);
            break;
    }
    fr_set_error("unsupported workgroup width");
    return FR_EINVAL;
}

template <int P, bool VISC, bool MOV>
fr_status run_mode(const Solver& sv, const Group& gr, int mode, const KArgs& a, const Tune& t, hipStream_t s) {
    switch (mode) {
        case MODE_R: return run_lanes<P, VISC, MOV, MODE_R>(sv, gr, a, t, s);
        case MODE_JVP: return run_lanes<P, VISC, MOV, MODE_JVP>(sv, gr, a, t, s);
        case MODE_AOP: return run_lanes<P, VISC, MOV, MODE_AOP>(sv, gr, a, t, s);
        case MODE_BLK: return run_lanes<P, VISC, MOV, MODE_BLK>(sv, gr, a, t, s);
        case MODE_PREP: return run_lanes<P, VISC, MOV, MODE_PREP>(sv, gr, a, t, s);
        case MODE_LIN: return run_lanes<P, VISC, MOV, MODE_LIN>(sv, gr, a, t, s);
        case MODE_LINBLK: return run_lanes<P, VISC, MOV, MODE_LINBLK>(sv, gr, a, t, s);
    }
    fr_set_error("unknown residual mode");
    return FR_EINVAL;
}

}  // namespace fused

#define FR_FUSED_INSTANTIATE(P)                                                                          \
    template <>                                                                                          \
    fr_status launch_fused_p<P>(const Solver& sv, const Group& gr, int mode, const KArgs& a, const Tune& t, \
                                hipStream_t s) {                                                         \
        if (gr.visc)                                                                                     \
            return gr.mov ? fused::run_mode<P, true, true>(sv, gr, mode, a, t, s)                         \
                          : fused::run_mode<P, true, false>(sv, gr, mode, a, t, s);                       \
        return gr.mov ? fused::run_mode<P, false, true>(sv, gr, mode, a, t, s)                            \
                      : fused::run_mode<P, false, false>(sv, gr, mode, a, t, s);                          \
    }
