// Restarted, right-preconditioned FP64 GMRES(m) and the BDF2 dual-time Newton loop for
// every case of a solver at once, with the small dense state of each case (Hessenberg
// matrix, Givens rotations, least-squares right-hand side, counters) on the device.
//
// One restart cycle is a fixed sequence of launches over all cases:
//   cycle init (per case: idle test, g = beta e1, V_0 = r / beta) |
//   m x [ z = P^-1 V_j ; w = A z ; classical Gram-Schmidt (2 streaming passes over V, or
//         4 when re-orthogonalised: option "gram_schmidt" = 2) ;
//         Givens update of column j and of g, convergence test ; V_{j+1} = w / h_{j+1,j} ] |
//   y = H^-1 g ; x += P^-1 (V y) ; r = b - A x ; beta = |r|
// Per-case flags decide which cases a launch touches: a case whose Arnoldi process has
// stopped (|g_{j+1}| <= tol |b|, breakdown, iteration cap) is skipped by the rest of the
// cycle's Arnoldi launches; a case that did not start the cycle is skipped by its update
// too.  The sequence holds no host decision, so it is captured once into a hipGraph and
// replayed; the host synchronises once per cycle to read one "needs another cycle" flag
// per case.  The Newton loop (paper Sec. 3.2) keeps per-case convergence on the device
// as well and synchronises once per Newton iteration.
#include <cmath>
#include <cstring>

#include "fr_internal.hpp"

namespace {

// layout of one case's GMRES state (doubles) for restart length m
struct GsLayout {
    int m, H, CS, SN, G, Y, H1, H2, NRM, BN, BETA, INVHN, SCALE0, total;
    __host__ __device__ explicit GsLayout(int m_) : m(m_) {
        H = 0;
        CS = H + (m + 1) * m;
        SN = CS + m;
        G = SN + m;
        Y = G + m + 1;
        H1 = Y + m;
        H2 = H1 + MAXV;
        NRM = H2 + MAXV;
        BN = NRM + 8;
        BETA = BN + 1;
        INVHN = BETA + 1;
        SCALE0 = INVHN + 1;
        total = ((SCALE0 + 1 + 7) / 8) * 8;
    }
};

struct Ctl {
    double* gs;
    int gs_stride;
    int* gi;
    CaseStep* step;   // written only by the Newton check (SER)
    double* sum;
    int n;
};

__device__ __forceinline__ int case_index() { return blockIdx.x * blockDim.x + threadIdx.x; }

// start of a solve: counters and flags of the solve
__global__ void k_gm_start(Ctl k, int maxit) {
    const int c = case_index();
    if (c >= k.n) return;
    int* gi = k.gi + c * GI_STRIDE;
    gi[GI_TOTAL] = 0;
    gi[GI_CYC] = 0;
    gi[GI_MAXIT] = maxit;
    gi[GI_DONE] = 1;
    gi[GI_IDLE] = 1;
}

// beta = bn = |b|
__global__ void k_gm_norm0(Ctl k, int m) {
    const int c = case_index();
    if (c >= k.n) return;
    if (k.gi[c * GI_STRIDE + GI_NDONE]) return;
    const GsLayout L(m);
    double* gs = k.gs + (size_t)c * k.gs_stride;
    const double b = sqrt(gs[L.NRM]);
    gs[L.BN] = b;
    gs[L.BETA] = b;
}

// the case's test for another cycle (also used by the host through the summary)
__device__ __forceinline__ bool wants_cycle(const int* gi, double beta, double bn, double tol) {
    return !gi[GI_NDONE] && isfinite(beta) && beta > 0.0 && beta > tol * bn && gi[GI_TOTAL] < gi[GI_MAXIT];
}

// per case: does it take part in this cycle?  g = beta e1, scale of V_0
__global__ void k_cycle_init(Ctl k, int m) {
    const int c = case_index();
    if (c >= k.n) return;
    const GsLayout L(m);
    double* gs = k.gs + (size_t)c * k.gs_stride;
    int* gi = k.gi + c * GI_STRIDE;
    const double beta = gs[L.BETA], bn = gs[L.BN];
    const bool run = wants_cycle(gi, beta, bn, k.step[c].tol_res);
    gi[GI_IDLE] = run ? 0 : 1;
    gi[GI_DONE] = run ? 0 : 1;
    gi[GI_CYC] = 0;
    if (!run) return;
    for (int i = 0; i <= m; ++i) gs[L.G + i] = 0.0;
    gs[L.G] = beta;
    gs[L.SCALE0] = 1.0 / beta;
}

// column j of each case's Hessenberg matrix, Givens rotations, convergence flag
// Column j of H: the Gram-Schmidt coefficients h_0..h_j (one or two passes summed) through the
// previous rotations.  Rows 0..j-1 are stored; the rotated row-j entry is returned.  The running
// entry stays in a register and the inputs are read through pointers that alias nothing written,
// so the loads of later rows need not wait for the stores of earlier ones.
__device__ __forceinline__ double rotate_column(const double* __restrict__ h1, const double* __restrict__ h2,
                                                const double* __restrict__ cs, const double* __restrict__ sn,
                                                double* __restrict__ Hj, int j, int m, bool two) {
    constexpr int CH = 8;   // rows whose inputs are loaded together
    double a = two ? h1[0] + h2[0] : h1[0];
    for (int i0 = 0; i0 < j; i0 += CH) {
        double hb[CH], c8[CH], s8[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const int i = i0 + t < j ? i0 + t : j - 1;   // rows past j - 1 load row j - 1 again, unused
            const double x1 = h1[i + 1], x2 = h2[i + 1];
            hb[t] = two ? x1 + x2 : x1;
            c8[t] = cs[i];
            s8[t] = sn[i];
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            if (i0 + t < j) {
                Hj[(size_t)(i0 + t) * m] = c8[t] * a + s8[t] * hb[t];
                a = -s8[t] * a + c8[t] * hb[t];
            }
        }
    }
    return a;
}

// One workgroup of 256 threads per case: the second stage of |w|^2 (the update pass's chunk
// partials in slot 0, summed in the order of the solver's other second stages), then the Givens
// update on thread 0.
__global__ void __launch_bounds__(256) k_norm_givens(Ctl k, const int* __restrict__ case_chunk,
                                                     const double* __restrict__ partial, int j, int m, int passes) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    int* gi = k.gi + c * GI_STRIDE;
    if (gi[GI_DONE]) return;   // uniform per workgroup
    const GsLayout L(m);
    double* gs = k.gs + (size_t)c * k.gs_stride;
    {
        const int c0 = case_chunk[c], c1 = case_chunk[c + 1];
        double v = 0.0;
        for (int b = c0 + threadIdx.x; b < c1; b += blockDim.x) v += partial[(size_t)b * MAXV];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x != 0) return;
        gs[L.NRM] = red[0];
    }
    double* H = gs + L.H;
    double* cs = gs + L.CS;
    double* sn = gs + L.SN;
    double* g = gs + L.G;
    const double hn = sqrt(gs[L.NRM]);
    const double a0 = rotate_column(gs + L.H1, gs + L.H2, cs, sn, H + j, j, m, passes == 2), a1 = hn;
    const double den = sqrt(a0 * a0 + a1 * a1);
    cs[j] = den == 0.0 ? 1.0 : a0 / den;
    sn[j] = den == 0.0 ? 0.0 : a1 / den;
    H[j * m + j] = cs[j] * a0 + sn[j] * a1;
    H[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    gi[GI_CYC] = j + 1;
    gi[GI_TOTAL] += 1;
    gs[L.INVHN] = hn > 0.0 ? 1.0 / hn : 0.0;
    const bool conv = fabs(g[j + 1]) <= k.step[c].tol_res * gs[L.BN];
    if (conv || !(hn > 0.0) || !isfinite(hn) || gi[GI_TOTAL] >= gi[GI_MAXIT] || j == m - 1) gi[GI_DONE] = 1;
}

// y = H^-1 g on the iterations of this cycle
__global__ void k_backsub(Ctl k, int m) {
    const int c = case_index();
    if (c >= k.n) return;
    const int* gi = k.gi + c * GI_STRIDE;
    if (gi[GI_IDLE]) return;
    const GsLayout L(m);
    double* gs = k.gs + (size_t)c * k.gs_stride;
    const int jd = gi[GI_CYC];
    const double* H = gs + L.H;
    double* y = gs + L.Y;
    for (int i = jd - 1; i >= 0; --i) {
        double s = gs[L.G + i];
        // eight terms' loads a pass, subtracted in order (past jd - 1: reload jd - 1, unused)
        for (int q0 = i + 1; q0 < jd; q0 += 8) {
            double h8[8], y8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + u < jd ? q0 + u : jd - 1;
                h8[u] = H[i * m + q];
                y8[u] = y[q];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q0 + u < jd) s -= h8[u] * y8[u];
        }
        y[i] = s / H[i * m + i];
    }
    for (int i = jd; i < m; ++i) y[i] = 0.0;
}

// beta = |r| after the update; a non-finite beta retires the case; summary for the host
__global__ void k_cycle_end(Ctl k, int m) {
    const int c = case_index();
    if (c >= k.n) return;
    const GsLayout L(m);
    double* gs = k.gs + (size_t)c * k.gs_stride;
    int* gi = k.gi + c * GI_STRIDE;
    if (!gi[GI_IDLE]) {
        const double beta = sqrt(gs[L.NRM]);
        gs[L.BETA] = beta;
        if (!isfinite(beta)) { gi[GI_STATUS] = 1; gi[GI_NDONE] = 1; }
    }
    double* s = k.sum + (size_t)c * SUM_STRIDE;
    s[S_BN] = gs[L.BN];
    s[S_BETA] = gs[L.BETA];
    s[S_TOTAL] = gi[GI_TOTAL];
    s[S_MORE] = (!gi[GI_IDLE] && gi[GI_CYC] > 0 && wants_cycle(gi, gs[L.BETA], gs[L.BN], k.step[c].tol_res)) ? 1.0 : 0.0;
}

// GMRES iterations of this Newton step into the case's total
__global__ void k_gm_finish(Ctl k) {
    const int c = case_index();
    if (c >= k.n) return;
    k.sum[(size_t)c * SUM_STRIDE + S_GMRES] += k.gi[c * GI_STRIDE + GI_TOTAL];
}

// ---- chunk-walking vector kernels (every chunk belongs to one case)
struct Vec {
    const int* chunk_case;
    int nchunks;
    const int* gi;
    int flag;   // skip flag
};

#define FR_CHUNKS(vc, ...)                                                                                \
    for (int ch = blockIdx.x; ch < (vc).nchunks; ch += gridDim.x) {                                       \
        const int c = (vc).chunk_case[ch];                                                                 \
        if ((vc).gi[c * GI_STRIDE + (vc).flag]) continue;                                                  \
        for (size_t t = (size_t)ch * CHUNK + threadIdx.x; t < (size_t)(ch + 1) * CHUNK; t += blockDim.x) { \
            __VA_ARGS__                                                                                    \
        }                                                                                                  \
    }

// out = s_c * in, s_c = gs[c * stride + field]; launched with 256 threads
static_assert(CHUNK % (4 * 256) == 0, "k_scale_case covers a chunk in passes of 4 x 256 entries");
__global__ void k_scale_case(Vec vc, const double* __restrict__ in, double* __restrict__ out, const double* gs,
                             int stride, int field) {
    for (int ch = blockIdx.x; ch < vc.nchunks; ch += gridDim.x) {
        const int c = vc.chunk_case[ch];
        if (vc.gi[c * GI_STRIDE + vc.flag]) continue;
        const double a = gs[(size_t)c * stride + field];
        // four entries a pass, loaded before the first store (CHUNK is a multiple of 4 blockDim)
        for (size_t t = (size_t)ch * CHUNK + threadIdx.x; t < (size_t)(ch + 1) * CHUNK; t += 4 * blockDim.x) {
            double x[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k] = in[t + (size_t)k * blockDim.x];
#pragma unroll
            for (int k = 0; k < 4; ++k) out[t + (size_t)k * blockDim.x] = a * x[k];
        }
    }
}

// out = sum_{i < cyc_c} y_c[i] V_i (launched with 256 threads: one per coefficient)
static_assert(MAXV <= 256, "k_combine_case stages one coefficient per thread");
__global__ void k_combine_case(Vec vc, const double* __restrict__ V, size_t ldv, const double* gs, int stride,
                               int yfield, double* __restrict__ out) {
    __shared__ double y[MAXV];
    for (int ch = blockIdx.x; ch < vc.nchunks; ch += gridDim.x) {
        const int c = vc.chunk_case[ch];
        if (vc.gi[c * GI_STRIDE + vc.flag]) continue;
        const int nv = vc.gi[c * GI_STRIDE + GI_CYC];
        __syncthreads();
        if ((int)threadIdx.x < MAXV) y[threadIdx.x] = (int)threadIdx.x < nv ? gs[(size_t)c * stride + yfield + threadIdx.x] : 0.0;
        __syncthreads();
        for (size_t t = (size_t)ch * CHUNK + threadIdx.x; t < (size_t)(ch + 1) * CHUNK; t += blockDim.x) {
            double s = 0.0;
            int i = 0;
            // 16 basis entries loaded before any is used, added in order
            for (; i + 16 <= nv; i += 16) {
                double x[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) x[u] = V[(size_t)(i + u) * ldv + t];
#pragma unroll
                for (int u = 0; u < 16; ++u) s += y[i + u] * x[u];
            }
            for (; i < nv; ++i) s += y[i] * V[i * ldv + t];
            out[t] = s;
        }
    }
}

__global__ void k_add(Vec vc, const double* __restrict__ z, double* __restrict__ x) { FR_CHUNKS(vc, x[t] += z[t];) }
__global__ void k_sub(Vec vc, const double* __restrict__ b, const double* __restrict__ w, double* __restrict__ r) {
    FR_CHUNKS(vc, r[t] = b[t] - w[t];)
}
__global__ void k_fill(Vec vc, double v, double* __restrict__ x) { FR_CHUNKS(vc, x[t] = v;) }
__global__ void k_copy(Vec vc, const double* __restrict__ a, double* __restrict__ b) { FR_CHUNKS(vc, b[t] = a[t];) }

unsigned vgrid(const Solver& sv) { return (unsigned)(sv.nchunks < 8192 ? sv.nchunks : 8192); }
unsigned cgrid(const Solver& sv) { return (unsigned)((sv.n + 63) / 64); }

Ctl ctl(const Solver& sv) { return Ctl{sv.d_gs, sv.gs_stride, sv.d_gi, sv.d_step, sv.d_sum, sv.n}; }
Vec vec(const Solver& sv, int flag) { return Vec{sv.d_chunk_case, sv.nchunks, sv.d_gi, flag}; }

double* wv(const Solver& sv, int i) { return sv.d_w + (size_t)i * sv.Ntot; }

// Newton operator at the iterate whose linearisation packs the Newton loop has written
KArgs bdf_args(const Solver& sv, const double* q) {
    KArgs a{};
    a.q = q; a.cstep = sv.d_step; a.flags = sv.d_gi;
    a.fpack = sv.d_fpack; a.spack = sv.d_spack;
    return a;
}

fr_status bdf_op(const Solver& sv, const double* q, const double* v, double* Av, int flag, hipStream_t s) {
    KArgs a = bdf_args(sv, q);
    a.v = v; a.out = Av; a.flag = flag;
    return solver_fused(sv, MODE_LIN, a, s);
}

// the launches of one cycle (enqueued eagerly or under capture)
fr_status enqueue_cycle(Solver& sv, int m, hipStream_t s) {
    const size_t N = sv.Ntot;
    const GsLayout L(m);
    const double* q = sv.d_q;
    const double* b = wv(sv, WB);
    double* x = wv(sv, WDQ);
    double* r = wv(sv, WRES);
    double* w = wv(sv, WW);
    double* z = wv(sv, WZ);
    double* V = sv.d_V;
    double* gs = sv.d_gs;
    const int gst = sv.gs_stride;
    const Ctl k = ctl(sv);
    hipLaunchKernelGGL(k_cycle_init, dim3(cgrid(sv)), dim3(64), 0, s, k, m);
    FR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scale_case, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_DONE), r, V, gs, gst, L.SCALE0);
    FR_HIP(hipGetLastError());
    for (int j = 0; j < m; ++j) {
        double* vj = V + (size_t)j * N;
        FR_TRY(precond_apply(sv, vj, z, bdf_args(sv, q), sv.d_gi, GI_DONE, s));
        FR_TRY(bdf_op(sv, q, z, w, GI_DONE, s));
        // classical Gram-Schmidt: h = V^T w, w -= V h (and once more when re-orthogonalising)
        FR_TRY(la_krylov(sv, V, N, 0, nullptr, 0, j + 1, w, nullptr, false, false, gs + L.H1, gst, sv.d_gi, GI_DONE, s));
        // each pass over the basis walks its chunks the other way from the pass before it
        if (sv.gs_passes == 2) {
            FR_TRY(la_krylov(sv, V, N, j + 1, gs + L.H1, gst, j + 1, w, w, false, false, gs + L.H2, gst, sv.d_gi,
                             GI_DONE, s, sv.fuse_gs));
            FR_TRY(la_krylov(sv, V, N, j + 1, gs + L.H2, gst, 0, w, w, true, false, nullptr, gst, sv.d_gi,
                             GI_DONE, s, !sv.fuse_gs));
        } else {
            FR_TRY(la_krylov(sv, V, N, j + 1, gs + L.H1, gst, 0, w, w, true, false, nullptr, gst, sv.d_gi,
                             GI_DONE, s, true));
        }
        // |w|^2's second stage and the Givens update in one launch
        hipLaunchKernelGGL(k_norm_givens, dim3(sv.n), dim3(256), 0, s, k, sv.d_case_chunk, sv.d_part, j, m,
                           sv.gs_passes);
        FR_HIP(hipGetLastError());
        if (j + 1 < m) {
            hipLaunchKernelGGL(k_scale_case, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_DONE), w,
                               V + (size_t)(j + 1) * N, gs, gst, L.INVHN);
            FR_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_backsub, dim3(cgrid(sv)), dim3(64), 0, s, k, m);
    FR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_combine_case, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_IDLE), V, N, gs, gst, L.Y, w);
    FR_HIP(hipGetLastError());
    FR_TRY(precond_apply(sv, w, z, bdf_args(sv, q), sv.d_gi, GI_IDLE, s));
    hipLaunchKernelGGL(k_add, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_IDLE), z, x);
    FR_HIP(hipGetLastError());
    FR_TRY(bdf_op(sv, q, x, w, GI_IDLE, s));
    hipLaunchKernelGGL(k_sub, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_IDLE), b, w, r);
    FR_HIP(hipGetLastError());
    FR_TRY(la_krylov(sv, r, N, 0, nullptr, 0, 0, r, nullptr, true, false, gs + L.NRM, gst, sv.d_gi, GI_IDLE, s));
    hipLaunchKernelGGL(k_cycle_end, dim3(cgrid(sv)), dim3(64), 0, s, k, m);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

// ---- Newton-level kernels
__global__ void k_step_init(Ctl k) {
    const int c = case_index();
    if (c >= k.n) return;
    int* gi = k.gi + c * GI_STRIDE;
    for (int f = 0; f < GI_STRIDE; ++f) gi[f] = 0;
    double* s = k.sum + (size_t)c * SUM_STRIDE;
    for (int f = 0; f < SUM_STRIDE; ++f) s[f] = 0.0;
}

// per case: Newton test on the mass-row norm of b (in the NRM slot).  With SER (steady
// solves, paper Eq. SER) the pseudo-time step of this iteration follows from the previous
// one and the residual ratio Res_{m-1}/Res_m, clipped to [dtau_min, dtau_max].
__global__ void k_newton_check(Ctl k, int m, int it) {
    const int c = case_index();
    if (c >= k.n) return;
    int* gi = k.gi + c * GI_STRIDE;
    double* s = k.sum + (size_t)c * SUM_STRIDE;
    if (gi[GI_NDONE]) return;
    const GsLayout L(m);
    const double rr = sqrt(k.gs[(size_t)c * k.gs_stride + L.NRM]);
    if (it == 0) s[S_RES0] = rr;
    s[S_RES] = rr;
    s[S_NEWTON] = it;
    CaseStep& st = k.step[c];
    if (st.ser && st.reject_growth > 0.0 && it > 0 && !st.retry && !(rr <= st.reject_growth * st.res_prev)) {
        // step rejection (not in the paper; off unless requested): the step just taken is undone
        // by k_reject_restore and retried from the same state with a ten times smaller dtau;
        // the case sits out the rest of this iteration and recomputes its residual in the next
        st.dtau *= 0.1;
        st.idt = 1.0 / st.dtau;
        st.retry = 1;
        s[S_DTAU] = st.dtau;
        s[S_REJ] += 1.0;
        gi[GI_REJECT] = 1;
        gi[GI_NDONE] = 1;
        return;
    }
    if (!isfinite(rr)) { gi[GI_STATUS] = 1; gi[GI_NDONE] = 1; return; }
    if (rr <= st.tol_abs || rr <= st.tol_pseudo * s[S_RES0]) { gi[GI_CONV] = 1; gi[GI_NDONE] = 1; return; }
    if (it >= st.max_newton) { gi[GI_STATUS] = 2; gi[GI_NDONE] = 1; return; }
    if (st.ser) {
        if (it > 0 && !st.retry) {
            const double d = st.dtau * pow(st.res_prev / rr, st.r_ser);
            st.dtau = fmax(st.dtau_min, fmin(st.dtau_max, d));
            st.idt = 1.0 / st.dtau;
        }
        st.retry = 0;
        st.res_prev = rr;
        s[S_DTAU] = st.dtau;
    }
}

// q -= dq for the cases whose step k_newton_check undid
__global__ void k_reject_restore(Vec vc, const double* __restrict__ dq, double* __restrict__ q) {
    for (int ch = blockIdx.x; ch < vc.nchunks; ch += gridDim.x) {
        const int c = vc.chunk_case[ch];
        if (!vc.gi[c * GI_STRIDE + GI_REJECT]) continue;
        for (size_t t = (size_t)ch * CHUNK + threadIdx.x; t < (size_t)(ch + 1) * CHUNK; t += blockDim.x) q[t] -= dq[t];
    }
}

// a case whose step was undone takes part again, from its restored state
__global__ void k_retry(Ctl k) {
    const int c = case_index();
    if (c >= k.n) return;
    int* gi = k.gi + c * GI_STRIDE;
    if (gi[GI_REJECT]) { gi[GI_REJECT] = 0; gi[GI_NDONE] = 0; }
}

// a singular block (status 3) takes its case out of the iteration; flags to the summary
__global__ void k_after_factor(Ctl k) {
    const int c = case_index();
    if (c >= k.n) return;
    int* gi = k.gi + c * GI_STRIDE;
    if (gi[GI_STATUS] == 3) gi[GI_NDONE] = 1;
}

__global__ void k_publish(Ctl k) {
    const int c = case_index();
    if (c >= k.n) return;
    const int* gi = k.gi + c * GI_STRIDE;
    double* s = k.sum + (size_t)c * SUM_STRIDE;
    s[S_NDONE] = gi[GI_NDONE] && !gi[GI_REJECT];
    s[S_CONV] = gi[GI_CONV];
    s[S_STATUS] = gi[GI_STATUS];
}

__global__ void k_axpy_case(Vec vc, const double* __restrict__ dq, double* __restrict__ q) {
    FR_CHUNKS(vc, q[t] += dq[t];)
}

}  // namespace

size_t gmres_state_doubles(int m) { return (size_t)GsLayout(m).total; }

void gmres_release(Solver& sv) {
    if (sv.graph_exec) {
        (void)hipGraphExecDestroy((hipGraphExec_t)sv.graph_exec);
        sv.graph_exec = nullptr;
    }
}

// GMRES on every case still in the Newton iteration: A dq = b with b = WB, dq = WDQ
fr_status gmres_device(Solver& sv, int m, int prec, int max_it, hipStream_t s) {
    PhaseRange range("lmfr: GMRES solve");
    const GsLayout L(m);
    const Ctl k = ctl(sv);
    hipLaunchKernelGGL(k_gm_start, dim3(cgrid(sv)), dim3(64), 0, s, k, max_it);
    FR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fill, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_NDONE), 0.0, wv(sv, WDQ));
    FR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_copy, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_NDONE), wv(sv, WB), wv(sv, WRES));
    FR_HIP(hipGetLastError());
    FR_TRY(la_krylov(sv, wv(sv, WB), sv.Ntot, 0, nullptr, 0, 0, wv(sv, WB), nullptr, true, false, sv.d_gs + L.NRM,
                     sv.gs_stride, sv.d_gi, GI_NDONE, s));
    hipLaunchKernelGGL(k_gm_norm0, dim3(cgrid(sv)), dim3(64), 0, s, k, m);
    FR_HIP(hipGetLastError());

    if (sv.precond != 0) {   // the sweeps' work vector exists before any capture
        FR_TRY(dalloc(&sv.d_gst, sv.Ntot));
    }
    const bool graph = sv.use_graph;
    // the operator kernel of a group depends on whether its elements are all affine
    std::vector<char> aff(sv.groups.size());
    for (size_t g = 0; g < sv.groups.size(); ++g) {
        bool all = true;
        for (int id : sv.groups[g].ids) all = all && sv.cs[id]->all_affine;
        aff[g] = all ? 1 : 0;
    }
    if (graph && (!sv.graph_exec || sv.graph_m != m || sv.graph_prec != prec || sv.graph_passes != sv.gs_passes ||
                  sv.graph_precond != sv.precond || sv.graph_cl != (int)sv.inv_colour || sv.graph_aff != aff)) {
        gmres_release(sv);
        // capture one cycle (all buffers are solver-owned; tolerances, time coefficients and
        // caps are read on the device, so the graph depends on m, the block precision and
        // layout, the Gram-Schmidt passes and the preconditioner only)
        hipGraph_t gr;
        FR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        fr_status cst = enqueue_cycle(sv, m, s);
        hipError_t ee = hipStreamEndCapture(s, &gr);
        if (cst != FR_OK) { if (ee == hipSuccess) (void)hipGraphDestroy(gr); return cst; }
        FR_HIP(ee);
        hipGraphExec_t ex;
        hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        FR_HIP(ie);
        sv.graph_exec = ex;
        sv.graph_m = m;
        sv.graph_prec = prec;
        sv.graph_passes = sv.gs_passes;
        sv.graph_precond = sv.precond;
        sv.graph_cl = (int)sv.inv_colour;
        sv.graph_aff = aff;
    }
    double* hs = sv.h_pin;
    for (;;) {
        if (graph) {
            FR_HIP(hipGraphLaunch((hipGraphExec_t)sv.graph_exec, s));
        } else {
            FR_TRY(enqueue_cycle(sv, m, s));
        }
        FR_HIP(hipMemcpyAsync(hs, sv.d_sum, (size_t)sv.n * SUM_STRIDE * sizeof(double), hipMemcpyDeviceToHost, s));
        FR_HIP(hipStreamSynchronize(s));
        bool more = false;
        for (int c = 0; c < sv.n; ++c) more |= hs[(size_t)c * SUM_STRIDE + S_MORE] != 0.0;
        if (!more) break;
    }
    hipLaunchKernelGGL(k_gm_finish, dim3(cgrid(sv)), dim3(64), 0, s, k);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

// The BDF2 (BDF1 for cases without q^{n-1}) dual-time Newton iteration of every case,
// paper Sec. 3.2, Eq. (unsteady_pre_discretized_3): the iterate and Q^n, Q^{n-1} are in
// the solver's vectors (WQN, WQNM1 hold the states on entry; converted here).
fr_status solver_newton(Solver& sv, const fr_step_opts* o, hipStream_t s) {
    PhaseRange range("lmfr: BDF2 step (Newton loop)");
    const Ctl k = ctl(sv);
    const GsLayout L(o->krylov);
    hipLaunchKernelGGL(k_step_init, dim3(cgrid(sv)), dim3(64), 0, s, k);
    FR_HIP(hipGetLastError());
    FR_TRY(launch_cons(sv, sv.d_q, wv(sv, WQN), sv.d_gi, s));
    FR_TRY(launch_cons_nm1(sv, wv(sv, WQNM1), s));
    double* hs = sv.h_pin;
    for (int it = 0;; ++it) {
        PhaseRange it_range("lmfr: Newton iteration");
        if (sv.reject_on) {
            hipLaunchKernelGGL(k_retry, dim3(cgrid(sv)), dim3(64), 0, s, k);
            FR_HIP(hipGetLastError());
        }
        // R at the iterate, and the linearisation packs the GMRES operator reads
        KArgs a{};
        a.q = sv.d_q; a.out = wv(sv, WR); a.flags = sv.d_gi; a.flag = GI_NDONE;
        a.fpack = sv.d_fpack; a.spack = sv.d_spack;
        FR_TRY(solver_fused(sv, MODE_PREP, a, s));
        FR_TRY(launch_bdf_rhs(sv, sv.d_q, wv(sv, WQN), wv(sv, WQNM1), wv(sv, WR), wv(sv, WB), sv.d_gi, s));
        FR_TRY(la_krylov(sv, wv(sv, WB), sv.Ntot, 0, nullptr, 0, 0, wv(sv, WB), nullptr, true, true, sv.d_gs + L.NRM,
                         sv.gs_stride, sv.d_gi, GI_NDONE, s));
        hipLaunchKernelGGL(k_newton_check, dim3(cgrid(sv)), dim3(64), 0, s, k, o->krylov, it);
        FR_HIP(hipGetLastError());
        if (sv.reject_on) {
            hipLaunchKernelGGL(k_reject_restore, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_NDONE), wv(sv, WDQ),
                               sv.d_q);
            FR_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_publish, dim3(cgrid(sv)), dim3(64), 0, s, k);
        FR_HIP(hipGetLastError());
        FR_HIP(hipMemcpyAsync(hs, sv.d_sum, (size_t)sv.n * SUM_STRIDE * sizeof(double), hipMemcpyDeviceToHost, s));
        FR_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int c = 0; c < sv.n; ++c) any |= hs[(size_t)c * SUM_STRIDE + S_NDONE] == 0.0;
        if (!any) break;
        if (it % o->jac_lag == 0) {
            PhaseRange refresh_range("lmfr: preconditioner refresh (enqueue)");
            KArgs b{};
            b.cstep = sv.d_step; b.flags = sv.d_gi; b.flag = GI_NDONE;
            b.fpack = sv.d_fpack; b.spack = sv.d_spack;   // written by this iteration's residual pass
            FR_TRY(launch_block_assembly(sv, sv.d_q, b, s));
            if (sv.keep_blocks) {
                FR_HIP(hipMemcpyAsync(sv.d_blk_keep, sv.d_blk, sv.Btot * sizeof(double), hipMemcpyDeviceToDevice, s));
            }
            FR_TRY(launch_block_invert(sv, o->prec, sv.d_gi, s));
            hipLaunchKernelGGL(k_after_factor, dim3(cgrid(sv)), dim3(64), 0, s, k);
            FR_HIP(hipGetLastError());
        }
        FR_TRY(gmres_device(sv, o->krylov, o->prec, o->max_lin_it, s));
        hipLaunchKernelGGL(k_axpy_case, dim3(vgrid(sv)), dim3(256), 0, s, vec(sv, GI_NDONE), wv(sv, WDQ), sv.d_q);
        FR_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_publish, dim3(cgrid(sv)), dim3(64), 0, s, k);
    FR_HIP(hipGetLastError());
    FR_HIP(hipMemcpyAsync(hs, sv.d_sum, (size_t)sv.n * SUM_STRIDE * sizeof(double), hipMemcpyDeviceToHost, s));
    FR_HIP(hipStreamSynchronize(s));
    return FR_OK;
}
