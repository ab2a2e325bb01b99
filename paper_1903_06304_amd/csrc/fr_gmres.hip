// Restarted, right-preconditioned FP64 GMRES(m) with its small dense state on the device.
//
// One restart cycle is a fixed sequence of launches:
//   cycle init (g = beta e1, V_0 = r / beta) |
//   m x [ z = P^-1 V_j ; w = A z ; classical Gram-Schmidt twice (3 streaming passes) ;
//         Givens update of column j and of g, convergence test ; V_{j+1} = w / h_{j+1,j} ] |
//   y = H^-1 g ; x += P^-1 (V y) ; r = b - A x ; beta = |r|
// The Givens kernel raises a device flag when |g_{j+1}| <= tol |b| (or on breakdown or
// the iteration cap); every later launch of the cycle reads the flag and returns at once.
// The sequence therefore contains no host decision and is captured once into a hipGraph
// and replayed; the host synchronises once per cycle to read beta and the counters.
#include <cmath>
#include <cstring>

#include "fr_internal.hpp"

namespace {

// layout of d_gs (doubles) for restart length m
struct GsLayout {
    int m, H, CS, SN, G, Y, H1, H2, NRM, BN, BETA, INVHN, SCALE0, total;
    explicit GsLayout(int m_) : m(m_) {
        H = 0;
        CS = H + (m + 1) * m;
        SN = CS + m;
        G = SN + m;
        Y = G + m + 1;
        H1 = Y + m;
        H2 = H1 + 64;
        NRM = H2 + 64;
        BN = NRM + 64;
        BETA = BN + 1;
        INVHN = BETA + 1;
        SCALE0 = INVHN + 1;
        total = SCALE0 + 1;
    }
};
enum { GI_DONE = 0, GI_CYC, GI_TOTAL, GI_MAXIT, GI_TOTAL_INT };

// g = beta e1, counters of the cycle reset, scale of V_0
__global__ void k_cycle_init(int m, double* gs, int* gi, GsLayout L) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double beta = gs[L.BETA];
    for (int i = 0; i <= m; ++i) gs[L.G + i] = 0.0;
    gs[L.G] = beta;
    gs[L.SCALE0] = beta > 0.0 ? 1.0 / beta : 0.0;
    gi[GI_CYC] = 0;
    gi[GI_DONE] = (beta > 0.0 && gi[GI_TOTAL] < gi[GI_MAXIT]) ? 0 : 1;
}

// column j of the Hessenberg matrix, Givens rotations, convergence flag
__global__ void k_givens(int j, int m, double tol, double* gs, int* gi, GsLayout L) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (gi[GI_DONE]) return;
    double* H = gs + L.H;
    double* cs = gs + L.CS;
    double* sn = gs + L.SN;
    double* g = gs + L.G;
    for (int i = 0; i <= j; ++i) H[i * m + j] = gs[L.H1 + i] + gs[L.H2 + i];
    const double hn = sqrt(gs[L.NRM]);
    H[(j + 1) * m + j] = hn;
    for (int i = 0; i < j; ++i) {
        const double a0 = H[i * m + j], a1 = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a0 + sn[i] * a1;
        H[(i + 1) * m + j] = -sn[i] * a0 + cs[i] * a1;
    }
    const double a0 = H[j * m + j], a1 = H[(j + 1) * m + j];
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
    const bool conv = fabs(g[j + 1]) <= tol * gs[L.BN];
    if (conv || !(hn > 0.0) || !isfinite(hn) || gi[GI_TOTAL] >= gi[GI_MAXIT] || j == m - 1) gi[GI_DONE] = 1;
}

// y = H^-1 g on the iterations of this cycle
__global__ void k_backsub(int m, double* gs, const int* gi, GsLayout L) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int jd = gi[GI_CYC];
    const double* H = gs + L.H;
    double* y = gs + L.Y;
    for (int i = jd - 1; i >= 0; --i) {
        double s = gs[L.G + i];
        for (int k = i + 1; k < jd; ++k) s -= H[i * m + k] * y[k];
        y[i] = s / H[i * m + i];
    }
    for (int i = jd; i < m; ++i) y[i] = 0.0;
}

// out = scale * in, scale read on the device; skipped when *skip != 0
__global__ void k_scale_dev(size_t N, const double* __restrict__ in, double* __restrict__ out, const double* scale,
                            const int* skip) {
    if (skip && *skip) return;
    const double a = *scale;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x)
        out[t] = a * in[t];
}

// out = sum_{i < count} y_i V_i
__global__ void k_combine_dev(size_t N, const double* __restrict__ V, size_t ldv, const double* __restrict__ y,
                              const int* count, double* __restrict__ out) {
    const int nv = *count;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < nv; ++i) s += y[i] * V[i * ldv + t];
        out[t] = s;
    }
}

// x += z ; r = b - w
__global__ void k_add(size_t N, const double* __restrict__ z, double* __restrict__ x) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x)
        x[t] += z[t];
}
__global__ void k_sub(size_t N, const double* __restrict__ b, const double* __restrict__ w, double* __restrict__ r) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x)
        r[t] = b[t] - w[t];
}
__global__ void k_fill(size_t N, double v, double* __restrict__ x) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x)
        x[t] = v;
}
// beta = sqrt(|r|^2) (and bn = beta on the first call of a solve)
__global__ void k_sqrt_to(const double* in, double* beta, double* bn) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double b = sqrt(*in);
    *beta = b;
    if (bn) *bn = b;
}
__global__ void k_set_int(int* p, int v0, int v1, int v2, int v3) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    p[0] = v0; p[1] = v1; p[2] = v2; p[3] = v3;
}

unsigned gridN(size_t N) {
    size_t g = (N + 255) / 256;
    if (g > 4096) g = 4096;
    return (unsigned)(g < 1 ? 1 : g);
}

// work vectors of the solve inside d_w
enum { WR = 4, WW = 5, WZ = 6 };

fr_status bdf_op(fr_ctx c, const double* q, const double* v, double ct, double idt, double* Av, const int* skip,
                 hipStream_t s) {
    KArgs a{};
    a.E = c->E; a.q = q; a.v = v; a.out = Av; a.c_time = ct; a.inv_dtau = idt; a.skip = skip;
    return launch_residual(c, MODE_AOP, a, s);
}

// the launches of one cycle (enqueued eagerly or under capture)
fr_status enqueue_cycle(fr_ctx c, const double* q, const double* b, double* x, int m, double tol, double ct,
                        double idt, hipStream_t s) {
    const size_t N = c->N();
    const GsLayout L(m);
    double* V = c->d_V;
    double* r = c->d_w + (size_t)WR * N;
    double* w = c->d_w + (size_t)WW * N;
    double* z = c->d_w + (size_t)WZ * N;
    double* gs = c->d_gs;
    int* gi = c->d_gi;
    const int* done = gi + GI_DONE;
    hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(64), 0, s, m, gs, gi, L);
    FR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scale_dev, dim3(gridN(N)), dim3(256), 0, s, N, r, V, gs + L.SCALE0, done);
    FR_HIP(hipGetLastError());
    for (int j = 0; j < m; ++j) {
        double* vj = V + (size_t)j * N;
        fr_status st;
        if ((st = launch_block_apply(c, vj, z, s, done)) != FR_OK) return st;
        if ((st = bdf_op(c, q, z, ct, idt, w, done, s)) != FR_OK) return st;
        if ((st = la_krylov(c, N, V, 0, nullptr, j + 1, w, nullptr, false, gs + L.H1, s, done)) != FR_OK) return st;
        if ((st = la_krylov(c, N, V, j + 1, gs + L.H1, j + 1, w, w, false, gs + L.H2, s, done)) != FR_OK) return st;
        if ((st = la_krylov(c, N, V, j + 1, gs + L.H2, 0, w, w, true, gs + L.NRM, s, done)) != FR_OK) return st;
        hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, j, m, tol, gs, gi, L);
        FR_HIP(hipGetLastError());
        if (j + 1 < m) {
            hipLaunchKernelGGL(k_scale_dev, dim3(gridN(N)), dim3(256), 0, s, N, w, V + (size_t)(j + 1) * N,
                               gs + L.INVHN, done);
            FR_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_backsub, dim3(1), dim3(64), 0, s, m, gs, gi, L);
    FR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_combine_dev, dim3(gridN(N)), dim3(256), 0, s, N, V, N, gs + L.Y, gi + GI_CYC, w);
    FR_HIP(hipGetLastError());
    fr_status st;
    if ((st = launch_block_apply(c, w, z, s, nullptr)) != FR_OK) return st;
    hipLaunchKernelGGL(k_add, dim3(gridN(N)), dim3(256), 0, s, N, z, x);
    FR_HIP(hipGetLastError());
    if ((st = bdf_op(c, q, x, ct, idt, w, nullptr, s)) != FR_OK) return st;
    hipLaunchKernelGGL(k_sub, dim3(gridN(N)), dim3(256), 0, s, N, b, w, r);
    FR_HIP(hipGetLastError());
    if ((st = la_krylov(c, N, r, 0, nullptr, 0, r, nullptr, true, gs + L.NRM, s, nullptr)) != FR_OK) return st;
    hipLaunchKernelGGL(k_sqrt_to, dim3(1), dim3(64), 0, s, gs + L.NRM, gs + L.BETA, (double*)nullptr);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

}  // namespace

void gmres_release(fr_ctx c) {
    if (c->graph_exec) {
        (void)hipGraphExecDestroy((hipGraphExec_t)c->graph_exec);
        c->graph_exec = nullptr;
    }
}

fr_status gmres_device(fr_ctx c, const double* q, const double* b, double* x, int m, double tol, int max_it,
                       double ct, double idt, int prec, GmresResult& out, hipStream_t s) {
    const size_t N = c->N();
    const GsLayout L(m);
    double* gs = c->d_gs;
    int* gi = c->d_gi;
    double* r = c->d_w + (size_t)WR * N;
    // x = 0, r = b, beta = bn = |b|, counters
    hipLaunchKernelGGL(k_fill, dim3(gridN(N)), dim3(256), 0, s, N, 0.0, x);
    FR_HIP(hipGetLastError());
    FR_HIP(hipMemcpyAsync(r, b, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    fr_status st = la_krylov(c, N, b, 0, nullptr, 0, b, nullptr, true, gs + L.NRM, s, nullptr);
    if (st != FR_OK) return st;
    hipLaunchKernelGGL(k_sqrt_to, dim3(1), dim3(64), 0, s, gs + L.NRM, gs + L.BETA, gs + L.BN);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, gi, 0, 0, 0, max_it);
    FR_HIP(hipGetLastError());

    const bool graph = c->use_graph;
    if (graph && (!c->graph_exec || c->graph_m != m || c->graph_ct != ct || c->graph_idt != idt ||
                  c->graph_prec != prec || c->graph_tol != tol)) {
        gmres_release(c);
        // capture one cycle (all buffers are context-owned; the key is what the launches bake in)
        hipGraph_t gr;
        FR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        fr_status cst = enqueue_cycle(c, q, b, x, m, tol, ct, idt, s);
        hipError_t ee = hipStreamEndCapture(s, &gr);
        if (cst != FR_OK) { if (ee == hipSuccess) (void)hipGraphDestroy(gr); return cst; }
        FR_HIP(ee);
        hipGraphExec_t ex;
        hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        FR_HIP(ie);
        c->graph_exec = ex;
        c->graph_m = m; c->graph_ct = ct; c->graph_idt = idt; c->graph_prec = prec;
        c->graph_tol = tol;
    }
    out.its = 0;
    out.rel = 0.0;
    for (int cycle = 0;; ++cycle) {
        if (graph) {
            FR_HIP(hipGraphLaunch((hipGraphExec_t)c->graph_exec, s));
        } else {
            st = enqueue_cycle(c, q, b, x, m, tol, ct, idt, s);
            if (st != FR_OK) return st;
        }
        FR_HIP(hipMemcpyAsync(c->h_scal + 2048, gs + L.BN, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        FR_HIP(hipMemcpyAsync(c->h_scal + 2052, gi, GI_TOTAL_INT * sizeof(int), hipMemcpyDeviceToHost, s));
        FR_HIP(hipStreamSynchronize(s));
        const double bn = c->h_scal[2048], beta = c->h_scal[2049];
        int ic[GI_TOTAL_INT];
        memcpy(ic, c->h_scal + 2052, sizeof(ic));
        out.its = ic[GI_TOTAL];
        out.rel = bn > 0.0 ? beta / bn : 0.0;
        if (!std::isfinite(beta)) { fr_set_error("non-finite GMRES residual"); return FR_ENONFINITE; }
        if (bn == 0.0 || beta <= tol * bn || ic[GI_TOTAL] >= max_it || ic[GI_CYC] == 0) break;
    }
    return FR_OK;
}

size_t gmres_state_doubles(int m) { return (size_t)GsLayout(m).total; }
