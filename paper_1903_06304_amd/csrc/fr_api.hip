// C ABI of the lmfr library: context, operator tables, residual / JVP / VJP entry
// points, the element-block-Jacobi preconditioner, the BDF2 dual-time Newton step, and
// batches of cases advanced together.  A context's own entry points run through its
// one-case solver; a batch is a solver over many contexts.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fr_internal.hpp"

// ----------------------------------------------------------------------------- errors
static thread_local std::string g_err;
void fr_set_error(const std::string& s) { g_err = s; }
extern "C" const char* fr_last_error(void) { return g_err.c_str(); }

static fr_status bad(const char* msg) { fr_set_error(msg); return FR_EINVAL; }

// ----------------------------------------------------------------------------- 1-D tables
namespace {

// Legendre P_n and P_n' at x (three-term recurrence)
void leg(int nn, double x, double& P, double& dP) {
    double a = 1.0, b = x;
    if (nn == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 2; k <= nn; ++k) { double c = ((2 * k - 1) * x * b - (k - 1) * a) / k; a = b; b = c; }
    P = b;
    dP = nn * (x * b - a) / (x * x - 1.0);
}

// Gauss-Legendre points (Newton from Chebyshev guesses) and weights
void gl_nodes(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n); w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = -std::cos(M_PI * (2 * i + 1) / (2.0 * n));
        for (int it = 0; it < 60; ++it) {
            double P, dP; leg(n, z, P, dP);
            double dz = P / dP; z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        double P, dP; leg(n, z, P, dP);
        x[i] = z; w[i] = 2.0 / ((1.0 - z * z) * dP * dP);
    }
}

// Gauss-Lobatto points: +-1 and the roots of P'_{m-1} (Newton on P'_{m-1})
void gll_nodes(int m, std::vector<double>& x) {
    x.resize(m);
    x[0] = -1.0; x[m - 1] = 1.0;
    const int N = m - 1;
    for (int i = 1; i < N; ++i) {
        double z = -std::cos(M_PI * i / N);
        for (int it = 0; it < 60; ++it) {
            double P, dP; leg(N, z, P, dP);
            // (1 - z^2) P'' = 2 z P' - N (N+1) P
            double d2P = (2.0 * z * dP - N * (N + 1) * P) / (1.0 - z * z);
            double dz = dP / d2P; z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[i] = z;
    }
}

// barycentric weights of a node set
std::vector<double> bary(const std::vector<double>& x) {
    std::vector<double> b(x.size(), 1.0);
    for (size_t a = 0; a < x.size(); ++a)
        for (size_t m = 0; m < x.size(); ++m)
            if (m != a) b[a] /= (x[a] - x[m]);
    return b;
}

// Lagrange values and derivatives of the basis on nodes x at point z
void lag_eval(const std::vector<double>& x, const std::vector<double>& bw, double z, double* L, double* dL) {
    const int n = (int)x.size();
    for (int a = 0; a < n; ++a) {
        if (z == x[a]) {
            // z is a node: values are a Kronecker delta, derivatives the differentiation row
            for (int c = 0; c < n; ++c) L[c] = (c == a) ? 1.0 : 0.0;
            double diag = 0.0;
            for (int c = 0; c < n; ++c) {
                if (c == a) continue;
                dL[c] = (bw[c] / bw[a]) / (x[a] - x[c]);
                diag -= dL[c];
            }
            dL[a] = diag;
            return;
        }
    }
    double den = 0.0;
    for (int a = 0; a < n; ++a) den += bw[a] / (z - x[a]);
    for (int a = 0; a < n; ++a) {
        L[a] = (bw[a] / (z - x[a])) / den;
        double s = 0.0;
        for (int m = 0; m < n; ++m) if (m != a) s += 1.0 / (z - x[m]);
        dL[a] = L[a] * s;
    }
}

void build_tables(fr_ctx c) {
    const int n = c->n, m = c->m;
    std::vector<double> x, w;
    gl_nodes(n, x, w);
    std::vector<double> bw = bary(x);
    memset(&c->op, 0, sizeof(OpTab));
    double L[FR_MAXN], dL[FR_MAXN];
    for (int i = 0; i < n; ++i) {
        lag_eval(x, bw, x[i], L, dL);
        for (int a = 0; a < n; ++a) c->op.D[i * n + a] = dL[a];
    }
    lag_eval(x, bw, -1.0, L, dL);
    for (int a = 0; a < n; ++a) { c->op.lamL[a] = L[a]; c->op.dlamL[a] = dL[a]; }
    lag_eval(x, bw, 1.0, L, dL);
    for (int a = 0; a < n; ++a) { c->op.lamR[a] = L[a]; c->op.dlamR[a] = dL[a]; }
    // Radau correction functions (g_L right Radau, g_R left Radau) have nodal slopes
    // -l_i(-1)/w_i and l_i(+1)/w_i on the Gauss-Legendre points
    for (int i = 0; i < n; ++i) {
        c->op.gamL[i] = -c->op.lamL[i] / w[i];
        c->op.gamR[i] = c->op.lamR[i] / w[i];
    }
    // geometry basis on Gauss-Lobatto nodes of degree m-1
    std::vector<double> g;
    gll_nodes(m, g);
    std::vector<double> gb = bary(g);
    memset(&c->gt, 0, sizeof(GeoTab));
    c->gt.m = m;
    for (int i = 0; i < n; ++i) {
        lag_eval(g, gb, x[i], L, dL);
        for (int a = 0; a < m; ++a) { c->gt.Ls[i * m + a] = L[a]; c->gt.dLs[i * m + a] = dL[a]; }
    }
    lag_eval(g, gb, -1.0, L, dL);
    for (int a = 0; a < m; ++a) c->gt.dLm[a] = dL[a];
    lag_eval(g, gb, 1.0, L, dL);
    for (int a = 0; a < m; ++a) c->gt.dLp[a] = dL[a];
}

}  // namespace

// ----------------------------------------------------------------------------- context
extern "C" fr_status fr_create(const fr_params* prm, const int32_t* h_nbr, const int32_t* h_nbr_face,
                               const int8_t* h_flip, fr_ctx* out) {
    if (!prm || !h_nbr || !h_nbr_face || !out) return bad("fr_create: null argument");
    *out = nullptr;
    if (prm->order < 1 || prm->order > 4 || prm->geom_order < 1 || prm->geom_order > 4) {
        fr_set_error("fr_create: order and geom_order must be in 1..4");
        return FR_EUNSUPPORTED;
    }
    if (prm->n_elem <= 0 || prm->n_elem >= (1 << 27)) return bad("fr_create: n_elem out of range");
    {
        // kernels index state arrays with 32-bit offsets: 4 * n_elem * (p+1)^2 < 2^31; the fused
        // kernels form the byte offset of a per-field point index (solution or flux point) in
        // 32 bits: 8 * n_elem * max((p+1)^2, 4(p+1)) < 2^32
        const long long np1 = prm->order + 1;
        if (4LL * prm->n_elem * np1 * np1 >= (1LL << 31)) return bad("fr_create: state arrays above 2^31 entries");
        const long long npt = np1 * np1 > 4 * np1 ? np1 * np1 : 4 * np1;
        if (8LL * prm->n_elem * npt >= (1LL << 32)) return bad("fr_create: flux-point arrays above 2^32 bytes");
    }
    if (!(prm->gamma > 1.0) || !(prm->mach_ref > 0.0) || !(prm->prandtl > 0.0) || !(prm->mach_inf >= 0.0) ||
        !(prm->kappa >= 0.0))
        return bad("fr_create: invalid physical parameters");
    if (prm->viscous && !(prm->reynolds > 0.0)) return bad("fr_create: reynolds must be positive");
    const int E = prm->n_elem;
    std::vector<int32_t> packed((size_t)E * 4), bcode((size_t)E, 0);
    bool any_bc = false, any_far = false;
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f) {
            const int nb = h_nbr[e * 4 + f];
            if (nb < 0) {
                // boundary face: its kind in the element's code, the element itself as the
                // (unused) neighbour so that every gather stays in bounds
                if (nb < FR_BC_NOSLIP_WALL) return bad("fr_create: unknown boundary code");
                const int kind = -nb;
                static_assert(-FR_BC_FARFIELD == BC_FARFIELD && -FR_BC_SLIP_WALL == BC_SLIP &&
                              -FR_BC_NOSLIP_WALL == BC_WALL, "boundary codes");
                bcode[e] |= kind << (2 * f);
                any_bc = true;
                any_far = any_far || kind == BC_FARFIELD;
                packed[(size_t)e * 4 + f] = e * 8 + f * 2;
                continue;
            }
            const int nf = h_nbr_face[e * 4 + f];
            const int fl = h_flip ? (h_flip[e * 4 + f] != 0) : 0;
            if (nb < 0 || nb >= E || nf < 0 || nf > 3) return bad("fr_create: neighbour table out of range");
            if (h_nbr[nb * 4 + nf] != e || h_nbr_face[nb * 4 + nf] != f)
                return bad("fr_create: neighbour table is not symmetric");
            if (nb == e && nf == f) return bad("fr_create: a face cannot neighbour itself");
            packed[(size_t)e * 4 + f] = nb * 8 + nf * 2 + fl;
        }
    // colours of the Gauss-Seidel sweeps: in element order, the smallest colour no face
    // neighbour has yet (a checkerboard on even periodic meshes; at most 5 colours)
    std::vector<int32_t> colour((size_t)E, -1);
    int ncol = 0;
    for (int e = 0; e < E; ++e) {
        bool used[5] = {false, false, false, false, false};
        for (int f = 0; f < 4; ++f) {
            const int nb = h_nbr[e * 4 + f];
            if (nb >= 0 && nb != e && colour[nb] >= 0) used[colour[nb]] = true;
        }
        int k = 0;
        while (used[k]) ++k;
        colour[e] = k;
        ncol = k + 1 > ncol ? k + 1 : ncol;
    }
    // the elements sorted by colour: the Gauss-Seidel sweeps run over one colour at a time
    std::vector<int32_t> corder;
    corder.reserve((size_t)E);
    std::array<int, 6> cofs{};
    for (int k = 0; k < ncol; ++k) {
        cofs[k] = (int)corder.size();
        for (int e = 0; e < E; ++e)
            if (colour[e] == k) corder.push_back(e);
    }
    for (int k = ncol; k < 6; ++k) cofs[k] = E;
    fr_ctx c = new fr_ctx_s();
    c->prm = *prm;
    c->ncolors = ncol;
    c->cofs = cofs;
    c->p = prm->order; c->n = c->p + 1; c->Np = c->n * c->n;
    c->pg = prm->geom_order; c->m = c->pg + 1; c->E = E;
    const double g = prm->gamma, Ma = prm->mach_ref;
    PhysConst& pc = c->pc;
    pc.gam = g;
    pc.Rg = 1.0 / (g * Ma * Ma);
    pc.Cp = 1.0 / ((g - 1.0) * Ma * Ma);
    pc.inv_gm1 = 1.0 / (g - 1.0);
    pc.gRg = g * pc.Rg;
    pc.inv_Cp = 1.0 / pc.Cp;
    pc.inv_Rg = 1.0 / pc.Rg;
    pc.mu_re = prm->viscous ? prm->mu / prm->reynolds : 0.0;
    pc.kc_re = prm->viscous ? prm->mu * pc.Cp / prm->prandtl / prm->reynolds : 0.0;
    pc.eps_min = prm->kappa * prm->mach_inf;
    pc.br2 = 0.5 * c->n * c->n;
    build_tables(c);
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; fr_set_error("no HIP device"); return FR_EHIP; }
    const size_t EN = (size_t)E * c->Np, FE = (size_t)E * 4 * c->n;
    fr_status st = FR_OK;
    if ((st = dalloc(&c->d_nbr, (size_t)E * 4)) != FR_OK ||
        (st = dalloc(&c->d_gsp, NGSP * EN)) != FR_OK ||
        (st = dalloc(&c->d_gfp, NGFP * FE)) != FR_OK ||
        (st = dalloc(&c->d_aff, (size_t)E)) != FR_OK ||
        (st = dalloc(&c->d_color, (size_t)E)) != FR_OK ||
        (st = dalloc(&c->d_corder, (size_t)E)) != FR_OK ||
        (st = dalloc(&c->d_trace, FE * 10)) != FR_OK ||
        (st = dalloc(&c->d_vj, FE * 10)) != FR_OK ||
        (st = dalloc(&c->d_qinf, (size_t)4)) != FR_OK ||
        (any_bc && (st = dalloc(&c->d_bc, (size_t)E)) != FR_OK)) {
        fr_destroy(c);
        return st;
    }
    c->has_farfield = any_far;
    if (any_bc && hipMemcpy(c->d_bc, bcode.data(), bcode.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        fr_destroy(c);
        fr_set_error("copy of the boundary codes failed");
        return FR_EHIP;
    }
    if (hipMemcpy(c->d_nbr, packed.data(), packed.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_color, colour.data(), colour.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_corder, corder.data(), corder.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        fr_destroy(c);
        fr_set_error("copy of the neighbour table failed");
        return FR_EHIP;
    }
    c->self = new Solver();
    if ((st = solver_init(*c->self, &c, 1)) != FR_OK) {
        fr_destroy(c);
        return st;
    }
    *out = c;
    return FR_OK;
}

extern "C" void fr_destroy(fr_ctx c) {
    if (!c) return;
    if (c->self) { solver_free(*c->self); delete c->self; }
    dfree(c->d_nbr); dfree(c->d_gsp); dfree(c->d_gfp); dfree(c->d_aff); dfree(c->d_color); dfree(c->d_corder); dfree(c->d_trace);
    dfree(c->d_vj); dfree(c->d_bc); dfree(c->d_qinf);
    delete c;
}

static bool is_tile_option(const char* name);
static fr_status set_tile_option(Solver& sv, const char* name, int64_t value);

static bool is_tile_option(const char* name) {
    return !strcmp(name, "tile_lanes") || !strcmp(name, "tile_grid") || !strcmp(name, "tile_xcd");
}

// solver options shared by contexts and batches; returns FR_EINVAL with no message for
// names it does not know
static fr_status solver_option(Solver& sv, const char* name, int64_t value) {
    if (!strcmp(name, "graph")) { sv.use_graph = value != 0; gmres_release(sv); return FR_OK; }
    if (!strcmp(name, "gram_schmidt")) {
        if (value != 1 && value != 2) return bad("gram_schmidt must be 1 or 2");
        sv.gs_passes = (int)value;
        gmres_release(sv);
        return FR_OK;
    }
    if (!strcmp(name, "fused_gram_schmidt")) { sv.fuse_gs = value != 0; gmres_release(sv); return FR_OK; }
    if (!strcmp(name, "preconditioner")) {
        if (value < 0 || value > 2)
            return bad("preconditioner must be 0 (block Jacobi), 1 (symmetric block Gauss-Seidel) or 2 (forward block Gauss-Seidel)");
        if (value != 0) {   // the sweeps apply the Newton operator through the linearisation packs
            FR_TRY(dalloc(&sv.d_fpack, sv.fpack_len));
            FR_TRY(dalloc(&sv.d_spack, sv.spack_len));
            FR_TRY(dalloc(&sv.d_rscratch, sv.Ntot));
        }
        sv.precond = (int)value;
        gmres_release(sv);
        return FR_OK;
    }
    if (is_tile_option(name)) return set_tile_option(sv, name, value);
    fr_set_error(std::string("unknown option ") + name);
    return FR_EINVAL;
}

// manual launch shape of every group and mode of a solver
static fr_status set_tile_option(Solver& sv, const char* name, int64_t value) {
    if (value < 0 || value > (1 << 24)) return bad("tile option out of range");
    if (!strcmp(name, "tile_lanes") && value != 0 && value != 64 && value != 128 && value != 256)
        return bad("tile_lanes must be 0, 64, 128 or 256");
    for (Group& g : sv.groups)
        for (int m = 0; m < NMODES; ++m) {
            Tune& t = g.tune[m];
            const bool dual = m != MODE_R;   // only the residual is built with 256 lanes
            if (!strcmp(name, "tile_lanes")) t.lanes = (dual && value == 256) ? 128 : (int)value;
            else if (!strcmp(name, "tile_grid")) t.grid = (int)value;
            else t.xcd = value != 0;
        }
    gmres_release(sv);
    return FR_OK;
}

extern "C" fr_status fr_set_option(fr_ctx c, const char* name, int64_t value) {
    if (!c || !name) return bad("fr_set_option: null argument");
    Solver& sv = *c->self;
    if (!strcmp(name, "keep_blocks")) { sv.keep_blocks = value != 0; return FR_OK; }
    if (!strcmp(name, "operator_packs")) {
        if (value) {
            FR_TRY(dalloc(&sv.d_fpack, sv.fpack_len));
            FR_TRY(dalloc(&sv.d_spack, sv.spack_len));
            FR_TRY(dalloc(&sv.d_rscratch, sv.Ntot));
        }
        sv.op_packs = value != 0;
        return FR_OK;
    }
    return solver_option(sv, name, value);
}

extern "C" fr_status fr_set_geometry(fr_ctx c, const double* xg, const double* vg, void* stream) {
    if (!c || !xg) return bad("fr_set_geometry: null argument");
    if (c->prm.moving && !vg) return bad("fr_set_geometry: moving mesh needs grid velocities");
    FR_TRY(launch_geometry(c, xg, c->prm.moving ? vg : nullptr, (hipStream_t)stream));
    // whether every element is affine decides the residual kernel variant: read the flags back
    std::vector<int32_t> h((size_t)c->E);
    FR_HIP(hipMemcpyAsync(h.data(), c->d_aff, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, (hipStream_t)stream));
    FR_HIP(hipStreamSynchronize((hipStream_t)stream));
    bool all = true;
    for (int32_t x : h) all = all && x != 0;
    c->all_affine = all;
    c->geometry_set = true;
    return FR_OK;
}

extern "C" fr_status fr_set_farfield(fr_ctx c, const double* h_qinf) {
    if (!c || !h_qinf) return bad("fr_set_farfield: null argument");
    for (int r = 0; r < 4; ++r)
        if (!std::isfinite(h_qinf[r])) return bad("fr_set_farfield: non-finite state");
    if (!(h_qinf[0] > 0.0) || !(h_qinf[3] > 0.0)) return bad("fr_set_farfield: p and T must be positive");
    FR_HIP(hipMemcpy(c->d_qinf, h_qinf, 4 * sizeof(double), hipMemcpyHostToDevice));
    c->farfield_set = true;
    return FR_OK;
}

static fr_status ready(fr_ctx c) {
    if (!c) return bad("null context");
    if (const char* m = ctx_not_ready(c)) return bad(m);
    return FR_OK;
}

static KArgs plain_args(const double* q, const double* v, double* out, double* out2) {
    KArgs a{};
    a.q = q; a.v = v; a.out = out; a.out2 = out2;
    return a;
}

extern "C" fr_status fr_residual(fr_ctx c, const double* q, double* R, void* stream) {
    FR_TRY(ready(c));
    if (!q || !R) return bad("fr_residual: null argument");
    return solver_fused(*c->self, MODE_R, plain_args(q, nullptr, R, nullptr), (hipStream_t)stream);
}

extern "C" fr_status fr_jvp(fr_ctx c, const double* q, const double* v, double* Jv, double* R_or_null, void* stream) {
    FR_TRY(ready(c));
    if (!q || !v || !Jv) return bad("fr_jvp: null argument");
    return solver_fused(*c->self, MODE_JVP, plain_args(q, v, Jv, R_or_null), (hipStream_t)stream);
}

extern "C" fr_status fr_bdf_operator(fr_ctx c, const double* q, const double* v, double c_time, double inv_dtau,
                                     double* Av, void* stream) {
    FR_TRY(ready(c));
    if (!q || !v || !Av) return bad("fr_bdf_operator: null argument");
    Solver& sv = *c->self;
    KArgs a = plain_args(q, v, Av, nullptr);
    a.c_time = c_time; a.inv_dtau = inv_dtau;
    if (!sv.op_packs) return solver_fused(sv, MODE_AOP, a, (hipStream_t)stream);
    // linearisation packs of q (R into the scratch vector), then the tangent-only operator
    KArgs p = plain_args(q, nullptr, sv.d_rscratch, nullptr);
    p.fpack = sv.d_fpack; p.spack = sv.d_spack;
    FR_TRY(solver_fused(sv, MODE_PREP, p, (hipStream_t)stream));
    a.fpack = sv.d_fpack; a.spack = sv.d_spack;
    return solver_fused(sv, MODE_LIN, a, (hipStream_t)stream);
}

extern "C" fr_status fr_vjp(fr_ctx c, const double* q, const double* w, double* JTw, void* stream) {
    FR_TRY(ready(c));
    if (!q || !w || !JTw) return bad("fr_vjp: null argument");
    return launch_vjp(c, q, w, JTw, (hipStream_t)stream);
}

extern "C" fr_status fr_block_jacobi_factor(fr_ctx c, const double* q, double c_time, double inv_dtau, int32_t prec,
                                            void* stream) {
    FR_TRY(ready(c));
    if (!q) return bad("fr_block_jacobi_factor: null argument");
    if (prec < FR_FP64 || prec > FR_BF16) return bad("fr_block_jacobi_factor: unknown precision");
    Solver& sv = *c->self;
    hipStream_t s = (hipStream_t)stream;
    FR_TRY(solver_ensure_blocks(sv, prec));
    KArgs a{};
    a.c_time = c_time; a.inv_dtau = inv_dtau;
    sv.f_ct = c_time; sv.f_idt = inv_dtau;
    if (sv.op_packs || sv.precond != 0) {
        // linearisation packs of q, then tangent-only block columns
        KArgs p = plain_args(q, nullptr, sv.d_rscratch, nullptr);
        p.fpack = sv.d_fpack; p.spack = sv.d_spack;
        FR_TRY(solver_fused(sv, MODE_PREP, p, s));
        a.fpack = sv.d_fpack; a.spack = sv.d_spack;
    }
    FR_TRY(launch_block_assembly(sv, q, a, s));
    if (sv.keep_blocks) FR_HIP(hipMemcpyAsync(sv.d_blk_keep, sv.d_blk, sv.Btot * sizeof(double), hipMemcpyDeviceToDevice, s));
    // a zero pivot marks the case status; reading it synchronises once per refresh
    FR_HIP(hipMemsetAsync(sv.d_gi, 0, GI_STRIDE * sizeof(int), s));
    FR_TRY(launch_block_invert(sv, prec, nullptr, s));
    int* flags = reinterpret_cast<int*>(sv.h_pin);
    FR_HIP(hipMemcpyAsync(flags, sv.d_gi, GI_STRIDE * sizeof(int), hipMemcpyDeviceToHost, s));
    FR_HIP(hipStreamSynchronize(s));
    if (flags[GI_STATUS] == 3) {
        sv.inv_prec = -1;
        fr_set_error("fr_block_jacobi_factor: singular element block");
        return FR_ENOCONV;
    }
    return FR_OK;
}

extern "C" fr_status fr_block_jacobi_apply(fr_ctx c, const double* r, double* z, void* stream) {
    FR_TRY(ready(c));
    if (!r || !z) return bad("fr_block_jacobi_apply: null argument");
    if (r == z) return bad("fr_block_jacobi_apply: r and z may not alias");
    Solver& sv = *c->self;
    KArgs op{};   // the Newton operator of the last factor (its packs, time coefficients)
    op.c_time = sv.f_ct; op.inv_dtau = sv.f_idt;
    op.fpack = sv.d_fpack; op.spack = sv.d_spack;
    return precond_apply(sv, r, z, op, nullptr, 0, (hipStream_t)stream);
}

// blocks as assembled (column-major per element) -> caller's array row-major
namespace {
__global__ void k_transpose_blocks(size_t E, int nb, const double* __restrict__ src, double* __restrict__ dst) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nn = (size_t)nb * nb;
    if (t >= E * nn) return;
    const size_t e = t / nn, rc = t % nn, col = rc / nb, row = rc % nb;
    dst[e * nn + row * nb + col] = src[t];
}
}  // namespace

extern "C" fr_status fr_affine_elements(fr_ctx c, int32_t* n_affine, void* stream) {
    FR_TRY(ready(c));
    if (!n_affine) return bad("fr_affine_elements: null argument");
    std::vector<int32_t> h((size_t)c->E);
    FR_HIP(hipMemcpyAsync(h.data(), c->d_aff, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                          (hipStream_t)stream));
    FR_HIP(hipStreamSynchronize((hipStream_t)stream));
    int32_t n = 0;
    for (int32_t a : h) n += a;
    *n_affine = n;
    return FR_OK;
}

extern "C" fr_status fr_get_blocks(fr_ctx c, double* blk, void* stream) {
    FR_TRY(ready(c));
    if (!blk) return bad("fr_get_blocks: null argument");
    const Solver& sv = *c->self;
    if (!sv.d_blk_keep) return bad("fr_get_blocks: enable keep_blocks before fr_block_jacobi_factor");
    const int nb = 4 * c->Np;
    const size_t tot = (size_t)c->E * nb * nb;
    hipLaunchKernelGGL(k_transpose_blocks, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (size_t)c->E, nb, sv.d_blk_keep, blk);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

// stored inverse (precision of the last factor, column-major per element) -> caller's FP64
// array, row-major per element, widened exactly
namespace {
template <class Tin> __device__ __forceinline__ double widen(Tin x);
template <> __device__ __forceinline__ double widen<double>(double x) { return x; }
template <> __device__ __forceinline__ double widen<float>(float x) { return (double)x; }
template <> __device__ __forceinline__ double widen<uint16_t>(uint16_t x) {
    return (double)__uint_as_float((uint32_t)x << 16);
}
// slot k of the stored inverse holds element corder[k]'s block in the colour layout (corder
// set), element k's otherwise; the output is in element order
template <class Tin>
__global__ void k_widen_inverse(size_t E, int nb, const Tin* __restrict__ src, const int32_t* __restrict__ corder,
                                double* __restrict__ dst) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t nn = (size_t)nb * nb;
    if (t >= E * nn) return;
    const size_t k = t / nn, rc = t % nn, col = rc / nb, row = rc % nb;
    const size_t e = corder ? (size_t)corder[k] : k;
    dst[e * nn + row * nb + col] = widen<Tin>(src[t]);
}
}  // namespace

extern "C" fr_status fr_get_inverse(fr_ctx c, double* inv, void* stream) {
    FR_TRY(ready(c));
    if (!inv) return bad("fr_get_inverse: null argument");
    const Solver& sv = *c->self;
    if (sv.inv_prec < 0 || !sv.d_inv) return bad("fr_get_inverse: no factored blocks");
    const int nb = 4 * c->Np;
    const size_t tot = (size_t)c->E * nb * nb;
    const dim3 grid((unsigned)((tot + 255) / 256));
    hipStream_t s = (hipStream_t)stream;
    const int32_t* cl = sv.inv_colour ? c->d_corder : nullptr;
    switch (sv.inv_prec) {
        case FR_FP64:
            hipLaunchKernelGGL(k_widen_inverse<double>, grid, dim3(256), 0, s, (size_t)c->E, nb,
                               (const double*)sv.d_inv, cl, inv);
            break;
        case FR_FP32:
            hipLaunchKernelGGL(k_widen_inverse<float>, grid, dim3(256), 0, s, (size_t)c->E, nb,
                               (const float*)sv.d_inv, cl, inv);
            break;
        default:
            hipLaunchKernelGGL(k_widen_inverse<uint16_t>, grid, dim3(256), 0, s, (size_t)c->E, nb,
                               (const uint16_t*)sv.d_inv, cl, inv);
    }
    FR_HIP(hipGetLastError());
    return FR_OK;
}

extern "C" fr_status fr_reserve(fr_ctx c, int32_t krylov_max, int32_t prec) {
    if (!c) return bad("fr_reserve: null context");
    return solver_reserve(*c->self, krylov_max, prec);
}

extern "C" fr_status fr_bdf2_step(fr_ctx c, double* q_io, const double* q_nm1, const fr_step_opts* o,
                                  fr_step_stats* h_stats, void* stream) {
    FR_TRY(ready(c));
    if (!q_io || !o) return bad("fr_bdf2_step: null argument");
    double* qs[1] = {q_io};
    const double* qm[1] = {q_nm1};
    return solver_step(*c->self, qs, qm, o, h_stats, (hipStream_t)stream);
}

extern "C" fr_status fr_steady_solve(fr_ctx c, double* q_io, const fr_steady_opts* o, fr_steady_stats* h_stats,
                                     void* stream) {
    FR_TRY(ready(c));
    if (!q_io || !o) return bad("fr_steady_solve: null argument");
    double* qs[1] = {q_io};
    return solver_steady(*c->self, qs, o, h_stats, (hipStream_t)stream);
}

extern "C" fr_status fr_autotune(fr_ctx c, const char* cache_path, void* stream) {
    FR_TRY(ready(c));
    return solver_autotune(*c->self, cache_path, (hipStream_t)stream);
}

// ----------------------------------------------------------------------------- batches
extern "C" fr_status fr_batch_create(const fr_ctx* ctxs, int32_t n, fr_batch* out) {
    if (!ctxs || !out || n < 1) return bad("fr_batch_create: invalid argument");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return bad("fr_batch_create: null context");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return bad("fr_batch_create: a context appears twice");
    }
    fr_batch b = new fr_batch_s();
    fr_status st = solver_init(b->sv, ctxs, n);
    if (st != FR_OK) {
        solver_free(b->sv);
        delete b;
        return st;
    }
    *out = b;
    return FR_OK;
}

extern "C" void fr_batch_destroy(fr_batch b) {
    if (!b) return;
    solver_free(b->sv);
    delete b;
}

extern "C" fr_status fr_batch_layout(fr_batch b, int64_t* n_total, int64_t* offsets) {
    if (!b || !n_total) return bad("fr_batch_layout: null argument");
    *n_total = (int64_t)b->sv.Ntot;
    if (offsets)
        for (int c = 0; c < b->sv.n; ++c) offsets[c] = (int64_t)b->sv.off[c];
    return FR_OK;
}

static fr_status batch_ready(fr_batch b) {
    if (!b) return bad("null batch");
    for (fr_ctx c : b->sv.cs)
        if (const char* m = ctx_not_ready(c)) return bad(m);
    return FR_OK;
}

extern "C" fr_status fr_batch_residual(fr_batch b, const double* q, double* R, void* stream) {
    FR_TRY(batch_ready(b));
    if (!q || !R) return bad("fr_batch_residual: null argument");
    return solver_fused(b->sv, MODE_R, plain_args(q, nullptr, R, nullptr), (hipStream_t)stream);
}

extern "C" fr_status fr_batch_jvp(fr_batch b, const double* q, const double* v, double* Jv, void* stream) {
    FR_TRY(batch_ready(b));
    if (!q || !v || !Jv) return bad("fr_batch_jvp: null argument");
    return solver_fused(b->sv, MODE_JVP, plain_args(q, v, Jv, nullptr), (hipStream_t)stream);
}

extern "C" fr_status fr_batch_bdf2_step(fr_batch b, double* const* q, const double* const* q_nm1,
                                        const fr_step_opts* opts, fr_step_stats* h_stats, void* stream) {
    FR_TRY(batch_ready(b));
    if (!q || !opts) return bad("fr_batch_bdf2_step: null argument");
    return solver_step(b->sv, q, q_nm1, opts, h_stats, (hipStream_t)stream);
}

extern "C" fr_status fr_batch_steady_solve(fr_batch b, double* const* q, const fr_steady_opts* opts,
                                           fr_steady_stats* h_stats, void* stream) {
    FR_TRY(batch_ready(b));
    if (!q || !opts) return bad("fr_batch_steady_solve: null argument");
    return solver_steady(b->sv, q, opts, h_stats, (hipStream_t)stream);
}

extern "C" fr_status fr_batch_reserve(fr_batch b, int32_t krylov_max, int32_t prec) {
    if (!b) return bad("fr_batch_reserve: null batch");
    return solver_reserve(b->sv, krylov_max, prec);
}

extern "C" fr_status fr_batch_set_option(fr_batch b, const char* name, int64_t value) {
    if (!b || !name) return bad("fr_batch_set_option: null argument");
    return solver_option(b->sv, name, value);
}

extern "C" fr_status fr_batch_autotune(fr_batch b, const char* cache_path, void* stream) {
    FR_TRY(batch_ready(b));
    return solver_autotune(b->sv, cache_path, (hipStream_t)stream);
}
