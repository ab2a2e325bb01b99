// Solvers: the layout that lets many cases (meshes of different sizes, orders, flow
// parameters, static or deforming) share every launch of the hot path, the BDF2 step
// driver shared by a context and a batch, and the autotuner of the fused kernels'
// launch shape.
//
// Layout.  Case c's state vector [4][E_c][Np_c] starts at off_c, a multiple of CHUNK
// doubles, and is zero-padded to the next multiple; chunk k of the concatenated vector
// belongs to exactly one case (chunk_case), so segmented reductions and per-case vector
// operations walk chunks.  Cases are grouped by (order, viscous, moving); each group
// is one launch of the fused kernel whose tiles (EPB elements of one case) are listed
// by a prefix over the group's members for every tile width a kernel may use.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "fr_internal.hpp"

namespace {

template <class T>
fr_status upload(T** d, const std::vector<T>& h) {
    FR_TRY(dalloc(d, h.size()));
    FR_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return FR_OK;
}

}  // namespace

fr_status solver_init(Solver& sv, const fr_ctx* ctxs, int n) {
    sv.cs.assign(ctxs, ctxs + n);
    sv.n = n;
    FR_HIP(hipGetDevice(&sv.device));
    sv.off.resize(n);
    sv.len.resize(n);
    sv.boff.resize(n);
    size_t o = 0, bo = 0, fo = 0, so = 0;
    std::vector<CaseDev> cd(n);
    for (int c = 0; c < n; ++c) {
        const fr_ctx x = ctxs[c];
        if (x->device != sv.device) { fr_set_error("every case must live on the current device"); return FR_EINVAL; }
        const size_t N = x->N();
        const size_t nb = 4 * (size_t)x->Np;
        sv.off[c] = o;
        sv.len[c] = ((N + CHUNK - 1) / CHUNK) * CHUNK;
        sv.boff[c] = bo;
        o += sv.len[c];
        bo += (size_t)x->E * nb * nb;
        cd[c].E = x->E;
        cd[c].Np = x->Np;
        cd[c].off = sv.off[c];
        cd[c].boff = sv.boff[c];
        cd[c].fpoff = fo;
        cd[c].spoff = so;
        fo += (size_t)npf(x->prm.viscous != 0) * x->E * 4 * x->n;
        so += (size_t)nps(x->prm.viscous != 0) * x->E * x->Np;
        cd[c].g = x->geo();
        cd[c].pc = x->pc;
        sv.ncolors = x->ncolors > sv.ncolors ? x->ncolors : sv.ncolors;
    }
    sv.Ntot = o;
    sv.Btot = bo;
    sv.fpack_len = fo;
    sv.spack_len = so;
    sv.nchunks = (int)(o / CHUNK);
    if ((size_t)sv.nchunks * CHUNK != o || o / CHUNK > (size_t)1 << 30) { fr_set_error("solver too large"); return FR_EINVAL; }
    std::vector<int> chunk_case(sv.nchunks), case_chunk(n + 1);
    for (int c = 0; c < n; ++c) {
        case_chunk[c] = (int)(sv.off[c] / CHUNK);
        for (size_t k = sv.off[c] / CHUNK; k < (sv.off[c] + sv.len[c]) / CHUNK; ++k) chunk_case[k] = c;
    }
    case_chunk[n] = sv.nchunks;
    FR_TRY(upload(&sv.d_cases, cd));
    FR_TRY(upload(&sv.d_chunk_case, chunk_case));
    FR_TRY(upload(&sv.d_case_chunk, case_chunk));
    // launch groups: cases of one order, viscous and moving kind, with or without boundary
    // faces, and (as the geometry stands when the solver is made) affine or not, so that a
    // case runs the same kernel variant alone and in a batch; whether a group is affine is
    // checked again at every launch
    for (int c = 0; c < n; ++c) {
        const fr_ctx x = ctxs[c];
        Group* g = nullptr;
        for (Group& h : sv.groups)
            if (h.p == x->p && h.visc == (x->prm.viscous != 0) && h.mov == (x->prm.moving != 0) &&
                h.aff0 == x->all_affine && h.bnd == (x->d_bc != nullptr))
                g = &h;
        if (!g) {
            sv.groups.emplace_back();
            g = &sv.groups.back();
            g->p = x->p;
            g->visc = x->prm.viscous != 0;
            g->mov = x->prm.moving != 0;
            g->aff0 = x->all_affine;
            g->bnd = x->d_bc != nullptr;
        }
        g->ids.push_back(c);
        g->elems.push_back(x->E);
        g->cofs.push_back(x->cofs);
    }
    for (Group& g : sv.groups) {
        FR_TRY(upload(&g.d_ids, g.ids));
        std::vector<int> widths = fused_tile_widths(g.p);
        widths.push_back(1);
        for (int w : block_apply_widths(g.p)) widths.push_back(w);
        for (int w : widths) {
            if (g.tile_pfx(w)) continue;
            std::vector<int> pfx(g.ids.size() + 1, 0);
            for (size_t k = 0; k < g.ids.size(); ++k) pfx[k + 1] = pfx[k] + (int)((g.elems[k] + w - 1) / w);
            int* d = nullptr;
            FR_TRY(upload(&d, pfx));
            g.pfx.emplace_back(w, d);
        }
        // the Gauss-Seidel sweeps (coupling passes and block applies): per colour, tiles over
        // each member's elements of it
        std::vector<int> cwidths = fused_tile_widths(g.p);
        for (int w : block_apply_widths(g.p)) cwidths.push_back(w);
        for (int w : cwidths) {
            for (int k = 0; k < sv.ncolors; ++k) {
                if (g.color_tiles(w, k)) continue;
                std::vector<int> pfx(g.ids.size() + 1, 0), csel(2 * g.ids.size());
                for (size_t m = 0; m < g.ids.size(); ++m) {
                    const int cnt = g.cofs[m][k + 1] - g.cofs[m][k];
                    csel[2 * m] = g.cofs[m][k];
                    csel[2 * m + 1] = cnt;
                    pfx[m + 1] = pfx[m] + (cnt + w - 1) / w;
                }
                Group::ColorTiles ct{w, k, pfx.back(), nullptr, nullptr};
                FR_TRY(upload(&ct.d_pfx, pfx));
                const fr_status st = upload(&ct.d_csel, csel);
                if (st != FR_OK) { dfree(ct.d_pfx); return st; }
                g.ctiles.push_back(ct);
            }
        }
    }
    // per-case flags, step scalars, summary, reduction partials, pinned staging
    FR_TRY(dalloc(&sv.d_gi, (size_t)n * GI_STRIDE));
    FR_HIP(hipMemset(sv.d_gi, 0, (size_t)n * GI_STRIDE * sizeof(int)));
    FR_TRY(dalloc(&sv.d_sum, (size_t)n * SUM_STRIDE));
    FR_HIP(hipMemset(sv.d_sum, 0, (size_t)n * SUM_STRIDE * sizeof(double)));
    FR_TRY(dalloc(&sv.d_step, (size_t)n));
    FR_TRY(dalloc(&sv.d_part, (size_t)sv.nchunks * MAXV));
    sv.h_pin_doubles = (size_t)n * (SUM_STRIDE + sizeof(CaseStep) / sizeof(double) + 2) + 64;
    if (hipHostMalloc((void**)&sv.h_pin, sv.h_pin_doubles * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        sv.h_pin = nullptr;
        fr_set_error("hipHostMalloc failed");
        return FR_ENOMEM;
    }
    return FR_OK;
}

void solver_free(Solver& sv) {
    gmres_release(sv);
    for (Group& g : sv.groups) {
        dfree(g.d_ids);
        for (auto& x : g.pfx) dfree(x.second);
        for (auto& x : g.ctiles) { dfree(x.d_pfx); dfree(x.d_csel); }
    }
    sv.groups.clear();
    dfree(sv.d_cases); dfree(sv.d_chunk_case); dfree(sv.d_case_chunk);
    dfree(sv.d_blk); dfree(sv.d_inv); dfree(sv.d_blk_keep);
    dfree(sv.d_q); dfree(sv.d_w); dfree(sv.d_V); dfree(sv.d_gs); dfree(sv.d_gi); dfree(sv.d_part);
    dfree(sv.d_step); dfree(sv.d_sum); dfree(sv.d_fpack); dfree(sv.d_spack); dfree(sv.d_rscratch);
    dfree(sv.d_gst);
    if (sv.h_pin) (void)hipHostFree(sv.h_pin);
    if (sv.ws) (void)hipStreamDestroy(sv.ws);
    if (sv.ev_in) (void)hipEventDestroy(sv.ev_in);
    if (sv.ev_out) (void)hipEventDestroy(sv.ev_out);
    sv = Solver();
}

size_t prec_bytes(int prec) { return prec == FR_FP64 ? 8 : prec == FR_FP32 ? 4 : 2; }

fr_status solver_ensure_blocks(Solver& sv, int prec) {
    FR_TRY(dalloc(&sv.d_blk, sv.Btot));
    // the inverse in the stored precision; a wider precision than the buffer was sized for
    // replaces it (the inverse of the previous factor is then gone: inv_prec is reset)
    const size_t need = sv.Btot * prec_bytes(prec);
    if (sv.inv_bytes < need) {
        gmres_release(sv);   // a captured cycle holds the old buffer's address
        dfree(sv.d_inv);
        sv.d_inv = nullptr;
        sv.inv_bytes = 0;
        sv.inv_prec = -1;
        char* p = nullptr;
        FR_TRY(dalloc(&p, need));
        sv.d_inv = p;
        sv.inv_bytes = need;
    }
    if (sv.keep_blocks) FR_TRY(dalloc(&sv.d_blk_keep, sv.Btot));
    return FR_OK;
}

fr_status solver_reserve(Solver& sv, int m, int prec) {
    if (m < 1 || m > MAXV - 4 || prec < FR_FP64 || prec > FR_BF16) {
        fr_set_error("reserve: krylov must be in 1..156 and prec an fr_prec");
        return FR_EINVAL;
    }
    FR_TRY(solver_ensure_step(sv, m, prec));
    FR_TRY(dalloc(&sv.d_gst, sv.Ntot));   // Gauss-Seidel sweeps
    FR_TRY(dalloc(&sv.d_rscratch, sv.Ntot));   // R of the two-pass Newton operator
    return FR_OK;
}

fr_status solver_ensure_step(Solver& sv, int m, int prec) {
    FR_TRY(solver_ensure_blocks(sv, prec));
    if (sv.kry_m < m || !sv.d_V) {
        gmres_release(sv);
        dfree(sv.d_V); sv.d_V = nullptr;
        dfree(sv.d_gs); sv.d_gs = nullptr;
        FR_TRY(dalloc(&sv.d_V, (size_t)(m + 1) * sv.Ntot));
        FR_HIP(hipMemset(sv.d_V, 0, (size_t)(m + 1) * sv.Ntot * sizeof(double)));
        sv.gs_stride = (int)gmres_state_doubles(m);
        FR_TRY(dalloc(&sv.d_gs, (size_t)sv.n * sv.gs_stride));
        FR_HIP(hipMemset(sv.d_gs, 0, (size_t)sv.n * sv.gs_stride * sizeof(double)));
        sv.kry_m = m;
    }
    if (!sv.d_w) {
        // padding entries of every vector stay zero: kernels only ever write zeros there
        FR_TRY(dalloc(&sv.d_w, (size_t)NWORK * sv.Ntot));
        FR_HIP(hipMemset(sv.d_w, 0, (size_t)NWORK * sv.Ntot * sizeof(double)));
    }
    FR_TRY(dalloc(&sv.d_fpack, sv.fpack_len));
    FR_TRY(dalloc(&sv.d_spack, sv.spack_len));
    if (!sv.d_q) {
        FR_TRY(dalloc(&sv.d_q, sv.Ntot));
        FR_HIP(hipMemset(sv.d_q, 0, sv.Ntot * sizeof(double)));
    }
    if (!sv.ws) {
        FR_HIP(hipStreamCreateWithFlags(&sv.ws, hipStreamNonBlocking));
        FR_HIP(hipEventCreateWithFlags(&sv.ev_in, hipEventDisableTiming));
        FR_HIP(hipEventCreateWithFlags(&sv.ev_out, hipEventDisableTiming));
    }
    return FR_OK;
}

// ----------------------------------------------------------------------------- step driver
namespace {

// Runs the device Newton loop over every case with the per-case scalars already in the
// pinned staging area: states in, iteration, states out, all on the solver stream ordered
// after and before the caller's stream.  The per-case summary is left in h_pin.
fr_status run_newton(Solver& sv, double* const* q, const double* const* q_nm1, const fr_step_opts& common,
                     hipStream_t caller) {
    const int n = sv.n;
    FR_HIP(hipEventRecord(sv.ev_in, caller));
    FR_HIP(hipStreamWaitEvent(sv.ws, sv.ev_in, 0));
    hipStream_t s = sv.ws;
    const CaseStep* hst = reinterpret_cast<const CaseStep*>(sv.h_pin + (size_t)n * SUM_STRIDE);
    FR_HIP(hipMemcpyAsync(sv.d_step, hst, (size_t)n * sizeof(CaseStep), hipMemcpyHostToDevice, s));
    double* wq = sv.d_w + (size_t)WQNM1 * sv.Ntot;
    for (int c = 0; c < n; ++c) {
        const size_t bytes = sv.N(c) * sizeof(double);
        FR_HIP(hipMemcpyAsync(sv.d_q + sv.off[c], q[c], bytes, hipMemcpyDeviceToDevice, s));
        if (q_nm1 && q_nm1[c]) FR_HIP(hipMemcpyAsync(wq + sv.off[c], q_nm1[c], bytes, hipMemcpyDeviceToDevice, s));
    }
    const fr_status st = solver_newton(sv, &common, s);
    if (st == FR_OK) {
        for (int c = 0; c < n; ++c)
            FR_HIP(hipMemcpyAsync(q[c], sv.d_q + sv.off[c], sv.N(c) * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    FR_HIP(hipEventRecord(sv.ev_out, s));
    FR_HIP(hipStreamWaitEvent(caller, sv.ev_out, 0));
    return st;
}

// status of the cases from the summary: the first non-finite case, else the first that
// hit the iteration cap or a singular block
fr_status case_status(const Solver& sv) {
    fr_status ret = FR_OK;
    for (int c = 0; c < sv.n; ++c) {
        const int status = (int)sv.h_pin[(size_t)c * SUM_STRIDE + S_STATUS];
        char buf[160];
        if (status == 1 && ret != FR_ENONFINITE) {
            snprintf(buf, sizeof buf, "case %d: non-finite residual", c);
            fr_set_error(buf);
            ret = FR_ENONFINITE;
        } else if ((status == 2 || status == 3) && ret == FR_OK) {
            snprintf(buf, sizeof buf, "case %d: %s", c,
                     status == 2 ? "Newton iteration limit reached" : "singular element block");
            fr_set_error(buf);
            ret = FR_ENOCONV;
        }
    }
    return ret;
}

fr_status check_cases(const Solver& sv, double* const* q) {
    for (int c = 0; c < sv.n; ++c) {
        if (const char* m = ctx_not_ready(sv.cs[c])) { fr_set_error(m); return FR_EINVAL; }
        if (!q[c]) { fr_set_error("null state pointer"); return FR_EINVAL; }
    }
    return FR_OK;
}

}  // namespace

fr_status solver_step(Solver& sv, double* const* q, const double* const* q_nm1, const fr_step_opts* o,
                      fr_step_stats* stats, hipStream_t caller) {
    const int n = sv.n;
    FR_TRY(check_cases(sv, q));
    for (int c = 0; c < n; ++c) {
        const fr_step_opts& x = o[c];
        if (!(x.dt > 0.0) || x.krylov < 1 || x.krylov > MAXV - 4 || x.max_lin_it < 1 || x.max_newton < 0 ||
            x.jac_lag < 1 || x.prec < FR_FP64 || x.prec > FR_BF16 || !(x.inv_dtau >= 0.0)) {
            fr_set_error("invalid step options");
            return FR_EINVAL;
        }
        if (x.krylov != o[0].krylov || x.max_lin_it != o[0].max_lin_it || x.max_newton != o[0].max_newton ||
            x.jac_lag != o[0].jac_lag || x.prec != o[0].prec) {
            fr_set_error("krylov, max_lin_it, max_newton, jac_lag and prec must agree across a batch");
            return FR_EINVAL;
        }
    }
    FR_TRY(solver_ensure_step(sv, o[0].krylov, o[0].prec));
    // per-case step scalars through the pinned staging area (the previous step has synchronised)
    CaseStep* hst = reinterpret_cast<CaseStep*>(sv.h_pin + (size_t)n * SUM_STRIDE);
    for (int c = 0; c < n; ++c) {
        const bool b2 = q_nm1 && q_nm1[c];
        CaseStep st{};
        st.a0 = b2 ? 1.5 : 1.0;
        st.a1 = b2 ? -2.0 : -1.0;
        st.a2 = b2 ? 0.5 : 0.0;
        st.inv_dt = 1.0 / o[c].dt;
        st.ct = st.a0 / o[c].dt;
        st.idt = o[c].inv_dtau;
        st.tol_res = o[c].tol_res;
        st.tol_pseudo = o[c].tol_pseudo;
        st.tol_abs = o[c].tol_abs;
        st.has_nm1 = b2 ? 1 : 0;
        st.max_newton = o[c].max_newton;
        st.ser = 0;
        hst[c] = st;
    }
    FR_TRY(run_newton(sv, q, q_nm1, o[0], caller));
    for (int c = 0; c < n && stats; ++c) {
        const double* x = sv.h_pin + (size_t)c * SUM_STRIDE;
        stats[c].newton_its = (int32_t)x[S_NEWTON];
        stats[c].gmres_its = (int32_t)x[S_GMRES];
        stats[c].converged = x[S_CONV] != 0.0;
        stats[c].res0 = x[S_RES0];
        stats[c].res_final = x[S_RES];
    }
    return case_status(sv);
}

// Steady pseudo-transient continuation (paper Sec. 3.2, Eq. steady_pre_discretized_1):
// the Newton loop with no physical-time terms (c_time = 0, right-hand side R) and the
// pseudo-time step under SER control, Eq. (SER), updated per case on the device.
fr_status solver_steady(Solver& sv, double* const* q, const fr_steady_opts* o, fr_steady_stats* stats,
                        hipStream_t caller) {
    PhaseRange range("lmfr: steady solve");
    const int n = sv.n;
    FR_TRY(check_cases(sv, q));
    for (int c = 0; c < n; ++c) {
        const fr_steady_opts& x = o[c];
        if (!(x.dtau0 > 0.0) || !(x.dtau_min > 0.0) || !(x.dtau_max >= x.dtau_min) || !(x.r_ser >= 0.0) ||
            !(x.tol_pseudo >= 0.0) || !(x.tol_res >= 0.0) || !(x.tol_abs >= 0.0) || !(x.reject_growth >= 0.0) ||
            !std::isfinite(x.reject_growth) || x.krylov < 1 ||
            x.krylov > MAXV - 4 || x.max_lin_it < 1 || x.max_steps < 0 || x.jac_lag < 1 || x.prec < FR_FP64 ||
            x.prec > FR_BF16) {
            fr_set_error("invalid steady options");
            return FR_EINVAL;
        }
        if (x.krylov != o[0].krylov || x.max_lin_it != o[0].max_lin_it || x.max_steps != o[0].max_steps ||
            x.jac_lag != o[0].jac_lag || x.prec != o[0].prec) {
            fr_set_error("krylov, max_lin_it, max_steps, jac_lag and prec must agree across a batch");
            return FR_EINVAL;
        }
    }
    FR_TRY(solver_ensure_step(sv, o[0].krylov, o[0].prec));
    CaseStep* hst = reinterpret_cast<CaseStep*>(sv.h_pin + (size_t)n * SUM_STRIDE);
    sv.reject_on = false;
    for (int c = 0; c < n; ++c) {
        CaseStep st{};   // no physical-time terms: c_time = inv_dt = a0 = a1 = a2 = 0
        st.dtau = o[c].dtau0;
        st.idt = 1.0 / o[c].dtau0;
        st.dtau_min = o[c].dtau_min;
        st.dtau_max = o[c].dtau_max;
        st.r_ser = o[c].r_ser;
        st.tol_res = o[c].tol_res;
        st.tol_pseudo = o[c].tol_pseudo;
        st.tol_abs = o[c].tol_abs;
        st.max_newton = o[c].max_steps;
        st.ser = 1;
        st.reject_growth = o[c].reject_growth;
        sv.reject_on = sv.reject_on || o[c].reject_growth > 0.0;
        hst[c] = st;
    }
    fr_step_opts common{};
    common.krylov = o[0].krylov;
    common.max_lin_it = o[0].max_lin_it;
    common.max_newton = o[0].max_steps;
    common.jac_lag = o[0].jac_lag;
    common.prec = o[0].prec;
    const fr_status rs = run_newton(sv, q, nullptr, common, caller);
    sv.reject_on = false;
    FR_TRY(rs);
    for (int c = 0; c < n && stats; ++c) {
        const double* x = sv.h_pin + (size_t)c * SUM_STRIDE;
        stats[c].steps = (int32_t)x[S_NEWTON];
        stats[c].gmres_its = (int32_t)x[S_GMRES];
        stats[c].converged = x[S_CONV] != 0.0;
        stats[c].res0 = x[S_RES0];
        stats[c].res_final = x[S_RES];
        stats[c].dtau_final = x[S_DTAU] > 0.0 ? x[S_DTAU] : o[c].dtau0;
        stats[c].rejected = (int32_t)x[S_REJ];
    }
    return case_status(sv);
}

// ----------------------------------------------------------------------------- autotuner
namespace {

// free-stream state of every case (rho = T = 1, |v| = 1): inputs for timing
__global__ void k_tune_state(const CaseDev* cases, const int* chunk_case, int nchunks, double* q, double* v) {
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int c = chunk_case[ch];
        const CaseDev& cd = cases[c];
        const size_t EN = (size_t)cd.E * cd.Np;
        for (size_t t = (size_t)ch * CHUNK + threadIdx.x; t < (size_t)(ch + 1) * CHUNK; t += blockDim.x) {
            const size_t r = t - cd.off;
            const int var = (int)(r / EN);
            double x = 0.0, d = 0.0;
            if (var < 4) {
                const double phase = 0.001 * (double)(r % EN);
                x = var == 0 ? cd.pc.Rg : var == 1 ? 0.8 + 0.1 * sin(phase) : var == 2 ? 0.6 : 1.0 + 0.01 * cos(phase);
                d = 1e-3 * cos(3.0 * phase + var);
            }
            q[t] = x;
            v[t] = d;
        }
    }
}

std::string arch_name(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string s = p.gcnArchName;
    for (char& ch : s) if (ch == ' ') ch = '_';
    return s;
}

std::string tune_key(const std::string& arch, const Solver& sv, const Group& g, int mode) {
    long long E = 0;
    for (long long e : g.elems) E += e;
    int bucket = 0;
    while ((1LL << (bucket + 1)) <= E) ++bucket;
    bool aff = true;   // all-affine groups run other kernel variants
    for (int id : g.ids) aff = aff && sv.cs[id]->all_affine;
    std::ostringstream o;
    o << arch << " p" << g.p << " v" << g.visc << " m" << g.mov << " a" << (aff ? 1 : 0) << " mode" << mode
      << " e2^" << bucket;
    return o.str();
}

}  // namespace

fr_status solver_autotune(Solver& sv, const char* cache_path, hipStream_t s) {
    PhaseRange range("lmfr: autotune");
    const std::string arch = arch_name(sv.device);
    // cached choices
    std::vector<std::pair<std::string, Tune>> cache;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            const size_t bar = line.find('|');
            if (bar == std::string::npos) continue;
            std::istringstream v(line.substr(bar + 1));
            Tune t;
            if (v >> t.lanes >> t.grid >> t.xcd) cache.emplace_back(line.substr(0, bar), t);
        }
    }
    // the timed launches rotate through input/output pairs totalling > 512 MB, so that they
    // stream from HBM as in use rather than from the 256 MB Infinity Cache
    const int nrot = (int)std::min<size_t>(8, std::max<size_t>(1, (size_t)(512e6 / (16.0 * (double)sv.Ntot)) + 1));
    std::vector<double*> qr(nrot, nullptr), outr(nrot, nullptr);
    double *v = nullptr, *out2 = nullptr, *pf = nullptr, *ps = nullptr;
    auto release = [&]() {
        for (double* x : qr) dfree(x);
        for (double* x : outr) dfree(x);
        dfree(v); dfree(out2); dfree(pf); dfree(ps);
    };
    bool ok = dalloc(&v, sv.Ntot) == FR_OK && dalloc(&out2, sv.Ntot) == FR_OK && dalloc(&pf, sv.fpack_len) == FR_OK &&
              dalloc(&ps, sv.spack_len) == FR_OK;
    for (int r = 0; r < nrot && ok; ++r) ok = dalloc(&qr[r], sv.Ntot) == FR_OK && dalloc(&outr[r], sv.Ntot) == FR_OK;
    if (!ok) {
        release();
        return FR_ENOMEM;
    }
    for (int r = 0; r < nrot; ++r)
        hipLaunchKernelGGL(k_tune_state, dim3((unsigned)std::min(sv.nchunks, 8192)), dim3(256), 0, s, sv.d_cases,
                           sv.d_chunk_case, sv.nchunks, qr[r], v);
    double* q = qr[0];
    double* out = outr[0];
    hipEvent_t e0, e1;
    FR_HIP(hipEventCreate(&e0));
    FR_HIP(hipEventCreate(&e1));
    fr_status ret = FR_OK;
    std::string appended;
    // persistent grids up to 6144 workgroups: the lighter variants run 3 waves per SIMD, and
    // 768 / 1536 / 3072 workgroups of 256 / 128 / 64 lanes are one resident round at that rate
    const int grids[] = {0, 512, 1024, 1536, 2048, 3072, 4096, 6144};
    constexpr int NGRID = 8;
    for (Group& g : sv.groups) {
        for (int mode : {MODE_R, MODE_JVP, MODE_AOP, MODE_PREP, MODE_LIN}) {
            const std::string key = tune_key(arch, sv, g, mode);
            bool found = false;
            for (auto& kv : cache)
                if (kv.first == key) { g.tune[mode] = kv.second; found = true; }
            if (found) continue;
            KArgs a{};
            a.q = q; a.v = (mode == MODE_R || mode == MODE_PREP) ? nullptr : v; a.out = out; a.out2 = nullptr;
            a.c_time = 1.0; a.inv_dtau = 0.0;
            a.fpack = pf; a.spack = ps;
            if (mode == MODE_LIN) {
                // the linearisation packs of the tuning state
                KArgs pa = a;
                pa.v = nullptr;
                if ((ret = launch_fused(sv, g, MODE_PREP, pa, g.tune[MODE_PREP], s)) != FR_OK) break;
            }
            Tune best;
            float best_ms = 1e30f;
            // two sweeps, each candidate keeping its faster time: the GPU raises its clocks over
            // the first tens of milliseconds of work, which would favour the later candidates
            for (int pass = 0; pass < 2 && ret == FR_OK; ++pass)
            for (int lanes : {64, 128, 256}) {
                if (lanes == 256 && mode != MODE_R) continue;
                for (int gx = 0; gx < 2 * NGRID; ++gx) {
                    Tune t;
                    t.lanes = lanes;
                    t.grid = grids[gx % NGRID];
                    t.xcd = gx / NGRID;
                    if ((ret = launch_fused(sv, g, mode, a, t, s)) != FR_OK) break;   // warm-up
                    FR_HIP(hipEventRecord(e0, s));
                    const int reps = 8;
                    for (int r = 0; r < reps && ret == FR_OK; ++r) {
                        KArgs ar = a;
                        if (mode == MODE_R || mode == MODE_PREP) ar.q = qr[r % nrot];
                        ar.out = outr[r % nrot];
                        ret = launch_fused(sv, g, mode, ar, t, s);
                    }
                    FR_HIP(hipEventRecord(e1, s));
                    FR_HIP(hipEventSynchronize(e1));
                    if (ret != FR_OK) break;
                    float ms = 0.f;
                    FR_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best_ms) { best_ms = ms; best = t; }
                }
                if (ret != FR_OK) break;
            }
            if (ret != FR_OK) break;
            g.tune[mode] = best;
            std::ostringstream o;
            o << key << "|" << best.lanes << " " << best.grid << " " << best.xcd << "\n";
            appended += o.str();
        }
        if (ret != FR_OK) break;
        // block columns use the shapes of the matching Newton operators
        g.tune[MODE_BLK] = g.tune[MODE_AOP];
        g.tune[MODE_LINBLK] = g.tune[MODE_LIN];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FR_HIP(hipStreamSynchronize(s));
    release();
    if (ret != FR_OK) return ret;
    gmres_release(sv);   // captured cycles baked the previous shapes
    if (cache_path && !appended.empty()) {
        std::ofstream outf(cache_path, std::ios::app);
        outf << appended;
    }
    return FR_OK;
}
