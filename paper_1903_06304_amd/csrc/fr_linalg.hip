// Element-block-Jacobi preconditioner and Krylov building blocks for gfx950.
//
//  - block assembly: seeded forward tangents of the residual kernel (one column per
//    launch lane) give the true diagonal block dR_e/dq_e; the time terms
//    inv_dtau Gamma + c_time M are added pointwise (paper Eq. unsteady_pre_discretized_3)
//  - block inversion: Gauss-Jordan with partial pivoting in FP64, one workgroup per
//    element, the block resident in LDS; the explicit inverse is stored in FP64, FP32
//    or BF16 (round to nearest even), column-major so the apply reads it coalesced
//  - block apply z_e = P_e^-1 r_e: memory-bound GEMV, FP64 accumulation
//  - Krylov reductions: two-stage, fixed-order (deterministic) dot products
#include "fr_internal.hpp"

#include <hip/hip_bf16.h>

namespace {

constexpr int RED_THREADS = 256;
static_assert(MAXV <= RED_THREADS, "the coefficient staging takes one thread per Krylov vector");
constexpr int MAX_GRID = 8192;    // workgroups of the chunk-walking kernels

// case of tile t of a group (binary search over the group's tile prefix); uniform
__device__ __forceinline__ int tile_member(const GroupArgs& ga, int t) {
    int lo = 0, hi = ga.nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ga.pfx[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// z_e = Ainv_e r_e for the elements of one group; state layout [4][E][Np] per case,
// block row/col index v*Np + s.  Each thread owns RPT consecutive rows and reads them
// from every column of the column-major inverse with one load (1 double, 4 floats in 16
// bytes, or 4 bfloat16 in 8 bytes), so every precision streams its blocks with wide loads;
// FP64 accumulation over the columns in ascending order.
template <class Tin> struct Pack8;
template <> struct Pack8<double> {   // 8-byte loads: 1 row per thread
    static constexpr int R = 1;
    using Raw = double;
    __device__ static Raw ld(const double* p) { return *p; }
    __device__ static void expand(const Raw& v, double* x) { x[0] = v; }
};
template <> struct Pack8<float> {    // 16-byte loads: 4 rows per thread
    static constexpr int R = 4;
    using Raw = float4;
    __device__ static Raw ld(const float* p) { return *reinterpret_cast<const float4*>(p); }
    __device__ static void expand(const Raw& v, double* x) { x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w; }
};
template <> struct Pack8<uint16_t> { // 8-byte loads: 4 rows per thread
    static constexpr int R = 4;
    using Raw = uint2;
    __device__ static Raw ld(const uint16_t* p) { return *reinterpret_cast<const uint2*>(p); }
    __device__ static void expand(const Raw& v, double* x) {
        x[0] = (double)__uint_as_float(v.x << 16);
        x[1] = (double)__uint_as_float(v.x & 0xffff0000u);
        x[2] = (double)__uint_as_float(v.y << 16);
        x[3] = (double)__uint_as_float(v.y & 0xffff0000u);
    }
};

template <class Tin, int NB>
struct ApplyShape {
    static constexpr int RPT = Pack8<Tin>::R, TPE = NB / RPT, EPB = 256 / TPE, threads = EPB * TPE;
    static_assert(NB % RPT == 0, "block size must be a multiple of the rows per thread");
};

// z_e = D_e^-1 r_e for every element, or, for the Gauss-Seidel sweeps, for the elements of
// one colour only (tiles over that colour, ga.csel): z_e = D_e^-1 (r_e - b_e) (b may be null),
// or z_e -= D_e^-1 r_e (sub).
template <class Tin, int NB>
__global__ void __launch_bounds__(256) k_block_apply(GroupArgs ga, const Tin* __restrict__ inv,
                                                     const double* __restrict__ r, const double* __restrict__ b,
                                                     double* __restrict__ z, int sub,
                                                     const int* __restrict__ flags, int flag, int cl) {
    using SH = ApplyShape<Tin, NB>;
    constexpr int Np = NB / 4, RPT = SH::RPT, TPE = SH::TPE, EPB = SH::EPB;
    __shared__ double rs[EPB][NB + 1];
    const int t = blockIdx.x;
    if (t >= ga.ntiles) return;
    const int lo = tile_member(ga, t);
    const int cid = ga.ids[lo];
    if (flags && flags[cid * GI_STRIDE + flag]) return;
    const CaseDev& cd = ga.cases[cid];
    const int el = threadIdx.x / TPE, r0 = (threadIdx.x % TPE) * RPT;
    // one colour of the Gauss-Seidel sweeps (ga.csel set): the tiles run over the member's
    // elements of that colour, taken from its colour-sorted element list.  slot: the
    // element's block in the stored inverse (its position in that list in the colour layout)
    int slot = (t - ga.pfx[lo]) * EPB + el;
    bool act = (el < EPB) && (slot < cd.E);
    if (ga.csel) {
        act = (el < EPB) && (slot < ga.csel[2 * lo + 1]);
        slot += ga.csel[2 * lo];
    }
    int e = slot;
    if (ga.csel || cl) e = act ? cd.g.corder[slot] : 0;
    if (!cl) slot = e;
    const size_t EN = (size_t)cd.E * Np;
    size_t gid[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int row = r0 + k;
        gid[k] = cd.off + (row / Np) * EN + (size_t)e * Np + (row % Np);
        if (act) rs[el][row] = b ? r[gid[k]] - b[gid[k]] : r[gid[k]];
    }
    __syncthreads();
    if (!act) return;
    const Tin* A = inv + cd.boff + (size_t)slot * NB * NB + r0;
    double acc[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) acc[k] = 0.0;
    // columns in batches of U, every load of a batch issued before any is used (so that
    // U loads per thread are in flight), summed in ascending column order
    constexpr int U = 16, NBU = NB - NB % U;
    for (int c0 = 0; c0 < NBU; c0 += U) {
        typename Pack8<Tin>::Raw raw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) raw[u] = Pack8<Tin>::ld(A + (size_t)(c0 + u) * NB);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double x[RPT];
            Pack8<Tin>::expand(raw[u], x);
            const double rc = rs[el][c0 + u];
#pragma unroll
            for (int k = 0; k < RPT; ++k) acc[k] += x[k] * rc;
        }
    }
    if (NBU < NB) {
        typename Pack8<Tin>::Raw raw[NB % U > 0 ? NB % U : 1];
#pragma unroll
        for (int u = 0; u < NB - NBU; ++u) raw[u] = Pack8<Tin>::ld(A + (size_t)(NBU + u) * NB);
#pragma unroll
        for (int u = 0; u < NB - NBU; ++u) {
            double x[RPT];
            Pack8<Tin>::expand(raw[u], x);
            const double rc = rs[el][NBU + u];
#pragma unroll
            for (int k = 0; k < RPT; ++k) acc[k] += x[k] * rc;
        }
    }
    if (sub) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) z[gid[k]] -= acc[k];
    } else {
#pragma unroll
        for (int k = 0; k < RPT; ++k) z[gid[k]] = acc[k];
    }
}

// ------------------------------------------------------------------ segmented Krylov reductions
// The solver vectors are concatenations of per-case segments aligned to CHUNK doubles;
// every chunk belongs to one case.  First stage: one partial sum per chunk and output;
// second stage: per case, a fixed-order tree over its chunks (deterministic).
struct ChunkArgs {
    const CaseDev* cases;
    const int* chunk_case;   // [nchunks]
    const int* case_chunk;   // [ncase + 1]
    int nchunks;
    const int* flags;        // per-case skip flags or NULL
    int flag;
};

__device__ __forceinline__ bool chunk_skipped(const ChunkArgs& ca, int c) {
    return ca.flags && ca.flags[c * GI_STRIDE + ca.flag];
}

// End of chunk ch within its case's entries: the padding after a case's 4 E Np entries is
// neither read nor written by the reductions, so a non-finite value that arithmetic on the
// padding once produced (a scaling by a non-finite coefficient) cannot reach a dot product
// or norm of a later iteration, step or solve.
__device__ __forceinline__ size_t case_end(const CaseDev& cd, int ch) {
    const size_t e = cd.off + (size_t)4 * cd.E * cd.Np, ce = (size_t)(ch + 1) * CHUNK;
    return e < ce ? e : ce;
}

// Dot products V_i . w for i in [DB*blockIdx.y, DB*blockIdx.y + DB) ∩ [0, nv), plus |w|^2 in
// slot nv when want_norm (y-block 0 only; mass_only: first E Np entries of the case).
// DB = 8 vectors per pass (16 measured slower: fewer workgroups, heavier reduction).
constexpr int DB = 8;
__global__ void __launch_bounds__(RED_THREADS) k_dots8(ChunkArgs ca, const double* __restrict__ V, size_t ldv, int nv,
                                                       const double* __restrict__ w, int want_norm, int mass_only,
                                                       double* __restrict__ partial) {
    __shared__ double red[RED_THREADS / 64][DB + 1];
    const int i0 = blockIdx.y * DB;
    const int cnt = nv - i0 < DB ? nv - i0 : DB;
    const bool nrm = want_norm && blockIdx.y == 0;
    const double* Vc = V + (size_t)i0 * ldv;
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    for (int ch = blockIdx.x; ch < ca.nchunks; ch += gridDim.x) {
        const int c = ca.chunk_case[ch];
        if (chunk_skipped(ca, c)) continue;
        const CaseDev& cd = ca.cases[c];
        const size_t end = case_end(cd, ch);
        size_t lim = end;
        if (mass_only) {
            const size_t m = cd.off + (size_t)cd.E * cd.Np;
            lim = m < lim ? m : lim;
        }
        double acc[DB];
#pragma unroll
        for (int i = 0; i < DB; ++i) acc[i] = 0.0;
        double nacc = 0.0;
        for (size_t t = (size_t)ch * CHUNK + threadIdx.x; t < end; t += RED_THREADS) {
            const double wt = w[t];
            if (cnt > 0) {
                // all rows loaded before any is used (rows past cnt - 1 reload row cnt - 1, unused)
                double x[DB];
#pragma unroll
                for (int i = 0; i < DB; ++i) x[i] = Vc[(size_t)(i < cnt ? i : cnt - 1) * ldv + t];
#pragma unroll
                for (int i = 0; i < DB; ++i)
                    if (i < cnt) acc[i] += x[i] * wt;
            }
            if (nrm && t < lim) nacc += wt * wt;
        }
        __syncthreads();   // red[] of the previous chunk consumed
#pragma unroll
        for (int i = 0; i < DB + 1; ++i) {
            const bool live = (i < cnt) || (i == DB && nrm);
            if (!live) continue;
            double v = (i < DB) ? acc[i] : nacc;
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) red[wid][i] = v;
        }
        __syncthreads();
        const int k = threadIdx.x;
        if (k < cnt || (k == DB && nrm)) {
            double v = 0.0;
            for (int q = 0; q < RED_THREADS / 64; ++q) v += red[q][k];
            partial[(size_t)ch * MAXV + (k < DB ? i0 + k : nv)] = v;
        }
    }
}

// w_out = w_in - sum_{i < nv} coef_c[i] V_i (coef_c = coef + c * cstride), and the partial
// |w_out|^2 in slot 0 when want_norm
__global__ void __launch_bounds__(RED_THREADS) k_update(ChunkArgs ca, const double* __restrict__ V, size_t ldv, int nv,
                                                        const double* __restrict__ coef, int cstride,
                                                        const double* w_in, double* w_out, int want_norm,
                                                        double* __restrict__ partial, int rev) {
    __shared__ double cf[MAXV];
    __shared__ double red[RED_THREADS / 64];
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    for (int ci = blockIdx.x; ci < ca.nchunks; ci += gridDim.x) {
        const int ch = rev ? ca.nchunks - 1 - ci : ci;   // chunks last to first (partials by chunk)
        const int c = ca.chunk_case[ch];
        if (chunk_skipped(ca, c)) continue;
        const size_t end = case_end(ca.cases[c], ch);
        __syncthreads();   // cf[] / red[] of the previous chunk consumed
        if ((int)threadIdx.x < MAXV) cf[threadIdx.x] = ((int)threadIdx.x < nv) ? coef[(size_t)c * cstride + threadIdx.x] : 0.0;
        __syncthreads();
        double nacc = 0.0;
        for (size_t t = (size_t)ch * CHUNK + threadIdx.x; t < end; t += RED_THREADS) {
            double wt = w_in[t];
            int i = 0;
            // 16 basis entries loaded before any is used, summed in the groups of four below
            for (; i + 16 <= nv; i += 16) {
                double x[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) x[u] = V[(size_t)(i + u) * ldv + t];
#pragma unroll
                for (int u = 0; u < 16; u += 4)
                    wt -= cf[i + u] * x[u] + cf[i + u + 1] * x[u + 1] + cf[i + u + 2] * x[u + 2] + cf[i + u + 3] * x[u + 3];
            }
            for (; i + 4 <= nv; i += 4)
                wt -= cf[i] * V[i * ldv + t] + cf[i + 1] * V[(i + 1) * ldv + t] + cf[i + 2] * V[(i + 2) * ldv + t] +
                      cf[i + 3] * V[(i + 3) * ldv + t];
            for (; i < nv; ++i) wt -= cf[i] * V[i * ldv + t];
            w_out[t] = wt;
            nacc += wt * wt;
        }
        if (!want_norm) continue;
        for (int off = 32; off > 0; off >>= 1) nacc += __shfl_down(nacc, off, 64);
        if (lane == 0) red[wid] = nacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = 0.0;
            for (int q = 0; q < RED_THREADS / 64; ++q) v += red[q];
            partial[(size_t)ch * MAXV] = v;
        }
    }
}

// The re-orthogonalising pass of classical Gram-Schmidt applied twice, in one read of the basis:
// w_out = w_in - sum_{i < nv} coef_c[i] V_i (as k_update) and the partial dots V_k . w_out,
// k < nv, of each chunk (as k_dots8 on w_out), from the basis entries already loaded for the
// update.  The update's grouping and the reductions' order are those of the two kernels, so the
// results are theirs bit for bit.  NV bounds nv.
template <int NV>
__global__ void __launch_bounds__(RED_THREADS) k_update_dots(ChunkArgs ca, const double* __restrict__ V, size_t ldv,
                                                             int nv, const double* __restrict__ coef, int cstride,
                                                             const double* w_in, double* w_out,
                                                             double* __restrict__ partial, int rev) {
    __shared__ double cf[NV];
    __shared__ double red[RED_THREADS / 64][NV];
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    for (int ci = blockIdx.x; ci < ca.nchunks; ci += gridDim.x) {
        const int ch = rev ? ca.nchunks - 1 - ci : ci;   // chunks last to first (partials by chunk)
        const int c = ca.chunk_case[ch];
        if (chunk_skipped(ca, c)) continue;
        const size_t end = case_end(ca.cases[c], ch);
        __syncthreads();   // cf[] / red[] of the previous chunk consumed
        if ((int)threadIdx.x < NV) cf[threadIdx.x] = ((int)threadIdx.x < nv) ? coef[(size_t)c * cstride + threadIdx.x] : 0.0;
        __syncthreads();
        double acc[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] = 0.0;
        for (size_t t = (size_t)ch * CHUNK + threadIdx.x; t < end; t += RED_THREADS) {
            // all rows loaded before any is used (rows past nv - 1 reload row nv - 1, unused)
            double x[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) x[k] = V[(size_t)(k < nv ? k : nv - 1) * ldv + t];
            double wt = w_in[t];
            const int n4 = nv & ~3;
#pragma unroll
            for (int k = 0; k < NV; k += 4)
                if (k < n4) wt -= cf[k] * x[k] + cf[k + 1] * x[k + 1] + cf[k + 2] * x[k + 2] + cf[k + 3] * x[k + 3];
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (k >= n4 && k < nv) wt -= cf[k] * x[k];
            w_out[t] = wt;
#pragma unroll
            for (int k = 0; k < NV; ++k)
                if (k < nv) acc[k] += x[k] * wt;
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            if (k >= nv) continue;
            double v = acc[k];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) red[wid][k] = v;
        }
        __syncthreads();
        const int k = threadIdx.x;
        if (k < nv) {
            double v = 0.0;
            for (int q = 0; q < RED_THREADS / 64; ++q) v += red[q][k];
            partial[(size_t)ch * MAXV + k] = v;
        }
    }
}

// out_c[i] = sum over the chunks of case c of partial[chunk][i]; grid (ncase, nout)
__global__ void __launch_bounds__(256) k_final(ChunkArgs ca, const double* __restrict__ partial,
                                               double* __restrict__ out, int ostride) {
    __shared__ double red[256];
    const int c = blockIdx.x, i = blockIdx.y;
    if (chunk_skipped(ca, c)) return;
    const int c0 = ca.case_chunk[c], c1 = ca.case_chunk[c + 1];
    double v = 0.0;
    for (int b = c0 + threadIdx.x; b < c1; b += blockDim.x) v += partial[(size_t)b * MAXV + i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)c * ostride + i] = red[0];
}

// ------------------------------------------------------------------ pointwise physics per case
// Walk the chunks that hold solution points of the first variable of each case: point
// t of case c covers entries v * E Np + t, v = 0..3.
#define FR_POINT_LOOP(ca, ...)                                                                  \
    for (int ch = blockIdx.x; ch < (ca).nchunks; ch += gridDim.x) {                             \
        const int c = (ca).chunk_case[ch];                                                       \
        if (chunk_skipped((ca), c)) continue;                                                    \
        const CaseDev& cd = (ca).cases[c];                                                       \
        const size_t EN = (size_t)cd.E * cd.Np;                                                  \
        const size_t r0 = (size_t)ch * CHUNK - cd.off;                                           \
        if (r0 >= EN) continue;                                                                  \
        for (size_t t = r0 + threadIdx.x; t < r0 + CHUNK && t < EN; t += blockDim.x) {           \
            const size_t base = cd.off + t;                                                      \
            __VA_ARGS__                                                                          \
        }                                                                                        \
    }

// q^c of the state
__global__ void k_cons(ChunkArgs ca, const double* __restrict__ q, double* __restrict__ Qc) {
    FR_POINT_LOOP(ca, {
        double qs[4], qc[4];
        for (int v = 0; v < 4; ++v) qs[v] = q[base + v * EN];
        fr_cons(cd.pc, qs, qc);
        for (int v = 0; v < 4; ++v) Qc[base + v * EN] = qc[v];
    })
}

// b = R - (a0 q^c(q) + a1 Q^n + a2 Q^{n-1}) / dt with the case's BDF coefficients
__global__ void k_bdf_rhs(ChunkArgs ca, const CaseStep* __restrict__ st, const double* __restrict__ q,
                          const double* __restrict__ Qn, const double* __restrict__ Qnm1, const double* __restrict__ R,
                          double* __restrict__ b) {
    FR_POINT_LOOP(ca, {
        const CaseStep& cs = st[c];
        double qs[4], qc[4];
        for (int v = 0; v < 4; ++v) qs[v] = q[base + v * EN];
        fr_cons(cd.pc, qs, qc);
        for (int v = 0; v < 4; ++v) {
            double acc = cs.a0 * qc[v] + cs.a1 * Qn[base + v * EN];
            if (cs.has_nm1) acc += cs.a2 * Qnm1[base + v * EN];
            b[base + v * EN] = R[base + v * EN] - acc * cs.inv_dt;
        }
    })
}

// q^c in place for the cases with a q^{n-1}
__global__ void k_cons_nm1(ChunkArgs ca, const CaseStep* __restrict__ st, double* __restrict__ buf) {
    FR_POINT_LOOP(ca, {
        if (st[c].has_nm1) {
            double qs[4], qc[4];
            for (int v = 0; v < 4; ++v) qs[v] = buf[base + v * EN];
            fr_cons(cd.pc, qs, qc);
            for (int v = 0; v < 4; ++v) buf[base + v * EN] = qc[v];
        }
    })
}

ChunkArgs chunk_args(const Solver& sv, const int* flags, int flag) {
    ChunkArgs ca;
    ca.cases = sv.d_cases;
    ca.chunk_case = sv.d_chunk_case;
    ca.case_chunk = sv.d_case_chunk;
    ca.nchunks = sv.nchunks;
    ca.flags = flags;
    ca.flag = flag;
    return ca;
}

unsigned chunk_grid(const Solver& sv) {
    return (unsigned)(sv.nchunks < MAX_GRID ? sv.nchunks : MAX_GRID);
}

// the tiles of a group at a tile width; color >= 0: the tiles over the members' elements of
// that colour (pfx null when a table is missing)
GroupArgs group_args(const Solver& sv, const Group& gr, int epb, int color = -1) {
    GroupArgs ga;
    ga.cases = sv.d_cases;
    ga.ids = gr.d_ids;
    ga.pfx = gr.tile_pfx(epb);
    ga.nmem = (int)gr.ids.size();
    ga.ntiles = gr.ntiles(epb);
    ga.xcd = 0;
    if (color >= 0) {
        const Group::ColorTiles* ct = gr.color_tiles(epb, color);
        ga.pfx = ct ? ct->d_pfx : nullptr;
        ga.ntiles = ct ? ct->ntiles : 0;
        ga.csel = ct ? ct->d_csel : nullptr;
    }
    return ga;
}

}  // namespace

// ----------------------------------------------------------------------------- launchers
fr_status launch_block_assembly(Solver& sv, const double* q, const KArgs& base, hipStream_t s) {
    PhaseRange range("lmfr: block assembly (enqueue)");
    // one seeded column of every element's block per launch and group (every column at once
    // on affine static groups, below); with the linearisation packs of q in base
    // (fpack/spack), tangents only
    KArgs a = base;
    a.q = q; a.v = nullptr; a.out = sv.d_blk; a.out2 = nullptr;
    const int mode = (a.fpack && a.spack) ? MODE_LINBLK : MODE_BLK;
    for (const Group& gr : sv.groups) {
        const int nb = 4 * (gr.p + 1) * (gr.p + 1);
        // the affine kernel over the packs (static groups whose elements are all affine)
        // assembles every column in one launch, reading the packs of an element once
        bool all_aff = !gr.mov;
        for (int id : gr.ids) all_aff = all_aff && sv.cs[id]->all_affine;
        if (mode == MODE_LINBLK && all_aff) {
            a.seed0 = 0;
            a.ncols = nb;
            FR_TRY(launch_fused(sv, gr, mode, a, gr.tune[mode], s));
            a.ncols = 0;
            continue;
        }
        for (int col = 0; col < nb; ++col) {
            a.seed0 = col;
            FR_TRY(launch_fused(sv, gr, mode, a, gr.tune[mode], s));
        }
    }
    return FR_OK;
}

// explicit inverse of every element block, on the matrix cores (fr_invert.hip)
static fr_status invert_all(Solver& sv, int prec, const int* flags, hipStream_t s) {
    for (const Group& gr : sv.groups) {
        GroupArgs ga = group_args(sv, gr, 1);
        if (!ga.pfx) { fr_set_error("tile prefix missing"); return FR_EINVAL; }
        FR_TRY(launch_block_invert_group(sv, gr.p, ga, prec, flags, s));
    }
    return FR_OK;
}

fr_status launch_block_invert(Solver& sv, int prec, const int* flags, hipStream_t s) {
    PhaseRange range("lmfr: block inversion (enqueue)");
    if (prec < FR_FP64 || prec > FR_BF16) { fr_set_error("unknown precision"); return FR_EINVAL; }
    // the Gauss-Seidel sweeps apply one colour at a time: colour-sorted blocks keep each
    // colour's reads contiguous (every other block of the element order reads at about half
    // the bandwidth)
    sv.inv_colour = sv.precond != 0;
    FR_TRY(invert_all(sv, prec, flags, s));
    sv.inv_prec = prec;
    return FR_OK;
}

// tile widths (elements per workgroup) of the block apply, per stored precision (FP32 and
// BF16 both take 4 rows per thread)
std::vector<int> block_apply_widths(int p) {
    const int nb = 4 * (p + 1) * (p + 1);
    return {256 / nb, 1024 / nb};
}

struct ApplyArgs {
    const double* r;
    const double* b;
    double* z;
    int color;
    int sub;
    const int* flags;
    int flag;
};

template <class Tin, int NB>
static fr_status apply_as(const Solver& sv, const Group& gr, const ApplyArgs& x, hipStream_t s) {
    using SH = ApplyShape<Tin, NB>;
    GroupArgs ga = group_args(sv, gr, SH::EPB, x.color);
    if (!ga.pfx) { fr_set_error("tile prefix missing"); return FR_EINVAL; }
    if (ga.ntiles == 0) return FR_OK;
    hipLaunchKernelGGL((k_block_apply<Tin, NB>), dim3(ga.ntiles), dim3(SH::threads), 0, s, ga, (const Tin*)sv.d_inv,
                       x.r, x.b, x.z, x.sub, x.flags, x.flag, sv.inv_colour ? 1 : 0);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

template <class Tin>
static fr_status apply_p(const Solver& sv, const Group& gr, const ApplyArgs& x, hipStream_t s) {
    switch (gr.p) {
        case 1: return apply_as<Tin, 16>(sv, gr, x, s);
        case 2: return apply_as<Tin, 36>(sv, gr, x, s);
        case 3: return apply_as<Tin, 64>(sv, gr, x, s);
        case 4: return apply_as<Tin, 100>(sv, gr, x, s);
    }
    fr_set_error("order outside 1..4");
    return FR_EUNSUPPORTED;
}

fr_status launch_block_apply_ex(const Solver& sv, const double* r, const double* b, double* z, int color, bool sub,
                                const int* flags, int flag, hipStream_t s) {
    const ApplyArgs x{r, b, z, color, sub ? 1 : 0, flags, flag};
    for (const Group& gr : sv.groups) {
        switch (sv.inv_prec) {
            case FR_FP64: FR_TRY(apply_p<double>(sv, gr, x, s)); break;
            case FR_FP32: FR_TRY(apply_p<float>(sv, gr, x, s)); break;
            case FR_BF16: FR_TRY(apply_p<uint16_t>(sv, gr, x, s)); break;
            default: fr_set_error("preconditioner not factored"); return FR_EINVAL;
        }
    }
    return FR_OK;
}

fr_status launch_block_apply(const Solver& sv, const double* r, double* z, const int* flags, int flag, hipStream_t s) {
    return launch_block_apply_ex(sv, r, nullptr, z, -1, false, flags, flag, s);
}

// Symmetric block Gauss-Seidel over the elements in colour order, P = (D + L) D^-1 (D + U)
// with L / U the couplings of the Newton operator A to elements of lower / higher colour
// (elements of one colour never share a face, so A restricted to a colour is D):
//   forward   z_k = D_k^-1 (r_k - [A z_{<k}]_k),   k = 0 .. K-1
//   backward  z_k -= D_k^-1 [A z_{>k}]_k,          k = K-2 .. 0
// where z_{<k} (z_{>k}) is z on the colours below (above) k and zero elsewhere.  Costs
// 2 (K - 1) operator applications and about 1.5 block-apply passes per application.
// Forward block Gauss-Seidel (option value 2), P = D + L, is the forward sweep alone:
// K - 1 operator applications over one colour each and one block-apply pass.
fr_status precond_apply(Solver& sv, const double* r, double* z, const KArgs& op, const int* flags, int flag,
                        hipStream_t s) {
    if (sv.precond == 0) return launch_block_apply(sv, r, z, flags, flag, s);
    FR_TRY(dalloc(&sv.d_gst, sv.Ntot));
    const int K = sv.ncolors;
    KArgs a = op;
    a.v = z;
    a.out = sv.d_gst;
    a.flags = flags;
    a.flag = flag;
    // each coupling pass computes the rows of the colour that its block apply updates, from z
    // on the elements of lower colours (forward sweep) or of higher colours (backward sweep)
    for (int k = 0; k < K; ++k) {
        if (k > 0) {
            a.csweep = 1 + k;
            a.cbelow = 1;
            FR_TRY(solver_fused(sv, MODE_LIN, a, s));
        }
        FR_TRY(launch_block_apply_ex(sv, r, k > 0 ? sv.d_gst : nullptr, z, k, false, flags, flag, s));
    }
    for (int k = K - 2; k >= 0 && sv.precond == 1; --k) {
        a.csweep = 1 + k;
        a.cbelow = 0;
        FR_TRY(solver_fused(sv, MODE_LIN, a, s));
        FR_TRY(launch_block_apply_ex(sv, sv.d_gst, nullptr, z, k, true, flags, flag, s));
    }
    return FR_OK;
}

fr_status la_krylov(const Solver& sv, const double* V, size_t ldv, int nv_upd, const double* coef, int cstride,
                    int nv_dot, const double* w_in, double* w_out, bool want_norm, bool mass_only, double* out,
                    int ostride, const int* flags, int flag, hipStream_t s, bool rev) {
    if (nv_upd > MAXV - 1 || nv_dot > MAXV - 1) { fr_set_error("too many Krylov vectors"); return FR_EINVAL; }
    if (mass_only && nv_upd > 0) { fr_set_error("mass-row norm only on a plain norm pass"); return FR_EINVAL; }
    const ChunkArgs ca = chunk_args(sv, flags, flag);
    double* partial = sv.d_part;
    const unsigned grid = chunk_grid(sv);
    const double* w = w_in;
    if (sv.fuse_gs && nv_upd > 0 && nv_dot == nv_upd && w_out && !want_norm && !mass_only && nv_upd <= 32) {
        // update and re-orthogonalising dots share one read of the basis
        if (nv_upd <= 8)
            hipLaunchKernelGGL(k_update_dots<8>, dim3(grid), dim3(RED_THREADS), 0, s, ca, V, ldv, nv_upd, coef, cstride,
                               w_in, w_out, partial, rev ? 1 : 0);
        else if (nv_upd <= 16)
            hipLaunchKernelGGL(k_update_dots<16>, dim3(grid), dim3(RED_THREADS), 0, s, ca, V, ldv, nv_upd, coef,
                               cstride, w_in, w_out, partial, rev ? 1 : 0);
        else
            hipLaunchKernelGGL(k_update_dots<32>, dim3(grid), dim3(RED_THREADS), 0, s, ca, V, ldv, nv_upd, coef,
                               cstride, w_in, w_out, partial, rev ? 1 : 0);
        FR_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_final, dim3(sv.n, nv_dot), dim3(256), 0, s, ca, partial, out, ostride);
        FR_HIP(hipGetLastError());
        return FR_OK;
    }
    if (nv_upd > 0) {
        // the norm of the updated vector rides on the update pass when no dots follow
        const int nrm = (want_norm && nv_dot == 0) ? 1 : 0;
        hipLaunchKernelGGL(k_update, dim3(grid), dim3(RED_THREADS), 0, s, ca, V, ldv, nv_upd, coef, cstride, w_in,
                           w_out, nrm, partial, rev ? 1 : 0);
        FR_HIP(hipGetLastError());
        w = w_out;
        if (nv_dot == 0) {
            if (nrm && out) {   // (no out: the caller reduces the partials in slot 0 itself)
                hipLaunchKernelGGL(k_final, dim3(sv.n, 1), dim3(256), 0, s, ca, partial, out, ostride);
                FR_HIP(hipGetLastError());
            }
            return FR_OK;
        }
    }
    const int ychunks = nv_dot > 0 ? (nv_dot + DB - 1) / DB : 1;
    hipLaunchKernelGGL(k_dots8, dim3(grid, ychunks), dim3(RED_THREADS), 0, s, ca, V, ldv, nv_dot, w,
                       want_norm ? 1 : 0, mass_only ? 1 : 0, partial);
    FR_HIP(hipGetLastError());
    const int nout = nv_dot + (want_norm ? 1 : 0);
    if (nout > 0) {
        hipLaunchKernelGGL(k_final, dim3(sv.n, nout), dim3(256), 0, s, ca, partial, out, ostride);
        FR_HIP(hipGetLastError());
    }
    return FR_OK;
}

fr_status launch_cons(const Solver& sv, const double* q, double* Qc, const int* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_cons, dim3(chunk_grid(sv)), dim3(256), 0, s, chunk_args(sv, flags, GI_NDONE), q, Qc);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status launch_bdf_rhs(const Solver& sv, const double* q, const double* Qn, const double* Qnm1, const double* R,
                         double* b, const int* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_bdf_rhs, dim3(chunk_grid(sv)), dim3(256), 0, s, chunk_args(sv, flags, GI_NDONE), sv.d_step, q,
                       Qn, Qnm1, R, b);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status launch_cons_nm1(const Solver& sv, double* buf, hipStream_t s) {
    hipLaunchKernelGGL(k_cons_nm1, dim3(chunk_grid(sv)), dim3(256), 0, s, chunk_args(sv, nullptr, 0), sv.d_step, buf);
    FR_HIP(hipGetLastError());
    return FR_OK;
}
