// Internal declarations of the lmfr library (host side + kernel argument structs).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <array>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/lmfr.h"
#include "fr_physics.hpp"

// Named host-side range (roctx) over a solver phase, shown by rocprofv3 --marker-trace.  The
// ranges time the host thread: they bracket GPU work where the phase ends with a stream
// synchronisation (a BDF2 step, a Newton iteration, a GMRES solve, a steady solve, the
// autotuner); elsewhere they cover the enqueueing only.
struct PhaseRange {
    explicit PhaseRange(const char* name) { roctxRangePushA(name); }
    ~PhaseRange() { roctxRangePop(); }
    PhaseRange(const PhaseRange&) = delete;
    PhaseRange& operator=(const PhaseRange&) = delete;
};

#define FR_MAXN 5   // up to p = 4

// 1-D operators on the Gauss-Legendre solution points
struct OpTab {
    double D[FR_MAXN * FR_MAXN];   // D[i*n+a] = l_a'(xi_i)
    double lamL[FR_MAXN], lamR[FR_MAXN];   // l_a(-1), l_a(+1)
    double gamL[FR_MAXN], gamR[FR_MAXN];   // Radau correction slopes at xi_i
    double dlamL[FR_MAXN], dlamR[FR_MAXN]; // l_a'(-1), l_a'(+1): derivative traces
};

// Gauss-Lobatto geometry basis evaluated where the metrics are needed
struct GeoTab {
    int m;                                   // geom_order + 1
    double Ls[FR_MAXN * FR_MAXN];            // Ls[i*m+a] = L_a(xi_i)
    double dLs[FR_MAXN * FR_MAXN];           // dLs[i*m+a] = L_a'(xi_i)
    double dLm[FR_MAXN], dLp[FR_MAXN];       // L_a'(-1), L_a'(+1)
};

// Field indices of the per-solution-point geometry array gsp[NGSP][E][Np]
enum { G_XIX = 0, G_XIY, G_ETX, G_ETY, G_IJ, G_UG, G_VG, NGSP };
// Field indices of the per-side geometry array gfp[NGFP][E][4][n]: unit outward normal,
// signed scale sc = sign * |S| (the element-oriented face vector is sc * n), BR2
// coefficient cc = (p+1)^2/8 |S| (1/|J|^- + 1/|J|^+), grid velocity at the face point
enum { F_NX = 0, F_NY, F_SC, F_CC, F_UG, F_VG, NGFP };

struct Geo {
    const double* sp;     // [NGSP][E][Np]
    const double* fp;     // [NGFP][E][4n]
    const int32_t* nbr;   // [E][4]: nb*8 + nb_face*2 + flip
    const int32_t* aff;   // [E]: 1 when the element's metrics are constant (affine map)
    const int32_t* color; // [E]: element colour of the Gauss-Seidel sweeps (no face neighbour shares it)
    const int32_t* corder;// [E]: the elements sorted by colour (ascending; element order within a colour)
    const int32_t* bc;    // [E]: boundary kind of face f in bits 2f..2f+1 (BC_*), 0 interior;
                          // null when the mesh has no boundary face.  A boundary face's
                          // entry in nbr names the element itself, same face, no reversal.
    const double* qinf;   // [4]: far-field primitive state
};

// boundary kinds of the per-element face codes (the ABI codes are -1, -2, -3)
enum { BC_NONE = 0, BC_FARFIELD = 1, BC_SLIP = 2, BC_WALL = 3 };

// R; exact JVP; Newton operator; one seeded block column; R plus the linearisation packs;
// Newton operator from the packs (tangent-only staging)
enum FrMode { MODE_R = 0, MODE_JVP = 1, MODE_AOP = 2, MODE_BLK = 3, MODE_PREP = 4, MODE_LIN = 5, MODE_LINBLK = 6,
              NMODES = 7 };   // MODE_LINBLK: block columns from the packs

// Linearisation packs of a state (written by MODE_PREP, read by MODE_LIN): the values the
// Newton operator's nonlinear point functions need, so that its staged data are tangents.
//   face pack [NPF][E][4n]: own and neighbour traces q^-, q^+ (4 + 4) and the sum of the
//                           uncorrected gradient traces g^- + g^+ (6, viscous only: the BR2
//                           common gradient depends on the two only through their sum)
//   point pack [NPS][E][Np]: q (4) and the corrected gradient (6, viscous only)
constexpr int npf(bool visc) { return visc ? 14 : 8; }
constexpr int nps(bool visc) { return visc ? 10 : 4; }

// Device view of one case (one mesh) of a solver.  A solver concatenates the state
// vectors [4][E][Np] of its cases, each starting at a multiple of CHUNK doubles, and
// the element blocks [E][nb][nb] of its cases.
struct CaseDev {
    int E, Np;
    unsigned long long off;    // first entry of the case's state vector
    unsigned long long boff;   // first entry of the case's element blocks
    unsigned long long fpoff;  // first entry of the case's face pack
    unsigned long long spoff;  // first entry of the case's point pack
    Geo g;
    PhysConst pc;
};

// Per-case scalars of one dual-time step or steady solve (written by the host before it;
// with SER the Newton check updates dtau, idt and res_prev on the device).
struct CaseStep {
    double ct, idt;             // c_time (a0/dt) and inv_dtau of the Newton operator
    double inv_dt, a0, a1, a2;  // BDF coefficients: a0 q^c(q) + a1 Q^n + a2 Q^{n-1}
    double tol_res, tol_pseudo, tol_abs;
    double dtau, dtau_min, dtau_max, r_ser, res_prev;   // SER pseudo-time step control
    double reject_growth;       // step rejection: undo a step whose residual grows beyond this factor (0: off)
    int has_nm1, max_newton, ser;
    int retry;                  // the previous step was undone: keep dtau for the retry
};

// per-case summary published to the host: sum[case * SUM_STRIDE + field]
enum { S_BN = 0, S_BETA, S_TOTAL, S_MORE,      // GMRES: |b|, |r|, iterations, wants another cycle
       S_RES0, S_RES, S_NEWTON, S_GMRES,       // Newton: Res_0, Res_m, iterations, GMRES iterations
       S_NDONE, S_CONV, S_STATUS, S_DTAU,      // flags, status, last pseudo-time step (SER)
       S_REJ,                                  // pseudo-time steps undone (step rejection)
       SUM_STRIDE = 16 };

// work vectors of a step inside Solver::d_w
enum { WB = 0, WR, WQN, WQNM1, WRES, WW, WZ, WDQ, NWORK };

// per-case integer state of a step: gi[case * GI_STRIDE + field]
enum { GI_DONE = 0,   // Arnoldi of the current cycle stopped (skip flag of the cycle's kernels)
       GI_CYC,        // iterations of the current cycle
       GI_TOTAL,      // GMRES iterations of the current Newton step
       GI_MAXIT,      // GMRES iteration cap
       GI_IDLE,       // the case takes no part in the current cycle (skip flag of its update)
       GI_NDONE,      // the case has left the Newton iteration (skip flag of everything)
       GI_STATUS,     // 0 running/converged, 1 non-finite, 2 iteration limit, 3 singular block
       GI_CONV,       // Newton converged
       GI_REJECT,     // the last step was undone: out of this iteration (GI_NDONE set), back in the next
       GI_STRIDE };

// Arguments of the fused residual kernels.  State-sized pointers are bases of the
// concatenated vectors (per-case offsets come from CaseDev).
struct KArgs {
    const double* q;      // state
    const double* v;      // tangent direction (JVP / AOP)
    double* out;          // R, Jv, Av, or the block assembly buffer (block mode)
    double* out2;         // R (JVP) or NULL
    double c_time, inv_dtau;   // time-term coefficients when cstep is NULL
    const CaseStep* cstep;     // per-case coefficients (solver steps) or NULL
    int seed0;            // first seeded column (block mode)
    int ncols;            // block columns from the packs (MODE_LINBLK) on affine static groups: the
                          // columns seed0 .. seed0 + ncols - 1 in one launch (0: one column)
    const int* flags;     // per-case flags (gi layout) or NULL
    int flag;             // which flag skips a case
    double* fpack;        // linearisation packs (MODE_PREP writes, MODE_LIN reads)
    double* spack;
    int csweep;           // MODE_LIN: 1 + the colour whose rows a Gauss-Seidel coupling pass computes
                          // (the elements of other colours are skipped); 0: every element
    int cbelow;           // coupling pass: the tangent v is taken on elements of lower colours (1) or
                          // of higher colours (0), zero elsewhere (the element itself included)
};

// tiles of one launch group (cases of one order / viscous / moving combination)
struct GroupArgs {
    const CaseDev* cases;
    const int* ids;       // case index of each group member
    const int* pfx;       // first tile of each member, [nmem + 1]
    int nmem;
    int ntiles;
    int xcd;              // tile order (Tune::xcd)
    // a Gauss-Seidel coupling pass: per member, the first entry of its colour in Geo::corder and
    // the colour's element count [nmem][2]; the tiles then cover that colour only.  null: every
    // element, in element order
    const int* csel = nullptr;
};

// launch shape of the fused kernel: workgroup width (lanes) and persistent grid size
struct Tune {
    int lanes = 0;        // 0: default of the variant
    int grid = 0;         // 0: one workgroup per tile
    int xcd = 1;          // 1: each XCD walks a contiguous eighth of the tiles; 0: round robin
};

struct Group {
    int p, visc, mov;
    bool aff0 = false;                       // all members affine when the solver was made
    bool bnd = false;                        // the members' meshes have boundary faces
    std::vector<int> ids;
    int* d_ids = nullptr;
    std::vector<std::pair<int, int*>> pfx;   // tile width (elements) -> device prefix
    std::vector<long long> elems;            // elements of each member
    std::vector<std::array<int, 6>> cofs;    // per member: first entry of each colour in corder (6: end)
    struct ColorTiles { int epb, color, ntiles; int* d_pfx; int* d_csel; };
    std::vector<ColorTiles> ctiles;          // tile prefixes of the Gauss-Seidel coupling passes
    Tune tune[NMODES];                       // per mode
    const int* tile_pfx(int epb) const {
        for (auto& x : pfx) if (x.first == epb) return x.second;
        return nullptr;
    }
    const ColorTiles* color_tiles(int epb, int color) const {
        for (auto& x : ctiles) if (x.epb == epb && x.color == color) return &x;
        return nullptr;
    }
    int ntiles(int epb) const {
        long long t = 0;
        for (long long e : elems) t += (e + epb - 1) / epb;
        return (int)t;
    }
};

struct Solver;

struct fr_ctx_s {
    fr_params prm;
    int p, n, Np, pg, m, E;
    PhysConst pc;
    OpTab op;
    GeoTab gt;
    int device;
    bool geometry_set = false;
    // device storage
    int32_t* d_nbr = nullptr;       // packed [E][4]
    double* d_gsp = nullptr;        // [NGSP][E][Np]
    double* d_gfp = nullptr;        // [NGFP][E][4n]
    int32_t* d_aff = nullptr;       // [E] affine-element flags
    int32_t* d_color = nullptr;     // [E] element colours
    int32_t* d_corder = nullptr;    // [E] elements sorted by colour
    std::array<int, 6> cofs{};      // first entry of each colour in d_corder (entry ncolors: E)
    int32_t* d_bc = nullptr;        // [E] boundary face codes (null: no boundary face)
    double* d_qinf = nullptr;       // [4] far-field state
    bool has_farfield = false, farfield_set = false;
    int ncolors = 0;
    bool all_affine = false;        // every element affine at the current geometry
    double* d_trace = nullptr;      // neighbour traces (adjoint path)
    double* d_vj = nullptr;         // adjoint trace buffer
    Solver* self = nullptr;         // one-case solver of the context's own entry points
    size_t N() const { return (size_t)4 * E * Np; }
    Geo geo() const { return Geo{d_gsp, d_gfp, d_nbr, d_aff, d_color, d_corder, d_bc, d_qinf}; }
};

// why a context cannot be evaluated yet, or null
inline const char* ctx_not_ready(const fr_ctx_s* c) {
    if (!c->geometry_set) return "fr_set_geometry has not been called";
    if (c->has_farfield && !c->farfield_set) return "the mesh has far-field faces: fr_set_farfield has not been called";
    return nullptr;
}

// A solver: one or more cases advanced together (fr_batch, or the one-case solver of a
// context).  Owns the concatenated work vectors, blocks and device GMRES state.
struct Solver {
    std::vector<fr_ctx> cs;
    int n = 0;
    std::vector<size_t> off, len, boff;    // state offset / padded length, block offset per case
    size_t Ntot = 0, Btot = 0;
    int nchunks = 0;
    CaseDev* d_cases = nullptr;
    int* d_chunk_case = nullptr;           // [nchunks]
    int* d_case_chunk = nullptr;           // [n + 1] first chunk of each case
    std::vector<Group> groups;
    int device = 0;
    // preconditioner
    double* d_blk = nullptr;               // FP64 assembly buffer (column-major blocks)
    void* d_inv = nullptr;                 // inverse blocks in the stored precision
    size_t inv_bytes = 0;                  // capacity of d_inv
    int inv_prec = -1;
    // inverse blocks in colour order (chosen at factor time with the Gauss-Seidel sweeps): slot
    // k of a case holds the block of its element corder[k], so each colour's blocks are one
    // contiguous range; otherwise slot e holds element e's block
    bool inv_colour = false;
    bool keep_blocks = false;
    double* d_blk_keep = nullptr;
    int precond = 0;                       // 0: element-block Jacobi, 1: symmetric block Gauss-Seidel
    int ncolors = 1;                       // colours of the sweeps (max over the cases)
    double* d_gst = nullptr;               // Gauss-Seidel couplings [Ntot]
    double f_ct = 0.0, f_idt = 0.0;        // time coefficients of the last context-level factor
    bool reject_on = false;                // the running steady solve undoes steps that raise the residual
    // step workspace
    int kry_m = 0;
    double* d_q = nullptr;                 // Newton iterate
    double* d_w = nullptr;                 // NWORK vectors
    double* d_V = nullptr;                 // (m+1) Krylov vectors
    double* d_gs = nullptr;                // per-case GMRES state [n][gs_stride]
    int gs_stride = 0;
    int* d_gi = nullptr;                   // per-case flags [n][GI_STRIDE]
    double* d_part = nullptr;              // reduction partials [nchunks][MAXV]
    CaseStep* d_step = nullptr;            // [n]
    double* d_sum = nullptr;               // per-case summary [n][SUM_STRIDE]
    double* d_fpack = nullptr;             // linearisation packs of the Newton iterate
    double* d_spack = nullptr;
    size_t fpack_len = 0, spack_len = 0;
    bool op_packs = false;                 // fr_bdf_operator through the packs (two passes)
    double* d_rscratch = nullptr;          // R of that path
    double* h_pin = nullptr;               // pinned host staging
    size_t h_pin_doubles = 0;
    hipStream_t ws = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    bool use_graph = true;
    void* graph_exec = nullptr;
    int graph_m = 0, graph_prec = -1, graph_passes = 0, graph_precond = -1, graph_cl = -1;
    std::vector<char> graph_aff;           // per group: all members affine when the cycle was captured
    int gs_passes = 1;                     // classical Gram-Schmidt passes per Arnoldi step (1 or 2)
    bool fuse_gs = true;                   // two passes: update and re-orthogonalising dots in one read
    size_t N(int c) const { return (size_t)4 * cs[c]->E * cs[c]->Np; }
};

struct fr_batch_s {
    Solver sv;
};

constexpr int CHUNK = 4096;   // alignment of case vectors; unit of the segmented reductions
constexpr int MAXV = 160;     // max vectors in one multi-dot: Krylov dimension up to MAXV - 4

// error handling
void fr_set_error(const std::string& s);
#define FR_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            fr_set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
            return FR_EHIP;                                                          \
        }                                                                            \
    } while (0)

#define FR_TRY(x)                              \
    do {                                       \
        fr_status st_ = (x);                   \
        if (st_ != FR_OK) return st_;          \
    } while (0)

template <class T>
fr_status dalloc(T** p, size_t count) {
    if (*p) return FR_OK;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T) + 16);
    if (e != hipSuccess) {
        *p = nullptr;
        fr_set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return FR_ENOMEM;
    }
    return FR_OK;
}
inline void dfree(void* p) { if (p) (void)hipFree(p); }

// geometry and traces (fr_kernels.hip)
fr_status launch_geometry(fr_ctx c, const double* xg, const double* vg, hipStream_t s);
fr_status launch_traces(fr_ctx c, const double* q, double* trace, hipStream_t s);
fr_status launch_vjp(fr_ctx c, const double* q, const double* w, double* out, hipStream_t s);

// fused residual kernels of one group (fr_fused_p*.hip)
fr_status launch_fused(const Solver& sv, const Group& gr, int mode, const KArgs& a, const Tune& t, hipStream_t s);
template <int P>
fr_status launch_fused_p(const Solver& sv, const Group& gr, int mode, const KArgs& a, const Tune& t, hipStream_t s);
template <> fr_status launch_fused_p<1>(const Solver&, const Group&, int, const KArgs&, const Tune&, hipStream_t);
template <> fr_status launch_fused_p<2>(const Solver&, const Group&, int, const KArgs&, const Tune&, hipStream_t);
template <> fr_status launch_fused_p<3>(const Solver&, const Group&, int, const KArgs&, const Tune&, hipStream_t);
template <> fr_status launch_fused_p<4>(const Solver&, const Group&, int, const KArgs&, const Tune&, hipStream_t);
// every group of the solver with its tuned shape
fr_status solver_fused(const Solver& sv, int mode, const KArgs& a, hipStream_t s);
// tile widths (elements per workgroup) a group may be launched with
std::vector<int> fused_tile_widths(int p);

// solver set-up (fr_solver.hip)
fr_status solver_init(Solver& sv, const fr_ctx* ctxs, int n);
void solver_free(Solver& sv);
fr_status solver_ensure_blocks(Solver& sv, int prec);
fr_status solver_ensure_step(Solver& sv, int m, int prec);
fr_status solver_reserve(Solver& sv, int m, int prec);
size_t prec_bytes(int prec);

// preconditioner (fr_linalg.hip)
fr_status launch_block_assembly(Solver& sv, const double* q, const KArgs& base, hipStream_t s);
fr_status launch_block_invert(Solver& sv, int prec, const int* flags, hipStream_t s);
// explicit inverses of one group's element blocks, Gauss-Jordan on the matrix cores (fr_invert.hip)
fr_status launch_block_invert_group(Solver& sv, int p, const GroupArgs& ga, int prec, const int* flags,
                                    hipStream_t s);
fr_status launch_block_apply(const Solver& sv, const double* r, double* z, const int* flags, int flag, hipStream_t s);
// restricted to the elements of one colour (color >= 0; -1: all):
//   sub = false: z_e = D_e^-1 (r_e - b_e) (b may be null);  sub = true: z_e -= D_e^-1 r_e
fr_status launch_block_apply_ex(const Solver& sv, const double* r, const double* b, double* z, int color, bool sub,
                                const int* flags, int flag, hipStream_t s);
// z = P^-1 r with the solver's preconditioner; the Gauss-Seidel sweeps apply the Newton
// operator described by op (its v and out are set here)
fr_status precond_apply(Solver& sv, const double* r, double* z, const KArgs& op, const int* flags, int flag,
                        hipStream_t s);
// segmented reductions over the concatenated vectors: for every case c (not skipped),
//   w_out = w_in - sum_{i<nv_upd} coef_c[i] V_i            (coef_c = coef + c * cstride)
//   out_c[i] = V_i . w_out (i < nv_dot), out_c[nv_dot] = |w_out|^2 (want_norm)
// (out_c = out + c * ostride); mass_only restricts the norm to the first E Np entries.
// rev: the update passes walk the chunks from the last to the first, so that a pass that follows
// one over the same basis starts on the chunks still in the Infinity Cache (same results)
fr_status la_krylov(const Solver& sv, const double* V, size_t ldv, int nv_upd, const double* coef, int cstride,
                    int nv_dot, const double* w_in, double* w_out, bool want_norm, bool mass_only, double* out,
                    int ostride, const int* flags, int flag, hipStream_t s, bool rev = false);
fr_status launch_bdf_rhs(const Solver& sv, const double* q, const double* Qn, const double* Qnm1, const double* R,
                         double* b, const int* flags, hipStream_t s);
fr_status launch_cons(const Solver& sv, const double* q, double* Qc, const int* flags, hipStream_t s);
// q^c in place for the cases that have a q^{n-1}
fr_status launch_cons_nm1(const Solver& sv, double* buf, hipStream_t s);
std::vector<int> block_apply_widths(int p);

// device GMRES (fr_gmres.hip)
size_t gmres_state_doubles(int m);
fr_status gmres_device(Solver& sv, int m, int prec, int max_it, hipStream_t s);
void gmres_release(Solver& sv);
// Newton loop of a step: iterate in d_q, q^{n-1} states in WQNM1; leaves the per-case
// summary in h_pin
fr_status solver_newton(Solver& sv, const fr_step_opts* opts, hipStream_t s);
// one dual-time step of every case (copies in and out of the caller's arrays)
fr_status solver_steady(Solver& sv, double* const* q, const fr_steady_opts* opts, fr_steady_stats* stats,
                        hipStream_t s);
fr_status solver_step(Solver& sv, double* const* q, const double* const* q_nm1, const fr_step_opts* opts,
                      fr_step_stats* stats, hipStream_t caller);
fr_status solver_autotune(Solver& sv, const char* cache_path, hipStream_t s);
