// Internal declarations of the lmfr library (host side + kernel argument structs).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lmfr.h"
#include "fr_physics.hpp"

#define FR_MAXN 5   // up to p = 4

// 1-D operators on the Gauss-Legendre solution points
struct OpTab {
    double D[FR_MAXN * FR_MAXN];   // D[i*n+a] = l_a'(xi_i)
    double lamL[FR_MAXN], lamR[FR_MAXN];   // l_a(-1), l_a(+1)
    double gamL[FR_MAXN], gamR[FR_MAXN];   // Radau correction slopes at xi_i
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
};

enum FrMode { MODE_R = 0, MODE_JVP = 1, MODE_AOP = 2, MODE_BLK = 3 };

struct KArgs {
    int E;
    const double* q;      // state [4][E][Np]
    const double* v;      // tangent direction (JVP / AOP)
    const double* tr;     // neighbour traces [E][4][NTV][n] of the scalar type
    double* out;          // R, Jv, Av, or block column base
    double* out2;         // R (JVP) or NULL
    double c_time, inv_dtau;
    int seed0;            // first seeded column (block mode)
    const int* skip;      // device flag: non-zero => the launch does nothing (finished GMRES cycle)
};

struct fr_ctx_s {
    fr_params prm;
    int p, n, Np, pg, m, E;
    PhysConst pc;
    OpTab op;
    GeoTab gt;
    int device;
    bool keep_blocks = false;
    bool geometry_set = false;
    // device storage
    int32_t* d_nbr = nullptr;       // packed [E][4]
    double* d_gsp = nullptr;        // [NGSP][E][Np]
    double* d_gfp = nullptr;        // [NGFP][E][4n]
    double* d_trace = nullptr;      // neighbour traces, sized for Dual<KBLK>
    double* d_trace0 = nullptr;     // value-only traces (block assembly)
    double* d_blk = nullptr;        // [E][nb][nb] FP64 assembly buffer (column-major per element)
    void* d_inv = nullptr;          // [E][nb][nb] inverse blocks in the stored precision
    int inv_prec = -1;
    double* d_blk_keep = nullptr;
    double* d_scal = nullptr;       // small reduction scratch, layout SC_* below
    double* h_scal = nullptr;       // pinned host mirror
    // Krylov workspace
    int kry_m = 0;
    double* d_V = nullptr;          // [(m+1)][N]
    double* d_w = nullptr;          // [N] x 6 work vectors
    double* d_vj = nullptr;         // [vjp adjoint trace buffer]
    double* d_qw = nullptr;         // Newton iterate (ctx-owned so captured graphs stay valid)
    double* d_gs = nullptr;         // device GMRES state (Hessenberg, rotations, scalars)
    int* d_gi = nullptr;            // device GMRES counters and flags
    bool use_graph = true;
    hipStream_t ws = nullptr;       // context stream of the BDF2 step (capturable, default priority)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    void* graph_exec = nullptr;     // hipGraphExec_t of one GMRES(m) cycle
    double graph_ct = 0, graph_idt = 0;
    int graph_m = 0, graph_prec = -1;
    double graph_tol = 0;
    size_t N() const { return (size_t)4 * E * Np; }
};

// layout of the reduction scratch d_scal (doubles)
enum { SC_H1 = 0, SC_H2 = 64, SC_NRM = 128, SC_Y = 192, SC_STATUS = 256, SC_PART = 320,
       SC_TOTAL = 320 + 2048 * 64 };

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

// launchers (fr_kernels.hip)
fr_status launch_geometry(fr_ctx c, const double* xg, const double* vg, hipStream_t s);
fr_status launch_traces(fr_ctx c, const double* q, const double* v, double* trace, int lanes, hipStream_t s);
fr_status launch_residual(fr_ctx c, int mode, const KArgs& a, hipStream_t s);
fr_status launch_vjp(fr_ctx c, const double* q, const double* w, double* out, hipStream_t s);

// linear algebra (fr_linalg.hip)
fr_status launch_block_assembly(fr_ctx c, const double* q, double c_time, double inv_dtau, hipStream_t s);
fr_status launch_block_invert(fr_ctx c, int prec, hipStream_t s);
fr_status launch_block_apply(fr_ctx c, const double* r, double* z, hipStream_t s, const int* skip = nullptr);
// dots of the first N entries; V_i = V + i * c->N()
fr_status la_dots(fr_ctx c, size_t N, const double* V, int nv, const double* w, double* d_out, hipStream_t s);
// w_out = w_in - sum_{i<nv_upd} coef_i V_i; d_out[i] = V_i . w_out (i < nv_dot); d_out[nv_dot] = |w_out|^2
fr_status la_krylov(fr_ctx c, size_t N, const double* V, int nv_upd, const double* d_coef, int nv_dot,
                    const double* w_in, double* w_out, bool want_norm, double* d_out, hipStream_t s,
                    const int* skip = nullptr);
fr_status la_axpy(size_t N, double a, const double* x, double* y, hipStream_t s);
fr_status la_scale_copy(size_t N, double a, const double* x, double* y, hipStream_t s);
fr_status la_norm2(size_t N, const double* x, double* d_out, double* scratch, hipStream_t s);
fr_status launch_bdf_rhs(fr_ctx c, const double* q, const double* Qn, const double* Qnm1, const double* R,
                         double a0, double a1, double a2, double dt, double* b, hipStream_t s);
fr_status launch_cons(fr_ctx c, const double* q, double* Qc, hipStream_t s);
fr_status la_combine(size_t N, const double* V, int nv, const double* d_y, double* out, hipStream_t s);

// device GMRES (fr_gmres.hip)
struct GmresResult { int its; double rel; };
fr_status gmres_device(fr_ctx c, const double* q, const double* b, double* x, int m, double tol, int max_it,
                       double ct, double idt, int prec, GmresResult& out, hipStream_t s);
void gmres_release(fr_ctx c);
size_t gmres_state_doubles(int m);
