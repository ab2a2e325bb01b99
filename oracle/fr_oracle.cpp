// ORACLE -- test infrastructure only.
//
// A plain, serial, double-precision CPU implementation of the implicit
// Weiss-Smith-preconditioned flux reconstruction (FR/CPR) method of
// Wang & Yu, "An Implicit High-Order Preconditioned Flux Reconstruction Method
// for Low-Mach-Number Flow Simulation with Dynamic Meshes" (arXiv:1903.06304).
// It exists only to check the GPU library: only the tests, the smoke check and
// the benchmark's CPU-baseline leg may load it. It shares no code, header,
// table or constant with the GPU library.
//
// Everything is templated on the scalar type so that the same code runs in
// double (residual) and in std::complex<double> (complex-step derivatives:
// JVP, dense Jacobian, VJP, diagonal blocks).  Non-analytic operations
// (abs, max, min) compare real parts; ties pick the first argument, and
// d|x|/dx = +1 at x = 0.
//
// Paper passages followed (sections / equations of the paper):
//   non-dimensional NS, fluxes, stresses ........ Sec. 2.1, Eqs. (comp_ns),
//                                                 (convection), (diffusion), (shear_stress)
//   M, Gamma, Theta, eigenvalues, epsilon ....... Sec. 2.2, Eqs. (jacobian),
//                                                 (preconditioning), (theta), (eigenvalues),
//                                                 (eigenvalues_para), (eps_nonmove)
//   moving-mesh form, implicit GCL .............. Sec. 2.3, Eqs. (unsteady_pre_mov_pdomain),
//                                                 (eps_move) and A_n,mov
//   FR/CPR residual, Radau correction ........... Sec. 3.1, Eq. (cpr_ns), F^cor/G^cor
//   common flux mapping, Rusanov, BR2 ........... Sec. 3.1, Eqs. (norm_f_2), (Rosanov)
//   BDF2 dual-time Newton system ................ Sec. 3.2, Eqs. (unsteady_pre_discretized_1..3)
//   GMRES, block Jacobi, Jacobian lag ........... Sec. 3.2 and the parallel-setup paragraph of Sec. 4
//
// Readings where the paper is silent (solution points, BR2 details, trace of
// the flux polynomial, ...) are the ones listed in the design notes of the
// repository; each is marked "reading" where it is used.
//
// Derivatives: complex step, Im R(q + i h v) / h with h = 1e-30.
// Parity of this oracle is pinned by the "not gpu" tests (operators, M, Gamma,
// eigenvalues, flux consistency, free-stream preservation, conservation,
// FR == DG, consistency order, BDF2 order, LU / GMRES, FD derivatives).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <functional>
#include <vector>

using cplx = std::complex<double>;

namespace ora {

// ---------------------------------------------------------------- scalars
inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }
template <class T> inline T sabs(const T& x) { return re(x) >= 0.0 ? x : T(-x); }
template <class T> inline T smax(const T& a, const T& b) { return re(a) >= re(b) ? a : b; }
template <class T> inline T smin(const T& a, const T& b) { return re(a) <= re(b) ? a : b; }
inline double ssqrt(double x) { return std::sqrt(x); }
inline cplx ssqrt(const cplx& x) { return std::sqrt(x); }

// Op-counting scalar: a double that tallies every arithmetic operation applied to it
// (additions and subtractions, multiplications, divisions, square roots).  Running the
// residual on it counts the floating-point work one evaluation does on the state; pure
// geometry and operator-table arithmetic (doubles) is set-up work and is not counted.
struct OpTally { unsigned long long add = 0, mul = 0, div = 0, sqrt = 0; };
static OpTally g_tally;
struct Cnt {
    double v;
    Cnt() : v(0.0) {}
    Cnt(double x) : v(x) {}
    Cnt operator-() const { return Cnt(-v); }
    Cnt& operator+=(const Cnt& b) { ++g_tally.add; v += b.v; return *this; }
    Cnt& operator-=(const Cnt& b) { ++g_tally.add; v -= b.v; return *this; }
    Cnt& operator*=(const Cnt& b) { ++g_tally.mul; v *= b.v; return *this; }
    Cnt& operator/=(const Cnt& b) { ++g_tally.div; v /= b.v; return *this; }
};
inline Cnt operator+(const Cnt& a, const Cnt& b) { ++g_tally.add; return Cnt(a.v + b.v); }
inline Cnt operator-(const Cnt& a, const Cnt& b) { ++g_tally.add; return Cnt(a.v - b.v); }
inline Cnt operator*(const Cnt& a, const Cnt& b) { ++g_tally.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(const Cnt& a, const Cnt& b) { ++g_tally.div; return Cnt(a.v / b.v); }
inline double re(const Cnt& x) { return x.v; }
inline Cnt ssqrt(const Cnt& x) { ++g_tally.sqrt; return Cnt(std::sqrt(x.v)); }

// ---------------------------------------------------------------- 1-D operators
// Legendre P_k and P_k' by the three-term recurrence.
static void legendre(int k, double x, double& P, double& dP) {
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (k == 0) { P = 1.0; dP = 0.0; return; }
    for (int m = 1; m < k; ++m) {
        double p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
        double d2 = d0 + (2 * m + 1) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    P = p1; dP = d1;
}

// Gauss-Legendre nodes and weights (Newton on P_n), ascending.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0); w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP; legendre(n, z, P, dP);
            double dz = P / dP; z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double P, dP; legendre(n, z, P, dP);
        x[i] = z; w[i] = 2.0 / ((1.0 - z * z) * dP * dP);
    }
}

// Gauss-Lobatto nodes: -1, roots of P'_{n-1}, +1.
static void gauss_lobatto(int n, std::vector<double>& x) {
    x.assign(n, 0.0);
    x[0] = -1.0; x[n - 1] = 1.0;
    for (int i = 1; i < n - 1; ++i) {
        double z = -std::cos(M_PI * i / (n - 1));
        for (int it = 0; it < 100; ++it) {
            // f = P'_{n-1}(z); f' from the Legendre ODE: (1-z^2)P'' = 2zP' - m(m+1)P
            int m = n - 1; double P, dP; legendre(m, z, P, dP);
            double d2P = (2 * z * dP - m * (m + 1) * P) / (1 - z * z);
            double dz = dP / d2P; z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
    }
}

// Lagrange basis l_a(x) on nodes, and its derivative.
static double lagrange(const std::vector<double>& nd, int a, double x) {
    double v = 1.0;
    for (int m = 0; m < (int)nd.size(); ++m) if (m != a) v *= (x - nd[m]) / (nd[a] - nd[m]);
    return v;
}
static double lagrange_d(const std::vector<double>& nd, int a, double x) {
    double s = 0.0;
    for (int k = 0; k < (int)nd.size(); ++k) {
        if (k == a) continue;
        double t = 1.0 / (nd[a] - nd[k]);
        for (int m = 0; m < (int)nd.size(); ++m) if (m != a && m != k) t *= (x - nd[m]) / (nd[a] - nd[m]);
        s += t;
    }
    return s;
}

struct Ops {
    int p, n, pg, ng1;
    std::vector<double> xi, w;        // Gauss-Legendre solution points (reading: GL)
    std::vector<double> D;            // D[i*n+a] = l_a'(xi_i)
    std::vector<double> lamL, lamR;   // l_a(-1), l_a(+1)
    std::vector<double> gamL, gamR;   // g_L'(xi_i), g_R'(xi_i), Radau corrections
    std::vector<double> gll;          // geometry nodes
    void build(int p_, int pg_) {
        p = p_; n = p + 1; pg = pg_; ng1 = pg + 1;
        gauss_legendre(n, xi, w);
        D.assign(n * n, 0.0); lamL.assign(n, 0.0); lamR.assign(n, 0.0);
        gamL.assign(n, 0.0); gamR.assign(n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < n; ++a) D[i * n + a] = lagrange_d(xi, a, xi[i]);
        for (int a = 0; a < n; ++a) { lamL[a] = lagrange(xi, a, -1.0); lamR[a] = lagrange(xi, a, 1.0); }
        // Sec. 3.1: g_L = right Radau polynomial of degree p+1, g_R = left Radau polynomial.
        //   g_L = ((-1)^(p+1)/2) (P_{p+1} - P_p),   g_R = (1/2)(P_{p+1} + P_p)
        double sgn = ((p + 1) % 2 == 0) ? 1.0 : -1.0;
        for (int i = 0; i < n; ++i) {
            double P1, dP1, P0, dP0;
            legendre(p + 1, xi[i], P1, dP1); legendre(p, xi[i], P0, dP0);
            gamL[i] = 0.5 * sgn * (dP1 - dP0);
            gamR[i] = 0.5 * (dP1 + dP0);
        }
        gauss_lobatto(ng1, gll);
    }
};

// ---------------------------------------------------------------- context
struct Ctx {
    // parameters, Sec. 2.1 non-dimensionalisation
    int p, n, Np, pg, ng, E, viscous, moving;
    double gam, Ma, Re, Pr, mu, kappa, Ma_inf, Rg, Cp, kc;
    Ops op;
    // nbr[e*4+f] >= 0: neighbour element; < 0: boundary face of kind -nbr (1 far field,
    // 2 slip wall, 3 adiabatic no-slip wall)
    std::vector<int> nbr, nbr_face; std::vector<signed char> flip;
    double qinf[4] = {0.0, 0.0, 0.0, 0.0};   // far-field primitive state (p, u, v, T)
    // geometry at solution points, [E][Np]
    std::vector<double> xs, ys, jac, xix, xiy, etx, ety, ugs, vgs;
    // per element side [E][4][n]: element-oriented face vector S = |J| grad(xi) (faces 0,1)
    // or |J| grad(eta) (faces 2,3), |J| at the flux point, grid velocity at the flux point
    std::vector<double> Sx, Sy, Jf, ugf, vgf;
    std::vector<double> xg, vg;
    int threads = 1;   // element-loop threads of the residual (OpenMP builds only)
};

static inline double face_sign(int f) { return (f == 1 || f == 3) ? 1.0 : -1.0; }

// index of solution point on the line through face point k of face f, a-th along the normal
static inline int line_pt(int n, int f, int k, int a) {
    return (f < 2) ? (a + n * k) : (k + n * a);
}

// Evaluate the isoparametric map and its derivatives at reference point (r, s).
static void map_eval(const Ctx& c, int e, double r, double s, double& x, double& y,
                     double& xr, double& xs_, double& yr, double& ys_, double& u, double& v) {
    const int m = c.op.ng1;
    x = y = xr = xs_ = yr = ys_ = u = v = 0.0;
    for (int b = 0; b < m; ++b)
        for (int a = 0; a < m; ++a) {
            double La = lagrange(c.op.gll, a, r), Lb = lagrange(c.op.gll, b, s);
            double dLa = lagrange_d(c.op.gll, a, r), dLb = lagrange_d(c.op.gll, b, s);
            size_t id = (size_t)e * c.ng + a + m * b;
            double X = c.xg[id], Y = c.xg[(size_t)c.E * c.ng + id];
            x += X * La * Lb; y += Y * La * Lb;
            xr += X * dLa * Lb; xs_ += X * La * dLb;
            yr += Y * dLa * Lb; ys_ += Y * La * dLb;
            if (c.moving) {
                u += c.vg[id] * La * Lb; v += c.vg[(size_t)c.E * c.ng + id] * La * Lb;
            }
        }
}

// Sec. 2.3: |J| = x_xi y_eta - x_eta y_xi; xi_x = y_eta/|J|, xi_y = -x_eta/|J|,
// eta_x = -y_xi/|J|, eta_y = x_xi/|J|.  Face vectors |J| grad(xi) = (y_eta, -x_eta),
// |J| grad(eta) = (-y_xi, x_xi), computed once per face from its owner side.
static void build_geometry(Ctx& c) {
    const int n = c.n, Np = c.Np, E = c.E;
    c.xs.assign((size_t)E * Np, 0); c.ys = c.jac = c.xix = c.xiy = c.etx = c.ety = c.ugs = c.vgs = c.xs;
    c.Sx.assign((size_t)E * 4 * n, 0); c.Sy = c.Jf = c.ugf = c.vgf = c.Sx;
    for (int e = 0; e < E; ++e)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double x, y, xr, xs_, yr, ys_, u, v;
                map_eval(c, e, c.op.xi[i], c.op.xi[j], x, y, xr, xs_, yr, ys_, u, v);
                size_t id = (size_t)e * Np + i + n * j;
                double J = xr * ys_ - xs_ * yr;
                c.xs[id] = x; c.ys[id] = y; c.jac[id] = J;
                c.xix[id] = ys_ / J; c.xiy[id] = -xs_ / J;
                c.etx[id] = -yr / J; c.ety[id] = xr / J;
                c.ugs[id] = u; c.vgs[id] = v;
            }
    // own-side evaluation of every side
    std::vector<double> sx(c.Sx.size()), sy(c.Sx.size()), ug(c.Sx.size()), vg(c.Sx.size());
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f)
            for (int k = 0; k < n; ++k) {
                double r = (f == 0) ? -1.0 : (f == 1) ? 1.0 : c.op.xi[k];
                double s = (f == 2) ? -1.0 : (f == 3) ? 1.0 : c.op.xi[k];
                double x, y, xr, xs_, yr, ys_, u, v;
                map_eval(c, e, r, s, x, y, xr, xs_, yr, ys_, u, v);
                size_t id = ((size_t)e * 4 + f) * n + k;
                if (f < 2) { sx[id] = ys_; sy[id] = -xs_; } else { sx[id] = -yr; sy[id] = xr; }
                c.Jf[id] = xr * ys_ - xs_ * yr;
                ug[id] = u; vg[id] = v;
            }
    // share the face vector and grid velocity from the owner (smaller (e,f) index)
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f) {
            int e2 = c.nbr[e * 4 + f], f2 = c.nbr_face[e * 4 + f], fl = c.flip[e * 4 + f];
            bool own = e2 < 0 || (e * 4 + f) <= (e2 * 4 + f2);
            for (int k = 0; k < n; ++k) {
                size_t id = ((size_t)e * 4 + f) * n + k;
                if (own) { c.Sx[id] = sx[id]; c.Sy[id] = sy[id]; c.ugf[id] = ug[id]; c.vgf[id] = vg[id]; continue; }
                int k2 = fl ? n - 1 - k : k;
                size_t id2 = ((size_t)e2 * 4 + f2) * n + k2;
                // owner's outward vector, negated, is this side's outward vector
                double ox = face_sign(f2) * sx[id2], oy = face_sign(f2) * sy[id2];
                c.Sx[id] = -face_sign(f) * ox; c.Sy[id] = -face_sign(f) * oy;
                c.ugf[id] = ug[id2]; c.vgf[id] = vg[id2];
            }
        }
}

// ---------------------------------------------------------------- physics
// Sec. 2.1: rho = p/(R T), E = p/(gamma-1) + rho|v|^2/2, q^c = (rho, rho u, rho v, E).
template <class T> static void cons(const Ctx& c, const T* q, T* qc) {
    T rho = q[0] / (c.Rg * q[3]);
    T E = q[0] / (c.gam - 1.0) + 0.5 * rho * (q[1] * q[1] + q[2] * q[2]);
    qc[0] = rho; qc[1] = rho * q[1]; qc[2] = rho * q[2]; qc[3] = E;
}

// Sec. 2.1 Eqs. (convection), (diffusion), (shear_stress): f = f_inv - f_vis, g = g_inv - g_vis.
// gx, gy: gradient of (p, u, v, T).
template <class T> static void phys_flux(const Ctx& c, const T* q, const T* gx, const T* gy, T* f, T* g) {
    T qc[4]; cons(c, q, qc);
    T p = q[0], u = q[1], v = q[2];
    f[0] = qc[0] * u; f[1] = qc[0] * u * u + p; f[2] = qc[0] * u * v; f[3] = (qc[3] + p) * u;
    g[0] = qc[0] * v; g[1] = qc[0] * u * v; g[2] = qc[0] * v * v + p; g[3] = (qc[3] + p) * v;
    if (c.viscous) {
        T ux = gx[1], uy = gy[1], vx = gx[2], vy = gy[2], Tx = gx[3], Ty = gy[3];
        T txx = c.mu * (4.0 / 3.0 * ux - 2.0 / 3.0 * vy);
        T tyy = c.mu * (4.0 / 3.0 * vy - 2.0 / 3.0 * ux);
        T txy = c.mu * (uy + vx);
        double ir = 1.0 / c.Re;
        f[1] -= ir * txx; f[2] -= ir * txy; f[3] -= ir * (u * txx + v * txy + c.kc * Tx);
        g[1] -= ir * txy; g[2] -= ir * tyy; g[3] -= ir * (u * txy + v * tyy + c.kc * Ty);
    }
}

// Sec. 2.2 Eq. (jacobian): M = d q^c / d q^p, rho_p = 1/(RT), rho_T = -rho/T, h = Cp T + |v|^2/2.
template <class T> static void mat_M(const Ctx& c, const T* q, T M[4][4]) {
    T u = q[1], v = q[2], Tt = q[3];
    T rho = q[0] / (c.Rg * Tt);
    T rp = 1.0 / (c.Rg * Tt), rT = -rho / Tt;
    T h = c.Cp * Tt + 0.5 * (u * u + v * v);
    M[0][0] = rp;         M[0][1] = 0.0;     M[0][2] = 0.0;     M[0][3] = rT;
    M[1][0] = rp * u;     M[1][1] = rho;     M[1][2] = 0.0;     M[1][3] = rT * u;
    M[2][0] = rp * v;     M[2][1] = 0.0;     M[2][2] = rho;     M[2][3] = rT * v;
    M[3][0] = rp * h - 1.0; M[3][1] = rho * u; M[3][2] = rho * v; M[3][3] = rT * h + rho * c.Cp;
}

// Sec. 2.2 Eqs. (eps_nonmove), (eps_move): eps = min(1, max(kappa Ma_inf, Ma)), Ma from
// v - v_g; U_r = eps c, c^2 = gamma R T.
template <class T> static T ref_velocity(const Ctx& c, const T* q, double ug, double vg) {
    T cs = ssqrt(c.gam * c.Rg * q[3]);
    T du = q[1] - ug, dv = q[2] - vg;
    T Ma = ssqrt(du * du + dv * dv) / cs;
    T eps = smin(T(1.0), smax(T(c.kappa * c.Ma_inf), Ma));
    return eps * cs;
}

// Sec. 2.2 Eqs. (preconditioning), (theta): Gamma = M with rho_p replaced by
// Theta = 1/U_r^2 - rho_T/(rho Cp).
template <class T> static void mat_Gamma(const Ctx& c, const T* q, double ug, double vg, T G[4][4]) {
    T u = q[1], v = q[2], Tt = q[3];
    T rho = q[0] / (c.Rg * Tt);
    T rT = -rho / Tt;
    T Ur = ref_velocity(c, q, ug, vg);
    T Th = 1.0 / (Ur * Ur) - rT / (rho * c.Cp);
    T h = c.Cp * Tt + 0.5 * (u * u + v * v);
    G[0][0] = Th;         G[0][1] = 0.0;     G[0][2] = 0.0;     G[0][3] = rT;
    G[1][0] = Th * u;     G[1][1] = rho;     G[1][2] = 0.0;     G[1][3] = rT * u;
    G[2][0] = Th * v;     G[2][1] = 0.0;     G[2][2] = rho;     G[2][3] = rT * v;
    G[3][0] = Th * h - 1.0; G[3][1] = rho * u; G[3][2] = rho * v; G[3][3] = rT * h + rho * c.Cp;
}

// Sec. 2.2 Eqs. (eigenvalues), (eigenvalues_para) with u_n = (v - v_g).n (Sec. 2.3):
// largest |eigenvalue| of Gamma^-1 A_n,mov.
template <class T> static T max_eig(const Ctx& c, const T* q, double nx, double ny, double ug, double vg) {
    T Tt = q[3];
    T rho = q[0] / (c.Rg * Tt);
    T rp = 1.0 / (c.Rg * Tt), rT = -rho / Tt;
    T Ur = ref_velocity(c, q, ug, vg);
    T un = (q[1] - ug) * nx + (q[2] - vg) * ny;
    T beta = rp + rT / (rho * c.Cp);
    T alpha = (1.0 - beta * Ur * Ur) / 2.0;
    T unp = un * (1.0 - alpha);
    T cp = ssqrt(alpha * alpha * un * un + Ur * Ur);
    return smax(smax(sabs(un), sabs(unp + cp)), sabs(unp - cp));
}

// Sec. 3.1: normal inviscid flux on a (moving) face, f_n = f n_x + g n_y - (v_g.n) q^c.
template <class T> static void normal_inviscid(const Ctx& c, const T* q, double nx, double ny,
                                               double ug, double vg, T* fn) {
    T qc[4]; cons(c, q, qc);
    T p = q[0], u = q[1], v = q[2];
    T f[4] = {qc[0] * u, qc[0] * u * u + p, qc[0] * u * v, (qc[3] + p) * u};
    T g[4] = {qc[0] * v, qc[0] * u * v, qc[0] * v * v + p, (qc[3] + p) * v};
    double vgn = ug * nx + vg * ny;
    for (int r = 0; r < 4; ++r) fn[r] = f[r] * nx + g[r] * ny - vgn * qc[r];
}

// NS physics for the generic FR driver (4 variables).
struct NSPhys {
    static constexpr int NV = 4;
    const Ctx* c;
    template <class T> void flux(const T* q, const T* gx, const T* gy, T* f, T* g, T* qc) const {
        phys_flux(*c, q, gx, gy, f, g); cons(*c, q, qc);
    }
    // Common normal flux for unit normal n pointing out of the "-" (own) side.
    // Inviscid: preconditioned Rusanov, Eq. (Rosanov), Gamma~ and |lambda|max at the
    // averaged primitive state. Viscous: q^com = average; BR2 common gradient
    // (reading: face-local Radau lifting at the face, no extra penalty).
    template <class T> void common(const T* qL, const T* qR, const T* gxL, const T* gyL,
                                   const T* gxR, const T* gyR, double nx, double ny, double Smag,
                                   double JfL, double JfR, double ug, double vg, T* fn, T* qcom) const {
        const Ctx& C = *c;
        T fL[4], fR[4]; normal_inviscid(C, qL, nx, ny, ug, vg, fL); normal_inviscid(C, qR, nx, ny, ug, vg, fR);
        T qb[4]; for (int r = 0; r < 4; ++r) qb[r] = 0.5 * (qL[r] + qR[r]);
        T G[4][4]; mat_Gamma(C, qb, ug, vg, G);
        T lam = max_eig(C, qb, nx, ny, ug, vg);
        for (int r = 0; r < 4; ++r) {
            T gd = 0.0;
            for (int s = 0; s < 4; ++s) gd += G[r][s] * (qR[s] - qL[s]);
            fn[r] = 0.5 * (fL[r] + fR[r]) - 0.5 * lam * gd;
        }
        for (int r = 0; r < 4; ++r) qcom[r] = qb[r];
        if (!C.viscous) return;
        const double pf = 0.5 * (C.p + 1) * (C.p + 1);
        double cL = pf * Smag / JfL, cR = pf * Smag / JfR;
        T gx[4], gy[4];
        for (int r = 0; r < 4; ++r) {
            // r^- = cL (q^com - q^-) n,  r^+ = cR (q^com - q^+) (-n)
            T rxL = cL * (qcom[r] - qL[r]) * nx, ryL = cL * (qcom[r] - qL[r]) * ny;
            T rxR = -cR * (qcom[r] - qR[r]) * nx, ryR = -cR * (qcom[r] - qR[r]) * ny;
            gx[r] = 0.5 * ((gxL[r] + rxL) + (gxR[r] + rxR));
            gy[r] = 0.5 * ((gyL[r] + ryL) + (gyR[r] + ryR));
        }
        T u = qcom[1], v = qcom[2];
        T txx = C.mu * (4.0 / 3.0 * gx[1] - 2.0 / 3.0 * gy[2]);
        T tyy = C.mu * (4.0 / 3.0 * gy[2] - 2.0 / 3.0 * gx[1]);
        T txy = C.mu * (gy[1] + gx[2]);
        double ir = 1.0 / C.Re;
        T fv[4] = {T(0.0), ir * txx, ir * txy, ir * (u * txx + v * txy + C.kc * gx[3])};
        T gv[4] = {T(0.0), ir * txy, ir * tyy, ir * (u * txy + v * tyy + C.kc * gy[3])};
        for (int r = 0; r < 4; ++r) fn[r] -= fv[r] * nx + gv[r] * ny;
    }
    // Sec. "Boundary Conditions": the state on the far side of a boundary face, which then
    // enters the same common flux as an interior neighbour's trace (the approximate Riemann
    // solver enforces the condition).  n: unit outward normal, (ug, vg): face velocity.
    //  1 far field: the free stream q^inf, uniform (zero gradient);
    //  2 slip wall: the mirror image of the own side across the wall, with the velocity
    //    taken relative to the moving wall (reading: a symmetry plane, so that viscous
    //    terms see the mirrored gradients too);
    //  3 adiabatic no-slip wall: velocity 2 v_wall - v (the average is the wall velocity),
    //    same p and T, same velocity gradient, temperature gradient mirrored (the average
    //    has no normal component: no heat flux through the wall).
    template <class T> void exterior(int kind, const T* qL, const T* gxL, const T* gyL, double nx, double ny,
                                     double ug, double vg, T* qR, T* gxR, T* gyR) const {
        const Ctx& C = *c;
        if (kind == 1) {
            for (int r = 0; r < 4; ++r) { qR[r] = C.qinf[r]; gxR[r] = 0.0; gyR[r] = 0.0; }
            return;
        }
        // reflection across the wall line: Rm = I - 2 n n^T
        const double Rm[2][2] = {{1.0 - 2.0 * nx * nx, -2.0 * nx * ny}, {-2.0 * ny * nx, 1.0 - 2.0 * ny * ny}};
        const double w[2] = {ug, vg};
        auto mirror_vec = [&](const T* a, T* b) {   // b = Rm a
            for (int r = 0; r < 2; ++r) b[r] = Rm[r][0] * a[0] + Rm[r][1] * a[1];
        };
        qR[0] = qL[0]; qR[3] = qL[3];
        T gp[2] = {gxL[0], gyL[0]}, gT[2] = {gxL[3], gyL[3]}, mp[2], mT[2];
        mirror_vec(gT, mT);
        gxR[3] = mT[0]; gyR[3] = mT[1];
        if (kind == 2) {
            T rel[2] = {qL[1] - w[0], qL[2] - w[1]}, mr[2];
            mirror_vec(rel, mr);
            qR[1] = w[0] + mr[0]; qR[2] = w[1] + mr[1];
            mirror_vec(gp, mp);
            gxR[0] = mp[0]; gyR[0] = mp[1];
            // velocity gradient G[a][b] = d u_a / d x_b of the mirror image: Rm G Rm
            T G[2][2] = {{gxL[1], gyL[1]}, {gxL[2], gyL[2]}}, H[2][2];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    T acc = 0.0;
                    for (int k = 0; k < 2; ++k)
                        for (int l = 0; l < 2; ++l) acc += Rm[a][k] * G[k][l] * Rm[l][b];
                    H[a][b] = acc;
                }
            gxR[1] = H[0][0]; gyR[1] = H[0][1]; gxR[2] = H[1][0]; gyR[2] = H[1][1];
        } else {
            qR[1] = 2.0 * w[0] - qL[1]; qR[2] = 2.0 * w[1] - qL[2];
            gxR[0] = gxL[0]; gyR[0] = gyL[0];
            gxR[1] = gxL[1]; gyR[1] = gyL[1]; gxR[2] = gxL[2]; gyR[2] = gyL[2];
        }
    }
};

// Scalar advection-diffusion physics (1 variable): f = a_x u - nu u_x, g = a_y u - nu u_y,
// upwind common advective flux, same BR2 viscous treatment. Used to pin the FR machinery
// against an independent DG weak form.
struct ScalarPhys {
    static constexpr int NV = 1;
    const Ctx* c; double ax, ay, nu;
    template <class T> void flux(const T* q, const T* gx, const T* gy, T* f, T* g, T* qc) const {
        f[0] = ax * q[0] - nu * gx[0]; g[0] = ay * q[0] - nu * gy[0]; qc[0] = q[0];
    }
    template <class T> void common(const T* qL, const T* qR, const T* gxL, const T* gyL,
                                   const T* gxR, const T* gyR, double nx, double ny, double Smag,
                                   double JfL, double JfR, double ug, double vg, T* fn, T* qcom) const {
        double an = ax * nx + ay * ny - (ug * nx + vg * ny);
        fn[0] = 0.5 * an * (qL[0] + qR[0]) - 0.5 * std::fabs(an) * (qR[0] - qL[0]);
        qcom[0] = 0.5 * (qL[0] + qR[0]);
        if (nu == 0.0) return;
        const double pf = 0.5 * (c->p + 1) * (c->p + 1);
        double cL = pf * Smag / JfL, cR = pf * Smag / JfR;
        T gx = 0.5 * ((gxL[0] + cL * (qcom[0] - qL[0]) * nx) + (gxR[0] - cR * (qcom[0] - qR[0]) * nx));
        T gy = 0.5 * ((gyL[0] + cL * (qcom[0] - qL[0]) * ny) + (gyR[0] - cR * (qcom[0] - qR[0]) * ny));
        fn[0] -= nu * (gx * nx + gy * ny);
    }
    // the scalar path checks the interior machinery only: a boundary face sees its own trace
    template <class T> void exterior(int, const T* qL, const T* gxL, const T* gyL, double, double, double, double,
                                     T* qR, T* gxR, T* gyR) const {
        qR[0] = qL[0]; gxR[0] = gxL[0]; gyR[0] = gyL[0];
    }
};

// ---------------------------------------------------------------- FR residual
// Traces of the solution and of the uncorrected chain-rule gradient at the 4n flux
// points of element e.  tq[f][v][k], tgx/tgy[f][v][k].
template <class Phys, class T>
static void element_traces(const Ctx& c, const Phys&, int e, const T* q, T* tq, T* tgx, T* tgy) {
    const int n = c.n, Np = c.Np, NV = Phys::NV;
    std::vector<T> gx((size_t)NV * Np), gy((size_t)NV * Np);
    for (int v = 0; v < NV; ++v) {
        const T* qv = q + ((size_t)v * c.E + e) * Np;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                T dxi = 0.0, deta = 0.0;
                for (int a = 0; a < n; ++a) dxi += c.op.D[i * n + a] * qv[a + n * j];
                for (int b = 0; b < n; ++b) deta += c.op.D[j * n + b] * qv[i + n * b];
                size_t id = (size_t)e * Np + i + n * j;
                gx[v * Np + i + n * j] = c.xix[id] * dxi + c.etx[id] * deta;
                gy[v * Np + i + n * j] = c.xiy[id] * dxi + c.ety[id] * deta;
            }
    }
    for (int f = 0; f < 4; ++f) {
        const std::vector<double>& lam = (f == 0 || f == 2) ? c.op.lamL : c.op.lamR;
        for (int v = 0; v < NV; ++v)
            for (int k = 0; k < n; ++k) {
                T sq = 0.0, sx = 0.0, sy = 0.0;
                const T* qv = q + ((size_t)v * c.E + e) * Np;
                for (int a = 0; a < n; ++a) {
                    int s = line_pt(n, f, k, a);
                    sq += lam[a] * qv[s]; sx += lam[a] * gx[v * Np + s]; sy += lam[a] * gy[v * Np + s];
                }
                size_t id = ((size_t)f * NV + v) * n + k;
                tq[id] = sq; tgx[id] = sx; tgy[id] = sy;
            }
    }
}

template <class T> struct Traces {
    int NV, n;
    std::vector<T> q, gx, gy;  // [E][4][NV][n]
    void init(int E, int NV_, int n_) { NV = NV_; n = n_; q.assign((size_t)E * 4 * NV * n, T(0.0)); gx = gy = q; }
    T* pq(int e) { return q.data() + (size_t)e * 4 * NV * n; }
    T* pgx(int e) { return gx.data() + (size_t)e * 4 * NV * n; }
    T* pgy(int e) { return gy.data() + (size_t)e * 4 * NV * n; }
};

// Residual of element e (Eq. (cpr_ns) with the F^cor/G^cor corrections and the
// moving-mesh terms), given the traces of every element.
// R = -[ xi_x d_xi f + eta_x d_eta f + xi_y d_xi g + eta_y d_eta g
//        - u_g (xi_x d_xi q^c + eta_x d_eta q^c) - v_g (xi_y d_xi q^c + eta_y d_eta q^c)
//        + (1/|J|)(dF_L g_L' + dF_R g_R' + dG_B g_L'(eta) + dG_T g_R'(eta)) ]
template <class Phys, class T>
static void element_residual(const Ctx& c, const Phys& ph, int e, const T* q, Traces<T>& tr, T* Re) {
    const int n = c.n, Np = c.Np, NV = Phys::NV;
    T* tq = tr.pq(e); T* tgx = tr.pgx(e); T* tgy = tr.pgy(e);
    // --- face stage: common fluxes and common solution
    std::vector<T> Fnum((size_t)4 * NV * n), dqf((size_t)4 * NV * n);
    for (int f = 0; f < 4; ++f) {
        int e2 = c.nbr[e * 4 + f], f2 = c.nbr_face[e * 4 + f], fl = c.flip[e * 4 + f];
        for (int k = 0; k < n; ++k) {
            int k2 = fl ? n - 1 - k : k;
            size_t sid = ((size_t)e * 4 + f) * n + k, sid2 = e2 >= 0 ? ((size_t)e2 * 4 + f2) * n + k2 : sid;
            double Sox = face_sign(f) * c.Sx[sid], Soy = face_sign(f) * c.Sy[sid];
            double Smag = std::sqrt(Sox * Sox + Soy * Soy);
            double nx = Sox / Smag, ny = Soy / Smag;
            T qL[4], qR[4], gxL[4], gyL[4], gxR[4], gyR[4];
            for (int v = 0; v < NV; ++v) {
                qL[v] = tq[((size_t)f * NV + v) * n + k];
                gxL[v] = tgx[((size_t)f * NV + v) * n + k];
                gyL[v] = tgy[((size_t)f * NV + v) * n + k];
            }
            double JfR;
            if (e2 >= 0) {
                for (int v = 0; v < NV; ++v) {
                    qR[v] = tr.pq(e2)[((size_t)f2 * NV + v) * n + k2];
                    gxR[v] = tr.pgx(e2)[((size_t)f2 * NV + v) * n + k2];
                    gyR[v] = tr.pgy(e2)[((size_t)f2 * NV + v) * n + k2];
                }
                JfR = c.Jf[sid2];
            } else {
                // boundary face; reading: the BR2 lifting of the far side uses the own |J|
                ph.exterior(-e2, qL, gxL, gyL, nx, ny, c.ugf[sid], c.vgf[sid], qR, gxR, gyR);
                JfR = c.Jf[sid];
            }
            T fn[4], qcom[4];
            ph.common(qL, qR, gxL, gyL, gxR, gyR, nx, ny, Smag, c.Jf[sid], JfR,
                      c.ugf[sid], c.vgf[sid], fn, qcom);
            // Eq. (norm_f_2): F^num = |J||grad xi| f_n^com sign(n . grad xi); n is this side's
            // outward normal, so the sign is face_sign(f).
            for (int v = 0; v < NV; ++v) {
                Fnum[((size_t)f * NV + v) * n + k] = face_sign(f) * Smag * fn[v];
                dqf[((size_t)f * NV + v) * n + k] = qcom[v] - qL[v];
            }
        }
    }
    // --- corrected gradient at solution points (reading: FR lifting of q^com - q^- on all 4 faces)
    std::vector<T> gx((size_t)NV * Np), gy((size_t)NV * Np);
    for (int v = 0; v < NV; ++v) {
        const T* qv = q + ((size_t)v * c.E + e) * Np;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t id = (size_t)e * Np + i + n * j;
                T dxi = 0.0, deta = 0.0;
                for (int a = 0; a < n; ++a) dxi += c.op.D[i * n + a] * qv[a + n * j];
                for (int b = 0; b < n; ++b) deta += c.op.D[j * n + b] * qv[i + n * b];
                T cx = 0.0, cy = 0.0;
                // faces 0/1 at point j, faces 2/3 at point i
                const int fk[4] = {j, j, i, i};
                const double gm[4] = {c.op.gamL[i], c.op.gamR[i], c.op.gamL[j], c.op.gamR[j]};
                for (int f = 0; f < 4; ++f) {
                    size_t sid = ((size_t)e * 4 + f) * n + fk[f];
                    T d = dqf[((size_t)f * NV + v) * n + fk[f]];
                    cx += d * c.Sx[sid] * gm[f]; cy += d * c.Sy[sid] * gm[f];
                }
                gx[v * Np + i + n * j] = c.xix[id] * dxi + c.etx[id] * deta + cx / c.jac[id];
                gy[v * Np + i + n * j] = c.xiy[id] * dxi + c.ety[id] * deta + cy / c.jac[id];
            }
    }
    // --- pointwise fluxes at solution points
    std::vector<T> F((size_t)NV * Np), G((size_t)NV * Np), QC((size_t)NV * Np);
    for (int s = 0; s < Np; ++s) {
        T qs[4], gxs[4], gys[4], fs[4], gs[4], qcs[4];
        for (int v = 0; v < NV; ++v) {
            qs[v] = q[((size_t)v * c.E + e) * Np + s]; gxs[v] = gx[v * Np + s]; gys[v] = gy[v * Np + s];
        }
        ph.flux(qs, gxs, gys, fs, gs, qcs);
        for (int v = 0; v < NV; ++v) { F[v * Np + s] = fs[v]; G[v * Np + s] = gs[v]; QC[v * Np + s] = qcs[v]; }
    }
    // --- flux differences at flux points: dF = F^num - F^loc, F^loc = S.(Pi f, Pi g) - (S.v_g) Pi q^c
    //     (reading: traces of the same flux polynomials that are differentiated)
    std::vector<T> dF((size_t)4 * NV * n);
    for (int f = 0; f < 4; ++f) {
        const std::vector<double>& lam = (f == 0 || f == 2) ? c.op.lamL : c.op.lamR;
        for (int k = 0; k < n; ++k) {
            size_t sid = ((size_t)e * 4 + f) * n + k;
            double Sxk = c.Sx[sid], Syk = c.Sy[sid];
            double Svg = Sxk * c.ugf[sid] + Syk * c.vgf[sid];
            for (int v = 0; v < NV; ++v) {
                T pf = 0.0, pg = 0.0, pq = 0.0;
                for (int a = 0; a < n; ++a) {
                    int s = line_pt(n, f, k, a);
                    pf += lam[a] * F[v * Np + s]; pg += lam[a] * G[v * Np + s]; pq += lam[a] * QC[v * Np + s];
                }
                T Floc = Sxk * pf + Syk * pg - Svg * pq;
                dF[((size_t)f * NV + v) * n + k] = Fnum[((size_t)f * NV + v) * n + k] - Floc;
            }
        }
    }
    // --- volume terms and correction lift
    for (int v = 0; v < NV; ++v)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t id = (size_t)e * Np + i + n * j;
                T dfx = 0.0, dfe = 0.0, dgx = 0.0, dge = 0.0, dqx = 0.0, dqe = 0.0;
                for (int a = 0; a < n; ++a) {
                    double Dx = c.op.D[i * n + a];
                    dfx += Dx * F[v * Np + a + n * j]; dgx += Dx * G[v * Np + a + n * j]; dqx += Dx * QC[v * Np + a + n * j];
                }
                for (int b = 0; b < n; ++b) {
                    double De = c.op.D[j * n + b];
                    dfe += De * F[v * Np + i + n * b]; dge += De * G[v * Np + i + n * b]; dqe += De * QC[v * Np + i + n * b];
                }
                T vol = c.xix[id] * dfx + c.etx[id] * dfe + c.xiy[id] * dgx + c.ety[id] * dge
                      - c.ugs[id] * (c.xix[id] * dqx + c.etx[id] * dqe)
                      - c.vgs[id] * (c.xiy[id] * dqx + c.ety[id] * dqe);
                T cor = dF[((size_t)0 * NV + v) * n + j] * c.op.gamL[i] + dF[((size_t)1 * NV + v) * n + j] * c.op.gamR[i]
                      + dF[((size_t)2 * NV + v) * n + i] * c.op.gamL[j] + dF[((size_t)3 * NV + v) * n + i] * c.op.gamR[j];
                Re[(size_t)v * Np + i + n * j] = -(vol + cor / c.jac[id]);
            }
}

template <class Phys, class T>
static void compute_traces(const Ctx& c, const Phys& ph, const T* q, Traces<T>& tr) {
    tr.init(c.E, Phys::NV, c.n);
#pragma omp parallel for schedule(static) num_threads(c.threads) if (c.threads > 1)
    for (int e = 0; e < c.E; ++e) element_traces(c, ph, e, q, tr.pq(e), tr.pgx(e), tr.pgy(e));
}

// Full residual R[NV][E][Np].
template <class Phys, class T>
static void residual(const Ctx& c, const Phys& ph, const T* q, T* R) {
    const int NV = Phys::NV, Np = c.Np;
    Traces<T> tr; compute_traces(c, ph, q, tr);
    // elements are independent once the traces exist: an OpenMP build may split them over
    // threads (each with its own element buffer); the arithmetic per element is unchanged
#pragma omp parallel num_threads(c.threads) if (c.threads > 1)
    {
        std::vector<T> Re((size_t)NV * Np);
#pragma omp for schedule(static)
        for (int e = 0; e < c.E; ++e) {
            element_residual(c, ph, e, q, tr, Re.data());
            for (int v = 0; v < NV; ++v)
                for (int s = 0; s < Np; ++s) R[((size_t)v * c.E + e) * Np + s] = Re[(size_t)v * Np + s];
        }
    }
}

static const double CS_H = 1e-30;

// JVP by complex step: J v = Im R(q + i h v)/h.
static void jvp_cs(const Ctx& c, const double* q, const double* v, double* Jv) {
    NSPhys ph{&c};
    size_t N = (size_t)4 * c.E * c.Np;
    std::vector<cplx> qz(N), Rz(N);
    for (size_t i = 0; i < N; ++i) qz[i] = cplx(q[i], CS_H * v[i]);
    residual(c, ph, qz.data(), Rz.data());
    for (size_t i = 0; i < N; ++i) Jv[i] = Rz[i].imag() / CS_H;
}

// Diagonal block d R_e / d q_e (4Np x 4Np, row/col index v*Np + s) by complex step with
// seeds on element e only; neighbours keep their real traces (unless e neighbours itself).
static void element_block_cs(const Ctx& c, const double* q, Traces<cplx>& trz, int e, double* B) {
    NSPhys ph{&c};
    const int Np = c.Np, nb = 4 * Np;
    std::vector<cplx> qe((size_t)4 * c.E * Np);  // only element e's entries are touched
    // copy element e's state (complex) into a full-size buffer view
    std::vector<cplx> qz((size_t)4 * c.E * Np);
    for (int v = 0; v < 4; ++v)
        for (int s = 0; s < Np; ++s) qz[((size_t)v * c.E + e) * Np + s] = q[((size_t)v * c.E + e) * Np + s];
    size_t tsz = (size_t)4 * 4 * c.n;
    std::vector<cplx> save_q(trz.pq(e), trz.pq(e) + tsz), save_x(trz.pgx(e), trz.pgx(e) + tsz),
                      save_y(trz.pgy(e), trz.pgy(e) + tsz);
    std::vector<cplx> Re((size_t)nb);
    for (int col = 0; col < nb; ++col) {
        int cv = col / Np, cs = col % Np;
        size_t gid = ((size_t)cv * c.E + e) * Np + cs;
        qz[gid] += cplx(0.0, CS_H);
        element_traces(c, ph, e, qz.data(), trz.pq(e), trz.pgx(e), trz.pgy(e));
        element_residual(c, ph, e, qz.data(), trz, Re.data());
        for (int r = 0; r < nb; ++r) B[(size_t)r * nb + col] = Re[r].imag() / CS_H;
        qz[gid] -= cplx(0.0, CS_H);
        qz[gid] = cplx(qz[gid].real(), 0.0);
    }
    std::copy(save_q.begin(), save_q.end(), trz.pq(e));
    std::copy(save_x.begin(), save_x.end(), trz.pgx(e));
    std::copy(save_y.begin(), save_y.end(), trz.pgy(e));
}

// ---------------------------------------------------------------- dense LU (partial pivoting)
static int lu_factor(int n, double* A, int* piv) {
    for (int k = 0; k < n; ++k) {
        int pr = k; double best = std::fabs(A[(size_t)k * n + k]);
        for (int r = k + 1; r < n; ++r) if (std::fabs(A[(size_t)r * n + k]) > best) { best = std::fabs(A[(size_t)r * n + k]); pr = r; }
        piv[k] = pr;
        if (best == 0.0) return -1;
        if (pr != k) for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)pr * n + j]);
        for (int r = k + 1; r < n; ++r) {
            double l = A[(size_t)r * n + k] / A[(size_t)k * n + k];
            A[(size_t)r * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[(size_t)r * n + j] -= l * A[(size_t)k * n + j];
        }
    }
    return 0;
}
static void lu_solve(int n, const double* LU, const int* piv, double* b) {
    for (int k = 0; k < n; ++k) if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int r = 0; r < n; ++r) for (int j = 0; j < r; ++j) b[r] -= LU[(size_t)r * n + j] * b[j];
    for (int r = n - 1; r >= 0; --r) {
        for (int j = r + 1; j < n; ++j) b[r] -= LU[(size_t)r * n + j] * b[j];
        b[r] /= LU[(size_t)r * n + r];
    }
}

// ---------------------------------------------------------------- GMRES(m), right preconditioned, MGS
struct GmresOut { int its; double rel; };
static GmresOut gmres(size_t N, const std::function<void(const double*, double*)>& A,
                      const std::function<void(const double*, double*)>& Pinv,
                      const double* b, double* x, int m, double tol, int max_it) {
    auto dot = [N](const double* a, const double* c) { double s = 0; for (size_t i = 0; i < N; ++i) s += a[i] * c[i]; return s; };
    std::fill(x, x + N, 0.0);
    double bn = std::sqrt(dot(b, b));
    GmresOut out{0, 0.0};
    if (bn == 0.0) return out;
    std::vector<double> r(b, b + N), z(N), w(N);
    std::vector<std::vector<double>> V(m + 1, std::vector<double>(N));
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
    double beta = bn;
    while (out.its < max_it) {
        for (size_t i = 0; i < N; ++i) V[0][i] = r[i] / beta;
        std::fill(g.begin(), g.end(), 0.0); g[0] = beta;
        int j = 0;
        for (; j < m && out.its < max_it; ++j) {
            Pinv(V[j].data(), z.data()); A(z.data(), w.data());
            for (int i = 0; i <= j; ++i) {
                double h = dot(w.data(), V[i].data()); H[(size_t)i * m + j] = h;
                for (size_t t = 0; t < N; ++t) w[t] -= h * V[i][t];
            }
            double hn = std::sqrt(dot(w.data(), w.data())); H[(size_t)(j + 1) * m + j] = hn;
            if (hn != 0.0) for (size_t t = 0; t < N; ++t) V[j + 1][t] = w[t] / hn;
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            double den = std::sqrt(a * a + bb * bb);
            cs[j] = den == 0.0 ? 1.0 : a / den; sn[j] = den == 0.0 ? 0.0 : bb / den;
            H[(size_t)j * m + j] = cs[j] * a + sn[j] * bb; H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j]; g[j] = cs[j] * g[j];
            out.its++;
            if (std::fabs(g[j + 1]) <= tol * bn || hn == 0.0) { ++j; break; }
        }
        // back substitution H y = g, x += Pinv(V y)
        std::vector<double> y(j);
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= H[(size_t)i * m + k] * y[k];
            y[i] = s / H[(size_t)i * m + i];
        }
        std::fill(w.begin(), w.end(), 0.0);
        for (int i = 0; i < j; ++i) for (size_t t = 0; t < N; ++t) w[t] += y[i] * V[i][t];
        Pinv(w.data(), z.data());
        for (size_t t = 0; t < N; ++t) x[t] += z[t];
        A(x, w.data());
        for (size_t t = 0; t < N; ++t) r[t] = b[t] - w[t];
        beta = std::sqrt(dot(r.data(), r.data()));
        out.rel = beta / bn;
        if (beta <= tol * bn) break;
    }
    return out;
}

// ---------------------------------------------------------------- preconditioners
// Element colouring for the Gauss-Seidel sweeps: elements in index order take the smallest
// colour that no face neighbour already has.
static std::vector<int> colour_elements(const Ctx& c, int& ncol) {
    std::vector<int> col(c.E, -1);
    ncol = 0;
    for (int e = 0; e < c.E; ++e) {
        bool used[5] = {false, false, false, false, false};
        for (int f = 0; f < 4; ++f) {
            const int nb = c.nbr[e * 4 + f];
            if (nb >= 0 && nb != e && col[nb] >= 0) used[col[nb]] = true;
        }
        int k = 0;
        while (used[k]) ++k;
        col[e] = k;
        ncol = std::max(ncol, k + 1);
    }
    return col;
}

// z = P^-1 r.  precond 0: element-block Jacobi, z_e = D_e^-1 r_e with D_e the diagonal
// block of the Newton operator A (factored in blk/piv).  precond 1: symmetric block
// Gauss-Seidel over the elements in colour order (reading: the element-block form of the
// relaxation-type preconditioning the paper's solver setup names, ILU(0)),
// P = (D + L) D^-1 (D + U), L / U the couplings of A to elements of lower / higher colour:
//   forward  y_k = D_k^-1 (r_k - sum_{k' < k} A_{k k'} y_{k'})   for k = 0 .. K-1,
//   backward z_k = y_k - D_k^-1 sum_{k' > k} A_{k k'} z_{k'}      for k = K-2 .. 0,
// with the off-diagonal products taken as A applied to y (z) restricted to those colours.
// precond 2: forward block Gauss-Seidel, P = D + L: the forward sweep alone (z = y).
static void precond_apply(const Ctx& c, int precond, const std::vector<int>& col, int ncol,
                          const std::vector<double>& blk, const std::vector<int>& piv,
                          const std::function<void(const double*, double*)>& A, const double* r, double* z) {
    const int Np = c.Np, E = c.E, nb = 4 * Np;
    const size_t N = (size_t)4 * E * Np;
    std::vector<double> tmp(nb);
    // z_e = D_e^-1 (a_e - b_e) (b may be null), or z_e -= D_e^-1 a_e when sub
    auto dsolve = [&](int e, const double* a, const double* b, bool sub) {
        for (int v = 0; v < 4; ++v)
            for (int s = 0; s < Np; ++s) {
                const size_t id = ((size_t)v * E + e) * Np + s;
                tmp[v * Np + s] = a[id] - (b ? b[id] : 0.0);
            }
        lu_solve(nb, blk.data() + (size_t)e * nb * nb, piv.data() + (size_t)e * nb, tmp.data());
        for (int v = 0; v < 4; ++v)
            for (int s = 0; s < Np; ++s) {
                const size_t id = ((size_t)v * E + e) * Np + s;
                z[id] = sub ? z[id] - tmp[v * Np + s] : tmp[v * Np + s];
            }
    };
    if (precond == 0) {
        for (int e = 0; e < E; ++e) dsolve(e, r, nullptr, false);
        return;
    }
    std::fill(z, z + N, 0.0);
    std::vector<double> u(N), t(N);
    auto restrict_to = [&](int lo, int hi) {   // u = z on colours lo..hi, 0 elsewhere
        for (int v = 0; v < 4; ++v)
            for (int e = 0; e < E; ++e)
                for (int s = 0; s < Np; ++s) {
                    const size_t id = ((size_t)v * E + e) * Np + s;
                    u[id] = (col[e] >= lo && col[e] <= hi) ? z[id] : 0.0;
                }
    };
    for (int k = 0; k < ncol; ++k) {
        if (k > 0) { restrict_to(0, k - 1); A(u.data(), t.data()); }
        for (int e = 0; e < E; ++e)
            if (col[e] == k) dsolve(e, r, k > 0 ? t.data() : nullptr, false);
    }
    if (precond != 1) return;
    for (int k = ncol - 2; k >= 0; --k) {
        restrict_to(k + 1, ncol - 1);
        A(u.data(), t.data());
        for (int e = 0; e < E; ++e)
            if (col[e] == k) dsolve(e, t.data(), nullptr, true);
    }
}

// ---------------------------------------------------------------- BDF2 dual-time Newton step
struct StepOpts { double dt, inv_dtau, tol_pseudo, tol_res, tol_abs; int krylov, max_lin_it, max_newton, jac_lag, precond; };
struct StepStats { int newton_its, gmres_its, converged; double res0, res_final; };

// Sec. 3.2 Eq. (unsteady_pre_discretized_3):
// (Gamma/dtau + 3/(2dt) M - dR/dq) dq = -(3 q^c,m - 4 q^c,n + q^c,n-1)/(2dt) + R^m,
// initial iterate q^n; BDF1 (coefficients 1, -1) when q^{n-1} is absent (reading).
static int bdf2_step(const Ctx& c, double* q, const double* q_nm1, const StepOpts& o, StepStats& st) {
    const int Np = c.Np, E = c.E, nb = 4 * Np;
    const size_t N = (size_t)4 * E * Np;
    double a0 = q_nm1 ? 1.5 : 1.0, a1 = q_nm1 ? -2.0 : -1.0, a2 = q_nm1 ? 0.5 : 0.0;
    double ct = a0 / o.dt;
    NSPhys ph{&c};
    auto qc_field = [&](const double* qq, std::vector<double>& out) {
        out.assign(N, 0.0);
        for (int e = 0; e < E; ++e)
            for (int s = 0; s < Np; ++s) {
                double qs[4], qcs[4];
                for (int v = 0; v < 4; ++v) qs[v] = qq[((size_t)v * E + e) * Np + s];
                cons(c, qs, qcs);
                for (int v = 0; v < 4; ++v) out[((size_t)v * E + e) * Np + s] = qcs[v];
            }
    };
    std::vector<double> Qn, Qnm1, Qm, R(N), b(N), dq(N);
    qc_field(q, Qn);
    if (q_nm1) qc_field(q_nm1, Qnm1); else Qnm1.assign(N, 0.0);
    std::vector<double> blk((size_t)E * nb * nb); std::vector<int> piv((size_t)E * nb);
    int ncol = 0;
    const std::vector<int> col = colour_elements(c, ncol);
    st = StepStats{0, 0, 0, 0.0, 0.0};
    // time-term matrices at the current iterate: Gamma/dtau + ct M per solution point
    auto time_mat = [&](const double* qq, int e, int s, double T4[4][4]) {
        double qs[4]; for (int v = 0; v < 4; ++v) qs[v] = qq[((size_t)v * E + e) * Np + s];
        double M[4][4], G[4][4]; mat_M(c, qs, M);
        size_t id = (size_t)e * Np + s;
        mat_Gamma(c, qs, c.ugs[id], c.vgs[id], G);
        for (int r = 0; r < 4; ++r) for (int k = 0; k < 4; ++k) T4[r][k] = o.inv_dtau * G[r][k] + ct * M[r][k];
    };
    for (int m = 0; ; ++m) {
        residual(c, ph, q, R.data());
        qc_field(q, Qm);
        for (size_t i = 0; i < N; ++i) b[i] = -(a0 * Qm[i] + a1 * Qn[i] + a2 * Qnm1[i]) / o.dt + R[i];
        double res = 0.0;
        for (size_t i = 0; i < (size_t)E * Np; ++i) res += b[i] * b[i];   // continuity rows
        res = std::sqrt(res);
        if (!std::isfinite(res)) return -4;
        if (m == 0) st.res0 = res;
        st.res_final = res;
        if (res <= o.tol_abs || res <= o.tol_pseudo * st.res0) { st.converged = 1; break; }
        if (m >= o.max_newton) break;
        if (m % o.jac_lag == 0) {
            Traces<cplx> trz;
            std::vector<cplx> qz(q, q + N);
            compute_traces(c, ph, qz.data(), trz);
            for (int e = 0; e < E; ++e) {
                double* B = blk.data() + (size_t)e * nb * nb;
                element_block_cs(c, q, trz, e, B);
                for (int r = 0; r < nb * nb; ++r) B[r] = -B[r];
                for (int s = 0; s < Np; ++s) {
                    double T4[4][4]; time_mat(q, e, s, T4);
                    for (int r = 0; r < 4; ++r) for (int k = 0; k < 4; ++k) B[(size_t)(r * Np + s) * nb + k * Np + s] += T4[r][k];
                }
                if (lu_factor(nb, B, piv.data() + (size_t)e * nb) != 0) return -5;
            }
        }
        std::vector<double> qcur(q, q + N);
        auto Aop = [&](const double* v, double* out) {
            jvp_cs(c, qcur.data(), v, out);
            for (int e = 0; e < E; ++e)
                for (int s = 0; s < Np; ++s) {
                    double T4[4][4]; time_mat(qcur.data(), e, s, T4);
                    for (int r = 0; r < 4; ++r) {
                        double t = 0.0;
                        for (int k = 0; k < 4; ++k) t += T4[r][k] * v[((size_t)k * E + e) * Np + s];
                        size_t id = ((size_t)r * E + e) * Np + s;
                        out[id] = t - out[id];
                    }
                }
        };
        auto Pop = [&](const double* v, double* out) { precond_apply(c, o.precond, col, ncol, blk, piv, Aop, v, out); };
        GmresOut go = gmres(N, Aop, Pop, b.data(), dq.data(), o.krylov, o.tol_res, o.max_lin_it);
        st.gmres_its += go.its;
        for (size_t i = 0; i < N; ++i) q[i] += dq[i];
        st.newton_its++;
    }
    return st.converged ? 0 : -5;
}

// ---------------------------------------------------------------- steady pseudo-transient continuation
struct SteadyOpts { double dtau0, dtau_min, dtau_max, r_ser, tol_pseudo, tol_res, tol_abs, reject_growth; int krylov, max_lin_it, max_steps, jac_lag, precond; };

// Sec. 3.2 Eq. (steady_pre_discretized_1): (Gamma^m/dtau - dR/dq^m) dq^m = R^m, backward Euler
// in pseudo time linearised about q^m, with dtau from Eq. (SER): the step size used at pseudo-step
// m is that of step m-1 times (Res_{m-1}/Res_m)^r_ser, clipped to [dtau_min, dtau_max], and dtau0
// at m = 0 (reading: the freshest residual ratio sets the next step); Res is the 2-norm of the
// continuity (pressure) rows of R.  hist (may be null) receives (Res_m, dtau_m) per step taken.
//
// Step rejection (not in the paper, which leaves globalisation of SER to other work; off when
// reject_growth = 0): when the residual after a step is not finite or exceeds reject_growth times
// the one before it, the step is undone (q -= dq) and retried from the same state with a ten
// times smaller dtau (the SER update and its clipping are skipped for that retry, since the
// residual ratio is 1).  A rejected step is recorded in hist as (Res, -dtau of the retry) and
// counts towards max_steps.
static int steady_solve(const Ctx& c, double* q, const SteadyOpts& o, StepStats& st, double* dtau_final,
                        std::vector<double>* hist, int* rejected = nullptr) {
    const int Np = c.Np, E = c.E, nb = 4 * Np;
    const size_t N = (size_t)4 * E * Np;
    NSPhys ph{&c};
    std::vector<double> R(N), dq(N);
    std::vector<double> blk((size_t)E * nb * nb); std::vector<int> piv((size_t)E * nb);
    int ncol = 0;
    const std::vector<int> col = colour_elements(c, ncol);
    st = StepStats{0, 0, 0, 0.0, 0.0};
    double dtau = o.dtau0, res_prev = 0.0;
    bool retry = false;
    int nrej = 0;
    auto gamma_pt = [&](const double* qq, int e, int s, double G[4][4]) {
        double qs[4]; for (int v = 0; v < 4; ++v) qs[v] = qq[((size_t)v * E + e) * Np + s];
        const size_t id = (size_t)e * Np + s;
        mat_Gamma(c, qs, c.ugs[id], c.vgs[id], G);
    };
    for (int m = 0; ; ++m) {
        residual(c, ph, q, R.data());
        double res = 0.0;
        for (size_t i = 0; i < (size_t)E * Np; ++i) res += R[i] * R[i];
        res = std::sqrt(res);
        if (o.reject_growth > 0.0 && m > 0 && !retry && !(res <= o.reject_growth * res_prev)) {
            for (size_t i = 0; i < N; ++i) q[i] -= dq[i];
            dtau *= 0.1;
            retry = true;
            ++nrej;
            if (hist) { hist->push_back(res); hist->push_back(-dtau); }
            if (m >= o.max_steps) break;
            continue;
        }
        if (!std::isfinite(res)) return -4;
        if (m == 0) st.res0 = res;
        st.res_final = res;
        if (res <= o.tol_abs || res <= o.tol_pseudo * st.res0) { st.converged = 1; break; }
        if (m >= o.max_steps) break;
        if (m > 0 && !retry) dtau = std::max(o.dtau_min, std::min(o.dtau_max, dtau * std::pow(res_prev / res, o.r_ser)));
        retry = false;
        res_prev = res;
        if (hist) { hist->push_back(res); hist->push_back(dtau); }
        const double idt = 1.0 / dtau;
        if (m % o.jac_lag == 0) {
            Traces<cplx> trz;
            std::vector<cplx> qz(q, q + N);
            compute_traces(c, ph, qz.data(), trz);
            for (int e = 0; e < E; ++e) {
                double* B = blk.data() + (size_t)e * nb * nb;
                element_block_cs(c, q, trz, e, B);
                for (int r = 0; r < nb * nb; ++r) B[r] = -B[r];
                for (int s = 0; s < Np; ++s) {
                    double G[4][4]; gamma_pt(q, e, s, G);
                    for (int r = 0; r < 4; ++r) for (int k = 0; k < 4; ++k) B[(size_t)(r * Np + s) * nb + k * Np + s] += idt * G[r][k];
                }
                if (lu_factor(nb, B, piv.data() + (size_t)e * nb) != 0) return -5;
            }
        }
        std::vector<double> qcur(q, q + N);
        auto Aop = [&](const double* v, double* out) {
            jvp_cs(c, qcur.data(), v, out);
            for (int e = 0; e < E; ++e)
                for (int s = 0; s < Np; ++s) {
                    double G[4][4]; gamma_pt(qcur.data(), e, s, G);
                    for (int r = 0; r < 4; ++r) {
                        double t = 0.0;
                        for (int k = 0; k < 4; ++k) t += idt * G[r][k] * v[((size_t)k * E + e) * Np + s];
                        const size_t id = ((size_t)r * E + e) * Np + s;
                        out[id] = t - out[id];
                    }
                }
        };
        auto Pop = [&](const double* v, double* out) { precond_apply(c, o.precond, col, ncol, blk, piv, Aop, v, out); };
        GmresOut go = gmres(N, Aop, Pop, R.data(), dq.data(), o.krylov, o.tol_res, o.max_lin_it);
        st.gmres_its += go.its;
        for (size_t i = 0; i < N; ++i) q[i] += dq[i];
        st.newton_its++;
    }
    if (dtau_final) *dtau_final = dtau;
    if (rejected) *rejected = nrej;
    return st.converged ? 0 : -5;
}

}  // namespace ora

// =====================================================================================
// C API (ctypes).  All arrays are host arrays; layouts as in the GPU library:
// state [4][E][Np], geometry nodes [2][E][(pg+1)^2], face tables [E][4].
// =====================================================================================
using namespace ora;

extern "C" {

int ora_operators(int p, int pg, double* xi, double* w, double* D, double* lamL, double* lamR,
                  double* gamL, double* gamR, double* gll) {
    Ops o; o.build(p, pg);
    int n = p + 1;
    std::memcpy(xi, o.xi.data(), n * sizeof(double)); std::memcpy(w, o.w.data(), n * sizeof(double));
    std::memcpy(D, o.D.data(), n * n * sizeof(double));
    std::memcpy(lamL, o.lamL.data(), n * sizeof(double)); std::memcpy(lamR, o.lamR.data(), n * sizeof(double));
    std::memcpy(gamL, o.gamL.data(), n * sizeof(double)); std::memcpy(gamR, o.gamR.data(), n * sizeof(double));
    std::memcpy(gll, o.gll.data(), (pg + 1) * sizeof(double));
    return 0;
}

// dprm: gamma, mach_ref, reynolds, prandtl, mu, kappa, mach_inf
// iprm: order, geom_order, n_elem, viscous, moving
void* ora_create(const double* dprm, const int* iprm, const int* nbr, const int* nbr_face,
                 const signed char* flip, const double* xg, const double* vg) {
    Ctx* c = new Ctx();
    c->gam = dprm[0]; c->Ma = dprm[1]; c->Re = dprm[2]; c->Pr = dprm[3]; c->mu = dprm[4];
    c->kappa = dprm[5]; c->Ma_inf = dprm[6];
    c->p = iprm[0]; c->pg = iprm[1]; c->E = iprm[2]; c->viscous = iprm[3]; c->moving = iprm[4];
    c->n = c->p + 1; c->Np = c->n * c->n; c->ng = (c->pg + 1) * (c->pg + 1);
    // Sec. 2.1: R = 1/(gamma Ma^2), Cp = 1/((gamma-1) Ma^2), k = mu Cp / Pr
    c->Rg = 1.0 / (c->gam * c->Ma * c->Ma);
    c->Cp = 1.0 / ((c->gam - 1.0) * c->Ma * c->Ma);
    c->kc = c->mu * c->Cp / c->Pr;
    c->op.build(c->p, c->pg);
    c->nbr.assign(nbr, nbr + 4 * c->E); c->nbr_face.assign(nbr_face, nbr_face + 4 * c->E);
    c->flip.assign(4 * c->E, 0);
    if (flip) c->flip.assign(flip, flip + 4 * c->E);
    c->xg.assign(xg, xg + (size_t)2 * c->E * c->ng);
    if (c->moving && vg) c->vg.assign(vg, vg + (size_t)2 * c->E * c->ng);
    else { c->vg.assign((size_t)2 * c->E * c->ng, 0.0); }
    build_geometry(*c);
    return c;
}

void ora_destroy(void* h) { delete (Ctx*)h; }

// far-field primitive state (p, u, v, T) of the boundary faces of kind 1
void ora_set_farfield(void* h, const double* qinf) {
    Ctx& c = *(Ctx*)h;
    for (int r = 0; r < 4; ++r) c.qinf[r] = qinf[r];
}

// geometry at solution points: out[9][E][Np] = x, y, |J|, xi_x, xi_y, eta_x, eta_y, u_g, v_g
// faces: fout[5][E][4][n] = Sx, Sy, Jf, u_g, v_g
int ora_geometry(void* h, double* out, double* fout) {
    Ctx& c = *(Ctx*)h; size_t M = (size_t)c.E * c.Np, F = (size_t)c.E * 4 * c.n;
    const std::vector<double>* a[9] = {&c.xs, &c.ys, &c.jac, &c.xix, &c.xiy, &c.etx, &c.ety, &c.ugs, &c.vgs};
    for (int i = 0; i < 9; ++i) std::memcpy(out + i * M, a[i]->data(), M * sizeof(double));
    const std::vector<double>* b[5] = {&c.Sx, &c.Sy, &c.Jf, &c.ugf, &c.vgf};
    for (int i = 0; i < 5; ++i) std::memcpy(fout + i * F, b[i]->data(), F * sizeof(double));
    return 0;
}

void ora_set_threads(void* h, int n) { ((Ctx*)h)->threads = n < 1 ? 1 : n; }

int ora_openmp(void) {
#ifdef _OPENMP
    return 1;
#else
    return 0;
#endif
}

// R(q) on the op-counting scalar: R (equal to ora_residual's bit for bit) and the counts
// {add/sub, mul, div, sqrt} of one evaluation.  Serial.
int ora_count_residual(void* h, const double* q, double* R, unsigned long long* counts) {
    Ctx& c = *(Ctx*)h;
    const int keep = c.threads;
    c.threads = 1;
    NSPhys ph{&c};
    const size_t N = (size_t)4 * c.E * c.Np;
    std::vector<Cnt> qc(q, q + N), Rc(N);
    g_tally = OpTally();
    residual(c, ph, qc.data(), Rc.data());
    for (size_t i = 0; i < N; ++i) R[i] = Rc[i].v;
    counts[0] = g_tally.add; counts[1] = g_tally.mul; counts[2] = g_tally.div; counts[3] = g_tally.sqrt;
    c.threads = keep;
    return 0;
}

int ora_residual(void* h, const double* q, double* R) {
    Ctx& c = *(Ctx*)h; NSPhys ph{&c}; residual(c, ph, q, R); return 0;
}

// complex residual (real/imag parts separately), for derivative pins
int ora_residual_cplx(void* h, const double* qr, const double* qi, double* Rr, double* Ri) {
    Ctx& c = *(Ctx*)h; NSPhys ph{&c};
    size_t N = (size_t)4 * c.E * c.Np;
    std::vector<cplx> qz(N), Rz(N);
    for (size_t i = 0; i < N; ++i) qz[i] = cplx(qr[i], qi[i]);
    residual(c, ph, qz.data(), Rz.data());
    for (size_t i = 0; i < N; ++i) { Rr[i] = Rz[i].real(); Ri[i] = Rz[i].imag(); }
    return 0;
}

int ora_scalar_residual(void* h, double ax, double ay, double nu, const double* u, double* R) {
    Ctx& c = *(Ctx*)h; ScalarPhys ph{&c, ax, ay, nu}; residual(c, ph, u, R); return 0;
}

int ora_jvp(void* h, const double* q, const double* v, double* Jv) {
    jvp_cs(*(Ctx*)h, q, v, Jv); return 0;
}

// dense Jacobian J[N][N] (row-major), N = 4 E Np, by complex step column by column
int ora_dense_jacobian(void* h, const double* q, double* J) {
    Ctx& c = *(Ctx*)h; NSPhys ph{&c};
    size_t N = (size_t)4 * c.E * c.Np;
    std::vector<cplx> qz(q, q + N), Rz(N);
    for (size_t k = 0; k < N; ++k) {
        qz[k] = cplx(q[k], CS_H);
        residual(c, ph, qz.data(), Rz.data());
        for (size_t r = 0; r < N; ++r) J[r * N + k] = Rz[r].imag() / CS_H;
        qz[k] = cplx(q[k], 0.0);
    }
    return 0;
}

// (J^T w)_k for a list of global DOF indices k: Im <w, R(q + i h e_k)>/h, re-evaluating only
// the element of k and its face neighbours.
int ora_vjp_dofs(void* h, const double* q, const double* w, const long long* dofs, long long nd, double* out) {
    Ctx& c = *(Ctx*)h; NSPhys ph{&c};
    const int Np = c.Np; const size_t N = (size_t)4 * c.E * Np;
    std::vector<cplx> qz(q, q + N);
    Traces<cplx> trz; compute_traces(c, ph, qz.data(), trz);
    size_t tsz = (size_t)4 * 4 * c.n;
    std::vector<cplx> Re((size_t)4 * Np);
    for (long long t = 0; t < nd; ++t) {
        long long k = dofs[t];
        int v = (int)(k / ((long long)c.E * Np)); long long rem = k % ((long long)c.E * Np);
        int e = (int)(rem / Np);
        std::vector<cplx> sq(trz.pq(e), trz.pq(e) + tsz), sx(trz.pgx(e), trz.pgx(e) + tsz), sy(trz.pgy(e), trz.pgy(e) + tsz);
        qz[k] += cplx(0.0, CS_H);
        element_traces(c, ph, e, qz.data(), trz.pq(e), trz.pgx(e), trz.pgy(e));
        std::vector<int> els{e};
        for (int f = 0; f < 4; ++f) {
            int e2 = c.nbr[e * 4 + f];
            if (e2 >= 0 && std::find(els.begin(), els.end(), e2) == els.end()) els.push_back(e2);
        }
        double acc = 0.0;
        for (int e2 : els) {
            element_residual(c, ph, e2, qz.data(), trz, Re.data());
            for (int r = 0; r < 4; ++r)
                for (int s = 0; s < Np; ++s) acc += w[((size_t)r * c.E + e2) * Np + s] * Re[(size_t)r * Np + s].imag();
        }
        out[t] = acc / CS_H;
        qz[k] = cplx(q[k], 0.0);
        std::copy(sq.begin(), sq.end(), trz.pq(e)); std::copy(sx.begin(), sx.end(), trz.pgx(e));
        std::copy(sy.begin(), sy.end(), trz.pgy(e));
        (void)v;
    }
    return 0;
}

// Element blocks P_e = inv_dtau Gamma_e + c_time M_e - dR_e/dq_e, [E][4Np][4Np], for the
// listed elements (els == NULL: all elements, in order).
int ora_blocks(void* h, const double* q, double c_time, double inv_dtau, const int* els, int nel, double* blk) {
    Ctx& c = *(Ctx*)h; NSPhys ph{&c};
    const int Np = c.Np, nb = 4 * Np, E = c.E;
    std::vector<cplx> qz(q, q + (size_t)4 * E * Np);
    Traces<cplx> trz; compute_traces(c, ph, qz.data(), trz);
    int cnt = els ? nel : E;
    for (int t = 0; t < cnt; ++t) {
        int e = els ? els[t] : t;
        double* B = blk + (size_t)t * nb * nb;
        element_block_cs(c, q, trz, e, B);
        for (int r = 0; r < nb * nb; ++r) B[r] = -B[r];
        for (int s = 0; s < Np; ++s) {
            double qs[4]; for (int v = 0; v < 4; ++v) qs[v] = q[((size_t)v * E + e) * Np + s];
            double M[4][4], G[4][4]; mat_M(c, qs, M);
            size_t id = (size_t)e * Np + s;
            mat_Gamma(c, qs, c.ugs[id], c.vgs[id], G);
            for (int r = 0; r < 4; ++r) for (int k = 0; k < 4; ++k)
                B[(size_t)(r * Np + s) * nb + k * Np + s] += inv_dtau * G[r][k] + c_time * M[r][k];
        }
    }
    return 0;
}

// pointwise physics at one state (for pins): qc[4], M[16], Gamma[16], fn[4] (inviscid normal
// flux), lam (|lambda|max); aux = (nx, ny, ug, vg)
int ora_point(void* h, const double* q, const double* aux, double* qc, double* M, double* G, double* fn, double* lam) {
    Ctx& c = *(Ctx*)h;
    cons(c, q, qc);
    double Mm[4][4], Gm[4][4]; mat_M(c, q, Mm); mat_Gamma(c, q, aux[2], aux[3], Gm);
    for (int r = 0; r < 4; ++r) for (int k = 0; k < 4; ++k) { M[r * 4 + k] = Mm[r][k]; G[r * 4 + k] = Gm[r][k]; }
    normal_inviscid(c, q, aux[0], aux[1], aux[2], aux[3], fn);
    *lam = max_eig(c, q, aux[0], aux[1], aux[2], aux[3]);
    return 0;
}

// complex-state pointwise q^c (for the M pin by complex step)
int ora_cons_cplx(void* h, const double* qr, const double* qi, double* outr, double* outi) {
    Ctx& c = *(Ctx*)h; cplx q[4], o[4];
    for (int i = 0; i < 4; ++i) q[i] = cplx(qr[i], qi[i]);
    cons(c, q, o);
    for (int i = 0; i < 4; ++i) { outr[i] = o[i].real(); outi[i] = o[i].imag(); }
    return 0;
}

// common normal flux at one face point (for consistency / symmetry pins)
// aux = (nx, ny, Smag, JfL, JfR, ug, vg); g* = gradients [4] each
int ora_common_flux(void* h, const double* qL, const double* qR, const double* gxL, const double* gyL,
                    const double* gxR, const double* gyR, const double* aux, double* fn, double* qcom) {
    Ctx& c = *(Ctx*)h; NSPhys ph{&c};
    ph.common(qL, qR, gxL, gyL, gxR, gyR, aux[0], aux[1], aux[2], aux[3], aux[4], aux[5], aux[6], fn, qcom);
    return 0;
}

// physical flux at one point (for pins)
int ora_phys_flux(void* h, const double* q, const double* gx, const double* gy, double* f, double* g) {
    Ctx& c = *(Ctx*)h; phys_flux(c, q, gx, gy, f, g); return 0;
}

int ora_lu_factor(int n, double* A, int* piv) { return lu_factor(n, A, piv); }
int ora_lu_solve(int n, const double* LU, const int* piv, double* b) { lu_solve(n, LU, piv, b); return 0; }

// GMRES on a dense matrix with an optional dense preconditioner inverse (row-major); for pins
int ora_gmres_dense(int n, const double* A, const double* Pinv, const double* b, double* x,
                    int m, double tol, int max_it, int* its, double* rel) {
    auto Aop = [&](const double* v, double* o) {
        for (int r = 0; r < n; ++r) { double s = 0; for (int k = 0; k < n; ++k) s += A[(size_t)r * n + k] * v[k]; o[r] = s; } };
    auto Pop = [&](const double* v, double* o) {
        if (!Pinv) { std::copy(v, v + n, o); return; }
        for (int r = 0; r < n; ++r) { double s = 0; for (int k = 0; k < n; ++k) s += Pinv[(size_t)r * n + k] * v[k]; o[r] = s; } };
    GmresOut g = gmres((size_t)n, Aop, Pop, b, x, m, tol, max_it);
    *its = g.its; *rel = g.rel;
    return 0;
}

// One BDF2 (or BDF1 when q_nm1 == NULL) dual-time Newton step; q updated in place.
// dopt: dt, inv_dtau, tol_pseudo, tol_res, tol_abs; iopt: krylov, max_lin_it, max_newton, jac_lag, precond
// istat: newton_its, gmres_its, converged; dstat: res0, res_final
int ora_bdf2_step(void* h, double* q, const double* q_nm1, const double* dopt, const int* iopt,
                  int* istat, double* dstat) {
    Ctx& c = *(Ctx*)h;
    StepOpts o{dopt[0], dopt[1], dopt[2], dopt[3], dopt[4], iopt[0], iopt[1], iopt[2], iopt[3], iopt[4]};
    StepStats st;
    int rc = bdf2_step(c, q, q_nm1, o, st);
    istat[0] = st.newton_its; istat[1] = st.gmres_its; istat[2] = st.converged;
    dstat[0] = st.res0; dstat[1] = st.res_final;
    return rc;
}

// Steady pseudo-transient continuation with SER; q updated in place.
// dopt: dtau0, dtau_min, dtau_max, r_ser, tol_pseudo, tol_res, tol_abs, reject_growth;
// iopt: krylov, max_lin_it, max_steps, jac_lag, precond
// istat: steps (accepted and rejected), gmres_its, converged, rejected steps;
// dstat: res0, res_final, dtau of the last step taken;
// hist (length 2 * (max_steps + 1), may be null): Res_m, dtau_m of every step (rejected: -dtau)
int ora_steady_solve(void* h, double* q, const double* dopt, const int* iopt, int* istat, double* dstat,
                     double* hist) {
    Ctx& c = *(Ctx*)h;
    SteadyOpts o{dopt[0], dopt[1], dopt[2], dopt[3], dopt[4], dopt[5], dopt[6], dopt[7], iopt[0], iopt[1], iopt[2],
                 iopt[3], iopt[4]};
    StepStats st;
    double dtf = 0.0;
    std::vector<double> hv;
    int nrej = 0;
    int rc = steady_solve(c, q, o, st, &dtf, &hv, &nrej);
    istat[0] = st.newton_its + nrej; istat[1] = st.gmres_its; istat[2] = st.converged; istat[3] = nrej;
    dstat[0] = st.res0; dstat[1] = st.res_final; dstat[2] = dtf;
    if (hist) std::copy(hv.begin(), hv.end(), hist);
    return rc;
}

// z = P^-1 r for the Newton operator A v = inv_dtau Gamma v + c_time M v - J v at q:
// precond 0 block Jacobi, 1 symmetric block Gauss-Seidel in colour order, 2 forward block
// Gauss-Seidel in colour order.  colours (may be null) receives the element colours.
int ora_precond_apply(void* h, const double* q, double c_time, double inv_dtau, int precond, const double* r,
                      double* z, int* colours) {
    Ctx& c = *(Ctx*)h;
    const int Np = c.Np, E = c.E, nb = 4 * Np;
    const size_t N = (size_t)4 * E * Np;
    NSPhys ph{&c};
    auto time_mat = [&](int e, int s, double T4[4][4]) {
        double qs[4]; for (int v = 0; v < 4; ++v) qs[v] = q[((size_t)v * E + e) * Np + s];
        double M[4][4], G[4][4]; mat_M(c, qs, M);
        const size_t id = (size_t)e * Np + s;
        mat_Gamma(c, qs, c.ugs[id], c.vgs[id], G);
        for (int a = 0; a < 4; ++a) for (int k = 0; k < 4; ++k) T4[a][k] = inv_dtau * G[a][k] + c_time * M[a][k];
    };
    std::vector<double> blk((size_t)E * nb * nb); std::vector<int> piv((size_t)E * nb);
    Traces<cplx> trz;
    std::vector<cplx> qz(q, q + N);
    compute_traces(c, ph, qz.data(), trz);
    for (int e = 0; e < E; ++e) {
        double* B = blk.data() + (size_t)e * nb * nb;
        element_block_cs(c, q, trz, e, B);
        for (int a = 0; a < nb * nb; ++a) B[a] = -B[a];
        for (int s = 0; s < Np; ++s) {
            double T4[4][4]; time_mat(e, s, T4);
            for (int a = 0; a < 4; ++a) for (int k = 0; k < 4; ++k) B[(size_t)(a * Np + s) * nb + k * Np + s] += T4[a][k];
        }
        if (lu_factor(nb, B, piv.data() + (size_t)e * nb) != 0) return -5;
    }
    auto Aop = [&](const double* v, double* out) {
        jvp_cs(c, q, v, out);
        for (int e = 0; e < E; ++e)
            for (int s = 0; s < Np; ++s) {
                double T4[4][4]; time_mat(e, s, T4);
                for (int a = 0; a < 4; ++a) {
                    double t = 0.0;
                    for (int k = 0; k < 4; ++k) t += T4[a][k] * v[((size_t)k * E + e) * Np + s];
                    const size_t id = ((size_t)a * E + e) * Np + s;
                    out[id] = t - out[id];
                }
            }
    };
    int ncol = 0;
    const std::vector<int> col = colour_elements(c, ncol);
    if (colours) std::copy(col.begin(), col.end(), colours);
    precond_apply(c, precond, col, ncol, blk, piv, Aop, r, z);
    return 0;
}

}  // extern "C"
