// Scalar types of the device code: double, and forward-mode dual numbers with K
// tangent lanes (exact Jacobian-vector products and K seeded columns of the element
// blocks).  Non-smooth operations follow one convention everywhere: max/min return
// the first argument on ties, |x| has slope +1 at x = 0, and the tangent of the
// branch not taken is never propagated.
#pragma once
#include <hip/hip_runtime.h>

#define FR_HD __host__ __device__ __forceinline__

template <int K>
struct Dual {
    double v;
    double d[K];
};

FR_HD double val(double x) { return x; }
template <int K> FR_HD double val(const Dual<K>& x) { return x.v; }

// ---- reciprocal: hardware estimate refined by two Newton steps (error well below 1 ulp
// of the quantities it feeds; replaces the much longer IEEE division sequence)
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ double rcp(double x) { return frcp(x); }
template <int K> __device__ __forceinline__ Dual<K> rcp(const Dual<K>& a) { Dual<K> r; r.v = frcp(a.v);
    const double s = -r.v * r.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * s; return r; }

template <int K> FR_HD Dual<K> mkconst(double a) { Dual<K> r; r.v = a;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = 0.0; return r; }

// ---- arithmetic
template <int K> FR_HD Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) { Dual<K> r; r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int K> FR_HD Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) { Dual<K> r; r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int K> FR_HD Dual<K> operator-(const Dual<K>& a) { Dual<K> r; r.v = -a.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r; }
template <int K> FR_HD Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) { Dual<K> r; r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int K> __device__ __forceinline__ Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) { Dual<K> r;
    const double ib = frcp(b.v);
    r.v = a.v * ib;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib; return r; }
template <int K> FR_HD Dual<K> operator+(const Dual<K>& a, double b) { Dual<K> r = a; r.v += b; return r; }
template <int K> FR_HD Dual<K> operator+(double b, const Dual<K>& a) { Dual<K> r = a; r.v += b; return r; }
template <int K> FR_HD Dual<K> operator-(const Dual<K>& a, double b) { Dual<K> r = a; r.v -= b; return r; }
template <int K> FR_HD Dual<K> operator-(double b, const Dual<K>& a) { Dual<K> r; r.v = b - a.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = -a.d[k]; return r; }
template <int K> FR_HD Dual<K> operator*(const Dual<K>& a, double b) { Dual<K> r; r.v = a.v * b;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b; return r; }
template <int K> FR_HD Dual<K> operator*(double b, const Dual<K>& a) { return a * b; }
template <int K> FR_HD Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K> FR_HD Dual<K> operator/(double a, const Dual<K>& b) { Dual<K> r; r.v = a / b.v;
    const double s = -r.v / b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = s * b.d[k]; return r; }
template <int K> FR_HD Dual<K>& operator+=(Dual<K>& a, const Dual<K>& b) { a = a + b; return a; }
template <int K> FR_HD Dual<K>& operator-=(Dual<K>& a, const Dual<K>& b) { a = a - b; return a; }

// fused multiply-add on the value; tangent by the product rule
FR_HD double fma_(double a, double b, double c) { return fma(a, b, c); }
template <int K> FR_HD Dual<K> fma_(double a, const Dual<K>& b, const Dual<K>& c) { Dual<K> r; r.v = fma(a, b.v, c.v);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = fma(a, b.d[k], c.d[k]); return r; }

// ---- elementary functions
FR_HD double ssqrt(double x) { return sqrt(x); }
template <int K> FR_HD Dual<K> ssqrt(const Dual<K>& a) { Dual<K> r; r.v = sqrt(a.v);
    const double s = 0.5 / r.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * s; return r; }
FR_HD double sabs(double x) { return x >= 0.0 ? x : -x; }
template <int K> FR_HD Dual<K> sabs(const Dual<K>& a) { return a.v >= 0.0 ? a : -a; }
template <class T> FR_HD T smax(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }
template <class T> FR_HD T smin(const T& a, const T& b) { return val(a) <= val(b) ? a : b; }

// generic constant constructor
template <class T> struct Make { FR_HD static T c(double a) { return T(a); } };
template <int K> struct Make<Dual<K>> { FR_HD static Dual<K> c(double a) { return mkconst<K>(a); } };
template <class T> FR_HD T cst(double a) { return Make<T>::c(a); }

// ---- memory helpers: a T is stored as (1 + K) consecutive doubles
template <class T> struct Store;
template <> struct Store<double> {
    static constexpr int W = 1;
    FR_HD static double ld(const double* p) { return *p; }
    FR_HD static void st(double* p, double x) { *p = x; }
};
template <int K> struct Store<Dual<K>> {
    static constexpr int W = 1 + K;
    FR_HD static Dual<K> ld(const double* p) { Dual<K> r; r.v = p[0];
#pragma unroll
        for (int k = 0; k < K; ++k) r.d[k] = p[1 + k]; return r; }
    FR_HD static void st(double* p, const Dual<K>& x) { p[0] = x.v;
#pragma unroll
        for (int k = 0; k < K; ++k) p[1 + k] = x.d[k]; }
};
