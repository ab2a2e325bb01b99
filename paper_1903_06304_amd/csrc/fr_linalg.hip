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

constexpr int RED_BLOCKS = 2048;  // first-stage partial sums per reduction (8 workgroups per CU)
constexpr int RED_THREADS = 256;
constexpr int MAXV = 64;          // max vectors in one multi-dot

// ------------------------------------------------------------------ block inversion
template <class Tout>
__device__ __forceinline__ Tout to_store(double x);
template <> __device__ __forceinline__ double to_store<double>(double x) { return x; }
template <> __device__ __forceinline__ float to_store<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ uint16_t to_store<uint16_t>(double x) {
    float f = (float)x;
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);                       // round to nearest even
    return (uint16_t)(r >> 16);
}
__device__ __forceinline__ double from_store(double x) { return x; }
__device__ __forceinline__ double from_store(float x) { return (double)x; }
__device__ __forceinline__ double from_store(uint16_t x) { return (double)__uint_as_float(((uint32_t)x) << 16); }

// A is column-major in global (a[col*nb + row]); LDS holds it row-major with a padded stride.
template <class Tout>
__global__ void __launch_bounds__(256) k_block_invert(int E, int nb, const double* __restrict__ blk,
                                                      Tout* __restrict__ inv, int* __restrict__ status) {
    extern __shared__ double lds[];
    const int ld = nb + 1;
    double* A = lds;                       // [nb][ld]
    double* colk = lds + (size_t)nb * ld;  // [nb]
    int* perm = (int*)(colk + nb);         // [nb]
    __shared__ int s_piv;
    __shared__ double s_pval;
    const int e = blockIdx.x;
    if (e >= E) return;
    const double* src = blk + (size_t)e * nb * nb;
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int c = t / nb, r = t % nb;
        A[r * ld + c] = src[t];
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        // pivot search over rows k..nb-1 by the first wave (ties -> smallest row)
        if (threadIdx.x < 64) {
            double best = -1.0;
            int br = k;
            for (int r = k + (int)threadIdx.x; r < nb; r += 64) {
                const double a = fabs(A[r * ld + k]);
                if (a > best) { best = a; br = r; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_down(best, off, 64);
                const int orr = __shfl_down(br, off, 64);
                if (ob > best || (ob == best && orr < br)) { best = ob; br = orr; }
            }
            if (threadIdx.x == 0) { s_piv = br; s_pval = A[br * ld + k]; perm[k] = br; }
        }
        __syncthreads();
        const int pr = s_piv;
        const double pv = s_pval;
        if (pv == 0.0) {
            if (threadIdx.x == 0) *status = 1;   // plain vector store
            return;   // uniform across the workgroup
        }
        if (pr != k) {
            for (int c = threadIdx.x; c < nb; c += blockDim.x) {
                const double t0 = A[k * ld + c];
                A[k * ld + c] = A[pr * ld + c];
                A[pr * ld + c] = t0;
            }
        }
        __syncthreads();
        // scale the pivot row (A[k][k] := 1 first so the inverse accumulates in place)
        const double ip = 1.0 / pv;
        for (int c = threadIdx.x; c < nb; c += blockDim.x) {
            const double a = (c == k) ? 1.0 : A[k * ld + c];
            A[k * ld + c] = a * ip;
        }
        for (int r = threadIdx.x; r < nb; r += blockDim.x) colk[r] = (r == k) ? 0.0 : A[r * ld + k];
        __syncthreads();
        for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
            const int r = t / nb, c = t % nb;
            if (r == k) continue;
            const double a = (c == k) ? 0.0 : A[r * ld + c];
            A[r * ld + c] = a - colk[r] * A[k * ld + c];
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges, last first
    for (int k = nb - 1; k >= 0; --k) {
        const int pr = perm[k];
        if (pr != k) {
            for (int r = threadIdx.x; r < nb; r += blockDim.x) {
                const double t0 = A[r * ld + k];
                A[r * ld + k] = A[r * ld + pr];
                A[r * ld + pr] = t0;
            }
        }
        __syncthreads();
    }
    Tout* dst = inv + (size_t)e * nb * nb;
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int c = t / nb, r = t % nb;
        dst[t] = to_store<Tout>(A[r * ld + c]);   // column-major inverse
    }
}

// z_e = Ainv_e r_e; state layout [4][E][Np], block row/col index v*Np + s
template <class Tin>
__global__ void __launch_bounds__(256) k_block_apply(int E, int Np, const Tin* __restrict__ inv,
                                                     const double* __restrict__ r, double* __restrict__ z,
                                                     const int* skip) {
    extern __shared__ double rs[];
    if (skip && *skip) return;
    const int nb = 4 * Np;
    const int epb = blockDim.x / nb;
    const int el = threadIdx.x / nb, row = threadIdx.x % nb;
    const int e = blockIdx.x * epb + el;
    const bool act = (el < epb) && (e < E);
    const size_t EN = (size_t)E * Np;
    if (act) rs[el * nb + row] = r[(row / Np) * EN + (size_t)e * Np + (row % Np)];
    __syncthreads();
    if (!act) return;
    const Tin* A = inv + (size_t)e * nb * nb;
    double acc = 0.0;
    for (int c = 0; c < nb; ++c) acc += from_store(A[(size_t)c * nb + row]) * rs[el * nb + c];
    z[(row / Np) * EN + (size_t)e * Np + (row % Np)] = acc;
}

// ------------------------------------------------------------------ Krylov reductions
// Dot products V_i . w for i in [8*blockIdx.y, 8*blockIdx.y + 8) ∩ [0, nv), plus |w|^2 in slot
// nv when want_norm (chunk 0 only): per-block partial sums partial[b][i].
__global__ void __launch_bounds__(RED_THREADS) k_dots8(size_t N, const double* __restrict__ V, size_t ldv, int nv,
                                                       const double* __restrict__ w, int want_norm,
                                                       double* __restrict__ partial, const int* skip) {
    __shared__ double red[RED_THREADS / 64][9];
    if (skip && *skip) return;
    const int i0 = blockIdx.y * 8;
    const int cnt = nv - i0 < 8 ? nv - i0 : 8;
    const bool nrm = want_norm && blockIdx.y == 0;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double nacc = 0.0;
    const double* Vc = V + (size_t)i0 * ldv;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x) {
        const double wt = w[t];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < cnt) acc[i] += Vc[i * ldv + t] * wt;
        if (nrm) nacc += wt * wt;
    }
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const bool live = (i < cnt) || (i == 8 && nrm);
        if (!live) continue;
        double v = (i < 8) ? acc[i] : nacc;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wid][i] = v;
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < cnt || (k == 8 && nrm)) {
        double v = 0.0;
        for (int q = 0; q < RED_THREADS / 64; ++q) v += red[q][k];
        partial[(size_t)blockIdx.x * MAXV + (k < 8 ? i0 + k : nv)] = v;
    }
}

// w_out = w_in - sum_{i < nv} coef[i] V_i, and partial |w_out|^2 in slot 0 when want_norm
__global__ void __launch_bounds__(RED_THREADS) k_update(size_t N, const double* __restrict__ V, size_t ldv, int nv,
                                                        const double* __restrict__ coef, const double* w_in,
                                                        double* w_out, int want_norm, double* __restrict__ partial,
                                                        const int* skip) {
    __shared__ double cf[MAXV];
    __shared__ double red[RED_THREADS / 64];
    if (skip && *skip) return;
    if ((int)threadIdx.x < MAXV) cf[threadIdx.x] = ((int)threadIdx.x < nv) ? coef[threadIdx.x] : 0.0;
    __syncthreads();
    double nacc = 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x) {
        double wt = w_in[t];
        int i = 0;
        for (; i + 4 <= nv; i += 4)
            wt -= cf[i] * V[i * ldv + t] + cf[i + 1] * V[(i + 1) * ldv + t] + cf[i + 2] * V[(i + 2) * ldv + t] +
                  cf[i + 3] * V[(i + 3) * ldv + t];
        for (; i < nv; ++i) wt -= cf[i] * V[i * ldv + t];
        w_out[t] = wt;
        nacc += wt * wt;
    }
    if (!want_norm) return;
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    for (int off = 32; off > 0; off >>= 1) nacc += __shfl_down(nacc, off, 64);
    if (lane == 0) red[wid] = nacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int q = 0; q < RED_THREADS / 64; ++q) v += red[q];
        partial[(size_t)blockIdx.x * MAXV] = v;
    }
}

// out[i] = sum over blocks of partial[b][i]; one workgroup per output, fixed-order tree
__global__ void __launch_bounds__(256) k_final(int nblocks, const double* __restrict__ partial, double* __restrict__ out,
                                               const int* skip) {
    __shared__ double red[256];
    if (skip && *skip) return;
    const int i = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partial[(size_t)b * MAXV + i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
}

// out = sum_i y[i] V_i
__global__ void k_combine(size_t N, double* __restrict__ out, const double* __restrict__ V, size_t ldv, int nv,
                          const double* __restrict__ y) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < nv; ++i) s += y[i] * V[i * ldv + t];
        out[t] = s;
    }
}

__global__ void k_axpy(size_t N, double a, const double* __restrict__ x, double* __restrict__ y) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x)
        y[t] += a * x[t];
}

__global__ void k_scale_copy(size_t N, double a, const double* __restrict__ x, double* __restrict__ y) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (size_t)gridDim.x * blockDim.x)
        y[t] = a * x[t];
}

// q^c of the state (per solution point)
__global__ void k_cons(size_t EN, PhysConst pc, const double* __restrict__ q, double* __restrict__ Qc) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= EN) return;
    double qs[4], qc[4];
    for (int v = 0; v < 4; ++v) qs[v] = q[v * EN + t];
    fr_cons(pc, qs, qc);
    for (int v = 0; v < 4; ++v) Qc[v * EN + t] = qc[v];
}

// b = -(a0 q^c(q) + a1 Q^n + a2 Q^{n-1}) / dt + R
__global__ void k_bdf_rhs(size_t EN, PhysConst pc, const double* __restrict__ q, const double* __restrict__ Qn,
                          const double* __restrict__ Qnm1, const double* __restrict__ R, double a0, double a1, double a2,
                          double idt, double* __restrict__ b) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= EN) return;
    double qs[4], qc[4];
    for (int v = 0; v < 4; ++v) qs[v] = q[v * EN + t];
    fr_cons(pc, qs, qc);
    for (int v = 0; v < 4; ++v) {
        double acc = a0 * qc[v] + a1 * Qn[v * EN + t];
        if (Qnm1) acc += a2 * Qnm1[v * EN + t];
        b[v * EN + t] = R[v * EN + t] - acc * idt;
    }
}

unsigned grid_for(size_t N, int bs) {
    size_t g = (N + bs - 1) / bs;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

// ----------------------------------------------------------------------------- launchers
fr_status launch_block_assembly(fr_ctx c, const double* q, double c_time, double inv_dtau, hipStream_t s) {
    // one seeded column of every element's block per launch
    fr_status st = FR_OK;
    const int nb = 4 * c->Np;
    KArgs a{};
    a.E = c->E; a.q = q; a.v = nullptr; a.out = c->d_blk;
    a.c_time = c_time; a.inv_dtau = inv_dtau;
    for (int col = 0; col < nb; ++col) {
        a.seed0 = col;
        st = launch_residual(c, MODE_BLK, a, s);
        if (st != FR_OK) return st;
    }
    return FR_OK;
}

fr_status launch_block_invert(fr_ctx c, int prec, hipStream_t s) {
    const int nb = 4 * c->Np;
    const size_t lds = ((size_t)nb * (nb + 1) + nb) * sizeof(double) + nb * sizeof(int);
    int* d_status = (int*)(c->d_scal + SC_STATUS);
    FR_HIP(hipMemsetAsync(d_status, 0, sizeof(int), s));
    switch (prec) {
        case FR_FP64:
            FR_HIP(hipFuncSetAttribute((const void*)k_block_invert<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(k_block_invert<double>, dim3(c->E), dim3(256), lds, s, c->E, nb, c->d_blk, (double*)c->d_inv, d_status);
            break;
        case FR_FP32:
            FR_HIP(hipFuncSetAttribute((const void*)k_block_invert<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(k_block_invert<float>, dim3(c->E), dim3(256), lds, s, c->E, nb, c->d_blk, (float*)c->d_inv, d_status);
            break;
        case FR_BF16:
            FR_HIP(hipFuncSetAttribute((const void*)k_block_invert<uint16_t>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(k_block_invert<uint16_t>, dim3(c->E), dim3(256), lds, s, c->E, nb, c->d_blk, (uint16_t*)c->d_inv, d_status);
            break;
        default:
            fr_set_error("unknown precision");
            return FR_EINVAL;
    }
    FR_HIP(hipGetLastError());
    c->inv_prec = prec;
    return FR_OK;
}

fr_status launch_block_apply(fr_ctx c, const double* r, double* z, hipStream_t s, const int* skip) {
    const int nb = 4 * c->Np;
    const int epb = 256 / nb;
    const int threads = epb * nb;
    const unsigned grid = (unsigned)((c->E + epb - 1) / epb);
    const size_t lds = (size_t)threads * sizeof(double);
    switch (c->inv_prec) {
        case FR_FP64: hipLaunchKernelGGL(k_block_apply<double>, dim3(grid), dim3(threads), lds, s, c->E, c->Np, (const double*)c->d_inv, r, z, skip); break;
        case FR_FP32: hipLaunchKernelGGL(k_block_apply<float>, dim3(grid), dim3(threads), lds, s, c->E, c->Np, (const float*)c->d_inv, r, z, skip); break;
        case FR_BF16: hipLaunchKernelGGL(k_block_apply<uint16_t>, dim3(grid), dim3(threads), lds, s, c->E, c->Np, (const uint16_t*)c->d_inv, r, z, skip); break;
        default: fr_set_error("preconditioner not factored"); return FR_EINVAL;
    }
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status la_krylov(fr_ctx c, size_t N, const double* V, int nv_upd, const double* d_coef, int nv_dot,
                    const double* w_in, double* w_out, bool want_norm, double* d_out, hipStream_t s,
                    const int* skip) {
    if (nv_upd > MAXV - 1 || nv_dot > MAXV - 1) { fr_set_error("too many Krylov vectors"); return FR_EINVAL; }
    double* partial = c->d_scal + SC_PART;
    const size_t ldv = c->N();
    const double* w = w_in;
    if (nv_upd > 0) {
        // the norm of the updated vector rides on the update pass when no dots follow
        const int nrm = (want_norm && nv_dot == 0) ? 1 : 0;
        hipLaunchKernelGGL(k_update, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, N, V, ldv, nv_upd, d_coef, w_in, w_out,
                           nrm, partial, skip);
        FR_HIP(hipGetLastError());
        w = w_out;
        if (nv_dot == 0) {
            if (nrm) {
                hipLaunchKernelGGL(k_final, dim3(1), dim3(256), 0, s, RED_BLOCKS, partial, d_out, skip);
                FR_HIP(hipGetLastError());
            }
            return FR_OK;
        }
    }
    const int chunks = nv_dot > 0 ? (nv_dot + 7) / 8 : 1;
    hipLaunchKernelGGL(k_dots8, dim3(RED_BLOCKS, chunks), dim3(RED_THREADS), 0, s, N, V, ldv, nv_dot, w,
                       want_norm ? 1 : 0, partial, skip);
    FR_HIP(hipGetLastError());
    const int nout = nv_dot + (want_norm ? 1 : 0);
    if (nout > 0) {
        hipLaunchKernelGGL(k_final, dim3(nout), dim3(256), 0, s, RED_BLOCKS, partial, d_out, skip);
        FR_HIP(hipGetLastError());
    }
    return FR_OK;
}

fr_status la_dots(fr_ctx c, size_t N, const double* V, int nv, const double* w, double* d_out, hipStream_t s) {
    return la_krylov(c, N, V, 0, nullptr, nv, w, nullptr, false, d_out, s);
}

fr_status la_combine(size_t N, const double* V, int nv, const double* d_y, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3(grid_for(N, 256)), dim3(256), 0, s, N, out, V, N, nv, d_y);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status la_axpy(size_t N, double a, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(N, 256)), dim3(256), 0, s, N, a, x, y);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status la_scale_copy(size_t N, double a, const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(N, 256)), dim3(256), 0, s, N, a, x, y);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status launch_cons(fr_ctx c, const double* q, double* Qc, hipStream_t s) {
    const size_t EN = (size_t)c->E * c->Np;
    hipLaunchKernelGGL(k_cons, dim3((unsigned)((EN + 255) / 256)), dim3(256), 0, s, EN, c->pc, q, Qc);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

fr_status launch_bdf_rhs(fr_ctx c, const double* q, const double* Qn, const double* Qnm1, const double* R,
                         double a0, double a1, double a2, double dt, double* b, hipStream_t s) {
    const size_t EN = (size_t)c->E * c->Np;
    hipLaunchKernelGGL(k_bdf_rhs, dim3((unsigned)((EN + 255) / 256)), dim3(256), 0, s, EN, c->pc, q, Qn, Qnm1, R, a0, a1,
                       a2, 1.0 / dt, b);
    FR_HIP(hipGetLastError());
    return FR_OK;
}
