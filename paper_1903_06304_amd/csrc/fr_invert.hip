// Gauss-Jordan inversion with partial pivoting of element blocks larger than one wave
// (p = 4: 100 rows), two waves per element, the block held in registers (lane L of wave
// w owns row 64 w + L).  Step k: each wave proposes its largest |a[k]| among the rows not
// used yet (lowest row on ties), the workgroup takes the larger proposal (wave 0 on
// ties), the owner of the pivot row publishes it in LDS, and every row eliminates column
// k with the in-place inverse trick.  Same per-entry arithmetic as the one-wave kernel;
// pivoting is implicit (rows stay in place) and the output is permuted as there.
// The LDS proposal and pivot-row buffers alternate between even and odd steps, so two
// barriers per step suffice.
#include "fr_internal.hpp"

#include <climits>

namespace {

template <class Tout> __device__ __forceinline__ Tout store_as(double x);
template <> __device__ __forceinline__ double store_as<double>(double x) { return x; }
template <> __device__ __forceinline__ float store_as<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ uint16_t store_as<uint16_t>(double x) {
    const float f = (float)x;
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);           // round to nearest even
}

__device__ __forceinline__ int member_of(const GroupArgs& ga, int t) {
    int lo = 0, hi = ga.nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ga.pfx[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int NB, class Tout>
__global__ void __launch_bounds__(128) k_block_invert_2w(GroupArgs ga, const double* __restrict__ blk,
                                                        Tout* __restrict__ inv, int* __restrict__ gi,
                                                        const int* __restrict__ flags) {
    static_assert(NB > 64 && NB <= 128, "two waves per element");
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, row = 64 * w + lane;
    const int t = blockIdx.x;
    if (t >= ga.ntiles) return;
    const int lo = member_of(ga, t);
    const int cid = ga.ids[lo];
    if (flags && flags[cid * GI_STRIDE + GI_NDONE]) return;
    const CaseDev& cd = ga.cases[cid];
    const int e = t - ga.pfx[lo];
    const double* src = blk + cd.boff + (size_t)e * NB * NB;
    const bool live = row < NB;
    __shared__ double s_cand[2][2];
    __shared__ int s_crow[2][2];
    __shared__ double s_prow[2][NB];
    __shared__ int s_piv[NB];
    double a[NB];
#pragma clang loop unroll(full)
    for (int c = 0; c < NB; ++c) a[c] = live ? src[(size_t)c * NB + row] : 0.0;
    bool used = !live;
    int mystep = 0;
#pragma clang loop unroll(full)
    for (int k = 0; k < NB; ++k) {
        const int bs = k & 1;
        // this wave's proposal
        double m = used ? -1.0 : fabs(a[k]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
        const unsigned long long cand = __ballot(!used && fabs(a[k]) == m);
        if (lane == 0) {
            s_cand[bs][w] = m;
            s_crow[bs][w] = cand ? 64 * w + (int)__ffsll((long long)cand) - 1 : INT_MAX;
        }
        __syncthreads();
        double best = s_cand[bs][0];
        int prow = s_crow[bs][0];
        if (s_cand[bs][1] > best) { best = s_cand[bs][1]; prow = s_crow[bs][1]; }
        if (row == prow) {
#pragma clang loop unroll(full)
            for (int c = 0; c < NB; ++c) s_prow[bs][c] = a[c];
        }
        if (threadIdx.x == 0) s_piv[k] = prow;
        __syncthreads();
        const double pv = s_prow[bs][k];
        if (!(pv != 0.0)) {
            if (threadIdx.x == 0) gi[cid * GI_STRIDE + GI_STATUS] = 3;   // plain vector store
            return;                                                       // uniform per workgroup
        }
        const bool isp = row == prow;
        if (isp) { used = true; mystep = k; }
        const double ip = 1.0 / pv;
        const double f = a[k];
#pragma clang loop unroll(full)
        for (int c = 0; c < NB; ++c) {
            const double pc = ((c == k) ? 1.0 : s_prow[bs][c]) * ip;
            const double ac = (c == k) ? 0.0 : a[c];
            a[c] = isp ? pc : ac - f * pc;
        }
    }
    if (!live) return;
    Tout* dst = inv + cd.boff + (size_t)e * NB * NB;
#pragma clang loop unroll(full)
    for (int k = 0; k < NB; ++k) dst[(size_t)s_piv[k] * NB + mystep] = store_as<Tout>(a[k]);   // column-major
}

template <class Tout>
fr_status run(Solver& sv, const Group& gr, const GroupArgs& ga, const int* flags, hipStream_t s) {
    hipLaunchKernelGGL((k_block_invert_2w<100, Tout>), dim3(ga.ntiles), dim3(128), 0, s, ga, sv.d_blk,
                       (Tout*)sv.d_inv, sv.d_gi, flags);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

}  // namespace

fr_status launch_block_invert_p4(Solver& sv, const Group& gr, const GroupArgs& ga, int prec, const int* flags,
                                 hipStream_t s) {
    switch (prec) {
        case FR_FP64: return run<double>(sv, gr, ga, flags, s);
        case FR_FP32: return run<float>(sv, gr, ga, flags, s);
        case FR_BF16: return run<uint16_t>(sv, gr, ga, flags, s);
    }
    fr_set_error("unknown precision");
    return FR_EINVAL;
}
