// Explicit inverse of every element block (the element-block-Jacobi preconditioner of the
// paper's Sec. 4 set-up): Gauss-Jordan elimination with partial pivoting, blocked by
// panels of 16 columns, with the trailing update of each panel on the matrix cores.
//
// One workgroup (4 waves) per element; the block, padded to NBP = 16 ceil(nb / 16) rows
// and columns with an identity on the padding, sits in LDS column-major.  Per panel of
// columns kb .. kb + 15:
//   1. wave 0 runs the 16 Gauss-Jordan steps on the panel columns only, over every row
//      (lane l holds rows l and l + 64, where they exist, in registers).  Step j takes as pivot the unused
//      row with the largest |a(r, kb + j)| (lowest row on ties) and applies the in-place
//      inverse update: rows stay where they are, column kb + j becomes the transformed
//      unit vector of the pivot row.  The panel then holds W = M [e_p(0) .. e_p(15)], M
//      the product of the 16 elementary transforms;
//   2. every other column c becomes M c = W c(pivot rows) + (c with the panel's pivot rows
//      zeroed): a rank-16 product W (NBP x 16) times the pivot rows (16 x NBP - 16) added
//      to the rest, formed as 16 x 16 output tiles of v_mfma_*_16x16x4 (4 k-steps each).
//      Wave w owns the column tiles J = w mod 4 and reads its pivot-row operands into
//      registers before it writes any tile of its columns, so no copy is needed.
// After the last panel the block holds the inverse with rows and columns permuted by
// the pivot order: inverse(pos(r), piv(k)) = a(r, k), pos the step at which row r was
// the pivot.  Padding columns pick their own padding row with pivot 1 and change nothing.
//
// Arithmetic type TC: FP64 (MFMA f64 16x16x4) for an FP64 inverse; FP32 (MFMA f32
// 16x16x4, FP32 accumulation) for an FP32 or BF16 inverse, the FP64 block rounded to
// FP32 on load and the FP32 result rounded to nearest even for BF16.
#include "fr_internal.hpp"

namespace {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

// 16x16x4 products D = A B + C on one wave: lane l supplies A(l % 16, l / 16) and
// B(l / 16, l % 16); its r-th accumulator element is D(row(l, r), l % 16).  The output row
// order differs between the FP64 and FP32 instructions (checked on the device).
template <class TC> struct Mfma;
template <> struct Mfma<double> {
    using V = mf_d4;
    __device__ __forceinline__ static V step(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
    using V = mf_f4;
    __device__ __forceinline__ static V step(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <class TO, class TC> __device__ __forceinline__ TO store_as(TC x);
template <> __device__ __forceinline__ double store_as<double, double>(double x) { return x; }
template <> __device__ __forceinline__ float store_as<float, float>(float x) { return x; }
template <> __device__ __forceinline__ uint16_t store_as<uint16_t, float>(float x) {
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);           // round to nearest even
}

// Cross-lane moves of a double, no LDS: a DPP move within rows of 16 lanes, and a read
// of one lane into scalar registers.
template <int CTRL> __device__ __forceinline__ double dpp_mov(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL> __device__ __forceinline__ float dpp_mov(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_value(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane_value(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
// maximum over the wave: DPP within each row of 16 lanes (quad swaps, then rotations by 4
// and 8), then the four row maxima read into scalar registers
template <class T> __device__ __forceinline__ T wave_max(T m) {
    m = fmax(m, dpp_mov<0xB1>(m));    // quad_perm [1, 0, 3, 2]
    m = fmax(m, dpp_mov<0x4E>(m));    // quad_perm [2, 3, 0, 1]
    m = fmax(m, dpp_mov<0x124>(m));   // row_ror 4
    m = fmax(m, dpp_mov<0x128>(m));   // row_ror 8
    return fmax(fmax(lane_value(m, 0), lane_value(m, 16)), fmax(lane_value(m, 32), lane_value(m, 48)));
}

__device__ __forceinline__ int case_of_tile(const GroupArgs& ga, int t) {
    int lo = 0, hi = ga.nmem - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ga.pfx[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int NB, class TC, class TO>
__global__ void __launch_bounds__(256) k_block_invert_mfma(GroupArgs ga, const double* __restrict__ blk,
                                                           TO* __restrict__ inv, int* __restrict__ gi,
                                                           const int* __restrict__ flags, int cl) {
    constexpr int NBP = (NB + 15) / 16 * 16, NT = NBP / 16;
    // column stride: one element of padding against bank conflicts where LDS allows two
    // blocks per CU either way (an FP64 100 x 100 block takes LD = NB to fit twice)
    constexpr int LD = (NB * (NB + 1) * sizeof(TC) <= 80000) ? NB + 1 : NB;
    static_assert(NB < 255, "pivot bookkeeping in bytes");
    __shared__ TC A[NB * LD];          // the real block, column c at A + c * LD; the padding is
                                       // an identity that the elimination never changes
    __shared__ uint8_t s_piv[NB];      // pivot row of each step
    __shared__ uint8_t s_pos[NB];      // step at which each row was the pivot, 255 before
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int t = blockIdx.x;
    if (t >= ga.ntiles) return;                                   // uniform per workgroup
    const int lo = case_of_tile(ga, t);
    const int cid = ga.ids[lo];
    if (flags && flags[cid * GI_STRIDE + GI_NDONE]) return;       // uniform per workgroup
    const CaseDev& cd = ga.cases[cid];
    // slot of the stored inverse; its element is the same index, or the slot's entry of the
    // colour-sorted element list in the colour layout
    const int slot = t - ga.pfx[lo];
    const int e = cl ? cd.g.corder[slot] : slot;
    const double* src = blk + cd.boff + (size_t)e * NB * NB;
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int c = idx / NB, r = idx % NB;
        A[c * LD + r] = (TC)src[idx];
    }
    for (int r = tid; r < NB; r += 256) s_pos[r] = 255;
    if (tid == 0) s_bad = 0;
    __syncthreads();

    for (int kb = 0; kb < NB; kb += 16) {
        const int nk = NB - kb < 16 ? NB - kb : 16;   // real steps of this panel
        if (wave == 0) {
            // the panel's Gauss-Jordan steps on one wave: lane l holds rows l and l + 64
            // (where they exist) of the panel columns in registers; pivot search and pivot
            // row broadcast through DPP moves and scalar reads, no LDS
            constexpr bool TWO = NB > 64;
            const int r0 = lane, r1 = lane + 64;
            const bool h0 = r0 < NB, h1 = TWO && r1 < NB;
            TC p0[16], p1[TWO ? 16 : 1];
#pragma unroll
            for (int c = 0; c < 16; ++c) p0[c] = (h0 && c < nk) ? A[(kb + c) * LD + r0] : TC(0);
            if (TWO) {
#pragma unroll
                for (int c = 0; c < 16; ++c) p1[TWO ? c : 0] = (h1 && c < nk) ? A[(kb + c) * LD + r1] : TC(0);
            }
            bool u0 = h0 ? s_pos[r0] != 255 : true;
            bool u1 = h1 ? s_pos[r1] != 255 : true;
            bool bad = false;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < nk) {   // uniform
                    const TC m0 = u0 ? TC(-1) : fabs(p0[j]);
                    const TC m1 = u1 ? TC(-1) : fabs(p1[TWO ? j : 0]);
                    const TC m = wave_max(fmax(m0, m1));
                    const unsigned long long c0 = __ballot(!u0 && m0 == m);
                    const unsigned long long c1 = __ballot(!u1 && m1 == m);
                    int prow = __builtin_amdgcn_readfirstlane(
                        c0 ? (int)__ffsll((long long)c0) - 1 : (c1 ? 64 + (int)__ffsll((long long)c1) - 1 : -1));
                    // no usable pivot: the block is singular (or not finite); the steps run on
                    // with row 0 so that the loop stays straight-line code, and the block is
                    // discarded
                    const bool ok = prow >= 0 && m > TC(0);
                    bad = bad || !ok;
                    prow = ok ? prow : 0;
                    const bool own0 = h0 && r0 == prow, own1 = h1 && r1 == prow;
                    TC pr[16];
                    const int pl = prow & 63;
                    if (!TWO || prow < 64) {
#pragma unroll
                        for (int c = 0; c < 16; ++c) pr[c] = lane_value(p0[c], pl);
                    } else {
#pragma unroll
                        for (int c = 0; c < 16; ++c) pr[c] = lane_value(p1[TWO ? c : 0], pl);
                    }
                    const TC ip = TC(1) / pr[j];
                    const TC f0 = p0[j], f1 = p1[TWO ? j : 0];
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const TC pc = (c == j ? TC(1) : pr[c]) * ip;   // normalised pivot row
                        p0[c] = own0 ? pc : ((c == j) ? TC(0) : p0[c]) - f0 * pc;
                        if (TWO) p1[TWO ? c : 0] = own1 ? pc : ((c == j) ? TC(0) : p1[TWO ? c : 0]) - f1 * pc;
                    }
                    u0 = u0 || own0;
                    u1 = u1 || own1;
                    if (lane == 0) {
                        s_piv[kb + j] = (uint8_t)prow;
                        s_pos[prow] = (uint8_t)(kb + j);
                    }
                }
            }
            if (bad && lane == 0) s_bad = 1;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                if (c < nk) {
                    if (h0) A[(kb + c) * LD + r0] = p0[c];
                    if (h1) A[(kb + c) * LD + r1] = p1[TWO ? c : 0];
                }
            }
        }
        __syncthreads();
        if (s_bad) {
            if (tid == 0) gi[cid * GI_STRIDE + GI_STATUS] = 3;   // plain vector store
            return;                                               // uniform per workgroup
        }
        // trailing update: every column tile but the panel's, D = W Y + Z, with the padding
        // read as zeros (its identity part never meets a real row or column here) and
        // padding results dropped
        const int pj = kb / 16;
        for (int J = wave; J < NT; J += 4) {
            if (J == pj) continue;
            const int col = 16 * J + (lane & 15);
            const bool cin = col < NB;
            TC b[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 4 * s + (lane >> 4);
                b[s] = (cin && k < nk) ? A[col * LD + s_piv[kb + k]] : TC(0);
            }
            for (int I = 0; I < NT; ++I) {
                typename Mfma<TC>::V acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * I + Mfma<TC>::row(lane, r);
                    const bool in = cin && row < NB;
                    const int ps = in ? s_pos[row] : 255;
                    acc[r] = (!in || (ps >= kb && ps < kb + nk)) ? TC(0) : A[col * LD + row];
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = 4 * s + (lane >> 4), row = 16 * I + (lane & 15);
                    const TC a = (k < nk && row < NB) ? A[(kb + k) * LD + row] : TC(0);
                    acc = Mfma<TC>::step(a, b[s], acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * I + Mfma<TC>::row(lane, r);
                    if (cin && row < NB) A[col * LD + row] = acc[r];
                }
            }
        }
        __syncthreads();
    }
    // inverse(row R, col C) = a(piv(R), pos(C)); written column-major, consecutive threads
    // on consecutive rows
    TO* dst = inv + cd.boff + (size_t)slot * NB * NB;
    for (int idx = tid; idx < NB * NB; idx += 256) {
        const int C = idx / NB, R = idx % NB;
        dst[idx] = store_as<TO, TC>(A[s_pos[C] * LD + s_piv[R]]);
    }
}

template <int NB, class TC, class TO>
fr_status launch_nb(Solver& sv, const GroupArgs& ga, const int* flags, hipStream_t s) {
    hipLaunchKernelGGL((k_block_invert_mfma<NB, TC, TO>), dim3(ga.ntiles), dim3(256), 0, s, ga, sv.d_blk,
                       (TO*)sv.d_inv, sv.d_gi, flags, sv.inv_colour ? 1 : 0);
    FR_HIP(hipGetLastError());
    return FR_OK;
}

template <class TC, class TO>
fr_status launch_p(Solver& sv, int p, const GroupArgs& ga, const int* flags, hipStream_t s) {
    switch (p) {
        case 1: return launch_nb<16, TC, TO>(sv, ga, flags, s);
        case 2: return launch_nb<36, TC, TO>(sv, ga, flags, s);
        case 3: return launch_nb<64, TC, TO>(sv, ga, flags, s);
        case 4: return launch_nb<100, TC, TO>(sv, ga, flags, s);
    }
    fr_set_error("order outside 1..4");
    return FR_EUNSUPPORTED;
}

}  // namespace

fr_status launch_block_invert_group(Solver& sv, int p, const GroupArgs& ga, int prec, const int* flags,
                                    hipStream_t s) {
    if (ga.ntiles == 0) return FR_OK;
    switch (prec) {
        case FR_FP64: return launch_p<double, double>(sv, p, ga, flags, s);
        case FR_FP32: return launch_p<float, float>(sv, p, ga, flags, s);
        case FR_BF16: return launch_p<float, uint16_t>(sv, p, ga, flags, s);
    }
    fr_set_error("unknown precision");
    return FR_EINVAL;
}
