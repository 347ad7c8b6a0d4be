// Device-side bodies of the fused dense sweep, shared by the single-state
// kernels and the batched (many states per launch) kernels.
#pragma once

#include "sv_internal.h"

namespace sv {

template <typename R> struct Vec2;
template <> struct Vec2<float> { using T = float2; };
template <> struct Vec2<double> { using T = double2; };

typedef float f4 __attribute__((ext_vector_type(4)));

// Spread group counter g over the non-target positions.
template <int K>
__device__ __forceinline__ uint64_t group_base(const Sweep& a, uint64_t g)
{
    uint64_t base = g;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const uint64_t low = base & a.lowmask[j];
        base = ((base ^ low) << 1) | low;
    }
    return base;
}

__device__ __forceinline__ uint32_t fold_index(const Sweep& a, uint64_t idx)
{
    uint32_t b = 0;
    for (int j = 0; j < a.fold_m; ++j) b |= (uint32_t)((idx >> a.fold_pos[j]) & 1u) << j;
    return b;
}

// VALU form: one lane owns one group and its 2^k amplitudes.  The matrix is
// wave-uniform and read one row per iteration with scalar loads; the row
// loop is not unrolled so only one row (2^(k+1) values) is live in SGPRs.
template <typename R, int K, bool FOLD>
__device__ __forceinline__ void dense_group(const Sweep& a, uint64_t g)
{
    using V = typename Vec2<R>::T;
    constexpr int D = 1 << K;
    V* __restrict__ psi = (V*)a.psi;
    const V* __restrict__ mat = (const V*)a.mat;
    const uint64_t base = group_base<K>(a, g);
    uint64_t bitv[K];
#pragma unroll
    for (int j = 0; j < K; ++j) bitv[j] = 1ull << a.tpos[j];
    V x[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        uint64_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if ((c >> j) & 1) o |= bitv[j];
        x[c] = psi[base + o];
    }
    uint32_t fb = 0;
    if (FOLD) fb = fold_index(a, base + a.idx_offset);
#pragma unroll 1
    for (int r = 0; r < D; ++r) {
        R re = 0, im = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const V m = mat[r * D + c];
            re = fma(m.x, x[c].x, re);
            re = fma(-m.y, x[c].y, re);
            im = fma(m.x, x[c].y, im);
            im = fma(m.y, x[c].x, im);
        }
        // row offset from the target positions (a dynamic index into a
        // per-row table would spill SGPRs)
        uint64_t orow = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) orow |= ((r >> j) & 1) ? bitv[j] : 0ull;
        if (FOLD) {
            const V p = ((const V*)a.ftab)[fb | fold_index(a, orow)];
            const R t = re * p.x - im * p.y;
            im = re * p.y + im * p.x;
            re = t;
        }
        psi[base + orow] = V{re, im};
    }
}

// ---------------------------------------------------------------------------
// Matrix-core form (complex64, k = 4..6), v_mfma_f32_16x16x4f32.
//
// y = M x is the real product [yr; yi] = [[Mr, -Mi], [Mi, Mr]] [xr; xi] of a
// (2D x 2D) matrix A (D = 2^k) with one 2D-vector per group; sixteen groups
// are the 16 columns of the B operand.  Operand layouts (wave64): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its 4 results are
// D[4 (l / 16) + v][l % 16].  So lane l = j + 16 h works on group j:
//   * the K index of k-step s for lane h is (amplitude 4 (s >> 1) + h, part
//     s & 1): the lane loads the D/4 complete amplitudes c = 4 m + h of its
//     group and feeds re / im on alternate k-steps;
//   * output row R = 16 rb + 4 h + v is (amplitude R >> 1, part R & 1): the
//     lane ends with complete (re, im) pairs of amplitudes 8 rb + 2 h + {0, 1}.
// A is staged in LDS in operand order: one ds_read_b128 gives a lane its A
// operands for four consecutive k-steps.
// ---------------------------------------------------------------------------
template <int K>
struct MfmaShape {
    static constexpr int D = 1 << K;
    static constexpr int RB = 2 * D / 16;    // 16-row blocks of A
    static constexpr int KQ = 2 * D / 16;    // groups of four k-steps
    static constexpr int NA = RB * KQ * 256; // floats of A
};

template <int K>
__device__ __forceinline__ void mfma_stage_matrix(f4* As, const float2* __restrict__ mat)
{
    using S = MfmaShape<K>;
    for (int i = threadIdx.x; i < S::NA; i += blockDim.x) {
        const int s4 = i & 3, l = (i >> 2) & 63, blk = i >> 8;
        const int sq = blk % S::KQ, rb = blk / S::KQ;
        const int s = 4 * sq + s4;
        const int R = 16 * rb + (l & 15);
        const int c = 4 * (s >> 1) + (l >> 4), p = s & 1;
        const int r = R >> 1, q = R & 1;
        const float2 m = mat[r * S::D + c];
        ((float*)As)[i] = (q == 0) ? (p == 0 ? m.x : -m.y) : (p == 0 ? m.y : m.x);
    }
}

// Tiles [t0, t_end) with stride `step` of one sweep, for the calling wave.
template <int K, bool FOLD>
__device__ __forceinline__ void mfma_tiles(const Sweep& a, const f4* As, uint64_t t0, uint64_t step,
                                           uint64_t t_end)
{
    using S = MfmaShape<K>;
    constexpr int D = S::D, RB = S::RB, KQ = S::KQ;
    float2* __restrict__ psi = (float2*)a.psi;
    const int lane = threadIdx.x & 63;
    const int j = lane & 15, h = lane >> 4;
    uint64_t bitv[K];
#pragma unroll
    for (int t = 0; t < K; ++t) bitv[t] = 1ull << a.tpos[t];

    auto load_tile = [&](uint64_t t, float2* xx, uint64_t& b) {
        b = group_base<K>(a, t * 16 + j);
#pragma unroll
        for (int m = 0; m < D / 4; ++m) {
            uint64_t o = (h & 1) ? bitv[0] : 0ull;
            o |= (h & 2) ? bitv[1] : 0ull;
#pragma unroll
            for (int u = 2; u < K; ++u)
                if (((4 * m) >> u) & 1) o |= bitv[u];
            xx[m] = psi[b + o];
        }
    };

    // software pipeline: the next tile's loads are in flight while the
    // matrix cores work on the current one (tiles touch disjoint amplitudes)
    float2 xn[D / 4];
    uint64_t base_n = 0;
    if (t0 < t_end) load_tile(t0, xn, base_n);
    for (uint64_t tile = t0; tile < t_end; tile += step) {
        float2 x[D / 4];
#pragma unroll
        for (int m = 0; m < D / 4; ++m) x[m] = xn[m];
        const uint64_t base = base_n;
        if (tile + step < t_end) load_tile(tile + step, xn, base_n);
        f4 acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int sq = 0; sq < KQ; ++sq) {
            f4 av[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) av[rb] = As[(rb * KQ + sq) * 64 + lane];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int s = 4 * sq + s4;
                const float b = (s & 1) ? x[s >> 1].y : x[s >> 1].x;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rb][s4], b, acc[rb], 0, 0, 0);
            }
            // keep the next group's LDS operand reads from being hoisted:
            // with k = 6 hoisting all of them exceeds the register file
            if (K == 6) __builtin_amdgcn_sched_barrier(0);
        }
        uint32_t fb = 0;
        if (FOLD) fb = fold_index(a, base + a.idx_offset);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int pr = 0; pr < 2; ++pr) {
                // amplitude r = 8 rb + 2 h + pr: bit 0 = pr, bits 1-2 = h, bits 3.. = rb
                uint64_t o = pr ? bitv[0] : 0ull;
                o |= (h & 1) ? bitv[1] : 0ull;
                o |= (h & 2) ? bitv[2] : 0ull;
#pragma unroll
                for (int t = 3; t < K; ++t)
                    if ((rb >> (t - 3)) & 1) o |= bitv[t];
                float re = acc[rb][2 * pr], im = acc[rb][2 * pr + 1];
                if (FOLD) {
                    const float2 ph = ((const float2*)a.ftab)[fb | fold_index(a, o)];
                    const float tr = re * ph.x - im * ph.y;
                    im = re * ph.y + im * ph.x;
                    re = tr;
                }
                psi[base + o] = float2{re, im};
            }
        }
    }
}

}  // namespace sv
