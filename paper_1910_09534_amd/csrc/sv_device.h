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
//
// psi and mat are separate restrict parameters: the matrix must be known not
// to alias the amplitudes, or its rows cannot stay in scalar loads across the
// stores of earlier rows.
template <typename R, int K, bool FOLD, typename PT, typename MT>
__device__ __forceinline__ void dense_group(PT __restrict__ psi, MT __restrict__ mat, const Sweep& a,
                                            uint64_t g)
{
    using V = typename Vec2<R>::T;
    constexpr int D = 1 << K;
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
// y = M x for sixteen groups at once, as three real D x D products (D = 2^k)
// on a D x 16 block whose columns are the groups (the 3-multiplication form
// of a complex product):
//     P1 = Mr Xr,  P2 = Mi Xi,  P3 = (Mr + Mi)(Xr + Xi),
//     Yr = P1 - P2,  Yi = P3 - P1 - P2.
// Operand layouts (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; its 4 results are D[4 (l / 16) + v][l % 16].  So lane
// l = j + 16 h works on group j: at k-step s it supplies amplitude 4 s + h,
// and it ends with amplitudes 16 rb + 4 h + v (v = 0..3) of row block rb.
// The three real matrices are staged once per workgroup in LDS in operand
// order: one ds_read_b128 gives a lane its A operands for four k-steps.
//
// Loads and stores: direct (each lane reads its own amplitudes; 16 lanes
// cover 16 consecutive groups) or, when target bits sit among the lowest
// four positions, staged through LDS in address order: the tile's 16 D
// amplitudes are read as 64-lane runs of ascending addresses, parked in a
// per-wave LDS block (row = amplitude index within the group, column =
// group, one column of padding), and then read in operand order.
// ---------------------------------------------------------------------------
template <int K>
struct MfmaShape {
    static constexpr int D = 1 << K;
    static constexpr int RB = D / 16;            // 16-row blocks per product
    static constexpr int KS = D / 4;             // k-steps
    static constexpr int KQ = KS / 4;            // groups of four k-steps
    static constexpr int NA = 3 * RB * KQ * 256; // floats of the three matrices
    static constexpr int XS = D * 17;            // float2 per wave for staging
};

template <int K>
__device__ __forceinline__ void mfma_stage_matrix(f4* As, const float2* __restrict__ mat)
{
    using S = MfmaShape<K>;
    for (int i = threadIdx.x; i < S::NA; i += blockDim.x) {
        const int s4 = i & 3, l = (i >> 2) & 63, blk = i >> 8;
        const int sq = blk % S::KQ, rb = (blk / S::KQ) % S::RB, p = blk / (S::KQ * S::RB);
        const int R = 16 * rb + (l & 15);
        const int C = 4 * (4 * sq + s4) + (l >> 4);
        const float2 m = mat[R * S::D + C];
        ((float*)As)[i] = p == 0 ? m.x : (p == 1 ? m.y : m.x + m.y);
    }
}

// Tiles [t0, t_end) with stride `step` of one sweep, for the calling wave.
// Xs: this wave's staging block (STAGED only).
template <int K, bool FOLD, bool STAGED>
__device__ __forceinline__ void mfma_tiles(const Sweep& a, const f4* As, float2* Xs, uint64_t t0,
                                           uint64_t step, uint64_t t_end)
{
    using S = MfmaShape<K>;
    constexpr int D = S::D, RB = S::RB, KQ = S::KQ, NE = D / 4;
    float2* __restrict__ psi = (float2*)a.psi;
    const int lane = threadIdx.x & 63;
    const int j = lane & 15, h = lane >> 4;
    uint64_t bitv[K];
#pragma unroll
    for (int t = 0; t < K; ++t) bitv[t] = 1ull << a.tpos[t];

    // staged: this lane's part of the address / LDS slot of element 64 i + lane
    uint64_t addr_lane = 0;
    int slot_lane = 0;
    if (STAGED) {
#pragma unroll
        for (int b = 0; b < 6; ++b)
            if ((lane >> b) & 1) {
                addr_lane |= a.st_addr_bit[b];
                slot_lane += a.st_slot_bit[b];
            }
    }

    auto load_tile = [&](uint64_t t, float2* xx) {
        if (STAGED) {
            const uint64_t b0 = group_base<K>(a, t * 16);
#pragma unroll
            for (int i = 0; i < NE; ++i) xx[i] = psi[b0 + addr_lane + a.st_addr_i[i]];
        } else {
            const uint64_t b = group_base<K>(a, t * 16 + j);
#pragma unroll
            for (int m = 0; m < NE; ++m) {
                uint64_t o = (h & 1) ? bitv[0] : 0ull;
                o |= (h & 2) ? bitv[1] : 0ull;
#pragma unroll
                for (int u = 2; u < K; ++u)
                    if ((m >> (u - 2)) & 1) o |= bitv[u];
                xx[m] = psi[b + o];
            }
        }
    };

    // software pipeline: the next tile's loads are in flight while the
    // matrix cores work on the current one (tiles touch disjoint amplitudes)
    float2 xn[NE];
    if (t0 < t_end) load_tile(t0, xn);
    for (uint64_t tile = t0; tile < t_end; tile += step) {
        float2 x[NE];
        if (STAGED) {
#pragma unroll
            for (int i = 0; i < NE; ++i) Xs[slot_lane + a.st_slot_i[i]] = xn[i];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int s = 0; s < NE; ++s) x[s] = Xs[(4 * s + h) * 17 + j];
        } else {
#pragma unroll
            for (int s = 0; s < NE; ++s) x[s] = xn[s];
        }
        if (tile + step < t_end) load_tile(tile + step, xn);
        f4 acc[3][RB];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[p][rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int sq = 0; sq < KQ; ++sq) {
            f4 av[3][RB];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) av[p][rb] = As[((p * RB + rb) * KQ + sq) * 64 + lane];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const float2 xv = x[4 * sq + s4];
                const float bs = xv.x + xv.y;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc[0][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0][rb][s4], xv.x, acc[0][rb], 0, 0, 0);
                    acc[1][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1][rb][s4], xv.y, acc[1][rb], 0, 0, 0);
                    acc[2][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2][rb][s4], bs, acc[2][rb], 0, 0, 0);
                }
            }
            // keep later LDS operand reads from being hoisted: with k = 6
            // hoisting all of them exceeds the register file
            if (K == 6) __builtin_amdgcn_sched_barrier(0);
        }
        const uint64_t base = group_base<K>(a, tile * 16 + j);
        uint32_t fb = 0;
        if (FOLD) fb = fold_index(a, base + a.idx_offset);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // amplitude r = 16 rb + 4 h + v: bits 0-1 = v, bits 2-3 = h, bits 4.. = rb
                uint64_t o = (v & 1) ? bitv[0] : 0ull;
                o |= (v & 2) ? bitv[1] : 0ull;
                o |= (h & 1) ? bitv[2] : 0ull;
                o |= (h & 2) ? bitv[3] : 0ull;
#pragma unroll
                for (int t = 4; t < K; ++t)
                    if ((rb >> (t - 4)) & 1) o |= bitv[t];
                const float p1 = acc[0][rb][v], p2 = acc[1][rb][v], p3 = acc[2][rb][v];
                float re = p1 - p2, im = p3 - p1 - p2;
                if (FOLD) {
                    const float2 ph = ((const float2*)a.ftab)[fb | fold_index(a, o)];
                    const float tr = re * ph.x - im * ph.y;
                    im = re * ph.y + im * ph.x;
                    re = tr;
                }
                if (STAGED) Xs[(16 * rb + 4 * h + v) * 17 + j] = float2{re, im};
                else psi[base + o] = float2{re, im};
            }
        }
        if (STAGED) {
            __builtin_amdgcn_wave_barrier();
            const uint64_t b0 = group_base<K>(a, tile * 16);
#pragma unroll
            for (int i = 0; i < NE; ++i) psi[b0 + addr_lane + a.st_addr_i[i]] = Xs[slot_lane + a.st_slot_i[i]];
            __builtin_amdgcn_wave_barrier();
        }
    }
}

}  // namespace sv
