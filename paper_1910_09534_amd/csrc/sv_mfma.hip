// Fused dense sweep on the matrix cores (complex64, k = 4..6).
//
// A 2^k x 2^k complex block y = M x is the real product
//     [yr; yi] = [[Mr, -Mi], [Mi, Mr]] [xr; xi]
// of a (2D x 2D) matrix A (D = 2^k) with one 2D-vector per group.  Sixteen
// groups form the 16 columns of the B operand of v_mfma_f32_16x16x4f32, so
// one wave computes A (2D x 2D) times B (2D x 16) with (2D/16) x (2D/4)
// MFMAs and FP32 accumulation.
//
// Operand layouts of v_mfma_f32_16x16x4f32 (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; the 4 results of lane l are
// D[4 (l / 16) + v][l % 16], v = 0..3.  Hence lane l = j + 16 h works on
// group j of the tile:
//   * K index of k-step s for lane h is (amplitude c = 4 (s >> 1) + h,
//     part s & 1): each lane loads the D/4 complete amplitudes c = 4 m + h
//     of its group (8-byte loads) and feeds re / im on alternate k-steps;
//   * output row R = 16 rb + 4 h + v is (amplitude R >> 1, part R & 1): each
//     lane ends with complete (re, im) pairs of amplitudes 8 rb + 2 h + {0,1}.
// A is staged once per workgroup in LDS, pre-arranged so that one
// ds_read_b128 gives a lane its operands for four consecutive k-steps.
#include "sv_internal.h"

namespace sv {

typedef float f4 __attribute__((ext_vector_type(4)));

struct MfmaK {
    uint64_t tiles;             // groups / 16
    uint64_t idx_offset;
    uint64_t lowmask[kMaxDense];
    int tpos[kMaxDense];
    int fold_m;
    int fold_pos[kMaxDiag];
};

template <int K, bool FOLD>
__global__ __launch_bounds__(256) void k_dense_mfma(float2* __restrict__ psi,
                                                                   const float2* __restrict__ mat,
                                                                   const float2* __restrict__ ftab,
                                                                   MfmaK a)
{
    constexpr int D = 1 << K;
    constexpr int RB = 2 * D / 16;      // 16-row blocks of A
    constexpr int KQ = 2 * D / 16;      // groups of four k-steps
    constexpr int NA = RB * KQ * 256;   // floats of A
    __shared__ f4 As[NA / 4];

    // A in operand order: As[(rb * KQ + sq) * 64 + l][s4] = A[16 rb + l % 16][k-step 4 sq + s4, lane l / 16]
    for (int i = threadIdx.x; i < NA; i += blockDim.x) {
        const int s4 = i & 3, l = (i >> 2) & 63, blk = i >> 8;
        const int sq = blk % KQ, rb = blk / KQ;
        const int s = 4 * sq + s4;
        const int R = 16 * rb + (l & 15);
        const int c = 4 * (s >> 1) + (l >> 4), p = s & 1;
        const int r = R >> 1, q = R & 1;
        const float2 m = mat[r * D + c];
        const float v = (q == 0) ? (p == 0 ? m.x : -m.y) : (p == 0 ? m.y : m.x);
        ((float*)As)[i] = v;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int j = lane & 15, h = lane >> 4;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    uint64_t bitv[K];
#pragma unroll
    for (int t = 0; t < K; ++t) bitv[t] = 1ull << a.tpos[t];

    // group base and amplitudes of tile t (lane: group j, amplitudes 4 m + h)
    auto load_tile = [&](uint64_t t, float2* xx, uint64_t& b) {
        b = t * 16 + j;
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const uint64_t low = b & a.lowmask[u];
            b = ((b ^ low) << 1) | low;
        }
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
    if (wave < a.tiles) load_tile(wave, xn, base_n);
    for (uint64_t tile = wave; tile < a.tiles; tile += nwaves) {
        float2 x[D / 4];
#pragma unroll
        for (int m = 0; m < D / 4; ++m) x[m] = xn[m];
        const uint64_t base = base_n;
        if (tile + nwaves < a.tiles) load_tile(tile + nwaves, xn, base_n);
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
            // keep the next group's LDS operand reads from being hoisted here:
            // with k = 6 hoisting all of them exceeds the register file
            if (K == 6) __builtin_amdgcn_sched_barrier(0);
        }
        uint32_t fb = 0;
        if (FOLD) {
            const uint64_t gi = base + a.idx_offset;
            for (int t = 0; t < a.fold_m; ++t) fb |= (uint32_t)((gi >> a.fold_pos[t]) & 1u) << t;
        }
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
                    uint32_t fr = 0;
                    for (int t = 0; t < a.fold_m; ++t) fr |= (uint32_t)((o >> a.fold_pos[t]) & 1u) << t;
                    const float2 ph = ftab[fb | fr];
                    const float tr = re * ph.x - im * ph.y;
                    im = re * ph.y + im * ph.x;
                    re = tr;
                }
                psi[base + o] = float2{re, im};
            }
        }
    }
}

template <int K>
static hipError_t mfma_dispatch(hipStream_t st, void* psi, const void* mat, const void* ftab,
                                const MfmaK& a, bool fold)
{
    const int block = 256;
    const uint64_t waves = a.tiles;
    uint64_t g = (waves + block / 64 - 1) / (block / 64);
    const uint64_t cap = 256 * (K == 6 ? 2 : 6);
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    if (fold)
        hipLaunchKernelGGL((k_dense_mfma<K, true>), dim3((unsigned)g), dim3(block), 0, st, (float2*)psi,
                           (const float2*)mat, (const float2*)ftab, a);
    else
        hipLaunchKernelGGL((k_dense_mfma<K, false>), dim3((unsigned)g), dim3(block), 0, st, (float2*)psi,
                           (const float2*)mat, (const float2*)ftab, a);
    return hipGetLastError();
}

hipError_t launch_dense_mfma(hipStream_t st, void* psi, int nloc, int k, const int* pos, const void* mat,
                             const DiagSpec* fold, uint64_t idx_offset)
{
    if (k < 4 || k > 6 || nloc < k + 4) return hipErrorInvalidValue;
    MfmaK a{};
    a.tiles = 1ull << (nloc - k - 4);
    a.idx_offset = idx_offset;
    int sp[kMaxDense];
    for (int j = 0; j < k; ++j) sp[j] = pos[j];
    for (int j = 1; j < k; ++j)
        for (int l = j; l > 0 && sp[l - 1] > sp[l]; --l) {
            const int t = sp[l]; sp[l] = sp[l - 1]; sp[l - 1] = t;
        }
    for (int j = 0; j < k; ++j) a.lowmask[j] = (1ull << sp[j]) - 1;
    for (int j = 0; j < k; ++j) a.tpos[j] = pos[j];
    const bool do_fold = fold && fold->m > 0;
    if (do_fold) {
        a.fold_m = fold->m;
        for (int j = 0; j < fold->m; ++j) a.fold_pos[j] = fold->pos[j];
    }
    const void* ft = do_fold ? fold->table : nullptr;
    switch (k) {
        case 4: return mfma_dispatch<4>(st, psi, mat, ft, a, do_fold);
        case 5: return mfma_dispatch<5>(st, psi, mat, ft, a, do_fold);
        case 6: return mfma_dispatch<6>(st, psi, mat, ft, a, do_fold);
    }
    return hipErrorInvalidValue;
}

}  // namespace sv
