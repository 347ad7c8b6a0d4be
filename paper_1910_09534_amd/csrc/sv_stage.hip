// Staged sweep: several dense blocks applied in one pass over HBM.  The
// appendix uses cache blocking to form the 5-qubit aggregate gates
// themselves (each "cache" line of its listing is one aggregate); here a
// second level of blocking applies a run of aggregates to an LDS-resident
// tile, so the run costs one HBM round trip instead of one per aggregate.
//
// A stage is a run of consecutive dense blocks (k = 4 or 5, complex64) whose
// target positions, together with positions 0..3, fit in t <= 13 tile
// positions P[0] < ... < P[t-1] (P[0..3] = 0..3; free low positions widen
// the tile to 13 when the LDS budget allows).  A tile is the 2^t amplitudes whose other bits equal the
// tile id.  A persistent workgroup (256 lanes) loops over tiles:
//   1. the next tile's loads are issued (into registers; each lane holds
//      pairs of adjacent amplitudes, 16 bytes per access: position 0 is
//      always a tile position);
//   2. each block runs on the LDS tile: pairs of 16-group units per wave
//      through the three real products of the matrix-core form
//      (v_mfma_f32_16x16x4f32, same operand layout as the single sweep),
//      reading and writing LDS, with a workgroup barrier between blocks;
//   3. the tile is written back, then the next tile is parked in LDS.
// The next tile's loads precede this tile's stores, so parking never waits
// for stores.  Re M and Im M of every block are staged in LDS once per
// workgroup.  Every workgroup runs the same number of tile iterations, so
// the barriers are reached uniformly.
#include <atomic>
#include <cmath>

#include "sv_device.h"

#include <type_traits>

namespace sv {

constexpr int kStageMaxOps = 8;
constexpr int kStageMaxT = 14;
constexpr int kStageMaxLds = 80 * 1024;     // tiles of up to 13 positions: two 256-lane workgroups per CU
constexpr int kStageMaxLds14 = 160 * 1024;  // 14 positions: one workgroup per CU

// LDS a tile of t positions may use, and its workgroup size
static inline int stage_lds_limit_t(int t) { return t >= 14 ? kStageMaxLds14 : kStageMaxLds; }
// lanes of a complex64 staged-pass workgroup: 256 for tiles of up to 13
// positions; 14 positions take the whole LDS, one workgroup per CU, of 1024
// lanes in the split form (four waves per SIMD to hide each tile's LDS and
// barrier latency; the kernel fits 128 VGPRs with one 5-qubit or two
// 4-qubit units per wave at a time) and 512 in the fp32 form (its 3M units
// need more registers)
static inline int stage_threads(int t, bool split) { return t >= 14 ? (split ? 1024 : 512) : 256; }

struct StageK {
    uint64_t tiles;                          // 2^(nloc - t)
    // tile id bits go, in ascending order, to the set bits of tmask (the
    // positions outside the tile that can be non-zero); consecutive tiles of
    // a workgroup are gridDim.x apart, their bases tstep = that stride
    // spread onto tmask apart (added in the masked number system)
    uint64_t tmask;
    uint64_t tstep;
    // amplitudes on tile positions no earlier operation has reached are
    // zero but their memory may hold older values: tile-local index bits
    // (bit b = position P[b]) of such elements, parked in LDS as zeros
    uint32_t newmask_t;
    uint64_t dep_lane[10];                   // global offset of lane bit b (8 lane bits; 9 or 10 at t = 14)
    uint64_t dep_i[32];                      // global offset of the pair (element) index bits above the lane bits
    int t;
    int nops;
    int from_e0;                             // 1: input is |0...0>, not read
    double* norm_out;                        // non-null: per-workgroup FP64 sum of |psi|^2 of the result
    float split_scale, split_unscale;        // split form: the tile's scale in LDS (a power of two) and its inverse
    int op_k[kStageMaxOps];
    int op_bits[kStageMaxOps][kMaxDense];    // tile-local bit of matrix bit j
    int op_lowmask_bits[kStageMaxOps][kMaxDense];  // the same bits, ascending
    int op_aoff[kStageMaxOps];               // float offset of the op's operand matrices in LDS
    const float2* op_mat[kStageMaxOps];      // row-major complex matrices (device)
};

// tile-local index -> LDS slot (one pad element per 16)
__device__ __forceinline__ int lslot(int i) { return i + (i >> 4); }

// Group index -> tile-local index: zero bits inserted at the block's target
// bits (low[u] = (1 << target_u) - 1, ascending).  The map acts bit by bit,
// so spread(a | b) = spread(a) | spread(b) for disjoint a, b; likewise
// lslot(a | b) = lslot(a) + lslot(b), which splits every LDS address into a
// wave-uniform part (the unit) and per-lane constants of the block.
template <int K>
__device__ __forceinline__ int spread(int g, const int (&low)[K])
{
#pragma unroll
    for (int u = 0; u < K; ++u) {
        const int lw = g & low[u];
        g = ((g ^ lw) << 1) | lw;
    }
    return g;
}

// NU (1 or 2) 16-group units of one block on the LDS tile, processed together
// by the calling wave: their loads are issued together and their 6 NU
// accumulator chains interleave on the matrix core.  The LDS slot of operand
// element m (matrix column 4 m + h) of unit q is su[q] + sx[m] + cx and that
// of result r = 16 rb + 4 h + v is su[q] + sy[4 rb + v] + cy: su, sx, sy are
// wave-uniform, cx, cy per lane.
template <int K, int NU>
__device__ __forceinline__ void stage_units(const f4 (&av)[3][MfmaShape<K>::RB][MfmaShape<K>::KQ],
                                            const int (&sx)[MfmaShape<K>::D / 4],
                                            const int (&sy)[MfmaShape<K>::D / 4], int cx, int cy,
                                            const int (&su)[2], float2* __restrict__ T)
{
    using S = MfmaShape<K>;
    constexpr int RB = S::RB, KQ = S::KQ, NE = S::D / 4;
    float2 x[NU][NE];
#pragma unroll
    for (int m = 0; m < NE; ++m)
#pragma unroll
        for (int q = 0; q < NU; ++q) x[q][m] = T[(su[q] + sx[m]) + cx];
    f4 acc[NU][3][RB];
#pragma unroll
    for (int q = 0; q < NU; ++q)
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[q][p][rb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int sq = 0; sq < KQ; ++sq) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
            for (int q = 0; q < NU; ++q) {
                const float2 xv = x[q][4 * sq + s4];
                const float bs = xv.x + xv.y;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc[q][0][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[0][rb][sq][s4], xv.x, acc[q][0][rb], 0, 0, 0);
                    acc[q][1][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[1][rb][sq][s4], xv.y, acc[q][1][rb], 0, 0, 0);
                    acc[q][2][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[2][rb][sq][s4], bs, acc[q][2][rb], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int q = 0; q < NU; ++q) {
                const float p1 = acc[q][0][rb][v], p2 = acc[q][1][rb][v], p3 = acc[q][2][rb][v];
                T[(su[q] + sy[4 * rb + v]) + cy] = float2{p1 - p2, p3 - p1 - p2};
            }
}

template <int K, int NT>
__device__ __forceinline__ void stage_block(const StageK& a, int o, const f4* __restrict__ As,
                                            float2* __restrict__ T, int wave)
{
    using S = MfmaShape<K>;
    constexpr int RB = S::RB, KQ = S::KQ, NE = S::D / 4;
    const int lane = threadIdx.x & 63;
    constexpr int nw = NT / 64;
    const int j = lane & 15, h = lane >> 4;
    int bit[K], low[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        bit[u] = 1 << a.op_bits[o][u];
        low[u] = (1 << a.op_lowmask_bits[o][u]) - 1;
    }
    // this wave's operand fragments of Re M and Im M, read from LDS once per
    // block and tile; the third operand Re M + Im M is formed here
    f4 av[3][RB][KQ];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int sq = 0; sq < KQ; ++sq) av[p][rb][sq] = As[((p * RB + rb) * KQ + sq) * 64 + lane];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int sq = 0; sq < KQ; ++sq) av[2][rb][sq] = av[0][rb][sq] + av[1][rb][sq];
    // slot offsets: per lane, the unit's group j with the lane's h bits (h
    // selects matrix bits 0, 1 of an operand and bits 2, 3 of a result);
    // uniform, the remaining matrix bits of element m / result (rb, v)
    const int lj = lslot(spread<K>(j, low));
    const int cx = lj + lslot(((h & 1) ? bit[0] : 0) | ((h & 2) ? bit[1] : 0));
    const int cy = lj + lslot(((h & 1) ? bit[2] : 0) | ((h & 2) ? bit[3] : 0));
    int sx[NE], sy[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        int off = 0;
#pragma unroll
        for (int u = 2; u < K; ++u)
            if ((m >> (u - 2)) & 1) off |= bit[u];
        sx[m] = lslot(off);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int off = (v & 1) ? bit[0] : 0;
            off |= (v & 2) ? bit[1] : 0;
#pragma unroll
            for (int u = 4; u < K; ++u)
                if ((rb >> (u - 4)) & 1) off |= bit[u];
            sy[4 * rb + v] = lslot(off);
        }
    // units wave, wave + nw, ... in pairs (the wave's trip count is uniform)
    const int units = 1 << (a.t - K - 4);
    for (int unit = wave; unit < units; unit += 2 * nw) {
        const int su[2] = {lslot(spread<K>(unit * 16, low)), lslot(spread<K>((unit + nw) * 16, low))};
        if (unit + nw < units) stage_units<K, 2>(av, sx, sy, cx, cy, su, T);
        else stage_units<K, 1>(av, sx, sy, cx, cy, su, T);
    }
}

// ---- split-fp16 form -------------------------------------------------------
// Every real product of the block runs on the fp16 matrix cores with single-
// precision accuracy: each fp32 operand x is split into x_hi = f16(x) and
// x_lo = f16(x - x_hi) (both rounded to nearest), so x_hi + x_lo carries 22
// significant bits, and A x = A_hi x_hi + A_hi x_lo + A_lo x_hi up to a term
// of relative size 2^-22; the fp16 products are exact and accumulate in fp32
// (the split-precision scheme of Markidis et al. 2018 and Ootomo & Yokota
// 2022, without their rescaling of the low parts: the tile is parked in LDS
// scaled by a power of two chosen from a bound on the state's norm, so that
// every amplitude stays below 2^15 and typical ones lie far above the fp16
// subnormal range; the blocks are unitary, so their entries are at most 1).
// Complex products use four real ones: Re y = Ar xr - Ai xi and
// Im y = Ai xr + Ar xi.
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

// f16(a), f16(b) packed (low half a), rounded to nearest even
__device__ __forceinline__ uint32_t pk_hi(float a, float b)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// f16(a - hi.lo), f16(b - hi.hi) packed: each residual is formed exactly in
// fp32 inside the mixed-precision fma and rounded once to fp16
__device__ __forceinline__ uint32_t pk_lo(float a, float b, uint32_t hi)
{
    uint32_t r;
    asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %0, %1, -1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "=&v"(r)
        : "v"(hi), "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ h8 neg8(h8 v)
{
    return __builtin_bit_cast(h8, __builtin_bit_cast(u4, v) ^ 0x80008000u);
}

__device__ __forceinline__ f4 mma(h8 a, h8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Operand fragments of one block for the split form.  k = 5, per 16-row
// block rb: Ar_hi, Ar_lo, Ai_hi, Ai_lo, -Ai_hi, -Ai_lo, element e of lane
// (i, g) = matrix entry (16 rb + i, 4 e + g).  k = 4 (16 columns, so the
// real and imaginary columns share one 32-deep product): [Ar | -Ai] and
// [Ai | Ar], hi and lo, element e < 4 = entry (i, 4 e + g) of the first
// part, e >= 4 of the second.
template <int K>
struct SplitA;
template <>
struct SplitA<5> {
    h8 v[2][6];
};
template <>
struct SplitA<4> {
    h8 v[4];
};

// LDS image of a block's operands (what the kernel stages): k = 5: h8
// [(rb * 4 + p) * 64 + lane], p = Ar_hi, Ar_lo, Ai_hi, Ai_lo; k = 4: h4
// [p * 64 + lane].  Both take 8 bytes per matrix entry, as the fp32 form.
__device__ __forceinline__ void split_load(SplitA<5>& A, const void* As, int lane)
{
    const h8* a8 = (const h8*)As;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
        for (int p = 0; p < 4; ++p) A.v[rb][p] = a8[(rb * 4 + p) * 64 + lane];
        A.v[rb][4] = neg8(A.v[rb][2]);
        A.v[rb][5] = neg8(A.v[rb][3]);
    }
}

__device__ __forceinline__ void split_load(SplitA<4>& A, const void* As, int lane)
{
    const u2* a4 = (const u2*)As;
    const u2 rh = a4[0 * 64 + lane], rl = a4[1 * 64 + lane], ih = a4[2 * 64 + lane], il = a4[3 * 64 + lane];
    const uint32_t sg = 0x80008000u;
    A.v[0] = __builtin_bit_cast(h8, u4{rh.x, rh.y, ih.x ^ sg, ih.y ^ sg});
    A.v[1] = __builtin_bit_cast(h8, u4{rl.x, rl.y, il.x ^ sg, il.y ^ sg});
    A.v[2] = __builtin_bit_cast(h8, u4{ih.x, ih.y, rh.x, rh.y});
    A.v[3] = __builtin_bit_cast(h8, u4{il.x, il.y, rl.x, rl.y});
}

// NU units of a k = 5 block, split form (slots as in stage_units)
template <int NU>
__device__ __forceinline__ void split_units(const SplitA<5>& A, const int (&sx)[8], const int (&sy)[8], int cx,
                                            int cy, const int (&su)[NU], float2* __restrict__ T)
{
    float2 x[NU][8];
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int q = 0; q < NU; ++q) x[q][m] = T[(su[q] + sx[m]) + cx];
    h8 xrh[NU], xrl[NU], xih[NU], xil[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) {
        u4 rh, rl, ih, il;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float2 a = x[q][2 * w], b = x[q][2 * w + 1];
            rh[w] = pk_hi(a.x, b.x);
            ih[w] = pk_hi(a.y, b.y);
            rl[w] = pk_lo(a.x, b.x, rh[w]);
            il[w] = pk_lo(a.y, b.y, ih[w]);
        }
        xrh[q] = __builtin_bit_cast(h8, rh);
        xrl[q] = __builtin_bit_cast(h8, rl);
        xih[q] = __builtin_bit_cast(h8, ih);
        xil[q] = __builtin_bit_cast(h8, il);
    }
    f4 re[NU][2], im[NU][2];
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    // small terms first; 4 NU independent chains interleave
#pragma unroll
    for (int q = 0; q < NU; ++q)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            re[q][rb] = mma(A.v[rb][1], xrh[q], z);
            im[q][rb] = mma(A.v[rb][3], xrh[q], z);
        }
#pragma unroll
    for (int q = 0; q < NU; ++q)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            re[q][rb] = mma(A.v[rb][0], xrl[q], re[q][rb]);
            im[q][rb] = mma(A.v[rb][2], xrl[q], im[q][rb]);
        }
#pragma unroll
    for (int q = 0; q < NU; ++q)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            re[q][rb] = mma(A.v[rb][5], xih[q], re[q][rb]);
            im[q][rb] = mma(A.v[rb][1], xih[q], im[q][rb]);
        }
#pragma unroll
    for (int q = 0; q < NU; ++q)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            re[q][rb] = mma(A.v[rb][4], xil[q], re[q][rb]);
            im[q][rb] = mma(A.v[rb][0], xil[q], im[q][rb]);
        }
#pragma unroll
    for (int q = 0; q < NU; ++q)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            re[q][rb] = mma(A.v[rb][0], xrh[q], re[q][rb]);
            im[q][rb] = mma(A.v[rb][2], xrh[q], im[q][rb]);
        }
#pragma unroll
    for (int q = 0; q < NU; ++q)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            re[q][rb] = mma(A.v[rb][4], xih[q], re[q][rb]);
            im[q][rb] = mma(A.v[rb][0], xih[q], im[q][rb]);
        }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int q = 0; q < NU; ++q)
                T[(su[q] + sy[4 * rb + v]) + cy] = float2{re[q][rb][v], im[q][rb][v]};
}

// NU units of a k = 4 block, split form: operand element e < 4 is Re x of
// column 4 e + g, e >= 4 Im x of column 4 (e - 4) + g
template <int NU>
__device__ __forceinline__ void split_units(const SplitA<4>& A, const int (&sx)[4], const int (&sy)[4], int cx,
                                            int cy, const int (&su)[NU], float2* __restrict__ T)
{
    float2 x[NU][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < NU; ++q) x[q][m] = T[(su[q] + sx[m]) + cx];
    h8 xh[NU], xl[NU];
#pragma unroll
    for (int q = 0; q < NU; ++q) {
        u4 hh, ll;
        hh[0] = pk_hi(x[q][0].x, x[q][1].x);
        hh[1] = pk_hi(x[q][2].x, x[q][3].x);
        hh[2] = pk_hi(x[q][0].y, x[q][1].y);
        hh[3] = pk_hi(x[q][2].y, x[q][3].y);
        ll[0] = pk_lo(x[q][0].x, x[q][1].x, hh[0]);
        ll[1] = pk_lo(x[q][2].x, x[q][3].x, hh[1]);
        ll[2] = pk_lo(x[q][0].y, x[q][1].y, hh[2]);
        ll[3] = pk_lo(x[q][2].y, x[q][3].y, hh[3]);
        xh[q] = __builtin_bit_cast(h8, hh);
        xl[q] = __builtin_bit_cast(h8, ll);
    }
    f4 re[NU], im[NU];
    const f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NU; ++q) {
        re[q] = mma(A.v[1], xh[q], z);
        im[q] = mma(A.v[3], xh[q], z);
    }
#pragma unroll
    for (int q = 0; q < NU; ++q) {
        re[q] = mma(A.v[0], xl[q], re[q]);
        im[q] = mma(A.v[2], xl[q], im[q]);
    }
#pragma unroll
    for (int q = 0; q < NU; ++q) {
        re[q] = mma(A.v[0], xh[q], re[q]);
        im[q] = mma(A.v[2], xh[q], im[q]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int q = 0; q < NU; ++q) T[(su[q] + sy[v]) + cy] = float2{re[q][v], im[q][v]};
}

// one block on the LDS tile, split form (slot offsets as in stage_block)
template <int K, int NT>
__device__ __forceinline__ void split_block(const StageK& a, int o, const void* As, float2* __restrict__ T, int wave)
{
    constexpr int NE = (1 << K) / 4;
    const int lane = threadIdx.x & 63;
    constexpr int nw = NT / 64;
    const int j = lane & 15, h = lane >> 4;
    int bit[K], low[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        bit[u] = 1 << a.op_bits[o][u];
        low[u] = (1 << a.op_lowmask_bits[o][u]) - 1;
    }
    SplitA<K> A;
    split_load(A, As, lane);
    const int lj = lslot(spread<K>(j, low));
    const int cx = lj + lslot(((h & 1) ? bit[0] : 0) | ((h & 2) ? bit[1] : 0));
    const int cy = lj + lslot(((h & 1) ? bit[2] : 0) | ((h & 2) ? bit[3] : 0));
    int sx[NE], sy[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        int off = 0;
#pragma unroll
        for (int u = 2; u < K; ++u)
            if ((m >> (u - 2)) & 1) off |= bit[u];
        sx[m] = lslot(off);
    }
#pragma unroll
    for (int rb = 0; rb < NE / 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int off = (v & 1) ? bit[0] : 0;
            off |= (v & 2) ? bit[1] : 0;
#pragma unroll
            for (int u = 4; u < K; ++u)
                if ((rb >> (u - 4)) & 1) off |= bit[u];
            sy[4 * rb + v] = lslot(off);
        }
    // units wave, wave + nw, ... in groups of NG (4 for k = 4, whose units
    // are short, 2 for k = 5; half that with 1024 lanes, which must fit 128
    // VGPRs); units / nw is a power of two, so a wave runs whole groups or
    // fewer than NG units one by one
    constexpr int NG = NT >= 1024 ? (K == 4 ? 2 : 1) : (K == 4 ? 4 : 2);
    const int units = 1 << (a.t - K - 4);
    if (units >= NG * nw) {
        for (int unit = wave; unit < units; unit += NG * nw) {
            int su[NG];
#pragma unroll
            for (int q = 0; q < NG; ++q) su[q] = lslot(spread<K>((unit + q * nw) * 16, low));
            split_units<NG>(A, sx, sy, cx, cy, su, T);
        }
    } else {
        for (int unit = wave; unit < units; unit += nw) {
            const int su[1] = {lslot(spread<K>(unit * 16, low))};
            split_units<1>(A, sx, sy, cx, cy, su, T);
        }
    }
}

// TW: tile width t (9..14), PER = 2^t / lanes elements per lane.  WIDE: the
// lane part of an element's address needs more than 32 bits of byte offset
// (otherwise element addresses are a wave-uniform 64-bit base plus a 32-bit
// per-lane offset, so loads and stores take the scalar-base form).
// bits of x, in ascending order, onto the set bits of m (host and device)
__host__ __device__ inline uint64_t spread_bits(uint64_t x, uint64_t m)
{
    uint64_t r = 0;
    while (m && x) {
        const uint64_t low = m & (~m + 1);
        if (x & 1) r |= low;
        x >>= 1;
        m &= m - 1;
    }
    return r;
}

template <int TW, bool WIDE, bool ZERO, bool SPLIT>
__global__ __launch_bounds__(TW >= 14 ? (SPLIT ? 1024 : 512) : 256) void k_stage(float2* __restrict__ psi, StageK a)
{
    // lanes NT (2^LB), PER amplitudes per lane in PER / 2 adjacent pairs
    constexpr int NT = TW >= 14 ? (SPLIT ? 1024 : 512) : 256, LB = TW >= 14 ? (SPLIT ? 10 : 9) : 8;
    constexpr int PER = 1 << (TW - LB);
    extern __shared__ f4 smem[];
    float2* T = (float2*)smem;                                   // tile, padded
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    f4* Abase = smem + ((lslot(1 << TW) * 8 + 15) / 16);          // operand matrices
    // stage every block's operand matrices in operand order
    for (int o = 0; o < a.nops && SPLIT; ++o) {
        const int k = a.op_k[o];
        const float2* mat = a.op_mat[o];
        _Float16* dst = (_Float16*)((float*)Abase + a.op_aoff[o]);
        const int D = 1 << k, NA = 4 * D * D;
        for (int i = threadIdx.x; i < NA; i += NT) {
            int e, l, p, R;
            if (k == 5) {
                e = i & 7, l = (i >> 3) & 63, p = (i >> 9) & 3;
                R = 16 * (i >> 11) + (l & 15);
            } else {
                e = i & 3, l = (i >> 2) & 63, p = i >> 8;
                R = l & 15;
            }
            const float2 m = mat[R * D + 4 * e + (l >> 4)];
            const float v = p < 2 ? m.x : m.y;
            const _Float16 hv = (_Float16)v;
            dst[i] = (p & 1) ? (_Float16)(v - (float)hv) : hv;
        }
    }
    for (int o = 0; o < a.nops && !SPLIT; ++o) {
        const int k = a.op_k[o];
        const int D = 1 << k, RB = D / 16, KQ = D / 16, NA = 2 * RB * KQ * 256;
        float* dst = (float*)(Abase) + a.op_aoff[o];
        const float2* mat = a.op_mat[o];
        for (int i = threadIdx.x; i < NA; i += NT) {
            const int s4 = i & 3, l = (i >> 2) & 63, blk = i >> 8;
            const int sq = blk % KQ, rb = (blk / KQ) % RB, p = blk / (KQ * RB);
            const int R = 16 * rb + (l & 15);
            const int C = 4 * (4 * sq + s4) + (l >> 4);
            const float2 m = mat[R * D + C];
            dst[i] = p == 0 ? m.x : m.y;
        }
    }
    // element pair m of lane l: tile-local indices (l << 1) + 2 NT m + {0, 1}
    // (tile bit 0 is position 0: the pair is two adjacent amplitudes, one
    // 16-byte access); their LDS slots are lslot(2 l) + ES2 m + {0, 1}
    constexpr int PP = PER / 2, ES2 = 2 * NT + (2 * NT) / 16;
    uint64_t dl = 0;
    for (int b = 0; b < LB; ++b)
        if ((threadIdx.x >> b) & 1) dl |= a.dep_lane[b];
    const uint32_t dlb = (uint32_t)(dl * sizeof(float2));       // used when !WIDE
    auto elem = [&](uint64_t tb, int m) -> float4* {
        if (WIDE) return (float4*)(psi + (tb + dl + a.dep_i[m]));
        return (float4*)((char*)(psi + (tb + a.dep_i[m])) + dlb);
    };
    const int ls = lslot(2 * threadIdx.x);
    float4 xr[PP];
    auto load_tile = [&](uint64_t tile, uint64_t tb) {
        if (a.from_e0) {
#pragma unroll
            for (int m = 0; m < PP; ++m) xr[m] = float4{0.f, 0.f, 0.f, 0.f};
            if (tile == 0 && threadIdx.x == 0) xr[0].x = 1.f;
        } else {
#pragma unroll
            for (int m = 0; m < PP; ++m) {
                const f4 v = __builtin_nontemporal_load((const f4*)elem(tb, m));
                xr[m] = float4{v.x, v.y, v.z, v.w};
            }
        }
    };
    // pair m as parked: with ZERO, elements on positions no operation has
    // reached are zero (memory there may hold older values)
    auto parked = [&](int m, float2& e0, float2& e1) {
        e0 = float2{xr[m].x, xr[m].y};
        e1 = float2{xr[m].z, xr[m].w};
        if (SPLIT) {
            e0.x *= a.split_scale, e0.y *= a.split_scale;
            e1.x *= a.split_scale, e1.y *= a.split_scale;
        }
        if (ZERO) {
            const uint32_t pi = (uint32_t)((threadIdx.x << 1) + 2 * NT * m);
            if (pi & a.newmask_t) e0 = float2{0.f, 0.f};
            if ((pi | 1u) & a.newmask_t) e1 = float2{0.f, 0.f};
        }
    };
    auto park = [&]() {
#pragma unroll
        for (int m = 0; m < PP; ++m) {
            float2 e0, e1;
            parked(m, e0, e1);
            T[ls + ES2 * m] = e0;
            T[ls + ES2 * m + 1] = e1;
        }
    };
    double nacc = 0.0;                                           // this lane's sum of |psi|^2
    uint64_t tile = blockIdx.x;
    uint64_t tb = spread_bits(tile, a.tmask);
    if (tile < a.tiles) {
        load_tile(tile, tb);
        park();
    }
    __syncthreads();
    // Per tile: issue the next tile's loads, run the blocks on the LDS tile,
    // then store it while parking the next tile in its place.
    // The state streams through once per pass: its loads and stores are
    // non-temporal, and the waves raise their issue priority while they
    // issue them, so that the memory requests of one workgroup go out ahead
    // of the matrix-core work of the other on the same CU.
    for (; tile < a.tiles; tile += gridDim.x) {
        const uint64_t nt = tile + gridDim.x;
        const uint64_t nb = ((tb | ~a.tmask) + a.tstep) & a.tmask;
        const bool next = nt < a.tiles;
        __builtin_amdgcn_s_setprio(1);
        if (next) load_tile(nt, nb);
        __builtin_amdgcn_s_setprio(0);
        for (int o = 0; o < a.nops; ++o) {
            const f4* As = (const f4*)((const float*)Abase + a.op_aoff[o]);
            if (SPLIT) {
                if (a.op_k[o] == 5) split_block<5, NT>(a, o, As, T, wave);
                else split_block<4, NT>(a, o, As, T, wave);
            } else {
                if (a.op_k[o] == 5) stage_block<5, NT>(a, o, As, T, wave);
                else stage_block<4, NT>(a, o, As, T, wave);
            }
            __syncthreads();
        }
        // Each lane parks the next tile's pairs in the very slots it has just
        // read for its stores (no other lane touches them), pair by pair, so
        // the wait for a pair's load never covers the stores issued before it.
        __builtin_amdgcn_s_setprio(1);
        auto store_park = [&](auto park_next, auto sum_norm) {
#pragma unroll
            for (int m = 0; m < PP; ++m) {
                float2 v0 = T[ls + ES2 * m], v1 = T[ls + ES2 * m + 1];
                if (SPLIT) {
                    const float r = a.split_unscale;
                    v0.x *= r, v0.y *= r, v1.x *= r, v1.y *= r;
                }
                if constexpr (decltype(park_next)::value) {
                    float2 e0, e1;
                    parked(m, e0, e1);
                    T[ls + ES2 * m] = e0;
                    T[ls + ES2 * m + 1] = e1;
                }
                __builtin_nontemporal_store(f4{v0.x, v0.y, v1.x, v1.y}, (f4*)elem(tb, m));
                if constexpr (decltype(sum_norm)::value) {
                    nacc = fma((double)v0.x, (double)v0.x, nacc);
                    nacc = fma((double)v0.y, (double)v0.y, nacc);
                    nacc = fma((double)v1.x, (double)v1.x, nacc);
                    nacc = fma((double)v1.y, (double)v1.y, nacc);
                }
            }
        };
        using yes = std::true_type;
        using no = std::false_type;
        if (next) {
            if (a.norm_out) store_park(yes{}, yes{});
            else store_park(yes{}, no{});
        } else {
            if (a.norm_out) store_park(no{}, yes{});
            else store_park(no{}, no{});
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        tb = nb;
    }
    if (a.norm_out) {
        // fixed-order tree over the workgroup's lanes (the tile buffer is free)
        double* sh = (double*)smem;
        sh[threadIdx.x] = nacc;
        __syncthreads();
        for (int h = NT / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.norm_out[blockIdx.x] = sh[0];
    }
}


// ---- complex128 staged pass ---------------------------------------------------
// The FP64 form for complex128 states (Sec. 5 computes in double): the same
// tile scheme, with a tile of 2^t double-complex amplitudes taking twice the
// LDS of a complex64 one, so one 512-lane workgroup per CU holds the whole
// 160 KiB (a 13-position complex128 tile plus its blocks' matrices is the
// double of a 13-position complex64 tile plus its own).  Each lane moves one
// amplitude per 16-byte access (tile bits 0..8 are the lane, bits 9.. the
// element index), and every block's three real products (3M, as in the
// fp32 form) run on v_mfma_f64_16x16x4f64, whose operand layouts are those
// of v_mfma_f32_16x16x4f32 (its result rows are not: see stage64_block),
// one 16-group unit per wave at a time.
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double dd2 __attribute__((ext_vector_type(2)));

template <int K>
__device__ __forceinline__ void stage64_block(const StageK& a, int o, const d4* __restrict__ As,
                                              double2* __restrict__ T, int wave)
{
    using S = MfmaShape<K>;
    constexpr int RB = S::RB, KQ = S::KQ, NE = S::D / 4;
    constexpr int nw = 8;
    const int lane = threadIdx.x & 63;
    const int j = lane & 15, h = lane >> 4;
    int bit[K], low[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        bit[u] = 1 << a.op_bits[o][u];
        low[u] = (1 << a.op_lowmask_bits[o][u]) - 1;
    }
    // operands as in the fp32 form; results: v_mfma_f64_16x16x4f64 gives
    // item v of lane (j, h) row h + 4 v (the fp32 instruction 4 h + v), so
    // h selects result bits 0, 1 and v bits 2, 3
    const int lj = lslot(spread<K>(j, low));
    const int cx = lj + lslot(((h & 1) ? bit[0] : 0) | ((h & 2) ? bit[1] : 0));
    const int cy = cx;
    int sx[NE], sy[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        int off = 0;
#pragma unroll
        for (int u = 2; u < K; ++u)
            if ((m >> (u - 2)) & 1) off |= bit[u];
        sx[m] = lslot(off);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int off = (v & 1) ? bit[2] : 0;
            off |= (v & 2) ? bit[3] : 0;
#pragma unroll
            for (int u = 4; u < K; ++u)
                if ((rb >> (u - 4)) & 1) off |= bit[u];
            sy[4 * rb + v] = lslot(off);
        }
    const int units = 1 << (a.t - K - 4);
    for (int unit = wave; unit < units; unit += nw) {
        const int su = lslot(spread<K>(unit * 16, low));
        double2 x[NE];
#pragma unroll
        for (int m = 0; m < NE; ++m) x[m] = T[(su + sx[m]) + cx];
        d4 acc[3][RB];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[p][rb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int sq = 0; sq < KQ; ++sq) {
            d4 av[3][RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                av[0][rb] = As[((0 * RB + rb) * KQ + sq) * 64 + lane];
                av[1][rb] = As[((1 * RB + rb) * KQ + sq) * 64 + lane];
                av[2][rb] = av[0][rb] + av[1][rb];
            }
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const double2 xv = x[4 * sq + s4];
                const double bs = xv.x + xv.y;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc[0][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0][rb][s4], xv.x, acc[0][rb], 0, 0, 0);
                    acc[1][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1][rb][s4], xv.y, acc[1][rb], 0, 0, 0);
                    acc[2][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[2][rb][s4], bs, acc[2][rb], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double p1 = acc[0][rb][v], p2 = acc[1][rb][v], p3 = acc[2][rb][v];
                T[(su + sy[4 * rb + v]) + cy] = double2{p1 - p2, p3 - p1 - p2};
            }
    }
}

// TW: tile width t (9..13), PER = 2^(t-9) amplitudes per lane.  WIDE and
// ZERO as for k_stage.
template <int TW, bool WIDE, bool ZERO>
__global__ __launch_bounds__(512) void k_stage64(double2* __restrict__ psi, StageK a)
{
    constexpr int NT = 512, LB = 9, PER = 1 << (TW - LB);
    extern __shared__ d4 smem64[];
    double2* T = (double2*)smem64;                               // tile, padded
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    d4* Abase = smem64 + ((lslot(1 << TW) * 16 + 31) / 32);      // operand matrices
    for (int o = 0; o < a.nops; ++o) {
        const int k = a.op_k[o];
        const int D = 1 << k, RB = D / 16, KQ = D / 16, NA = 2 * RB * KQ * 256;
        double* dst = (double*)Abase + a.op_aoff[o];
        const double2* mat = (const double2*)a.op_mat[o];
        for (int i = threadIdx.x; i < NA; i += NT) {
            const int s4 = i & 3, l = (i >> 2) & 63, blk = i >> 8;
            const int sq = blk % KQ, rb = (blk / KQ) % RB, p = blk / (KQ * RB);
            const int R = 16 * rb + (l & 15);
            const int C = 4 * (4 * sq + s4) + (l >> 4);
            const double2 m = mat[R * D + C];
            dst[i] = p == 0 ? m.x : m.y;
        }
    }
    // element m of lane l: tile-local index l + NT m, LDS slot lslot(l) + ES m
    constexpr int ES = NT + NT / 16;
    uint64_t dl = 0;
    for (int b = 0; b < LB; ++b)
        if ((threadIdx.x >> b) & 1) dl |= a.dep_lane[b];
    const uint32_t dlb = (uint32_t)(dl * sizeof(double2));      // used when !WIDE
    auto elem = [&](uint64_t tb, int m) -> dd2* {
        if (WIDE) return (dd2*)(psi + (tb + dl + a.dep_i[m]));
        return (dd2*)((char*)(psi + (tb + a.dep_i[m])) + dlb);
    };
    const int ls = lslot(threadIdx.x);
    dd2 xr[PER];
    auto load_tile = [&](uint64_t tile, uint64_t tb) {
        if (a.from_e0) {
#pragma unroll
            for (int m = 0; m < PER; ++m) xr[m] = dd2{0.0, 0.0};
            if (tile == 0 && threadIdx.x == 0) xr[0].x = 1.0;
        } else {
#pragma unroll
            for (int m = 0; m < PER; ++m) xr[m] = __builtin_nontemporal_load(elem(tb, m));
        }
    };
    auto parked = [&](int m) -> double2 {
        double2 e = double2{xr[m].x, xr[m].y};
        if (ZERO && (((uint32_t)threadIdx.x + (uint32_t)(NT * m)) & a.newmask_t)) e = double2{0.0, 0.0};
        return e;
    };
    double nacc = 0.0;
    uint64_t tile = blockIdx.x;
    uint64_t tb = spread_bits(tile, a.tmask);
    if (tile < a.tiles) {
        load_tile(tile, tb);
#pragma unroll
        for (int m = 0; m < PER; ++m) T[ls + ES * m] = parked(m);
    }
    __syncthreads();
    for (; tile < a.tiles; tile += gridDim.x) {
        const uint64_t nt = tile + gridDim.x;
        const uint64_t nb = ((tb | ~a.tmask) + a.tstep) & a.tmask;
        const bool next = nt < a.tiles;
        __builtin_amdgcn_s_setprio(1);
        if (next) load_tile(nt, nb);
        __builtin_amdgcn_s_setprio(0);
        for (int o = 0; o < a.nops; ++o) {
            const d4* As = (const d4*)((const double*)Abase + a.op_aoff[o]);
            if (a.op_k[o] == 5) stage64_block<5>(a, o, As, T, wave);
            else stage64_block<4>(a, o, As, T, wave);
            __syncthreads();
        }
        // each lane parks the next tile's elements in the slots it has just
        // read for its stores
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const double2 v = T[ls + ES * m];
            if (next) T[ls + ES * m] = parked(m);
            __builtin_nontemporal_store(dd2{v.x, v.y}, elem(tb, m));
            if (a.norm_out) nacc = fma(v.x, v.x, fma(v.y, v.y, nacc));
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        tb = nb;
    }
    if (a.norm_out) {
        double* sh = (double*)smem64;
        sh[threadIdx.x] = nacc;
        __syncthreads();
        for (int hh = NT / 2; hh > 0; hh >>= 1) {
            if ((int)threadIdx.x < hh) sh[threadIdx.x] += sh[threadIdx.x + hh];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.norm_out[blockIdx.x] = sh[0];
    }
}

int stage_lds_bytes(int t, int nops, const int* ks, int dtype)
{
    int scalars = 0;
    for (int o = 0; o < nops; ++o) scalars += 2 * (1 << (2 * ks[o]));
    if (dtype) {
        // complex128: tile in 32-byte units, then the matrices in double
        const int tile_d4 = (((1 << t) + ((1 << t) >> 4)) * 16 + 31) / 32;
        return tile_d4 * 32 + scalars * 8;
    }
    // complex64: the padded tile (slots lslot(0 .. 2^t - 1), where the
    // operand matrices start: see k_stage), then the matrices in float
    const int tile_f4 = ((1 << t) + ((1 << t) >> 4)) * 8 / 16;
    return tile_f4 * 16 + scalars * 4;
}

// LDS a tile of t positions may use: complex64 as above; complex128 always
// the whole CU (one 512-lane workgroup)
static inline int stage_lds_limit_dt(int t, int dtype) { return dtype ? kStageMaxLds14 : stage_lds_limit_t(t); }

// the variant for a tile of t positions (9..14), 64-bit lane offsets, and
// zeroing of stale elements
static void (*stage_kernel(int t, bool wide, bool zero, bool split))(float2*, StageK)
{
#define SV_STAGE_W(T, W)                                                                         \
    (zero ? (split ? k_stage<T, W, true, true> : k_stage<T, W, true, false>)                     \
          : (split ? k_stage<T, W, false, true> : k_stage<T, W, false, false>))
#define SV_STAGE_CASE(T) \
    case T:              \
        return wide ? SV_STAGE_W(T, true) : SV_STAGE_W(T, false);
    switch (t) {
        SV_STAGE_CASE(9)
        SV_STAGE_CASE(10)
        SV_STAGE_CASE(11)
        SV_STAGE_CASE(12)
        SV_STAGE_CASE(13)
        SV_STAGE_CASE(14)
    }
#undef SV_STAGE_CASE
#undef SV_STAGE_W
    return nullptr;
}

static void (*stage64_kernel(int t, bool wide, bool zero))(double2*, StageK)
{
#define SV_STAGE64_CASE(T) \
    case T:                \
        return wide ? (zero ? k_stage64<T, true, true> : k_stage64<T, true, false>) \
                    : (zero ? k_stage64<T, false, true> : k_stage64<T, false, false>);
    switch (t) {
        SV_STAGE64_CASE(9)
        SV_STAGE64_CASE(10)
        SV_STAGE64_CASE(11)
        SV_STAGE64_CASE(12)
        SV_STAGE64_CASE(13)
    }
#undef SV_STAGE64_CASE
    return nullptr;
}

// 14-position tiles need the whole LDS of a CU for one workgroup; where the
// device refuses that, tiles stop at 13 positions (and complex128 states
// take no staged passes)
static std::atomic<bool> g_stage14{false};
static std::atomic<bool> g_stage64{false};

hipError_t stage_prepare()
{
    static std::atomic<bool> done{false};
    if (done) return hipSuccess;
    for (int t = 9; t <= 13; ++t)
        for (int v = 0; v < 8; ++v) {
            void (*k)(float2*, StageK) = stage_kernel(t, v & 1, v & 2, v & 4);
            const hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     kStageMaxLds);
            if (e != hipSuccess) return e;
        }
    bool ok14 = true;
    for (int v = 0; v < 8 && ok14; ++v) {
        void (*k)(float2*, StageK) = stage_kernel(14, v & 1, v & 2, v & 4);
        ok14 = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, kStageMaxLds14) ==
               hipSuccess;
    }
    if (!ok14) (void)hipGetLastError();
    g_stage14 = ok14;
    bool ok64 = true;
    for (int t = 9; t <= 13 && ok64; ++t)
        for (int v = 0; v < 4 && ok64; ++v) {
            void (*k)(double2*, StageK) = stage64_kernel(t, v & 1, v & 2);
            ok64 = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, kStageMaxLds14) ==
                   hipSuccess;
        }
    if (!ok64) (void)hipGetLastError();
    g_stage64 = ok64;
    done = true;
    return hipSuccess;
}

int split_exponent(double bound)
{
    if (!(bound >= 0.0) || !std::isfinite(bound)) return kNoSplit;
    if (bound < 0x1p-85) return 100;
    int e = 15 - (int)std::ceil(std::log2(bound));
    while (std::ldexp(bound, e) > 32768.0) --e;
    while (e < 100 && std::ldexp(bound, e + 1) <= 32768.0) ++e;
    return e < -100 ? kNoSplit : (e > 100 ? 100 : e);
}

int stage_max_t(int dtype)
{
    if (stage_prepare() != hipSuccess) return dtype ? 0 : 13;
    if (dtype) return g_stage64 ? 13 : 0;
    return g_stage14 ? kStageMaxT : 13;
}

int stage_lds_limit(int t, int dtype)
{
    return stage_lds_limit_dt(t, dtype);
}

// Tile positions of a staged pass, ascending, into P (returns t, or -1 when
// the run does not fit): 0..3 plus every target, widened with the lowest
// free positions to the widest tile within t_max that the LDS holds (a
// 14-position tile: one workgroup per CU; 13 and less: two or more 256-lane
// ones).  Wider tiles mean more 16-group units per wave and longer
// contiguous runs in memory: on the 30-qubit headline, widening to 14
// wherever it fits measured 35.2-35.5 ms per step against 36.4 when tiles
// widened to 13 at most.  Only positions inside the support widen it: one
// outside would double the amplitudes visited (beyond the 9 the kernel
// needs).
static int stage_positions(int nloc, int nops, const int* ks, const int* const* pos, int t_max,
                           uint64_t support, int* P, int dtype)
{
    if (t_max > stage_max_t(dtype)) t_max = stage_max_t(dtype);
    if (nops < 1 || nops > kStageMaxOps) return -1;
    bool in[64] = {};
    for (int p = 0; p < 4; ++p) in[p] = true;
    for (int o = 0; o < nops; ++o) {
        if (ks[o] < 4 || ks[o] > 5) return -1;
        for (int j = 0; j < ks[o]; ++j) in[pos[o][j]] = true;
    }
    int cnt = 0;
    for (int p = 0; p < 64; ++p) cnt += in[p];
    // support positions free to widen with, lowest first
    int cand[64], nc = 0;
    for (int p = 0; p < nloc; ++p)
        if (!in[p] && ((support >> p) & 1)) cand[nc++] = p;
    auto fits = [&](int tt) { return stage_lds_bytes(tt, nops, ks, dtype) <= stage_lds_limit_dt(tt, dtype); };
    // the widest tile within t_max whose LDS fits (up to 13 positions the
    // limit is the same, so past the first width that fails no narrower
    // one fits; 14 has a limit of its own)
    int want = cnt;
    for (int tt = t_max; tt > cnt; --tt)
        if (tt - cnt <= nc && fits(tt)) {
            want = tt;
            break;
        }
    for (int i = 0; i < want - cnt; ++i) in[cand[i]] = true;
    cnt = want;
    // at least 9 positions, from outside the support if need be
    for (int p = 0; p < nloc && cnt < 9; ++p) {
        if (in[p]) continue;
        if (!fits(cnt + 1)) break;
        in[p] = true;
        ++cnt;
    }
    int t = 0;
    for (int p = 0; p < 64; ++p)
        if (in[p]) P[t++] = p;
    if (t > t_max || t < 9 || nloc < t || !fits(t))
        return -1;
    return t;
}

uint64_t stage_visits(int nloc, int nops, const int* ks, const int* const* pos, int t_max, uint64_t support,
                      int dtype)
{
    int P[64];
    const int t = stage_positions(nloc, nops, ks, pos, t_max, support, P, dtype);
    if (t < 0) return 0;
    uint64_t pmask = 0;
    for (int b = 0; b < t; ++b) pmask |= 1ull << P[b];
    const uint64_t full = nloc >= 64 ? ~0ull : ((1ull << nloc) - 1);
    return (1ull << t) << __builtin_popcountll(full & ~pmask & support);
}

hipError_t launch_stage(hipStream_t st, void* psi, int nloc, int nops, const int* ks, const int* const* pos,
                        const void* const* mats, int t_max, bool from_e0, double* norm_out, int* norm_blocks,
                        int* t_out, uint64_t support, bool garbage, uint64_t* tile_mask_out,
                        uint64_t* amps_out, int split_exp, int dtype)
{
    int P[64];
    const int t = stage_positions(nloc, nops, ks, pos, t_max, support, P, dtype);
    if (t < 0) return hipErrorInvalidValue;
    if (dtype && split_exp != kNoSplit) return hipErrorInvalidValue;
    StageK a{};
    a.t = t;
    a.nops = nops;
    a.from_e0 = from_e0 ? 1 : 0;
    a.norm_out = norm_out;
    const bool split = split_exp != kNoSplit;
    if (split && (split_exp < -100 || split_exp > 100)) return hipErrorInvalidValue;
    a.split_scale = split ? std::ldexp(1.0f, split_exp) : 1.0f;
    a.split_unscale = split ? std::ldexp(1.0f, -split_exp) : 1.0f;
    // tiles: only those whose id bits lie on positions that may be non-zero
    // (support); the other tiles hold zeros and stay zero
    uint64_t pmask = 0;
    for (int b = 0; b < t; ++b) pmask |= 1ull << P[b];
    const uint64_t full = nloc >= 64 ? ~0ull : ((1ull << nloc) - 1);
    support &= full;
    a.tmask = full & ~pmask & support;
    a.tiles = 1ull << __builtin_popcountll(a.tmask);
    const uint64_t newmask = (garbage && !from_e0) ? (pmask & ~support) : 0;
    a.newmask_t = 0;
    for (int b = 0; b < t; ++b)
        if ((newmask >> P[b]) & 1) a.newmask_t |= 1u << b;
    const int lb = dtype ? 9 : (t >= 14 ? (split ? 10 : 9) : 8);  // lane bits of the tile index
    // complex64: tile bit 0 (position 0) pairs adjacent amplitudes; lane bit
    // b is tile bit b + 1; pair index bit c is tile bit lb + 1 + c.
    // complex128: lane bit b is tile bit b; element index bit c is tile bit
    // lb + c
    const int pb = dtype ? 0 : 1;
    for (int b = 0; b < lb; ++b) a.dep_lane[b] = 1ull << P[b + pb];
    for (int i = 0; i < (1 << (t - lb - pb)); ++i) {
        uint64_t d = 0;
        for (int b = lb + pb; b < t; ++b)
            if ((i >> (b - lb - pb)) & 1) d |= 1ull << P[b];
        a.dep_i[i] = d;
    }
    int aoff = 0;
    for (int o = 0; o < nops; ++o) {
        a.op_k[o] = ks[o];
        a.op_mat[o] = (const float2*)mats[o];
        a.op_aoff[o] = aoff;
        aoff += 2 * (1 << (2 * ks[o]));
        int tbit[kMaxDense];
        for (int j = 0; j < ks[o]; ++j) {
            int b = 0;
            while (P[b] != pos[o][j]) ++b;
            a.op_bits[o][j] = b;
            tbit[j] = b;
        }
        for (int j = 1; j < ks[o]; ++j)
            for (int l = j; l > 0 && tbit[l - 1] > tbit[l]; --l) {
                const int tmp = tbit[l]; tbit[l] = tbit[l - 1]; tbit[l - 1] = tmp;
            }
        for (int j = 0; j < ks[o]; ++j) a.op_lowmask_bits[o][j] = tbit[j];
    }
    const int lds = stage_lds_bytes(t, nops, ks, dtype);
    if (lds > stage_lds_limit_dt(t, dtype)) return hipErrorInvalidValue;
    // byte offset of the lane part of an element address
    uint64_t dl_max = 0;
    for (int b = 0; b < lb; ++b) dl_max |= a.dep_lane[b];
    const bool wide = dl_max * (dtype ? sizeof(double2) : sizeof(float2)) >= (1ull << 32);
    void (*kern)(float2*, StageK) = dtype ? nullptr : stage_kernel(t, wide, a.newmask_t != 0, split);
    void (*kern64)(double2*, StageK) = dtype ? stage64_kernel(t, wide, a.newmask_t != 0) : nullptr;
    if (!kern && !kern64) return hipErrorInvalidValue;
    {
        const hipError_t e = stage_prepare();
        if (e != hipSuccess) return e;
    }
    // persistent: as many workgroups as are resident (LDS-limited, at most 4
    // per CU; complex128: one 512-lane workgroup per CU)
    int per_cu = (160 * 1024) / lds;
    if (per_cu > 4) per_cu = 4;
    if (per_cu < 1 || dtype) per_cu = 1;
    uint64_t grid = a.tiles;
    const uint64_t cap = 256ull * per_cu;
    if (grid > cap) grid = cap;
    a.tstep = spread_bits(grid, a.tmask);
    if (dtype)
        hipLaunchKernelGGL(kern64, dim3((unsigned)grid), dim3(512), lds, st, (double2*)psi, a);
    else
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(stage_threads(t, split)), lds, st, (float2*)psi, a);
    if (t_out) *t_out = t;
    if (norm_blocks) *norm_blocks = norm_out ? (int)grid : 0;
    if (tile_mask_out) *tile_mask_out = pmask;
    if (amps_out) *amps_out = a.tiles << t;
    return hipGetLastError();
}

}  // namespace sv
