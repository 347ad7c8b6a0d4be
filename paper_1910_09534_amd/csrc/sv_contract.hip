// Contraction of two tensors over their entanglement indices (App. A: the
// equation that eliminates the indices introduced by EI and E2Q; Sec. 2:
// contraction deferral sums the shared indices and takes the outer product
// over the others):
//
//     out[x2 * 2^n1 + x1] = sum_e t1[e * 2^n1 + x1] * t2[e * 2^n2 + x2]
//
// With N = 2^n1, M = 2^n2 and K = 2^e this is the complex matrix product
// out (M x N) = t2^T (M x K) * t1 (K x N): dense, bound by the matrix
// cores once K reaches a few tens.
//
//   k_contract_mfma   complex64, M >= 128, N >= 64, K >= 16: 128 x 64 output
//                     tiles per 256-lane workgroup, 64 x 32 per wave, as
//                     three real products per 16 x 16 block (3M form:
//                     P1 = Br Ar, P2 = Bi Ai, P3 = (Br + Bi)(Ar + Ai);
//                     re = P1 - P2, im = P3 - P1 - P2) on v_mfma_f32_16x16x4f32,
//                     K in chunks of 16 through double-buffered LDS, the next
//                     chunk's global loads in flight during the products.
//   k_contract_plain  any size, complex64 (FP32 sums) or complex128 (FP64):
//                     one output per lane, a loop over K.
#include <hip/hip_runtime.h>

#include "sv_internal.h"

namespace sv {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kCM = 128;          // output rows (x2) per workgroup
constexpr int kCN = 64;           // output columns (x1) per workgroup
constexpr int kCK = 16;           // K per chunk
constexpr int kCThreads = 256;
constexpr int kBStride = kCM + 4; // LDS row strides in complex elements (padding staggers banks)
constexpr int kAStride = kCN + 4;

// t1 and t2 are not __restrict__: loads through such pointers count as
// invariant and are moved past the scheduling fence that keeps them ahead of
// the products
__global__ __launch_bounds__(kCThreads) void k_contract_mfma(const float2* t1, const float2* t2,
                                                             float2* __restrict__ out, int n1, int n2,
                                                             int e, uint32_t tiles_n, uint32_t group)
{
    __shared__ __attribute__((aligned(16))) float2 Bs[2][kCK * kBStride];
    __shared__ __attribute__((aligned(16))) float2 As[2][kCK * kAStride];
    const uint64_t N = 1ull << n1, M = 1ull << n2;
    const uint32_t K = 1u << e;
    // grouped order: `group` consecutive row blocks sweep the column blocks
    // together, so a t1 panel is read once per group of row blocks (per XCD
    // L2) and the group's t2 panels stay in cache across the sweep.  (Giving
    // each XCD a contiguous range of this order instead measured 2x the L2
    // refills.)
    const uint32_t per = group * tiles_n;
    const uint32_t g = blockIdx.x / per, r = blockIdx.x % per;
    const uint32_t tn = r / group, tm = g * group + r % group;
    const uint64_t m0 = (uint64_t)tm * kCM, n0 = (uint64_t)tn * kCN;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;

    // global -> register staging of one K chunk: 4 float4 of t2, 2 of t1 per
    // lane (plain unrolled loops: the arrays stay in registers)
    const uint32_t nchunks = K / kCK;
    // named values rather than arrays: private arrays get moved to LDS
    float4 gb0, gb1, gb2, gb3, ga0, ga1;
    // this lane's slots: t2 rows k = tid / 64 + 4 i, columns 2 (tid % 64);
    // t1 rows k = tid / 32 + 8 i, columns 2 (tid % 32)
    const int kb = tid >> 6, mb2 = 2 * (tid & 63);
    const int ka = tid >> 5, na2 = 2 * (tid & 31);
    const int bo = kb * kBStride + mb2, ao = ka * kAStride + na2;
    const uint64_t bg = (uint64_t)kb * M + m0 + mb2, ag = (uint64_t)ka * N + n0 + na2;
#define SV_CONTRACT_LOAD(kn)                                              \
    do {                                                                  \
        const float2* pb = t2 + bg + (uint64_t)(kn) * M;                  \
        const float2* pa = t1 + ag + (uint64_t)(kn) * N;                  \
        gb0 = *(const float4*)(pb);                                       \
        gb1 = *(const float4*)(pb + 4 * M);                               \
        gb2 = *(const float4*)(pb + 8 * M);                               \
        gb3 = *(const float4*)(pb + 12 * M);                              \
        ga0 = *(const float4*)(pa);                                       \
        ga1 = *(const float4*)(pa + 8 * N);                               \
    } while (0)
#define SV_CONTRACT_PARK(bf)                                              \
    do {                                                                  \
        *(float4*)(&Bs[bf][bo]) = gb0;                                    \
        *(float4*)(&Bs[bf][bo + 4 * kBStride]) = gb1;                     \
        *(float4*)(&Bs[bf][bo + 8 * kBStride]) = gb2;                     \
        *(float4*)(&Bs[bf][bo + 12 * kBStride]) = gb3;                    \
        *(float4*)(&As[bf][ao]) = ga0;                                    \
        *(float4*)(&As[bf][ao + 8 * kAStride]) = ga1;                     \
    } while (0)

    f4v p1[4][2], p2[4][2], p3[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            p1[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
            p2[a][b] = p1[a][b];
            p3[a][b] = p1[a][b];
        }

    SV_CONTRACT_LOAD(0);
    SV_CONTRACT_PARK(0);
    __syncthreads();
    for (uint32_t c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        // the next chunk's loads are in flight during this chunk's products
        // (the last iteration loads its own chunk again: in bounds, unused)
        SV_CONTRACT_LOAD((c + 1 < nchunks ? c + 1 : c) * kCK);
        // keep the loads ahead of the products (the scheduler would sink
        // them to their use, after the products)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < kCK / 4; ++s) {
            const int k = 4 * s + lk;
            float br[4], bi[4], bs[4], ar[2], ai[2], as_[2];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const float2 v = Bs[buf][k * kBStride + wm + 16 * a + li];
                br[a] = v.x;
                bi[a] = v.y;
                bs[a] = v.x + v.y;
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const float2 v = As[buf][k * kAStride + wn + 16 * b + li];
                ar[b] = v.x;
                ai[b] = v.y;
                as_[b] = v.x + v.y;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    p1[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(br[a], ar[b], p1[a][b], 0, 0, 0);
                    p2[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(bi[a], ai[b], p2[a][b], 0, 0, 0);
                    p3[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(bs[a], as_[b], p3[a][b], 0, 0, 0);
                }
        }
        // park the next chunk in the other buffer (read by nobody since the
        // previous barrier); after the products, so that only this waits
        // for the loads
        __builtin_amdgcn_sched_barrier(0);
        SV_CONTRACT_PARK(buf ^ 1);
        __syncthreads();
    }
#undef SV_CONTRACT_LOAD
#undef SV_CONTRACT_PARK
    // lane holds rows 4 lk + v of each 16-row block, column li of each 16-column block
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint64_t m = m0 + wm + 16 * a + 4 * lk + v;
                const uint64_t n = n0 + wn + 16 * b + li;
                const float x1 = p1[a][b][v], x2 = p2[a][b][v], x3 = p3[a][b][v];
                out[m * N + n] = float2{x1 - x2, x3 - x1 - x2};
            }
}

// ---- split-fp16 form of the matrix-core contraction -----------------------
// The same 128 x 64 output tiles and 16-deep K chunks, with the products on
// the fp16 matrix cores at single-precision accuracy: every input is scaled
// by a power of two (from the largest |component| of its tensor, so that it
// stays below 2^14) and split into hi = f16(x) and lo = f16(x - hi); the
// three products A_hi B_hi + A_hi B_lo + A_lo B_hi accumulate in fp32 on
// v_mfma_f32_16x16x32_f16.  A K chunk of 16 complex values is one 32-deep
// real product: Re = [Br | Bi] [Ar ; -Ai] and Im = [Br | Bi] [Ai ; Ar]
// (B = t2^T, A = t1): six products per 16 x 16 block per chunk, both
// sharing the B operand.  The chunk
// is parked in LDS already split, each row's 16 values contiguous (hi and
// lo of the real and imaginary parts), so a lane reads its 8 operand
// values with one 16-byte access.
typedef _Float16 ch8 __attribute__((ext_vector_type(8)));
typedef _Float16 ch4 __attribute__((ext_vector_type(4)));
typedef uint32_t cu4 __attribute__((ext_vector_type(4)));
typedef uint32_t cu2 __attribute__((ext_vector_type(2)));

constexpr int kSRow = 16;                  // f16 per LDS row: the chunk's 16 k values

// f16 pair (a, b), round to nearest
// f16(a s), f16(b s), each rounded once (s is a power of two, so a s is
// exact): the scale and the conversion in one mixed-precision fma
__device__ __forceinline__ uint32_t cpk_hi(float a, float b, float s)
{
    uint32_t r;
    asm("v_fma_mixlo_f16 %0, %1, %3, 0\n\t"
        "v_fma_mixhi_f16 %0, %2, %3, 0"
        : "=&v"(r)
        : "v"(a), "v"(b), "v"(s));
    return r;
}

// f16(a s - hi.lo), f16(b s - hi.hi): residuals formed exactly in the fma,
// rounded once
__device__ __forceinline__ uint32_t cpk_lo(float a, float b, float s, uint32_t hi)
{
    uint32_t r;
    asm("v_fma_mixlo_f16 %0, %1, %3, -%4 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %0, %2, %3, -%4 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
        : "=&v"(r)
        : "v"(a), "v"(b), "v"(s), "v"(hi));
    return r;
}

// element offset in a part of the LDS chunk of row r, k-octet o (0, 1):
// the two octets of a row swap places on every other group of four rows,
// which spreads the 16-byte reads of sixteen consecutive rows over the banks
__device__ __forceinline__ int srow(int r, int o)
{
    return r * kSRow + ((o ^ ((r >> 2) & 1)) << 3);
}

// largest |component| of count floats, as float bits, into *out (atomic
// max: non-negative floats order as their bit patterns)
__global__ __launch_bounds__(256) void k_absmax(const float* __restrict__ x, uint64_t count, uint32_t* out)
{
    __shared__ float sh[256];
    float m = 0.f;
    const uint64_t stride = (uint64_t)gridDim.x * 256 * 4;
    for (uint64_t i = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 4; i < count; i += stride) {
        const float4 v = *(const float4*)(x + i);
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, __float_as_uint(sh[0]));
}

// exponent s with max 2^s <= 2^14 (0 for an all-zero tensor)
__device__ __forceinline__ int scale_exp(uint32_t maxbits)
{
    const float m = __uint_as_float(maxbits);
    if (!(m > 0.f) || !isfinite(m)) return 0;
    int e = 14 - (int)ceilf(log2f(m));
    while (ldexpf(m, e) > 16384.f) --e;
    return e < -100 ? -100 : (e > 100 ? 100 : e);
}

__global__ __launch_bounds__(kCThreads) void k_contract_split(const float2* t1, const float2* t2,
                                                              float2* __restrict__ out, int n1, int n2, int e,
                                                              uint32_t tiles_n, uint32_t group,
                                                              const uint32_t* __restrict__ maxbits)
{
    // [buffer][part: re hi, re lo, im hi, im lo][row][k]
    __shared__ __attribute__((aligned(16))) _Float16 Bs[2][4][kCM * kSRow];
    __shared__ __attribute__((aligned(16))) _Float16 As[2][4][kCN * kSRow];
    const uint64_t N = 1ull << n1, M = 1ull << n2;
    const uint32_t K = 1u << e;
    const uint32_t per = group * tiles_n;
    const uint32_t gq = blockIdx.x / per, rr = blockIdx.x % per;
    const uint32_t tn = rr / group, tm = gq * group + rr % group;
    const uint64_t m0 = (uint64_t)tm * kCM, n0 = (uint64_t)tn * kCN;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 32;
    const int li = lane & 15, g = lane >> 4;
    const int eb = scale_exp(maxbits[0]), ea = scale_exp(maxbits[1]);
    // (the two factors are applied one after the other on the way out:
    // 2^-(eb + ea) alone can leave the float range)
    const float sb = ldexpf(1.f, eb), sa = ldexpf(1.f, ea), ub = ldexpf(1.f, -eb), ua = ldexpf(1.f, -ea);

    // staging: t2 column m = tid % 128, k = 8 (tid / 128) + 0..7; t1 column
    // n = tid % 64, k = 4 (tid / 64) + 0..3 (each load row is 64 lanes of
    // consecutive columns)
    const int bm = tid & 127, bo = tid >> 7;
    const int an = tid & 63, aq = tid >> 6;
    const uint32_t nchunks = K / kCK;
    float2 gb[8], ga[4];
    auto load = [&](uint32_t c) {
        const float2* pb = t2 + (uint64_t)(c * kCK + 8 * bo) * M + m0 + bm;
        const float2* pa = t1 + (uint64_t)(c * kCK + 4 * aq) * N + n0 + an;
#pragma unroll
        for (int k = 0; k < 8; ++k) gb[k] = pb[(uint64_t)k * M];
#pragma unroll
        for (int k = 0; k < 4; ++k) ga[k] = pa[(uint64_t)k * N];
    };
    auto park = [&](int buf) {
        cu4 rh, rl, ih, il;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float x0 = gb[2 * w].x, x1 = gb[2 * w + 1].x;
            const float y0 = gb[2 * w].y, y1 = gb[2 * w + 1].y;
            rh[w] = cpk_hi(x0, x1, sb);
            ih[w] = cpk_hi(y0, y1, sb);
            rl[w] = cpk_lo(x0, x1, sb, rh[w]);
            il[w] = cpk_lo(y0, y1, sb, ih[w]);
        }
        const int ob = srow(bm, bo);
        *(cu4*)&Bs[buf][0][ob] = rh;
        *(cu4*)&Bs[buf][1][ob] = rl;
        *(cu4*)&Bs[buf][2][ob] = ih;
        *(cu4*)&Bs[buf][3][ob] = il;
        cu2 arh, arl, aih, ail;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const float x0 = ga[2 * w].x, x1 = ga[2 * w + 1].x;
            const float y0 = ga[2 * w].y, y1 = ga[2 * w + 1].y;
            arh[w] = cpk_hi(x0, x1, sa);
            aih[w] = cpk_hi(y0, y1, sa);
            arl[w] = cpk_lo(x0, x1, sa, arh[w]);
            ail[w] = cpk_lo(y0, y1, sa, aih[w]);
        }
        const int oa = srow(an, aq >> 1) + 4 * (aq & 1);
        *(cu2*)&As[buf][0][oa] = arh;
        *(cu2*)&As[buf][1][oa] = arl;
        *(cu2*)&As[buf][2][oa] = aih;
        *(cu2*)&As[buf][3][oa] = ail;
    };

    f4v re[4][2], im[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            re[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
            im[a][b] = re[a][b];
        }
    // lane (li, g): operand element e is k = 8 (g & 1) + e of the real part
    // (g < 2) or the imaginary part (g >= 2).  Re = [Br | Bi] [Ar ; -Ai] and
    // Im = [Br | Bi] [Ai ; Ar]: both products share the A operand, and the
    // -Ai of the real one is the sign flipped in lanes g >= 2 of its other
    // operand (two 16-column blocks per wave, against four 16-row blocks
    // of the A operand)
    const int o = g & 1;
    const int pA = g < 2 ? 0 : 2;                 // A operand rows: Br or Bi
    const int pBr = g < 2 ? 0 : 2;                // [Ar ; Ai], Ai negated below
    const int pBi = g < 2 ? 2 : 0;                // [Ai ; Ar]
    const uint32_t neg = g < 2 ? 0u : 0x80008000u;

    load(0);
    park(0);
    __syncthreads();
    for (uint32_t c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) load(c + 1);
        __builtin_amdgcn_sched_barrier(0);
        ch8 xbr_h[2], xbr_l[2], xbi_h[2], xbi_l[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int ob = srow(wn + 16 * b + li, o);
            xbr_h[b] = __builtin_bit_cast(ch8, *(const cu4*)&As[buf][pBr][ob] ^ neg);
            xbr_l[b] = __builtin_bit_cast(ch8, *(const cu4*)&As[buf][pBr + 1][ob] ^ neg);
            xbi_h[b] = *(const ch8*)&As[buf][pBi][ob];
            xbi_l[b] = *(const ch8*)&As[buf][pBi + 1][ob];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int oa = srow(wm + 16 * a + li, o);
            const cu4 h = *(const cu4*)&Bs[buf][pA][oa];
            const cu4 l = *(const cu4*)&Bs[buf][pA + 1][oa];
            const ch8 a_h = __builtin_bit_cast(ch8, h), a_l = __builtin_bit_cast(ch8, l);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                re[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_l, xbr_h[b], re[a][b], 0, 0, 0);
                im[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_l, xbi_h[b], im[a][b], 0, 0, 0);
                re[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, xbr_l[b], re[a][b], 0, 0, 0);
                im[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, xbi_l[b], im[a][b], 0, 0, 0);
                re[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, xbr_h[b], re[a][b], 0, 0, 0);
                im[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, xbi_h[b], im[a][b], 0, 0, 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (c + 1 < nchunks) park(buf ^ 1);
        __syncthreads();
    }
    // lane holds rows 4 g + v of each 16-row block, column li of each 16-column block
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint64_t m = m0 + wm + 16 * a + 4 * g + v;
                const uint64_t n = n0 + wn + 16 * b + li;
                out[m * N + n] = float2{re[a][b][v] * ub * ua, im[a][b][v] * ub * ua};
            }
}

template <typename T, typename A>
__global__ __launch_bounds__(256) void k_contract_plain(const T* __restrict__ t1, const T* __restrict__ t2,
                                                        T* __restrict__ out, int n1, int n2, int e)
{
    const uint64_t N = 1ull << n1, M = 1ull << n2, K = 1ull << e;
    const uint64_t total = N * M;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total; o += stride) {
        const uint64_t n = o & (N - 1), m = o >> n1;
        A re = 0, im = 0;
        for (uint64_t k = 0; k < K; ++k) {
            const T a = t1[k * N + n], b = t2[k * M + m];
            re += (A)a.x * (A)b.x - (A)a.y * (A)b.y;
            im += (A)a.x * (A)b.y + (A)a.y * (A)b.x;
        }
        out[o].x = re;
        out[o].y = im;
    }
}

}  // namespace

bool contract_uses_mfma(int dtype, int n1, int n2, int e)
{
    return dtype == 0 && n2 >= 7 && n1 >= 6 && e >= 4;
}

hipError_t launch_contract(hipStream_t st, const void* t1, const void* t2, void* out, int n1, int n2, int e,
                           int dtype, bool split)
{
    if (contract_uses_mfma(dtype, n1, n2, e)) {
        const uint64_t tiles = (1ull << (n2 - 7)) * (1ull << (n1 - 6));
        if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
        const uint32_t tiles_m = 1u << (n2 - 7);
        const uint32_t group = tiles_m < 16 ? tiles_m : 16;
        if (split) {
            // the two tensors' largest |component|, in stream-ordered memory
            // (concurrent contractions on other streams keep their own)
            uint32_t* mx = nullptr;
            hipError_t err = hipMallocAsync((void**)&mx, 2 * sizeof(uint32_t), st);
            if (err != hipSuccess) return err;
            err = hipMemsetAsync(mx, 0, 2 * sizeof(uint32_t), st);
            if (err != hipSuccess) return err;
            const uint64_t c2 = 2ull << (n2 + e), c1 = 2ull << (n1 + e);
            auto grid_for = [](uint64_t count) {
                uint64_t gsz = (count / 4 + 255) / 256;
                return (unsigned)(gsz > 2048 ? 2048 : (gsz < 1 ? 1 : gsz));
            };
            hipLaunchKernelGGL(k_absmax, dim3(grid_for(c2)), dim3(256), 0, st, (const float*)t2, c2, mx);
            hipLaunchKernelGGL(k_absmax, dim3(grid_for(c1)), dim3(256), 0, st, (const float*)t1, c1, mx + 1);
            hipLaunchKernelGGL(k_contract_split, dim3((unsigned)tiles), dim3(kCThreads), 0, st, (const float2*)t1,
                               (const float2*)t2, (float2*)out, n1, n2, e, (uint32_t)(1ull << (n1 - 6)), group,
                               (const uint32_t*)mx);
            err = hipGetLastError();
            const hipError_t e2 = hipFreeAsync(mx, st);
            return err != hipSuccess ? err : e2;
        }
        hipLaunchKernelGGL(k_contract_mfma, dim3((unsigned)tiles), dim3(kCThreads), 0, st, (const float2*)t1,
                           (const float2*)t2, (float2*)out, n1, n2, e, (uint32_t)(1ull << (n1 - 6)), group);
        return hipGetLastError();
    }
    const uint64_t total = 1ull << (n1 + n2);
    uint64_t grid = (total + 255) / 256;
    if (grid > (1u << 20)) grid = 1u << 20;
    if (dtype == 0)
        hipLaunchKernelGGL((k_contract_plain<float2, float>), dim3((unsigned)grid), dim3(256), 0, st,
                           (const float2*)t1, (const float2*)t2, (float2*)out, n1, n2, e);
    else
        hipLaunchKernelGGL((k_contract_plain<double2, double>), dim3((unsigned)grid), dim3(256), 0, st,
                           (const double2*)t1, (const double2*)t2, (double2*)out, n1, n2, e);
    return hipGetLastError();
}

}  // namespace sv
