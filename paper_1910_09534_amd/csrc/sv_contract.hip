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
                           int dtype)
{
    if (contract_uses_mfma(dtype, n1, n2, e)) {
        const uint64_t tiles = (1ull << (n2 - 7)) * (1ull << (n1 - 6));
        if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
        const uint32_t tiles_m = 1u << (n2 - 7);
        const uint32_t group = tiles_m < 16 ? tiles_m : 16;
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
