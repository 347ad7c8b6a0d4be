// Fused dense sweep on the matrix cores (complex64, k = 4..6): single-state
// and batched launches.  The per-tile body (operand layouts, LDS staging of
// the real form of the block) is in sv_device.h.
#include "sv_device.h"

namespace sv {

template <int K, bool FOLD, bool STAGED>
__global__ __launch_bounds__(256) void k_dense_mfma(Sweep a)
{
    __shared__ f4 As[MfmaShape<K>::NA / 4];
    __shared__ float2 Xs[STAGED ? 4 * MfmaShape<K>::XS : 1];
    mfma_stage_matrix<K>(As, (const float2*)a.mat);
    __syncthreads();
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    mfma_tiles<K, FOLD, STAGED>(a, As, Xs + (STAGED ? (threadIdx.x >> 6) * MfmaShape<K>::XS : 0), wave,
                                nwaves, a.groups / 16);
}

// Many sweeps (of different states) in one launch: workgroup b belongs to
// the sweep i with items[i].block0 <= b < items[i + 1].block0 (the last
// sweep ends at gridDim.x); its waves stride over that sweep's tiles.
__device__ __forceinline__ int find_item(const Sweep* __restrict__ items, int nitems, uint64_t b)
{
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int K, bool FOLD, bool STAGED>
__global__ __launch_bounds__(256) void k_dense_mfma_batch(const Sweep* __restrict__ items, int nitems)
{
    __shared__ f4 As[MfmaShape<K>::NA / 4];
    __shared__ float2 Xs[STAGED ? 4 * MfmaShape<K>::XS : 1];
    const int i = find_item(items, nitems, blockIdx.x);
    const Sweep& a = items[i];
    const uint64_t b_end = (i + 1 < nitems) ? items[i + 1].block0 : gridDim.x;
    const uint64_t nb = b_end - a.block0;
    mfma_stage_matrix<K>(As, (const float2*)a.mat);
    __syncthreads();
    const uint64_t wave = (blockIdx.x - a.block0) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    mfma_tiles<K, FOLD, STAGED>(a, As, Xs + (STAGED ? (threadIdx.x >> 6) * MfmaShape<K>::XS : 0), wave,
                                nb * (blockDim.x >> 6), a.groups / 16);
}

template <int K, bool STAGED>
static hipError_t mfma_dispatch(hipStream_t st, const Sweep& a)
{
    const uint64_t tiles = a.groups / 16;
    uint64_t g = (tiles + 3) / 4;
    const uint64_t cap = 256 * (K == 6 ? 2 : 6);
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    if (a.ftab)
        hipLaunchKernelGGL((k_dense_mfma<K, true, STAGED>), dim3((unsigned)g), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_dense_mfma<K, false, STAGED>), dim3((unsigned)g), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_dense_mfma(hipStream_t st, void* psi, int nloc, int k, const int* pos, const void* mat,
                             const DiagSpec* fold, uint64_t idx_offset)
{
    if (k < 4 || k > 6 || nloc < k + 4) return hipErrorInvalidValue;
    const Sweep a = make_sweep(psi, nloc, k, pos, mat, fold, idx_offset);
    switch (k) {
        case 4: return a.staged ? mfma_dispatch<4, true>(st, a) : mfma_dispatch<4, false>(st, a);
        case 5: return a.staged ? mfma_dispatch<5, true>(st, a) : mfma_dispatch<5, false>(st, a);
        case 6: return mfma_dispatch<6, false>(st, a);
    }
    return hipErrorInvalidValue;
}

uint64_t mfma_batch_blocks(uint64_t groups)
{
    // about 8 tiles per wave, 4 waves per workgroup
    const uint64_t tiles = groups / 16;
    const uint64_t b = (tiles + 31) / 32;
    return b < 1 ? 1 : b;
}

hipError_t launch_dense_mfma_batch(hipStream_t st, int k, bool fold, bool staged, const Sweep* d_items,
                                   int nitems, uint64_t total_blocks)
{
    if (nitems <= 0) return hipSuccess;
    if (total_blocks == 0 || total_blocks > 0x7fffffffull) return hipErrorInvalidValue;
    if (staged && k == 6) return hipErrorInvalidValue;
    const dim3 grid((unsigned)total_blocks), block(256);
#define SV_MB(KK, SS)                                                                                 \
    if (fold)                                                                                         \
        hipLaunchKernelGGL((k_dense_mfma_batch<KK, true, SS>), grid, block, 0, st, d_items, nitems);  \
    else                                                                                              \
        hipLaunchKernelGGL((k_dense_mfma_batch<KK, false, SS>), grid, block, 0, st, d_items, nitems);
    switch (k) {
        case 4: if (staged) { SV_MB(4, true) } else { SV_MB(4, false) } break;
        case 5: if (staged) { SV_MB(5, true) } else { SV_MB(5, false) } break;
        case 6: SV_MB(6, false) break;
        default: return hipErrorInvalidValue;
    }
#undef SV_MB
    return hipGetLastError();
}

}  // namespace sv
