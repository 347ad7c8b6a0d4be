// Internal interface between the C-ABI host code (sv_api.cpp) and the gfx950
// kernels (sv_kernels.hip).  Not installed; not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sv {

constexpr int kMaxDense = 6;    // largest fused block (c64); c128 stops at 5
constexpr int kMaxDiag = 12;    // largest diagonal op
constexpr int kMaxRuns = 48;    // bit-move runs of a permutation

// A diagonal table applied in the epilogue of a dense sweep (or on its own).
// phase index of amplitude i = sum_j bit(i + idx_offset, pos[j]) << j.
struct DiagSpec {
    int m = 0;
    int pos[kMaxDiag] = {};
    const void* table = nullptr;   // device, 2^m entries of the state dtype
};

// Bit-position moves: dst_index = sum_r shift(src_index & mask[r], sh[r]).
struct BitRuns {
    int count = 0;
    uint64_t mask[kMaxRuns] = {};
    int shift[kMaxRuns] = {};      // > 0 left shift, < 0 right shift
};

// One dense sweep: a 2^k x 2^k block on positions tpos of the amplitude
// range psi[0, 2^nloc), optionally followed (same sweep) by a diagonal table.
struct Sweep {
    void* psi;
    const void* mat;               // row-major 2^k x 2^k, state dtype
    const void* ftab;              // folded diagonal table or nullptr
    uint64_t groups;               // 2^(nloc - k)
    uint64_t idx_offset;           // global index of psi[0] (bits of sliced positions)
    uint64_t lowmask[kMaxDense];   // (1 << p) - 1 for the target positions, ascending
    uint64_t block0;               // batched launches: first block of this sweep
    int tpos[kMaxDense];           // target positions in matrix-bit order
    int k;
    int fold_m;
    int fold_pos[kMaxDiag];
    // matrix-core sweeps staged through LDS in address order (targets among
    // the lowest four positions): element e = 64 i + lane of a 16-group tile
    // sits at tile base + st_addr_bit(lane bits) + st_addr_i[i] and goes to
    // LDS slot st_slot_bit(lane bits) + st_slot_i[i] (slot = group + 17 amp)
    int staged;
    uint64_t st_addr_bit[6];
    uint64_t st_addr_i[16];
    int st_slot_bit[6];
    int st_slot_i[16];
};

// Fill a Sweep for positions pos[0..k) over 2^nloc amplitudes.
Sweep make_sweep(void* psi, int nloc, int k, const int* pos, const void* mat, const DiagSpec* fold,
                 uint64_t idx_offset);

// Build runs for "value at bit from[p] goes to bit to[p]" for p < nbits.
BitRuns make_runs(int nbits, const int* from, const int* to);

// Pooled allocation of small work buffers (device, or pinned host).  *got
// receives the usable size (a power of two >= bytes).  nullptr on failure.
void* pool_alloc(size_t bytes, bool pinned_host, size_t* got);
void pool_free(void* p, size_t bytes, bool pinned_host);

// Zero-fill count amplitudes, then set element 0 to 1 if one_at_zero.
hipError_t launch_init(hipStream_t st, void* psi, int dtype, uint64_t count, bool one_at_zero);

// Dense 2^k x 2^k block on physical positions pos[0..k) of a range of 2^nloc
// amplitudes.  mat: device, row-major, state dtype.  fold: optional diagonal
// applied to the outputs (same sweep).  idx_offset: global index of the
// range's first element (feeds fold's bits above nloc).
hipError_t launch_dense(hipStream_t st, void* psi, int dtype, int nloc, int k, const int* pos,
                        const void* mat, const DiagSpec* fold, uint64_t idx_offset,
                        int mfma_min_k);

// Matrix-core form of the dense sweep (complex64, 4 <= k <= 6, nloc >= k + 4).
hipError_t launch_dense_mfma(hipStream_t st, void* psi, int nloc, int k, const int* pos,
                             const void* mat, const DiagSpec* fold, uint64_t idx_offset);

// Batched dense sweeps: many states, one launch (same dtype, k and fold
// flag).  d_items: device array of Sweep descriptors whose
// block0 fields partition [0, total_blocks).  VALU form: one group per lane,
// 256 lanes per workgroup.  MFMA form (complex64, k >= 4): blocks per sweep
// from mfma_batch_blocks.
hipError_t launch_dense_batch(hipStream_t st, int dtype, int k, bool fold, const Sweep* d_items,
                              int nitems, uint64_t total_blocks);
hipError_t launch_dense_mfma_batch(hipStream_t st, int k, bool fold, bool staged, const Sweep* d_items,
                                   int nitems, uint64_t total_blocks);
uint64_t mfma_batch_blocks(uint64_t groups);

// Whether a complex64 k-qubit sweep over 2^nloc amplitudes runs on the
// matrix cores (else on the vector units).
inline bool dense_uses_mfma(int k, int nloc, int mfma_min_k)
{
    return mfma_min_k >= 4 && k >= mfma_min_k && nloc >= k + 4;
}

// Staged sweep: nops dense blocks (k = 4 or 5, complex64) applied to LDS
// tiles in one HBM pass.  pos[o] / mats[o]: block o's positions and device
// matrix.  The tile (positions 0..3 and every target) is widened with free
// low positions up to t_max (<= 13) within the LDS budget.  Fails
// (hipErrorInvalidValue) when the targets alone exceed t_max positions or
// the LDS budget; *t_out receives the tile width used.  from_e0: the input
// is |0...0> and is not read (the pass writes every amplitude).  norm_out
// (non-null): each workgroup writes the FP64 sum of |psi|^2 of the amplitudes
// it wrote to norm_out[workgroup]; *norm_blocks receives the workgroup count
// (at most 1024).  support: positions on which the state may be non-zero
// (every other bit of a non-zero amplitude's index is 0); only tiles whose
// id bits lie on support positions are visited, the others hold zeros and
// stay zero, and the tile is widened with support positions only.  garbage: the memory outside the support's reach is not zero,
// so tile amplitudes with a bit on a tile position outside the support are
// taken as zero instead of read.  *tile_mask_out: the tile's positions;
// *amps_out: amplitudes visited.
// dtype 0: complex64 (fp32 or split-fp16 form); 1: complex128 (FP64 form,
// one 512-lane workgroup per CU, tiles of 9..13 positions).
int stage_lds_bytes(int t, int nops, const int* ks, int dtype = 0);
// LDS budget of a tile of t positions (complex64: 80 KiB up to 13, two
// workgroups per CU; 160 KiB at 14, one 512-lane workgroup per CU;
// complex128: 160 KiB).
int stage_lds_limit(int t, int dtype = 0);
// Sets the staged kernels' LDS attribute for every tile width (idempotent;
// launch_stage does it on first use, graph capture needs it beforehand).
hipError_t stage_prepare();
// Widest tile the device runs: complex64 14, or 13 where a workgroup cannot
// have the whole LDS of a CU; complex128 13, or 0 (no staged passes) there.
int stage_max_t(int dtype = 0);
// split_exp: kNoSplit = fp32 matrix-core form; otherwise the split-fp16
// form with the tile scaled by 2^split_exp in LDS (-100..100).
constexpr int kNoSplit = -1000;
hipError_t launch_stage(hipStream_t st, void* psi, int nloc, int nops, const int* ks, const int* const* pos,
                        const void* const* mats, int t_max, bool from_e0, double* norm_out, int* norm_blocks,
                        int* t_out, uint64_t support = ~0ull, bool garbage = false,
                        uint64_t* tile_mask_out = nullptr, uint64_t* amps_out = nullptr,
                        int split_exp = kNoSplit, int dtype = 0);
// Exponent e of the split-fp16 form's tile scale 2^e for a run whose
// blocks are all unitary and whose state norm stays below bound: the
// largest e with 2^e bound <= 2^15 (-100..100); kNoSplit when bound is not
// finite (the run takes the fp32 form).
int split_exponent(double bound);

// Amplitudes a staged pass with these blocks visits (launch_stage's tile
// choice for this support); 0 when the run does not fit a tile.
uint64_t stage_visits(int nloc, int nops, const int* ks, const int* const* pos, int t_max, uint64_t support, int dtype = 0);

// Contraction over entanglement indices: out[x2 2^n1 + x1] =
// sum_e t1[e 2^n1 + x1] t2[e 2^n2 + x2] (complex64 or complex128).
bool contract_uses_mfma(int dtype, int n1, int n2, int e);
hipError_t launch_contract(hipStream_t st, const void* t1, const void* t2, void* out, int n1, int n2, int e,
                           int dtype, bool split = true);

// Zeroes every amplitude whose index has a bit outside `support`.
hipError_t launch_zero_outside(hipStream_t st, void* psi, int dtype, int nloc, uint64_t support);

// Diagonal op on its own: psi[i] *= table[c(i + idx_offset)].
hipError_t launch_diag(hipStream_t st, void* psi, int dtype, int nloc, uint64_t idx_offset,
                       const DiagSpec& d);

// Out-of-place bit permutation of 2^nbits amplitudes: out[dst(i)] = in[i],
// runs map destination index -> source index (dst-major gather form).
hipError_t launch_bitperm(hipStream_t st, const void* in, void* out, int dtype, int nbits,
                          const BitRuns& dst_to_src);

// Cross-slice accumulation for `count` bitstrings (FP64 accumulators acc,
// device, 2*count doubles).  For every j:
//   phys = runs(x_j)                   (logical bitstring -> physical index)
//   t    = phys >> nloc                (physical slice id of x_j)
//   if tcol == nullptr:  acc[j] += psi_slice[phys & lowmask]  when t == slice
//   else:                acc[j] += tcol[rowmap(t)] * psi_slice[...]  (any t)
// rowmap: 2^s table physical-slice-id -> row index of T (device, int32).
hipError_t launch_accumulate(hipStream_t st, const void* psi_slice, int dtype, int nloc,
                             uint64_t slice, const BitRuns& log_to_phys, int64_t count,
                             const uint64_t* bits, const void* tcol, const int* rowmap,
                             double* acc);

// Deterministic FP64 sum of |psi|^2 over 2^nloc amplitudes: writes
// nblocks partial sums to partial (device), returns the block count used.
hipError_t launch_norm_partials(hipStream_t st, const void* psi, int dtype, int nloc,
                                double* partial, int* nblocks);

// Sum of N |a_j|^2 and of ln(N |a_j|^2) over count FP64 amplitudes, written
// as per-block pairs to partial (2 * nblocks doubles).
hipError_t launch_xeb_partials(hipStream_t st, const double* amps, int64_t count, double logN,
                               double* partial, int* nblocks);

// Fixed-order sum of `count` runs of `width` doubles (single workgroup):
// out[w] = sum_b partial[b * width + w].
hipError_t launch_finish_sum(hipStream_t st, const double* partial, int count, int width,
                             double* out);

}  // namespace sv
