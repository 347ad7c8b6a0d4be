// Internal: the state handle behind the C-ABI's sv_handle (shared by the
// single-state executor and the batch executor).  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "sv_internal.h"

namespace sv {

enum OpKind { OP_DENSE = 0, OP_DIAG = 1, OP_LPERM = 2 };

struct Op {
    int kind = OP_DENSE;
    int k = 0;                 // dense: qubit count; diag: m
    int pos[kMaxDiag] = {};    // physical positions at queue time
    size_t off = 0;            // arena offset of matrix / table
    BitRuns runs;              // OP_LPERM: destination -> source over local bits
    // bound on the factor by which the op can raise the state's norm (its
    // largest singular value) and whether it is unitary within kUnitTol;
    // worked out from the queued data when first needed (size_op)
    double growth = 1.0;
    bool unit = true;
    bool sized = false;
};

// Unitarity tolerance of an op (largest entry of |M^H M - I|): staged runs
// of such blocks may take the split-fp16 form (entries at most ~1, largest
// singular value ~1).
constexpr double kUnitTol = 1e-3;

// Largest-singular-value bound of a k-qubit matrix (row-major complex64 if
// amp == 8, else complex128) and whether it is unitary within kUnitTol.
// Allocates nothing (per-thread buffers).
double op_growth(const void* m, int k, size_t amp, bool* unit);

// Fills op.growth / op.unit from its data in the host arena (once).
void size_op(Op& op, const uint8_t* arena, size_t amp);

// Writes |0...0> into a resident state whose reset was deferred (no-op
// otherwise); on the handle's stream.
int materialize_e0(sv_state* h);

// Device work buffers of a reduction (and the matrices of the queue it
// flushes) taken from caller-provided memory instead of the handle's pool:
// the entry point that allocates nothing hands these in.
struct WorkBufs {
    void* bits;          // count uint64 bitstrings
    void* acc;           // count complex128 accumulators
    void* part;          // kPartDoubles FP64 partial sums
    void* tcol;          // T columns (ns * ns complex128) + ns FP64 slice norms
    void* rowmap;        // ns int
    void* small;         // 8 doubles
    void* arena;         // queued matrices / tables
    size_t arena_cap;
};
constexpr size_t kPartDoubles = 4096 * 2;

// The reduction behind reduce_slices with its work buffers taken from wb
// (nullptr: the handle's own, allocated on demand).
int reduce_with(sv_state* h, const void* trailing, int64_t count, const uint64_t* bits, void* out,
                double* stats, const WorkBufs* wb);

// Staged run starting at ops[i]: consecutive 4/5-qubit dense ops (none with
// a diagonal to fold after it when fold is set) whose positions, with
// positions 0..3, fit a tile of at most stage_t (and nloc, and the device's
// widest) positions within the LDS budget, at most kStageRunMax ops.  Returns the op count (0 when
// ops[i] cannot start one) and their widths in ks.
constexpr int kStageRunMax = 8;
int form_stage_run(const Op* ops, size_t nops, size_t i, int stage_t, int nloc, bool fold, int* ks,
                   int dtype = 0);

}  // namespace sv

struct sv_state {
    using Op = sv::Op;
    int n = 0, s = 0, L = 0, dtype = 0;
    size_t amp = 8;
    uint64_t slice_mask = 0;
    std::vector<int> order, pos;          // order[p] = logical at p; pos[q] = position of q

    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool tier = false;

    // resident storage
    void* dev = nullptr;
    size_t dev_bytes = 0;
    bool own_dev = false;
    void* scratch = nullptr;              // permute target (resident)

    // host tier
    std::vector<void*> files;             // [t * 2^s + u], 2^(L-s) amplitudes each
    bool pinned_tier = true;              // files pinned (hipHostMalloc) or pageable (mmap)
    bool store32 = false;                 // complex128 state whose files hold complex64
    int famp = 8;                         // bytes per amplitude in the files
    std::vector<int> file_fds;            // file-backed tier: one open file per logical file
    std::vector<std::string> file_paths;  //   (removed when the handle is destroyed)
    std::vector<void*> file_maps;         //   and where each is mapped (files[] gets relabelled)
    std::string tier_dir;                 // their directory (checkpoint metadata lives there too)
    bool keep_files = false;              // destroy keeps the files and the checkpoint
    std::vector<uint8_t> slice_zero;      // slice known to be all zero
    std::vector<void*> slots;             // device slice buffers
    void* pslot = nullptr;                // device buffer for local permutes
    hipStream_t s_in = nullptr, s_out = nullptr;
    std::vector<hipEvent_t> ev_in, ev_comp, ev_out;

    // operation queue
    std::vector<Op> ops;
    std::vector<uint8_t> arena;
    void* d_arena = nullptr;
    size_t d_arena_cap = 0;
    const void* d_arena_use = nullptr;    // where the last upload put the queue's matrices
    void* h_arena = nullptr;
    size_t h_arena_cap = 0;
    hipEvent_t ev_arena = nullptr;

    // reduction work buffers
    void* d_bits = nullptr;  size_t d_bits_cap = 0;
    void* d_acc = nullptr;   size_t d_acc_cap = 0;
    void* d_part = nullptr;  size_t d_part_cap = 0;
    void* d_tcol = nullptr;  size_t d_tcol_cap = 0;
    void* d_rowmap = nullptr; size_t d_rowmap_cap = 0;
    void* d_small = nullptr;              // 8 doubles

    // options and accounting
    bool timing = false, fold = true;
    int mfma_min_k = 4;
    int stage_t = 13;            // widest tile of staged multi-block passes (0: off)
    bool split = true;           // staged passes in the split-fp16 form where the amplitude bound allows
    bool e0_pending = false;     // resident state is |0...0> but not yet written (sv_reset)
    // Resident states after sv_reset: every amplitude whose index has a bit
    // outside `support` is zero (the positions no operation has touched since
    // the reset), and while `garbage` is set the memory there may still hold
    // older values.  Staged passes visit only the tiles inside the support.
    uint64_t support = ~0ull;
    bool garbage = false;
    bool sparse_start = true;
    int64_t fail_io_at = 0;               // failure injection: remaining transfers before a forced SV_EIO
    int nslots = 3;
    std::vector<hipEvent_t> tev_pool;
    struct TimedLaunch {
        int kind;           // 0 single sweep, 1 staged pass
        double flops;       // algorithmic: (8 2^k - 2) per amplitude per block
        double issued;      // as executed: 6 2^k (3M, matrix cores) or 8 2^k (vector units)
        double bytes;       // HBM bytes the launch must move: amplitudes read + written
    };
    std::vector<TimedLaunch> tev_info;              // per event pair
    size_t tev_used = 0;
    double t_ms = 0.0;
    int64_t t_count = 0;
    double tk_ms[2] = {0.0, 0.0};                   // by kind: single sweeps, staged passes
    int64_t tk_count[2] = {0, 0};
    double tk_flops[2] = {0.0, 0.0};
    double tk_issued[2] = {0.0, 0.0};
    double tk_bytes[2] = {0.0, 0.0};
    int64_t counters[8] = {};
    // bound on the norm of the amplitudes in memory (so on every
    // |amplitude|), before the queued ops: 1 after creation or sv_reset,
    // times each applied op's growth; infinite once the device buffer has
    // been handed out or when a restored tier does not state it
    double amp_bound = 1.0;
    int64_t stage_forms[2] = {};  // staged passes run in the split-fp16 / fp32 form

    bool poisoned = false;
    std::string err;
};

