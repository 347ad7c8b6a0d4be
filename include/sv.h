/*
 * libsv -- sliced state-vector contraction on one MI355X (gfx950).
 *
 * C-ABI of the hot path of the tensor-contraction-deferral simulator of
 * Pednault et al., "Leveraging Secondary Storage to Simulate Deep 54-qubit
 * Sycamore Circuits": Schroedinger-style evolution of one subcircuit slice's
 * amplitude tensor (Sec. 2), with gates aggregated into dense k-qubit blocks
 * (Sec. 5, aggregate gates of at most 5 qubits), diagonal (hyperedge) gates
 * applied as element-wise phases (Sec. 2, diagonal and separable tensors),
 * index permutes that re-choose the sliced ("global") qubits (Sec. 4, the
 * local/global reorganisation between subcircuits), slices staged to a
 * secondary tier (Sec. 4, logical files read and written whole), and the
 * accumulation of amplitudes across slices (Sec. 2, tensor slicing).
 *
 * Conventions
 *   - Qubits are logical labels 0..n-1.  A bitstring / amplitude index has
 *     bit q = value of qubit q (little-endian).
 *   - A k-qubit matrix on qubits (q_0, ..., q_{k-1}) is row-major 2^k x 2^k
 *     with row/column index c = sum_j b(q_j) 2^j.
 *   - The library keeps a logical-to-physical layout.  The top s =
 *     popcount(slice_mask) physical positions are the sliced qubits; a slice
 *     is one fixed assignment of them and holds 2^(n-s) amplitudes.
 *   - Matrices and phase tables are passed in the state's dtype: interleaved
 *     (re, im) float pairs for SV_C64, double pairs for SV_C128.  Outputs of
 *     gather/reduce are always complex128 (double pairs).
 *
 * Return values: SV_OK (0) or a negative SV_E* code.  No call throws or
 * aborts.  Argument errors are detected before anything is queued and leave
 * the state unchanged.  A device or transfer error poisons the handle: every
 * later call on it returns SV_ESTATE until destroy_state.  last_error()
 * describes the most recent failure.
 *
 * Ordering and ownership: apply_fused / apply_diag validate, copy their
 * inputs and queue the operation; the caller may free its buffers on return.
 * Queued operations run, in order, on the handle's HIP stream at the next
 * permute_qubits, gather_amplitudes, reduce_slices or sync_state (or when the
 * queue is large).  gather_amplitudes and reduce_slices return complete host
 * results.  One host thread may use a handle at a time; different handles are
 * independent.  Identical call sequences give bitwise identical results.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SV_OK = 0,
    SV_EINVAL = -1,   /* bad argument (qubit out of range, duplicate, NULL, k out of range) */
    SV_ENOMEM = -2,   /* device or pinned-host allocation failed */
    SV_EDEVICE = -3,  /* HIP runtime or kernel error (handle poisoned) */
    SV_ESLICED = -4,  /* non-diagonal operation on a sliced qubit */
    SV_ESTATE = -5,   /* handle poisoned by an earlier device/transfer error */
    SV_EIO = -6       /* slice staging to / from the host tier failed (handle poisoned) */
};

enum { SV_C64 = 0, SV_C128 = 1 };

/* Flags OR-ed into the dtype argument of create_state. */
enum {
    SV_FLAG_TIER = 0x100,     /* keep slices in the host tier even if they fit in HBM */
    SV_FLAG_PAGEABLE = 0x400, /* host tier in pageable memory even if it would fit the
                                 pinned budget (48 GiB; larger tiers are pageable) */
    SV_FLAG_STORE32 = 0x800   /* SV_C128 only: the host tier (implied) stores single
                                 precision, 8 bytes per amplitude, while the device
                                 computes in double (Sec. 5: storage in single precision,
                                 in-memory calculations in double); every write to the
                                 tier rounds the amplitudes to complex64 */
};

typedef struct sv_state* sv_handle;

/*
 * create_state -- allocate an n-qubit state |0...0> (Sec. 2: each qubit
 * starts in |0>).  slice_mask selects the sliced qubits (Sec. 2, tensor
 * slicing; Sec. 4, global qubits); they take the top physical positions in
 * ascending label order, the rest take positions 0.. in ascending order.
 * dtype: SV_C64 or SV_C128, optionally | SV_FLAG_TIER.  hip_stream: a
 * hipStream_t to run on, or NULL for a stream owned by the handle.
 * If the whole state fits in device memory all slices are resident in one
 * HBM buffer; otherwise (or with SV_FLAG_TIER) slices live in host memory
 * (pinned up to 48 GiB, pageable beyond) and are staged through device
 * slots.  n in [1, 40], s <= 12; the tier needs n >= 2s.
 * Errors: SV_EINVAL, SV_ENOMEM, SV_EDEVICE.  *out is set only on success.
 */
int create_state(int n, uint64_t slice_mask, int dtype, void* hip_stream, sv_handle* out);

/*
 * create_state_ext -- as create_state, but the amplitudes live in the
 * caller's device buffer dev_buf (at least 2^n amplitudes of the dtype,
 * e.g. a torch tensor), which the handle neither frees nor reallocates.
 * The buffer is initialised to |0...0> unless dtype has SV_FLAG_KEEP set, in
 * which case its current contents (in the initial layout) are the state.
 * All slices are resident.  Errors: SV_EINVAL (buffer NULL, too small or
 * not 16-byte aligned).
 */
enum { SV_FLAG_KEEP = 0x200 };
int create_state_ext(int n, uint64_t slice_mask, int dtype, void* hip_stream,
                     void* dev_buf, size_t bytes, sv_handle* out);

/*
 * create_state_files -- as create_state with SV_FLAG_TIER, but the host tier
 * lives in files on a file system (Sec. 4: the slices of the state go to
 * secondary storage, each logical file written and read whole; App. A,
 * the "write" and "read" modes): one file per logical file, created in
 * directory dir (which must exist and be writable), memory-mapped shared,
 * so the page cache moves the data to and from storage, and removed by
 * destroy_state.  The state needs 1 <= s <= n/2 sliced qubits; the files
 * hold 2^(n-s) amplitudes in total.  Errors: SV_EINVAL (dir NULL or empty,
 * bad sizes), SV_EIO (a file cannot be created, sized or mapped),
 * SV_ENOMEM, SV_EDEVICE.
 */
int create_state_files(int n, uint64_t slice_mask, int dtype, void* hip_stream, const char* dir,
                       sv_handle* out);

/*
 * sv_checkpoint -- make a state whose host tier lives in files a restart
 * point (Sec. 4: each phase ends with every logical file written whole to
 * secondary storage, so the files are a complete copy of the state): every
 * queued operation is applied and written back, the files are flushed to
 * storage, and a small metadata file (sv_checkpoint.meta: sizes, layout,
 * slices known to be zero, file names, and the caller's tag, e.g. the index
 * of the next phase) replaces the previous one atomically.  Errors:
 * SV_EINVAL (the tier is not in files), SV_EIO, SV_EDEVICE.
 *
 * open_state_files -- a new handle on the state of the last checkpoint in
 * dir: the existing files, mapped shared, with the checkpoint's layout;
 * *tag receives its tag (tag may be NULL).  The new handle owns the files
 * (destroy_state removes them and the metadata unless SV_OPT_KEEP_FILES).
 * Errors: SV_EINVAL (dir or out NULL, malformed metadata), SV_EIO (no
 * checkpoint, a file missing or of the wrong size), SV_ENOMEM, SV_EDEVICE.
 */
int sv_checkpoint(sv_handle h, int64_t tag);
int open_state_files(const char* dir, void* hip_stream, sv_handle* out, int64_t* tag);

/* destroy_state -- wait for queued work, free everything the handle owns.
   Accepts a poisoned handle; NULL is a no-op.  */
int destroy_state(sv_handle h);

/*
 * apply_fused -- queue a dense k-qubit block (Sec. 5: gates aggregated into a
 * k-qubit kernel represented by a 2^k x 2^k unitary), 1 <= k <= 6 for SV_C64,
 * 1 <= k <= 5 for SV_C128; every qubit must be unsliced.  qubits: k distinct logical labels; matrix:
 * row-major 2^k x 2^k in the state dtype (need not be unitary).
 * Errors: SV_EINVAL; SV_ESLICED if a qubit is currently sliced.
 */
int apply_fused(sv_handle h, int k, const int* qubits, const void* matrix);

/*
 * apply_diag -- queue a diagonal gate on m qubits (Sec. 2: a diagonal tensor
 * is a hyperedge; it mixes no amplitudes): psi[i] *= phases[c(i)],
 * c(i) = sum_j b_{q_j}(i) 2^j.  1 <= m <= 12.  Sliced qubits are allowed:
 * their bits come from the slice being processed.  Errors: SV_EINVAL.
 */
int apply_diag(sv_handle h, int m, const int* qubits, const void* phases);

/*
 * apply_ops -- queue a planned sequence of operations in one call (Sec. 5:
 * a subcircuit runs as its list of aggregate kernels, applied in order;
 * App. A: the listing gives each subcircuit as such a list of rows).
 * Operation i is kinds[i] = SV_OP_FUSED (as apply_fused) or SV_OP_DIAG (as
 * apply_diag) on widths[i] qubits.  qubits: the operations' qubit lists,
 * concatenated; data: their matrices (2^k x 2^k, row-major) or phase tables
 * (2^m entries), concatenated, in the state dtype with no padding.  Every
 * operation is validated before any is queued: on an error nothing is
 * queued.  Inputs are copied; the caller may free them on return.
 * Errors: SV_EINVAL (count < 0, a NULL array with count > 0, an unknown
 * kind, or any error apply_fused / apply_diag would report), SV_ESLICED.
 */
enum { SV_OP_FUSED = 0, SV_OP_DIAG = 1 };
int apply_ops(sv_handle h, int count, const int* kinds, const int* widths, const int* qubits,
              const void* data);

/*
 * permute_qubits -- choose a new layout (Sec. 4: switching subcircuits
 * reorganises which indices are local and which are global; the listing's
 * all2all rows give the new index order).  order[p] = logical qubit placed
 * at physical position p (p = 0 least significant); the top s positions
 * become the sliced qubits.  Flushes queued work.  Results of later calls
 * are unaffected (operations address logical qubits).  For a resident state
 * the library allocated, the re-laid-out amplitudes may end up in another
 * buffer of the handle (sv_device_buffer gives the current one); a state in
 * a caller's buffer (create_state_ext) keeps it.  A resident state
 * that is still |0...0> with nothing queued (after sv_reset, or created and
 * not yet operated on) only takes the new layout: no data moves.  Choosing
 * the layout there decides which positions the first operations touch.
 * Errors: SV_EINVAL (not a permutation), SV_ENOMEM (no room for the
 * re-arrangement), SV_EDEVICE / SV_EIO (handle poisoned).
 */
int permute_qubits(sv_handle h, const int* order);

/*
 * gather_amplitudes -- flush, then out[j] = psi[bitstrings[j]] as complex128
 * for j < count (bit q of a bitstring = qubit q; must be < 2^n).  out is a
 * host buffer of 2*count doubles.  Errors: SV_EINVAL (bitstring >= 2^n or
 * NULL with count > 0), SV_EDEVICE.
 */
int gather_amplitudes(sv_handle h, int64_t count, const uint64_t* bitstrings, void* out_c128);

/*
 * reduce_slices -- flush, then accumulate across slices in FP64 (Sec. 2:
 * iterating over the slices and summing their contributions):
 *     out[j] = sum_t T[r(x_j), t] * psi_t(x_j with its sliced bits set to t)
 * where r(x) is x's sliced bits and t runs over the 2^s slices; bit i of r
 * and t belongs to the i-th sliced qubit in ascending label order.
 * trailing_c128: host 2^s x 2^s row-major complex128 T, or NULL for the
 * identity (then out[j] = psi[x_j]).  T lets the last gates on sliced qubits
 * be applied in the reduction instead of by a permute.
 * stats (may be NULL): [0] = sum over all amplitudes of |psi|^2 (before T),
 * [1] = sum_j N |out[j]|^2, [2] = sum_j ln(N |out[j]|^2), N = 2^n, all FP64.
 * Errors as gather_amplitudes.
 */
int reduce_slices(sv_handle h, const void* trailing_c128, int64_t count,
                  const uint64_t* bitstrings, void* out_c128, double stats[3]);

/*
 * reduce_slices_noalloc -- reduce_slices for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * reduce_slices, but no device or pinned memory is allocated or freed: the
 * work buffers of the reduction and the device copy of the queued matrices
 * live in one fixed device array of the library (about 32 MiB, held on each
 * GPU the library runs on until the process ends).  Limits: a resident
 * state (not the host tier), SV_OPT_TIMING off, count <=
 * SV_NOALLOC_MAX_BITSTRINGS, at most SV_NOALLOC_MAX_SLICED sliced qubits,
 * queued matrices and tables of at most SV_NOALLOC_MAX_QUEUED_BYTES; beyond
 * them: SV_EINVAL, nothing run.  All calls on one GPU share the array: the
 * library lets one such call per GPU run at a time (calls from other
 * threads wait), and the array keeps nothing from one call to the next.
 * The state itself must have been created beforehand (creation allocates).
 */
enum {
    SV_NOALLOC_MAX_BITSTRINGS = 1 << 20,
    SV_NOALLOC_MAX_SLICED = 6,
    SV_NOALLOC_MAX_QUEUED_BYTES = 8 << 20
};
int reduce_slices_noalloc(sv_handle h, const void* trailing_c128, int64_t count,
                          const uint64_t* bitstrings, void* out_c128, double stats[3]);

/* sync_state -- run everything queued and wait for it.  */
int sync_state(sv_handle h);

/* sv_reset -- drop queued operations and set the state back to |0...0>
   (the layout is kept; |0...0> is index 0 in every layout).  Reuses the
   handle's memory: nothing is allocated.  For a resident state the write
   is deferred: the first staged pass builds its input from |0...0>
   without reading HBM, and any other first use writes |0...0> first.
   Until every qubit position has been touched, staged passes visit only
   the tiles that can be non-zero (SV_OPT_SPARSE_START); the state is
   complete in memory again when the queue has run (sync_state, reads). */
int sv_reset(sv_handle h);

/* last_error -- text of the most recent failure on h (or of the last failed
   create or sv_contract when h is NULL).  Valid until the next call on the same handle. */
const char* last_error(sv_handle h);

/* ---- introspection and tuning (not part of the paper's operation set) ---- */

/* Current layout: order[p] = logical qubit at physical position p. */
int sv_get_order(sv_handle h, int* order);

/* Copy of the raw device amplitude buffer pointer (resident states) and its
   size in bytes; *dev = NULL for tiered states. */
int sv_device_buffer(sv_handle h, void** dev, size_t* bytes);

enum {
    SV_OPT_TIMING = 1,     /* 1: time every dense sweep with HIP events on the handle's stream */
    SV_OPT_MFMA = 2,       /* smallest k (4..6) whose complex64 blocks run on the matrix
                              cores (default 4); 0 or > 6: never */
    SV_OPT_FOLD_DIAG = 3,  /* 1 (default): fold a diagonal op into the preceding dense sweep */
    SV_OPT_SLOTS = 4,      /* tier: number of device slice slots (>= 2) */
    SV_OPT_STAGE = 5,      /* widest LDS tile (9..14 positions, default 13) for running a
                              run of consecutive 4/5-qubit blocks in one pass over HBM
                              (complex64: 14 = one workgroup per CU, 1024 lanes in the split
                              form and 512 in the fp32 form, holding the
                              whole LDS; a pass widens its tile with free positions
                              to the widest width the LDS holds for its blocks'
                              matrices; in the split-fp16 form 14 measured fastest
                              for states of 2^23 to 2^30 amplitudes, in the fp32 form
                              13 at 2^30; complex128: one 512-lane workgroup per CU, tiles
                              of at most 13 positions, products on the FP64 matrix
                              cores); 0: one pass per block; other values: SV_EINVAL */
    SV_OPT_FAIL_IO = 6,    /* failure injection for tests: the n-th host-tier transfer
                              from now on (n >= 1) is not issued and reports SV_EIO,
                              poisoning the handle; 0 (default): off */
    SV_OPT_KEEP_FILES = 8,  /* states whose tier is in files: 1 = destroy_state keeps the
                              files and the checkpoint (so a later open_state_files
                              can resume); 0 (default) = they are removed */
    SV_OPT_SPLIT = 9,       /* 1 (default): a staged pass runs its complex64 products on
                              the fp16 matrix cores with single-precision accuracy
                              (each fp32 operand split into two fp16 parts, fp32
                              accumulation, the tile scaled by a power of two taken
                              from the state's amplitude bound, see sv_stage_forms)
                              when every block of the pass is unitary within 1e-3
                              (largest entry of |M^H M - I|) and the bound is
                              finite; otherwise, or with 0, on the fp32 matrix
                              cores.  A batch takes the form at sv_batch_prepare, in
                              its variant run from a reset only. */
    SV_OPT_SPARSE_START = 7 /* 1 (default): a resident state created as |0...0> or
                              reset with sv_reset is non-zero only on index bits some
                              operation has targeted since; staged passes visit only
                              the tiles inside them and widen their tile with them
                              only; after a reset the rest is zero-filled before the
                              amplitudes are read.  0: every pass visits the whole
                              state.  Takes effect at the next sv_reset. */
};
int sv_set_option(sv_handle h, int option, int64_t value);

/*
 * sv_counters -- work done since creation: [0] dense sweeps (HBM passes),
 * [1] diagonal sweeps, [2] permute sweeps, [3] amplitudes touched by sweeps
 * (staged passes: the amplitudes they visit),
 * [4] bytes staged host->device, [5] bytes staged device->host, [6] slices
 * skipped because they are known to be zero, [7] blocks applied in staged
 * multi-block passes.
 * sv_sweep_time -- with SV_OPT_TIMING: total milliseconds and count of timed
 * dense sweeps (HIP events on the handle's stream), reset by the call.
 */
int sv_counters(sv_handle h, int64_t counters[8]);

/*
 * sv_stage_forms -- staged multi-block passes run since creation in the
 * split-fp16 form (passes[0]) and in the fp32 form (passes[1]), and the
 * state's amplitude bound: an upper bound on its norm, so on every
 * |amplitude|, kept on the host.  It is 1 after creation and sv_reset, is
 * multiplied by each queued op's growth (a bound on its largest singular
 * value: the square root of the largest absolute row sum of M^H M; for a
 * diagonal op its largest |entry|), and becomes infinite when
 * sv_device_buffer hands out the amplitudes (the caller may write them) or
 * when open_state_files restores a checkpoint that does not state it, or
 * create_state_ext adopts the caller's amplitudes (SV_FLAG_KEEP).  A
 * resident state with an unknown bound gets one from its norm, measured on
 * the device when its next queue holds 4/5-qubit complex64 blocks (one read
 * pass and a wait on the handle's stream).  The split form scales the tile
 * by the largest power of two 2^e with 2^e * bound <= 2^15, so amplitudes
 * stay in fp16 range (Sec. 5 computes in single precision; the split keeps
 * that accuracy).  A batch counts its passes at sv_batch_prepare, in the
 * form of its variant run from a reset.  Either pointer may be NULL.
 */
int sv_stage_forms(sv_handle h, int64_t passes[2], double* amp_bound);
int sv_sweep_time(sv_handle h, double* total_ms, int64_t* count);

/* sv_sweep_profile -- with SV_OPT_TIMING: the timed launches split by kind,
 * [0] single dense sweeps, [1] staged multi-block passes: total
 * milliseconds, launch count, algorithmic flops (a k-qubit block is a
 * complex 2^k-term dot product per amplitude: 8 2^k - 2 flops), the flops
 * the kernels issued (6 2^k per amplitude per complex64 block on the
 * fp32 matrix cores, 3 real products; 24 2^k on the fp16 matrix cores in
 * the split form, 4 real products of 3 split terms; 8 2^k on the vector
 * units) and the HBM
 * bytes the launches had to move (amplitudes read and written; after
 * sv_reset a staged pass visits only the amplitudes that can be non-zero,
 * reads none from |0...0> and none on positions no operation has reached).
 * Flops count the amplitudes visited.  Resets the same accumulators as
 * sv_sweep_time.  Any pointer may be NULL. */
int sv_sweep_profile(sv_handle h, double ms[2], int64_t count[2], double flops[2], double issued[2],
                     double bytes[2]);

/* ---- batches of independent states ----------------------------------------
 * Many circuits of different qubit counts run as one recorded execution: the
 * queued operations of each state (its plan) are taken over, sweep r of every
 * state goes into round r, and each round is one launch per kernel form
 * (matrix-core / VALU), block width k and fold flag, whose workgroups are
 * divided among the states in proportion to their size.  With
 * SV_BATCH_GRAPH all rounds are captured into one HIP graph, so a batch is
 * one graph launch and can be replayed (e.g. after sv_reset of every state).
 * A second variant (and graph) serves launches where every state was reset
 * since its last use (SV_OPT_SPARSE_START on): staged passes start from
 * |0...0> and visit only the tiles that can be non-zero, |0...0> is written
 * only ahead of a plain sweep, and what no pass reached is cleared at the
 * end.  A state's own operation order is kept; results are bitwise
 * identical to running the same operations on the state alone.
 *
 * sv_batch_prepare -- handles: `count` distinct resident states of one dtype
 *   (HBM, not tiered) with no queued permutes; their queues are emptied.
 *   hip_stream: stream for the batch (NULL: owned).  The states must outlive
 *   the batch.  Errors: SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_ESTATE.
 * sv_batch_launch  -- enqueue the batch after the work already queued on the
 *   states' streams; later work on those streams waits for it.  Asynchronous.
 *   Runs the reset variant when every state is reset and not yet used.
 *   SV_EINVAL if a state has queued operations or was permuted since the
 *   batch was prepared (the recorded launches address its old layout).
 * sv_batch_sync    -- wait for the last launch.
 * sv_batch_info    -- [0] launches per run, [1] sweeps per run, [2]
 *   amplitudes the sweeps visit per run, [3] 1 if captured in a graph;
 *   [0] and [2] for the variant launched last (before any launch: the
 *   ordinary one).
 * sv_batch_destroy -- free the batch (not the states).
 * sv_batch_error   -- text of the last batch failure (b may be NULL).
 */
typedef struct sv_batch_s* sv_batch;
enum { SV_BATCH_GRAPH = 1 };
int sv_batch_prepare(int count, sv_handle* handles, int flags, void* hip_stream, sv_batch* out);
int sv_batch_launch(sv_batch b);
int sv_batch_sync(sv_batch b);
int sv_batch_info(sv_batch b, int64_t info[4]);
int sv_batch_destroy(sv_batch b);
const char* sv_batch_error(sv_batch b);

/* ---- contraction deferral ---------------------------------------------------
 * sv_contract -- the contraction that eliminates entanglement indices (App.
 *   A, the equation summing phi' chi' over the indices a', a introduced by
 *   the EI and E2Q synthesized gates; Sec. 2, contraction deferral: sum over
 *   the shared indices, outer product over the others), for two tensors
 *   that share e entanglement indices:
 *       out[x2 * 2^n1 + x1] = sum_{c < 2^e} t1[c * 2^n1 + x1] * t2[c * 2^n2 + x2].
 *   t1: device buffer of 2^(n1+e) amplitudes whose index bits n1.. are the
 *   entanglement indices (e.g. a state permuted so that they sit at the top
 *   positions); t2 likewise with n2 open bits and the same entanglement
 *   indices in the same order; out: device buffer of 2^(n1+n2) amplitudes
 *   (caller-owned, overwritten, not overlapping the inputs).  dtype SV_C64
 *   (FP32 sums, on the matrix cores when 2^n2 >= 128, 2^n1 >= 64 and
 *   2^e >= 16: by default on the fp16 matrix cores at single-precision
 *   accuracy, each tensor scaled by a power of two from its largest
 *   |component| and every value split into two fp16 parts, with two 8-byte
 *   words of stream-ordered device memory for the scales; | SV_CONTRACT_FP32
 *   for the 3M form on the fp32 matrix cores) or SV_C128 (FP64 sums).  All
 *   buffers 16-byte aligned.
 *   hip_stream: stream to run on (NULL: the null stream); asynchronous.
 *   Errors: SV_EINVAL (NULL or misaligned buffer, e above 30, n1 + n2, n1 + e
 *   or n2 + e above 40, overlap), SV_EDEVICE; the text is last_error(NULL). */
enum { SV_CONTRACT_FP32 = 0x1000 };
int sv_contract(const void* t1, const void* t2, void* out, int n1, int n2, int e, int dtype, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SV_H */
