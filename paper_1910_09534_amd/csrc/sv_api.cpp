// C-ABI of libsv: handles, argument checks, the operation queue and its
// executor, slicing with a pinned host tier, permutes, gathers and the
// cross-slice FP64 reduction.  See include/sv.h for the contract.
//
// Layout.  Physical bit positions of an n-qubit state: [0, L) are local
// (L = n - s), [L, n) are sliced.  A slice t holds the 2^L amplitudes whose
// sliced bits equal t.  In the host tier the top s local positions
// [L - s, L) form the "file" index (Sec. 4: the logical files are indexed by
// the union of the two alternating slice sets and always read or written
// whole): slice t is 2^s files of 2^(L - s) amplitudes, and re-choosing the
// sliced qubits among the 2s top positions only relabels files.
#include <fcntl.h>
#include <hip/hip_runtime.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <deque>
#include <new>
#include <thread>
#include <cctype>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sv.h"
#include "sv_internal.h"
#include "sv_state.h"

using namespace sv;

double sv::op_growth(const void* m, int k, size_t amp, bool* unit)
{
    // G = M^H M (Hermitian: the upper triangle, in fp32, is enough for a
    // tolerance of 1e-3); ||M||_2^2 = lambda_max(G) <= max_r sum_c |G_rc|
    constexpr int DM = 1 << kMaxDense;
    thread_local float re[DM * DM], im[DM * DM], gr[DM * DM], gi[DM * DM];
    thread_local double row[DM];
    const int D = 1 << k;
    for (size_t i = 0; i < (size_t)D * D; ++i) {
        if (amp == 8) {
            re[i] = ((const float*)m)[2 * i];
            im[i] = ((const float*)m)[2 * i + 1];
        } else {
            re[i] = (float)((const double*)m)[2 * i];
            im[i] = (float)((const double*)m)[2 * i + 1];
        }
        gr[i] = gi[i] = 0.f;
    }
    for (int x = 0; x < D; ++x) {
        const float* ar = &re[(size_t)x * D];
        const float* ai = &im[(size_t)x * D];
        for (int r = 0; r < D; ++r) {
            const float cr = ar[r], ci = -ai[r];
            float* pr = &gr[(size_t)r * D];
            float* pi = &gi[(size_t)r * D];
            for (int c = r; c < D; ++c) {
                pr[c] += cr * ar[c] - ci * ai[c];
                pi[c] += cr * ai[c] + ci * ar[c];
            }
        }
    }
    for (int r = 0; r < D; ++r) row[r] = 0.0;
    double dev = 0.0;
    for (int r = 0; r < D; ++r)
        for (int c = r; c < D; ++c) {
            const double a = std::hypot((double)gr[(size_t)r * D + c], (double)gi[(size_t)r * D + c]);
            row[r] += a;
            if (c != r) row[c] += a;
            const double d = c == r ? std::hypot((double)gr[(size_t)r * D + c] - 1.0, (double)gi[(size_t)r * D + c]) : a;
            dev = std::max(dev, d);
        }
    double worst = 0.0;
    for (int r = 0; r < D; ++r) worst = std::max(worst, row[r]);
    if (unit) *unit = dev <= kUnitTol;
    // not finite (NaN / inf entries): no bound
    return std::isfinite(worst) ? std::sqrt(worst) : HUGE_VAL;
}

void sv::size_op(Op& op, const uint8_t* arena, size_t amp)
{
    if (op.sized) return;
    op.sized = true;
    if (op.kind == OP_DENSE) {
        op.growth = op_growth(arena + op.off, op.k, amp, &op.unit);
    } else if (op.kind == OP_DIAG) {
        // a diagonal op scales amplitudes by its entries
        double lo = HUGE_VAL, hi = 0.0;
        for (size_t i = 0; i < ((size_t)1 << op.k); ++i) {
            const double a = amp == 8 ? std::hypot((double)((const float*)(arena + op.off))[2 * i],
                                                   (double)((const float*)(arena + op.off))[2 * i + 1])
                                      : std::hypot(((const double*)(arena + op.off))[2 * i],
                                                   ((const double*)(arena + op.off))[2 * i + 1]);
            lo = std::min(lo, a);
            hi = std::max(hi, a);
        }
        op.growth = std::isfinite(hi) ? hi : HUGE_VAL;
        op.unit = hi - 1.0 <= kUnitTol && 1.0 - lo <= kUnitTol;
    }
}

namespace {

thread_local std::string g_create_error;

}  // namespace

namespace {

int set_err(sv_state* h, int code, const std::string& msg)
{
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

int fail_dev(sv_state* h, const char* what, hipError_t e, int code = SV_EDEVICE)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (h) {
        h->poisoned = true;
        h->err = m;
    } else {
        g_create_error = m;
    }
    return code;
}

#define TRY(h, expr)                                                 \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return fail_dev((h), #expr, e_);       \
    } while (0)

#define TRY_IO(h, expr)                                              \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return fail_dev((h), #expr, e_, SV_EIO); \
    } while (0)

#define CHECK_HANDLE(h)                                                          \
    do {                                                                         \
        if (!(h)) return set_err(nullptr, SV_EINVAL, "NULL handle");              \
        if ((h)->poisoned) return SV_ESTATE;                                     \
    } while (0)

int ensure_dev(sv_state* h, void** p, size_t* cap, size_t need)
{
    if (*cap >= need) return SV_OK;
    if (*p) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail_dev(h, "hipStreamSynchronize", e);
        pool_free(*p, *cap, false);
        *p = nullptr;
        *cap = 0;
    }
    size_t got = 0;
    *p = pool_alloc(std::max(need, (size_t)4096), false, &got);
    if (!*p) return set_err(h, SV_ENOMEM, "device allocation of work buffer failed");
    *cap = got;
    return SV_OK;
}

int check_qubit_list(sv_state* h, int k, const int* q, int kmax)
{
    if (!q) return set_err(h, SV_EINVAL, "qubit list is NULL");
    if (k < 1 || k > kmax) return set_err(h, SV_EINVAL, "qubit count out of range");
    for (int j = 0; j < k; ++j) {
        if (q[j] < 0 || q[j] >= h->n) return set_err(h, SV_EINVAL, "qubit label out of range");
        for (int l = 0; l < j; ++l)
            if (q[l] == q[j]) return set_err(h, SV_EINVAL, "duplicate qubit label");
    }
    return SV_OK;
}

size_t push_arena(sv_state* h, const void* src, size_t bytes)
{
    size_t off = (h->arena.size() + 255) & ~(size_t)255;
    h->arena.resize(off + bytes);
    std::memcpy(h->arena.data() + off, src, bytes);
    return off;
}

// ---- timing of dense sweeps ----------------------------------------------
hipEvent_t next_event(sv_state* h)
{
    if (h->tev_used == h->tev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->tev_pool.push_back(e);
    }
    return h->tev_pool[h->tev_used++];
}

int collect_timing(sv_state* h)
{
    if (h->tev_used == 0) return SV_OK;
    TRY(h, hipEventSynchronize(h->tev_pool[h->tev_used - 1]));
    for (size_t i = 0; i + 1 < h->tev_used; i += 2) {
        float ms = 0.f;
        TRY(h, hipEventElapsedTime(&ms, h->tev_pool[i], h->tev_pool[i + 1]));
        h->t_ms += ms;
        h->t_count += 1;
        const auto& info = h->tev_info[i / 2];
        h->tk_ms[info.kind] += ms;
        h->tk_count[info.kind] += 1;
        h->tk_flops[info.kind] += info.flops;
        h->tk_issued[info.kind] += info.issued;
        h->tk_bytes[info.kind] += info.bytes;
    }
    h->tev_used = 0;
    h->tev_info.clear();
    return SV_OK;
}

// Arithmetic of one dense k-qubit block per amplitude.  Algorithmic: a
// complex 2^k-term dot product per output, 8 2^k - 2 flops.  Issued: 6 2^k
// in the matrix-core form (three real products), 8 2^k on the vector units
// (complex multiply-adds).
static double block_flops_alg(int k)
{
    return 8.0 * (double)(1 << k) - 2.0;
}

static double block_flops_issued(int dtype, int k, int nloc, int mfma_min_k)
{
    const double d = (double)(1 << k);
    if (dtype == 0 && dense_uses_mfma(k, nloc, mfma_min_k)) return 6.0 * d;
    return 8.0 * d;
}

// ---- deferred reset --------------------------------------------------------
// sv_reset leaves a resident state marked |0...0> without writing it; the
// first staged pass then builds its tiles from |0...0> instead of reading
// HBM, and anything else that needs the amplitudes writes them first.
// Until every position has been touched, staged passes skip the tiles that
// are still zero (the support, in sv_state), so the memory there is written
// here before anything else reads it.
int materialize_state(sv_state* h)
{
    if (h->e0_pending) {
        h->e0_pending = false;
        h->garbage = false;
        TRY(h, launch_init(h->stream, h->dev, h->dtype, (uint64_t)1 << h->n, true));
        return SV_OK;
    }
    if (h->garbage) {
        h->garbage = false;
        TRY(h, launch_zero_outside(h->stream, h->dev, h->dtype, h->n, h->support));
    }
    return SV_OK;
}

// ---- running the queue over one range of amplitudes ----------------------
// psi: 2^nloc amplitudes whose global index starts at idx_offset.
// norm_out (resident states): when the queue ends with a staged run, that
// pass also writes per-workgroup FP64 sums of |psi|^2 there and
// *norm_blocks receives their count (else 0).
int run_ops(sv_state* h, hipStream_t st, void** psi, void* alt, int nloc, uint64_t idx_offset,
            double* norm_out = nullptr, int* norm_blocks = nullptr)
{
    if (norm_blocks) *norm_blocks = 0;
    const char* dbase = (const char*)h->d_arena_use;
    const size_t nops = h->ops.size();
    // the amplitude bound before op i (ops are sized as they are reached,
    // so the host work overlaps the launches already queued)
    double bnd = h->amp_bound;
    for (size_t i = 0; i < nops; ++i) {
        const Op& op = h->ops[i];
        // a run of consecutive 4/5-qubit complex64 blocks whose targets fit in
        // one LDS tile goes through a single staged HBM pass
        // (complex64 with the matrix-core sweeps on from k = 4; complex128
        // always: its single sweeps run on the vector units)
        const int stage_t = h->stage_t;
        if (op.kind == OP_DENSE && stage_t >= 9 && (h->dtype != 0 || h->mfma_min_k == 4) &&
            (op.k == 4 || op.k == 5)) {
            int ks[kStageRunMax];
            const int* pp[kStageRunMax];
            const void* mm[kStageRunMax];
            const int cnt = form_stage_run(h->ops.data(), nops, i, stage_t, nloc, h->fold, ks, h->dtype);
            for (int c = 0; c < cnt; ++c) {
                pp[c] = h->ops[i + c].pos;
                mm[c] = dbase + h->ops[i + c].off;
            }
            const size_t j = i + cnt;
            // a single block goes through a staged pass when it takes the
            // split-fp16 form (the pass reads and writes its tiles in long
            // runs, where a single sweep reads 16-group tiles scattered over
            // the block's target bits), or when it is the queue's last op and
            // the pass also sums the norm (saving a read)
            bool lone_split = false;
            if (cnt == 1 && h->split && h->dtype == 0) {
                size_op(h->ops[i], h->arena.data(), h->amp);
                lone_split = h->ops[i].unit &&
                             split_exponent(bnd * std::max(1.0, h->ops[i].growth)) != kNoSplit;
            }
            if (cnt >= 2 || (cnt == 1 && (lone_split || (j == nops && norm_out != nullptr)))) {
                const bool from_e0 = h->e0_pending && i == 0 && !h->tier;
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (h->timing) {
                    e0 = next_event(h);
                    e1 = next_event(h);
                    if (!e0 || !e1) return set_err(h, SV_EDEVICE, "event creation failed");
                    TRY(h, hipEventRecord(e0, st));
                }
                int tused = 0;
                const bool last = j == nops && norm_out != nullptr;
                const bool track = !h->tier;
                const bool h_garbage_before = h->garbage;
                const uint64_t support_before = h->support;
                uint64_t pmask = 0, visited = 0;
                // split-fp16 form: unitary blocks, the tile scaled from the
                // state's amplitude bound through the run
                bool unit = h->split && h->dtype == 0;
                double bmax = bnd;
                for (int c = 0; c < cnt; ++c) {
                    Op& oc = h->ops[i + c];
                    size_op(oc, h->arena.data(), h->amp);
                    unit = unit && oc.unit;
                    bmax *= std::max(1.0, oc.growth);
                    bnd *= oc.growth;
                }
                const int split_exp = unit ? split_exponent(bmax) : kNoSplit;
                TRY(h, launch_stage(st, *psi, nloc, cnt, ks, pp, mm, stage_t, from_e0,
                                    last ? norm_out : nullptr, last ? norm_blocks : nullptr, &tused,
                                    track ? h->support : ~0ull, track && h->garbage, &pmask, &visited,
                                    split_exp, h->dtype));
                h->stage_forms[split_exp != kNoSplit ? 0 : 1] += 1;
                h->e0_pending = false;
                if (track) {
                    // the other tile positions were zero and stay zero
                    const uint64_t full = ((uint64_t)1 << nloc) - 1;
                    for (int c = 0; c < cnt; ++c)
                        for (int q = 0; q < ks[c]; ++q) h->support |= (uint64_t)1 << pp[c][q];
                    if ((h->support & full) == full) h->garbage = false;
                }
                if (h->timing) {
                    TRY(h, hipEventRecord(e1, st));
                    double f = 0.0, fi = 0.0;
                    // issued per amplitude: 3 real products (3M form, fp32 or
                    // FP64), or 4 real products x 3 split terms (fp16), 2 2^k
                    // flops each
                    for (int c = 0; c < cnt; ++c) {
                        f += block_flops_alg(ks[c]);
                        fi += (split_exp != kNoSplit ? 24.0 : 6.0) * (double)(1 << ks[c]);
                    }
                    // from |0...0> nothing is read; amplitudes on positions
                    // not reached yet are taken as zero, not read
                    const double amps = (double)visited;
                    double rd = from_e0 ? 0.0 : amps;
                    if (!from_e0 && track && h_garbage_before)
                        rd = std::ldexp(amps, -__builtin_popcountll(pmask & ~support_before));
                    h->tev_info.push_back({1, f * amps, fi * amps, (double)h->amp * (amps + rd)});
                }
                h->counters[0] += 1;
                h->counters[3] += (int64_t)visited;
                h->counters[7] += cnt;
                i = j - 1;
                continue;
            }
        }
        if (h->e0_pending || h->garbage) {
            const int rc = materialize_state(h);
            if (rc) return rc;
        }
        h->support = ~0ull;
        if (op.kind != OP_LPERM) {
            size_op(h->ops[i], h->arena.data(), h->amp);
            bnd *= h->ops[i].growth;
        }
        if (op.kind == OP_DENSE) {
            DiagSpec fold;
            const DiagSpec* fp = nullptr;
            if (h->fold && i + 1 < nops && h->ops[i + 1].kind == OP_DIAG) {
                const Op& d = h->ops[i + 1];
                fold.m = d.k;
                for (int j = 0; j < d.k; ++j) fold.pos[j] = d.pos[j];
                fold.table = dbase + d.off;
                fp = &fold;
                size_op(h->ops[i + 1], h->arena.data(), h->amp);
                bnd *= h->ops[i + 1].growth;
                ++i;
            }
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (h->timing) {
                e0 = next_event(h);
                e1 = next_event(h);
                if (!e0 || !e1) return set_err(h, SV_EDEVICE, "event creation failed");
                TRY(h, hipEventRecord(e0, st));
            }
            TRY(h, launch_dense(st, *psi, h->dtype, nloc, op.k, op.pos, dbase + op.off, fp,
                                idx_offset, h->mfma_min_k));
            if (h->timing) {
                TRY(h, hipEventRecord(e1, st));
                const double amps = (double)((uint64_t)1 << nloc);
                h->tev_info.push_back({0, block_flops_alg(op.k) * amps,
                                       block_flops_issued(h->dtype, op.k, nloc, h->mfma_min_k) * amps,
                                       2.0 * (double)h->amp * amps});
            }
            h->counters[0] += 1;
            h->counters[3] += (int64_t)1 << nloc;
        } else if (op.kind == OP_DIAG) {
            DiagSpec d;
            d.m = op.k;
            for (int j = 0; j < op.k; ++j) d.pos[j] = op.pos[j];
            d.table = dbase + op.off;
            TRY(h, launch_diag(st, *psi, h->dtype, nloc, idx_offset, d));
            h->counters[1] += 1;
            h->counters[3] += (int64_t)1 << nloc;
        } else {
            TRY(h, launch_bitperm(st, *psi, alt, h->dtype, nloc, op.runs));
            std::swap(*psi, alt);
            h->counters[2] += 1;
            h->counters[3] += (int64_t)1 << nloc;
        }
    }
    return SV_OK;
}

int upload_arena(sv_state* h, const WorkBufs* wb = nullptr)
{
    const size_t bytes = h->arena.size();
    if (bytes == 0) return SV_OK;
    if (wb) {
        // caller-provided device memory; the copy reads the queue's own host
        // buffer, which nothing changes before the caller's call returns
        if (bytes > wb->arena_cap) return set_err(h, SV_EINVAL, "queued matrices exceed the work area");
        TRY(h, hipMemcpyAsync(wb->arena, h->arena.data(), bytes, hipMemcpyHostToDevice, h->stream));
        h->d_arena_use = wb->arena;
        return SV_OK;
    }
    if (h->ev_arena) TRY(h, hipEventSynchronize(h->ev_arena));   // pinned staging reusable
    if (h->h_arena_cap < bytes) {
        if (h->h_arena) pool_free(h->h_arena, h->h_arena_cap, true);
        h->h_arena = nullptr;
        h->h_arena_cap = 0;
        size_t got = 0;
        h->h_arena = pool_alloc(std::max(bytes * 2, (size_t)1 << 20), true, &got);
        if (!h->h_arena) return set_err(h, SV_ENOMEM, "pinned staging allocation failed");
        h->h_arena_cap = got;
    }
    int rc = ensure_dev(h, &h->d_arena, &h->d_arena_cap, std::max(bytes * 2, (size_t)1 << 20));
    if (rc) return rc;
    std::memcpy(h->h_arena, h->arena.data(), bytes);
    TRY(h, hipMemcpyAsync(h->d_arena, h->h_arena, bytes, hipMemcpyHostToDevice, h->stream));
    h->d_arena_use = h->d_arena;
    if (!h->ev_arena) TRY(h, hipEventCreateWithFlags(&h->ev_arena, hipEventDisableTiming));
    TRY(h, hipEventRecord(h->ev_arena, h->stream));
    return SV_OK;
}

// ---- tier staging ------------------------------------------------------------
size_t file_amps(const sv_state* h) { return (size_t)1 << (h->L - h->s); }

// failure injection: true when this transfer must fail (see SV_OPT_FAIL_IO)
bool injected_io_failure(sv_state* h)
{
    if (h->fail_io_at <= 0) return false;
    return --h->fail_io_at == 0;
}

#define CHECK_INJECTED_IO(h)                                                         \
    do {                                                                             \
        if (injected_io_failure(h))                                                  \
            return fail_dev((h), "host-tier transfer (injected failure)", hipErrorUnknown, SV_EIO); \
    } while (0)

int stage_in(sv_state* h, hipStream_t st, uint64_t t, void* slot)
{
    const size_t fa = file_amps(h), fb = fa * h->amp;
    const int nf = 1 << h->s;
    for (int u = 0; u < nf; ++u) {
        char* dst = (char*)slot + (size_t)u * fb;
        CHECK_INJECTED_IO(h);
        TRY_IO(h, hipMemcpyAsync(dst, h->files[t * nf + u], fb, hipMemcpyHostToDevice, st));
        h->counters[4] += (int64_t)fb;
    }
    return SV_OK;
}

int stage_out(sv_state* h, hipStream_t st, uint64_t t, const void* slot)
{
    const size_t fa = file_amps(h), fb = fa * h->amp;
    const int nf = 1 << h->s;
    for (int u = 0; u < nf; ++u) {
        const char* src = (const char*)slot + (size_t)u * fb;
        CHECK_INJECTED_IO(h);
        TRY_IO(h, hipMemcpyAsync(h->files[t * nf + u], src, fb, hipMemcpyDeviceToHost, st));
        h->counters[5] += (int64_t)fb;
    }
    return SV_OK;
}

// Run the queue over every non-zero slice of the tier: stage in (copy-in
// stream), compute (handle stream), stage out (copy-out stream), pipelined
// over the device slots.  visit (optional) runs on the compute stream after
// the ops of each slice, with the slice's buffer.
template <typename F>
int tier_pass_pinned(sv_state* h, bool write_back, F&& visit)
{
    const int ns = 1 << h->s;
    const int R = (int)h->slots.size();
    int idx = 0;
    for (int t = 0; t < ns; ++t) {
        if (h->slice_zero[t]) {
            h->counters[6] += 1;
            continue;
        }
        const int k = idx % R;
        void* slot = h->slots[k];
        if (idx >= R) TRY(h, hipStreamWaitEvent(h->s_in, h->ev_out[k], 0));
        if (idx >= R) TRY(h, hipStreamWaitEvent(h->s_in, h->ev_comp[k], 0));
        int rc = stage_in(h, h->s_in, (uint64_t)t, slot);
        if (rc) return rc;
        TRY(h, hipEventRecord(h->ev_in[k], h->s_in));
        TRY(h, hipStreamWaitEvent(h->stream, h->ev_in[k], 0));
        void* cur = slot;
        void* alt = h->pslot;
        rc = run_ops(h, h->stream, &cur, alt, h->L, (uint64_t)t << h->L);
        if (rc) return rc;
        if (cur != slot) {
            // an odd number of local permutes left the data in the permute
            // buffer: swap roles so the slot keeps pointing at live data
            h->slots[k] = cur;
            h->pslot = slot;
            slot = cur;
        }
        rc = visit(t, slot);
        if (rc) return rc;
        TRY(h, hipEventRecord(h->ev_comp[k], h->stream));
        if (write_back) {
            TRY(h, hipStreamWaitEvent(h->s_out, h->ev_comp[k], 0));
            rc = stage_out(h, h->s_out, (uint64_t)t, slot);
            if (rc) return rc;
        }
        TRY(h, hipEventRecord(h->ev_out[k], h->s_out));
        ++idx;
    }
    TRY(h, hipStreamSynchronize(h->s_in));
    TRY(h, hipStreamSynchronize(h->stream));
    TRY(h, hipStreamSynchronize(h->s_out));
    return SV_OK;
}

// ---- pageable tier: pinned bounce buffers -----------------------------------
// Pageable files cannot be the source or target of asynchronous DMA, so
// every chunk (<= kChunk bytes) goes through a pinned bounce buffer: host
// threads copy file <-> bounce, the copy streams move bounce <-> slot.  One
// host thread drives both directions chunk by chunk, so the host-to-device
// and device-to-host links and the host copies overlap with each other and
// with the kernels of the slice in between.
constexpr size_t kChunk = (size_t)64 << 20;
constexpr int kBounce = 4;
constexpr int kCopyThreads = 8;

void par_memcpy(void* dst, const void* src, size_t bytes)
{
    if (bytes < ((size_t)4 << 20)) {
        std::memcpy(dst, src, bytes);
        return;
    }
    std::thread th[kCopyThreads];
    const size_t part = (bytes / kCopyThreads + 4095) & ~(size_t)4095;
    for (int i = 0; i < kCopyThreads; ++i) {
        const size_t lo = std::min(bytes, part * i), hi = std::min(bytes, part * (i + 1));
        th[i] = std::thread([=] { if (hi > lo) std::memcpy((char*)dst + lo, (const char*)src + lo, hi - lo); });
    }
    for (auto& t : th) t.join();
}

// Complex128 <-> complex64 between host buffers (files of a tier that stores
// single precision), split over threads like par_memcpy.
void par_widen(double* dst, const float* src, size_t count)
{
    auto run = [=](size_t lo, size_t hi) {
        for (size_t i = lo; i < hi; ++i) dst[i] = (double)src[i];
    };
    if (count < ((size_t)1 << 19)) { run(0, count); return; }
    std::thread th[kCopyThreads];
    const size_t part = (count + kCopyThreads - 1) / kCopyThreads;
    for (int i = 0; i < kCopyThreads; ++i)
        th[i] = std::thread(run, std::min(count, part * i), std::min(count, part * (i + 1)));
    for (auto& t : th) t.join();
}

void par_narrow(float* dst, const double* src, size_t count)
{
    auto run = [=](size_t lo, size_t hi) {
        for (size_t i = lo; i < hi; ++i) dst[i] = (float)src[i];
    };
    if (count < ((size_t)1 << 19)) { run(0, count); return; }
    std::thread th[kCopyThreads];
    const size_t part = (count + kCopyThreads - 1) / kCopyThreads;
    for (int i = 0; i < kCopyThreads; ++i)
        th[i] = std::thread(run, std::min(count, part * i), std::min(count, part * (i + 1)));
    for (auto& t : th) t.join();
}

struct OutChunk {
    const char* src;   // device
    char* dst;         // pageable file memory
    size_t bytes;
    int slice_idx;
    int slot;          // device slot the slice occupies
    bool last;         // last chunk of its slice: releases the slot
};

struct BouncePipe {
    sv_state* h;
    void* bin[kBounce] = {};
    void* bout[kBounce] = {};
    hipEvent_t ev_bin[kBounce] = {}, ev_bout[kBounce] = {};
    int next_in = 0;
    std::deque<OutChunk> pending;                    // not issued yet
    std::deque<std::pair<int, OutChunk>> inflight;   // (bounce index, chunk) issued D2H
    int free_out[kBounce];
    int nfree_out = 0;
    int err = SV_OK;

    int init()
    {
        for (int b = 0; b < kBounce; ++b) {
            size_t got = 0;
            bin[b] = pool_alloc(kChunk, true, &got);
            bout[b] = pool_alloc(kChunk, true, &got);
            if (!bin[b] || !bout[b]) return set_err(h, SV_ENOMEM, "pinned bounce buffer allocation failed");
            TRY(h, hipEventCreateWithFlags(&ev_bin[b], hipEventDisableTiming));
            TRY(h, hipEventCreateWithFlags(&ev_bout[b], hipEventDisableTiming));
            TRY(h, hipEventRecord(ev_bin[b], h->s_in));
            free_out[nfree_out++] = b;
        }
        return SV_OK;
    }
    ~BouncePipe()
    {
        for (int b = 0; b < kBounce; ++b) {
            if (ev_bin[b]) { (void)hipEventSynchronize(ev_bin[b]); (void)hipEventDestroy(ev_bin[b]); }
            if (ev_bout[b]) { (void)hipEventSynchronize(ev_bout[b]); (void)hipEventDestroy(ev_bout[b]); }
            pool_free(bin[b], kChunk, true);
            pool_free(bout[b], kChunk, true);
        }
    }
    // finish the oldest issued D2H chunk: wait for it, copy bounce -> file
    int complete_one()
    {
        auto [b, c] = inflight.front();
        inflight.pop_front();
        TRY_IO(h, hipEventSynchronize(ev_bout[b]));
        if (h->store32) par_narrow((float*)c.dst, (const double*)bout[b], c.bytes / sizeof(double));
        else par_memcpy(c.dst, bout[b], c.bytes);
        free_out[nfree_out++] = b;
        return SV_OK;
    }
    // issue D2H chunks while bounce buffers are free; finish chunks whose
    // copy is done (blocking only when `block` and nothing can be issued)
    int pump(bool block)
    {
        for (;;) {
            while (!pending.empty() && nfree_out > 0) {
                const OutChunk c = pending.front();
                pending.pop_front();
                CHECK_INJECTED_IO(h);
                const int b = free_out[--nfree_out];
                TRY_IO(h, hipMemcpyAsync(bout[b], c.src, c.bytes, hipMemcpyDeviceToHost, h->s_out));
                TRY_IO(h, hipEventRecord(ev_bout[b], h->s_out));
                if (c.last) TRY_IO(h, hipEventRecord(h->ev_out[c.slot], h->s_out));
                inflight.emplace_back(b, c);
                h->counters[5] += (int64_t)c.bytes;
            }
            bool progressed = false;
            while (!inflight.empty() && hipEventQuery(ev_bout[inflight.front().first]) == hipSuccess) {
                int rc = complete_one();
                if (rc) return rc;
                progressed = true;
            }
            if (!block || (pending.empty() && inflight.empty())) return SV_OK;
            if (!progressed) {
                int rc = complete_one();
                if (rc) return rc;
            }
        }
    }
    // every out-chunk of slices <= idx issued and finished
    int drain_upto(int idx)
    {
        for (;;) {
            bool any = false;
            for (const auto& c : pending) any = any || c.slice_idx <= idx;
            for (const auto& c : inflight) any = any || c.second.slice_idx <= idx;
            if (!any) return SV_OK;
            int rc = pump(false);
            if (rc) return rc;
            if (!inflight.empty()) {
                rc = complete_one();
                if (rc) return rc;
            }
        }
    }
    // stage a slice in: file chunk -> bounce (host) -> slot (s_in); out-chunks
    // are pumped between chunks so both directions stay busy
    // (offsets are in device bytes; a single-precision file holds
    // famp / amp of them)
    int stage_in(uint64_t t, void* slot)
    {
        const size_t fb = file_amps(h) * h->amp;
        const int nf = 1 << h->s;
        for (int u = 0; u < nf; ++u)
            for (size_t off = 0; off < fb; off += kChunk) {
                const size_t n = std::min(kChunk, fb - off);
                const int b = next_in;
                next_in = (next_in + 1) % kBounce;
                TRY_IO(h, hipEventSynchronize(ev_bin[b]));
                CHECK_INJECTED_IO(h);
                const char* src = (const char*)h->files[t * nf + u] + off / h->amp * h->famp;
                if (h->store32) par_widen((double*)bin[b], (const float*)src, n / sizeof(double));
                else par_memcpy(bin[b], src, n);
                TRY_IO(h, hipMemcpyAsync((char*)slot + (size_t)u * fb + off, bin[b], n,
                                         hipMemcpyHostToDevice, h->s_in));
                TRY_IO(h, hipEventRecord(ev_bin[b], h->s_in));
                h->counters[4] += (int64_t)n;
                int rc = pump(false);
                if (rc) return rc;
            }
        return SV_OK;
    }
    void queue_out(uint64_t t, const void* slot, int idx, int k)
    {
        const size_t fb = file_amps(h) * h->amp;
        const int nf = 1 << h->s;
        for (int u = 0; u < nf; ++u)
            for (size_t off = 0; off < fb; off += kChunk)
                pending.push_back({(const char*)slot + (size_t)u * fb + off,
                                   (char*)h->files[t * nf + u] + off / h->amp * h->famp,
                                   std::min(kChunk, fb - off), idx, k,
                                   u == nf - 1 && off + kChunk >= fb});
    }
};

template <typename F>
int tier_pass_pageable(sv_state* h, bool write_back, F&& visit)
{
    const int ns = 1 << h->s;
    const int R = (int)h->slots.size();
    std::vector<int> act;
    for (int t = 0; t < ns; ++t) {
        if (h->slice_zero[t]) h->counters[6] += 1;
        else act.push_back(t);
    }
    BouncePipe bp;
    bp.h = h;
    int rc = bp.init();
    if (rc) return rc;
    const int N = (int)act.size();
    auto slot_of = [&](int idx) { return idx % R; };
    // stage-in of idx into its slot, after the slot's previous slice left it
    auto prefetch = [&](int idx) -> int {
        const int k = slot_of(idx);
        if (idx >= R) {
            int r = bp.drain_upto(idx - R);
            if (r) return r;
            TRY(h, hipStreamWaitEvent(h->s_in, h->ev_out[k], 0));
            TRY(h, hipStreamWaitEvent(h->s_in, h->ev_comp[k], 0));
        }
        int r = bp.stage_in((uint64_t)act[idx], h->slots[k]);
        if (r) return r;
        TRY(h, hipEventRecord(h->ev_in[k], h->s_in));
        return SV_OK;
    };
    if (N > 0) {
        rc = prefetch(0);
        if (rc) return rc;
    }
    for (int idx = 0; idx < N; ++idx) {
        const int k = slot_of(idx);
        const int t = act[idx];
        void* slot = h->slots[k];
        TRY(h, hipStreamWaitEvent(h->stream, h->ev_in[k], 0));
        void* cur = slot;
        rc = run_ops(h, h->stream, &cur, h->pslot, h->L, (uint64_t)t << h->L);
        if (rc) return rc;
        if (cur != slot) {
            h->slots[k] = cur;
            h->pslot = slot;
            slot = cur;
        }
        rc = visit(t, slot);
        if (rc) return rc;
        TRY(h, hipEventRecord(h->ev_comp[k], h->stream));
        if (write_back) {
            TRY(h, hipStreamWaitEvent(h->s_out, h->ev_comp[k], 0));
            bp.queue_out((uint64_t)t, slot, idx, k);      // its last chunk records ev_out[k]
        }
        // the next slice streams in while this one computes and earlier ones
        // stream out; a slot is reused only after its slice left it (prefetch
        // drains that slice's chunks first)
        if (idx + 1 < N) {
            rc = prefetch(idx + 1);
            if (rc) return rc;
        }
        rc = bp.pump(false);
        if (rc) return rc;
    }
    rc = bp.pump(true);
    if (rc) return rc;
    TRY(h, hipStreamSynchronize(h->s_in));
    TRY(h, hipStreamSynchronize(h->stream));
    TRY(h, hipStreamSynchronize(h->s_out));
    return SV_OK;
}

template <typename F>
int tier_pass(sv_state* h, bool write_back, F&& visit)
{
    if (h->pinned_tier) return tier_pass_pinned(h, write_back, std::forward<F>(visit));
    return tier_pass_pageable(h, write_back, std::forward<F>(visit));
}

// An amplitude bound for a resident state whose bound is unknown (its
// buffer was written by the caller): its norm, an FP64 sum of |psi|^2 on the
// device (one read pass and a host wait).  Only when a staged pass of the
// queue could take the split form.
int measure_bound(sv_state* h, const WorkBufs* wb)
{
    if (h->tier || !h->split || h->dtype != 0 || h->stage_t < 9 || h->mfma_min_k != 4 || h->ops.empty() ||
        std::isfinite(h->amp_bound))
        return SV_OK;
    bool stageable = false;
    for (const Op& op : h->ops) stageable = stageable || (op.kind == OP_DENSE && (op.k == 4 || op.k == 5));
    if (!stageable) return SV_OK;
    double* part;
    double* small;
    if (wb) {
        part = (double*)wb->part;
        small = (double*)wb->small;
    } else {
        const int rc = ensure_dev(h, &h->d_part, &h->d_part_cap, kPartDoubles * sizeof(double));
        if (rc) return rc;
        part = (double*)h->d_part;
        small = (double*)h->d_small;
    }
    int nb = 0;
    TRY(h, launch_norm_partials(h->stream, h->dev, h->dtype, h->n, part, &nb));
    TRY(h, launch_finish_sum(h->stream, part, nb, 1, small));
    double nrm2 = HUGE_VAL;
    TRY(h, hipMemcpyAsync(&nrm2, small, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    TRY(h, hipStreamSynchronize(h->stream));
    h->amp_bound = std::isfinite(nrm2) ? std::sqrt(nrm2) * (1.0 + 1e-6) : HUGE_VAL;
    return SV_OK;
}

int flush(sv_state* h, double* norm_out = nullptr, int* norm_blocks = nullptr, const WorkBufs* wb = nullptr)
{
    if (norm_blocks) *norm_blocks = 0;
    if (h->ops.empty()) return materialize_state(h);
    int rc = upload_arena(h, wb);
    if (rc) return rc;
    if (!h->tier) {
        rc = measure_bound(h, wb);
        if (rc) return rc;
        void* cur = h->dev;
        rc = run_ops(h, h->stream, &cur, h->scratch, h->n, 0, norm_out, norm_blocks);
        if (rc) return rc;
        if (cur != h->dev) return set_err(h, SV_EDEVICE, "internal: permute left in scratch");
        rc = materialize_state(h);   // tiles the passes skipped hold older values
        if (rc) return rc;
    } else {
        TRY(h, hipEventRecord(h->ev_arena, h->stream));
        TRY(h, hipStreamWaitEvent(h->s_in, h->ev_arena, 0));
        rc = tier_pass(h, true, [](int, void*) { return SV_OK; });
        if (rc) return rc;
    }
    // the queue is applied: the bound advances over it
    for (Op& op : h->ops) {
        size_op(op, h->arena.data(), h->amp);
        h->amp_bound *= op.growth;
    }
    h->ops.clear();
    h->arena.clear();
    if (h->timing) return collect_timing(h);
    return SV_OK;
}

// checkpoint metadata of a file-backed tier, in the tier's directory
const char* const kCheckpointName = "sv_checkpoint.meta";

// What open_state_files restores: the layout, the slices known to be zero
// and the names of the existing files.
struct Restore {
    std::vector<int> order;
    std::vector<uint8_t> slice_zero;
    std::vector<std::string> names;
};

void release(sv_state* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->s_in) (void)hipStreamSynchronize(h->s_in);
    if (h->s_out) (void)hipStreamSynchronize(h->s_out);
    if (h->own_dev && h->dev) (void)hipFree(h->dev);
    if (h->scratch) (void)hipFree(h->scratch);
    const size_t fbytes = h->files.empty() ? 0 : ((size_t)1 << (h->L - h->s)) * h->famp;
    for (void* p : h->files) {
        if (!p) continue;
        if (h->pinned_tier) (void)hipHostFree(p);
        else munmap(p, fbytes);
    }
    for (int fd : h->file_fds) (void)close(fd);
    if (!h->keep_files) {
        for (const auto& path : h->file_paths) (void)unlink(path.c_str());
        if (!h->tier_dir.empty()) (void)unlink((h->tier_dir + "/" + kCheckpointName).c_str());
    }
    for (void* p : h->slots)
        if (p) (void)hipFree(p);
    if (h->pslot) (void)hipFree(h->pslot);
    const std::pair<void*, size_t> work[] = {{h->d_arena, h->d_arena_cap}, {h->d_bits, h->d_bits_cap},
                                             {h->d_acc, h->d_acc_cap}, {h->d_part, h->d_part_cap},
                                             {h->d_tcol, h->d_tcol_cap}, {h->d_rowmap, h->d_rowmap_cap},
                                             {h->d_small, 64}};
    for (const auto& w : work)
        if (w.first) pool_free(w.first, w.second, false);
    if (h->h_arena) pool_free(h->h_arena, h->h_arena_cap, true);
    for (auto* v : {&h->ev_in, &h->ev_comp, &h->ev_out, &h->tev_pool})
        for (hipEvent_t e : *v) (void)hipEventDestroy(e);
    if (h->ev_arena) (void)hipEventDestroy(h->ev_arena);
    if (h->s_in) (void)hipStreamDestroy(h->s_in);
    if (h->s_out) (void)hipStreamDestroy(h->s_out);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

void default_layout(sv_state* h)
{
    h->order.clear();
    for (int q = 0; q < h->n; ++q)
        if (!((h->slice_mask >> q) & 1)) h->order.push_back(q);
    for (int q = 0; q < h->n; ++q)
        if ((h->slice_mask >> q) & 1) h->order.push_back(q);
    h->pos.assign(h->n, 0);
    for (int p = 0; p < h->n; ++p) h->pos[h->order[p]] = p;
}

int create_common(int n, uint64_t slice_mask, int dtype, void* stream, void* ext, size_t ext_bytes,
                  sv_handle* out, const char* dir = nullptr, const Restore* rs = nullptr)
{
    if (!out) return set_err(nullptr, SV_EINVAL, "out is NULL");
    const int base = dtype & 0xff;
    if (base != SV_C64 && base != SV_C128) return set_err(nullptr, SV_EINVAL, "bad dtype");
    if (n < 1 || n > 40) return set_err(nullptr, SV_EINVAL, "n out of range [1, 40]");
    if (n < 64 && (slice_mask >> n)) return set_err(nullptr, SV_EINVAL, "slice_mask names a qubit >= n");
    const int s = __builtin_popcountll(slice_mask);
    if (s > 12 || s > n - 1) return set_err(nullptr, SV_EINVAL, "too many sliced qubits");

    sv_state* h = new (std::nothrow) sv_state();
    if (!h) return set_err(nullptr, SV_ENOMEM, "host allocation failed");
    h->n = n;
    h->s = s;
    h->L = n - s;
    h->dtype = base;
    h->amp = base ? 16 : 8;
    h->store32 = base == SV_C128 && (dtype & SV_FLAG_STORE32);
    h->famp = h->store32 ? 8 : h->amp;
    h->slice_mask = slice_mask;
    default_layout(h);
    hipError_t e;
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { release(h); return fail_dev(nullptr, "hipStreamCreate", e); }
        h->own_stream = true;
    }
    const size_t total = ((size_t)1 << n) * h->amp;
    bool tier = (dtype & SV_FLAG_TIER) != 0 || dir != nullptr || h->store32;
    if (ext) {
        if (tier) { release(h); return set_err(nullptr, SV_EINVAL, "external buffer cannot be tiered"); }
        if (ext_bytes < total) { release(h); return set_err(nullptr, SV_EINVAL, "external buffer too small"); }
        if ((uintptr_t)ext & 15) { release(h); return set_err(nullptr, SV_EINVAL, "external buffer not 16-byte aligned"); }
        h->dev = ext;
        h->dev_bytes = ext_bytes;
    } else if (!tier) {
        size_t freeb = 0, totb = 0;
        e = hipMemGetInfo(&freeb, &totb);
        if (e != hipSuccess) { release(h); return fail_dev(nullptr, "hipMemGetInfo", e); }
        const size_t margin = (size_t)2 << 30;
        if (total + margin > freeb) {
            if (s == 0) { release(h); return set_err(nullptr, SV_ENOMEM, "state does not fit in device memory and is not sliced"); }
            tier = true;
        } else {
            if (hipMalloc(&h->dev, total) != hipSuccess) {
                (void)hipGetLastError();
                release(h);
                return set_err(nullptr, SV_ENOMEM, "device allocation of the state failed");
            }
            h->own_dev = true;
            h->dev_bytes = total;
        }
    }
    h->tier = tier;
    if (tier) {
        if (s < 1 || h->L - s < 0) { release(h); return set_err(nullptr, SV_EINVAL, "tier needs 1 <= s <= n/2"); }
        const int ns = 1 << s;
        const size_t fb = file_amps(h) * h->famp;
        h->files.assign((size_t)ns * ns, nullptr);
        // Pinned memory is scarce (the driver caps it well below host RAM):
        // the tier is pinned up to kPinnedBudget and pageable beyond that
        // (or when pinning fails); pageable files are anonymous mappings whose
        // pages stay unbacked until written.
        const size_t kPinnedBudget = (size_t)48 << 30;
        // (a single-precision tier converts in the host copies of the bounce path)
        h->pinned_tier = (fb * h->files.size() <= kPinnedBudget) && !(dtype & SV_FLAG_PAGEABLE) && !dir &&
                         !h->store32;
        if (h->pinned_tier) {
            for (auto& f : h->files) {
                if (hipHostMalloc(&f, fb, hipHostMallocDefault) != hipSuccess) {
                    f = nullptr;
                    (void)hipGetLastError();
                    h->pinned_tier = false;
                    break;
                }
                std::memset(f, 0, fb);
            }
            if (!h->pinned_tier)
                for (auto& f : h->files) {
                    if (f) (void)hipHostFree(f);
                    f = nullptr;
                }
        }
        if (dir) {
            // one file per logical file (Sec. 4: slices go to secondary storage
            // as whole files), mapped shared: the page cache does the I/O
            static std::atomic<unsigned> seq{0};
            const unsigned id = seq.fetch_add(1);
            h->tier_dir = dir;
            if (rs) h->keep_files = true;       // until opened, the files are the checkpoint's
            for (size_t i = 0; i < h->files.size(); ++i) {
                const std::string path = rs ? std::string(dir) + "/" + rs->names[i]
                                            : std::string(dir) + "/sv_tier_" + std::to_string((long)getpid()) + "_" +
                                                  std::to_string(id) + "_" + std::to_string(i) + ".bin";
                const int fd = rs ? open(path.c_str(), O_RDWR) : open(path.c_str(), O_RDWR | O_CREAT | O_EXCL, 0600);
                if (fd < 0) {
                    release(h);
                    return set_err(nullptr, SV_EIO, (rs ? "cannot open tier file " : "cannot create tier file ") + path);
                }
                h->file_fds.push_back(fd);
                h->file_paths.push_back(path);
                void* p = MAP_FAILED;
                struct stat sb_;
                const bool sized = rs ? (fstat(fd, &sb_) == 0 && (size_t)sb_.st_size == fb)
                                      : ftruncate(fd, (off_t)fb) == 0;
                if (sized)
                    p = mmap(nullptr, fb, PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
                if (p == MAP_FAILED) {
                    release(h);
                    return set_err(nullptr, SV_EIO, "cannot size or map tier file " + path);
                }
                h->files[i] = p;
                h->file_maps.push_back(p);
            }
        } else if (!h->pinned_tier) {
            for (auto& f : h->files) {
                void* p = mmap(nullptr, fb, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
                if (p == MAP_FAILED) {
                    f = nullptr;
                    release(h);
                    return set_err(nullptr, SV_ENOMEM, "host tier allocation failed");
                }
                (void)madvise(p, fb, MADV_HUGEPAGE);     // fewer first-touch faults
                f = p;
            }
        }
        if (rs) {
            // the checkpoint's state: its layout, its zero slices, its files as they are
            h->order = rs->order;
            for (int p = 0; p < n; ++p) h->pos[h->order[p]] = p;
            h->slice_zero = rs->slice_zero;
            h->keep_files = false;
        } else {
            // |0...0>: amplitude 0 lives in file (t = 0, u = 0)
            if (h->famp == 16) { double one[2] = {1.0, 0.0}; std::memcpy(h->files[0], one, 16); }
            else { float one[2] = {1.0f, 0.0f}; std::memcpy(h->files[0], one, 8); }
            h->slice_zero.assign(ns, 1);
            h->slice_zero[0] = 0;
        }
        const size_t sb = ((size_t)1 << h->L) * h->amp;
        h->slots.assign(h->nslots, nullptr);
        for (auto& p : h->slots)
            if (hipMalloc(&p, sb) != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                release(h);
                return set_err(nullptr, SV_ENOMEM, "device slot allocation failed");
            }
        if (hipMalloc(&h->pslot, sb) != hipSuccess) {
            h->pslot = nullptr;
            (void)hipGetLastError();
            release(h);
            return set_err(nullptr, SV_ENOMEM, "device slot allocation failed");
        }
        e = hipStreamCreateWithFlags(&h->s_in, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->s_out, hipStreamNonBlocking);
        if (e != hipSuccess) { release(h); return fail_dev(nullptr, "hipStreamCreate", e); }
        for (auto* v : {&h->ev_in, &h->ev_comp, &h->ev_out}) {
            v->assign(h->nslots, nullptr);
            for (auto& ev : *v) {
                e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (e != hipSuccess) { release(h); return fail_dev(nullptr, "hipEventCreate", e); }
            }
        }
        e = hipEventCreateWithFlags(&h->ev_arena, hipEventDisableTiming);
        if (e != hipSuccess) { release(h); return fail_dev(nullptr, "hipEventCreate", e); }
    } else if (!(ext && (dtype & SV_FLAG_KEEP))) {
        e = launch_init(h->stream, h->dev, h->dtype, (uint64_t)1 << n, true);
        if (e != hipSuccess) { release(h); return fail_dev(nullptr, "init kernel", e); }
        h->support = 0;              // |0...0>, written in full: nothing stale
    } else {
        h->amp_bound = HUGE_VAL;     // the caller's amplitudes
    }
    h->d_small = pool_alloc(64, false, nullptr);
    if (!h->d_small) {
        release(h);
        return set_err(nullptr, SV_ENOMEM, "device allocation failed");
    }
    *out = h;
    return SV_OK;
}

// FP64 host reduction helpers ------------------------------------------------
int finish_sum(sv_state* h, hipStream_t st, const WorkBufs& w, int nblocks, int width, double* host_out)
{
    TRY(h, launch_finish_sum(st, (const double*)w.part, nblocks, width, (double*)w.small));
    TRY(h, hipMemcpyAsync(host_out, w.small, sizeof(double) * width, hipMemcpyDeviceToHost, st));
    TRY(h, hipStreamSynchronize(st));
    return SV_OK;
}

int do_reduce(sv_state* h, const void* trailing, int64_t count, const uint64_t* bits, void* out,
              double* stats, const WorkBufs* wb = nullptr)
{
    CHECK_HANDLE(h);
    if (count < 0 || (count > 0 && (!bits || !out))) return set_err(h, SV_EINVAL, "bad output arguments");
    const uint64_t lim = h->n >= 64 ? ~0ull : ((1ull << h->n) - 1);
    for (int64_t j = 0; j < count; ++j)
        if (bits[j] > lim) return set_err(h, SV_EINVAL, "bitstring >= 2^n");
    int rc;
    const int ns = 1 << h->s;
    const size_t cnt = (size_t)std::max<int64_t>(count, 1);
    WorkBufs w;
    if (wb) {
        w = *wb;
    } else {
        if ((rc = ensure_dev(h, &h->d_bits, &h->d_bits_cap, cnt * 8))) return rc;
        if ((rc = ensure_dev(h, &h->d_acc, &h->d_acc_cap, cnt * 16))) return rc;
        if ((rc = ensure_dev(h, &h->d_part, &h->d_part_cap, kPartDoubles * sizeof(double)))) return rc;
        // T (all columns, gathered per physical slice) + per-slice norms
        if ((rc = ensure_dev(h, &h->d_tcol, &h->d_tcol_cap, (size_t)ns * ns * 16 + (size_t)ns * 8))) return rc;
        if ((rc = ensure_dev(h, &h->d_rowmap, &h->d_rowmap_cap, (size_t)ns * 4))) return rc;
        w = WorkBufs{h->d_bits, h->d_acc, h->d_part, h->d_tcol, h->d_rowmap, h->d_small, nullptr, 0};
    }

    // logical bitstring -> physical index
    std::vector<int> from(h->n), to(h->n);
    for (int q = 0; q < h->n; ++q) { from[q] = q; to[q] = h->pos[q]; }
    const BitRuns l2p = make_runs(h->n, from.data(), to.data());
    // physical slice id -> T index (bit i = i-th sliced qubit in ascending label order)
    std::vector<int> sl;
    for (int q = 0; q < h->n; ++q)
        if (h->pos[q] >= h->L) sl.push_back(q);
    std::vector<int> rowmap(ns);
    for (int t = 0; t < ns; ++t) {
        int r = 0;
        for (int i = 0; i < h->s; ++i)
            if ((t >> (h->pos[sl[i]] - h->L)) & 1) r |= 1 << i;
        rowmap[t] = r;
    }
    const double* T = (const double*)trailing;
    // tcols[t][r] = T[r][rowmap[t]]: the column a physical slice t multiplies
    std::vector<double> tcols;
    if (T) {
        tcols.assign((size_t)ns * ns * 2, 0.0);
        for (int t = 0; t < ns; ++t)
            for (int r = 0; r < ns; ++r) {
                const size_t src = 2 * ((size_t)r * ns + rowmap[t]);
                tcols[2 * ((size_t)t * ns + r)] = T[src];
                tcols[2 * ((size_t)t * ns + r) + 1] = T[src + 1];
            }
    }
    hipStream_t st = h->stream;
    double* d_snorm = (double*)((char*)w.tcol + (size_t)ns * ns * 16);
    if (count > 0) {
        TRY(h, hipMemcpyAsync(w.bits, bits, (size_t)count * 8, hipMemcpyHostToDevice, st));
        TRY(h, hipMemsetAsync(w.acc, 0, (size_t)count * 16, st));
    }
    TRY(h, hipMemcpyAsync(w.rowmap, rowmap.data(), (size_t)ns * 4, hipMemcpyHostToDevice, st));
    if (T) TRY(h, hipMemcpyAsync(w.tcol, tcols.data(), tcols.size() * 8, hipMemcpyHostToDevice, st));
    TRY(h, hipMemsetAsync(d_snorm, 0, (size_t)ns * 8, st));
    int folded_blocks = 0;
    // nothing below synchronises the host per slice: the tier pipeline keeps
    // staging the next slice while this one is reduced
    auto visit = [&](int t, const void* slice_buf) -> int {
        const void* tc = T ? (const void*)((const char*)w.tcol + (size_t)t * ns * 16) : nullptr;
        TRY(h, launch_accumulate(st, slice_buf, h->dtype, h->L, (uint64_t)t, l2p, count,
                                 (const uint64_t*)w.bits, tc, (const int*)w.rowmap,
                                 (double*)w.acc));
        if (stats) {
            int nb = folded_blocks;      // partials already written by the last staged pass
            if (nb == 0)
                TRY(h, launch_norm_partials(st, slice_buf, h->dtype, h->L, (double*)w.part, &nb));
            TRY(h, launch_finish_sum(st, (const double*)w.part, nb, 1, d_snorm + t));
        }
        return SV_OK;
    };
    if (!h->tier) {
        // unsliced: the norm rides on the queue's last staged pass when it has one
        rc = (stats && ns == 1) ? flush(h, (double*)w.part, &folded_blocks, wb) : flush(h, nullptr, nullptr, wb);
        if (rc) return rc;
        for (int t = 0; t < ns && !rc; ++t)
            rc = visit(t, (const char*)h->dev + ((size_t)t << h->L) * h->amp);
    } else {
        // one pass over the tier: pending ops, then the reduction, then write back
        const bool pending = !h->ops.empty();
        if (pending) {
            rc = upload_arena(h);
            if (rc) return rc;
        }
        rc = tier_pass(h, pending, visit);
        if (rc) return rc;
        h->ops.clear();
        h->arena.clear();
        if (h->timing) rc = collect_timing(h);
    }
    if (rc) return rc;
    if (count > 0)
        TRY(h, hipMemcpyAsync(out, w.acc, (size_t)count * 16, hipMemcpyDeviceToHost, st));
    if (stats) {
        std::vector<double> snorm(ns, 0.0);
        TRY(h, hipMemcpyAsync(snorm.data(), d_snorm, (size_t)ns * 8, hipMemcpyDeviceToHost, st));
        double x[2] = {0.0, 0.0};
        if (count > 0) {
            int nb = 0;
            TRY(h, launch_xeb_partials(st, (const double*)w.acc, count, (double)h->n,
                                       (double*)w.part, &nb));
            rc = finish_sum(h, st, w, nb, 2, x);
            if (rc) return rc;
        }
        TRY(h, hipStreamSynchronize(st));
        double norm = 0.0;
        for (int t = 0; t < ns; ++t) norm += snorm[t];    // fixed slice order
        stats[0] = norm;
        stats[1] = x[0];
        stats[2] = x[1];
    }
    TRY(h, hipStreamSynchronize(st));
    return SV_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

int create_state(int n, uint64_t slice_mask, int dtype, void* hip_stream, sv_handle* out)
{
    return create_common(n, slice_mask, dtype, hip_stream, nullptr, 0, out);
}

int create_state_files(int n, uint64_t slice_mask, int dtype, void* hip_stream, const char* dir,
                       sv_handle* out)
{
    if (!dir || !*dir) return set_err(nullptr, SV_EINVAL, "directory is NULL or empty");
    return create_common(n, slice_mask, dtype | SV_FLAG_TIER, hip_stream, nullptr, 0, out, dir);
}

int create_state_ext(int n, uint64_t slice_mask, int dtype, void* hip_stream, void* dev_buf,
                     size_t bytes, sv_handle* out)
{
    if (!dev_buf) return set_err(nullptr, SV_EINVAL, "dev_buf is NULL");
    return create_common(n, slice_mask, dtype, hip_stream, dev_buf, bytes, out);
}

int destroy_state(sv_handle h)
{
    if (!h) return SV_OK;
    release(h);
    return SV_OK;
}

int apply_fused(sv_handle h, int k, const int* qubits, const void* matrix)
{
    CHECK_HANDLE(h);
    const int kmax = h->dtype ? 5 : 6;
    int rc = check_qubit_list(h, k, qubits, kmax);
    if (rc) return rc;
    if (!matrix) return set_err(h, SV_EINVAL, "matrix is NULL");
    if (k > h->L) return set_err(h, SV_EINVAL, "block wider than the local qubits");
    for (int j = 0; j < k; ++j)
        if (h->pos[qubits[j]] >= h->L) return set_err(h, SV_ESLICED, "dense op on a sliced qubit");
    Op op;
    op.kind = OP_DENSE;
    op.k = k;
    for (int j = 0; j < k; ++j) op.pos[j] = h->pos[qubits[j]];
    int minp = 64;
    for (int j = 0; j < k; ++j) minp = std::min(minp, op.pos[j]);
    if (h->dtype == 0 && h->mfma_min_k == 4 && k < 4 && minp < 4 && h->L >= 8) {
        // A small block whose targets sit among the lowest four positions
        // reads and writes partial cache lines on the VALU path.  Widen it
        // to four qubits with identity on the lowest free positions (M' = I
        // (x) M, extra bits on top) so it runs as an address-ordered staged
        // matrix-core sweep over whole cache lines.
        const int D = 1 << k;
        for (int p = 0; op.k < 4; ++p) {
            bool used = false;
            for (int j = 0; j < op.k; ++j) used = used || (op.pos[j] == p);
            if (!used) op.pos[op.k++] = p;
        }
        const int D4 = 16;
        std::vector<float> big((size_t)D4 * D4 * 2, 0.0f);
        const float* m = (const float*)matrix;
        for (int hi = 0; hi < D4 / D; ++hi)
            for (int r = 0; r < D; ++r)
                for (int c = 0; c < D; ++c) {
                    const size_t dst = ((size_t)(hi * D + r) * D4 + (hi * D + c)) * 2;
                    big[dst] = m[2 * (r * D + c)];
                    big[dst + 1] = m[2 * (r * D + c) + 1];
                }
        op.off = push_arena(h, big.data(), big.size() * sizeof(float));
    } else {
        op.off = push_arena(h, matrix, ((size_t)1 << (2 * k)) * h->amp);
    }
    h->ops.push_back(op);
    if (h->arena.size() > ((size_t)64 << 20) || h->ops.size() > 65536) return flush(h);
    return SV_OK;
}

int apply_diag(sv_handle h, int m, const int* qubits, const void* phases)
{
    CHECK_HANDLE(h);
    int rc = check_qubit_list(h, m, qubits, kMaxDiag);
    if (rc) return rc;
    if (!phases) return set_err(h, SV_EINVAL, "phase table is NULL");
    Op op;
    op.kind = OP_DIAG;
    op.k = m;
    for (int j = 0; j < m; ++j) op.pos[j] = h->pos[qubits[j]];
    op.off = push_arena(h, phases, ((size_t)1 << m) * h->amp);
    h->ops.push_back(op);
    if (h->arena.size() > ((size_t)64 << 20) || h->ops.size() > 65536) return flush(h);
    return SV_OK;
}

int apply_ops(sv_handle h, int count, const int* kinds, const int* widths, const int* qubits,
              const void* data)
{
    CHECK_HANDLE(h);
    if (count < 0) return set_err(h, SV_EINVAL, "negative operation count");
    if (count == 0) return SV_OK;
    if (!kinds || !widths || !qubits || !data) return set_err(h, SV_EINVAL, "NULL operation array");
    // every operation is checked before any is queued
    const int kmax = h->dtype ? 5 : 6;
    size_t qo = 0;
    for (int i = 0; i < count; ++i) {
        const int k = widths[i];
        int rc;
        if (kinds[i] == SV_OP_FUSED) {
            rc = check_qubit_list(h, k, qubits + qo, kmax);
            if (rc) return rc;
            if (k > h->L) return set_err(h, SV_EINVAL, "block wider than the local qubits");
            for (int j = 0; j < k; ++j)
                if (h->pos[qubits[qo + j]] >= h->L) return set_err(h, SV_ESLICED, "dense op on a sliced qubit");
        } else if (kinds[i] == SV_OP_DIAG) {
            rc = check_qubit_list(h, k, qubits + qo, kMaxDiag);
            if (rc) return rc;
        } else {
            return set_err(h, SV_EINVAL, "unknown operation kind");
        }
        qo += (size_t)k;
    }
    qo = 0;
    const char* d = (const char*)data;
    for (int i = 0; i < count; ++i) {
        const int k = widths[i];
        const int rc = kinds[i] == SV_OP_FUSED ? apply_fused(h, k, qubits + qo, d)
                                               : apply_diag(h, k, qubits + qo, d);
        if (rc) return rc;
        d += (kinds[i] == SV_OP_FUSED ? ((size_t)1 << (2 * k)) : ((size_t)1 << k)) * h->amp;
        qo += (size_t)k;
    }
    return SV_OK;
}

int permute_qubits(sv_handle h, const int* order)
{
    CHECK_HANDLE(h);
    if (!order) return set_err(h, SV_EINVAL, "order is NULL");
    std::vector<int> seen(h->n, 0);
    for (int p = 0; p < h->n; ++p) {
        if (order[p] < 0 || order[p] >= h->n || seen[order[p]]) return set_err(h, SV_EINVAL, "order is not a permutation");
        seen[order[p]] = 1;
    }
    std::vector<int> npos(h->n);
    for (int p = 0; p < h->n; ++p) npos[order[p]] = p;
    bool same = true;
    for (int q = 0; q < h->n; ++q) same = same && (npos[q] == h->pos[q]);
    if (same) return SV_OK;

    // |0...0> is the same in every layout: a resident state that is still
    // |0...0> (reset, or no operation since it was created as |0...0>) only
    // takes the new layout
    if (!h->tier && h->ops.empty() && (h->e0_pending || h->support == 0)) {
        h->pos = npos;
        for (int p = 0; p < h->n; ++p) h->order[p] = order[p];
        return SV_OK;
    }

    if (!h->tier) {
        int rc = flush(h);
        if (rc) return rc;
        if (!h->scratch) {
            if (hipMalloc(&h->scratch, h->dev_bytes) != hipSuccess) {
                h->scratch = nullptr;
                (void)hipGetLastError();
                return set_err(h, SV_ENOMEM, "no device memory for the permute buffer");
            }
        }
        // out[new index] = in[old index]: destination bit npos[q] <- source bit pos[q]
        std::vector<int> from(h->n), to(h->n);
        for (int q = 0; q < h->n; ++q) { from[q] = npos[q]; to[q] = h->pos[q]; }
        const BitRuns r = make_runs(h->n, from.data(), to.data());
        TRY(h, launch_bitperm(h->stream, h->dev, h->scratch, h->dtype, h->n, r));
        if (h->own_dev) {
            std::swap(h->dev, h->scratch);       // both buffers are the handle's own
        } else {
            // the amplitudes stay in the caller's buffer
            TRY(h, hipMemcpyAsync(h->dev, h->scratch, ((size_t)1 << h->n) * h->amp,
                                  hipMemcpyDeviceToDevice, h->stream));
        }
        // the positions that can be non-zero move with their qubits
        uint64_t moved = 0;
        for (int q = 0; q < h->n; ++q)
            if ((h->support >> h->pos[q]) & 1) moved |= (uint64_t)1 << npos[q];
        h->support = moved;
        h->counters[2] += 1;
        h->counters[3] += (int64_t)1 << h->n;
    } else {
        // (1) per-slice local permute bringing the qubits that become sliced
        //     into the file positions [L-s, L); (2) relabel files; (3) per-slice
        //     local permute to the requested local order (queued for the next pass).
        const int L = h->L, s = h->s, F = L - s;
        std::vector<int> mid(h->n);              // intermediate position of each qubit
        for (int q = 0; q < h->n; ++q) mid[q] = h->pos[q];
        std::vector<int> incoming;               // new sliced qubits now in [0, F)
        for (int q = 0; q < h->n; ++q)
            if (npos[q] >= L && h->pos[q] < F) incoming.push_back(q);
        std::vector<int> evict;                  // file-region qubits that stay local
        for (int p = F; p < L; ++p) {
            const int q = h->order[p];
            if (npos[q] < L) evict.push_back(q);
        }
        if (evict.size() < incoming.size()) return set_err(h, SV_EINVAL, "internal: file region too small");
        for (size_t i = 0; i < incoming.size(); ++i) std::swap(mid[incoming[i]], mid[evict[i]]);
        bool moved1 = false;
        for (int q = 0; q < h->n; ++q) moved1 = moved1 || (mid[q] != h->pos[q]);
        if (moved1) {
            Op op;
            op.kind = OP_LPERM;
            std::vector<int> from, to;
            for (int q = 0; q < h->n; ++q)
                if (h->pos[q] < L) { from.push_back(mid[q]); to.push_back(h->pos[q]); }
            op.runs = make_runs((int)from.size(), from.data(), to.data());
            h->ops.push_back(op);
        }
        int rc = flush(h);
        if (rc) return rc;
        // (2) top 2s positions [F, n): after (1) every new sliced qubit is there.
        // new positions within the top block: sliced ones go to npos; the others
        // (becoming or staying file-region) keep npos if it is in [F, L), else
        // take the remaining file slots in ascending order.
        std::vector<int> top_new(h->n, -1);
        std::vector<int> used(h->n, 0);
        for (int q = 0; q < h->n; ++q)
            if (mid[q] >= F && npos[q] >= F) { top_new[q] = npos[q]; used[npos[q]] = 1; }
        int slot = F;
        for (int q = 0; q < h->n; ++q) {
            if (mid[q] >= F && top_new[q] < 0) {
                while (used[slot]) ++slot;
                top_new[q] = slot;
                used[slot] = 1;
            }
        }
        // file pointer relabel: old top index (bits at mid positions) -> new top index
        const int ns = 1 << s, nf = 1 << (2 * s);
        std::vector<void*> nfiles(nf, nullptr);
        std::vector<uint8_t> nzero(ns, 1);
        for (int oldidx = 0; oldidx < nf; ++oldidx) {
            int newidx = 0;
            for (int q = 0; q < h->n; ++q)
                if (mid[q] >= F && ((oldidx >> (mid[q] - F)) & 1)) newidx |= 1 << (top_new[q] - F);
            const int ot = oldidx >> s, nt = newidx >> s;
            nfiles[newidx] = h->files[oldidx];
            if (!h->slice_zero[ot]) nzero[nt] = 0;
        }
        // files of slice t are stored at [t * 2^s + u]: the index above is (t << s) | u
        h->files.swap(nfiles);
        h->slice_zero.swap(nzero);
        // (3) remaining local permutation
        std::vector<int> cur(h->n);
        for (int q = 0; q < h->n; ++q) cur[q] = mid[q] >= F ? top_new[q] : mid[q];
        bool moved3 = false;
        for (int q = 0; q < h->n; ++q) moved3 = moved3 || (cur[q] != npos[q]);
        if (moved3) {
            Op op;
            op.kind = OP_LPERM;
            std::vector<int> from, to;
            for (int q = 0; q < h->n; ++q)
                if (npos[q] < L) { from.push_back(npos[q]); to.push_back(cur[q]); }
            op.runs = make_runs((int)from.size(), from.data(), to.data());
            h->ops.push_back(op);
        }
    }
    h->pos = npos;
    for (int p = 0; p < h->n; ++p) h->order[p] = order[p];
    return SV_OK;
}

int gather_amplitudes(sv_handle h, int64_t count, const uint64_t* bitstrings, void* out_c128)
{
    return do_reduce(h, nullptr, count, bitstrings, out_c128, nullptr);
}

int reduce_slices(sv_handle h, const void* trailing_c128, int64_t count, const uint64_t* bitstrings,
                  void* out_c128, double stats[3])
{
    return do_reduce(h, trailing_c128, count, bitstrings, out_c128, stats);
}

int sv_checkpoint(sv_handle h, int64_t tag)
{
    CHECK_HANDLE(h);
    if (h->file_fds.empty() || h->tier_dir.empty())
        return set_err(h, SV_EINVAL, "checkpoints need a host tier in files (create_state_files)");
    int rc = sync_state(h);                 // every queued operation applied, every file written back
    if (rc) return rc;
    const size_t fb = file_amps(h) * h->famp;
    for (size_t i = 0; i < h->files.size(); ++i)
        if (msync(h->files[i], fb, MS_SYNC) != 0) return set_err(h, SV_EIO, "msync of a tier file failed");
    std::string meta = "sv_checkpoint 1\n";
    meta += "n " + std::to_string(h->n) + "\n";
    // the qubits sliced now (those at the top positions), not at creation
    uint64_t sliced = 0;
    for (int p = h->L; p < h->n; ++p) sliced |= 1ull << h->order[p];
    meta += "slice_mask " + std::to_string((unsigned long long)sliced) + "\n";
    meta += "dtype " + std::to_string(h->dtype | (h->store32 ? SV_FLAG_STORE32 : 0)) + "\n";
    meta += "tag " + std::to_string((long long)tag) + "\n";
    meta += "order";
    for (int p = 0; p < h->n; ++p) meta += " " + std::to_string(h->order[p]);
    meta += "\nslice_zero";
    for (uint8_t z : h->slice_zero) meta += z ? " 1" : " 0";
    // logical file i is the file now mapped at files[i] (a change of the
    // sliced set relabels files instead of moving them)
    meta += "\nfiles " + std::to_string(h->files.size()) + "\n";
    for (void* p : h->files) {
        size_t j = 0;
        while (j < h->file_maps.size() && h->file_maps[j] != p) ++j;
        if (j == h->file_maps.size()) return set_err(h, SV_EIO, "internal: tier file without a path");
        meta += h->file_paths[j].substr(h->file_paths[j].rfind('/') + 1) + "\n";
    }
    {
        char b[64];
        std::snprintf(b, sizeof b, "bound %.17g\n", h->amp_bound);
        meta += b;
    }
    // write, flush and rename: a crash leaves the previous checkpoint or this one whole
    const std::string final_path = h->tier_dir + "/" + kCheckpointName;
    const std::string tmp = final_path + ".tmp";
    const int fd = open(tmp.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0600);
    if (fd < 0) return set_err(h, SV_EIO, "cannot write " + tmp);
    const bool ok = write(fd, meta.data(), meta.size()) == (ssize_t)meta.size() && fsync(fd) == 0;
    (void)close(fd);
    if (!ok || rename(tmp.c_str(), final_path.c_str()) != 0) {
        (void)unlink(tmp.c_str());
        return set_err(h, SV_EIO, "cannot write " + final_path);
    }
    const int dfd = open(h->tier_dir.c_str(), O_RDONLY | O_DIRECTORY);
    if (dfd >= 0) { (void)fsync(dfd); (void)close(dfd); }
    return SV_OK;
}

int open_state_files(const char* dir, void* hip_stream, sv_handle* out, int64_t* tag)
{
    if (!dir || !*dir || !out) return set_err(nullptr, SV_EINVAL, "directory or out is NULL");
    const std::string path = std::string(dir) + "/" + kCheckpointName;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return set_err(nullptr, SV_EIO, "no checkpoint in " + std::string(dir));
    std::vector<char> buf(1 << 20);
    const size_t got = std::fread(buf.data(), 1, buf.size() - 1, f);
    std::fclose(f);
    buf[got] = 0;
    std::string text(buf.data());
    size_t at = 0;
    auto word = [&]() -> std::string {
        while (at < text.size() && std::isspace((unsigned char)text[at])) ++at;
        const size_t b = at;
        while (at < text.size() && !std::isspace((unsigned char)text[at])) ++at;
        return text.substr(b, at - b);
    };
    auto num = [&](long long lo, long long hi, long long* v) -> bool {
        const std::string w = word();
        if (w.empty()) return false;
        char* end = nullptr;
        errno = 0;
        const long long x = std::strtoll(w.c_str(), &end, 10);
        if (errno || *end || x < lo || x > hi) return false;
        *v = x;
        return true;
    };
    long long version = 0, n = 0, dtype = 0, t = 0, nfiles = 0;
    unsigned long long mask = 0;
    bool ok = word() == "sv_checkpoint" && num(1, 1, &version) && word() == "n" && num(1, 40, &n) &&
              word() == "slice_mask";
    if (ok) {
        const std::string w = word();
        char* end = nullptr;
        mask = std::strtoull(w.c_str(), &end, 10);
        ok = !w.empty() && !*end && (n >= 64 || (mask >> n) == 0);
    }
    ok = ok && word() == "dtype" && num(0, 0xfff, &dtype) && word() == "tag" &&
         num(-(1ll << 62), 1ll << 62, &t) && word() == "order";
    const int s = __builtin_popcountll(mask);
    Restore rs;
    if (ok) {
        std::vector<int> seen(n, 0);
        for (long long p = 0; p < n && ok; ++p) {
            long long q = 0;
            ok = num(0, n - 1, &q) && !seen[q];
            if (ok) { seen[q] = 1; rs.order.push_back((int)q); }
        }
        // the top s positions must hold the sliced qubits
        for (long long p = n - s; p < n && ok; ++p) ok = (mask >> rs.order[p]) & 1;
    }
    ok = ok && s >= 1 && s <= 12 && word() == "slice_zero";
    for (int i = 0; ok && i < (1 << s); ++i) {
        long long z = 0;
        ok = num(0, 1, &z);
        rs.slice_zero.push_back((uint8_t)z);
    }
    ok = ok && word() == "files" && num(1, 1 << 24, &nfiles) && nfiles == (1ll << (2 * s));
    for (long long i = 0; ok && i < nfiles; ++i) {
        const std::string w = word();
        ok = !w.empty() && w.find('/') == std::string::npos && w != "." && w != "..";
        rs.names.push_back(w);
    }
    // the amplitude bound (infinite when absent or unreadable)
    double bound = HUGE_VAL;
    if (ok && word() == "bound") {
        const std::string w = word();
        char* end = nullptr;
        const double v = std::strtod(w.c_str(), &end);
        if (!w.empty() && !*end && v >= 0.0) bound = v;
    }
    if (!ok) return set_err(nullptr, SV_EINVAL, "malformed checkpoint " + path);
    const int rc = create_common((int)n, mask, (int)dtype | SV_FLAG_TIER, hip_stream, nullptr, 0, out, dir, &rs);
    if (rc) return rc;
    (*out)->amp_bound = bound;
    if (tag) *tag = t;
    return SV_OK;
}

int sync_state(sv_handle h)
{
    CHECK_HANDLE(h);
    int rc = flush(h);
    if (rc) return rc;
    TRY(h, hipStreamSynchronize(h->stream));
    return SV_OK;
}

int sv_reset(sv_handle h)
{
    CHECK_HANDLE(h);
    h->ops.clear();
    h->arena.clear();
    h->amp_bound = 1.0;
    if (!h->tier) {
        h->e0_pending = true;        // written by the first pass or on demand
        h->support = h->sparse_start ? 0 : ~0ull;
        h->garbage = h->sparse_start;
        return SV_OK;
    }
    TRY(h, hipStreamSynchronize(h->stream));
    TRY(h, hipStreamSynchronize(h->s_in));
    TRY(h, hipStreamSynchronize(h->s_out));
    const size_t fb = file_amps(h) * h->famp;
    for (size_t i = 0; i < h->files.size(); ++i) {
        void* f = h->files[i];
        if (h->pinned_tier) {
            std::memset(f, 0, fb);
        } else if (!h->file_fds.empty()) {
            // file blocks freed: they read back as zero
            if (fallocate(h->file_fds[i], FALLOC_FL_PUNCH_HOLE | FALLOC_FL_KEEP_SIZE, 0, (off_t)fb) != 0)
                std::memset(f, 0, fb);
        } else {
            (void)madvise(f, fb, MADV_DONTNEED);      // pages read back as zero
        }
    }
    if (h->famp == 16) { double one[2] = {1.0, 0.0}; std::memcpy(h->files[0], one, 16); }
    else { float one[2] = {1.0f, 0.0f}; std::memcpy(h->files[0], one, 8); }
    // |0...0> sits in slice 0, file 0 only if index 0 maps there: it does in
    // every layout (all bits zero)
    std::fill(h->slice_zero.begin(), h->slice_zero.end(), (uint8_t)1);
    h->slice_zero[0] = 0;
    return SV_OK;
}

const char* last_error(sv_handle h)
{
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

int sv_get_order(sv_handle h, int* order)
{
    if (!h || !order) return SV_EINVAL;
    for (int p = 0; p < h->n; ++p) order[p] = h->order[p];
    return SV_OK;
}

int sv_device_buffer(sv_handle h, void** dev, size_t* bytes)
{
    if (!h || !dev || !bytes) return SV_EINVAL;
    CHECK_HANDLE(h);
    {
        const int rc = materialize_state(h);
        if (rc) return rc;
    }
    h->support = ~0ull;              // the caller may write it
    if (!h->tier) h->amp_bound = HUGE_VAL;
    *dev = h->tier ? nullptr : h->dev;
    *bytes = h->tier ? 0 : ((size_t)1 << h->n) * h->amp;
    return SV_OK;
}

int sv_set_option(sv_handle h, int option, int64_t value)
{
    CHECK_HANDLE(h);
    switch (option) {
        case SV_OPT_TIMING: h->timing = value != 0; return SV_OK;
        case SV_OPT_MFMA:
            if (value < 0 || value > 64) return set_err(h, SV_EINVAL, "SV_OPT_MFMA: k out of range");
            h->mfma_min_k = (int)value;
            return SV_OK;
        case SV_OPT_FOLD_DIAG: h->fold = value != 0; return SV_OK;
        case SV_OPT_SLOTS: return set_err(h, SV_EINVAL, "slot count is fixed at creation");
        case SV_OPT_STAGE:
            if (value != 0 && (value < 9 || value > 14))
                return set_err(h, SV_EINVAL, "SV_OPT_STAGE: 0 or 9..14 positions");
            h->stage_t = (int)value;
            return SV_OK;
        case SV_OPT_FAIL_IO: h->fail_io_at = value; return SV_OK;
        case SV_OPT_SPARSE_START: h->sparse_start = value != 0; return SV_OK;
        case SV_OPT_SPLIT: h->split = value != 0; return SV_OK;
        case SV_OPT_KEEP_FILES:
            if (h->file_fds.empty()) return set_err(h, SV_EINVAL, "SV_OPT_KEEP_FILES: the tier is not in files");
            h->keep_files = value != 0;
            return SV_OK;
    }
    return set_err(h, SV_EINVAL, "unknown option");
}

int sv_counters(sv_handle h, int64_t counters[8])
{
    if (!h || !counters) return SV_EINVAL;
    for (int i = 0; i < 8; ++i) counters[i] = h->counters[i];
    return SV_OK;
}

int sv_stage_forms(sv_handle h, int64_t passes[2], double* amp_bound)
{
    if (!h) return SV_EINVAL;
    if (passes) {
        passes[0] = h->stage_forms[0];
        passes[1] = h->stage_forms[1];
    }
    if (amp_bound) {
        double b = h->amp_bound;
        for (Op& op : h->ops) {
            size_op(op, h->arena.data(), h->amp);
            b *= op.growth;
        }
        *amp_bound = b;
    }
    return SV_OK;
}

static void reset_timing(sv_state* h)
{
    h->t_ms = 0.0;
    h->t_count = 0;
    for (int k = 0; k < 2; ++k) {
        h->tk_ms[k] = 0.0;
        h->tk_count[k] = 0;
        h->tk_flops[k] = 0.0;
        h->tk_issued[k] = 0.0;
        h->tk_bytes[k] = 0.0;
    }
}

int sv_sweep_time(sv_handle h, double* total_ms, int64_t* count)
{
    CHECK_HANDLE(h);
    int rc = collect_timing(h);
    if (rc) return rc;
    if (total_ms) *total_ms = h->t_ms;
    if (count) *count = h->t_count;
    reset_timing(h);
    return SV_OK;
}

int sv_contract(const void* t1, const void* t2, void* out, int n1, int n2, int e, int dtype, void* hip_stream)
{
    const bool split = !(dtype & SV_CONTRACT_FP32);
    dtype &= ~SV_CONTRACT_FP32;
    if (!t1 || !t2 || !out) return set_err(nullptr, SV_EINVAL, "sv_contract: NULL buffer");
    if (dtype != SV_C64 && dtype != SV_C128) return set_err(nullptr, SV_EINVAL, "sv_contract: bad dtype");
    if (n1 < 0 || n2 < 0 || e < 0 || e > 30 || n1 + n2 > 40 || n1 + e > 40 || n2 + e > 40)
        return set_err(nullptr, SV_EINVAL, "sv_contract: sizes out of range");
    if (((uintptr_t)t1 | (uintptr_t)t2 | (uintptr_t)out) & 15)
        return set_err(nullptr, SV_EINVAL, "sv_contract: buffers must be 16-byte aligned");
    const size_t amp = dtype == SV_C64 ? 8 : 16;
    const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (amp << (n1 + n2));
    for (const void* p : {t1, t2}) {
        const int np = p == t1 ? n1 : n2;
        const uintptr_t p0 = (uintptr_t)p, p1 = p0 + (amp << (np + e));
        if (p0 < o1 && o0 < p1) return set_err(nullptr, SV_EINVAL, "sv_contract: output overlaps an input");
    }
    const hipError_t err = launch_contract((hipStream_t)hip_stream, t1, t2, out, n1, n2, e, dtype, split);
    if (err != hipSuccess) return fail_dev(nullptr, "sv_contract launch", err);
    return SV_OK;
}

int sv_sweep_profile(sv_handle h, double ms[2], int64_t count[2], double flops[2], double issued[2],
                     double bytes[2])
{
    CHECK_HANDLE(h);
    int rc = collect_timing(h);
    if (rc) return rc;
    for (int k = 0; k < 2; ++k) {
        if (ms) ms[k] = h->tk_ms[k];
        if (count) count[k] = h->tk_count[k];
        if (flops) flops[k] = h->tk_flops[k];
        if (issued) issued[k] = h->tk_issued[k];
        if (bytes) bytes[k] = h->tk_bytes[k];
    }
    reset_timing(h);
    return SV_OK;
}

}  // extern "C"

int sv::materialize_e0(sv_state* h)
{
    return materialize_state(h);
}

// ---- staged-run formation (shared with the batch executor) -----------------
int sv::form_stage_run(const Op* ops, size_t nops, size_t i, int stage_t, int nloc, bool fold, int* ks, int dtype)
{
    bool in[64] = {};
    for (int p = 0; p < 4; ++p) in[p] = true;
    int cnt = 0;
    for (size_t j = i; j < nops && cnt < kStageRunMax; ++j) {
        const Op& q = ops[j];
        if (q.kind != OP_DENSE || (q.k != 4 && q.k != 5)) break;
        if (fold && j + 1 < nops && ops[j + 1].kind == OP_DIAG) break;
        bool in2[64];
        for (int p = 0; p < 64; ++p) in2[p] = in[p];
        for (int u = 0; u < q.k; ++u) in2[q.pos[u]] = true;
        int t = 0;
        for (int p = 0; p < 64; ++p) t += in2[p];
        if (t < 9) t = 9;
        ks[cnt] = q.k;
        if (t > stage_t || t > stage_max_t(dtype) || t > nloc ||
            stage_lds_bytes(t, cnt + 1, ks, dtype) > stage_lds_limit(t, dtype))
            break;
        for (int p = 0; p < 64; ++p) in[p] = in2[p];
        ++cnt;
    }
    return cnt;
}

int sv::reduce_with(sv_state* h, const void* trailing, int64_t count, const uint64_t* bits, void* out,
                    double* stats, const WorkBufs* wb)
{
    return do_reduce(h, trailing, count, bits, out, stats, wb);
}
