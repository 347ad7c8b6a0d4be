// Batch executor: many resident states, their queued operations applied
// round by round with one launch per (kernel form, k, fold) per round, all
// rounds optionally captured into one HIP graph (see sv_batch_prepare in
// include/sv.h).
//
// Sweep r of every state goes into round r.  Within a round the sweeps of
// different states touch different buffers, so they share a launch; rounds
// are ordered on one stream, which keeps every state's own op order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sv.h"
#include "sv_internal.h"
#include "sv_state.h"

using namespace sv;

namespace {

struct Launch {
    int kind;          // 0 dense VALU, 1 dense MFMA, 2 diagonal, 3 staged pass (one state each),
                       // 4 write |0...0>, 5 zero outside the support (one state each)
    int dtype, k;
    bool fold;
    bool staged;       // MFMA: address-ordered LDS staging
    size_t first;      // index of the first Sweep item
    int nitems;
    uint64_t blocks;
    // diagonal and staged launches
    void* psi;
    int nloc;
    DiagSpec diag;
    int cnt, t_max;                           // staged: blocks, tile limit
    int ks[kStageRunMax];
    int spos[kStageRunMax][6];
    const void* smat[kStageRunMax];
    // run from a reset: staged passes start from |0...0> or visit only the
    // support's tiles; kind 5 clears outside `support`
    bool from_e0 = false, garbage = false;
    uint64_t support = ~0ull;
    int split_exp = kNoSplit;                 // staged: split-fp16 tile scale exponent
};

}  // namespace

struct sv_batch_s {
    std::vector<sv_state*> states;
    // each state's buffer and layout when the batch was prepared: the
    // recorded launches address both
    std::vector<void*> devs;
    std::vector<std::vector<int>> orders;
    // per state: the product of its ops' growth factors (the amplitude
    // bound advances by it at every launch)
    std::vector<double> gprod;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* d_arena = nullptr;
    void* d_items = nullptr;
    std::vector<Launch> launches;
    // the same rounds for states all reset since their last use: no |0...0>
    // writes ahead, staged passes visit only the tiles that can be non-zero
    std::vector<Launch> launches_reset;
    hipGraph_t graph = nullptr, graph_reset = nullptr;
    hipGraphExec_t exec = nullptr, exec_reset = nullptr;
    hipEvent_t ev_done = nullptr;
    std::vector<hipEvent_t> ev_in;
    int64_t sweeps = 0;
    double amps_swept = 0, amps_swept_reset = 0;
    bool last_reset = false;                 // variant of the last launch
    std::string err;
};

namespace {

thread_local std::string g_batch_error;

int berr(sv_batch_s* b, int code, const std::string& m)
{
    if (b) b->err = m;
    else g_batch_error = m;
    return code;
}

void free_batch(sv_batch_s* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->exec_reset) (void)hipGraphExecDestroy(b->exec_reset);
    if (b->graph_reset) (void)hipGraphDestroy(b->graph_reset);
    if (b->d_arena) (void)hipFree(b->d_arena);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->ev_done) (void)hipEventDestroy(b->ev_done);
    for (hipEvent_t e : b->ev_in) (void)hipEventDestroy(e);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

hipError_t enqueue_all(sv_batch_s* b, const std::vector<Launch>& launches)
{
    const Sweep* items = (const Sweep*)b->d_items;
    for (const Launch& L : launches) {
        hipError_t e = hipSuccess;
        if (L.kind == 0)
            e = launch_dense_batch(b->stream, L.dtype, L.k, L.fold, items + L.first, L.nitems, L.blocks);
        else if (L.kind == 1)
            e = launch_dense_mfma_batch(b->stream, L.k, L.fold, L.staged, items + L.first, L.nitems,
                                        L.blocks);
        else if (L.kind == 2)
            e = launch_diag(b->stream, L.psi, L.dtype, L.nloc, 0, L.diag);
        else if (L.kind == 4)
            e = launch_init(b->stream, L.psi, L.dtype, (uint64_t)1 << L.nloc, true);
        else if (L.kind == 5)
            e = launch_zero_outside(b->stream, L.psi, L.dtype, L.nloc, L.support);
        else {
            const int* pp[kStageRunMax];
            for (int c = 0; c < L.cnt; ++c) pp[c] = L.spos[c];
            int t = 0;
            e = launch_stage(b->stream, L.psi, L.nloc, L.cnt, L.ks, pp, L.smat, L.t_max, L.from_e0, nullptr,
                             nullptr, &t, L.support, L.garbage, nullptr, nullptr, L.split_exp);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int sv_batch_prepare(int count, sv_handle* handles, int flags, void* hip_stream, sv_batch* out)
{
    if (!out || !handles || count < 1) return berr(nullptr, SV_EINVAL, "bad batch arguments");
    const int dtype = handles[0] ? handles[0]->dtype : -1;
    for (int i = 0; i < count; ++i) {
        sv_state* h = handles[i];
        if (!h) return berr(nullptr, SV_EINVAL, "NULL handle in batch");
        if (h->poisoned) return SV_ESTATE;
        if (h->tier) return berr(nullptr, SV_EINVAL, "batched states must be resident in HBM");
        if (h->dtype != dtype) return berr(nullptr, SV_EINVAL, "batched states must share a dtype");
        for (int j = 0; j < i; ++j)
            if (handles[j] == h) return berr(nullptr, SV_EINVAL, "duplicate handle in batch");
        for (const auto& op : h->ops)
            if (op.kind == OP_LPERM) return berr(nullptr, SV_EINVAL, "queued permute in a batched state");
    }
    sv_batch_s* b = new (std::nothrow) sv_batch_s();
    if (!b) return berr(nullptr, SV_ENOMEM, "host allocation failed");
    b->states.assign(handles, handles + count);
    for (int i = 0; i < count; ++i) {
        sv_state* h = handles[i];
        b->devs.push_back(h->dev);
        b->orders.push_back(h->order);
        double gp = 1.0;
        for (Op& op : h->ops) {
            size_op(op, h->arena.data(), h->amp);
            gp *= op.growth;
        }
        b->gprod.push_back(gp);
    }
    hipError_t e;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { free_batch(b); return berr(nullptr, SV_EDEVICE, "stream creation failed"); }
        b->own_stream = true;
    }

    // one device arena holding every state's matrices and tables
    std::vector<size_t> abase(count);
    size_t atot = 0;
    for (int i = 0; i < count; ++i) {
        abase[i] = atot;
        atot += (handles[i]->arena.size() + 255) & ~(size_t)255;
    }
    if (atot) {
        if (hipMalloc(&b->d_arena, atot) != hipSuccess) {
            (void)hipGetLastError();
            free_batch(b);
            return berr(nullptr, SV_ENOMEM, "device allocation of the batch arena failed");
        }
        for (int i = 0; i < count; ++i)
            if (!handles[i]->arena.empty()) {
                e = hipMemcpy((char*)b->d_arena + abase[i], handles[i]->arena.data(),
                              handles[i]->arena.size(), hipMemcpyHostToDevice);
                if (e != hipSuccess) { free_batch(b); return berr(nullptr, SV_EDEVICE, "arena upload failed"); }
            }
    }

    // per state: its sweeps (dense + folded diagonal, diagonal alone, or a
    // staged run of 4/5-qubit blocks formed as for the state alone)
    struct Sw { int kind; const Op* op; const Op* fold; int cnt; int ks[kStageRunMax]; };
    std::vector<std::vector<Sw>> sweeps(count);
    size_t rounds = 0;
    bool any_staged = false;
    for (int i = 0; i < count; ++i) {
        sv_state* h = handles[i];
        const auto& ops = h->ops;
        const bool can_stage = h->dtype == 0 && h->stage_t >= 9 && h->mfma_min_k == 4;
        for (size_t j = 0; j < ops.size(); ++j) {
            if (can_stage && ops[j].kind == OP_DENSE && (ops[j].k == 4 || ops[j].k == 5)) {
                Sw w{3, &ops[j], nullptr, 0, {}};
                w.cnt = form_stage_run(ops.data(), ops.size(), j, h->stage_t, h->n, h->fold, w.ks);
                // a lone unitary block also takes a staged pass, as run_ops
                // gives it (split-fp16 form in the reset variant)
                if (w.cnt >= 2 || (w.cnt == 1 && h->split && ops[j].unit)) {
                    sweeps[i].push_back(w);
                    j += w.cnt - 1;
                    any_staged = true;
                    continue;
                }
            }
            if (ops[j].kind == OP_DENSE) {
                const Op* f = nullptr;
                if (h->fold && j + 1 < ops.size() && ops[j + 1].kind == OP_DIAG) f = &ops[++j];
                sweeps[i].push_back({0, &ops[j - (f ? 1 : 0)], f, 0, {}});
            } else {
                sweeps[i].push_back({2, &ops[j], nullptr, 0, {}});
            }
        }
        rounds = std::max(rounds, sweeps[i].size());
    }

    // the reset variant: per state, the positions reached since the reset,
    // whether |0...0> is still unwritten and whether memory outside the
    // support still holds older values
    std::vector<uint64_t> rs_support(count, 0);
    std::vector<double> rs_bound(count, 1.0);     // amplitude bound through the ops, from |0...0>
    std::vector<char> rs_e0(count, 1), rs_garbage(count, 1);
    auto rs_full = [&](int i) { return ((uint64_t)1 << handles[i]->n) - 1; };
    auto rs_materialize = [&](int i) {
        sv_state* h = handles[i];
        Launch M{};
        M.dtype = h->dtype;
        M.psi = h->dev;
        M.nloc = h->n;
        if (rs_e0[i]) {
            M.kind = 4;
            b->launches_reset.push_back(M);
        } else if (rs_garbage[i] && (rs_support[i] & rs_full(i)) != rs_full(i)) {
            M.kind = 5;
            M.support = rs_support[i];
            b->launches_reset.push_back(M);
        }
        rs_e0[i] = 0;
        rs_garbage[i] = 0;
    };

    std::vector<Sweep> items;
    for (size_t r = 0; r < rounds; ++r) {
        // (form, k, fold) -> item indices of this round, in state order
        std::map<std::tuple<int, int, int>, std::vector<Sweep>> groups;
        for (int i = 0; i < count; ++i) {
            if (r >= sweeps[i].size()) continue;
            sv_state* h = handles[i];
            const Sw& w = sweeps[i][r];
            const char* ab = (const char*)b->d_arena + abase[i];
            b->sweeps += 1;
            b->amps_swept += (double)((uint64_t)1 << h->n);
            if (w.kind == 3) {
                Launch L{};
                L.kind = 3;
                L.dtype = h->dtype;
                L.psi = h->dev;
                L.nloc = h->n;
                L.cnt = w.cnt;
                L.t_max = h->stage_t;
                bool unit = h->split;
                double bmax = rs_bound[i];
                for (int c = 0; c < w.cnt; ++c) {
                    L.ks[c] = w.ks[c];
                    for (int u = 0; u < w.ks[c]; ++u) L.spos[c][u] = w.op[c].pos[u];
                    L.smat[c] = ab + w.op[c].off;
                    unit = unit && w.op[c].unit;
                    bmax *= std::max(1.0, w.op[c].growth);
                    rs_bound[i] *= w.op[c].growth;
                }
                b->launches.push_back(L);
                // from a reset the amplitude bound is known (1): that variant
                // takes the split-fp16 form, the other the fp32 form
                Launch R = L;
                R.split_exp = unit ? split_exponent(bmax) : kNoSplit;
                h->stage_forms[R.split_exp != kNoSplit ? 0 : 1] += 1;
                R.from_e0 = rs_e0[i] != 0;
                R.support = rs_support[i];
                R.garbage = rs_garbage[i] != 0;
                b->launches_reset.push_back(R);
                {
                    const int* pp[kStageRunMax];
                    for (int c = 0; c < w.cnt; ++c) pp[c] = L.spos[c];
                    b->amps_swept_reset += (double)stage_visits(h->n, w.cnt, w.ks, pp, h->stage_t, rs_support[i]);
                }
                for (int c = 0; c < w.cnt; ++c)
                    for (int u = 0; u < w.ks[c]; ++u) rs_support[i] |= (uint64_t)1 << w.op[c].pos[u];
                rs_e0[i] = 0;
                if ((rs_support[i] & rs_full(i)) == rs_full(i)) rs_garbage[i] = 0;
                h->counters[0] += 1;
                h->counters[3] += (int64_t)1 << h->n;
                h->counters[7] += w.cnt;
                continue;
            }
            rs_bound[i] *= w.op->growth * (w.fold ? w.fold->growth : 1.0);
            // a plain sweep needs every amplitude in memory
            rs_materialize(i);
            rs_support[i] = ~0ull;
            b->amps_swept_reset += (double)((uint64_t)1 << h->n);
            if (w.kind == 2) {
                Launch L{};
                L.kind = 2;
                L.dtype = h->dtype;
                L.psi = h->dev;
                L.nloc = h->n;
                L.diag.m = w.op->k;
                for (int t = 0; t < w.op->k; ++t) L.diag.pos[t] = w.op->pos[t];
                L.diag.table = ab + w.op->off;
                b->launches.push_back(L);
                b->launches_reset.push_back(L);
                h->counters[1] += 1;
                h->counters[3] += (int64_t)1 << h->n;
                continue;
            }
            DiagSpec fd;
            if (w.fold) {
                fd.m = w.fold->k;
                for (int t = 0; t < w.fold->k; ++t) fd.pos[t] = w.fold->pos[t];
                fd.table = ab + w.fold->off;
            }
            const int k = w.op->k;
            Sweep s = make_sweep(h->dev, h->n, k, w.op->pos, ab + w.op->off, w.fold ? &fd : nullptr, 0);
            const bool mf = h->dtype == 0 && h->mfma_min_k >= 4 && k >= h->mfma_min_k && h->n >= k + 4;
            // form: 0 VALU, 1 MFMA direct, 3 MFMA staged
            groups[std::make_tuple(mf ? (s.staged ? 3 : 1) : 0, k, w.fold ? 1 : 0)].push_back(s);
            h->counters[0] += 1;
            h->counters[3] += (int64_t)1 << h->n;
        }
        for (auto& kv : groups) {
            Launch L{};
            L.kind = std::get<0>(kv.first) == 3 ? 1 : std::get<0>(kv.first);
            L.staged = std::get<0>(kv.first) == 3;
            L.k = std::get<1>(kv.first);
            L.fold = std::get<2>(kv.first) != 0;
            L.dtype = dtype;
            L.first = items.size();
            L.nitems = (int)kv.second.size();
            uint64_t blk = 0;
            for (Sweep& s : kv.second) {
                s.block0 = blk;
                blk += L.kind == 1 ? mfma_batch_blocks(s.groups) : (s.groups + 255) / 256;
                items.push_back(s);
            }
            L.blocks = blk;
            if (blk > 0x7fffffffull) { free_batch(b); return berr(nullptr, SV_EINVAL, "batch round too large"); }
            b->launches.push_back(L);
            b->launches_reset.push_back(L);
        }
    }
    // the state is read after the batch: everything in memory
    for (int i = 0; i < count; ++i) rs_materialize(i);
    if (!items.empty()) {
        if (hipMalloc(&b->d_items, items.size() * sizeof(Sweep)) != hipSuccess) {
            (void)hipGetLastError();
            free_batch(b);
            return berr(nullptr, SV_ENOMEM, "device allocation of the batch table failed");
        }
        e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(Sweep), hipMemcpyHostToDevice);
        if (e != hipSuccess) { free_batch(b); return berr(nullptr, SV_EDEVICE, "batch table upload failed"); }
    }
    for (int i = 0; i < count; ++i) {
        handles[i]->ops.clear();
        handles[i]->arena.clear();
    }
    e = hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming);
    if (e != hipSuccess) { free_batch(b); return berr(nullptr, SV_EDEVICE, "event creation failed"); }
    b->ev_in.assign(count, nullptr);
    for (auto& ev : b->ev_in)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            free_batch(b);
            return berr(nullptr, SV_EDEVICE, "event creation failed");
        }
    if (flags & SV_BATCH_GRAPH) {
        // kernel attributes are set outside the capture
        if (any_staged && (e = stage_prepare()) != hipSuccess) {
            free_batch(b);
            return berr(nullptr, SV_EDEVICE, "staged kernel set-up failed");
        }
        e = hipSuccess;
        for (int v = 0; v < 2 && e == hipSuccess; ++v) {
            hipGraph_t& g = v ? b->graph_reset : b->graph;
            e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = enqueue_all(b, v ? b->launches_reset : b->launches);
                e = hipStreamEndCapture(b->stream, &g);
                if (e2 != hipSuccess) e = e2;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(v ? &b->exec_reset : &b->exec, g, nullptr, nullptr, 0);
        }
        if (e != hipSuccess) {
            free_batch(b);
            return berr(nullptr, SV_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
        }
    }
    *out = b;
    return SV_OK;
}

int sv_batch_launch(sv_batch b)
{
    if (!b) return berr(nullptr, SV_EINVAL, "NULL batch");
    // every state reset since its last use (sparse start on): the reset
    // variant, which writes |0...0> only where a plain sweep needs it
    bool reset = true;
    for (sv_state* h : b->states) reset = reset && h->e0_pending && h->sparse_start;
    // order after everything already queued on the states' own streams
    for (size_t i = 0; i < b->states.size(); ++i) {
        sv_state* h = b->states[i];
        if (h->poisoned) return SV_ESTATE;
        if (!h->ops.empty()) return berr(b, SV_EINVAL, "state has operations queued after the batch was prepared");
        if (h->dev != b->devs[i] || h->order != b->orders[i])
            return berr(b, SV_EINVAL, "state was re-laid out (permute_qubits) after the batch was prepared");
        // otherwise a deferred reset is written on the state's stream, ahead of the batch
        if (!reset && (h->e0_pending || h->garbage)) {
            const int rc = materialize_e0(h);
            if (rc) return rc;
        }
        h->e0_pending = false;
        h->garbage = false;
        h->support = ~0ull;
        if (hipEventRecord(b->ev_in[i], h->stream) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->ev_in[i], 0) != hipSuccess)
            return berr(b, SV_EDEVICE, "stream ordering failed");
    }
    hipGraphExec_t ex = reset ? b->exec_reset : b->exec;
    b->last_reset = reset;
    hipError_t e = ex ? hipGraphLaunch(ex, b->stream) : enqueue_all(b, reset ? b->launches_reset : b->launches);
    if (e != hipSuccess) {
        for (sv_state* h : b->states) { h->poisoned = true; h->err = "batch launch failed"; }
        return berr(b, SV_EDEVICE, std::string("batch launch failed: ") + hipGetErrorString(e));
    }
    for (size_t i = 0; i < b->states.size(); ++i) {
        sv_state* h = b->states[i];
        h->amp_bound = (reset ? 1.0 : h->amp_bound) * b->gprod[i];
    }
    if (hipEventRecord(b->ev_done, b->stream) != hipSuccess) return berr(b, SV_EDEVICE, "event record failed");
    for (sv_state* h : b->states)
        if (hipStreamWaitEvent(h->stream, b->ev_done, 0) != hipSuccess)
            return berr(b, SV_EDEVICE, "stream ordering failed");
    return SV_OK;
}

int sv_batch_sync(sv_batch b)
{
    if (!b) return berr(nullptr, SV_EINVAL, "NULL batch");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        for (sv_state* h : b->states) { h->poisoned = true; h->err = "batch execution failed"; }
        return berr(b, SV_EDEVICE, std::string("batch execution failed: ") + hipGetErrorString(e));
    }
    return SV_OK;
}

int sv_batch_info(sv_batch b, int64_t info[4])
{
    if (!b || !info) return SV_EINVAL;
    info[0] = (int64_t)(b->last_reset ? b->launches_reset.size() : b->launches.size());
    info[1] = b->sweeps;
    info[2] = (int64_t)(b->last_reset ? b->amps_swept_reset : b->amps_swept);
    info[3] = b->exec ? 1 : 0;
    return SV_OK;
}

int sv_batch_destroy(sv_batch b)
{
    free_batch(b);
    return SV_OK;
}

const char* sv_batch_error(sv_batch b)
{
    return b ? b->err.c_str() : g_batch_error.c_str();
}

}  // extern "C"
