"""Host-side planning of a circuit into library operations (untimed).

* Gate aggregation (Sec. 5): gates are grouped into clusters spanning at most
  k qubits; each cluster becomes one 2^k x 2^k matrix, i.e. one dense sweep.
  Clustering is greedy over the gate list: each open cluster owns a disjoint
  set of qubits; a gate joins (and merges) the clusters it touches when the
  union stays within k qubits, otherwise those clusters are emitted and the
  gate starts a new one.  Per qubit, gate order is preserved, and clusters
  on disjoint qubits commute, so the product is unchanged.
* Diagonal extraction (Sec. 2: diagonal tensors are hyperedges; Eq. 1 has a
  diagonal |11> phase): a two-qubit gate of the Eq. (1) sparsity pattern
  splits exactly into diag(m00, 1, 1, m33) times a gate acting only on the
  |01>, |10> block.  With fold_diag the diagonal part is emitted as its own
  op right after the cluster holding the non-diagonal part, and the library
  folds it into that cluster's sweep as an element-wise phase.
* Staged passes (a second level of cache blocking over the appendix's
  aggregate gates): the device applies a run of consecutive 4/5-qubit
  blocks whose positions, with positions 0..3, fit in one 13-position tile
  in a single HBM pass.
  `order_for_staging` reorders commuting blocks so that such runs are
  consecutive, and `plan` picks among aggregations by a cost model of
  staged and single passes.
* Slice phases (Sec. 4): `phase_schedule` splits the gate list into phases,
  each with a set of sliced qubits on which only diagonal work may happen,
  alternating between two slice sets like the paper's subcircuits 3..9.

All arithmetic here is FP64 on tiny matrices; the results are handed to the
library in the state's dtype.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Op:
    kind: str                       # "dense" | "diag" | "perm"
    qubits: Tuple[int, ...] = ()
    matrix: Optional[np.ndarray] = None   # dense: (2^k, 2^k); diag: (2^m,)
    order: Optional[List[int]] = None     # perm
    ngates: int = 0                 # circuit gates this op carries


def embed_in(block_qubits: Sequence[int], gate_qubits: Sequence[int], g: np.ndarray) -> np.ndarray:
    """Matrix of gate g (index = sum_j b(gate_qubits[j]) 2^j) on the index
    space of block_qubits (a superset), as a 2^k x 2^k array."""
    k = len(block_qubits)
    where = [list(block_qubits).index(q) for q in gate_qubits]
    idx = np.arange(1 << k)
    sub = np.zeros(1 << k, dtype=np.int64)
    rest = idx.copy()
    for j, w in enumerate(where):
        bit = (idx >> w) & 1
        sub |= bit << j
        rest &= ~(1 << w)
    same = rest[:, None] == rest[None, :]
    return np.where(same, g[sub[:, None], sub[None, :]], 0).astype(np.complex128)


def split_eq1(m: np.ndarray):
    """Split a 4x4 of the Eq. (1) pattern into (diag, middle-block gate):
    m = diag(m00, 1, 1, m33) @ x.  Returns None for other matrices."""
    if m.shape != (4, 4):
        return None
    mask = np.zeros((4, 4), dtype=bool)
    mask[0, 0] = mask[3, 3] = True
    mask[1:3, 1:3] = True
    if np.any(m[~mask] != 0):
        return None
    d = np.array([m[0, 0], 1.0, 1.0, m[3, 3]], dtype=np.complex128)
    x = np.eye(4, dtype=np.complex128)
    x[1:3, 1:3] = m[1:3, 1:3]
    return d, x


class _Block:
    __slots__ = ("qubits", "m", "ngates", "first")

    def __init__(self, qubits, m, ngates, first):
        self.qubits = list(qubits)
        self.m = m
        self.ngates = ngates
        self.first = first


def fuse(gates, kmax: int, fold_diag: bool = False) -> List[Op]:
    """Greedy aggregation of `gates` (objects with .qubits, .matrix) into
    dense blocks of at most kmax qubits (and diagonal ops with fold_diag)."""
    ops: List[Op] = []
    owner: Dict[int, _Block] = {}
    counter = [0]

    def emit(b: _Block):
        for q in b.qubits:
            del owner[q]
        ops.append(Op("dense", tuple(b.qubits), b.m, ngates=b.ngates))

    def add_dense(qs, m, ng):
        touching = []
        for q in qs:
            b = owner.get(q)
            if b is not None and b not in touching:
                touching.append(b)
        union = []
        for b in touching:
            union += b.qubits
        for q in qs:
            if q not in union:
                union.append(q)
        if len(union) <= kmax:
            # merge the touching blocks (disjoint: they commute) by Kronecker product
            if touching:
                cur_q = list(touching[0].qubits)
                cur_m = touching[0].m
                ngs = touching[0].ngates
                first = min(b.first for b in touching)
                for b in touching[1:]:
                    cur_m = np.kron(b.m, cur_m)
                    cur_q += b.qubits
                    ngs += b.ngates
                for b in touching:
                    for q in b.qubits:
                        del owner[q]
            else:
                cur_q, cur_m, ngs, first = [], np.eye(1, dtype=np.complex128), 0, counter[0]
            for q in qs:
                if q not in cur_q:
                    cur_m = np.kron(np.eye(2, dtype=np.complex128), cur_m)
                    cur_q.append(q)
            cur_m = embed_in(cur_q, qs, m) @ cur_m
            nb = _Block(cur_q, cur_m, ngs + ng, first)
        else:
            for b in touching:
                emit(b)
            nb = _Block(list(qs), np.array(m, dtype=np.complex128), ng, counter[0])
        for q in nb.qubits:
            owner[q] = nb
        counter[0] += 1

    for g in gates:
        qs = tuple(g.qubits)
        m = np.asarray(g.matrix, dtype=np.complex128)
        parts = split_eq1(m) if (fold_diag and len(qs) == 2) else None
        if parts is None:
            add_dense(qs, m, 1)
            continue
        d, x = parts
        add_dense(qs, x, 1)
        # the diagonal commutes with x (same qubits); emit it right after the
        # block that now holds x, and close that block so no later gate on
        # these qubits is applied before the phase
        b = owner[qs[0]]
        emit(b)
        ops.append(Op("diag", qs, d, ngates=0))
    for b in sorted(set(owner.values()), key=lambda b: b.first):
        ops.append(Op("dense", tuple(b.qubits), b.m, ngates=b.ngates))
    return ops


def fuse_grow(gates, kmax: int, window: int = 4, last_gain: float = 0.0) -> List[Op]:
    """Aggregation by growing qubit sets (Sec. 5 aggregate gates, clusters that
    span several depths as in the appendix listing's cache rows).

    Repeatedly: start from the qubits of the earliest pending gate, add one
    qubit at a time (among the qubits of the pending gates that touch the
    set; `window` next gates per qubit) choosing the one that lets the most
    pending gates be applied inside
    the set, up to kmax qubits; then emit one block holding every pending
    gate that lies inside the set and whose predecessors on each of its
    qubits are already applied (its causal closure within the set).  Per
    qubit, gates keep their order, so the product is unchanged.

    last_gain > 0: the last qubit (growing to kmax) is only added when it
    raises the block's gate weight by that fraction or more; a kmax block
    costs twice the arithmetic of a kmax-1 block, so one that absorbs few
    more gates is not worth it when the passes are compute bound."""
    ng = len(gates)
    qs_of = [tuple(g.qubits) for g in gates]
    per_q: Dict[int, List[int]] = {}
    for i, qs in enumerate(qs_of):
        for q in qs:
            per_q.setdefault(q, []).append(i)
    ptr = {q: 0 for q in per_q}                 # index into per_q[q] of the next pending gate
    done = [False] * ng

    def closure(Q):
        """Pending gates applicable inside Q, in a valid order."""
        loc = {q: ptr[q] for q in Q}
        taken = []
        progress = True
        while progress:
            progress = False
            for q in Q:
                lst = per_q.get(q, [])
                while loc[q] < len(lst):
                    gi = lst[loc[q]]
                    qs = qs_of[gi]
                    if any(x not in Q for x in qs):
                        break
                    if any(per_q[x][loc[x]] != gi for x in qs):
                        break
                    for x in qs:
                        loc[x] += 1
                    taken.append(gi)
                    progress = True
        return taken

    ops: List[Op] = []
    remaining = ng
    while remaining:
        first = min(per_q[q][ptr[q]] for q in per_q if ptr[q] < len(per_q[q]))
        Q = list(qs_of[first])
        best = closure(Q)
        while len(Q) < kmax:
            cands = set()
            for q in Q:
                lst = per_q[q]
                for t in range(ptr[q], min(ptr[q] + window, len(lst))):
                    cands.update(x for x in qs_of[lst[t]] if x not in Q)
            if not cands:
                break
            scored = []
            for c in sorted(cands):
                cl = closure(Q + [c])
                w = sum(len(qs_of[i]) for i in cl)
                scored.append((w, -c, c, cl))
            scored.sort(reverse=True)
            w, _, c, cl = scored[0]
            if last_gain > 0 and len(Q) == kmax - 1 and \
                    w < (1.0 + last_gain) * sum(len(qs_of[i]) for i in best):
                break
            Q.append(c)
            best = cl
        # emit the block
        qlist = []
        for gi in best:
            for q in qs_of[gi]:
                if q not in qlist:
                    qlist.append(q)
        m = np.eye(1 << len(qlist), dtype=np.complex128)
        for gi in best:
            m = embed_in(qlist, qs_of[gi], np.asarray(gates[gi].matrix, dtype=np.complex128)) @ m
            for q in qs_of[gi]:
                ptr[q] += 1
            done[gi] = True
        remaining -= len(best)
        ops.append(Op("dense", tuple(qlist), m, ngates=len(best)))
    return ops


# Staged-pass formation on the device (mirrored here for planning): a run
# holds at most STAGE_MAX_OPS 4/5-qubit blocks, the tile at most STAGE_T
# positions (0..3 always), and the LDS budget covers the tile (2^t complex64
# plus one pad per 16) and Re/Im of every block's matrix: STAGE_LDS up to
# 13 positions (two workgroups per CU), STAGE_LDS14 at 14 (one
# workgroup per CU).  Tiles are widened with support positions to the
# widest width within the limit whose LDS fits (`_tile_positions`).
STAGE_T = 14
STAGE_MAX_OPS = 8
STAGE_LDS = 80 * 1024
STAGE_LDS14 = 160 * 1024


def _lds_limit(t: int) -> int:
    return STAGE_LDS14 if t >= 14 else STAGE_LDS


# Widest tile per state: 14 positions for complex64 (one workgroup
# per CU, fewer passes).  In the split-fp16 form, the default, it measured
# faster at every size: 36.2-36.4 against 39.4-40.5 ms per 30-qubit step
# (14 instead of 17 passes), batches of 20-28 qubits tuned to 14 from 23
# qubits.  The fp32 form (SV_OPT_SPLIT 0) measured slower with 14 at 2^30
# amplitudes (45.8 against 44.6 ms per step), where two workgroups per CU
# overlap its longer block work better; such callers pass 13.  Complex128
# tiles hold at most 13 positions.
STAGE_T_C128 = 13


def stage_tmax(nloc: int, dtype: str = "c64") -> int:
    """Tile limit for a state of 2^nloc amplitudes: at most nloc - 9
    positions, so that a pass has at least 512 tiles, and at most 14 for
    complex64 (13 for complex128); 0 (no staged passes) below 9.  Callers
    pass it to the device as SV_OPT_STAGE for the state."""
    t = min(STAGE_T if dtype == "c64" else STAGE_T_C128, nloc - 9)
    return t if t >= 9 else 0


def _stage_lds(t: int, ks: Sequence[int]) -> int:
    tile = ((1 << t) + ((1 << t) >> 4)) * 8
    return tile + sum(2 * (1 << (2 * k)) for k in ks) * 4


def _stageable(o: "Op") -> bool:
    return o.kind == "dense" and len(o.qubits) in (4, 5)


def _fits(pos: set, ks: Sequence[int], tmax: int) -> bool:
    t = max(9, len(pos))
    return t <= tmax and len(ks) <= STAGE_MAX_OPS and _stage_lds(t, ks) <= _lds_limit(t)


def stage_runs(ops: Sequence["Op"], pos_of=None, tmax: Optional[int] = None) -> List[List[int]]:
    """The runs the device forms from `ops` in this order (lists of indices;
    a single-element list is a sweep of its own)."""
    tmax = STAGE_T if tmax is None else tmax
    pos = (lambda q: q) if pos_of is None else pos_of
    runs: List[List[int]] = []
    i = 0
    while i < len(ops):
        if _stageable(ops[i]):
            P, ks, j = set(range(4)), [], i
            while j < len(ops) and _stageable(ops[j]):
                P2 = P | {pos(q) for q in ops[j].qubits}
                if not _fits(P2, ks + [len(ops[j].qubits)], tmax):
                    break
                P, ks, j = P2, ks + [len(ops[j].qubits)], j + 1
            if j - i >= 2:
                runs.append(list(range(i, j)))
                i = j
                continue
        runs.append([i])
        i += 1
    return runs


def order_for_staging(ops: Sequence["Op"], pos_of=None, tmax: Optional[int] = None) -> List["Op"]:
    """Reorder ops so that blocks which can share a staged pass are adjacent.

    Ops are nodes of a dependency graph (an op depends on the last earlier op
    sharing a qubit); only ops with no path between them change relative
    order, so the product is unchanged (ops on disjoint qubits commute).
    Greedy: take the earliest ready op; if it is a 4/5-qubit block, keep
    adding the ready block that adds the fewest new tile positions (earliest
    first) while the tile and LDS limits hold."""
    tmax = STAGE_T if tmax is None else tmax
    pos = (lambda q: q) if pos_of is None else pos_of
    n = len(ops)
    npred = [0] * n
    succ: List[List[int]] = [[] for _ in range(n)]
    last: Dict[int, int] = {}
    for i, o in enumerate(ops):
        ps = {last[q] for q in o.qubits if q in last}
        for p in ps:
            succ[p].append(i)
        npred[i] = len(ps)
        for q in o.qubits:
            last[q] = i
    ready = {i for i in range(n) if npred[i] == 0}
    out: List[Op] = []

    def take(i):
        ready.discard(i)
        out.append(ops[i])
        for s_ in succ[i]:
            npred[s_] -= 1
            if npred[s_] == 0:
                ready.add(s_)

    while ready:
        first = min(ready)
        take(first)
        if not _stageable(ops[first]):
            continue
        P = set(range(4)) | {pos(q) for q in ops[first].qubits}
        ks = [len(ops[first].qubits)]
        while True:
            best = None
            for i in ready:
                if not _stageable(ops[i]):
                    continue
                P2 = P | {pos(q) for q in ops[i].qubits}
                if not _fits(P2, ks + [len(ops[i].qubits)], tmax):
                    continue
                key = (len(P2) - len(P), i)
                if best is None or key < best[0]:
                    best = (key, i, P2)
            if best is None:
                break
            _, i, P = best
            ks.append(len(ops[i].qubits))
            take(i)
    assert len(out) == n
    return out


# Modelled device time (ms per 2^30 complex64 amplitudes) of a single sweep
# of a k-qubit block, and of a staged pass: the larger of its memory time
# and a fixed part plus a cost per block.  Only the ranking of candidate
# plans uses these figures.  Two forms of the staged kernel:
#  * "split" (the library's default, SV_OPT_SPLIT 1): products on the fp16
#    matrix cores; a block costs its LDS round trip, split and barrier more
#    than its matrix-core work (least squares over 80 measured single
#    passes on a dense 30-qubit state, tile limits 12..14, 2..8 blocks:
#    memory 3.5, fixed 0.55, per 4-qubit block 0.83, per 5-qubit block 0.95;
#    rms error 0.24 ms);
#  * "fp32" (SV_OPT_SPLIT 0): the fp32 matrix cores bound the pass (fitted
#    to measured 30-qubit step times of 31 aggregations: memory 3.35, fixed
#    1.475, per 5-qubit block 1.78, per 4-qubit block 1.10).
# STAGE_FORM selects the model.  It defaults to the split fit, the form
# the device takes for unitary blocks: with 14-position tiles the 30-qubit
# depth-14 circuit planned from |0...0> gets the same plan either way (41
# blocks in 13 passes), and planned for passes over the whole state the
# split fit's plan (33 blocks, 29 of them 5-qubit, in 13 passes) runs
# 48.0-48.9 ms per step against 50.5-51.4 for the fp32 figures' (37
# blocks, 11 of them 5-qubit).  With 13-position tiles the fp32 figures
# had ranked better (0.2-1.0 ms on that circuit): the split fit's max()
# prices blocks under the memory time as free, which they are not quite.
SWEEP_MS = {1: 2.9, 2: 2.9, 3: 3.4, 4: 3.5, 5: 3.57, 6: 3.7}
STAGE_MODELS = {
    "split": (3.5, 0.55, {4: 0.83, 5: 0.95}),
    "fp32": (3.35, 1.475, {4: 1.10, 5: 1.78}),
}
STAGE_FORM = "split"


def stage_pass_ms(ks: Sequence[int]) -> float:
    """Modelled time of one staged pass of blocks of widths `ks` over 2^30
    amplitudes (STAGE_FORM's model)."""
    mem, fixed, per = STAGE_MODELS[STAGE_FORM]
    return max(mem, fixed + sum(per[k] for k in ks))


def staged_cost(ops: Sequence["Op"], pos_of=None, tmax: Optional[int] = None) -> float:
    """Modelled time of `ops` in this order, staged runs formed as the
    device forms them."""
    tmax = STAGE_T if tmax is None else tmax
    tot = 0.0
    for r in stage_runs(ops, pos_of, tmax):
        if len(r) >= 2:
            tot += stage_pass_ms([len(ops[i].qubits) for i in r])
        else:
            o = ops[r[0]]
            tot += SWEEP_MS.get(len(o.qubits), 4.0) if o.kind == "dense" else SWEEP_MS[1]
    return tot


# Launch overhead of a staged pass (ms) that touches only a few tiles.
STAGE_MS_LAUNCH = 0.02


def _tile_positions(P: int, ks: Sequence[int], S: int, nloc: int, tmax: int) -> Tuple[int, int]:
    """The device's tile of a staged pass (mask, width): targets and 0..3
    (P), widened with the lowest support positions to the widest tile
    within tmax whose LDS fits, then with any positions up to 9."""
    t = bin(P).count("1")
    cand = [p for p in range(nloc) if not (P >> p) & 1 and (S >> p) & 1]
    for tt in range(tmax, t, -1):
        if tt - t <= len(cand) and _stage_lds(tt, ks) <= _lds_limit(tt):
            for p in cand[:tt - t]:
                P |= 1 << p
            t = tt
            break
    for p in range(nloc):
        if t >= 9:
            break
        if (P >> p) & 1:
            continue
        if _stage_lds(t + 1, ks) > _lds_limit(t + 1):
            break
        P |= 1 << p
        t += 1
    return P, t


def sparse_passes(ops: Sequence["Op"], nloc: int, pos_of=None, tmax: Optional[int] = None,
                  support: int = 0) -> List[Tuple[List[int], int]]:
    """The passes `ops` run as from |0...0> (after sv_reset), each with the
    log2 of the amplitudes it visits, mirroring the device: a staged pass
    visits only the tiles whose id bits lie on positions some earlier op
    targeted (`support`), widens its tile with support positions only
    (others only up to the 9 a tile needs), and adds its targets to the
    support; any other sweep visits the whole state and makes the support
    full."""
    tmax = STAGE_T if tmax is None else tmax
    pos = (lambda q: q) if pos_of is None else pos_of
    full = (1 << nloc) - 1
    S = support & full
    out: List[Tuple[List[int], int]] = []
    for r in stage_runs(ops, pos_of, tmax):
        if len(r) < 2:
            out.append((r, nloc))
            S = full
            continue
        ks = [len(ops[i].qubits) for i in r]
        tg = 0
        for i in r:
            for q in ops[i].qubits:
                tg |= 1 << pos(q)
        P, t = _tile_positions(tg | 0xF, ks, S, nloc, tmax)
        out.append((r, t + bin(S & ~P).count("1")))
        S |= tg
    return out


def sparse_cost(ops: Sequence["Op"], nloc: int, pos_of=None, tmax: Optional[int] = None,
                support: int = 0) -> float:
    """Modelled time of `ops` run from |0...0> (`sparse_passes`): a pass
    costs its full-state model time scaled by the share of the state it
    visits, plus a launch overhead for staged passes."""
    tot = 0.0
    for r, lv in sparse_passes(ops, nloc, pos_of, tmax, support):
        if len(r) < 2:
            o = ops[r[0]]
            tot += SWEEP_MS.get(len(o.qubits), 4.0) if o.kind == "dense" else SWEEP_MS[1]
            continue
        base = stage_pass_ms([len(ops[i].qubits) for i in r])
        tot += base * 2.0 ** (lv - nloc) + STAGE_MS_LAUNCH
    return tot


def activation_orders(gates, n: int) -> List[List[int]]:
    """Orders in which to bring qubits into play when running from
    |0...0>: both directions of the Fiedler vector of the coupling graph
    (the qubits sorted along the graph's longest axis, so the front
    between touched and untouched qubits stays a narrow cut), and both
    directions of the qubit index."""
    A = np.zeros((n, n))
    for g in gates:
        qs = list(g.qubits)
        for a in qs:
            for b in qs:
                if a != b:
                    A[a, b] = 1.0
    Lp = np.diag(A.sum(1)) - A
    _, vec = np.linalg.eigh(Lp)
    f = vec[:, 1] if n > 1 else np.zeros(n)
    fied = sorted(range(n), key=lambda q: (f[q], q))
    return [fied, fied[::-1], list(range(n)), list(range(n))[::-1]]


def support_order(gates, act: Sequence[int]) -> list:
    """The gates in a dependency-respecting order that touches new qubits as
    late as possible: every gate whose qubits are all in play runs (earliest
    first) before the next qubit of `act` is brought into play."""
    n_g = len(gates)
    npred = [0] * n_g
    succ: List[List[int]] = [[] for _ in range(n_g)]
    last: Dict[int, int] = {}
    for i, g in enumerate(gates):
        ps = {last[q] for q in g.qubits if q in last}
        for p_ in ps:
            succ[p_].append(i)
        npred[i] = len(ps)
        for q in g.qubits:
            last[q] = i
    ready = {i for i in range(n_g) if npred[i] == 0}
    live: set = set()
    out: list = []
    k = 0
    while ready:
        ins = [i for i in ready if all(q in live for q in gates[i].qubits)]
        if not ins:
            live.add(act[k])
            k += 1
            continue
        i = min(ins)
        ready.discard(i)
        out.append(gates[i])
        for s_ in succ[i]:
            npred[s_] -= 1
            if npred[s_] == 0:
                ready.add(s_)
    assert len(out) == n_g
    return out


def widen_small_blocks(ops: Sequence["Op"], pos_of=None) -> List["Op"]:
    """Dense blocks on fewer than 4 qubits become 4-qubit blocks (identity on
    the added qubits, exact) by adding the qubits at positions 0..3, which
    every staged tile holds anyway: they can then join staged passes."""
    pos = (lambda q: q) if pos_of is None else pos_of
    where = {}
    for o in ops:
        for q in o.qubits:
            where[pos(q)] = q
    out: List[Op] = []
    for o in ops:
        if o.kind != "dense" or len(o.qubits) >= 4:
            out.append(o)
            continue
        extra = [where[p] for p in range(4) if p in where and where[p] not in o.qubits]
        extra = extra[:4 - len(o.qubits)]
        if len(o.qubits) + len(extra) < 4:
            out.append(o)
            continue
        qs = tuple(o.qubits) + tuple(extra)
        m = embed_in(qs, o.qubits, np.asarray(o.matrix, dtype=np.complex128))
        out.append(Op("dense", qs, m, ngates=o.ngates))
    return out


def plan_cost(ops: Sequence[Op]) -> float:
    """Relative cost of a plan: one unit per HBM sweep plus the block's
    arithmetic (8 2^k flop per amplitude) in units of a 6-qubit block."""
    return sum(1.0 + (8 << len(o.qubits)) / 4096.0 if o.kind == "dense" else 1.0 for o in ops)


def _nloc_of(gates) -> int:
    return 1 + max((q for g in gates for q in g.qubits), default=0)


def plan_fast(gates, kmax: int, pos_of=None, nloc: Optional[int] = None,
              sparse_start: bool = False, tmax: Optional[int] = None) -> List[Op]:
    """One staged aggregation (grow-based, window 4, last qubit only when it
    adds 40 % more gate weight), widened and ordered for staged passes: for
    request paths where planning time counts (tens of ms for ~600 gates).
    sparse_start: the same aggregation also of the gates in the Fiedler
    orders of `support_order`, the cheapest by `sparse_cost` kept.
    tmax: widest staged tile (default stage_tmax(nloc); 0 = no staging)."""
    n_loc = _nloc_of(gates) if nloc is None else nloc
    tmax = stage_tmax(n_loc) if tmax is None else tmax
    gain = 0.4 if kmax >= 5 and tmax else 0.0
    ops = fuse_grow(gates, kmax, window=4, last_gain=gain)
    if not tmax:
        return ops
    ops = order_for_staging(widen_small_blocks(ops, pos_of), pos_of, tmax)
    if not sparse_start:
        return ops
    cands = [ops]
    n_q = 1 + max((q for g in gates for q in g.qubits), default=0)
    for act in activation_orders(gates, n_q)[:2]:
        c = fuse_grow(support_order(gates, act), kmax, window=4, last_gain=gain)
        cands.append(order_for_staging(widen_small_blocks(c, pos_of), pos_of, tmax))
    return min(cands, key=lambda c: sparse_cost(c, n_loc, pos_of, tmax))


def _staged_candidates(gates, kmax: int, pos_of, tmax: int) -> List[List[Op]]:
    cands = [fuse(gates, kmax)]
    for w in (3, 4, 5, 6, 8):
        cands.append(fuse_grow(gates, kmax, window=w))
    if kmax >= 3:
        for w in (3, 4, 5, 6, 8):
            for g in (0.2, 0.4, 0.6, 0.8, 1.0):
                cands.append(fuse_grow(gates, kmax, window=w, last_gain=g))
    return [order_for_staging(widen_small_blocks(c, pos_of), pos_of, tmax) for c in cands]


def plan(gates, kmax: int, fold_diag: bool = False, staged: bool = True, pos_of=None,
         nloc: Optional[int] = None, sparse_start: bool = False, tmax: Optional[int] = None) -> List[Op]:
    """Aggregate with every available heuristic and keep the cheapest plan.

    staged (complex64 states): blocks on fewer than 4 qubits are widened to
    4 (`widen_small_blocks`), commuting blocks are ordered for staged passes
    (`order_for_staging`; positions given by pos_of, default position =
    qubit) and the candidates are ranked by `staged_cost`; otherwise they
    are ranked by `plan_cost`.  sparse_start (the ops run right after
    sv_reset): the gates are also tried in orders that bring qubits into
    play late (`support_order` over `activation_orders`), and the
    candidates are ranked by `sparse_cost`.  tmax: widest staged tile
    (default stage_tmax(nloc), the complex64 limit)."""
    n_loc = _nloc_of(gates) if nloc is None else nloc
    tmax = (stage_tmax(n_loc) if tmax is None else tmax) if staged else 0
    if not tmax or fold_diag:
        cands = [fuse(gates, kmax, fold_diag=fold_diag)]
        if not fold_diag:
            for w in (3, 4, 5, 6, 8):
                cands.append(fuse_grow(gates, kmax, window=w))
        return min(cands, key=plan_cost)
    cands = _staged_candidates(gates, kmax, pos_of, tmax)
    if not sparse_start:
        return min(cands, key=lambda c: staged_cost(c, pos_of, tmax))
    n_q = 1 + max((q for g in gates for q in g.qubits), default=0)
    for act in activation_orders(gates, n_q):
        cands += _staged_candidates(support_order(gates, act), kmax, pos_of, tmax)
    return min(cands, key=lambda c: sparse_cost(c, n_loc, pos_of, tmax))


@dataclasses.dataclass
class Phase:
    sliced: Tuple[int, ...]          # qubits fixed (sliced) during the phase
    order: List[int]                 # layout: order[p] = qubit at position p
    gate_ids: List[int]              # circuit gates applied in the phase
    ops: List[Op] = dataclasses.field(default_factory=list)


@dataclasses.dataclass
class SlicedPlan:
    n: int
    phases: List[Phase]
    trailing_qubits: Tuple[int, ...]     # = the last phase's sliced set, ascending
    trailing: Optional[np.ndarray]       # 2^s x 2^s over trailing_qubits, or None (identity)
    trailing_gate_ids: List[int]


def phase_layout(n: int, sliced: Sequence[int], other: Sequence[int]) -> List[int]:
    """[qubits in neither set ascending] [other set] [sliced set]: the other
    set sits in the top local ("file") positions, so switching the two sets
    only relabels whole files (Sec. 4, logical files indexed by both sets)."""
    both = set(sliced) | set(other)
    inner = [q for q in range(n) if q not in both]
    return inner + sorted(other) + sorted(sliced)


def phase_schedule(circuit, set_a: Sequence[int], set_b: Sequence[int], kmax: int,
                   max_phases: int = 64) -> SlicedPlan:
    """Split the gate list into phases with alternating sliced sets (Sec. 4:
    subcircuits 3, 5, 7, 9 slice one set and 4, 6, 8 the other).  A phase
    applies, in order, every pending gate that touches no sliced qubit and
    whose predecessors are applied (a light-cone scan).  When the pending
    gates act only on the current sliced set they are multiplied into the
    trailing operator that the cross-slice reduction applies."""
    n = circuit.n
    gates = circuit.gates
    pending = list(range(len(gates)))
    phases: List[Phase] = []
    cur, nxt = tuple(sorted(set_a)), tuple(sorted(set_b))
    trailing_ids: List[int] = []
    stall = 0
    while pending:
        blocked = set(cur)
        take, rest = [], []
        for i in pending:
            qs = set(gates[i].qubits)
            if qs & blocked:
                blocked |= qs
                rest.append(i)
            else:
                take.append(i)
        ph = Phase(cur, phase_layout(n, cur, nxt), take)
        where = {q: p for p, q in enumerate(ph.order)}
        ph.ops = plan([gates[i] for i in take], kmax, pos_of=where.__getitem__,
                      nloc=n - len(cur)) if take else []
        phases.append(ph)
        stall = stall + 1 if not take else 0
        if stall >= 2 or len(phases) > max_phases:
            raise ValueError("phase schedule makes no progress (a gate spans both slice sets?)")
        pending = rest
        if pending and all(set(gates[i].qubits) <= set(cur) for i in pending):
            trailing_ids = list(pending)        # only sliced qubits left: fold into T
            pending = []
            break
        cur, nxt = nxt, cur
    last = phases[-1].sliced
    T = None
    if trailing_ids:
        ql = list(last)
        T = np.eye(1 << len(ql), dtype=np.complex128)
        for i in trailing_ids:
            T = embed_in(ql, gates[i].qubits, np.asarray(gates[i].matrix, dtype=np.complex128)) @ T
    return SlicedPlan(n, phases, tuple(last), T, trailing_ids)


def stats(ops: Sequence[Op]) -> Dict[str, object]:
    hist: Dict[int, int] = {}
    for o in ops:
        if o.kind == "dense":
            hist[len(o.qubits)] = hist.get(len(o.qubits), 0) + 1
    return {"dense": sum(1 for o in ops if o.kind == "dense"),
            "diag": sum(1 for o in ops if o.kind == "diag"),
            "perm": sum(1 for o in ops if o.kind == "perm"),
            "k_hist": dict(sorted(hist.items())),
            "flops_per_amp": sum((8 * (1 << len(o.qubits)) - 2) for o in ops if o.kind == "dense")}


class PackedPlan(list):
    """pack()'s result: PackedOps items and permute ops, in plan order."""


def pack(ops: Sequence[Op], dtype) -> PackedPlan:
    """The op list as library calls: runs of dense / diagonal ops packed for
    one apply_ops call each, permutes as their own items."""
    from . import sv
    out, run = PackedPlan(), []
    for o in ops:
        if o.kind in ("dense", "diag"):
            run.append((o.kind, o.qubits, o.matrix))
            continue
        if run:
            out.append(sv.PackedOps(run, dtype))
            run = []
        out.append(o)
    if run:
        out.append(sv.PackedOps(run, dtype))
    return out


def enqueue(state_handle, ops, dtype) -> None:
    """Hand a planned op list (or its pack()) to the library (argument
    marshalling only)."""
    from . import sv
    for it in (ops if isinstance(ops, PackedPlan) else pack(ops, dtype)):
        if isinstance(it, sv.PackedOps):
            sv.apply_ops(state_handle, it)
        else:
            sv.permute_qubits(state_handle, it.order)
