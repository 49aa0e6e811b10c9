"""A host model of the persistent walk schedule's control flow (walk.hip,
k_walk_persistent), run on the CPU: per-wave id claims with guided sizes and
one claim issued ahead, the two start stages (a claimed id whose source is
loading; a ready query whose row range is loading), 1, 2 or 4 walkers per
lane, the LDS staging of lengths and status with per-range `left` counters and
the coalesced flush, the rejection walkers' missed dart (the walker keeps its
state and throws its next dart in the next iteration) and the exit test at the
bottom of the loop.  Waves run round-robin, one iteration each.

Moves: REJ (as the kernel has it), Node2Vec with its dart loop inside the move
(as the kernel has it), and Node2Vec with one dart per iteration, a variant
that used to hang the device with two walkers per lane and is not in the
library.  In every configuration the model must finish, record every query
exactly once and give the oracle's walks: the schedule's own logic, which REJ
still shares, is not what made that variant hang.
"""
import numpy as np
import pytest

import oracle
import synth

KIDLE = 0xFFFFFFFF
KDIRECT = 0xFFFFFFFF
KMISSED = -2
KSTAGE = 256
KMAXDARTS = 1 << 24


class Philox:
    def __init__(self, seed):
        self.key = (seed & 0xFFFFFFFF, seed >> 32)
        self.cache = {}

    def __call__(self, k, t, qid):
        key = (k, t, qid)
        if key not in self.cache:
            self.cache[key] = [int(x) for x in oracle.philox4x32_10((k, t, qid & 0xFFFFFFFF, qid >> 32), self.key)]
        return self.cache[key]


def mulhi(r, d):
    return (r * d) >> 32


class Walker:
    def __init__(self):
        self.qi = KIDLE


def emulate(g, src, move_kind, WPL, n_waves, chunk, n_slots, seed, max_len, thr, pmax=None, max_iters=200000):
    n = g.n
    nq = len(src)
    rp, col = g.row_ptr, g.col
    ph = Philox(seed)
    head = [0]
    lengths = np.full(nq, -1, np.int64)
    status = np.zeros(nq, np.int64)
    recorded = np.zeros(nq, np.int64)
    paths = {}

    def guided(seen):
        left = nq - seen if seen < nq else 0
        take = min(left // (2 * n_waves), chunk)
        return max(take, min(64, chunk))

    waves = []
    for wv in range(n_waves):
        W = dict(lanes=[dict(w=[Walker() for _ in range(WPL)], s_qi=KIDLE, r_qi=KIDLE, s_code=KDIRECT,
                             r_code=KDIRECT, s_src=0, r_src=0, r_lo=0, r_hi=0, r_deg=0, r_pm=0, s_bad=False,
                             done_slots=0) for _ in range(64)],
                 slots=[dict(base=0, size=0, left=0, len=[0] * KSTAGE, st=[0] * KSTAGE) for _ in range(n_slots)],
                 pool_next=0, pool_end=0, pool_base=0, pool_slot=KDIRECT, exhausted=False, more=True)
        W["ahead_take"] = guided(0)
        W["ahead_base"] = head[0]; head[0] += W["ahead_take"]
        W["ahead_seen"] = W["ahead_base"]
        W["ahead_pending"] = False
        waves.append(W)

    def record(W, L, code, qi, k, st):
        recorded[qi] += 1
        if code == KDIRECT:
            lengths[qi] = k; status[qi] = st
        else:
            sl = W["slots"][code // KSTAGE]
            sl["len"][code % KSTAGE] = k; sl["st"][code % KSTAGE] = st
            sl["left"] -= 1
            if sl["left"] == 0:
                L["done_slots"] |= 1 << (code // KSTAGE)

    def n2v_accept(w, x, r):
        y = r[1] >> 16
        if x == w.prev:
            return y < thr[0]
        adjacent = x in set(col[rp[w.prev]:rp[w.prev + 1]].tolist())
        return y < (thr[1] if adjacent else thr[2])

    it = 0
    while any(W["more"] for W in waves):
        it += 1
        if it > max_iters:
            raise AssertionError("the schedule did not finish")
        for W in waves:
            if not W["more"]:
                continue
            lanes = W["lanes"]
            # Start
            for L in lanes:
                for w in L["w"]:
                    if w.qi == KIDLE and L["r_qi"] != KIDLE:
                        w.qi = L["r_qi"]; w.code = L["r_code"]; w.cur = L["r_src"]; w.prev = -1; w.k = 0
                        w.poff = 0; w.pdeg = 0; w.need_row = False; w.dart = 0; w.pm = L["r_pm"]
                        w.off = L["r_lo"]; w.deg = L["r_deg"]
                        paths[w.qi] = [w.cur]
                        L["r_qi"] = KIDLE
            # S -> R
            for L in lanes:
                if L["r_qi"] == KIDLE and L["s_qi"] != KIDLE:
                    if L["s_bad"]:
                        record(W, L, L["s_code"], L["s_qi"], 0, 4)
                    else:
                        L["r_qi"], L["r_code"], L["r_src"] = L["s_qi"], L["s_code"], L["s_src"]
                        L["r_lo"], L["r_hi"] = int(rp[L["s_src"]]), int(rp[L["s_src"] + 1])
                        if pmax is not None:
                            L["r_pm"] = int(pmax[L["s_src"]])
                    L["s_qi"] = KIDLE
            # Claim
            need = [L["s_qi"] == KIDLE for L in lanes]
            while any(need) and not W["exhausted"]:
                avail = W["pool_end"] - W["pool_next"]
                if avail == 0:
                    if W["ahead_pending"]:
                        W["ahead_seen"] = W["ahead_base"]; W["ahead_pending"] = False
                    base = W["ahead_seen"]
                    if base >= nq:
                        W["exhausted"] = True
                        break
                    W["pool_next"] = base
                    W["pool_end"] = min(base + W["ahead_take"], nq)
                    avail = W["pool_end"] - W["pool_next"]
                    W["pool_base"] = W["pool_next"]
                    W["pool_slot"] = KDIRECT
                    for i, sl in enumerate(W["slots"]):
                        if sl["size"] == 0:
                            sl["base"], sl["size"], sl["left"] = W["pool_base"], avail, avail
                            W["pool_slot"] = i
                            break
                    W["ahead_take"] = guided(base + W["ahead_take"])
                    W["ahead_base"] = head[0]; head[0] += W["ahead_take"]
                    W["ahead_pending"] = True
                rk = 0
                for li, L in enumerate(lanes):
                    if need[li]:
                        if rk < avail:
                            L["s_qi"] = W["pool_next"] + rk
                            L["s_code"] = KDIRECT if W["pool_slot"] == KDIRECT else \
                                W["pool_slot"] * KSTAGE + (L["s_qi"] - W["pool_base"])
                            L["s_src"] = int(src[L["s_qi"]])
                        rk += 1
                W["pool_next"] += min(sum(need), avail)
                need = [L["s_qi"] == KIDLE for L in lanes]
            # Gather
            for L in lanes:
                for w in L["w"]:
                    if w.qi != KIDLE and w.need_row:
                        w.off, w.deg = int(rp[w.cur]), int(rp[w.cur + 1] - rp[w.cur])
                        w.need_row = False
            # Move
            nxts = []
            for L in lanes:
                row = []
                for w in L["w"]:
                    nxt = -1
                    if w.qi != KIDLE and w.deg != 0:
                        qid = w.qi
                        if move_kind == "rej":
                            if w.pm != 0:
                                r = ph(w.k, w.dart, qid)
                                e = w.off + mulhi(r[0], w.deg)
                                hit = r[1] * w.pm < (int(g.weight[e]) << 32)
                                if hit or w.dart + 1 == KMAXDARTS:
                                    nxt = int(col[e])
                                    w.pm = int(pmax[nxt]); w.dart = 0
                                    w.off, w.deg = int(rp[nxt]), int(rp[nxt + 1] - rp[nxt])
                                else:
                                    nxt = KMISSED; w.dart += 1
                        elif move_kind == "n2v_loop":
                            t = 0
                            while True:
                                r = ph(w.k, t, qid)
                                x = int(col[w.off + mulhi(r[0], w.deg)])
                                if w.k == 0 or t + 1 == KMAXDARTS or n2v_accept(w, x, r):
                                    nxt = x
                                    break
                                t += 1
                            w.poff, w.pdeg = w.off, w.deg
                            w.need_row = True
                        else:   # n2v_one: one dart per iteration
                            r = ph(w.k, w.dart, qid)
                            x = int(col[w.off + mulhi(r[0], w.deg)])
                            if w.k == 0 or w.dart + 1 == KMAXDARTS or n2v_accept(w, x, r):
                                nxt = x
                                w.poff, w.pdeg = w.off, w.deg
                                w.need_row = True
                                w.dart = 0
                            else:
                                nxt = KMISSED
                                w.dart += 1
                    row.append(nxt)
                nxts.append(row)
            # end of iteration: prepared loads complete
            for L in lanes:
                L["s_bad"] = not (0 <= L["s_src"] < n)
                L["r_deg"] = L["r_hi"] - L["r_lo"]
            W["ahead_seen"] = W["ahead_base"]; W["ahead_pending"] = False
            # Update
            for L, row in zip(lanes, nxts):
                for w, nxt in zip(L["w"], row):
                    if w.qi == KIDLE or nxt == KMISSED:
                        continue
                    st = 0
                    if nxt < 0:
                        st = 3
                    else:
                        paths[w.qi].append(nxt)
                        w.prev, w.cur, w.k = w.cur, nxt, w.k + 1
                        if w.k == max_len:
                            st = 1
                    if st:
                        record(W, L, w.code, w.qi, w.k, st)
                        w.qi = KIDLE
            # flush finished ranges
            wave_done = 0
            for L in lanes:
                wave_done |= L["done_slots"]; L["done_slots"] = 0
            for i, sl in enumerate(W["slots"]):
                if wave_done >> i & 1:
                    for j in range(sl["size"]):
                        lengths[sl["base"] + j] = sl["len"][j]; status[sl["base"] + j] = sl["st"][j]
                    sl["size"] = 0
            anyl = any(L["r_qi"] != KIDLE or L["s_qi"] != KIDLE or any(w.qi != KIDLE for w in L["w"]) for L in lanes)
            W["more"] = (not W["exhausted"]) or anyl
    return lengths, status, recorded, paths, it


@pytest.fixture(scope="module")
def case(oracle_lib, synth_lib):
    g = synth.rmat(8, 8, True, 0x5EED)
    synth.attach_attrs(g, 0x5EED ^ 1, weights=True)
    rng = np.random.default_rng(3)
    nq = 700
    src = synth.sources(nq, g.n, 77).astype(np.int32)
    src[rng.choice(nq, 9, replace=False)] = -1                 # bad sources
    thr = oracle.n2v_thresholds(2.0, 0.5)
    pmax = oracle.rej_build(g.row_ptr, g.weight)
    max_len = 10
    ref = {"n2v": oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.NODE2VEC, oracle.OREJ, max_len, 9,
                                                                  n2v_thr_q16=thr), src),
           "rej": oracle.walk(g.row_ptr, g.col, oracle.WalkParams(oracle.DEEPWALK, oracle.REJ, max_len, 9), src,
                              weight=g.weight, pmax=pmax)}
    return dict(g=g, src=src, thr=thr, pmax=pmax, max_len=max_len, ref=ref)


@pytest.mark.parametrize("n_slots", [0, 8])
@pytest.mark.parametrize("wpl", [1, 2, 4])
@pytest.mark.parametrize("kind", ["rej", "n2v_loop", "n2v_one"])
def test_schedule_finishes_once_per_query(case, kind, wpl, n_slots):
    ref = case["ref"]["rej" if kind == "rej" else "n2v"]
    L, S, rec, P, iters = emulate(case["g"], case["src"], kind, wpl, n_waves=3, chunk=128, n_slots=n_slots,
                                  seed=9, max_len=case["max_len"], thr=case["thr"], pmax=case["pmax"])
    assert (rec == 1).all()
    assert np.array_equal(L, ref.lengths.astype(np.int64)) and np.array_equal(S, ref.status.astype(np.int64))
    for q, p in P.items():
        assert p == list(ref.paths[q, :len(p)])
