"""The library's netlist builders against the oracle's (identical gate
lists), and the engine's host-side analysis (CPU only, no GPU calls)."""
import numpy as np
import pytest

from oracle import circuits as C
from oracle import lr
from oracle import params as OP
from tests import helpers


def _same(lib, ora):
    assert lib.n_wires == ora.n_wires
    assert lib.inputs.tolist() == ora.inputs
    assert lib.outputs.tolist() == ora.outputs
    assert lib.gates.tolist() == ora.gates


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 16])
def test_operator_netlists_match_oracle(k):
    import paper_2205_05825_amd as mk
    _same(mk.build_operator(mk.OP_ADD, k), C.adder(k))
    _same(mk.build_operator(mk.OP_SUB, k), C.subtractor(k))
    if k >= 2:
        _same(mk.build_operator(mk.OP_MUL, k), C.multiplier(k))
        _same(mk.build_operator(mk.OP_DIV, k), C.divider(k))
        _same(mk.build_operator(mk.OP_DIV2, k), C.divider(k, 2 * k))


@pytest.mark.parametrize("m,d", [(1, 1), (3, 2), (64, 4)])
def test_lr_netlist_matches_oracle(m, d):
    import paper_2205_05825_amd as mk
    _same(mk.build_lr_step(m, d), lr.build_netlist(m, d))


@pytest.mark.parametrize("m,frac", [(1, 8), (3, 0), (16, 8), (64, 8)])
def test_lr_formula_netlist_matches_oracle(m, frac):
    import paper_2205_05825_amd as mk
    _same(mk.build_lr_formula(m, frac), lr.build_formula_netlist(m, frac))


@pytest.mark.parametrize("t", range(7))
def test_naive_gate_netlists_match_oracle(t):
    import paper_2205_05825_amd as mk
    _same(mk.build_naive_gate(t), C.naive_gate(t))


def test_circuit_stats():
    import paper_2205_05825_amd as mk
    add = mk.build_operator(mk.OP_ADD, 8)
    levels, live, width, slots = mk.circuit_stats(add)
    # the final carry of the adder is dead: 4 gates dropped
    assert live == 5 * 8 - 3
    assert levels >= 8 and width >= 1 and slots >= 16
    mul = mk.build_operator(mk.OP_MUL, 8)
    levels, live, width, slots = mk.circuit_stats(mul)
    assert live == C.gate_count(C.multiplier(8))
    # slot reuse keeps the wire buffer well below one slot per gate
    assert slots < 16 + live


def test_engine_rejects_malformed_netlists():
    import paper_2205_05825_amd as mk
    good = mk.build_operator(mk.OP_ADD, 2)
    bad = mk.Circuit(good.n_wires, good.inputs, good.outputs, good.gates[::-1].copy())
    with pytest.raises(mk.MkError) as e:
        mk.circuit_stats(bad)
    assert e.value.code == -1
    dup = mk.Circuit(good.n_wires, np.array([2, 2, 3, 4]), good.outputs, good.gates)
    with pytest.raises(mk.MkError):
        mk.circuit_stats(dup)


def test_graph_entry_points_without_a_device_key():
    """Graph creation refuses a context whose key is not uploaded (checked on
    the host, before any device work); destroying a null graph is a no-op."""
    import ctypes
    import paper_2205_05825_amd as mk
    from paper_2205_05825_amd import _lib
    ctx = mk.Context(helpers.lib_params(OP.C1B), 3)
    circ = mk.build_operator(mk.OP_ADD, 2)
    h = ctypes.c_void_p()
    rc = _lib._L.mk_circuit_graph_create(ctx._h, ctypes.byref(circ.c()), ctypes.c_void_p(16),
                                         ctypes.c_void_p(16), 4, OP.C1B.lwe_words, 1,
                                         ctypes.byref(h))
    assert rc == -4 and not h.value
    assert _lib._L.mk_circuit_graph_create(ctx._h, ctypes.byref(circ.c()), None, None, 4,
                                           OP.C1B.lwe_words, 1, None) == -1
    assert _lib._L.mk_graph_destroy(None) == 0
    assert _lib._L.mk_graph_launch(None, None) == -1


def test_graph_piece_bound_is_enforced_on_the_host():
    """mk_set_graph_piece refuses piece sizes outside [64, 4096] kernels
    (4096 is the largest piece the GPU tests replay) before any device
    work; sizes inside the range are taken."""
    import paper_2205_05825_amd as mk
    ctx = mk.Context(helpers.lib_params(OP.C1B), 3)
    for bad in (0, 63, 4097, 1 << 20, -1):
        with pytest.raises(mk.MkError) as e:
            ctx.set_graph_piece(bad)
        assert e.value.code == -1
    for good in (64, 1024, 4096):
        ctx.set_graph_piece(good)


def _plan_slots(circ, release_when_read_at_level):
    """Model of the engine's wire-slot planner (first fit over a coalesced
    free list; the inputs' range first, then one range per level).  A range
    is released before level l allocates once no level >= l reads it, or,
    with release_when_read_at_level, already when l is its last reader (the
    rule that let a chunked level overwrite its own inputs)."""
    NOT = 6
    base, level = {}, {}
    for w in list(circ.inputs) + [0, 1]:
        base[int(w)] = int(w) if w not in (0, 1) else None
        level[int(w)] = 0
    gates = [tuple(int(x) for x in g) for g in circ.gates]
    for t, a, b, o in gates:
        if t == NOT:
            base[o], level[o] = base[a], level[a]
        else:
            base[o], level[o] = o, 1 + max(level[a], level[b])
    live = helpers.live_levels(circ)
    L = max(live.values(), default=0)
    by_level = {l: [] for l in range(1, L + 1)}
    for gi in sorted(live):
        by_level[live[gi]].append(gi)
    last = {}
    for l in range(1, L + 1):
        for gi in by_level[l]:
            for w in gates[gi][1:3]:
                if base[w] is not None:
                    last[base[w]] = max(last.get(base[w], 0), l)
    for w in circ.outputs:
        if base[int(w)] is not None:
            last[base[int(w)]] = L + 1
    free, top, ranges, slot = [], 0, [], {}

    def alloc(n):
        nonlocal top
        for i, (st, sz) in enumerate(free):
            if sz >= n:
                free[i] = (st + n, sz - n)
                if free[i][1] == 0:
                    free.pop(i)
                return st
        st, top = top, top + n
        return st

    def release(st, n):
        free.append((st, n))
        free.sort()
        merged = []
        for s, z in free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + z)
            else:
                merged.append((s, z))
        free[:] = merged

    st = alloc(len(circ.inputs))
    for i, w in enumerate(circ.inputs):
        slot[int(w)] = st + i
    ranges.append((st, len(circ.inputs), max([last.get(int(w), 0) for w in circ.inputs], default=0)))
    for l in range(1, L + 1):
        keep = []
        for r in ranges:
            done = r[2] <= l if release_when_read_at_level else r[2] < l
            if done:
                if r[1]:
                    release(r[0], r[1])
            else:
                keep.append(r)
        ranges = keep
        outs = [gates[gi][3] for gi in by_level[l]]
        st = alloc(len(outs))
        for i, w in enumerate(outs):
            slot[w] = st + i
        ranges.append((st, len(outs), max([last.get(w, 0) for w in outs], default=0)))
    return slot, live, last, gates


def _clashes(circ, slot, live, last, gates):
    """(level, slot) pairs where a level's output takes the slot of a wire
    that this level or a later one still reads."""
    holder = {slot[int(w)]: int(w) for w in circ.inputs}
    out = []
    for l in sorted(set(live.values())):
        gis = [gi for gi in live if live[gi] == l]
        for gi in gis:
            h = holder.get(slot[gates[gi][3]])
            if h is not None and last.get(h, 0) >= l:
                out.append((l, slot[gates[gi][3]]))
        for gi in gis:
            holder[slot[gates[gi][3]]] = gates[gi][3]
    return out


_NETLISTS = {
    "add16": lambda mk: mk.build_operator(mk.OP_ADD, 16),
    "mul8": lambda mk: mk.build_operator(mk.OP_MUL, 8),
    "div8": lambda mk: mk.build_operator(mk.OP_DIV, 8),
    "lr_step": lambda mk: mk.build_lr_step(4, 2),
    "lr_formula": lambda mk: mk.build_lr_formula(2, 8),
}


@pytest.mark.parametrize("name", sorted(_NETLISTS))
def test_slot_plan_never_overwrites_a_wire_still_read(name):
    """The library's slot assignment equals the planner model's, and no
    level writes a slot whose wire that level or a later one still reads
    (a level wider than one rotation launch runs in chunks, so it reads its
    inputs while writing its outputs).  The model under the earlier release
    rule clashes on the 16-bit adder, so a return to that rule fails here."""
    import paper_2205_05825_amd as mk
    circ = _NETLISTS[name](mk)
    lib_slot, lib_level = mk.circuit_slots(circ)
    slot, live, last, gates = _plan_slots(circ, False)
    for w in range(circ.n_wires):
        assert lib_slot[w] == slot.get(w, -1), w
    for gi, l in live.items():
        assert lib_level[gates[gi][3]] == l
    assert not _clashes(circ, slot, live, last, gates)
    if name == "add16":
        old = _plan_slots(circ, True)
        assert _clashes(circ, *old)


def _plain_eval(circ, values):
    """Plaintext evaluation of a netlist: values maps input wires to bits
    (arrays over instances); returns {wire: bits} for every defined wire."""
    import mk_inputs as mi
    v = dict(values)
    n = len(next(iter(values.values())))
    v[0], v[1] = np.zeros(n, np.int64), np.ones(n, np.int64)
    for t, a, b, o in (tuple(int(x) for x in g) for g in circ.gates):
        if t == 6:
            v[o] = 1 - v[a]
        else:
            v[o] = np.array([mi.plain_gate(t, int(x), int(y)) for x, y in zip(v[a], v[b])])
    return v


@pytest.mark.parametrize("name", ["lr_formula", "div8"])
def test_split_by_levels_computes_the_same_outputs(name):
    """Evaluating the level-range parts in order gives the whole circuit's
    outputs (plaintext evaluation, random inputs), and every part is a
    valid netlist for the engine (circuit_stats accepts it)."""
    import paper_2205_05825_amd as mk
    circ = _NETLISTS[name](mk)
    rng = np.random.default_rng(3)
    ins = {int(w): rng.integers(0, 2, 5) for w in circ.inputs}
    whole = _plain_eval(circ, ins)
    parts = helpers.split_by_levels(circ, 4)
    wires = dict(ins)
    total_levels = 0
    for p in parts:
        total_levels += mk.circuit_stats(p)[0]
        got = _plain_eval(p, {int(w): wires[int(w)] for w in p.inputs})
        for w in p.outputs:
            wires[int(w)] = got[int(w)]
    for w in circ.outputs:
        w = int(w)
        ref = whole[w]
        val = wires[w] if w > 1 else np.full(5, w)
        assert np.array_equal(val, ref), w
    assert total_levels == mk.circuit_stats(circ)[0]
