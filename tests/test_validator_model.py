"""The code-stream validator in its two forms, as models on the CPU.

The structure passes validate every code stream before the interpreter may
run it.  After two-pass emission a sequential simulation does it (one lane
per segment, code after code).  The placement pass does the same checks 64
codes at a time: the state before each code (window index, slab depth, slot
writes since the last FLUSH, REF count, FLUSH and END seen) is a prefix sum
or prefix OR over the batch, carried from batch to batch.  These tests model
both forms in Python, with the kernel's kinds and window sizes, and check
that they flag exactly the same streams, valid and corrupted alike: a
corrupted stream is not something to run on the device.
"""
import os
import random
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", "paper_1902_09215_amd", "csrc"))
import gen_interp as g  # noqa: E402

K = {k: i for i, k in enumerate(g.KINDS)}
NK, W, H, RING = g.NK, g.VSTACK, g.HALF, g.RING
OPS3, OPS00, OPS22 = K["OPS3"], K["OPS00"], K["OPS22"]
PR0, LR0 = K["PUSHREF0"], K["LOADREF0"]
FLUSH, END, OUTB, OUTM, OUTT, OUTX = K["FLUSH"], K["END"], K["OUTBOT"], K["OUTMEM"], K["OUTT"], K["OUTX"]
SPILL, FILL = K["SPILL"], K["FILL"]


def norm_base(m):
    return 0 if m < W - H // 2 else (m - H // 2) // H * H


def classes(k):
    ops1 = k <= OPS3
    ops2 = OPS00 <= k <= OPS22
    pref = PR0 <= k < PR0 + RING
    lref = LR0 <= k < LR0 + RING
    push1 = K["CH0"] <= k <= K["CH3"] or k == K["PUSHX"] or pref
    push2 = k == K["PUSH2X"] or K["PXCH0"] <= k <= K["PXCH3"]
    need = 1 if ops1 else (2 if ops2 else 0)
    d = -1 if ops1 else (-2 if ops2 else (1 if push1 else (2 if push2 else 0)))
    return need, d, pref, lref


def sequential(kinds, m0, ref0, last, n_out, n_in, slab_entries):
    """The simulation after two-pass emission, code by code."""
    slab = norm_base(m0)
    idx = m0 - slab
    fl = outs = ins = bad = 0
    ended = tail = False
    for k in kinds:
        if k >= NK:
            bad |= 1
        if ended:
            bad |= 4
        if tail:
            isF, isB, isM = k == FLUSH, k == OUTB, k == OUTM
            w = not (isF or isB or isM or k in (OUTT, OUTX, END)) or (isB and fl >= idx) or (isM and fl >= slab)
            fl = 0 if isF else fl + (1 if isB or isM else 0)
            outs += 1 if k in (OUTB, OUTM, OUTT, OUTX) else 0
            ended |= k == END
            if w:
                bad |= 2
            continue
        need, d, pref, lref = classes(k)
        w = idx < need
        slot = (ref0 + ins) & (RING - 1)
        if (pref and k - PR0 != slot) or (lref and k - LR0 != slot):
            bad |= 1
        idx += d
        ins += 1 if pref or lref else 0
        if k == END:
            ended = True
        elif k == FLUSH:
            fl, tail = 0, True
        elif k == OUTB:
            w |= fl >= idx
            fl += 1
        elif k == OUTM:
            w |= fl >= slab
            fl += 1
        elif k == SPILL:
            w |= idx < H
            idx -= H
            slab += H
        elif k == FILL:
            w |= slab < H or idx > H - 1
            idx += H
            slab -= H
        outs += 1 if k in (OUTT, OUTX, OUTB, OUTM) else 0
        w |= idx < 0 or idx > W - 1 or slab < 0 or slab > slab_entries
        if w:
            bad |= 2
    if ended != last:
        bad |= 4
    if not last and slab != norm_base(idx + slab):
        bad |= 8
    if outs != n_out:
        bad |= 16
    if ins != n_in:
        bad |= 32
    return bad


def batched(kinds, m0, ref0, last, n_out, n_in, slab_entries):
    """The placement pass's form: 64 codes at a time, the state before each
    code from prefix sums over the batch plus what earlier batches carried."""
    slab = norm_base(m0)
    idx = m0 - slab
    ins = nbm = nbm_flush = outs = bad = 0
    tail = ended = False
    for i0 in range(0, len(kinds), 64):
        ks = kinds[i0:i0 + 64]
        n = len(ks)
        isF = [k == FLUSH for k in ks]
        isE = [k == END for k in ks]
        isBM = [k in (OUTB, OUTM) for k in ks]
        tail_b = [tail or any(isF[:j]) for j in range(n)]
        ended_b = [ended or any(isE[:j]) for j in range(n)]
        fl = []
        for j in range(n):
            flushes = [l for l in range(j) if isF[l]]
            at_flush = nbm + sum(isBM[:flushes[-1]]) if flushes else nbm_flush
            fl.append(nbm + sum(isBM[:j]) - at_flush)
        di, ds, isref = [], [], []
        for j, k in enumerate(ks):
            need, d, pref, lref = classes(k)
            d += -H if k == SPILL else (H if k == FILL else 0)
            s = H if k == SPILL else (-H if k == FILL else 0)
            if tail_b[j]:
                d = s = 0
            di.append(d)
            ds.append(s)
            isref.append((pref or lref) and not tail_b[j])
        for j, k in enumerate(ks):
            need, _, pref, lref = classes(k)
            ib, sb = idx + sum(di[:j]), slab + sum(ds[:j])
            ia, sa = ib + di[j], sb + ds[j]
            ins_b = ins + sum(isref[:j])
            if k >= NK:
                bad |= 1
            if ended_b[j]:
                bad |= 4
            w = False
            isB, isM = k == OUTB, k == OUTM
            if tail_b[j]:
                w |= not (isF[j] or isB or isM or k in (OUTT, OUTX) or isE[j])
                w |= (isB and fl[j] >= ib) or (isM and fl[j] >= sb)
            else:
                w |= ib < need
                slot = (ref0 + ins_b) & (RING - 1)
                if (pref and k - PR0 != slot) or (lref and k - LR0 != slot):
                    bad |= 1
                w |= (isB and fl[j] >= ib) or (isM and fl[j] >= sb)
                w |= k == SPILL and ib < H
                w |= k == FILL and (sb < H or ib > H - 1)
                w |= ia < 0 or ia > W - 1 or sa < 0 or sa > slab_entries
            if w:
                bad |= 2
        idx += sum(di)
        slab += sum(ds)
        ins += sum(isref)
        flushes = [l for l in range(n) if isF[l]]
        if flushes:
            nbm_flush = nbm + sum(isBM[:flushes[-1]])
        nbm += sum(isBM)
        outs += sum(1 for k in ks if k in (OUTB, OUTM, OUTT, OUTX))
        tail = tail or any(isF)
        ended = ended or any(isE)
    if ended != last:
        bad |= 4
    if not last and slab != norm_base(idx + slab):
        bad |= 8
    if outs != n_out:
        bad |= 16
    if ins != n_in:
        bad |= 32
    return bad


def random_stream(rng, length, last):
    """A plausible stream: stack actions, REFs in ring order, spills and
    fills, then (last) the chunk end's flushes and slot writes."""
    ks = []
    ref = rng.randrange(RING)
    for _ in range(length):
        r = rng.random()
        if r < 0.3:
            ks.append(rng.choice([K["PUSHX"], K["PUSH2X"], K["CH0"], K["PXCH1"]]))
        elif r < 0.6:
            ks.append(rng.choice([K["OPS0"], K["OPS3"], K["OPS12"], K["OPX2"], K["LOADX"]]))
        elif r < 0.75:
            ks.append((PR0 if rng.random() < 0.5 else LR0) + ref % RING)
            ref += 1
        elif r < 0.8:
            ks.append(rng.choice([SPILL, FILL]))
        else:
            ks.append(rng.choice([K["OPS1"], K["PUSHX"], OUTT]))
    if last:
        ks += [FLUSH] + [OUTM] * rng.randrange(4) + [FLUSH] + [OUTB] * rng.randrange(70) + [OUTT, END]
    return ks


def corrupt(rng, ks):
    ks = list(ks)
    what = rng.randrange(5)
    if what == 0 and ks:
        ks[rng.randrange(len(ks))] = rng.randrange(NK + 3)
    elif what == 1 and ks:
        del ks[rng.randrange(len(ks))]
    elif what == 2:
        ks.insert(rng.randrange(len(ks) + 1), rng.choice([FLUSH, END, SPILL, FILL, OUTB, OUTM]))
    elif what == 3 and len(ks) > 1:
        i = rng.randrange(len(ks) - 1)
        ks[i], ks[i + 1] = ks[i + 1], ks[i]
    else:
        ks = ks + ks[: rng.randrange(8)]
    return ks


@pytest.mark.parametrize("seed", range(6))
def test_batched_validation_equals_sequential(seed):
    rng = random.Random(1000 + seed)
    flagged = clean = 0
    for case in range(150):
        last = rng.random() < 0.4
        length = rng.choice([0, 1, 5, 63, 64, 65, 130, 200])
        ks = random_stream(rng, length, last)
        if rng.random() < 0.6:
            ks = corrupt(rng, ks)
        m0 = rng.choice([0, 1, 5, 30, 50, 60, 120])
        ref0 = rng.randrange(RING)
        slab_entries = rng.choice([0, 28, 56, 200])
        # the counts the plan would claim: the stream's own, or off by one
        n_out = sum(1 for k in ks if k in (OUTB, OUTM, OUTT, OUTX)) + (rng.random() < 0.1)
        n_in = sum(1 for k in ks if PR0 <= k < LR0 + RING) + (rng.random() < 0.1)
        want = sequential(ks, m0, ref0, last, n_out, n_in, slab_entries)
        got = batched(ks, m0, ref0, last, n_out, n_in, slab_entries)
        assert got == want, f"case {case}: batched {got:#x} sequential {want:#x} ({len(ks)} codes)"
        flagged += want != 0
        clean += want == 0
    # both outcomes occur, so the comparison covers accepted and rejected streams
    assert flagged > 10 and clean > 5


def test_a_valid_window_walk_passes_both():
    # fill the window, spill half, push and pop, fill back, pop, and end the
    # segment in its boundary position (a final spill): a stream the emitter
    # could write, accepted by both forms
    ks = [K["LOADX"]] + [K["PUSHX"]] * (W - 1) + [SPILL] + [K["PUSHX"]] * 10 + [K["OPS0"]] * 10
    ks += [FILL] + [K["OPS1"]] * 5 + [SPILL]
    assert norm_base(W - 1 - 5) == H
    for f in (sequential, batched):
        assert f(ks, 0, 0, False, 0, 0, 64) == 0
        # the same stream claiming a slot write it does not make
        assert f(ks, 0, 0, False, 1, 0, 64) == 16
