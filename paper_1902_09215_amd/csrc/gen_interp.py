"""Generate the gfx950 threaded-code interpreter used by k_run (ev_interp.inc).

The structure passes (k_seg_count / k_seg_emit) turn each work item's tokens
into a stream of 32-bit codes, one per action of the right-to-left stack
machine, with leaves folded into the functions that consume them and common
pairs of actions fused into one code.  A code's value is the byte offset of
its handler from the handler table: handlers are unrolled per position
(the code's index modulo 32), because each must find the next code in a
fixed SGPR of the 128-byte code block held in s[64:95].

Code blocks: s[64:79] holds positions 0..15 and s[80:95] positions 16..31.
Position 15's handler waits for the upper half and starts loading the next
block's lower half into s[64:79]; position 31's handler advances the block
pointer, waits for that lower half and starts loading the upper half.  So a
refill costs one scalar load per 16 codes and no register copies.

Dispatch is `s_add_u32 s44, s42, s[next]` + `s_setpc_b64 s[44:45]`.  A code
whose work lives in a shared routine (division, slot reads and writes,
spills) sets s[44:45] to the next handler first and jumps to the routine,
which ends by jumping there: one jump more than a plain code, not a call
and a return.  s45 (and s47, for routine jumps) equal the table's high
address word: the table must
not cross a 4 GiB boundary, which the prologue checks (a launch that finds a
carry writes 1 to the flag word and evaluates nothing; the library probes
this once per device and falls back to k_eval if ever needed).  Every
handler is placed with .org at its exact offset, so a handler that outgrew
its slot is an assembler error, never a wrong jump.

Register use inside the block (W0 = 7):
  v[W0 + m]       top of the operand stack (T); v[W0..W0+m-1] the entries
                  below it, oldest first.  m = M0[7:0].  Relative access
                  uses GPR-index mode with SRC0, SRC1 and DST relative,
                  switched on once per work item: a handler changes M0 only
                  when the depth changes, and writes a value from a fixed
                  register (x, x+x, a ring value) into the stack with
                  v_bfi_b32 d, 0, 0, src, whose third source stays absolute.
                  Division switches SRC2 on for its fused operations and
                  back; memory instructions run with the mode off.
  v[W0+VSTACK ..] HEAD registers above the window: a division works in
                  place, its temporaries just above T (relative, like the
                  stack), so it moves no operand in or out
  then            the ring of slot values read ahead at the skeleton levels
  then            x+x, x-x, x*x and x%x, made once per work item: a
                  function of two x leaves (about one function in four in a
                  random tree) is then a register move, a division included
  v4, v5          staging registers
  %[x], %[lane4]  the lane's input value and byte offset (not clobbered)
  s[40:41] code block pointer (128-byte aligned), s[42:43] handler table,
  s[44:45] jump target (the next handler), s[46:47] routine target,
  s[50:51] read-ahead pointer into the input slot rows, s[52:53] output-slot row pointer,
  s54 row bytes (cases * 4), M0 window index of T (and the mode bits),
  s[56:57] division scratch, s58 scratch, s59 flush index, s[60:61] next
  free entry of the wave's spill slab in global memory, s[62:63] the slab's
  base, s48 = 1 while the wave's LDS chunk (%[lds]: HALF rows of 64 lanes)
  holds the slab's top HALF entries.

When the structure machine sees the stack outgrow the window it emits SPILL
(store the bottom half of the window to the slab, shift the window down);
when a function needs an entry below the window it emits FILL (the
reverse).  So the kernel never tests the stack depth; the device validator
simulates the window index and slab depth of every code stream before it
may run.
"""
from __future__ import annotations

import os
import sys

W0 = 7  # T at v[W0 + m]; v[W0 - 1 + m] the entry below it
VSTACK = int(os.environ.get("EV_VSTACK", "48"))  # register-stack entries: v[W0] .. v[W0+VSTACK-1]
HALF = VSTACK // 2  # entries moved by one spill or fill
HEAD = 6  # division temporaries above the window (relative to T)
RING = int(os.environ.get("EV_RING", "8"))  # slot values read ahead
assert RING in (4, 8, 16, 32), "the ring size must be a power of two up to 32"
RING0 = W0 + VSTACK + HEAD
XX0 = RING0 + RING  # x+x, x-x, x*x, x%x
NREG = XX0 + 4
POS = 32  # positions per 128-byte code block
NSTRIDE = 32  # bytes per handler at ordinary positions
TSTRIDE = 64  # bytes per handler at positions 15 and 31 (they also refill)
# Kinds in table order: within each position's block the kinds a level-0
# stream uses come first, the rare ones (slot writes, flushes, spills) after,
# and the skeleton levels' REF kinds last, so that a level-0 launch's hot
# handlers are one contiguous kilobyte per position and the table's working
# set stays well inside the instruction cache whatever its alignment.
# OPS0..OPS2 must be kinds 0..2, and each group (and OUTT..OUTMEM) contiguous.
KINDS = ["OPS0", "OPS1", "OPS2", "OPS3", "OPX0", "OPX1", "OPX2", "OPX3",
         "CH0", "CH1", "CH2", "CH3", "LCH0", "LCH1", "LCH2", "LCH3",
         "PUSHX", "LOADX", "PUSH2X"] + [f"OPS{a}{b}" for a in range(3) for b in range(3)] \
    + ["PXCH0", "PXCH1", "PXCH2", "PXCH3"] \
    + ["OUTT", "OUTX", "FLUSH", "OUTBOT", "END", "SPILL", "FILL", "OUTMEM"] \
    + [f"PUSHREF{r}" for r in range(RING)] + [f"LOADREF{r}" for r in range(RING)]
NK = len(KINDS)
TBASE = (POS - 2) * NK * NSTRIDE  # first byte of the position-15 and -31 handlers
TABLE_BYTES = TBASE + 2 * NK * TSTRIDE
VOP = {0: "v_add_f32_e32", 1: "v_sub_f32_e32", 2: "v_mul_f32_e32"}


def is_transition(pos: int) -> bool:
    return pos % 16 == 15


def code_of(pos: int, kind: int) -> int:
    """Handler offset from the table base for a code at this position."""
    if is_transition(pos):
        return TBASE + (pos // 16) * NK * TSTRIDE + kind * TSTRIDE
    return (pos - pos // 16) * NK * NSTRIDE + kind * NSTRIDE


def div_body(a: int, b: int, t: int, r: int) -> list[str]:
    """Correctly rounded binary32 division a/b (the sequence hipcc emits for
    IEEE-mode division on gfx950), then protection: b != 0 ? a/b : 1.0f.
    Operands v[a], v[b], temporaries v[t] .. v[t+4], result v[r]; under
    full GPR-index mode all of them are relative to T."""
    d, rc, n, e, q = (f"v{t + i}" for i in range(5))
    A, B, R = f"v{a}", f"v{b}", f"v{r}"
    return [
        f"v_div_scale_f32 {d}, s[56:57], {B}, {B}, {A}",
        f"v_rcp_f32_e32 {rc}, {d}",
        f"v_div_scale_f32 {n}, vcc, {A}, {B}, {A}",
        f"v_fma_f32 {e}, -{d}, {rc}, 1.0",
        f"v_fmac_f32_e32 {rc}, {e}, {rc}",
        f"v_mul_f32_e32 {e}, {n}, {rc}",
        f"v_fma_f32 {q}, -{d}, {e}, {n}",
        f"v_fmac_f32_e32 {e}, {q}, {rc}",
        f"v_fma_f32 {d}, -{d}, {e}, {n}",
        f"v_div_fmas_f32 {d}, {d}, {rc}, {e}",
        f"v_div_fixup_f32 {d}, {d}, {B}, {A}",
        f"v_cmp_neq_f32_e32 vcc, 0, {B}",
        "s_nop 1",
        f"v_cndmask_b32_e32 {R}, 1.0, {d}, vcc",
    ]


FULL = "gpr_idx(SRC0,SRC1,SRC2,DST)"
MODE = "gpr_idx(SRC0,SRC1,DST)"  # the handlers' mode: SRC2 absolute
T, BELOW, ABOVE, ABOVE2 = f"v{W0}", f"v{W0 - 1}", f"v{W0 + 1}", f"v{W0 + 2}"
MODE_ON = f"s_set_gpr_idx_on m0, {MODE}"  # back to the handlers' mode (index unchanged)


def put(dst: str, src: str) -> str:
    """dst (relative) = src (a fixed register), bit for bit."""
    return f"v_bfi_b32 {dst}, 0, 0, {src}"


def next_target(pos: int) -> list[str]:
    """s[44:45] = the handler of the code at position pos+1 (refilling the
    code block halves at positions 15 and 31)."""
    nxt = (pos + 1) % POS
    pre: list[str] = []
    if pos == 15:
        pre = ["s_waitcnt lgkmcnt(0)", "s_load_dwordx16 s[64:79], s[40:41], 0x80"]
    elif pos == 31:
        pre = ["s_add_u32 s40, s40, 0x80", "s_addc_u32 s41, s41, 0", "s_waitcnt lgkmcnt(0)",
               "s_load_dwordx16 s[80:95], s[40:41], 0x40"]
    return pre + [f"s_add_u32 s44, s42, s{64 + nxt}"]


def dispatch(pos: int) -> list[str]:
    """Jump to the handler of the code at position pos+1."""
    return next_target(pos) + ["s_setpc_b64 s[44:45]"]


def tail_jump(routine: str) -> list[str]:
    """Jump to a shared routine, which ends by jumping to s[44:45]: the next
    code's handler, set up before the jump (one jump instead of a call, a
    return and a dispatch)."""
    return [f"s_add_u32 s46, s42, .L{routine}%= - .Ltab%=", "s_setpc_b64 s[46:47]"]


def row_dec(lo: int) -> list[str]:
    return [f"s_sub_u32 s{lo}, s{lo}, s54", f"s_subb_u32 s{lo + 1}, s{lo + 1}, 0"]


def handler(kind: str, pos: int, cp: str = "") -> list[str]:
    k = kind
    body: list[str]
    routine = None
    if k in ("OPS0", "OPS1", "OPS2"):
        # T' = op(T, below): the entry below becomes T
        body = [f"{VOP[int(k[3])]} {BELOW}, {T}, {BELOW}", "s_sub_u32 m0, m0, 1"]
    elif k == "OPS3":
        routine = "divops"
    elif len(k) == 5 and k.startswith("OPS"):
        # two pops in a row: the second works one entry lower
        a, b = int(k[3]), int(k[4])
        body = [f"{VOP[a]} {BELOW}, {T}, {BELOW}", f"{VOP[b]} v{W0 - 2}, {BELOW}, v{W0 - 2}", "s_sub_u32 m0, m0, 2"]
    elif k.startswith("OPX"):
        op = int(k[3])
        # T = op(x, T).  x + T and x - T are one fused multiply-add with x as
        # the (absolute) third source: T * 1 + x and T * -1 + x round once,
        # exactly as the sum and the difference do.  x * T copies x just
        # above T first.
        if op == 3:
            routine = "divopx"
        elif op < 2:
            body = [f"v_fma_f32 {T}, {T}, {'1.0' if op == 0 else '-1.0'}, %[x]"]
        else:
            body = [put(ABOVE, "%[x]"), f"{VOP[op]} {T}, {ABOVE}, {T}"]
    elif k.startswith("CH"):
        op = int(k[2])
        # push T; T = op(x, x), made once per work item
        body = [put(ABOVE, f"v{XX0 + op}"), "s_add_u32 m0, m0, 1"]
    elif k.startswith("LCH"):
        op = int(k[3])
        # T = op(x, x) with no value below
        body = [put(T, f"v{XX0 + op}")]
    elif k == "PUSHX":
        body = [put(ABOVE, "%[x]"), "s_add_u32 m0, m0, 1"]
    elif k == "PUSH2X":
        body = [put(ABOVE, "%[x]"), put(ABOVE2, "%[x]"), "s_add_u32 m0, m0, 2"]
    elif k.startswith("PXCH"):
        op = int(k[4])
        # two pushes of x, then a function of x: push x; push op(x, x)
        body = [put(ABOVE, "%[x]"), put(ABOVE2, f"v{XX0 + op}"), "s_add_u32 m0, m0, 2"]
    elif k == "LOADX":
        body = [put(T, "%[x]")]
    elif k in ("OUTT", "OUTBOT", "SPILL", "FILL", "OUTMEM") or k.startswith("PUSHREF") or k.startswith("LOADREF"):
        routine = k.lower()
    elif k == "OUTX":
        body = ["s_set_gpr_idx_off"] + row_dec(52) + ["global_store_dword %[lane4], %[x], s[52:53]" + cp, MODE_ON]
    elif k == "FLUSH":
        body = ["s_mov_b32 s59, 0"]
    elif k == "END":
        return ["s_set_gpr_idx_off", "s_branch .Lexit%="]
    else:
        raise KeyError(k)
    if routine is not None:
        return next_target(pos) + tail_jump(routine)
    return body + dispatch(pos)


def routines(cp: str = "") -> list[str]:
    out = []
    # T' = T / below (the entry below becomes T), worked in place: every
    # operand relative to T, the temporaries just above it
    out += [".Ldivops%=:", f"s_set_gpr_idx_on m0, {FULL}"]
    out += div_body(W0, W0 - 1, W0 + 1, W0 - 1)
    out += ["s_sub_u32 m0, m0, 1", MODE_ON, "s_setpc_b64 s[44:45]"]
    # T = x / T: x copied just above T first
    out += [".Ldivopx%=:", put(ABOVE, "%[x]"), f"s_set_gpr_idx_on m0, {FULL}"]
    out += div_body(W0 + 1, W0, W0 + 2, W0)
    out += [MODE_ON, "s_setpc_b64 s[44:45]"]
    # a value from the previous level's slots (rows read downwards): REF j of
    # a work item takes ring register j % RING, loaded RING REFs earlier, and
    # starts the load of the row REF j + RING will take.  Vector memory
    # operations complete in issue order, so at most RING-1 later loads can
    # still be outstanding when REF j's row has arrived.
    for r in range(RING):
        for name, dst, inc in ((f"pushref{r}", ABOVE, True), (f"loadref{r}", T, False)):
            out += [f".L{name}%=:", f"s_waitcnt vmcnt({RING - 1})", put(dst, f"v{RING0 + r}")]
            if inc:
                out += ["s_add_u32 m0, m0, 1"]
            out += ["s_set_gpr_idx_off"] + row_dec(50) + [
                f"global_load_dword v{RING0 + r}, %[lane4], s[50:51]" + cp, MODE_ON, "s_setpc_b64 s[44:45]"]
    # T to the next output slot (rows written downwards)
    out += [".Loutt%=:", "s_set_gpr_idx_on m0, gpr_idx(SRC0)", f"v_mov_b32_e32 v4, {T}", "s_set_gpr_idx_off"]
    out += row_dec(52) + ["global_store_dword %[lane4], v4, s[52:53]" + cp, MODE_ON, "s_setpc_b64 s[44:45]"]
    # chunk-end flush of the window entry s59 (the index of T is kept in s58)
    out += [".Loutbot%=:", "s_mov_b32 s58, m0", "s_set_gpr_idx_on s59, gpr_idx(SRC0)", f"v_mov_b32_e32 v4, {T}",
            "s_set_gpr_idx_off", "s_add_u32 s59, s59, 1"] + row_dec(52) + [
            "global_store_dword %[lane4], v4, s[52:53]" + cp, f"s_set_gpr_idx_on s58, {MODE}",
            "s_setpc_b64 s[44:45]"]
    # spill: the window's bottom HALF entries to the wave's LDS chunk, which
    # holds the top HALF entries of the slab; what it held goes on to the
    # slab in global memory first.  A stack that goes back and forth across a
    # window boundary then spills and fills through LDS only.
    tmp = ["v4", "v5"] + [f"v{W0 + VSTACK + i}" for i in range(HEAD)]  # free outside a division
    out += [".Lspill%=:", "s_set_gpr_idx_off", "s_cmp_eq_u32 s48, 0", "s_cbranch_scc1 .Lspilll%="]
    for r0 in range(0, HALF, len(tmp)):
        n = min(len(tmp), HALF - r0)
        out += [f"ds_read_b32 {tmp[k]}, %[lds] offset:{256 * (r0 + k)}" for k in range(n)]
        out += ["s_waitcnt lgkmcnt(0)"]
        out += [f"global_store_dword %[slane], {tmp[k]}, s[60:61]" + (f" offset:{256 * k}" if k else "")
                for k in range(n)]
        out += [f"s_add_u32 s60, s60, {256 * n}", "s_addc_u32 s61, s61, 0"]
    out += [".Lspilll%=:"]
    out += [f"ds_write_b32 %[lds], v{W0 + i}" + (f" offset:{256 * i}" if i else "") for i in range(HALF)]
    out += ["s_mov_b32 s48, 1"]
    out += [f"v_mov_b32_e32 v{W0 + i}, v{W0 + HALF + i}" for i in range(VSTACK - HALF)]
    out += [f"s_sub_u32 m0, m0, {HALF}", MODE_ON, "s_setpc_b64 s[44:45]"]
    # fill: shift up, then the slab's top HALF entries into the bottom: from
    # the LDS chunk when it holds them, else from global memory
    groups = [(g0, min(16, HALF - g0)) for g0 in range(0, HALF, 16)]
    out += [".Lfill%=:", "s_set_gpr_idx_off"]
    out += [f"v_mov_b32_e32 v{W0 + HALF + i}, v{W0 + i}" for i in range(VSTACK - HALF)]
    out += ["s_cmp_eq_u32 s48, 0", "s_cbranch_scc1 .Lfillg%="]
    out += [f"ds_read_b32 v{W0 + i}, %[lds]" + (f" offset:{256 * i}" if i else "") for i in range(HALF)]
    out += ["s_mov_b32 s48, 0", "s_waitcnt lgkmcnt(0)", f"s_add_u32 m0, m0, {HALF}", MODE_ON, "s_setpc_b64 s[44:45]"]
    out += [".Lfillg%=:"]
    for g0, n in reversed(groups):
        out += [f"s_sub_u32 s60, s60, {256 * n}", "s_subb_u32 s61, s61, 0"]
        out += [f"global_load_dword v{W0 + g0 + i}, %[slane], s[60:61]" + (f" offset:{256 * i}" if i else "")
                for i in range(n)]
    out += ["s_waitcnt vmcnt(0)", f"s_add_u32 m0, m0, {HALF}", MODE_ON, "s_setpc_b64 s[44:45]"]
    # chunk-end flush of an entry that lives in the slab (entry s59): in
    # global memory below the slab pointer, else in the LDS chunk
    out += [".Loutmem%=:", "s_set_gpr_idx_off", "s_sub_u32 s56, s60, s62", "s_lshr_b32 s56, s56, 8",
            "s_cmp_lt_u32 s59, s56", "s_cbranch_scc1 .Loutmemg%=",
            "s_sub_u32 s57, s59, s56", "s_lshl_b32 s57, s57, 8", "v_add_u32_e32 v5, s57, %[lds]",
            "ds_read_b32 v4, v5", "s_waitcnt lgkmcnt(0)", "s_branch .Loutmemst%=",
            ".Loutmemg%=:", "s_lshl_b32 s46, s59, 8", "s_add_u32 s46, s62, s46",
            "s_addc_u32 s47, s63, 0", "global_load_dword v4, %[slane], s[46:47]", "s_waitcnt vmcnt(0)",
            "s_mov_b32 s47, s43", ".Loutmemst%=:", "s_add_u32 s59, s59, 1"] + row_dec(52) + [
            "global_store_dword %[lane4], v4, s[52:53]" + cp, MODE_ON, "s_setpc_b64 s[44:45]"]
    return out


def generate(cp: str = "") -> str:
    lines = [
        # inputs -> the block's own registers
        "s_mov_b64 s[40:41], %[cptr]",
        "s_mov_b32 s59, %[j0]",
        "s_mov_b64 s[50:51], %[inp]",
        "s_mov_b64 s[52:53], %[outp]",
        "s_mov_b32 s54, %[rowb]",
        "s_mov_b32 s55, 0",
        "s_mov_b64 s[60:61], %[smem]",
        "s_mov_b64 s[62:63], %[smem]",
        "s_mov_b32 s48, 0",
        # skeleton levels: start reading the first RING slot rows
        "s_cmp_eq_u32 %[refs], 0",
        "s_cbranch_scc1 .Lnoref%=",
    ] + sum((row_dec(50) + [f"global_load_dword v{RING0 + r}, %[lane4], s[50:51]" + cp] for r in range(RING)), []) + [
        ".Lnoref%=:",
        # x+x, x-x, x*x and x%x, once per work item (no index mode is on)
        f"v_add_f32_e32 v{XX0}, %[x], %[x]",
        f"v_sub_f32_e32 v{XX0 + 1}, %[x], %[x]",
        f"v_mul_f32_e32 v{XX0 + 2}, %[x], %[x]",
        f"v_mov_b32_e32 v{W0}, %[x]",
    ] + div_body(W0, W0, W0 + 1, XX0 + 3) + [
        # the lower half holds the next block's codes when we start in the upper half
        "s_cmp_lt_u32 s59, 16",
        "s_cselect_b32 s58, 0, 0x80",
        "s_load_dwordx16 s[64:79], s[40:41], s58",
        "s_load_dwordx16 s[80:95], s[40:41], 0x40",
        "s_getpc_b64 s[42:43]",
        ".Lpc%=:",
        "s_add_u32 s42, s42, .Ltab%= - .Lpc%=",
        "s_addc_u32 s43, s43, 0",
        # the whole table and its routines must share the high address word
        "s_add_u32 s46, s42, .Lend%= - .Ltab%=",
        "s_cbranch_scc1 .Lcarry%=",
        "s_mov_b32 s45, s43",
        "s_mov_b32 s47, s43",
        "s_waitcnt lgkmcnt(0)",
        "s_mov_b32 m0, s59",
        "s_nop 0",
        "s_movrels_b32 s58, s64",
        # the handlers' index mode, on until END: T at window place 0
        f"s_set_gpr_idx_on s55, {MODE}",
        "s_add_u32 s44, s42, s58",
        "s_setpc_b64 s[44:45]",
        ".Lcarry%=:",
        "s_waitcnt lgkmcnt(0)",
        "v_mov_b32_e32 v4, 1",
        "v_mov_b32_e32 v5, 0",
        "global_store_dword v5, v4, %[flag]",
        "s_branch .Lexit%=",
        # the table starts on a 16 KB boundary: its place relative to the
        # instruction cache's sets then does not move with unrelated code
        # (measured: up to 12% apart between placements)
        ".p2align 14",
        ".Ltab%=:",
    ]
    # handlers in address order (positions 15 and 31 sit after the others)
    for off, pos, ki in sorted((code_of(pos, ki), pos, ki) for pos in range(POS) for ki in range(NK)):
        lines.append(f".org .Ltab%= + {off}")
        lines += handler(KINDS[ki], pos, cp)
    lines.append(f".org .Ltab%= + {TABLE_BYTES}")
    lines += routines(cp)
    lines.append(".Lend%=:")
    # no scalar load may still be writing s[64:95] once the block is left
    # nor a vector load still be writing the ring registers
    lines += [".Lexit%=:", "s_waitcnt vmcnt(0) lgkmcnt(0)"]
    return "\n".join(lines) + "\n"


def asm_macro(name: str, text: str) -> str:
    body = "\n".join('    "' + ln.replace('"', '\\"') + '\\n"' for ln in text.splitlines())
    return f"#define {name} \\\n" + body.replace("\n", " \\\n") + "\n"


def write(path: str) -> None:
    clob = ", ".join([f'"v{i}"' for i in range(4, NREG)] + [f'"s{i}"' for i in range(40, 64)]
                     + [f'"s{i}"' for i in range(64, 96)] + ['"m0"', '"vcc"', '"scc"'])
    src = ("// Generated by gen_interp.py: threaded-code interpreter for k_run.\n"
           f"#define EV_CODE_POS {POS}u\n#define EV_CODE_NSTRIDE {NSTRIDE}u\n#define EV_CODE_TSTRIDE {TSTRIDE}u\n"
           f"#define EV_CODE_TBASE {TBASE}u\n#define EV_NK {NK}u\n"
           f"#define EV_VSTACK {VSTACK}u\n#define EV_VHALF {HALF}u\n#define EV_RING {RING}u\n"
           f"#define EV_INTERP_CLOBBERS {clob}\n"
           + "".join(f"#define EV_K_{k} {i}u\n" for i, k in enumerate(KINDS))
           + asm_macro("EV_INTERP_ASM", generate())
           # slot rows read and written at device scope (sc1): coherent with
           # other work groups of the same launch without cache maintenance
           + asm_macro("EV_INTERP_ASM_COH", generate(" sc1")))
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write(src)
    os.replace(tmp, path)


if __name__ == "__main__":
    write(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                               "ev_interp.inc"))
