// Device kernels of libev (gfx950).
//
// Trees are prefix words of one-byte tokens (Sec. 2.2 of Langdon & Banzhaf
// 2019): 0 ADD, 1 SUB, 2 MUL, 3 DIV (protected), 4 X; the split plan adds
// 5 REF, a leaf whose value is an intermediate result slot.
//
// Evaluation is the paper's single pass over each buffer for all test cases
// with an operand stack whose frames hold one float per case (Sec. 2.2),
// re-mapped to the GPU: one wavefront interprets one work item, the token
// stream is read with scalar loads and is uniform across the wave, and lane
// i carries test case i.  The tokens of a work item are processed right to
// left, so a function finds its first argument on top of the stack and its
// second below it.
//
// A work item ("chunk") is a contiguous token range of one tree.  Values
// inside it whose enclosing function lies outside it are written to result
// slots and replaced by REF tokens in the next level's skeleton, which is
// again split into chunks until each tree is a single value.  Every
// function node still combines exactly the operands it would in a
// sequential pass, so the results do not depend on the split.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ev_internal.h"
#include "ev_interp.inc"

namespace ev {

// Read-only data that is wave-uniform goes through the scalar cache.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) u32x4* const_u4p;
typedef const __attribute__((address_space(1))) u32x4* global_u4p;

// ------------------------------------------------------------ utilities

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// A copy between device memory and the host's pinned staging buffer, done
// by the stream's own compute queue: a small transfer then needs no handoff
// to a DMA engine and back (which costs more than the copy).  16-byte moves
// when both ends and the size allow, else 4-byte, else bytes.
__global__ void k_fill_u8(uint8_t* __restrict__ p, uint64_t n, uint8_t v)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_copy(uint8_t* __restrict__ dst, const uint8_t* __restrict__ src, uint64_t n, uint32_t w)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i * w >= n) return;
    if (w == 16)
        reinterpret_cast<u32x4*>(dst)[i] = reinterpret_cast<const u32x4*>(src)[i];
    else if (w == 4)
        reinterpret_cast<uint32_t*>(dst)[i] = reinterpret_cast<const uint32_t*>(src)[i];
    else
        dst[i] = src[i];
    __threadfence_system();  // host-visible before the stream's next marker
}

// Protected division and the three other functions (Sec. 2.1, Table 1).
__device__ __forceinline__ float apply_op(uint32_t t, float a, float b)
{
    switch (t) {
    case TOK_ADD: return a + b;
    case TOK_SUB: return a - b;
    case TOK_MUL: return a * b;
    default: return (b != 0.0f) ? a / b : 1.0f;
    }
}

// ------------------------------------------------------ structure machine
//
// The right-to-left stack machine of both interpreters, run without values:
//   tv  the top value T is live      P  an X sits on top, not yet placed
//   m   values below T               base  of those, how many live in the
//                                          wave's spill slab (a multiple of
//                                          the half window)
// A function meeting fewer than two values is a "spine" node: its subtree
// leaves the chunk; the value it would take from the chunk (at most one)
// becomes a result slot (or stays an X when it is a bare input) and the
// node goes into the next level's skeleton.  At the chunk's first token all
// values still on the stack become result slots.  For the register-stack
// interpreter every action is also written as one code, an X folded into
// the function or push that consumes it, and a push or load of x directly
// followed by a function of x fused into one code; SPILL and FILL keep T
// inside the window of EV_VSTACK register entries.
//
// The structure passes run in parallel over 256-token segments.  The number
// of values on the stack, cnt, changes as cnt+1 for a leaf and max(cnt-1, 0)
// for a function (spine included), maps of the form c -> max(c+a, b) that
// compose associatively; so a per-segment map, folded over a chunk's
// segments, gives each segment its starting state (cnt; P is whether the
// previously read token was an X; tv and m follow).  The window is put in a
// fixed position for the starting m at every segment boundary (extra SPILL
// or FILL codes), so each segment's codes depend on its own tokens only.
// One implementation serves counting and emission, so they cannot disagree.

// Window base for a given m at a segment boundary: T at index m if m < 48,
// else at an index in [16, 47].
__device__ __forceinline__ uint32_t norm_base(uint32_t m)
{
    return m < EV_VSTACK - EV_VHALF / 2 ? 0u : (m - EV_VHALF / 2) / EV_VHALF * EV_VHALF;
}

// Handler offset of a code at index `at` (its position is at mod 32): the
// layout written by gen_interp.py.  Arithmetic only, so that no branch
// appears around it.
static_assert(EV_CODE_POS == 32 && EV_CODE_NSTRIDE == 32 && EV_CODE_TSTRIDE == 64, "code layout");
// tr: 1 at the refill positions 15 and 31, whose handlers are 64 bytes apart
__device__ __forceinline__ uint32_t code_tr(uint32_t pos) { return ((pos & 15u) + 1u) >> 4; }
// offset of kind 0's handler at a position
__device__ __forceinline__ uint32_t code_base(uint32_t pos)
{
    const uint32_t hi = pos >> 4;  // second half of the block
    const uint32_t nb = (pos - hi) * (EV_NK * EV_CODE_NSTRIDE);
    const uint32_t tb = EV_CODE_TBASE + hi * (EV_NK * EV_CODE_TSTRIDE);
    const uint32_t mask = 0u - code_tr(pos);
    return (nb & ~mask) | (tb & mask);
}
__device__ __forceinline__ uint32_t code_value(uint64_t at, uint32_t kind)
{
    const uint32_t pos = (uint32_t)at & 31u;
    return code_base(pos) + (kind << (5u + code_tr(pos)));
}

struct Sink {
    uint32_t* codes;   // nullptr: count codes only
    uint64_t at;       // global index of the next code
    uint8_t* frag;     // nullptr: count fragment tokens only
    uint64_t w;        // one past the next fragment token (written backwards)
    uint32_t n_codes, n_frag, n_out, n_in;
    uint32_t pending;  // an action waiting for a partner to fuse with, or ~0u
    uint32_t ref;      // index of the next REF within the work item (its ring slot mod EV_RING)
    // Recording (the count pass): the segment's code kinds, one byte each,
    // stored four at a time (rk is 4-byte aligned), and its fragment tokens
    // in emission order, each into a region of the given capacity (nullptr:
    // not recorded); ovf is set if one overflows.  The chunk-end runs of slot
    // writes are not recorded, only where they go (rec).
    uint8_t* rk;
    uint8_t* rf;
    uint32_t rk_cap, rf_cap, ovf;
    uint32_t nr, kacc;  // kinds recorded, and the word being filled
    SegRec rec;

    __device__ __forceinline__ void rec_kind(uint32_t kind)
    {
        const uint32_t j = nr++;
        kacc |= kind << (8u * (j & 3u));
        if ((j & 3u) == 3u) {
            if ((j & ~3u) + 4u <= rk_cap)
                *reinterpret_cast<uint32_t*>(rk + (j & ~3u)) = kacc;
            else
                ovf = 1;
            kacc = 0;
        }
    }
    // the last, partly filled word
    __device__ __forceinline__ void rec_end()
    {
        if (rk && (nr & 3u)) {
            if ((nr & ~3u) + 4u <= rk_cap)
                *reinterpret_cast<uint32_t*>(rk + (nr & ~3u)) = kacc;
            else
                ovf = 1;
        }
    }
    __device__ __forceinline__ void put(uint32_t kind)
    {
        if (codes) codes[at] = code_value(at, kind);
        if (rk) rec_kind(kind);
        at++;
        n_codes++;
    }
    // count codes of one kind (which: 1 the memory run, 2 the window run)
    __device__ __forceinline__ void run(uint32_t kind, uint32_t count, uint32_t which)
    {
        if (rk) {
            if (which == 1) {
                rec.a1 = nr;
                rec.n1 = count;
            } else {
                rec.a2 = nr;
                rec.n2 = count;
            }
        } else if (codes) {
            for (uint32_t i = 0; i < count; i++) codes[at + i] = code_value(at + i, kind);
        }
        at += count;
        n_codes += count;
    }
    __device__ void flush()
    {
        if (pending != ~0u) {
            put(pending);
            pending = ~0u;
        }
    }
    // Fusions: a push or load of x then a function of x (CH, LCH); two
    // pushes of x (PUSH2X), which waits in turn for a function of x
    // (PXCH: push x, push op(x, x)); two pops by + - * in a row (OPSab).
    __device__ void code(uint32_t kind)
    {
        if (pending != ~0u) {
            const uint32_t p = pending;
            if ((p == EV_K_PUSHX || p == EV_K_LOADX) && kind >= EV_K_OPX0 && kind <= EV_K_OPX3) {
                pending = ~0u;
                put((p == EV_K_PUSHX ? EV_K_CH0 : EV_K_LCH0) + (kind - EV_K_OPX0));
                return;
            }
            if (p == EV_K_PUSH2X && kind >= EV_K_OPX0 && kind <= EV_K_OPX3) {
                pending = ~0u;
                put(EV_K_PXCH0 + (kind - EV_K_OPX0));
                return;
            }
            if (p == EV_K_PUSHX && kind == EV_K_PUSHX) {
                pending = EV_K_PUSH2X;
                return;
            }
            if (p <= EV_K_OPS2 && kind <= EV_K_OPS2) {
                pending = ~0u;
                put(EV_K_OPS00 + p * 3u + kind);
                return;
            }
            flush();
        }
        if (kind == EV_K_PUSHX || kind == EV_K_LOADX || kind <= EV_K_OPS2) {
            pending = kind;
            return;
        }
        put(kind);
    }
    __device__ __forceinline__ void ftok(uint32_t t)
    {
        if (frag) frag[--w] = (uint8_t)t;
        if (rf) {
            if (n_frag < rf_cap)
                rf[n_frag] = (uint8_t)t;
            else
                ovf = 1;
        }
        n_frag++;
    }
    // count fragment tokens t (the chunk-end REFs, last in emission order;
    // not recorded)
    __device__ __forceinline__ void ftok_run(uint32_t t, uint32_t count)
    {
        if (frag)
            for (uint32_t i = 0; i < count; i++) frag[--w] = (uint8_t)t;
        n_frag += count;
    }
    // put(e) unless e is ~0u, without branching on e
    __device__ __forceinline__ void put_if(uint32_t e)
    {
        const uint32_t has = e != ~0u ? 1u : 0u;
        if (codes && has) codes[at] = code_value(at, e);
        if (rk && has) rec_kind(e);
        at += has;
        n_codes += has;
    }
    // code() for kind in {none (~0u), OPX*, OPS*, PUSHX, LOADX}, with selects:
    // the same fusions and the same order of codes as code()
    __device__ __forceinline__ void code_fast(uint32_t kind)
    {
        const uint32_t p = pending;
        const bool none = kind == ~0u;
        const bool opx = kind - EV_K_OPX0 < 4u;
        const bool ch = (p == EV_K_PUSHX || p == EV_K_LOADX) && opx;
        const bool pxch = p == EV_K_PUSH2X && opx;
        const bool xx = p == EV_K_PUSHX && kind == EV_K_PUSHX;  // fused into a pending PUSH2X
        const bool ops = p <= EV_K_OPS2 && kind <= EV_K_OPS2;
        const bool fused = ch || pxch || ops;
        const uint32_t fk = ch ? (p == EV_K_PUSHX ? EV_K_CH0 : EV_K_LCH0) + (kind - EV_K_OPX0)
                               : (pxch ? EV_K_PXCH0 + (kind - EV_K_OPX0) : EV_K_OPS00 + p * 3u + kind);
        const bool defer = kind == EV_K_PUSHX || kind == EV_K_LOADX || kind <= EV_K_OPS2;
        const uint32_t e1 = (none || xx) ? ~0u : (fused ? fk : p);
        const uint32_t e2 = (none || xx || fused || defer) ? ~0u : kind;
        pending = none ? p : (xx ? EV_K_PUSH2X : ((fused || !defer) ? ~0u : kind));
        put_if(e1);
        put_if(e2);
    }
};

// Calls f(t) for the tokens of [start, start+len) right to left.  Tokens
// are read in aligned 16-byte blocks, the next block to the left in flight
// while a block's tokens are worked (a block loop around a token loop, so
// that the prefetched block needs no conditional copy).  Whole blocks are
// read: up to 15 bytes on either side of the range, and the range's first
// block once more at the end, all inside the buffers' padding.
template <class F>
__device__ __forceinline__ void for_tokens_rev(const uint8_t* __restrict__ seq, uint64_t start, uint32_t len, F&& f)
{
    if (!len) return;
    const uint64_t first = start & ~(uint64_t)15;
    uint64_t b = (start + len - 1) & ~(uint64_t)15;
    uint32_t jhi = (uint32_t)((start + len - 1) & 15);
    u32x4 nxt = *reinterpret_cast<const u32x4*>(seq + b);
    for (;;) {
        const u32x4 cur = nxt;
        nxt = *reinterpret_cast<const u32x4*>(seq + (b > first ? b - 16 : b));
        const uint32_t jlo = b == first ? (uint32_t)(start & 15) : 0u;
        for (uint32_t j = jhi + 1; j-- > jlo;) {
            const uint32_t word = j >= 8 ? (j >= 12 ? cur.w : cur.z) : (j >= 4 ? cur.y : cur.x);
            f((word >> (8 * (j & 3))) & 255u);
        }
        if (b == first) break;
        b -= 16;
        jhi = 15;
    }
}

// Machine over one segment from a given start.  last: the segment holding
// the chunk's first token (it ends with the chunk's flush and END); other
// segments end by putting the window in its boundary position.
__device__ uint32_t run_segment(const uint8_t* __restrict__ seq, uint64_t start, uint32_t len, uint32_t cnt_in,
                                uint32_t P_in, uint32_t ptok_in, bool last, Sink& o)
{
    // P: the token read before is a leaf whose push is still pending: x, or
    // an ephemeral random constant (token ptok), which the structure treats
    // alike (a plan holding constants runs on k_eval, which reads tokens)
    uint32_t P = P_in, ptok = ptok_in;
    uint32_t tv = cnt_in > P ? 1u : 0u;
    uint32_t m = cnt_in - tv - P;
    uint32_t base = norm_base(m), maxtop = m;
    for_tokens_rev(seq, start, len, [&](const uint32_t t) {
        // Common tokens, decided with selects so that lanes on different
        // token kinds do not diverge: a function finding two values without
        // a FILL, and an x needing no SPILL.  The rest take the full path.
        const uint32_t cnt = m + tv + P;
        const bool leaf = t == TOK_X || t >= TOK_C0;
        const bool fast_fn = t < TOK_X && cnt >= 2 && (P || m != base || base == 0);
        const bool fast_x = leaf && !(P && tv && m + 1 - base > EV_VSTACK - 1);
        if (fast_fn || fast_x) {
            const uint32_t kx = !P ? ~0u : (tv ? EV_K_PUSHX : EV_K_LOADX);
            const uint32_t kind = fast_fn ? (P ? EV_K_OPX0 + t : EV_K_OPS0 + t) : kx;
            m = fast_fn ? m - (P ? 0u : 1u) : m + ((P && tv) ? 1u : 0u);
            tv = fast_fn ? tv : (tv | P);
            P = fast_fn ? 0u : 1u;
            ptok = fast_fn ? ptok : t;
            o.code_fast(kind);
            maxtop = m > maxtop ? m : maxtop;
            return;
        }
        if (leaf) {
            ptok = t;
            if (!P) {
                P = 1;
            } else if (tv) {
                if (m + 1 - base > EV_VSTACK - 1) { o.code(EV_K_SPILL); base += EV_VHALF; }
                o.code(EV_K_PUSHX);
                m++;
            } else {
                o.code(EV_K_LOADX);
                tv = 1;
            }
        } else if (t == TOK_REF) {
            o.n_in++;
            if (P) {
                if (tv) {
                    if (m + 1 - base > EV_VSTACK - 1) { o.code(EV_K_SPILL); base += EV_VHALF; }
                    o.code(EV_K_PUSHX);
                    m++;
                } else {
                    o.code(EV_K_LOADX);
                    tv = 1;
                }
                P = 0;
            }
            const uint32_t slot = o.ref++ & (EV_RING - 1);
            if (tv) {
                if (m + 1 - base > EV_VSTACK - 1) { o.code(EV_K_SPILL); base += EV_VHALF; }
                o.code(EV_K_PUSHREF0 + slot);
                m++;
            } else {
                o.code(EV_K_LOADREF0 + slot);
                tv = 1;
            }
        } else if (t < TOK_X) {
            const uint32_t cnt = m + tv + P;
            if (cnt >= 2) {
                if (P) {
                    o.code(EV_K_OPX0 + t);
                    P = 0;
                } else {
                    if (m == base && base > 0) { o.code(EV_K_FILL); base -= EV_VHALF; }
                    o.code(EV_K_OPS0 + t);
                    m--;
                }
            } else {
                if (cnt == 1) {
                    if (!P) { o.code(EV_K_OUTT); o.n_out++; }
                    o.ftok(P ? ptok : TOK_REF);
                }
                o.ftok(t);
                tv = 0; P = 0; m = 0;
            }
        }
        maxtop = m > maxtop ? m : maxtop;
    });
    if (!last) {
        o.flush();
        const uint32_t nb = norm_base(m);
        while (base < nb) { o.put(EV_K_SPILL); base += EV_VHALF; }
        while (base > nb) { o.put(EV_K_FILL); base -= EV_VHALF; }
        return maxtop;
    }
    // the chunk's first token: every value left becomes a slot, bottom first
    // (nothing is pending after a FLUSH, so the runs are put directly)
    if (base > 0) {
        o.code(EV_K_FLUSH);
        o.run(EV_K_OUTMEM, base, 1);
    }
    if (m > base) {
        o.code(EV_K_FLUSH);
        o.run(EV_K_OUTBOT, m - base, 2);
    }
    if (tv) o.code(EV_K_OUTT);
    if (P) o.code(EV_K_OUTX);
    o.code(EV_K_END);
    const uint32_t left = m + tv + P;
    o.n_out += left;
    o.rec.nfr = o.n_frag;
    o.ftok_run(TOK_REF, left);
    return maxtop;
}

// Segments of a level: segment s of chunk c covers tokens
// [c.start + s*SEG, ...) and is read after segment s+1.

// The segments of every chunk: block j writes chunk j's.  Segment 0 holds
// the chunk's first `head` tokens and the others `seg_len` each: segment 0
// also emits the chunk's final flush (a slot per value left), so it is kept
// short to keep its lane from lagging behind the wave.
__global__ void k_seg_build(const ChunkIn* __restrict__ ch, const ChunkSegs* __restrict__ cg, uint32_t n,
                            uint32_t seg_len, uint32_t head, SegIn* __restrict__ seg, const GLevel* __restrict__ gl)
{
    if (gl) n = gl->n;
    const uint32_t j = blockIdx.x;
    if (j >= n) return;
    const ChunkIn c = ch[j];
    const ChunkSegs g = cg[j];
    for (uint32_t k = threadIdx.x; k < g.n_seg; k += blockDim.x) {
        const uint32_t o = k == 0 ? 0u : head + (k - 1) * seg_len;
        const uint32_t cap = k == 0 ? head : seg_len;
        const uint32_t len = c.len - o < cap ? c.len - o : cap;
        seg[g.first + k] = SegIn{c.start + o, len, k == 0 ? 1u : 0u};
    }
}

// ------------------------------------------------- split plan on the device
//
// A level's chunks and segments from its trees: block i writes the chunks
// of tree i (all but the last hold C tokens) and their segment records.
__device__ __forceinline__ uint32_t seg_count(uint32_t len, uint32_t seg_len, uint32_t head)
{
    return len <= head ? 1u : 1u + (len - head + seg_len - 1) / seg_len;
}

__global__ __launch_bounds__(64) void k_plan_chunks(const TreeLvl* __restrict__ trees, uint32_t n_trees,
                                                    uint32_t seg_len, uint32_t head, ChunkIn* __restrict__ ch,
                                                    ChunkSegs* __restrict__ cg, uint32_t* __restrict__ err_init,
                                                    uint32_t n_err, const GLevel* __restrict__ gl)
{
    if (gl) n_trees = gl->nt;
    const uint32_t i = blockIdx.x;
    if (i == 0 && err_init)  // the validator's words of every level: no flags, no failing segment
        for (uint32_t k = threadIdx.x; k < n_err; k += blockDim.x) err_init[k] = (k & 1u) ? UINT32_MAX : 0u;
    if (i >= n_trees) return;
    const TreeLvl tl = trees[i];
    const uint32_t full = seg_count(tl.C, seg_len, head);
    for (uint32_t k = threadIdx.x; k < tl.n_chunks; k += blockDim.x) {
        const uint64_t o = (uint64_t)k * tl.C;
        const uint32_t len = tl.len - o < tl.C ? (uint32_t)(tl.len - o) : tl.C;
        const uint32_t j = tl.chunk_first + k;
        ch[j] = ChunkIn{tl.start + o, len, tl.tree};
        cg[j] = ChunkSegs{tl.seg_first + k * full, seg_count(len, seg_len, head)};
    }
}

__device__ __forceinline__ uint32_t len_bucket(uint32_t len) { return len ? (uint32_t)__clz(len) : 32u; }


// One wave per tree: the numbering of its chunks' slots, fragment tokens and
// codes relative to the tree (exclusive for codes, inclusive for slots and
// fragments), its chunks' input slots (the k-th REF of a level reads the
// previous level's slot k), the tree's totals and, at level 0, its validity
// (Sec. 2.2: every token fills one open slot and a function opens two; a
// tree is valid iff a slot is open before each token and none after the
// last).
__global__ __launch_bounds__(64) void k_plan_trees(const TreeLvl* __restrict__ trees, uint32_t n_trees,
                                                   const ChunkStat* __restrict__ cs, uint32_t level, uint64_t prev_out,
                                                   uint64_t* __restrict__ code_loc, uint64_t* __restrict__ out_loc,
                                                   uint64_t* __restrict__ frag_loc, uint32_t* __restrict__ in_end,
                                                   TreeSum* __restrict__ sum, const GLevel* __restrict__ gl)
{
    if (gl) {
        n_trees = gl->nt;
        prev_out = gl->prev_out;
    }
    const uint32_t i = blockIdx.x;
    if (i >= n_trees) return;
    const int lane = (int)threadIdx.x;
    const TreeLvl tl = trees[i];
    uint64_t c_out = 0, c_frag = 0, c_code = 0, c_in = tl.ref_base;
    int64_t c_open = 1;
    uint32_t bad = 0, maxtop = 0, max_m = 0;
    for (uint32_t g = 0; g < tl.n_chunks; g += 64) {
        const uint32_t k = g + (uint32_t)lane;
        const bool in = k < tl.n_chunks;
        const uint32_t j = tl.chunk_first + (in ? k : 0);
        ChunkStat q = {};
        if (in) q = cs[j];
        // every chunk's codes start a 128-byte block (its codes are then the
        // same words wherever the block lands, so a child's plan can copy them)
        const uint64_t padc = ((uint64_t)q.n_codes + (EV_CODE_POS - 1)) & ~(uint64_t)(EV_CODE_POS - 1);
        uint64_t so = q.n_out, sf = q.n_frag, sc = padc, si = q.n_in;
        int64_t sn = q.net;
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t a = __shfl_up(so, d, 64), b = __shfl_up(sf, d, 64), c = __shfl_up(sc, d, 64),
                           e = __shfl_up(si, d, 64);
            const int64_t f = __shfl_up(sn, d, 64);
            if (lane >= d) {
                so += a;
                sf += b;
                sc += c;
                si += e;
                sn += f;
            }
        }
        if (in) {
            code_loc[j] = c_code + sc - padc;
            out_loc[j] = c_out + so;
            frag_loc[j] = c_frag + sf;
            const uint64_t ie = c_in + si;
            in_end[j] = (uint32_t)ie;
            if (ie > prev_out) bad |= 2u;
            if (level == 0 && ((q.bad & BAD_TOKEN) || c_open + (sn - q.net) + q.minpref < 1)) bad |= 1u;
            if (q.bad & BAD_TOKEN) bad |= level == 0 ? 1u : 2u;
            bad |= q.bad & HAS_CONST;
            maxtop = q.maxtop > maxtop ? q.maxtop : maxtop;
            max_m = q.max_m > max_m ? q.max_m : max_m;
        }
        c_out += __shfl(so, 63, 64);
        c_frag += __shfl(sf, 63, 64);
        c_code += __shfl(sc, 63, 64);
        c_in += __shfl(si, 63, 64);
        c_open += __shfl(sn, 63, 64);
    }
    for (int d = 32; d > 0; d >>= 1) {
        bad |= __shfl_xor(bad, d, 64);
        const uint32_t a = __shfl_xor(maxtop, d, 64), b = __shfl_xor(max_m, d, 64);
        maxtop = a > maxtop ? a : maxtop;
        max_m = b > max_m ? b : max_m;
    }
    if (level == 0 && c_open != 0) bad |= 1u;
    if (lane == 0) sum[i] = TreeSum{c_out, c_frag, c_code, bad, maxtop, max_m, 0};
}

// One block: the trees' bases over the level's chunks, in sequence order
// (which is tree order): exclusive sums of their slots, fragment tokens and
// codes, stored by tree id with the tree's chunk range and bucket ranks.
// Rounds of 1024 consecutive trees (coalesced reads), each scanned by wave
// shuffles and the waves' totals, on top of the previous rounds' total.
__global__ __launch_bounds__(1024) void k_plan_bases(const TreeLvl* __restrict__ trees, uint32_t n_trees,
                                                     const TreeSum* __restrict__ sum, TreeBase* __restrict__ base,
                                                     const GLevel* __restrict__ gl)
{
    if (gl) n_trees = gl->nt;
    __shared__ uint64_t wo[16], wf[16], wc[16], carry[3];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    if (t == 0) carry[0] = carry[1] = carry[2] = 0;
    __syncthreads();
    for (uint32_t r0 = 0; r0 < n_trees; r0 += 1024) {
        const uint32_t i = r0 + t;
        uint64_t o = 0, f = 0, c = 0;
        if (i < n_trees) {
            o = sum[i].n_out;
            f = sum[i].n_frag;
            c = sum[i].n_codes;
        }
        uint64_t so = o, sf = f, sc = c;  // inclusive sums within the wave
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t ao = __shfl_up(so, d), af = __shfl_up(sf, d), ac = __shfl_up(sc, d);
            if (lane >= d) {
                so += ao;
                sf += af;
                sc += ac;
            }
        }
        if (lane == 63) {
            wo[w] = so;
            wf[w] = sf;
            wc[w] = sc;
        }
        __syncthreads();
        uint64_t bo = carry[0], bf = carry[1], bc = carry[2];
        for (uint32_t k = 0; k < w; k++) {
            bo += wo[k];
            bf += wf[k];
            bc += wc[k];
        }
        if (i < n_trees) {
            const TreeLvl tl = trees[i];
            base[tl.tree] = TreeBase{bo + so - o, bf + sf - f, bc + sc - c, tl.chunk_first, tl.n_chunks, tl.rank_full,
                                     tl.rank_last};
        }
        __syncthreads();  // every thread has read carry and the waves' totals
        if (t == 1023) {  // the round's total (trees past the end add zero)
            carry[0] = bo + so;
            carry[1] = bf + sf;
            carry[2] = bc + sc;
        }
        __syncthreads();
    }
}

// Per chunk: its global numbering from its tree's bases, and its work item,
// placed longest first (bucket_start: the first place of each length
// bucket, zero where the tree's ranks are places already; the tree gives
// the chunk's rank inside its bucket).
__global__ void k_plan_items(const ChunkIn* __restrict__ ch, uint32_t n, const TreeBase* __restrict__ base,
                             const uint64_t* __restrict__ code_loc, const uint64_t* __restrict__ out_loc,
                             const uint64_t* __restrict__ frag_loc, const uint32_t* __restrict__ in_end,
                             const uint32_t* __restrict__ bucket_start, uint64_t* __restrict__ code_begin,
                             uint64_t* __restrict__ frag_end, RunChunk* __restrict__ run, EvalChunk* __restrict__ slow,
                             uint32_t* __restrict__ code_tail, uint8_t* __restrict__ frag_tail,
                             const GLevel* __restrict__ gl, uint32_t* __restrict__ item_tree)
{
    if (gl) {  // the tails follow the level's live totals
        n = gl->n;
        if (code_tail) code_tail += gl->sc;
        if (frag_tail) frag_tail += gl->sf;
    }
    if (blockIdx.x == 0) {
        // the padding after the level's code stream (zeros) and after the
        // next level's skeleton (0xFF): the readers' wide loads reach it
        for (uint32_t i = threadIdx.x; code_tail && i < 128; i += blockDim.x) code_tail[i] = 0;
        for (uint32_t i = threadIdx.x; frag_tail && i < 64; i += blockDim.x) frag_tail[i] = 0xFF;
    }
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const ChunkIn c = ch[j];
    const TreeBase b = base[c.tree];
    const uint64_t cb = b.code + code_loc[j];
    const uint32_t oe = (uint32_t)(b.out + out_loc[j]);
    code_begin[j] = run ? cb : ~0ull;
    frag_end[j] = b.frag + frag_loc[j];
    const uint32_t k = j - b.chunk_first;
    const uint32_t at = bucket_start[len_bucket(c.len)] + (k + 1 < b.n_chunks ? b.rank_full + k : b.rank_last);
    if (item_tree) item_tree[at] = c.tree;
    if (run)
        run[at] = RunChunk{cb, in_end[j], oe};
    else
        slow[at] = EvalChunk{c.start, c.len, in_end[j], oe, c.tree, 0, 0};
}

// ------------------------------------------ children reusing their mum's level 0
//
// A child of Sec. 3.1's crossover is its mum with the subtree at p (ending
// at ep) replaced by a subtree of the dad.  The right-to-left structure
// machine of a level-0 chunk starts from an empty stack at the chunk's end,
// so a chunk's codes and skeleton fragment depend on its own tokens alone:
// the mum's chunks wholly before p and wholly after ep are the child's too.
// Only the tokens between them are planned; the rest is copied.

// One thread per child: which of its mum's chunks it keeps, and the tokens
// to plan.  A child over the size cap is a copy of its mum and keeps every
// chunk.  The mum's chunks lie in token order, so the chunk holding p and
// the first chunk after ep are found by binary search.
__global__ void k_reuse_runs(const XoPlan* __restrict__ plan, const int32_t* __restrict__ mum,
                             const L0Tree* __restrict__ trees, const ChunkIn* __restrict__ mum_ch, uint32_t n,
                             ReuseRun* __restrict__ out)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const XoPlan x = plan[j];
    const L0Tree t = trees[mum[j]];
    ReuseRun r;
    r.src_first = t.chunk_first;
    r.mum_off = x.mum_off;
    r.mum = (uint32_t)mum[j];
    r.pad = 0;
    r.n_pre = r.ks = r.n_suf = 0;
    r.mid_start = 0;
    r.mid_len = x.child_len;
    r.shift = 0;
    if (x.copy_mum) {
        r.n_pre = t.n_chunks;
        r.ks = t.n_chunks;
        r.mid_start = x.child_len;
        r.mid_len = 0;
    } else if (t.n_chunks > 1) {
        const ChunkIn* c = mum_ch + t.chunk_first;
        // kp: the chunks ending at or before p; ks: the first starting after ep
        uint32_t lo = 0, hi = t.n_chunks;
        while (lo < hi) {
            const uint32_t m = (lo + hi) / 2;
            if (c[m].start - x.mum_off + c[m].len <= x.p) lo = m + 1; else hi = m;
        }
        const uint32_t kp = lo;
        lo = kp;
        hi = t.n_chunks;
        while (lo < hi) {
            const uint32_t m = (lo + hi) / 2;
            if (c[m].start - x.mum_off <= x.ep) lo = m + 1; else hi = m;
        }
        const uint32_t ks = lo;
        const uint64_t mum_len = c[t.n_chunks - 1].start - x.mum_off + c[t.n_chunks - 1].len;
        r.n_pre = kp;
        r.ks = ks;
        r.n_suf = t.n_chunks - ks;
        r.shift = (int64_t)x.child_len - (int64_t)mum_len;
        r.mid_start = c[kp].start - x.mum_off;
        const uint64_t mid_end = ks < t.n_chunks ? (uint64_t)((int64_t)(c[ks].start - x.mum_off) + r.shift) : x.child_len;
        r.mid_len = mid_end - r.mid_start;
    }
    out[j] = r;
}

// One block per child: its chunk records in token order (kept prefix,
// fresh chunks, kept suffix), the segments of its fresh chunks, and each
// chunk's source (the mum's chunk index, or ~0u for a fresh chunk).  Block
// 0 also initializes the validator's words, as k_plan_chunks does.
__global__ __launch_bounds__(64) void k_reuse_chunks(const TreeReuse* __restrict__ trees, uint32_t n_trees,
                                                     const ChunkIn* __restrict__ mum_ch, uint32_t seg_len, uint32_t head,
                                                     ChunkIn* __restrict__ ch, ChunkSegs* __restrict__ cg,
                                                     uint32_t* __restrict__ src, uint32_t* __restrict__ err_init,
                                                     uint32_t n_err)
{
    const uint32_t i = blockIdx.x;
    if (i == 0 && err_init)
        for (uint32_t k = threadIdx.x; k < n_err; k += blockDim.x) err_init[k] = (k & 1u) ? UINT32_MAX : 0u;
    if (i >= n_trees) return;
    const TreeReuse t = trees[i];
    const uint32_t n_chunks = t.r.n_pre + t.n_mid + t.r.n_suf;
    const uint32_t full = seg_count(t.C, seg_len, head);
    for (uint32_t k = threadIdx.x; k < n_chunks; k += blockDim.x) {
        uint64_t off;
        uint32_t len, from = ~0u, first = 0, nseg = 0;
        if (k < t.r.n_pre || k >= t.r.n_pre + t.n_mid) {
            const bool pre = k < t.r.n_pre;
            from = t.r.src_first + (pre ? k : t.r.ks + (k - t.r.n_pre - t.n_mid));
            const ChunkIn mc = mum_ch[from];
            off = (uint64_t)((int64_t)(mc.start - t.r.mum_off) + (pre ? 0 : t.r.shift));
            len = mc.len;
        } else {
            const uint32_t m = k - t.r.n_pre;
            off = t.r.mid_start + (uint64_t)m * t.C;
            len = m + 1 == t.n_mid ? t.mid_last : t.C;
            first = t.seg_first + m * full;
            nseg = seg_count(len, seg_len, head);
        }
        const uint32_t j = t.chunk_first + k;
        ch[j] = ChunkIn{t.start + off, len, t.tree};
        cg[j] = ChunkSegs{first, nseg};
        src[j] = from;
    }
}

// Kept chunks take their mum's totals (after the fresh chunks' were made).
__global__ void k_reuse_stats(const uint32_t* __restrict__ src, uint32_t n, const ChunkStat* __restrict__ mum_stat,
                              ChunkStat* __restrict__ cstat)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t f = src[j];
    if (f != ~0u) cstat[j] = mum_stat[f];
}

// One block per chunk: a kept chunk's codes (whole 128-byte blocks: every
// chunk's codes start a block in both plans) and its skeleton fragment
// (bytes [frag_end - n_frag, frag_end) of each level-1 skeleton).
__global__ __launch_bounds__(256) void k_reuse_copy(const uint32_t* __restrict__ src, uint32_t n,
                                                    const ChunkStat* __restrict__ cstat,
                                                    const uint64_t* __restrict__ code_begin,
                                                    const uint64_t* __restrict__ frag_end,
                                                    const uint64_t* __restrict__ mum_code,
                                                    const uint64_t* __restrict__ mum_frag,
                                                    const uint32_t* __restrict__ mum_codes,
                                                    const uint8_t* __restrict__ mum_skel, uint32_t* __restrict__ codes,
                                                    uint8_t* __restrict__ skel)
{
    const uint32_t j = blockIdx.x;
    if (j >= n) return;
    const uint32_t f = src[j];
    if (f == ~0u) return;
    const ChunkStat q = cstat[j];
    if (codes) {
        const u32x4* a = reinterpret_cast<const u32x4*>(mum_codes + mum_code[f]);
        u32x4* b = reinterpret_cast<u32x4*>(codes + code_begin[j]);
        const uint32_t words = ((q.n_codes + (EV_CODE_POS - 1)) & ~(EV_CODE_POS - 1)) / 4u;
        const uint32_t step = blockDim.x;
        uint32_t w = threadIdx.x;
        // four loads in flight per thread; streamed past the caches (measured
        // 6% faster on the largest populations' copies)
        for (; w + 3 * step < words; w += 4 * step) {
            const u32x4 v0 = __builtin_nontemporal_load(&a[w]), v1 = __builtin_nontemporal_load(&a[w + step]),
                        v2 = __builtin_nontemporal_load(&a[w + 2 * step]),
                        v3 = __builtin_nontemporal_load(&a[w + 3 * step]);
            __builtin_nontemporal_store(v0, &b[w]);
            __builtin_nontemporal_store(v1, &b[w + step]);
            __builtin_nontemporal_store(v2, &b[w + 2 * step]);
            __builtin_nontemporal_store(v3, &b[w + 3 * step]);
        }
        for (; w < words; w += step) b[w] = a[w];
    }
    if (skel) {
        const uint8_t* a = mum_skel + (mum_frag[f] - q.n_frag);
        uint8_t* b = skel + (frag_end[j] - q.n_frag);
        for (uint32_t w = threadIdx.x; w < q.n_frag; w += blockDim.x) b[w] = a[w];
    }
}

// Per segment: its cnt map (a, b), validity counters and input references.
__global__ void k_seg_fn(const uint8_t* __restrict__ seq, const SegIn* __restrict__ segs, uint32_t n,
                         SegFn* __restrict__ out, uint32_t ref_ok, uint32_t n_consts, const GLevel* __restrict__ gl)
{
    if (gl) n = gl->n_seg;
    const uint32_t si = blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= n) return;
    const SegIn g = segs[si];
    int32_t a = 0, b = INT32_MIN / 2, R = 0, maxR = INT32_MIN;
    uint32_t bad = 0, n_in = 0, last_t = 0;
    for_tokens_rev(seq, g.start, g.len, [&](const uint32_t t) {
        const bool is_const = t >= TOK_C0 && t < TOK_C0 + n_consts;
        bad |= (t > TOK_REF && !is_const) || (t == TOK_REF && !ref_ok) ? BAD_TOKEN : 0u;
        bad |= is_const ? HAS_CONST : 0u;
        n_in += t == TOK_REF;
        if (t < TOK_X) {
            a -= 1;
            b = b - 1 > 0 ? b - 1 : 0;
            R += 1;
        } else {
            a += 1;
            b += 1;
            R -= 1;
        }
        maxR = R > maxR ? R : maxR;
        last_t = t;
    });
    SegFn f;
    f.a = a;
    f.b = b;
    f.net = R;
    f.minpref = R - maxR;
    f.bad = bad;
    f.n_in = n_in;
    f.left_x = last_t == TOK_X || last_t >= TOK_C0;
    f.left_tok = last_t;
    out[si] = f;
}

// Per chunk, one wave: fold the segment maps in reading order (last segment
// first) to give every segment its start (cnt, P, REFs read before it), and
// combine the validity counters.  The maps compose as
//   (a1, b1) then (a2, b2) = (a1 + a2, max(b1 + a2, b2)),
// so each group of 64 segments is an exclusive scan across the lanes.  The
// minimum running sum before a token, over token order, is
//   S + min_k (minpref_k - suffix_k),  S the chunk's sum and suffix_k the sum
// over segments k.. n-1, which reading order accumulates.
__global__ __launch_bounds__(64) void k_seg_scan(const ChunkSegs* __restrict__ cseg, uint32_t n,
                                                 const SegFn* __restrict__ fn, SegStart* __restrict__ st,
                                                 ChunkStat* __restrict__ cstat, const GLevel* __restrict__ gl)
{
    if (gl) n = gl->n;
    const uint32_t ci = blockIdx.x;
    if (ci >= n) return;
    const int lane = (int)threadIdx.x;
    const ChunkSegs cs = cseg[ci];
    constexpr int32_t NONE = INT32_MIN / 2;
    int32_t c = 0, suf = 0, mmin = INT32_MAX;
    uint32_t P = 0, Ptok = TOK_X, refs = 0, bad = 0;
    for (uint32_t g = 0; g < cs.n_seg; g += 64) {
        const uint32_t r = g + (uint32_t)lane;
        const bool in = r < cs.n_seg;
        const uint32_t k = in ? cs.n_seg - 1 - r : 0;
        SegFn f = {0, NONE, 0, 0, 0, 0, 0, TOK_X};
        if (in) f = fn[cs.first + k];
        int32_t A = f.a, B = f.b, net = f.net;
        uint32_t nin = f.n_in;
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t A0 = __shfl_up(A, d, 64), B0 = __shfl_up(B, d, 64), t0 = __shfl_up(net, d, 64);
            const uint32_t n0 = __shfl_up(nin, d, 64);
            if (lane >= d) {
                B = B0 + A > B ? B0 + A : B;
                A = A0 + A;
                net += t0;
                nin += n0;
            }
        }
        int32_t Ae = __shfl_up(A, 1, 64), Be = __shfl_up(B, 1, 64);
        uint32_t ne = __shfl_up(nin, 1, 64), Pe = __shfl_up(f.left_x, 1, 64), Te = __shfl_up(f.left_tok, 1, 64);
        if (lane == 0) {
            Ae = 0;
            Be = NONE;
            ne = 0;
            Pe = P;
            Te = Ptok;
        }
        if (in) {
            const int32_t cnt = c + Ae > Be ? c + Ae : Be;
            st[cs.first + k] = SegStart{(uint32_t)cnt, Pe, refs + ne, Te};
            const int32_t v = f.minpref - (suf + net);
            mmin = v < mmin ? v : mmin;
            bad |= f.bad;
        }
        const int32_t A63 = __shfl(A, 63, 64), B63 = __shfl(B, 63, 64);
        c = c + A63 > B63 ? c + A63 : B63;
        const uint32_t last = (cs.n_seg - g < 64u ? cs.n_seg - g : 64u) - 1u;
        P = __shfl(f.left_x, (int)last, 64);
        Ptok = __shfl(f.left_tok, (int)last, 64);
        refs += __shfl(nin, 63, 64);
        suf += __shfl(net, 63, 64);
    }
    for (int d = 32; d > 0; d >>= 1) {
        const int32_t o = __shfl_xor(mmin, d, 64);
        mmin = o < mmin ? o : mmin;
        bad |= __shfl_xor(bad, d, 64);
    }
    if (lane == 0) {
        ChunkStat r = {};
        r.net = suf;
        r.minpref = cs.n_seg ? suf + mmin : 0;
        r.bad = bad;
        cstat[ci] = r;
    }
}

// Where a segment's recording goes: one region per segment, by its index,
// each as large as the longest segment of the level needs (kinds: at most 4
// per token plus the boundary's spills and fills, or the chunk end's flushes
// and last codes; fragment tokens: at most 2 per token), so that they never
// overlap whichever tokens the level's segments cover.  Kind regions are
// 8-byte aligned.
__device__ __forceinline__ uint64_t rec_kinds_at(uint32_t si, uint32_t seg_len) { return rec_kinds_stride(seg_len) * si; }
__device__ __forceinline__ uint64_t rec_frags_at(uint32_t si, uint32_t seg_len) { return rec_frags_stride(seg_len) * si; }

// Per segment: its counts; with rk/rf, also the recording of its codes'
// kinds and fragment tokens (set *ovf if a region was too small).
__global__ void k_seg_count(const uint8_t* __restrict__ seq, const SegIn* __restrict__ segs, uint32_t n,
                            const SegStart* __restrict__ st, SegCount* __restrict__ out, uint8_t* __restrict__ rk,
                            uint8_t* __restrict__ rf, SegRec* __restrict__ rec, uint32_t* __restrict__ ovf,
                            uint32_t seg_len, const GLevel* __restrict__ gl)
{
    if (gl) n = gl->n_seg;
    const uint32_t si = blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= n) return;
    const SegIn g = segs[si];
    Sink o{nullptr, 0, nullptr, 0, 0, 0, 0, 0, ~0u, st[si].ref0, nullptr, nullptr, 0, 0, 0, 0, 0, SegRec{}};
    if (rk) {
        o.rk = rk + rec_kinds_at(si, seg_len);
        o.rf = rf + rec_frags_at(si, seg_len);
        o.rk_cap = 4u * g.len + 40u;
        o.rf_cap = 2u * g.len + 16u;
    }
    const uint32_t maxtop = run_segment(seq, g.start, g.len, st[si].cnt, st[si].P, st[si].ptok, g.last != 0, o);
    out[si] = SegCount{o.n_codes, o.n_frag, o.n_out, o.n_in, maxtop, 0};
    if (rk) {
        o.rec_end();
        if (!g.last) o.rec.nfr = o.n_frag;
        rec[si] = o.rec;
        if (o.ovf) atomicOr(ovf, 1u);
    }
}

// Per chunk, one wave: totals for the plan (first launch, no code_begin),
// or each segment's code and fragment positions once the chunk's own bases
// are known (second launch).  Codes run in reading order (last segment
// first); fragments and slots lie in token order, a segment's fragment
// ending where the next one's begins.
__global__ __launch_bounds__(64) void k_seg_chunk(const ChunkSegs* __restrict__ cseg, uint32_t n,
                                                  const SegCount* __restrict__ cnt, ChunkStat* __restrict__ cstat,
                                                  const uint64_t* __restrict__ code_begin,
                                                  const uint64_t* __restrict__ frag_end, uint64_t* __restrict__ seg_code,
                                                  uint64_t* __restrict__ seg_frag, const GLevel* __restrict__ gl)
{
    if (gl) n = gl->n;
    const uint32_t ci = blockIdx.x;
    if (ci >= n) return;
    const int lane = (int)threadIdx.x;
    const ChunkSegs cs = cseg[ci];
    if (!code_begin) {
        uint32_t nc = 0, nf = 0, no = 0, ni = 0, mt = 0;
        for (uint32_t k = (uint32_t)lane; k < cs.n_seg; k += 64) {
            const SegCount q = cnt[cs.first + k];
            nc += q.n_codes;
            nf += q.n_frag;
            no += q.n_out;
            ni += q.n_in;
            mt = q.maxtop > mt ? q.maxtop : mt;
        }
        for (int d = 32; d > 0; d >>= 1) {
            nc += __shfl_xor(nc, d, 64);
            nf += __shfl_xor(nf, d, 64);
            no += __shfl_xor(no, d, 64);
            ni += __shfl_xor(ni, d, 64);
            const uint32_t o = __shfl_xor(mt, d, 64);
            mt = o > mt ? o : mt;
        }
        if (lane == 0) {
            ChunkStat r = cstat[ci];
            r.n_codes = nc;
            r.n_frag = nf;
            r.n_out = no;
            r.n_in = ni;
            r.maxtop = mt;
            r.max_m = mt + 1;
            r.code_out = no;
            r.code_in = ni;
            cstat[ci] = r;
        }
        return;
    }
    const uint64_t cb = code_begin[ci];
    uint64_t at = cb, w = frag_end ? frag_end[ci] : 0;
    for (uint32_t g = 0; g < cs.n_seg; g += 64) {
        const uint32_t r = g + (uint32_t)lane;
        const bool in = r < cs.n_seg;
        const uint32_t k = in ? cs.n_seg - 1 - r : 0;
        uint64_t c = 0, f = 0;
        if (in) {
            c = cnt[cs.first + k].n_codes;
            f = cnt[cs.first + k].n_frag;
        }
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t c0 = __shfl_up(c, d, 64), f0 = __shfl_up(f, d, 64);
            if (lane >= d) {
                c += c0;
                f += f0;
            }
        }
        uint64_t ce = __shfl_up(c, 1, 64), fe = __shfl_up(f, 1, 64);
        if (lane == 0) ce = fe = 0;
        if (in) {
            seg_code[cs.first + k] = cb == ~0ull ? ~0ull : at + ce;
            seg_frag[cs.first + k] = w - fe;
        }
        at += __shfl(c, 63, 64);
        w -= __shfl(f, 63, 64);
    }
}

__device__ __forceinline__ void emit_segment(const uint8_t* __restrict__ seq, const SegIn* __restrict__ segs,
                                             uint32_t si, const SegStart* __restrict__ st,
                                             const uint64_t* __restrict__ seg_code, const uint64_t* __restrict__ seg_frag,
                                             uint8_t* __restrict__ dst, uint32_t* __restrict__ codes)
{
    const SegIn g = segs[si];
    const bool has_codes = codes && seg_code[si] != ~0ull;
    if (!dst && !has_codes) return;
    Sink o{has_codes ? codes : nullptr, has_codes ? seg_code[si] : 0, dst, dst ? seg_frag[si] : 0, 0, 0, 0, 0, ~0u,
           st[si].ref0, nullptr, nullptr, 0, 0, 0, 0, 0, SegRec{}};
    run_segment(seq, g.start, g.len, st[si].cnt, st[si].P, st[si].ptok, g.last != 0, o);
}

__global__ void k_seg_emit(const uint8_t* __restrict__ seq, const SegIn* __restrict__ segs, uint32_t n,
                           const SegStart* __restrict__ st, const uint64_t* __restrict__ seg_code,
                           const uint64_t* __restrict__ seg_frag, uint8_t* __restrict__ dst, uint32_t* __restrict__ codes,
                           const GLevel* __restrict__ gl)
{
    if (gl) {  // the fallback of a recording level only
        if (gl->record && !gl->record_ovf) return;
        n = gl->n_seg;
    }
    const uint32_t si = blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= n) return;
    emit_segment(seq, segs, si, st, seg_code, seg_frag, dst, codes);
}

// A recorded segment's codes and fragment tokens to their places, one wave
// per segment: each kind becomes its handler's offset at the code's final
// position, and a chunk's end gets its runs of slot writes and REF tokens
// back.  Writes outside [0, n_codes) or [0, n_frag), and reads past a
// recording, are skipped and flagged.
//
// The wave also validates the segment's codes as k_seg_check does, 64 codes
// at a time: the window index, slab depth, slot-write count since the last
// FLUSH, REF count and the FLUSH and END states before each code are
// prefix sums (or prefix ORs) of per-code steps, taken with ballots and
// shuffles, carried from batch to batch.  Flags go to err[0] (0x200 for a
// placement fault), the first failing segment to err[1].
__global__ __launch_bounds__(64) void k_seg_place(const SegIn* __restrict__ segs, uint32_t n,
                                                  const SegCount* __restrict__ cnt, const SegRec* __restrict__ rec,
                                                  const SegStart* __restrict__ st,
                                                  const uint64_t* __restrict__ seg_code,
                                                  const uint64_t* __restrict__ seg_frag, const uint8_t* __restrict__ rk,
                                                  const uint8_t* __restrict__ rf, uint32_t* __restrict__ codes,
                                                  uint64_t n_codes, uint8_t* __restrict__ dst, uint64_t n_frag,
                                                  uint32_t slab_entries, uint32_t* __restrict__ err, uint32_t seg_len,
                                                  const GLevel* __restrict__ gl)
{
    if (gl) {  // not when a recording region overflowed (emit and check run instead)
        if (gl->record_ovf) return;
        n = gl->n_seg;
        n_codes = gl->sc;
        n_frag = gl->sf;
        slab_entries = gl->slab_entries;
    }
    const uint32_t lane = threadIdx.x;
    const uint64_t lt = (1ull << lane) - 1ull;  // the lanes before this one
    for (uint32_t si = blockIdx.x; si < n; si += gridDim.x) {
        const SegIn g = segs[si];
        const SegCount q = cnt[si];
        const SegRec r = rec[si];
        const uint32_t cap_k = 4u * g.len + 40u, cap_f = 2u * g.len + 16u;
        uint32_t bad = 0;
        if (codes && seg_code[si] != ~0ull) {
            const uint64_t b = seg_code[si];
            const uint8_t* kp = rk + rec_kinds_at(si, seg_len);
            // the machine's state before the batch
            const SegStart s0 = st[si];
            const uint32_t tv0 = s0.cnt > s0.P ? 1u : 0u, m0 = s0.cnt - tv0 - s0.P;
            int32_t slab = (int32_t)norm_base(m0), idx = (int32_t)(m0 - (uint32_t)slab);
            uint32_t ins = 0, nbm = 0, nbm_flush = 0, outs = 0;
            bool tail = false, ended = false;
            for (uint32_t i0 = 0; i0 < q.n_codes; i0 += 64) {
                const uint32_t i = i0 + lane;
                const bool live = i < q.n_codes;
                // recorded kinds, with the memory run (n1 codes) inserted
                // before recorded kind a1 and the window run (n2) before a2
                uint32_t k = EV_NK;  // none
                if (live) {
                    uint32_t src = i;
                    if (i >= r.a1 && i < r.a1 + r.n1) {
                        k = EV_K_OUTMEM;
                    } else {
                        if (i >= r.a1 + r.n1) src -= r.n1;
                        if (src >= r.a2 && src < r.a2 + r.n2) {
                            k = EV_K_OUTBOT;
                        } else {
                            if (src >= r.a2 + r.n2) src -= r.n2;
                            k = src < cap_k ? kp[src] : 0u;
                            bad |= src < cap_k ? 0u : 0x200u;
                        }
                    }
                    const uint64_t at = b + i;
                    if (at < n_codes)
                        codes[at] = code_value(at, k);
                    else
                        bad |= 0x200u;
                    if (k >= EV_NK) bad |= 1u;
                }
                // the code's kind class
                const bool isF = k == EV_K_FLUSH, isE = k == EV_K_END, isB = k == EV_K_OUTBOT, isM = k == EV_K_OUTMEM;
                const bool isT = k == EV_K_OUTT, isX = k == EV_K_OUTX;
                const bool ops1 = k <= EV_K_OPS3;
                const bool ops2 = k >= EV_K_OPS00 && k <= EV_K_OPS22;
                const bool pref = k >= EV_K_PUSHREF0 && k < EV_K_PUSHREF0 + EV_RING;
                const bool lref = k >= EV_K_LOADREF0 && k < EV_K_LOADREF0 + EV_RING;
                const bool push1 = (k >= EV_K_CH0 && k <= EV_K_CH3) || k == EV_K_PUSHX || pref;
                const bool push2 = k == EV_K_PUSH2X || (k >= EV_K_PXCH0 && k <= EV_K_PXCH3);
                const bool spill = k == EV_K_SPILL, fill = k == EV_K_FILL;
                // FLUSH, END and slot-write states before this code
                const uint64_t bF = __ballot(isF), bE = __ballot(isE), bBM = __ballot(isB || isM);
                const bool tail_b = tail || (bF & lt) != 0;
                const bool ended_b = ended || (bE & lt) != 0;
                uint32_t at_flush = nbm_flush;  // slot writes before the last FLUSH before this code
                if (bF & lt) {
                    const uint32_t l = 63u - (uint32_t)__clzll(bF & lt);
                    at_flush = nbm + (uint32_t)__popcll(bBM & ((1ull << l) - 1ull));
                }
                const int32_t fl = (int32_t)(nbm + (uint32_t)__popcll(bBM & lt) - at_flush);
                // window and slab steps (none after a FLUSH)
                const int32_t need = ops1 ? 1 : (ops2 ? 2 : 0);
                int32_t di = ops1 ? -1 : ops2 ? -2 : push1 ? 1 : (push2 ? 2 : 0);
                di += spill ? -(int32_t)EV_VHALF : (fill ? (int32_t)EV_VHALF : 0);
                int32_t ds = spill ? (int32_t)EV_VHALF : (fill ? -(int32_t)EV_VHALF : 0);
                const bool isref = (pref || lref) && !tail_b;
                if (tail_b) di = ds = 0;
                // inclusive sums over the batch, both in one word: each step
                // biased by 32 into its own 16 bits (at most 64 x 64 each)
                static_assert(EV_VHALF <= 32u, "window steps must fit the 16-bit scan halves");
                uint32_t ps = (uint32_t)(di + 32) | ((uint32_t)(ds + 32) << 16);
                for (uint32_t d = 1; d < 64; d <<= 1) {
                    const uint32_t t = __shfl_up(ps, d, 64);
                    if (lane >= d) ps += t;
                }
                const int32_t si_ = (int32_t)(ps & 0xFFFFu) - 32 * (int32_t)(lane + 1);
                const int32_t ss_ = (int32_t)(ps >> 16) - 32 * (int32_t)(lane + 1);
                const int32_t ib = idx + si_ - di, sb = slab + ss_ - ds;  // before this code
                const int32_t ia = idx + si_, sa = slab + ss_;           // after it
                const uint64_t bR = __ballot(isref);
                const uint32_t ins_b = ins + (uint32_t)__popcll(bR & lt);
                if (live) {
                    if (ended_b) bad |= 4u;
                    uint32_t w = 0;
                    if (tail_b) {
                        // only the chunk's final slot writes and END, none
                        // of which moves the window
                        w |= !(isF || isB || isM || isT || isX || isE) ? 1u : 0u;
                        w |= (isB && fl >= ib) || (isM && fl >= sb) ? 1u : 0u;
                    } else {
                        w |= ib < need ? 1u : 0u;
                        const uint32_t slot = (s0.ref0 + ins_b) & (EV_RING - 1u);
                        if ((pref && k - EV_K_PUSHREF0 != slot) || (lref && k - EV_K_LOADREF0 != slot)) bad |= 1u;
                        w |= (isB && fl >= ib) || (isM && fl >= sb) ? 1u : 0u;
                        w |= spill && ib < (int32_t)EV_VHALF ? 1u : 0u;
                        w |= fill && (sb < (int32_t)EV_VHALF || ib > (int32_t)EV_VHALF - 1) ? 1u : 0u;
                        w |= ia < 0 || ia > (int32_t)EV_VSTACK - 1 || sa < 0 || sa > (int32_t)slab_entries ? 1u : 0u;
                    }
                    if (w) bad |= 2u;
                }
                // carry to the next batch
                idx += __shfl(si_, 63, 64);
                slab += __shfl(ss_, 63, 64);
                ins += (uint32_t)__popcll(bR);
                if (bF) {
                    const uint32_t l = 63u - (uint32_t)__clzll(bF);
                    nbm_flush = nbm + (uint32_t)__popcll(bBM & ((1ull << l) - 1ull));
                }
                nbm += (uint32_t)__popcll(bBM);
                outs += (uint32_t)__popcll(__ballot(isB || isM || isT || isX));
                tail = tail || bF != 0;
                ended = ended || bE != 0;
            }
            if (lane == 0) {
                if (ended != (g.last != 0)) bad |= 4u;
                // a segment hands the next one the window in its boundary position
                if (!g.last && (uint32_t)slab != norm_base((uint32_t)(idx + slab))) bad |= 8u;
                if (outs != q.n_out) bad |= 16u;
                if (ins != q.n_in) bad |= 32u;
            }
        }
        if (dst) {
            const uint64_t w = seg_frag[si];
            const uint8_t* f = rf + rec_frags_at(si, seg_len);
            for (uint32_t i = lane; i < q.n_frag; i += 64) {
                const uint8_t t = i < r.nfr ? (i < cap_f ? f[i] : (uint8_t)0xFF) : (uint8_t)TOK_REF;
                bad |= (i < r.nfr && i >= cap_f) ? 0x200u : 0u;
                if (i < w && w - 1 - i < n_frag)
                    dst[w - 1 - i] = t;
                else
                    bad |= 0x200u;
            }
        }
        if (bad) {
            atomicOr(err, bad);
            atomicMin(err + 1, si);
        }
    }
}

// Every code must name a handler of its own position and only a chunk's
// last segment may (and must) end with END; simulating the codes from the
// segment's start must keep T inside the register window, every read entry
// below it, the slab within its rows, must end with the window in its
// boundary position and must write and read exactly the slots the plan
// gave the segment.  Anything else fails the plan before a code runs.
__global__ void k_seg_check(const uint32_t* __restrict__ codes, const SegIn* __restrict__ segs, uint32_t n,
                            const SegStart* __restrict__ st, const uint64_t* __restrict__ seg_code,
                            const SegCount* __restrict__ cnt, uint32_t slab_entries, uint32_t* __restrict__ err,
                            const GLevel* __restrict__ gl)
{
    if (gl) {  // with emission (the fallback of a recording level)
        if (gl->record && !gl->record_ovf) return;
        n = gl->n_seg;
        slab_entries = gl->slab_entries;
    }
    const uint32_t si = blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= n) return;
    const uint64_t b = seg_code[si];
    if (b == ~0ull) return;
    const SegIn g = segs[si];
    const SegCount sc = cnt[si];
    const uint32_t len = sc.n_codes;
    const uint32_t P = st[si].P, tv = st[si].cnt > P ? 1u : 0u, m0 = st[si].cnt - tv - P, ref0 = st[si].ref0;
    int32_t slab = (int32_t)norm_base(m0), idx = (int32_t)(m0 - (uint32_t)slab), fl = 0;
    uint32_t outs = 0, ins = 0, bad = 0, ended = 0, tail = 0, m = m0;
    // bad: 1 a code names another position or no handler, 2 the window or
    // slab leaves its bounds, 4 END misplaced, 8 boundary position, 16/32
    // slots written/read differ from the plan
    // codes are read in aligned blocks of four, sixteen codes a step with
    // the next sixteen in flight (one lane per segment leaves few waves to
    // hide a load's latency); at most 31 codes past the stream are read,
    // inside the buffer's zero tail
    const uint32_t sk = (uint32_t)(b & 3u), total = sk + len;
    const uint32_t* cb = codes + (b - sk);
    auto ld = [&](uint32_t q) { return *reinterpret_cast<const u32x4*>(cb + q); };
    u32x4 n0 = ld(0), n1 = ld(4), n2 = ld(8), n3 = ld(12);
    for (uint32_t q0 = 0; q0 < total; q0 += 16) {
        const u32x4 c0 = n0, c1 = n1, c2 = n2, c3 = n3;
        n0 = ld(q0 + 16);
        n1 = ld(q0 + 20);
        n2 = ld(q0 + 24);
        n3 = ld(q0 + 28);
#pragma unroll
        for (uint32_t h = 0; h < 4; h++) {
            const uint32_t qb = q0 + 4 * h;
            if (qb >= total) break;
            const u32x4 cur = h == 0 ? c0 : (h == 1 ? c1 : (h == 2 ? c2 : c3));
            const uint32_t jlo = qb ? 0u : sk, jend = total - qb < 4u ? total - qb : 4u;
            for (uint32_t j = jlo; j < jend; j++) {
                const uint32_t i = qb + j - sk;
                const uint32_t v = j >= 2 ? (j == 3 ? cur.w : cur.z) : (j == 1 ? cur.y : cur.x);
                // decode: handler base and stride of this position
                const uint32_t pos = (uint32_t)((b + i) & (EV_CODE_POS - 1));
                const uint32_t sh = 5u + code_tr(pos);  // log2 of the stride
                const uint32_t base = code_base(pos);
                const uint32_t rel = v - base;
                const uint32_t k = rel >> sh;
                if (v < base || (rel & ((1u << sh) - 1u)) || k >= EV_NK) bad |= 1;
                if (ended) bad |= 4;
                if (tail) {
                    // after a FLUSH only the chunk's final slot writes and END may
                    // follow, none of which moves the window (a short path for
                    // the long runs of OUTMEM and OUTBOT)
                    const bool isF = k == EV_K_FLUSH, isB = k == EV_K_OUTBOT, isM = k == EV_K_OUTMEM;
                    const bool isT = k == EV_K_OUTT, isX = k == EV_K_OUTX, isE = k == EV_K_END;
                    const bool w =
                        !(isF || isB || isM || isT || isX || isE) || (isB && fl >= idx) || (isM && fl >= slab);
                    fl = isF ? 0 : fl + ((isB || isM) ? 1 : 0);
                    outs += (isB || isM || isT || isX) ? 1u : 0u;
                    ended |= isE ? 1u : 0u;
                    if (w) bad |= 2;
                    continue;
                }
                // stack actions of the common kinds, with selects
                const bool ops1 = k <= EV_K_OPS3;
                const bool ops2 = k >= EV_K_OPS00 && k <= EV_K_OPS22;
                const bool pref = k >= EV_K_PUSHREF0 && k < EV_K_PUSHREF0 + EV_RING;
                const bool lref = k >= EV_K_LOADREF0 && k < EV_K_LOADREF0 + EV_RING;
                const bool push1 = (k >= EV_K_CH0 && k <= EV_K_CH3) || k == EV_K_PUSHX || pref;
                const int32_t need = ops1 ? 1 : (ops2 ? 2 : 0);
                const bool push2 = k == EV_K_PUSH2X || (k >= EV_K_PXCH0 && k <= EV_K_PXCH3);
                const int32_t d = ops1 ? -1 : ops2 ? -2 : push1 ? 1 : (push2 ? 2 : 0);
                uint32_t w = idx < need ? 1u : 0u;
                // a REF's ring slot follows from its index within the work item
                const uint32_t slot = (ref0 + ins) & (EV_RING - 1);
                if ((pref && k - EV_K_PUSHREF0 != slot) || (lref && k - EV_K_LOADREF0 != slot)) bad |= 1;
                idx += d;
                m += (uint32_t)d;
                ins += (pref || lref) ? 1u : 0u;
                if (k >= EV_K_OUTT && k <= EV_K_OUTMEM) {  // the rare kinds
                    if (k == EV_K_END) ended = 1;
                    if (k == EV_K_FLUSH) {
                        fl = 0;
                        tail = 1;
                    } else if (k == EV_K_OUTBOT) {
                        w |= fl >= idx;
                        fl++;
                    } else if (k == EV_K_OUTMEM) {
                        w |= fl >= slab;
                        fl++;
                    } else if (k == EV_K_SPILL) {
                        w |= idx < (int32_t)EV_VHALF;
                        idx -= EV_VHALF;
                        slab += EV_VHALF;
                    } else if (k == EV_K_FILL) {
                        w |= slab < (int32_t)EV_VHALF || idx > (int32_t)EV_VHALF - 1;
                        idx += EV_VHALF;
                        slab -= EV_VHALF;
                    }
                    outs += (k == EV_K_OUTT || k == EV_K_OUTX || k == EV_K_OUTBOT || k == EV_K_OUTMEM);
                }
                w |= idx < 0 || idx > (int32_t)EV_VSTACK - 1 || slab < 0 || slab > (int32_t)slab_entries;
                if (w) bad |= 2;
            }
        }
    }
    if ((ended != 0) != (g.last != 0)) bad |= 4;
    // a segment hands the next one the window in its boundary position
    if (!g.last && (uint32_t)slab != norm_base((uint32_t)(idx + slab))) bad |= 8;
    if (outs != sc.n_out) bad |= 16;
    if (ins != sc.n_in) bad |= 32;
    if (bad) {
        atomicOr(err, bad);
        atomicMin(err + 1, si);
    }
}

// ------------------------------------------------------------ evaluation

__device__ __forceinline__ EvalChunk load_chunk(const_u4p base, uint32_t i)
{
    const u32x4 a = base[2 * i], b = base[2 * i + 1];
    EvalChunk c;
    c.start = (uint64_t)a.x | ((uint64_t)a.y << 32);
    c.len = a.z;
    c.in_end = a.w;
    c.out_end = b.x;
    c.tree = b.y;
    c.pad0 = b.z;
    c.pad1 = b.w;
    return c;
}


__device__ __forceinline__ uint32_t wave_pop(uint32_t* ctr)
{
    uint32_t v = 0;
    if (threadIdx.x == 0) v = atomicAdd(ctr, 1u);
    return __builtin_amdgcn_readfirstlane(v);
}

// One wave = one work item at a time; lane = test case.  Operand stack:
// top in a register (T), the next D entries in an LDS ring, deeper entries
// spilled to this wave's slab of global memory in groups of 16.
template <int D>
__global__ __launch_bounds__(64) void k_eval(EvalArgs a)
{
    extern __shared__ float ring[];  // D * 64 floats
    const uint32_t lane = threadIdx.x;
    const_u4p tok16 = (const_u4p)(global_u4p)(const void*)a.seq;  // 16-byte token blocks
    const_u4p chunks = (const_u4p)(global_u4p)(const void*)a.chunks;
    const float* __restrict__ in_res = a.in_res;
    float* __restrict__ out_res = a.out_res;
    float* __restrict__ gs = a.gstack + (size_t)blockIdx.x * (size_t)a.gstack_entries * 64u;
    const int32_t N = a.N;

    uint32_t item = wave_pop(a.counter);
    while (item < a.n_items) {
        const uint32_t next = wave_pop(a.counter);
        const uint32_t ci = item / a.n_cb;
        const uint32_t cb = item - ci * a.n_cb;
        const EvalChunk c = load_chunk(chunks, ci);
        const int32_t cs = (int32_t)(cb * 64u + lane);
        const bool act = cs < N;
        const float xv = act ? a.x[cs] : 0.0f;

        uint32_t cnt = 0, P = 0, m = 0, lo = 0;
        uint32_t in_slot = c.in_end, out_slot = c.out_end;
        float T = 0.0f, pv = 0.0f;  // pv: the pending leaf's value (x or a constant) while P

#define RING(e) ring[((e) & (D - 1)) * 64u + lane]
#define STEP(tok)                                                                   \
    do {                                                                            \
        const uint32_t t_ = (tok);                                                  \
        if (t_ == TOK_X || t_ >= TOK_C0) {                                          \
            const float lv_ = t_ == TOK_X ? xv : a.consts[t_ - TOK_C0];             \
            if (P) { RING(m) = T; m++; T = pv; } else { P = 1; }                    \
            pv = lv_;                                                               \
            cnt++;                                                                  \
        } else if (t_ < TOK_X) {                                                    \
            if (cnt < 2) {                                                          \
                if (cnt == 1 && !P) {                                               \
                    out_slot--;                                                     \
                    if (act) out_res[(size_t)out_slot * (size_t)N + cs] = T;        \
                }                                                                   \
                cnt = 0; P = 0; m = 0; lo = 0;                                      \
            } else {                                                                \
                float av, bv;                                                       \
                if (P) { av = pv; bv = T; P = 0; }                                  \
                else { m--; av = T; bv = RING(m); }                                 \
                T = apply_op(t_, av, bv);                                           \
                cnt--;                                                              \
            }                                                                       \
        } else {                                                                    \
            in_slot--;                                                              \
            const float r_ = act ? in_res[(size_t)in_slot * (size_t)N + cs] : 0.0f; \
            if (P) { RING(m) = T; m++; T = pv; P = 0; }                             \
            RING(m) = T; m++; T = r_;                                               \
            cnt++;                                                                  \
        }                                                                           \
    } while (0)

        const uint64_t s = c.start, e = c.start + c.len;
        uint64_t b = (e - 1) & ~(uint64_t)15;
        const uint64_t blo = s & ~(uint64_t)15;
        u32x4 wn = tok16[b >> 4];
        for (;;) {
            const u32x4 w = wn;
            if (b != blo) wn = tok16[(b >> 4) - 1];
            // keep at least 16 resident entries (or all of them) and 16 free
            if (m - lo > (uint32_t)D - 16u) {
                for (uint32_t i = 0; i < 16; i++) gs[(size_t)(lo + i) * 64u + lane] = RING(lo + i);
                lo += 16;
            } else if (lo > 0 && m - lo < 16u) {
                const uint32_t k = lo < 16u ? lo : 16u;
                for (uint32_t i = 0; i < k; i++) {
                    const uint32_t en = lo - 1 - i;
                    RING(en) = gs[(size_t)en * 64u + lane];
                }
                lo -= k;
            }
            if (b >= s && b + 16 <= e) {
                STEP(w.w >> 24); STEP((w.w >> 16) & 255u); STEP((w.w >> 8) & 255u); STEP(w.w & 255u);
                STEP(w.z >> 24); STEP((w.z >> 16) & 255u); STEP((w.z >> 8) & 255u); STEP(w.z & 255u);
                STEP(w.y >> 24); STEP((w.y >> 16) & 255u); STEP((w.y >> 8) & 255u); STEP(w.y & 255u);
                STEP(w.x >> 24); STEP((w.x >> 16) & 255u); STEP((w.x >> 8) & 255u); STEP(w.x & 255u);
            } else {
                const int jhi = (b + 16 <= e) ? 15 : (int)(e - 1 - b);
                const int jlo = (b >= s) ? 0 : (int)(s - b);
                for (int j = jhi; j >= jlo; --j) {
                    const uint32_t word = j >= 12 ? w.w : j >= 8 ? w.z : j >= 4 ? w.y : w.x;
                    STEP((word >> (8 * (j & 3))) & 255u);
                }
            }
            if (b == blo) break;
            b -= 16;
        }
#undef STEP
        // chunk start: every value left becomes a slot, rightmost first
        {
            const uint32_t real = (cnt >= 1 + P) ? cnt - 1 - P : 0u;
            for (uint32_t i = 0; i < real; i++) {
                const uint32_t en = m - real + i;
                const float v = (en >= lo) ? RING(en) : gs[(size_t)en * 64u + lane];
                out_slot--;
                if (act) out_res[(size_t)out_slot * (size_t)N + cs] = v;
            }
            if (cnt >= 1 + P) {
                out_slot--;
                if (act) out_res[(size_t)out_slot * (size_t)N + cs] = T;
            }
            if (P) {
                out_slot--;
                if (act) out_res[(size_t)out_slot * (size_t)N + cs] = pv;
            }
        }
#undef RING
        item = next;
    }
}

template __global__ void k_eval<64>(EvalArgs);
template __global__ void k_eval<128>(EvalArgs);

// ----------------------------------------------------------------- fitness
//
// Table 1: (1/N) sum |GP(x_i) - y_i|; the sum runs over i in ascending order
// in binary32 (Sec. 2.2) and is then divided by (float)N.
__global__ void k_fitness(FitArgs a)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.M) return;
    const uint32_t lv = a.fin[2 * t], slot = a.fin[2 * t + 1];
    if (lv >= a.n_levels || slot >= (a.gl ? a.gl[lv].so : (uint64_t)a.n_out[lv])) {
        // no such slot: a plan inconsistency, reported as NaN, never read
        a.fit[t] = __int_as_float(0x7fc00000);
        if (a.hits) a.hits[t] = 0;
        for (int32_t i = 0; a.per_case && i < a.N; i++) a.per_case[(size_t)t * (size_t)a.N + i] = a.fit[t];
        return;
    }
    const float* r = a.res[lv] + (size_t)slot * (size_t)a.N;
    float s = 0.0f;
    int32_t h = 0;
    for (int32_t i = 0; i < a.N; i++) {
        const float v = r[i];
        const float e = fabsf(v - a.y[i]);
        s = s + e;
        h += e <= 0.01f ? 1 : 0;  // a hit (Sec. 3.2); a NaN error is none
        if (a.per_case) a.per_case[(size_t)t * (size_t)a.N + i] = v;
    }
    a.fit[t] = s / (float)a.N;
    if (a.hits) a.hits[t] = h;
}

// ---------------------------------------------------------------- crossover
//
// Sec. 3.1: the subtree rooted at p ends where the open-slot count started at
// p first drops to zero.  One wave scans 4096 tokens per step: each lane
// takes 64, the wave prefix-sums their net effect, and the first lane whose
// running count reaches zero holds the end.
__global__ __launch_bounds__(64) void k_subtree_end(const uint8_t* __restrict__ buf, const uint64_t* __restrict__ base,
                                                    const uint64_t* __restrict__ pos, uint32_t n,
                                                    uint64_t* __restrict__ end_out)
{
    // One wave per query; it reads 4 KiB per step, 64 aligned bytes per
    // lane (the population buffer carries EV_POP_PAD >= 4 KiB of padding,
    // so the last step stays inside it).
    const uint32_t qi = blockIdx.x;
    if (qi >= n) return;
    const uint32_t lane = threadIdx.x;
    const uint64_t a = base[qi] + pos[qi];
    uint64_t w = a & ~(uint64_t)15;
    int32_t open = 1;  // slots still to fill before the subtree is complete
    for (;;) {
        const uint64_t addr = w + (uint64_t)lane * 64u;
        const u32x4* src = reinterpret_cast<const u32x4*>(buf + addr);
        const u32x4 v0 = src[0], v1 = src[1], v2 = src[2], v3 = src[3];
        auto tok_at = [&](int j) {
            const u32x4& v = j >= 32 ? (j >= 48 ? v3 : v2) : (j >= 16 ? v1 : v0);
            const int i = j & 15;
            const uint32_t word = i >= 8 ? (i >= 12 ? v.w : v.z) : (i >= 4 ? v.y : v.x);
            return (word >> (8 * (i & 3))) & 255u;
        };
        // the lane's net count and its lowest running value
        int32_t c = 0, cmin = 0;
#pragma unroll
        for (int j = 0; j < 64; j++) {
            c += addr + j >= a ? (tok_at(j) < TOK_X ? 1 : -1) : 0;
            cmin = c < cmin ? c : cmin;
        }
        int32_t pre = c;
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t o = __shfl_up(pre, d, 64);
            if ((int)lane >= d) pre += o;
        }
        const int32_t before = pre - c;
        // no lane whose running count reaches zero: the end is further on
        if (!__ballot(open + before + cmin <= 0)) {
            open += __shfl(pre, 63, 64);
            w += 4096;
            continue;
        }
        int32_t hit = -1, cc = 0;
#pragma unroll
        for (int j = 0; j < 64; j++) {
            if (addr + j >= a) {
                cc += tok_at(j) < TOK_X ? 1 : -1;
                if (hit < 0 && open + before + cc == 0) hit = j;
            }
        }
        const uint64_t mask = __ballot(hit >= 0);
        if (mask) {
            const int first = __ffsll((unsigned long long)mask) - 1;
            const int j = __shfl(hit, first, 64);
            if (lane == 0) end_out[qi] = w + (uint64_t)first * 64u + (uint64_t)j - base[qi];
            return;
        }
        open += __shfl(pre, 63, 64);
        w += 4096;
    }
}

// Copy children: mum[0,p) + dad[q, eq] + mum(ep, nm), in 4 KiB pieces of
// each child.  Whole aligned words inside a child are written with one store
// each; the child's first and last partial words byte by byte (a
// neighbouring child may share them).
__device__ __forceinline__ uint8_t child_byte(const uint8_t* __restrict__ mums, const uint8_t* __restrict__ dads,
                                              const XoPlan& x, uint64_t i, uint64_t a, uint64_t b)
{
    if (x.copy_mum || i < a) return mums[x.mum_off + i];
    if (i < b) return dads[x.dad_off + x.q + (i - a)];
    return mums[x.mum_off + x.ep + 1 + (i - b)];
}

// 16 bytes from p (any alignment) in two steps, so that a thread can have
// several in flight: the five aligned words around them (a 16-byte load and
// one more word, read even when p is aligned, so that no branch separates
// the loads), then the shift.  It reads up to 3 bytes before p and 4 after
// p + 15, inside the buffer (its base is aligned) or its padding.
struct Raw16 {
    uint32_t r[5];
    uint32_t sh;
};

__device__ __forceinline__ Raw16 load16_raw(const uint8_t* __restrict__ p)
{
    Raw16 w;
    const uint64_t addr = (uint64_t)(uintptr_t)p;
    const uint32_t* q = reinterpret_cast<const uint32_t*>(addr & ~(uint64_t)3);
    w.sh = (uint32_t)(addr & 3u) * 8u;
    w.r[0] = q[0];
    w.r[1] = q[1];
    w.r[2] = q[2];
    w.r[3] = q[3];
    w.r[4] = q[4];
    return w;
}

__device__ __forceinline__ u32x4 shift16(const Raw16& w)
{
    if (!w.sh) return u32x4{w.r[0], w.r[1], w.r[2], w.r[3]};
    const uint32_t sh = w.sh, up = 32u - sh;
    return u32x4{(w.r[0] >> sh) | (w.r[1] << up), (w.r[1] >> sh) | (w.r[2] << up), (w.r[2] >> sh) | (w.r[3] << up),
                 (w.r[3] >> sh) | (w.r[4] << up)};
}

// Where the child's 16 bytes from i come from: one run of the mum or the
// dad, or (nullptr) bytes from both sides of a cut.  Every population buffer
// has EV_POP_PAD bytes of padding after its last tree, so 20 bytes from any
// tree's start may be read.
__device__ __forceinline__ const uint8_t* word_src(const uint8_t* __restrict__ mums, const uint8_t* __restrict__ dads,
                                                   const XoPlan& x, uint64_t i, uint64_t a, uint64_t b)
{
    if (x.copy_mum || i + 15 < a) return mums + x.mum_off + i;
    if (i >= a && i + 15 < b) return dads + x.dad_off + x.q + (i - a);
    if (i >= b) return mums + x.mum_off + x.ep + 1 + (i - b);
    return nullptr;
}

__device__ __forceinline__ u32x4 cut_word(const uint8_t* __restrict__ mums, const uint8_t* __restrict__ dads,
                                          const XoPlan& x, uint64_t i, uint64_t a, uint64_t b)
{
    uint32_t r[4];
    for (int k = 0; k < 4; k++)
        r[k] = (uint32_t)child_byte(mums, dads, x, i + 4 * k, a, b) |
               ((uint32_t)child_byte(mums, dads, x, i + 4 * k + 1, a, b) << 8) |
               ((uint32_t)child_byte(mums, dads, x, i + 4 * k + 2, a, b) << 16) |
               ((uint32_t)child_byte(mums, dads, x, i + 4 * k + 3, a, b) << 24);
    return u32x4{r[0], r[1], r[2], r[3]};
}

// Bytes [lo, hi) of child x (x.child_off: where its bytes go in dst), by the
// whole block.  The output's aligned 16-byte words inside the range take one
// store each, with four words' loads in flight per thread; the partial
// words at the range's ends are written byte by byte (the neighbouring
// range, of this child or another, writes the rest of them).
__device__ __forceinline__ void xo_copy_range(const uint8_t* __restrict__ mums, const uint8_t* __restrict__ dads,
                                              const XoPlan& x, uint64_t lo, uint64_t hi, uint8_t* __restrict__ dst)
{
    if (hi > x.child_len) hi = x.child_len;
    if (lo >= hi) return;
    const uint64_t a = x.p, b = x.p + (x.eq - x.q + 1);
    const uint64_t o0 = x.child_off + lo, o1 = x.child_off + hi;
    const uint64_t w0 = (o0 + 15) & ~(uint64_t)15, w1 = o1 & ~(uint64_t)15;
    if (w0 >= w1) {
        for (uint64_t o = o0 + threadIdx.x; o < o1; o += blockDim.x)
            dst[o] = child_byte(mums, dads, x, o - x.child_off, a, b);
        return;
    }
    const uint64_t step = 16u * blockDim.x;
    uint64_t w = w0 + 16u * threadIdx.x;
    for (; w + 3 * step < w1; w += 4 * step) {
        const uint8_t* src[4];
        Raw16 raw[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            src[u] = word_src(mums, dads, x, w + u * step - x.child_off, a, b);
            // a word across a cut is put together byte by byte below; its
            // loads here read the mum's first bytes and are not used
            raw[u] = load16_raw(src[u] ? src[u] : mums + x.mum_off);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const u32x4 v = src[u] ? shift16(raw[u]) : cut_word(mums, dads, x, w + u * step - x.child_off, a, b);
            *reinterpret_cast<u32x4*>(dst + w + u * step) = v;
        }
    }
    for (; w < w1; w += step) {
        const uint8_t* sp = word_src(mums, dads, x, w - x.child_off, a, b);
        const u32x4 v = sp ? shift16(load16_raw(sp)) : cut_word(mums, dads, x, w - x.child_off, a, b);
        *reinterpret_cast<u32x4*>(dst + w) = v;
    }
    const uint32_t t = threadIdx.x;
    if (t < w0 - o0) dst[o0 + t] = child_byte(mums, dads, x, o0 + t - x.child_off, a, b);
    if (t < o1 - w1) dst[w1 + t] = child_byte(mums, dads, x, w1 + t - x.child_off, a, b);
}

// Piece `piece` (4 KiB) of child x.
__device__ __forceinline__ void xo_copy_piece(const uint8_t* __restrict__ mums, const uint8_t* __restrict__ dads,
                                              const XoPlan& x, uint64_t piece, uint8_t* __restrict__ dst)
{
    xo_copy_range(mums, dads, x, piece * 4096u, piece * 4096u + 4096u, dst);
}

// The child holding copy piece pb: the j with pf[j] <= pb < pf[j + 1].
__device__ __forceinline__ uint32_t piece_child(const uint64_t* __restrict__ pf, uint32_t n, uint64_t pb)
{
    uint32_t j = 0, hi_j = n;
    while (hi_j - j > 1) {
        const uint32_t mid = (j + hi_j) / 2;
        if (pf[mid] <= pb)
            j = mid;
        else
            hi_j = mid;
    }
    return j;
}

// 4 KiB pieces per block of k_xo_copy (64 KiB: enough bytes per block that
// finding the block's child costs little beside them).
static constexpr uint32_t XO_BLOCK_PIECES = 16;

// Block b copies the 4 KiB pieces [b * XO_BLOCK_PIECES, (b + 1) *
// XO_BLOCK_PIECES) of the children (pf: each child's first piece, pf[n] the
// total), one run of a child's pieces at a time.
__global__ __launch_bounds__(256) void k_xo_copy(const uint8_t* __restrict__ mums, const uint8_t* __restrict__ dads,
                                                 const XoPlan* __restrict__ plan, const uint64_t* __restrict__ off,
                                                 uint32_t n_children, uint8_t* __restrict__ dst,
                                                 uint8_t* __restrict__ pad, uint32_t pad_len,
                                                 const uint32_t* __restrict__ stop)
{
    // with stop (a replayed generation): nothing when the children do not
    // fit their buffer, and the padding goes after their total
    if (stop && *stop) return;
    if (!pad) pad = dst + off[n_children];
    if (blockIdx.x == 0)  // the buffer's padding of 0xFF after the children
        for (uint32_t i = threadIdx.x; i < pad_len; i += blockDim.x) pad[i] = 0xFF;
    const uint64_t* pf = off + n_children + 4;
    const uint64_t pb0 = (uint64_t)blockIdx.x * XO_BLOCK_PIECES;
    const uint64_t total = pf[n_children];
    const uint64_t end = pb0 + XO_BLOCK_PIECES < total ? pb0 + XO_BLOCK_PIECES : total;
    uint64_t pb = pb0;
    uint32_t j = pb < end ? piece_child(pf, n_children, pb) : 0u;
    while (pb < end) {
        while (j + 1 < n_children && pf[j + 1] <= pb) j++;
        const uint64_t pe = pf[j + 1] < end ? pf[j + 1] : end;
        XoPlan x = plan[j];
        x.child_off = off[j];
        xo_copy_range(mums, dads, x, (pb - pf[j]) * 4096u, (pe - pf[j]) * 4096u, dst);
        pb = pe;
    }
}

// A batch of children to places of their own, for a population kept as a
// heap of trees: child k of the batch is plan[idx[k]], written at
// dst + at[k]; pf is the batch's prefix of 4 KiB copy pieces (n + 1
// entries).  Both parents live in `src`.
__global__ void k_xo_copy_at(const uint8_t* __restrict__ src, const XoPlan* __restrict__ plan,
                             const uint32_t* __restrict__ idx, const uint64_t* __restrict__ at,
                             const uint64_t* __restrict__ pf, uint32_t n, uint8_t* __restrict__ dst)
{
    const uint64_t pb = blockIdx.x;
    const uint32_t k = piece_child(pf, n, pb);
    if (pb < pf[k] || pb >= pf[n]) return;
    XoPlan x = plan[idx[k]];
    x.child_off = at[k];
    xo_copy_piece(src, src, x, pb - pf[k], dst);
}

// Per child j: the two subtree queries, (tree start, point) in the mum's
// and the dad's buffer, at j and n + j.
__global__ void k_xo_query(const uint64_t* __restrict__ moff, const uint64_t* __restrict__ doff,
                           const int32_t* __restrict__ mum, const int32_t* __restrict__ dad,
                           const uint64_t* __restrict__ p, const uint64_t* __restrict__ q, uint32_t n,
                           uint64_t* __restrict__ qb, uint64_t* __restrict__ qp)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    qb[j] = moff[mum[j]];
    qp[j] = p[j];
    qb[n + j] = doff[dad[j]];
    qp[n + j] = q[j];
}

// Child plans of Sec. 2.3's crossover, one thread per child: the child's
// length is the mum's with its subtree at p replaced by the dad's subtree
// at q, or the mum's own when that exceeds the size cap.  len[j] gets the
// length, with bit 63 set for a capped child.
__global__ void k_xo_plan(const uint64_t* __restrict__ moff, const uint64_t* __restrict__ doff,
                          const int32_t* __restrict__ mum, const int32_t* __restrict__ dad,
                          const uint64_t* __restrict__ p, const uint64_t* __restrict__ q,
                          const uint64_t* __restrict__ ends, uint32_t n, uint64_t cap, XoPlan* __restrict__ plan,
                          uint64_t* __restrict__ len, const uint64_t* __restrict__ mlen)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    XoPlan x;
    // the mum's start, and its length from the offsets or (a heap of trees)
    // from mlen
    const uint64_t m0 = moff[mum[j]], nm = mlen ? mlen[mum[j]] : moff[mum[j] + 1] - m0;
    x.mum_off = m0;
    x.dad_off = doff[dad[j]];
    x.p = p[j];
    x.ep = ends[j];
    x.q = q[j];
    x.eq = ends[n + j];
    const uint64_t l = nm - (x.ep - x.p + 1) + (x.eq - x.q + 1);
    x.copy_mum = l > cap ? 1u : 0u;
    x.child_len = x.copy_mum ? nm : l;
    x.child_off = 0;
    x.pad = 0;
    plan[j] = x;
    len[j] = x.child_len | ((uint64_t)x.copy_mum << 63);
}

// One block: the children's offsets (exclusive scan of the lengths in
// off[0, n), in place; off[n] the total), off[n + 1] the number capped and
// off[n + 2] the longest child.
__global__ __launch_bounds__(1024) void k_xo_offsets(uint64_t* __restrict__ off, uint32_t n)
{
    __shared__ uint64_t part[1024], partp[1024];
    __shared__ unsigned long long s_max;
    __shared__ uint32_t s_capped;
    const uint32_t t = threadIdx.x;
    if (t == 0) {
        s_max = 0;
        s_capped = 0;
    }
    const uint32_t per = (n + 1023u) / 1024u;
    const uint32_t j0 = t * per < n ? t * per : n, j1 = j0 + per < n ? j0 + per : n;
    uint64_t mine = 0, minep = 0, mx = 0;
    uint32_t capped = 0;
    for (uint32_t j = j0; j < j1; j++) {
        const uint64_t v = off[j], l = v & ~(1ull << 63);
        mine += l;
        minep += (l + 4095) / 4096;  // the child's 4 KiB copy pieces
        mx = l > mx ? l : mx;
        capped += (uint32_t)(v >> 63);
    }
    part[t] = mine;
    partp[t] = minep;
    __syncthreads();
    atomicMax(&s_max, (unsigned long long)mx);
    atomicAdd(&s_capped, capped);
    for (uint32_t d = 1; d < 1024; d <<= 1) {
        const uint64_t v = t >= d ? part[t - d] : 0, vp = t >= d ? partp[t - d] : 0;
        __syncthreads();
        part[t] += v;
        partp[t] += vp;
        __syncthreads();
    }
    uint64_t at = part[t] - mine, atp = partp[t] - minep;
    uint64_t* pf = off + n + 4;  // first copy piece of each child
    for (uint32_t j = j0; j < j1; j++) {
        const uint64_t l = off[j] & ~(1ull << 63);
        off[j] = at;
        pf[j] = atp;
        at += l;
        atp += (l + 4095) / 4096;
    }
    if (t == 1023) {
        off[n] = part[1023];
        pf[n] = partp[1023];
        off[n + 3] = partp[1023];
    }
    if (t == 0) {
        off[n + 1] = s_capped;
        off[n + 2] = s_max;
    }
}

// ------------------------------------------------------ selection (Table 1)

__device__ __forceinline__ void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

// Philox4x32 with 10 rounds (Salmon et al., SC'11).
__device__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        philox_round(c, k0, k1);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ bool fit_better(float a, float b)
{
    if (a != a) return false;
    if (b != b) return true;
    return a < b;
}

__device__ int32_t tournament(const float* __restrict__ fit, uint32_t M, int32_t k, uint32_t k0, uint32_t k1,
                              uint64_t gen, uint32_t child, uint32_t role)
{
    int32_t best = -1;
    uint32_t w[4] = {0, 0, 0, 0};
    for (int32_t c = 0; c < k; c++) {
        if ((c & 3) == 0) {
            w[0] = child;
            w[1] = ((role + 1u) << 8) | (uint32_t)(c >> 2);
            w[2] = (uint32_t)gen;
            w[3] = (uint32_t)(gen >> 32);
            philox10(w, k0, k1);
        }
        const int32_t cand = (int32_t)(((uint64_t)w[c & 3] * (uint64_t)M) >> 32);
        if (best < 0 || fit_better(fit[cand], fit[best])) best = cand;
    }
    return best;
}

__device__ __forceinline__ uint64_t mulhi_u64(uint64_t u, uint64_t n) { return __umul64hi(u, n); }

__global__ void k_select(const float* __restrict__ fit, const uint64_t* __restrict__ off, uint32_t M, int32_t k,
                         uint64_t seed, uint64_t gen, int32_t* __restrict__ mum, int32_t* __restrict__ dad,
                         uint64_t* __restrict__ p, uint64_t* __restrict__ q, const uint64_t* __restrict__ gen_at,
                         const uint64_t* __restrict__ len)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    if (gen_at) gen = *gen_at;  // a replayed generation's number
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int32_t mm = tournament(fit, M, k, k0, k1, gen, j, 0);
    const int32_t dd = tournament(fit, M, k, k0, k1, gen, j, 1);
    uint32_t w[4] = {j, 0x300u, (uint32_t)gen, (uint32_t)(gen >> 32)};
    philox10(w, k0, k1);
    const uint64_t up = ((uint64_t)w[1] << 32) | w[0];
    const uint64_t uq = ((uint64_t)w[3] << 32) | w[2];
    mum[j] = mm;
    dad[j] = dd;
    // sizes: from the offsets, or (a heap of trees) from the lengths
    p[j] = mulhi_u64(up, len ? len[mm] : off[mm + 1] - off[mm]);
    q[j] = mulhi_u64(uq, len ? len[dd] : off[dd + 1] - off[dd]);
}

}  // namespace ev

namespace ev {

// ---------------------------------------------- population statistics (Sec. 4)

__device__ __forceinline__ bool stat_better(float a, uint32_t ia, float b, uint32_t ib)
{
    // lower MAE wins, NaN is worst, and of equals the lower index (the first)
    if (a != a) return (b != b) && ia < ib;
    if (b != b) return true;
    return a < b || (a == b && ia < ib);
}

// One block: the best tree (least fitness, NaN worst, the first of equals),
// how many trees share its fitness bit for bit (or are NaN with a NaN best),
// the sum and count of the finite fitness values and the sizes' sum, minimum
// and maximum.
__global__ __launch_bounds__(1024) void k_pop_stats(const float* __restrict__ fit, const uint64_t* __restrict__ off,
                                                    uint32_t M, PopStatsDev* __restrict__ out)
{
    __shared__ float sf[1024];
    __shared__ uint32_t si[1024];
    __shared__ double sd[1024], ss[1024];
    __shared__ uint64_t smin[1024], smax[1024];
    __shared__ uint32_t sc[1024];
    const uint32_t t = threadIdx.x;
    float bf = __int_as_float(0x7fc00000);
    uint32_t bi = 0xFFFFFFFFu, nfin = 0;
    double sum = 0.0, size_sum = 0.0;
    uint64_t mn = ~0ull, mx = 0;
    for (uint32_t i = t; i < M; i += blockDim.x) {
        const float f = fit[i];
        if (bi == 0xFFFFFFFFu || stat_better(f, i, bf, bi)) {
            bf = f;
            bi = i;
        }
        if (isfinite(f)) {
            sum += (double)f;
            nfin++;
        }
        const uint64_t n = off[i + 1] - off[i];
        size_sum += (double)n;
        mn = n < mn ? n : mn;
        mx = n > mx ? n : mx;
    }
    sf[t] = bf;
    si[t] = bi;
    sd[t] = sum;
    ss[t] = size_sum;
    smin[t] = mn;
    smax[t] = mx;
    sc[t] = nfin;
    __syncthreads();
    for (uint32_t d = 512; d > 0; d >>= 1) {
        if (t < d) {
            if (si[t + d] != 0xFFFFFFFFu && (si[t] == 0xFFFFFFFFu || stat_better(sf[t + d], si[t + d], sf[t], si[t]))) {
                sf[t] = sf[t + d];
                si[t] = si[t + d];
            }
            sd[t] += sd[t + d];
            ss[t] += ss[t + d];
            smin[t] = smin[t + d] < smin[t] ? smin[t + d] : smin[t];
            smax[t] = smax[t + d] > smax[t] ? smax[t + d] : smax[t];
            sc[t] += sc[t + d];
        }
        __syncthreads();
    }
    const float best = sf[0];
    const uint32_t bu = __float_as_uint(best);
    const bool best_nan = best != best;
    uint32_t conv = 0;
    for (uint32_t i = t; i < M; i += blockDim.x) {
        const float f = fit[i];
        conv += (__float_as_uint(f) == bu || (best_nan && f != f)) ? 1u : 0u;
    }
    __syncthreads();
    const uint32_t nfin_all = sc[0];
    __syncthreads();
    sc[t] = conv;
    __syncthreads();
    for (uint32_t d = 512; d > 0; d >>= 1) {
        if (t < d) sc[t] += sc[t + d];
        __syncthreads();
    }
    if (t == 0) *out = PopStatsDev{sd[0], ss[0], smin[0], smax[0], si[0], nfin_all, sc[0], 0};
}

// One wave per tree: the greatest height the right-to-left stack machine
// reaches on it (a leaf pushes, a function pops two and pushes one), which
// bounds the depth pass's stack.  Lane l takes the l-th of 64 consecutive
// parts; the parts combine from the right.
__global__ __launch_bounds__(64) void k_tree_height(const uint8_t* __restrict__ buf, const uint64_t* __restrict__ off,
                                                    uint32_t M, uint32_t* __restrict__ height)
{
    const uint32_t t = blockIdx.x;
    if (t >= M) return;
    const uint32_t lane = threadIdx.x;
    const uint64_t a = off[t], n = off[t + 1] - a;
    const uint64_t per = (n + 63) / 64;
    const uint64_t lo = a + per * lane < a + n ? a + per * lane : a + n;
    const uint64_t hi = lo + per < a + n ? lo + per : a + n;
    int64_t run = 0, best = 0;  // the part's running height from its right end, and its peak
    for (uint64_t k = hi; k-- > lo;) {
        run += buf[k] < TOK_X ? -1 : 1;  // a function pops two and pushes one, a leaf pushes
        best = run > best ? run : best;
    }
    // the height entering each part from its right: sum of the parts to its right
    int64_t suf = run;
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t o = __shfl_down(suf, d, 64);
        if ((int)lane + d < 64) suf += o;
    }
    const int64_t enter = suf - run;
    int64_t peak = enter + best;
    for (int d = 32; d > 0; d >>= 1) {
        const int64_t o = __shfl_xor(peak, d, 64);
        peak = o > peak ? o : peak;
    }
    if (lane == 0) height[t] = (uint32_t)(peak > 0 ? peak : 1);
}

// One thread per tree: its depth (root at 0), right to left: a leaf is a
// subtree of depth 0, a function one more than the deeper of its two
// arguments; the subtrees' depths wait on a stack in [stack + base[t], ...).
__global__ void k_tree_depth(const uint8_t* __restrict__ buf, const uint64_t* __restrict__ off, uint32_t M,
                             const uint64_t* __restrict__ base, uint32_t* __restrict__ stack, uint32_t* __restrict__ depth)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    uint32_t* st = stack + base[t];
    const uint64_t cap = base[t + 1] - base[t];
    uint64_t sp = 0;
    for (uint64_t k = off[t + 1]; k-- > off[t];) {
        if (buf[k] >= TOK_X) {  // a leaf: x or a constant
            if (sp < cap) st[sp] = 0;
            sp++;
        } else {
            const uint32_t x = sp >= 1 && sp - 1 < cap ? st[sp - 1] : 0u;
            const uint32_t y = sp >= 2 && sp - 2 < cap ? st[sp - 2] : 0u;
            sp = sp >= 1 ? sp - 1 : 0;
            if (sp >= 1 && sp - 1 < cap) st[sp - 1] = 1u + (x > y ? x : y);
        }
    }
    depth[t] = cap ? st[0] : 0u;
}

// --------------------------------------------------- register-stack kernel
//
// One wave runs the threaded codes of one work item (lane = test case); see
// gen_interp.py for the handlers.  Chunks whose stack would outgrow the
// register window run on k_eval instead.
__global__ __launch_bounds__(64) void k_run(RunArgs a)
{
    // a level whose code streams failed validation runs none of them (the
    // host reports the failure when it reads the verdict)
    if (a.verdict && *a.verdict) return;
    if (a.gl) {  // a device-made level: its live item count and spill rows
        a.n_items = a.gl->n * a.n_cb;
        a.slab_entries = a.gl->slab_entries;
    }
    const uint32_t lane = threadIdx.x;
    const_u4p chunks = (const_u4p)(global_u4p)(const void*)a.chunks;
    // this wave's spill slab: slab_entries rows of 64 lanes, whose top
    // EV_VHALF rows may sit in LDS (the low 32 bits of a shared address are
    // its LDS offset)
    const uint64_t smem = (uint64_t)(uintptr_t)a.slab + (uint64_t)blockIdx.x * a.slab_entries * 256u;
    __shared__ float spill_lds[EV_VHALF * 64];
    const uint32_t lds = (uint32_t)(uintptr_t)spill_lds + lane * 4u;
    uint32_t item = wave_pop(a.counter);
    while (item < a.n_items) {
        const uint32_t next = wave_pop(a.counter);
        const uint32_t ci = item / a.n_cb;
        const uint32_t cb = item - ci * a.n_cb;
        const u32x4 d = chunks[ci];
        const uint64_t code_begin = (uint64_t)d.x | ((uint64_t)d.y << 32);
        const int32_t cs = (int32_t)(cb * 64u + lane);
        if (cs < a.N) {
            const float xv = a.x[cs];
            const uint32_t lane4 = (uint32_t)cs * 4u;
            const uint64_t cptr = (uint64_t)(uintptr_t)a.codes + (code_begin & ~(uint64_t)31) * 4u;
            const uint32_t j0 = (uint32_t)(code_begin & 31u);
            const uint64_t inp = (uint64_t)(uintptr_t)a.in_res + (uint64_t)d.z * a.rowb;
            const uint64_t outp = (uint64_t)(uintptr_t)a.out_res + (uint64_t)d.w * a.rowb;
            const uint32_t slane = lane * 4u;
            asm volatile(EV_INTERP_ASM
                         :
                         : [x] "v"(xv), [lane4] "v"(lane4), [slane] "v"(slane), [cptr] "s"(cptr), [j0] "s"(j0),
                           [inp] "s"(inp), [outp] "s"(outp), [rowb] "s"(a.rowb), [smem] "s"(smem),
                           [flag] "s"(a.flag), [refs] "s"(a.refs), [lds] "v"(lds)
                         : EV_INTERP_CLOBBERS);
        }
        item = next;
    }
}


}  // namespace ev

namespace ev {

// ------------------------------------------- a generation replayed from a graph
//
// Sec. 2.3's generation with no host wait inside it: the children's plan is
// made level by level on the device.  k_g_init takes the children's
// offsets, k_g_begin lays out a level's work items from the trees still
// active (the host-driven plan's rules: items of C tokens, one item for a
// small tree or a skeleton that did not halve), the structure kernels run on
// the level's live counts, and k_g_end reads the trees' totals, places each
// tree's value or its next range, and checks the totals against the
// capacities the buffers were made for.  Any overflow voids the generation
// (GStatus.poison) and stops every later step of it.

__device__ __forceinline__ void g_poison(GStatus* st, uint32_t bits, uint32_t level)
{
    const uint32_t old = atomicOr(&st->poison, bits);
    if (!old) st->level = level;
}

// The children from their offsets (k_xo_offsets' layout: off[M] the total,
// off[M + 1] the number capped, off[M + 3] the copy pieces): each tree
// active at level 0 over its own bytes.  Block 0 also starts the
// generation's status and clears the interpreter's work counters.
__global__ void k_g_init(const uint64_t* __restrict__ off, uint32_t M, GTree* __restrict__ tr, uint64_t bytes_cap,
                         uint32_t pad_len, uint64_t pieces_cap, GStatus* __restrict__ st,
                         uint32_t* __restrict__ counters, uint32_t n_counters)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0)
        for (uint32_t k = threadIdx.x; k < n_counters; k += blockDim.x) counters[k] = 0;
    if (j == 0) {
        const uint64_t total = off[M], pieces = off[M + 3];
        GStatus s0 = {};
        s0.child_bytes = total;
        s0.capped = off[M + 1];
        if (total + pad_len > bytes_cap || pieces > pieces_cap) s0.poison = G_OVF_BYTES;
        *st = s0;
    }
    if (j < M) tr[j] = GTree{off[j], off[j + 1] - off[j], 0, 0, 1};
}

__device__ __forceinline__ uint64_t g_nseg(uint64_t len, uint32_t seg_len, uint32_t head)
{
    return len <= head ? 1 : 1 + (len - head + seg_len - 1) / seg_len;
}

// One block: the level's trees, in tree order, with their chunks and
// segments numbered by exclusive scans (rounds of 1024 trees, each scanned
// by wave shuffles and the waves' totals on top of the rounds before), and
// their work items' places longest first: each length bucket's first place
// (bucket_start, after the counts of every tree) and each tree's ranks in
// its buckets (taken with shared atomics: the order inside a bucket does
// not matter).
__global__ __launch_bounds__(1024) void k_g_begin(const GTree* __restrict__ tr, uint32_t M, GLevel* __restrict__ gls,
                                                  uint32_t level, const GCap* __restrict__ caps, uint64_t C,
                                                  uint32_t seg_len, uint32_t head, uint32_t record,
                                                  TreeLvl* __restrict__ tl, uint32_t* __restrict__ bucket_start,
                                                  GStatus* __restrict__ st)
{
    __shared__ uint64_t wsum[3][16], carry[3];
    __shared__ unsigned long long s_tok;
    __shared__ uint32_t s_bad, hist[EV_LEN_BUCKETS], rank[EV_LEN_BUCKETS];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const bool live = st->poison == 0 && (level == 0 || gls[level - 1].any != 0);
    if (!live) {
        if (t == 0) {
            GLevel v = {};
            v.record = record;
            gls[level] = v;
        }
        return;
    }
    if (t == 0) {
        carry[0] = carry[1] = carry[2] = 0;
        s_tok = 0;
        s_bad = 0;
    }
    if (t < EV_LEN_BUCKETS) hist[t] = rank[t] = 0;
    __syncthreads();
    for (uint32_t r0 = 0; r0 < M; r0 += 1024) {
        const uint32_t i = r0 + t;
        GTree q = {};
        if (i < M) q = tr[i];
        const bool act = i < M && q.active != 0;
        const uint64_t len = act ? q.rl : 0;
        const bool whole = len <= C || (level > 0 && len * 2 > q.prev_len);
        const uint64_t Ct = whole ? len : C;
        const uint64_t nc = act ? (whole ? 1 : (len + C - 1) / C) : 0;
        const uint64_t last = act ? len - (nc - 1) * Ct : 0;
        const uint64_t ns = act ? (nc - 1) * g_nseg(Ct, seg_len, head) + g_nseg(last, seg_len, head) : 0;
        if (act && whole && len > 0xFFFFFFFFull) atomicOr(&s_bad, 1u);
        if (act) {
            if (nc > 1) atomicAdd(&hist[len_bucket((uint32_t)Ct)], (uint32_t)(nc - 1));
            atomicAdd(&hist[len_bucket((uint32_t)last)], 1u);
        }
        uint64_t a = act ? 1 : 0, b = nc, c = ns, tok = len;
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t a0 = __shfl_up(a, d, 64), b0 = __shfl_up(b, d, 64), c0 = __shfl_up(c, d, 64);
            if (lane >= d) {
                a += a0;
                b += b0;
                c += c0;
            }
        }
        for (int d = 32; d > 0; d >>= 1) tok += __shfl_xor(tok, d, 64);
        if (lane == 63) {
            wsum[0][w] = a;
            wsum[1][w] = b;
            wsum[2][w] = c;
        }
        if (lane == 0 && tok) atomicAdd(&s_tok, (unsigned long long)tok);
        __syncthreads();
        uint64_t ba = carry[0], bb = carry[1], bc = carry[2];
        for (uint32_t k = 0; k < w; k++) {
            ba += wsum[0][k];
            bb += wsum[1][k];
            bc += wsum[2][k];
        }
        if (act) {
            TreeLvl v;
            v.start = q.rs;
            v.len = len;
            v.chunk_first = (uint32_t)(bb + b - nc);
            v.n_chunks = (uint32_t)nc;
            v.seg_first = (uint32_t)(bc + c - ns);
            v.C = (uint32_t)Ct;
            v.tree = i;
            v.ref_base = q.ref_base;
            v.rank_full = v.rank_last = 0;  // below
            tl[(uint32_t)(ba + a - 1)] = v;
        }
        __syncthreads();  // every thread has read carry and the waves' totals
        if (t == 1023) {
            carry[0] = ba + a;
            carry[1] = bb + b;
            carry[2] = bc + c;
        }
        __syncthreads();
    }
    const uint32_t nt = (uint32_t)carry[0];
    const GCap cp = caps[level];
    const bool over = s_bad || carry[1] > cp.n || carry[2] > cp.n_seg;
    if (t == 0) {
        GLevel v = {};
        v.record = record;
        v.tokens = s_tok;
        v.prev_out = level ? gls[level - 1].so : 0;
        if (over) {
            g_poison(st, G_OVF_ITEMS, level);
        } else {
            v.nt = nt;
            v.n = (uint32_t)carry[1];
            v.n_seg = (uint32_t)carry[2];
            // each bucket's first place
            for (uint32_t k = 0, acc = 0; k < EV_LEN_BUCKETS; k++) {
                bucket_start[k] = acc;
                acc += hist[k];
            }
        }
        gls[level] = v;
    }
    if (over) return;
    // the trees' ranks in their buckets (their records were written above
    // by this block)
    __syncthreads();
    for (uint32_t i = t; i < nt; i += blockDim.x) {
        TreeLvl v = tl[i];
        const uint32_t nc = v.n_chunks;
        const uint32_t last = (uint32_t)(v.len - (uint64_t)(nc - 1) * v.C);
        v.rank_full = nc > 1 ? atomicAdd(&rank[len_bucket(v.C)], nc - 1) : 0u;
        v.rank_last = atomicAdd(&rank[len_bucket(last)], 1u);
        tl[i] = v;
    }
}

// One block: the trees' bases over the level's chunks, in the level's order
// (exclusive sums of their slots, fragment tokens and codes, stored by tree
// id with the tree's chunk range and bucket ranks, as k_plan_bases makes
// them), the trees that end here (their value's level and slot) and the
// next level's ranges; the level's totals are checked against the
// capacities.
__global__ __launch_bounds__(1024) void k_g_end(GTree* __restrict__ tr, GLevel* __restrict__ gls, uint32_t level,
                                                const GCap* __restrict__ caps, uint32_t n_levels,
                                                const TreeLvl* __restrict__ tl, const TreeSum* __restrict__ sum,
                                                TreeBase* __restrict__ tb, uint32_t* __restrict__ fin,
                                                GStatus* __restrict__ st)
{
    __shared__ uint64_t wo[16], wf[16], wc[16], carry[3];
    __shared__ uint32_t s_top, s_bad, s_any;
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const uint32_t nt = gls[level].nt;
    if (nt == 0) return;  // no work at this level, or voided
    if (t == 0) {
        carry[0] = carry[1] = carry[2] = 0;
        s_top = s_bad = s_any = 0;
    }
    __syncthreads();
    for (uint32_t r0 = 0; r0 < nt; r0 += 1024) {
        const uint32_t i = r0 + t;
        TreeSum q = {};
        if (i < nt) q = sum[i];
        const uint64_t o = q.n_out, f = q.n_frag, c = q.n_codes;
        uint64_t so = o, sf = f, sc = c;  // inclusive sums within the wave
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t ao = __shfl_up(so, d), af = __shfl_up(sf, d), ac = __shfl_up(sc, d);
            if (lane >= d) {
                so += ao;
                sf += af;
                sc += ac;
            }
        }
        if (lane == 63) {
            wo[w] = so;
            wf[w] = sf;
            wc[w] = sc;
        }
        __syncthreads();
        uint64_t bo = carry[0], bf = carry[1], bc = carry[2];
        for (uint32_t k = 0; k < w; k++) {
            bo += wo[k];
            bf += wf[k];
            bc += wc[k];
        }
        if (i < nt) {
            const TreeLvl v = tl[i];
            const uint32_t tree = v.tree;
            const TreeBase b{bo + so - o, bf + sf - f, bc + sc - c, v.chunk_first, v.n_chunks, v.rank_full, v.rank_last};
            tb[tree] = b;
            uint32_t bad = 0;
            if (q.bad & 1u) bad |= G_MALFORMED;
            if (q.bad & 2u) bad |= G_INCONSISTENT;
            if (q.bad & HAS_CONST) bad |= G_CONSTS;
            if (bad) atomicOr(&s_bad, bad);
            atomicMax(&s_top, q.maxtop);
            if (q.n_frag == 1) {
                fin[2 * (size_t)tree] = level;
                fin[2 * (size_t)tree + 1] = (uint32_t)(b.out + q.n_out - 1);
                tr[tree].active = 0;
            } else {
                s_any = 1;
                GTree r = tr[tree];
                r.prev_len = r.rl;
                r.rs = b.frag;
                r.rl = q.n_frag;
                r.ref_base = (uint32_t)b.out;
                tr[tree] = r;
            }
        }
        __syncthreads();  // every thread has read carry and the waves' totals
        if (t == 1023) {
            carry[0] = bo + so;
            carry[1] = bf + sf;
            carry[2] = bc + sc;
        }
        __syncthreads();
    }
    if (t == 0) {
        const GCap cp = caps[level];
        GLevel& g = gls[level];
        uint32_t bad = s_bad;
        const uint32_t top = s_top;
        const uint64_t so = carry[0], sf = carry[1], sc = carry[2];
        // the host-driven plan's rule: spill rows when the stack reaches
        // past the window's re-centring point
        const uint32_t slab = top + 1 > EV_VSTACK_ENTRIES - EV_VHALF / 2 ? top + EV_VHALF : 0u;
        if (so > cp.so || sf > cp.sf || sc > cp.sc || so > 0xFFFFFFF0ull) bad |= G_OVF_SIZES;
        if (slab > cp.slab) bad |= G_OVF_SLAB;
        if (s_any && level + 1 >= n_levels) bad |= G_OVF_LEVELS;
        if (g.record && g.record_ovf) bad |= G_OVF_ITEMS;  // a recording region was too small
        if (bad) {
            g_poison(st, bad, level);
            g.nt = g.n = g.n_seg = 0;
            g.any = 0;
        } else {
            g.so = so;
            g.sf = sf;
            g.sc = sc;
            g.slab_entries = slab;
            g.any = s_any;
            st->levels = level + 1;
        }
    }
}

// The generation's verdict: code streams that failed validation void it
// too.  The status, the levels' counts and the children's fitness go to
// pinned host memory (read after the replay), and the generation number
// steps on.
__global__ __launch_bounds__(256) void k_g_finish(GStatus* __restrict__ st, const GLevel* __restrict__ gls,
                                                  uint32_t n_levels, const uint32_t* __restrict__ err,
                                                  const float* __restrict__ fit, uint32_t M,
                                                  uint64_t* __restrict__ gen_at, GStatus* __restrict__ h_st,
                                                  GLevel* __restrict__ h_levels, float* __restrict__ h_fit)
{
    const uint32_t t = threadIdx.x;
    if (t == 0) {
        const uint32_t used = st->levels;
        for (uint32_t l = 0; l < used && l < n_levels; l++)
            if (err[2 * l]) {
                g_poison(st, G_INVALID_CODES, l);
                break;
            }
        *h_st = *st;
        *gen_at += 1;
    }
    for (uint32_t l = t; l < n_levels; l += blockDim.x) h_levels[l] = gls[l];
    for (uint32_t j = t; j < M; j += blockDim.x) h_fit[j] = fit[j];
}

// Several plan levels in one persistent launch (Sec. 2.2's subtrees
// combined level by level, without a barrier between levels): the queue
// holds runs of the levels' work items, and an item of level l of tree t
// waits until every item of level l - 1 of tree t has finished.  Every item
// it waits for sits earlier in the queue.  A wave holds its current item
// and the next one it took, and starts that one only after finishing the
// current; so the earliest unfinished item is some wave's current item,
// everything it waits for is done, and the wait ends.  Slot rows cross compute
// units (and the XCDs' separate L2s) without any cache maintenance: every
// slot-row load and store of the interpreter is made at device scope (sc1),
// the item's stores have completed (the interpreter's last vmcnt wait)
// before its done count is raised, and a waiting item issues its row loads
// only after it has read the count it waits for.  Write-back or invalidate
// of a whole L2 would also reach the kernels of other streams.
__global__ __launch_bounds__(64) void k_run_chain(ChainArgs a)
{
    const uint32_t lane = threadIdx.x;
    const uint64_t smem = (uint64_t)(uintptr_t)a.slab + (uint64_t)blockIdx.x * a.slab_entries * 256u;
    __shared__ float spill_lds[EV_VHALF * 64];  // the slab's top rows (as in k_run)
    const uint32_t lds = (uint32_t)(uintptr_t)spill_lds + lane * 4u;
    uint32_t item = wave_pop(a.counter);
    while (item < a.total) {
        const uint32_t next = wave_pop(a.counter);
        uint32_t l = 0;
        while (l + 1 < a.n_levels && item >= a.levels[l + 1].first) l++;
        const RunLevel L = a.levels[l];
        const uint32_t local = item - L.first;
        const uint32_t ci = local / a.n_cb;
        const uint32_t cb = local - ci * a.n_cb;
        const uint32_t tree = (uint32_t)__builtin_amdgcn_readfirstlane(L.item_tree[ci]);
        const uint32_t pl = L.plevel;
        if (pl > 0) {
            const uint32_t* dp = a.done + (size_t)(pl - 1) * a.M + tree;
            const uint32_t want = a.need[(size_t)(pl - 1) * a.M + tree] * a.n_cb;
            while (__hip_atomic_load(dp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want)
                __builtin_amdgcn_s_sleep(4);
        }
        // a level whose code streams failed validation runs none of them
        // (its items still count as done)
        if (!(L.verdict && *L.verdict)) {
            const_u4p chunks = (const_u4p)(global_u4p)(const void*)L.chunks;
            const u32x4 d = chunks[ci];
            const uint64_t code_begin = (uint64_t)d.x | ((uint64_t)d.y << 32);
            const int32_t cs = (int32_t)(cb * 64u + lane);
            if (cs < a.N) {
                // wave-uniform operands in scalar registers (readfirstlane
                // returns an int: each half goes through uint32_t, so that
                // the low word is not sign-extended into the high one)
                auto uni = [](uint64_t v) {
                    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
                    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
                    return (uint64_t)lo | ((uint64_t)hi << 32);
                };
                const float xv = a.x[cs];
                const uint32_t lane4 = (uint32_t)cs * 4u;
                const uint64_t cptr = uni((uint64_t)(uintptr_t)L.codes + (code_begin & ~(uint64_t)31) * 4u);
                const uint32_t j0 = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(code_begin & 31u));
                const uint64_t inp = uni((uint64_t)(uintptr_t)L.in_res + (uint64_t)d.z * a.rowb);
                const uint64_t outp = uni((uint64_t)(uintptr_t)L.out_res + (uint64_t)d.w * a.rowb);
                const uint32_t slane = lane * 4u;
                const uint32_t refs = (uint32_t)__builtin_amdgcn_readfirstlane(L.refs);
                // a skeleton item (it reads slots) is on its tree's critical
                // path: its wave issues ahead of the level-0 waves sharing
                // its SIMD
                if (refs) __builtin_amdgcn_s_setprio(3);
                asm volatile(EV_INTERP_ASM_COH
                             :
                             : [x] "v"(xv), [lane4] "v"(lane4), [slane] "v"(slane), [cptr] "s"(cptr), [j0] "s"(j0),
                               [inp] "s"(inp), [outp] "s"(outp), [rowb] "s"(a.rowb), [smem] "s"(smem),
                               [flag] "s"(a.flag), [refs] "s"(refs), [lds] "v"(lds)
                             : EV_INTERP_CLOBBERS, "memory");
                if (refs) __builtin_amdgcn_s_setprio(0);
            }
        }
        if (lane == 0) __hip_atomic_fetch_add(a.done + (size_t)pl * a.M + tree, 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        item = next;
    }
}

}  // namespace ev

// ------------------------------------------------------------ launchers

namespace ev {

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(cdiv(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3(cdiv(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t a = (uint64_t)(uintptr_t)dst | (uint64_t)(uintptr_t)src | n;
    const uint32_t w = (a & 15) == 0 ? 16u : ((a & 3) == 0 ? 4u : 1u);
    hipLaunchKernelGGL(k_copy, dim3(cdiv(n / w, 256)), dim3(256), 0, s, (uint8_t*)dst, (const uint8_t*)src, n, w);
    return hipGetLastError();
}

hipError_t launch_seg_build(const ChunkIn* ch, const ChunkSegs* cg, uint32_t n, uint32_t seg_len, uint32_t head,
                            SegIn* seg, hipStream_t s, const GLevel* gl)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_build, dim3(n), dim3(64), 0, s, ch, cg, n, seg_len, head, seg, gl);
    return hipGetLastError();
}

hipError_t launch_plan_chunks(const TreeLvl* trees, uint32_t n_trees, uint32_t seg_len, uint32_t head, ChunkIn* ch,
                              ChunkSegs* cg, uint32_t* err_init, uint32_t n_err, hipStream_t s, const GLevel* gl)
{
    if (n_trees == 0) return hipSuccess;
    hipLaunchKernelGGL(k_plan_chunks, dim3(n_trees), dim3(64), 0, s, trees, n_trees, seg_len, head, ch, cg, err_init,
                       n_err, gl);
    return hipGetLastError();
}

hipError_t launch_plan_bases(const TreeLvl* trees, uint32_t n_trees, const TreeSum* sum, TreeBase* base, hipStream_t s,
                             const GLevel* gl)
{
    if (n_trees == 0) return hipSuccess;
    hipLaunchKernelGGL(k_plan_bases, dim3(1), dim3(1024), 0, s, trees, n_trees, sum, base, gl);
    return hipGetLastError();
}

hipError_t launch_plan_trees(const TreeLvl* trees, uint32_t n_trees, const ChunkStat* cs, uint32_t level,
                             uint64_t prev_out, uint64_t* code_loc, uint64_t* out_loc, uint64_t* frag_loc,
                             uint32_t* in_end, TreeSum* sum, hipStream_t s, const GLevel* gl)
{
    if (n_trees == 0) return hipSuccess;
    hipLaunchKernelGGL(k_plan_trees, dim3(n_trees), dim3(64), 0, s, trees, n_trees, cs, level, prev_out, code_loc,
                       out_loc, frag_loc, in_end, sum, gl);
    return hipGetLastError();
}

hipError_t launch_plan_items(const ChunkIn* ch, uint32_t n, const TreeBase* base, const uint64_t* code_loc,
                             const uint64_t* out_loc, const uint64_t* frag_loc, const uint32_t* in_end,
                             const uint32_t* cursor,
                             uint64_t* code_begin, uint64_t* frag_end, RunChunk* run, EvalChunk* slow,
                             uint32_t* code_tail, uint8_t* frag_tail, hipStream_t s, const GLevel* gl,
                             uint32_t* item_tree)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_plan_items, dim3(cdiv(n, 256)), dim3(256), 0, s, ch, n, base, code_loc, out_loc, frag_loc,
                       in_end, cursor, code_begin, frag_end, run, slow, code_tail, frag_tail, gl, item_tree);
    return hipGetLastError();
}

hipError_t launch_reuse_runs(const XoPlan* plan, const int32_t* mum, const L0Tree* trees, const ChunkIn* mum_ch,
                             uint32_t n, ReuseRun* out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reuse_runs, dim3(cdiv(n, 256)), dim3(256), 0, s, plan, mum, trees, mum_ch, n, out);
    return hipGetLastError();
}

hipError_t launch_reuse_chunks(const TreeReuse* trees, uint32_t n_trees, const ChunkIn* mum_ch, uint32_t seg_len,
                               uint32_t head, ChunkIn* ch, ChunkSegs* cg, uint32_t* src, uint32_t* err_init,
                               uint32_t n_err, hipStream_t s)
{
    if (n_trees == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reuse_chunks, dim3(n_trees), dim3(64), 0, s, trees, n_trees, mum_ch, seg_len, head, ch, cg,
                       src, err_init, n_err);
    return hipGetLastError();
}

hipError_t launch_reuse_stats(const uint32_t* src, uint32_t n, const ChunkStat* mum_stat, ChunkStat* cstat,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reuse_stats, dim3(cdiv(n, 256)), dim3(256), 0, s, src, n, mum_stat, cstat);
    return hipGetLastError();
}

hipError_t launch_reuse_copy(const uint32_t* src, uint32_t n, const ChunkStat* cstat, const uint64_t* code_begin,
                             const uint64_t* frag_end, const uint64_t* mum_code, const uint64_t* mum_frag,
                             const uint32_t* mum_codes, const uint8_t* mum_skel, uint32_t* codes, uint8_t* skel,
                             hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reuse_copy, dim3(n), dim3(256), 0, s, src, n, cstat, code_begin, frag_end, mum_code, mum_frag,
                       mum_codes, mum_skel, codes, skel);
    return hipGetLastError();
}

hipError_t launch_pop_stats(const float* fit, const uint64_t* off, uint32_t M, PopStatsDev* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_pop_stats, dim3(1), dim3(1024), 0, s, fit, off, M, out);
    return hipGetLastError();
}

hipError_t launch_tree_height(const uint8_t* buf, const uint64_t* off, uint32_t M, uint32_t* height, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tree_height, dim3(M), dim3(64), 0, s, buf, off, M, height);
    return hipGetLastError();
}

hipError_t launch_tree_depth(const uint8_t* buf, const uint64_t* off, uint32_t M, const uint64_t* base, uint32_t* stack,
                             uint32_t* depth, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tree_depth, dim3(cdiv(M, 64)), dim3(64), 0, s, buf, off, M, base, stack, depth);
    return hipGetLastError();
}

hipError_t launch_seg_fn(const uint8_t* seq, const SegIn* segs, uint32_t n, SegFn* out, uint32_t ref_ok,
                         uint32_t n_consts, hipStream_t s, const GLevel* gl)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_fn, dim3(cdiv(n, 64)), dim3(64), 0, s, seq, segs, n, out, ref_ok, n_consts, gl);
    return hipGetLastError();
}

hipError_t launch_seg_scan(const ChunkSegs* cseg, uint32_t n, const SegFn* fn, SegStart* st, ChunkStat* cstat,
                           hipStream_t s, const GLevel* gl)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_scan, dim3(n), dim3(64), 0, s, cseg, n, fn, st, cstat, gl);
    return hipGetLastError();
}

hipError_t launch_seg_count(const uint8_t* seq, const SegIn* segs, uint32_t n, const SegStart* st, SegCount* out,
                            uint8_t* rk, uint8_t* rf, SegRec* rec, uint32_t* ovf, uint32_t seg_len, hipStream_t s,
                            const GLevel* gl)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_count, dim3(cdiv(n, 64)), dim3(64), 0, s, seq, segs, n, st, out, rk, rf, rec, ovf,
                       seg_len, gl);
    return hipGetLastError();
}

hipError_t launch_seg_place(const SegIn* segs, uint32_t n, const SegCount* cnt, const SegRec* rec, const SegStart* st,
                            const uint64_t* seg_code, const uint64_t* seg_frag, const uint8_t* rk, const uint8_t* rf,
                            uint32_t* codes, uint64_t n_codes, uint8_t* dst, uint64_t n_frag, uint32_t slab_entries,
                            uint32_t* err, uint32_t seg_len, hipStream_t s, const GLevel* gl)
{
    if (n == 0) return hipSuccess;
    const uint32_t grid = n < 16384u ? n : 16384u;
    hipLaunchKernelGGL(k_seg_place, dim3(grid), dim3(64), 0, s, segs, n, cnt, rec, st, seg_code, seg_frag, rk, rf,
                       codes, n_codes, dst, n_frag, slab_entries, err, seg_len, gl);
    return hipGetLastError();
}

hipError_t launch_seg_chunk(const ChunkSegs* cseg, uint32_t n, const SegCount* cnt, ChunkStat* cstat,
                            const uint64_t* code_begin, const uint64_t* frag_end, uint64_t* seg_code, uint64_t* seg_frag,
                            hipStream_t s, const GLevel* gl)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_chunk, dim3(n), dim3(64), 0, s, cseg, n, cnt, cstat, code_begin, frag_end,
                       seg_code, seg_frag, gl);
    return hipGetLastError();
}

hipError_t launch_seg_emit(const uint8_t* seq, const SegIn* segs, uint32_t n, const SegStart* st, const uint64_t* seg_code,
                           const uint64_t* seg_frag, uint8_t* dst, uint32_t* codes, hipStream_t s, const GLevel* gl)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_emit, dim3(cdiv(n, 64)), dim3(64), 0, s, seq, segs, n, st, seg_code, seg_frag, dst, codes,
                       gl);
    return hipGetLastError();
}

hipError_t launch_seg_check(const uint32_t* codes, const SegIn* segs, uint32_t n, const SegStart* st,
                            const uint64_t* seg_code, const SegCount* cnt, uint32_t slab_entries, uint32_t* err,
                            hipStream_t s, const GLevel* gl)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_check, dim3(cdiv(n, 64)), dim3(64), 0, s, codes, segs, n, st, seg_code, cnt, slab_entries,
                       err, gl);
    return hipGetLastError();
}

size_t eval_lds_bytes(int D) { return (size_t)D * 64u * sizeof(float); }

hipError_t eval_occupancy(int D, int* blocks_per_cu)
{
    if (D == 128)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(&k_eval<128>), 64,
                                                            eval_lds_bytes(D));
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(&k_eval<64>), 64,
                                                        eval_lds_bytes(64));
}

hipError_t launch_eval(int D, const EvalArgs& a, uint32_t grid, hipStream_t s)
{
    if (a.n_items == 0 || grid == 0) return hipSuccess;
    if (D == 128)
        hipLaunchKernelGGL(k_eval<128>, dim3(grid), dim3(64), eval_lds_bytes(128), s, a);
    else
        hipLaunchKernelGGL(k_eval<64>, dim3(grid), dim3(64), eval_lds_bytes(64), s, a);
    return hipGetLastError();
}

hipError_t run_occupancy(int* blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(&k_run), 64, 0);
}

hipError_t chain_occupancy(int* blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(&k_run_chain), 64,
                                                        0);
}

hipError_t launch_run_chain(const ChainArgs& a, uint32_t grid, hipStream_t s)
{
    if (a.total == 0 || grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_run_chain, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_run(const RunArgs& a, uint32_t grid, hipStream_t s)
{
    if (a.n_items == 0 || grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_run, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}



hipError_t launch_fitness(const FitArgs& a, hipStream_t s)
{
    if (a.M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fitness, dim3(cdiv(a.M, 64)), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_subtree_end(const uint8_t* buf, const uint64_t* base, const uint64_t* pos, uint32_t n,
                              uint64_t* end_out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_subtree_end, dim3(n), dim3(64), 0, s, buf, base, pos, n, end_out);
    return hipGetLastError();
}

hipError_t launch_xo_copy(const uint8_t* mums, const uint8_t* dads, const XoPlan* plan, const uint64_t* off,
                          uint32_t n, uint64_t pieces, uint8_t* dst, uint8_t* pad, uint32_t pad_len, hipStream_t s,
                          const uint32_t* stop)
{
    if (n == 0 || pieces == 0) return launch_fill_u8(pad, pad_len, 0xFF, s);
    if (pieces > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_xo_copy, dim3(cdiv(pieces, XO_BLOCK_PIECES)), dim3(256), 0, s, mums, dads, plan, off, n, dst,
                       pad, pad_len, stop);
    return hipGetLastError();
}

hipError_t launch_xo_copy_at(const uint8_t* src, const XoPlan* plan, const uint32_t* idx, const uint64_t* at,
                            const uint64_t* pf, uint32_t n, uint64_t pieces, uint8_t* dst, hipStream_t s)
{
    if (n == 0 || pieces == 0) return hipSuccess;
    if (pieces > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_xo_copy_at, dim3((uint32_t)pieces), dim3(256), 0, s, src, plan, idx, at, pf, n, dst);
    return hipGetLastError();
}

hipError_t launch_xo_query(const uint64_t* moff, const uint64_t* doff, const int32_t* mum, const int32_t* dad,
                           const uint64_t* p, const uint64_t* q, uint32_t n, uint64_t* qb, uint64_t* qp, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_xo_query, dim3(cdiv(n, 256)), dim3(256), 0, s, moff, doff, mum, dad, p, q, n, qb, qp);
    return hipGetLastError();
}

hipError_t launch_xo_plan(const uint64_t* moff, const uint64_t* doff, const int32_t* mum, const int32_t* dad,
                          const uint64_t* p, const uint64_t* q, const uint64_t* ends, uint32_t n, uint64_t cap,
                          XoPlan* plan, uint64_t* off, hipStream_t s, const uint64_t* mlen)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_xo_plan, dim3(cdiv(n, 256)), dim3(256), 0, s, moff, doff, mum, dad, p, q, ends, n, cap, plan, off,
                       mlen);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_xo_offsets, dim3(1), dim3(1024), 0, s, off, n);
    return hipGetLastError();
}

hipError_t launch_select(const float* fit, const uint64_t* off, uint32_t M, int32_t k, uint64_t seed, uint64_t gen,
                         int32_t* mum, int32_t* dad, uint64_t* p, uint64_t* q, hipStream_t s, const uint64_t* gen_at,
                         const uint64_t* len)
{
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3(cdiv(M, 64)), dim3(64), 0, s, fit, off, M, k, seed, gen, mum, dad, p, q, gen_at,
                       len);
    return hipGetLastError();
}


hipError_t launch_g_init(const uint64_t* off, uint32_t M, GTree* tr, uint64_t bytes_cap, uint32_t pad_len,
                         uint64_t pieces_cap, GStatus* st, uint32_t* counters, uint32_t n_counters, hipStream_t s)
{
    hipLaunchKernelGGL(k_g_init, dim3(cdiv(M ? M : 1, 256)), dim3(256), 0, s, off, M, tr, bytes_cap, pad_len,
                       pieces_cap, st, counters, n_counters);
    return hipGetLastError();
}

hipError_t launch_g_begin(const GTree* tr, uint32_t M, GLevel* gls, uint32_t level, const GCap* caps, uint64_t C,
                          uint32_t seg_len, uint32_t head, uint32_t record, TreeLvl* tl, uint32_t* bucket_start,
                          GStatus* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_g_begin, dim3(1), dim3(1024), 0, s, tr, M, gls, level, caps, C, seg_len, head, record, tl,
                       bucket_start, st);
    return hipGetLastError();
}

hipError_t launch_g_end(GTree* tr, GLevel* gls, uint32_t level, const GCap* caps, uint32_t n_levels, const TreeLvl* tl,
                        const TreeSum* sum, TreeBase* tb, uint32_t* fin, GStatus* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_g_end, dim3(1), dim3(1024), 0, s, tr, gls, level, caps, n_levels, tl, sum, tb, fin, st);
    return hipGetLastError();
}

hipError_t launch_g_finish(GStatus* st, const GLevel* gls, uint32_t n_levels, const uint32_t* err, const float* fit,
                           uint32_t M, uint64_t* gen_at, GStatus* h_st, GLevel* h_levels, float* h_fit, hipStream_t s)
{
    hipLaunchKernelGGL(k_g_finish, dim3(1), dim3(256), 0, s, st, gls, n_levels, err, fit, M, gen_at, h_st, h_levels,
                       h_fit);
    return hipGetLastError();
}

}  // namespace ev
