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

// -------------------------------------------- structure passes (integer)
//
// The stack machine of the evaluator, without values.  State:
//   cnt  values of the chunk on the logical stack
//   P    1 when the top of the stack is an X not yet written anywhere
//   m    physical stack entries (entries below the register-held top,
//        plus possibly one unused bottom entry)
// A function meeting fewer than two values is a "spine" node: its subtree
// leaves the chunk.  The value it would take from the chunk (at most one)
// becomes a result slot (or stays an X when it is a bare input), and the
// spine node itself goes into the skeleton.  At the chunk's first token all
// values still on the stack become result slots.

// ------------------------------------------------------ structure machine
//
// The right-to-left stack machine of both interpreters, run without values:
//   tv  the top value T is live      P  an X sits on top, not yet placed
//   m   values below T               base  of those, how many live in the
//                                          wave's spill slab (multiple of
//                                          the half window)
// A function meeting fewer than two values is a "spine" node: its subtree
// leaves the chunk; the value it would take from the chunk (at most one)
// becomes a result slot (or stays an X when it is a bare input) and the
// node goes into the next level's skeleton.  At the chunk's first token all
// values still on the stack become result slots.  For the register-stack
// interpreter every action is also written as one code, an X folded into
// the function or push that consumes it, and a push or load of x directly
// followed by a function of x fused into one code; SPILL and FILL keep T
// inside the window of EV_VSTACK register entries.  One implementation
// serves counting and emission, so the two cannot disagree.

struct Sink {
    uint16_t* codes;   // nullptr: count codes only
    uint64_t at;       // global index of the next code
    uint8_t* frag;     // nullptr: count fragment tokens only
    uint64_t w;        // one past the next fragment token (written backwards)
    uint32_t n_codes, n_frag, n_out, n_in;
    uint32_t pending;  // EV_K_PUSHX / EV_K_LOADX waiting for fusion, or ~0u

    __device__ void put(uint32_t kind)
    {
        if (codes) codes[at] = (uint16_t)((uint32_t)(at & (EV_CODE_POS - 1)) * EV_CODE_BLOCK + kind * EV_CODE_STRIDE);
        at++;
        n_codes++;
    }
    __device__ void code(uint32_t kind)
    {
        if (pending != ~0u) {
            if (kind >= EV_K_OPX0 && kind <= EV_K_OPX3) {
                put((pending == EV_K_PUSHX ? EV_K_CH0 : EV_K_LCH0) + (kind - EV_K_OPX0));
                pending = ~0u;
                return;
            }
            put(pending);
            pending = ~0u;
        }
        if (kind == EV_K_PUSHX || kind == EV_K_LOADX) {
            pending = kind;
            return;
        }
        put(kind);
    }
    __device__ void ftok(uint32_t t)
    {
        if (frag) frag[--w] = (uint8_t)t;
        n_frag++;
    }
};

// Reads one chunk's tokens right to left, 16 bytes per load.
struct RevTokens {
    const uint8_t* seq;
    uint64_t k, lo, wb;
    u32x4 wd;
    __device__ RevTokens(const uint8_t* s, uint64_t start, uint32_t len) : seq(s), k(start + len), lo(start), wb(~0ull) {}
    __device__ bool next(uint32_t& t)
    {
        if (k <= lo) return false;
        k--;
        const uint64_t b = k & ~(uint64_t)15;
        if (b != wb) {
            wd = *reinterpret_cast<const u32x4*>(seq + b);
            wb = b;
        }
        const uint32_t j = (uint32_t)(k & 15);
        const uint32_t word = j >= 8 ? (j >= 12 ? wd.w : wd.z) : (j >= 4 ? wd.y : wd.x);
        t = (word >> (8 * (j & 3))) & 255u;
        return true;
    }
};

struct MachineOut {
    uint32_t maxtop;  // deepest m
    int32_t net;      // sum over tokens of (+1 function, -1 leaf)
    int32_t minpref;  // minimum of that running sum before a token
    uint32_t bad;     // a token above max_tok
};

__device__ MachineOut run_machine(const uint8_t* __restrict__ seq, uint64_t start, uint32_t len, uint32_t max_tok,
                                  Sink& o)
{
    uint32_t tv = 0, P = 0, m = 0, base = 0, maxtop = 0, bad = 0;
    int32_t R = 0, maxR = INT32_MIN;
    RevTokens rt(seq, start, len);
    uint32_t t;
    while (rt.next(t)) {
        bad |= t > max_tok;
        R += t < TOK_X ? 1 : -1;
        maxR = R > maxR ? R : maxR;
        if (t == TOK_X) {
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
            if (tv) {
                if (m + 1 - base > EV_VSTACK - 1) { o.code(EV_K_SPILL); base += EV_VHALF; }
                o.code(EV_K_PUSHREF);
                m++;
            } else {
                o.code(EV_K_LOADREF);
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
                    o.ftok(P ? TOK_X : TOK_REF);
                }
                o.ftok(t);
                tv = 0; P = 0; m = 0;
            }
        }
        maxtop = m > maxtop ? m : maxtop;
    }
    // chunk start: every value left becomes a slot, the bottom one first
    if (base > 0) {
        o.code(EV_K_FLUSH);
        for (uint32_t i = 0; i < base; i++) o.code(EV_K_OUTMEM);
    }
    if (m > base) {
        o.code(EV_K_FLUSH);
        for (uint32_t i = base; i < m; i++) o.code(EV_K_OUTBOT);
    }
    if (tv) o.code(EV_K_OUTT);
    if (P) o.code(EV_K_OUTX);
    o.code(EV_K_END);
    const uint32_t left = m + tv + P;
    o.n_out += left;
    for (uint32_t i = 0; i < left; i++) o.ftok(TOK_REF);
    MachineOut r;
    r.maxtop = maxtop;
    r.net = R;
    r.minpref = len ? R - maxR : 0;
    r.bad = bad;
    return r;
}

__global__ void k_count(const uint8_t* __restrict__ seq, const ChunkIn* __restrict__ in, uint32_t n,
                        ChunkStat* __restrict__ out, uint32_t max_tok)
{
    const uint32_t ci = blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= n) return;
    const ChunkIn c = in[ci];
    Sink o{nullptr, 0, nullptr, 0, 0, 0, 0, 0, ~0u};
    const MachineOut r = run_machine(seq, c.start, c.len, max_tok, o);
    ChunkStat s;
    s.n_out = o.n_out;
    s.n_frag = o.n_frag;
    s.n_in = o.n_in;
    s.max_m = r.maxtop + 1;
    s.net = r.net;
    s.minpref = r.minpref;
    s.bad = r.bad;
    s.n_codes = o.n_codes;
    s.maxtop = r.maxtop;
    s.code_out = o.n_out;
    s.code_in = o.n_in;
    out[ci] = s;
}

// Emission: the chunk's skeleton fragment (ending at frag_end[ci]) and, for
// register-stack items, its codes (from code_begin[ci]).
__global__ void k_emit(const uint8_t* __restrict__ seq, const ChunkIn* __restrict__ in,
                       const uint64_t* __restrict__ frag_end, const uint64_t* __restrict__ code_begin, uint32_t n,
                       uint8_t* __restrict__ dst, uint16_t* __restrict__ codes)
{
    const uint32_t ci = blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= n) return;
    const ChunkIn c = in[ci];
    const bool has_codes = codes && code_begin[ci] != ~0ull;
    if (!dst && !has_codes) return;
    Sink o{has_codes ? codes : nullptr, has_codes ? code_begin[ci] : 0, dst, dst ? frag_end[ci] : 0, 0, 0, 0, 0, ~0u};
    run_machine(seq, c.start, c.len, TOK_REF, o);
}

// Every code of a register-stack item must name a handler of its own
// position and the item must end with its only END; simulating the codes
// must keep T inside the register window, every read entry below it, the
// slab within its entries, and must write and read exactly the slots the
// plan gave the item.  Anything else fails the plan before a code runs.
__global__ void k_check_codes(const uint16_t* __restrict__ codes, const uint64_t* __restrict__ begin,
                              const uint32_t* __restrict__ expect, uint32_t n, uint32_t slab_entries,
                              uint32_t* __restrict__ err)
{
    const uint32_t ci = blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= n) return;
    const uint64_t b = begin[ci];
    const uint32_t len = expect[3 * ci], want_out = expect[3 * ci + 1], want_in = expect[3 * ci + 2];
    uint32_t outs = 0, ins = 0, bad = len == 0;
    int32_t idx = 0, slab = 0, fl = 0;
    for (uint32_t i = 0; i < len; i++) {
        const uint32_t v = codes[b + i];
        const uint32_t pos = v / EV_CODE_BLOCK, r = v % EV_CODE_BLOCK, k = r / EV_CODE_STRIDE;
        if (r % EV_CODE_STRIDE || pos != (uint32_t)((b + i) & (EV_CODE_POS - 1)) || k > EV_K_OUTMEM) bad = 1;
        if ((k == EV_K_END) != (i + 1 == len)) bad = 1;
        if (k <= EV_K_OPS3) {
            bad |= idx < 1;
            idx--;
        } else if ((k >= EV_K_CH0 && k <= EV_K_CH3) || k == EV_K_PUSHX || k == EV_K_PUSHREF) {
            idx++;
        } else if (k == EV_K_FLUSH) {
            fl = 0;
        } else if (k == EV_K_OUTBOT) {
            bad |= fl >= idx;
            fl++;
        } else if (k == EV_K_OUTMEM) {
            bad |= fl >= slab;
            fl++;
        } else if (k == EV_K_SPILL) {
            bad |= idx < (int32_t)EV_VHALF;
            idx -= EV_VHALF;
            slab += EV_VHALF;
        } else if (k == EV_K_FILL) {
            bad |= slab < (int32_t)EV_VHALF || idx != 0;
            idx += EV_VHALF;
            slab -= EV_VHALF;
        }
        bad |= idx < 0 || idx > (int32_t)EV_VSTACK - 1 || slab < 0 || slab > (int32_t)slab_entries;
        outs += (k == EV_K_OUTT || k == EV_K_OUTX || k == EV_K_OUTBOT || k == EV_K_OUTMEM);
        ins += (k == EV_K_PUSHREF || k == EV_K_LOADREF);
    }
    if (bad || outs != want_out || ins != want_in) atomicOr(err, 1u);
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
        float T = 0.0f;

#define RING(e) ring[((e) & (D - 1)) * 64u + lane]
#define STEP(tok)                                                                   \
    do {                                                                            \
        const uint32_t t_ = (tok);                                                  \
        if (t_ == TOK_X) {                                                          \
            if (P) { RING(m) = T; m++; T = xv; } else { P = 1; }                    \
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
                if (P) { av = xv; bv = T; P = 0; }                                  \
                else { m--; av = T; bv = RING(m); }                                 \
                T = apply_op(t_, av, bv);                                           \
                cnt--;                                                              \
            }                                                                       \
        } else {                                                                    \
            in_slot--;                                                              \
            const float r_ = act ? in_res[(size_t)in_slot * (size_t)N + cs] : 0.0f; \
            if (P) { RING(m) = T; m++; T = xv; P = 0; }                             \
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
                if (act) out_res[(size_t)out_slot * (size_t)N + cs] = xv;
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
__global__ void k_fitness(const uint64_t* __restrict__ rows, const float* __restrict__ y, int32_t N, uint32_t M,
                          float* __restrict__ fit, float* __restrict__ per_case)
{
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    const float* r = reinterpret_cast<const float*>(rows[t]);
    float s = 0.0f;
    for (int32_t i = 0; i < N; i++) {
        const float v = r[i];
        s = s + fabsf(v - y[i]);
        if (per_case) per_case[(size_t)t * (size_t)N + i] = v;
    }
    fit[t] = s / (float)N;
}

// ---------------------------------------------------------------- crossover
//
// Sec. 3.1: the subtree rooted at p ends where the open-slot count started at
// p first drops to zero.  One wave scans 256 tokens per step: each lane takes
// four, the wave prefix-sums their net effect and the first lane whose
// running minimum reaches zero holds the end.
__global__ __launch_bounds__(64) void k_subtree_end(const uint8_t* __restrict__ buf, const uint64_t* __restrict__ base,
                                                    const uint64_t* __restrict__ pos, uint32_t n,
                                                    uint64_t* __restrict__ end_out)
{
    const uint32_t qi = blockIdx.x;
    if (qi >= n) return;
    const uint32_t lane = threadIdx.x;
    const uint8_t* t = buf + base[qi];
    uint64_t k = pos[qi];
    int32_t open = 1;  // slots still to fill before the subtree is complete
    for (;;) {
        const uint8_t* tb = t + k + lane * 4u;
        const uint32_t wv = (uint32_t)tb[0] | ((uint32_t)tb[1] << 8) | ((uint32_t)tb[2] << 16) | ((uint32_t)tb[3] << 24);
        int32_t c = 0;
        for (int j = 0; j < 4; j++) c += (((wv >> (8 * j)) & 255u) < TOK_X) ? 1 : -1;
        int32_t pre = c;
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t o = __shfl_up(pre, d, 64);
            if ((int)lane >= d) pre += o;
        }
        const int32_t before = pre - c;
        int32_t hit = -1, cc = 0;
        for (int j = 0; j < 4; j++) {
            cc += (((wv >> (8 * j)) & 255u) < TOK_X) ? 1 : -1;
            if (hit < 0 && open + before + cc == 0) hit = j;
        }
        const uint64_t mask = __ballot(hit >= 0);
        if (mask) {
            const int first = __ffsll((unsigned long long)mask) - 1;
            const int j = __shfl(hit, first, 64);
            if (lane == 0) end_out[qi] = k + (uint64_t)first * 4u + (uint64_t)j;
            return;
        }
        open += __shfl(pre, 63, 64);
        k += 256;
    }
}

// Copy children: mum[0,p) + dad[q, eq] + mum(ep, nm).  Grid: x = 4 KiB pieces
// of the child, y = child.
__global__ void k_xo_copy(const uint8_t* __restrict__ mums, const uint8_t* __restrict__ dads,
                          const XoPlan* __restrict__ plan, uint32_t n_children, uint8_t* __restrict__ dst)
{
    const uint32_t j = blockIdx.y;
    if (j >= n_children) return;
    const XoPlan x = plan[j];
    const uint64_t lo = (uint64_t)blockIdx.x * 4096u;
    if (lo >= x.child_len) return;
    const uint64_t hi = lo + 4096u < x.child_len ? lo + 4096u : x.child_len;
    const uint64_t a = x.p, b = x.p + (x.eq - x.q + 1);
    uint8_t* out = dst + x.child_off;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        uint8_t v;
        if (x.copy_mum) v = mums[x.mum_off + i];
        else if (i < a) v = mums[x.mum_off + i];
        else if (i < b) v = dads[x.dad_off + x.q + (i - a)];
        else v = mums[x.mum_off + x.ep + 1 + (i - b)];
        out[i] = v;
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
                         uint64_t* __restrict__ p, uint64_t* __restrict__ q)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int32_t mm = tournament(fit, M, k, k0, k1, gen, j, 0);
    const int32_t dd = tournament(fit, M, k, k0, k1, gen, j, 1);
    uint32_t w[4] = {j, 0x300u, (uint32_t)gen, (uint32_t)(gen >> 32)};
    philox10(w, k0, k1);
    const uint64_t up = ((uint64_t)w[1] << 32) | w[0];
    const uint64_t uq = ((uint64_t)w[3] << 32) | w[2];
    mum[j] = mm;
    dad[j] = dd;
    p[j] = mulhi_u64(up, off[mm + 1] - off[mm]);
    q[j] = mulhi_u64(uq, off[dd + 1] - off[dd]);
}

}  // namespace ev

namespace ev {

// --------------------------------------------------- register-stack kernel
//
// One wave runs the threaded codes of one work item (lane = test case); see
// gen_interp.py for the handlers.  Chunks whose stack would outgrow the
// register window run on k_eval instead.
__global__ __launch_bounds__(64) void k_run(RunArgs a)
{
    const uint32_t lane = threadIdx.x;
    const_u4p chunks = (const_u4p)(global_u4p)(const void*)a.chunks;
    // this wave's spill slab: slab_entries rows of 64 lanes
    const uint64_t smem = (uint64_t)(uintptr_t)a.slab + (uint64_t)blockIdx.x * a.slab_entries * 256u;
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
            const uint64_t cptr = (uint64_t)(uintptr_t)a.codes + (code_begin & ~(uint64_t)31) * 2u;
            const uint32_t j0 = (uint32_t)(code_begin & 31u);
            const uint64_t inp = (uint64_t)(uintptr_t)a.in_res + (uint64_t)d.z * a.rowb;
            const uint64_t outp = (uint64_t)(uintptr_t)a.out_res + (uint64_t)d.w * a.rowb;
            const uint32_t slane = lane * 4u;
            asm volatile(EV_INTERP_ASM
                         :
                         : [x] "v"(xv), [lane4] "v"(lane4), [slane] "v"(slane), [cptr] "s"(cptr), [j0] "s"(j0),
                           [inp] "s"(inp), [outp] "s"(outp), [rowb] "s"(a.rowb), [smem] "s"(smem)
                         : EV_INTERP_CLOBBERS);
        }
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

hipError_t launch_count(const uint8_t* seq, const ChunkIn* in, uint32_t n, ChunkStat* out, uint32_t max_tok,
                        hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count, dim3(cdiv(n, 64)), dim3(64), 0, s, seq, in, n, out, max_tok);
    return hipGetLastError();
}

hipError_t launch_emit(const uint8_t* seq, const ChunkIn* in, const uint64_t* frag_end, const uint64_t* code_begin,
                       uint32_t n, uint8_t* dst, uint16_t* codes, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_emit, dim3(cdiv(n, 64)), dim3(64), 0, s, seq, in, frag_end, code_begin, n, dst, codes);
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

hipError_t launch_run(const RunArgs& a, uint32_t grid, hipStream_t s)
{
    if (a.n_items == 0 || grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_run, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}


hipError_t launch_check_codes(const uint16_t* codes, const uint64_t* begin, const uint32_t* expect, uint32_t n,
                              uint32_t slab_entries, uint32_t* err, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_codes, dim3(cdiv(n, 64)), dim3(64), 0, s, codes, begin, expect, n, slab_entries, err);
    return hipGetLastError();
}

hipError_t launch_fitness(const uint64_t* rows, const float* y, int32_t N, uint32_t M, float* fit, float* per_case,
                          hipStream_t s)
{
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fitness, dim3(cdiv(M, 64)), dim3(64), 0, s, rows, y, N, M, fit, per_case);
    return hipGetLastError();
}

hipError_t launch_subtree_end(const uint8_t* buf, const uint64_t* base, const uint64_t* pos, uint32_t n,
                              uint64_t* end_out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_subtree_end, dim3(n), dim3(64), 0, s, buf, base, pos, n, end_out);
    return hipGetLastError();
}

hipError_t launch_xo_copy(const uint8_t* mums, const uint8_t* dads, const XoPlan* plan, uint32_t n,
                          uint64_t max_child, uint8_t* dst, hipStream_t s)
{
    if (n == 0 || max_child == 0) return hipSuccess;
    hipLaunchKernelGGL(k_xo_copy, dim3(cdiv(max_child, 4096), n), dim3(256), 0, s, mums, dads, plan, n, dst);
    return hipGetLastError();
}

hipError_t launch_select(const float* fit, const uint64_t* off, uint32_t M, int32_t k, uint64_t seed, uint64_t gen,
                         int32_t* mum, int32_t* dad, uint64_t* p, uint64_t* q, hipStream_t s)
{
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3(cdiv(M, 64)), dim3(64), 0, s, fit, off, M, k, seed, gen, mum, dad, p, q);
    return hipGetLastError();
}

}  // namespace ev
