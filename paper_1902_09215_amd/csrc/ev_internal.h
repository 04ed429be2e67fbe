// Internal types shared by the libev kernels and the host runtime.
#pragma once
#include <stdint.h>

namespace ev {

enum : uint32_t { TOK_ADD = 0, TOK_SUB = 1, TOK_MUL = 2, TOK_DIV = 3, TOK_X = 4, TOK_REF = 5 };
// Tokens TOK_C0 .. TOK_C0 + n_consts - 1: ephemeral random constants (leaves
// whose value is the same on every case).
constexpr uint32_t TOK_C0 = 6;
constexpr uint32_t MAX_CONSTS = 250;
// ChunkStat.bad / SegFn.bad flags: a token outside the level's alphabet, and
// (not an error) a constant seen
constexpr uint32_t BAD_TOKEN = 1u, HAS_CONST = 4u;

struct GLevel;  // a level's live counts in a device-made plan (below)

// Register-stack entries of k_run (the interpreter's VGPR window).
#include "ev_interp.inc"
constexpr uint32_t EV_VSTACK_ENTRIES = EV_VSTACK;

// A work item of the split plan as the structure passes see it.
struct ChunkIn {
    uint64_t start;  // first token, offset into the level's sequence
    uint32_t len;    // tokens
    uint32_t tree;   // owning tree
};

struct ChunkStat {
    uint32_t n_out;   // values written to result slots
    uint32_t n_frag;  // tokens of the chunk's skeleton fragment
    uint32_t n_in;    // REF tokens read
    uint32_t max_m;   // deepest physical operand stack
    int32_t net;      // sum over tokens of (+1 function, -1 leaf)
    int32_t minpref;  // minimum of that running sum before a token
    uint32_t bad;     // a token outside the level's alphabet was seen
    uint32_t n_codes; // threaded codes of the chunk (register-stack kernel)
    uint32_t maxtop;  // highest register-stack index the codes touch
    uint32_t code_out;  // slot-writing codes (must equal n_out)
    uint32_t code_in;   // slot-reading codes (must equal n_in)
};

// Bytes of 0xFF after a population's trees: room for the wide reads of
// the subtree scan (up to 4 KiB past a subtree's end) and the token readers.
constexpr uint64_t EV_POP_PAD = 4096 + 64;

// Structure segments (SEG_TOKENS tokens of one chunk).
constexpr uint32_t SEG_TOKENS = 256;
struct SegIn {
    uint64_t start;
    uint32_t len;
    uint32_t last;  // holds the chunk's first token (read last)
};

// A level's segment length: SEG_TOKENS at a large level 0, a quarter of it
// at a smaller one and at the skeleton levels, which need the extra lanes
// (each segment is one lane of the structure passes), and 16 tokens at a
// level of under 2^20 tokens, whose passes take about the time of one
// lane's segment.
constexpr uint64_t SEG_BIG_LEVEL = 1ull << 26;
constexpr uint64_t SEG_SMALL_LEVEL = 1ull << 20;
constexpr uint32_t seg_len_for(int level, uint64_t tokens)
{
    return level == 0 && tokens >= SEG_BIG_LEVEL ? SEG_TOKENS : tokens < SEG_SMALL_LEVEL ? 16u : SEG_TOKENS / 4;
}

// Bytes of one segment's recording regions (its code kinds, its fragment
// tokens) at a level whose segments hold at most seg_len tokens.
constexpr uint64_t rec_kinds_stride(uint32_t seg_len) { return 4ull * seg_len + 64ull; }
constexpr uint64_t rec_frags_stride(uint32_t seg_len) { return 2ull * seg_len + 16ull; }

struct ChunkSegs {
    uint32_t first;  // first segment (token order)
    uint32_t n_seg;
};

// A tree's part of one level of the split plan (host to device): its range
// in the level's sequence and where its chunks and segments go.
struct TreeLvl {
    uint64_t start, len;  // the tree's tokens at this level
    uint32_t chunk_first, n_chunks;
    uint32_t seg_first;   // first segment of its first chunk
    uint32_t C;           // tokens per chunk (all but the last are full)
    uint32_t tree;
    uint32_t ref_base;    // its first input slot: the previous level's slot index
    uint32_t rank_full;   // places of its work items in their length buckets:
    uint32_t rank_last;   //   full chunks rank_full, rank_full + 1, ...; the last rank_last
};

// A tree's totals over its chunks at one level (device to host).
struct TreeSum {
    uint64_t n_out, n_frag, n_codes;
    uint32_t bad;     // 1: not a valid prefix tree (level 0); 2: input slots out of range
    uint32_t maxtop;  // highest register-stack index of its chunks' codes
    uint32_t max_m;   // deepest physical stack of its chunks
    uint32_t pad;
};

// Per tree id: its bases over the level's chunks (made on the device from
// the trees' totals), and its chunks and their places in the length
// buckets (copied from its TreeLvl).
struct TreeBase {
    uint64_t out, frag, code;
    uint32_t chunk_first, n_chunks;
    uint32_t rank_full, rank_last;
};

// Work items, longest first: the number of buckets of the counting sort on
// a length's bit count.
constexpr uint32_t EV_LEN_BUCKETS = 33;

// Levels a split plan may have.
constexpr int EV_MAX_LEVELS = 64;

// Where each tree's value ends up: its level's result rows, and its slot.
struct FitArgs {
    const float* res[EV_MAX_LEVELS + 1];
    uint32_t n_out[EV_MAX_LEVELS + 1];  // slots of each level
    uint32_t n_levels;
    const uint32_t* fin;  // per tree: level, slot
    const float* y;
    int32_t N;
    uint32_t M;
    float* fit;
    float* per_case;
    int32_t* hits;  // nullable: per tree, the cases within 0.01 of the target
    const GLevel* gl;  // nullable: a device-made plan's levels (their slot counts replace n_out)
};

struct SegFn {
    int32_t a, b;      // the segment maps cnt to max(cnt + a, b)
    int32_t net;       // sum over tokens of (+1 function, -1 leaf)
    int32_t minpref;   // minimum of that running sum before a token
    uint32_t bad, n_in;
    uint32_t left_x;   // its first token is a leaf (x or a constant)
    uint32_t left_tok; // and which
};

struct SegStart {
    uint32_t cnt, P;
    uint32_t ref0;  // REF tokens the chunk's later segments hold (read before this one)
    uint32_t ptok;  // with P: the pending leaf's token (x or a constant)
};

struct SegCount {
    uint32_t n_codes, n_frag, n_out, n_in, maxtop, pad;
};

// What a segment's recording leaves out: the chunk end's runs of n1 slot
// writes from the slab (inserted before recorded kind a1) and n2 from the
// window (before a2), and the REF tokens after its nfr recorded fragment
// tokens.
struct SegRec {
    uint32_t a1, n1, a2, n2, nfr, pad;
};

// A work item of the register-stack kernel (16 bytes).
struct RunChunk {
    uint64_t code_begin;  // index of its first code in the level's code stream
    uint32_t in_end;
    uint32_t out_end;
};

struct RunArgs {
    const uint32_t* codes;
    const RunChunk* chunks;
    uint32_t n_items;
    uint32_t n_cb;
    uint32_t* counter;
    const float* x;
    int32_t N;
    uint32_t rowb;  // bytes per result slot row (N * 4)
    const float* in_res;
    float* out_res;
    float* slab;            // spill slabs, one per wave of the grid
    uint64_t slab_entries;  // rows of 64 floats per slab
    uint32_t* flag;         // set to 1 if the interpreter's table cannot be used (see gen_interp.py)
    uint32_t refs;          // 1 at the skeleton levels: REF slots are read ahead
    const uint32_t* verdict;  // the validator's flags for these code streams: nonzero runs nothing
    const GLevel* gl;         // nullable: a device-made level (its item count and spill rows replace n_items, slab_entries)
};

// One plan level of a chained launch of the register-stack kernel.
struct RunLevel {
    const uint32_t* codes;
    const RunChunk* chunks;
    const uint32_t* item_tree;  // per work item: its tree
    const float* in_res;        // the previous level's slot rows
    float* out_res;
    const uint32_t* verdict;    // the validator's flags for the level's code streams
    uint32_t first;             // the record's first place in the launch's queue
    uint32_t n_items;           // work items x case blocks
    uint32_t refs;
    uint32_t plevel;            // its plan level, counted from the launch's first
};

// Several levels in one launch: a work item of a level waits for its tree's
// items of the level before (need: work items per level and tree; done:
// finished items x case blocks, cleared before the launch).  The queue is a
// list of records, each a run of one level's work items (chunks and
// item_tree point at the run's first); a level may be split over several
// records, each of them after every record that holds work its items wait
// for.
struct ChainArgs {
    const RunLevel* levels;
    uint32_t n_levels;  // records
    uint32_t total;  // items of every level
    uint32_t n_cb;
    uint32_t M;      // trees (the stride of need and done)
    uint32_t* counter;
    const uint32_t* need;
    uint32_t* done;
    const float* x;
    int32_t N;
    uint32_t rowb;
    float* slab;
    uint64_t slab_entries;
    uint32_t* flag;
};

// A work item as the evaluator sees it (32 bytes).
struct EvalChunk {
    uint64_t start;
    uint32_t len;
    uint32_t in_end;   // one past the last input slot this chunk reads
    uint32_t out_end;  // one past the last output slot this chunk writes
    uint32_t tree;
    uint32_t pad0, pad1;
};

struct EvalArgs {
    const uint8_t* seq;
    const EvalChunk* chunks;
    uint32_t n_items;  // chunks * n_cb
    uint32_t n_cb;     // 64-case blocks per chunk
    uint32_t* counter;
    const float* x;
    int32_t N;
    uint32_t gstack_entries;  // stack entries per wave in gstack
    const float* in_res;
    float* out_res;
    float* gstack;
    const float* consts;  // the constants' values (token TOK_C0 + i is consts[i])
};

static_assert(sizeof(EvalChunk) == 32, "EvalChunk layout");

// Level 0 of a planned population, per tree: its range of chunks (the
// chunks themselves, in token order, are kept with the plan so that a child
// can take over those crossover leaves intact).
struct L0Tree {
    uint32_t chunk_first, n_chunks;
};

// A child's level 0 from its mum's (Sec. 3.1: the child is its mum with the
// subtree at p replaced): the mum's chunks wholly before p and wholly after
// the end ep of that subtree keep their tokens, so their codes and skeleton
// fragments are the mum's; only the tokens between them are planned.
struct ReuseRun {
    uint64_t mid_start, mid_len;  // the child's tokens planned afresh (child offsets)
    int64_t shift;                // child length - mum length: where the kept suffix lands
    uint64_t mum_off;             // the mum's first token in its population
    uint32_t src_first;           // the mum's first level-0 chunk (index into its chunk tables)
    uint32_t n_pre;               // mum chunks 0 .. n_pre-1 kept, at their own offsets
    uint32_t ks, n_suf;           // mum chunks ks .. ks+n_suf-1 kept, at their offsets + shift
    uint32_t mum, pad;            // the mum's index in its population
};

// A child as the chunk kernel of a reusing plan sees it.
struct TreeReuse {
    uint64_t start;  // the child's first token in the level's sequence
    ReuseRun r;
    uint32_t chunk_first, seg_first, tree, C;  // C: the fresh chunks' size
    uint32_t n_mid, mid_last;                  // fresh chunks (all C tokens but the last)
};

// A population's statistics as the device reduces them (see ev_pop_stats).
struct PopStatsDev {
    double sum_fit;      // over finite fitness values
    double sum_size;
    uint64_t min_size, max_size;
    uint32_t best, n_finite, converged, pad;
};

// A generation replayed from a captured graph (Sec. 2.3's loop with no
// host wait inside a generation) plans its children on the device.  Its
// buffers are sized for capacities fixed at capture and its launches for
// those capacities; each level's live counts are made on the device
// (k_g_begin, k_g_end) and the kernels take them from the level's GLevel,
// doing nothing past them.  A count over its capacity voids the generation
// (GStatus), which the host then runs again on the host-driven path.
struct GLevel {
    uint32_t nt, n, n_seg;   // the level's trees, work items and structure segments
    uint32_t record;         // the count pass records codes (fixed at capture)
    uint32_t record_ovf;     // a recording region overflowed: emit and check instead of place
    uint32_t slab_entries;   // spill rows per wave of k_run
    uint32_t any;            // some tree goes on to the next level
    uint32_t pad;
    uint64_t tokens, prev_out;  // the level's tokens; the previous level's slots
    uint64_t so, sf, sc;        // slots, next skeleton tokens, codes (with each item's padding)
};

// A tree's state between the levels of a device-made plan.
struct GTree {
    uint64_t rs, rl, prev_len;  // its range in the level's sequence; its length a level before
    uint32_t ref_base, active;  // its first input slot; it has work at the level
};

// A level's capacities (fixed at capture).
struct GCap {
    uint64_t n, n_seg, so, sf, sc;
    uint32_t slab, pad;
};

// Why a replayed generation is void (GStatus.poison bits).
enum : uint32_t {
    G_OVF_BYTES = 1u,       // the children's bytes or copy pieces
    G_OVF_ITEMS = 2u,       // work items or segments of a level
    G_OVF_SIZES = 4u,       // slots, skeleton tokens or codes of a level
    G_OVF_SLAB = 8u,        // spill rows
    G_OVF_LEVELS = 16u,     // more levels than captured
    G_MALFORMED = 32u,      // a child is not a valid prefix tree
    G_INCONSISTENT = 64u,   // input slots out of range
    G_CONSTS = 128u,        // a constant token (not planned for the register-stack kernel)
    G_INVALID_CODES = 256u  // a level's code streams failed validation
};

struct GStatus {
    uint32_t poison, level;  // the reasons; the level of the first
    uint32_t levels, pad;    // levels the plan used
    uint64_t child_bytes, capped;
};

struct XoPlan {
    uint64_t mum_off, dad_off;  // tree starts in the parents' buffers
    uint64_t p, ep, q, eq;      // points and the ends of their subtrees
    uint64_t child_off, child_len;
    uint32_t copy_mum;          // child over the size cap: copy of the mum
    uint32_t pad;
};

}  // namespace ev
