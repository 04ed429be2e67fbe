// The generational loop of Sec. 2.3 replayed from captured HIP graphs:
// ev_evolve.
//
// One generation is selection (Table 1's tournaments, Philox draws),
// subtree crossover (Sec. 3.1), the children's split plan, their
// evaluation and their fitness.  On the host-driven path the host waits
// inside a generation: for the children's offsets (to size their buffer)
// and for each plan level's totals (to size the next level's).  Here the
// whole generation is one graph of fixed launches over buffers sized for
// capacities: the plan is made on the device (k_g_begin / k_g_end and the
// structure kernels reading each level's live counts), and the host only
// launches the graph and, after it, reads a status word, the levels' counts
// and the children's fitness from pinned memory.
//
// The population rotates through three buffers, and one graph is captured
// per buffer (parents there, children in the next).  Replays are pipelined:
// generation i + 1 is launched before the host reads generation i's status,
// so the host's checks and the next launch overlap the device's work.  The
// third buffer keeps generation i's parents intact while i + 1 runs, so a
// voided generation can still be redone.  A generation whose counts exceed
// a capacity voids itself (every later step of it does nothing) and is done
// again on the host-driven path, whose results are the same bit for bit;
// the generation launched after it is discarded, the capacities are
// re-derived from the redone generation's plan and the graphs captured
// again.  Counts nearing a capacity trigger the same re-capture after a
// good generation, so that growing trees (Sec. 4's bloat) rarely reach the
// fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>

#include "ev_runtime.h"

namespace ev {

// Sizes of one plan level (observed, or capacities).
struct LevelSize {
    uint64_t n = 0, n_seg = 0, so = 0, sf = 0, sc = 0, slab = 0, tokens = 0;
};

static constexpr uint32_t G_N_ERR = 2 * (EV_MAX_LEVELS + 1);
static constexpr int NB = 3;  // population buffers (and graphs) in the rotation
static int nxt(int a) { return a + 1 < NB ? a + 1 : 0; }
static constexpr uint64_t G_RECORD_MAX = (uint64_t)2 << 30;

struct GenGraph {
    int device = 0;
    int32_t M = 0, table = -1, N = 0, k = 2;
    uint64_t seed = 0, cap = 0;
    uint32_t C0 = 0, C1 = 0;
    int run_grid = 0;
    bool use_record = true;
    float* d_x = nullptr;
    const float* d_y = nullptr;

    // the population's buffers (bytes with their padding, offsets in the
    // crossover layout, fitness)
    uint64_t bytes_cap = 0, pieces_cap = 0;
    uint8_t* bytes[NB] = {};
    uint64_t* off[NB] = {};
    float* fit[NB] = {};
    int cur = 0;  // the buffer holding the current parents

    // per-generation scratch: selection and crossover
    int32_t *mum = nullptr, *dad = nullptr;
    uint64_t *p = nullptr, *q = nullptr, *qb = nullptr, *qp = nullptr, *ends = nullptr;
    XoPlan* plan = nullptr;
    uint64_t* gen_at = nullptr;

    // the plan made on the device (its capacities, levels, state)
    uint32_t L = 0;
    std::vector<LevelSize> caps;
    bool record = false;
    uint64_t n_max = 0, nseg_max = 0, slab_max = 0;
    std::vector<void*> blocks;  // every plan block, freed together
    GTree* tr = nullptr;
    TreeLvl* tl = nullptr;
    GLevel* gls = nullptr;
    GCap* d_caps = nullptr;
    GStatus* st = nullptr;
    uint32_t *fin = nullptr, *err = nullptr, *counters = nullptr;
    ChunkIn* ch = nullptr;
    ChunkSegs* cseg = nullptr;
    SegIn* seg = nullptr;
    SegFn* fn = nullptr;
    SegStart* sst = nullptr;
    SegCount* cnt = nullptr;
    ChunkStat* stat = nullptr;
    uint64_t* loc = nullptr;
    uint32_t* inend = nullptr;
    TreeSum* sum = nullptr;
    TreeBase* tb = nullptr;
    uint64_t *cb = nullptr, *fe = nullptr, *scode = nullptr, *sfrag = nullptr;
    uint8_t *rk = nullptr, *rf = nullptr;
    SegRec* rec = nullptr;
    uint32_t* cursor = nullptr;  // each length bucket's first place
    std::vector<uint32_t> seg_len;  // per level
    uint8_t* skel[2] = {nullptr, nullptr};
    std::vector<uint32_t*> codes;
    std::vector<RunChunk*> run;
    std::vector<float*> res;
    float* slab = nullptr;
    uint32_t grid = 0;

    // pinned host, per graph: the status, the levels' counts and the
    // children's fitness of its last replay
    uint8_t* pin[NB] = {};
    GStatus* h_st[NB] = {};
    GLevel* h_lv[NB] = {};
    float* h_fit[NB] = {};
    hipEvent_t done[NB] = {};  // the end of each graph's last replay

    // per buffer: the graph of all L levels, and one of the first L - 1
    // (the last level is room to grow; while recent generations have not
    // needed it, its launches are left out)
    hipGraph_t graph[NB] = {}, graph_s[NB] = {};
    hipGraphExec_t exec[NB] = {}, exec_s[NB] = {};
};

static void graphs_drop(GenGraph& g)
{
    for (int i = 0; i < NB; i++) {
        for (hipGraphExec_t* e : {&g.exec[i], &g.exec_s[i]}) {
            if (*e) (void)hipGraphExecDestroy(*e);
            *e = nullptr;
        }
        for (hipGraph_t* h : {&g.graph[i], &g.graph_s[i]}) {
            if (*h) (void)hipGraphDestroy(*h);
            *h = nullptr;
        }
    }
}

// The plan's buffers (not the population's).  The caller has synchronized.
static void plan_blocks_free(ev_ctx* c, GenGraph& g)
{
    graphs_drop(g);
    for (void* b : g.blocks) dev_free(c, b);
    g.blocks.clear();
    g.codes.clear();
    g.run.clear();
    g.res.clear();
}

static void pop_blocks_free(ev_ctx* c, GenGraph& g)
{
    for (int i = 0; i < NB; i++) {
        dev_free(c, g.bytes[i]);
        dev_free(c, g.off[i]);
        dev_free(c, g.fit[i]);
        g.bytes[i] = nullptr;
        g.off[i] = nullptr;
        g.fit[i] = nullptr;
    }
    g.bytes_cap = g.pieces_cap = 0;
}

static void xo_blocks_free(ev_ctx* c, GenGraph& g)
{
    for (void* b : {(void*)g.mum, (void*)g.p, (void*)g.qb, (void*)g.plan, (void*)g.gen_at}) dev_free(c, b);
    g.mum = g.dad = nullptr;
    g.p = g.q = g.qb = g.qp = g.ends = nullptr;
    g.plan = nullptr;
    g.gen_at = nullptr;
}

static void gengraph_free(ev_ctx* c, GenGraph* g)
{
    if (!g) return;
    (void)sync(c->main);
    plan_blocks_free(c, *g);
    pop_blocks_free(c, *g);
    xo_blocks_free(c, *g);
    for (int i = 0; i < NB; i++) {
        if (g->pin[i]) (void)hipHostFree(g->pin[i]);
        if (g->done[i]) (void)hipEventDestroy(g->done[i]);
    }
    delete g;
}

void evolve_release(ev_ctx* c)
{
    gengraph_free(c, c->evolve);
    c->evolve = nullptr;
}

// Observed sizes of a host-driven plan's levels.
static std::vector<LevelSize> sizes_of(const Plan& pl)
{
    std::vector<LevelSize> v;
    for (const Level& L : pl.levels) {
        LevelSize s;
        s.n = L.n_run;
        s.n_seg = L.n_seg;
        s.so = L.n_out;
        s.sf = L.n_frag;
        s.sc = L.n_codes;
        s.slab = L.slab_entries;
        s.tokens = L.tokens;
        v.push_back(s);
    }
    return v;
}

// ... and of a replayed generation's (its levels' counts, read back).
static std::vector<LevelSize> sizes_of(const GLevel* lv, uint32_t levels)
{
    std::vector<LevelSize> v;
    for (uint32_t l = 0; l < levels; l++) {
        LevelSize s;
        s.n = lv[l].n;
        s.n_seg = lv[l].n_seg;
        s.so = lv[l].so;
        s.sf = lv[l].sf;
        s.sc = lv[l].sc;
        s.slab = lv[l].slab_entries;
        s.tokens = lv[l].tokens;
        v.push_back(s);
    }
    return v;
}

// Capacities with room to grow: four times what was seen (twice for plans
// of over 2^24 tokens, whose buffers are large), with floors that keep small
// plans from re-capturing at every step, and one level more than seen (sized
// like the largest skeleton level).  Segments are bounded through the
// tokens and items, whatever segment length the sizes were seen with.
static std::vector<LevelSize> caps_from(const std::vector<LevelSize>& seen, uint32_t* levels)
{
    const uint64_t f = !seen.empty() && seen[0].tokens > (1ull << 24) ? 2 : 4;
    auto grow = [f](uint64_t v, uint64_t floor) { return std::max<uint64_t>(f * v, floor); };
    std::vector<LevelSize> caps;
    LevelSize hi;  // the largest skeleton level
    for (size_t l = 0; l < seen.size(); l++) {
        const LevelSize& s = seen[l];
        LevelSize k;
        k.n = grow(s.n, 64);
        k.tokens = grow(s.tokens, 1 << 16);
        k.so = grow(s.so, 256);
        k.sf = grow(s.sf, 4096);
        k.sc = grow(s.sc, 8192);
        k.slab = 0;
        caps.push_back(k);
        if (l > 0) {
            hi.n = std::max(hi.n, k.n);
            hi.tokens = std::max(hi.tokens, k.tokens);
            hi.so = std::max(hi.so, k.so);
            hi.sf = std::max(hi.sf, k.sf);
            hi.sc = std::max(hi.sc, k.sc);
        }
    }
    if (caps.empty()) caps.push_back(LevelSize{64, 0, 256, 4096, 8192, 0, 1 << 16});
    if (hi.n == 0) hi = caps[0];
    const size_t want = std::min<size_t>(caps.size() + 1, EV_MAX_LEVELS);
    while (caps.size() < want) caps.push_back(hi);
    *levels = (uint32_t)caps.size();
    return caps;
}

static bool near_caps(const std::vector<LevelSize>& seen, const std::vector<LevelSize>& caps, uint64_t slab_max)
{
    if (seen.size() >= caps.size()) return true;
    auto near = [](uint64_t v, uint64_t cap) { return v * 4 > cap * 3; };
    for (size_t l = 0; l < seen.size(); l++) {
        const LevelSize &s = seen[l], &k = caps[l];
        if (near(s.n, k.n) || near(s.n_seg, k.n_seg) || near(s.tokens, k.tokens) || near(s.so, k.so) ||
            near(s.sf, k.sf) || near(s.sc, k.sc) || near(s.slab, slab_max))
            return true;
    }
    return false;
}

template <typename T>
static ev_status g_alloc(ev_ctx* c, GenGraph& g, size_t count, T** out)
{
    void* b = nullptr;
    ev_status st = dev_alloc(c, std::max<size_t>(count, 1) * sizeof(T), &b);
    if (st != EV_OK) return st;
    g.blocks.push_back(b);
    *out = (T*)b;
    return EV_OK;
}

// The plan's buffers for capacities `caps` (the previous ones are freed).
static ev_status plan_blocks_make(ev_ctx* c, GenGraph& g, const std::vector<LevelSize>& caps_in, uint32_t levels,
                                  uint64_t slab_rows)
{
    plan_blocks_free(c, g);
    g.caps = caps_in;
    g.L = levels;
    g.n_max = g.nseg_max = 0;
    g.seg_len.assign(levels, 0);
    uint64_t sf_max = 0, rk_bytes = 0, rf_bytes = 0;
    for (uint32_t l = 0; l < levels; l++) {
        // each level's segment length, and its segments through its tokens
        // and items: a chunk of len tokens has at most 2 + len / seg_len
        const uint32_t seg_len = seg_len_for((int)l, g.caps[l].tokens);
        g.seg_len[l] = seg_len;
        g.caps[l].n_seg = std::max<uint64_t>(g.caps[l].n_seg, 2 * g.caps[l].n + g.caps[l].tokens / seg_len + 1);
        const std::vector<LevelSize>& caps = g.caps;
        g.n_max = std::max(g.n_max, caps[l].n);
        g.nseg_max = std::max(g.nseg_max, caps[l].n_seg);
        sf_max = std::max(sf_max, caps[l].sf);
        rk_bytes = std::max(rk_bytes, rec_kinds_stride(seg_len) * caps[l].n_seg + 64);
        rf_bytes = std::max(rf_bytes, rec_frags_stride(seg_len) * caps[l].n_seg + 64);
    }
    if (g.n_max > 0xFFFFFFF0ull || g.nseg_max > 0xFFFFFFF0ull) return fail(EV_ECAP, "ev_evolve: plan too large");
    g.record = g.use_record && rk_bytes + rf_bytes <= G_RECORD_MAX;
    g.slab_max = slab_rows;
    const std::vector<LevelSize>& caps = g.caps;
    const size_t M = (size_t)g.M;
    ev_status st = EV_OK;
    auto A = [&](auto count, auto** out) {
        if (st == EV_OK) st = g_alloc(c, g, (size_t)count, out);
    };
    A(M, &g.tr);
    A(M, &g.tl);
    A(levels, &g.gls);
    A(levels, &g.d_caps);
    A(1, &g.st);
    A(2 * M, &g.fin);
    A(G_N_ERR, &g.err);
    A(2 * (size_t)levels, &g.counters);
    A(g.n_max, &g.ch);
    A(g.n_max, &g.cseg);
    A(g.nseg_max, &g.seg);
    A(g.nseg_max, &g.fn);
    A(g.nseg_max, &g.sst);
    A(g.nseg_max, &g.cnt);
    A(g.n_max, &g.stat);
    A(3 * g.n_max, &g.loc);
    A(g.n_max, &g.inend);
    A(M + 1, &g.sum);
    A(M, &g.tb);
    A(g.n_max, &g.cb);
    A(g.n_max, &g.fe);
    A(g.nseg_max, &g.scode);
    A(g.nseg_max, &g.sfrag);
    A(EV_LEN_BUCKETS, &g.cursor);
    if (g.record) {
        A(rk_bytes, &g.rk);
        A(rf_bytes, &g.rf);
        A(g.nseg_max, &g.rec);
    }
    A(sf_max + 64, &g.skel[0]);
    A(sf_max + 64, &g.skel[1]);
    for (uint32_t l = 0; l < levels && st == EV_OK; l++) {
        uint32_t* cd = nullptr;
        RunChunk* rn = nullptr;
        float* rs = nullptr;
        A(caps[l].sc + 128, &cd);  // 512 bytes of the readers' tail after the codes
        A(caps[l].n, &rn);
        A((caps[l].so + EV_RING) * (uint64_t)g.N, &rs);
        g.codes.push_back(cd);
        g.run.push_back(rn);
        g.res.push_back(rs + (size_t)EV_RING * g.N);
    }
    // the spill slabs: as many waves as c->grid_run, each with slab_rows
    // rows of 64 lanes
    g.grid = (uint32_t)g.run_grid;
    if (slab_rows) A((size_t)g.grid * slab_rows * 64, &g.slab);
    if (st != EV_OK) {
        plan_blocks_free(c, g);
        return st;
    }
    std::vector<GCap> dc(levels);
    for (uint32_t l = 0; l < levels; l++)
        dc[l] = GCap{caps[l].n, caps[l].n_seg, caps[l].so, caps[l].sf, caps[l].sc, (uint32_t)slab_rows, 0};
    return put(c->main, g.d_caps, dc.data(), dc.size() * sizeof(GCap));
}

// Room for a population of `bytes`: four times as much while small (fewer
// re-captures as trees grow), twice from 16 MB on.
static uint64_t pop_room(uint64_t bytes) { return (bytes < (1ull << 24) ? 4 : 2) * bytes; }

// The population's buffers for bytes_cap bytes each (with padding),
// the current population (buffer `keep` of the old ones, `total` bytes)
// copied over.  The caller has dropped the graphs (they name the old ones).
static ev_status pop_blocks_make(ev_ctx* c, GenGraph& g, uint64_t bytes_cap, int keep, uint64_t total)
{
    const size_t M = (size_t)std::max(1, g.M);
    GenGraph n;
    ev_status st = EV_OK;
    for (int i = 0; i < NB && st == EV_OK; i++) {
        if ((st = dev_alloc(c, bytes_cap, (void**)&n.bytes[i])) == EV_OK &&
            (st = dev_alloc(c, (2 * M + 6) * 8, (void**)&n.off[i])) == EV_OK)
            st = dev_alloc(c, M * 4, (void**)&n.fit[i]);
    }
    if (st != EV_OK) {
        pop_blocks_free(c, n);
        return st;
    }
    hipStream_t s = c->stream;
    if (keep >= 0 && g.bytes[keep]) {
        HIPCHK(hipMemcpyAsync(n.bytes[keep], g.bytes[keep], total + EV_POP_PAD, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(n.off[keep], g.off[keep], (M + 1) * 8, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(n.fit[keep], g.fit[keep], M * 4, hipMemcpyDeviceToDevice, s));
    }
    pop_blocks_free(c, g);  // reused by later work on this stream only, after the copies
    for (int i = 0; i < NB; i++) {
        g.bytes[i] = n.bytes[i];
        g.off[i] = n.off[i];
        g.fit[i] = n.fit[i];
    }
    g.bytes_cap = bytes_cap;
    g.pieces_cap = bytes_cap / 4096 + M + 1;
    return EV_OK;
}

static ev_status xo_blocks_make(ev_ctx* c, GenGraph& g)
{
    const size_t M = (size_t)std::max(1, g.M);
    ev_status st = dev_alloc(c, M * 8, (void**)&g.mum);
    if (st == EV_OK) {
        g.dad = g.mum + M;
        st = dev_alloc(c, M * 16, (void**)&g.p);
    }
    if (st == EV_OK) {
        g.q = g.p + M;
        st = dev_alloc(c, M * 48, (void**)&g.qb);
    }
    if (st == EV_OK) {
        g.qp = g.qb + 2 * M;
        g.ends = g.qp + 2 * M;
        st = dev_alloc(c, M * sizeof(XoPlan), (void**)&g.plan);
    }
    if (st == EV_OK) st = dev_alloc(c, 8, (void**)&g.gen_at);
    if (st != EV_OK) xo_blocks_free(c, g);
    return st;
}

// Queue one generation, parents in buffer a and children in the next, over
// the first nl plan levels (a generation that needs more voids itself).
static hipError_t enqueue_generation(ev_ctx* c, GenGraph& g, int a, uint32_t nl, hipStream_t s)
{
    const int b = nxt(a);
    const uint32_t M = (uint32_t)g.M;
    const uint32_t n_cb = (uint32_t)((g.N + 63) / 64);
    hipError_t e = hipSuccess;
    auto E = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    E(launch_select(g.fit[a], g.off[a], M, g.k, g.seed, 0, g.mum, g.dad, g.p, g.q, s, g.gen_at));
    E(launch_xo_query(g.off[a], g.off[a], g.mum, g.dad, g.p, g.q, M, g.qb, g.qp, s));
    E(launch_subtree_end(g.bytes[a], g.qb, g.qp, 2 * M, g.ends, s));
    E(launch_xo_plan(g.off[a], g.off[a], g.mum, g.dad, g.p, g.q, g.ends, M, g.cap, g.plan, g.off[b], s));
    E(launch_g_init(g.off[b], M, g.tr, g.bytes_cap, (uint32_t)EV_POP_PAD, g.pieces_cap, g.st, g.counters, 2 * g.L,
                    s));
    E(launch_xo_copy(g.bytes[a], g.bytes[a], g.plan, g.off[b], M, g.pieces_cap, g.bytes[b], nullptr,
                     (uint32_t)EV_POP_PAD, s, &g.st->poison));
    uint64_t* cloc = g.loc;
    uint64_t* oloc = g.loc + g.n_max;
    uint64_t* floc = g.loc + 2 * g.n_max;
    for (uint32_t l = 0; l < nl; l++) {
        const uint64_t C = l == 0 ? g.C0 : g.C1;
        const uint32_t seg_len = g.seg_len[l], head = seg_len / 4;
        const LevelSize& k = g.caps[l];
        const uint32_t kn = (uint32_t)k.n, kns = (uint32_t)k.n_seg;
        GLevel* gl = g.gls + l;
        const uint8_t* seq = l == 0 ? g.bytes[b] : g.skel[l & 1];
        uint8_t* next = g.skel[(l + 1) & 1];
        E(launch_g_begin(g.tr, M, g.gls, l, g.d_caps, C, seg_len, head, g.record ? 1u : 0u, g.tl, g.cursor, g.st,
                         s));
        E(launch_plan_chunks(g.tl, M, seg_len, head, g.ch, g.cseg, l == 0 ? g.err : nullptr, G_N_ERR, s, gl));
        E(launch_seg_build(g.ch, g.cseg, kn, seg_len, head, g.seg, s, gl));
        E(launch_seg_fn(seq, g.seg, kns, g.fn, l ? 1u : 0u, 0u, s, gl));
        E(launch_seg_scan(g.cseg, kn, g.fn, g.sst, g.stat, s, gl));
        E(launch_seg_count(seq, g.seg, kns, g.sst, g.cnt, g.record ? g.rk : nullptr, g.record ? g.rf : nullptr,
                           g.record ? g.rec : nullptr, &gl->record_ovf, seg_len, s, gl));
        E(launch_seg_chunk(g.cseg, kn, g.cnt, g.stat, nullptr, nullptr, nullptr, nullptr, s, gl));
        E(launch_plan_trees(g.tl, M, g.stat, l, 0, cloc, oloc, floc, g.inend, g.sum, s, gl));
        E(launch_g_end(g.tr, g.gls, l, g.d_caps, nl, g.tl, g.sum, g.tb, g.fin, g.st, s));
        E(launch_plan_items(g.ch, kn, g.tb, cloc, oloc, floc, g.inend, g.cursor, g.cb, g.fe, g.run[l], nullptr,
                            g.codes[l], next, s, gl));
        E(launch_seg_chunk(g.cseg, kn, g.cnt, g.stat, g.cb, g.fe, g.scode, g.sfrag, s, gl));
        // placement of the recording (a recording that overflowed voids the
        // generation), or emission and validation when the level is too
        // large to record
        if (g.record) {
            E(launch_seg_place(g.seg, kns, g.cnt, g.rec, g.sst, g.scode, g.sfrag, g.rk, g.rf, g.codes[l], k.sc, next,
                               k.sf, 0, g.err + 2 * l, seg_len, s, gl));
        } else {
            E(launch_seg_emit(seq, g.seg, kns, g.sst, g.scode, g.sfrag, next, g.codes[l], s, gl));
            E(launch_seg_check(g.codes[l], g.seg, kns, g.sst, g.scode, g.cnt, 0, g.err + 2 * l, s, gl));
        }
    }
    for (uint32_t l = 0; l < nl; l++) {
        RunArgs r{};
        r.codes = g.codes[l];
        r.chunks = g.run[l];
        r.n_items = (uint32_t)g.caps[l].n * n_cb;
        r.n_cb = n_cb;
        r.counter = g.counters + g.L + l;
        r.x = g.d_x;
        r.N = g.N;
        r.rowb = (uint32_t)g.N * 4u;
        r.in_res = l ? g.res[l - 1] : nullptr;
        r.out_res = g.res[l];
        r.slab = g.slab;
        r.slab_entries = g.slab_max;
        r.flag = c->d_flag;
        r.refs = l ? 1u : 0u;
        r.verdict = g.err + 2 * l;
        r.gl = g.gls + l;
        E(launch_run(r, (uint32_t)std::min<uint64_t>(g.grid, (uint64_t)r.n_items), s));
    }
    FitArgs fa = {};
    for (uint32_t l = 0; l < nl; l++) fa.res[l] = g.res[l];
    fa.n_levels = nl;
    fa.fin = g.fin;
    fa.y = g.d_y;
    fa.N = g.N;
    fa.M = M;
    fa.fit = g.fit[b];
    fa.gl = g.gls;
    E(launch_fitness(fa, s));
    E(launch_g_finish(g.st, g.gls, nl, g.err, g.fit[b], M, g.gen_at, g.h_st[a], g.h_lv[a], g.h_fit[a], s));
    return e;
}

// Capture the generation with parents in buffer a, over all levels or
// (short) all but the last.
static ev_status capture(ev_ctx* c, GenGraph& g, int a, bool short_form)
{
    hipStream_t s = c->stream;
    ev_status st = sync(c->main);  // staged uploads have landed; nothing else is queued
    if (st != EV_OK) return st;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const hipError_t e = enqueue_generation(c, g, a, short_form ? g.L - 1 : g.L, s);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return hip_fail(e != hipSuccess ? e : e2, "capturing a generation");
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e3, "hipGraphInstantiate");
    }
    (short_form ? g.graph_s : g.graph)[a] = graph;
    (short_form ? g.exec_s : g.exec)[a] = ex;
    return EV_OK;
}

// One generation on the host-driven path from buffer a into the next (the
// same kernels and draws as the graph's): its children's plan sizes and
// capped count, their fitness in h_fit[a].  The population buffers grow
// when the children need it.
static ev_status host_generation(ev_ctx* c, GenGraph& g, int a, uint64_t gen, std::vector<LevelSize>* seen,
                                 int32_t* capped, uint64_t* nodes)
{
    Exec& x = c->main;
    hipStream_t s = c->stream;
    const int b = nxt(a);
    const int32_t M = g.M;
    std::vector<uint64_t> h_off((size_t)M + 1);
    ev_status st = get(x, h_off.data(), g.off[a], h_off.size() * 8);
    if (st == EV_OK) st = sync(x);
    if (st != EV_OK) return st;
    // the parents, as a population that owns nothing
    Pop view;
    view.d_bytes = g.bytes[a];
    view.d_off = g.off[a];
    view.h_off = h_off;
    view.M = M;
    view.total = h_off.back();
    HIPCHK(launch_select(g.fit[a], g.off[a], (uint32_t)M, g.k, g.seed, gen, g.mum, g.dad, g.p, g.q, s));
    Pop* kids = nullptr;
    st = crossover_build_dev(c, x, &view, &view, g.mum, g.dad, g.p, g.q, M, g.cap, &kids, capped, false);
    if (st != EV_OK) return st;
    if ((st = eval_enqueue(c, x, kids, g.table, kids->d_fit, nullptr, false, nullptr)) != EV_OK ||
        (st = get(x, g.h_fit[a], kids->d_fit, (size_t)M * 4)) != EV_OK || (st = sync(x)) != EV_OK) {
        pop_free(c, kids);
        return st;
    }
    if (kids->total + EV_POP_PAD > g.bytes_cap) {
        graphs_drop(g);
        // the parents are done with: nothing to keep
        if ((st = pop_blocks_make(c, g, pop_room(kids->total + EV_POP_PAD), -1, 0)) != EV_OK) {
            pop_free(c, kids);
            return st;
        }
    }
    HIPCHK(hipMemcpyAsync(g.bytes[b], kids->d_bytes, kids->total + EV_POP_PAD, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(g.off[b], kids->d_off, ((size_t)M + 1) * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(g.fit[b], kids->d_fit, (size_t)M * 4, hipMemcpyDeviceToDevice, s));
    *seen = sizes_of(kids->plan);
    *nodes = kids->total;
    const uint64_t next = gen + 1;
    if ((st = put(x, g.gen_at, &next, 8)) == EV_OK) st = sync(x);
    pop_free(c, kids);
    return st;
}

// New plan buffers (and, at the next replay, graphs) for sizes `seen`.
static ev_status replan(ev_ctx* c, GenGraph& g, const std::vector<LevelSize>& seen, bool tight)
{
    uint32_t levels = 0;
    std::vector<LevelSize> caps;
    uint64_t slab = 0;
    for (const LevelSize& l : seen) slab = std::max(slab, l.slab);
    if (tight) {
        // exactly what was seen (tests of the fallback)
        caps = seen;
        if (caps.empty()) caps.push_back(LevelSize{1, 1, 1, 1, 1, 0});
        levels = (uint32_t)caps.size();
    } else {
        caps = caps_from(seen, &levels);
        slab = std::max<uint64_t>(2 * slab, 64 + EV_VHALF);
    }
    const ev_status st = sync(c->main);  // the old buffers are idle
    if (st != EV_OK) return st;
    return plan_blocks_make(c, g, caps, levels, slab);
}

}  // namespace ev

using namespace ev;

extern "C" ev_status ev_evolve(ev_ctx* c, ev_pop parents, const float* fitness, int32_t table, uint64_t seed,
                               uint64_t gen0, int32_t n_gen, int32_t tournament, uint64_t size_cap, uint32_t flags,
                               ev_pop* out, float* fit_history, int32_t* capped_history, ev_evolve_report* report)
{
    if (!c || !out || n_gen < 0 || tournament < 1) return fail(EV_EINVAL, "ev_evolve: bad arguments");
    Pop* P = pop_get(c, parents);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", parents);
    if (!fitness && !P->fit_valid) return fail(EV_EINVAL, "ev_evolve: parents have no fitness yet");
    CaseTable ct;
    if (!table_get(c, table, &ct)) return fail(EV_EINVAL, "no case table %d", table);
    HIPCHK(hipSetDevice(c->device));
    *out = 0;
    ev_evolve_report rep = {};
    const auto t0 = std::chrono::steady_clock::now();
    auto ms_since = [](std::chrono::steady_clock::time_point a) {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
    };
    Exec& x = c->main;
    hipStream_t s = c->stream;
    const int32_t M = P->M;
    if ((flags & EV_EVOLVE_LEAN) && M > 0) {
        ev_status st = evolve_lean(c, P, fitness, table, seed, gen0, n_gen, tournament, size_cap, out, fit_history,
                                   capped_history, &rep);
        rep.ms = ms_since(t0);
        if (report) *report = rep;
        return st;
    }
    const bool graphs = !(flags & EV_EVOLVE_NO_GRAPH) && c->use_run && c->n_consts == 0 && M > 0;
    ev_status st = EV_OK;

    if (!graphs) {
        // the plain form: every generation on the host-driven path
        Pop* cur = P;
        const size_t m = (size_t)std::max(1, M);
        float* d_fit = nullptr;
        void* d_sel = nullptr;
        if ((st = dev_alloc(c, m * 4, (void**)&d_fit)) != EV_OK) return st;
        if ((st = dev_alloc(c, m * 24, &d_sel)) != EV_OK) {
            dev_free(c, d_fit);
            return st;
        }
        if (M) HIPCHK(hipMemcpyAsync(d_fit, fitness ? fitness : P->d_fit, (size_t)M * 4, hipMemcpyDeviceToDevice, s));
        int32_t* d_mum = (int32_t*)d_sel;
        int32_t* d_dad = d_mum + m;
        uint64_t* d_p = (uint64_t*)((char*)d_sel + m * 8);
        uint64_t* d_q = d_p + m;
        for (int32_t i = 0; i < n_gen && st == EV_OK; i++) {
            Pop* kids = nullptr;
            int32_t capped = 0;
            hipError_t e = launch_select(d_fit, cur->d_off, (uint32_t)M, tournament, seed, gen0 + (uint64_t)i, d_mum,
                                         d_dad, d_p, d_q, s);
            if (e != hipSuccess) {
                st = hip_fail(e, "selection");
                break;
            }
            if ((st = crossover_build_dev(c, x, cur, cur, d_mum, d_dad, d_p, d_q, M, size_cap, &kids, &capped)) !=
                EV_OK)
                break;
            st = eval_enqueue(c, x, kids, table, kids->d_fit, nullptr, false, nullptr);
            if (st == EV_OK && M) {
                e = hipMemcpyAsync(d_fit, kids->d_fit, (size_t)M * 4, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) st = hip_fail(e, "hipMemcpyAsync");
            }
            if (st == EV_OK && fit_history) st = get(x, fit_history + (size_t)i * M, kids->d_fit, (size_t)M * 4);
            if (st == EV_OK) st = sync(x);
            if (st != EV_OK) {
                pop_free(c, kids);
                break;
            }
            kids->fit_valid = true;
            if (capped_history) capped_history[i] = capped;
            rep.capped += (uint64_t)capped;
            rep.nodes += kids->total;
            rep.generations++;
            if (cur != P) pop_free(c, cur);
            cur = kids;
        }
        if (st == EV_OK && cur == P) {
            // no generation: a copy of the parents
            uint8_t* d = nullptr;
            Pop* Q = nullptr;
            if ((st = dev_alloc(c, P->total + EV_POP_PAD, (void**)&d)) == EV_OK) {
                const hipError_t e = hipMemcpyAsync(d, P->d_bytes, P->total + EV_POP_PAD, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) {
                    dev_free(c, d);
                    st = hip_fail(e, "hipMemcpyAsync");
                } else {
                    st = pop_build(c, x, d, P->h_off, &Q, nullptr);
                }
            }
            if (st == EV_OK && M) {
                const hipError_t e = hipMemcpyAsync(Q->d_fit, d_fit, (size_t)M * 4, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) st = hip_fail(e, "hipMemcpyAsync");
            }
            if (st == EV_OK) st = sync(x);
            if (st == EV_OK) {
                Q->fit_valid = true;
                cur = Q;
            } else if (Q) {
                pop_free(c, Q);
            }
        }
        (void)sync(x);
        dev_free(c, d_sel);
        dev_free(c, d_fit);
        if (st != EV_OK) {
            if (cur != P) pop_free(c, cur);
            return st;
        }
        rep.ms = ms_since(t0);
        if (report) *report = rep;
        *out = pop_register(c, cur);
        return EV_OK;
    }

    // the graphs of an earlier call serve if they were made for the same loop
    GenGraph* g = c->evolve;
    const bool tight = (flags & EV_EVOLVE_TEST_TIGHT) != 0;
    const uint32_t C1 = c->chunk_hi ? c->chunk_hi : 2 * c->chunk;
    if (g && (g->M != M || g->table != table || g->N != ct.N || g->d_x != ct.d_x || g->k != tournament ||
              g->seed != seed || g->cap != size_cap || g->C0 != c->chunk || g->C1 != C1 ||
              g->run_grid != c->grid_run || g->use_record != c->use_record || tight)) {
        evolve_release(c);
        g = nullptr;
    }
    if (!g) {
        g = new GenGraph();
        g->device = c->device;
        g->M = M;
        g->table = table;
        g->N = ct.N;
        g->k = tournament;
        g->seed = seed;
        g->cap = size_cap;
        g->C0 = c->chunk;
        g->C1 = C1;
        g->run_grid = c->grid_run;
        g->use_record = c->use_record;
        g->d_x = ct.d_x;
        g->d_y = ct.d_y;
        const size_t pin_bytes = 256 + EV_MAX_LEVELS * sizeof(GLevel) + (size_t)M * 4;
        for (int i = 0; i < NB; i++) {
            hipError_t e = hipHostMalloc((void**)&g->pin[i], pin_bytes, hipHostMallocCoherent);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&g->done[i], hipEventDisableTiming);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                gengraph_free(c, g);
                return fail(EV_ENOMEM, "ev_evolve: pinned status or event: %s", hipGetErrorString(e));
            }
            g->h_st[i] = (GStatus*)g->pin[i];
            g->h_lv[i] = (GLevel*)(g->pin[i] + 256);
            g->h_fit[i] = (float*)(g->pin[i] + 256 + EV_MAX_LEVELS * sizeof(GLevel));
        }
        if ((st = xo_blocks_make(c, *g)) != EV_OK) {
            gengraph_free(c, g);
            return st;
        }
        c->evolve = g;
    }
    GenGraph& G = *g;
    // the parents into buffer 0
    if (!G.bytes[0] || P->total + EV_POP_PAD > G.bytes_cap * 3 / 4) {
        if ((st = sync(x)) != EV_OK) return st;
        graphs_drop(G);
        if ((st = pop_blocks_make(c, G, pop_room(P->total + EV_POP_PAD), -1, 0)) != EV_OK) return st;
    }
    G.cur = 0;
    HIPCHK(hipMemcpyAsync(G.bytes[0], P->d_bytes, P->total + EV_POP_PAD, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(G.off[0], P->d_off, ((size_t)M + 1) * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(G.fit[0], fitness ? fitness : P->d_fit, (size_t)M * 4, hipMemcpyDeviceToDevice, s));
    st = put(x, G.gen_at, &gen0, 8);
    if (st == EV_OK && G.blocks.empty()) st = replan(c, G, sizes_of(P->plan), tight);
    if (st == EV_OK) st = sync(x);
    if (st != EV_OK) return st;

    // every buffer's graph, captured while nothing else is queued
    auto capture_timed = [&](int k, bool sf) -> ev_status {
        const auto tc = std::chrono::steady_clock::now();
        const ev_status r = capture(c, G, k, sf);
        if (r != EV_OK) return r;
        rep.captures++;
        rep.ms_capture += ms_since(tc);
        return EV_OK;
    };
    auto ensure_graphs = [&]() -> ev_status {
        for (int k = 0; k < NB; k++) {
            if (G.exec[k]) continue;
            const ev_status r = capture_timed(k, false);
            if (r != EV_OK) return r;
        }
        return EV_OK;
    };
    // The short graph serves while the last SHORT_AFTER generations read
    // all used fewer than L levels; a generation that needs the last level
    // voids itself and is redone, and the full graph serves again.  Short
    // graphs are captured when first needed after a re-capture (the capture
    // waits for the generation in flight).
    constexpr int SHORT_AFTER = 2;
    int fits_short = 0;
    auto launch = [&](int a) -> ev_status {
        const bool sf = fits_short >= SHORT_AFTER && G.L >= 2;
        if (sf && !G.exec_s[a]) {
            const ev_status r = capture_timed(a, true);
            if (r != EV_OK) return r;
        }
        HIPCHK(hipGraphLaunch(sf ? G.exec_s[a] : G.exec[a], s));
        HIPCHK(hipEventRecord(G.done[a], s));
        return EV_OK;
    };
    // generation i + 1, launched before generation i's status was read, is
    // thrown away: the device's generation counter is set back to it
    bool ahead = false;
    auto discard_ahead = [&](uint64_t next_gen) -> ev_status {
        if (!ahead) return EV_OK;
        ahead = false;
        ev_status r = sync(x);
        if (r == EV_OK) r = put(x, G.gen_at, &next_gen, 8);
        if (r == EV_OK) r = sync(x);
        return r;
    };
    if (n_gen > 0) {
        if ((st = ensure_graphs()) != EV_OK) return st;
        if ((st = launch(G.cur)) != EV_OK) return st;
    }
    for (int32_t i = 0; i < n_gen; i++) {
        const int a = G.cur, b = nxt(a);
        const uint64_t gen = gen0 + (uint64_t)i;
        // generation i was launched (by the iteration before, or above);
        // launch i + 1 from its children before looking at its status
        if (i + 1 < n_gen && !ahead && G.exec[b]) {
            if ((st = launch(b)) != EV_OK) return st;
            ahead = true;
        }
        HIPCHK(hipEventSynchronize(G.done[a]));
        const GStatus gs = *G.h_st[a];
        std::vector<LevelSize> seen;
        int32_t capped = 0;
        uint64_t nodes = gs.child_bytes;
        bool regraph = false;
        const uint32_t L_read = G.L;  // the capacities generation i ran under
        if (gs.poison) {
            // void: done again on the host-driven path, then new capacities
            if ((st = discard_ahead(gen + 1)) != EV_OK) return st;
            if ((st = host_generation(c, G, a, gen, &seen, &capped, &nodes)) != EV_OK) return st;
            rep.fallbacks++;
            if ((st = replan(c, G, seen, tight)) != EV_OK) return st;
            regraph = true;
        } else {
            capped = (int32_t)gs.capped;
            rep.replayed++;
            seen = sizes_of(G.h_lv[a], gs.levels);
            if (gs.child_bytes + EV_POP_PAD > G.bytes_cap * 3 / 4) {
                // larger population buffers, keeping the children (the
                // generation after them runs again on the new buffers)
                if ((st = discard_ahead(gen + 1)) != EV_OK) return st;
                graphs_drop(G);
                if ((st = pop_blocks_make(c, G, pop_room(gs.child_bytes + EV_POP_PAD), b, gs.child_bytes)) != EV_OK)
                    return st;
                regraph = true;
            }
            if (!tight && near_caps(seen, G.caps, G.slab_max)) {
                // the generation ahead (if any) finishes under the old
                // capacities; its status is read like any other
                if ((st = replan(c, G, seen, false)) != EV_OK) return st;
                regraph = true;
            }
        }
        // how many generations in a row fit the short graph (re-capture
        // starts the count again)
        const uint32_t used = gs.poison ? (uint32_t)seen.size() : gs.levels;
        fits_short = (regraph || used + 1 > L_read) ? 0 : fits_short + 1;
        if (fit_history) std::memcpy(fit_history + (size_t)i * M, G.h_fit[a], (size_t)M * 4);
        if (capped_history) capped_history[i] = capped;
        rep.capped += (uint64_t)capped;
        rep.nodes += nodes;
        rep.generations++;
        G.cur = b;
        if (i + 1 < n_gen) {
            if (regraph && (st = ensure_graphs()) != EV_OK) return st;
            if (!ahead && (st = launch(b)) != EV_OK) return st;
        }
        ahead = false;
    }
    if ((st = sync(x)) != EV_OK) return st;

    // the last generation as a population of its own (planned afresh)
    std::vector<uint64_t> h_off((size_t)M + 1);
    if ((st = get(x, h_off.data(), G.off[G.cur], h_off.size() * 8)) != EV_OK || (st = sync(x)) != EV_OK) return st;
    uint8_t* d = nullptr;
    if ((st = dev_alloc(c, h_off.back() + EV_POP_PAD, (void**)&d)) != EV_OK) return st;
    HIPCHK(hipMemcpyAsync(d, G.bytes[G.cur], h_off.back() + EV_POP_PAD, hipMemcpyDeviceToDevice, s));
    Pop* Q = nullptr;
    if ((st = pop_build(c, x, d, h_off, &Q, nullptr)) != EV_OK) return st;
    if (M) HIPCHK(hipMemcpyAsync(Q->d_fit, G.fit[G.cur], (size_t)M * 4, hipMemcpyDeviceToDevice, s));
    if ((st = sync(x)) != EV_OK) {
        pop_free(c, Q);
        return st;
    }
    Q->fit_valid = true;
    rep.ms = ms_since(t0);
    if (report) *report = rep;
    *out = pop_register(c, Q);
    return EV_OK;
}
