// Host runtime of libev: contexts, device populations, the split plan,
// evaluation, crossover and generations.  See include/ev.h for the ABI.
#include "ev_runtime.h"

#include <algorithm>
#include <tuple>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>

namespace ev {

thread_local std::string g_err;

ev_status fail(ev_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

ev_status hip_fail(hipError_t e, const char* what)
{
    return fail(EV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------- memory

// Device memory goes through a per-context cache: freed blocks are kept in
// size classes and handed out again, so the plan and crossover temporaries
// of every generation cost no hipMalloc/hipFree (hipFree synchronizes the
// device).  A block goes back to the cache while work that uses it may
// still be queued on the freeing thread's stream; the cache (ev_cache.h)
// hands it out again at once on that stream, whose later work is ordered
// after it, but on another stream only after the freeing stream has been
// waited for.  The budget bounds live bytes; when live plus cached bytes
// would exceed what the device can hold, the cached blocks idle the longest
// are released first.
// Powers of two up to 256 MiB, then steps of 2^(1/4) (rounded to 2 MiB): a
// large block serves requests from about 84% of its size up, so the large
// buffers of successive generations, whose sizes wander by a few percent,
// keep finding one in the cache (a fresh multi-GB hipMalloc on a nearly
// full device has taken over a second).
static size_t size_class(size_t bytes)
{
    if (bytes <= 256) return 256;
    if (bytes <= (256ull << 20)) {
        size_t c = 256;
        while (c < bytes) c <<= 1;
        return c;
    }
    const size_t g = 2ull << 20;
    double c = (double)(256ull << 20);
    size_t cls = 256ull << 20;
    while (cls < bytes) {
        c *= 1.189207115002721;  // 2^(1/4)
        cls = ((size_t)c + g - 1) / g * g;
    }
    return cls;
}

static thread_local Exec* tl_exec = nullptr;

ExecScope::ExecScope(Exec* x) : prev(tl_exec) { tl_exec = x; }
ExecScope::~ExecScope() { tl_exec = prev; }

Exec* current_exec(ev_ctx* c) { return tl_exec ? tl_exec : &c->main; }

bool table_get(ev_ctx* c, int32_t table, CaseTable* out)
{
    std::lock_guard<std::mutex> g(c->pop_mu);
    if (table < 0 || table >= (int32_t)c->tables.size()) return false;
    *out = c->tables[(size_t)table];
    return true;
}

// Hand cached blocks back: to the caller's allocator once every stream of
// the device has finished with them (hipFree waits by itself).
static void blocks_free(ev_ctx* c, const std::vector<std::pair<void*, size_t>>& blocks)
{
    if (blocks.empty()) return;
    if (c->ext.alloc) (void)hipDeviceSynchronize();
    for (auto& b : blocks) {
        if (c->ext.alloc)
            c->ext.free(b.first, c->ext.user);
        else
            (void)hipFree(b.first);
    }
}

static hipError_t block_alloc(ev_ctx* c, void** out, size_t bytes)
{
    if (!c->ext.alloc) return hipMalloc(out, bytes);
    *out = c->ext.alloc(bytes, c->ext.user);
    return *out ? hipSuccess : hipErrorOutOfMemory;
}

ev_status dev_alloc(ev_ctx* c, size_t bytes, void** out)
{
    *out = nullptr;
    const size_t cls = size_class(bytes);
    const StreamClock* clk = &current_exec(c)->clock;
    std::vector<std::pair<void*, size_t>> release;
    {
        std::lock_guard<std::mutex> g(c->mem_mu);
        if (c->budget && c->in_use + cls > c->budget)
            return fail(EV_ENOMEM, "memory budget exceeded (%zu + %zu > %zu bytes)", (size_t)c->in_use, cls,
                        (size_t)c->budget);
        // the same size class, or for a large request up to a class a
        // quarter larger, within the budget
        size_t hi = cls + (cls >= (256ull << 20) ? cls / 4 : 0);
        if (c->budget) hi = std::min<size_t>(hi, std::max<size_t>(cls, c->budget - c->in_use));
        size_t got = 0;
        if ((*out = c->cache.take(cls, hi, clk, &got)) != nullptr) {
            c->in_use += got;
            c->sizes[*out] = got;
            return EV_OK;
        }
        // Live and cached blocks together stay below the device's free
        // memory: the driver accepts allocations beyond it and then moves
        // buffers out of HBM while kernels use them.
        if (c->in_use + c->cache.bytes() + cls > c->hold_limit)
            release = c->cache.evict_oldest(c->in_use + c->cache.bytes() + cls - c->hold_limit);
        if (c->in_use + cls > c->hold_limit) {
            // not even with an empty cache
            blocks_free(c, release);
            return fail(EV_ENOMEM, "device memory exhausted (%zu + %zu > %zu bytes held)", (size_t)c->in_use, cls,
                        (size_t)c->hold_limit);
        }
        c->in_use += cls;
    }
    blocks_free(c, release);
    hipError_t e = block_alloc(c, out, cls);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        dev_cache_release(c);
        e = block_alloc(c, out, cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            std::lock_guard<std::mutex> g(c->mem_mu);
            c->in_use -= cls;
            *out = nullptr;
            return fail(EV_ENOMEM, "hipMalloc(%zu): %s", cls, hipGetErrorString(e));
        }
    }
    std::lock_guard<std::mutex> g(c->mem_mu);
    c->sizes[*out] = cls;
    return EV_OK;
}

void dev_free(ev_ctx* c, void* p)
{
    if (!p) return;
    const StreamClock* clk = &current_exec(c)->clock;
    std::lock_guard<std::mutex> g(c->mem_mu);
    auto it = c->sizes.find(p);
    if (it == c->sizes.end()) return;
    const size_t cls = it->second;
    c->sizes.erase(it);
    c->in_use -= cls;
    c->cache.put(p, cls, clk);
}

void dev_cache_release(ev_ctx* c)
{
    std::vector<std::pair<void*, size_t>> release;
    {
        std::lock_guard<std::mutex> g(c->mem_mu);
        release = c->cache.evict_all();
    }
    blocks_free(c, release);
}

// ------------------------------------------------------------- plans

void plan_free(ev_ctx* c, Plan& pl)
{
    for (auto& L : pl.levels) {
        if (L.owned) dev_free(c, L.seq);
        dev_free(c, L.d_chunks);
        dev_free(c, L.codes);
        dev_free(c, L.d_run);
        dev_free(c, L.d_item_tree);
    }
    pl.levels.clear();
    dev_free(c, pl.d_need);
    pl.d_need = nullptr;
    pl.h_need.clear();
    pl.h_pos.clear();
    pl.fin_level.clear();
    pl.fin_slot.clear();
    dev_free(c, pl.d_fin);
    pl.d_fin = nullptr;
    dev_free(c, pl.d_err);
    pl.d_err = nullptr;
    pl.err_pending = false;
    for (void* q : {(void*)pl.l0_ch, (void*)pl.l0_stat, (void*)pl.l0_code, (void*)pl.l0_frag, (void*)pl.l0_tree})
        dev_free(c, q);
    pl.l0_ch = nullptr;
    pl.l0_stat = nullptr;
    pl.l0_code = pl.l0_frag = nullptr;
    pl.l0_tree = nullptr;
    pl.l0_n = 0;
}

ev_status plan_verdict(Pop* P)
{
    Plan& pl = P->plan;
    if (!pl.err_pending) return EV_OK;
    if (pl.h_err[0])  // stays pending: every later evaluation fails the same way
        return fail(EV_EDEVICE, "internal: malformed code stream at level %d (flags %u, segment %u)", pl.err_level,
                    pl.h_err[0], pl.h_err[1]);
    pl.err_pending = false;
    return EV_OK;
}

void rescache_free(ev_ctx* c, ResCache& r)
{
    for (float* p : r.res) dev_free(c, p - (size_t)EV_RING * r.N);
    r.res.clear();

    dev_free(c, r.d_per_case);
    r.d_per_case = nullptr;
    dev_free(c, r.d_chain);
    r.d_chain = nullptr;
    r.chain_first = -1;
    r.chain_records = 0;
}

void pop_free(ev_ctx* c, Pop* P)
{
    if (!P) return;
    plan_free(c, P->plan);
    for (auto& kv : P->res) rescache_free(c, kv.second);
    P->res.clear();
    dev_free(c, P->d_bytes);
    dev_free(c, P->d_off);
    dev_free(c, P->d_fit);
    dev_free(c, P->d_hits);
    delete P;
}

// Largest recording of a level's codes and fragments (about 7.3 bytes per
// token in 64-token segments); larger levels count, then emit.  6 GiB takes
// the skeleton level of the largest populations (4.7e8 tokens) while their
// trees hold most of the device.
static constexpr uint64_t RECORD_MAX = (uint64_t)6 << 30;

// Recording buffer k of x (0: code kinds, 1: fragment tokens, 2: segment
// records), at least `bytes`.  It stays with x for later plans on x's
// stream, so that successive generations' plans find it at once: a fresh
// multi-GB block on a nearly full device costs milliseconds, and the cache
// may have given its last one back.  It grows by an eighth more than asked.
static ev_status ensure_rec(ev_ctx* c, Exec& x, int k, size_t bytes, void** out)
{
    if (bytes > x.rec_cap[k]) {
        // queued readers on x's stream finish before the block is used again
        dev_free(c, x.d_rec_buf[k]);
        x.d_rec_buf[k] = nullptr;
        x.rec_cap[k] = 0;
        const size_t want = bytes + bytes / 8;
        if (ev_status st = dev_alloc(c, want, &x.d_rec_buf[k])) return st;
        x.rec_cap[k] = want;
    }
    *out = x.d_rec_buf[k];
    return EV_OK;
}

static void release_rec(ev_ctx* c, Exec& x)
{
    for (int k = 0; k < 3; k++) {
        dev_free(c, x.d_rec_buf[k]);
        x.d_rec_buf[k] = nullptr;
        x.rec_cap[k] = 0;
    }
}

// Build the split plan of a population whose bytes are on the device.
// Level 0 is the trees themselves; each level's chunks produce the next
// level's skeleton until every tree is one value.  The host keeps what is
// per tree (its range at the level, its first input slot, where it ends);
// chunks, segments and their numbering are made on the device, and the host
// waits once per level, for the trees' totals that size the level's buffers.
// With reuse, level 0 takes over the chunks of each child's mum that its
// crossover left intact (their codes and skeleton fragments are copied) and
// plans only the tokens between them.
ev_status plan_build(ev_ctx* c, Exec& x, Pop* P, int32_t* bad_tree, bool defer_check, const ReuseSpec* reuse)
{
    hipStream_t s = x.stream;
    const int32_t M = P->M;
    const uint64_t C0 = c->chunk;
    // work-item size of the skeleton levels (by default twice level 0's: a
    // skeleton level has few tokens, and longer items there end more trees
    // a level earlier, which saves a level's fixed latency)
    const uint64_t C1 = c->chunk_hi ? c->chunk_hi : 2 * C0;
    Plan& pl = P->plan;
    pl.chunk = (uint32_t)C0;
    pl.D = c->lds_depth;
    pl.fin_level.assign(M, -1);
    pl.fin_slot.assign(M, 0);
    pl.chunks_total = 0;
    pl.slots_total = 0;
    pl.max_stack = 0;

    PlanScratch& W = x.plan;
    auto& rs = W.rs;
    auto& rl = W.rl;
    auto& prev_len = W.prev_len;
    auto& ref_base = W.ref_base;
    auto& active = W.active;
    rs.assign(M, 0);
    rl.assign(M, 0);
    prev_len.assign(M, 0);
    ref_base.assign(M, 0);
    active.assign(M, 1);
    for (int32_t t = 0; t < M; t++) {
        // a heap of trees (h_start) keeps each tree anywhere in the buffer
        rs[t] = P->h_start.empty() ? P->h_off[t] : P->h_start[t];
        rl[t] = P->h_off[t + 1] - P->h_off[t];
        if (rl[t] == 0) {
            if (bad_tree) *bad_tree = t;
            return fail(EV_EMALFORMED, "tree %d is empty", t);
        }
    }
    uint8_t* cur = P->d_bytes;
    uint64_t cur_len = P->total;  // bytes of the level's sequence
    bool cur_owned = false;
    int level = 0;
    // per-level device scratch: the level's trees, chunks and segments, the
    // segments' maps, starts, counts and positions, the chunks' numbering
    void *d_tl = nullptr, *d_ch = nullptr, *d_cseg = nullptr, *d_seg = nullptr, *d_fn = nullptr, *d_st = nullptr,
         *d_cnt = nullptr, *d_stat = nullptr, *d_loc = nullptr, *d_inend = nullptr, *d_sum = nullptr, *d_tb = nullptr,
         *d_cb = nullptr, *d_fe = nullptr, *d_scode = nullptr, *d_sfrag = nullptr, *d_err = nullptr, *d_tr = nullptr,
         *d_src = nullptr, *d_l0t = nullptr;
    // the recordings: x's own buffers (see ensure_rec), not freed here
    void *d_rk = nullptr, *d_rf = nullptr, *d_rec = nullptr;
    ev_status st = EV_OK;
    // also frees a skeleton not yet handed to a level
    auto cleanup = [&]() {
        for (void** p : {&d_tl, &d_ch, &d_cseg, &d_seg, &d_fn, &d_st, &d_cnt, &d_stat, &d_loc, &d_inend, &d_sum, &d_tb,
                         &d_cb, &d_fe, &d_scode, &d_sfrag, &d_err, &d_tr, &d_src, &d_l0t}) {
            dev_free(c, *p);
            *p = nullptr;
        }
        if (cur_owned) dev_free(c, cur);
        cur_owned = false;
    };
    auto realloc = [&](void** p, size_t bytes) -> ev_status {
        dev_free(c, *p);
        *p = nullptr;
        return dev_alloc(c, bytes, p);
    };
    // validator flags of every level, two words each (flags, first failing
    // segment), read back with the next level's totals or after the last
    // level, so that validation costs no wait of its own
    // (set by the first level's chunk kernel)
    constexpr int MAX_LEVELS = EV_MAX_LEVELS;
    constexpr uint32_t N_ERR = 2 * (MAX_LEVELS + 1);
    uint32_t verr[2] = {0, 0};
    if ((st = dev_alloc(c, N_ERR * 4, &d_err)) != EV_OK) {
        cleanup();
        return st;
    }
    auto code_error = [&](int lv, const uint32_t* e) -> ev_status {
        return fail(EV_EDEVICE, "internal: malformed code stream at level %d (flags %u, segment %u)", lv, e[0], e[1]);
    };
    auto& tl = W.tl;      // the level's trees
    auto& tsum = W.tsum;  // their totals
    auto& tb = W.tb;      // per tree id: its bases over the level's chunks
    tb.resize((size_t)std::max(1, M));
    uint32_t hist[EV_LEN_BUCKETS];
    // work items go biggest tree first, a tree's items together: a tree's
    // next level waits for all of its items at this one (the chained launch
    // starts it as soon as they are done), and long trees have the long
    // items, which the kernels' dynamic work queues want first.  A counting
    // sort on the tree length's bit count (the order inside a power of two
    // does not matter).
    auto bucket = [](uint64_t len) {
        return len >> 32 ? 0u : len ? (uint32_t)__builtin_clz((uint32_t)len) : 32u;
    };

    bool plan_run = c->use_run;  // items on the register-stack kernel (no constants seen)
    std::vector<uint32_t> need_all;  // per level and tree: work items (register-stack levels)
    std::vector<uint32_t> pos_all;   // and the place of the tree's first item (~0u: not known)
    std::vector<TreeReuse> trv;  // level 0 of a reusing plan: the children's runs
    if (reuse) {
        const Plan& mp = reuse->mum->plan;
        if (!mp.l0_n || (int64_t)reuse->runs->size() != M || !c->use_run) {
            cleanup();
            return fail(EV_EDEVICE, "internal: reuse without the mum's level-0 chunks");
        }
    }
    for (;;) {
        const uint64_t C = level == 0 ? C0 : C1;
        const bool reusing = level == 0 && reuse != nullptr;
        // Segments are 256 tokens at a large level 0, 64 at a smaller one
        // and at the skeleton levels, which need the extra parallelism, and
        // 16 at a level of under 2^20 tokens; a chunk's first segment, which
        // also emits the chunk's final flush, is a quarter of that.
        const uint32_t seg_len = seg_len_for(level, cur_len);
        const uint32_t head = seg_len / 4;
        auto nseg = [&](uint64_t len) -> uint64_t { return len <= head ? 1 : 1 + (len - head + seg_len - 1) / seg_len; };
        tl.clear();
        trv.clear();
        std::fill(hist, hist + EV_LEN_BUCKETS, 0u);
        uint64_t n = 0, ns = 0, tokens = 0;
        for (int32_t t = 0; reusing && t < M; t++) {
            // the child's kept chunks (from the mum's tables, checked against
            // the child's length here so that no kernel reads past them) and
            // its fresh tokens in chunks of C
            const ReuseRun& r = (*reuse->runs)[t];
            const Pop* mp_pop = reuse->mum;
            const Plan& mp = mp_pop->plan;
            const uint64_t len = rl[t];
            const uint64_t n_mid = (r.mid_len + C - 1) / C;
            const bool mum_ok =
                r.mum < (uint32_t)mp_pop->M && r.mum_off == mp_pop->h_off[r.mum] &&
                (r.n_suf == 0 || r.shift == (int64_t)len - (int64_t)(mp_pop->h_off[r.mum + 1] - r.mum_off));
            const bool ok = mum_ok && (uint64_t)r.src_first + r.ks + r.n_suf <= mp.l0_n && r.n_pre <= r.ks &&
                            (uint64_t)r.src_first + r.n_pre <= mp.l0_n && r.mid_start <= len &&
                            r.mid_len <= len - r.mid_start && n_mid < 0xFFFFFFF0ull &&
                            (r.n_pre > 0 || r.mid_start == 0) && (r.n_suf > 0 || r.mid_start + r.mid_len == len);
            if (!ok) {
                cleanup();
                return fail(EV_EDEVICE, "internal: inconsistent reuse of tree %d's mum", t);
            }
            TreeReuse v{};
            v.start = rs[t];
            v.r = r;
            v.chunk_first = (uint32_t)n;
            v.seg_first = (uint32_t)ns;
            v.tree = (uint32_t)t;
            v.C = (uint32_t)C;
            v.n_mid = (uint32_t)n_mid;
            v.mid_last = n_mid ? (uint32_t)(r.mid_len - (n_mid - 1) * C) : 0u;
            trv.push_back(v);
            const uint64_t nc = r.n_pre + n_mid + r.n_suf;
            TreeLvl w{};
            w.start = rs[t];
            w.len = len;
            w.chunk_first = (uint32_t)n;
            w.n_chunks = (uint32_t)nc;
            w.seg_first = (uint32_t)ns;
            w.C = (uint32_t)C;
            w.tree = (uint32_t)t;
            // the ranks of its work items in its length bucket (made
            // absolute below)
            w.rank_full = hist[bucket(len)];
            hist[bucket(len)] += (uint32_t)nc;
            w.rank_last = w.rank_full + (uint32_t)(nc - 1);
            tl.push_back(w);
            n += nc;
            if (n_mid) ns += (n_mid - 1) * nseg(C) + nseg(v.mid_last);
            tokens += len;
            if (n > 0xFFFFFFF0ull || ns > 0xFFFFFFF0ull) {
                cleanup();
                return fail(EV_ECAP, "too many work items or structure segments at level %d", level);
            }
        }
        for (int32_t t = 0; !reusing && t < M; t++) {
            if (!active[t]) continue;
            const uint64_t len = rl[t];
            // One work item when the tree is small, or when the last split
            // did not halve it.  A skeleton dense in long spine paths
            // shrinks slowly (only items holding a path's bottom reduce;
            // the others copy slot values into new slots), so it is cheaper
            // to finish it in one item than to split it level after level.
            const bool whole = len <= C || (level > 0 && len * 2 > prev_len[t]);
            if (whole && len > 0xFFFFFFFFull) {
                cleanup();
                return fail(EV_ECAP, "work item of %llu tokens", (unsigned long long)len);
            }
            const uint64_t Ct = whole ? len : C;
            const uint64_t nc = whole ? 1 : (len + C - 1) / C;
            TreeLvl v;
            v.start = rs[t];
            v.len = len;
            v.chunk_first = (uint32_t)n;
            v.n_chunks = (uint32_t)nc;
            v.seg_first = (uint32_t)ns;
            v.C = (uint32_t)Ct;
            v.tree = (uint32_t)t;
            v.ref_base = (uint32_t)ref_base[t];
            // the ranks of its work items in its length bucket (made
            // absolute below)
            v.rank_full = hist[bucket(len)];
            hist[bucket(len)] += (uint32_t)nc;
            v.rank_last = v.rank_full + (uint32_t)(nc - 1);
            tl.push_back(v);
            n += nc;
            ns += (nc - 1) * nseg(Ct) + nseg(len - (nc - 1) * Ct);
            tokens += len;
            if (n > 0xFFFFFFF0ull || ns > 0xFFFFFFF0ull) {
                cleanup();
                return fail(EV_ECAP, "too many work items or structure segments at level %d", level);
            }
        }
        if (tl.empty()) break;
        const uint32_t nt = (uint32_t)tl.size(), n_seg = (uint32_t)ns;

        // each length bucket's first place; the trees' ranks become places
        // (the item kernel's per-chunk bucket offsets are then zero)
        uint32_t cursor[EV_LEN_BUCKETS];
        for (uint32_t k = 0, a = 0; k < EV_LEN_BUCKETS; k++) {
            cursor[k] = a;
            a += hist[k];
        }
        for (TreeLvl& v : tl) {
            v.rank_full += cursor[bucket(v.len)];
            v.rank_last += cursor[bucket(v.len)];
        }
        std::fill(cursor, cursor + EV_LEN_BUCKETS, 0u);
        // device: chunks, segments, their counts, and each tree's numbering
        const size_t tl_bytes = nt * sizeof(TreeLvl);
        if ((st = realloc(&d_tl, tl_bytes + sizeof(cursor))) || (st = realloc(&d_ch, n * sizeof(ChunkIn))) ||
            (st = realloc(&d_cseg, n * sizeof(ChunkSegs))) || (st = realloc(&d_seg, n_seg * sizeof(SegIn))) ||
            (st = realloc(&d_fn, n_seg * sizeof(SegFn))) || (st = realloc(&d_st, n_seg * sizeof(SegStart))) ||
            (st = realloc(&d_cnt, n_seg * sizeof(SegCount))) || (st = realloc(&d_stat, n * sizeof(ChunkStat))) ||
            (st = realloc(&d_loc, n * 3 * sizeof(uint64_t))) || (st = realloc(&d_inend, n * sizeof(uint32_t))) ||
            (st = realloc(&d_sum, (nt + 1) * sizeof(TreeSum))) ||
            (st = realloc(&d_tb, (size_t)std::max(1, M) * sizeof(TreeBase))) ||
            (st = put2(x, d_tl, tl.data(), tl_bytes, cursor, sizeof(cursor)))) {
            cleanup();
            return st;
        }
        uint64_t* d_cloc = (uint64_t*)d_loc;
        uint64_t* d_oloc = d_cloc + n;
        uint64_t* d_floc = d_oloc + n;
        const uint64_t prev_out = pl.levels.empty() ? 0 : pl.levels.back().n_out;
        if (reusing) {
            if ((st = realloc(&d_tr, nt * sizeof(TreeReuse))) || (st = realloc(&d_src, n * sizeof(uint32_t))) ||
                (st = put(x, d_tr, trv.data(), nt * sizeof(TreeReuse)))) {
                cleanup();
                return st;
            }
            HIPCHK(launch_reuse_chunks((TreeReuse*)d_tr, nt, reuse->mum->plan.l0_ch, seg_len, head, (ChunkIn*)d_ch,
                                       (ChunkSegs*)d_cseg, (uint32_t*)d_src, (uint32_t*)d_err, N_ERR, s));
        } else {
            HIPCHK(launch_plan_chunks((TreeLvl*)d_tl, nt, seg_len, head, (ChunkIn*)d_ch, (ChunkSegs*)d_cseg,
                                      level == 0 ? (uint32_t*)d_err : nullptr, N_ERR, s));
        }
        HIPCHK(launch_seg_build((ChunkIn*)d_ch, (ChunkSegs*)d_cseg, (uint32_t)n, seg_len, head, (SegIn*)d_seg, s));
        HIPCHK(launch_seg_fn(cur, (SegIn*)d_seg, n_seg, (SegFn*)d_fn, level == 0 ? 0u : 1u, (uint32_t)c->n_consts, s));
        HIPCHK(launch_seg_scan((ChunkSegs*)d_cseg, (uint32_t)n, (SegFn*)d_fn, (SegStart*)d_st, (ChunkStat*)d_stat, s));
        // The count pass also records the segments' code kinds and fragment
        // tokens when the recording fits, so that emission only has to place
        // them (and run the chunks' first segments); the overflow flag rides
        // in the totals' extra record.
        const uint64_t rk_bytes = rec_kinds_stride(seg_len) * n_seg + 64;
        const uint64_t rf_bytes = rec_frags_stride(seg_len) * n_seg + 64;
        bool record = c->use_record && rk_bytes + rf_bytes <= RECORD_MAX;
        uint32_t* d_ovf = &((TreeSum*)d_sum)[nt].bad;
        if (record && ((st = ensure_rec(c, x, 0, rk_bytes, &d_rk)) || (st = ensure_rec(c, x, 1, rf_bytes, &d_rf)) ||
                       (st = ensure_rec(c, x, 2, (uint64_t)n_seg * sizeof(SegRec), &d_rec)))) {
            if (st != EV_ENOMEM) {
                cleanup();
                return st;
            }
            // no room to record: count, then emit
            release_rec(c, x);
            d_rk = d_rf = d_rec = nullptr;
            record = false;
            st = EV_OK;
        }
        HIPCHK(launch_fill_u32((uint32_t*)((TreeSum*)d_sum + nt), sizeof(TreeSum) / 4, 0u, s));
        HIPCHK(launch_seg_count(cur, (SegIn*)d_seg, n_seg, (SegStart*)d_st, (SegCount*)d_cnt,
                                record ? (uint8_t*)d_rk : nullptr, record ? (uint8_t*)d_rf : nullptr,
                                record ? (SegRec*)d_rec : nullptr, d_ovf, seg_len, s));
        HIPCHK(launch_seg_chunk((ChunkSegs*)d_cseg, (uint32_t)n, (SegCount*)d_cnt, (ChunkStat*)d_stat, nullptr, nullptr,
                                nullptr, nullptr, s));
        if (reusing)
            HIPCHK(launch_reuse_stats((uint32_t*)d_src, (uint32_t)n, reuse->mum->plan.l0_stat, (ChunkStat*)d_stat, s));
        HIPCHK(launch_plan_trees((TreeLvl*)d_tl, nt, (ChunkStat*)d_stat, (uint32_t)level, prev_out, d_cloc, d_oloc,
                                 d_floc, (uint32_t*)d_inend, (TreeSum*)d_sum, s));
        HIPCHK(launch_plan_bases((TreeLvl*)d_tl, nt, (TreeSum*)d_sum, (TreeBase*)d_tb, s));
        tsum.resize(nt + 1);
        if ((st = get(x, tsum.data(), d_sum, (nt + 1) * sizeof(TreeSum))) ||
            (level > 0 && (st = get(x, verr, (uint32_t*)d_err + 2 * (level - 1), 8))) || (st = sync(x))) {
            cleanup();
            return st;
        }
        if (level > 0 && verr[0]) {
            cleanup();
            return code_error(level - 1, verr);
        }

        // host: the trees' bases (sequence order is tree order), validity
        // and the level's totals
        uint64_t so = 0, sf = 0, sc = 0;
        uint32_t slab_top = 0, max_m = 0;
        for (uint32_t i = 0; i < nt; i++) {
            const TreeSum& q = tsum[i];
            const uint32_t t = tl[i].tree;
            // trees with constants run on the token-reading interpreter,
            // at every level (their skeletons may hold constants too)
            if (q.bad & HAS_CONST) plan_run = false;
            if (q.bad & 1u) {
                cleanup();
                if (bad_tree) *bad_tree = (int32_t)t;
                return fail(EV_EMALFORMED, "tree %u is not a valid prefix tree", t);
            }
            if (q.bad & 2u) {
                cleanup();
                return fail(EV_EDEVICE, "inconsistent split plan at level %d", level);
            }
            tb[t].out = so;
            tb[t].frag = sf;
            tb[t].code = sc;
            so += q.n_out;
            sf += q.n_frag;
            sc += q.n_codes;
            slab_top = std::max(slab_top, q.maxtop);
            max_m = std::max(max_m, q.max_m);
            pl.max_stack = std::max<uint64_t>(pl.max_stack, q.maxtop + 1);
        }
        if (so > 0xFFFFFFF0ull) { cleanup(); return fail(EV_ECAP, "too many intermediate results"); }
        if (reusing && !plan_run) {
            cleanup();
            return fail(EV_EDEVICE, "internal: reused level-0 chunks in a plan without the register-stack kernel");
        }
        const bool run_items = plan_run;
        if (run_items && need_all.size() == (size_t)level * M) {
            // each tree's work items at this level, for the chained launch
            need_all.resize((size_t)(level + 1) * M, 0u);
            pos_all.resize((size_t)(level + 1) * M, ~0u);
            for (uint32_t i = 0; i < nt; i++) {
                need_all[(size_t)level * M + tl[i].tree] = tl[i].n_chunks;
                pos_all[(size_t)level * M + tl[i].tree] = tl[i].rank_full;
            }
        }

        Level L;
        L.seq = cur;
        L.owned = cur_owned;
        L.n_out = (uint32_t)so;
        L.max_m = run_items ? 0 : max_m;
        L.tokens = tokens;
        L.trees = nt;
        // a stack deeper than the register window spills half-windows to a
        // slab; so does one that reaches the window's upper quarter at a
        // segment boundary, where the window is re-centred
        L.slab_entries = run_items && slab_top + 1 > EV_VSTACK_ENTRIES - EV_VHALF / 2 ? slab_top + EV_VHALF : 0;
        L.n_chunks = run_items ? 0 : (uint32_t)n;
        L.n_run = run_items ? (uint32_t)n : 0;
        L.n_seg = n_seg;
        L.n_codes = run_items ? sc : 0;
        L.n_frag = sf;
        pl.chunks_total += n;
        pl.slots_total += so;
        pl.levels.push_back(L);  // owns what is allocated below, freed with the plan
        Level& LL = pl.levels.back();
        cur_owned = false;
        if (!run_items) {
            if ((st = dev_alloc(c, n * sizeof(EvalChunk), (void**)&LL.d_chunks)) != EV_OK) { cleanup(); return st; }
        } else {
            if ((st = dev_alloc(c, n * sizeof(RunChunk), (void**)&LL.d_run)) != EV_OK) { cleanup(); return st; }
            if ((st = dev_alloc(c, n * sizeof(uint32_t), (void**)&LL.d_item_tree)) != EV_OK) { cleanup(); return st; }
            // 512 zero bytes after the stream (written with the work items):
            // the interpreter reads up to 192 bytes past a stream's last code
            // block, the validator up to 124
            if ((st = dev_alloc(c, sc * 4 + 512, (void**)&LL.codes)) != EV_OK) { cleanup(); return st; }
        }

        // trees finished at this level and the next level's ranges
        bool any = false;
        for (uint32_t i = 0; i < nt; i++) {
            const uint32_t t = tl[i].tree;
            const TreeSum& q = tsum[i];
            if (q.n_frag == 1) {
                pl.fin_level[t] = level;
                pl.fin_slot[t] = (uint32_t)(tb[t].out + q.n_out - 1);
                active[t] = 0;
            } else {
                any = true;
                prev_len[t] = rl[t];
                rs[t] = tb[t].frag;
                rl[t] = q.n_frag;
                ref_base[t] = tb[t].out;
            }
        }

        // the chunks' numbering and work items (longest first, from each
        // length bucket's first place), then one pass writes the next level's
        // skeleton and this level's codes, and every code stream is
        // validated before anything may run it
        // emission writes every byte of the next skeleton, [0, sf); 64 bytes
        // of padding follow (written with the work items)
        uint8_t* d_next = nullptr;
        if (any && (st = dev_alloc(c, sf + 64, (void**)&d_next)) != EV_OK) { cleanup(); return st; }
        if ((st = realloc(&d_cb, n * sizeof(uint64_t))) || (st = realloc(&d_fe, n * sizeof(uint64_t))) ||
            (st = realloc(&d_scode, n_seg * sizeof(uint64_t))) || (st = realloc(&d_sfrag, n_seg * sizeof(uint64_t)))) {
            dev_free(c, d_next);
            cleanup();
            return st;
        }
        HIPCHK(launch_plan_items((ChunkIn*)d_ch, (uint32_t)n, (TreeBase*)d_tb, d_cloc, d_oloc, d_floc,
                                 (uint32_t*)d_inend, (uint32_t*)((uint8_t*)d_tl + tl_bytes), (uint64_t*)d_cb,
                                 (uint64_t*)d_fe, run_items ? LL.d_run : nullptr, run_items ? nullptr : LL.d_chunks,
                                 run_items ? LL.codes + sc : nullptr, any ? d_next + sf : nullptr,
                                 s, nullptr, run_items ? LL.d_item_tree : nullptr));
        if (any || run_items) {
            HIPCHK(launch_seg_chunk((ChunkSegs*)d_cseg, (uint32_t)n, (SegCount*)d_cnt, (ChunkStat*)d_stat,
                                    (uint64_t*)d_cb, (uint64_t*)d_fe, (uint64_t*)d_scode, (uint64_t*)d_sfrag, s));
            if (record && tsum[nt].bad == 0) {
                // placement validates the codes as it writes them
                HIPCHK(launch_seg_place((SegIn*)d_seg, n_seg, (SegCount*)d_cnt, (SegRec*)d_rec, (SegStart*)d_st,
                                        (uint64_t*)d_scode, (uint64_t*)d_sfrag, (uint8_t*)d_rk, (uint8_t*)d_rf,
                                        run_items ? LL.codes : nullptr, sc, d_next, sf, LL.slab_entries,
                                        (uint32_t*)d_err + 2 * level, seg_len, s));
            } else {
                HIPCHK(launch_seg_emit(cur, (SegIn*)d_seg, n_seg, (SegStart*)d_st, (uint64_t*)d_scode,
                                       (uint64_t*)d_sfrag, d_next, run_items ? LL.codes : nullptr, s));
                if (run_items)
                    HIPCHK(launch_seg_check(LL.codes, (SegIn*)d_seg, n_seg, (SegStart*)d_st, (uint64_t*)d_scode,
                                            (SegCount*)d_cnt, LL.slab_entries, (uint32_t*)d_err + 2 * level, s));
            }
        }
        if (reusing) {
            const Plan& mp = reuse->mum->plan;
            HIPCHK(launch_reuse_copy((uint32_t*)d_src, (uint32_t)n, (ChunkStat*)d_stat, (uint64_t*)d_cb,
                                     (uint64_t*)d_fe, mp.l0_code, mp.l0_frag, mp.levels[0].codes,
                                     mp.levels.size() > 1 ? mp.levels[1].seq : nullptr, LL.codes, any ? d_next : nullptr,
                                     s));
        }
        if (level == 0 && run_items && any) {
            // level 0's chunks stay with the plan (for children that reuse them)
            std::vector<L0Tree> l0t((size_t)std::max(1, M), L0Tree{0, 0});
            for (uint32_t i = 0; i < nt; i++) l0t[tl[i].tree] = L0Tree{tl[i].chunk_first, tl[i].n_chunks};
            if ((st = dev_alloc(c, l0t.size() * sizeof(L0Tree), &d_l0t)) ||
                (st = put(x, d_l0t, l0t.data(), l0t.size() * sizeof(L0Tree)))) {
                cleanup();
                return st;
            }
            pl.l0_n = (uint32_t)n;
            pl.l0_ch = (ChunkIn*)d_ch;
            pl.l0_stat = (ChunkStat*)d_stat;
            pl.l0_code = (uint64_t*)d_cb;
            pl.l0_frag = (uint64_t*)d_fe;
            pl.l0_tree = (L0Tree*)d_l0t;
            d_ch = d_stat = d_cb = d_fe = d_l0t = nullptr;
        }
        if (!any) {
            // where each tree's value is, for the fitness kernel
            auto& fin = W.fin;
            fin.resize(2 * (size_t)std::max(1, M));
            for (int32_t t = 0; t < M; t++) {
                fin[2 * (size_t)t] = (uint32_t)pl.fin_level[t];
                fin[2 * (size_t)t + 1] = pl.fin_slot[t];
            }
            if ((st = dev_alloc(c, fin.size() * 4, (void**)&pl.d_fin)) || (st = put(x, pl.d_fin, fin.data(), fin.size() * 4))) {
                cleanup();
                return st;
            }
            // the last level: its validation must pass before the plan is
            // used, checked here, or (defer_check) by its k_run launches on
            // the device and by the host with the first evaluation
            if (c->test_fail_check && run_items)
                HIPCHK(launch_fill_u32((uint32_t*)d_err + 2 * level, 1, 0x100u, s));
            if (defer_check) {
                pl.err_level = level;
                pl.err_pending = true;
                break;
            }
            if ((st = get(x, verr, (uint32_t*)d_err + 2 * level, 8)) || (st = sync(x))) {
                cleanup();
                return st;
            }
            if (verr[0]) {
                cleanup();
                return code_error(level, verr);
            }
            break;
        }
        cur = d_next;
        cur_len = sf;
        cur_owned = true;
        level++;
        if (level > MAX_LEVELS) {
            cleanup();
            int32_t t = 0;
            while (t < M && !active[t]) t++;
            return fail(EV_ECAP, "split plan did not converge (tree %d: %llu tokens after %llu)", t,
                        (unsigned long long)(t < M ? rl[t] : 0), (unsigned long long)(t < M ? prev_len[t] : 0));
        }
    }
    pl.d_err = (uint32_t*)d_err;  // the plan keeps the validator's words
    d_err = nullptr;
    if (pl.levels.size() >= 2 && need_all.size() == pl.levels.size() * (size_t)M) {
        if ((st = dev_alloc(c, need_all.size() * sizeof(uint32_t), (void**)&pl.d_need)) != EV_OK ||
            (st = put(x, pl.d_need, need_all.data(), need_all.size() * sizeof(uint32_t))) != EV_OK) {
            cleanup();
            return st;
        }
        pl.h_need = std::move(need_all);
        pl.h_pos = std::move(pos_all);
    }
    cleanup();
    pl.bytes = 0;
    for (auto& L : pl.levels) pl.bytes += (uint64_t)L.n_chunks * sizeof(EvalChunk) + (uint64_t)L.n_run * sizeof(RunChunk);
    return EV_OK;
}

// Make a population from device bytes (takes ownership of d_bytes, also on
// failure).
ev_status pop_build(ev_ctx* c, Exec& x, uint8_t* d_bytes, const std::vector<uint64_t>& h_off, Pop** out, int32_t* bad,
                    uint64_t* d_off, bool defer_check, const ReuseSpec* reuse)
{
    *out = nullptr;
    Pop* P = new Pop();
    P->d_bytes = d_bytes;
    P->d_off = d_off;
    P->h_off = h_off;
    P->M = (int32_t)h_off.size() - 1;
    P->total = h_off.back();
    ev_status st;
    if (!d_off) {
        if ((st = dev_alloc(c, h_off.size() * sizeof(uint64_t), (void**)&P->d_off)) != EV_OK) { pop_free(c, P); return st; }
        if ((st = put(x, P->d_off, h_off.data(), h_off.size() * sizeof(uint64_t))) != EV_OK) { pop_free(c, P); return st; }
    }
    if ((st = dev_alloc(c, (size_t)std::max(1, P->M) * sizeof(float), (void**)&P->d_fit)) != EV_OK) { pop_free(c, P); return st; }
    if ((st = plan_build(c, x, P, bad, defer_check, reuse)) != EV_OK) { pop_free(c, P); return st; }
    *out = P;
    return EV_OK;
}

ev_pop pop_register(ev_ctx* c, Pop* P)
{
    std::lock_guard<std::mutex> g(c->pop_mu);
    const ev_pop id = c->next_pop++;
    c->pops[id] = P;
    return id;
}

Pop* pop_get(ev_ctx* c, ev_pop id)
{
    std::lock_guard<std::mutex> g(c->pop_mu);
    auto it = c->pops.find(id);
    return it == c->pops.end() ? nullptr : it->second;
}

Pop* pop_acquire(ev_ctx* c, ev_pop id)
{
    std::lock_guard<std::mutex> g(c->pop_mu);
    auto it = c->pops.find(id);
    if (it == c->pops.end()) return nullptr;
    it->second->refs++;
    return it->second;
}

// The caller has waited for its own work on P; if P was freed meanwhile and
// this was its last user, its blocks go to the cache for the caller's stream.
void pop_release(ev_ctx* c, Pop* P)
{
    bool last = false;
    {
        std::lock_guard<std::mutex> g(c->pop_mu);
        last = --P->refs == 0 && P->dead;
    }
    if (last) pop_free(c, P);
}

// ----------------------------------------------------------- evaluation

ev_status ensure_gstack(ev_ctx* c, Exec& x, size_t bytes)
{
    if (bytes <= x.gstack_bytes) return EV_OK;
    if (ev_status st = sync(x)) return st;
    dev_free(c, x.d_gstack);
    x.d_gstack = nullptr;
    x.gstack_bytes = 0;
    ev_status st = dev_alloc(c, bytes, (void**)&x.d_gstack);
    if (st == EV_OK) x.gstack_bytes = bytes;
    return st;
}

ev_status ensure_counters(ev_ctx* c, Exec& x, size_t n)
{
    if (n <= x.n_counters) return EV_OK;
    if (ev_status st = sync(x)) return st;
    dev_free(c, x.d_counters);
    x.d_counters = nullptr;
    x.n_counters = 0;
    ev_status st = dev_alloc(c, n * sizeof(uint32_t), (void**)&x.d_counters);
    if (st == EV_OK) x.n_counters = n;
    return st;
}

ev_status exec_init(Exec& x, hipStream_t given)
{
    if (given) {
        x.stream = given;
        x.own_stream = false;
    } else {
        // default priority (streams of other priorities are not used)
        hipError_t e = hipStreamCreateWithFlags(&x.stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        x.own_stream = true;
    }
    x.clock.stream = x.stream;
    (void)hipEventCreateWithFlags(&x.done, hipEventDisableTiming);
    (void)hipEventCreate(&x.ev0);
    (void)hipEventCreate(&x.ev1);
    (void)hipEventCreate(&x.evi0);
    (void)hipEventCreate(&x.evi1);
    return EV_OK;
}

// A region of n bytes in x's pinned staging buffer.  When the buffer is
// full the stream is synchronized first (every staged copy has then landed)
// and the buffer is reused, or replaced by a larger one.
ev_status stage(Exec& x, size_t n, void** out)
{
    n = (n + 255) & ~(size_t)255;
    if (x.pin_off + n > x.pin_cap) {
        ev_status st = sync(x);
        if (st != EV_OK) return st;
        if (n > x.pin_cap) {
            if (x.pin) (void)hipHostFree(x.pin);
            x.pin = nullptr;
            x.pin_cap = 0;
            const size_t cap = std::max<size_t>(n, (size_t)4 << 20);
            // coherent: the copy kernel reads and writes it directly
            hipError_t e = hipHostMalloc((void**)&x.pin, cap, hipHostMallocCoherent);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                x.pin = nullptr;
                return fail(EV_ENOMEM, "hipHostMalloc(%zu): %s", cap, hipGetErrorString(e));
            }
            x.pin_cap = cap;
        }
    }
    *out = x.pin + x.pin_off;
    x.pin_off += n;
    return EV_OK;
}

// Large transfers pass through the staging buffer in pieces of this size.
static constexpr size_t STAGE_PIECE = (size_t)64 << 20;
// Transfers up to this size are copied by a kernel on the stream's compute
// queue: a DMA-engine copy between kernels costs a handoff between queues
// (measured 15-40 us around each), far more than such a copy itself.
static constexpr size_t KERNEL_COPY_MAX = (size_t)1 << 20;

// Host-to-device copy on x's stream (src may be reused on return).
ev_status put(Exec& x, void* dst, const void* src, size_t n)
{
    for (size_t o = 0; o < n; o += STAGE_PIECE) {
        const size_t k = std::min(STAGE_PIECE, n - o);
        void* p = nullptr;
        ev_status st = stage(x, k, &p);
        if (st != EV_OK) return st;
        std::memcpy(p, (const uint8_t*)src + o, k);
        if (k <= KERNEL_COPY_MAX)
            HIPCHK(launch_copy((uint8_t*)dst + o, p, k, x.stream));
        else
            HIPCHK(hipMemcpyAsync((uint8_t*)dst + o, p, k, hipMemcpyHostToDevice, x.stream));
    }
    return EV_OK;
}

// Two host buffers to consecutive device bytes, as one transfer.
ev_status put2(Exec& x, void* dst, const void* a, size_t na, const void* b, size_t nb)
{
    if (na + nb > KERNEL_COPY_MAX) {
        ev_status st = put(x, dst, a, na);
        return st != EV_OK ? st : put(x, (uint8_t*)dst + na, b, nb);
    }
    void* p = nullptr;
    ev_status st = stage(x, na + nb, &p);
    if (st != EV_OK) return st;
    std::memcpy(p, a, na);
    std::memcpy((uint8_t*)p + na, b, nb);
    HIPCHK(launch_copy(dst, p, na + nb, x.stream));
    return EV_OK;
}

// Device-to-host copy on x's stream; dst holds the data once sync(x) returns.
ev_status get(Exec& x, void* dst, const void* src, size_t n)
{
    for (size_t o = 0; o < n; o += STAGE_PIECE) {
        const size_t k = std::min(STAGE_PIECE, n - o);
        void* p = nullptr;
        ev_status st = stage(x, k, &p);
        if (st != EV_OK) return st;
        if (k <= KERNEL_COPY_MAX)
            HIPCHK(launch_copy(p, (const uint8_t*)src + o, k, x.stream));
        else
            HIPCHK(hipMemcpyAsync(p, (const uint8_t*)src + o, k, hipMemcpyDeviceToHost, x.stream));
        x.pin_out.push_back(Exec::Out{(uint8_t*)dst + o, p, k});
    }
    return EV_OK;
}

// Waits for everything enqueued on x's stream so far (the stream may be
// shared with other Execs: their later work is not waited for).
ev_status sync(Exec& x)
{
    hipError_t e = hipEventRecord(x.done, x.stream);
    if (e == hipSuccess) e = hipEventSynchronize(x.done);
    if (e == hipSuccess) {
        for (const Exec::Out& o : x.pin_out) std::memcpy(o.dst, o.src, o.n);
        x.clock.waits.fetch_add(1);  // everything queued before this call has finished
    }
    x.pin_out.clear();
    x.pin_off = 0;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return EV_OK;
}

void exec_free(ev_ctx* c, Exec& x)
{
    if (x.stream) (void)hipStreamSynchronize(x.stream);
    ExecScope scope(&x);
    if (x.pin) (void)hipHostFree(x.pin);
    x.pin = nullptr;
    x.pin_cap = x.pin_off = 0;
    x.pin_out.clear();
    dev_free(c, x.d_gstack);
    dev_free(c, x.d_counters);
    x.d_gstack = nullptr;
    x.d_counters = nullptr;
    x.gstack_bytes = x.n_counters = 0;
    release_rec(c, x);
    for (hipEvent_t e : x.evl) (void)hipEventDestroy(e);
    x.evl.clear();
    if (x.done) (void)hipEventDestroy(x.done);
    if (x.ev0) (void)hipEventDestroy(x.ev0);
    if (x.ev1) (void)hipEventDestroy(x.ev1);
    if (x.evi0) (void)hipEventDestroy(x.evi0);
    if (x.evi1) (void)hipEventDestroy(x.evi1);
    x.done = x.ev0 = x.ev1 = x.evi0 = x.evi1 = nullptr;
    {
        // the stream has drained: what it freed is free for every stream
        std::lock_guard<std::mutex> g(c->mem_mu);
        c->cache.forget(&x.clock);
    }
    if (x.own_stream && x.stream) (void)hipStreamDestroy(x.stream);
    x.stream = nullptr;
}

ev_status rescache_build(ev_ctx* c, Exec& x, Pop* P, int32_t table, ResCache** out);

// Drop the cached result slots of every population but P (they are
// rebuilt on their next evaluation).  Waits for the context's stream first,
// since queued evaluations may still use them.
static void rescache_evict_others(ev_ctx* c, Exec& x, Pop* P)
{
    (void)sync(x);
    std::lock_guard<std::mutex> g(c->pop_mu);
    for (auto& kv : c->pops) {
        if (kv.second == P) continue;
        for (auto& r : kv.second->res) rescache_free(c, r.second);
        kv.second->res.clear();
    }
}

ev_status rescache_get(ev_ctx* c, Exec& x, Pop* P, int32_t table, ResCache** out)
{
    auto it = P->res.find(table);
    if (it != P->res.end()) { *out = &it->second; return EV_OK; }
    ev_status st0 = rescache_build(c, x, P, table, out);
    // only the synchronous API (the context's own Exec) evicts: serving
    // workers never touch registered populations' slots, the API might
    if (st0 != EV_ENOMEM || &x != &c->main) return st0;
    rescache_evict_others(c, x, P);
    return rescache_build(c, x, P, table, out);
}

ev_status rescache_build(ev_ctx* c, Exec& x, Pop* P, int32_t table, ResCache** out)
{
    ResCache r;
    CaseTable ct;
    if (!table_get(c, table, &ct)) return fail(EV_EINVAL, "no case table %d", table);
    const int32_t N = ct.N;
    r.N = N;
    ev_status st;
    for (auto& L : P->plan.levels) {
        float* p = nullptr;
        // EV_RING rows in front: the next level reads up to that many rows
        // ahead of (below) its lowest slot
        const size_t rows = (size_t)std::max<uint32_t>(L.n_out, 1) + EV_RING;
        if ((st = dev_alloc(c, rows * N * sizeof(float), (void**)&p)) != EV_OK) {
            rescache_free(c, r);
            return st;
        }
        r.res.push_back(p + (size_t)EV_RING * N);
    }
    P->res[table] = r;
    *out = &P->res[table];
    return EV_OK;
}

// The buffers an evaluation's kernels use besides the plan: the work
// counters (two per level), each level's result slots (with EV_RING rows in
// front of the pointer) and the spill slabs of the waves.
struct EvalBufs {
    uint32_t* counters = nullptr;
    std::vector<float*> res;
    float* slab = nullptr;
    size_t slab_bytes = 0;
    // levels chain_first .. levels-1 in one launch: their RunLevel records
    // and the done counters (chained levels x trees words); null: a launch
    // per level
    const RunLevel* chain = nullptr;
    uint32_t* done = nullptr;
    int chain_first = -1;
    uint32_t chain_records = 0;  // runs of work items in the chained launch's queue
};

// Level-0 sizes (tokens) up to which level 0 joins the chained launch: a
// tree's skeleton items then start as soon as its own level-0 items are
// done, beside the rest of level 0.  Larger level 0s keep a launch of their
// own (their trees' level-0 items cover the whole launch anyway).
static constexpr uint64_t CHAIN_LEVEL0_MAX = 1ull << 27;

// The first level of P that goes in the chained launch, or -1: every level
// on the register-stack kernel, on a stream that allows it; from level 0
// when level 0 is small and there is a level after it, else from level 1
// when there are two levels after it.
static int chain_first(ev_ctx* c, const Exec& x, const Pop* P)
{
    const Plan& pl = P->plan;
    const size_t nl = pl.levels.size();
    if (!c->use_chain || !x.chain_ok || !pl.d_need || nl < 2) return -1;
    for (const Level& L : pl.levels)
        if (L.n_chunks || !L.n_run || !L.d_item_tree) return -1;
    if (pl.levels[0].tokens <= CHAIN_LEVEL0_MAX) return 0;
    return nl >= 3 ? 1 : -1;
}

// Spill-slab bytes one wave of a level's interpreter needs (0: none).
static size_t slab_per_wave(const Level& L, int D)
{
    if (L.n_run) return L.slab_entries ? (size_t)L.slab_entries * 64 * sizeof(float) : 0;
    if (L.n_chunks && L.max_m + 16 > (uint32_t)D) return (size_t)(L.max_m + 16) * 64 * sizeof(float);
    return 0;
}

// Queue the kernels of one evaluation of P on x's stream.  A level's grid is
// cut to the waves whose spill slabs fit b.slab_bytes.
static ev_status eval_launch(ev_ctx* c, Exec& x, Pop* P, const CaseTable& ct, const EvalBufs& b, float* d_fit,
                             float* d_per_case, int32_t* d_hits, bool timed)
{
    const int32_t N = ct.N;
    const uint32_t n_cb = (uint32_t)((N + 63) / 64);
    const int D = P->plan.D;
    const size_t nl = P->plan.levels.size();
    const uint32_t grid_max = (uint32_t)c->grid_eval[D == 128 ? 1 : 0];
    auto grid_for = [&](const Level& L, uint64_t items, uint32_t grid) -> uint32_t {
        uint64_t g = std::min<uint64_t>(grid, items);
        const size_t w = slab_per_wave(L, D);
        if (w) g = std::min<uint64_t>(g, b.slab_bytes / w);
        return (uint32_t)g;
    };
    for (const Level& L : P->plan.levels)
        if ((L.n_run || L.n_chunks) && grid_for(L, 1, 1) == 0)
            return fail(EV_ECAP, "no room for one wave's spill slab (%zu bytes)", slab_per_wave(L, D));
    hipStream_t s = x.stream;
    if (timed) {
        while (x.evl.size() < nl) {
            hipEvent_t e = nullptr;
            HIPCHK(hipEventCreate(&e));
            x.evl.push_back(e);
        }
        x.n_levels_timed = (uint32_t)nl;
    }
    if (timed) HIPCHK(hipEventRecord(x.ev0, s));
    HIPCHK(launch_fill_u32(b.counters, (uint32_t)(2 * nl), 0u, s));
    const size_t cf = b.chain && b.done && b.chain_first >= 0 ? (size_t)b.chain_first : nl;
    const bool chained = cf < nl;
    if (chained) HIPCHK(launch_fill_u32(b.done, (uint32_t)((nl - cf) * (size_t)P->M), 0u, s));
    for (size_t li = 0; li < nl; li++) {
        const Level& L = P->plan.levels[li];
        if (chained && li >= cf) {
            if (li == cf) {
                // levels cf .. nl-1 in one launch (k_run_chain)
                if (timed && li == 0) HIPCHK(hipEventRecord(x.evi0, s));
                ChainArgs ca{};
                ca.levels = b.chain;
                ca.n_levels = b.chain_records;
                uint64_t total = 0, rows = 0;
                for (size_t k = cf; k < nl; k++) {
                    total += (uint64_t)P->plan.levels[k].n_run * n_cb;
                    rows = std::max<uint64_t>(rows, P->plan.levels[k].slab_entries);
                }
                if (total > 0xFFFFFFF0ull) return fail(EV_ECAP, "too many chained work items for one launch");
                ca.total = (uint32_t)total;
                ca.n_cb = n_cb;
                ca.M = (uint32_t)P->M;
                ca.counter = b.counters + nl + cf;
                ca.need = P->plan.d_need + cf * (size_t)P->M;  // from level cf on
                ca.done = b.done;
                ca.x = ct.d_x;
                ca.N = N;
                ca.rowb = (uint32_t)N * 4u;
                ca.slab = b.slab;
                ca.slab_entries = rows;
                ca.flag = c->d_flag;
                uint64_t g = std::min<uint64_t>((uint64_t)c->grid_chain, total);
                if (rows) g = std::min<uint64_t>(g, b.slab_bytes / (rows * 64 * sizeof(float)));
                if (g == 0) return fail(EV_ECAP, "no room for one wave's spill slab (%llu rows)", (unsigned long long)rows);
                HIPCHK(launch_run_chain(ca, (uint32_t)g, s));
                if (timed && li == 0) HIPCHK(hipEventRecord(x.evi1, s));
            }
            if (timed) HIPCHK(hipEventRecord(x.evl[li], s));
            continue;
        }
        if (timed && li == 0) HIPCHK(hipEventRecord(x.evi0, s));
        if (L.n_run) {
            RunArgs r{};
            r.codes = L.codes;
            r.chunks = L.d_run;
            r.n_items = L.n_run * n_cb;
            r.n_cb = n_cb;
            r.counter = b.counters + nl + li;
            r.x = ct.d_x;
            r.N = N;
            r.rowb = (uint32_t)N * 4u;
            r.in_res = li ? b.res[li - 1] : nullptr;
            r.refs = li ? 1u : 0u;
            r.out_res = b.res[li];
            r.slab = b.slab;
            r.slab_entries = L.slab_entries;
            r.flag = c->d_flag;
            r.verdict = P->plan.d_err ? P->plan.d_err + 2 * li : nullptr;
            HIPCHK(launch_run(r, grid_for(L, r.n_items, (uint32_t)c->grid_run), s));
        }
        if (L.n_chunks == 0) {
            if (timed && li == 0) HIPCHK(hipEventRecord(x.evi1, s));
            if (timed) HIPCHK(hipEventRecord(x.evl[li], s));
            continue;
        }
        EvalArgs a;
        a.seq = L.seq;
        a.chunks = L.d_chunks;
        a.n_items = L.n_chunks * n_cb;
        a.n_cb = n_cb;
        a.counter = b.counters + li;
        a.x = ct.d_x;
        a.N = N;
        a.gstack_entries = L.max_m + 16;
        a.in_res = li ? b.res[li - 1] : nullptr;
        a.out_res = b.res[li];
        a.gstack = b.slab;
        a.consts = c->d_const;
        HIPCHK(launch_eval(D, a, grid_for(L, a.n_items, grid_max), s));
        if (timed && li == 0) HIPCHK(hipEventRecord(x.evi1, s));
        if (timed) HIPCHK(hipEventRecord(x.evl[li], s));
    }
    FitArgs fa = {};
    for (size_t li = 0; li < nl; li++) {
        fa.res[li] = b.res[li];
        fa.n_out[li] = P->plan.levels[li].n_out;
    }
    fa.n_levels = (uint32_t)nl;
    fa.fin = P->plan.d_fin;
    fa.y = ct.d_y;
    fa.N = N;
    fa.M = (uint32_t)P->M;
    fa.fit = d_fit;
    fa.per_case = d_per_case;
    fa.hits = d_hits;
    HIPCHK(launch_fitness(fa, s));
    if (timed) HIPCHK(hipEventRecord(x.ev1, s));
    return EV_OK;
}

// Queue the evaluation of P on table on c->stream; fit/per_case are device
// pointers (per_case nullable).
ev_status eval_enqueue(ev_ctx* c, Exec& x, Pop* P, int32_t table, float* d_fit, float* d_per_case, bool timed,
                       int32_t* d_hits, bool verdict_at_sync)
{
    if (P->plan.err_pending) {
        // the plan's last validation verdict: read with the caller's next
        // sync (then checked by plan_verdict), or here
        ev_status st = get(x, P->plan.h_err, P->plan.d_err + 2 * P->plan.err_level, 8);
        if (st == EV_OK && !verdict_at_sync && (st = sync(x)) == EV_OK) st = plan_verdict(P);
        if (st != EV_OK) return st;
    }
    CaseTable ct;
    if (!table_get(c, table, &ct)) return fail(EV_EINVAL, "no case table %d", table);
    const int32_t N = ct.N;
    const uint32_t n_cb = (uint32_t)((N + 63) / 64);
    const int D = P->plan.D;
    ResCache* rc = nullptr;
    ev_status st;
    if ((st = rescache_get(c, x, P, table, &rc)) != EV_OK) return st;
    const size_t nl = P->plan.levels.size();
    const int cfi = chain_first(c, x, P);
    const bool chain = cfi >= 0;
    const size_t cf = chain ? (size_t)cfi : nl;
    // the work counters, then (chained) the done counters of the chained levels
    if ((st = ensure_counters(c, x, 2 * nl + (chain ? (nl - cf) * (size_t)P->M : 0))) != EV_OK) return st;
    // spill slabs for every wave of each level's grid
    const uint32_t grid_max = (uint32_t)c->grid_eval[D == 128 ? 1 : 0];
    size_t need = 0, chain_rows = 0;
    uint64_t chain_items = 0;
    for (size_t li = 0; li < nl; li++) {
        const Level& L = P->plan.levels[li];
        const uint64_t items = (uint64_t)(L.n_run + L.n_chunks) * n_cb;
        if (chain && li >= cf) {
            chain_rows = std::max<size_t>(chain_rows, L.slab_entries);
            chain_items += items;
            continue;
        }
        const uint64_t grid = std::min<uint64_t>(L.n_run ? (uint64_t)c->grid_run : grid_max, items);
        need = std::max(need, (size_t)grid * slab_per_wave(L, D));
    }
    if (chain)
        need = std::max(need, (size_t)std::min<uint64_t>(c->grid_chain, chain_items) * chain_rows * 64 * sizeof(float));
    if ((st = ensure_gstack(c, x, need)) != EV_OK) return st;
    if (chain && rc->d_chain && rc->chain_first != cfi) {
        // made for another first level (queued launches on this stream may
        // still read it: freed in stream order)
        dev_free(c, rc->d_chain);
        rc->d_chain = nullptr;
    }
    if (chain && !rc->d_chain) {
        // the chained launch's queue, kept with the result slots of this
        // case table: runs of work items (level, first item, count)
        struct Run {
            size_t li;
            uint32_t start, count;
        };
        std::vector<Run> runs;
        const Plan& pl = P->plan;
        const size_t M = (size_t)P->M;
        const bool known = cf == 0 && nl >= 2 && pl.h_pos.size() >= 2 * M && pl.h_need.size() >= 2 * M &&
                           pl.h_pos[0] != ~0u && pl.h_pos[M] != ~0u;
        if (known) {
            // Level 0's first wave of items (as many as the launch has
            // waves), then the skeleton items of the trees whose level-0
            // items all lie in it (taken in their own order, as long as that
            // holds), then the rest of level 0, then the other skeleton
            // items.  Those trees' skeleton items start when their level-0
            // items end, not after every level-0 item has been taken.
            const uint32_t n0 = pl.levels[0].n_run, n1 = pl.levels[1].n_run;
            const uint32_t P0 =
                (uint32_t)std::min<uint64_t>(n0, std::max<uint64_t>(1, (uint64_t)c->grid_chain / n_cb));
            std::vector<std::pair<uint32_t, uint32_t>> by1;  // (first level-1 place, tree)
            for (size_t t = 0; t < M; t++)
                if (pl.h_need[M + t]) by1.push_back({pl.h_pos[M + t], (uint32_t)t});
            std::sort(by1.begin(), by1.end());
            uint32_t K = 0;
            for (auto& e : by1) {
                const size_t t = e.second;
                if (e.first != K || pl.h_pos[t] == ~0u || (uint64_t)pl.h_pos[t] + pl.h_need[t] > P0) break;
                K += pl.h_need[M + t];
            }
            runs.push_back({0, 0, P0});
            if (K) runs.push_back({1, 0, K});
            if (n0 > P0) runs.push_back({0, P0, n0 - P0});
            if (n1 > K) runs.push_back({1, K, n1 - K});
            for (size_t li = 2; li < nl; li++) runs.push_back({li, 0, pl.levels[li].n_run});
        } else {
            for (size_t li = cf; li < nl; li++) runs.push_back({li, 0, pl.levels[li].n_run});
        }
        std::vector<RunLevel> rl;
        uint64_t first = 0;
        for (const Run& u : runs) {
            if (!u.count) continue;
            const Level& L = pl.levels[u.li];
            RunLevel r{};
            r.codes = L.codes;
            r.chunks = L.d_run + u.start;
            r.item_tree = L.d_item_tree + u.start;
            r.in_res = u.li ? rc->res[u.li - 1] : nullptr;
            r.out_res = rc->res[u.li];
            r.verdict = pl.d_err ? pl.d_err + 2 * u.li : nullptr;
            r.first = (uint32_t)first;
            r.n_items = u.count * n_cb;
            r.refs = u.li ? 1u : 0u;
            r.plevel = (uint32_t)(u.li - cf);
            rl.push_back(r);
            first += (uint64_t)u.count * n_cb;
        }
        if (rl.empty()) rl.push_back(RunLevel{});
        if ((st = dev_alloc(c, rl.size() * sizeof(RunLevel), (void**)&rc->d_chain)) != EV_OK ||
            (st = put(x, rc->d_chain, rl.data(), rl.size() * sizeof(RunLevel))) != EV_OK)
            return st;
        rc->chain_first = cfi;
        rc->chain_records = (uint32_t)rl.size();
    }
    EvalBufs b;
    b.counters = x.d_counters;
    b.res = rc->res;
    b.slab = x.d_gstack;
    b.slab_bytes = x.gstack_bytes;
    if (chain) {
        b.chain = rc->d_chain;
        b.done = x.d_counters + 2 * nl;
        b.chain_first = cfi;
        b.chain_records = rc->chain_records;
    }
    return eval_launch(c, x, P, ct, b, d_fit, d_per_case, d_hits, timed);
}

// The same with every buffer of the kernels carved from [scratch, scratch +
// bytes) and no allocation: the population's plan must be settled (its
// validation verdict read), the outputs are device pointers.
ev_status eval_in_scratch(ev_ctx* c, Pop* P, int32_t table, float* d_fit, float* d_per_case, int32_t* d_hits,
                          uint8_t* scratch, size_t bytes)
{
    if (P->plan.err_pending)
        return fail(EV_EINVAL, "population not evaluated yet: its plan's validation verdict is still to be read");
    CaseTable ct;
    if (!table_get(c, table, &ct)) return fail(EV_EINVAL, "no case table %d", table);
    const size_t nl = P->plan.levels.size();
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t at = up(2 * nl * sizeof(uint32_t));
    EvalBufs b;
    b.counters = (uint32_t*)scratch;
    for (const Level& L : P->plan.levels) {
        const size_t rows = (size_t)std::max<uint32_t>(L.n_out, 1) + EV_RING;
        const size_t need = rows * (size_t)ct.N * sizeof(float);
        if (at + need > bytes)
            return fail(EV_ECAP, "the population's result slots need more than the %zu bytes of static scratch", bytes);
        b.res.push_back((float*)(scratch + at) + (size_t)EV_RING * ct.N);
        at = up(at + need);
    }
    b.slab = (float*)(scratch + std::min(at, bytes));
    b.slab_bytes = at < bytes ? bytes - at : 0;
    return eval_launch(c, c->main, P, ct, b, d_fit, d_per_case, d_hits, false);
}

// ----------------------------------------------------------- crossover

// Children from explicit parents and points; all arrays on the host.
// Children of Sec. 2.3's crossover from parent indices and points already on
// the device (d_mum, d_dad, d_p, d_q; n each, valid for the parents): the
// subtree ends, child lengths and offsets are found on the device, so the
// host waits once, for the offsets it needs to size the new buffer.
ev_status crossover_build_dev(ev_ctx* c, Exec& x, Pop* mums, Pop* dads, const int32_t* d_mum, const int32_t* d_dad,
                              const uint64_t* d_p, const uint64_t* d_q, int32_t n, uint64_t cap, Pop** out,
                              int32_t* n_capped, bool defer_check)
{
    hipStream_t s = x.stream;
    const size_t qn = std::max<size_t>(1, 2 * (size_t)n);
    void *d_b = nullptr, *d_qp = nullptr, *d_e = nullptr, *d_plan = nullptr;
    uint64_t* d_off = nullptr;
    auto cleanup = [&]() {
        for (void* p : {d_b, d_qp, d_e, d_plan}) dev_free(c, p);
    };
    ev_status st;
    if ((st = dev_alloc(c, qn * 8, &d_b)) || (st = dev_alloc(c, qn * 8, &d_qp)) || (st = dev_alloc(c, qn * 8, &d_e)) ||
        (st = dev_alloc(c, std::max<size_t>(1, n) * sizeof(XoPlan), &d_plan)) ||
        (st = dev_alloc(c, (2 * (size_t)n + 5) * 8, (void**)&d_off))) {
        cleanup();
        dev_free(c, d_off);
        return st;
    }
    // the offsets, then the number capped, the longest child and the number
    // of 4 KiB copy pieces (each child's first piece follows on the device)
    std::vector<uint64_t> off((size_t)n + 4, 0);
    // the mum's level-0 chunks each child keeps (read with the offsets)
    const bool reuse_ok = c->use_reuse && c->use_run && c->n_consts == 0 && mums->plan.l0_n > 0 && n > 0;
    std::vector<ReuseRun> runs;
    void* d_runs = nullptr;
    if (reuse_ok && (st = dev_alloc(c, (size_t)n * sizeof(ReuseRun), &d_runs)) != EV_OK) {
        cleanup();
        dev_free(c, d_off);
        return st;
    }
    if (n > 0) {
        uint64_t* qb = (uint64_t*)d_b;
        uint64_t* qp = (uint64_t*)d_qp;
        uint64_t* ends = (uint64_t*)d_e;
        HIPCHK(launch_xo_query(mums->d_off, dads->d_off, d_mum, d_dad, d_p, d_q, (uint32_t)n, qb, qp, s));
        if (mums == dads) {
            HIPCHK(launch_subtree_end(mums->d_bytes, qb, qp, 2u * (uint32_t)n, ends, s));
        } else {
            HIPCHK(launch_subtree_end(mums->d_bytes, qb, qp, (uint32_t)n, ends, s));
            HIPCHK(launch_subtree_end(dads->d_bytes, qb + n, qp + n, (uint32_t)n, ends + n, s));
        }
        HIPCHK(launch_xo_plan(mums->d_off, dads->d_off, d_mum, d_dad, d_p, d_q, ends, (uint32_t)n, cap, (XoPlan*)d_plan,
                              d_off, s));
        if (reuse_ok) {
            runs.resize((size_t)n);
            HIPCHK(launch_reuse_runs((XoPlan*)d_plan, d_mum, mums->plan.l0_tree, mums->plan.l0_ch, (uint32_t)n,
                                     (ReuseRun*)d_runs, s));
            st = get(x, runs.data(), d_runs, (size_t)n * sizeof(ReuseRun));
        }
        if (st || (st = get(x, off.data(), d_off, ((size_t)n + 4) * 8)) || (st = sync(x))) {
            cleanup();
            dev_free(c, d_runs);
            dev_free(c, d_off);
            return st;
        }
        dev_free(c, d_runs);
    } else if ((st = put(x, d_off, off.data(), 8)) != EV_OK) {
        cleanup();
        dev_free(c, d_off);
        return st;
    }
    uint8_t* d_child = nullptr;
    if ((st = dev_alloc(c, off[n] + EV_POP_PAD, (void**)&d_child)) != EV_OK) {
        cleanup();
        dev_free(c, d_off);
        return st;
    }
    const uint64_t capped = off[n + 1], pieces = off[n + 3];
    off.resize((size_t)n + 1);
    HIPCHK(launch_xo_copy(mums->d_bytes, dads->d_bytes, (XoPlan*)d_plan, d_off, (uint32_t)n, pieces, d_child,
                          d_child + off[n], (uint32_t)EV_POP_PAD, s));
    // the scratch goes back to the cache while the copy may still run: every
    // later use of it is ordered after the copy on the context's one stream
    cleanup();
    if (n_capped) *n_capped = (int32_t)capped;
    const ReuseSpec spec{mums, &runs};
    return pop_build(c, x, d_child, off, out, nullptr, d_off, defer_check, reuse_ok ? &spec : nullptr);
}

// The same from host arrays, checked against the parents first.
ev_status crossover_build(ev_ctx* c, Exec& x, Pop* mums, Pop* dads, const int32_t* mum, const int32_t* dad,
                          const uint64_t* p, const uint64_t* q, int32_t n, uint64_t cap, Pop** out, int32_t* n_capped)
{
    for (int32_t j = 0; j < n; j++) {
        if (mum[j] < 0 || mum[j] >= mums->M || dad[j] < 0 || dad[j] >= dads->M)
            return fail(EV_EINVAL, "child %d: parent index out of range", j);
        const uint64_t nm = mums->h_off[mum[j] + 1] - mums->h_off[mum[j]];
        const uint64_t nd = dads->h_off[dad[j] + 1] - dads->h_off[dad[j]];
        if (p[j] >= nm || q[j] >= nd) return fail(EV_EINVAL, "child %d: crossover point out of range", j);
    }
    void* d_in = nullptr;
    const size_t m = std::max<size_t>(1, n);
    ev_status st = dev_alloc(c, m * 24, &d_in);
    if (st != EV_OK) return st;
    int32_t* d_mum = (int32_t*)d_in;
    int32_t* d_dad = d_mum + m;
    uint64_t* d_p = (uint64_t*)((char*)d_in + m * 8);
    uint64_t* d_q = d_p + m;
    if (n > 0 && ((st = put(x, d_mum, mum, (size_t)n * 4)) || (st = put(x, d_dad, dad, (size_t)n * 4)) ||
                  (st = put(x, d_p, p, (size_t)n * 8)) || (st = put(x, d_q, q, (size_t)n * 8)))) {
        dev_free(c, d_in);
        return st;
    }
    st = crossover_build_dev(c, x, mums, dads, d_mum, d_dad, d_p, d_q, n, cap, out, n_capped);
    dev_free(c, d_in);
    return st;
}

}  // namespace ev

// =================================================================== C ABI

using namespace ev;

extern "C" {

static ev_status run_probe(ev_ctx* c);

const char* ev_last_error(void) { return g_err.c_str(); }

ev_status ev_create(ev_ctx** out, int device, const float* x, const float* y, int32_t n_cases,
                    uint64_t mem_budget_bytes, const ev_allocator* alloc, void* stream)
{
    if (!out || !x || !y || n_cases < 1) return fail(EV_EINVAL, "ev_create: bad arguments");
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(EV_EINVAL, "ev_create: allocator needs alloc and free");
    *out = nullptr;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(EV_EINVAL, "ev_create: no device %d", device);
    HIPCHK(hipSetDevice(device));
    ev_ctx* c = new ev_ctx();
    c->device = device;
    if (alloc) c->ext = *alloc;
    c->budget = mem_budget_bytes;
    {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { delete c; return fail(EV_EDEVICE, "hipMemGetInfo"); }
        // leave room for the runtime's own buffers and other contexts
        const size_t margin = std::max<size_t>((size_t)4 << 30, free_b / 32);
        c->hold_limit = free_b > margin ? free_b - margin : free_b / 2;
        if (c->budget == 0 || c->budget > c->hold_limit) c->budget = c->hold_limit;
    }
    if (exec_init(c->main, (hipStream_t)stream) != EV_OK) { delete c; return EV_EDEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete c; return fail(EV_EDEVICE, "device properties"); }
    c->num_cus = prop.multiProcessorCount;
    for (int i = 0; i < 2; i++) {
        int bpc = 0;
        if (eval_occupancy(i ? 128 : 64, &bpc) != hipSuccess || bpc < 1) bpc = 1;
        c->grid_eval[i] = bpc * c->num_cus;
    }
    {
        int bpc = 0;
        if (run_occupancy(&bpc) != hipSuccess || bpc < 1) bpc = 1;
        c->run_bpc = bpc;
        c->grid_run = bpc * c->num_cus;
        bpc = 0;
        if (chain_occupancy(&bpc) != hipSuccess || bpc < 1) bpc = 1;
        c->grid_chain = bpc * c->num_cus;
    }
    int32_t tid = 0;
    ev_status st = ev_add_cases(c, x, y, n_cases, &tid);
    if (st == EV_OK) st = dev_alloc(c, 256, (void**)&c->d_flag);
    if (st == EV_OK && (st = dev_alloc(c, 256 * sizeof(float), (void**)&c->d_const)) == EV_OK) {
        const std::vector<float> zero(256, 0.0f);
        st = put(c->main, c->d_const, zero.data(), zero.size() * sizeof(float));
    }
    if (st == EV_OK) st = run_probe(c);
    if (st == EV_OK) st = static_scratch_init(device);
    if (st != EV_OK) { ev_destroy(c); return st; }
    *out = c;
    return EV_OK;
}

// One launch of k_run over a one-code stream (END) on case table 0: the
// interpreter's prologue sets the flag word when its jump table cannot be
// used from the address the code object was loaded at; the register-stack
// path is then switched off for the context.
static ev_status run_probe(ev_ctx* c)
{
    Exec& x = c->main;
    void* buf = nullptr;
    ev_status st = dev_alloc(c, 4096, &buf);
    if (st != EV_OK) return st;
    uint32_t* codes = (uint32_t*)buf;                    // [0, 1024): one code and zeros
    RunChunk* chunk = (RunChunk*)((char*)buf + 1024);  // [1024, 1040)
    uint32_t* counter = (uint32_t*)((char*)buf + 1280);
    float* slot = (float*)((char*)buf + 2048);
    std::vector<uint8_t> h(1536, 0);
    const uint32_t end_code = EV_K_END * EV_CODE_NSTRIDE;  // END at position 0
    std::memcpy(h.data(), &end_code, 4);
    const RunChunk rc{0, 0, 0};
    std::memcpy(h.data() + 1024, &rc, sizeof rc);
    const uint32_t zero = 0;
    if ((st = put(x, buf, h.data(), h.size())) == EV_OK) st = put(x, c->d_flag, &zero, 4);
    RunArgs r{};
    r.codes = codes;
    r.chunks = chunk;
    r.n_items = 1;
    r.n_cb = 1;
    r.counter = counter;
    CaseTable t0;
    (void)table_get(c, 0, &t0);
    r.x = t0.d_x;
    r.N = 1;
    r.rowb = 4;
    r.in_res = slot;
    r.out_res = slot;
    r.slab = nullptr;
    r.slab_entries = 0;
    r.flag = c->d_flag;
    r.refs = 0;
    uint32_t flag = 0, flag2 = 0;
    if (st == EV_OK) {
        hipError_t e = launch_run(r, 1, x.stream);
        if (e != hipSuccess) st = hip_fail(e, "probe launch");
    }
    if (st == EV_OK) st = get(x, &flag, c->d_flag, 4);
    // the same one-code stream through the chained launch (its own copy of
    // the handler table): one level, one item, its tree's done counter
    RunLevel* lv = (RunLevel*)((char*)buf + 3072);       // [3072, 3136)
    uint32_t* done = (uint32_t*)((char*)buf + 1536);       // [1536, 1540)
    uint32_t* counter2 = (uint32_t*)((char*)buf + 1792);   // [1792, 1796)
    uint32_t* item_tree = (uint32_t*)((char*)buf + 1800);  // [1800, 1804)
    if (st == EV_OK) {
        RunLevel l0{};
        l0.codes = codes;
        l0.chunks = chunk;
        l0.item_tree = item_tree;
        l0.in_res = slot;
        l0.out_res = slot;
        l0.first = 0;
        l0.n_items = 1;
        l0.refs = 0;
        const uint32_t z4[4] = {0, 0, 0, 0};
        if ((st = put(x, lv, &l0, sizeof l0)) == EV_OK && (st = put(x, done, z4, 4)) == EV_OK &&
            (st = put(x, counter2, z4, 4)) == EV_OK && (st = put(x, item_tree, z4, 4)) == EV_OK &&
            (st = put(x, c->d_flag, &zero, 4)) == EV_OK) {
            ChainArgs ca{};
            ca.levels = lv;
            ca.n_levels = 1;
            ca.total = 1;
            ca.n_cb = 1;
            ca.M = 1;
            ca.counter = counter2;
            ca.need = done;
            ca.done = done;
            ca.x = t0.d_x;
            ca.N = 1;
            ca.rowb = 4;
            ca.flag = c->d_flag;
            hipError_t e = launch_run_chain(ca, 1, x.stream);
            if (e != hipSuccess) st = hip_fail(e, "probe launch");
        }
    }
    if (st == EV_OK) st = get(x, &flag2, c->d_flag, 4);
    if (st == EV_OK) st = sync(x);
    else (void)sync(x);
    dev_free(c, buf);
    if (st == EV_OK && flag) {
        c->run_ok = false;
        c->use_run = false;
    }
    if (st == EV_OK && (flag || flag2)) {
        c->grid_chain = 0;
        c->use_chain = false;
    }
    return st;
}

ev_status ev_add_cases(ev_ctx* c, const float* x, const float* y, int32_t n, int32_t* table)
{
    if (!c || !x || !y || n < 1) return fail(EV_EINVAL, "ev_add_cases: bad arguments");
    HIPCHK(hipSetDevice(c->device));
    CaseTable t;
    t.N = n;
    ev_status st;
    if ((st = dev_alloc(c, (size_t)n * 4, (void**)&t.d_x)) != EV_OK) return st;
    if ((st = dev_alloc(c, (size_t)n * 4, (void**)&t.d_y)) != EV_OK) { dev_free(c, t.d_x); return st; }
    if ((st = put(c->main, t.d_x, x, (size_t)n * 4)) || (st = put(c->main, t.d_y, y, (size_t)n * 4)) ||
        (st = sync(c->main))) {
        dev_free(c, t.d_x);
        dev_free(c, t.d_y);
        return st;
    }
    std::lock_guard<std::mutex> g(c->pop_mu);
    c->tables.push_back(t);
    if (table) *table = (int32_t)c->tables.size() - 1;
    return EV_OK;
}

ev_status ev_destroy(ev_ctx* c)
{
    if (!c) return fail(EV_EINVAL, "ev_destroy: NULL context");
    (void)hipSetDevice(c->device);
    serve_stop(c);
    evolve_release(c);
    (void)sync(c->main);
    for (auto& kv : c->pops) pop_free(c, kv.second);
    c->pops.clear();
    for (auto& t : c->tables) { dev_free(c, t.d_x); dev_free(c, t.d_y); }
    dev_free(c, c->d_flag);
    dev_free(c, c->d_const);
    exec_free(c, c->main);
    dev_cache_release(c);
    delete c;
    return EV_OK;
}

ev_status ev_load_trees(ev_ctx* c, const uint8_t* bytes, const uint64_t* off, int32_t n, uint32_t flags,
                        ev_pop* out_pop, int32_t* bad_tree)
{
    if (!c || !off || n < 0 || !out_pop) return fail(EV_EINVAL, "ev_load_trees: bad arguments");
    if (bad_tree) *bad_tree = -1;
    HIPCHK(hipSetDevice(c->device));
    std::vector<uint64_t> h_off(n + 1);
    if (flags & EV_DEVICE_PTR) {
        ev_status st0 = get(c->main, h_off.data(), off, (n + 1) * sizeof(uint64_t));
        if (st0 == EV_OK) st0 = sync(c->main);
        if (st0 != EV_OK) return st0;
    } else {
        std::memcpy(h_off.data(), off, (n + 1) * sizeof(uint64_t));
    }
    if (h_off[0] != 0) return fail(EV_EINVAL, "ev_load_trees: off[0] must be 0");
    for (int32_t t = 0; t < n; t++) {
        if (h_off[t + 1] <= h_off[t]) {
            if (bad_tree) *bad_tree = t;
            return fail(EV_EMALFORMED, "tree %d is empty or offsets decrease", t);
        }
    }
    const uint64_t total = h_off[n];
    if (total > 0 && !bytes) return fail(EV_EINVAL, "ev_load_trees: NULL bytes");
    uint8_t* d = nullptr;
    ev_status st = dev_alloc(c, total + EV_POP_PAD, (void**)&d);
    if (st != EV_OK) return st;
    hipError_t e = hipSuccess;
    if (flags & EV_DEVICE_PTR) {
        e = hipMemcpyAsync(d, bytes, total, hipMemcpyDeviceToDevice, c->stream);
    } else if ((st = put(c->main, d, bytes, total)) != EV_OK) {
        dev_free(c, d);
        return st;
    }
    if (e == hipSuccess) e = launch_fill_u8(d + total, EV_POP_PAD, 0xFF, c->stream);
    if (e != hipSuccess) { dev_free(c, d); return hip_fail(e, "upload trees"); }
    Pop* P = nullptr;
    ev_status st2 = pop_build(c, c->main, d, h_off, &P, bad_tree);
    if (st2 != EV_OK) return st2;
    *out_pop = pop_register(c, P);
    return EV_OK;
}

ev_status ev_pop_info(ev_ctx* c, ev_pop pop, int32_t* n_trees, uint64_t* total_bytes)
{
    if (!c) return fail(EV_EINVAL, "NULL context");
    Pop* P = pop_get(c, pop);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", pop);
    if (n_trees) *n_trees = P->M;
    if (total_bytes) *total_bytes = P->total;
    return EV_OK;
}

ev_status ev_get_trees(ev_ctx* c, ev_pop pop, uint8_t* bytes, uint64_t* off, uint64_t cap_bytes)
{
    if (!c) return fail(EV_EINVAL, "NULL context");
    Pop* P = pop_get(c, pop);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", pop);
    if (cap_bytes < P->total || (!bytes && P->total) || !off) return fail(EV_EINVAL, "ev_get_trees: buffer too small");
    HIPCHK(hipSetDevice(c->device));
    ev_status st = get(c->main, bytes, P->d_bytes, P->total);
    if (st == EV_OK) st = sync(c->main);
    if (st != EV_OK) return st;
    std::memcpy(off, P->h_off.data(), P->h_off.size() * sizeof(uint64_t));
    return EV_OK;
}

ev_status ev_free_pop(ev_ctx* c, ev_pop pop)
{
    if (!c) return fail(EV_EINVAL, "NULL context");
    Pop* P = nullptr;
    {
        std::lock_guard<std::mutex> g(c->pop_mu);
        auto it = c->pops.find(pop);
        if (it == c->pops.end()) return fail(EV_ENOTFOUND, "no population %d", pop);
        P = it->second;
        c->pops.erase(it);
        if (P->refs > 0) {
            P->dead = true;  // a serving job still reads it: freed when it is done
            return EV_OK;
        }
    }
    (void)hipSetDevice(c->device);
    (void)sync(c->main);
    pop_free(c, P);
    return EV_OK;
}

ev_status ev_eval_fitness(ev_ctx* c, ev_pop pop, int32_t table, float* fitness, float* per_case, int32_t* hits,
                          uint32_t flags)
{
    if (!c || !fitness) return fail(EV_EINVAL, "ev_eval_fitness: bad arguments");
    Pop* P = pop_get(c, pop);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", pop);
    CaseTable ct;
    if (!table_get(c, table, &ct)) return fail(EV_EINVAL, "no case table %d", table);
    HIPCHK(hipSetDevice(c->device));
    const int32_t N = ct.N;
    float* d_pc = nullptr;
    if (per_case) {
        if (flags & EV_OUT_DEVICE) {
            d_pc = per_case;
        } else {
            ResCache* rc = nullptr;
            ev_status st = rescache_get(c, c->main, P, table, &rc);
            if (st != EV_OK) return st;
            if (!rc->d_per_case) {
                st = dev_alloc(c, (size_t)std::max(1, P->M) * N * sizeof(float), (void**)&rc->d_per_case);
                if (st != EV_OK) return st;
            }
            d_pc = rc->d_per_case;
        }
    }
    int32_t* d_hits = nullptr;
    if (hits) {
        if (flags & EV_OUT_DEVICE) {
            d_hits = hits;
        } else {
            if (!P->d_hits) {
                ev_status st = dev_alloc(c, (size_t)std::max(1, P->M) * sizeof(int32_t), (void**)&P->d_hits);
                if (st != EV_OK) return st;
            }
            d_hits = P->d_hits;
        }
    }
    const bool verdict = P->plan.err_pending;
    ev_status st = eval_enqueue(c, c->main, P, table, P->d_fit, d_pc, true, d_hits, true);
    if (st != EV_OK) return st;
    P->hits_valid = false;
    if (flags & EV_OUT_DEVICE) {
        if (P->M) HIPCHK(hipMemcpyAsync(fitness, P->d_fit, (size_t)P->M * 4, hipMemcpyDeviceToDevice, c->stream));
        if (verdict && ((st = sync(c->main)) != EV_OK || (st = plan_verdict(P)) != EV_OK)) return st;
        P->fit_valid = true;
        return EV_OK;
    }
    if ((st = get(c->main, fitness, P->d_fit, (size_t)P->M * 4)) != EV_OK) return st;
    if (per_case && (st = get(c->main, per_case, d_pc, (size_t)P->M * N * 4)) != EV_OK) return st;
    if (hits && (st = get(c->main, hits, d_hits, (size_t)P->M * 4)) != EV_OK) return st;
    if ((st = sync(c->main)) != EV_OK || (st = plan_verdict(P)) != EV_OK) return st;
    P->fit_valid = true;
    P->hits_valid = hits != nullptr;
    return EV_OK;
}

ev_status ev_population_stats(ev_ctx* c, ev_pop pop, ev_pop_stats* out, uint32_t* depth)
{
    if (!c || !out) return fail(EV_EINVAL, "ev_population_stats: bad arguments");
    Pop* P = pop_get(c, pop);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", pop);
    if (!P->fit_valid) return fail(EV_EINVAL, "ev_population_stats: the population has not been evaluated");
    HIPCHK(hipSetDevice(c->device));
    Exec& x = c->main;
    const uint32_t M = (uint32_t)P->M;
    *out = ev_pop_stats{};
    if (M == 0) return EV_OK;
    void *d_ps = nullptr, *d_h = nullptr, *d_base = nullptr, *d_stack = nullptr;
    auto cleanup = [&]() {
        (void)sync(x);
        for (void* q : {d_ps, d_h, d_base, d_stack}) dev_free(c, q);
    };
    ev_status st;
    PopStatsDev ps{};
    std::vector<uint32_t> h(M), d(M);
    if ((st = dev_alloc(c, sizeof(PopStatsDev), &d_ps)) || (st = dev_alloc(c, (size_t)M * 8, &d_h))) {
        cleanup();
        return st;
    }
    HIPCHK(launch_pop_stats(P->d_fit, P->d_off, M, (PopStatsDev*)d_ps, x.stream));
    HIPCHK(launch_tree_height(P->d_bytes, P->d_off, M, (uint32_t*)d_h, x.stream));
    if ((st = get(x, &ps, d_ps, sizeof ps)) || (st = get(x, h.data(), d_h, (size_t)M * 4)) || (st = sync(x))) {
        cleanup();
        return st;
    }
    // each tree's depth stack: as many entries as its stack machine's height
    std::vector<uint64_t> base((size_t)M + 1, 0);
    for (uint32_t t = 0; t < M; t++) base[t + 1] = base[t] + h[t];
    int32_t best_hits = -1;
    if ((st = dev_alloc(c, base.size() * 8, &d_base)) || (st = dev_alloc(c, base[M] * 4 + 4, &d_stack)) ||
        (st = put(x, d_base, base.data(), base.size() * 8))) {
        cleanup();
        return st;
    }
    HIPCHK(launch_tree_depth(P->d_bytes, P->d_off, M, (uint64_t*)d_base, (uint32_t*)d_stack, (uint32_t*)d_h,
                             x.stream));
    float bf = 0;
    if (ps.best >= M) {
        cleanup();
        return fail(EV_EDEVICE, "internal: no best tree among %u", M);
    }
    if ((st = get(x, d.data(), d_h, (size_t)M * 4)) || (st = get(x, &bf, P->d_fit + ps.best, 4)) ||
        (P->hits_valid && (st = get(x, &best_hits, P->d_hits + ps.best, 4))) || (st = sync(x))) {
        cleanup();
        return st;
    }
    cleanup();
    out->best_fitness = bf;
    out->best_tree = (int32_t)ps.best;
    out->best_hits = best_hits;
    out->converged = (int32_t)ps.converged;
    out->mean_fitness = ps.n_finite ? ps.sum_fit / ps.n_finite : std::nan("");
    out->best_size = P->h_off[ps.best + 1] - P->h_off[ps.best];
    out->min_size = ps.min_size;
    out->max_size = ps.max_size;
    out->mean_size = ps.sum_size / M;
    uint64_t dsum = 0;
    uint32_t dmin = UINT32_MAX, dmax = 0;
    for (uint32_t t = 0; t < M; t++) {
        dsum += d[t];
        dmin = std::min(dmin, d[t]);
        dmax = std::max(dmax, d[t]);
    }
    out->best_depth = d[ps.best];
    out->min_depth = dmin;
    out->max_depth = dmax;
    out->mean_depth = (double)dsum / M;
    if (depth) std::memcpy(depth, d.data(), (size_t)M * 4);
    return EV_OK;
}

ev_status ev_crossover(ev_ctx* c, ev_pop mums_pop, ev_pop dads_pop, const int32_t* mum, const int32_t* dad,
                       const uint64_t* p, const uint64_t* q, int32_t n, uint64_t size_cap, ev_pop* out,
                       int32_t* n_capped)
{
    if (!c || n < 0 || !out || (n > 0 && (!mum || !dad || !p || !q))) return fail(EV_EINVAL, "ev_crossover: bad arguments");
    Pop* A = pop_get(c, mums_pop);
    Pop* B = pop_get(c, dads_pop);
    if (!A || !B) return fail(EV_ENOTFOUND, "ev_crossover: unknown population");
    HIPCHK(hipSetDevice(c->device));
    Pop* C = nullptr;
    ev_status st = crossover_build(c, c->main, A, B, mum, dad, p, q, n, size_cap, &C, n_capped);
    if (st != EV_OK) return st;
    *out = pop_register(c, C);
    return EV_OK;
}

ev_status ev_generation(ev_ctx* c, ev_pop parents, const float* fitness, uint64_t seed, uint64_t gen,
                        int32_t tournament, uint64_t size_cap, ev_pop* out, int32_t* n_capped)
{
    if (!c || !out || tournament < 1) return fail(EV_EINVAL, "ev_generation: bad arguments");
    Pop* P = pop_get(c, parents);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", parents);
    if (!fitness && !P->fit_valid) return fail(EV_EINVAL, "ev_generation: parents have no fitness yet");
    HIPCHK(hipSetDevice(c->device));
    const int32_t M = P->M;
    void* d_sel = nullptr;
    ev_status st = dev_alloc(c, (size_t)std::max(1, M) * 24, &d_sel);
    if (st != EV_OK) return st;
    int32_t* d_mum = (int32_t*)d_sel;
    int32_t* d_dad = d_mum + std::max(1, M);
    uint64_t* d_p = (uint64_t*)((char*)d_sel + (size_t)std::max(1, M) * 8);
    uint64_t* d_q = d_p + std::max(1, M);
    hipError_t e = launch_select(fitness ? fitness : P->d_fit, P->d_off, (uint32_t)M, tournament, seed, gen, d_mum,
                                 d_dad, d_p, d_q, c->stream);
    if (e != hipSuccess) {
        dev_free(c, d_sel);
        return hip_fail(e, "selection");
    }
    Pop* C = nullptr;
    // the children's last validation verdict is read with their first
    // evaluation (their k_run launches check it on the device)
    st = crossover_build_dev(c, c->main, P, P, d_mum, d_dad, d_p, d_q, M, size_cap, &C, n_capped, true);
    dev_free(c, d_sel);
    if (st != EV_OK) return st;
    *out = pop_register(c, C);
    return EV_OK;
}

ev_status ev_get_plan_info(ev_ctx* c, ev_pop pop, ev_plan_info* info)
{
    if (!c || !info) return fail(EV_EINVAL, "bad arguments");
    Pop* P = pop_get(c, pop);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", pop);
    info->levels = (int32_t)P->plan.levels.size();
    info->chunks = P->plan.chunks_total;
    info->slots = P->plan.slots_total;
    info->max_stack = P->plan.max_stack;
    info->plan_bytes = P->plan.bytes;
    return EV_OK;
}

ev_status ev_set_constants(ev_ctx* c, const float* consts, int32_t n)
{
    if (!c || n < 0 || n > (int32_t)MAX_CONSTS || (n > 0 && !consts))
        return fail(EV_EINVAL, "ev_set_constants: bad arguments");
    {
        std::lock_guard<std::mutex> g(c->pop_mu);
        if (!c->pops.empty()) return fail(EV_EINVAL, "ev_set_constants: the context holds populations");
    }
    if (c->serve) return fail(EV_EINVAL, "ev_set_constants: the serving loop has started");
    HIPCHK(hipSetDevice(c->device));
    std::vector<float> v(256, 0.0f);
    for (int32_t i = 0; i < n; i++) v[(size_t)i] = consts[i];
    ev_status st = put(c->main, c->d_const, v.data(), v.size() * sizeof(float));
    if (st == EV_OK) st = sync(c->main);
    if (st != EV_OK) return st;
    c->n_consts = n;
    return EV_OK;
}

ev_status ev_get_level_info(ev_ctx* c, ev_pop pop, int32_t level, ev_level_info* info)
{
    if (!c || !info) return fail(EV_EINVAL, "bad arguments");
    Pop* P = pop_get(c, pop);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", pop);
    if (level < 0 || level >= (int32_t)P->plan.levels.size()) return fail(EV_EINVAL, "no plan level %d", level);
    const Level& L = P->plan.levels[level];
    info->tokens = L.tokens;
    info->trees = L.trees;
    info->items = L.n_run + L.n_chunks;
    info->slots = L.n_out;
    // the launch of an evaluation on the context's stream that runs the level
    const int cf = chain_first(c, c->main, P);
    info->launch = (uint32_t)(cf >= 0 && level >= cf ? cf : level);
    info->codes = L.n_codes;
    return EV_OK;
}

ev_status ev_set_tuning(ev_ctx* c, uint32_t chunk, uint32_t chunk_hi, uint32_t lds_depth, uint32_t flags)
{
    if (!c) return fail(EV_EINVAL, "NULL context");
    if (lds_depth != 0 && lds_depth != 64 && lds_depth != 128) return fail(EV_EINVAL, "lds_depth must be 64 or 128");
    if ((chunk != 0 && chunk < 64) || (chunk_hi != 0 && chunk_hi < 64))
        return fail(EV_EINVAL, "work items must be at least 64 tokens");
    c->use_run = c->run_ok && (flags & EV_TUNE_NO_REGSTACK) == 0;
    c->test_fail_check = (flags & EV_TUNE_TEST_FAIL_CHECK) != 0;
    c->use_record = (flags & EV_TUNE_NO_RECORD) == 0;
    c->use_reuse = (flags & EV_TUNE_NO_REUSE) == 0;
    c->use_chain = c->grid_chain > 0 && (flags & EV_TUNE_NO_CHAIN) == 0;
    if (chunk) c->chunk = chunk;
    if (chunk_hi) c->chunk_hi = chunk_hi;
    if (lds_depth) c->lds_depth = (int)lds_depth;
    return EV_OK;
}

// ------------------------------------------------------------- autotuner

struct TuneKey {
    std::string arch;
    int32_t n_cases;
    int32_t size_bin, tree_bin;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(arch, n_cases, size_bin, tree_bin) < std::tie(o.arch, o.n_cases, o.size_bin, o.tree_bin);
    }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, ev_tune_choice> g_tune_cache;

static int32_t log2_bin(uint64_t v)
{
    int32_t b = 0;
    while (v > 1) {
        v >>= 1;
        b++;
    }
    return b;
}

// Apply a choice to the context: work-item sizes and the interpreter's grid.
static void tune_apply(ev_ctx* c, const ev_tune_choice& t)
{
    if (t.chunk) c->chunk = t.chunk;
    c->chunk_hi = t.chunk_hi;
    const int w = t.waves_per_cu && (int)t.waves_per_cu < c->run_bpc ? (int)t.waves_per_cu : c->run_bpc;
    c->grid_run = std::max(1, w) * c->num_cus;
}

extern "C" ev_status ev_autotune_ex(ev_ctx* c, ev_pop pop, int32_t table, int32_t reps, uint32_t flags,
                                    ev_tune_choice* choice)
{
    if (!c || reps < 1) return fail(EV_EINVAL, "ev_autotune_ex: bad arguments");
    Pop* P = pop_get(c, pop);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", pop);
    CaseTable ct;
    if (!table_get(c, table, &ct)) return fail(EV_EINVAL, "no case table %d", table);
    HIPCHK(hipSetDevice(c->device));
    Exec& x = c->main;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, c->device));
    const TuneKey key{prop.gcnArchName, ct.N, log2_bin(std::max<uint64_t>(1, P->total)),
                      log2_bin((uint64_t)std::max(1, P->M))};
    // re-plan P with the context's current sizes
    auto replan = [&]() -> ev_status {
        if (ev_status st = sync(x)) return st;
        for (auto& kv : P->res) rescache_free(c, kv.second);
        P->res.clear();
        plan_free(c, P->plan);
        return plan_build(c, x, P, nullptr);
    };
    // median device time of `reps` evaluations (after one that warms up)
    auto measure = [&](float* med) -> ev_status {
        std::vector<float> t;
        for (int32_t r = 0; r <= reps; r++) {
            ev_status st = eval_enqueue(c, x, P, table, P->d_fit, nullptr, true, nullptr);
            if (st == EV_OK) st = sync(x);
            if (st != EV_OK) return st;
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, x.ev0, x.ev1));
            if (r) t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        *med = t[t.size() / 2];
        return EV_OK;
    };
    if (!(flags & EV_AUTOTUNE_NO_CACHE)) {
        ev_tune_choice hit{};
        bool found = false;
        {
            std::lock_guard<std::mutex> g(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                hit = it->second;
                found = true;
            }
        }
        if (found) {
            tune_apply(c, hit);
            if (ev_status st = replan()) return st;
            hit.from_cache = 1;
            if (choice) *choice = hit;
            return EV_OK;
        }
    }
    const ev_tune_choice start{c->chunk, c->chunk_hi, 0, 0, 0.0f};
    ev_tune_choice best = start;
    bool have = false;
    // try one setting; keep it if faster.  A setting whose plan does not fit
    // in memory is skipped.
    auto trial = [&](ev_tune_choice t, bool plan) -> ev_status {
        tune_apply(c, t);
        if (plan) {
            ev_status st = replan();
            if (st == EV_ENOMEM) return EV_OK;
            if (st != EV_OK) return st;
        }
        float ms = 0;
        if (ev_status st = measure(&ms)) {
            if (st != EV_ENOMEM) return st;
            // result slots that do not fit beside the rest: skip the setting
            for (auto& kv : P->res) rescache_free(c, kv.second);
            P->res.clear();
            return EV_OK;
        }
        t.ms = ms;
        if (!have || ms < best.ms) {
            best = t;
            have = true;
        }
        return EV_OK;
    };
    static const uint32_t cand[] = {1024, 2048, 4096, 6144, 8192, 12288, 16384, 32768};
    ev_status st = EV_OK;
    for (uint32_t ch : cand) {
        if (ch > 2 * std::max<uint64_t>(64, P->total)) break;  // no split from here on
        // very large populations: items under 4096 tokens multiply the plan and slots
        if (P->total > (1ull << 30) && ch < 4096) continue;
        if ((st = trial(ev_tune_choice{ch, 0, 0, 0, 0.0f}, true)) != EV_OK) break;
    }
    if (st == EV_OK && have) {
        const uint32_t ch = best.chunk;
        for (uint32_t mul : {1u, 4u})
            if ((st = trial(ev_tune_choice{ch, ch * mul, 0, 0, 0.0f}, true)) != EV_OK) break;
    }
    if (st == EV_OK && have) {
        // the grid: the plan of the best sizes, fewer waves per CU
        const ev_tune_choice b = best;
        tune_apply(c, b);
        if ((st = replan()) == EV_OK) {
            for (int less : {4, 8}) {
                if (c->run_bpc - less < 1) break;
                ev_tune_choice t = b;
                t.waves_per_cu = (uint32_t)(c->run_bpc - less);
                if ((st = trial(t, false)) != EV_OK) break;
            }
        }
    }
    if (st != EV_OK) {
        tune_apply(c, start);
        return st;
    }
    if (!have) {
        tune_apply(c, start);
        return fail(EV_ENOMEM, "ev_autotune: no candidate plan fits in memory");
    }
    tune_apply(c, best);
    if ((st = replan()) != EV_OK) return st;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = best;
    }
    if (choice) *choice = best;
    return EV_OK;
}

extern "C" ev_status ev_tune_cache_save(const char* path)
{
    if (!path) return fail(EV_EINVAL, "ev_tune_cache_save: NULL path");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(EV_EINVAL, "ev_tune_cache_save: cannot write %s", path);
    std::lock_guard<std::mutex> g(g_tune_mu);
    std::fprintf(f, "# arch n_cases size_bin tree_bin chunk chunk_hi waves_per_cu ms\n");
    for (auto& kv : g_tune_cache)
        std::fprintf(f, "%s %d %d %d %u %u %u %.6g\n", kv.first.arch.c_str(), kv.first.n_cases, kv.first.size_bin,
                     kv.first.tree_bin, kv.second.chunk, kv.second.chunk_hi, kv.second.waves_per_cu, kv.second.ms);
    const bool ok = std::fclose(f) == 0;
    return ok ? EV_OK : fail(EV_EINVAL, "ev_tune_cache_save: write to %s failed", path);
}

extern "C" ev_status ev_tune_cache_load(const char* path)
{
    if (!path) return fail(EV_EINVAL, "ev_tune_cache_load: NULL path");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(EV_EINVAL, "ev_tune_cache_load: cannot read %s", path);
    std::map<TuneKey, ev_tune_choice> got;
    char line[512];
    int ln = 0;
    while (std::fgets(line, sizeof line, f)) {
        ln++;
        if (line[0] == '#' || line[0] == '\n') continue;
        char arch[256];
        int n, sb, tb;
        unsigned ch, hi, w;
        float ms;
        if (std::sscanf(line, "%255s %d %d %d %u %u %u %f", arch, &n, &sb, &tb, &ch, &hi, &w, &ms) != 8 || ch < 64 ||
            (hi != 0 && hi < 64)) {
            std::fclose(f);
            return fail(EV_EINVAL, "ev_tune_cache_load: %s line %d is malformed", path, ln);
        }
        got[TuneKey{arch, n, sb, tb}] = ev_tune_choice{ch, hi, w, 0, ms};
    }
    std::fclose(f);
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (auto& kv : got) g_tune_cache[kv.first] = kv.second;
    return EV_OK;
}

extern "C" ev_status ev_autotune(ev_ctx* c, ev_pop pop, int32_t table, int32_t reps, uint32_t* best_chunk,
                                 float* best_ms)
{
    ev_tune_choice t{};
    ev_status st = ev_autotune_ex(c, pop, table, reps, EV_AUTOTUNE_NO_CACHE, &t);
    if (st != EV_OK) return st;
    if (best_chunk) *best_chunk = t.chunk;
    if (best_ms) *best_ms = t.ms;
    return EV_OK;
}

ev_status ev_last_level_times(ev_ctx* c, float* ms, int32_t cap, int32_t* n_levels)
{
    if (!c || (cap > 0 && !ms)) return fail(EV_EINVAL, "ev_last_level_times: bad arguments");
    Exec& x = c->main;
    const int32_t n = (int32_t)x.n_levels_timed;
    if (n_levels) *n_levels = n;
    if (n == 0) return EV_OK;
    HIPCHK(hipEventSynchronize(x.evl[n - 1]));
    hipEvent_t prev = x.ev0;
    for (int32_t i = 0; i < n && i < cap; i++) {
        HIPCHK(hipEventElapsedTime(&ms[i], prev, x.evl[i]));
        prev = x.evl[i];
    }
    return EV_OK;
}

ev_status ev_last_timing(ev_ctx* c, float* eval_ms, float* interp_ms)
{
    if (!c) return fail(EV_EINVAL, "NULL context");
    HIPCHK(hipEventSynchronize(c->main.ev1));
    float a = 0, b = 0;
    HIPCHK(hipEventElapsedTime(&a, c->main.ev0, c->main.ev1));
    HIPCHK(hipEventElapsedTime(&b, c->main.evi0, c->main.evi1));
    if (eval_ms) *eval_ms = a;
    if (interp_ms) *interp_ms = b;
    return EV_OK;
}

}  // extern "C"
