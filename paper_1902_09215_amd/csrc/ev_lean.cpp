// The memory-lean generational loop: ev_evolve with EV_EVOLVE_LEAN.
//
// Sec. 2.3 notes that a generation need not hold 2M trees (all parents and
// all children) if each parent is deleted as soon as its last child has
// been made, and that a heap of its own for the population would do this
// without the cost of general-purpose freeing.  Here the population is such
// a heap: one device arena in which every tree lies anywhere (a start and a
// length each), managed on the host as a list of free byte ranges.
//
// A generation selects and plans every child first (on the device, as on
// the host-driven path), reads the children's lengths back, and then makes
// them in batches, in the order of their lower parent index.  In that order
// parent i is no longer needed once every child whose lower parent is at
// most i has been made, so parents die from the front of the index range
// while children are made; after each batch the bytes of the parents whose
// last child it held become free for the next batches' children.  The
// placement of the whole generation is worked out on the host before its
// copies are queued (the copies of a batch are queued after those of the
// batches before it, so no child overwrites a parent still being read).
// With parents drawn evenly, at most about 1.25 populations' worth of trees
// are alive at once (against 2 for separate parent and child buffers), plus
// a batch.
//
// The children are evaluated in place (their plan reads the arena at each
// tree's start), so the heap is the only copy of a generation.  If a child
// finds no free range, the arena is replaced by a larger one, the parents
// are packed at its front, and the placement is worked out again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <numeric>

#include "ev_runtime.h"

namespace ev {

// Free byte ranges of the arena, first fit, merged with their neighbours.
class Holes {
public:
    void reset(uint64_t cap) { free_.clear(); if (cap) free_[0] = cap; }
    void add(uint64_t at, uint64_t n)
    {
        if (!n) return;
        auto next = free_.lower_bound(at);
        if (next != free_.end() && at + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == at) {
                prev->second += n;
                return;
            }
        }
        free_[at] = n;
    }
    bool take(uint64_t n, uint64_t* at)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *at = it->first;
            const uint64_t rest = it->second - n, from = it->first + n;
            free_.erase(it);
            if (rest) free_[from] = rest;
            return true;
        }
        return false;
    }

private:
    std::map<uint64_t, uint64_t> free_;
};

struct LeanHeap {
    uint8_t* arena = nullptr;
    uint64_t cap = 0;  // bytes for trees (EV_POP_PAD bytes of 0xFF follow)
    std::vector<uint64_t> start, len;
};

// A new arena of cap bytes holding the trees of `h` packed in index order
// (the old arena is freed when free_old is set).
static ev_status heap_repack(ev_ctx* c, LeanHeap& h, uint64_t cap, bool free_old)
{
    Exec& x = c->main;
    hipStream_t s = c->stream;
    const size_t M = h.start.size();
    uint8_t* na = nullptr;
    ev_status st = dev_alloc(c, cap + EV_POP_PAD, (void**)&na);
    if (st != EV_OK) return st;
    HIPCHK(launch_fill_u8(na + cap, EV_POP_PAD, 0xFF, s));
    std::vector<uint64_t> ns(M);
    uint64_t o = 0;
    for (size_t t = 0; t < M; t++) {
        ns[t] = o;
        o += h.len[t];
    }
    if (M) {
        // each tree as a child that is a copy of its mum, to its packed place
        std::vector<XoPlan> pl(M);
        std::vector<uint32_t> idx(M);
        std::vector<uint64_t> pf(M + 1, 0);
        for (size_t t = 0; t < M; t++) {
            XoPlan v{};
            v.mum_off = h.start[t];
            v.child_len = h.len[t];
            v.copy_mum = 1;
            pl[t] = v;
            idx[t] = (uint32_t)t;
            pf[t + 1] = pf[t] + (h.len[t] + 4095) / 4096;
        }
        void* buf = nullptr;
        const size_t o_idx = M * sizeof(XoPlan), o_at = (o_idx + M * 4 + 7) & ~(size_t)7, o_pf = o_at + M * 8;
        if ((st = dev_alloc(c, o_pf + (M + 1) * 8, &buf)) != EV_OK) {
            dev_free(c, na);
            return st;
        }
        XoPlan* d_pl = (XoPlan*)buf;
        uint32_t* d_idx = (uint32_t*)((char*)buf + o_idx);
        uint64_t* d_at = (uint64_t*)((char*)buf + o_at);
        uint64_t* d_pf = (uint64_t*)((char*)buf + o_pf);
        hipError_t e = hipSuccess;
        if ((st = put(x, d_pl, pl.data(), M * sizeof(XoPlan))) == EV_OK &&
            (st = put(x, d_idx, idx.data(), M * 4)) == EV_OK && (st = put(x, d_at, ns.data(), M * 8)) == EV_OK &&
            (st = put(x, d_pf, pf.data(), (M + 1) * 8)) == EV_OK)
            e = launch_xo_copy_at(h.arena, d_pl, d_idx, d_at, d_pf, (uint32_t)M, pf[M], na, s);
        if (st == EV_OK && e != hipSuccess) st = hip_fail(e, "packing the heap");
        if (st == EV_OK) st = sync(x);
        dev_free(c, buf);
        if (st != EV_OK) {
            dev_free(c, na);
            return st;
        }
    }
    if (free_old) dev_free(c, h.arena);
    h.arena = na;
    h.cap = cap;
    h.start = ns;
    return EV_OK;
}

// The placement of one generation's children: per child its start, the
// batches (positions in `order`), and the most bytes alive at once.
struct Placement {
    std::vector<uint64_t> at;
    std::vector<uint32_t> order;
    std::vector<uint32_t> batch_end;  // exclusive ends of the batches in `order`
    uint64_t peak = 0;
};

static bool place(const LeanHeap& h, const std::vector<int32_t>& mum, const std::vector<int32_t>& dad,
                  const std::vector<uint64_t>& clen, uint32_t batch, Placement* out)
{
    const uint32_t M = (uint32_t)h.start.size();
    Placement p;
    p.at.assign(M, 0);
    p.order.resize(M);
    std::iota(p.order.begin(), p.order.end(), 0u);
    auto key = [&](uint32_t j) { return (uint32_t)std::min(mum[j], dad[j]); };
    std::stable_sort(p.order.begin(), p.order.end(), [&](uint32_t a, uint32_t b) { return key(a) < key(b); });
    // each parent's last use (its position in `order`), -1 for none
    std::vector<int64_t> last(M, -1);
    for (uint32_t pos = 0; pos < M; pos++) {
        const uint32_t j = p.order[pos];
        last[mum[j]] = std::max<int64_t>(last[mum[j]], pos);
        last[dad[j]] = std::max<int64_t>(last[dad[j]], pos);
    }
    // parents freed after each position
    std::vector<std::vector<uint32_t>> free_after(M);
    Holes holes;
    holes.reset(h.cap);
    // the parents' bytes are taken; unused parents are free at once
    std::vector<std::pair<uint64_t, uint64_t>> used;
    uint64_t live = 0;
    for (uint32_t i = 0; i < M; i++)
        if (last[i] >= 0) {
            used.push_back({h.start[i], h.len[i]});
            free_after[last[i]].push_back(i);
            live += h.len[i];
        }
    {
        // holes = [0, cap) minus the used ranges
        std::sort(used.begin(), used.end());
        holes.reset(0);
        uint64_t o = 0;
        for (auto& u : used) {
            if (u.first > o) holes.add(o, u.first - o);
            o = std::max(o, u.first + u.second);
        }
        if (h.cap > o) holes.add(o, h.cap - o);
    }
    p.peak = live;
    for (uint32_t b0 = 0; b0 < M; b0 += batch) {
        const uint32_t b1 = std::min(M, b0 + batch);
        for (uint32_t pos = b0; pos < b1; pos++) {
            const uint32_t j = p.order[pos];
            if (!holes.take(clen[j], &p.at[j])) return false;
            live += clen[j];
        }
        p.peak = std::max(p.peak, live);
        for (uint32_t pos = b0; pos < b1; pos++)
            for (uint32_t i : free_after[pos]) {
                holes.add(h.start[i], h.len[i]);
                live -= h.len[i];
            }
        p.batch_end.push_back(b1);
    }
    *out = std::move(p);
    return true;
}

// Release what evaluate_heap made, but not the arena it read.
static void view_release(ev_ctx* c, Pop* v)
{
    if (!v) return;
    v->d_bytes = nullptr;  // the arena's
    pop_free(c, v);
}

// The heap's trees evaluated in place: fitness into d_fit (device).
static ev_status evaluate_heap(ev_ctx* c, const LeanHeap& h, int32_t table, float* d_fit)
{
    Exec& x = c->main;
    Pop* v = new Pop();
    v->d_bytes = h.arena;
    v->M = (int32_t)h.start.size();
    v->h_off.assign(h.start.size() + 1, 0);
    for (size_t t = 0; t < h.start.size(); t++) v->h_off[t + 1] = v->h_off[t] + h.len[t];
    v->h_start = h.start;
    v->total = v->h_off.back();
    // the plan reads the trees at their starts; fitness goes to d_fit
    ev_status st = plan_build(c, x, v, nullptr);
    if (st == EV_OK) st = eval_enqueue(c, x, v, table, d_fit, nullptr, false, nullptr);
    if (st == EV_OK) st = sync(x);
    view_release(c, v);
    return st;
}

ev_status evolve_lean(ev_ctx* c, Pop* P, const float* fitness, int32_t table, uint64_t seed, uint64_t gen0,
                      int32_t n_gen, int32_t tournament, uint64_t size_cap, ev_pop* out, float* fit_history,
                      int32_t* capped_history, ev_evolve_report* rep)
{
    Exec& x = c->main;
    hipStream_t s = c->stream;
    const int32_t M = P->M;
    const size_t m = (size_t)std::max(1, M);
    LeanHeap h;
    h.start.resize(M);
    h.len.resize(M);
    for (int32_t t = 0; t < M; t++) {
        h.start[t] = P->h_off[t];
        h.len[t] = P->h_off[t + 1] - P->h_off[t];
    }
    // per-generation device scratch
    float* d_fit = nullptr;
    void* d_sel = nullptr;  // mum, dad (int32), p, q, qb (2M), qp (2M), ends (2M), start, len, off (2M + 6)
    XoPlan* d_plan = nullptr;
    void* d_batch = nullptr;  // idx (u32 x M), at (u64 x M), pf (u64 x M + batches)
    ev_status st = EV_OK;
    auto cleanup = [&]() {
        (void)sync(x);
        for (void* q : {(void*)d_fit, d_sel, (void*)d_plan, d_batch, (void*)h.arena}) dev_free(c, q);
        h.arena = nullptr;
    };
    const uint32_t batch = (uint32_t)std::max<int32_t>(1, (M + 15) / 16);
    const size_t n_batches = (m + batch - 1) / batch;
    const size_t sel_bytes = m * 8 + m * 16 + m * 48 + m * 16 + (2 * m + 6) * 8;
    const size_t o_at = (m * 4 + 7) & ~(size_t)7, o_pf = o_at + m * 8;
    if ((st = dev_alloc(c, m * 4, (void**)&d_fit)) != EV_OK || (st = dev_alloc(c, sel_bytes, &d_sel)) != EV_OK ||
        (st = dev_alloc(c, m * sizeof(XoPlan), (void**)&d_plan)) != EV_OK ||
        (st = dev_alloc(c, o_pf + (m + n_batches) * 8, &d_batch)) != EV_OK) {
        cleanup();
        return st;
    }
    int32_t* d_mum = (int32_t*)d_sel;
    int32_t* d_dad = d_mum + m;
    uint64_t* d_p = (uint64_t*)((char*)d_sel + m * 8);
    uint64_t* d_q = d_p + m;
    uint64_t* d_qb = d_q + m;
    uint64_t* d_qp = d_qb + 2 * m;
    uint64_t* d_ends = d_qp + 2 * m;
    uint64_t* d_start = d_ends + 2 * m;
    uint64_t* d_len = d_start + m;
    uint64_t* d_off = d_len + m;
    uint32_t* d_idx = (uint32_t*)d_batch;
    uint64_t* d_at = (uint64_t*)((char*)d_batch + o_at);
    uint64_t* d_pf = (uint64_t*)((char*)d_batch + o_pf);
    // the parents, copied into an arena of their own with room for half a
    // population more (the caller's population is left as it is)
    h.arena = P->d_bytes;
    if ((st = heap_repack(c, h, P->total + P->total / 2 + ((uint64_t)64 << 10), false)) != EV_OK) {
        h.arena = nullptr;
        cleanup();
        return st;
    }
    HIPCHK(hipMemcpyAsync(d_fit, fitness ? fitness : P->d_fit, (size_t)M * 4, hipMemcpyDeviceToDevice, s));
    std::vector<int32_t> mum(M), dad(M);
    std::vector<uint64_t> off((size_t)M + 4), clen(M);
    std::vector<uint32_t> idx(M);
    std::vector<uint64_t> at(M), pf;
    for (int32_t i = 0; i < n_gen; i++) {
        const uint64_t gen = gen0 + (uint64_t)i;
        if ((st = put(x, d_start, h.start.data(), (size_t)M * 8)) != EV_OK ||
            (st = put(x, d_len, h.len.data(), (size_t)M * 8)) != EV_OK) {
            cleanup();
            return st;
        }
        // selection and the children's plans, as on the host-driven path
        hipError_t e = launch_select(d_fit, d_start, (uint32_t)M, tournament, seed, gen, d_mum, d_dad, d_p, d_q, s,
                                     nullptr, d_len);
        if (e == hipSuccess) e = launch_xo_query(d_start, d_start, d_mum, d_dad, d_p, d_q, (uint32_t)M, d_qb, d_qp, s);
        if (e == hipSuccess) e = launch_subtree_end(h.arena, d_qb, d_qp, 2u * (uint32_t)M, d_ends, s);
        if (e == hipSuccess)
            e = launch_xo_plan(d_start, d_start, d_mum, d_dad, d_p, d_q, d_ends, (uint32_t)M, size_cap, d_plan, d_off, s,
                               d_len);
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e, "lean generation");
        }
        if ((st = get(x, mum.data(), d_mum, (size_t)M * 4)) != EV_OK ||
            (st = get(x, dad.data(), d_dad, (size_t)M * 4)) != EV_OK ||
            (st = get(x, off.data(), d_off, ((size_t)M + 4) * 8)) != EV_OK || (st = sync(x)) != EV_OK) {
            cleanup();
            return st;
        }
        uint64_t total = 0;
        for (int32_t j = 0; j < M; j++) {
            clen[j] = off[j + 1] - off[j];  // off[M] is the total
            total += clen[j];
        }
        const uint64_t parents = std::accumulate(h.len.begin(), h.len.end(), (uint64_t)0);
        Placement pl;
        if (!place(h, mum, dad, clen, batch, &pl)) {
            // no free range for a child: a larger arena, parents packed in front
            const uint64_t cap = std::max<uint64_t>(2 * h.cap, parents + total + (parents + total) / 2);
            if ((st = heap_repack(c, h, cap, true)) != EV_OK) {
                cleanup();
                return st;
            }
            rep->lean_repacks++;
            // the children's plans name their parents' places: made again
            // for the packed ones (lengths and points are unchanged)
            if ((st = put(x, d_start, h.start.data(), (size_t)M * 8)) != EV_OK) {
                cleanup();
                return st;
            }
            e = launch_xo_plan(d_start, d_start, d_mum, d_dad, d_p, d_q, d_ends, (uint32_t)M, size_cap, d_plan, d_off,
                               s, d_len);
            if (e != hipSuccess) {
                cleanup();
                return hip_fail(e, "lean generation");
            }
            if (!place(h, mum, dad, clen, batch, &pl)) {
                cleanup();
                return fail(EV_EDEVICE, "internal: no room for the children after repacking the heap");
            }
        }
        // the batches' copies, in order (batch k's piece prefix at b0 + k)
        pf.assign((size_t)M + n_batches, 0);
        uint32_t b0 = 0;
        for (size_t k = 0; k < pl.batch_end.size(); k++) {
            const uint32_t b1 = pl.batch_end[k];
            uint64_t* f = pf.data() + b0 + k;
            for (uint32_t pos = b0; pos < b1; pos++) {
                idx[pos] = pl.order[pos];
                at[pos] = pl.at[pl.order[pos]];
                f[pos - b0 + 1] = f[pos - b0] + (clen[pl.order[pos]] + 4095) / 4096;
            }
            b0 = b1;
        }
        if ((st = put(x, d_idx, idx.data(), (size_t)M * 4)) != EV_OK ||
            (st = put(x, d_at, at.data(), (size_t)M * 8)) != EV_OK ||
            (st = put(x, d_pf, pf.data(), pf.size() * 8)) != EV_OK) {
            cleanup();
            return st;
        }
        b0 = 0;
        for (size_t k = 0; k < pl.batch_end.size() && e == hipSuccess; k++) {
            const uint32_t b1 = pl.batch_end[k];
            const uint64_t* f = pf.data() + b0 + k;
            e = launch_xo_copy_at(h.arena, d_plan, d_idx + b0, d_at + b0, d_pf + b0 + k, b1 - b0, f[b1 - b0], h.arena,
                                  s);
            b0 = b1;
        }
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e, "lean copies");
        }
        h.start = pl.at;
        h.len = clen;
        rep->lean_peak_bytes = std::max(rep->lean_peak_bytes, pl.peak);
        rep->lean_two_buffer_bytes = std::max(rep->lean_two_buffer_bytes, parents + total);
        rep->lean_arena_bytes = std::max(rep->lean_arena_bytes, h.cap);
        // the children evaluated in place
        if ((st = evaluate_heap(c, h, table, d_fit)) != EV_OK) {
            cleanup();
            return st;
        }
        if (fit_history && (st = get(x, fit_history + (size_t)i * M, d_fit, (size_t)M * 4)) != EV_OK) {
            cleanup();
            return st;
        }
        if ((st = sync(x)) != EV_OK) {
            cleanup();
            return st;
        }
        if (capped_history) capped_history[i] = (int32_t)off[M + 1];
        rep->capped += off[M + 1];
        rep->nodes += total;
        rep->generations++;
    }
    // the last generation, packed in index order, as a population of its own
    std::vector<uint64_t> h_off((size_t)M + 1, 0);
    for (int32_t t = 0; t < M; t++) h_off[t + 1] = h_off[t] + h.len[t];
    if ((st = heap_repack(c, h, h_off.back(), true)) != EV_OK) {
        cleanup();
        return st;
    }
    Pop* Q = nullptr;
    uint8_t* bytes = h.arena;
    h.arena = nullptr;  // handed to the population (pop_build owns it, also on failure)
    if ((st = pop_build(c, x, bytes, h_off, &Q, nullptr)) != EV_OK) {
        cleanup();
        return st;
    }
    const hipError_t e = hipMemcpyAsync(Q->d_fit, d_fit, (size_t)M * 4, hipMemcpyDeviceToDevice, s);
    cleanup();
    if (e != hipSuccess) {
        pop_free(c, Q);
        return hip_fail(e, "hipMemcpyAsync");
    }
    Q->fit_valid = true;
    *out = pop_register(c, Q);
    return EV_OK;
}

}  // namespace ev
