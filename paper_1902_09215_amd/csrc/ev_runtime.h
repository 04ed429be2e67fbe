// Host-side state of libev.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ev.h"
#include "ev_cache.h"
#include "ev_internal.h"
#include "ev_launch.h"

namespace ev {

struct CaseTable {
    float* d_x = nullptr;
    float* d_y = nullptr;
    int32_t N = 0;
};

// One level of a population's split plan.
struct Level {
    uint8_t* seq = nullptr;  // level 0: the population's bytes; later: skeleton
    bool owned = false;
    EvalChunk* d_chunks = nullptr;  // work items of the general kernel (k_eval)
    uint32_t n_chunks = 0;
    uint32_t* codes = nullptr;      // threaded codes of the register-stack items
    RunChunk* d_run = nullptr;      // work items of the register-stack kernel (k_run)
    uint32_t n_run = 0;
    uint32_t* d_item_tree = nullptr;  // per register-stack work item: its tree
    uint64_t tokens = 0;            // tokens over all work items of the level
    uint32_t trees = 0;             // trees with work at the level
    uint32_t slab_entries = 0;      // spill-slab rows per wave of k_run (0: no spills)
    uint32_t n_out = 0;  // result slots written by this level
    uint32_t max_m = 0;  // deepest physical operand stack of a k_eval item
    uint32_t n_seg = 0;     // structure segments
    uint64_t n_codes = 0;   // codes of the register-stack items (with each item's padding)
    uint64_t n_frag = 0;    // tokens of the next level's skeleton
};

struct Plan {
    std::vector<Level> levels;
    std::vector<int32_t> fin_level;  // per tree: level holding its value
    std::vector<uint32_t> fin_slot;  // and the slot
    uint32_t* d_fin = nullptr;       // both on the device: level, slot per tree
    // The validator's words, two per level (flags, first failing segment).
    // err_pending: the last level's were not yet read by the host; its k_run
    // launches check them on the device, and the host reads them with the
    // first evaluation (h_err).
    uint32_t* d_err = nullptr;
    int err_level = 0;
    bool err_pending = false;
    uint32_t h_err[2] = {0, 0};
    // per level and tree (levels x trees): the tree's work items, for the
    // chained launch (null when it does not apply); on the host, with the
    // place of the tree's first item at the level (its items are together;
    // ~0u where the places were made on the device and are not known here)
    uint32_t* d_need = nullptr;
    std::vector<uint32_t> h_need, h_pos;
    uint32_t chunk = 0;
    int D = 64;
    uint64_t chunks_total = 0, slots_total = 0, max_stack = 0, bytes = 0;
    // Level 0's chunks, kept when the level was planned for the
    // register-stack kernel and has a next level, so that children can take
    // over the ones crossover leaves intact: per chunk (token order) its
    // record, totals, first code and fragment end in levels[1].seq; per tree
    // its range of chunks.
    uint32_t l0_n = 0;
    ChunkIn* l0_ch = nullptr;
    ChunkStat* l0_stat = nullptr;
    uint64_t* l0_code = nullptr;
    uint64_t* l0_frag = nullptr;
    L0Tree* l0_tree = nullptr;
};

struct Pop;

// Children planned from their mum's level 0 (one ReuseRun per child).
struct ReuseSpec {
    const Pop* mum;
    const std::vector<ReuseRun>* runs;
};

// Intermediate results of one population for one case table.
struct ResCache {
    int32_t N = 0;
    std::vector<float*> res;     // per level: n_out * N floats (EV_RING padding rows before)
    float* d_per_case = nullptr;
    RunLevel* d_chain = nullptr;  // the chained launch's queue: runs of the chained levels' items
    int chain_first = -1;         // the first level d_chain holds
    uint32_t chain_records = 0;   // and its runs
};

struct Pop {
    uint8_t* d_bytes = nullptr;
    uint64_t* d_off = nullptr;
    std::vector<uint64_t> h_off;
    // when not empty, tree t's bytes start at d_bytes + h_start[t] (a heap of
    // trees, used only inside the memory-lean loop); h_off then holds the
    // prefix sums of the lengths
    std::vector<uint64_t> h_start;
    int32_t M = 0;
    uint64_t total = 0;
    Plan plan;
    float* d_fit = nullptr;
    int32_t* d_hits = nullptr;  // the last evaluation's hits, when asked for
    bool fit_valid = false;
    bool hits_valid = false;    // d_hits holds the last evaluation's hits
    std::map<int32_t, ResCache> res;
    // serving jobs using the population off the caller's thread (guarded by
    // the context's pop_mu); ev_free_pop of a population still in use only
    // unregisters it, and the last job to release it frees it
    int32_t refs = 0;
    bool dead = false;
};

// Host-side working vectors of plan_build, kept across calls so that their
// (large) buffers are reused instead of freshly mapped and faulted in.
struct PlanScratch {
    std::vector<uint64_t> rs, rl, prev_len, ref_base;
    std::vector<char> active;
    std::vector<uint32_t> fin;
    std::vector<TreeLvl> tl;
    std::vector<TreeSum> tsum;
    std::vector<TreeBase> tb;
};

// Per-thread execution resources: a stream (possibly shared) and the scratch
// its launches use.
struct Exec {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // the stream's identity and completed waits, for the block cache: a
    // block this Exec frees is reused at once on its own stream, and on
    // another only after a later wait here
    StreamClock clock;
    uint32_t* d_counters = nullptr;
    size_t n_counters = 0;
    float* d_gstack = nullptr;
    size_t gstack_bytes = 0;
    // the structure pass's recordings (code kinds, fragment tokens, segment
    // records), kept from plan to plan on this stream and grown as needed
    void* d_rec_buf[3] = {nullptr, nullptr, nullptr};
    size_t rec_cap[3] = {0, 0, 0};
    // the skeleton levels may go in one chained launch (k_run_chain) on
    // this stream; off on the serving workers' streams
    bool chain_ok = true;
    hipEvent_t done = nullptr;  // completion marker of sync()
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evi0 = nullptr, evi1 = nullptr;
    std::vector<hipEvent_t> evl;  // timed evaluations: one event after each plan level
    uint32_t n_levels_timed = 0;
    // Pinned host staging of the stream's transfers: copies are plain DMA
    // from and to it; device-to-host data is handed out at the next sync().
    uint8_t* pin = nullptr;
    size_t pin_cap = 0, pin_off = 0;
    struct Out {
        void* dst;
        const void* src;
        size_t n;
    };
    std::vector<Out> pin_out;
    PlanScratch plan;
};

struct Job;
struct Serve;
struct GenGraph;

}  // namespace ev

struct ev_ctx {
    int device = 0;
    int num_cus = 0;
    int grid_eval[2] = {0, 0};
    int grid_run = 0;
    int run_bpc = 0;  // interpreter waves per compute unit that fit (occupancy)
    bool use_run = true;  // register-stack kernel for the items that fit it
    bool run_ok = true;   // the register-stack kernel can run here (probed at creation)
    bool test_fail_check = false;  // EV_TUNE_TEST_FAIL_CHECK
    bool use_record = true;        // the count pass records codes for emission (EV_TUNE_NO_RECORD clears it)
    bool use_reuse = true;         // children take over their mums' level-0 chunks (EV_TUNE_NO_REUSE clears it)
    bool use_chain = true;         // the skeleton levels in one launch (EV_TUNE_NO_CHAIN clears it)
    int grid_chain = 0;
    uint32_t* d_flag = nullptr;  // the probe's flag word
    // ephemeral random constants (Sec. 2.1): token 6 + i is d_const[i]
    int32_t n_consts = 0;
    float* d_const = nullptr;
    uint32_t chunk = 6144;     // tokens per work item at level 0
    uint32_t chunk_hi = 0;     // at the skeleton levels (0: twice chunk)
    int lds_depth = 64;

    ev::Exec main;
    hipStream_t& stream = main.stream;  // the context's stream for the synchronous calls

    std::mutex mem_mu;
    ev_allocator ext = {};     // the caller's allocator (ext.alloc == nullptr: hipMalloc)
    uint64_t budget = 0, in_use = 0;
    uint64_t hold_limit = ~0ull;  // live + cached bytes, below the device's free memory
    std::unordered_map<void*, size_t> sizes;   // live blocks and their size class
    ev::BlockCache cache;                        // freed blocks, stream-ordered

    std::mutex pop_mu;
    std::deque<ev::CaseTable> tables;  // stable: serving workers hold references while tables are added
    std::map<ev_pop, ev::Pop*> pops;
    ev_pop next_pop = 1;

    ev::Serve* serve = nullptr;
    std::mutex serve_init_mu;

    ev::GenGraph* evolve = nullptr;  // ev_evolve's captured generations, kept for the next call
};

namespace ev {

extern thread_local std::string g_err;
ev_status fail(ev_status code, const char* fmt, ...);
ev_status hip_fail(hipError_t e, const char* what);
// return the failure of a HIP call
#define HIPCHK(x)                                      \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #x); \
    } while (0)

// Device blocks.  Both act for the calling thread's Exec (set with
// ExecScope; the context's own Exec when none is set): a block freed while
// that Exec's queued work may still use it is reused at once on the same
// stream, and on other streams only after that Exec's next wait.
ev_status dev_alloc(ev_ctx* c, size_t bytes, void** out);
void dev_free(ev_ctx* c, void* p);
void dev_cache_release(ev_ctx* c);

// The Exec on whose stream the calling thread queues its work.
struct ExecScope {
    explicit ExecScope(Exec* x);
    ~ExecScope();
    Exec* prev;
};
Exec* current_exec(ev_ctx* c);

// A case table by index (copied under the lock); false if there is none.
bool table_get(ev_ctx* c, int32_t table, CaseTable* out);

ev_status exec_init(Exec& x, hipStream_t given);
ev_status stage(Exec& x, size_t n, void** out);
ev_status put(Exec& x, void* dst, const void* src, size_t n);
ev_status put2(Exec& x, void* dst, const void* a, size_t na, const void* b, size_t nb);
ev_status get(Exec& x, void* dst, const void* src, size_t n);
ev_status sync(Exec& x);
void exec_free(ev_ctx* c, Exec& x);

void pop_free(ev_ctx* c, Pop* P);
// d_off: the offsets already on the device (adopted), or nullptr to upload h_off
// defer_check: leave the last plan level's validation verdict to the device
// and to the first evaluation (Plan::err_pending)
// reuse: the children's level 0 taken over from their mums' where it can be
ev_status pop_build(ev_ctx* c, Exec& x, uint8_t* d_bytes, const std::vector<uint64_t>& h_off, Pop** out,
                    int32_t* bad, uint64_t* d_off = nullptr, bool defer_check = false,
                    const ReuseSpec* reuse = nullptr);
// after a sync that followed eval_enqueue(P): the deferred verdict, if any
ev_status plan_verdict(Pop* P);
ev_pop pop_register(ev_ctx* c, Pop* P);
Pop* pop_get(ev_ctx* c, ev_pop id);
// pin / unpin a registered population for work on another thread
Pop* pop_acquire(ev_ctx* c, ev_pop id);
void pop_release(ev_ctx* c, Pop* P);

// verdict_at_sync: a plan's deferred validation verdict (Plan::err_pending)
// is fetched with the caller's next sync(x), after which the caller calls
// plan_verdict(P); otherwise it is checked here, with a sync of its own
ev_status eval_enqueue(ev_ctx* c, Exec& x, Pop* P, int32_t table, float* d_fit, float* d_per_case, bool timed,
                       int32_t* d_hits, bool verdict_at_sync = false);
// Look up this device's copy of the static scratch array (device current).
ev_status static_scratch_init(int device);
// eval_enqueue on the context's stream with no allocation: counters,
// result slots and spill slabs carved from [scratch, scratch + bytes)
ev_status eval_in_scratch(ev_ctx* c, Pop* P, int32_t table, float* d_fit, float* d_per_case, int32_t* d_hits,
                          uint8_t* scratch, size_t bytes);
ev_status crossover_build(ev_ctx* c, Exec& x, Pop* mums, Pop* dads, const int32_t* mum, const int32_t* dad,
                          const uint64_t* p, const uint64_t* q, int32_t n, uint64_t cap, Pop** out,
                          int32_t* n_capped);
ev_status crossover_build_dev(ev_ctx* c, Exec& x, Pop* mums, Pop* dads, const int32_t* d_mum, const int32_t* d_dad,
                              const uint64_t* d_p, const uint64_t* d_q, int32_t n, uint64_t cap, Pop** out,
                              int32_t* n_capped, bool defer_check = false);

void serve_stop(ev_ctx* c);

// Release a context's replayed-generation graphs and their buffers.
void evolve_release(ev_ctx* c);
// The memory-lean loop of ev_evolve (EV_EVOLVE_LEAN): arguments as there.
ev_status evolve_lean(ev_ctx* c, Pop* P, const float* fitness, int32_t table, uint64_t seed, uint64_t gen0,
                      int32_t n_gen, int32_t tournament, uint64_t size_cap, ev_pop* out, float* fit_history,
                      int32_t* capped_history, ev_evolve_report* rep);
// build a population's split plan (bad_tree: the first malformed tree)
ev_status plan_build(ev_ctx* c, Exec& x, Pop* P, int32_t* bad_tree, bool defer_check = false,
                     const ReuseSpec* reuse = nullptr);

}  // namespace ev
