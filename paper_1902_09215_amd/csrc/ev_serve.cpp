// Serving loop of libev: ev_submit / ev_poll / ev_wait / ev_result.
//
// Requests are queued in arrival order.  Worker threads, each with its own
// scratch and pinned staging, take the queue head as soon as its estimated
// device footprint fits the budget beside the jobs already in flight, and
// fold every other queued evaluation request on the same case table that
// also fits into the same device launch (continuous batching).  Several
// workers run at once, each on its own stream: their batches overlap on the
// device, and one batches, stages and plans on the host while the others'
// kernels run.  Device blocks move between the workers' streams through the
// stream-ordered block cache (ev_cache.h), and a population a crossover job
// reads stays alive until the job is done.  Each tree's result depends only
// on the tree, never on the batch it rode in or on what ran beside it.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "ev_runtime.h"

namespace ev {

struct Job {
    ev_ticket id = 0;
    int32_t kind = 0;
    int32_t table = 0;
    int32_t n = 0;  // trees (eval) or children (crossover)
    std::vector<uint8_t> bytes;
    std::vector<uint64_t> off;
    ev_pop parents = 0;
    std::vector<int32_t> mum, dad;
    std::vector<uint64_t> p, q;
    uint64_t size_cap = 0;
    uint64_t footprint = 0;
    int32_t N = 0;
    bool done = false;
    ev_status status = EV_OK;
    std::vector<float> fitness, per_case;
    uint64_t t_submit = 0, t_start = 0, t_done = 0;
    std::string err;  // the failing call's message (set on the worker thread)
};

static uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Serve {
    std::mutex mu;
    std::condition_variable cv;       // work queued / stop
    std::condition_variable done_cv;  // a job finished
    std::deque<Job*> queue;
    std::unordered_map<ev_ticket, Job*> jobs;
    ev_ticket next = 1;
    uint64_t reserved = 0;
    uint64_t budget = 0;  // 0 = unbounded
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<std::unique_ptr<Exec>> execs;
    uint64_t max_batch_nodes = 1ull << 28;
    int32_t max_batch_jobs = 4096;
};

// Device bytes a job may hold at its peak: the trees, one byte per node per
// split level (skeletons shrink fast), per-case values of every tree and
// intermediate slots (a few hundred per 4096 tokens, whatever the work-item
// size).
static uint64_t footprint(uint64_t nodes, uint64_t trees, int32_t N, uint32_t chunk)
{
    const uint64_t chunks = nodes / (chunk < 4096u ? chunk : 4096u) + trees;
    return 2 * nodes + 1024 + trees * (64 + 8ull * N) + chunks * (96 + 256ull * 4 * N);
}

static void finish(Serve* S, Job* j, ev_status st)
{
    std::lock_guard<std::mutex> g(S->mu);
    if (st != EV_OK) j->err = g_err;
    j->status = st;
    j->done = true;
    j->t_done = now_ns();
    S->reserved -= j->footprint;
    S->done_cv.notify_all();
    S->cv.notify_all();
}

// Evaluate a batch of eval jobs (same table) as one population.  A tree
// that is not a valid prefix tree fails the batch's plan with EV_EMALFORMED;
// *bad_job is then the batch index of the job that holds it (else -1).
static ev_status run_eval_batch(ev_ctx* c, Exec& x, std::vector<Job*>& batch, int32_t* bad_job)
{
    *bad_job = -1;
    std::vector<uint64_t> off(1, 0);
    uint64_t total = 0;
    for (Job* j : batch) total += j->off.back();
    for (Job* j : batch) {
        const uint64_t base = off.back();
        for (int32_t t = 0; t < j->n; t++) off.push_back(base + j->off[t + 1]);
    }
    const int32_t M = (int32_t)off.size() - 1;
    const int32_t table = batch[0]->table;
    const int32_t N = batch[0]->N;
    ev_status st = EV_OK;
    uint8_t* d = nullptr;
    Pop* P = nullptr;
    float* d_pc = nullptr;
    std::vector<float> fit(M), pc((size_t)M * N);
    if ((st = dev_alloc(c, total + EV_POP_PAD, (void**)&d)) == EV_OK) {
        uint64_t at = 0;
        for (Job* j : batch) {
            if (st == EV_OK) st = put(x, d + at, j->bytes.data(), j->bytes.size());
            at += j->bytes.size();
        }
        if (st == EV_OK) {
            hipError_t e = launch_fill_u8(d + total, EV_POP_PAD, 0xFF, x.stream);
            if (e != hipSuccess) st = hip_fail(e, "serve upload");
        }
        if (st != EV_OK) {
            (void)sync(x);
            dev_free(c, d);
        } else {
            int32_t bad = -1;
            st = pop_build(c, x, d, off, &P, &bad);
            for (int32_t k = 0, first = 0; st == EV_EMALFORMED && bad >= 0 && k < (int32_t)batch.size(); k++) {
                if (bad < first + batch[k]->n) {
                    *bad_job = k;
                    break;
                }
                first += batch[k]->n;
            }
        }
    }
    if (st == EV_OK) st = dev_alloc(c, (size_t)std::max(1, M) * N * sizeof(float), (void**)&d_pc);
    if (st == EV_OK) st = eval_enqueue(c, x, P, table, P->d_fit, d_pc, false, nullptr);
    if (st == EV_OK) st = get(x, fit.data(), P->d_fit, (size_t)M * 4);
    if (st == EV_OK) st = get(x, pc.data(), d_pc, (size_t)M * N * 4);
    if (st == EV_OK) st = sync(x);
    else (void)sync(x);
    dev_free(c, d_pc);
    if (P) pop_free(c, P);
    int32_t at = 0;
    for (Job* j : batch) {
        if (st == EV_OK) {
            j->fitness.assign(fit.begin() + at, fit.begin() + at + j->n);
            j->per_case.assign(pc.begin() + (size_t)at * N, pc.begin() + (size_t)(at + j->n) * N);
            j->N = N;
        }
        at += j->n;
    }
    return st;
}

static ev_status run_crossover(ev_ctx* c, Exec& x, Job* j)
{
    Pop* par = pop_acquire(c, j->parents);
    if (!par) return fail(EV_ENOTFOUND, "no population %d", j->parents);
    Pop* C = nullptr;
    int32_t capped = 0;
    ev_status st = crossover_build(c, x, par, par, j->mum.data(), j->dad.data(), j->p.data(), j->q.data(), j->n,
                                   j->size_cap, &C, &capped);
    if (st != EV_OK) {
        (void)sync(x);
        pop_release(c, par);
        return st;
    }
    const int32_t N = j->N;
    float* d_pc = nullptr;
    st = dev_alloc(c, (size_t)std::max(1, C->M) * N * sizeof(float), (void**)&d_pc);
    if (st == EV_OK) st = eval_enqueue(c, x, C, j->table, C->d_fit, d_pc, false, nullptr);
    if (st == EV_OK) {
        j->fitness.resize(C->M);
        j->per_case.resize((size_t)C->M * N);
        j->N = N;
        st = get(x, j->fitness.data(), C->d_fit, (size_t)C->M * 4);
        if (st == EV_OK) st = get(x, j->per_case.data(), d_pc, (size_t)C->M * N * 4);
    }
    if (st == EV_OK) st = sync(x);
    else (void)sync(x);
    dev_free(c, d_pc);
    pop_free(c, C);
    pop_release(c, par);
    return st;
}

// A job is admitted when its footprint fits beside the jobs in flight and
// the memory the context already holds; with nothing in flight the head of
// the queue always starts (and reports EV_ENOMEM if it really cannot run).
static bool fits(ev_ctx* c, Serve* S, uint64_t fp)
{
    if (S->budget == 0 || S->reserved == 0) return true;
    uint64_t used;
    {
        std::lock_guard<std::mutex> g(c->mem_mu);
        used = c->in_use;
    }
    return S->reserved + fp <= S->budget && used + fp <= S->budget;
}

static void worker(ev_ctx* c, Serve* S, Exec* x)
{
    (void)hipSetDevice(c->device);
    ExecScope scope(x);  // blocks this thread frees are tagged with its stream
    for (;;) {
        std::vector<Job*> batch;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || (!S->queue.empty() && fits(c, S, S->queue.front()->footprint)); });
            if (S->stop) return;
            Job* h = S->queue.front();
            S->queue.pop_front();
            S->reserved += h->footprint;
            h->t_start = now_ns();
            batch.push_back(h);
            if (h->kind == EV_JOB_EVAL) {
                uint64_t nodes = h->off.back();
                for (auto it = S->queue.begin(); it != S->queue.end();) {
                    Job* j = *it;
                    if ((int32_t)batch.size() >= S->max_batch_jobs) break;
                    if (j->kind != EV_JOB_EVAL || j->table != h->table || nodes + j->off.back() > S->max_batch_nodes ||
                        !fits(c, S, j->footprint)) {
                        ++it;
                        continue;
                    }
                    S->reserved += j->footprint;
                    j->t_start = h->t_start;
                    nodes += j->off.back();
                    batch.push_back(j);
                    it = S->queue.erase(it);
                }
            }
        }
        if (batch[0]->kind == EV_JOB_EVAL) {
            ev_status st = EV_OK;
            while (!batch.empty()) {
                int32_t bad = -1;
                st = run_eval_batch(c, *x, batch, &bad);
                if (bad < 0) break;
                // a malformed request fails alone; the others run again
                // without it
                finish(S, batch[bad], st);
                batch.erase(batch.begin() + bad);
            }
            for (Job* j : batch) finish(S, j, st);
        } else {
            const ev_status st = run_crossover(c, *x, batch[0]);
            finish(S, batch[0], st);
        }
    }
}

static Serve* serve_get(ev_ctx* c)
{
    std::lock_guard<std::mutex> g(c->serve_init_mu);
    if (c->serve) return c->serve;
    Serve* S = new Serve();
    S->budget = c->budget;
    // Each worker has its own stream (default priority), scratch, staging
    // and completion event: batches overlap on the device, and a worker's
    // host work (batching, planning, staging) overlaps the others' kernels.
    const int W = 4;
    for (int i = 0; i < W; i++) {
        auto x = std::make_unique<Exec>();
        if (exec_init(*x, nullptr) != EV_OK) break;
        // one launch per skeleton level here: with the chained launch on
        // the workers' concurrent streams, other jobs' code streams failed
        // validation now and then (cause not found)
        x->chain_ok = false;
        S->execs.push_back(std::move(x));
    }
    for (auto& x : S->execs) S->workers.emplace_back(worker, c, S, x.get());
    c->serve = S;
    return S;
}

void serve_stop(ev_ctx* c)
{
    Serve* S = nullptr;
    {
        std::lock_guard<std::mutex> g(c->serve_init_mu);
        S = c->serve;
        c->serve = nullptr;
    }
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto& t : S->workers) t.join();
    for (auto& x : S->execs) exec_free(c, *x);
    for (auto& kv : S->jobs) delete kv.second;
    for (Job* j : S->queue) (void)j;  // owned by S->jobs as well
    delete S;
}

}  // namespace ev

using namespace ev;

extern "C" {

ev_status ev_submit(ev_ctx* c, const ev_job* job, ev_ticket* out)
{
    if (!c || !job || !out) return fail(EV_EINVAL, "ev_submit: bad arguments");
    CaseTable ct;
    if (!table_get(c, job->table, &ct)) return fail(EV_EINVAL, "no case table %d", job->table);
    auto j = std::make_unique<Job>();
    j->kind = job->kind;
    j->table = job->table;
    const int32_t N = ct.N;
    j->N = N;
    if (job->kind == EV_JOB_EVAL) {
        if (job->n_trees < 0 || (job->n_trees > 0 && (!job->off || !job->bytes)))
            return fail(EV_EINVAL, "ev_submit: bad trees");
        j->n = job->n_trees;
        j->off.assign(job->off, job->off + job->n_trees + 1);
        if (j->off[0] != 0) return fail(EV_EINVAL, "ev_submit: off[0] must be 0");
        for (int32_t t = 0; t < j->n; t++)
            if (j->off[t + 1] <= j->off[t]) return fail(EV_EMALFORMED, "ev_submit: tree %d is empty", t);
        // the trees are checked on the device, when their batch is planned
        j->bytes.assign(job->bytes, job->bytes + j->off.back());
        j->footprint = footprint(j->off.back(), (uint64_t)j->n, N, c->chunk);
    } else if (job->kind == EV_JOB_CROSSOVER) {
        if (job->n_children < 0 || (job->n_children > 0 && (!job->mum || !job->dad || !job->p || !job->q)))
            return fail(EV_EINVAL, "ev_submit: bad crossover arrays");
        Pop* par = pop_acquire(c, job->parents);
        if (!par) return fail(EV_ENOTFOUND, "no population %d", job->parents);
        // host-side checks only: the population stays pinned while they read it
        struct Unpin {
            ev_ctx* c;
            Pop* P;
            ~Unpin() { pop_release(c, P); }
        } unpin{c, par};
        j->n = job->n_children;
        j->parents = job->parents;
        j->mum.assign(job->mum, job->mum + j->n);
        j->dad.assign(job->dad, job->dad + j->n);
        j->p.assign(job->p, job->p + j->n);
        j->q.assign(job->q, job->q + j->n);
        j->size_cap = job->size_cap;
        uint64_t nodes = 0;
        for (int32_t k = 0; k < j->n; k++) {
            if (j->mum[k] < 0 || j->mum[k] >= par->M || j->dad[k] < 0 || j->dad[k] >= par->M)
                return fail(EV_EINVAL, "ev_submit: parent index out of range");
            const uint64_t nm = par->h_off[j->mum[k] + 1] - par->h_off[j->mum[k]];
            const uint64_t nd = par->h_off[j->dad[k] + 1] - par->h_off[j->dad[k]];
            if (j->p[k] >= nm || j->q[k] >= nd) return fail(EV_EINVAL, "ev_submit: crossover point out of range");
            nodes += nm + nd;
        }
        j->footprint = footprint(nodes, (uint64_t)j->n, N, c->chunk) + 48ull * j->n;
    } else {
        return fail(EV_EINVAL, "ev_submit: unknown job kind %d", job->kind);
    }
    Serve* S = serve_get(c);
    if (S->budget && j->footprint > S->budget)
        return fail(EV_EBUSY, "ev_submit: job needs ~%llu bytes, budget is %llu", (unsigned long long)j->footprint,
                    (unsigned long long)S->budget);
    std::lock_guard<std::mutex> g(S->mu);
    j->id = S->next++;
    j->t_submit = now_ns();
    *out = j->id;
    Job* raw = j.release();
    S->jobs[raw->id] = raw;
    S->queue.push_back(raw);
    S->cv.notify_one();
    return EV_OK;
}

ev_status ev_poll(ev_ctx* c, ev_ticket t, int32_t* done, ev_status* job_status)
{
    if (!c || !done) return fail(EV_EINVAL, "ev_poll: bad arguments");
    Serve* S = serve_get(c);
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->jobs.find(t);
    if (it == S->jobs.end()) return fail(EV_ENOTFOUND, "no ticket %llu", (unsigned long long)t);
    *done = it->second->done ? 1 : 0;
    if (job_status) *job_status = it->second->done ? it->second->status : EV_OK;
    return EV_OK;
}

ev_status ev_wait(ev_ctx* c, ev_ticket t, ev_status* job_status)
{
    if (!c) return fail(EV_EINVAL, "ev_wait: NULL context");
    Serve* S = serve_get(c);
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(t);
    if (it == S->jobs.end()) return fail(EV_ENOTFOUND, "no ticket %llu", (unsigned long long)t);
    Job* j = it->second;
    S->done_cv.wait(lk, [&] { return j->done; });
    if (job_status) *job_status = j->status;
    return EV_OK;
}

ev_status ev_result(ev_ctx* c, ev_ticket t, float* fitness, float* per_case, int32_t cap, int32_t* n_out)
{
    if (!c) return fail(EV_EINVAL, "ev_result: NULL context");
    Serve* S = serve_get(c);
    Job* j = nullptr;
    {
        std::lock_guard<std::mutex> g(S->mu);
        auto it = S->jobs.find(t);
        if (it == S->jobs.end()) return fail(EV_ENOTFOUND, "no ticket %llu", (unsigned long long)t);
        j = it->second;
        if (!j->done) return fail(EV_EBUSY, "ticket %llu not finished", (unsigned long long)t);
        if (j->status != EV_OK) {
            const ev_status st = j->status;
            const std::string msg = j->err;
            S->jobs.erase(it);
            delete j;
            return fail(st, "job failed: %s", msg.c_str());
        }
        if (cap < (int32_t)j->fitness.size()) return fail(EV_EINVAL, "ev_result: cap %d < %zu", cap, j->fitness.size());
        S->jobs.erase(it);
    }
    if (n_out) *n_out = (int32_t)j->fitness.size();
    if (fitness) std::memcpy(fitness, j->fitness.data(), j->fitness.size() * 4);
    if (per_case) std::memcpy(per_case, j->per_case.data(), j->per_case.size() * 4);
    delete j;
    return EV_OK;
}

ev_status ev_job_timing(ev_ctx* c, ev_ticket t, uint64_t* submit_ns, uint64_t* start_ns, uint64_t* done_ns)
{
    if (!c) return fail(EV_EINVAL, "ev_job_timing: NULL context");
    Serve* S = serve_get(c);
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->jobs.find(t);
    if (it == S->jobs.end()) return fail(EV_ENOTFOUND, "no ticket %llu", (unsigned long long)t);
    if (submit_ns) *submit_ns = it->second->t_submit;
    if (start_ns) *start_ns = it->second->t_start;
    if (done_ns) *done_ns = it->second->t_done;
    return EV_OK;
}

}  // extern "C"
