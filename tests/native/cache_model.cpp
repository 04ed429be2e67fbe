// Host model of device streams around the block cache of libev
// (paper_1902_09215_amd/csrc/ev_cache.h): no block may be handed to a
// stream while another stream still has queued work that uses it.
//
// A stream is a FIFO of queued uses of blocks.  The host allocates a block
// for a stream (and queues a use of it there), frees blocks, lets the
// device run queued work in an adversarial order, and waits for streams.
// Built with g++ by tests/test_cache_model.py; exits non-zero on a
// violation and prints the number of checked hand-outs.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "ev_cache.h"

using ev::BlockCache;
using ev::StreamClock;

struct SimStream {
    StreamClock clock;
    std::deque<void*> queued;  // blocks used by queued, not yet finished work
    std::set<void*> live;      // blocks allocated by this stream's owner
};

static int fails = 0;
static long checks = 0;

#define CHECK(c, ...)                      \
    do {                                   \
        if (!(c)) {                        \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");    \
            fails++;                       \
        }                                  \
    } while (0)

static void* fresh_block()
{
    static uintptr_t next = 0x100000;
    next += 0x1000;
    return (void*)next;
}

// A block handed to stream t must have no queued use on any other stream.
static void check_handout(std::vector<SimStream>& S, size_t t, void* p)
{
    checks++;
    for (size_t s = 0; s < S.size(); s++) {
        if (s == t) continue;
        for (void* q : S[s].queued) CHECK(q != p, "block %p handed to stream %zu while stream %zu still uses it", p, t, s);
    }
}

static void scripted()
{
    // plan building on stream A frees its scratch while the kernel that
    // reads it is still queued; another worker's stream B allocates
    std::vector<SimStream> S(2);
    S[0].clock.stream = (void*)0xA;
    S[1].clock.stream = (void*)0xB;
    BlockCache c;
    void* scratch = fresh_block();
    S[0].queued.push_back(scratch);  // k_seg_place reads it
    c.put(scratch, 4096, &S[0].clock);
    size_t got = 0;
    CHECK(c.take(4096, 4096, &S[1].clock, &got) == nullptr, "other stream got a block still in use");
    // the same stream may reuse it at once: its next kernel runs after
    void* again = c.take(4096, 4096, &S[0].clock, &got);
    CHECK(again == scratch, "same stream did not reuse its block");
    c.put(again, 4096, &S[0].clock);
    // once stream A has been waited for, B may take it
    S[0].queued.clear();
    S[0].clock.waits++;
    CHECK(c.take(4096, 4096, &S[1].clock, &got) == scratch, "block not reusable after the wait");
    // a wait that happened before the free does not count
    c.put(scratch, 4096, &S[0].clock);
    S[0].queued.push_back(scratch);
    CHECK(c.take(4096, 4096, &S[1].clock, &got) == nullptr, "an earlier wait released a later free");
    // a stream that drained and went away releases its blocks
    S[0].queued.clear();
    c.forget(&S[0].clock);
    CHECK(c.take(4096, 4096, &S[1].clock, &got) == scratch, "forgotten stream's block not released");
    // blocks freed with no stream are free for all
    c.put(scratch, 256, nullptr);
    CHECK(c.take(256, 256, &S[1].clock, &got) == scratch, "stream-less block not handed out");
    // size classes: a request takes a block of a class in [lo, hi] only
    void* big = fresh_block();
    c.put(big, 8192, nullptr);
    CHECK(c.take(4096, 4096, &S[1].clock, &got) == nullptr, "class above the range handed out");
    CHECK(c.take(4096, 8192, &S[1].clock, &got) == big && got == 8192, "class within the range not handed out");
    // eviction: oldest first, until the bytes are released
    void* a = fresh_block();
    void* b = fresh_block();
    c.put(a, 256, nullptr);
    c.put(b, 512, nullptr);
    auto ev = c.evict_oldest(100);
    CHECK(ev.size() == 1 && ev[0].first == a, "eviction did not take the oldest block first");
    CHECK(c.bytes() == 512 && c.blocks() == 1, "byte count after eviction");
}

static void random_walk(unsigned seed)
{
    std::mt19937_64 rng(seed);
    const size_t n_streams = 1 + rng() % 4;
    std::vector<SimStream> S(n_streams);
    for (size_t i = 0; i < n_streams; i++) S[i].clock.stream = (void*)(0x1000 + i);
    BlockCache c;
    std::map<void*, size_t> cls_of;
    const size_t classes[] = {256, 512, 1024};
    for (int step = 0; step < 4000; step++) {
        const size_t t = rng() % n_streams;
        SimStream& st = S[t];
        switch (rng() % 6) {
        case 0:
        case 1: {  // allocate on t and queue a use of the block there
            const size_t cls = classes[rng() % 3];
            size_t got = 0;
            void* p = c.take(cls, cls, &st.clock, &got);
            if (p) check_handout(S, t, p);
            else p = fresh_block();
            cls_of[p] = p && got ? got : cls;
            st.live.insert(p);
            st.queued.push_back(p);
            break;
        }
        case 2: {  // queue another use of a live block, then maybe free it
            if (st.live.empty()) break;
            auto it = st.live.begin();
            std::advance(it, rng() % st.live.size());
            void* p = *it;
            if (rng() % 2) st.queued.push_back(p);
            st.live.erase(it);
            c.put(p, cls_of[p], &st.clock);
            break;
        }
        case 3: {  // the device finishes some queued work of t
            size_t k = rng() % (st.queued.size() + 1);
            while (k-- > 0) st.queued.pop_front();
            break;
        }
        case 4:  // the host waits for t: everything queued has finished
            st.queued.clear();
            st.clock.waits++;
            break;
        case 5:  // nothing
            break;
        }
    }
}

int main()
{
    scripted();
    for (unsigned seed = 1; seed <= 300; seed++) random_walk(seed);
    std::printf("%ld\n", checks);
    return fails ? 1 : 0;
}
