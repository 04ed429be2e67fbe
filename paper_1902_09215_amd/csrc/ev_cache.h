// Stream-ordered cache of freed device blocks (host logic only, no HIP).
//
// A block handed back while kernels queued on some stream may still use it
// is kept here, tagged with that stream and with how many completed host
// waits the stream had seen when the block was freed.  It is handed out
// again only where that is safe without a device-side wait:
//   * on the same stream: the new user's work is queued behind the old one;
//   * on another stream: only once the freeing stream has completed a wait
//     that began after the free (every use queued before the free is then
//     finished).
// A stream that is going away drains first, so its blocks become free for
// every stream.  The caller serialises all calls (one mutex).
#pragma once
#include <algorithm>
#include <atomic>
#include <cstddef>
#include <cstdint>
#include <map>
#include <unordered_map>
#include <utility>
#include <vector>

namespace ev {

// One per execution stream: its identity and its count of completed waits
// (a wait covers everything queued on the stream before it began).
struct StreamClock {
    const void* stream = nullptr;
    std::atomic<uint64_t> waits{0};
};

class BlockCache {
public:
    // Keep block p of size class cls, last used on clk's stream (clk may be
    // null: no stream may still use the block).
    void put(void* p, size_t cls, const StreamClock* clk)
    {
        Tag t;
        t.cls = cls;
        t.tick = tick_++;
        t.clock = clk;
        t.stream = clk ? clk->stream : nullptr;
        t.waits_at_free = clk ? clk->waits.load() : 0;
        bins_[cls].push_back(p);
        tags_[p] = t;
        bytes_ += cls;
    }

    // A block of a class in [lo, hi] that work queued on `clk`'s stream may
    // use now; nullptr if there is none.  *got receives its class.
    void* take(size_t lo, size_t hi, const StreamClock* clk, size_t* got)
    {
        for (auto it = bins_.lower_bound(lo); it != bins_.end() && it->first <= hi; ++it) {
            auto& bin = it->second;
            // most recently freed first (warm in the caches, and the likeliest
            // to come from the same stream)
            for (size_t i = bin.size(); i-- > 0;) {
                void* p = bin[i];
                if (!usable(tags_[p], clk)) continue;
                bin.erase(bin.begin() + (ptrdiff_t)i);
                *got = it->first;
                bytes_ -= it->first;
                tags_.erase(p);
                return p;
            }
        }
        return nullptr;
    }

    // The clock's stream has drained and is going away: its blocks may be
    // used by every stream from now on.
    void forget(const StreamClock* clk)
    {
        for (auto& kv : tags_)
            if (kv.second.clock == clk) {
                kv.second.clock = nullptr;
                kv.second.stream = nullptr;
            }
    }

    // Remove and return the blocks idle the longest until `need` bytes are
    // released (or the cache is empty); the caller frees them.
    std::vector<std::pair<void*, size_t>> evict_oldest(uint64_t need)
    {
        std::vector<std::pair<uint64_t, void*>> order;
        order.reserve(tags_.size());
        for (auto& kv : tags_) order.push_back({kv.second.tick, kv.first});
        std::sort(order.begin(), order.end());
        std::vector<std::pair<void*, size_t>> out;
        uint64_t got = 0;
        for (auto& o : order) {
            if (got >= need) break;
            void* p = o.second;
            const size_t cls = tags_[p].cls;
            auto& bin = bins_[cls];
            bin.erase(std::find(bin.begin(), bin.end(), p));
            tags_.erase(p);
            bytes_ -= cls;
            got += cls;
            out.push_back({p, cls});
        }
        return out;
    }

    // Remove and return every block; the caller frees them.
    std::vector<std::pair<void*, size_t>> evict_all() { return evict_oldest(~0ull); }

    uint64_t bytes() const { return bytes_; }
    size_t blocks() const { return tags_.size(); }

private:
    struct Tag {
        size_t cls = 0;
        uint64_t tick = 0;
        const StreamClock* clock = nullptr;
        const void* stream = nullptr;
        uint64_t waits_at_free = 0;
    };

    static bool usable(const Tag& t, const StreamClock* clk)
    {
        if (!t.clock) return true;                               // no stream can still use it
        if (clk && clk->stream == t.stream) return true;         // ordered behind its last use
        return t.clock->waits.load() > t.waits_at_free;          // its stream was waited for since
    }

    std::map<size_t, std::vector<void*>> bins_;
    std::unordered_map<void*, Tag> tags_;
    uint64_t tick_ = 0;
    uint64_t bytes_ = 0;
};

}  // namespace ev
