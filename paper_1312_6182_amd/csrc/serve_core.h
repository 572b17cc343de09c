// Host-side bookkeeping of the GP-SPCA solve server: the device-arena
// allocator, the residency of registered matrices and the admission policy.
//
// This header has no HIP dependency: the server (serve.cpp) drives it with
// real device memory and streams, and a host-only build drives it with a
// simulated device in the CPU tests.
//
// Policy:
//  - every request needs its matrix resident (uploaded once, kept for later
//    requests on the same matrix, together with its cached column norms) and a
//    private workspace for the duration of its solve;
//  - a free slot admits the oldest waiting request whose memory can be found:
//    first from free arena space, then by evicting resident matrices that no
//    admitted request uses, least recently used first; a request that cannot
//    fit even in an empty arena is rejected at submission;
//  - to keep a large request from starving, once the oldest waiting request
//    has been passed over `max_bypass` times, nothing behind it is admitted
//    until it is.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

namespace gpspca {
namespace serve {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
  public:
    explicit Arena(size_t size = 0) { reset(size); }

    void reset(size_t size) {
        size_ = size / kAlign * kAlign;
        free_.clear();
        used_.clear();
        if (size_) free_[0] = size_;
    }

    // Offset of a block of `bytes` (aligned), or SIZE_MAX.
    size_t alloc(size_t bytes) {
        const size_t need = align_up(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > need) free_[off + need] = len - need;
                used_[off] = need;
                return off;
            }
        }
        return SIZE_MAX;
    }

    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t start = off, len = u->second;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
        return true;
    }

    size_t size() const { return size_; }
    size_t free_bytes() const {
        size_t s = 0;
        for (auto& f : free_) s += f.second;
        return s;
    }
    size_t largest_free() const {
        size_t s = 0;
        for (auto& f : free_) s = std::max(s, f.second);
        return s;
    }
    size_t used_blocks() const { return used_.size(); }
    // Blocks in use as (offset, length), for invariant checks.
    std::vector<std::pair<size_t, size_t>> used_list() const {
        return std::vector<std::pair<size_t, size_t>>(used_.begin(), used_.end());
    }

  private:
    size_t size_ = 0;
    std::map<size_t, size_t> free_;
    std::map<size_t, size_t> used_;
};

struct MatrixEntry {
    uint64_t id = 0;
    size_t bytes = 0;        // device bytes when resident (data + cached norms)
    bool resident = false;
    size_t offset = SIZE_MAX;
    int refs = 0;            // admitted requests using it
    uint64_t last_use = 0;   // admission tick of the last request
    uint64_t uploads = 0;
};

struct Waiting {
    uint64_t req = 0;
    uint64_t matrix = 0;
    size_t ws_bytes = 0;
};

struct Admission {
    uint64_t req = 0;
    uint64_t matrix = 0;
    size_t ws_offset = SIZE_MAX;
    size_t matrix_offset = SIZE_MAX;
    bool upload = false;                 // the matrix must be copied in first
    std::vector<uint64_t> evicted;       // matrices whose memory was reclaimed
};

// Residency and admission state (not thread-safe: the server holds a lock).
class Scheduler {
  public:
    explicit Scheduler(size_t arena_bytes = 0, int max_bypass = 8)
        : arena_(arena_bytes), max_bypass_(max_bypass) {}

    Arena& arena() { return arena_; }
    const Arena& arena() const { return arena_; }

    void add_matrix(uint64_t id, size_t bytes) {
        MatrixEntry e;
        e.id = id;
        e.bytes = bytes;
        mats_[id] = e;
    }
    const MatrixEntry* matrix(uint64_t id) const {
        auto it = mats_.find(id);
        return it == mats_.end() ? nullptr : &it->second;
    }
    // Drop a matrix (must be unused); frees its memory.
    bool remove_matrix(uint64_t id) {
        auto it = mats_.find(id);
        if (it == mats_.end() || it->second.refs > 0) return false;
        if (it->second.resident) arena_.release(it->second.offset);
        mats_.erase(it);
        return true;
    }

    // Whether the request could ever run (alone in an empty arena).
    bool fits_alone(uint64_t matrix, size_t ws_bytes) const {
        auto it = mats_.find(matrix);
        if (it == mats_.end()) return false;
        return align_up(it->second.bytes) + align_up(ws_bytes) <= arena_.size();
    }

    void enqueue(const Waiting& w) { queue_.push_back(w); }
    size_t waiting() const { return queue_.size(); }

    // Admit the first waiting request that fits (see the policy above).
    bool admit(Admission* out) {
        for (size_t qi = 0; qi < queue_.size(); ++qi) {
            if (qi > 0 && head_bypassed_ >= max_bypass_) return false;
            Waiting w = queue_[qi];
            if (try_place(w, out)) {
                queue_.erase(queue_.begin() + (std::ptrdiff_t)qi);
                if (qi > 0) ++head_bypassed_;
                else head_bypassed_ = 0;
                return true;
            }
        }
        return false;
    }

    // A request finished: free its workspace and drop its matrix reference.
    void finish(uint64_t matrix, size_t ws_offset) {
        arena_.release(ws_offset);
        auto it = mats_.find(matrix);
        if (it != mats_.end() && it->second.refs > 0) it->second.refs -= 1;
    }

    // Upload failed: forget the residency claimed by try_place.
    void drop_residency(uint64_t matrix) {
        auto it = mats_.find(matrix);
        if (it != mats_.end() && it->second.resident) {
            arena_.release(it->second.offset);
            it->second.resident = false;
            it->second.offset = SIZE_MAX;
        }
    }

    size_t resident_bytes() const {
        size_t s = 0;
        for (auto& kv : mats_)
            if (kv.second.resident) s += align_up(kv.second.bytes);
        return s;
    }
    uint64_t evictions() const { return evictions_; }

  private:
    bool try_place(const Waiting& w, Admission* out) {
        auto it = mats_.find(w.matrix);
        if (it == mats_.end()) return false;
        MatrixEntry& me = it->second;
        std::vector<uint64_t> evicted;
        size_t ws = arena_.alloc(w.ws_bytes);
        size_t moff = me.resident ? me.offset : SIZE_MAX;
        bool upload = false;
        if (!me.resident) {
            moff = (ws == SIZE_MAX) ? SIZE_MAX : arena_.alloc(me.bytes);
            upload = true;
        }
        // evict idle matrices (least recently used first) until both fit, but
        // only if the free space plus all idle matrices could hold the request
        if (ws == SIZE_MAX || moff == SIZE_MAX) {
            size_t avail = arena_.free_bytes();
            for (auto& kv : mats_)
                if (kv.second.resident && kv.second.refs == 0 && kv.second.id != w.matrix)
                    avail += align_up(kv.second.bytes);
            const size_t need = (ws == SIZE_MAX ? align_up(w.ws_bytes) : 0) +
                                (moff == SIZE_MAX ? align_up(me.bytes) : 0);
            if (avail < need) {
                if (ws != SIZE_MAX) arena_.release(ws);
                if (upload && moff != SIZE_MAX) arena_.release(moff);
                return false;
            }
        }
        while (ws == SIZE_MAX || moff == SIZE_MAX) {
            MatrixEntry* victim = nullptr;
            for (auto& kv : mats_) {
                MatrixEntry& c = kv.second;
                if (!c.resident || c.refs > 0 || c.id == w.matrix) continue;
                if (!victim || c.last_use < victim->last_use ||
                    (c.last_use == victim->last_use && c.id < victim->id))
                    victim = &c;
            }
            if (!victim) break;
            arena_.release(victim->offset);
            victim->resident = false;
            victim->offset = SIZE_MAX;
            evicted.push_back(victim->id);
            ++evictions_;
            if (ws == SIZE_MAX) ws = arena_.alloc(w.ws_bytes);
            if (ws != SIZE_MAX && moff == SIZE_MAX) moff = arena_.alloc(me.bytes);
        }
        if (ws == SIZE_MAX || moff == SIZE_MAX) {
            if (ws != SIZE_MAX) arena_.release(ws);
            if (upload && moff != SIZE_MAX) arena_.release(moff);
            // evicted matrices stay evicted: their memory is free for later
            out->evicted = evicted;
            return false;
        }
        if (upload) {
            me.resident = true;
            me.offset = moff;
            me.uploads += 1;
        }
        me.refs += 1;
        me.last_use = ++tick_;
        out->req = w.req;
        out->matrix = w.matrix;
        out->ws_offset = ws;
        out->matrix_offset = moff;
        out->upload = upload;
        out->evicted = evicted;
        return true;
    }

    Arena arena_;
    int max_bypass_;
    int head_bypassed_ = 0;
    uint64_t tick_ = 0;
    uint64_t evictions_ = 0;
    std::unordered_map<uint64_t, MatrixEntry> mats_;
    std::deque<Waiting> queue_;
};

}  // namespace serve
}  // namespace gpspca
