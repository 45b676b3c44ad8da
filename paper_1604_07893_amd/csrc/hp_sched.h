// Admission control of the serving layer (hp_serve_*): plain C++ with no GPU
// dependence. Requests wait in arrival order and are admitted while a slot is
// free and their workspace fits in the server's HBM arena (first fit over a
// coalescing free list); a request that does not fit blocks the ones behind it
// (no overtaking, so a large request cannot starve). Finished requests return
// their space.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace hp {

// First-fit placement of byte ranges in [0, total).
class FirstFit {
public:
    explicit FirstFit(size_t total = 0) { reset(total); }
    void reset(size_t total) {
        free_.clear();
        if (total) free_[0] = total;
    }
    // Lowest-offset free range of at least `bytes`; false if none.
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t roff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                return true;
            }
        }
        return false;
    }
    // Returns a range from alloc, merging it with free neighbours.
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    const std::map<size_t, size_t>& free_ranges() const { return free_; }

private:
    std::map<size_t, size_t> free_;  // offset -> bytes
};

class Admission {
public:
    Admission(size_t budget = 0, int max_slots = 0) : arena_(budget), slots_(max_slots) {}
    void submit(uint64_t ticket, size_t bytes) { waiting_.push_back({ticket, bytes, 0}); }
    // Admits waiting requests in arrival order while a slot is free and the
    // first waiting one fits; enter(ticket, offset) places each admitted
    // request (a nonzero return stops admission and is returned, the request
    // staying admitted). Returns 0 otherwise.
    template <class Enter>
    int admit(Enter&& enter) {
        while (!waiting_.empty() && (int)active_.size() < slots_) {
            Entry e = waiting_.front();
            if (!arena_.alloc(e.bytes, &e.off)) break;
            waiting_.pop_front();
            active_.push_back(e);
            const int rc = enter(e.ticket, e.off);
            if (rc != 0) return rc;
        }
        return 0;
    }
    // Removes an active request and frees its range.
    void finish(uint64_t ticket) {
        for (size_t i = 0; i < active_.size(); ++i) {
            if (active_[i].ticket == ticket) {
                arena_.release(active_[i].off, active_[i].bytes);
                active_.erase(active_.begin() + (long)i);
                return;
            }
        }
    }
    std::vector<uint64_t> active() const {
        std::vector<uint64_t> t;
        for (const Entry& e : active_) t.push_back(e.ticket);
        return t;
    }
    size_t waiting() const { return waiting_.size(); }
    size_t active_count() const { return active_.size(); }
    const FirstFit& arena() const { return arena_; }

private:
    struct Entry {
        uint64_t ticket;
        size_t bytes, off;
    };
    FirstFit arena_;
    int slots_;
    std::deque<Entry> waiting_;
    std::vector<Entry> active_;
};

}  // namespace hp
