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
    // request. A nonzero return from enter takes that request back out (its
    // slot and range are free again; it does not return to the queue),
    // stops admission and is returned. Returns 0 otherwise.
    template <class Enter>
    int admit(Enter&& enter) {
        while (!waiting_.empty() && (int)active_.size() < slots_) {
            Entry e = waiting_.front();
            if (!arena_.alloc(e.bytes, &e.off)) break;
            waiting_.pop_front();
            active_.push_back(e);
            const int rc = enter(e.ticket, e.off);
            if (rc != 0) {
                finish(e.ticket);
                return rc;
            }
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

// One scheduling step of the server: admission, one loop of every active
// request, then the bookkeeping of the requests that finished in it. Kept
// apart from the GPU work (the executor) so that its error paths can be
// checked on the CPU. Exec provides:
//   int  enter(t, offset)  set up an admitted request in its arena range;
//                          on failure it is out of the active set again
//   int  run(active)       one loop of every active request (marks those
//                          that finish; may fail after marking some)
//   bool finished(t)
//   bool wants_retry(t)    finished, failed, and may run again from its
//                          start in its own range (once)
//   int  reenter(t)        set that run up
//   void fail(t, rc)       finish a request with error rc
//   void settle(t)         record a finished request's times
// A request whose set-up or rerun set-up fails is finished with that error
// (its slot and range freed); every request that finished is settled and
// its space freed even when the loop failed. Returns the first error (the
// step's other work still done), else 0.
template <class Exec>
int serve_step(Admission& adm, Exec& ex) {
    uint64_t failed = 0;
    int rc = adm.admit([&](uint64_t t, size_t off) {
        const int r = ex.enter(t, off);
        if (r != 0) failed = t;
        return r;
    });
    if (rc != 0) ex.fail(failed, rc);
    const std::vector<uint64_t> act = adm.active();
    if (act.empty()) return rc;
    const int rl = ex.run(act);
    if (rc == 0) rc = rl;
    for (uint64_t t : act) {
        if (ex.finished(t) && ex.wants_retry(t)) {
            const int r = ex.reenter(t);
            if (r == 0) continue;  // runs again from its start
            ex.fail(t, r);
            if (rc == 0) rc = r;
        }
        if (ex.finished(t)) {
            ex.settle(t);
            adm.finish(t);
        }
    }
    return rc;
}

}  // namespace hp
