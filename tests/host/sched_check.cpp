// Checks the serving layer's admission control (hp_sched.h) on the CPU with a
// fake executor: every admitted request runs one loop per step and finishes
// after its own loop count. Test infrastructure; exits non-zero on the first
// failed check and prints "ok" otherwise.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "hp_sched.h"

#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);   \
            std::exit(1);                                                \
        }                                                                \
    } while (0)

static void first_fit() {
    hp::FirstFit f(1000);
    size_t a, b, c, d;
    CHECK(f.alloc(100, &a) && a == 0);
    CHECK(f.alloc(200, &b) && b == 100);
    CHECK(f.alloc(300, &c) && c == 300);
    f.release(b, 200);  // hole [100, 300)
    CHECK(f.free_ranges().size() == 2);
    CHECK(f.alloc(250, &d) && d == 600);  // the 200-byte hole is skipped
    size_t e;
    CHECK(!f.alloc(500, &e));
    f.release(a, 100);  // merges with the hole: [0, 300)
    CHECK(f.free_ranges().size() == 2 && f.free_ranges().begin()->second == 300);
    f.release(c, 300);  // [0, 600)
    f.release(d, 250);  // [0, 1000)
    CHECK(f.free_ranges().size() == 1 && f.free_ranges().begin()->second == 1000);
    CHECK(f.alloc(1000, &e) && e == 0 && f.free_ranges().empty());
}

static void arrival_order_and_slots() {
    hp::Admission adm(1000, 2);
    std::vector<uint64_t> order;
    auto enter = [&](uint64_t t, size_t) {
        order.push_back(t);
        return 0;
    };
    adm.submit(1, 600);
    adm.submit(2, 300);
    adm.submit(3, 200);
    adm.submit(4, 100);
    CHECK(adm.admit(enter) == 0);
    CHECK(order == (std::vector<uint64_t>{1, 2}));  // two slots
    adm.finish(1);
    CHECK(adm.admit(enter) == 0);
    CHECK(order == (std::vector<uint64_t>{1, 2, 3}));  // slots full again (2, 3)
    adm.finish(2);
    adm.finish(3);
    CHECK(adm.admit(enter) == 0 && order.back() == 4);
    // head of line: 5 needs more than is free, 6 would fit but must wait
    adm.submit(5, 950);
    adm.submit(6, 50);
    CHECK(adm.admit(enter) == 0 && order.back() == 4 && adm.waiting() == 2);
    adm.finish(4);
    CHECK(adm.admit(enter) == 0);
    CHECK(order.size() == 6 && order[4] == 5 && order[5] == 6);
    adm.finish(5);
    adm.finish(6);
    CHECK(adm.active_count() == 0 && adm.arena().free_ranges().size() == 1);
    // a failing placement is reported, stops admission and is taken back out
    // (its slot and range free again)
    adm.submit(7, 10);
    adm.submit(8, 10);
    CHECK(adm.admit([](uint64_t, size_t) { return -4; }) == -4 && adm.waiting() == 1);
    CHECK(adm.active_count() == 0 && adm.arena().free_ranges().size() == 1 &&
          adm.arena().free_ranges().begin()->second == 1000);
}

// hp::serve_step's error paths with a fake executor: a request whose set-up
// fails, one whose rerun set-up fails, a loop that fails after finishing some
// requests, and a successful rerun.
struct FakeReq {
    int loops = 1, done = 0, status = 0;
    bool finished = false, retried = false, settled = false;
    bool fail_enter = false, fail_reenter = false, fails_first_run = false;
};
struct FakeExec {
    std::map<uint64_t, FakeReq>& reqs;
    int loop_error = 0;  // returned by run() after its bookkeeping
    int enter(uint64_t t, size_t) {
        FakeReq& r = reqs[t];
        if (r.fail_enter) {
            r.status = -4;
            r.finished = true;
            return -4;
        }
        r.finished = false;
        return 0;
    }
    int run(const std::vector<uint64_t>& act) {
        for (uint64_t t : act) {
            FakeReq& r = reqs[t];
            CHECK(!r.finished);  // no loop on a finished or half-set-up request
            if (++r.done >= r.loops) {
                r.finished = true;
                r.status = (r.fails_first_run && !r.retried) ? 2 : 0;
            }
        }
        return loop_error;
    }
    bool finished(uint64_t t) { return reqs[t].finished; }
    bool wants_retry(uint64_t t) { return reqs[t].status > 0 && !reqs[t].retried; }
    int reenter(uint64_t t) {
        FakeReq& r = reqs[t];
        r.retried = true;
        r.done = 0;
        if (r.fail_reenter) {
            r.status = -4;
            r.finished = true;
            return -4;
        }
        r.status = 0;
        r.finished = false;
        return 0;
    }
    void fail(uint64_t t, int rc) {
        reqs[t].status = rc;
        reqs[t].finished = true;
    }
    void settle(uint64_t t) { reqs[t].settled = true; }
};

static void serve_step_error_paths() {
    std::map<uint64_t, FakeReq> reqs;
    hp::Admission adm(1000, 4);
    FakeExec ex{reqs};
    reqs[1].loops = 2;
    reqs[2].fail_enter = true;
    reqs[3].loops = 1;
    for (uint64_t t = 1; t <= 3; ++t) adm.submit(t, 300);
    // step 1: 2's set-up fails: it ends with the error, out of the active set,
    // its range free; admission stopped there (3 waits); 1 runs a loop
    CHECK(hp::serve_step(adm, ex) == -4);
    CHECK(reqs[2].finished && reqs[2].status == -4 && !reqs[2].settled);
    CHECK(adm.active_count() == 1 && adm.waiting() == 1);
    // step 2: 3 is admitted into 2's range; 1 and 3 finish
    CHECK(hp::serve_step(adm, ex) == 0);
    CHECK(reqs[1].settled && reqs[3].settled && reqs[1].status == 0 && reqs[3].status == 0);
    CHECK(adm.active_count() == 0 && adm.arena().free_ranges().begin()->second == 1000);

    // a failed solve is rerun; a rerun whose set-up fails ends with the error
    reqs[4].fails_first_run = true;
    reqs[5].fails_first_run = true;
    reqs[5].fail_reenter = true;
    adm.submit(4, 300);
    adm.submit(5, 300);
    CHECK(hp::serve_step(adm, ex) == -4);
    CHECK(!reqs[4].finished && reqs[4].retried && !reqs[4].settled);      // rerunning
    CHECK(reqs[5].finished && reqs[5].status == -4 && reqs[5].settled);   // not "ok"
    CHECK(adm.active_count() == 1);
    CHECK(hp::serve_step(adm, ex) == 0);
    CHECK(reqs[4].finished && reqs[4].status == 0 && reqs[4].settled);
    CHECK(adm.active_count() == 0 && adm.arena().free_ranges().begin()->second == 1000);

    // a loop that fails after finishing a request: that request is still
    // settled and its space freed; the error is returned
    reqs[6].loops = 1;
    reqs[7].loops = 3;
    adm.submit(6, 300);
    adm.submit(7, 300);
    ex.loop_error = -4;
    CHECK(hp::serve_step(adm, ex) == -4);
    CHECK(reqs[6].settled && adm.active_count() == 1);
    ex.loop_error = 0;
    CHECK(hp::serve_step(adm, ex) == 0 && hp::serve_step(adm, ex) == 0);
    CHECK(reqs[7].settled && adm.active_count() == 0);
    CHECK(adm.arena().free_ranges().size() == 1 &&
          adm.arena().free_ranges().begin()->second == 1000);
}

// Poisson-like replay: random sizes and loop counts; the invariants of the
// admission policy must hold at every step and every request must finish.
static void replay(unsigned seed) {
    std::mt19937_64 rng(seed);
    const size_t budget = 1 << 20;
    const int slots = 8;
    hp::Admission adm(budget, slots);
    struct Req {
        size_t bytes, off = 0;
        int loops, done = 0;
        bool admitted = false, finished = false;
    };
    std::map<uint64_t, Req> reqs;
    std::vector<uint64_t> admitted_order;
    uint64_t next = 1;
    const int total = 400;
    int steps = 0;
    while ((int)admitted_order.size() < total || adm.active_count() > 0) {
        CHECK(++steps < 100000);
        // arrivals: 0-2 per step
        for (int a = (int)(rng() % 3); a > 0 && next <= (uint64_t)total; --a) {
            Req r;
            r.bytes = 256 * (1 + rng() % 1024);  // up to 256 KiB
            r.loops = 1 + (int)(rng() % 12);
            reqs[next] = r;
            adm.submit(next, r.bytes);
            ++next;
        }
        CHECK(adm.admit([&](uint64_t t, size_t off) {
                  Req& r = reqs[t];
                  r.admitted = true;
                  r.off = off;
                  admitted_order.push_back(t);
                  return 0;
              }) == 0);
        // invariants: slot cap, budget, disjoint placements, arrival order
        const std::vector<uint64_t> act = adm.active();
        CHECK((int)act.size() <= slots);
        size_t used = 0;
        for (size_t i = 0; i < act.size(); ++i) {
            const Req& r = reqs[act[i]];
            CHECK(r.off + r.bytes <= budget);
            used += r.bytes;
            for (size_t j = i + 1; j < act.size(); ++j) {
                const Req& q = reqs[act[j]];
                CHECK(r.off + r.bytes <= q.off || q.off + q.bytes <= r.off);
            }
        }
        CHECK(used <= budget);
        for (size_t i = 1; i < admitted_order.size(); ++i)
            CHECK(admitted_order[i] == admitted_order[i - 1] + 1);
        // the fake executor: one loop for every active request
        for (uint64_t t : act) {
            Req& r = reqs[t];
            if (++r.done == r.loops) {
                r.finished = true;
                adm.finish(t);
            }
        }
        if (next > (uint64_t)total && adm.waiting() == 0 && adm.active_count() == 0) break;
    }
    for (auto& kv : reqs) CHECK(kv.second.finished && kv.second.done == kv.second.loops);
    CHECK(adm.arena().free_ranges().size() == 1 && adm.arena().free_ranges().begin()->second == budget);
}

int main() {
    first_fit();
    arrival_order_and_slots();
    serve_step_error_paths();
    for (unsigned s = 1; s <= 20; ++s) replay(s);
    std::printf("ok\n");
    return 0;
}
