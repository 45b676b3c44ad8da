// LoopState::sym_ok: the loops that may form their s x s products symmetric
// are, in FP64 solves, the first and those after a change d with
// (d/2)^p >= tol (so the loop expected to meet the stopping test, after a
// change below tol^(1/p), forms full products), at most L loops with
// p^L 2^-52 <= 1e-7; staged solves form full products throughout. Test infrastructure; prints "ok" or the first failed
// check.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "hp_loop.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);  \
            std::exit(1);                                               \
        }                                                               \
    } while (0)

static hp_params params(int method, int precision) {
    hp_params p{};
    p.method = method;
    p.precision = precision;
    p.tol = 1e-10;
    p.tau_switch = 0.1;
    p.max_iter = 100;
    p.diverge_limit = 1e6;
    return p;
}

int main() {
    hp_result r{};
    {
        // PM (order 18): threshold d >= 2 tol^(1/18) = 0.556
        hp_params p = params(HP_METHOD_PM, HP_PREC_FP64);
        hp::LoopState st;
        st.init(&p, &r, 1.0);
        CHECK(st.sym_ok());  // first loop
        CHECK(st.step(4.0, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 2
        CHECK(st.sym_ok());
        CHECK(st.step(0.36, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 0.6
        CHECK(st.sym_ok());
        CHECK(st.step(0.25, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 0.5
        CHECK(!st.sym_ok());
        CHECK(st.step(1e-12, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 1e-6
        CHECK(!st.sym_ok());
        // a re-initialised state starts over
        st.init(&p, &r, 1.0);
        CHECK(st.sym_ok());
    }
    {
        // SM (order 2): threshold 2 tol^(1/2) = 2e-5
        hp_params p = params(HP_METHOD_SM, HP_PREC_FP64);
        hp::LoopState st;
        st.init(&p, &r, 1.0);
        CHECK(st.step(1.0, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 1
        CHECK(st.step(1e-8, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 1e-4
        CHECK(st.sym_ok());
        CHECK(st.step(1e-10, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 1e-5
        CHECK(!st.sym_ok());
    }
    {
        // staged solves (X from FP32 or 16 bits) form full products throughout
        for (int prec : {HP_PREC_FP32_FP64, HP_PREC_MIXED, HP_PREC_FP32}) {
            hp_params p = params(HP_METHOD_PM, prec);
            hp::LoopState st;
            st.init(&p, &r, 1.0);
            CHECK(!st.sym_ok());
            CHECK(st.step(4.0, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 2
            CHECK(!st.sym_ok());
        }
    }
    {
        // the loop budget: 18^(k+1) 2^-52 <= 1e-7 for k + 1 <= 6
        hp_params p = params(HP_METHOD_PM, HP_PREC_FP64);
        hp::LoopState st;
        st.init(&p, &r, 1.0);
        for (int k = 0; k < 6; ++k) {
            CHECK(st.sym_ok());
            CHECK(st.step(16.0, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 4
        }
        CHECK(!st.sym_ok());
        // SM (order 2): 2^(k+1) 2^-52 <= 1e-7 up to k + 1 = 28
        hp_params q = params(HP_METHOD_SM, HP_PREC_FP64);
        st.init(&q, &r, 1.0);
        for (int k = 0; k < 28; ++k) {
            CHECK(st.sym_ok());
            CHECK(st.step(1.0, 1.0, 0.0, false) == hp::LoopState::CONTINUE);  // d = 1
        }
        CHECK(!st.sym_ok());
    }
    std::printf("ok\n");
    return 0;
}
