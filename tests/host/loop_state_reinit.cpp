// LoopState::init must clear every flag a previous solve of the same problem
// left behind (a served request that is run again in FP64 only reuses its
// state: a stale "projection pending" once sent that run into the Penrose
// projection of a plan without its buffers). Test infrastructure; prints
// "ok" or the first failed check.
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

int main() {
    hp_params p{};
    p.precision = HP_PREC_FP32_FP64;
    p.tol = 1e-10;
    p.tau_switch = 0.1;
    p.max_iter = 100;
    p.diverge_limit = 1e6;
    hp_result r{};
    hp::LoopState st;
    st.init(&p, &r, 1.0);
    // a failed first attempt: non-finite FP32 loop, projection deferred
    CHECK(st.step(1.0, 0.0, 0.0, false) == hp::LoopState::NEXT_STAGE);
    CHECK(!st.exit_converged);
    st.proj_pending = true;
    st.enter_stage(2);
    CHECK(st.step(1.0, 0.0, 0.0, false) == hp::LoopState::DONE && st.status == HP_NONFINITE);
    // the retry, FP64 only
    p.precision = HP_PREC_FP64;
    st.init(&p, &r, 1.0);
    CHECK(!st.proj_pending && !st.exit_converged && !st.probe && st.result_idx == -1);
    CHECK(st.stage == 2 && st.ik == 0 && st.in_ == 1 && st.k == 0);
    CHECK(st.step(1e-8, 1.0, 0.0, false) == hp::LoopState::CONTINUE);
    CHECK(!st.projection_due());
    std::printf("ok\n");
    return 0;
}
