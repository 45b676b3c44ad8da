// Drives hp::LoopState (the library's per-loop control: stopping rules,
// stabilised switch, precision stages, guards) from a scripted sequence of
// per-loop stopping sums, with no GPU. Test infrastructure.
//
// stdin:  precision stop_rule tol tau_switch variant max_iter method alpha
//         diverge_limit low_dtype
//         then one line per loop: diff2 ref2 dinf [rnorm]; rnorm is the norm
//         of the next loop's residual, handed to probe_exit when the loop
//         asks for it (LoopState::probe)
// stdout: one JSON object with the action after each loop, the final status,
//         loop count, switch loop, per-stage loop counts, whether the returned
//         iterate is the newest one, the last stopping-rule value, and (for an
//         input that needs the Penrose projection on entering FP64) the loop
//         after which the projection runs (0: at the stage change; -1: never).
#include <cstdio>
#include <vector>

#include "hp_loop.h"

int main() {
    hp_params p{};  // the fields the loop control reads come from stdin
    if (std::scanf("%d %d %lf %lf %d %d %d %lf %lf %d", &p.precision, &p.stop_rule, &p.tol,
                   &p.tau_switch, &p.variant, &p.max_iter, &p.method, &p.alpha, &p.diverge_limit,
                   &p.low_dtype) != 10)
        return 2;
    hp_result r{};
    hp::LoopState st;
    st.init(&p, &r, p.alpha);
    st.keep_best = true;  // as the single-solve driver sets it
    // which iterate X_j each buffer of the current stage's set holds (the
    // driver's buffers: the loop writes X_{k+1} into in_; slot kBest takes a
    // copy of save_from when asked; entering FP64 copies from_idx into 0)
    int buf[4] = {0, -1, -1, -1};
    std::vector<int> actions;
    int projected_at = -1;
    bool returns_new = false, done = false;
    char line[512];
    while (!done && st.k < p.max_iter && std::fgets(line, sizeof line, stdin)) {
        double diff2, ref2, dinf, rnorm = -1.0;
        const int got = std::sscanf(line, "%lf %lf %lf %lf", &diff2, &ref2, &dinf, &rnorm);
        if (got < 3) continue;
        const int newest = st.in_;
        buf[st.in_] = st.k + 1;
        hp::LoopState::Action a = st.step(diff2, ref2, dinf, p.stop_rule == HP_STOP_ABS_INF);
        if (st.save_best) buf[hp::LoopState::kBest] = buf[st.save_from];
        if (a == hp::LoopState::CONTINUE && st.k < p.max_iter && st.probe && got == 4 &&
            st.probe_exit(rnorm))
            a = hp::LoopState::NEXT_STAGE;
        actions.push_back((int)a);
        if (a == hp::LoopState::CONTINUE && st.projection_due()) {
            st.projected();
            projected_at = st.k;
        }
        if (a == hp::LoopState::DONE) {
            done = true;
            returns_new = st.result_idx == newest;
        } else if (a == hp::LoopState::NEXT_STAGE) {
            if (st.stage + 1 == st.final_stage) {  // as for an input that needs the projection
                if (st.exit_converged) projected_at = 0;
                else st.proj_pending = true;
            }
            const int from = buf[st.from_idx];
            st.enter_stage(st.stage + 1);
            if (st.stage == 2) {
                buf[0] = from;
                buf[1] = buf[2] = buf[3] = -1;
            }
        }
    }
    if (!done) {
        st.finish_maxiter();
        returns_new = true;  // after a CONTINUE the newest iterate is the current one
    }
    const int returned = buf[st.result_idx];
    std::printf("{\"actions\": [");
    for (size_t i = 0; i < actions.size(); ++i) std::printf("%s%d", i ? ", " : "", actions[i]);
    std::printf("], \"status\": %d, \"iters\": %d, \"switch_iter\": %d, \"iters_stage\": [%d, %d, %d], "
                "\"returns_new\": %s, \"returned\": %d, \"stop_last\": %.17g, "
                "\"projected_at\": %d}\n",
                st.status, r.iters, r.switch_iter, r.iters_stage[0], r.iters_stage[1],
                r.iters_stage[2], returns_new ? "true" : "false", returned, r.stop_last,
                projected_at);
    return 0;
}
