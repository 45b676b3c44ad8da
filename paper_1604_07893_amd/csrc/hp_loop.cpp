// LoopState: the decisions taken after each loop from its two stopping sums.
#include "hp_loop.h"

#include <algorithm>

namespace hp {

static constexpr double kUnitRoundoffF32 = 5.960464477539063e-08;
// A lower stage ends after a loop (other than its first) whose relative
// change falls below this. That change measures the error of the loop's
// input; the loop's output has about that error to the 18th power (0.2^18 <
// 1e-12), i.e. it is already at the stage's rounding floor, and a further
// loop would only confirm it.
static constexpr double kPredict = 0.2;

void LoopState::init(const hp_params* prm, hp_result* r, double a) {
    p = prm;
    res = r;
    alpha = a;
    stage = p->precision == HP_PREC_MIXED ? 0
            : (p->precision == HP_PREC_FP32 || p->precision == HP_PREC_FP32_FP64) ? 1
                                                                                  : 2;
    final_stage = p->precision == HP_PREC_FP32 ? 1 : 2;
    first_stage = stage;
    stabilising = p->variant == HP_VARIANT_STAB_ALWAYS;
    res->switch_iter = stabilising ? 0 : -1;
    converging = false;
    stage_first = true;
    d_prev = 0.0;
    ik = 0;
    in_ = 1;
    k = 0;
    status = HP_MAXITER;
    result_idx = -1;
    from_idx = 0;
    probe = false;
    exit_converged = false;
    proj_pending = false;
    keep_best = false;
    have_best = false;
    save_best = false;
    save_from = 0;
    best_d = 0.0;
}

Engine LoopState::engine() const {
    if (stage == 2) return ENG_F64;
    if (stage == 1) return ENG_F32;
    return p->low_dtype == HP_LOWP_F16 ? ENG_F16 : ENG_BF16;
}

void LoopState::enter_stage(int next) {
    stage = next;
    stage_first = true;
    if (next == 2) {
        ik = 0;
        in_ = 1;
    } else {
        ik = from_idx;
        in_ = from_idx == 0 ? 1 : 0;
    }
}

LoopState::Action LoopState::step(double diff2, double ref2, double dinf, bool have_dinf) {
    probe = false;
    save_best = false;
    res->iters = k + 1;
    res->iters_stage[stage] += 1;
    // alpha = 0 (A = 0 under the norm rule, or a caller's 0): X0 = 0 is the
    // outer inverse with range {0}, and X_k = X_{k+1} = 0 is no change. Any
    // other zero iterate (e.g. X0 below FP32's range) leaves 0/0: non-finite.
    const double d = (diff2 == 0.0 && ref2 == 0.0 && alpha == 0.0)
                         ? 0.0
                         : std::sqrt(diff2) / std::sqrt(ref2);
    if (k < HP_HIST) {
        res->d_hist[k] = d;
        if (have_dinf) res->dinf_hist[k] = dinf;
    }
    res->d_stage[stage] = d;
    res->d_last = d;
    ++k;
    const bool finite = std::isfinite(d) && std::isfinite(diff2) && (!have_dinf || std::isfinite(dinf));
    auto note_switch = [&]() {
        if (d < tau_switch()) {
            converging = true;
            if (p->variant == HP_VARIANT_STABILISED && !stabilising) {
                stabilising = true;
                res->switch_iter = k;
            }
        }
    };

    if (stage != final_stage) {
        // a lower stage ends when its change stops halving, reaches its
        // rounding floor, or goes non-finite (16-bit overflow); the next stage
        // continues from the better of the last two iterates
        const double u = stage == 0 ? (p->low_dtype == HP_LOWP_F16 ? 4.8828125e-4 : 3.90625e-3)
                                    : kUnitRoundoffF32;
        // (two changes below 1 in a row: while the slow directions still grow,
        // on ill-conditioned input, the change can rise and fall above and
        // around 1 without any stall)
        const bool stalled = !stage_first && d < 1.0 && d_prev < 1.0 && d >= 0.5 * d_prev;
        const bool floor = d < 10.0 * u || d < p->tol;
        if (finite) note_switch();
        // (not on a stage's first loop: its change is mostly the step between
        // the two precisions and says little about the slow directions)
        const bool settled = finite && d < kPredict && !stage_first;
        if (!finite || stalled || floor || settled) {
            const bool keep_new = finite && !(stalled && d >= d_prev);
            from_idx = keep_new ? in_ : ik;
            exit_converged = finite && d < kPredict;
            d_prev = d;
            return NEXT_STAGE;
        }
        // the first FP32 loop's change says little about the slow directions
        // (above), but the residual of its output measures them directly
        probe = stage == 1 && final_stage == 2 && stage_first && d < kPredict;
        stage_first = false;
        d_prev = d;
        std::swap(ik, in_);
        return CONTINUE;
    }

    // before convergence sets in, a blow-up returns the best iterate seen
    const int fallback = (keep_best && have_best && !converging) ? kBest : ik;
    if (!finite) {
        status = HP_NONFINITE;
        result_idx = fallback;
        return DONE;
    }
    double sval;
    bool passed;
    if (p->stop_rule == HP_STOP_REL_FRO || p->stop_rule == HP_STOP_REL_FRO_BOUND) {
        sval = d;
        passed = d < p->tol;
    } else if (p->stop_rule == HP_STOP_ABS_INF) {
        sval = dinf;
        passed = dinf <= p->tol;
    } else {
        sval = diff2 == 0.0 ? 0.0
                            : std::sqrt(diff2) /
                                  (std::pow((double)method_order(p->method), (double)(k - 1)) * alpha);
        passed = sval < p->tol;
    }
    res->stop_last = sval;
    if (passed) {
        status = HP_OK;
        result_idx = in_;
        return DONE;
    }
    // the first stabilised loop after the switch is not compared: its change
    // also removes the null-space block (Theorem 7.1)
    const bool first_stab = p->variant == HP_VARIANT_STABILISED && res->switch_iter > 0 &&
                            k == res->switch_iter + 1;
    if (converging && !stage_first && !first_stab && d >= d_prev) {
        status = HP_STAGNATED;
        result_idx = ik;
        return DONE;
    }
    if (!converging && d > p->diverge_limit) {
        status = HP_DIVERGED;
        result_idx = fallback;
        return DONE;
    }
    note_switch();
    if (keep_best && !converging && (!have_best || d < best_d)) {
        best_d = d;
        have_best = true;
        save_best = true;
        save_from = ik;
    }
    stage_first = false;
    d_prev = d;
    std::swap(ik, in_);
    return CONTINUE;
}

bool LoopState::projection_due() const {
    return proj_pending && stage == final_stage && d_prev < kPredict;
}

bool LoopState::bound_ready() const {
    if (p->stop_rule != HP_STOP_REL_FRO_BOUND || stage != final_stage || stabilising) return false;
    return std::pow(d_prev, (double)method_order(p->method)) < p->tol;
}

}  // namespace hp
