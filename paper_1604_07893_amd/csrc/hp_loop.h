// The host-side control of one problem's iteration (stopping rules, the
// switch to the stabilised variant, precision stages, guards): plain C++ with
// no GPU dependence, shared by single, batched and served solves.
#pragma once

#include <cmath>
#include <cstdint>
#include <utility>

#include "hyperpower.h"

namespace hp {

// Which MFMA path a product runs on.
enum Engine { ENG_F64, ENG_F32, ENG_BF16, ENG_F16 };

// Order p of each HP_METHOD_* (the p of rule (stopreliable)).
inline int method_order(int method) {
    static const int kOrder[] = {18, 2, 3, 7, 18};
    return kOrder[method];
}

// Host-side state of one problem's iteration: the stopping rule, the switch
// to the stabilised variant, the precision stages and the guards.
struct LoopState {
    enum Action { CONTINUE, NEXT_STAGE, DONE };
    const hp_params* p = nullptr;
    hp_result* res = nullptr;
    double alpha = 0.0;
    int stage = 2;        // 0 16-bit, 1 FP32, 2 FP64
    int final_stage = 2;
    int first_stage = 2;  // the stage the solve started in
    bool stabilising = false;
    bool converging = false;
    bool stage_first = true;  // no stagnation test on a stage's first loop
    double d_prev = 0.0;
    int ik = 0, in_ = 1;  // current and next iterate (index into the stage's set)
    int k = 0;            // loops run
    int status = HP_MAXITER;
    int result_idx = -1;  // iterate to return (index into the final stage's set)
    int from_idx = 0;     // NEXT_STAGE: iterate the next stage starts from

    // The iterate returned on HP_DIVERGED, and on HP_NONFINITE before
    // convergence sets in (Section 6 warns that the loops can diverge; the
    // iterate just before the blow-up is already far off): the input of the
    // final-stage loop with the smallest relative change among the loops
    // before the change first fell below tau_switch. With keep_best (set by
    // the caller after init) the caller keeps a copy of that iterate: after a
    // step() that sets save_best it copies iterate save_from of the final
    // stage's set to slot kBest before the next loop runs. Without keep_best
    // those outcomes return X_k, the input of the loop that detected them.
    static constexpr int kBest = 3;

    // The change below which the stabilised loops start (and the stagnation
    // guard is armed): hp_params.tau_switch, but at least kTauFp32 when the
    // last stage is FP32. FP32 rounding seeds the null-space block of a
    // rank-deficient input 2^29 times above FP64's and it grows 18x per plain
    // loop (Theorem 6.2), so FP32 must switch a loop earlier (measured on the
    // 4096 x 2048 rank-1536 input: changes 0.81, 0.20, then 3.5 and growing).
    static constexpr double kTauFp32 = 0.25;
    double tau_switch() const {
        return final_stage == 1 && p->tau_switch < kTauFp32 ? kTauFp32 : p->tau_switch;
    }
    bool keep_best = false;
    bool have_best = false;
    bool save_best = false;
    int save_from = 0;
    double best_d = 0.0;

    // Set by step() after the first loop of the FP32 stage (when the FP64
    // stage follows) if that loop changed X by less than kPredict: the caller
    // may then form the next loop's residual R = I - A X_{k+1} (its first
    // product) and call probe_exit(||R||_F).
    bool probe = false;

    void init(const hp_params* prm, hp_result* r, double a);
    Engine engine() const;
    // Digest one loop's sums; `dinf` is used if have_dinf.
    Action step(double diff2, double ref2, double dinf, bool have_dinf);
    // After NEXT_STAGE the caller moves the iterate `from_idx` into the next
    // stage's set; this resets the indices (FP64 stage: X[0]).
    void enter_stage(int next);
    bool done() const { return result_idx >= 0; }
    // HP_STOP_REL_FRO_BOUND: after a CONTINUE, whether the next loop is a
    // plain loop of the final stage whose change the residual bound may
    // already settle (the last change d has d^p < tol).
    bool bound_ready() const;
    // After a probe: true (and the FP64 stage is to start from X_{k+1}) when
    // one loop of order p from there would take the residual below tol,
    // r^p < tol; otherwise the stage goes on (reusing R).
    bool probe_exit(double r) {
        if (!(std::isfinite(r) && std::pow(r, (double)method_order(p->method)) < p->tol)) return false;
        from_idx = ik;
        exit_converged = true;
        return true;
    }
    // On NEXT_STAGE: whether the lower stage ended in the converging regime
    // (last change below kPredict). The Penrose projection on entering FP64
    // assumes it; otherwise the caller defers the projection (proj_pending)
    // until projection_due(), after an FP64 loop whose change is that small,
    // and then calls projected().
    bool exit_converged = false;
    bool proj_pending = false;
    bool projection_due() const;
    void projected() {
        proj_pending = false;
        stage_first = true;  // the projection's own change is not a stall
    }
    // HP_STOP_REL_FRO_BOUND with PM, after a residual check that did not
    // settle (r = ||R||_F < 1): the scheme with the fewest products (SM, CM,
    // FM, PM) whose order q has r^q < tol/2, so that the check after the
    // loop settles.
    int scheme_for(double r) const {
        if (p->method != HP_METHOD_PM || !(r < 1.0)) return p->method;
        static const int kByCost[] = {HP_METHOD_SM, HP_METHOD_CM, HP_METHOD_FM, HP_METHOD_PM};
        for (int m : kByCost)
            if (std::pow(r, (double)method_order(m)) < p->tol / 2) return m;
        return HP_METHOD_PM;
    }
    // Whether the next loop may form its s x s products symmetric. They are
    // symmetric in exact arithmetic for X0 = alpha A^T; computing the upper
    // triangle and mirroring it turns the part K of R that is not symmetric
    // into a symmetric error of the same size, and that error grows by the
    // order p per loop in the directions not yet converged. So: FP64 solves
    // only (K at 1e-16; an FP32 stage's symmetric loops reached order one),
    // at most the first L loops with p^L * 2^-52 <= 1e-7, and after the first
    // loop only while the last change d has (d/2)^p >= tol. The loop expected
    // to meet the stopping test follows a change below tol^(1/p) and so forms
    // full products, which correct what the symmetric loops left.
    bool sym_ok() const {
        if (stage != 2 || first_stage != 2) return false;
        const double order = (double)method_order(p->method);
        if (std::pow(order, (double)(k + 1)) * 0x1p-52 > 1e-7) return false;
        if (k == 0) return true;
        if (stage_first || !std::isfinite(d_prev)) return false;
        return std::pow(d_prev / 2.0, order) >= p->tol;
    }
    // The residual bound settled it: return the current iterate.
    void stop_bound(double bound) {
        status = HP_OK;
        result_idx = ik;
        res->stop_last = bound;
    }
    void finish_maxiter() {
        if (result_idx < 0) result_idx = ik;
    }
};

}  // namespace hp
