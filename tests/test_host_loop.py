"""The library's per-loop control, hp::LoopState (paper_1604_07893_amd/csrc/
hp_loop.cpp: stopping rules of Section 4 and Example 8.1, the switch to
(PM-modified) of Section 7, the guards, the precision stages), compiled for
the CPU with g++ and driven by tests/host/loop_state_check.cpp; no GPU.

Against the oracle: fed the oracle's own per-loop sums (||X_{k+1}-X_k||_F^2,
||X_k||_F^2 and the inf-norm change), it must take the oracle's decisions --
loop count, status, switch loop, and whether the newest iterate or its
predecessor is returned. The precision-stage exits have no counterpart in the
paper or the oracle (they are this library's rule); they are checked on
scripted change sequences against the rule as documented in hp_loop.cpp.
"""

import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_1604_07893_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STOP = {"rel_fro": 0, "paper_4_1": 1, "abs_inf": 2}
VARIANT = {"plain": 0, "stabilised": 1, "stab_always": 2}
METHOD = {"pm": 0, "sm": 1, "cm": 2, "fm": 3, "hm": 4}
STATUS = {0: "ok", 1: "maxiter", 2: "stagnated", 3: "diverged", 4: "nonfinite"}
CONTINUE, NEXT_STAGE, DONE = 0, 1, 2


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("host") / "loop_state_check"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1604_07893_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "loop_state_check.cpp"),
                    os.path.join(ROOT, "paper_1604_07893_amd", "csrc", "hp_loop.cpp"),
                    "-o", str(exe)], check=True)

    def run(loops, *, precision=0, stop="rel_fro", tol=1e-12, tau=0.1, variant="plain",
            max_iter=100, method="pm", alpha=1.0, diverge=1e6, low=0):
        head = (f"{precision} {STOP[stop]} {tol!r} {tau!r} {VARIANT[variant]} {max_iter} "
                f"{METHOD[method]} {float(alpha)!r} {diverge!r} {low}\n")
        body = "".join(" ".join(repr(float(v)) for v in row) + "\n" for row in loops)
        out = subprocess.run([str(exe)], input=head + body, capture_output=True, text=True,
                             check=True)
        return json.loads(out.stdout)
    return run


def oracle_loops(res):
    return [(float(nD) ** 2, float(nX) ** 2, float(di))
            for (nD, nX), di in zip(res.fro_hist, res.diff_inf_hist)]


def check_against_oracle(harness, res, **kw):
    got = harness(oracle_loops(res), **kw)
    assert STATUS[got["status"]] == res.status
    assert got["iters"] == res.iters
    assert got["switch_iter"] == res.switch_iter
    # the same iterate is returned: X_{k+1} on success and at the loop cap,
    # X_k on stagnation, the best one before the blow-up on divergence
    assert got["returned"] == res.returned_iter
    assert got["returns_new"] == (res.status in ("ok", "maxiter"))
    assert got["actions"][-1] == (DONE if res.status != "maxiter" else CONTINUE)
    return got


def test_relative_change_stop_on_full_rank_input(harness):
    A = inputs.uniform(60, 30, seed=1)
    res = O.solve(A, tol=1e-12)
    assert res.status == "ok"
    check_against_oracle(harness, res, tol=1e-12)


@pytest.mark.parametrize("variant", ["plain", "stabilised", "stab_always"])
def test_guard_and_switch_on_rank_deficient_input(harness, variant):
    """Plain PM stagnates (the guard of Section 6); the stabilised variant
    switches at the first change below tau_switch and passes."""
    lr = inputs.lowrank_svd(120, 60, 40, smin=1e-3, seed=6)
    res = O.solve(lr.A, variant=variant, tol=1e-10)
    check_against_oracle(harness, res, variant=variant, tol=1e-10)


@pytest.mark.parametrize("alpha_scale", [2.5, 4.0])
def test_divergence_guard(harness, alpha_scale):
    """alpha sigma_1^2 > 2 breaks the convergence condition of Section 4."""
    A = inputs.uniform(60, 30, seed=1)
    a = alpha_scale / np.linalg.svd(A, compute_uv=False)[0] ** 2
    res = O.solve(A, alpha_rule="user", alpha=a, tol=1e-12)
    assert res.status == "diverged"
    check_against_oracle(harness, res, alpha=a, tol=1e-12)


@pytest.mark.parametrize("method", ["pm", "sm", "cm", "fm", "hm"])
def test_paper_rule_divides_by_p_to_the_k_alpha(harness, method):
    d = inputs.square_svd(48, smin=1e-2, seed=7)
    res = O.solve(d.A, method=method, stop="paper_4_1", tol=1e-8)
    got = check_against_oracle(harness, res, method=method, stop="paper_4_1", tol=1e-8,
                               alpha=float(res.alpha))
    assert got["stop_last"] == pytest.approx(float(res.stop_hist[-1]), rel=1e-12)


def test_absolute_inf_norm_rule_on_drazin_input(harness):
    dz = inputs.drazin_jordan(n=40, nb=30, seed=5)
    res = O.solve(dz.A, kind="drazin", l=dz.index, stop="abs_inf", tol=1e-10)
    check_against_oracle(harness, res, stop="abs_inf", tol=1e-10)


def test_loop_cap(harness):
    A = inputs.uniform(60, 30, seed=1)
    res = O.solve(A, tol=1e-12, max_iter=3)
    assert res.status == "maxiter"
    check_against_oracle(harness, res, tol=1e-12, max_iter=3)


def test_non_finite_change_returns_the_best_iterate_before_it(harness):
    got = harness([(1.0, 1.0, 0.0), (float("nan"), 1.0, 0.0), (1e-30, 1.0, 0.0)])
    assert STATUS[got["status"]] == "nonfinite" and got["iters"] == 2
    assert got["returns_new"] is False and got["returned"] == 0
    # after convergence set in (a change below tau_switch), the last finite one
    got = harness(rel_loops([3.0, 0.05, 1e-3]) + [(float("nan"), 1.0, 0.0)])
    assert STATUS[got["status"]] == "nonfinite" and got["returned"] == 3


def test_divergence_returns_the_input_of_the_smallest_change(harness):
    """A blow-up before convergence returns the iterate with the smallest
    change seen, not the one the blow-up started from (Section 6)."""
    got = harness(rel_loops([4.3, 3.7, 0.81, 0.14, 2.4, 15.9, 2e6]))
    assert STATUS[got["status"]] == "diverged" and got["iters"] == 7
    assert got["returned"] == 3  # X_3, the input of the loop that changed it by 0.14


def test_fp32_emulation_of_the_rank_deficient_4096x2048_run(harness):
    """The relative changes of the plain loops on the 4096x2048 rank-1536
    input with every product in FP32 (numpy float32 emulation of the GPU
    loops): the null-space block, seeded by rounding, grows 18x per loop
    (Theorem 6.2) before any change falls below 0.1. With that threshold
    (the FP64 default) the loops never switch and the guard returns X_7
    (error 8e-3 against the closed form in the emulation), not X_12 (1.6e4)."""
    ds = [4.285, 3.690, 3.655, 3.652, 3.625, 3.191, 0.810, 0.1355, 2.414, 15.85, 16.99, 18.21,
          2.19e6]
    got = harness(rel_loops(ds), variant="stabilised", tol=1e-10)
    assert STATUS[got["status"]] == "diverged" and got["iters"] == 13
    assert got["returned"] == 7 and got["switch_iter"] == -1


def test_fp32_solve_switches_before_the_null_space_block_grows(harness):
    """The same input solved in FP32 (precision 1): the switch threshold is at
    least 0.25, so the change 0.1355 of loop 8 starts the stabilised loops.
    Changes from the emulation of that run: loop 9, the first stabilised one,
    changes X by 0.142 (more than loop 8: it also removes the null-space
    block, Theorem 7.1) and is not tested for stagnation; loops 10-12 settle
    at the FP32 floor and loop 13's change rises, so the solve ends
    "stagnated" with X_12 (error 2.2e-3 against the closed form in the
    emulation)."""
    ds = [4.285, 3.690, 3.655, 3.652, 3.625, 3.191, 0.810, 0.1355, 0.142, 1.022e-3, 9.236e-4,
          9.230e-4, 9.258e-4]
    got = harness(rel_loops(ds), precision=1, variant="stabilised", tol=1e-10)
    assert got["switch_iter"] == 8
    assert STATUS[got["status"]] == "stagnated" and got["iters"] == 13
    assert got["returned"] == 12
    # an explicit threshold above 0.25 is kept: 0.9 switches after loop 7
    got = harness(rel_loops(ds[:8]), precision=1, variant="stabilised", tau=0.9, tol=1e-10)
    assert got["switch_iter"] == 7


def test_zero_iterate_reads_as_no_change(harness):
    """A = 0 gives alpha = 0, X0 = 0 and zero stopping sums: the change 0/0 is
    read as 0, so the first loop passes (the zero matrix's inverse is 0), as
    the oracle decides. With alpha > 0 a zero iterate (X0 below a precision's
    range) is not a result: 0/0 is non-finite."""
    got = harness([(0.0, 0.0, 0.0)], tol=1e-12, alpha=0.0)
    assert STATUS[got["status"]] == "ok" and got["iters"] == 1 and got["returns_new"]
    got = harness([(0.0, 0.0, 0.0)], stop="paper_4_1", tol=1e-12, alpha=0.0)
    assert STATUS[got["status"]] == "ok" and got["iters"] == 1
    got = harness([(0.0, 0.0, 0.0)], tol=1e-12, alpha=1e-90)
    assert STATUS[got["status"]] == "nonfinite"
    res = O.solve(np.zeros((4, 3)), kind="mp", tol=1e-12)
    assert res.alpha == 0
    check_against_oracle(harness, res, tol=1e-12, alpha=0.0)


def test_first_stabilised_loop_is_not_tested_for_stagnation(harness):
    """FP64: the loop right after the switch may change X more than the loop
    that triggered it; the next loops are tested again."""
    got = harness(rel_loops([3.0, 0.05, 0.08, 1e-3, 2e-3]), variant="stabilised", tol=1e-12)
    assert got["switch_iter"] == 2
    assert STATUS[got["status"]] == "stagnated" and got["iters"] == 5
    assert got["returned"] == 4
    # without the switch (plain variant) loop 3 is tested: 0.08 >= 0.05
    got = harness(rel_loops([3.0, 0.05, 0.08]), variant="plain", tol=1e-12)
    assert STATUS[got["status"]] == "stagnated" and got["iters"] == 3


# ---- precision stages (HP_PREC_MIXED = 2, HP_PREC_FP32 = 1) ------------------

def rel_loops(ds):
    return [(d * d, 1.0, 0.0) for d in ds]


def test_mixed_stages_exit_on_a_settled_change(harness):
    """16-bit: 0.9 (first), 0.4 (halved), then 0.15 < 0.2 on a non-first loop
    -> next stage; FP32: its first loop never exits on that rule, 1e-3 does;
    FP64 runs the stopping rule."""
    got = harness(rel_loops([0.9, 0.4, 0.15, 0.1, 1e-3, 1e-6, 1e-13]), precision=2, tol=1e-10)
    assert got["actions"] == [CONTINUE, CONTINUE, NEXT_STAGE, CONTINUE, NEXT_STAGE, CONTINUE, DONE]
    assert got["iters_stage"] == [3, 2, 2] and STATUS[got["status"]] == "ok"
    assert got["returns_new"] is True


def test_mixed_stage_exits_when_the_change_stops_halving(harness):
    # 0.6 >= 0.5 * 0.9: stalled -> next stage; then 1e-8 is below the FP32
    # floor on the FP32 stage's first loop -> FP64
    got = harness(rel_loops([0.9, 0.6, 1e-8, 1e-13]), precision=2, tol=1e-10)
    assert got["actions"] == [CONTINUE, NEXT_STAGE, NEXT_STAGE, DONE]
    assert got["iters_stage"] == [2, 1, 1]


def test_fp32_floor_exits_even_on_a_first_loop(harness):
    # below 10 u_fp32 = 6e-7: the FP32 stage has nothing left to gain
    got = harness(rel_loops([0.5, 1e-7, 1e-9, 1e-13]), precision=3, tol=1e-10)
    assert got["actions"] == [CONTINUE, NEXT_STAGE, CONTINUE, DONE]
    assert got["iters_stage"] == [0, 2, 2]


def test_fp32_only_precision_stops_on_its_own_tolerance(harness):
    got = harness(rel_loops([0.5, 1e-3, 1e-6]), precision=1, tol=1e-5)
    assert got["actions"] == [CONTINUE, CONTINUE, DONE]
    assert got["iters_stage"] == [0, 3, 0] and STATUS[got["status"]] == "ok"


def test_fp32_stage_leaves_after_one_loop_when_its_residual_allows(harness):
    """The first FP32 loop after the 16-bit stage changed X by 0.1 < 0.2; the
    residual of its output, ||R||_F = 0.05, satisfies 0.05^18 < tol, so the FP64
    stage starts from that output at once; with ||R||_F = 0.5 the FP32 stage
    goes on (and its next loop reuses R)."""
    seq = [(0.81, 1.0, 0.0), (0.16, 1.0, 0.0), (0.0225, 1.0, 0.0), (0.01, 1.0, 0.0, 0.05),
           (1e-12, 1.0, 0.0), (1e-26, 1.0, 0.0)]
    got = harness(seq, precision=2, tol=1e-10)
    assert got["actions"] == [CONTINUE, CONTINUE, NEXT_STAGE, NEXT_STAGE, CONTINUE, DONE]
    assert got["iters_stage"] == [3, 1, 2] and got["returns_new"] is True
    seq[3] = (0.01, 1.0, 0.0, 0.5)
    got = harness(seq, precision=2, tol=1e-10)
    assert got["actions"][:5] == [CONTINUE, CONTINUE, NEXT_STAGE, CONTINUE, NEXT_STAGE]
    assert got["iters_stage"][1] == 2


def test_fp32_stage_rides_out_the_transient_of_an_ill_conditioned_input(harness):
    """Changes of a square N(0,1) 340x340 request (kappa 2.6e3) under FP32
    loops: they rise and fall around 1 while the slow directions grow. A change
    of 0.79 after 1.43 is no stall; the stage ends only at 1.5e-5 (settled), in
    the converging regime, where the projection may run at once."""
    seq = rel_loops([15.9, 7.97, 2.27, 1.62, 1.43, 0.79, 4.5, 0.34, 1.5e-5, 1.3e-5, 1e-16])
    got = harness(seq, precision=3, tol=1e-10, variant="stabilised")
    assert got["actions"][:9] == [CONTINUE] * 8 + [NEXT_STAGE]
    assert got["iters_stage"] == [0, 9, 2] and STATUS[got["status"]] == "ok"
    assert got["projected_at"] == 0


def test_projection_waits_for_the_converging_regime(harness):
    """A lower stage that ends on a stall above kPredict (0.6 after 0.9) hands
    over an iterate that is not yet converging: the projection waits for the
    first FP64 change below 0.2."""
    got = harness(rel_loops([0.9, 0.6, 0.3, 0.01, 1e-9, 1e-16]), precision=3, tol=1e-12)
    assert got["actions"][:2] == [CONTINUE, NEXT_STAGE]
    assert got["projected_at"] == 4          # after the FP64 loop whose change was 0.01
    assert STATUS[got["status"]] == "ok"


def test_reinit_clears_the_state_of_a_previous_attempt(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "reinit"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1604_07893_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "loop_state_reinit.cpp"),
                    os.path.join(ROOT, "paper_1604_07893_amd", "csrc", "hp_loop.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout


def test_symmetric_products_only_far_from_the_tolerance(tmp_path):
    """LoopState::sym_ok (tests/host/loop_state_sym.cpp): the loop expected to
    meet the stopping test forms full products."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "sym"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1604_07893_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "loop_state_sym.cpp"),
                    os.path.join(ROOT, "paper_1604_07893_amd", "csrc", "hp_loop.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout


def test_symmetric_product_partition(tmp_path):
    """The stream-K partition of the symmetric product (hp_symk.h, shared with
    the kernel): every K-step once, pieces on consecutive blocks, whole tiles
    on single blocks, distinct partial slots below 2 * grid
    (tests/host/sym_partition_check.cpp)."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "symk"
    subprocess.run([gxx, "-std=c++17", "-O2", "-Wall",
                    "-I", os.path.join(ROOT, "paper_1604_07893_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "sym_partition_check.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
