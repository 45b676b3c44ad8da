"""Literal CPU implementation of the hyperpower iterations (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this
module; the product path never does.

Citations name the paper's sections, equations (by their LaTeX labels, e.g.
``(PM)``, ``(PM-modified)``, ``(stopreliable)``) and tables.

Pins (what ties this file to something other than itself) live in
``tests/test_oracle_pins.py``:
  * the PM constants: the polynomial identity of Section 2, checked exactly;
  * ``pm_step``: equals the 18-term definition (hyper18) and gives
    F_{k+1} = F_k^18 (Theorem 3.1) in multiple precision;
  * ``solve`` (loop, X0 rules, stop rule, iteration counting, COC): the paper's
    worked Example 8.1 / Table 1 at 150 digits, for SM, CM, FM and PM;
  * Moore-Penrose results: LAPACK SVD pseudo-inverse and closed forms from
    the factors, plus the four Penrose equations;
  * Drazin results: the Jordan-form closed form;
  * the iteration limit: classical order-2 Newton-Schulz reaches the same X;
  * Theorem 6.2 / 7.1: the E22 block grows 18x per plain loop and is removed by
    the stabilising product;
  * ``norm_1`` / ``norm_inf`` (the alpha of Section 4): hand-summed values and
    numpy's matrix norms;
  * ``penrose_residuals`` / ``drazin_residuals``: closed forms on iterates
    with a known error built in the factors' bases.
Parity unpinned: the (stopreliable) branch of ``solve`` (stop="paper_4_1"):
the paper prints no outcome of that rule, so only its quantity is checked.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

try:  # multiple precision is only needed for the 150-digit worked example
    import mpmath
except ImportError:  # pragma: no cover
    mpmath = None


# ---------------------------------------------------------------------------
# Element arithmetic: IEEE binary64 or mpmath numbers in numpy object arrays.
# ---------------------------------------------------------------------------

class Arith:
    """Scalar/array helpers for one element type."""

    def __init__(self, name: str):
        self.name = name

    # scalars -----------------------------------------------------------
    def num(self, v):
        if self.name == "f64":
            return float(v)
        return mpmath.mpf(v)

    def sqrt(self, v):
        return math.sqrt(v) if self.name == "f64" else mpmath.sqrt(v)

    def log(self, v):
        return math.log(v) if self.name == "f64" else mpmath.log(v)

    # arrays ------------------------------------------------------------
    def asarray(self, a):
        if self.name == "f64":
            return np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
        a = np.asarray(a, dtype=object)
        return np.vectorize(mpmath.mpf, otypes=[object])(a)

    def eye(self, n):
        if self.name == "f64":
            return np.eye(n)
        e = np.empty((n, n), dtype=object)
        e[...] = mpmath.mpf(0)
        for i in range(n):
            e[i, i] = mpmath.mpf(1)
        return e

    def isfinite(self, a) -> bool:
        if self.name == "f64":
            return bool(np.all(np.isfinite(a)))
        return all(mpmath.isfinite(x) for x in a.ravel())


F64 = Arith("f64")
MP = Arith("mp")


# ---------------------------------------------------------------------------
# Constants of the factored polynomial, Section 2.
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class PMConstants:
    c1: object
    c2: object
    c3: object
    d1: object
    d2: object
    mu: object
    psi: object


def octic_constants(ar: Arith = F64) -> dict:
    """a1, a2, a3, b1, b2, mu, psi: the solution of the seven-equation system
    that splits the even-power sum of (hyper18-3) into two octics in R^2 plus
    mu R^2 + psi R^4 (Section 2, (hyper18-33) and the closed forms after it)."""
    n = ar.num
    r93 = ar.sqrt(n(93))
    return dict(
        a1=n(5) / 496 * (31 + r93),
        a2=(3 + r93) / 8,
        a3=n(1) / 2,
        b1=n(-5) / 496 * (r93 - 31),
        b2=(3 - r93) / 8,
        mu=n(3) / 8,
        psi=n(321) / 1984,
    )


def pm_constants(ar: Arith = F64) -> PMConstants:
    """c1, c2, c3 of (simplify1), d1, d2 of (simplify2), mu and psi of
    (hyper18-33): the closed forms printed in Section 2, evaluated in the
    arithmetic ``ar``."""
    n = ar.num
    r93 = ar.sqrt(n(93))
    q = ar.sqrt(27 - 2 * r93)
    return PMConstants(
        c1=(q + 1) / 4,
        c2=(1 - q) / 4,
        c3=(5 * r93 - 93) / 496,
        d1=(-93 - 5 * r93) / 496,
        d2=-r93 / 4,
        mu=n(3) / 8,
        psi=n(321) / 1984,
    )


# ---------------------------------------------------------------------------
# Norms (plain definitions).
# ---------------------------------------------------------------------------

def norm_1(a):
    """Largest absolute column sum."""
    return np.abs(a).sum(axis=0).max()


def norm_inf(a):
    """Largest absolute row sum."""
    return np.abs(a).sum(axis=1).max()


def norm_fro(a, ar: Arith = F64):
    if np.iscomplexobj(a):
        return ar.sqrt(float((np.abs(a) ** 2).sum()))
    return ar.sqrt((a * a).sum())


def adjoint(A):
    """A^* (conjugate transpose; the transpose for real A)."""
    return A.conj().T if np.iscomplexobj(A) else A.T


# ---------------------------------------------------------------------------
# Initial approximations, Section 4.
# ---------------------------------------------------------------------------

def x0_moore_penrose(A, rule: str = "norm1inf", alpha=None, ar: Arith = F64):
    """X0 = alpha * A^* for the Moore-Penrose inverse (A^T for real A).

    rule "norm1inf":   alpha = 1 / (||A||_1 ||A||_inf)          (Section 4)
    rule "sigma_max2": alpha = 1 / sigma_1^2                    (scaling that
                       keeps ||I - A X0||_2 < 1, condition of Theorem 3.1)
    rule "sigma_opt":  alpha = 2 / (sigma_1^2 + sigma_r^2)       (Section 4, the
                       Pan-Schreiber choice; sigma read as singular values of A)
    rule "user":       alpha given.
    Singular values come from LAPACK; that is allowed here (oracle only).
    Returns (X0, alpha).
    """
    if rule == "norm1inf":
        # A = 0: the rule's denominator vanishes; X0 = alpha A^* = 0 for any
        # alpha (G = 0, so the outer inverse with range R(G) = {0} is 0)
        den = norm_1(A) * norm_inf(A)
        alpha = 1 / den if den != 0 else den * 0
    elif rule in ("sigma_max2", "sigma_opt"):
        s = np.linalg.svd(np.asarray(A, dtype=np.complex128 if np.iscomplexobj(A) else np.float64),
                          compute_uv=False)
        s1 = s[0]
        if rule == "sigma_max2":
            alpha = 1.0 / (s1 * s1)
        else:
            sr = s[s > s1 * max(A.shape) * np.finfo(float).eps][-1]
            alpha = 2.0 / (s1 * s1 + sr * sr)
        alpha = ar.num(alpha)
    elif rule == "user":
        if alpha is None:
            raise ValueError("rule 'user' needs alpha")
        alpha = ar.num(alpha)
    else:
        raise ValueError(f"unknown alpha rule {rule!r}")
    return alpha * adjoint(A), alpha


def x0_diag(A, ar: Arith = F64):
    """X0 = diag(1/a_11, ..., 1/a_nn), the initial matrix (choice3) of
    Example 8.3 (square A). Here G = X0 itself, so the limit is A^{-1} when A
    is nonsingular and the loops converge. Returns (X0, 1)."""
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("the diagonal initial matrix needs a square A")
    X0 = ar.eye(n) * 0
    for i in range(n):
        X0[i, i] = 1 / A[i, i]
    return X0, ar.num(1)


def chop(X, eps):
    """The sparsity control of Example 8.3 (Mathematica's Chop[X, eps]): every
    entry with |x| < eps becomes 0."""
    Y = X.copy()
    Y[np.abs(X) < eps] = 0
    return Y


def x0_drazin(A, l: int, ar: Arith = F64):
    """X0 = A^l / Tr(A^{l+1}) with l >= ind(A) (Section 4; Example 8.1).
    Returns (X0, alpha) with alpha = 1 / Tr(A^{l+1})."""
    n = A.shape[0]
    Al = ar.eye(n)
    for _ in range(l):
        Al = Al @ A
    tr = np.trace(Al @ A)
    alpha = 1 / tr
    return alpha * Al, alpha


# ---------------------------------------------------------------------------
# One loop of each iteration.
# ---------------------------------------------------------------------------

def pm_step(A, X, K: PMConstants, ar: Arith = F64):
    """One loop of PM, Section 2, iteration (PM): seven products, in the
    association the paper prints."""
    I = ar.eye(A.shape[0])
    R = I - A @ X                                   # product 1
    R2 = R @ R                                      # product 2
    R4 = R2 @ R2                                    # product 3
    M = (I + K.c1 * R2 + R4) @ (I + K.c2 * R2 + R4)  # product 4
    T = M + K.c3 * R2
    S = M + K.d1 * R2 + K.d2 * R4
    V = T @ S + K.mu * R2 + K.psi * R4              # product 5
    return X @ ((I + R) @ V)                        # products 6 and 7


def stabilise(A, Xh):
    """The extra step of (PM-modified), Section 7: X_{k+1} = X_{k+1/2} A X_{k+1/2}."""
    return Xh @ A @ Xh


def hyperpower_direct_step(A, X, p: int, ar: Arith = F64):
    """The hyperpower family (Hyperpower1), Section 1.3, by its definition:
    X_{k+1} = X_k (I + R + R^2 + ... + R^{p-1}), R = I - A X_k."""
    I = ar.eye(A.shape[0])
    R = I - A @ X
    P = I
    acc = I
    for _ in range(1, p):
        P = P @ R
        acc = acc + P
    return X @ acc


def sm_step(A, X, K=None, ar: Arith = F64):
    """Newton-Schulz-Hotelling (schulz), Section 1.3: X (2I - A X)."""
    I = ar.eye(A.shape[0])
    return X @ (2 * I - A @ X)


def cm_step(A, X, K=None, ar: Arith = F64):
    """Chebyshev-Sen-Prabhu (chebyshev), Section 1.3: X (3I - A X (3I - A X))."""
    I = ar.eye(A.shape[0])
    AX = A @ X
    return X @ (3 * I - AX @ (3 * I - AX))


def fm_step(A, X, K=None, ar: Arith = F64):
    """The seventh-order factorisation (SoleymaniN), Section 1.3."""
    I = ar.eye(A.shape[0])
    psi = I - A @ X
    psi2 = psi @ psi
    zeta = I + psi + psi2
    ups = psi + psi2 @ psi2
    return X @ (I + ups @ zeta)


def hm_step(A, X, K=None, ar: Arith = F64):
    """The 18th-order product of five factors (hyper18-2), Section 2."""
    I = ar.eye(A.shape[0])
    R = I - A @ X
    R2 = R @ R
    R3 = R2 @ R
    R6 = R3 @ R3
    return X @ (R + I) @ (R2 - R + I) @ (R2 + R + I) @ (R6 - R3 + I) @ (R6 + R3 + I)


STEP_FUNCTIONS = {"pm": pm_step, "sm": sm_step, "cm": cm_step, "fm": fm_step, "hm": hm_step}
ORDER = {"pm": 18, "sm": 2, "cm": 3, "fm": 7, "hm": 18}


# ---------------------------------------------------------------------------
# The iteration with its stopping rule, variant switch and guards.
# ---------------------------------------------------------------------------

@dataclass
class Result:
    X: object
    status: str                 # ok | maxiter | stagnated | diverged | nonfinite
    iters: int                  # loops run, including the one whose test passed
    alpha: object
    d_hist: list = field(default_factory=list)      # relative Frobenius changes
    stop_hist: list = field(default_factory=list)   # the stopping rule's values
    diff_inf_hist: list = field(default_factory=list)  # ||X_{k+1}-X_k||_inf
    switch_iter: int = -1       # first loop run stabilised (-1: never)
    bound_hist: list = field(default_factory=list)  # ||R||_F of "rel_fro_bound" checks
    fro_hist: list = field(default_factory=list)    # (||X_{k+1}-X_k||_F, ||X_k||_F) per loop
    method_hist: list = field(default_factory=list) # scheme run by each loop
    returned_iter: int = 0      # k of the returned iterate X_k (X_0 = X0)


def solve(A, *, kind: str = "mp", l: int | None = None, alpha_rule: str = "norm1inf",
          alpha=None, X0=None, method: str = "pm", variant: str = "plain",
          tau_switch: float = 0.1, stop: str = "rel_fro", tol: float = 1e-12,
          max_iter: int = 100, diverge_limit: float = 1e6, chop_eps: float = 0.0,
          ar: Arith = F64) -> Result:
    """Run a hyperpower iteration to a generalized inverse of A.

    kind      "mp": Moore-Penrose, X0 = alpha A^T (Section 4); with
              alpha_rule "diag", X0 = diag(1/a_ii) of Example 8.3 instead
              (square A, limit A^{-1}).
              "drazin": X0 = A^l / Tr(A^{l+1}), l >= ind(A) (Section 4).
    method    "pm" (the paper's 7-product scheme) or one of the comparison
              schemes "sm", "cm", "fm", "hm" (Sections 1.3 and 2).
    variant   "plain": (PM) every loop.
              "stabilised": plain loops until the relative change first drops
              below tau_switch, then (PM-modified) for every later loop -- the
              switch recipe that closes Section 7.
              "stab_always": (PM-modified) from X0 (kept for the test that
              shows why the switch is needed).
    stop      "rel_fro":  ||X_{k+1}-X_k||_F / ||X_k||_F < tol.
              "abs_inf":  ||X_{k+1}-X_k||_inf <= tol (Example 8.1).
              "paper_4_1": ||X_{k+1}-X_k||_F / (p^k alpha) < tol, rule
              (stopreliable) of Section 4 with the Frobenius norm (Example 8.2).
              "rel_fro_bound": "rel_fro", and before a plain loop that follows
              a change d with d^p < tol, r = ||I - A X_{k+1}||_F is formed;
              r/(1-r) < tol (r < 1) bounds the change that loop would make
              below tol, so X_{k+1} is returned without it; otherwise, for
              method "pm", that loop runs the scheme with the fewest products
              (SM, CM, FM, PM: orders 2, 3, 7, 18) whose order q has
              r^q < tol/2, which makes the next check settle (additions to the
              paper's rules).
    chop_eps  > 0: entries of each new iterate below chop_eps in magnitude are
              set to 0 at the end of the loop, before its change is measured
              (Example 8.3).
    Guards (the warning of Section 6 that looping past convergence can
    diverge): a non-finite iterate ends with "nonfinite" and the last finite
    iterate; once some relative change below tau_switch has been seen, a change
    that does not decrease ends with "stagnated" and returns X_k, the input of
    that loop (the first stabilised loop after the switch is exempt: its change
    also removes the null-space block of Theorem 7.1, which no plain loop
    measured); a relative change above diverge_limit before then ends with
    "diverged"; max_iter loops end with "maxiter" (Section 8 uses 100).
    On "diverged", and on "nonfinite" before some change below tau_switch has
    been seen, the returned iterate is the best one before the blow-up: the
    input of the loop with the smallest relative change so far (X_k itself if
    no earlier loop qualifies).
    The returned iterate on success is X_{k+1}, and iters counts the loops run.
    """
    if not (isinstance(A, np.ndarray) and (A.dtype == object) == (ar is MP)):
        A = ar.asarray(A)
    if X0 is not None:
        X = X0
        alpha = ar.num(alpha) if alpha is not None else ar.num(1)
    elif kind == "mp" and alpha_rule == "diag":
        X, alpha = x0_diag(A, ar)
    elif kind == "mp":
        X, alpha = x0_moore_penrose(A, alpha_rule, alpha, ar)
    elif kind == "drazin":
        if l is None:
            raise ValueError("drazin needs l >= ind(A)")
        X, alpha = x0_drazin(A, l, ar)
    else:
        raise ValueError(f"unknown kind {kind!r}")

    p = ORDER[method]
    K = pm_constants(ar)
    res = Result(X=X, status="maxiter", iters=0, alpha=alpha)
    stabilising = variant == "stab_always"
    if stabilising:
        res.switch_iter = 0
    converging = False
    next_method = None
    best = None  # (d, k, X_k): the input of the loop with the smallest change
    for k in range(max_iter):
        use = next_method or method
        next_method = None
        res.method_hist.append(use)
        Xn = STEP_FUNCTIONS[use](A, X, K, ar)
        if stabilising:
            Xn = stabilise(A, Xn)
        if chop_eps > 0:
            Xn = chop(Xn, chop_eps)
        res.iters = k + 1
        if not ar.isfinite(Xn):
            if best is not None and not converging:
                res.status, res.X, res.returned_iter = "nonfinite", best[2], best[1]
            else:
                res.status, res.X, res.returned_iter = "nonfinite", X, k
            return res
        D = Xn - X
        nD, nX = norm_fro(D, ar), norm_fro(X, ar)
        # alpha = 0 (A = 0 under the rule of Section 4, or a user's 0): X0 = 0 is
        # the outer inverse with range R(X0) = {0}; X_k = X_{k+1} = 0 is read as
        # no change. Any other zero iterate leaves the change undefined.
        if nX != 0:
            d = nD / nX
        elif nD == 0 and alpha == 0:
            d = nD
        else:
            d = ar.num(np.nan)
        res.fro_hist.append((nD, nX))
        res.d_hist.append(d)
        res.diff_inf_hist.append(norm_inf(D))
        if stop in ("rel_fro", "rel_fro_bound"):
            sval, passed = d, d < tol
        elif stop == "abs_inf":
            sval = res.diff_inf_hist[-1]
            passed = sval <= tol
        elif stop == "paper_4_1":
            sval = nD / (ar.num(p) ** k * alpha) if nD != 0 else nD
            passed = sval < tol
        else:
            raise ValueError(f"unknown stop rule {stop!r}")
        res.stop_hist.append(sval)
        if not (bool(np.isfinite(d)) if ar.name == "f64" else mpmath.isfinite(d)):
            res.status, res.X, res.returned_iter = "nonfinite", X, k
            return res
        if passed:
            res.status, res.X, res.returned_iter = "ok", Xn, k + 1
            return res
        # the first stabilised loop after the switch is not compared: its
        # change includes the removal of the null-space block (Theorem 7.1),
        # which the plain loops before it did not measure
        first_stab = variant == "stabilised" and res.switch_iter == k
        if converging and not first_stab and d >= res.d_hist[-2]:
            res.status, res.X, res.returned_iter = "stagnated", X, k
            return res
        if not converging and d > diverge_limit:
            if best is not None:
                res.status, res.X, res.returned_iter = "diverged", best[2], best[1]
            else:
                res.status, res.X, res.returned_iter = "diverged", X, k
            return res
        if d < tau_switch:
            converging = True
            if variant == "stabilised" and not stabilising:
                stabilising = True
                res.switch_iter = k + 1
        if not converging and (best is None or d < best[0]):
            best = (d, k, X)
        if (stop == "rel_fro_bound" and not stabilising and k + 1 < max_iter
                and d ** p < tol):
            # The next (plain) loop changes X by X (R + R^2 + ... + R^{p-1})
            # with R = I - A X, whose Frobenius norm is at most
            # ||X||_F ||R||_2 / (1 - ||R||_2) <= ||X||_F r / (1 - r),
            # r = ||R||_F < 1: when that is below tol the loop need not run.
            # (An addition to the paper's stopping rules.)
            R = ar.eye(A.shape[0]) - A @ Xn
            r = norm_fro(R, ar)
            res.bound_hist.append(r)
            if r < 1 and r / (1 - r) < tol:
                res.status, res.X, res.returned_iter = "ok", Xn, k + 1
                return res
            if method == "pm" and r < 1:
                # the next loop's residual is R^q: an order q with r^q < tol/2
                # makes the check after it settle
                for m in ("sm", "cm", "fm", "pm"):
                    if r ** ORDER[m] < tol / 2:
                        next_method = m
                        break
        X = Xn
    res.X = X
    res.returned_iter = res.iters
    return res


def coc(diff_inf_hist, ar: Arith = F64):
    """Computational order of convergence (COC), Section 8, from the last three
    infinity-norm changes e_k = ||X_k - X_{k-1}||_inf:
    rho = ln(e_{k+1}/e_k) / ln(e_k/e_{k-1})."""
    e0, e1, e2 = diff_inf_hist[-3:]
    return ar.log(e2 / e1) / ar.log(e1 / e0)


# ---------------------------------------------------------------------------
# Residuals of the defining equations.
# ---------------------------------------------------------------------------

def penrose_residuals(A, X):
    """Relative residuals of the four Penrose equations for X = A^dagger:
    ||AXA - A||/||A||, ||XAX - X||/||X||, ||AX - (AX)^T||/||AX||,
    ||XA - (XA)^T||/||XA|| (Frobenius norms)."""
    f = np.linalg.norm
    AX = A @ X
    XA = X @ A
    return (f(AX @ A - A) / f(A), f(XA @ X - X) / f(X),
            f(AX - adjoint(AX)) / f(AX), f(XA - adjoint(XA)) / f(XA))


def drazin_residuals(A, X, l: int):
    """Relative residuals of the Drazin equations A^{l+1} X = A^l, XAX = X,
    AX = XA (Frobenius norms)."""
    f = np.linalg.norm
    Al = np.linalg.matrix_power(A, l)
    AX = A @ X
    return (f(Al @ A @ X - Al) / f(Al), f(X @ A @ X - X) / f(X),
            f(AX - X @ A) / f(AX))
