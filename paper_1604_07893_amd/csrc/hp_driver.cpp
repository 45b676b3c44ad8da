// Host driver and C ABI of libhyperpower.
//
// One hp_solve call runs the loop of Section 2, iteration (PM), optionally
// switching to (PM-modified) of Section 7, on the caller's stream: every
// product is one k_gemm_f64 launch whose epilogue forms the next linear
// combination, and the two stopping sums come back to the host once per loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "hp_internal.h"
#include "hyperpower.h"

struct hp_handle {
    int device = 0;
    int forced_tile = -1;         // HP_GEMM_TILE: one tile configuration for every product
    double* host_scal = nullptr;  // pinned, hp::SLOT_COUNT doubles
    static constexpr int kEvents = 64;
    hipEvent_t ev[kEvents] = {};
};

namespace {

using hp::Epilogue;

// Constants of the factored polynomial: the closed forms printed in Section 2
// (c1, c2, c3 of (simplify1); d1, d2 of (simplify2); mu, psi of (hyper18-33)).
struct PMConst {
    double c1, c2, c3, d1, d2, mu, psi;
};

PMConst pm_const() {
    const double r93 = std::sqrt(93.0);
    const double q = std::sqrt(27.0 - 2.0 * r93);
    PMConst k;
    k.c1 = (q + 1.0) / 4.0;
    k.c2 = (1.0 - q) / 4.0;
    k.c3 = (5.0 * r93 - 93.0) / 496.0;
    k.d1 = (-93.0 - 5.0 * r93) / 496.0;
    k.d2 = -r93 / 4.0;
    k.mu = 3.0 / 8.0;
    k.psi = 321.0 / 1984.0;
    return k;
}

#define HIPCHK(x)                           \
    do {                                    \
        if ((x) != hipSuccess) return HP_EHIP; \
    } while (0)

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Leading dimension of the library's internal matrices: a multiple of 8
// doubles (64 bytes) so every row start is aligned for 16-byte loads, nudged
// off multiples of 1 KiB so that the rows of a tile do not all start on the
// same memory channel.
inline int64_t pad_ld(int64_t cols) {
    int64_t ld = round_up(cols, 8);
    if (ld % 128 == 0) ld += 8;
    return ld;
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout. FP64 set: A, three n x m iterates (X_k, X_{k+1}, X_{k+1/2})
// and seven s x s loop matrices. FP32 set (FP32 and mixed precision): the same
// in single precision. FP32-only solves keep just A and one iterate in FP64
// (X0 is formed there).
struct Plan {
    int64_t m = 0, n = 0;
    bool left = false;
    int64_t s = 0;          // side of the residual R (n for left, m for right)
    int64_t ldA = 0, ldX = 0, ldS = 0;  // FP64 leading dimensions (elements)
    int64_t ldA32 = 0, ldX32 = 0, ldS32 = 0;
    int nX64 = 0, nS64 = 0, nX32 = 0, nS32 = 0;
    bool has32 = false;
    size_t offA = 0, offX[3] = {}, offS[7] = {};
    size_t offA32 = 0, offX32[3] = {}, offS32[7] = {};
    size_t offSmall = 0, nSmall = 0, offScal = 0, total = 0;
};

bool choose_left(const hp_params* p, int64_t m, int64_t n) {
    if (p->side == HP_SIDE_LEFT) return true;
    if (p->side == HP_SIDE_RIGHT) return false;
    return m > n;
}

Plan make_plan(const hp_params* p, int64_t m, int64_t n) {
    Plan pl;
    pl.m = m;
    pl.n = n;
    pl.left = choose_left(p, m, n);
    pl.s = pl.left ? n : m;
    pl.ldA = pad_ld(n);
    pl.ldX = pad_ld(m);
    pl.ldS = pad_ld(pl.s);
    pl.ldA32 = pad_ld(n);
    pl.ldX32 = pad_ld(m);
    pl.ldS32 = pad_ld(pl.s);
    const bool fp32only = p->precision == HP_PREC_FP32;
    pl.has32 = p->precision != HP_PREC_FP64;
    pl.nX64 = fp32only ? 1 : 3;
    pl.nS64 = fp32only ? 0 : 7;
    pl.nX32 = pl.has32 ? 3 : 0;
    pl.nS32 = pl.has32 ? 7 : 0;
    // Drazin set-up forms A^l in two s x s buffers of the FP64 set
    if (fp32only && p->kind == HP_KIND_DRAZIN) pl.nS64 = 2;
    size_t off = 0;
    pl.offA = off;
    off = align_up(off + sizeof(double) * (size_t)(m * pl.ldA));
    for (int i = 0; i < pl.nX64; ++i) {
        pl.offX[i] = off;
        off = align_up(off + sizeof(double) * (size_t)(n * pl.ldX));
    }
    for (int i = 0; i < pl.nS64; ++i) {
        pl.offS[i] = off;
        off = align_up(off + sizeof(double) * (size_t)(pl.s * pl.ldS));
    }
    if (pl.has32) {
        pl.offA32 = off;
        off = align_up(off + sizeof(float) * (size_t)(m * pl.ldA32));
        for (int i = 0; i < pl.nX32; ++i) {
            pl.offX32[i] = off;
            off = align_up(off + sizeof(float) * (size_t)(n * pl.ldX32));
        }
        for (int i = 0; i < pl.nS32; ++i) {
            pl.offS32[i] = off;
            off = align_up(off + sizeof(float) * (size_t)(pl.s * pl.ldS32));
        }
    }
    // small area: GEMM partial pairs, norm sums, trace partials, row sums
    const int64_t big = std::max(m, n);
    const int64_t blocks = (int64_t)hp::gemm_max_blocks(big, big);
    int64_t small = 2 * blocks;
    small = std::max<int64_t>(small, ((m + 255) / 256 + 1) * n + m);
    small = std::max<int64_t>(small, ((n + 31) / 32) * ((n + 31) / 32));
    small = std::max<int64_t>(small, big);
    pl.offSmall = off;
    pl.nSmall = (size_t)small;
    off = align_up(off + sizeof(double) * (size_t)small);
    pl.offScal = off;
    off = align_up(off + sizeof(double) * hp::SLOT_COUNT);
    pl.total = off;
    return pl;
}

int validate(const hp_params* p, int64_t m, int64_t n) {
    if (!p) return HP_EINVAL;
    if (m < 1 || n < 1 || m > 65535 || n > 65535) return HP_EINVAL;
    if (p->kind != HP_KIND_MOORE_PENROSE && p->kind != HP_KIND_DRAZIN) return HP_EINVAL;
    if (p->kind == HP_KIND_DRAZIN) {
        if (m != n || p->drazin_l < 1 || p->drazin_l > 64) return HP_EINVAL;
        if (p->alpha_rule != HP_ALPHA_TRACE && p->alpha_rule != HP_ALPHA_USER) return HP_EINVAL;
    } else if (p->alpha_rule != HP_ALPHA_NORM1INF && p->alpha_rule != HP_ALPHA_USER) {
        return HP_EINVAL;
    }
    if (p->alpha_rule == HP_ALPHA_USER && !(p->alpha > 0.0 && std::isfinite(p->alpha))) return HP_EINVAL;
    if (p->variant < HP_VARIANT_PLAIN || p->variant > HP_VARIANT_STAB_ALWAYS) return HP_EINVAL;
    if (p->side < HP_SIDE_AUTO || p->side > HP_SIDE_LEFT) return HP_EINVAL;
    if (p->stop_rule < HP_STOP_REL_FRO || p->stop_rule > HP_STOP_ABS_INF) return HP_EINVAL;
    if (p->precision < HP_PREC_FP64 || p->precision > HP_PREC_MIXED) return HP_EINVAL;
    if (p->low_dtype != HP_LOWP_BF16 && p->low_dtype != HP_LOWP_F16) return HP_EINVAL;
    if (p->max_iter < 1 || p->max_iter > 100000) return HP_EINVAL;
    if (!(p->tol >= 0.0) || !(p->tau_switch > 0.0) || !(p->diverge_limit > 0.0)) return HP_EINVAL;
    for (int i = 0; i < 6; ++i)
        if (p->reserved[i] != 0) return HP_EINVAL;
    return HP_OK;
}

// Pairs of hipEvents around GEMM launches, harvested after each stream sync.
struct GemmTimer {
    hp_handle* h;
    bool on;
    int used = 0;
    double total_ms = 0.0;
    hipStream_t s;
    void before() {
        if (on && used + 2 <= hp_handle::kEvents) (void)hipEventRecord(h->ev[used], s);
    }
    void after() {
        if (on && used + 2 <= hp_handle::kEvents) {
            (void)hipEventRecord(h->ev[used + 1], s);
            used += 2;
        }
    }
    void harvest() {  // stream must be synchronised
        for (int i = 0; i < used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess) total_ms += ms;
        }
        used = 0;
    }
};

// Which MFMA path a product runs on.
enum Engine { ENG_F64, ENG_F32, ENG_BF16, ENG_F16 };

// The buffers of one precision.
template <typename T>
struct Set {
    T* A = nullptr;
    T* X[3] = {};
    T* S[7] = {};
    int64_t ldA = 0, ldX = 0, ldS = 0;
};

struct Solver {
    hp_handle* h;
    const hp_params* p;
    hipStream_t s;
    Plan pl;
    char* ws;
    hp_result* res;
    GemmTimer timer;
    double gflop = 0.0;
    int gemms = 0;
    int last_blocks = 0;  // blocks (partial pairs) of the latest product
    int stage = 2;        // 0 16-bit, 1 FP32, 2 FP64 (for per-stage accounting)

    template <typename T>
    T* ptr(size_t off) { return reinterpret_cast<T*>(ws + off); }

    template <typename T>
    int gemm(Engine eng, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
             int64_t ldb, const hp::EpilogueT<T>& ep) {
        const hp::GemmTile t = h->forced_tile >= 0 ? (hp::GemmTile)h->forced_tile
                                                   : hp::gemm_pick_tile(M, N, K);
        timer.before();
        hipError_t e;
        if constexpr (std::is_same<T, double>::value) {
            e = hp::gemm(t, M, N, K, A, lda, B, ldb, ep, s);
        } else {
            if (eng == ENG_F32) e = hp::gemm(t, M, N, K, A, lda, B, ldb, ep, s);
            else e = hp::gemm_lowp(t, eng == ENG_BF16 ? hp::LOWP_BF16 : hp::LOWP_F16, M, N, K, A,
                                   lda, B, ldb, ep, s);
        }
        timer.after();
        last_blocks = hp::gemm_blocks(t, M, N);
        if (e != hipSuccess) return HP_EHIP;
        const double g = 2.0 * (double)M * (double)N * (double)K * 1e-9;
        gflop += g;
        res->gflop_stage[stage] += g;
        ++gemms;
        return HP_OK;
    }
};

#define CHK(x)                      \
    do {                            \
        int rc_ = (x);              \
        if (rc_ != HP_OK) return rc_; \
    } while (0)

// One loop of (PM), Section 2, in the association printed there, on buffers
// of one precision: R, R^2, R^4 (epilogue: F1, F2), F1 F2 (epilogue: T, S),
// T S (+ mu R^2 + psi R^4), R V (+ V), and the update; if `stab`, the
// stabilising product X A X of (PM-modified), Section 7, follows. The update
// (or the stabilising product) writes the partial sums of the stopping test
// against X_k into `partials`.
template <typename T>
int pm_loop(Solver& S, Engine eng, const Set<T>& b, T* Xk, T* Xn, T* Xh, bool stab,
            double* partials) {
    const PMConst K = pm_const();
    const int64_t m = S.pl.m, n = S.pl.n, sd = S.pl.s;
    const int64_t ldS = b.ldS, ldX = b.ldX, ldA = b.ldA;
    T* R = b.S[0];
    T* R2 = b.S[1];
    T* R4 = b.S[2];
    T* F1 = b.S[3];
    T* F2 = b.S[4];
    T* Tm = b.S[5];
    T* Sm = b.S[6];
    T* V = F1;  // F1, F2 are dead once T and S exist
    T* W = F2;
    {   // R = I - A X (right, m x m) or I - X A (left, n x n)
        hp::EpilogueT<T> e = hp::epilogue_plain(R, ldS, -1.0, 1.0);
        if (S.pl.left) CHK(S.gemm<T>(eng, n, n, m, Xk, ldX, b.A, ldA, e));
        else CHK(S.gemm<T>(eng, m, m, n, b.A, ldA, Xk, ldX, e));
    }
    CHK(S.gemm<T>(eng, sd, sd, sd, R, ldS, R, ldS, hp::epilogue_plain(R2, ldS)));
    {   // R4 = R2 R2; F1 = I + c1 R2 + R4; F2 = I + c2 R2 + R4
        hp::EpilogueT<T> e{};
        e.out[0] = R4; e.ldo[0] = ldS; e.acc_c[0] = 1.0;
        e.out[1] = F1; e.ldo[1] = ldS; e.acc_c[1] = 1.0; e.id[1] = 1.0; e.g1[1] = K.c1;
        e.out[2] = F2; e.ldo[2] = ldS; e.acc_c[2] = 1.0; e.id[2] = 1.0; e.g1[2] = K.c2;
        e.D1 = R2; e.ld1 = ldS;
        CHK(S.gemm<T>(eng, sd, sd, sd, R2, ldS, R2, ldS, e));
    }
    {   // M = F1 F2; T = M + c3 R2; S = M + d1 R2 + d2 R4
        hp::EpilogueT<T> e{};
        e.out[0] = Tm; e.ldo[0] = ldS; e.acc_c[0] = 1.0; e.g1[0] = K.c3;
        e.out[1] = Sm; e.ldo[1] = ldS; e.acc_c[1] = 1.0; e.g1[1] = K.d1; e.g2[1] = K.d2;
        e.D1 = R2; e.ld1 = ldS; e.D2 = R4; e.ld2 = ldS;
        CHK(S.gemm<T>(eng, sd, sd, sd, F1, ldS, F2, ldS, e));
    }
    {   // V = T S + mu R2 + psi R4
        hp::EpilogueT<T> e{};
        e.out[0] = V; e.ldo[0] = ldS; e.acc_c[0] = 1.0; e.g1[0] = K.mu; e.g2[0] = K.psi;
        e.D1 = R2; e.ld1 = ldS; e.D2 = R4; e.ld2 = ldS;
        CHK(S.gemm<T>(eng, sd, sd, sd, Tm, ldS, Sm, ldS, e));
    }
    {   // W = (I + R) V = V + R V
        hp::EpilogueT<T> e{};
        e.out[0] = W; e.ldo[0] = ldS; e.acc_c[0] = 1.0; e.g1[0] = 1.0;
        e.D1 = V; e.ld1 = ldS;
        CHK(S.gemm<T>(eng, sd, sd, sd, R, ldS, V, ldS, e));
    }
    {   // update: X W (right) or W X (left)
        hp::EpilogueT<T> e = hp::epilogue_plain(stab ? Xh : Xn, ldX);
        if (!stab) {
            e.ref = Xk; e.ldref = ldX; e.partials = partials;
        }
        if (S.pl.left) CHK(S.gemm<T>(eng, n, m, n, W, ldS, Xk, ldX, e));
        else CHK(S.gemm<T>(eng, n, m, m, Xk, ldX, W, ldS, e));
    }
    if (stab) {
        // X_{k+1} = X_{k+1/2} A X_{k+1/2}, associated so that the middle
        // product is the smaller square
        hp::EpilogueT<T> e = hp::epilogue_plain(Xn, ldX);
        e.ref = Xk; e.ldref = ldX; e.partials = partials;
        if (m >= n) {
            CHK(S.gemm<T>(eng, n, n, m, Xh, ldX, b.A, ldA, hp::epilogue_plain(R, ldS)));
            CHK(S.gemm<T>(eng, n, m, n, R, ldS, Xh, ldX, e));
        } else {
            CHK(S.gemm<T>(eng, m, m, n, b.A, ldA, Xh, ldX, hp::epilogue_plain(R, ldS)));
            CHK(S.gemm<T>(eng, n, m, m, Xh, ldX, R, ldS, e));
        }
    }
    return HP_OK;
}

constexpr double kUnitRoundoff[3] = {0.0, 5.960464477539063e-08, 1.1102230246251565e-16};

int run_solve(Solver& S, const double* A, int64_t lda, const double* X0, int64_t ldx0, double* X,
              int64_t ldx) {
    const hp_params* p = S.p;
    const Plan& pl = S.pl;
    hipStream_t s = S.s;
    hp_result* res = S.res;
    const int64_t m = pl.m, n = pl.n;

    Set<double> b64;
    b64.A = S.ptr<double>(pl.offA);
    for (int i = 0; i < pl.nX64; ++i) b64.X[i] = S.ptr<double>(pl.offX[i]);
    for (int i = 0; i < pl.nS64; ++i) b64.S[i] = S.ptr<double>(pl.offS[i]);
    b64.ldA = pl.ldA; b64.ldX = pl.ldX; b64.ldS = pl.ldS;
    Set<float> b32;
    if (pl.has32) {
        b32.A = S.ptr<float>(pl.offA32);
        for (int i = 0; i < pl.nX32; ++i) b32.X[i] = S.ptr<float>(pl.offX32[i]);
        for (int i = 0; i < pl.nS32; ++i) b32.S[i] = S.ptr<float>(pl.offS32[i]);
        b32.ldA = pl.ldA32; b32.ldX = pl.ldX32; b32.ldS = pl.ldS32;
    }
    double* small = S.ptr<double>(pl.offSmall);
    double* scal = S.ptr<double>(pl.offScal);
    double* hs = S.h->host_scal;
    const int64_t ldA = pl.ldA, ldX = pl.ldX, ldS = pl.ldS;

    // A -> padded internal copy
    HIPCHK(hipMemcpy2DAsync(b64.A, ldA * sizeof(double), A, lda * sizeof(double),
                            n * sizeof(double), m, hipMemcpyDeviceToDevice, s));

    // ---- X0 (Section 4), formed in FP64 ----
    double* X0w = b64.X[0];
    double alpha = 0.0;
    S.stage = 2;
    if (X0) {
        HIPCHK(hipMemcpy2DAsync(X0w, ldX * sizeof(double), X0, ldx0 * sizeof(double),
                                m * sizeof(double), n, hipMemcpyDeviceToDevice, s));
        alpha = p->alpha > 0.0 ? p->alpha : 1.0;
    } else {
        if (p->alpha_rule == HP_ALPHA_USER) {
            hs[hp::SLOT_ALPHA] = p->alpha;
            HIPCHK(hipMemcpyAsync(scal + hp::SLOT_ALPHA, hs + hp::SLOT_ALPHA, sizeof(double),
                                  hipMemcpyHostToDevice, s));
        }
        if (p->kind == HP_KIND_MOORE_PENROSE) {
            if (p->alpha_rule == HP_ALPHA_NORM1INF)
                HIPCHK(hp::alpha_norm1inf(b64.A, ldA, m, n, small, scal, s));
            HIPCHK(hp::transpose_scale(b64.A, ldA, m, n, X0w, ldX, scal + hp::SLOT_ALPHA, s));
        } else {
            // G = A^l by repeated products, alpha = 1/Tr(A^{l+1}) = 1/Tr(A^l A)
            const double* P = b64.A;
            int64_t ldp = ldA;
            double* pp[2] = {b64.S[0], b64.S[1]};
            for (int i = 1; i < p->drazin_l; ++i) {
                double* dst = pp[i & 1];
                CHK(S.gemm<double>(ENG_F64, n, n, n, P, ldp, b64.A, ldA,
                                   hp::epilogue_plain(dst, ldS)));
                P = dst;
                ldp = ldS;
            }
            if (p->alpha_rule == HP_ALPHA_TRACE)
                HIPCHK(hp::alpha_trace(P, ldp, b64.A, ldA, n, small, scal, s));
            HIPCHK(hp::scale(P, ldp, n, n, X0w, ldX, scal + hp::SLOT_ALPHA, s));
        }
        HIPCHK(hipMemcpyAsync(hs, scal, sizeof(double) * hp::SLOT_COUNT, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        S.timer.harvest();
        alpha = hs[hp::SLOT_ALPHA];
    }
    res->alpha = alpha;

    // ---- stages ----
    int stage = p->precision == HP_PREC_MIXED ? 0 : (p->precision == HP_PREC_FP32 ? 1 : 2);
    const int final_stage = p->precision == HP_PREC_FP32 ? 1 : 2;
    const Engine low_eng = p->low_dtype == HP_LOWP_F16 ? ENG_F16 : ENG_BF16;
    // current iterate indices into the X sets
    int ik = 0, in_ = 1;
    if (stage < 2) {
        HIPCHK(hp::convert(b64.A, ldA, m, n, b32.A, b32.ldA, s));
        HIPCHK(hp::convert(X0w, ldX, n, m, b32.X[0], b32.ldX, s));
    }

    const bool want_inf = (p->flags & HP_FLAG_INF_NORM) || p->stop_rule == HP_STOP_ABS_INF;
    bool stabilising = p->variant == HP_VARIANT_STAB_ALWAYS;
    res->switch_iter = stabilising ? 0 : -1;
    bool converging = false;
    bool stage_first = true;  // no stagnation test on a stage's first loop
    double d_prev = 0.0;
    int status = HP_MAXITER;
    int result_idx = -1;      // index into the final set's X buffers

    for (int k = 0; k < p->max_iter; ++k) {
        S.stage = stage;
        if (stage == 2) {
            CHK(pm_loop<double>(S, ENG_F64, b64, b64.X[ik], b64.X[in_], b64.X[2], stabilising, small));
        } else {
            CHK(pm_loop<float>(S, stage == 0 ? low_eng : ENG_F32, b32, b32.X[ik], b32.X[in_],
                               b32.X[2], stabilising, small));
        }
        HIPCHK(hp::reduce_pairs(small, S.last_blocks, scal, s));
        if (want_inf && stage == 2)
            HIPCHK(hp::diff_norm_inf(b64.X[in_], ldX, b64.X[ik], ldX, n, m, small, scal, s));
        HIPCHK(hipMemcpyAsync(hs, scal, sizeof(double) * hp::SLOT_COUNT, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        S.timer.harvest();

        res->iters = k + 1;
        res->iters_stage[stage] += 1;
        const double diff2 = hs[hp::SLOT_DIFF2], ref2 = hs[hp::SLOT_REF2];
        const double d = std::sqrt(diff2) / std::sqrt(ref2);
        if (k < HP_HIST) res->d_hist[k] = d;
        res->d_stage[stage] = d;
        double dinf = 0.0;
        if (want_inf && stage == 2) {
            dinf = hs[hp::SLOT_DINF];
            if (k < HP_HIST) res->dinf_hist[k] = dinf;
        }
        res->d_last = d;
        const bool finite = std::isfinite(d) && std::isfinite(diff2) && (!want_inf || std::isfinite(dinf));

        if (stage != final_stage) {
            // a lower stage ends when its change stops halving, reaches its
            // rounding floor, or goes non-finite (16-bit overflow); the next
            // stage continues from the better of the last two iterates
            const double u = stage == 0 ? (p->low_dtype == HP_LOWP_F16 ? 4.8828125e-4 : 3.90625e-3)
                                        : kUnitRoundoff[1];
            const bool stalled = !stage_first && d < 1.0 && d >= 0.5 * d_prev;
            const bool floor = d < 10.0 * u || d < p->tol;
            if (d < p->tau_switch) {
                converging = true;
                if (p->variant == HP_VARIANT_STABILISED && !stabilising) {
                    stabilising = true;
                    res->switch_iter = k + 1;
                }
            }
            if (!finite || stalled || floor) {
                const bool keep_new = finite && !(stalled && d >= d_prev);
                const int from = keep_new ? in_ : ik;
                const int next = stage + 1;
                if (next == 2) {
                    HIPCHK(hp::convert(b32.X[from], b32.ldX, n, m, b64.X[0], ldX, s));
                    ik = 0;
                    in_ = 1;
                } else {
                    ik = from;
                    in_ = from == 0 ? 1 : 0;
                }
                stage = next;
                stage_first = true;
                d_prev = d;
                continue;
            }
            stage_first = false;
            d_prev = d;
            std::swap(ik, in_);
            continue;
        }

        if (!finite) {
            status = HP_NONFINITE;
            result_idx = ik;
            break;
        }
        double sval;
        bool passed;
        if (p->stop_rule == HP_STOP_REL_FRO) {
            sval = d;
            passed = d < p->tol;
        } else if (p->stop_rule == HP_STOP_ABS_INF) {
            sval = dinf;
            passed = dinf <= p->tol;
        } else {
            sval = std::sqrt(diff2) / (std::pow(18.0, (double)k) * alpha);
            passed = sval < p->tol;
        }
        res->stop_last = sval;
        if (passed) {
            status = HP_OK;
            result_idx = in_;
            break;
        }
        if (converging && !stage_first && d >= d_prev) {
            status = HP_STAGNATED;
            result_idx = ik;
            break;
        }
        if (!converging && d > p->diverge_limit) {
            status = HP_DIVERGED;
            result_idx = ik;
            break;
        }
        if (d < p->tau_switch) {
            converging = true;
            if (p->variant == HP_VARIANT_STABILISED && !stabilising) {
                stabilising = true;
                res->switch_iter = k + 1;
            }
        }
        stage_first = false;
        d_prev = d;
        std::swap(ik, in_);
    }
    if (result_idx < 0) result_idx = ik;  // HP_MAXITER: the last iterate

    const int it = std::min(res->iters, HP_HIST);
    if (want_inf && it >= 3) {
        const double e0 = res->dinf_hist[it - 3], e1 = res->dinf_hist[it - 2], e2 = res->dinf_hist[it - 1];
        if (e0 > 0 && e1 > 0 && e2 > 0) res->coc = std::log(e2 / e1) / std::log(e1 / e0);
    }
    if (stage == 2) {
        HIPCHK(hipMemcpy2DAsync(X, ldx * sizeof(double), b64.X[result_idx], ldX * sizeof(double),
                                m * sizeof(double), n, hipMemcpyDeviceToDevice, s));
    } else {
        HIPCHK(hp::convert(b32.X[result_idx], b32.ldX, n, m, X, ldx, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return status;
}

const char* const kStatusText[] = {"ok", "max_iter reached", "stagnated", "diverged",
                                   "non-finite value", "pending"};
const char* const kErrorText[] = {"", "invalid argument", "workspace too small", "over HBM budget",
                                  "HIP runtime error", "unsupported"};

}  // namespace

extern "C" {

int hp_version(void) { return HP_ABI_VERSION; }

const char* hp_status_string(int status) {
    if (status >= 0 && status <= HP_PENDING) return kStatusText[status];
    if (status < 0 && status >= HP_EUNSUPPORTED) return kErrorText[-status];
    return "unknown status";
}

void hp_params_default(hp_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->kind = HP_KIND_MOORE_PENROSE;
    p->drazin_l = 0;
    p->alpha_rule = HP_ALPHA_NORM1INF;
    p->variant = HP_VARIANT_PLAIN;
    p->alpha = 0.0;
    p->tau_switch = 0.1;
    p->tol = 1e-12;
    p->diverge_limit = 1e6;
    p->max_iter = 100;
    p->stop_rule = HP_STOP_REL_FRO;
    p->side = HP_SIDE_AUTO;
    p->precision = HP_PREC_FP64;
    p->flags = 0;
}

int hp_create(hp_handle** out, int device) {
    if (!out) return HP_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return HP_EHIP;
    if (device < 0 || device >= count) return HP_EINVAL;
    HIPCHK(hipSetDevice(device));
    hp_handle* h = new hp_handle();
    h->device = device;
    if (const char* t = std::getenv("HP_GEMM_TILE")) {
        const int v = std::atoi(t);
        if (v >= 0 && v < hp::TILE_COUNT) h->forced_tile = v;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&h->host_scal), sizeof(double) * hp::SLOT_COUNT,
                      hipHostMallocDefault) != hipSuccess) {
        delete h;
        return HP_EHIP;
    }
    for (int i = 0; i < hp_handle::kEvents; ++i) {
        if (hipEventCreate(&h->ev[i]) != hipSuccess) {
            hp_destroy(h);
            return HP_EHIP;
        }
    }
    *out = h;
    return HP_OK;
}

int hp_destroy(hp_handle* h) {
    if (!h) return HP_EINVAL;
    (void)hipSetDevice(h->device);
    for (int i = 0; i < hp_handle::kEvents; ++i)
        if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
    if (h->host_scal) (void)hipHostFree(h->host_scal);
    delete h;
    return HP_OK;
}

int hp_workspace_bytes(const hp_params* p, int64_t m, int64_t n, size_t* bytes) {
    if (!bytes) return HP_EINVAL;
    int rc = validate(p, m, n);
    if (rc != HP_OK) return rc;
    *bytes = make_plan(p, m, n).total;
    return HP_OK;
}

int hp_solve(hp_handle* h, const hp_params* p, const double* A, int64_t m, int64_t n, int64_t lda,
             const double* X0, int64_t ldx0, double* X, int64_t ldx, void* workspace,
             size_t ws_bytes, void* stream, hp_result* out) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!h || !A || !X) return HP_EINVAL;
    int rc = validate(p, m, n);
    if (rc != HP_OK) return rc;
    if (lda < n || ldx < m || (X0 && ldx0 < m)) return HP_EINVAL;
    const Plan pl = make_plan(p, m, n);
    if (!workspace || ws_bytes < pl.total) return HP_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return HP_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;

    hp_result local{};
    hp_result* res = out ? out : &local;
    std::memset(res, 0, sizeof(*res));
    res->switch_iter = -1;
    res->side_used = pl.left ? HP_SIDE_LEFT : HP_SIDE_RIGHT;

    Solver S{h, p, reinterpret_cast<hipStream_t>(stream), pl, static_cast<char*>(workspace), res,
             GemmTimer{h, (p->flags & HP_FLAG_TIME_KERNELS) != 0, 0, 0.0,
                       reinterpret_cast<hipStream_t>(stream)}};
    rc = run_solve(S, A, lda, X0, ldx0, X, ldx);
    res->status = rc;
    res->gflop = S.gflop;
    res->gemms = S.gemms;
    res->gemm_ms = S.timer.total_ms;
    res->time_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int hp_gemm(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K, double alpha, const void* A,
            int64_t lda, const void* B, int64_t ldb, double beta_identity, void* C, int64_t ldc,
            void* stream) {
    if (!h || !A || !B || !C) return HP_EINVAL;
    if (dtype < HP_DTYPE_F64 || dtype > HP_DTYPE_F16_F32) return HP_EINVAL;
    if (M < 1 || N < 1 || K < 1 || M > (1 << 24) || N > (1 << 24) || K > (1 << 24)) return HP_EINVAL;
    if (lda < K || ldb < N || ldc < N) return HP_EINVAL;
    const int64_t vec = dtype == HP_DTYPE_F64 ? 2 : 4;  // elements per 16 bytes
    if (lda % vec || ldb % vec) return HP_EINVAL;
    if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
         reinterpret_cast<uintptr_t>(C)) & 15)
        return HP_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
    const hp::GemmTile t =
        h->forced_tile >= 0 ? (hp::GemmTile)h->forced_tile : hp::gemm_pick_tile(M, N, K);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (dtype == HP_DTYPE_F64) {
        e = hp::gemm(t, M, N, K, static_cast<const double*>(A), lda, static_cast<const double*>(B),
                     ldb, hp::epilogue_plain(static_cast<double*>(C), ldc, alpha, beta_identity), s);
    } else if (dtype == HP_DTYPE_F32) {
        e = hp::gemm(t, M, N, K, static_cast<const float*>(A), lda, static_cast<const float*>(B),
                     ldb, hp::epilogue_plain(static_cast<float*>(C), ldc, alpha, beta_identity), s);
    } else {
        e = hp::gemm_lowp(t, dtype == HP_DTYPE_BF16_F32 ? hp::LOWP_BF16 : hp::LOWP_F16, M, N, K,
                          static_cast<const float*>(A), lda, static_cast<const float*>(B), ldb,
                          hp::epilogue_plain(static_cast<float*>(C), ldc, alpha, beta_identity), s);
    }
    if (e != hipSuccess) return HP_EHIP;
    return HP_OK;
}

}  // extern "C"
