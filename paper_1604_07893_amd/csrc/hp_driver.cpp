// Host driver and C ABI of libhyperpower: single solves.
//
// One hp_solve call runs the loop of Section 2, iteration (PM), optionally
// switching to (PM-modified) of Section 7, on the caller's stream: every
// product is one MFMA GEMM launch whose epilogue forms the next linear
// combination, and the two stopping sums come back to the host once per loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "hp_host.h"

namespace hp {

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

static inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Leading dimension of the library's internal matrices: a multiple of 8
// elements so every row start is aligned for 16-byte loads, nudged off
// multiples of 128 elements so that the rows of a tile do not all start on
// the same memory channel.
int64_t pad_ld(int64_t cols) {
    int64_t ld = round_up(cols, 8);
    if (ld % 128 == 0) ld += 8;
    return ld;
}

static bool choose_left(const hp_params* p, int64_t m, int64_t n) {
    if (p->side == HP_SIDE_LEFT) return true;
    if (p->side == HP_SIDE_RIGHT) return false;
    return m > n;
}

Plan make_plan(const hp_params* p, int64_t m, int64_t n, bool single) {
    const bool split_area = single;
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
    pl.nX64 = fp32only ? 1 : (single ? 4 : 3);
    pl.nS64 = fp32only ? 0 : 7;
    pl.nX32 = pl.has32 ? (single && fp32only ? 4 : 3) : 0;
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
    pl.has_proj = pl.has32 && p->kind == HP_KIND_MOORE_PENROSE &&
                  (p->precision == HP_PREC_MIXED || p->precision == HP_PREC_FP32_FP64);
    pl.delta = p->precision == HP_PREC_DELTA32 ||
               ((p->precision == HP_PREC_MIXED || p->precision == HP_PREC_FP32_FP64) &&
                !(p->flags & HP_FLAG_FP64_POLY));
    if (pl.has_proj) {
        pl.offAt = off;
        off = align_up(off + sizeof(double) * (size_t)(n * pl.ldX));
        pl.offXt = off;
        off = align_up(off + sizeof(double) * (size_t)(m * pl.ldA));
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
    pl.has16 = p->precision == HP_PREC_MIXED;
    if (pl.has16) {
        constexpr size_t h = 2;  // bytes per 16-bit element
        pl.ldA16 = pad_ld(n);
        pl.ldAt16 = pad_ld(m);
        pl.ldX16 = pad_ld(m);
        pl.ldXt16 = pad_ld(n);
        pl.ldS16 = pad_ld(pl.s);
        pl.offA16 = off;
        off = align_up(off + h * (size_t)(m * pl.ldA16));
        pl.offAt16 = off;
        off = align_up(off + h * (size_t)(n * pl.ldAt16));
        for (int i = 0; i < 3; ++i) {
            pl.offX16[i] = off;
            off = align_up(off + h * (size_t)(n * pl.ldX16));
            pl.offXt16[i] = off;
            off = align_up(off + h * (size_t)(m * pl.ldXt16));
        }
        for (int i = 0; i < 7; ++i) {
            pl.offS16[i] = off;
            off = align_up(off + h * (size_t)(pl.s * pl.ldS16));
            pl.offSt16[i] = off;
            off = align_up(off + h * (size_t)(pl.s * pl.ldS16));
        }
    }
    if (split_area) {
        // every product of a solve is (m or n) x (m or n) x (m or n)
        const int64_t dims[2] = {m, n};
        const hp::GemmType types[2] = {hp::GT_F64, hp::GT_F32};
        for (hp::GemmType gt : types)
            for (int64_t M : dims)
                for (int64_t N : dims)
                    for (int64_t K : dims)
                        pl.splitSlots = std::max(
                            pl.splitSlots,
                            hp::gemm_split_slots(hp::gemm_pick_tile(M, N, K, gt), M, N, K));
        pl.splitCnt = pl.splitSlots;
        // the symmetric launches of the loop's s x s products (K = s, or m or
        // n for the residual and the stabilising middle product); FP64 solves
        // only (LoopState::sym_ok)
        pl.sym = p->kind == HP_KIND_MOORE_PENROSE && p->alpha_rule != HP_ALPHA_DIAG &&
                 !(p->chop > 0.0) && p->precision == HP_PREC_FP64 &&
                 (p->flags & HP_FLAG_SYMMETRIC);
        if (pl.sym) {
            for (int64_t K : dims) {
                int64_t slots = 0, cnt = 0;
                hp::gemm_sym_scratch(hp::gemm_pick_tile(pl.s, pl.s, K, hp::GT_F64), hp::GT_F64,
                                     pl.s, &slots, &cnt);
                pl.splitSlots = std::max(pl.splitSlots, slots);
                pl.splitCnt = std::max(pl.splitCnt, cnt);
            }
        }
        if (pl.splitSlots > 0) {
            pl.splitCnt = std::max(pl.splitCnt, pl.splitSlots);
            pl.offSplit = off;
            off = align_up(off + sizeof(double) * 128 * 128 * (size_t)pl.splitSlots);
            pl.offSplitCnt = off;
            off = align_up(off + sizeof(unsigned) * (size_t)pl.splitCnt);
        }
    }
    // small area: GEMM partial pairs, norm sums, trace partials, row sums
    const int64_t big = std::max(m, n);
    const int64_t blocks = (int64_t)hp::gemm_max_blocks(big, big);
    int64_t small = 2 * blocks;
    small = std::max<int64_t>(small, ((m + hp::kColChunk - 1) / hp::kColChunk + 2) * n + m);
    small = std::max<int64_t>(small, ((n + 31) / 32) * ((n + 31) / 32));
    small = std::max<int64_t>(small, big);
    pl.offSmall = off;
    pl.nSmall = (size_t)small;
    off = align_up(off + sizeof(double) * (size_t)small);
    pl.offScal = off;
    off = align_up(off + sizeof(double) * hp::SLOT_COUNT);
    pl.offDev = off;  // DevLoop and StepParams (hp_params.device_stop)
    off = align_up(off + sizeof(hp::DevLoop));
    pl.offStep = off;
    off = align_up(off + sizeof(hp::StepParams));
    pl.total = off;
    return pl;
}

int validate(const hp_params* p, int64_t m, int64_t n) {
    if (!p) return HP_EINVAL;
    if (m < 1 || n < 1 || m > 65535 || n > 65535) return HP_EINVAL;
    if (p->kind != HP_KIND_MOORE_PENROSE && p->kind != HP_KIND_DRAZIN) return HP_EINVAL;
    if (p->kind == HP_KIND_DRAZIN) {
        if (m != n || p->drazin_l < 1 || p->drazin_l > 64) return HP_EINVAL;
        // lower-precision stages are not stable on the nilpotent part
        if (p->precision != HP_PREC_FP64) return HP_EUNSUPPORTED;
        if (p->alpha_rule != HP_ALPHA_TRACE && p->alpha_rule != HP_ALPHA_USER) return HP_EINVAL;
    } else if (p->alpha_rule != HP_ALPHA_NORM1INF && p->alpha_rule != HP_ALPHA_USER &&
               p->alpha_rule != HP_ALPHA_SIGMA_MAX2 && p->alpha_rule != HP_ALPHA_DIAG) {
        return HP_EINVAL;
    }
    if (p->alpha_rule == HP_ALPHA_DIAG && m != n) return HP_EINVAL;
    if (!(p->chop >= 0.0) || !std::isfinite(p->chop)) return HP_EINVAL;
    if (p->chop > 0.0 && ((p->precision != HP_PREC_FP64 && p->precision != HP_PREC_FP32) ||
                          p->stop_rule == HP_STOP_REL_FRO_BOUND))
        return HP_EUNSUPPORTED;
    if (p->alpha_rule == HP_ALPHA_USER && !(p->alpha > 0.0 && std::isfinite(p->alpha))) return HP_EINVAL;
    if (p->variant < HP_VARIANT_PLAIN || p->variant > HP_VARIANT_STAB_ALWAYS) return HP_EINVAL;
    if (p->side < HP_SIDE_AUTO || p->side > HP_SIDE_LEFT) return HP_EINVAL;
    if (p->stop_rule < HP_STOP_REL_FRO || p->stop_rule > HP_STOP_REL_FRO_BOUND) return HP_EINVAL;
    if (p->precision < HP_PREC_FP64 || p->precision > HP_PREC_DELTA32) return HP_EINVAL;
    if (p->low_dtype != HP_LOWP_BF16 && p->low_dtype != HP_LOWP_F16) return HP_EINVAL;
    if (p->method < HP_METHOD_PM || p->method > HP_METHOD_HM) return HP_EINVAL;
    // the comparison methods run without precision stages (the stage exits
    // are tuned to the contraction of an order-18 loop)
    if (p->method != HP_METHOD_PM && p->precision != HP_PREC_FP64 && p->precision != HP_PREC_FP32)
        return HP_EUNSUPPORTED;
    if (p->max_iter < 1 || p->max_iter > 100000) return HP_EINVAL;
    if (!(p->tol >= 0.0) || !(p->tau_switch > 0.0) || !(p->diverge_limit > 0.0)) return HP_EINVAL;
    if (p->reserved[0] != 0 || p->reserved[1] != 0) return HP_EINVAL;
    if (p->device_stop != 0 && p->device_stop != 1) return HP_EINVAL;
    // the device-side decision covers FP64 loops with the plain stopping rules
    if (p->device_stop && (p->precision != HP_PREC_FP64 || p->stop_rule == HP_STOP_REL_FRO_BOUND ||
                           (p->flags & HP_FLAG_SYMMETRIC) || p->chop > 0.0))
        return HP_EUNSUPPORTED;
    return HP_OK;
}

Buffers carve(const Plan& pl, char* ws) {
    Buffers bf;
    auto d = [&](size_t off) { return reinterpret_cast<double*>(ws + off); };
    auto f = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
    bf.b64.A = d(pl.offA);
    for (int i = 0; i < pl.nX64; ++i) bf.b64.X[i] = d(pl.offX[i]);
    for (int i = 0; i < pl.nS64; ++i) bf.b64.S[i] = d(pl.offS[i]);
    bf.b64.ldA = pl.ldA;
    bf.b64.ldX = pl.ldX;
    bf.b64.ldS = pl.ldS;
    if (pl.has32) {
        bf.b32.A = f(pl.offA32);
        for (int i = 0; i < pl.nX32; ++i) bf.b32.X[i] = f(pl.offX32[i]);
        for (int i = 0; i < pl.nS32; ++i) bf.b32.S[i] = f(pl.offS32[i]);
        bf.b32.ldA = pl.ldA32;
        bf.b32.ldX = pl.ldX32;
        bf.b32.ldS = pl.ldS32;
    }
    if (pl.has16) {
        bf.A16 = {ws + pl.offA16, pl.ldA16, ws + pl.offAt16, pl.ldAt16};
        for (int i = 0; i < 3; ++i)
            bf.X16[i] = {ws + pl.offX16[i], pl.ldX16, ws + pl.offXt16[i], pl.ldXt16};
        for (int i = 0; i < 7; ++i)
            bf.S16[i] = {ws + pl.offS16[i], pl.ldS16, ws + pl.offSt16[i], pl.ldS16};
    }
    if (pl.has_proj) {
        bf.At = d(pl.offAt);
        bf.Xt = d(pl.offXt);
    }
    bf.small = d(pl.offSmall);
    bf.scal = d(pl.offScal);
    bf.dev = reinterpret_cast<DevLoop*>(ws + pl.offDev);
    bf.step = reinterpret_cast<StepParams*>(ws + pl.offStep);
    if (pl.splitSlots > 0) {
        bf.split_part = d(pl.offSplit);
        bf.split_cnt = reinterpret_cast<unsigned*>(ws + pl.offSplitCnt);
    }
    return bf;
}

}  // namespace hp

namespace {

using namespace hp;

// Pairs of hipEvents around GEMM launches, harvested after each stream sync.
struct GemmTimer {
    hp_handle* h;
    bool on;
    int used = 0;
    double total_ms = 0.0;
    hipStream_t s;
    double sym_ms = 0.0;  // the part of total_ms spent in symmetric launches
    double eng_ms[3] = {};  // ... by MFMA path: 16-bit, FP32, FP64
    bool is_sym[hp_handle::kEvents / 2] = {};
    int eng[hp_handle::kEvents / 2] = {};
    void before() {
        if (on && used + 2 <= hp_handle::kEvents) (void)hipEventRecord(h->ev[used], s);
    }
    void after(bool sym, int engine_idx) {
        if (on && used + 2 <= hp_handle::kEvents) {
            (void)hipEventRecord(h->ev[used + 1], s);
            is_sym[used / 2] = sym;
            eng[used / 2] = engine_idx;
            used += 2;
        }
    }
    void harvest() {  // stream must be synchronised
        for (int i = 0; i < used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess) {
                total_ms += ms;
                if (is_sym[i / 2]) sym_ms += ms;
                eng_ms[eng[i / 2]] += ms;
            }
        }
        used = 0;
    }
};

struct Solver {
    hp_handle* h;
    const hp_params* p;
    hipStream_t s;
    Plan pl;
    hp_result* res;
    GemmTimer timer;
    double gflop = 0.0;
    int gemms = 0;
    int last_blocks = 0;  // blocks (partial pairs) of the latest product
    int stage = 2;        // for per-stage accounting
    double gflop_sym = 0.0;
    int gemms_sym = 0;
    bool sym = false;  // the loop's products may run symmetric (Plan::sym, no user X0)
    bool sym_loop = false;  // ... and this loop may (LoopState::sym_ok)
    double* split_part = nullptr;  // split-K scratch of the workspace (Plan)
    unsigned* split_cnt = nullptr;
    const Buffers* bf = nullptr;   // for the 16-bit copies of the first mixed stage
    bool may_allocate = true;      // false under hp_solve_noalloc

    template <typename T>
    int gemm(Engine eng, const GemmCall<T>& g, const CopyUse* use = nullptr) {
        // every operand and the first output must exist in this plan
        if (!g.A || !g.B || !g.ep.out[0]) return HP_EINVAL;
        int dt = HP_DTYPE_F64;
        if constexpr (!std::is_same<T, double>::value)
            dt = eng == ENG_F32 ? HP_DTYPE_F32 : (eng == ENG_BF16 ? HP_DTYPE_BF16_F32 : HP_DTYPE_F16_F32);
        EpilogueT<T> ep = g.ep;
        if (split_part) {
            ep.split_part = reinterpret_cast<T*>(split_part);
            ep.split_cnt = split_cnt;
            ep.split_slots = pl.splitSlots * (int64_t)(sizeof(double) / sizeof(T));
            ep.split_ncnt = pl.splitCnt;
        }
        if (!(sym && sym_loop)) ep.sym = 0;
        const GemmTile t = choose_tile(h, dt, g.M, g.N, g.K, ep.split_slots);
        const bool sym_launch = eng == ENG_F64 || eng == ENG_F32
                                    ? gemm_sym_launches(t, g.M, g.N, g.K, g.A, g.lda, g.B, g.ldb, ep)
                                    : false;
        timer.before();
        hipError_t e;
        if constexpr (std::is_same<T, double>::value) {
            (void)eng;
            e = hp::gemm(t, g.M, g.N, g.K, g.A, g.lda, g.B, g.ldb, ep, s);
        } else {
            const Copy16* ca = (eng != ENG_F32 && bf) ? bf->copy16(g.A) : nullptr;
            const Copy16* cb = (eng != ENG_F32 && bf) ? bf->copy16(g.B) : nullptr;
            if (eng == ENG_F32) {
                e = hp::gemm(t, g.M, g.N, g.K, g.A, g.lda, g.B, g.ldb, ep, s);
            } else if (ca && cb) {
                // operands from their 16-bit copies (A row-major, B transposed);
                // the outputs leave their own copies for the next products
                const int dt16 = eng == ENG_BF16 ? HP_DTYPE_BF16 : HP_DTYPE_F16;
                const GemmTile t16 = choose_tile(h, dt16, g.M, g.N, g.K);
                for (int o = 0; o < 3; ++o) {
                    const Copy16* co = ep.out[o] ? bf->copy16(ep.out[o]) : nullptr;
                    if (!co) continue;
                    if (!use || use->row[o]) {
                        ep.h[o] = co->h;
                        ep.ldh[o] = co->ld;
                    }
                    if (!use || use->t[o]) {
                        ep.ht[o] = co->ht;
                        ep.ldht[o] = co->ldt;
                    }
                    if (use && !use->f32[o]) ep.skip32[o] = 1;
                }
                e = gemm_h16(t16, eng == ENG_BF16 ? LOWP_BF16 : LOWP_F16, g.M, g.N, g.K, ca->h,
                             ca->ld, cb->ht, cb->ldt, ep, s);
                last_blocks = gemm_blocks(t16, g.M, g.N);
                timer.after(false, 0);
                if (e != hipSuccess) return HP_EHIP;
                const double gf = 2.0 * (double)g.M * (double)g.N * (double)g.K * 1e-9;
                gflop += gf;
                res->gflop_stage[stage] += gf;
                res->gflop_engine[0] += gf;
                ++gemms;
                return HP_OK;
            } else {
                e = gemm_lowp(t, eng == ENG_BF16 ? LOWP_BF16 : LOWP_F16, g.M, g.N, g.K, g.A, g.lda,
                              g.B, g.ldb, ep, s);
            }
        }
        const int ei = eng == ENG_F64 ? 2 : eng == ENG_F32 ? 1 : 0;
        timer.after(sym_launch, ei);
        last_blocks = gemm_blocks(t, g.M, g.N);
        if (e != hipSuccess) return HP_EHIP;
        // a symmetric launch forms N (N + 1) / 2 distinct elements
        const double gf = (sym_launch ? (double)g.N + 1.0 : 2.0 * (double)g.N) * (double)g.M *
                          (double)g.K * 1e-9;
        gflop += gf;
        res->gflop_stage[stage] += gf;
        res->gflop_engine[ei] += gf;
        ++gemms;
        if (sym_launch) {
            gflop_sym += gf;
            ++gemms_sym;
        }
        return HP_OK;
    }
};

// hp_params.chop: the product that writes X_{k+1} (the update, or the
// stabilising product after it) drops its entries below `chop`.
template <typename T>
void set_chop(GemmCall<T>* calls, int nc, const T* Xn, double chop) {
    if (chop <= 0.0) return;
    for (int i = 0; i < nc; ++i)
        if (calls[i].ep.out[0] == Xn) calls[i].ep.chop = chop;
}

// hp_params.device_stop: the loops of an FP64 solve enqueued in chunks, each
// loop's decision taken on the device by loop_step (LoopState::step's rules),
// every kernel of the loop gated on it. A loop is enqueued in both forms --
// the plain update (writing X_{k+1} with the stopping sums) and the
// stabilised one (update into X_{k+1/2}, then X_{k+1/2} A X_{k+1/2} with the
// sums) -- and the flag the previous decision left selects which runs, so the
// iterates and decisions are those of run_solve, bitwise.
}  // namespace

namespace hp {

// Spins for at most max_us microseconds until *flag (pinned host memory that
// a kernel writes) equals `want`. Returns false when the time is up (the
// caller then waits for the stream).
bool poll_host(const double* flag, double want, double max_us) {
    const double kPollUs = max_us;
    const auto t0 = std::chrono::steady_clock::now();
    const volatile double* f = flag;
    for (int i = 0;; ++i) {
        if (*f == want) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return true;
        }
        if ((i & 63) == 63 &&
            std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
                    .count() > kPollUs)
            return false;
    }
}

}  // namespace hp

namespace {

int run_solve_device(Solver& S, char* ws, const double* A, int64_t lda, const double* X0,
                     int64_t ldx0, double* X, int64_t ldx) {
    const hp_params* p = S.p;
    const Plan& pl = S.pl;
    hipStream_t s = S.s;
    hp_result* res = S.res;
    const int64_t m = pl.m, n = pl.n;
    const Buffers bf = carve(pl, ws);
    double* hs = S.h->host_scal;
    if (bf.split_cnt) {
        HIPCHK(zero_u32(bf.split_cnt, pl.splitCnt, s));
        S.split_part = bf.split_part;
        S.split_cnt = bf.split_cnt;
    }
    S.sym = false;
    S.bf = &bf;
    S.stage = 2;
    double alpha = 0.0;
    {
        Range setup_range("set-up X0");
        CHK(setup_x0(p, pl, bf, A, lda, X0, ldx0, hs, s,
                     [&](const GemmCall<double>& g) { return S.gemm<double>(ENG_F64, g); }, &alpha));
    }
    S.timer.harvest();
    res->alpha = alpha;
    const double gf_setup = S.gflop;
    const int ng_setup = S.gemms;

    DevLoop* L = bf.dev;
    const int* gate = reinterpret_cast<const int*>(L);
    HIPCHK(loop_init(L, p->variant == HP_VARIANT_STAB_ALWAYS ? 1 : 0, s));
    const bool want_inf = (p->flags & HP_FLAG_INF_NORM) || p->stop_rule == HP_STOP_ABS_INF;
    // the decision's parameters, staged through pinned memory (the stream
    // reads them before the host touches that area again)
    StepParams& P = *reinterpret_cast<StepParams*>(hs + SLOT_COUNT);
    static_assert(sizeof(StepParams) <= sizeof(double) * hp_handle::kHostExtra, "staging");
    P = StepParams{};
    P.stop_rule = p->stop_rule;
    P.variant = p->variant;
    P.max_iter = p->max_iter;
    P.have_dinf = want_inf ? 1 : 0;
    P.keep_best = 1;
    P.tol = p->tol;
    P.tau = p->tau_switch;
    P.diverge = p->diverge_limit;
    P.alpha = alpha;
    P.order = (double)method_order(p->method);
    HIPCHK(hipMemcpyAsync(bf.step, &P, sizeof(StepParams), hipMemcpyHostToDevice, s));

    // executed work of one loop in each form (the accounting after the solve)
    double gf_plain = 0.0, gf_stab = 0.0;
    int ng_plain = 0, ng_stab = 0;
    auto flops = [](const GemmCall<double>& c) {
        return 2.0 * (double)c.M * (double)c.N * (double)c.K * 1e-9;
    };
    auto gated = [&](GemmCall<double> c, int mode) {
        c.ep.gate = gate;
        c.ep.gate_mode = mode;
        return S.gemm<double>(ENG_F64, c);
    };
    int calls_per_loop = 0;
    auto enqueue = [&](int j) -> int {
        const hipStream_t s = S.s;  // the solve stream, or the capture stream
        Range loop_range("loop %d (device decision)", j + 1);
        double* Xk = bf.b64.X[j & 1];
        double* Xn = bf.b64.X[(j + 1) & 1];
        GemmCall<double> cp[kMaxLoopGemms], cs[kMaxLoopGemms];
        const int np = describe_loop<double>(p->method, pl, bf.b64, Xk, Xn, bf.b64.X[2], false,
                                             bf.small, cp);
        const int ns = describe_loop<double>(p->method, pl, bf.b64, Xk, Xn, bf.b64.X[2], true,
                                             bf.small, cs);
        const int common = np - 1;  // the products before the update
        for (int i = 0; i < common; ++i) CHK(gated(cp[i], GATE_LIVE));
        // a variant that never switches enqueues only the form it runs
        int nb_plain = 0, nb_stab = 0;
        if (p->variant != HP_VARIANT_STAB_ALWAYS) {
            CHK(gated(cp[common], GATE_PLAIN));
            nb_plain = S.last_blocks;
        }
        if (p->variant != HP_VARIANT_PLAIN) {
            for (int i = common; i < ns; ++i) CHK(gated(cs[i], GATE_STAB));
            nb_stab = S.last_blocks;
        }
        HIPCHK(reduce_pairs_gated(bf.small, nb_plain, nb_stab, bf.scal, L, s));
        if (want_inf)
            HIPCHK(diff_norm_inf_gated(Xn, bf.b64.ldX, Xk, bf.b64.ldX, n, m, bf.small, bf.scal, L,
                                       s));
        HIPCHK(loop_step(bf.scal, L, bf.step, s));
        // the decision may ask to keep this loop's input as the best iterate
        HIPCHK(copy_gated(Xk, bf.b64.ldX, bf.b64.X[LoopState::kBest], bf.b64.ldX, n, m, L,
                          GATE_SAVE, s));
        return HP_OK;
    };
    {
        // the products of one loop in each form (host-side descriptions only)
        GemmCall<double> cp[kMaxLoopGemms], cs[kMaxLoopGemms];
        const int np = describe_loop<double>(p->method, pl, bf.b64, bf.b64.X[0], bf.b64.X[1],
                                             bf.b64.X[2], false, bf.small, cp);
        const int ns = describe_loop<double>(p->method, pl, bf.b64, bf.b64.X[0], bf.b64.X[1],
                                             bf.b64.X[2], true, bf.small, cs);
        const int common = np - 1;
        for (int i = 0; i < np; ++i) gf_plain += flops(cp[i]);
        for (int i = 0; i < common; ++i) gf_stab += flops(cp[i]);
        for (int i = common; i < ns; ++i) gf_stab += flops(cs[i]);
        ng_plain = np;
        ng_stab = ns;
        calls_per_loop = common + (p->variant != HP_VARIANT_STAB_ALWAYS ? 1 : 0) +
                         (p->variant != HP_VARIANT_PLAIN ? ns - common : 0);
    }

    // Two loops (input X[0], then X[1]) captured once (on the handle's
    // capture stream) as a graph per (workspace, shape, loop form) and
    // replayed on the solve stream; without allocation (or with per-kernel
    // timing, or HP_FLAG_NO_GRAPH) the loops are launched one by one instead.
    hp_handle* h = S.h;
    hipGraphExec_t exec = nullptr;
    const bool use_graph = S.may_allocate && !S.timer.on && !(p->flags & HP_FLAG_NO_GRAPH);
    if (use_graph) {
        const std::array<int64_t, 10> key = {
            (int64_t)reinterpret_cast<uintptr_t>(ws), m, n, pl.left ? 1 : 0, p->method,
            p->variant, want_inf ? 1 : 0, h->tune_gen, h->forced_tile, (int64_t)pl.total};
        for (auto& g : h->graphs)
            if (g.key == key) {
                g.used = ++h->graph_clock;
                exec = g.exec;
            }
        if (!exec) {
            if (!h->cap_stream)
                HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
            Range cap_range("capture two loops");
            HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            S.s = h->cap_stream;
            int rc = enqueue(0);
            if (rc == HP_OK) rc = enqueue(1);
            S.s = s;
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
            if (rc != HP_OK || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc != HP_OK ? rc : HP_EHIP;
            }
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return HP_EHIP;
            }
            if ((int)h->graphs.size() >= hp_handle::kGraphs) {
                auto lru = std::min_element(h->graphs.begin(), h->graphs.end(),
                                            [](const auto& a, const auto& b) { return a.used < b.used; });
                HIPCHK(hipStreamSynchronize(h->cap_stream));
                (void)hipGraphExecDestroy(lru->exec);
                (void)hipGraphDestroy(lru->graph);
                h->graphs.erase(lru);
            }
            h->graphs.push_back({key, graph, exec, ++h->graph_clock});
        }
    }
    // Chunks of loops between host reads of the decision state: 4 loops
    // first; then one loop when the last change d, in the converging regime,
    // has d^p < tol (the next loop is expected to pass the test), else two.
    // A chunk starting at an even loop takes whole replays of the graph (on
    // the solve stream); an odd remainder is launched loop by loop. Loops past
    // max_iter find the solve done and return at once. (The event pairs of
    // HP_FLAG_TIME_KERNELS bound a chunk too.)
    const double order = (double)method_order(p->method);
    int j = 0, chunk = std::min(p->max_iter, 4);
    for (;;) {
        int c = 0;
        while (c < chunk && j < p->max_iter) {
            if (exec && (j & 1) == 0 && chunk - c >= 2) {
                HIPCHK(hipGraphLaunch(exec, s));
                j += 2;
                c += 2;
            } else {
                CHK(enqueue(j));
                ++j;
                ++c;
            }
        }
        double* direct = S.h->host_loop_dev;
        const double seq = (double)++S.h->loop_seq;
        if (direct)
            CHK(loop_report(L, direct, seq, s));
        else
            HIPCHK(hipMemcpyAsync(hs, L, offsetof(DevLoop, d_hist), hipMemcpyDeviceToHost, s));
        if (!direct || S.timer.on ||
            !poll_host(S.h->host_loop + kLoopReportDoubles, seq, 1000.0))
            HIPCHK(hipStreamSynchronize(s));
        if (direct) std::memcpy(hs, S.h->host_loop, offsetof(DevLoop, d_hist));
        S.timer.harvest();
        const DevLoop& hl = *reinterpret_cast<const DevLoop*>(hs);
        if (hl.done || j >= p->max_iter) break;
        chunk = hl.converging && std::pow(hl.d_last, order) < p->tol ? 1 : 2;
        if (S.timer.on && calls_per_loop > 0)
            chunk = std::max(1, std::min(chunk, (hp_handle::kEvents / 2) / calls_per_loop));
    }
    DevLoop st{};
    HIPCHK(hipMemcpyAsync(&st, L, sizeof(DevLoop), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int k = st.k;
    res->iters = k;
    res->iters_stage[2] = k;
    res->switch_iter = st.switch_iter;
    res->d_last = st.d_last;
    res->d_stage[2] = st.d_last;
    res->stop_last = st.stop_last;
    const int it = std::min(k, HP_HIST);
    for (int i = 0; i < it; ++i) {
        res->d_hist[i] = st.d_hist[i];
        if (want_inf) res->dinf_hist[i] = st.dinf_hist[i];
    }
    if (want_inf && it >= 3) {
        const double e0 = res->dinf_hist[it - 3], e1 = res->dinf_hist[it - 2], e2 = res->dinf_hist[it - 1];
        if (e0 > 0 && e1 > 0 && e2 > 0) res->coc = std::log(e2 / e1) / std::log(e1 / e0);
    }
    // work of the loops that ran (the gated-off launches did none)
    const int n_stab = st.switch_iter >= 0 ? std::max(0, k - st.switch_iter) : 0;
    const int n_plain = k - n_stab;
    S.gflop = gf_setup + n_plain * gf_plain + n_stab * gf_stab;
    S.gemms = ng_setup + n_plain * ng_plain + n_stab * ng_stab;
    res->gflop_stage[2] = S.gflop;
    res->gflop_engine[2] = S.gflop;
    const int ri = st.result_idx >= 0 ? st.result_idx : (k & 1);
    HIPCHK(hipMemcpy2DAsync(X, ldx * sizeof(double), bf.b64.X[ri], bf.b64.ldX * sizeof(double),
                            m * sizeof(double), n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return st.done ? st.status : HP_MAXITER;
}

int run_solve(Solver& S, char* ws, const double* A, int64_t lda, const double* X0, int64_t ldx0,
              double* X, int64_t ldx) {
    const hp_params* p = S.p;
    const Plan& pl = S.pl;
    hipStream_t s = S.s;
    hp_result* res = S.res;
    const int64_t m = pl.m, n = pl.n;
    const Buffers bf = carve(pl, ws);
    double* hs = S.h->host_scal;
    if (bf.split_cnt) {
        HIPCHK(zero_u32(bf.split_cnt, pl.splitCnt, s));
        S.split_part = bf.split_part;
        S.split_cnt = bf.split_cnt;
    }
    // X_k = p(A^T A) A^T needs X0 = alpha A^T (not a caller's X0)
    S.sym = pl.sym && X0 == nullptr;
    S.bf = &bf;

    double alpha = 0.0;
    S.stage = 2;
    {
        Range setup_range("set-up X0");
        CHK(setup_x0(p, pl, bf, A, lda, X0, ldx0, hs, s,
                     [&](const GemmCall<double>& g) { return S.gemm<double>(ENG_F64, g); }, &alpha));
    }
    S.timer.harvest();
    res->alpha = alpha;

    LoopState st;
    st.init(p, res, alpha);
    st.keep_best = true;
    if (st.stage < 2) {
        HIPCHK(convert(bf.b64.A, bf.b64.ldA, m, n, bf.b32.A, bf.b32.ldA, s));
        HIPCHK(convert(bf.b64.X[0], bf.b64.ldX, n, m, bf.b32.X[0], bf.b32.ldX, s));
    }
    if (st.stage == 0 && pl.has16) {
        // the 16-bit stage's operands: A and X0 rounded, row-major and transposed
        const LowPrec lp = p->low_dtype == HP_LOWP_F16 ? LOWP_F16 : LOWP_BF16;
        HIPCHK(convert_h16(bf.b32.A, bf.b32.ldA, m, n, lp, bf.A16.h, bf.A16.ld, bf.A16.ht,
                           bf.A16.ldt, s));
        HIPCHK(convert_h16(bf.b32.X[0], bf.b32.ldX, n, m, lp, bf.X16[0].h, bf.X16[0].ld,
                           bf.X16[0].ht, bf.X16[0].ldt, s));
    }
    const bool want_inf = (p->flags & HP_FLAG_INF_NORM) || p->stop_rule == HP_STOP_ABS_INF;

    // The loop's products from `first` on (the residual product, call 0, may
    // already have run for the residual bound).
    // `scheme`: a plain final-stage loop after a residual check (first == 1) may run
    // a lower-order scheme (LoopState::scheme_for)
    // The delta form (describe_delta_poly): R and the update in FP64, the
    // polynomial's products in FP32. HP_PREC_DELTA32 runs every loop so;
    // staged precisions run an FP64-stage loop so when the latest residual
    // norm it knows (r_last) is below kDeltaR, i.e. R is going to 0: then
    // the FP32 rounding of W - I is relative to ||R|| and costs no accuracy.
    // With a null space on the residual's side R tends to a projector
    // (||R||_F >= 1) and every product stays FP64.
    constexpr double kDeltaR = 0.5;
    const bool delta_all = p->precision == HP_PREC_DELTA32;
    const bool track_r = pl.delta && !delta_all;  // ||R||_F of each FP64-stage loop
    double r_last = INFINITY;
    auto delta_now = [&]() { return pl.delta && (delta_all || r_last < kDeltaR); };
    auto run_delta = [&](int first, int scheme) -> int {
        S.sym_loop = false;
        const int64_t sd = pl.s;
        double* Xk = bf.b64.X[st.ik];
        if (first == 0) {
            GemmCall<double> c0[1];
            describe_residual<double>(pl, bf.b64, Xk,
                                      epilogue_plain(bf.b64.S[0], bf.b64.ldS, -1.0, 1.0), c0, 0);
            CHK(S.gemm<double>(ENG_F64, c0[0]));
            if (track_r)
                HIPCHK(diffsq(bf.b64.S[0], bf.b64.ldS, nullptr, 0, 0.0, sd, sd, bf.small, bf.scal,
                              SLOT_RNORM2, s));
        }
        const double* W64 = bf.b64.S[0];  // SM: W - I = R
        if (scheme != HP_METHOD_SM) {
            HIPCHK(convert(bf.b64.S[0], bf.b64.ldS, sd, sd, bf.b32.S[0], bf.b32.ldS, s));
            GemmCall<float> calls[kMaxLoopGemms];
            float* Wd = nullptr;
            const int nc = describe_delta_poly<float>(scheme, pl, bf.b32, calls, &Wd);
            for (int i = 0; i < nc; ++i) CHK(S.gemm<float>(ENG_F32, calls[i]));
            HIPCHK(convert(Wd, bf.b32.ldS, sd, sd, bf.b64.S[1], bf.b64.ldS, s));
            W64 = bf.b64.S[1];
        }
        GemmCall<double> u[3];
        const int nu = describe_update<double>(pl, bf.b64, W64, Xk, bf.b64.X[st.in_], bf.b64.X[2],
                                               st.stabilising, bf.small, bf.b64.S[2], u, 0, true);
        for (int i = 0; i < nu; ++i) CHK(S.gemm<double>(ENG_F64, u[i]));
        ++res->iters_delta;
        return HP_OK;
    };
    auto run_loop = [&](int first, int scheme) -> int {
        if (st.stage == 2 && delta_now()) return run_delta(first, scheme);
        S.sym_loop = st.sym_ok();
        if (st.stage == 2) {
            GemmCall<double> calls[kMaxLoopGemms];
            const int nc =
                scheme != p->method && first == 1 && !st.stabilising
                    ? describe_after_residual<double>(scheme, pl, bf.b64, bf.b64.X[st.ik],
                                                      bf.b64.X[st.in_], bf.small, calls)
                    : describe_loop<double>(p->method, pl, bf.b64, bf.b64.X[st.ik],
                                            bf.b64.X[st.in_], bf.b64.X[2], st.stabilising,
                                            bf.small, calls);
            set_chop(calls, nc, bf.b64.X[st.in_], p->chop);
            for (int i = first; i < nc; ++i) {
                CHK(S.gemm<double>(ENG_F64, calls[i]));
                if (i == 0 && track_r)  // the residual's norm decides the next loop's form
                    HIPCHK(diffsq(bf.b64.S[0], bf.b64.ldS, nullptr, 0, 0.0, pl.s, pl.s, bf.small,
                                  bf.scal, SLOT_RNORM2, s));
            }
        } else {
            GemmCall<float> calls[kMaxLoopGemms];
            const int nc =
                scheme != p->method && first == 1 && !st.stabilising
                    ? describe_after_residual<float>(scheme, pl, bf.b32, bf.b32.X[st.ik],
                                                     bf.b32.X[st.in_], bf.small, calls)
                    : describe_loop<float>(p->method, pl, bf.b32, bf.b32.X[st.ik],
                                           bf.b32.X[st.in_], bf.b32.X[2], st.stabilising,
                                           bf.small, calls);
            set_chop(calls, nc, bf.b32.X[st.in_], p->chop);
            CopyUse use[kMaxLoopGemms];
            copy_uses(calls, nc, bf.b32, use);
            for (int i = first; i < nc; ++i)
                CHK(S.gemm<float>(st.engine(), calls[i], st.stage == 0 ? &use[i] : nullptr));
        }
        return HP_OK;
    };
    // Form the next loop's residual R (its first product, into S[0]) and
    // return ||R||_F in *r.
    auto next_residual = [&](double* r) -> int {
        const int64_t sd = pl.s;
        S.sym_loop = false;  // the bound reads the full residual
        if (st.stage == 2) {
            GemmCall<double> calls[kMaxLoopGemms];
            describe_loop<double>(p->method, pl, bf.b64, bf.b64.X[st.ik], bf.b64.X[st.in_],
                                  bf.b64.X[2], false, bf.small, calls);
            CHK(S.gemm<double>(ENG_F64, calls[0]));
            HIPCHK(diffsq(bf.b64.S[0], bf.b64.ldS, nullptr, 0, 0.0, sd, sd, bf.small, bf.scal,
                          SLOT_RNORM2, s));
        } else {
            GemmCall<float> calls[kMaxLoopGemms];
            describe_loop<float>(p->method, pl, bf.b32, bf.b32.X[st.ik], bf.b32.X[st.in_],
                                 bf.b32.X[2], false, bf.small, calls);
            CHK(S.gemm<float>(st.engine(), calls[0]));
            HIPCHK(sumsq(bf.b32.S[0], bf.b32.ldS, sd, sd, bf.small, bf.scal, SLOT_RNORM2, s));
        }
        HIPCHK(hipMemcpyAsync(hs, bf.scal, sizeof(double) * SLOT_COUNT, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        S.timer.harvest();
        *r = std::sqrt(hs[SLOT_RNORM2]);
        return HP_OK;
    };
    // HP_STOP_REL_FRO_BOUND: R as above; true if ||R||_F/(1-||R||_F) < tol,
    // else the scheme for the loop that reuses R.
    int scheme = p->method;
    auto residual_bound = [&](bool* settled) -> int {
        *settled = false;
        double r = 0.0;
        CHK(next_residual(&r));
        if (track_r) r_last = r;
        if (std::isfinite(r) && r < 1.0 && r / (1.0 - r) < p->tol) {
            st.stop_bound(r / (1.0 - r));
            *settled = true;
        } else if (std::isfinite(r)) {
            scheme = st.scheme_for(r);
        }
        return HP_OK;
    };
    bool r_ready = false;

    while (st.k < p->max_iter) {
        Range loop_range("loop %d stage %d%s", st.k + 1, st.stage,
                         st.stabilising ? " stabilised" : "");
        S.stage = st.stage;
        const bool r_ready_prev = r_ready;
        CHK(run_loop(r_ready ? 1 : 0, scheme));
        r_ready = false;
        scheme = p->method;
        // the inf-norm change in the precision the stage holds its iterates in
        // (rule HP_STOP_ABS_INF reads it in whichever stage is final)
        const bool inf_now = want_inf;
        // without it, the reduction itself hands the scalars to the host
        double* direct = inf_now ? nullptr : S.h->host_sums_dev;
        const double seq = (double)++S.h->sums_seq;
        HIPCHK(reduce_pairs(bf.small, S.last_blocks, bf.scal, s, direct, seq));
        if (inf_now && st.stage == 2)
            HIPCHK(diff_norm_inf(bf.b64.X[st.in_], bf.b64.ldX, bf.b64.X[st.ik], bf.b64.ldX, n, m,
                                 bf.small, bf.scal, s));
        else if (inf_now)
            HIPCHK(diff_norm_inf(bf.b32.X[st.in_], bf.b32.ldX, bf.b32.X[st.ik], bf.b32.ldX, n, m,
                                 bf.small, bf.scal, s));
        if (!direct)
            HIPCHK(hipMemcpyAsync(hs, bf.scal, sizeof(double) * SLOT_COUNT, hipMemcpyDeviceToHost, s));
        // a short loop's sums arrive within microseconds: poll for them rather
        // than sleep in the stream wait (kernel timing needs the wait)
        if (!direct || S.timer.on || !poll_host(S.h->host_sums + SLOT_COUNT, seq, 300.0))
            HIPCHK(hipStreamSynchronize(s));
        if (direct) std::memcpy(hs, S.h->host_sums, sizeof(double) * SLOT_COUNT);
        S.timer.harvest();

        // (a loop that reused the bound check's R keeps the r_last of that check)
        if (track_r && st.stage == 2 && !r_ready_prev) r_last = std::sqrt(hs[SLOT_RNORM2]);
        LoopState::Action a = st.step(hs[SLOT_DIFF2], hs[SLOT_REF2], hs[SLOT_DINF], inf_now);
        if (st.save_best) {
            // keep the input of this loop: the best iterate so far (the next
            // loop overwrites its buffer)
            const int b = LoopState::kBest;
            if (st.stage == 2)
                HIPCHK(hipMemcpy2DAsync(bf.b64.X[b], bf.b64.ldX * sizeof(double),
                                        bf.b64.X[st.save_from], bf.b64.ldX * sizeof(double),
                                        m * sizeof(double), n, hipMemcpyDeviceToDevice, s));
            else
                HIPCHK(hipMemcpy2DAsync(bf.b32.X[b], bf.b32.ldX * sizeof(float),
                                        bf.b32.X[st.save_from], bf.b32.ldX * sizeof(float),
                                        m * sizeof(float), n, hipMemcpyDeviceToDevice, s));
        }
        if (a == LoopState::DONE) break;
        if (a == LoopState::CONTINUE && st.k < p->max_iter && st.probe) {
            double r = 0.0;
            CHK(next_residual(&r));
            if (st.probe_exit(r)) a = LoopState::NEXT_STAGE;
            else r_ready = true;
        }
        auto project = [&](int xi) {
            Range proj_range("projection");
            S.stage = 2;
            return project_mp(pl, bf, xi, s, [&](const GemmCall<double>& g) {
                return S.gemm<double>(ENG_F64, g);
            });
        };
        if (a == LoopState::CONTINUE && st.projection_due() && pl.has_proj) {
            CHK(project(st.ik));  // deferred from the stage change (below)
            st.projected();
        } else if (a == LoopState::CONTINUE && st.k < p->max_iter && st.bound_ready()) {
            bool settled = false;
            CHK(residual_bound(&settled));
            if (settled) break;
            r_ready = true;
        }
        if (a == LoopState::NEXT_STAGE) {
            const int next = st.stage + 1;
            if (next == 2) {
                HIPCHK(convert(bf.b32.X[st.from_idx], bf.b32.ldX, n, m, bf.b64.X[0], bf.b64.ldX, s));
                if (track_r) {
                    // the lower stage's last residual (of the iterate's
                    // predecessor, or of the iterate itself after a probe)
                    // decides the form of the first FP64 loop
                    HIPCHK(sumsq(bf.b32.S[0], bf.b32.ldS, pl.s, pl.s, bf.small, bf.scal,
                                 SLOT_RNORM2, s));
                    HIPCHK(hipMemcpyAsync(hs + SLOT_RNORM2, bf.scal + SLOT_RNORM2, sizeof(double),
                                          hipMemcpyDeviceToHost, s));
                    HIPCHK(hipStreamSynchronize(s));
                    r_last = std::sqrt(hs[SLOT_RNORM2]);
                }
                bool proj = false;
                CHK(needs_projection(pl, bf, hs, s, &proj));
                // the projection assumes an iterate in the converging regime;
                // after an earlier exit it waits for the FP64 loops to get there
                if (proj && st.exit_converged) CHK(project(0));
                else if (proj) st.proj_pending = true;
            }
            st.enter_stage(next);
            // entering the final stage from a converged lower one: its first
            // loop gets the residual check too (and with it its scheme)
            if (st.k < p->max_iter && st.bound_ready() && !st.proj_pending) {
                bool settled = false;
                CHK(residual_bound(&settled));
                if (settled) break;
                r_ready = true;
            }
        }
    }
    st.finish_maxiter();

    const int it = std::min(res->iters, HP_HIST);
    if (want_inf && it >= 3) {
        const double e0 = res->dinf_hist[it - 3], e1 = res->dinf_hist[it - 2], e2 = res->dinf_hist[it - 1];
        if (e0 > 0 && e1 > 0 && e2 > 0) res->coc = std::log(e2 / e1) / std::log(e1 / e0);
    }
    if (st.stage == 2) {
        HIPCHK(hipMemcpy2DAsync(X, ldx * sizeof(double), bf.b64.X[st.result_idx],
                                bf.b64.ldX * sizeof(double), m * sizeof(double), n,
                                hipMemcpyDeviceToDevice, s));
    } else {
        HIPCHK(convert(bf.b32.X[st.result_idx], bf.b32.ldX, n, m, X, ldx, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return st.status;
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
    if (hipHostMalloc(reinterpret_cast<void**>(&h->host_scal),
                      sizeof(double) * (hp::SLOT_COUNT + hp_handle::kHostExtra),
                      hipHostMallocDefault) != hipSuccess) {
        delete h;
        return HP_EHIP;
    }
    // (without it the loop falls back to a copy of the device scalars)
    if (hipHostMalloc(reinterpret_cast<void**>(&h->host_sums), sizeof(double) * (hp::SLOT_COUNT + 1),
                      hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess &&
        hipHostGetDevicePointer(reinterpret_cast<void**>(&h->host_sums_dev), h->host_sums, 0) !=
            hipSuccess)
        h->host_sums_dev = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&h->host_loop),
                      sizeof(double) * (hp::kLoopReportDoubles + 1),
                      hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess &&
        hipHostGetDevicePointer(reinterpret_cast<void**>(&h->host_loop_dev), h->host_loop, 0) !=
            hipSuccess)
        h->host_loop_dev = nullptr;
    for (int i = 0; i < hp_handle::kEvents; ++i) {
        if (hipEventCreate(&h->ev[i]) != hipSuccess) {
            hp_destroy(h);
            return HP_EHIP;
        }
    }
    // the fixed workspace of hp_solve_noalloc on this device (if this fails,
    // that entry point tries again on its first call and reports HP_EHIP)
    (void)hp::noalloc_init(device);
    *out = h;
    return HP_OK;
}

int hp_destroy(hp_handle* h) {
    if (!h) return HP_EINVAL;
    (void)hipSetDevice(h->device);
    if (h->cap_stream) (void)hipStreamSynchronize(h->cap_stream);
    for (auto& g : h->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    h->graphs.clear();
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (int i = 0; i < hp_handle::kEvents; ++i)
        if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
    if (h->host_scal) (void)hipHostFree(h->host_scal);
    if (h->host_sums) (void)hipHostFree(h->host_sums);
    if (h->host_loop) (void)hipHostFree(h->host_loop);
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
    return hp::solve_entry(h, p, A, m, n, lda, X0, ldx0, X, ldx, workspace, ws_bytes, stream, out,
                           true);
}

}  // extern "C"

int hp::solve_entry(hp_handle* h, const hp_params* p, const double* A, int64_t m, int64_t n,
                    int64_t lda, const double* X0, int64_t ldx0, double* X, int64_t ldx,
                    void* workspace, size_t ws_bytes, void* stream, hp_result* out,
                    bool may_allocate) {
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

    Range range("hp_solve %lldx%lld", (long long)m, (long long)n);
    Solver S{h, p, reinterpret_cast<hipStream_t>(stream), pl, res,
             GemmTimer{h, (p->flags & HP_FLAG_TIME_KERNELS) != 0, 0, 0.0,
                       reinterpret_cast<hipStream_t>(stream)}};
    S.may_allocate = may_allocate;
    rc = p->device_stop ? run_solve_device(S, static_cast<char*>(workspace), A, lda, X0, ldx0, X, ldx)
                        : run_solve(S, static_cast<char*>(workspace), A, lda, X0, ldx0, X, ldx);
    res->status = rc;
    res->gflop = S.gflop;
    res->gemms = S.gemms;
    res->gemm_ms = S.timer.total_ms;
    res->gemms_sym = S.gemms_sym;
    res->gflop_sym = S.gflop_sym;
    res->gemm_ms_sym = S.timer.sym_ms;
    for (int i = 0; i < 3; ++i) res->gemm_ms_engine[i] = S.timer.eng_ms[i];
    res->time_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

extern "C" {

// Split-K workspace of hp_gemm_ws: `slots` partial tiles of 128 x 128
// elements of the dtype's storage type, then `slots` counters.
static int64_t gemm_ws_slots(const hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K) {
    const hp::GemmTile t = h ? hp::choose_tile(h, dtype, M, N, K, INT64_MAX)
                             : hp::gemm_pick_tile(M, N, K, hp::gemm_type(dtype));
    return hp::gemm_split_slots(t, M, N, K);
}
static size_t gemm_ws_bytes(int dtype, int64_t slots) {
    if (slots <= 0) return 0;
    const size_t esz = dtype == HP_DTYPE_F64 ? 8 : 4;
    return hp::align_up(esz * 128 * 128 * (size_t)slots) + sizeof(unsigned) * (size_t)slots;
}

static int gemm_args(int dtype, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                     const void* B, int64_t ldb, const void* C, int64_t ldc) {
    if (!A || !B || !C) return HP_EINVAL;
    if (dtype < HP_DTYPE_F64 || dtype > HP_DTYPE_F16) return HP_EINVAL;
    if (M < 1 || N < 1 || K < 1 || M > (1 << 24) || N > (1 << 24) || K > (1 << 24)) return HP_EINVAL;
    const bool h16 = dtype == HP_DTYPE_BF16 || dtype == HP_DTYPE_F16;  // B given as B^T
    if (lda < K || ldb < (h16 ? K : N) || ldc < N) return HP_EINVAL;
    const int64_t vec = dtype == HP_DTYPE_F64 ? 2 : h16 ? 8 : 4;  // elements per 16 bytes
    if (lda % vec || ldb % vec) return HP_EINVAL;
    if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
         reinterpret_cast<uintptr_t>(C)) & 15)
        return HP_EINVAL;
    return HP_OK;
}

static int gemm_run(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K, double alpha,
                    const void* A, int64_t lda, const void* B, int64_t ldb, double beta_identity,
                    void* C, int64_t ldc, void* workspace, int64_t slots, void* stream) {
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
    const hp::GemmTile t = hp::choose_tile(h, dtype, M, N, K, workspace ? slots : 0);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned* cnt = nullptr;
    if (workspace && slots > 0) {
        const size_t esz = dtype == HP_DTYPE_F64 ? 8 : 4;
        cnt = reinterpret_cast<unsigned*>(static_cast<char*>(workspace) +
                                          hp::align_up(esz * 128 * 128 * (size_t)slots));
        HIPCHK(hp::zero_u32(cnt, slots, s));
    }
    auto split = [&](auto ep) {
        using E = std::remove_pointer_t<decltype(ep.split_part)>;
        if (cnt) {
            ep.split_part = static_cast<E*>(workspace);
            ep.split_cnt = cnt;
            ep.split_slots = slots;
        }
        return ep;
    };
    hipError_t e;
    if (dtype == HP_DTYPE_F64) {
        e = hp::gemm(t, M, N, K, static_cast<const double*>(A), lda, static_cast<const double*>(B),
                     ldb, split(hp::epilogue_plain(static_cast<double*>(C), ldc, alpha, beta_identity)), s);
    } else if (dtype == HP_DTYPE_F32) {
        e = hp::gemm(t, M, N, K, static_cast<const float*>(A), lda, static_cast<const float*>(B),
                     ldb, split(hp::epilogue_plain(static_cast<float*>(C), ldc, alpha, beta_identity)), s);
    } else if (dtype == HP_DTYPE_BF16 || dtype == HP_DTYPE_F16) {
        e = hp::gemm_h16(t, dtype == HP_DTYPE_BF16 ? hp::LOWP_BF16 : hp::LOWP_F16, M, N, K, A, lda, B,
                         ldb, hp::epilogue_plain(static_cast<float*>(C), ldc, alpha, beta_identity), s);
    } else {
        e = hp::gemm_lowp(t, dtype == HP_DTYPE_BF16_F32 ? hp::LOWP_BF16 : hp::LOWP_F16, M, N, K,
                          static_cast<const float*>(A), lda, static_cast<const float*>(B), ldb,
                          hp::epilogue_plain(static_cast<float*>(C), ldc, alpha, beta_identity), s);
    }
    if (e != hipSuccess) return HP_EHIP;
    return HP_OK;
}

int hp_gemm(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K, double alpha, const void* A,
            int64_t lda, const void* B, int64_t ldb, double beta_identity, void* C, int64_t ldc,
            void* stream) {
    if (!h) return HP_EINVAL;
    CHK(gemm_args(dtype, M, N, K, A, lda, B, ldb, C, ldc));
    return gemm_run(h, dtype, M, N, K, alpha, A, lda, B, ldb, beta_identity, C, ldc, nullptr, 0,
                    stream);
}

// Scratch of hp_gemm_sym: enough for either tile with a symmetric launch.
static void gemm_sym_ws(int dtype, int64_t N, int64_t* slots, int64_t* cnt) {
    *slots = *cnt = 0;
    const hp::GemmType gt = hp::gemm_type(dtype);
    for (hp::GemmTile t : {hp::TILE_128x128_W16_K2_P2, hp::TILE_128x128_W8, hp::TILE_128x128_W4_DMA}) {
        int64_t sl = 0, c = 0;
        hp::gemm_sym_scratch(t, gt, N, &sl, &c);
        *slots = std::max(*slots, sl);
        *cnt = std::max(*cnt, c);
    }
}
static size_t gemm_sym_ws_bytes(int dtype, int64_t slots, int64_t cnt) {
    if (slots <= 0 || cnt <= 0) return 0;
    const size_t esz = dtype == HP_DTYPE_F64 ? 8 : 4;
    return hp::align_up(esz * 128 * 128 * (size_t)slots) + sizeof(unsigned) * (size_t)cnt;
}

int hp_gemm_sym_workspace_bytes(int dtype, int64_t N, int64_t K, size_t* bytes) {
    if (!bytes) return HP_EINVAL;
    if (dtype != HP_DTYPE_F64 && dtype != HP_DTYPE_F32) return HP_EINVAL;
    if (N < 1 || K < 1 || N > (1 << 24) || K > (1 << 24)) return HP_EINVAL;
    int64_t slots = 0, cnt = 0;
    gemm_sym_ws(dtype, N, &slots, &cnt);
    *bytes = gemm_sym_ws_bytes(dtype, slots, cnt);
    return HP_OK;
}

int hp_gemm_sym(hp_handle* h, int dtype, int64_t N, int64_t K, double alpha, const void* A,
                int64_t lda, const void* B, int64_t ldb, double beta_identity, void* C,
                int64_t ldc, void* workspace, size_t ws_bytes, void* stream) {
    if (!h) return HP_EINVAL;
    if (dtype != HP_DTYPE_F64 && dtype != HP_DTYPE_F32) return HP_EINVAL;
    CHK(gemm_args(dtype, N, N, K, A, lda, B, ldb, C, ldc));
    if (!workspace && ws_bytes) return HP_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % hp::kAlign) return HP_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
    const hp::GemmType gt = hp::gemm_type(dtype);
    hp::GemmTile t = hp::choose_tile(h, dtype, N, N, K, 0);
    if (!hp::gemm_sym_runs(t, gt)) t = hp::TILE_128x128_W16_K2_P2;
    int64_t slots = 0, cnt = 0;
    gemm_sym_ws(dtype, N, &slots, &cnt);
    const bool fits = workspace && slots > 0 && ws_bytes >= gemm_sym_ws_bytes(dtype, slots, cnt);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned* cp = nullptr;
    if (fits) {
        const size_t esz = dtype == HP_DTYPE_F64 ? 8 : 4;
        cp = reinterpret_cast<unsigned*>(static_cast<char*>(workspace) +
                                         hp::align_up(esz * 128 * 128 * (size_t)slots));
        HIPCHK(hp::zero_u32(cp, cnt, s));
    }
    auto sym = [&](auto ep) {
        using E = std::remove_pointer_t<decltype(ep.split_part)>;
        ep.sym = 1;
        if (cp) {
            ep.split_part = static_cast<E*>(workspace);
            ep.split_cnt = cp;
            ep.split_slots = slots;
            ep.split_ncnt = cnt;
        }
        return ep;
    };
    hipError_t e;
    if (dtype == HP_DTYPE_F64)
        e = hp::gemm(t, N, N, K, static_cast<const double*>(A), lda, static_cast<const double*>(B),
                     ldb, sym(hp::epilogue_plain(static_cast<double*>(C), ldc, alpha, beta_identity)), s);
    else
        e = hp::gemm(t, N, N, K, static_cast<const float*>(A), lda, static_cast<const float*>(B),
                     ldb, sym(hp::epilogue_plain(static_cast<float*>(C), ldc, alpha, beta_identity)), s);
    return e == hipSuccess ? HP_OK : HP_EHIP;
}

int hp_gemm_workspace_bytes(int dtype, int64_t M, int64_t N, int64_t K, size_t* bytes) {
    if (!bytes) return HP_EINVAL;
    if (dtype < HP_DTYPE_F64 || dtype > HP_DTYPE_F16) return HP_EINVAL;
    if (M < 1 || N < 1 || K < 1 || M > (1 << 24) || N > (1 << 24) || K > (1 << 24)) return HP_EINVAL;
    *bytes = gemm_ws_bytes(dtype, gemm_ws_slots(nullptr, dtype, M, N, K));
    return HP_OK;
}

int hp_gemm_ws(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K, double alpha,
               const void* A, int64_t lda, const void* B, int64_t ldb, double beta_identity,
               void* C, int64_t ldc, void* workspace, size_t ws_bytes, void* stream) {
    if (!h) return HP_EINVAL;
    CHK(gemm_args(dtype, M, N, K, A, lda, B, ldb, C, ldc));
    if (!workspace && ws_bytes) return HP_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % hp::kAlign) return HP_EINVAL;
    // the tile the handle chooses (environment override, autotuned entry or
    // default) decides how much of the workspace is used; with less than that
    // the product runs unsplit
    int64_t slots = gemm_ws_slots(h, dtype, M, N, K);
    if (!workspace || ws_bytes < gemm_ws_bytes(dtype, slots)) slots = 0;
    return gemm_run(h, dtype, M, N, K, alpha, A, lda, B, ldb, beta_identity, C, ldc, workspace,
                    slots, stream);
}

static void residual_layout(int kind, int l, int64_t m, int64_t n, size_t off[8], size_t* total) {
    // AX (m x m), XA (n x n), AXA (m x n), XAX (n x m), then for Drazin two
    // n x n power buffers; then the small area and the scalar slots
    const int64_t ldm = hp::pad_ld(m), ldn = hp::pad_ld(n);
    size_t o = 0;
    off[0] = o; o = hp::align_up(o + 8 * (size_t)(m * ldm));
    off[1] = o; o = hp::align_up(o + 8 * (size_t)(n * ldn));
    off[2] = o; o = hp::align_up(o + 8 * (size_t)(m * ldn));
    off[3] = o; o = hp::align_up(o + 8 * (size_t)(n * ldm));
    off[4] = o; o = hp::align_up(o + (kind == HP_KIND_DRAZIN ? 8 * (size_t)(n * ldn) : 0));
    off[5] = o; o = hp::align_up(o + (kind == HP_KIND_DRAZIN ? 8 * (size_t)(n * ldn) : 0));
    const int64_t big = std::max(m, n);
    off[6] = o; o = hp::align_up(o + 8 * (size_t)std::max<int64_t>(big, ((big + 31) / 32) * ((big + 31) / 32)));
    off[7] = o; o = hp::align_up(o + 8 * 16);
    (void)l;
    *total = o;
}

// Complex input through its real 2m x 2n form: the real form's workspace
// after the two real-form matrices.
static void complex_layout(int64_t m, int64_t n, size_t* offX, size_t* offW, int64_t* ldE,
                           int64_t* ldXe) {
    *ldE = hp::pad_ld(2 * n);
    *ldXe = hp::pad_ld(2 * m);
    *offX = hp::align_up(sizeof(double) * (size_t)(2 * m) * (size_t)*ldE);
    *offW = *offX + hp::align_up(sizeof(double) * (size_t)(2 * n) * (size_t)*ldXe);
}

int hp_complex_workspace_bytes(const hp_params* p, int64_t m, int64_t n, size_t* bytes) {
    if (!bytes || m < 1 || n < 1 || m > 32767 || n > 32767) return HP_EINVAL;
    size_t inner = 0;
    CHK(hp_workspace_bytes(p, 2 * m, 2 * n, &inner));
    size_t offX, offW;
    int64_t ldE, ldXe;
    complex_layout(m, n, &offX, &offW, &ldE, &ldXe);
    *bytes = offW + inner;
    return HP_OK;
}

int hp_solve_complex(hp_handle* h, const hp_params* p, const double* A, int64_t m, int64_t n,
                     int64_t lda, double* X, int64_t ldx, void* workspace, size_t ws_bytes,
                     void* stream, hp_result* out) {
    if (!h || !A || !X || !p) return HP_EINVAL;
    // rules whose real form is not the complex rule: Tr(A^{l+1}) of the real
    // form is twice the real part of the complex trace, and its diagonal
    // holds only the real parts
    if ((p->kind == HP_KIND_DRAZIN && p->alpha_rule != HP_ALPHA_USER) ||
        p->alpha_rule == HP_ALPHA_DIAG)
        return HP_EUNSUPPORTED;
    size_t need = 0;
    CHK(hp_complex_workspace_bytes(p, m, n, &need));
    if (lda < n || ldx < m) return HP_EINVAL;
    if (!workspace || ws_bytes < need) return HP_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) % hp::kAlign) return HP_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
    size_t offX, offW;
    int64_t ldE, ldXe;
    complex_layout(m, n, &offX, &offW, &ldE, &ldXe);
    char* ws = static_cast<char*>(workspace);
    double* E = reinterpret_cast<double*>(ws);
    double* Xe = reinterpret_cast<double*>(ws + offX);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hp::Range range("hp_solve_complex %lldx%lld", (long long)m, (long long)n);
    HIPCHK(hp::embed_complex(A, lda, m, n, E, ldE, s));
    const int rc = hp_solve(h, p, E, 2 * m, 2 * n, ldE, nullptr, 0, Xe, ldXe, ws + offW,
                            ws_bytes - offW, stream, out);
    if (rc < 0) return rc;
    HIPCHK(hp::extract_complex(Xe, ldXe, n, m, X, ldx, s));
    HIPCHK(hipStreamSynchronize(s));
    return rc;
}

int hp_residuals_workspace_bytes(int kind, int l, int64_t m, int64_t n, size_t* bytes) {
    if (!bytes || m < 1 || n < 1 || m > 65535 || n > 65535) return HP_EINVAL;
    if (kind != HP_KIND_MOORE_PENROSE && kind != HP_KIND_DRAZIN) return HP_EINVAL;
    if (kind == HP_KIND_DRAZIN && (m != n || l < 1 || l > 64)) return HP_EINVAL;
    size_t off[8];
    residual_layout(kind, l, m, n, off, bytes);
    return HP_OK;
}

int hp_residuals(hp_handle* h, int kind, int l, const double* A, int64_t m, int64_t n, int64_t lda,
                 const double* X, int64_t ldx, void* workspace, size_t ws_bytes, void* stream,
                 double out[4]) {
    if (!h || !A || !X || !out) return HP_EINVAL;
    size_t need = 0;
    CHK(hp_residuals_workspace_bytes(kind, l, m, n, &need));
    if (lda < n || ldx < m || (lda & 1) || (ldx & 1)) return HP_EINVAL;
    if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(X)) & 15) return HP_EINVAL;
    if (!workspace || ws_bytes < need) return HP_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) % hp::kAlign) return HP_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    size_t off[8], total;
    residual_layout(kind, l, m, n, off, &total);
    char* w = static_cast<char*>(workspace);
    auto dp = [&](int i) { return reinterpret_cast<double*>(w + off[i]); };
    const int64_t ldm = hp::pad_ld(m), ldn = hp::pad_ld(n);
    double *AX = dp(0), *XA = dp(1), *AXA = dp(2), *XAX = dp(3), *tmp = dp(6), *scal = dp(7);
    auto mm = [&](int64_t M, int64_t N, int64_t K, const double* P, int64_t ldp, const double* Q,
                  int64_t ldq, double* C, int64_t ldc) -> int {
        const hp::GemmTile t = hp::choose_tile(h, HP_DTYPE_F64, M, N, K);
        return hp::gemm(t, M, N, K, P, ldp, Q, ldq, hp::epilogue_plain(C, ldc), s) == hipSuccess
                   ? HP_OK : HP_EHIP;
    };
    CHK(mm(m, m, n, A, lda, X, ldx, AX, ldm));     // AX
    CHK(mm(n, n, m, X, ldx, A, lda, XA, ldn));     // XA
    CHK(mm(n, m, n, XA, ldn, X, ldx, XAX, ldm));   // XAX
    double* hs = h->host_scal;
    if (kind == HP_KIND_MOORE_PENROSE) {
        CHK(mm(m, n, m, AX, ldm, A, lda, AXA, ldn));   // AXA
        HIPCHK(hp::diffsq(AXA, ldn, A, lda, 1.0, m, n, tmp, scal, 0, s));
        HIPCHK(hp::diffsq(A, lda, nullptr, 0, 0.0, m, n, tmp, scal, 1, s));
        HIPCHK(hp::diffsq(XAX, ldm, X, ldx, 1.0, n, m, tmp, scal, 2, s));
        HIPCHK(hp::diffsq(X, ldx, nullptr, 0, 0.0, n, m, tmp, scal, 3, s));
        HIPCHK(hp::asymsq(AX, ldm, m, tmp, scal, 4, s));
        HIPCHK(hp::diffsq(AX, ldm, nullptr, 0, 0.0, m, m, tmp, scal, 5, s));
        HIPCHK(hp::asymsq(XA, ldn, n, tmp, scal, 6, s));
        HIPCHK(hp::diffsq(XA, ldn, nullptr, 0, 0.0, n, n, tmp, scal, 7, s));
        HIPCHK(hipMemcpyAsync(hs, scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double v[8];
        std::memcpy(v, hs, sizeof(v));
        for (int i = 0; i < 4; ++i) out[i] = std::sqrt(v[2 * i]) / std::sqrt(v[2 * i + 1]);
        return HP_OK;
    }
    // Drazin: A^l by repeated products (A^1 = A), then A^{l+1} X = A^l (A X)
    double* pw[2] = {dp(4), dp(5)};
    const double* Al = A;
    int64_t ldl = lda;
    for (int i = 1; i < l; ++i) {
        double* dst = pw[i & 1];
        CHK(mm(n, n, n, Al, ldl, A, lda, dst, ldn));
        Al = dst;
        ldl = ldn;
    }
    double* other = (Al == pw[0]) ? pw[1] : pw[0];
    CHK(mm(n, n, n, Al, ldl, AX, ldm, other, ldn));  // A^l (A X) = A^{l+1} X
    HIPCHK(hp::diffsq(other, ldn, Al, ldl, 1.0, n, n, tmp, scal, 0, s));
    HIPCHK(hp::diffsq(Al, ldl, nullptr, 0, 0.0, n, n, tmp, scal, 1, s));
    HIPCHK(hp::diffsq(XAX, ldm, X, ldx, 1.0, n, n, tmp, scal, 2, s));
    HIPCHK(hp::diffsq(X, ldx, nullptr, 0, 0.0, n, n, tmp, scal, 3, s));
    HIPCHK(hp::diffsq(AX, ldm, XA, ldn, 1.0, n, n, tmp, scal, 4, s));
    HIPCHK(hp::diffsq(AX, ldm, nullptr, 0, 0.0, n, n, tmp, scal, 5, s));
    HIPCHK(hipMemcpyAsync(hs, scal, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double v[6];
    std::memcpy(v, hs, sizeof(v));
    for (int i = 0; i < 3; ++i) out[i] = std::sqrt(v[2 * i]) / std::sqrt(v[2 * i + 1]);
    out[3] = 0.0;
    return HP_OK;
}

// Scratch of hp_autotune: operands and result, then split-K scratch for 4
// partial tiles per output tile and as many counters. The grouped kinds hold
// A, B and `entries` results instead, then the launch table.
struct TuneLayout {
    int64_t lda, ldb, ldc, slots, entries;
    size_t ops, part, total;
};
static bool grouped_dtype(int dtype) {
    return dtype == HP_DTYPE_GROUPED_F64 || dtype == HP_DTYPE_GROUPED_F32;
}
static size_t operand_bytes(int dtype) {
    return (dtype == HP_DTYPE_F64 || dtype == HP_DTYPE_GROUPED_F64) ? 8
           : (dtype == HP_DTYPE_BF16 || dtype == HP_DTYPE_F16)      ? 2
                                                                     : 4;
}

static int tune_layout(int dtype, int64_t M, int64_t N, int64_t K, TuneLayout* L) {
    if (dtype < HP_DTYPE_F64 || dtype > HP_DTYPE_GROUPED_F32) return HP_EINVAL;
    if (M < 1 || N < 1 || K < 1 || M > 65535 || N > 65535 || K > 65535) return HP_EINVAL;
    if (grouped_dtype(dtype)) {
        // as many copies of the product as fill about 4 Mi outputs (1 to 64),
        // so that a table of small products is timed as the loop sees it
        const size_t esz = operand_bytes(dtype);
        const int64_t vec = 16 / (int64_t)esz;
        L->lda = (K + vec - 1) / vec * vec;
        L->ldb = L->ldc = (N + vec - 1) / vec * vec;
        L->slots = 0;
        L->entries = std::min<int64_t>(64, std::max<int64_t>(1, (int64_t(4) << 20) / (M * N)));
        L->ops = hp::align_up(esz * (size_t)(M * L->lda + K * L->ldb + L->entries * M * L->ldc));
        const size_t ent = dtype == HP_DTYPE_GROUPED_F64 ? sizeof(hp::GroupEntry<double>)
                                                         : sizeof(hp::GroupEntry<float>);
        L->part = hp::align_up(sizeof(hp::GroupHeader)) + ent * (size_t)L->entries;
        L->total = L->ops + L->part;
        return HP_OK;
    }
    L->entries = 0;
    const size_t esz = operand_bytes(dtype) == 2 ? 4 : operand_bytes(dtype);  // C is float
    const int64_t vec = 16 / (int64_t)operand_bytes(dtype);
    const bool h16 = operand_bytes(dtype) == 2;  // B held as B^T (N x K)
    L->lda = (K + vec - 1) / vec * vec;
    L->ldb = h16 ? L->lda : (N + vec - 1) / vec * vec;
    L->ldc = N;
    L->slots = 4 * ((M + 127) / 128) * ((N + 127) / 128);
    L->ops = hp::align_up(esz * (size_t)(M * L->lda + (h16 ? N : K) * L->ldb + M * L->ldc));
    L->part = hp::align_up(esz * 128 * 128 * (size_t)L->slots);
    L->total = L->ops + L->part + sizeof(unsigned) * (size_t)L->slots;
    return HP_OK;
}

int hp_autotune_scratch_bytes(int dtype, int64_t M, int64_t N, int64_t K, size_t* bytes) {
    if (!bytes) return HP_EINVAL;
    TuneLayout L;
    CHK(tune_layout(dtype, M, N, K, &L));
    *bytes = L.total;
    return HP_OK;
}

}  // extern "C"

namespace {

// hp_autotune of the grouped launch: every grouped tile on a table of
// L.entries copies of the product (shared operands, distinct results).
template <typename T>
int autotune_grouped(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K, const TuneLayout& L,
                     char* base, int reps, hipStream_t s, int* tile, double* ms) {
    T* A = reinterpret_cast<T*>(base);
    T* B = A + M * L.lda;
    T* C = B + K * L.ldb;
    char* tab = base + L.ops;
    auto* hdr_d = reinterpret_cast<hp::GroupHeader*>(tab);
    auto* ents_d = reinterpret_cast<hp::GroupEntry<T>*>(tab + hp::align_up(sizeof(hp::GroupHeader)));
    HIPCHK(hipMemsetAsync(A, 0, sizeof(T) * (size_t)(M * L.lda), s));
    HIPCHK(hipMemsetAsync(B, 0, sizeof(T) * (size_t)(K * L.ldb), s));
    std::vector<hp::GroupEntry<T>> ents((size_t)L.entries);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int best = -1;
    double best_ms = 0.0;
    for (int cfg = 0; cfg < hp::GTILE_COUNT; ++cfg) {
        const int dim = hp::grouped_tile_dim(cfg);
        const int tm = (int)((M + dim - 1) / dim), tn = (int)((N + dim - 1) / dim);
        hp::GroupHeader hdr{(int)L.entries, (int)L.entries * tm * tn};
        for (int64_t e = 0; e < L.entries; ++e) {
            hp::GroupEntry<T>& g = ents[(size_t)e];
            g = hp::GroupEntry<T>{};
            g.M = (int)M;
            g.N = (int)N;
            g.K = (int)K;
            g.tiles_n = tn;
            g.tile_start = (int)e * tm * tn;
            g.A = A;
            g.lda = L.lda;
            g.B = B;
            g.ldb = L.ldb;
            g.ep = hp::epilogue_plain(C + e * M * L.ldc, L.ldc);
        }
        // ordered after the previous configuration's launches on s
        if (hipMemcpyAsync(hdr_d, &hdr, sizeof(hdr), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(ents_d, ents.data(), sizeof(hp::GroupEntry<T>) * ents.size(),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            break;
        auto launch = [&]() { return hp::gemm_grouped(hdr_d, ents_d, 1024, cfg, s); };
        if (launch() != hipSuccess) continue;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) (void)launch();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float el = 0.f;
        (void)hipEventElapsedTime(&el, e0, e1);
        const double avg = el / reps / (double)L.entries;  // per product
        if (best < 0 || avg < best_ms) {
            best = cfg;
            best_ms = avg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) return HP_EHIP;
    h->tuned[{dtype, M, N, K}] = best;
    h->grouped_cfg[dtype - HP_DTYPE_GROUPED_F64] = best;
    ++h->tune_gen;
    *tile = best;
    *ms = best_ms;
    return HP_OK;
}

}  // namespace

extern "C" {

int hp_autotune(hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K, void* scratch,
                size_t scratch_bytes, int reps, void* stream, int* tile, double* ms) {
    if (!h || !scratch || !tile || !ms || reps < 1) return HP_EINVAL;
    TuneLayout L;
    CHK(tune_layout(dtype, M, N, K, &L));
    if (grouped_dtype(dtype)) {
        if (scratch_bytes < L.total) return HP_EWORKSPACE;
        if (reinterpret_cast<uintptr_t>(scratch) % 16) return HP_EINVAL;
        if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        char* base = static_cast<char*>(scratch);
        return dtype == HP_DTYPE_GROUPED_F64
                   ? autotune_grouped<double>(h, dtype, M, N, K, L, base, reps, s, tile, ms)
                   : autotune_grouped<float>(h, dtype, M, N, K, L, base, reps, s, tile, ms);
    }
    const size_t esz = dtype == HP_DTYPE_F64 ? 8 : 4;  // 16-bit operands get 4-byte room
    const bool h16 = dtype == HP_DTYPE_BF16 || dtype == HP_DTYPE_F16;
    const int64_t lda = L.lda, ldb = L.ldb, ldc = L.ldc, slots = L.slots;
    const size_t ops = L.ops;
    if (scratch_bytes < L.total) return HP_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(scratch) % 16) return HP_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return HP_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(scratch);
    void* A = base;
    void* B = base + esz * (size_t)(M * lda);
    void* C = base + esz * (size_t)(M * lda + (h16 ? N : K) * ldb);
    void* split_part = base + ops;
    unsigned* split_cnt = reinterpret_cast<unsigned*>(base + ops + L.part);
    HIPCHK(hp::zero_u32(split_cnt, slots, s));
    auto with_split = [&](auto ep) {
        using E = std::remove_pointer_t<decltype(ep.split_part)>;
        ep.split_part = static_cast<E*>(split_part);
        ep.split_cnt = split_cnt;
        ep.split_slots = slots;
        return ep;
    };
    // operands: identity-like fills are enough for timing (no data dependence)
    if (dtype == HP_DTYPE_F64) {
        HIPCHK(hp::set_identity(static_cast<double*>(A), lda, M, K, s));
        HIPCHK(hp::set_identity(static_cast<double*>(B), ldb, K, N, s));
    } else {
        HIPCHK(hipMemsetAsync(A, 0, esz * (size_t)(M * lda), s));
        HIPCHK(hipMemsetAsync(B, 0, esz * (size_t)((h16 ? N : K) * ldb), s));
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int best = -1;
    double best_ms = 0.0;
    for (int t = 0; t < hp::TILE_COUNT; ++t) {
        auto launch = [&]() -> hipError_t {
            if (dtype == HP_DTYPE_F64)
                return hp::gemm((hp::GemmTile)t, M, N, K, static_cast<const double*>(A), lda,
                                static_cast<const double*>(B), ldb,
                                with_split(hp::epilogue_plain(static_cast<double*>(C), ldc)), s);
            if (dtype == HP_DTYPE_F32)
                return hp::gemm((hp::GemmTile)t, M, N, K, static_cast<const float*>(A), lda,
                                static_cast<const float*>(B), ldb,
                                with_split(hp::epilogue_plain(static_cast<float*>(C), ldc)), s);
            if (h16)
                return hp::gemm_h16((hp::GemmTile)t, dtype == HP_DTYPE_BF16 ? hp::LOWP_BF16 : hp::LOWP_F16,
                                    M, N, K, A, lda, B, ldb,
                                    hp::epilogue_plain(static_cast<float*>(C), ldc), s);
            return hp::gemm_lowp((hp::GemmTile)t, dtype == HP_DTYPE_BF16_F32 ? hp::LOWP_BF16 : hp::LOWP_F16,
                                 M, N, K, static_cast<const float*>(A), lda,
                                 static_cast<const float*>(B), ldb,
                                 hp::epilogue_plain(static_cast<float*>(C), ldc), s);
        };
        if (launch() != hipSuccess) continue;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) (void)launch();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float el = 0.f;
        (void)hipEventElapsedTime(&el, e0, e1);
        const double avg = el / reps;
        if (best < 0 || avg < best_ms) {
            best = t;
            best_ms = avg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) return HP_EHIP;
    h->tuned[{dtype, M, N, K}] = best;
    ++h->tune_gen;
    *tile = best;
    *ms = best_ms;
    return HP_OK;
}

int hp_tune_export(hp_handle* h, int64_t* rows, int cap, int* count) {
    if (!h || !count || (cap > 0 && !rows)) return HP_EINVAL;
    int i = 0;
    for (const auto& kv : h->tuned) {
        if (i < cap) {
            for (int j = 0; j < 4; ++j) rows[5 * i + j] = kv.first[j];
            rows[5 * i + 4] = kv.second;
        }
        ++i;
    }
    *count = i;
    return HP_OK;
}

int hp_tune_import(hp_handle* h, const int64_t* rows, int count) {
    if (!h || count < 0 || (count > 0 && !rows)) return HP_EINVAL;
    for (int i = 0; i < count; ++i) {
        const int64_t* r = rows + 5 * i;
        if (r[0] < HP_DTYPE_F64 || r[0] > HP_DTYPE_GROUPED_F32 || r[4] < 0 ||
            r[4] >= (grouped_dtype((int)r[0]) ? hp::GTILE_COUNT : hp::TILE_COUNT))
            return HP_EINVAL;
    }
    for (int i = 0; i < count; ++i) {
        const int64_t* r = rows + 5 * i;
        h->tuned[{r[0], r[1], r[2], r[3]}] = (int)r[4];
        if (grouped_dtype((int)r[0])) h->grouped_cfg[r[0] - HP_DTYPE_GROUPED_F64] = (int)r[4];
    }
    ++h->tune_gen;
    return HP_OK;
}

}  // extern "C"
