// Host-side pieces shared by the single, batched and served solvers.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <cstdint>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdarg>
#include <cstdio>

#include "hp_internal.h"
#include "hp_loop.h"
#include "hyperpower.h"

struct hp_handle {
    int device = 0;
    int forced_tile = -1;         // HP_GEMM_TILE: one tile configuration for every product
    // autotuned tiles: (dtype, M, N, K) -> tile index
    std::map<std::array<int64_t, 4>, int> tuned;
    int tune_gen = 0;             // bumped whenever `tuned` changes
    // grouped-launch tile (GroupedTile) per precision (FP64, FP32) for groups
    // created from now on: the latest autotuned or imported choice
    int grouped_cfg[2] = {0, 0};
    // pinned: hp::SLOT_COUNT doubles, then kHostExtra doubles of staging
    // (device_stop: the step parameters, and the head of the DevLoop state,
    // which is read back over the slots)
    double* host_scal = nullptr;
    // SLOT_COUNT doubles of fine-grained pinned memory that the end-of-loop
    // reduction writes directly (device address host_sums_dev), in place of
    // a device-to-host copy per loop
    // Slot SLOT_COUNT holds the number of the last loop whose sums arrived
    // (sums_seq counts them), so that the host can poll it instead of waiting
    // for the stream.
    double* host_sums = nullptr;
    double* host_sums_dev = nullptr;
    uint64_t sums_seq = 0;
    // device_stop: the head of the DevLoop state, written by the device at
    // the end of each chunk of loops, then the chunk's number (loop_seq)
    // after it, which the host polls in place of a copy and a stream wait
    double* host_loop = nullptr;
    double* host_loop_dev = nullptr;
    uint64_t loop_seq = 0;
    static constexpr int kHostExtra = 16;
    static constexpr int kEvents = 64;
    hipEvent_t ev[kEvents] = {};
    // hp_params.device_stop: two loops of a solve captured (on cap_stream) as
    // a hipGraph and replayed on the solve stream, cached per (workspace,
    // shape, loop form); least recently used evicted.
    struct LoopGraph {
        std::array<int64_t, 10> key;
        hipGraph_t graph;
        hipGraphExec_t exec;
        uint64_t used;
    };
    static constexpr int kGraphs = 8;
    std::vector<LoopGraph> graphs;
    uint64_t graph_clock = 0;
    hipStream_t cap_stream = nullptr;
};

#define HIPCHK(x)                              \
    do {                                       \
        if ((x) != hipSuccess) return HP_EHIP; \
    } while (0)

#define CHK(x)                        \
    do {                              \
        int rc_ = (x);                \
        if (rc_ != HP_OK) return rc_; \
    } while (0)

namespace hp {

// A named roctx range over a scope: shows the solve's phases (set-up, each
// loop with its stage, projection, grouped loops) on the timeline of
// `rocprofv3 --marker-trace`; without a tool attached it costs a call.
struct Range {
    explicit Range(const char* fmt, ...) {
        char buf[96];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        roctxRangePushA(buf);
    }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

inline GemmType gemm_type(int dtype) {
    if (dtype == HP_DTYPE_F64) return GT_F64;
    if (dtype == HP_DTYPE_F32) return GT_F32;
    if (dtype == HP_DTYPE_BF16 || dtype == HP_DTYPE_F16) return GT_H16;
    return GT_LOWP;
}

// The tile a product of this dtype (HP_DTYPE_*) and shape runs on: the
// environment override, else the handle's autotuned entry, else the default.
// A split tile that cannot run split (too little scratch: `split_slots`
// partial tiles available) is replaced by the default unsplit choice, so that
// gemm_blocks of the returned tile is the launch's block count.
inline GemmTile choose_tile(const hp_handle* h, int dtype, int64_t M, int64_t N, int64_t K,
                            int64_t split_slots = 0) {
    GemmTile t;
    auto it = h->tuned.find({dtype, M, N, K});
    if (h->forced_tile >= 0) t = (GemmTile)h->forced_tile;
    else if (it != h->tuned.end()) t = (GemmTile)it->second;
    else t = gemm_pick_tile(M, N, K, gemm_type(dtype));
    if ((t == TILE_128x128_W8_S2 || t == TILE_128x128_W8_S4) &&
        !gemm_split_runs(t, M, N, K, gemm_type(dtype), split_slots))
        t = gemm_pick_tile(M, N, K, gemm_type(dtype), false);
    // a forced or tuned tile that this GEMM type does not run: the default
    if (!gemm_runs(t, gemm_type(dtype))) t = gemm_pick_tile(M, N, K, gemm_type(dtype), false);
    return t;
}

// Constants of the factored polynomial: the closed forms printed in Section 2
// (c1, c2, c3 of (simplify1); d1, d2 of (simplify2); mu, psi of (hyper18-33)).
struct PMConst {
    double c1, c2, c3, d1, d2, mu, psi;
};
PMConst pm_const();

// Takes the device address of hp_solve_noalloc's fixed workspace on `device`
// (which must be current) once per device; hp_create calls it.
int noalloc_init(int device);

// hp_solve's body; `may_allocate` false (hp_solve_noalloc) keeps it from
// creating anything (the device_stop path then launches loop by loop
// instead of capturing a graph).
int solve_entry(hp_handle* h, const hp_params* p, const double* A, int64_t m, int64_t n,
                int64_t lda, const double* X0, int64_t ldx0, double* X, int64_t ldx,
                void* workspace, size_t ws_bytes, void* stream, hp_result* out,
                bool may_allocate);

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t pad_ld(int64_t cols);

// Workspace layout of one problem. FP64 set: A, three n x m iterates (X_k,
// X_{k+1}, X_{k+1/2}) and seven s x s loop matrices. FP32 set (FP32 and mixed
// precision): the same in single precision. FP32-only solves keep just A and
// one iterate in FP64 (X0 is formed there).
struct Plan {
    int64_t m = 0, n = 0;
    bool left = false;
    int64_t s = 0;  // side of the residual R (n for left, m for right)
    int64_t ldA = 0, ldX = 0, ldS = 0;
    int64_t ldA32 = 0, ldX32 = 0, ldS32 = 0;
    int nX64 = 0, nS64 = 0, nX32 = 0, nS32 = 0;
    bool has32 = false;
    // HP_PREC_MIXED: 16-bit copies of the FP32 set for the first stage's
    // products, each matrix row-major and transposed (k-contiguous operands)
    bool has16 = false;
    int64_t ldA16 = 0, ldAt16 = 0, ldX16 = 0, ldXt16 = 0, ldS16 = 0;
    size_t offA16 = 0, offAt16 = 0, offX16[3] = {}, offXt16[3] = {}, offS16[7] = {}, offSt16[7] = {};
    size_t offA = 0, offX[4] = {}, offS[7] = {};
    size_t offA32 = 0, offX32[4] = {}, offS32[7] = {};
    bool has_proj = false;      // A^T (n x m) and X^T (m x n) for the projection
    size_t offAt = 0, offXt = 0;
    // split-K scratch: splitSlots partial tiles (128 x 128 doubles), then
    // splitCnt arrival counters; none when no product of the solve splits.
    // The symmetric launches of the loop products share it.
    int64_t splitSlots = 0, splitCnt = 0;
    // the loop's s x s products may run symmetric (HP_FLAG_SYMMETRIC: X_k =
    // p(A^T A) A^T for a Moore-Penrose solve from alpha A^T without Chop)
    bool sym = false;
    // FP64-stage loops may run in the delta form (HP_PREC_DELTA32, or staged
    // precisions without HP_FLAG_FP64_POLY)
    bool delta = false;
    size_t offSplit = 0, offSplitCnt = 0;
    size_t offSmall = 0, nSmall = 0, offScal = 0, offDev = 0, offStep = 0, total = 0;
};
// `single`: a single solve, which reserves the split-K scratch the default
// tile choice needs for its products (the grouped launches never split) and a
// fourth iterate in the final stage's set for the best iterate kept before
// convergence sets in (LoopState::kBest; batched and served solves return X_k
// on divergence instead).
Plan make_plan(const hp_params* p, int64_t m, int64_t n, bool single = true);
// Spins for at most max_us microseconds until *flag (pinned host memory that
// a kernel writes) equals `want`; false when the time is up.
bool poll_host(const double* flag, double want, double max_us);
int validate(const hp_params* p, int64_t m, int64_t n);


// The buffers of one precision.
template <typename T>
struct Set {
    T* A = nullptr;
    T* X[4] = {};  // X_k, X_{k+1}, X_{k+1/2}; [3]: the best iterate (single solves)
    T* S[7] = {};
    int64_t ldA = 0, ldX = 0, ldS = 0;
};

// The 16-bit copies of one FP32 matrix: row-major (ld) and transposed (ldt).
struct Copy16 {
    void* h = nullptr;
    int64_t ld = 0;
    void* ht = nullptr;
    int64_t ldt = 0;
};

struct Buffers {
    Set<double> b64;
    Set<float> b32;
    // copies of b32.A, b32.X[i], b32.S[i] (HP_PREC_MIXED only)
    Copy16 A16, X16[3], S16[7];
    // the copies of an FP32 set matrix (given by its base pointer), or null
    const Copy16* copy16(const float* p) const {
        if (!A16.h) return nullptr;
        if (p == b32.A) return &A16;
        for (int i = 0; i < 3; ++i)
            if (p == b32.X[i]) return &X16[i];
        for (int i = 0; i < 7; ++i)
            if (p == b32.S[i]) return &S16[i];
        return nullptr;
    }
    double* At = nullptr;  // n x m, ld b64.ldX
    double* Xt = nullptr;  // m x n, ld b64.ldA
    double* small = nullptr;
    double* scal = nullptr;
    DevLoop* dev = nullptr;  // loop control on the device (hp_params.device_stop)
    StepParams* step = nullptr;  // its parameters
    double* split_part = nullptr;  // Plan::splitSlots tiles of 128 x 128 doubles
    unsigned* split_cnt = nullptr;
};
Buffers carve(const Plan& pl, char* ws);

// One product of a loop: C = epilogue(A B), A M x K, B K x N.
template <typename T>
struct GemmCall {
    int64_t M, N, K;
    const T* A;
    int64_t lda;
    const T* B;
    int64_t ldb;
    EpilogueT<T> ep;
};

// Which copies of its outputs a product of the 16-bit stage must leave: the
// row-major 16-bit copy where a later product of the loop reads the matrix as
// its left operand, the transposed copy where one reads it as its right
// operand, and the FP32 value where an epilogue or the stopping test reads it
// (or it is an iterate or R, which the next stage and the projection test
// read). Uses end where a later product writes the same buffer again.
struct CopyUse {
    bool row[3] = {}, t[3] = {}, f32[3] = {};
};
template <typename T>
void copy_uses(const GemmCall<T>* c, int nc, const Set<T>& b, CopyUse* u) {
    for (int i = 0; i < nc; ++i) {
        u[i] = CopyUse{};
        for (int o = 0; o < 3; ++o) {
            const T* P = c[i].ep.out[o];
            if (!P) continue;
            bool iterate = P == b.S[0];
            for (int x = 0; x < 3; ++x) iterate = iterate || P == b.X[x];
            if (iterate) {
                u[i].row[o] = u[i].t[o] = u[i].f32[o] = true;
                continue;
            }
            for (int j = i + 1; j < nc; ++j) {
                const EpilogueT<T>& e = c[j].ep;
                if (c[j].A == P) u[i].row[o] = true;
                if (c[j].B == P) u[i].t[o] = true;
                if (e.D1 == P || e.D2 == P || e.ref == P) u[i].f32[o] = true;
                if (e.out[0] == P || e.out[1] == P || e.out[2] == P) break;
            }
        }
    }
}

// Most products a loop can take (HM: 9, plus 2 for the stabilising product).
constexpr int kMaxLoopGemms = 11;


// The update product X_{k+1} = X W (right form) or W X (left form), writing
// the partial sums of the stopping test against X_k into `partials`; with
// `stab`, it writes X_{k+1/2} instead and the stabilising product
// X_{k+1/2} A X_{k+1/2} of (PM-modified), Section 7, follows, associated so
// that the middle product is the smaller square (into `mid`, an s x s buffer
// that is dead by then). Appends to out[c..]; returns the new count.
// With `plus_x` the product is X_k + X_k W (or X_k + W X_k) (with `stab`, that
// is X_{k+1/2}).
template <typename T>
int describe_update(const Plan& pl, const Set<T>& b, const T* W, T* Xk, T* Xn, T* Xh, bool stab,
                    double* partials, T* mid, GemmCall<T>* out, int c, bool plus_x = false) {
    const int64_t m = pl.m, n = pl.n;
    const int64_t ldS = b.ldS, ldX = b.ldX, ldA = b.ldA;
    {
        EpilogueT<T> e = epilogue_plain(stab ? Xh : Xn, ldX);
        if (!stab) {
            e.ref = Xk; e.ldref = ldX; e.partials = partials;
        }
        if (plus_x) {
            e.D1 = Xk; e.ld1 = ldX; e.g1[0] = 1.0;
        }
        if (pl.left) out[c++] = {n, m, n, W, ldS, Xk, ldX, e};
        else out[c++] = {n, m, m, Xk, ldX, W, ldS, e};
    }
    if (stab) {
        EpilogueT<T> e = epilogue_plain(Xn, ldX);
        e.ref = Xk; e.ldref = ldX; e.partials = partials;
        EpilogueT<T> em = epilogue_plain(mid, ldS);
        em.sym = 1;  // X A (or A X) is symmetric for X = p(A^T A) A^T
        if (m >= n) {
            out[c++] = {n, n, m, Xh, ldX, b.A, ldA, em};
            out[c++] = {n, m, n, mid, ldS, Xh, ldX, e};
        } else {
            out[c++] = {m, m, n, b.A, ldA, Xh, ldX, em};
            out[c++] = {n, m, m, Xh, ldX, mid, ldS, e};
        }
    }
    return c;
}

// out[c] = the residual product: out0 = id0 I + acc0 P (and more outputs as
// given in `e`), P = A X (right form, m x m) or X A (left form, n x n).
template <typename T>
int describe_residual(const Plan& pl, const Set<T>& b, const T* Xk, EpilogueT<T> e,
                      GemmCall<T>* out, int c) {
    const int64_t m = pl.m, n = pl.n;
    e.sym = 1;
    if (pl.left) out[c++] = {n, n, m, Xk, b.ldX, b.A, b.ldA, e};
    else out[c++] = {m, m, n, b.A, b.ldA, Xk, b.ldX, e};
    return c;
}

// The products of one loop of HP_METHOD_* `method`. Every method keeps
// R = I - AX (or I - XA) in b.S[0] through the loop (a lower precision stage's
// last R decides the projection).
//
// PM, Section 2, in the association printed there: R; R^2; R^4 with
// F1 = I + c1 R^2 + R^4 and F2 = I + c2 R^2 + R^4 in its epilogue; F1 F2 with
// T = M + c3 R^2 and S = M + d1 R^2 + d2 R^4; T S + mu R^2 + psi R^4 = V;
// V + R V = W; the update. 7 products.
// SM (schulz): R and W = I + R = 2I - AX from one product; the update. 2.
// CM (chebyshev): P = AX with R = I - P and Q = 3I - P; W = 3I - P Q; the
// update. 3.
// FM (SoleymaniN): psi; psi^2 with zeta = I + psi + psi^2; upsilon =
// psi + psi^4 from psi^2 psi^2; W = I + upsilon zeta; the update. 5.
// HM (hyper18-2): R; R^2 with F2 = R^2 - R + I and F3 = R^2 + R + I; R^3;
// R^6 only as F4 = R^6 - R^3 + I and F5 = R^6 + R^3 + I; G = F2 + R F2
// (= (I + R) F2); G F3; G F4; G F5; the update. 9.
// Returns the number of calls (at most kMaxLoopGemms).
template <typename T>
int describe_loop(int method, const Plan& pl, const Set<T>& b, T* Xk, T* Xn, T* Xh, bool stab,
                  double* partials, GemmCall<T> out[kMaxLoopGemms]) {
    const int64_t sd = pl.s, ldS = b.ldS;
    T* const* S = b.S;
    int c = 0;
    // every s x s product of a loop is a polynomial in R: symmetric when R is
    auto sq = [&](const T* A, const T* B, EpilogueT<T> e) {
        e.sym = 1;
        out[c++] = {sd, sd, sd, A, ldS, B, ldS, e};
    };
    auto ep = [&](T* o0, double acc0, double id0) { return epilogue_plain(o0, ldS, acc0, id0); };
    switch (method) {
        case HP_METHOD_SM: {
            EpilogueT<T> e = ep(S[0], -1.0, 1.0);
            e.out[1] = S[1]; e.ldo[1] = ldS; e.acc_c[1] = -1.0; e.id[1] = 2.0;
            c = describe_residual(pl, b, Xk, e, out, c);
            return describe_update(pl, b, S[1], Xk, Xn, Xh, stab, partials, S[2], out, c);
        }
        case HP_METHOD_CM: {
            EpilogueT<T> e = ep(S[0], -1.0, 1.0);
            e.out[1] = S[1]; e.ldo[1] = ldS; e.acc_c[1] = -1.0; e.id[1] = 3.0;
            e.out[2] = S[2]; e.ldo[2] = ldS; e.acc_c[2] = 1.0;
            c = describe_residual(pl, b, Xk, e, out, c);
            sq(S[2], S[1], ep(S[3], -1.0, 3.0));
            return describe_update(pl, b, S[3], Xk, Xn, Xh, stab, partials, S[1], out, c);
        }
        case HP_METHOD_FM: {
            c = describe_residual(pl, b, Xk, ep(S[0], -1.0, 1.0), out, c);
            EpilogueT<T> e2 = ep(S[1], 1.0, 0.0);
            e2.out[1] = S[2]; e2.ldo[1] = ldS; e2.acc_c[1] = 1.0; e2.id[1] = 1.0; e2.g1[1] = 1.0;
            e2.D1 = S[0]; e2.ld1 = ldS;
            sq(S[0], S[0], e2);
            EpilogueT<T> e3 = ep(S[3], 1.0, 0.0);
            e3.g1[0] = 1.0; e3.D1 = S[0]; e3.ld1 = ldS;
            sq(S[1], S[1], e3);
            sq(S[3], S[2], ep(S[4], 1.0, 1.0));
            return describe_update(pl, b, S[4], Xk, Xn, Xh, stab, partials, S[1], out, c);
        }
        case HP_METHOD_HM: {
            c = describe_residual(pl, b, Xk, ep(S[0], -1.0, 1.0), out, c);
            EpilogueT<T> e2 = ep(S[1], 1.0, 0.0);
            e2.out[1] = S[2]; e2.ldo[1] = ldS; e2.acc_c[1] = 1.0; e2.id[1] = 1.0; e2.g1[1] = -1.0;
            e2.out[2] = S[3]; e2.ldo[2] = ldS; e2.acc_c[2] = 1.0; e2.id[2] = 1.0; e2.g1[2] = 1.0;
            e2.D1 = S[0]; e2.ld1 = ldS;
            sq(S[0], S[0], e2);                       // R^2, F2, F3
            sq(S[1], S[0], ep(S[4], 1.0, 0.0));       // R^3
            EpilogueT<T> e4{};
            e4.out[0] = S[5]; e4.ldo[0] = ldS; e4.acc_c[0] = 1.0; e4.id[0] = 1.0; e4.g1[0] = -1.0;
            e4.out[1] = S[6]; e4.ldo[1] = ldS; e4.acc_c[1] = 1.0; e4.id[1] = 1.0; e4.g1[1] = 1.0;
            e4.D1 = S[4]; e4.ld1 = ldS;
            sq(S[4], S[4], e4);                       // F4, F5
            EpilogueT<T> e5 = ep(S[1], 1.0, 0.0);
            e5.g1[0] = 1.0; e5.D1 = S[2]; e5.ld1 = ldS;
            sq(S[0], S[2], e5);                       // G = (I + R) F2
            sq(S[1], S[3], ep(S[4], 1.0, 0.0));       // G F3
            sq(S[4], S[5], ep(S[1], 1.0, 0.0));       // G F3 F4
            sq(S[1], S[6], ep(S[4], 1.0, 0.0));       // G F3 F4 F5
            return describe_update(pl, b, S[4], Xk, Xn, Xh, stab, partials, S[1], out, c);
        }
        default:
            break;
    }
    // PM
    const PMConst K = pm_const();
    T* R = S[0];
    T* R2 = S[1];
    T* R4 = S[2];
    T* F1 = S[3];
    T* F2 = S[4];
    T* Tm = S[5];
    T* Sm = S[6];
    T* V = F1;  // F1, F2 are dead once T and S exist
    T* W = F2;
    c = describe_residual(pl, b, Xk, ep(R, -1.0, 1.0), out, c);
    sq(R, R, ep(R2, 1.0, 0.0));
    {
        EpilogueT<T> e{};
        e.out[0] = R4; e.ldo[0] = ldS; e.acc_c[0] = 1.0;
        e.out[1] = F1; e.ldo[1] = ldS; e.acc_c[1] = 1.0; e.id[1] = 1.0; e.g1[1] = K.c1;
        e.out[2] = F2; e.ldo[2] = ldS; e.acc_c[2] = 1.0; e.id[2] = 1.0; e.g1[2] = K.c2;
        e.D1 = R2; e.ld1 = ldS;
        sq(R2, R2, e);
    }
    {
        EpilogueT<T> e{};
        e.out[0] = Tm; e.ldo[0] = ldS; e.acc_c[0] = 1.0; e.g1[0] = K.c3;
        e.out[1] = Sm; e.ldo[1] = ldS; e.acc_c[1] = 1.0; e.g1[1] = K.d1; e.g2[1] = K.d2;
        e.D1 = R2; e.ld1 = ldS; e.D2 = R4; e.ld2 = ldS;
        sq(F1, F2, e);
    }
    {
        EpilogueT<T> e{};
        e.out[0] = V; e.ldo[0] = ldS; e.acc_c[0] = 1.0; e.g1[0] = K.mu; e.g2[0] = K.psi;
        e.D1 = R2; e.ld1 = ldS; e.D2 = R4; e.ld2 = ldS;
        sq(Tm, Sm, e);
    }
    {
        EpilogueT<T> e{};
        e.out[0] = W; e.ldo[0] = ldS; e.acc_c[0] = 1.0; e.g1[0] = 1.0;
        e.D1 = V; e.ld1 = ldS;
        sq(R, V, e);
    }
    // the middle product goes to R^2's buffer (dead by now) so that R stays
    // available after the loop
    return describe_update(pl, b, W, Xk, Xn, Xh, stab, partials, R2, out, c);
}

// A plain loop of `method` whose residual R = I - A X_k (or I - X_k A) is
// already in S[0] (formed by PM's first product): out[0] is that product (not
// to be run again), the rest complete the loop. SM: X_k + X_k R; CM: W = I +
// R + R^2 formed in one product, then X_k W; FM, PM: their own products after
// the residual.
template <typename T>
int describe_after_residual(int method, const Plan& pl, const Set<T>& b, T* Xk, T* Xn,
                            double* partials, GemmCall<T> out[kMaxLoopGemms]) {
    if (method != HP_METHOD_SM && method != HP_METHOD_CM)
        return describe_loop(method, pl, b, Xk, Xn, b.X[2], false, partials, out);
    T* const* S = b.S;
    const int64_t sd = pl.s, ldS = b.ldS;
    int c = describe_residual(pl, b, Xk, epilogue_plain(S[0], ldS, -1.0, 1.0), out, 0);
    if (method == HP_METHOD_SM)
        return describe_update(pl, b, S[0], Xk, Xn, b.X[2], false, partials, S[2], out, c, true);
    EpilogueT<T> e = epilogue_plain(S[1], ldS, 1.0, 1.0);
    e.g1[0] = 1.0; e.D1 = S[0]; e.ld1 = ldS;
    e.sym = 1;
    out[c++] = {sd, sd, sd, S[0], ldS, S[0], ldS, e};
    return describe_update(pl, b, S[1], Xk, Xn, b.X[2], false, partials, S[2], out, c);
}

// The polynomial of one loop in the delta form, an exact re-association of
// the products of Section 2: with R = I - A X_k (or I - X_k A) already in
// S[0], it forms W' = W - I without rounding any value of the form
// I + (small): (I + a)(I + b) = I + a + b + a b, so each product forms a b and
// its epilogue adds a + b. For PM, with F1' = c1 R^2 + R^4 and
// F2' = c2 R^2 + R^4 (F1 = I + F1', F2 = I + F2'):
//   M' = F1' F2' + F1' + F2' = acc + (c1 + c2) R^2 + 2 R^4   (never stored),
//   T' = M' + c3 R^2,   S' = M' + d1 R^2 + d2 R^4,
//   V' = T' S' + T' + S' + mu R^2 + psi R^4 = T' S' + U,
//   W' = (I + R)(I + V') - I = R V' + R + V',
// where the M product's epilogue writes T', S' and U (in its accumulator and
// R^2, R^4; U over R^4, which each element reads before it writes). Other
// schemes: SM W' = R (no product); CM W' = R R + R; FM zeta' = R R + R,
// upsilon = R^2 R^2 + R, W' = upsilon zeta' + upsilon. The update
// X_{k+1} = X_k + X_k W' (or X_k + W' X_k) is the caller's. Appends to out;
// returns the number of products; *Wd is the buffer holding W' (S[0] for SM).
template <typename T>
int describe_delta_poly(int method, const Plan& pl, const Set<T>& b, GemmCall<T>* out, T** Wd) {
    const int64_t sd = pl.s, ldS = b.ldS;
    T* const* S = b.S;
    int c = 0;
    auto sq = [&](const T* A, const T* B, const EpilogueT<T>& e) {
        out[c++] = {sd, sd, sd, A, ldS, B, ldS, e};
    };
    auto out_to = [&](EpilogueT<T>& e, int o, T* buf, double acc, double g1, double g2) {
        e.out[o] = buf; e.ldo[o] = ldS; e.acc_c[o] = acc; e.g1[o] = g1; e.g2[o] = g2;
    };
    T* R = S[0];
    if (method == HP_METHOD_SM) {
        *Wd = R;
        return 0;
    }
    if (method == HP_METHOD_CM) {
        EpilogueT<T> e{};
        out_to(e, 0, S[1], 1.0, 1.0, 0.0);
        e.D1 = R; e.ld1 = ldS;
        sq(R, R, e);
        *Wd = S[1];
        return c;
    }
    if (method == HP_METHOD_FM) {
        EpilogueT<T> e2{};
        out_to(e2, 0, S[1], 1.0, 0.0, 0.0);   // R^2
        out_to(e2, 1, S[2], 1.0, 1.0, 0.0);   // zeta' = R^2 + R
        e2.D1 = R; e2.ld1 = ldS;
        sq(R, R, e2);
        EpilogueT<T> e4{};
        out_to(e4, 0, S[3], 1.0, 1.0, 0.0);   // upsilon = R^4 + R
        e4.D1 = R; e4.ld1 = ldS;
        sq(S[1], S[1], e4);
        EpilogueT<T> ew{};
        out_to(ew, 0, S[4], 1.0, 1.0, 0.0);   // W' = upsilon zeta' + upsilon
        ew.D1 = S[3]; ew.ld1 = ldS;
        sq(S[3], S[2], ew);
        *Wd = S[4];
        return c;
    }
    // PM
    const PMConst K = pm_const();
    T* R2 = S[1];
    T* R4 = S[2];
    T* F1 = S[3];
    T* F2 = S[4];
    T* Tm = S[5];
    T* Sm = S[6];
    T* U = R4;  // written over R^4 by the product that last reads it
    T* V = F1;  // F1', F2' are dead once T', S', U exist
    T* W = F2;
    sq(R, R, epilogue_plain(R2, ldS));
    {
        EpilogueT<T> e{};
        out_to(e, 0, R4, 1.0, 0.0, 0.0);
        out_to(e, 1, F1, 1.0, K.c1, 0.0);
        out_to(e, 2, F2, 1.0, K.c2, 0.0);
        e.D1 = R2; e.ld1 = ldS;
        sq(R2, R2, e);
    }
    {
        const double c12 = K.c1 + K.c2;
        EpilogueT<T> e{};
        out_to(e, 0, Tm, 1.0, c12 + K.c3, 2.0);
        out_to(e, 1, Sm, 1.0, c12 + K.d1, 2.0 + K.d2);
        out_to(e, 2, U, 2.0, 2.0 * c12 + K.c3 + K.d1 + K.mu, 4.0 + K.d2 + K.psi);
        e.D1 = R2; e.ld1 = ldS; e.D2 = R4; e.ld2 = ldS;
        sq(F1, F2, e);
    }
    {
        EpilogueT<T> e{};
        out_to(e, 0, V, 1.0, 1.0, 0.0);
        e.D1 = U; e.ld1 = ldS;
        sq(Tm, Sm, e);
    }
    {
        EpilogueT<T> e{};
        out_to(e, 0, W, 1.0, 1.0, 1.0);
        e.D1 = R; e.ld1 = ldS; e.D2 = V; e.ld2 = ldS;
        sq(R, V, e);
    }
    *Wd = W;
    return c;
}

// Power-iteration steps of HP_ALPHA_SIGMA_MAX2.
constexpr int kPowerIters = 50;

// Forms X0 = alpha G (Section 4) in the FP64 iterate b64.X[0] on stream s
// (products go through `gemm`), synchronises, and returns alpha.
template <typename GemmFn>
int setup_x0(const hp_params* p, const Plan& pl, const Buffers& bf, const double* A, int64_t lda,
             const double* X0, int64_t ldx0, double* host_scal, hipStream_t s, GemmFn&& gemm,
             double* alpha_out) {
    const int64_t m = pl.m, n = pl.n;
    const Set<double>& b = bf.b64;
    HIPCHK(hipMemcpy2DAsync(b.A, b.ldA * sizeof(double), A, lda * sizeof(double),
                            n * sizeof(double), m, hipMemcpyDeviceToDevice, s));
    double* X0w = b.X[0];
    if (X0) {
        HIPCHK(hipMemcpy2DAsync(X0w, b.ldX * sizeof(double), X0, ldx0 * sizeof(double),
                                m * sizeof(double), n, hipMemcpyDeviceToDevice, s));
        *alpha_out = p->alpha > 0.0 ? p->alpha : 1.0;
        return HP_OK;
    }
    if (p->alpha_rule == HP_ALPHA_USER || p->alpha_rule == HP_ALPHA_DIAG) {
        host_scal[SLOT_ALPHA] = p->alpha_rule == HP_ALPHA_DIAG ? 1.0 : p->alpha;
        HIPCHK(hipMemcpyAsync(bf.scal + SLOT_ALPHA, host_scal + SLOT_ALPHA, sizeof(double),
                              hipMemcpyHostToDevice, s));
    }
    if (p->kind == HP_KIND_MOORE_PENROSE) {
        if (p->alpha_rule == HP_ALPHA_NORM1INF)
            HIPCHK(alpha_norm1inf(b.A, b.ldA, m, n, bf.small, bf.scal, s));
        else if (p->alpha_rule == HP_ALPHA_SIGMA_MAX2)
            HIPCHK(alpha_sigma_max2(b.A, b.ldA, m, n, kPowerIters, bf.small, bf.scal, s));
        if (p->alpha_rule == HP_ALPHA_DIAG)
            HIPCHK(diag_inv(b.A, b.ldA, n, X0w, b.ldX, s));  // (choice3), Example 8.3
        else
            HIPCHK(transpose_scale(b.A, b.ldA, m, n, X0w, b.ldX, bf.scal + SLOT_ALPHA, s));
    } else {
        // G = A^l by repeated products, alpha = 1/Tr(A^{l+1}) = 1/Tr(A^l A)
        const double* P = b.A;
        int64_t ldp = b.ldA;
        double* pp[2] = {b.S[0], b.S[1]};
        for (int i = 1; i < p->drazin_l; ++i) {
            double* dst = pp[i & 1];
            GemmCall<double> g{n, n, n, P, ldp, b.A, b.ldA, epilogue_plain(dst, b.ldS)};
            CHK(gemm(g));
            P = dst;
            ldp = b.ldS;
        }
        if (p->alpha_rule == HP_ALPHA_TRACE)
            HIPCHK(alpha_trace(P, ldp, b.A, b.ldA, n, bf.small, bf.scal, s));
        HIPCHK(scale(P, ldp, n, n, X0w, b.ldX, bf.scal + SLOT_ALPHA, s));
    }
    HIPCHK(hipMemcpyAsync(host_scal, bf.scal, sizeof(double) * SLOT_COUNT, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *alpha_out = host_scal[SLOT_ALPHA];
    return HP_OK;
}

// Moore-Penrose only, on entering the FP64 stage from a lower one:
//     X <- (X A)^T X (A X)^T = A^T X^T X X^T A^T
// in FP64, which removes the components of X outside R(A^T) x R(A) that
// rounding in the lower stages left behind and that the loops of (PM) do not
// correct (first-order analysis in the proof of Theorem 6.2: the off-diagonal
// error blocks are carried unchanged). This step is not part of the paper: it
// applies the third and fourth Penrose equations ((AX)^T = AX, (XA)^T = XA),
// which the Moore-Penrose inverse satisfies. Associated so that every
// intermediate is min(m, n) square; X is b64.X[xi] in and out. A square
// nonsingular input has no such blocks and skips it (see needs_projection).
template <typename GemmFn>
int project_mp(const Plan& pl, const Buffers& bf, int xi, hipStream_t s, GemmFn&& gemm) {
    const int64_t m = pl.m, n = pl.n;
    const Set<double>& b = bf.b64;
    // only plans with lower-precision stages carry the projection buffers
    if (!pl.has_proj || !bf.At || !bf.Xt || xi < 0 || xi > 2) return HP_EINVAL;
    double* X = b.X[xi];
    HIPCHK(transpose_scale(b.A, b.ldA, m, n, bf.At, b.ldX, nullptr, s));  // A^T: n x m
    HIPCHK(transpose_scale(X, b.ldX, n, m, bf.Xt, b.ldA, nullptr, s));    // X^T: m x n
    if (m > n) {
        // (A^T X^T)(X X^T) A^T with n x n intermediates
        CHK(gemm(GemmCall<double>{n, n, m, bf.At, b.ldX, bf.Xt, b.ldA, epilogue_plain(b.S[0], b.ldS)}));
        CHK(gemm(GemmCall<double>{n, n, m, X, b.ldX, bf.Xt, b.ldA, epilogue_plain(b.S[1], b.ldS)}));
        CHK(gemm(GemmCall<double>{n, n, n, b.S[0], b.ldS, b.S[1], b.ldS, epilogue_plain(b.S[2], b.ldS)}));
        CHK(gemm(GemmCall<double>{n, m, n, b.S[2], b.ldS, bf.At, b.ldX, epilogue_plain(X, b.ldX)}));
    } else {
        // A^T (X^T X)(X^T A^T) with m x m intermediates
        CHK(gemm(GemmCall<double>{m, m, n, bf.Xt, b.ldA, X, b.ldX, epilogue_plain(b.S[0], b.ldS)}));
        CHK(gemm(GemmCall<double>{m, m, n, bf.Xt, b.ldA, bf.At, b.ldX, epilogue_plain(b.S[1], b.ldS)}));
        CHK(gemm(GemmCall<double>{m, m, m, b.S[0], b.ldS, b.S[1], b.ldS, epilogue_plain(b.S[2], b.ldS)}));
        CHK(gemm(GemmCall<double>{n, m, m, bf.At, b.ldX, b.S[2], b.ldS, epilogue_plain(X, b.ldX)}));
    }
    return HP_OK;
}

// Whether the projection is needed on entering the FP64 stage: always for a
// non-square input; for a square one only if it is rank deficient, read off
// the last lower-stage residual R = I - A X (or I - X A): its squared
// Frobenius norm is about the number of directions X does not invert (each
// contributes 1) and is small for a nonsingular input. Synchronises `s`.
inline int needs_projection(const Plan& pl, const Buffers& bf, double* host_scal, hipStream_t s,
                            bool* out) {
    *out = false;
    if (!pl.has_proj) return HP_OK;
    if (pl.m != pl.n) {
        *out = true;
        return HP_OK;
    }
    HIPCHK(sumsq(bf.b32.S[0], bf.b32.ldS, pl.s, pl.s, bf.small, bf.scal, SLOT_RNORM2, s));
    HIPCHK(hipMemcpyAsync(host_scal + SLOT_RNORM2, bf.scal + SLOT_RNORM2, sizeof(double),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = !(host_scal[SLOT_RNORM2] < 0.5);
    return HP_OK;
}

}  // namespace hp
