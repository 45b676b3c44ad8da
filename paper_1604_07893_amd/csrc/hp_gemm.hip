// MFMA GEMM with the fused hyperpower epilogue, for gfx950 (CDNA4, wave64).
//
// C = epilogue(A * B), A M x K, B K x N, row-major, T = double
// (v_mfma_f64_16x16x4f64, FP64 accumulate) or T = float
// (v_mfma_f32_16x16x4f32, FP32 accumulate).
//
// Block tile BM x BN, K-tile BK, each wave a WM x WN sub-tile of 16x16 MFMA
// accumulators. A and B are read with 16-byte loads along their contiguous
// rows into registers one K-tile ahead and written, as 16-byte vectors, to
// double-buffered LDS in the layout they were read in (A m-major, B k-major),
// rows padded so that a fragment read spreads over the banks. One barrier per
// K-tile. Products with too few output tiles to occupy the chip can split K
// over 2 or 4 blocks per tile; the last block of a tile to finish adds the
// partial tiles in a fixed order, so the result does not depend on which
// block finishes last.
// Large FP64 products (from 512 output tiles) run instead on k_gemm_w4dma:
// 4 waves of 64 x 64 per 128 x 128 tile, tiles brought to LDS by the
// load-to-LDS instruction, two blocks per CU; large FP32 products (from 256
// tiles of 256 x 256) on k_gemm_w4dma_f32, 4 waves of 128 x 128 per tile.
// The epilogue forms up to three outputs
//     out_o = id_o * I + acc_o * (A B) + g1_o * D1 + g2_o * D2
// (the linear combinations of one loop of iteration (PM), Section 2) and,
// optionally, per-block FP64 partial sums of (out_0 - ref)^2 and ref^2 for the
// stopping test of Section 4.
#include "hp_gemm_common.h"
#include "hp_internal.h"
#include "hp_symk.h"

#include <atomic>
#include <type_traits>

namespace hp {
namespace {


template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef dbl4 acc_t;
    static __device__ inline acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // accumulator register r of lane l holds row (l/16) + 4r, column l%16
    static __device__ inline int row(int g, int r) { return g + 4 * r; }
};

template <>
struct Mfma<float> {
    typedef flt4 acc_t;
    static __device__ inline acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator register r of lane l holds row 4(l/16) + r, column l%16
    static __device__ inline int row(int g, int r) { return 4 * g + r; }
};

template <typename T>
struct Vec16;  // 16 bytes of T
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};


template <typename T, int BM, int BN, int BK, int WM, int WN>
struct Cfg {
    static constexpr int WAVES = (BM / WM) * (BN / WN);
    static constexpr int NT = 64 * WAVES;
    static constexpr int V = Vec16<T>::n;
    static constexpr int PAD = 16;
    // A is kept as read, As[m][k], rows padded by one 16-byte vector: the 16
    // lanes of a fragment read (16 rows, one k) fall on distinct banks and the
    // staging writes are whole 16-byte vectors.
    static constexpr int LDA_S = BK + V;
    static constexpr int LDB_S = BN + PAD;
    // A tile: BM rows of BK elements, BK/V threads per row
    static constexpr int A_TPR = BK / V;
    static constexpr int A_RPP = NT / A_TPR;
    static constexpr int A_PASS = BM / A_RPP;
    // B tile: BK rows of BN elements, BN/V threads per row
    static constexpr int B_TPR = BN / V;
    static constexpr int B_RPP = NT / B_TPR;
    static constexpr int B_PASS = BK / B_RPP;
    static constexpr int TI = WM / 16, TJ = WN / 16;
    static_assert(BM % WM == 0 && BN % WN == 0 && WM % 16 == 0 && WN % 16 == 0, "wave tiling");
    static_assert(BK % 4 == 0 && BK % V == 0, "K tile");
    static_assert(NT % A_TPR == 0 && A_RPP > 0 && BM % A_RPP == 0 && A_PASS >= 1, "A loads");
    static_assert(NT % B_TPR == 0 && B_RPP > 0 && BK % B_RPP == 0 && B_PASS >= 1, "B loads");
    static constexpr size_t LDS_BYTES = 2 * ((size_t)BM * LDA_S + (size_t)BK * LDB_S) * sizeof(T);
};

// The fused epilogue of a BM x BN tile held as TI x TJ MFMA accumulators per
// wave: up to three outputs id*I + acc_c*acc + g1*D1 + g2*D2 (output 0 chopped
// with ep.chop) and, with ep.ref, the block's FP64 partial sums of the stopping
// test in pair `part`.
// With SYM (a symmetric product, EpilogueT::sym), only the elements on and
// above the diagonal are formed, each stored at (row, col) and (col, row).
template <typename T, int TI, int TJ, int WAVES, bool SYM = false>
__device__ __attribute__((always_inline)) inline void tile_epilogue(
    typename Mfma<T>::acc_t (&acc)[TI][TJ], const EpilogueT<T>& ep, int M, int N, int bm, int bn,
    int wm, int wn, int part, double (*red)[WAVES]) {
    int tid = threadIdx.x;
    // in the stream-K loop, values derived from the thread index would
    // otherwise be computed once before the loop and held through it
    if constexpr (SYM) asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int fr = lane & 15, fg = lane >> 4;
    double s_diff = 0.0, s_ref = 0.0;
    // Per 16 x 16 accumulator, the reads of its 4 elements (D1, D2 and the
    // stopping test's reference) are all issued before any of its stores, so
    // that a lane waits once per accumulator rather than once per element.
    // An element reads those inputs only at its own position, so reading them
    // ahead of the other elements' stores changes no value.
#pragma unroll
    for (int i = 0; i < TI; ++i) {
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int col = bn + wn + j * 16 + fr;
            T d1[4], d2[4];
            double x0[4];
            bool ok[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = bm + wm + i * 16 + Mfma<T>::row(fg, r);
                ok[r] = row < M && col < N && (!SYM || row <= col);
                d1[r] = ok[r] && ep.D1 ? ep.D1[(int64_t)row * ep.ld1 + col] : T(0);
                d2[r] = ok[r] && ep.D2 ? ep.D2[(int64_t)row * ep.ld2 + col] : T(0);
                x0[r] = !SYM && ok[r] && ep.ref && ep.out[0] ? (double)ep.ref[(int64_t)row * ep.ldref + col]
                                                            : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = bm + wm + i * 16 + Mfma<T>::row(fg, r);
                if (ok[r]) {
                    const T a = acc[i][j][r];
#pragma unroll
                    for (int o = 0; o < 3; ++o) {
                        if (ep.out[o]) {
                            T v = T(ep.acc_c[o]) * a;
                            if (row == col && ep.id[o] != 0.0) v += T(ep.id[o]);
                            if (ep.D1 && ep.g1[o] != 0.0) v += T(ep.g1[o]) * d1[r];
                            if (ep.D2 && ep.g2[o] != 0.0) v += T(ep.g2[o]) * d2[r];
                            if (o == 0 && ep.chop > 0.0 && fabs((double)v) < ep.chop) v = T(0);
                            ep.out[o][(int64_t)row * ep.ldo[o] + col] = v;
                            if (SYM && row != col) ep.out[o][(int64_t)col * ep.ldo[o] + row] = v;
                            if (!SYM && o == 0 && ep.ref) {
                                const double df = (double)v - x0[r];
                                s_diff += df * df;
                                s_ref += x0[r] * x0[r];
                            }
                        }
                    }
                }
            }
        }
    }
    if (!SYM && ep.ref) {
        const double sd = wave_sum(s_diff), sr = wave_sum(s_ref);
        if (lane == 0) {
            red[0][wave] = sd;
            red[1][wave] = sr;
        }
        __syncthreads();
        if (tid == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < WAVES; ++w) {
                a += red[0][w];
                b += red[1][w];
            }
            ep.partials[2 * part] = a;
            ep.partials[2 * part + 1] = b;
        }
    }
}

// Stream-K: the block holds piece `split` (in K order) of the sk_np pieces of
// output tile `part`; piece 0's partial tile is slot sk_slot0 of
// ep.split_part and piece i > 0's is slot 2 (sk_b0 + i). As the split-K path
// of gemm_tile, with a tile-dependent piece count: every piece is stored, and
// the last block to arrive reads them all back and adds them in K order (the
// same bits whichever block is last) into acc and returns true; the other
// blocks return false (uniformly over the block). A tile in one piece
// returns true at once.
template <typename T, int TI, int TJ, int NT, int TILE>
__device__ inline bool streamk_gather(typename Mfma<T>::acc_t (&acc)[TI][TJ], const EpilogueT<T>& ep,
                                      int tid, int part, int split, int sk_np, int sk_slot0, int sk_b0) {
    if (sk_np <= 1) return true;
    static_assert(TILE == TI * TJ * 4 * NT, "partial layout");
    auto slot = [&](int i) {
        return ep.split_part + (int64_t)(i == 0 ? sk_slot0 : 2 * (sk_b0 + i)) * TILE;
    };
    __shared__ unsigned sk_arrived;
    T* mine = slot(split);
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) mine[((i * TJ + j) * 4 + r) * NT + tid] = acc[i][j][r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        sk_arrived = __hip_atomic_fetch_add(&ep.split_cnt[part], 1u, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (sk_arrived != (unsigned)(sk_np - 1)) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            asm volatile("" ::: "memory");
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = ((i * TJ + j) * 4 + r) * NT + tid;
                T v = slot(0)[e];
                for (int q = 1; q < sk_np; ++q) v += slot(q)[e];
                asm volatile("" : "+v"(v));
                acc[i][j][r] = v;
            }
        }
    if (tid == 0) __hip_atomic_store(&ep.split_cnt[part], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// One BM x BN output tile (tm, tn) of C = epilogue(A * B); the block's
// partial sums (if any) go to pair `part` of ep.partials. SPLIT < 0 (the
// stream-K launch): the block holds piece `split` (in K order) of the
// sk_np pieces of tile `part`; piece 0's partial tile is slot sk_slot0 of
// ep.split_part and piece i > 0's is slot 2 (sk_b0 + i).
template <typename T, int BM, int BN, int BK, int WM, int WN, int PF = 1, int SPLIT = 1,
          bool SYM = false>
__device__ inline void gemm_tile(int M, int N, int K, const T* __restrict__ A, int64_t lda,
                                 const T* __restrict__ B, int64_t ldb, const EpilogueT<T>& ep,
                                 int tm, int tn, int part, int split = 0, int sk_np = 1,
                                 int sk_slot0 = 0, int sk_b0 = 0) {
    using C = Cfg<T, BM, BN, BK, WM, WN>;
    using VT = typename Vec16<T>::type;
    using ACC = typename Mfma<T>::acc_t;
    constexpr int V = C::V;
    __shared__ __attribute__((aligned(16))) T As[2][BM][C::LDA_S];
    __shared__ __attribute__((aligned(16))) T Bs[2][BK][C::LDB_S];
    __shared__ double red[2][C::WAVES];

    int tid = threadIdx.x;
    if constexpr (SPLIT < 0) asm volatile("" : "+v"(tid));  // as in tile_epilogue
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int bm = tm * BM, bn = tn * BN;
    const int wm = (wave / (BN / WN)) * WM, wn = (wave % (BN / WN)) * WN;

    // Global -> register staging. Every load is issued unconditionally from an
    // address that is always inside the operand (out-of-range rows/columns are
    // redirected to element 0) so the loads of a K-tile go out back to back;
    // out-of-range elements are zeroed when the registers are written to LDS.
    // Two register sets: the loads of K-tile t+2 are issued while tile t is
    // multiplied, so each load has two tiles of MFMA work to arrive.
    const int a_k = V * (tid % C::A_TPR), a_r = tid / C::A_TPR;
    const int b_n = V * (tid % C::B_TPR), b_k = tid / C::B_TPR;
    VT ra[PF][C::A_PASS], rb[PF][C::B_PASS];
    const T* a_ptr[C::A_PASS];
    bool a_row_ok[C::A_PASS];
#pragma unroll
    for (int p = 0; p < C::A_PASS; ++p) {
        const int row = bm + a_r + C::A_RPP * p;
        a_row_ok[p] = row < M;
        a_ptr[p] = A + (int64_t)(a_row_ok[p] ? row : 0) * lda + a_k;
    }
    const int b_col = bn + b_n;
    const bool b_col_ok = b_col < N;
    const T* b_ptr = B + (b_col_ok ? b_col : 0) + (int64_t)b_k * ldb;

    auto load = [&](int set, int k0) {
        const bool ka = k0 + a_k < K;
#pragma unroll
        for (int p = 0; p < C::A_PASS; ++p) {
            const T* src = (a_row_ok[p] && ka) ? a_ptr[p] + k0 : A;
            ra[set][p] = *reinterpret_cast<const VT*>(src);
        }
#pragma unroll
        for (int p = 0; p < C::B_PASS; ++p) {
            const int kr = k0 + b_k + C::B_RPP * p;
            const T* src = (b_col_ok && kr < K) ? b_ptr + (int64_t)(k0 + C::B_RPP * p) * ldb : B;
            rb[set][p] = *reinterpret_cast<const VT*>(src);
        }
    };
    auto store = [&](int set, int buf, int k0) {
#pragma unroll
        for (int p = 0; p < C::A_PASS; ++p) {
            VT v = ra[set][p];
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (!(a_row_ok[p] && (k0 + a_k + e < K))) v[e] = T(0);
            *reinterpret_cast<VT*>(&As[buf][a_r + C::A_RPP * p][a_k]) = v;
        }
#pragma unroll
        for (int p = 0; p < C::B_PASS; ++p) {
            const bool krow = k0 + b_k + C::B_RPP * p < K;
            VT v = rb[set][p];
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (!(krow && b_col + e < N)) v[e] = T(0);
            *reinterpret_cast<VT*>(&Bs[buf][b_k + C::B_RPP * p][b_n]) = v;
        }
    };

    ACC acc[C::TI][C::TJ];
#pragma unroll
    for (int i = 0; i < C::TI; ++i)
#pragma unroll
        for (int j = 0; j < C::TJ; ++j) acc[i][j] = ACC{};

    const int fr = lane & 15, fg = lane >> 4;
    const int nk = (K + BK - 1) / BK;
    if constexpr (PF == 1) {
        // One K-tile ahead: tile kt+1 is loaded into registers while tile kt
        // is multiplied. Each k-step q gives lane group fg the k = 4q + fg.
        auto compute = [&](int buf) {
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                T a[C::TI], b[C::TJ];
#pragma unroll
                for (int i = 0; i < C::TI; ++i) a[i] = As[buf][wm + i * 16 + fr][ks + fg];
#pragma unroll
                for (int j = 0; j < C::TJ; ++j) b[j] = Bs[buf][ks + fg][wn + j * 16 + fr];
#pragma unroll
                for (int i = 0; i < C::TI; ++i)
#pragma unroll
                    for (int j = 0; j < C::TJ; ++j) acc[i][j] = Mfma<T>::mma(a[i], b[j], acc[i][j]);
            }
        };
        load(0, 0);
        store(0, 0, 0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) load(0, (kt + 1) * BK);
            compute(cur);
            if (kt + 1 < nk) store(0, cur ^ 1, (kt + 1) * BK);
            __syncthreads();
        }
    } else {
        // Two K-tiles ahead, with the LDS reads spread over the MFMAs (for
        // blocks that have a compute unit to themselves and must hide their
        // own latencies). k-step q gives lane group fg the k = NQ*fg + q, so
        // the V steps of a fragment group are V consecutive elements of a row
        // of A (one 16-byte LDS read) and of V consecutive rows of B; a K-tile
        // is NG groups. The fragments of group g+1 are read while the MFMAs of
        // group g run; the block synchronises before the last group, so the
        // first group of the next tile is read while the last MFMAs of this
        // one run. The scheduling barriers keep the compiler from gathering
        // the LDS reads back together. Until stored, tile t sits in register
        // set t % 2; the loop body takes an even and an odd tile so both sets
        // are indexed statically. The loads are issued for every tile, also
        // past the end of K (they then read element 0 and are never stored):
        // with the same loads on every path the compiler's wait before a
        // store covers only the older set, not the loads just issued.
        constexpr int NQ = BK / 4, NG = NQ / V;
        static_assert(NQ % V == 0 && NG >= 2, "fragment groups");
        // tile kt+1 goes to LDS after the MFMAs of group STORE_G (its buffer
        // was last read before the previous barrier, its loads were issued a
        // tile earlier), so the LDS writes overlap MFMAs instead of sitting
        // in front of the barrier
        constexpr int STORE_G = NG > 2 ? 1 : NG - 1;
        VT fa[2][C::TI];
        T fb[2][C::TJ][V];
        auto frag = [&](int buf, int g, int slot) {
            const int k = NQ * fg + V * g;
#pragma unroll
            for (int i = 0; i < C::TI; ++i)
                fa[slot][i] = *reinterpret_cast<const VT*>(&As[buf][wm + i * 16 + fr][k]);
#pragma unroll
            for (int j = 0; j < C::TJ; ++j)
#pragma unroll
                for (int e = 0; e < V; ++e) fb[slot][j][e] = Bs[buf][k + e][wn + j * 16 + fr];
        };
        auto mma = [&](int slot) {
#pragma unroll
            for (int e = 0; e < V; ++e)
#pragma unroll
                for (int i = 0; i < C::TI; ++i)
#pragma unroll
                    for (int j = 0; j < C::TJ; ++j)
                        acc[i][j] = Mfma<T>::mma(fa[slot][i][e], fb[slot][j][e], acc[i][j]);
        };
        // register set `ld` receives tile kt+2, set `st` holds tile kt+1
        auto tile = [&](int kt, auto ld, auto st) {
            const int cur = kt & 1;
            load(decltype(ld)::value, (kt + 2) * BK);
#pragma unroll
            for (int g = 0; g + 1 < NG; ++g) {
                frag(cur, g + 1, (g + 1) & 1);
                mma(g & 1);
                if (g == STORE_G && kt + 1 < nk) store(decltype(st)::value, cur ^ 1, (kt + 1) * BK);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (STORE_G == NG - 1 && kt + 1 < nk) store(decltype(st)::value, cur ^ 1, (kt + 1) * BK);
            __syncthreads();
            if (kt + 1 < nk) frag(cur ^ 1, 0, 0);
            mma((NG - 1) & 1);
            __builtin_amdgcn_sched_barrier(0);
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        load(0, 0);
        store(0, 0, 0);
        load(1, BK);
        __syncthreads();
        frag(0, 0, 0);
        for (int kt = 0; kt < nk; kt += 2) {
            tile(kt, I0{}, I1{});
            if (kt + 1 < nk) tile(kt + 1, I1{}, I0{});
        }
    }

    if constexpr (SPLIT > 1) {
        // ---- split-K: this block holds the K-range `split` of tile `part` ----
        // Every block stores its partial tile (in accumulator order, so the
        // stores are contiguous across the block), publishes it, and counts
        // itself in; the last to arrive adds the SPLIT partials in an order
        // that does not depend on which block that is.
        constexpr int TILE = BM * BN;
        static_assert(TILE == C::TI * C::TJ * 4 * C::NT, "partial layout");
        T* slots = ep.split_part + (int64_t)part * SPLIT * TILE;
        __shared__ unsigned arrived;
#pragma unroll
        for (int i = 0; i < C::TI; ++i)
#pragma unroll
            for (int j = 0; j < C::TJ; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    slots[split * TILE + ((i * C::TJ + j) * 4 + r) * C::NT + tid] = acc[i][j][r];
        // Each thread's stores complete (workgroup release), then one thread
        // makes them all visible device-wide (an agent-scope release writes
        // back this XCD's L2) before counting the block in; an agent-scope
        // acquire after the count invalidates stale cached lines for the
        // whole block. One write-back and one invalidate per block.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            arrived = __hip_atomic_fetch_add(&ep.split_cnt[part], 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (arrived != SPLIT - 1) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
        for (int i = 0; i < C::TI; ++i)
#pragma unroll
            for (int j = 0; j < C::TJ; ++j) {
                // one fragment at a time: the empty asm statements keep the
                // compiler from issuing every fragment's loads at once (which
                // would hold them all in registers and spill)
                asm volatile("" ::: "memory");
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = ((i * C::TJ + j) * 4 + r) * C::NT + tid;
                    T v;
                    if constexpr (SPLIT == 2) {
                        // a + b == b + a exactly: same bits whichever block is last
                        v = acc[i][j][r] + slots[(split ^ 1) * TILE + e];
                    } else {
                        // all four from memory (its own as stored), summed in one order
                        v = (slots[e] + slots[TILE + e]) + (slots[2 * TILE + e] + slots[3 * TILE + e]);
                    }
                    asm volatile("" : "+v"(v));
                    acc[i][j][r] = v;
                }
            }
        if (tid == 0) __hip_atomic_store(&ep.split_cnt[part], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    if constexpr (SPLIT < 0) {
        if (!streamk_gather<T, C::TI, C::TJ, C::NT, BM * BN>(acc, ep, tid, part, split, sk_np, sk_slot0,
                                                             sk_b0))
            return;
    }

    tile_epilogue<T, C::TI, C::TJ, C::WAVES, SYM>(acc, ep, M, N, bm, bn, wm, wn, part, red);
}

template <typename T, int BM, int BN, int BK, int WM, int WN, int PF>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN)) void k_gemm(
    int M, int N, int K, const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
    int64_t ldb, EpilogueT<T> ep, int tiles_m, int tiles_n) {
    if (gate_closed(ep.gate, ep.gate_mode)) return;  // uniform over the launch
    int tm, tn;
    tile_of(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, tm, tn);
    gemm_tile<T, BM, BN, BK, WM, WN, PF>(M, N, K, A, lda, B, ldb, ep, tm, tn, blockIdx.x);
}

// Split-K launch: SPLIT consecutive (XCD-local) blocks per output tile, block
// `split` multiplying the K-range [split * kchunk, min(K, (split + 1) * kchunk)).
template <typename T, int BM, int BN, int BK, int WM, int WN, int SPLIT>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN))
__attribute__((amdgpu_waves_per_eu(4))) void k_gemm_split(
    int M, int N, int K, const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
    int64_t ldb, EpilogueT<T> ep, int tiles_m, int tiles_n, int kchunk) {
    if (gate_closed(ep.gate, ep.gate_mode)) return;  // uniform: no counter is touched
    const int p = xcd_contiguous(blockIdx.x, gridDim.x);
    const int t = p / SPLIT, split = p % SPLIT;
    int tm, tn;
    tile_of(t, tiles_m, tiles_n, tm, tn);
    const int k0 = split * kchunk;
    gemm_tile<T, BM, BN, BK, WM, WN, 1, SPLIT>(M, N, min(kchunk, K - k0), A + k0, lda,
                                               B + (int64_t)k0 * ldb, ldb, ep, tm, tn, t, split);
}

// Symmetric product (EpilogueT::sym) as one launch over the tiles on and
// above the diagonal (the partition in hp_symk.h): first `dp` tiles taken
// whole, gridDim.x at a time, then the rest as stream-K: their tiles * ipt
// K-steps (ipt = K-tiles per tile), laid end to end, cut into gridDim.x
// ranges of ipc steps, one per block. A block walks its range tile by tile;
// a tile that lies wholly in one range is finished there, one that spans
// several ranges by the last of their blocks to arrive. A block's first
// piece uses partial slot 2b and its last slot 2b + 1, so 2 * gridDim.x
// slots suffice.
template <typename T, int BM, int BN, int BK, int WM, int WN, int PF>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN)) void k_gemm_sym(
    int N, int K, const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb,
    EpilogueT<T> ep, int nt, int tiles, int ipt, int ipc, int dp) {
    static_assert(BM == 128 && BN == 128, "partial slots hold 128 x 128 tiles");
    if (gate_closed(ep.gate, ep.gate_mode)) return;  // uniform: no counter is touched
    const int b = xcd_contiguous(blockIdx.x, gridDim.x);
    for (int t = b; t < dp; t += gridDim.x) {
        int nt_p = nt;
        asm volatile("" : "+s"(nt_p));  // as below
        int tm, tn;
        sym_tile_of(t, nt_p, tm, tn);
        gemm_tile<T, BM, BN, BK, WM, WN, PF, -1, true>(N, N, K, A, lda, B, ldb, ep, tm, tn, t);
        __syncthreads();  // the next tile's staging reuses the LDS tiles
    }
    const int64_t total = (int64_t)(tiles - dp) * ipt;
    int64_t it = (int64_t)b * ipc;
    const int64_t end = min(it + (int64_t)ipc, total);
    while (it < end) {
        // the divisions below are redone per piece instead of keeping their
        // reciprocals in vector registers through the loop
        int ipt_p = ipt, ipc_p = ipc, nt_p = nt;
        asm volatile("" : "+s"(ipt_p), "+s"(ipc_p), "+s"(nt_p));
        const SymPiece pc = sym_piece(it, end, ipt_p, ipc_p, b);
        int tm, tn;
        sym_tile_of(dp + pc.t, nt_p, tm, tn);
        const int kb = pc.k0 * BK, ke = min(K, pc.k1 * BK);
        gemm_tile<T, BM, BN, BK, WM, WN, PF, -1, true>(N, N, ke - kb, A + kb, lda,
                                                      B + (int64_t)kb * ldb, ldb, ep, tm, tn,
                                                      dp + pc.t, pc.idx, pc.np, pc.slot0, pc.b0);
        it += pc.k1 - pc.k0;
        __syncthreads();  // the next piece's staging reuses the LDS tiles
    }
}

// Persistent grouped launch: the grid walks the tiles of every product in
// the table (entries in order, tiles of an entry row-major); each tile is
// computed exactly as a single launch of that product would compute it, so an
// entry's result does not depend on the other entries.
template <typename T, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN)) void k_gemm_grouped(
    const GroupHeader* __restrict__ hdr, const GroupEntry<T>* __restrict__ ents) {
    const int count = hdr->count;
    const int total = hdr->total_tiles;
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ents[mid].tile_start <= t) lo = mid;
            else hi = mid - 1;
        }
        const GroupEntry<T> g = ents[lo];
        const int local = t - g.tile_start;
        gemm_tile<T, BM, BN, BK, WM, WN>(g.M, g.N, g.K, g.A, g.lda, g.B, g.ldb, g.ep,
                                         local / g.tiles_n, local % g.tiles_n, local);
    }
}


// ---------------------------------------------------------------------------
// 16-bit MFMA GEMM on FP32 storage: C = epilogue(A * B) with A, B, C FP32 in
// memory, the operands rounded to bf16 or fp16 (round to nearest even) while
// they are staged into LDS, v_mfma_f32_16x16x32_{bf16,f16} with FP32
// accumulation. Each lane's fragment is 8 consecutive k of one row (A) or one
// column (B), so both operands are kept k-contiguous in LDS: A is written as
// read; each thread transposes a 4x4 block of B in registers.
// ---------------------------------------------------------------------------

template <int BM, int BN, int BK, int WM, int WN>
struct CfgLP {
    static constexpr int WAVES = (BM / WM) * (BN / WN);
    static constexpr int NT = 64 * WAVES;
    static constexpr int KP = BK + 8;  // LDS row pitch (16-bit elements): 16 lanes at one k hit distinct banks
    static constexpr int A_TPR = BK / 4;            // float4 loads per A row
    static constexpr int A_RPP = NT / A_TPR;
    static constexpr int A_PASS = BM / A_RPP;
    static constexpr int B_POS = (BK / 4) * (BN / 4);  // 4x4 blocks of B
    static constexpr int B_PASS = B_POS / NT;
    static constexpr int TI = WM / 16, TJ = WN / 16;
    static_assert(BK % 32 == 0, "K tile");
    static_assert((BN / 4) % 8 == 0, "B blocks");
    // 4x4 block `pos` of the B tile -> (column quad nq, k quad kq): runs of 8
    // lanes read 128 contiguous bytes of one row; the next lanes step in k so
    // the transposed 8-byte LDS writes spread over the banks.
    static __device__ inline void b_pos(int pos, int& nq, int& kq) {
        const int lo = pos % 8, rest = pos / 8;
        kq = rest % (BK / 4);
        nq = (rest / (BK / 4)) * 8 + lo;
    }
    static_assert(NT % A_TPR == 0 && BM % A_RPP == 0 && A_PASS >= 1, "A loads");
    static_assert(B_POS % NT == 0 && B_PASS >= 1, "B loads");
};

template <typename L, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN)) void k_gemm_lp(
    int M, int N, int K, const float* __restrict__ A, int64_t lda, const float* __restrict__ B,
    int64_t ldb, EpilogueT<float> ep, int tiles_m, int tiles_n) {
    using C = CfgLP<BM, BN, BK, WM, WN>;
    using FR = typename Mfma16<L>::frag_t;
    using QD = typename Mfma16<L>::quad_t;
    __shared__ __attribute__((aligned(16))) L As[2][BM][C::KP];
    __shared__ __attribute__((aligned(16))) L Bs[2][BN][C::KP];
    __shared__ double red[2][C::WAVES];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int tm, tn;
    tile_of(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, tm, tn);
    const int bm = tm * BM, bn = tn * BN;
    const int wm = (wave / (BN / WN)) * WM, wn = (wave % (BN / WN)) * WN;

    // Branch-free staging as in gemm_tile: loads from always-valid addresses,
    // masking when the registers are rounded and written to LDS.
    const int a_k = 4 * (tid % C::A_TPR), a_r = tid / C::A_TPR;
    flt4v ra[C::A_PASS];
    flt4v rb[C::B_PASS][4];
    bool a_row_ok[C::A_PASS];
    const float* a_ptr[C::A_PASS];
#pragma unroll
    for (int p = 0; p < C::A_PASS; ++p) {
        const int row = bm + a_r + C::A_RPP * p;
        a_row_ok[p] = row < M;
        a_ptr[p] = A + (int64_t)(a_row_ok[p] ? row : 0) * lda + a_k;
    }

    auto load = [&](int k0) {
        const bool ka = k0 + a_k < K;
#pragma unroll
        for (int p = 0; p < C::A_PASS; ++p)
            ra[p] = *reinterpret_cast<const flt4v*>((a_row_ok[p] && ka) ? a_ptr[p] + k0 : A);
#pragma unroll
        for (int p = 0; p < C::B_PASS; ++p) {
            int nq, kq;
            C::b_pos(tid + C::NT * p, nq, kq);
            const int c = bn + 4 * nq;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int kr = k0 + 4 * kq + r;
                const float* src = (kr < K && c < N) ? B + (int64_t)kr * ldb + c : B;
                rb[p][r] = *reinterpret_cast<const flt4v*>(src);
            }
        }
    };
    auto store = [&](int buf, int k0) {
#pragma unroll
        for (int p = 0; p < C::A_PASS; ++p) {
            QD q;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                q[e] = (a_row_ok[p] && k0 + a_k + e < K) ? (L)ra[p][e] : (L)0.f;
            *reinterpret_cast<QD*>(&As[buf][a_r + C::A_RPP * p][a_k]) = q;
        }
#pragma unroll
        for (int p = 0; p < C::B_PASS; ++p) {
            int nq, kq;
            C::b_pos(tid + C::NT * p, nq, kq);
            const int c = bn + 4 * nq;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                QD q;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool ok = (k0 + 4 * kq + r < K) && (c + cc < N);
                    q[r] = ok ? (L)rb[p][r][cc] : (L)0.f;
                }
                *reinterpret_cast<QD*>(&Bs[buf][4 * nq + cc][4 * kq]) = q;
            }
        }
    };

    flt4 acc[C::TI][C::TJ];
#pragma unroll
    for (int i = 0; i < C::TI; ++i)
#pragma unroll
        for (int j = 0; j < C::TJ; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

    const int nk = (K + BK - 1) / BK;
    load(0);
    store(0, 0);
    __syncthreads();
    const int fr = lane & 15, fg = lane >> 4;
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 32) {
            FR a[C::TI], b[C::TJ];
#pragma unroll
            for (int i = 0; i < C::TI; ++i)
                a[i] = *reinterpret_cast<const FR*>(&As[cur][wm + i * 16 + fr][ks + 8 * fg]);
#pragma unroll
            for (int j = 0; j < C::TJ; ++j)
                b[j] = *reinterpret_cast<const FR*>(&Bs[cur][wn + j * 16 + fr][ks + 8 * fg]);
#pragma unroll
            for (int i = 0; i < C::TI; ++i)
#pragma unroll
                for (int j = 0; j < C::TJ; ++j) acc[i][j] = Mfma16<L>::mma(a[i], b[j], acc[i][j]);
        }
        if (kt + 1 < nk) store(cur ^ 1, (kt + 1) * BK);
        __syncthreads();
    }

    double s_diff = 0.0, s_ref = 0.0;
#pragma unroll
    for (int i = 0; i < C::TI; ++i) {
#pragma unroll
        for (int j = 0; j < C::TJ; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = bm + wm + i * 16 + 4 * fg + r;
                const int col = bn + wn + j * 16 + fr;
                if (row < M && col < N) {
                    const float a = acc[i][j][r];
                    const float d1 = ep.D1 ? ep.D1[(int64_t)row * ep.ld1 + col] : 0.f;
                    const float d2 = ep.D2 ? ep.D2[(int64_t)row * ep.ld2 + col] : 0.f;
                    const float idv = (row == col) ? 1.f : 0.f;
#pragma unroll
                    for (int o = 0; o < 3; ++o) {
                        if (ep.out[o]) {
                            float v = (float)ep.acc_c[o] * a;
                            if (ep.id[o] != 0.0) v += (float)ep.id[o] * idv;
                            if (ep.g1[o] != 0.0) v += (float)ep.g1[o] * d1;
                            if (ep.g2[o] != 0.0) v += (float)ep.g2[o] * d2;
                            ep.out[o][(int64_t)row * ep.ldo[o] + col] = v;
                            if (o == 0 && ep.ref) {
                                const double x0 = (double)ep.ref[(int64_t)row * ep.ldref + col];
                                const double df = (double)v - x0;
                                s_diff += df * df;
                                s_ref += x0 * x0;
                            }
                        }
                    }
                }
            }
        }
    }
    if (ep.ref) {
        const double sd = wave_sum(s_diff), sr = wave_sum(s_ref);
        if (lane == 0) {
            red[0][wave] = sd;
            red[1][wave] = sr;
        }
        __syncthreads();
        if (tid == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < C::WAVES; ++w) {
                a += red[0][w];
                b += red[1][w];
            }
            ep.partials[2 * blockIdx.x] = a;
            ep.partials[2 * blockIdx.x + 1] = b;
        }
    }
}


// FP64 on 128 x 128 tiles of 4 waves (2 x 2), each wave a 64 x 64 sub-tile
// (16 accumulators, 128 VGPRs), K-tile 16, two blocks per CU (launch bounds:
// at least two waves per SIMD). The tiles come to LDS by the load-to-LDS
// instruction (global_load_lds_dwordx4: a wave's instruction fills 1 KB, 16
// bytes per lane in lane order), two stages, with no staging registers and no
// LDS store instructions. Per K-tile a wave reads all its fragments (8 reads
// of 16 bytes of A, 8 paired reads of B), then issues the next K-tile's loads
// into the other stage (so that no LDS read waits behind a load in flight),
// then runs its 64 MFMAs; one barrier per K-tile. Each block keeps one wave
// per SIMD, so the other block's MFMAs fill the matrix pipe while a block
// reads fragments or waits at its barrier.
// A stage: 128 rows of 16 elements; row r's 16-byte chunk c sits in slot
// c ^ (r % 8), so the lanes of a fragment read that share a cycle hit distinct
// banks. B stage: 16 rows of 128 elements as in memory. Rows beyond M and
// columns beyond N are read from the last row (column pair) and feed only
// outputs that are not stored. Needs N, lda, ldb even, K % 16 == 0 and A, B
// 16-byte aligned (w4dma_fits).
//
// The K loop of one tile: acc = A[bm.., 0..K) B[0..K, bn..) for the wave's
// 64 x 64 sub-tile at (wm, wn). All threads of the block call it; it returns
// with every load landed and every wave past its last LDS read, so the LDS
// stages can be filled again at once.
__device__ inline void w4dma_mainloop(dbl4 (&acc)[4][4], int M, int N, int K, const double* A,
                                      int64_t lda, const double* B, int64_t ldb, int bm, int bn,
                                      int wm, int wn, int wave, int lane) {
    constexpr int BN = 128, BK = 16, TI = 4, TJ = 4;
    __shared__ __attribute__((aligned(16))) double As[2][128 * BK];
    __shared__ __attribute__((aligned(16))) double Bs[2][BK * BN];
    // opaque per call: in the symmetric kernel's loops over tiles and pieces
    // the addresses derived from them would otherwise be computed once and
    // held through both loops (and spilled)
    asm volatile("" : "+v"(lane), "+v"(wave), "+v"(wm), "+v"(wn));
    // the wave's instruction d fills A tile rows 8 (wave + 4 d) .. + 7 (lane
    // l: row 8 (wave + 4 d) + l / 8, chunk (l % 8) ^ (row % 8)) and B tile row
    // wave + 4 d (lane l: columns 2 l, 2 l + 1)
    const double* a_src[4];
    const double* b_src[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int r = 8 * (wave + 4 * d) + (lane >> 3);
        a_src[d] = A + (int64_t)min(bm + r, M - 1) * lda + 2 * ((lane & 7) ^ (r & 7));
        b_src[d] = B + (int64_t)(wave + 4 * d) * ldb + min(bn + 2 * lane, N - 2);
    }
    // (the builtin takes an LDS address-space pointer, which exists only in
    // the device compilation; the host pass sees an empty body)
    auto issue = [&](int st, int k0) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
        for (int d = 0; d < 4; ++d)
            __builtin_amdgcn_global_load_lds(a_src[d] + k0, &As[st][8 * (wave + 4 * d) * BK], 16, 0, 0);
#pragma unroll
        for (int d = 0; d < 4; ++d)
            __builtin_amdgcn_global_load_lds(b_src[d] + (int64_t)k0 * ldb, &Bs[st][(wave + 4 * d) * BN],
                                             16, 0, 0);
#else
        (void)st;
        (void)k0;
#endif
    };
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = dbl4{};
    const int fr = lane & 15, fg = lane >> 4;
    typedef double dbl2 __attribute__((ext_vector_type(2)));
    dbl2 fa[2][TI];
    double fb[2][TJ][2];
    const int nk = K / BK;
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const int st = t & 1;
        // lane group fg supplies k = 4 fg + 2 g + e of the K-tile: chunk
        // 2 fg + g of an A row, rows 4 fg + 2 g + e of B
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int c = 2 * fg + g;
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                const int r = wm + 16 * i + fr;
                fa[g][i] = *reinterpret_cast<const dbl2*>(&As[st][r * BK + 2 * (c ^ (r & 7))]);
            }
#pragma unroll
            for (int j = 0; j < TJ; ++j)
#pragma unroll
                for (int e = 0; e < 2; ++e) fb[g][j][e] = Bs[st][(2 * c + e) * BN + wn + 16 * j + fr];
        }
        // issued on every K-tile (the last one re-reads its own K-range into
        // the stage nobody reads again), so that no branch lets the compiler
        // move the MFMAs above it; the scheduling barriers keep the loads
        // ahead of the MFMAs and the MFMAs ahead of the closing wait
        issue(st ^ 1, (t + 1 < nk ? t + 1 : t) * BK);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < TJ; ++j)
                        acc[i][j] = Mfma<double>::mma(fa[g][i][e], fb[g][j][e], acc[i][j]);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next K-tile
        __syncthreads();                // everyone's, and every read of this stage
    }
}

__global__ __launch_bounds__(256, 2) void k_gemm_w4dma(
    int M, int N, int K, const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
    int64_t ldb, EpilogueT<double> ep, int tiles_m, int tiles_n) {
    if (gate_closed(ep.gate, ep.gate_mode)) return;  // uniform over the launch
    __shared__ double red[2][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int tm, tn;
    tile_of(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, tm, tn);
    const int bm = tm * 128, bn = tn * 128;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    dbl4 acc[4][4];
    w4dma_mainloop(acc, M, N, K, A, lda, B, ldb, bm, bn, wm, wn, wave, lane);
    tile_epilogue<double, 4, 4, 4>(acc, ep, M, N, bm, bn, wm, wn, blockIdx.x, red);
}

// The symmetric product (EpilogueT::sym) on the same tile: the partition of
// k_gemm_sym (hp_symk.h) over the blocks the device holds at once (two per
// CU): whole upper-triangle tiles in rounds, then the rest split by K-steps
// of 16, pieces of a tile combined by streamk_gather.
__global__ __launch_bounds__(256, 2) void k_gemm_w4dma_sym(
    int N, int K, const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
    int64_t ldb, EpilogueT<double> ep, int nt, int tiles, int ipt, int ipc, int dp) {
    if (gate_closed(ep.gate, ep.gate_mode)) return;  // uniform: no counter is touched
    __shared__ double red[2][4];
    int tid = threadIdx.x;
    // as in gemm_tile: values derived from the thread index are recomputed
    // per piece instead of being held through the loops
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int b = xcd_contiguous(blockIdx.x, gridDim.x);
    // one loop over the block's whole tiles (b, b + grid, ... below dp) and
    // then its stream-K pieces, so that the K loop and the epilogue are
    // compiled once
    int t_whole = b;
    const int64_t total = (int64_t)(tiles - dp) * ipt;
    int64_t it = (int64_t)b * ipc;
    const int64_t end = min(it + (int64_t)ipc, total);
    for (;;) {
        int ipt_p = ipt, ipc_p = ipc, nt_p = nt;
        asm volatile("" : "+s"(ipt_p), "+s"(ipc_p), "+s"(nt_p));
        int t, kb, ke, idx = 0, np = 1, slot0 = 0, b0 = 0;
        if (t_whole < dp) {
            t = t_whole;
            kb = 0;
            ke = K;
            t_whole += gridDim.x;
        } else if (it < end) {
            const SymPiece pc = sym_piece(it, end, ipt_p, ipc_p, b);
            t = dp + pc.t;
            kb = pc.k0 * 16;
            ke = min(K, pc.k1 * 16);
            idx = pc.idx;
            np = pc.np;
            slot0 = pc.slot0;
            b0 = pc.b0;
            it += pc.k1 - pc.k0;
        } else {
            break;
        }
        int tm, tn;
        sym_tile_of(t, nt_p, tm, tn);
        dbl4 acc[4][4];
        w4dma_mainloop(acc, N, N, ke - kb, A + kb, lda, B + (int64_t)kb * ldb, ldb, tm * 128, tn * 128,
                       wm, wn, wave, lane);
        if (streamk_gather<double, 4, 4, 256, 128 * 128>(acc, ep, tid, t, idx, np, slot0, b0))
            tile_epilogue<double, 4, 4, 4, true>(acc, ep, N, N, tm * 128, tn * 128, wm, wn, t, red);
        __syncthreads();  // the next tile's loads refill the LDS stages
    }
}

bool w4dma_fits(int64_t N, int64_t K, int64_t lda, int64_t ldb, const void* A, const void* B) {
    return N >= 2 && N % 2 == 0 && K > 0 && K % 16 == 0 && lda % 2 == 0 && ldb % 2 == 0 &&
           (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
}

// FP32 on 256 x 256 tiles of 4 waves (2 x 2), each wave a 128 x 128
// sub-tile: 64 accumulators in the 256 AGPRs, one wave per SIMD, K-tile 32,
// two LDS stages of 64 KB. The structure of k_gemm_w4dma (tiles brought in
// by load-to-LDS; per K-tile all fragment reads, then the next K-tile's
// loads, then the MFMAs, then one barrier), with 512 MFMAs per wave per
// K-tile against 48 LDS reads: the larger wave tile makes up for the single
// wave per SIMD. A rows as in k_gemm_w4dma (16-byte chunk c of row r in slot
// c ^ (r % 8)); B rows keep their 16-byte chunks with chunk q of row k in slot
// q ^ (4 ((k / 8) % 2)), so that the two lane groups of a 4-byte fragment read
// that share an LDS cycle (rows k and k + 8) use different banks. Needs N,
// lda, ldb multiples of 4, K of 32, 16-byte aligned operands
// (w4dma_f32_fits).
__global__ __launch_bounds__(256, 1) void k_gemm_w4dma_f32(
    int M, int N, int K, const float* __restrict__ A, int64_t lda, const float* __restrict__ B,
    int64_t ldb, EpilogueT<float> ep, int tiles_m, int tiles_n) {
    constexpr int BM = 256, BN = 256, BK = 32, WAVES = 4, TI = 8, TJ = 8;
    if (gate_closed(ep.gate, ep.gate_mode)) return;  // uniform over the launch
    __shared__ __attribute__((aligned(16))) float As[2][BM * BK];
    __shared__ __attribute__((aligned(16))) float Bs[2][BK * BN];
    __shared__ double red[2][WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int tm, tn;
    tile_of(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, tm, tn);
    const int bm = tm * BM, bn = tn * BN;
    const int wm = (wave >> 1) * 128, wn = (wave & 1) * 128;
    // the wave's instruction d fills A tile rows 8 (wave + 4 d) .. + 7 and B
    // tile row wave + 4 d (1 KB each)
    const float* a_src[8];
    const float* b_src[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int r = 8 * (wave + 4 * d) + (lane >> 3);
        a_src[d] = A + (int64_t)min(bm + r, M - 1) * lda + 4 * ((lane & 7) ^ (r & 7));
        const int k = wave + 4 * d;
        b_src[d] = B + (int64_t)k * ldb + min(bn + 4 * (lane ^ (4 * ((k >> 3) & 1))), N - 4);
    }
    auto issue = [&](int st, int k0) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
        for (int d = 0; d < 8; ++d)
            __builtin_amdgcn_global_load_lds(a_src[d] + k0, &As[st][8 * (wave + 4 * d) * BK], 16, 0, 0);
#pragma unroll
        for (int d = 0; d < 8; ++d)
            __builtin_amdgcn_global_load_lds(b_src[d] + (int64_t)k0 * ldb, &Bs[st][(wave + 4 * d) * BN],
                                             16, 0, 0);
#else
        (void)st;
        (void)k0;
#endif
    };
    flt4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = flt4{};
    const int fr = lane & 15, fg = lane >> 4;
    typedef float flt4v_ __attribute__((ext_vector_type(4)));
    flt4v_ fa[2][TI];
    float fb[2][TJ][4];
    const int nk = K / BK;
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int t = 0; t < nk; ++t) {
        const int st = t & 1;
        // lane group fg supplies k = 8 fg + 4 g + e: chunk 2 fg + g of an A
        // row, rows 4 (2 fg + g) + e of B
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int c = 2 * fg + g;
#pragma unroll
            for (int i = 0; i < TI; ++i) {
                const int r = wm + 16 * i + fr;
                fa[g][i] = *reinterpret_cast<const flt4v_*>(&As[st][r * BK + 4 * (c ^ (r & 7))]);
            }
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
                const int col = wn + 16 * j + fr;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 4 * c + e;
                    fb[g][j][e] = Bs[st][k * BN + 4 * ((col >> 2) ^ (4 * ((k >> 3) & 1))) + (col & 3)];
                }
            }
        }
        // as in k_gemm_w4dma: loads on every K-tile, order pinned
        issue(st ^ 1, (t + 1 < nk ? t + 1 : t) * BK);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < TJ; ++j)
                        acc[i][j] = Mfma<float>::mma(fa[g][i][e], fb[g][j][e], acc[i][j]);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    tile_epilogue<float, TI, TJ, WAVES>(acc, ep, M, N, bm, bn, wm, wn, blockIdx.x, red);
}

bool w4dma_f32_fits(int64_t N, int64_t K, int64_t lda, int64_t ldb, const void* A, const void* B) {
    return N >= 4 && N % 4 == 0 && K > 0 && K % 32 == 0 && lda % 4 == 0 && ldb % 4 == 0 &&
           (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
}

template <typename T, int BM, int BN, int BK, int WM, int WN, int PF = 1>
hipError_t launch(int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                  int64_t ldb, const EpilogueT<T>& ep, hipStream_t s) {
    using C = Cfg<T, BM, BN, BK, WM, WN>;
    const int tm = (int)cdiv(M, BM), tn = (int)cdiv(N, BN);
    hipLaunchKernelGGL((k_gemm<T, BM, BN, BK, WM, WN, PF>), dim3(tm * tn), dim3(C::NT), 0, s,
                       (int)M, (int)N, (int)K, A, lda, B, ldb, ep, tm, tn);
    return hipGetLastError();
}

// Split-K launch of the 8-wave 128 x 128 tile. Runs unsplit, still on 128 x
// 128 tiles (so the block count, and the partial sums of the stopping test,
// match gemm_blocks), when the epilogue brings no scratch, too little, or K
// too short for every block to get a K-range.
template <typename T, int BK, int SPLIT>
hipError_t launch_split(int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                        int64_t ldb, const EpilogueT<T>& ep, hipStream_t s) {
    using C = Cfg<T, 128, 128, BK, 64, 32>;
    const int tm = (int)cdiv(M, 128), tn = (int)cdiv(N, 128);
    const int64_t tiles = (int64_t)tm * tn;
    const int64_t kchunk = cdiv(cdiv(K, SPLIT), BK) * BK;
    const bool ok = ep.split_part && ep.split_cnt && ep.split_slots >= SPLIT * tiles &&
                    (SPLIT - 1) * kchunk < K;
    if (!ok) {
        if (tiles >= 512) return launch<T, 128, 128, BK, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        return launch<T, 128, 128, 2 * BK, 32, 32, 2>(M, N, K, A, lda, B, ldb, ep, s);
    }
    hipLaunchKernelGGL((k_gemm_split<T, 128, 128, BK, 64, 32, SPLIT>), dim3(tiles * SPLIT),
                       dim3(C::NT), 0, s, (int)M, (int)N, (int)K, A, lda, B, ldb, ep, tm, tn,
                       (int)kchunk);
    return hipGetLastError();
}

// Blocks of k_gemm_sym<T, ...> that the device holds at once (compute units
// times blocks per unit): the stream-K grid. Queried once per kernel.
template <typename T, int BM, int BN, int BK, int WM, int WN, int PF>
int sym_grid() {
    // the same value whichever thread computes it first
    static std::atomic<int> g{0};
    int v = g.load(std::memory_order_relaxed);
    if (v == 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per, reinterpret_cast<const void*>(&k_gemm_sym<T, BM, BN, BK, WM, WN, PF>),
                64 * (BM / WM) * (BN / WN), 0) != hipSuccess)
            return 0;
        v = cus * std::max(per, 1);
        g.store(v, std::memory_order_relaxed);
    }
    return v;
}

struct SymShape {
    int grid, nt, tiles, ipt, ipc, dp;
};
template <typename T, int BM, int BN, int BK, int WM, int WN, int PF>
SymShape sym_shape(int64_t N, int64_t K) {
    SymShape sh{};
    const int g = sym_grid<T, BM, BN, BK, WM, WN, PF>();
    if (g <= 0) return sh;
    sh.nt = (int)cdiv(N, BM);
    sh.tiles = sh.nt * (sh.nt + 1) / 2;
    sh.ipt = (int)cdiv(K, BK);
    sym_layout(sh.tiles, sh.ipt, g, &sh.ipc, &sh.grid, &sh.dp);
    return sh;
}

template <typename T>
bool sym_fits(const SymShape& sh, const EpilogueT<T>& ep) {
    const int64_t ncnt = ep.split_ncnt > 0 ? ep.split_ncnt : ep.split_slots;
    return sh.grid > 0 && ep.split_part && ep.split_cnt && ep.split_slots >= 2 * (int64_t)sh.grid &&
           ncnt >= sh.tiles;
}

// The symmetric launch; returns false (nothing launched) when the epilogue
// brings too little scratch for it.
template <typename T, int BM, int BN, int BK, int WM, int WN, int PF>
bool launch_sym(int64_t N, int64_t K, const T* A, int64_t lda, const T* B, int64_t ldb,
                const EpilogueT<T>& ep, hipStream_t s, hipError_t* err) {
    using C = Cfg<T, BM, BN, BK, WM, WN>;
    if (K <= 0) return false;
    const SymShape sh = sym_shape<T, BM, BN, BK, WM, WN, PF>(N, K);
    if (!sym_fits(sh, ep)) return false;
    hipLaunchKernelGGL((k_gemm_sym<T, BM, BN, BK, WM, WN, PF>), dim3(sh.grid), dim3(C::NT), 0, s,
                       (int)N, (int)K, A, lda, B, ldb, ep, sh.nt, sh.tiles, sh.ipt, sh.ipc,
                       sh.dp);
    *err = hipGetLastError();
    return true;
}

// The same for k_gemm_w4dma_sym (K-steps of 16, two blocks per CU).
int sym_grid_w4dma() {
    static std::atomic<int> g{0};
    int v = g.load(std::memory_order_relaxed);
    if (v == 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per, reinterpret_cast<const void*>(&k_gemm_w4dma_sym), 256, 0) != hipSuccess)
            return 0;
        v = cus * std::max(per, 1);
        g.store(v, std::memory_order_relaxed);
    }
    return v;
}

SymShape sym_shape_w4dma(int64_t N, int64_t K) {
    SymShape sh{};
    const int g = sym_grid_w4dma();
    if (g <= 0) return sh;
    sh.nt = (int)cdiv(N, 128);
    sh.tiles = sh.nt * (sh.nt + 1) / 2;
    sh.ipt = (int)cdiv(K, 16);
    sym_layout(sh.tiles, sh.ipt, g, &sh.ipc, &sh.grid, &sh.dp);
    return sh;
}

// Which symmetric launch a call on the load-to-LDS tile takes: 1 for
// k_gemm_w4dma_sym (operands fit, scratch for its grid, and at least three
// rounds of whole tiles: 8192^3 8.44 ms against 8.68-8.75 for the 16-wave
// kernel, but 4096^3, one round, 1.37 against 1.16), 2 for the 16-wave
// stream-K kernel (otherwise, with scratch for it), 0 for none (the full
// product).
template <typename T>
int w4dma_sym_choice(int64_t N, int64_t K, const T* A, int64_t lda, const T* B, int64_t ldb,
                     const EpilogueT<T>& ep) {
    constexpr int BKF = 16 * sizeof(double) / sizeof(T);
    if constexpr (std::is_same<T, double>::value) {
        const SymShape sh = sym_shape_w4dma(N, K);
        if (w4dma_fits(N, K, lda, ldb, A, B) && sym_fits(sh, ep) && sh.tiles >= 3 * sh.grid) return 1;
    }
    return sym_fits(sym_shape<T, 128, 128, 2 * BKF, 32, 32, 2>(N, K), ep) ? 2 : 0;
}


template <typename T>
hipError_t dispatch(GemmTile t, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda,
                    const T* B, int64_t ldb, const EpilogueT<T>& ep, hipStream_t s) {
    constexpr int BKF = 16 * sizeof(double) / sizeof(T);  // 128-byte K-tile rows
    if (ep.sym && M == N && !ep.ref) {
        hipError_t e = hipSuccess;
        if constexpr (std::is_same<T, double>::value) {
            if (t == TILE_128x128_W4_DMA && K > 0 && w4dma_sym_choice(N, K, A, lda, B, ldb, ep) == 1) {
                const SymShape sh = sym_shape_w4dma(N, K);
                hipLaunchKernelGGL(k_gemm_w4dma_sym, dim3(sh.grid), dim3(256), 0, s, (int)N, (int)K, A,
                                   lda, B, ldb, ep, sh.nt, sh.tiles, sh.ipt, sh.ipc, sh.dp);
                return hipGetLastError();
            }
        }
        if ((t == TILE_128x128_W16_K2_P2 || t == TILE_128x128_W4_DMA) &&
            launch_sym<T, 128, 128, 2 * BKF, 32, 32, 2>(N, K, A, lda, B, ldb, ep, s, &e))
            return e;
        if (t == TILE_128x128_W8 && launch_sym<T, 128, 128, BKF, 64, 32, 1>(N, K, A, lda, B, ldb, ep, s, &e))
            return e;
    }
    switch (t) {
        case TILE_128x128_W4: return launch<T, 128, 128, BKF, 64, 64>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W8: return launch<T, 128, 128, BKF, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x64_W4: return launch<T, 128, 64, BKF, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_64x64_W4: return launch<T, 64, 64, BKF, 32, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_256x128_W8: return launch<T, 256, 128, BKF, 64, 64>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x64_W8: return launch<T, 128, 64, BKF, 32, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_64x128_W8: return launch<T, 64, 128, BKF, 32, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W8_K2: return launch<T, 128, 128, 2 * BKF, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W16: return launch<T, 128, 128, BKF, 32, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W8_P2: return launch<T, 128, 128, BKF, 64, 32, 2>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W16_P2: return launch<T, 128, 128, BKF, 32, 32, 2>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W8_S2: return launch_split<T, BKF, 2>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W8_S4: return launch_split<T, BKF, 4>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W16_K2_P2: return launch<T, 128, 128, 2 * BKF, 32, 32, 2>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_32x32_W4_K4: return launch<T, 32, 32, 4 * BKF, 16, 16>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W4_DMA:
            if constexpr (std::is_same<T, double>::value) {
                // otherwise the 16-wave kernel on the same 128 x 128 tiles
                // (the same blocks, so the same partial-sum slots)
                if (!w4dma_fits(N, K, lda, ldb, A, B))
                    return launch<T, 128, 128, 2 * BKF, 32, 32, 2>(M, N, K, A, lda, B, ldb, ep, s);
                const int tm = (int)cdiv(M, 128), tn = (int)cdiv(N, 128);
                hipLaunchKernelGGL(k_gemm_w4dma, dim3(tm * tn), dim3(256), 0, s, (int)M, (int)N,
                                   (int)K, A, lda, B, ldb, ep, tm, tn);
                return hipGetLastError();
            } else {
                return hipErrorInvalidValue;
            }
        case TILE_256x256_W4_DMA:
            if constexpr (std::is_same<T, float>::value) {
                // otherwise a register-staged kernel on the same 256 x 256
                // tiles (the same blocks, so the same partial-sum slots)
                if (!w4dma_f32_fits(N, K, lda, ldb, A, B))
                    return launch<T, 256, 256, BKF, 128, 64>(M, N, K, A, lda, B, ldb, ep, s);
                const int tm = (int)cdiv(M, 256), tn = (int)cdiv(N, 256);
                hipLaunchKernelGGL(k_gemm_w4dma_f32, dim3(tm * tn), dim3(256), 0, s, (int)M, (int)N,
                                   (int)K, A, lda, B, ldb, ep, tm, tn);
                return hipGetLastError();
            } else {
                return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
    }
}

template <typename L, int BM, int BN, int BK, int WM, int WN>
hipError_t launch_lp(int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, const float* B,
                     int64_t ldb, const EpilogueT<float>& ep, hipStream_t s) {
    using C = CfgLP<BM, BN, BK, WM, WN>;
    const int tm = (int)cdiv(M, BM), tn = (int)cdiv(N, BN);
    hipLaunchKernelGGL((k_gemm_lp<L, BM, BN, BK, WM, WN>), dim3(tm * tn), dim3(C::NT), 0, s,
                       (int)M, (int)N, (int)K, A, lda, B, ldb, ep, tm, tn);
    return hipGetLastError();
}

template <typename L>
hipError_t dispatch_lp(GemmTile t, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                       const float* B, int64_t ldb, const EpilogueT<float>& ep, hipStream_t s) {
    switch (t) {
        case TILE_128x128_W4: return launch_lp<L, 128, 128, 64, 64, 64>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W8: return launch_lp<L, 128, 128, 64, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x64_W4: return launch_lp<L, 128, 64, 64, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_64x64_W4: return launch_lp<L, 64, 64, 64, 32, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_256x128_W8: return launch_lp<L, 256, 128, 64, 64, 64>(M, N, K, A, lda, B, ldb, ep, s);
        // the 16-bit kernel stages B in 4x4 blocks: fewer blocks than threads
        // would leave lanes idle, so the smaller tiles keep 4 waves here
        case TILE_128x64_W8: return launch_lp<L, 128, 64, 64, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_64x128_W8: return launch_lp<L, 64, 128, 64, 32, 64>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W8_K2: return launch_lp<L, 128, 128, 128, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        case TILE_128x128_W16:
        case TILE_128x128_W8_P2:
        case TILE_128x128_W16_P2:
        case TILE_128x128_W8_S2:
        case TILE_128x128_W8_S4:
        case TILE_128x128_W16_K2_P2: return launch_lp<L, 128, 128, 64, 64, 32>(M, N, K, A, lda, B, ldb, ep, s);
        default: return hipErrorInvalidValue;
    }
}


}  // namespace

int grouped_tile_dim(int cfg) { return cfg == GTILE_128 ? 128 : cfg == GTILE_32 ? 32 : 64; }

template <typename T>
static hipError_t launch_grouped(const GroupHeader* hdr, const GroupEntry<T>* ents, int grid,
                                 int cfg, hipStream_t s) {
    constexpr int BKF = 16 * sizeof(double) / sizeof(T);  // 128-byte K-tile rows
    if (cfg == GTILE_128)
        hipLaunchKernelGGL((k_gemm_grouped<T, 128, 128, BKF, 64, 64>), dim3(grid), dim3(256), 0, s,
                           hdr, ents);
    else if (cfg == GTILE_32)
        hipLaunchKernelGGL((k_gemm_grouped<T, 32, 32, 4 * BKF, 16, 16>), dim3(grid), dim3(256), 0,
                           s, hdr, ents);
    else
        hipLaunchKernelGGL((k_gemm_grouped<T, 64, 64, BKF, 32, 32>), dim3(grid), dim3(256), 0, s,
                           hdr, ents);
    return hipGetLastError();
}

hipError_t gemm_grouped(const GroupHeader* hdr, const GroupEntry<double>* ents, int grid, int cfg,
                        hipStream_t s) {
    return launch_grouped(hdr, ents, grid, cfg, s);
}

hipError_t gemm_grouped(const GroupHeader* hdr, const GroupEntry<float>* ents, int grid, int cfg,
                        hipStream_t s) {
    return launch_grouped(hdr, ents, grid, cfg, s);
}

hipError_t gemm_lowp(GemmTile t, LowPrec lp, int64_t M, int64_t N, int64_t K, const float* A,
                     int64_t lda, const float* B, int64_t ldb, const EpilogueT<float>& ep,
                     hipStream_t s) {
    if (lp == LOWP_BF16) return dispatch_lp<__bf16>(t, M, N, K, A, lda, B, ldb, ep, s);
    return dispatch_lp<_Float16>(t, M, N, K, A, lda, B, ldb, ep, s);
}



template <typename T>
static bool sym_launches(GemmTile t, int64_t M, int64_t N, int64_t K, const T* A, int64_t lda,
                         const T* B, int64_t ldb, const EpilogueT<T>& ep) {
    constexpr int BKF = 16 * sizeof(double) / sizeof(T);
    if (!ep.sym || M != N || ep.ref || K <= 0) return false;
    if (t == TILE_128x128_W4_DMA) return w4dma_sym_choice(N, K, A, lda, B, ldb, ep) != 0;
    if (t == TILE_128x128_W16_K2_P2)
        return sym_fits(sym_shape<T, 128, 128, 2 * BKF, 32, 32, 2>(N, K), ep);
    if (t == TILE_128x128_W8) return sym_fits(sym_shape<T, 128, 128, BKF, 64, 32, 1>(N, K), ep);
    return false;
}
bool gemm_sym_launches(GemmTile t, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                       const double* B, int64_t ldb, const EpilogueT<double>& ep) {
    return sym_launches(t, M, N, K, A, lda, B, ldb, ep);
}
bool gemm_sym_launches(GemmTile t, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                       const float* B, int64_t ldb, const EpilogueT<float>& ep) {
    return sym_launches(t, M, N, K, A, lda, B, ldb, ep);
}

bool gemm_sym_runs(GemmTile t, GemmType gt) {
    // (the load-to-LDS tile's symmetric products run on k_gemm_w4dma_sym, or
    // on the 16-wave kernel where its operands or scratch do not fit)
    return ((gt == GT_F64 || gt == GT_F32) && (t == TILE_128x128_W16_K2_P2 || t == TILE_128x128_W8)) ||
           (gt == GT_F64 && t == TILE_128x128_W4_DMA);
}

void gemm_sym_scratch(GemmTile t, GemmType gt, int64_t n, int64_t* slots, int64_t* counters) {
    *slots = *counters = 0;
    if (!gemm_sym_runs(t, gt) || n <= 0) return;
    // the grid is at most the resident block count, whatever K is
    const int64_t nt = cdiv(n, 128);
    int g = 0;
    if (gt == GT_F64) {
        g = t == TILE_128x128_W8 ? sym_grid<double, 128, 128, 16, 64, 32, 1>()
                                 : sym_grid<double, 128, 128, 32, 32, 32, 2>();
        // the load-to-LDS tile's own symmetric kernel (a larger grid) runs
        // only on a triangle of at least three rounds (w4dma_sym_choice)
        if (t == TILE_128x128_W4_DMA) {
            const int gd = sym_grid_w4dma();
            if (nt * (nt + 1) / 2 >= 3 * (int64_t)gd) g = std::max(g, gd);
        }
    } else {
        g = t == TILE_128x128_W8 ? sym_grid<float, 128, 128, 32, 64, 32, 1>()
                                 : sym_grid<float, 128, 128, 64, 32, 32, 2>();
    }
    if (g <= 0) return;
    *slots = 2 * (int64_t)g;
    *counters = nt * (nt + 1) / 2;
}

template <int SPLIT>
static bool split_fits(int64_t M, int64_t N, int64_t K, int bk, int64_t slots) {
    const int64_t kchunk = cdiv(cdiv(K, SPLIT), bk) * bk;
    return slots >= SPLIT * cdiv(M, 128) * cdiv(N, 128) && (SPLIT - 1) * kchunk < K;
}

bool gemm_split_runs(GemmTile t, int64_t M, int64_t N, int64_t K, GemmType gt, int64_t slots) {
    if (gt == GT_LOWP || gt == GT_H16) return false;
    const int bk = gt == GT_F64 ? 16 : 32;  // BKF of the element type
    if (t == TILE_128x128_W8_S2) return split_fits<2>(M, N, K, bk, slots);
    if (t == TILE_128x128_W8_S4) return split_fits<4>(M, N, K, bk, slots);
    return false;
}

int64_t gemm_split_slots(GemmTile t, int64_t M, int64_t N, int64_t K) {
    (void)K;
    const int64_t tiles = cdiv(M, 128) * cdiv(N, 128);
    if (t == TILE_128x128_W8_S2) return 2 * tiles;
    if (t == TILE_128x128_W8_S4) return 4 * tiles;
    return 0;
}

hipError_t gemm(GemmTile t, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                const double* B, int64_t ldb, const EpilogueT<double>& ep, hipStream_t s) {
    return dispatch<double>(t, M, N, K, A, lda, B, ldb, ep, s);
}

hipError_t gemm(GemmTile t, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                const float* B, int64_t ldb, const EpilogueT<float>& ep, hipStream_t s) {
    return dispatch<float>(t, M, N, K, A, lda, B, ldb, ep, s);
}

}  // namespace hp
