// MFMA GEMM on 16-bit operands held in memory, for gfx950 (CDNA4, wave64):
// C = epilogue(A B) with A (M x K) and Bt = B^T (N x K) in bf16 or fp16,
// v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation and the FP32
// epilogue of the loop products (up to three outputs
// id*I + acc*(A B) + g1*D1 + g2*D2, optional FP64 partial sums of the
// stopping test), which can also leave 16-bit copies of its outputs,
// row-major and transposed, for the next products of a loop of Section 2.
#include "hp_gemm_common.h"
#include "hp_internal.h"

namespace hp {
namespace {

// ---------------------------------------------------------------------------
// 16-bit operands held in memory: A (M x K) and Bt = B^T (N x K), both
// row-major and so both k-contiguous, the layout a lane's fragment of
// v_mfma_f32_16x16x32_{bf16,f16} wants (8 consecutive k of one row of A or
// one column of B). Tiles are copied to LDS as read, 16 bytes at a time, with
// no conversion; a fragment is one 16-byte LDS read. FP32 accumulation and
// the FP32 epilogue of k_gemm_lp, which can also write the outputs rounded
// to 16 bits (nearest even), row-major and transposed, for later products.
// ---------------------------------------------------------------------------

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, int WM, int WN>
struct CfgH {
    static constexpr int WAVES = (BM / WM) * (BN / WN);
    static constexpr int NT = 64 * WAVES;
    static constexpr int KP = BK + 8;      // LDS row pitch (16-bit elements)
    static constexpr int TPR = BK / 8;     // 16-byte loads per tile row
    static constexpr int RPP = NT / TPR;   // tile rows per pass
    static constexpr int A_PASS = BM / RPP, B_PASS = BN / RPP;
    static constexpr int TI = WM / 16, TJ = WN / 16;
    static_assert(BK % 32 == 0 && NT % TPR == 0, "K tile");
    static_assert(BM % RPP == 0 && BN % RPP == 0 && A_PASS >= 1 && B_PASS >= 1, "loads");
    static_assert(BM % WM == 0 && BN % WN == 0 && WM % 16 == 0 && WN % 16 == 0, "waves");
};

// The FP32 epilogue of the 16-bit-operand kernels (accumulator register r
// of lane l: row 4(l/16) + r), with the 16-bit copies of the outputs.
template <typename L, int TI, int TJ, int WAVES>
__device__ __attribute__((always_inline)) inline void h16_epilogue(
    flt4 (&acc)[TI][TJ], const EpilogueT<float>& ep, int M, int N,
                                    int bm, int bn, int wm, int wn, double (*red)[WAVES]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int fr = lane & 15, fg = lane >> 4;
    double s_diff = 0.0, s_ref = 0.0;
#pragma unroll
    for (int i = 0; i < TI; ++i) {
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int row0 = bm + wm + i * 16 + 4 * fg;
            const int col = bn + wn + j * 16 + fr;
            float vo[3][4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + r;
                if (row < M && col < N) {
                    const float a = acc[i][j][r];
                    const float d1 = ep.D1 ? ep.D1[(int64_t)row * ep.ld1 + col] : 0.f;
                    const float d2 = ep.D2 ? ep.D2[(int64_t)row * ep.ld2 + col] : 0.f;
                    const float idv = (row == col) ? 1.f : 0.f;
#pragma unroll
                    for (int o = 0; o < 3; ++o) {
                        vo[o][r] = 0.f;
                        if (ep.out[o]) {
                            float v = (float)ep.acc_c[o] * a;
                            if (ep.id[o] != 0.0) v += (float)ep.id[o] * idv;
                            if (ep.g1[o] != 0.0) v += (float)ep.g1[o] * d1;
                            if (ep.g2[o] != 0.0) v += (float)ep.g2[o] * d2;
                            vo[o][r] = v;
                            if (!ep.skip32[o]) ep.out[o][(int64_t)row * ep.ldo[o] + col] = v;
                            if (ep.h[o]) static_cast<L*>(ep.h[o])[(int64_t)row * ep.ldh[o] + col] = (L)v;
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
            // transposed copies: the lane's 4 rows are 4 consecutive elements
            // of column `col` of the output, i.e. of row `col` of its transpose
            if (col < N) {
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    if (!ep.out[o] || !ep.ht[o]) continue;
                    L* dst = static_cast<L*>(ep.ht[o]) + (int64_t)col * ep.ldht[o] + row0;
                    if (row0 + 3 < M) {
                        typedef L l4 __attribute__((ext_vector_type(4)));
                        *reinterpret_cast<l4*>(dst) = l4{(L)vo[o][0], (L)vo[o][1], (L)vo[o][2], (L)vo[o][3]};
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (row0 + r < M) dst[r] = (L)vo[o][r];
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
            for (int w = 0; w < WAVES; ++w) {
                a += red[0][w];
                b += red[1][w];
            }
            ep.partials[2 * blockIdx.x] = a;
            ep.partials[2 * blockIdx.x + 1] = b;
        }
    }
}

template <typename L, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN)) void k_gemm_h16(
    int M, int N, int K, const L* __restrict__ A, int64_t lda, const L* __restrict__ Bt,
    int64_t ldbt, EpilogueT<float> ep, int tiles_m, int tiles_n) {
    using C = CfgH<BM, BN, BK, WM, WN>;
    using FR = typename Mfma16<L>::frag_t;
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

    // Branch-free staging: every 16-byte load comes from an address inside
    // the operand (rows or k beyond the edge read element 0 instead) and the
    // out-of-range 16-bit elements are zeroed on their way to LDS.
    const int kc = 8 * (tid % C::TPR), r0 = tid / C::TPR;
    u32x4 ra[C::A_PASS], rb[C::B_PASS];
    const L* a_ptr[C::A_PASS];
    const L* b_ptr[C::B_PASS];
    bool a_ok[C::A_PASS], b_ok[C::B_PASS];
#pragma unroll
    for (int p = 0; p < C::A_PASS; ++p) {
        const int row = bm + r0 + C::RPP * p;
        a_ok[p] = row < M;
        a_ptr[p] = A + (int64_t)(a_ok[p] ? row : 0) * lda + kc;
    }
#pragma unroll
    for (int p = 0; p < C::B_PASS; ++p) {
        const int row = bn + r0 + C::RPP * p;
        b_ok[p] = row < N;
        b_ptr[p] = Bt + (int64_t)(b_ok[p] ? row : 0) * ldbt + kc;
    }
    auto load = [&](int k0) {
        const bool kin = k0 + kc < K;
#pragma unroll
        for (int p = 0; p < C::A_PASS; ++p)
            ra[p] = *reinterpret_cast<const u32x4*>((a_ok[p] && kin) ? a_ptr[p] + k0 : A);
#pragma unroll
        for (int p = 0; p < C::B_PASS; ++p)
            rb[p] = *reinterpret_cast<const u32x4*>((b_ok[p] && kin) ? b_ptr[p] + k0 : Bt);
    };
    // keep the first `rem` 16-bit elements of v (all if rem >= 8)
    auto keep = [](u32x4 v, int rem) {
        if (rem >= 8) return v;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const unsigned lo = 2 * w < rem ? 0xFFFFu : 0u;
            const unsigned hi = 2 * w + 1 < rem ? 0xFFFF0000u : 0u;
            v[w] &= (lo | hi);
        }
        return v;
    };
    auto store = [&](int buf, int k0) {
        const int rem = K - (k0 + kc);
#pragma unroll
        for (int p = 0; p < C::A_PASS; ++p)
            *reinterpret_cast<u32x4*>(&As[buf][r0 + C::RPP * p][kc]) =
                a_ok[p] ? keep(ra[p], rem) : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int p = 0; p < C::B_PASS; ++p)
            *reinterpret_cast<u32x4*>(&Bs[buf][r0 + C::RPP * p][kc]) =
                b_ok[p] ? keep(rb[p], rem) : u32x4{0u, 0u, 0u, 0u};
    };

    flt4 acc[C::TI][C::TJ];
#pragma unroll
    for (int i = 0; i < C::TI; ++i)
#pragma unroll
        for (int j = 0; j < C::TJ; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

    const int fr = lane & 15, fg = lane >> 4;
    const int nk = (K + BK - 1) / BK;
    load(0);
    store(0, 0);
    __syncthreads();
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
            // one k-step's fragments live at a time (large wave tiles would
            // otherwise run out of registers)
            __builtin_amdgcn_sched_barrier(0);
        }
        if (kt + 1 < nk) store(cur ^ 1, (kt + 1) * BK);
        __syncthreads();
    }
    h16_epilogue<L, C::TI, C::TJ, C::WAVES>(acc, ep, M, N, bm, bn, wm, wn, red);
}

// The same product with the tiles brought into LDS by the load-to-LDS
// instruction (global_load_lds_dwordx4): no staging registers and no LDS
// store instructions. A wave's instruction fills 1 KB of LDS, 16 bytes per
// lane in lane order, i.e. 8 unpadded rows of a 64-wide K-tile; each lane
// picks its source chunk as (LDS slot) XOR (row mod 8), so that the 16 lanes
// of a fragment read (16 rows, one 16-byte chunk) spread over the banks.
// Needs K to be a multiple of BK = 64 (no masking); rows beyond M (N) read
// the last row and only feed outputs that are never stored. Two LDS stages:
// tile t+1 streams in while tile t is multiplied.
template <typename L, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * (BM / WM) * (BN / WN)) void k_gemm_h16_dma(
    int M, int N, int K, const L* __restrict__ A, int64_t lda, const L* __restrict__ Bt,
    int64_t ldbt, EpilogueT<float> ep, int tiles_m, int tiles_n) {
    constexpr int BK = 64;
    constexpr int WAVES = (BM / WM) * (BN / WN);
    constexpr int TI = WM / 16, TJ = WN / 16;
    constexpr int A_INS = BM / 8 / WAVES, B_INS = BN / 8 / WAVES;  // 8 rows per wave instruction
    static_assert(A_INS * 8 * WAVES == BM && B_INS * 8 * WAVES == BN, "DMA rows");
    // With two waves per SIMD (room for 256 registers) a wave reads the whole
    // K-tile's fragments before it issues the next tile's loads, so that its
    // MFMAs run while those loads are in flight (the compiler makes any LDS
    // read that follows a load-to-LDS wait for it).
    constexpr bool EARLY = WAVES <= 8 && TI * TJ * 4 + 2 * (TI + TJ) * 4 <= 224;
    using FR = typename Mfma16<L>::frag_t;
    __shared__ __attribute__((aligned(16))) L As[2][BM * BK];
    __shared__ __attribute__((aligned(16))) L Bs[2][BN * BK];
    __shared__ double red[2][WAVES];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int tm, tn;
    tile_of(xcd_contiguous(blockIdx.x, gridDim.x), tiles_m, tiles_n, tm, tn);
    const int bm = tm * BM, bn = tn * BN;
    const int wm = (wave / (BN / WN)) * WM, wn = (wave % (BN / WN)) * WN;

    // this lane's source in each of the wave's instructions: tile row
    // 8*q + lane/8 (clamped into the operand), chunk (lane%8) ^ (row%8)
    const int lrow = lane >> 3, slot = lane & 7;
    const L* a_src[A_INS];
    const L* b_src[B_INS];
#pragma unroll
    for (int i = 0; i < A_INS; ++i) {
        const int tr = 8 * (wave + WAVES * i) + lrow;
        a_src[i] = A + (int64_t)min(bm + tr, M - 1) * lda + 8 * (slot ^ (tr & 7));
    }
#pragma unroll
    for (int i = 0; i < B_INS; ++i) {
        const int tr = 8 * (wave + WAVES * i) + lrow;
        b_src[i] = Bt + (int64_t)min(bn + tr, N - 1) * ldbt + 8 * (slot ^ (tr & 7));
    }
    // (the builtin takes an LDS address-space pointer, which exists only in
    // the device compilation; the host pass sees an empty body)
    auto issue = [&](int buf, int k0) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
        for (int i = 0; i < A_INS; ++i)
            __builtin_amdgcn_global_load_lds(a_src[i] + k0, &As[buf][8 * (wave + WAVES * i) * BK], 16, 0, 0);
#pragma unroll
        for (int i = 0; i < B_INS; ++i)
            __builtin_amdgcn_global_load_lds(b_src[i] + k0, &Bs[buf][8 * (wave + WAVES * i) * BK], 16, 0, 0);
#else
        (void)buf;
        (void)k0;
#endif
    };

    flt4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

    const int fr = lane & 15, fg = lane >> 4;
    // fragments of k-step q (32 k) of the tile in stage `buf`
    auto frags = [&](int buf, int q, FR (&a)[TI], FR (&b)[TJ]) {
        const int c = 4 * q + fg;  // this lane's 16-byte chunk of the row
#pragma unroll
        for (int i = 0; i < TI; ++i) {
            const int r = wm + i * 16 + fr;
            a[i] = *reinterpret_cast<const FR*>(&As[buf][r * BK + 8 * (c ^ (r & 7))]);
        }
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int r = wn + j * 16 + fr;
            b[j] = *reinterpret_cast<const FR*>(&Bs[buf][r * BK + 8 * (c ^ (r & 7))]);
        }
    };
    auto mma = [&](FR (&a)[TI], FR (&b)[TJ]) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) acc[i][j] = Mfma16<L>::mma(a[i], b[j], acc[i][j]);
    };

    const int nk = K / BK;
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if constexpr (EARLY) {
            FR a0[TI], b0[TJ], a1[TI], b1[TJ];
            frags(cur, 0, a0, b0);
            frags(cur, 1, a1, b1);
            __builtin_amdgcn_sched_barrier(0);
            if (kt + 1 < nk) issue(cur ^ 1, (kt + 1) * BK);
            __builtin_amdgcn_sched_barrier(0);
            mma(a0, b0);
            mma(a1, b1);
            // keep the MFMAs above the wait below (they touch no memory, so
            // the scheduler would otherwise sink them past it)
            __builtin_amdgcn_sched_barrier(0);
        } else {
            if (kt + 1 < nk) issue(cur ^ 1, (kt + 1) * BK);
#pragma unroll
            for (int ks = 0; ks < BK; ks += 32) {
                const int c = ks / 8 + fg;
                FR a[TI], b[TJ];
#pragma unroll
                for (int i = 0; i < TI; ++i) {
                    const int r = wm + i * 16 + fr;
                    a[i] = *reinterpret_cast<const FR*>(&As[cur][r * BK + 8 * (c ^ (r & 7))]);
                }
#pragma unroll
                for (int j = 0; j < TJ; ++j) {
                    const int r = wn + j * 16 + fr;
                    b[j] = *reinterpret_cast<const FR*>(&Bs[cur][r * BK + 8 * (c ^ (r & 7))]);
                }
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < TJ; ++j) acc[i][j] = Mfma16<L>::mma(a[i], b[j], acc[i][j]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // this wave's loads of tile kt+1 have landed; the barrier makes every
        // wave's loads visible and ends every wave's reads of tile kt
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    h16_epilogue<L, TI, TJ, WAVES>(acc, ep, M, N, bm, bn, wm, wn, red);
}

template <typename L, int BM, int BN, int BK, int WM, int WN>
hipError_t launch_h16(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* Bt,
                      int64_t ldbt, const EpilogueT<float>& ep, hipStream_t s) {
    using C = CfgH<BM, BN, BK, WM, WN>;
    const int tm = (int)cdiv(M, BM), tn = (int)cdiv(N, BN);
    hipLaunchKernelGGL((k_gemm_h16<L, BM, BN, BK, WM, WN>), dim3(tm * tn), dim3(C::NT), 0, s,
                       (int)M, (int)N, (int)K, static_cast<const L*>(A), lda,
                       static_cast<const L*>(Bt), ldbt, ep, tm, tn);
    return hipGetLastError();
}

template <typename L, int BM, int BN, int WM, int WN>
hipError_t launch_h16_dma(int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                          const void* Bt, int64_t ldbt, const EpilogueT<float>& ep, hipStream_t s) {
    const int tm = (int)cdiv(M, BM), tn = (int)cdiv(N, BN);
    hipLaunchKernelGGL((k_gemm_h16_dma<L, BM, BN, WM, WN>), dim3(tm * tn),
                       dim3(64 * (BM / WM) * (BN / WN)), 0, s, (int)M, (int)N, (int)K,
                       static_cast<const L*>(A), lda, static_cast<const L*>(Bt), ldbt, ep, tm, tn);
    return hipGetLastError();
}

template <typename L>
hipError_t dispatch_h16(GemmTile t, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                        const void* Bt, int64_t ldbt, const EpilogueT<float>& ep, hipStream_t s) {
    // the load-to-LDS tiles copy whole 64-wide K-tiles: K a multiple of 64
    const bool dma = K % 64 == 0;
    switch (t) {
        case TILE_256x256_W8_DMA:
            if (dma) return launch_h16_dma<L, 256, 256, 128, 64>(M, N, K, A, lda, Bt, ldbt, ep, s);
            return launch_h16<L, 256, 256, 32, 128, 64>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_256x256_W16_DMA:
            if (dma) return launch_h16_dma<L, 256, 256, 64, 64>(M, N, K, A, lda, Bt, ldbt, ep, s);
            return launch_h16<L, 256, 256, 32, 64, 64>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_64x64_W4: return launch_h16<L, 64, 64, 64, 32, 32>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_128x64_W4: return launch_h16<L, 128, 64, 64, 64, 32>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_128x128_W4: return launch_h16<L, 128, 128, 64, 64, 64>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_256x128_W8: return launch_h16<L, 256, 128, 64, 64, 64>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_256x256_W8: return launch_h16<L, 256, 256, 32, 128, 64>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_256x256_W16: return launch_h16<L, 256, 256, 32, 64, 64>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_128x128_W16: return launch_h16<L, 128, 128, 64, 32, 32>(M, N, K, A, lda, Bt, ldbt, ep, s);
        case TILE_128x128_W8: return launch_h16<L, 128, 128, 64, 64, 32>(M, N, K, A, lda, Bt, ldbt, ep, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t gemm_h16(GemmTile t, LowPrec lp, int64_t M, int64_t N, int64_t K, const void* A,
                    int64_t lda, const void* Bt, int64_t ldbt, const EpilogueT<float>& ep,
                    hipStream_t s) {
    if (lp == LOWP_BF16) return dispatch_h16<__bf16>(t, M, N, K, A, lda, Bt, ldbt, ep, s);
    return dispatch_h16<_Float16>(t, M, N, K, A, lda, Bt, ldbt, ep, s);
}

}  // namespace hp
