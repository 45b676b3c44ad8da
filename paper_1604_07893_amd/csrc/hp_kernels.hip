// Small device kernels of libhyperpower for gfx950 (CDNA4, wave64): the X0
// rules of Section 4 (norms, trace, transpose-scale), the fixed-order
// reductions of the stopping test and precision conversions. The hot kernel,
// the MFMA GEMM with the fused loop epilogue, is in hp_gemm.hip.
#include "hp_internal.h"
#include "hyperpower.h"

namespace hp {
namespace {

constexpr int kThreads = 256;  // 4 waves of 64

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum over a 256-thread block in a fixed order; the result is valid in thread 0.
__device__ double block_sum(double v) {
    __shared__ double red[kThreads / 64];
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

__device__ double block_max(double v) {
    __shared__ double red[kThreads / 64];
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// Small helpers.
// ---------------------------------------------------------------------------

// Column sums of |A| over 256-row chunks: part[chunk][col].
__global__ __launch_bounds__(kThreads) void k_abs_colsum_part(const double* __restrict__ A, int64_t lda,
                                                              int M, int N, double* __restrict__ part) {
    const int col = blockIdx.x * kThreads + threadIdx.x;
    const int chunk = blockIdx.y;
    if (col >= N) return;
    const int r0 = chunk * kColChunk, r1 = min(M, r0 + kColChunk);
    double s = 0.0;
#pragma unroll 8
    for (int r = r0; r < r1; ++r) s += fabs(A[(int64_t)r * lda + col]);
    part[(int64_t)chunk * N + col] = s;
}

// Row sums of |A|: one block per row.
__global__ __launch_bounds__(kThreads) void k_abs_rowsum(const double* __restrict__ A, int64_t lda, int N,
                                                         double* __restrict__ rows) {
    const int r = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < N; c += kThreads) s += fabs(A[(int64_t)r * lda + c]);
    s = block_sum(s);
    if (threadIdx.x == 0) rows[r] = s;
}

__global__ __launch_bounds__(kThreads) void k_alpha_norm1inf(const double* __restrict__ part, int nchunk,
                                                             int N, const double* __restrict__ rows,
                                                             int M, double* __restrict__ scal) {
    double m1 = 0.0;
    for (int c = threadIdx.x; c < N; c += kThreads) {
        double s = 0.0;
        for (int ch = 0; ch < nchunk; ++ch) s += part[(int64_t)ch * N + c];
        m1 = fmax(m1, s);
    }
    double mi = 0.0;
    for (int r = threadIdx.x; r < M; r += kThreads) mi = fmax(mi, rows[r]);
    m1 = block_max(m1);
    mi = block_max(mi);
    if (threadIdx.x == 0) {
        scal[SLOT_NORM1] = m1;
        scal[SLOT_NORMINF] = mi;
        // A = 0: X0 = alpha A^T = 0 whatever alpha (the zero matrix's inverse)
        scal[SLOT_ALPHA] = m1 * mi > 0.0 ? 1.0 / (m1 * mi) : 0.0;
    }
}

// H = X and Ht = X^T rounded to 16 bits (nearest even), through a 32x32 LDS
// tile so that both the reads and the transposed writes run along rows.
template <typename L>
__global__ __launch_bounds__(kThreads) void k_convert_h16(const float* __restrict__ X, int64_t ldx,
                                                          int M, int N, L* __restrict__ H,
                                                          int64_t ldh, L* __restrict__ Ht,
                                                          int64_t ldht) {
    __shared__ float tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += kThreads / 32) {
        const int row = by + r, col = bx + tx;
        float v = 0.f;
        if (row < M && col < N) {
            v = X[(int64_t)row * ldx + col];
            if (H) H[(int64_t)row * ldh + col] = (L)v;
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    if (!Ht) return;
    for (int r = ty; r < 32; r += kThreads / 32) {
        const int col = bx + r, row = by + tx;
        if (col < N && row < M) Ht[(int64_t)col * ldht + row] = (L)tile[tx][r];
    }
}

// ---- power iteration on A^T A for sigma_max(A)^2 ----
// y = A v: one wave per row, lanes striding along the row.
__global__ __launch_bounds__(kThreads) void k_gemv_rows(const double* __restrict__ A, int64_t lda,
                                                        int M, int N, const double* __restrict__ v,
                                                        double* __restrict__ y) {
    const int r = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= M) return;
    double s = 0.0;
    for (int c = lane; c < N; c += 64) s += A[(int64_t)r * lda + c] * v[c];
    s = wave_sum(s);
    if (lane == 0) y[r] = s;
}

// part[chunk][col] = sum over the chunk's 256 rows of A[r][col] y[r].
__global__ __launch_bounds__(kThreads) void k_gemv_cols_part(const double* __restrict__ A,
                                                             int64_t lda, int M, int N,
                                                             const double* __restrict__ y,
                                                             double* __restrict__ part) {
    const int col = blockIdx.x * kThreads + threadIdx.x;
    const int chunk = blockIdx.y;
    if (col >= N) return;
    const int r0 = chunk * 256, r1 = min(M, r0 + 256);
    double s = 0.0;
    for (int r = r0; r < r1; ++r) s += A[(int64_t)r * lda + col] * y[r];
    part[(int64_t)chunk * N + col] = s;
}

// z = A^T y from the chunk partials (fixed order), then v = z / ||z|| and
// scal[SLOT_ALPHA] = 1 / ||y||^2 (||y||^2 = v_old^T A^T A v_old, the Rayleigh
// quotient of the unit vector the step started from). One block.
__global__ __launch_bounds__(kThreads) void k_power_step(const double* __restrict__ part, int nchunk,
                                                         int N, const double* __restrict__ y, int M,
                                                         double* __restrict__ v,
                                                         double* __restrict__ scal) {
    __shared__ double zz;
    double yy = 0.0;
    for (int r = threadIdx.x; r < M; r += kThreads) yy += y[r] * y[r];
    double sz = 0.0;
    for (int c = threadIdx.x; c < N; c += kThreads) {
        double z = 0.0;
        for (int ch = 0; ch < nchunk; ++ch) z += part[(int64_t)ch * N + c];
        v[c] = z;  // unnormalised for now; scaled below
        sz += z * z;
    }
    yy = block_sum(yy);
    sz = block_sum(sz);
    if (threadIdx.x == 0) {
        zz = sz;
        scal[SLOT_TRACE] = yy;  // the Rayleigh quotient, kept for the caller
        scal[SLOT_ALPHA] = 1.0 / yy;
    }
    __syncthreads();
    const double inv = zz > 0.0 ? 1.0 / sqrt(zz) : 0.0;
    for (int c = threadIdx.x; c < N; c += kThreads) v[c] *= inv;
}

// v0: a fixed, unit, generic start vector (a multiplicative hash of the index
// spread over [0.5, 1.5], normalised).
__global__ __launch_bounds__(kThreads) void k_power_start(int N, double* __restrict__ v) {
    double s = 0.0;
    for (int c = threadIdx.x; c < N; c += kThreads) {
        const uint32_t h = (uint32_t)c * 2654435761u;
        const double x = 0.5 + (double)h * (1.0 / 4294967296.0);
        v[c] = x;
        s += x * x;
    }
    s = block_sum(s);
    __shared__ double tot;
    if (threadIdx.x == 0) tot = s;
    __syncthreads();
    const double inv = 1.0 / sqrt(tot);
    for (int c = threadIdx.x; c < N; c += kThreads) v[c] *= inv;
}

// Partial sums of P[i][j] * A[j][i] over 32x32 tiles (A read through LDS so
// that both operands are read along rows).
__global__ __launch_bounds__(kThreads) void k_trace_part(const double* __restrict__ P, int64_t ldp,
                                                         const double* __restrict__ A, int64_t lda,
                                                         int n, double* __restrict__ part) {
    __shared__ double t[32][33];
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int y = ty; y < 32; y += 8) {
        const int j = bj + y, i = bi + tx;
        t[y][tx] = (j < n && i < n) ? A[(int64_t)j * lda + i] : 0.0;
    }
    __syncthreads();
    double s = 0.0;
    for (int y = ty; y < 32; y += 8) {
        const int i = bi + y, j = bj + tx;
        if (i < n && j < n) s += P[(int64_t)i * ldp + j] * t[tx][y];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_trace_final(const double* __restrict__ part, int np,
                                                          double* __restrict__ scal) {
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += kThreads) s += part[i];
    s = block_sum(s);
    if (threadIdx.x == 0) {
        scal[SLOT_TRACE] = s;
        scal[SLOT_ALPHA] = 1.0 / s;
    }
}

__global__ __launch_bounds__(kThreads) void k_transpose_scale(const double* __restrict__ A, int64_t lda,
                                                              int M, int N, double* __restrict__ Y,
                                                              int64_t ldy,
                                                              const double* __restrict__ alpha) {
    __shared__ double t[32][33];
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const double al = alpha ? *alpha : 1.0;
    for (int y = ty; y < 32; y += 8) {
        const int i = bi + y, j = bj + tx;
        if (i < M && j < N) t[y][tx] = A[(int64_t)i * lda + j];
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int j = bj + y, i = bi + tx;
        if (j < N && i < M) Y[(int64_t)j * ldy + i] = al * t[tx][y];
    }
}

__global__ __launch_bounds__(kThreads) void k_scale(const double* __restrict__ A, int64_t lda, int M,
                                                    int N, double* __restrict__ Y, int64_t ldy,
                                                    const double* __restrict__ alpha) {
    const double al = *alpha;
    const int r = blockIdx.y;
    for (int c = blockIdx.x * kThreads + threadIdx.x; c < N; c += gridDim.x * kThreads)
        Y[(int64_t)r * ldy + c] = al * A[(int64_t)r * lda + c];
}

__global__ __launch_bounds__(kThreads) void k_identity(double* __restrict__ Y, int64_t ldy, int M, int N) {
    const int r = blockIdx.y;
    for (int c = blockIdx.x * kThreads + threadIdx.x; c < N; c += gridDim.x * kThreads)
        Y[(int64_t)r * ldy + c] = (r == c) ? 1.0 : 0.0;
}

// X0 = diag(1/a_11, ..., 1/a_nn), zero elsewhere (n x n)
__global__ __launch_bounds__(kThreads) void k_diag_inv(const double* __restrict__ A, int64_t lda,
                                                       int n, double* __restrict__ Y, int64_t ldy) {
    const int r = blockIdx.y;
    const double d = 1.0 / A[(int64_t)r * lda + r];
    for (int c = blockIdx.x * kThreads + threadIdx.x; c < n; c += gridDim.x * kThreads)
        Y[(int64_t)r * ldy + c] = (r == c) ? d : 0.0;
}

// Real form of a complex M x N matrix (interleaved re, im):
// E = [[Re A, -Im A], [Im A, Re A]], 2M x 2N.
__global__ __launch_bounds__(kThreads) void k_embed_complex(const double* __restrict__ A, int64_t lda,
                                                            int M, int N, double* __restrict__ E,
                                                            int64_t lde) {
    const int r = blockIdx.y;
    for (int c = blockIdx.x * kThreads + threadIdx.x; c < N; c += gridDim.x * kThreads) {
        const double re = A[2 * ((int64_t)r * lda + c)], im = A[2 * ((int64_t)r * lda + c) + 1];
        E[(int64_t)r * lde + c] = re;
        E[(int64_t)r * lde + N + c] = -im;
        E[(int64_t)(M + r) * lde + c] = im;
        E[(int64_t)(M + r) * lde + N + c] = re;
    }
}

// The complex N x M matrix whose real form is E (2N x 2M): the real part is
// E's upper-left block, the imaginary part its lower-left block.
__global__ __launch_bounds__(kThreads) void k_extract_complex(const double* __restrict__ E, int64_t lde,
                                                              int N, int M, double* __restrict__ X,
                                                              int64_t ldx) {
    const int r = blockIdx.y;
    for (int c = blockIdx.x * kThreads + threadIdx.x; c < M; c += gridDim.x * kThreads) {
        X[2 * ((int64_t)r * ldx + c)] = E[(int64_t)r * lde + c];
        X[2 * ((int64_t)r * ldx + c) + 1] = E[(int64_t)(N + r) * lde + c];
    }
}

__global__ __launch_bounds__(kThreads) void k_zero_u32(unsigned* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = 0u;
}

__global__ __launch_bounds__(kThreads) void k_reduce_pairs(const double* __restrict__ part, int nb,
                                                           double* __restrict__ scal,
                                                           double* __restrict__ host,
                                                           double seq) {
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) {
        s0 += part[2 * b];
        s1 += part[2 * b + 1];
    }
    s0 = block_sum(s0);
    s1 = block_sum(s1);
    if (threadIdx.x == 0) {
        scal[SLOT_DIFF2] = s0;
        scal[SLOT_REF2] = s1;
        if (host) {
            // the other slots were written by earlier launches on this stream
            for (int i = 0; i < SLOT_COUNT; ++i)
                host[i] = i == SLOT_DIFF2 ? s0 : i == SLOT_REF2 ? s1 : scal[i];
            __threadfence_system();
            // last: the host polls this number before reading the sums
            host[SLOT_COUNT] = seq;
        }
    }
}

// Row sums of |X1 - X0| (one block per row), accumulated in FP64.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_diff_rowsum(const T* __restrict__ X1, int64_t ld1,
                                                          const T* __restrict__ X0, int64_t ld0,
                                                          int N, double* __restrict__ rows,
                                                          const int* gate) {
    if (gate_closed(gate, GATE_LIVE)) return;
    const int r = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < N; c += kThreads)
        s += fabs((double)X1[(int64_t)r * ld1 + c] - (double)X0[(int64_t)r * ld0 + c]);
    s = block_sum(s);
    if (threadIdx.x == 0) rows[r] = s;
}

__global__ __launch_bounds__(kThreads) void k_max_to_slot(const double* __restrict__ v, int n,
                                                          double* __restrict__ scal, int slot,
                                                          const int* gate) {
    if (gate_closed(gate, GATE_LIVE)) return;
    double m = 0.0;
    bool nan = false;
    for (int i = threadIdx.x; i < n; i += kThreads) {
        const double x = v[i];
        if (x != x) nan = true;
        m = fmax(m, x);
    }
    if (nan) m = __builtin_nan("");
    // NaN-propagating block max
    __shared__ int any_nan;
    if (threadIdx.x == 0) any_nan = 0;
    __syncthreads();
    if (nan) any_nan = 1;
    __syncthreads();
    const double r = block_max(nan ? 0.0 : m);
    if (threadIdx.x == 0) scal[slot] = any_nan ? __builtin_nan("") : r;
}

// Row sums of squares of an M x N matrix (one block per row).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_rowsumsq(const T* __restrict__ X, int64_t ldx, int N,
                                                       double* __restrict__ rows) {
    const int r = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < N; c += kThreads) {
        const double v = (double)X[(int64_t)r * ldx + c];
        s += v * v;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) rows[r] = s;
}

__global__ __launch_bounds__(kThreads) void k_sum_to_slot(const double* __restrict__ v, int n,
                                                          double* __restrict__ scal, int slot) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += v[i];
    s = block_sum(s);
    if (threadIdx.x == 0) scal[slot] = s;
}

// Row sums of (P - c Q)^2, or of (P - c Q^T)^2 when `transposed` (P, Q are
// M x N; for the transposed form M == N and Q^T is read through LDS tiles).
__global__ __launch_bounds__(kThreads) void k_rowdiffsq(const double* __restrict__ P, int64_t ldp,
                                                        const double* __restrict__ Q, int64_t ldq,
                                                        int M, int N, double c,
                                                        double* __restrict__ rows) {
    const int r = blockIdx.x;
    double s = 0.0;
    for (int j = threadIdx.x; j < N; j += kThreads) {
        const double v = P[(int64_t)r * ldp + j] - (Q ? c * Q[(int64_t)r * ldq + j] : 0.0);
        s += v * v;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) rows[r] = s;
}

// Partial sums of (P[i][j] - P[j][i])^2 over 32x32 tiles (n x n).
__global__ __launch_bounds__(kThreads) void k_asym_part(const double* __restrict__ P, int64_t ldp,
                                                        int n, double* __restrict__ part) {
    __shared__ double t[32][33];
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int y = ty; y < 32; y += 8) {
        const int j = bj + y, i = bi + tx;
        t[y][tx] = (j < n && i < n) ? P[(int64_t)j * ldp + i] : 0.0;
    }
    __syncthreads();
    double s = 0.0;
    for (int y = ty; y < 32; y += 8) {
        const int i = bi + y, j = bj + tx;
        if (i < n && j < n) {
            const double v = P[(int64_t)i * ldp + j] - t[tx][y];
            s += v * v;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// One block per problem: fixed-order sums of that problem's partial pairs.
struct ReduceEntryDev {
    const double* partials;
    int npairs;
    int pad;
};

__global__ __launch_bounds__(kThreads) void k_reduce_pairs_grouped(const int* __restrict__ count,
                                                                   const ReduceEntryDev* __restrict__ ents,
                                                                   double* __restrict__ out) {
    if ((int)blockIdx.x >= *count) return;  // uniform per block
    const ReduceEntryDev e = ents[blockIdx.x];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < e.npairs; b += kThreads) {
        s0 += e.partials[2 * b];
        s1 += e.partials[2 * b + 1];
    }
    s0 = block_sum(s0);
    s1 = block_sum(s1);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = s0;
        out[2 * blockIdx.x + 1] = s1;
        // (`out` may be pinned host memory: the signal launched after this
        // kernel orders these writes before its flag)
    }
}

// The decision fields of the device loop (the doubles before its change
// history) to pinned host memory, then `seq` after them.
__global__ void k_loop_report(const double* __restrict__ L, double* __restrict__ host, int n,
                              double seq) {
    if (threadIdx.x != 0) return;
    for (int i = 0; i < n; ++i) host[i] = L[i];
    __threadfence_system();
    host[n] = seq;
}

// One more loop signalled: the device counter, then its value in `flag`
// (pinned host memory), which the host polls.
__global__ void k_signal_host(unsigned long long* __restrict__ counter, double* __restrict__ flag) {
    if (threadIdx.x != 0) return;
    const unsigned long long v = *counter + 1;
    *counter = v;
    // the earlier launches' writes to host memory are complete; one system
    // fence per loop orders them before the flag
    __threadfence_system();
    *flag = (double)v;
}

// Elementwise precision conversion of an M x N matrix (round to nearest even
// when narrowing).
template <typename S, typename D>
__global__ __launch_bounds__(kThreads) void k_convert(const S* __restrict__ X, int64_t ldx, int M,
                                                      int N, D* __restrict__ Y, int64_t ldy) {
    const int r = blockIdx.y;
    for (int c = blockIdx.x * kThreads + threadIdx.x; c < N; c += gridDim.x * kThreads)
        Y[(int64_t)r * ldy + c] = (D)X[(int64_t)r * ldx + c];
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------

hipError_t alpha_norm1inf(const double* A, int64_t lda, int64_t M, int64_t N, double* tmp,
                          double* scal, hipStream_t s) {
    const int nchunk = (int)cdiv(M, kColChunk);
    double* part = tmp;
    double* rows = tmp + (int64_t)nchunk * N;
    hipLaunchKernelGGL(k_abs_colsum_part, dim3((unsigned)cdiv(N, kThreads), nchunk), dim3(kThreads),
                       0, s, A, lda, (int)M, (int)N, part);
    hipLaunchKernelGGL(k_abs_rowsum, dim3((unsigned)M), dim3(kThreads), 0, s, A, lda, (int)N, rows);
    hipLaunchKernelGGL(k_alpha_norm1inf, dim3(1), dim3(kThreads), 0, s, part, nchunk, (int)N, rows,
                       (int)M, scal);
    return hipGetLastError();
}

template <typename L>
hipError_t convert_h16_t(const float* X, int64_t ldx, int64_t M, int64_t N, L* H, int64_t ldh,
                         L* Ht, int64_t ldht, hipStream_t s) {
    hipLaunchKernelGGL(k_convert_h16<L>, dim3((unsigned)cdiv(N, 32), (unsigned)cdiv(M, 32)),
                       dim3(kThreads), 0, s, X, ldx, (int)M, (int)N, H, ldh, Ht, ldht);
    return hipGetLastError();
}

hipError_t convert_h16(const float* X, int64_t ldx, int64_t M, int64_t N, LowPrec lp, void* H,
                       int64_t ldh, void* Ht, int64_t ldht, hipStream_t s) {
    if (lp == LOWP_BF16)
        return convert_h16_t<__bf16>(X, ldx, M, N, static_cast<__bf16*>(H), ldh,
                                     static_cast<__bf16*>(Ht), ldht, s);
    return convert_h16_t<_Float16>(X, ldx, M, N, static_cast<_Float16*>(H), ldh,
                                   static_cast<_Float16*>(Ht), ldht, s);
}

hipError_t alpha_sigma_max2(const double* A, int64_t lda, int64_t M, int64_t N, int iters,
                            double* tmp, double* scal, hipStream_t s) {
    const int nchunk = (int)cdiv(M, 256);
    double* v = tmp;
    double* y = v + N;
    double* part = y + M;
    hipLaunchKernelGGL(k_power_start, dim3(1), dim3(kThreads), 0, s, (int)N, v);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_gemv_rows, dim3((unsigned)cdiv(M, kThreads / 64)), dim3(kThreads), 0, s,
                           A, lda, (int)M, (int)N, v, y);
        hipLaunchKernelGGL(k_gemv_cols_part, dim3((unsigned)cdiv(N, kThreads), nchunk),
                           dim3(kThreads), 0, s, A, lda, (int)M, (int)N, y, part);
        hipLaunchKernelGGL(k_power_step, dim3(1), dim3(kThreads), 0, s, part, nchunk, (int)N, y,
                           (int)M, v, scal);
    }
    return hipGetLastError();
}

hipError_t alpha_trace(const double* P, int64_t ldp, const double* A, int64_t lda, int64_t n,
                       double* tmp, double* scal, hipStream_t s) {
    const int nt = (int)cdiv(n, 32);
    hipLaunchKernelGGL(k_trace_part, dim3(nt, nt), dim3(kThreads), 0, s, P, ldp, A, lda, (int)n, tmp);
    hipLaunchKernelGGL(k_trace_final, dim3(1), dim3(kThreads), 0, s, tmp, nt * nt, scal);
    return hipGetLastError();
}

hipError_t transpose_scale(const double* A, int64_t lda, int64_t M, int64_t N, double* Y,
                           int64_t ldy, const double* alpha_dev, hipStream_t s) {
    if (!A || !Y) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_transpose_scale, dim3((unsigned)cdiv(N, 32), (unsigned)cdiv(M, 32)),
                       dim3(kThreads), 0, s, A, lda, (int)M, (int)N, Y, ldy, alpha_dev);
    return hipGetLastError();
}

hipError_t scale(const double* A, int64_t lda, int64_t M, int64_t N, double* Y, int64_t ldy,
                 const double* alpha_dev, hipStream_t s) {
    if (!A || !Y || !alpha_dev) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(N, kThreads), 16);
    hipLaunchKernelGGL(k_scale, dim3(gx, (unsigned)M), dim3(kThreads), 0, s, A, lda, (int)M, (int)N,
                       Y, ldy, alpha_dev);
    return hipGetLastError();
}

hipError_t set_identity(double* Y, int64_t ldy, int64_t M, int64_t N, hipStream_t s) {
    if (!Y) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(N, kThreads), 16);
    hipLaunchKernelGGL(k_identity, dim3(gx, (unsigned)M), dim3(kThreads), 0, s, Y, ldy, (int)M, (int)N);
    return hipGetLastError();
}

hipError_t diag_inv(const double* A, int64_t lda, int64_t n, double* Y, int64_t ldy, hipStream_t s) {
    if (!A || !Y) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(n, kThreads), 16);
    hipLaunchKernelGGL(k_diag_inv, dim3(gx, (unsigned)n), dim3(kThreads), 0, s, A, lda, (int)n, Y, ldy);
    return hipGetLastError();
}

hipError_t embed_complex(const double* A, int64_t lda, int64_t M, int64_t N, double* E, int64_t lde,
                         hipStream_t s) {
    if (!A || !E || M < 1 || N < 1) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(N, kThreads), 16);
    hipLaunchKernelGGL(k_embed_complex, dim3(gx, (unsigned)M), dim3(kThreads), 0, s, A, lda, (int)M,
                       (int)N, E, lde);
    return hipGetLastError();
}

hipError_t extract_complex(const double* E, int64_t lde, int64_t N, int64_t M, double* X, int64_t ldx,
                           hipStream_t s) {
    if (!E || !X || M < 1 || N < 1) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(M, kThreads), 16);
    hipLaunchKernelGGL(k_extract_complex, dim3(gx, (unsigned)N), dim3(kThreads), 0, s, E, lde, (int)N,
                       (int)M, X, ldx);
    return hipGetLastError();
}

hipError_t zero_u32(unsigned* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>(cdiv(n, kThreads), 1024);
    hipLaunchKernelGGL(k_zero_u32, dim3(g), dim3(kThreads), 0, s, p, n);
    return hipGetLastError();
}

hipError_t reduce_pairs(const double* partials, int nblocks, double* scal, hipStream_t s,
                        double* host, double seq) {
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(kThreads), 0, s, partials, nblocks, scal,
                       host, seq);
    return hipGetLastError();
}

template <typename T>
static hipError_t diff_norm_inf_t(const T* X1, int64_t ld1, const T* X0, int64_t ld0, int64_t M,
                                  int64_t N, double* tmp, double* scal, hipStream_t s,
                                  const int* gate = nullptr) {
    hipLaunchKernelGGL(k_diff_rowsum<T>, dim3((unsigned)M), dim3(kThreads), 0, s, X1, ld1, X0, ld0,
                       (int)N, tmp, gate);
    hipLaunchKernelGGL(k_max_to_slot, dim3(1), dim3(kThreads), 0, s, tmp, (int)M, scal,
                       (int)SLOT_DINF, gate);
    return hipGetLastError();
}

hipError_t diff_norm_inf(const double* X1, int64_t ld1, const double* X0, int64_t ld0, int64_t M,
                         int64_t N, double* tmp, double* scal, hipStream_t s) {
    return diff_norm_inf_t(X1, ld1, X0, ld0, M, N, tmp, scal, s);
}

hipError_t diff_norm_inf(const float* X1, int64_t ld1, const float* X0, int64_t ld0, int64_t M,
                         int64_t N, double* tmp, double* scal, hipStream_t s) {
    return diff_norm_inf_t(X1, ld1, X0, ld0, M, N, tmp, scal, s);
}

}  // namespace hp

namespace hp {

template <typename S, typename D>
static hipError_t convert_impl(const S* X, int64_t ldx, int64_t M, int64_t N, D* Y, int64_t ldy,
                               hipStream_t s) {
    if (!X || !Y) return hipErrorInvalidValue;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(N, kThreads), 16);
    hipLaunchKernelGGL((k_convert<S, D>), dim3(gx, (unsigned)M), dim3(kThreads), 0, s, X, ldx,
                       (int)M, (int)N, Y, ldy);
    return hipGetLastError();
}

hipError_t convert(const double* X, int64_t ldx, int64_t M, int64_t N, float* Y, int64_t ldy,
                   hipStream_t s) {
    return convert_impl(X, ldx, M, N, Y, ldy, s);
}

hipError_t convert(const float* X, int64_t ldx, int64_t M, int64_t N, double* Y, int64_t ldy,
                   hipStream_t s) {
    return convert_impl(X, ldx, M, N, Y, ldy, s);
}

}  // namespace hp

namespace hp {

struct ReduceEntry {
    const double* partials;
    int npairs;
    int pad;
};
static_assert(sizeof(ReduceEntry) == sizeof(ReduceEntryDev), "reduce table layout");

hipError_t loop_report(const DevLoop* L, double* host, double seq, hipStream_t s) {
    hipLaunchKernelGGL(k_loop_report, dim3(1), dim3(64), 0, s, reinterpret_cast<const double*>(L),
                       host, kLoopReportDoubles, seq);
    return hipGetLastError();
}

hipError_t signal_host(unsigned long long* counter, double* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_signal_host, dim3(1), dim3(64), 0, s, counter, flag);
    return hipGetLastError();
}

hipError_t reduce_pairs_grouped(const int* count, const ReduceEntry* ents, int grid, double* out,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_pairs_grouped, dim3((unsigned)grid), dim3(kThreads), 0, s, count,
                       reinterpret_cast<const ReduceEntryDev*>(ents), out);
    return hipGetLastError();
}

}  // namespace hp

namespace hp {

hipError_t sumsq(const float* X, int64_t ldx, int64_t M, int64_t N, double* tmp, double* scal,
                 int slot, hipStream_t s) {
    if (!X || !tmp || !scal) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rowsumsq<float>, dim3((unsigned)M), dim3(kThreads), 0, s, X, ldx, (int)N, tmp);
    hipLaunchKernelGGL(k_sum_to_slot, dim3(1), dim3(kThreads), 0, s, tmp, (int)M, scal, slot);
    return hipGetLastError();
}

}  // namespace hp

namespace hp {

hipError_t diffsq(const double* P, int64_t ldp, const double* Q, int64_t ldq, double c, int64_t M,
                  int64_t N, double* tmp, double* scal, int slot, hipStream_t s) {
    if (!P || !tmp || !scal) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rowdiffsq, dim3((unsigned)M), dim3(kThreads), 0, s, P, ldp, Q, ldq, (int)M,
                       (int)N, c, tmp);
    hipLaunchKernelGGL(k_sum_to_slot, dim3(1), dim3(kThreads), 0, s, tmp, (int)M, scal, slot);
    return hipGetLastError();
}

hipError_t asymsq(const double* P, int64_t ldp, int64_t n, double* tmp, double* scal, int slot,
                  hipStream_t s) {
    const int nt = (int)cdiv(n, 32);
    hipLaunchKernelGGL(k_asym_part, dim3(nt, nt), dim3(kThreads), 0, s, P, ldp, (int)n, tmp);
    hipLaunchKernelGGL(k_sum_to_slot, dim3(1), dim3(kThreads), 0, s, tmp, nt * nt, scal, slot);
    return hipGetLastError();
}

}  // namespace hp

// ---------------------------------------------------------------------------
// Loop control on the device (hp_params.device_stop): the decisions of
// LoopState::step for a solve whose every loop is FP64, taken from the
// stopping sums the loop's update product left, so that the host can enqueue
// loops without reading those sums; the kernels of a loop consult the flags
// (gate_closed) and skip their work once the solve is done, or when they
// belong to the other (plain / stabilised) form of the loop.
// ---------------------------------------------------------------------------

namespace hp {
namespace {

__global__ void k_loop_init(DevLoop* L, int stab_always) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    L->done = 0;
    L->stabilising = stab_always;
    L->save_best = 0;
    L->status = HP_MAXITER;
    L->k = 0;
    L->converging = 0;
    L->switch_iter = stab_always ? 0 : -1;
    L->result_idx = -1;
    L->have_best = 0;
    L->d_prev = 0.0;
    L->best_d = 0.0;
    L->stop_last = 0.0;
    L->d_last = 0.0;
}

__global__ __launch_bounds__(kThreads) void k_reduce_pairs_gated(const double* __restrict__ part,
                                                                 int nb_plain, int nb_stab,
                                                                 double* __restrict__ scal,
                                                                 const DevLoop* L) {
    if (L->done) return;
    const int nb = L->stabilising ? nb_stab : nb_plain;
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) {
        s0 += part[2 * b];
        s1 += part[2 * b + 1];
    }
    s0 = block_sum(s0);
    s1 = block_sum(s1);
    if (threadIdx.x == 0) {
        scal[SLOT_DIFF2] = s0;
        scal[SLOT_REF2] = s1;
    }
}

// The decision after loop k (its input iterate is index k % 2, its output
// (k + 1) % 2), in the order and arithmetic of LoopState::step.
__global__ void k_loop_step(const double* __restrict__ scal, DevLoop* L,
                            const StepParams* __restrict__ Pp) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || L->done) return;
    const StepParams P = *Pp;
    L->save_best = 0;
    const int k = L->k;
    const int ik = k & 1, in_ = ik ^ 1;
    const double diff2 = scal[SLOT_DIFF2], ref2 = scal[SLOT_REF2];
    const double dinf = P.have_dinf ? scal[SLOT_DINF] : 0.0;
    // a zero iterate from alpha = 0 (A = 0): no change, as in LoopState
    const double d = (diff2 == 0.0 && ref2 == 0.0 && P.alpha == 0.0) ? 0.0
                                                                   : sqrt(diff2) / sqrt(ref2);
    if (k < 128) {
        L->d_hist[k] = d;
        if (P.have_dinf) L->dinf_hist[k] = dinf;
    }
    L->d_last = d;
    L->k = k + 1;
    const bool finite = isfinite(d) && isfinite(diff2) && (!P.have_dinf || isfinite(dinf));
    const int fallback = (P.keep_best && L->have_best && !L->converging) ? 3 : ik;
    if (!finite) {
        L->status = HP_NONFINITE;
        L->result_idx = fallback;
        L->done = 1;
        return;
    }
    double sval;
    bool passed;
    if (P.stop_rule == HP_STOP_ABS_INF) {
        sval = dinf;
        passed = dinf <= P.tol;
    } else if (P.stop_rule == HP_STOP_PAPER_4_1) {
        sval = diff2 == 0.0 ? 0.0 : sqrt(diff2) / (pow(P.order, (double)k) * P.alpha);
        passed = sval < P.tol;
    } else {
        sval = d;
        passed = d < P.tol;
    }
    L->stop_last = sval;
    if (passed) {
        L->status = HP_OK;
        L->result_idx = in_;
        L->done = 1;
        return;
    }
    // the first stabilised loop after the switch is not compared (LoopState)
    const bool first_stab = P.variant == HP_VARIANT_STABILISED && L->switch_iter > 0 &&
                            k == L->switch_iter;
    if (L->converging && k > 0 && !first_stab && d >= L->d_prev) {
        L->status = HP_STAGNATED;
        L->result_idx = ik;
        L->done = 1;
        return;
    }
    if (!L->converging && d > P.diverge) {
        L->status = HP_DIVERGED;
        L->result_idx = fallback;
        L->done = 1;
        return;
    }
    if (d < P.tau) {
        L->converging = 1;
        if (P.variant == HP_VARIANT_STABILISED && !L->stabilising) {
            L->stabilising = 1;
            L->switch_iter = k + 1;
        }
    }
    if (P.keep_best && !L->converging && (!L->have_best || d < L->best_d)) {
        L->best_d = d;
        L->have_best = 1;
        L->save_best = 1;
    }
    L->d_prev = d;
    if (k + 1 >= P.max_iter) {
        L->status = HP_MAXITER;
        L->result_idx = in_;
        L->done = 1;
    }
}

__global__ __launch_bounds__(kThreads) void k_copy_gated(const double* __restrict__ X, int64_t ldx,
                                                         int M, int N, double* __restrict__ Y,
                                                         int64_t ldy, const int* gate, int mode) {
    if (gate_closed(gate, mode)) return;
    const int r = blockIdx.y;
    for (int c = blockIdx.x * kThreads + threadIdx.x; c < N; c += gridDim.x * kThreads)
        Y[(int64_t)r * ldy + c] = X[(int64_t)r * ldx + c];
}

}  // namespace

hipError_t loop_init(DevLoop* L, int stab_always, hipStream_t s) {
    hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(64), 0, s, L, stab_always);
    return hipGetLastError();
}

hipError_t reduce_pairs_gated(const double* partials, int nb_plain, int nb_stab, double* scal,
                              const DevLoop* L, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_pairs_gated, dim3(1), dim3(kThreads), 0, s, partials, nb_plain,
                       nb_stab, scal, L);
    return hipGetLastError();
}

hipError_t diff_norm_inf_gated(const double* X1, int64_t ld1, const double* X0, int64_t ld0,
                               int64_t M, int64_t N, double* tmp, double* scal, const DevLoop* L,
                               hipStream_t s) {
    return diff_norm_inf_t(X1, ld1, X0, ld0, M, N, tmp, scal, s,
                           reinterpret_cast<const int*>(L));
}

hipError_t loop_step(const double* scal, DevLoop* L, const StepParams* P, hipStream_t s) {
    hipLaunchKernelGGL(k_loop_step, dim3(1), dim3(64), 0, s, scal, L, P);
    return hipGetLastError();
}

hipError_t copy_gated(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                      int64_t cols, const DevLoop* L, int mode, hipStream_t s) {
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(cols, kThreads), 64);
    hipLaunchKernelGGL(k_copy_gated, dim3(gx, (unsigned)rows), dim3(kThreads), 0, s, src, lds,
                       (int)rows, (int)cols, dst, ldd, reinterpret_cast<const int*>(L), mode);
    return hipGetLastError();
}

}  // namespace hp
