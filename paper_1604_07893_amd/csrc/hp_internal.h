// Internal interface between the host driver (hp_driver.cpp) and the device
// kernels (hp_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace hp {

// Device scalar slots (doubles) in the workspace's scalar area.
enum ScalarSlot : int {
    SLOT_ALPHA = 0,      // alpha of X0
    SLOT_DIFF2 = 1,      // sum (X_{k+1} - X_k)^2
    SLOT_REF2 = 2,       // sum X_k^2
    SLOT_DINF = 3,       // ||X_{k+1} - X_k||_inf
    SLOT_TRACE = 4,      // Tr(A^{l+1})
    SLOT_NORM1 = 5,      // ||A||_1
    SLOT_NORMINF = 6,    // ||A||_inf
    SLOT_RNORM2 = 7,     // ||R||_F^2 of a lower stage's last residual
    SLOT_COUNT = 8
};

// Loop control kept on the device (hp_params.device_stop): the stop, switch
// and guard decisions of one FP64 solve, taken by k_loop_step from the
// reduced stopping sums of each loop, so that loops can be enqueued without
// the host reading those sums. The first three ints are what the kernels of a
// loop read to decide whether to run (gate_closed).
struct DevLoop {
    int done;          // a decision ended the solve: every later kernel skips
    int stabilising;   // the next loop runs the stabilising product
    int save_best;     // copy this loop's input to the best-iterate slot
    int status;        // HP_* outcome once done
    int k;             // loops run
    int converging;    // some change below tau_switch was seen
    int switch_iter;   // first loop run stabilised (-1: none)
    int result_idx;    // iterate to return (0, 1 or the best slot 3)
    int have_best;
    int pad[3];
    double d_prev, best_d, stop_last, d_last;
    double d_hist[128];     // HP_HIST
    double dinf_hist[128];
};

// When a gated kernel runs (EpilogueT::gate_mode, and the gated elementwise
// kernels): always; while the solve is live; in a live loop that is plain /
// stabilised (the flag as the previous loop's decision left it); when the
// last decision asked to keep the best iterate.
enum GateMode : int { GATE_NONE = 0, GATE_LIVE = 1, GATE_PLAIN = 2, GATE_STAB = 3, GATE_SAVE = 4 };

__host__ __device__ inline bool gate_closed(const int* g, int mode) {
    if (mode == GATE_NONE || !g) return false;
    if (mode == GATE_SAVE) return g[2] == 0;
    if (g[0]) return true;
    if (mode == GATE_PLAIN) return g[1] != 0;
    if (mode == GATE_STAB) return g[1] == 0;
    return false;
}

// Fused GEMM epilogue. For output o (0..2) with out[o] != nullptr:
//   out[o][i][j] = id[o]*[i==j] + acc_c[o]*acc + g1[o]*D1[i][j] + g2[o]*D2[i][j]
// If ref != nullptr, each block also writes FP64 partial sums
//   partials[2*b] = sum (out0 - ref)^2, partials[2*b+1] = sum ref^2
// over the elements it owns (b = linear block index).
template <typename T>
struct EpilogueT {
    T* out[3];
    int64_t ldo[3];
    double id[3];
    double acc_c[3];
    double g1[3];
    double g2[3];
    const T* D1;
    int64_t ld1;
    const T* D2;
    int64_t ld2;
    const T* ref;
    int64_t ldref;
    double* partials;
    // > 0: values of output 0 with |v| < chop are stored as 0 (and enter the
    // stopping sums as 0); 0 = off
    double chop;
    // Split-K scratch, read only by the split tiles (TILE_128x128_W8_S2/S4):
    // split_slots partial tiles of 128 x 128 elements, then one arrival
    // counter per output tile. The counters are zero before a launch and every
    // launch leaves them zero. Without scratch (or too little) those tiles run
    // unsplit.
    T* split_part;
    unsigned* split_cnt;
    int64_t split_slots;
    // arrival counters available at split_cnt (0: as many as split_slots)
    int64_t split_ncnt;
    // nonzero: the caller guarantees that the product is symmetric in exact
    // arithmetic (M == N; e.g. a polynomial in R = I - X A when X A is
    // symmetric). The symmetric launch (gemm_sym_runs) then computes the
    // tiles on and above the diagonal only, each element i <= j once, and
    // stores every output at (i, j) and (j, i); D1/D2 are read at i <= j only.
    // Requires ref == nullptr; other launches compute the full product.
    int sym;
    // 16-bit copies of the outputs, written by the 16-bit-operand kernel only
    // (gemm_h16) in its own operand type: h[o] row-major (ld ldh[o]) and ht[o]
    // transposed (ld ldht[o]); either may be null.
    void* h[3];
    int64_t ldh[3];
    void* ht[3];
    int64_t ldht[3];
    // gemm_h16 only: nonzero skips the FP32 store of output o (when only its
    // 16-bit copies are read later); the stopping sums still use the value
    int skip32[3];
    // FP64/FP32 kernels (gemm): with gate_mode != GATE_NONE the whole launch
    // returns at once when gate_closed(gate, gate_mode) (a DevLoop's flags)
    const int* gate;
    int gate_mode;
};
using Epilogue = EpilogueT<double>;

template <typename T>
inline EpilogueT<T> epilogue_plain(T* C, int64_t ldc, double acc_c = 1.0, double id = 0.0) {
    EpilogueT<T> e{};
    e.out[0] = C;
    e.ldo[0] = ldc;
    e.acc_c[0] = acc_c;
    e.id[0] = id;
    return e;
}

// Block-tile configurations of the MFMA GEMM (hp_gemm.hip).
enum GemmTile : int {
    TILE_128x128_W4 = 0,  // 4 waves, 64x64 each
    TILE_128x128_W8 = 1,  // 8 waves, 64x32 each
    TILE_128x64_W4 = 2,   // 4 waves, 64x32 each
    TILE_64x64_W4 = 3,    // 4 waves, 32x32 each
    TILE_256x128_W8 = 4,  // 8 waves, 64x64 each
    TILE_128x64_W8 = 5,   // 8 waves, 32x32 each
    TILE_64x128_W8 = 6,   // 8 waves, 32x32 each
    TILE_128x128_W8_K2 = 7,  // as TILE_128x128_W8 with a K-tile twice as deep
    TILE_128x128_W16 = 8, // 16 waves, 32x32 each
    TILE_128x128_W8_P2 = 9,   // TILE_128x128_W8 loading two K-tiles ahead
    TILE_128x128_W16_P2 = 10, // TILE_128x128_W16 loading two K-tiles ahead
    TILE_128x128_W8_S2 = 11,  // TILE_128x128_W8 with K split over 2 blocks per tile
    TILE_128x128_W8_S4 = 12,  // TILE_128x128_W8 with K split over 4 blocks per tile
    TILE_128x128_W16_K2_P2 = 13,  // TILE_128x128_W16_P2 with a K-tile twice as deep
    TILE_256x256_W8 = 14,   // 16-bit-operand kernel only: 8 waves, 128x64 each
    TILE_256x256_W16 = 15,  // 16-bit-operand kernel only: 16 waves, 64x64 each
    TILE_256x256_W8_DMA = 16,   // TILE_256x256_W8 with load-to-LDS tiles (K % 64 == 0)
    TILE_256x256_W16_DMA = 17,  // TILE_256x256_W16 with load-to-LDS tiles (K % 64 == 0)
    TILE_32x32_W4_K4 = 18,  // 4 waves, 16x16 each, K-tile four times as deep (small products)
    TILE_128x128_W4_DMA = 19,  // FP64 only: 4 waves of 64x64, load-to-LDS tiles (K % 16 == 0)
    TILE_256x256_W4_DMA = 20,  // FP32 only: 4 waves of 128x128, load-to-LDS tiles (K % 32 == 0)
    TILE_COUNT = 21
};

// Blocks (and partial-sum pairs) a launch with this tile uses for M x N.
int gemm_blocks(GemmTile t, int64_t M, int64_t N);
// The largest of gemm_blocks over every tile (sizes the partials buffer).
int gemm_max_blocks(int64_t M, int64_t N);
// Tile choice for an M x N x K product of element type `gt`.
// With allow_split false the choice is among the unsplit tiles.
enum GemmType : int { GT_F64 = 0, GT_F32 = 1, GT_LOWP = 2, GT_H16 = 3 };
// Whether the kernels of GEMM type gt run tile t (with the shape gemm_blocks
// assumes); gemm/gemm_lowp/gemm_h16 reject the others.
bool gemm_runs(GemmTile t, GemmType gt);
GemmTile gemm_pick_tile(int64_t M, int64_t N, int64_t K, GemmType gt, bool allow_split = true);
// Whether split tile t runs split for this product given `slots` partial
// tiles of scratch (it runs unsplit otherwise).
bool gemm_split_runs(GemmTile t, int64_t M, int64_t N, int64_t K, GemmType gt, int64_t slots);
// Split-K scratch (partial tiles of 128 x 128 elements; as many arrival
// counters) that tile t needs for an M x N x K product: 0 for unsplit tiles.
int64_t gemm_split_slots(GemmTile t, int64_t M, int64_t N, int64_t K);
// Symmetric products (EpilogueT::sym) of GEMM type gt run on tile t as one
// balanced launch over the upper-triangle tiles (stream-K: every block takes
// an equal share of the triangle's K-steps; a tile split between blocks is
// finished by the last of them to arrive, adding the pieces in K order).
bool gemm_sym_runs(GemmTile t, GemmType gt);
// Scratch the symmetric launch of an n x n x K product on tile t needs:
// partial tiles (of 128 x 128 elements of the GEMM type) and arrival counters;
// 0 and 0 when t has no symmetric launch.
void gemm_sym_scratch(GemmTile t, GemmType gt, int64_t n, int64_t* slots, int64_t* counters);
// Whether gemm() runs this call as the symmetric launch (ep.sym set, M == N,
// no stopping sums, a tile with that launch and enough scratch); it runs the
// full product otherwise. The operands decide whether the load-to-LDS tile's
// symmetric kernel applies.
bool gemm_sym_launches(GemmTile t, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                       const double* B, int64_t ldb, const EpilogueT<double>& ep);
bool gemm_sym_launches(GemmTile t, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                       const float* B, int64_t ldb, const EpilogueT<float>& ep);

// Zero n unsigned counters (a fill kernel: safe inside stream capture).
hipError_t zero_u32(unsigned* p, int64_t n, hipStream_t s);

// C = epilogue(A[M x K] * B[K x N]); all row-major, lda/ldb multiples of 16
// bytes, pointers 16-byte aligned.
hipError_t gemm(GemmTile t, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                const double* B, int64_t ldb, const EpilogueT<double>& ep, hipStream_t s);
hipError_t gemm(GemmTile t, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
                const float* B, int64_t ldb, const EpilogueT<float>& ep, hipStream_t s);

// Grouped products: one persistent launch computes every entry of a device
// table. Tiles are square, grouped_tile_dim(cfg) on a side, for the grouped
// tile configuration cfg (GroupedTile); entry e covers tiles
// [tile_start, tile_start + tiles_m * tiles_n) and writes its partial sums
// (if ep.ref) to ep.partials[2*local_tile ...].
struct GroupHeader {
    int count;        // entries in the table
    int total_tiles;  // sum of the entries' tile counts
};
template <typename T>
struct GroupEntry {
    int M, N, K, tiles_n;
    int tile_start, pad;
    const T* A;
    int64_t lda;
    const T* B;
    int64_t ldb;
    EpilogueT<T> ep;
};
// Tile configurations of the grouped kernel (each a tile shape of the
// single-launch kernel, 4 waves): 64 x 64 (the default), 128 x 128, and 32 x 32
// with a K-tile four times as deep (small products).
enum GroupedTile : int { GTILE_64 = 0, GTILE_128 = 1, GTILE_32 = 2, GTILE_COUNT = 3 };
int grouped_tile_dim(int cfg);
hipError_t gemm_grouped(const GroupHeader* hdr, const GroupEntry<double>* ents, int grid, int cfg,
                        hipStream_t s);
hipError_t gemm_grouped(const GroupHeader* hdr, const GroupEntry<float>* ents, int grid, int cfg,
                        hipStream_t s);

// 16-bit MFMA product of FP32 matrices (operands rounded to nearest even while
// staged, FP32 accumulation); lda/ldb multiples of 4 floats.
enum LowPrec : int { LOWP_BF16 = 0, LOWP_F16 = 1 };
hipError_t gemm_lowp(GemmTile t, LowPrec lp, int64_t M, int64_t N, int64_t K, const float* A,
                     int64_t lda, const float* B, int64_t ldb, const EpilogueT<float>& ep,
                     hipStream_t s);

// Product of 16-bit operands (type `lp`) held in memory: A M x K row-major,
// Bt = B^T N x K row-major (both k-contiguous; lda, ldbt multiples of 8
// elements, 16-byte aligned), v_mfma_f32_16x16x32 with FP32 accumulation;
// C = epilogue(A B) in FP32, plus the 16-bit copies ep.h / ep.ht if set.
hipError_t gemm_h16(GemmTile t, LowPrec lp, int64_t M, int64_t N, int64_t K, const void* A,
                    int64_t lda, const void* Bt, int64_t ldbt, const EpilogueT<float>& ep,
                    hipStream_t s);
// H = X rounded to 16 bits (row-major, ld ldh) and/or Ht = X^T rounded (ld
// ldht), X M x N FP32; either output may be null.
hipError_t convert_h16(const float* X, int64_t ldx, int64_t M, int64_t N, LowPrec lp, void* H,
                       int64_t ldh, void* Ht, int64_t ldht, hipStream_t s);

// Rows per partial column sum of alpha_norm1inf.
constexpr int kColChunk = 32;

// ||A||_1 and ||A||_inf of an M x N matrix, then scal[SLOT_ALPHA] =
// 1/(||A||_1 ||A||_inf). `tmp` needs (ceil(M/kColChunk)+1)*N + M doubles.
hipError_t alpha_norm1inf(const double* A, int64_t lda, int64_t M, int64_t N, double* tmp,
                          double* scal, hipStream_t s);

// Power iteration on A^T A (A M x N) from a fixed generic start vector:
// `iters` steps v <- A^T A v / ||A^T A v||; scal[SLOT_ALPHA] = 1/rho and
// scal[SLOT_TRACE] = rho, rho = ||A v||^2 for the last unit v (a lower bound
// on sigma_max(A)^2 that rises toward it). `tmp` needs N + M +
// ceil(M/256)*N doubles.
hipError_t alpha_sigma_max2(const double* A, int64_t lda, int64_t M, int64_t N, int iters,
                            double* tmp, double* scal, hipStream_t s);

// scal[SLOT_TRACE] = sum_ij P[i][j] * A[j][i] = Tr(P A), scal[SLOT_ALPHA] =
// 1/that (n x n). `tmp` needs ceil(n/32)^2 doubles.
hipError_t alpha_trace(const double* P, int64_t ldp, const double* A, int64_t lda, int64_t n,
                       double* tmp, double* scal, hipStream_t s);

// Y[j][i] = (*alpha_dev) * A[i][j] (alpha_dev NULL: 1); A is M x N, Y is N x M.
hipError_t transpose_scale(const double* A, int64_t lda, int64_t M, int64_t N, double* Y,
                           int64_t ldy, const double* alpha_dev, hipStream_t s);

// Y = (*alpha_dev) * A elementwise (M x N).
hipError_t scale(const double* A, int64_t lda, int64_t M, int64_t N, double* Y, int64_t ldy,
                 const double* alpha_dev, hipStream_t s);

// Y = diag(1/A[0][0], ..., 1/A[n-1][n-1]) (n x n, zero off the diagonal).
hipError_t diag_inv(const double* A, int64_t lda, int64_t n, double* Y, int64_t ldy, hipStream_t s);

// E (2M x 2N, ld lde) = [[Re A, -Im A], [Im A, Re A]] for a complex M x N
// matrix A stored as interleaved (re, im) doubles, leading dimension lda in
// complex elements.
hipError_t embed_complex(const double* A, int64_t lda, int64_t M, int64_t N, double* E, int64_t lde,
                         hipStream_t s);
// X (complex N x M, interleaved, ldx in complex elements) = the upper-left
// block of E (2N x 2M) + i times its lower-left block.
hipError_t extract_complex(const double* E, int64_t lde, int64_t N, int64_t M, double* X, int64_t ldx,
                           hipStream_t s);

// Y = I (M x N identity).
hipError_t set_identity(double* Y, int64_t ldy, int64_t M, int64_t N, hipStream_t s);

// scal[SLOT_DIFF2], scal[SLOT_REF2] = fixed-order sums of the pair partials.
// With `host` (a device-visible address of SLOT_COUNT + 1 doubles of pinned
// host memory), also writes all SLOT_COUNT scalars there and then `seq` to
// host[SLOT_COUNT], each write visible to the host in that order.
hipError_t reduce_pairs(const double* partials, int nblocks, double* scal, hipStream_t s,
                        double* host = nullptr, double seq = 0.0);

// Device-side loop control (hp_params.device_stop; hp_kernels.hip). Kept in
// device memory (not a kernel argument), so that captured loops do not
// depend on a solve's tolerance or alpha.
struct StepParams {
    int stop_rule, variant, max_iter, have_dinf, keep_best, pad;
    double tol, tau, diverge, alpha, order;
};
// Reset *L for a new solve (a fill kernel).
hipError_t loop_init(DevLoop* L, int stab_always, hipStream_t s);
// reduce_pairs of whichever update ran this loop (nb_plain or nb_stab
// partial pairs, by L->stabilising); skipped once the solve is done.
hipError_t reduce_pairs_gated(const double* partials, int nb_plain, int nb_stab, double* scal,
                              const DevLoop* L, hipStream_t s);
// diff_norm_inf, skipped once the solve is done.
hipError_t diff_norm_inf_gated(const double* X1, int64_t ld1, const double* X0, int64_t ld0,
                               int64_t M, int64_t N, double* tmp, double* scal, const DevLoop* L,
                               hipStream_t s);
// One loop's stop / switch / guard decision (LoopState::step for an FP64
// solve) from scal's sums; `ik` is the index (0 or 1) of the loop's input.
hipError_t loop_step(const double* scal, DevLoop* L, const StepParams* P, hipStream_t s);
// Copies the decision fields of *L (the bytes before d_hist) to `host` (the
// device address of pinned host memory with room for them and one more
// double), then writes `seq` into that last double: the host polls it.
hipError_t loop_report(const DevLoop* L, double* host, double seq, hipStream_t s);
constexpr int kLoopReportDoubles = (int)(offsetof(DevLoop, d_hist) / sizeof(double));
static_assert(offsetof(DevLoop, d_hist) % sizeof(double) == 0, "DevLoop header in whole doubles");
// dst = src (rows x cols doubles) when the gate is open.
hipError_t copy_gated(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                      int64_t cols, const DevLoop* L, int mode, hipStream_t s);

// scal[SLOT_DINF] = max_i sum_j |X1[i][j] - X0[i][j]|. `tmp` needs M doubles.
hipError_t diff_norm_inf(const double* X1, int64_t ld1, const double* X0, int64_t ld0,
                         int64_t M, int64_t N, double* tmp, double* scal, hipStream_t s);
hipError_t diff_norm_inf(const float* X1, int64_t ld1, const float* X0, int64_t ld0,
                         int64_t M, int64_t N, double* tmp, double* scal, hipStream_t s);

// scal[slot] = sum of squares of the M x N matrix X (fixed order). `tmp`
// needs M doubles.
hipError_t sumsq(const float* X, int64_t ldx, int64_t M, int64_t N, double* tmp, double* scal,
                 int slot, hipStream_t s);

// scal[slot] = sum over the M x N entries of (P - c Q)^2 (Q may be NULL).
// `tmp` needs M doubles.
hipError_t diffsq(const double* P, int64_t ldp, const double* Q, int64_t ldq, double c, int64_t M,
                  int64_t N, double* tmp, double* scal, int slot, hipStream_t s);
// scal[slot] = sum over the n x n entries of (P - P^T)^2. `tmp` needs
// ceil(n/32)^2 doubles.
hipError_t asymsq(const double* P, int64_t ldp, int64_t n, double* tmp, double* scal, int slot,
                  hipStream_t s);

// Y = X elementwise with a change of precision (M x N; narrowing rounds to
// nearest even).
hipError_t convert(const double* X, int64_t ldx, int64_t M, int64_t N, float* Y, int64_t ldy,
                   hipStream_t s);
hipError_t convert(const float* X, int64_t ldx, int64_t M, int64_t N, double* Y, int64_t ldy,
                   hipStream_t s);

}  // namespace hp
