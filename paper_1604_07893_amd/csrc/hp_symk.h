// Partition of a symmetric product's work over the blocks of its stream-K
// launch (k_gemm_sym in hp_gemm.hip). Plain integer arithmetic with no HIP
// dependence, so that the same code runs in the kernel and in the CPU check
// of its invariants (tests/host/sym_partition_check.cpp).
//
// The t_count = nt (nt + 1) / 2 tiles on and above the diagonal of an
// nt x nt tile grid are numbered row by row; tile t's K-steps (ipt of them)
// occupy the global step range [t ipt, (t + 1) ipt). Block b takes the steps
// [b ipc, min((b + 1) ipc, t_count ipt)). A tile covered by one block is
// finished there; one covered by several (its pieces, in K order, on
// consecutive blocks b0..b1) is finished by the last of them to arrive. A
// block's first piece uses partial slot 2 b and its last slot 2 b + 1.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define HP_SYMK_FN __host__ __device__ inline
#else
#define HP_SYMK_FN inline
#endif

namespace hp {

// Steps per block (ipc) and blocks (grid <= g) for t_count tiles of ipt
// K-steps on a launch of at most g resident blocks.
HP_SYMK_FN void sym_layout(int t_count, int ipt, int g, int* ipc, int* grid) {
    const int64_t total = (int64_t)t_count * ipt;
    *ipc = (int)((total + g - 1) / g);
    *grid = (int)((total + *ipc - 1) / *ipc);
}

// Upper-triangle tile t (row-major: row 0 holds tiles (0, 0..nt-1), row 1
// (1, 1..nt-1), ...) of an nt x nt tile grid.
HP_SYMK_FN void sym_tile_of(int t, int nt, int& tm, int& tn) {
    int r = 0;
    while (t >= nt - r) {
        t -= nt - r;
        ++r;
    }
    tm = r;
    tn = r + t;
}

// The piece that a block whose range ends at `end` takes from global step
// `it` on: tile t, its K-steps [k0, k1), the tile's piece count np, this
// piece's index, and the slot of the tile's piece 0 (pieces i > 0 are in
// slot 2 (b0 + i)).
struct SymPiece {
    int t, k0, k1, np, idx, slot0, b0;
};
HP_SYMK_FN SymPiece sym_piece(int64_t it, int64_t end, int ipt, int ipc, int b) {
    SymPiece p;
    p.t = (int)(it / ipt);
    p.k0 = (int)(it - (int64_t)p.t * ipt);
    const int64_t left = end - it;
    p.k1 = (int)((int64_t)p.k0 + left < (int64_t)ipt ? p.k0 + left : ipt);
    const int64_t ts = (int64_t)p.t * ipt;
    p.b0 = (int)(ts / ipc);
    const int b1 = (int)((ts + ipt - 1) / ipc);
    p.np = b1 - p.b0 + 1;
    p.idx = b - p.b0;
    // piece 0 is block b0's first piece when the tile starts with its range
    p.slot0 = 2 * p.b0 + ((int64_t)p.b0 * ipc >= ts ? 0 : 1);
    return p;
}

}  // namespace hp
