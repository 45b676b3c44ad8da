// Partition of a symmetric product's work over the blocks of its stream-K
// launch (k_gemm_sym in hp_gemm.hip). Plain integer arithmetic with no HIP
// dependence, so that the same code runs in the kernel and in the CPU check
// of its invariants (tests/host/sym_partition_check.cpp).
//
// The t_count = nt (nt + 1) / 2 tiles on and above the diagonal of an
// nt x nt tile grid are numbered row by row. With at least one tile per
// block, the first dp tiles are taken whole in rounds (round r gives tile
// r grid + b to block b, so the tiles in flight at once are neighbours in
// the numbering and share operand panels in L2); dp is the multiple of the
// grid that leaves between one and two tiles per block to the stream-K part
// (nothing when the grid divides the tile count). The remaining tiles
// dp .. t_count-1 are split by K-steps: tile
// dp + u's steps (ipt of them) occupy the stream-K step range
// [u ipt, (u + 1) ipt), and block b takes the steps [b ipc, min((b + 1) ipc,
// (t_count - dp) ipt)). A tile covered by one block is finished there; one
// covered by several (its pieces, in K order, on consecutive blocks b0..b1)
// is finished by the last of them to arrive. A block's first piece uses
// partial slot 2 b and its last slot 2 b + 1.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define HP_SYMK_FN __host__ __device__ inline
#else
#define HP_SYMK_FN inline
#endif

namespace hp {

// Blocks (grid <= g), whole tiles (dp) and stream-K steps per block (ipc)
// for t_count tiles of ipt K-steps on a launch of at most g resident blocks.
HP_SYMK_FN void sym_layout(int t_count, int ipt, int g, int* ipc, int* grid, int* dp) {
    const int q = t_count / g, r = t_count % g;
    // the remainder goes to stream-K with the last round, so that no tile is
    // cut into many small pieces (each piece costs a partial tile's round trip)
    *dp = q == 0 ? 0 : r == 0 ? q * g : (q - 1) * g;
    const int64_t total = (int64_t)(t_count - *dp) * ipt;
    *ipc = total > 0 ? (int)((total + g - 1) / g) : 1;
    *grid = *dp > 0 ? g : (int)((total + *ipc - 1) / *ipc);
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

// The piece that a block whose range ends at `end` takes from stream-K step
// `it` on: stream-K tile t (tile dp + t of the triangle), its K-steps
// [k0, k1), the tile's piece count np, this piece's index, and the slot of
// the tile's piece 0 (pieces i > 0 are in slot 2 (b0 + i)).
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
