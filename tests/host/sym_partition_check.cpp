// The partition of a symmetric product's launch (hp_symk.h), checked on the
// CPU for many shapes and grids: whole tiles in rounds, then stream-K. Every
// K-step of every upper-triangle tile is taken by exactly one block, every
// block has work, the rounds' tiles are whole and the rounds leave nothing
// or between one and two tiles per block to the stream-K part (no rounds
// below two tiles per block unless the grid divides them), a stream-K tile's pieces
// are on consecutive blocks in K order, a stream-K tile held by one block is
// whole, the partial slots of split tiles are distinct and below 2 * grid,
// the counter index (the tile) is below the tile count, and the triangle
// numbering visits each (tm <= tn) once. Test infrastructure; prints "ok" or
// the first failed check.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <utility>
#include <vector>

#include "hp_symk.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);  \
            std::exit(1);                                               \
        }                                                               \
    } while (0)

static void check(int nt, int K, int BK, int G) {
    const int tiles = nt * (nt + 1) / 2;
    const int ipt = (K + BK - 1) / BK;
    int ipc = 0, grid = 0, dp = 0;
    hp::sym_layout(tiles, ipt, G, &ipc, &grid, &dp);
    CHECK(grid >= 1 && grid <= G && ipc >= 1);
    CHECK(dp >= 0 && dp % grid == 0 && dp <= tiles);
    const int rest = tiles - dp;
    if (dp > 0)
        CHECK(grid == G && (rest == 0 || (rest > G && rest < 2 * G)));
    else
        CHECK(tiles < 2 * G);
    const int64_t total = (int64_t)tiles * ipt;
    const int64_t sk_total = (int64_t)(tiles - dp) * ipt;
    std::vector<int> owner(total, -1);
    std::vector<std::vector<int>> pieces(tiles);  // blocks holding each tile, in order
    std::set<int> slots;
    for (int b = 0; b < grid; ++b) {
        bool work = false;
        for (int t = b; t < dp; t += grid) {
            for (int k = 0; k < ipt; ++k) {
                CHECK(owner[(int64_t)t * ipt + k] == -1);
                owner[(int64_t)t * ipt + k] = b;
            }
            pieces[t].push_back(b);
            work = true;
        }
        int64_t it = (int64_t)b * ipc;
        const int64_t end = it + ipc < sk_total ? it + ipc : sk_total;
        CHECK(work || it < end);  // no block is left without work
        while (it < end) {
            const hp::SymPiece p = hp::sym_piece(it, end, ipt, ipc, b);
            const int t = dp + p.t;
            CHECK(p.t >= 0 && t < tiles);
            CHECK(0 <= p.k0 && p.k0 < p.k1 && p.k1 <= ipt);
            CHECK(p.np >= 1 && 0 <= p.idx && p.idx < p.np && p.b0 + p.idx == b);
            for (int k = p.k0; k < p.k1; ++k) {
                CHECK(owner[(int64_t)t * ipt + k] == -1);
                owner[(int64_t)t * ipt + k] = b;
            }
            if (p.np == 1) {
                CHECK(p.k0 == 0 && p.k1 == ipt);
            } else {
                const int slot = p.idx == 0 ? p.slot0 : 2 * (p.b0 + p.idx);
                CHECK(slot >= 0 && slot < 2 * grid);
                CHECK(slots.insert(slot).second);
            }
            pieces[t].push_back(b);
            it += p.k1 - p.k0;
        }
    }
    for (int64_t s = 0; s < total; ++s) CHECK(owner[s] >= 0);
    for (int t = 0; t < tiles; ++t) {
        const std::vector<int>& v = pieces[t];
        CHECK(!v.empty());
        if (t < dp) CHECK(v.size() == 1);
        for (size_t i = 1; i < v.size(); ++i) CHECK(v[i] == v[i - 1] + 1);
    }
    std::set<std::pair<int, int>> seen;
    for (int t = 0; t < tiles; ++t) {
        int tm = -1, tn = -1;
        hp::sym_tile_of(t, nt, tm, tn);
        CHECK(0 <= tm && tm <= tn && tn < nt);
        CHECK(seen.insert({tm, tn}).second);
    }
}

int main() {
    const int nts[] = {1, 2, 3, 7, 16, 17, 22, 23, 24, 31, 32, 33, 64};
    const int ks[] = {1, 31, 32, 33, 200, 333, 1000, 2048, 4096, 8192};
    const int bks[] = {16, 32, 64};
    const int gs[] = {1, 7, 256, 512};
    for (int nt : nts)
        for (int K : ks)
            for (int BK : bks)
                for (int G : gs) check(nt, K, BK, G);
    std::printf("ok\n");
    return 0;
}
