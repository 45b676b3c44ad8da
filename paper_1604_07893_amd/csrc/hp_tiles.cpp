// Tile shapes and the default tile choice of the MFMA GEMM kernels (host
// code: the launch configuration each product of a solve runs on).
#include <algorithm>

#include "hp_internal.h"

namespace hp {
namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tile configurations, indexed by GemmTile.
struct TileShape {
    int bm, bn;
};
constexpr TileShape kShapes[] = {
    {128, 128},  // TILE_128x128_W4: 4 waves of 64x64
    {128, 128},  // TILE_128x128_W8: 8 waves of 64x32
    {128, 64},   // TILE_128x64_W4: 4 waves of 64x32
    {64, 64},    // TILE_64x64_W4: 4 waves of 32x32
    {256, 128},  // TILE_256x128_W8: 8 waves of 64x64
    {128, 64},   // TILE_128x64_W8: 8 waves of 32x32
    {64, 128},   // TILE_64x128_W8: 8 waves of 32x32
    {128, 128},  // TILE_128x128_W8_K2: 8 waves of 64x32, double K-tile
    {128, 128},  // TILE_128x128_W16: 16 waves of 32x32
    {128, 128},  // TILE_128x128_W8_P2: 8 waves, loads two K-tiles ahead
    {128, 128},  // TILE_128x128_W16_P2: 16 waves, loads two K-tiles ahead
    {128, 128},  // TILE_128x128_W8_S2: K split over 2 blocks
    {128, 128},  // TILE_128x128_W8_S4: K split over 4 blocks
    {128, 128},  // TILE_128x128_W16_K2_P2: 16 waves, double K-tile, two ahead
    {256, 256},  // TILE_256x256_W8 (16-bit-operand kernel)
    {256, 256},  // TILE_256x256_W16 (16-bit-operand kernel)
    {256, 256},  // TILE_256x256_W8_DMA (16-bit-operand kernel, load-to-LDS)
    {256, 256},  // TILE_256x256_W16_DMA (16-bit-operand kernel, load-to-LDS)
    {32, 32},    // TILE_32x32_W4_K4: 4 waves of 16x16, 4x deeper K-tile
    {128, 128},  // TILE_128x128_W4_DMA: 4 waves of 64x64, load-to-LDS (FP64)
    {256, 256},  // TILE_256x256_W4_DMA: 4 waves of 128x128, load-to-LDS (FP32)
};
static_assert(sizeof(kShapes) / sizeof(kShapes[0]) == TILE_COUNT, "tile table");

}  // namespace

int gemm_blocks(GemmTile t, int64_t M, int64_t N) {
    const TileShape sh = kShapes[(int)t];
    return (int)(cdiv(M, sh.bm) * cdiv(N, sh.bn));
}

int gemm_max_blocks(int64_t M, int64_t N) {
    int b = 0;
    for (int t = 0; t < TILE_COUNT; ++t) b = std::max(b, gemm_blocks((GemmTile)t, M, N));
    return b;
}

bool gemm_runs(GemmTile t, GemmType gt) {
    switch (gt) {
        case GT_H16:
            return t == TILE_256x256_W8_DMA || t == TILE_256x256_W16_DMA || t == TILE_64x64_W4 ||
                   t == TILE_128x64_W4 || t == TILE_128x128_W4 || t == TILE_256x128_W8 ||
                   t == TILE_256x256_W8 || t == TILE_256x256_W16 || t == TILE_128x128_W16 ||
                   t == TILE_128x128_W8;
        case GT_LOWP: return t <= TILE_128x128_W16_K2_P2;
        default:
            return t <= TILE_128x128_W16_K2_P2 || t == TILE_32x32_W4_K4 ||
                   (gt == GT_F64 && t == TILE_128x128_W4_DMA) ||
                   (gt == GT_F32 && t == TILE_256x256_W4_DMA);
    }
}

GemmTile gemm_pick_tile(int64_t M, int64_t N, int64_t K, GemmType gt, bool allow_split) {
    // From MI355X sweeps of every tile over square and 2:1 products. FP64 with
    // at least one 128x128 tile per CU (256 CUs): the 16-wave tile with a
    // 32-deep K-tile, loading two K-tiles ahead with its LDS reads spread over
    // the MFMAs (2048^3: 52.8 TFLOP/s against 49.2 for the 8-wave tile
    // loading one ahead; 8192^3: 64.6 against 63.3). FP32: the 8-wave tile
    // from two tiles per CU (8192^3: 121.9 against 118.9), the 16-wave one
    // below. With fewer tiles than CUs and a long K, splitting K four ways
    // fills the chip (FP64 1024x1024x2048: 33.6 TFLOP/s against 14.6 unsplit
    // and 27.7 on 64x64 tiles); short K or the FP32 1536^2 case favour 64x64
    // tiles. The 16-bit kernel does not split. FP64 from two 128x128 tiles per
    // CU: the 4-wave 64x64-per-wave tile filled by load-to-LDS, two blocks
    // per CU (8192^3: 71.8 TFLOP/s against 65.5; 4096^3: 65.0 against 59-65).
    const int64_t tiles = cdiv(M, 128) * cdiv(N, 128);
    if (gt == GT_H16) {
        // 16-bit operands in memory: 256x256 tiles filled by load-to-LDS from
        // 64 such tiles (8192^3: 886 TFLOP/s on 8 waves reading each K-tile's
        // fragments before streaming the next; 708 with register staging);
        // the 16-wave 128x128 tile below (2048^3: 373 TFLOP/s)
        if (cdiv(M, 256) * cdiv(N, 256) >= 64) return TILE_256x256_W8_DMA;
        if (tiles >= 64) return TILE_128x128_W16;
        return TILE_64x64_W4;
    }
    if (gt == GT_LOWP) {
        if (tiles >= 512) return TILE_128x128_W8;
        if (tiles >= 64) return TILE_128x128_W16_P2;
        return TILE_64x64_W4;
    }
    // Small products (up to 144 tiles of 64^2, K up to 1024) are bound by the
    // latency of each K-tile's loads: 32x32 tiles with a 4x deeper K-tile
    // (FP64 256^3: 9.5 us against 23.1 on 64x64 tiles; 512^3: 14.1 against
    // 39.7; 768^3: 52.5 against 56.8; 1024^3 favours 64x64 again).
    const bool small = cdiv(M, 64) * cdiv(N, 64) <= 144 && K <= 1024;
    if (gt == GT_F64) {
        if (tiles >= 512) return TILE_128x128_W4_DMA;
        if (tiles >= 256) return TILE_128x128_W16_K2_P2;
        if (small) return TILE_32x32_W4_K4;
        if (allow_split && K >= 1024) return TILE_128x128_W8_S4;
        return TILE_64x64_W4;
    }
    // FP32 from one 256x256 tile per CU with K % 32 == 0: the 4-wave
    // 128x128-per-wave tile filled by load-to-LDS (8192^3: 130.9 TFLOP/s
    // against 122.8; 4096^3: 118.2 against 105.9; with 128 such tiles, half
    // the CUs idle: 65.1 against 113.6 for the 8-wave tile)
    if (cdiv(M, 256) * cdiv(N, 256) >= 256 && K % 32 == 0) return TILE_256x256_W4_DMA;
    if (tiles >= 512) return TILE_128x128_W8;
    if (tiles >= 256) return TILE_128x128_W16_K2_P2;
    if (small) return TILE_32x32_W4_K4;
    if (allow_split && ((tiles < 128 && K >= 2048) || K >= 4096)) return TILE_128x128_W8_S4;
    return TILE_64x64_W4;
}

}  // namespace hp
