// Tile shapes shared by the scheduler (task lists) and the kernels.
#pragma once
#include <cstddef>

namespace selinv {
constexpr int kThreads = 256;    // work-group size of every tiled kernel (4 waves)
constexpr int kMaxS = 256;       // widest supported block (cap)
constexpr int kTileM = 64;       // rows of an MFMA output tile (gather-GEMM, panel, Schur)
constexpr int kSchurTile = 64;   // edge of a Schur-update tile (lower c x c)
constexpr int kDiagTile = 32;    // edge of a diagonal-block tile (pairs (I,J), I >= J)
constexpr int kDiagTile64 = 64;  // the same on the per-level path (pipelined MFMA tile)
constexpr int kLdsDiagMax = 128; // diagonal blocks swept in registers up to this width
constexpr int kZMaxS = 64;       // widest block of the complex path (one 64-wide tile per diagonal step)
// Complex gather-GEMM and diagonal step: a level with fewer than
// kZSplitFill / 2 tasks cuts each task's contraction over C into pieces of
// at least kZSplitRows rows, about kZSplitFill work-groups in all; a piece
// writes its 64 x 64 complex partial product to a scratch slot of
// kZSlotDoubles doubles.
constexpr int kZSplitFill = 2048;
constexpr int kZSplitRows = 64;
// levels with fewer tasks than this (those of a single pole) cut pieces of
// kZSplitRows / 2 rows: one pole 5.85 -> 5.67 ms, while 32-row pieces in the
// batch's larger levels cost more in sums than they gained
constexpr int kZSplitFewTasks = 64;
constexpr size_t kZSlotDoubles = 2 * (size_t)kZMaxS * kZMaxS;
constexpr size_t kLdsDiagBytes = sizeof(double) * kLdsDiagMax * (kLdsDiagMax + 1);
constexpr bool kUseSweep = true;  // register Gauss-Jordan sweep for s <= kLdsDiagMax
constexpr size_t kDiagShmem = kUseSweep ? sizeof(double) * 2 * kLdsDiagMax : kLdsDiagBytes;

// small blocks run whole on one wave (all phases, 16 x 16 MFMA tiles)
constexpr int kSbS = 16;          // widest small block
constexpr int kSbC = 256;         // largest |C| of a small block
constexpr int kSbPerTask = 4;     // small blocks per work-group task (one per wave)
inline bool is_small(int s, int c, int smax) { return s <= smax && c <= kSbC; }
// per-level path: a wave per block only where |C| is small.  Blocks with a
// larger |C| sit in few, nearly empty levels near the leaves, where the tiled
// kernels spread them over many more work-groups (swept over 0..256: 32
// fastest at 40^3, 64^3 and molecular 16^3)
constexpr int kSbCLevel = 32;
// A level with at most this many panel tiles (a Schur colour group with at
// most this many tiles) loads each tile's whole contraction (s <= 128) before
// its first product: there the tiles' latency, not the device's throughput,
// sets the level time.
constexpr int kDeepMaxTiles = 256;
constexpr int kDeepK = 128;  // longest contraction of the whole-contraction kernels
constexpr int kZeroCols = 8;  // columns of Ainv(:, B) a task of the set-up kernel clears
// A level's Schur update runs in colour groups (read-modify-write, one launch
// each) only when its blocks need at most this many colours; more launches
// cost more than the atomics they save (molecular 16^3: 10.3 -> 9.5 ms).
constexpr int kMaxSchurColours = 3;
inline bool is_small_level(int s, int c) { return s <= kSbS && c <= kSbCLevel; }

// reverse sweep: split the contraction when a level has fewer tiles than this
// (swept over 256..2048: 1024 fastest at 64^3 and molecular 16^3)
constexpr int kFillTiles = 1024;
// resident work-groups of the gather-GEMM and diagonal-tile kernels on the
// target (256 CUs x 2); the per-level split is sized for them
constexpr long kGemmSlots = 512;
// fixed cost of one work-group of the split contractions, in 16-deep chunks
// (swept over 3..12 at 64^3: 6 fastest)
constexpr double kGemmTaskOvh = 6.0;
constexpr double kSdiagTaskOvh = 8.0;  // smaller epilogue (half a 64 x 64 tile)
constexpr int kMinSplitK = 128;  // rows of C per split piece, at least
constexpr int kMinSplitKDiag = 64;  // the same for the diagonal tile pairs

// output-column tile of a block of width s: 16, 32, 64 or 128
inline int tile_bn(int s) { return s <= 16 ? 16 : s <= 32 ? 32 : s <= 64 ? 64 : 128; }
}  // namespace selinv
