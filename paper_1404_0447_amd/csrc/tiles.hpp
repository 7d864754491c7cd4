// Tile shapes shared by the scheduler (task lists) and the kernels.
#pragma once

namespace selinv {
constexpr int kThreads = 256;   // work-group size of every tiled kernel
constexpr int kMaxS = 256;      // widest supported block (cap)
constexpr int kPanelRows = 16;  // rows of C(K) per factor panel task
constexpr int kSchurTile = 32;  // edge of a Schur-update tile (lower c x c)
constexpr int kGemmBM = 32;     // rows of X per gather-GEMM task
constexpr int kGemmBN = 32;     // columns of X per gather-GEMM task
constexpr int kGemmBK = 16;     // contraction chunk staged in LDS
}  // namespace selinv
