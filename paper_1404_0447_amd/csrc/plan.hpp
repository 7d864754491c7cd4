// Internal plan structures shared by the host analysis, the scheduler and
// the C ABI.  Not part of the public interface.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "selinv.h"

namespace selinv {

// A partition of the (permuted) columns into contiguous supernodes/blocks.
struct Partition {
    std::vector<int32_t> xs;     // block K = columns xs[K] .. xs[K+1]-1
    std::vector<int32_t> of;     // column -> block
    std::vector<int32_t> par;    // block tree parent, -1 for roots
    std::vector<int32_t> lev;    // Algorithm 2 priority (root = 1)
    std::vector<int64_t> cptr;   // C(K) = crows[cptr[K] .. cptr[K+1])
    std::vector<int32_t> crows;  // sorted row indices below each block
    int32_t depth = 0;

    int32_t nblocks() const { return (int32_t)xs.size() - 1; }
    int32_t first(int K) const { return xs[K]; }
    int32_t width(int K) const { return xs[K + 1] - xs[K]; }
    int32_t clen(int K) const { return (int32_t)(cptr[K + 1] - cptr[K]); }
    const int32_t* C(int K) const { return crows.data() + cptr[K]; }
};

// Device descriptor of one execution block (all offsets in doubles).
struct BlockDesc {
    int64_t poff;   // panel (s+c) x s, column-major, ld = s + c  (L and Ainv arenas)
    int64_t hoff;   // L_hat(C,K), c x s column-major, ld = c
    int64_t woff;   // s x s blocks: W = L_KK^{-1} and T = L_KK^{-T} D^{-1} L_KK^{-1}
    int64_t coff;   // offset into the per-position arrays (crow, cbase, rbase)
    int32_t first, s, c, level;
};
static_assert(sizeof(BlockDesc) == 48, "BlockDesc layout");

// One unit of device work; meaning of the fields depends on the kernel.
struct Task {
    int32_t b;       // execution block
    int32_t i0, j0;  // tile origin (rows, columns)
    int32_t bn;      // tile width (16, 32, 64, 128)
    int32_t kb, ke;  // contraction range [kb, ke)
    int32_t flags;   // bit 0: accumulate atomically (split contraction); bit 2: the
                     // block's Schur update is exclusive in its level (no atomics)
    int32_t pad;
};

struct LevelTasks {
    std::vector<Task> tasks;
    std::vector<int64_t> off;  // per level (index = level-1): tasks[off[l] .. off[l+1])
};

// Work-queue tasks of the persistent level kernels reuse Task: the operation
// sits in bits 8..15 of flags and `pad` holds the number of earlier tasks of
// the same block that must have finished first (its dependencies: the
// phases of one block run in the order below).
// Flags bit 1: other tasks of the level wait for this one (it signals its
// block's counter).  Small-block tasks (qSbFactor, qSbInvert) carry up to
// four block ids in b, i0, j0, bn (-1 = none), one per wave; medium-block
// tasks (qMbFactor, qMbInvert) run one block's every phase on one
// work-group, tile after tile.  Neither kind waits nor signals.
enum QOp { qLdlt = 0, qPanel, qSchur, qZero, qGemm, qSdiag, qSbFactor, qSbInvert, qMbFactor, qMbInvert };
inline int32_t q_flags(int op, int f) { return (op << 8) | f; }

// Schedule of the persistent path (chosen by the autotuner).
struct Sched {
    int32_t order = 1;        // queue order within a phase, see QOrder
    int32_t bn_cap = 128;     // widest output tile of the gather-GEMM / panel
    int32_t split_fill = 512; // split contractions when a level has fewer tiles (0: never)
    int32_t grid_mult = 2;    // resident work-groups per CU
    int32_t small_s = 16;     // blocks with s <= small_s (and |C| <= kSbC) run whole on one wave (0: none)
    int32_t mb_tiles = 8;     // other blocks with at most this many X tiles run whole on one work-group
};
enum QOrder { qoPlan = 0, qoLpt = 1, qoRoundRobin = 2, qoTileLpt = 3, qoNumOrders };

// Persistent kernel variants, chosen per level: only small blocks (light,
// wave-granular), else bounded by the widest diagonal block (factor) or
// output tile (inversion) of the level.
enum PersistVariant {
    kLightFactor = 0, kFactor32, kFactor64, kFactor128,
    kLightInvert, kInvert32, kInvert64, kInvert128, kNumVariants
};

// Kernel kinds (same numbering as SELINV_K_* in selinv.h).
enum Kind {
    kAssemble = 0, kLdlt, kPanel, kSchur, kGemm, kSdiag, kExport, kRevSel, kRevFac, kQFactor, kQInvert, kSbFactor,
    kSbInvert, kCheckpoint, kNumKinds
};

// Optional per-launch timing: start/stop events are stamped by the dispatch
// itself (hipExtLaunchKernelGGL), so no marker packets are added.
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<int> kinds;  // launch i used events 2i, 2i+1
    hipEvent_t next();
    ~Prof();
};

// The workspace has a persistent part (the factor, the index maps, the task
// lists and the checkpoint store: what must survive from the forward calls
// to selinv_backward) and a transient part (the inverse panels and the
// adjoint arenas), which may live in a separate buffer that the caller binds
// and releases (selinv_bind_transient).
struct DeviceLayout {
    // byte offsets into the persistent part
    size_t lp, hp, wp, tp, status, blocks, crow, cbase, rbase, cr2, rel, asm_off, exp_off, colblk, colptrL;
    size_t t_diag, t_ldlt, t_panel, t_schur, t_gemm, t_sdiag, t_zero, t_sb;
    size_t t_rs1, t_rs2, t_rs3, t_rf1a, t_rf1b, t_rf2;
    size_t q_fac, q_inv, q_done, q_head;  // persistent path: queues, counters
    size_t ck, ck_off;                    // checkpoint store (Ainv panels of checkpointed levels), its offsets
    size_t persist;                       // bytes of the persistent part
    // byte offsets into the transient part
    size_t ap, zb, hb, tb;  // inverse panels; adjoint arenas (backward)
    size_t zsp;             // complex plans: partial products of the split diagonal step
    size_t transient;       // bytes of the transient part
    size_t total;           // persistent + transient (one buffer holding both)
};

}  // namespace selinv

struct selinv_plan_s {
    int64_t n = 0, nnzA = 0;
    selinv_opts opts{};
    std::vector<int64_t> colptr;
    std::vector<int32_t> rowind;
    std::vector<int32_t> perm, iperm;  // perm[new] = original
    std::vector<int32_t> parent;       // column elimination tree
    std::vector<int32_t> cnt;          // |struct(j)| (below the diagonal)
    selinv::Partition fund;            // fundamental supernodes (reported)
    selinv::Partition exec;            // execution blocks (amalgamated chains)
    std::vector<int64_t> colptrL;      // canonical pattern of L
    std::vector<int32_t> rowindL;
    // execution-block device tables (host copies)
    std::vector<selinv::BlockDesc> blocks;
    std::vector<int32_t> crow;         // = exec.crows
    std::vector<int64_t> cbase, rbase;
    std::vector<int64_t> cr2;  // (cbase, rbase) interleaved; kept while an upload may read it
    std::vector<int32_t> rel;
    std::vector<int64_t> asm_off, exp_off;
    std::vector<int32_t> colblk;       // column -> execution block
    int64_t arena = 0, harena = 0, warena = 0;
    // forward, per level: small blocks (t_sb, four per task), and the tiled
    // path of the others (t_ldlt, t_panel, t_schur, t_gemm, t_sdiag, t_zero);
    // t_diag lists every block (used by the reverse sweep)
    selinv::LevelTasks t_diag, t_ldlt, t_panel, t_schur, t_gemm, t_sdiag, t_sb;
    std::vector<int64_t> ldlt_cut;     // per level: t_ldlt splits into s <= 32 | <= 64 | wider at 2l, 2l+1
    // per level: t_schur in colour groups [cut[g], cut[g+1]) whose blocks share no column of C
    std::vector<std::vector<int64_t>> schur_cuts;
    // per level: bit 0, panel tiles <= 64 wide and at most kDeepMaxTiles of
    // them (whole-contraction panel kernel); bit 1, every block of the level
    // at most kDeepK wide (whole-contraction kernels allowed at all)
    std::vector<char> panel_deep;
    // reverse sweep: selected inversion (leaves first) and factorization (root first)
    selinv::LevelTasks t_rs1, t_rs2, t_rs3, t_rf1a, t_rf1b, t_rf2;
    // per level: t_rs3 in colour groups (deterministic mode; otherwise one group)
    std::vector<std::vector<int64_t>> rs3_cuts;
    // per level: t_sdiag splits into [start, cut) and [cut, end) launches
    // (deterministic mode: the second half-products of off-diagonal tiles
    // run after the first; otherwise cut = end)
    std::vector<int64_t> sdiag_cut;
    // complex plans: scratch slots of the split gather-GEMM and diagonal
    // step (the most any level's launch uses; per level, t_gemm holds whole
    // tiles, pieces from zgemm_mid and one summing task per split tile from
    // zgemm_cut; t_sdiag likewise, its summing tasks from sdiag_cut)
    int64_t zsd_slots = 0;
    std::vector<int64_t> zgemm_mid, zgemm_cut;
    // column ranges [kb, ke) of blocks whose X or Ainv(B,B) accumulates, in
    // level order; level l owns t_zero[t_zero_off[l] .. t_zero_off[l+1])
    std::vector<selinv::Task> t_zero;
    std::vector<int64_t> t_zero_off;
    // checkpointing of the inverse panels for the adjoint: per block the
    // offset (doubles) of its copy in the store, -1 if its level is dropped
    std::vector<int64_t> ck_off;
    int64_t ck_size = 0;
    selinv::DeviceLayout lay{};
    selinv_info info{};
    // batch (block-diagonal union of independent matrices): per-matrix
    // offsets of columns, of A's entries and of L's entries (count + 1 each),
    // and the matrix of every execution block; a single matrix is a batch of 1
    std::vector<int64_t> b_noff, b_aoff, b_loff;
    std::vector<int32_t> blk_matrix;
    // persistent path: per-level work queues (factor leaves first, inversion
    // root first), their capacity in the workspace and the schedule
    selinv::Sched sched{};
    std::vector<selinv::Task> q_fac, q_inv;
    std::vector<int64_t> q_fac_off, q_inv_off;
    int64_t q_cap_fac = 0, q_cap_inv = 0;
    bool queues_on_device = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const void* graph_in = nullptr;
    void* graph_out = nullptr;
    hipStream_t cap_stream = nullptr;
    int n_cu = 0;                           // device of the bound workspace
    int occ[selinv::kNumVariants] = {1, 1, 1, 1, 1, 1, 1, 1};  // resident work-groups per CU, per variant
    std::vector<uint8_t> q_var_fac, q_var_inv;                  // per level: the PersistVariant to launch
    std::string dev_arch;
    unsigned spin_limit = 1u << 22;         // polls of a dependency wait before it is abandoned
    // binding state
    char* ws = nullptr;        // persistent part (and, when large enough, the transient part after it)
    size_t ws_bytes = 0;
    char* tr = nullptr;        // transient part in use (nullptr: none bound)
    bool tr_separate = false;  // bound with selinv_bind_transient
    bool factored = false;
    bool inverted = false;
    bool ap_valid = false;     // the inverse panels hold the last inversion's values
    uint64_t generation = 0;   // factorizations so far (selinv_factor, selinv_run)
    uint64_t static_uid = 0;   // identity in the static scratch (0: never used there)
    selinv::Prof prof;
    std::vector<double> work_flops, work_bytes;  // per kernel kind, per call
    ~selinv_plan_s();
};

namespace selinv {
// analyze.cpp
selinv_status analyze(selinv_plan_s* P, const selinv_geom* geom, const int32_t* perm_or_null,
                      std::string& err);
void nd_order_box(int ndim, const int32_t dims[3], int dofs, int rim_last, std::vector<int32_t>& perm);
void block_index_maps(const Partition& part, std::vector<int64_t>& rptr, std::vector<int32_t>& rel);
// schedule.cpp
void build_schedule(selinv_plan_s* P);
// Work queues of the persistent path for schedule `sc`: per level (index =
// level-1) the factor tasks qf[qf_off[l] .. qf_off[l+1]) and the inversion
// tasks qi[...], each level's tasks in phase order.
void build_queues(const selinv_plan_s* P, const Sched& sc, std::vector<Task>& qf, std::vector<int64_t>& qf_off,
                  std::vector<Task>& qi, std::vector<int64_t>& qi_off);
// upper bound on the factor / inversion queue entries of any schedule
void queue_bound(const selinv_plan_s* P, int64_t& nfac, int64_t& ninv);
// batch.cpp: merge independently analysed plans into their block-diagonal union
void merge_plans(const std::vector<selinv_plan_s*>& parts, selinv_plan_s* U);
}  // namespace selinv
