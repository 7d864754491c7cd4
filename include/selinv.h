/*
 * selinv.h -- C ABI of the MI355X supernodal selected-inversion library.
 *
 * Given a sparse symmetric matrix A, the library computes every entry of
 * A^{-1} that lies in the sparsity pattern of its LDL^T factor L (the
 * "selected elements", Section 2 of Jacquelin, Lin and Yang, PSelInv, ACM
 * TOMS; Algorithm 1 with the symmetric simplifications of Section 2.1).
 *
 * Pipeline: selinv_analyze (host: ordering, elimination tree, supernodes,
 * block index maps) -> selinv_bind_workspace (device memory owned by the
 * caller) -> selinv_factor (device supernodal LDL^T) -> selinv_invert
 * (device root-to-leaf selected inversion, written as values on the pattern
 * of L).  selinv_backward runs the adjoint of both.  selinv_analyze_batch
 * builds one plan for many independent matrices, and selinv_run executes
 * factor + inversion with one persistent work-queue launch per tree level
 * (optionally replayed from a captured HIP graph), with the schedule chosen
 * by selinv_tune.
 *
 * Conventions for every call:
 *  - Status codes are returned, never thrown.  selinv_last_error() gives a
 *    thread-local message for the last failing call.
 *  - Device pointers ("d_" prefix) are HIP device memory owned by the
 *    caller; host pointers are read during the call only.
 *  - Device work is asynchronous and ordered on the given stream; a zero
 *    pivot found on the device is latched and reported by
 *    selinv_sync_status.
 *  - A plan is not thread-safe; distinct plans are independent.
 *  - Numbering: "original" indices are those of the input CSC; L, the
 *    selected values and the pattern use the permuted numbering, with
 *    perm[new] = original.
 */
#ifndef SELINV_H
#define SELINV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct selinv_plan_s* selinv_plan;

typedef enum {
    SELINV_OK = 0,
    SELINV_EINVAL = -1,       /* bad argument or malformed input pattern      */
    SELINV_ESTATE = -2,       /* call out of order (e.g. invert before factor) */
    SELINV_EPIVOT = -3,       /* zero / non-finite / non-positive pivot        */
    SELINV_ENOMEM = -4,       /* host allocation failed or workspace too small */
    SELINV_EHIP = -5,         /* a HIP runtime call failed                     */
    SELINV_EUNSUPPORTED = -6, /* option not supported                          */
    SELINV_EQUEUE = -7        /* a persistent-kernel dependency wait gave up
                                 (poll limit reached); the results are invalid */
} selinv_status;

/* Geometry used by the nested-dissection ordering: a box grid of
 * dims[0] x dims[1] x dims[2] points (x fastest), dofs_per_point unknowns
 * per point stored contiguously (unknown = dofs*point + k).  ndim = 0 means
 * no geometry: natural order unless a permutation is given. */
typedef struct {
    int32_t ndim;
    int32_t dims[3];
    int32_t dofs_per_point;
} selinv_geom;

typedef struct {
    int32_t max_super;    /* cap on supernode width (columns), e.g. 128      */
    int32_t fuse_chains;  /* 1: run chains of single-child supernodes as one
                             amalgamated block (explicit zeros; results on the
                             fundamental pattern are unchanged up to rounding) */
    int32_t require_spd;  /* 1: a pivot <= 0 is an error (SELINV_EPIVOT)     */
    int32_t exec_cap;     /* cap on an execution block's width (<= 256); 0 =
                             min(max_super, 128).  Blocks wider than 128 take
                             a slow diagonal-factorization path.           */
    int32_t sep_order;    /* order of the points of a nested-dissection
                             separator plane: 0 lexicographic (x fastest);
                             1 rim last: the points on the plane's boundary
                             (a coordinate along another grid axis of more
                             than one point at the box's first or last
                             value) after the interior ones, each group
                             lexicographic.  Changes the pattern of L, never
                             the values of A^{-1}.                          */
    int32_t deterministic; /* 1: no floating-point atomics anywhere (no split
                             contractions, every Schur and adjoint scatter in
                             colour groups of disjoint updates, no small-block
                             kernels): results are bitwise reproducible from
                             run to run, through selinv_run and its graph, and
                             between a batch and its matrices run alone.
                             Slower.                                        */
    int32_t checkpoint_every; /* adjoint: the inverse panels of every k-th
                             level (levels 1, 1+k, 1+2k, ...; root = 1) are
                             copied to the persistent checkpoint store by
                             selinv_invert; selinv_backward restores them and
                             recomputes the other levels root first before
                             the reverse sweep, so the transient memory may be
                             released between the two.  <= 1: every level is
                             kept in place and nothing is recomputed.       */
    int32_t relaxed;      /* 1: report relaxed supernodes (Section 2.1): the
                             execution blocks, i.e. fundamental supernodes
                             cut into pieces of at most exec_cap columns and
                             chains of single-child pieces merged up to
                             exec_cap columns; the pattern (and the selected
                             values, the factor and the gradient input) then
                             includes the explicit zeros of L inside those
                             blocks, whose A^{-1} entries are computed too.
                             Needs fuse_chains = 1.                         */
    int32_t complex_values; /* 1: the values are complex (A(z) = H - z S of the
                             pole expansion, Section 4.3: symmetric, not
                             Hermitian); use selinv_factor_complex and
                             selinv_invert_complex.  Execution blocks are
                             then at most 64 columns wide and the schedule is
                             atomic-free and bitwise repeatable (long
                             contractions of sparse levels run as pieces
                             summed in a fixed order).                      */
    int32_t pivoting;     /* 1: symmetric indefinite A: each diagonal block
                             F_KK is inverted with 1x1 or 2x2 pivots chosen
                             inside the block by the Bunch-Kaufman rule
                             (symmetric pivoting, D block diagonal, Section
                             2.1).  Only T_K = F_KK^{-1} enters the rest of
                             the method, so Algorithm 1, the Schur updates
                             and the adjoint are unchanged.  No interchange
                             crosses a block: a singular F_KK is reported as
                             SELINV_EPIVOT with the block's first column.
                             Needs require_spd = 0 and real values;
                             execution blocks are then at most 128 columns,
                             every level runs as per-level launches (no
                             persistent queues, no small-block kernels), and
                             selinv_get_factor and selinv_tune refuse.     */
} selinv_opts;

typedef struct {
    int64_t n, nnzA, nnzL;      /* order, lower nonzeros of A and of L          */
    int64_t nsuper, depth;      /* fundamental supernodes, tree depth (levels)   */
    int64_t nblocks, exec_depth;/* execution blocks and their tree depth         */
    int64_t workspace_bytes;
    double flops_factor;        /* sum c^2 s + c s^2 + s^3/3 (fundamental)       */
    double flops_gemm;          /* sum 2 c^2 s + 2 c s^2      (fundamental)      */
    double flops_selinv;        /* sum 2 c^2 s + 3 c s^2 + 2/3 s^3 (fundamental) */
    double gather_bytes;        /* sum 8 c (c+1) / 2          (fundamental)      */
    double exec_flops_gemm;     /* same GEMM count on the execution blocks       */
} selinv_info;

/* Symbolic analysis (Sections 2.1-2.2 and Algorithm 2).
 * colptr[n+1], rowind[nnz]: lower triangle of A in CSC, diagonal included,
 * rows strictly increasing within a column, rowind[p] >= column.
 * geom: may be NULL (= ndim 0).  perm_or_null: perm[new] = original; when
 * given it overrides the geometric ordering.  opts: may be NULL (defaults
 * max_super 128, fuse_chains 1, require_spd 1).  On success *out owns a
 * copy of everything it needs; no device memory is touched. */
selinv_status selinv_analyze(int64_t n, const int64_t* colptr, const int32_t* rowind,
                             const selinv_geom* geom, const int32_t* perm_or_null,
                             const selinv_opts* opts, selinv_plan* out);

/* One symbolic analysis for `count` matrices of the same pattern (the poles
 * z_1 .. z_count of a pole expansion, Section 4.3: A(z_k) = H - z_k S all
 * share H's pattern): the plan is the block-diagonal union of count copies
 * of the analysed matrix, run with one launch per level for all of them.
 * Arguments as in selinv_analyze; values and results concatenate pole by
 * pole (selinv_batch_offsets). */
selinv_status selinv_analyze_poles(int64_t n, const int64_t* colptr, const int32_t* rowind,
                                   const selinv_geom* geom, const int32_t* perm_or_null,
                                   const selinv_opts* opts, int32_t count, selinv_plan* out);

/* Bytes of device workspace the plan needs (factor, inverse, index maps):
 * persistent + transient, for one buffer holding both. */
selinv_status selinv_workspace_size(selinv_plan p, size_t* bytes);

/* The two parts of the workspace.  Persistent: the factor, L_hat, T_K, the
 * index maps and task lists, and the checkpoint store; it must stay bound
 * from selinv_factor to selinv_backward.  Transient: the inverse panels and
 * the adjoint arenas (complex plans: the inverse panels and the partial
 * products of split diagonal steps), needed only inside selinv_invert,
 * selinv_invert_complex, selinv_backward and selinv_run.  Either pointer
 * may be NULL. */
selinv_status selinv_workspace_sizes(selinv_plan p, size_t* persistent, size_t* transient);

/* Bind caller-owned device memory (256-byte aligned) and upload the index
 * maps on stream s.  bytes >= selinv_workspace_size: the transient part
 * lives after the persistent part; persistent <= bytes < that: only the
 * persistent part, and a transient buffer must be bound with
 * selinv_bind_transient before an inversion.  The plan never allocates
 * device memory itself. */
selinv_status selinv_bind_workspace(selinv_plan p, void* d_ws, size_t bytes, hipStream_t s);

/* Bind a separate transient buffer (>= the transient size, 256-byte
 * aligned; the caller keeps ownership), or with d_tr = NULL release the one
 * bound (falling back to the workspace's own transient part if it has one).
 * The inverse panels it held are gone: after a release or a rebind,
 * selinv_backward needs checkpoint_every > 1 (it rebuilds them from the
 * checkpoints) or a new selinv_invert.  No device work; drops a captured
 * graph. */
selinv_status selinv_bind_transient(selinv_plan p, void* d_tr, size_t bytes);

/* Supernodal LDL^T of A (Section 2.1, LDL^T form; no pivoting, Section 4).
 * d_valsA: nnzA doubles in the CSC order given to selinv_analyze. */
selinv_status selinv_factor(selinv_plan p, const double* d_valsA, hipStream_t s);

/* Selected inversion (Algorithm 1, root first by the priority levels of
 * Algorithm 2): writes nnzL doubles of A^{-1} to d_sel in the canonical
 * order of selinv_get_pattern. */
selinv_status selinv_invert(selinv_plan p, double* d_sel, hipStream_t s);

/* Complex values (plans analysed with complex_values = 1).  d_valsA: nnzA
 * complex entries as (re, im) pairs of doubles in the CSC order of
 * selinv_analyze; d_sel: nnzL complex entries of A^{-1} on the canonical
 * pattern.  The LDL^T has complex pivots (no sign condition; a zero or
 * non-finite pivot is SELINV_EPIVOT through selinv_sync_status) and every
 * transpose in Algorithm 1 is a plain transpose.  The real-valued calls
 * (selinv_factor, selinv_invert, selinv_backward, selinv_run, selinv_tune,
 * selinv_get_factor) refuse such a plan with SELINV_EINVAL, and these two
 * refuse a real plan. */
selinv_status selinv_factor_complex(selinv_plan p, const double* d_valsA, hipStream_t s);
selinv_status selinv_invert_complex(selinv_plan p, double* d_sel, hipStream_t s);

/* Number of factorizations (selinv_factor, selinv_run) this plan has run.
 * A caller that keeps a plan across calls (an autograd node) records it
 * after the forward and checks it before selinv_backward: a different value
 * means the plan's factor and inverse now belong to other values. */
selinv_status selinv_generation(selinv_plan p, uint64_t* gen);

/* Reverse sweep (adjoint).  For f = sum over the pattern of L of
 * gsel_q * Ainv_q (d_gsel: nnzL doubles, canonical order), writes
 * d_gA[p] = df/da_p for every stored entry p of A (nnzA doubles, the CSC
 * order given to selinv_analyze); an off-diagonal entry stands for A_ij and
 * A_ji, so d_gA = -(A^{-1} S A^{-1}) off the diagonal and half of it on the
 * diagonal, S = G + G^T.  Runs the selected inversion in reverse (leaves
 * first, Algorithm 1 backwards) and then the factorization in reverse (root
 * first).  Needs selinv_factor and selinv_invert of the same values first;
 * uses only the workspace (no allocation).  With checkpoint_every > 1 it
 * first restores the checkpointed levels' inverse panels and recomputes the
 * others (root first); otherwise the inverse panels must still hold the
 * inversion (SELINV_ESTATE after the transient memory was released).
 * SELINV_EUNSUPPORTED if an execution block is wider than 128 columns. */
selinv_status selinv_backward(selinv_plan p, const double* d_gsel, double* d_gA, hipStream_t s);

/* Copy L (unit lower, D on the diagonal) on the canonical pattern to d_L. */
selinv_status selinv_get_factor(selinv_plan p, double* d_L, hipStream_t s);

/* Synchronise s and report a latched pivot failure: returns SELINV_EPIVOT
 * with *bad_col = original index of the first failing column (else -1). */
selinv_status selinv_sync_status(selinv_plan p, hipStream_t s, int64_t* bad_col);

selinv_status selinv_get_info(selinv_plan p, selinv_info* out);

/* Canonical pattern of L in permuted numbering: colptrL[n+1], rowindL[nnzL]
 * (rows ascending, diagonal first), perm[n] (new -> original).  Any pointer
 * may be NULL. */
selinv_status selinv_get_pattern(selinv_plan p, int64_t* colptrL, int32_t* rowindL, int32_t* perm);

/* Sizes of the arrays returned by selinv_get_symbolic. */
selinv_status selinv_symbolic_sizes(selinv_plan p, int64_t* nsuper, int64_t* ncrows, int64_t* nrel);

/* Fundamental-supernode symbolic data for parity checks (host copies):
 * parent[n] column elimination tree (-1 root); xsuper[N+1]; sparent[N];
 * level[N] (Algorithm 2 priority, root = 1); cptr[N+1], crows[] the row
 * structure C(K) below each supernode; rptr[N+1], rel[] the block index
 * maps: per supernode K, for each ancestor J met in C(K) in ascending order,
 * the record [J, a, pos(C[a]), ..., pos(C[c-1])] where a is the first
 * position of C(K) inside J's columns and pos(x) is the row of x within
 * rows(J) = cols(J) U C(J).  Any pointer may be NULL. */
selinv_status selinv_get_symbolic(selinv_plan p, int32_t* parent, int32_t* xsuper, int32_t* sparent,
                                  int32_t* level, int64_t* cptr, int32_t* crows, int64_t* rptr,
                                  int32_t* rel);

/* Kernel kinds reported by the timing calls below. */
enum {
    SELINV_K_ASSEMBLE = 0, /* zero the factor arena, scatter A into it            */
    SELINV_K_LDLT = 1,     /* diagonal block LDL^T, W = L_KK^{-1}, T_K           */
    SELINV_K_PANEL = 2,    /* L(C,K) and the normalised L_hat(C,K)               */
    SELINV_K_SCHUR = 3,    /* Schur update added into ancestor panels            */
    SELINV_K_GEMM = 4,     /* Ainv(C,K) = -Ainv(C,C) L_hat(C,K), gathered        */
    SELINV_K_SDIAG = 5,    /* Ainv(K,K) = T_K - L_hat^T Ainv(C,K), symmetrised   */
    SELINV_K_EXPORT = 6,   /* panels -> canonical values                         */
    SELINV_K_REVSEL = 7,   /* reverse selected inversion (adjoint), leaves first */
    SELINV_K_REVFAC = 8,   /* reverse factorization (adjoint), root first        */
    SELINV_K_QFACTOR = 9,  /* persistent factor level (LDLT, PANEL, SCHUR tasks)  */
    SELINV_K_QINVERT = 10, /* persistent inversion level (GEMM, SDIAG tasks)      */
    SELINV_K_SBFACTOR = 11, /* small blocks, whole factor step, one wave each      */
    SELINV_K_SBINVERT = 12, /* small blocks, whole inversion step, one wave each   */
    SELINV_K_CHECKPOINT = 13, /* inverse panels to / from the checkpoint store      */
    SELINV_NKINDS = 14
};

/* Enable (1) or disable (0) per-launch timing: every later kernel launch of
 * this plan is stamped with HIP start/stop events in its dispatch. */
selinv_status selinv_profile(selinv_plan p, int32_t enable);

/* Wait for the recorded launches and return, per kernel kind, the summed
 * duration in ms and the launch count (arrays of SELINV_NKINDS); clears the
 * record.  Either pointer may be NULL. */
selinv_status selinv_profile_read(selinv_plan p, double* ms, int64_t* launches);

/* Algorithmic flops and bytes per kernel kind (arrays of SELINV_NKINDS) on
 * the execution blocks: of one selinv_factor (ASSEMBLE..SCHUR and SBFACTOR),
 * one selinv_invert (GEMM, SDIAG, EXPORT, SBINVERT), one selinv_backward
 * (REVSEL, REVFAC) and, for selinv_run, of its factor and inversion levels
 * (QFACTOR, QINVERT).  Blocks of at most 16 columns and 256 rows below take
 * the small-block kinds in selinv_factor / selinv_invert. */
selinv_status selinv_kernel_work(selinv_plan p, double* flops, double* bytes);

/* Raw device arenas, for kernel-level checks: which = 0 factor panels
 * (L_KK with D on the diagonal; F(C,K) in the C rows), 1 inverse panels,
 * 2 L_hat(C,K) blocks, 3 scratch, 4 T_K blocks; after selinv_backward:
 * 5 the adjoint of the factor panels, 6 that of L_hat, 7 that of T_K.  The layout of
 * each execution block is given by selinv_get_blocks.  *count = number of
 * doubles (a complex plan: two per entry, (re, im); which = 5..7 is then
 * SELINV_EINVAL); d_out (device, may be NULL) receives a copy on stream s. */
selinv_status selinv_get_arena(selinv_plan p, int32_t which, double* d_out, int64_t* count, hipStream_t s);

/* Execution blocks (host copies, nblocks entries each; any may be NULL):
 * first column, width s, |C|, priority level, and the offsets (in doubles)
 * of the block's (s+c) x s panel, its c x s L_hat block and its s x s
 * W / T blocks; crow_off[b] indexes the rows C(b) in the order returned by
 * selinv_get_exec_rows. */
selinv_status selinv_get_blocks(selinv_plan p, int32_t* first, int32_t* s, int32_t* c, int32_t* level,
                                int64_t* poff, int64_t* hoff, int64_t* woff, int64_t* crow_off);

/* Row structures C(b) of the execution blocks, concatenated (host copy). */
selinv_status selinv_get_exec_rows(selinv_plan p, int32_t* rows);

/* ------------------------------------------------------------------------
 * Batched form and persistent execution.
 *
 * A batch of independent matrices is analysed as the block-diagonal matrix
 * they form: its elimination tree is the forest of their trees, and the
 * priority levels of Algorithm 2 (root = 1 in every tree) line up across the
 * batch (Section 3.4), so one launch per level serves every matrix; the
 * matrices are independent problems, like the pole matrices of the
 * electronic-structure application (Section 4.3).  The result
 * is an ordinary plan: every call above works on it, with the matrices'
 * unknowns, A entries and L entries concatenated in batch order.
 * ------------------------------------------------------------------------ */

/* Analyse `count` matrices (each as in selinv_analyze, with geoms[m] its
 * geometry; geoms may be NULL) into one plan.  Per matrix m: ns[m] order,
 * colptrs[m][ns[m]+1], rowinds[m][...] host arrays read during the call.
 * Columns of matrix m are ns[0] + ... + ns[m-1] + its own (permuted)
 * indices; perm maps within each matrix.  A failing matrix is named in the
 * error message.  The total order must stay below 2^31 - 1. */
selinv_status selinv_analyze_batch(int32_t count, const int64_t* ns, const int64_t* const* colptrs,
                                   const int32_t* const* rowinds, const selinv_geom* geoms, const selinv_opts* opts,
                                   selinv_plan* out);

/* Offsets of the matrices of a batch (count + 1 entries each; any pointer may
 * be NULL): columns, A's entries (the d_valsA layout) and L's entries (the
 * d_sel layout).  A plan from selinv_analyze is a batch of one. */
selinv_status selinv_batch_offsets(selinv_plan p, int32_t* count, int64_t* n_off, int64_t* nnzA_off,
                                   int64_t* nnzL_off);

/* Schedule of the persistent path.  Each level's queue lists its tasks phase
 * by phase (factor: diagonal block, L_hat tiles, Schur tiles; inversion:
 * zeroing of split blocks, gather-GEMM tiles, diagonal tiles) and, within a
 * phase, in `order`: 0 plan order (matrix by matrix), 1 largest block first,
 * 2 round robin over the matrices, 3 largest tile first.  bn_cap: widest
 * output tile of the gather-GEMM and panel products (16, 32, 64, 128).
 * split_fill (0..4096): contractions are split over work-groups while a
 * level has fewer output tiles than this (0 = never).  grid_mult: resident
 * work-groups per compute unit (capped by the kernel's occupancy).
 * small_s (0, 1, 2, 4, 8, 16): blocks of at most small_s columns and at most
 * 256 rows below run whole on one wave each, four to a task (0 = none); a
 * level with only such blocks runs a lighter kernel variant with as many
 * resident work-groups as it allows, each wave taking a fixed share.
 * mb_tiles (0..4096): other blocks with at most this many gather-GEMM output
 * tiles run whole on one work-group, phase after phase, so they wait for no
 * other work-group; larger blocks are split into tile tasks that wait for
 * their block's earlier phases. */
typedef struct {
    int32_t order;
    int32_t bn_cap;
    int32_t split_fill;
    int32_t grid_mult;
    int32_t small_s;
    int32_t mb_tiles;
} selinv_sched;

/* Rebuild the work queues for schedule *sc and upload them on stream s
 * (synchronises s; s is unused before selinv_bind_workspace); drops a
 * captured graph.  SELINV_EINVAL for a field out of range.  The workspace
 * reserves queue space for every valid schedule (a bound that holds for
 * any of them). */
selinv_status selinv_set_schedule(selinv_plan p, const selinv_sched* sc, hipStream_t s);
selinv_status selinv_get_schedule(selinv_plan p, selinv_sched* sc);

/* Host copy of one level's queue (sweep 0 factor, 1 inversion; level 1 =
 * roots) as 8 int32 per task: block, row origin, column origin, tile width,
 * contraction begin, end, flags (bit 0 atomic accumulation, bit 1 others
 * wait for it, bits 8..15 the operation: 0 LDLT, 1 PANEL, 2 SCHUR, 3 ZERO,
 * 4 GEMM, 5 SDIAG, 6 small-block factor, 7 small-block inversion, 8
 * medium-block factor, 9 medium-block inversion) and the number of earlier
 * tasks of the same block it waits for.  A small-block task lists up to four
 * block ids in its first four fields (-1 = none); a medium-block task names
 * its block and its tile width.
 * *count = tasks; tasks may be NULL. */
selinv_status selinv_get_queue(selinv_plan p, int32_t sweep, int32_t level, int32_t* tasks, int64_t* count);

/* Polls a dependency wait makes before it gives up and latches
 * SELINV_EQUEUE (default 2^22, far beyond any legitimate wait); the kernel
 * still runs every task, so it always finishes.  A small value forces the
 * error path for tests.  Drops a captured graph. */
selinv_status selinv_set_spin_limit(selinv_plan p, uint32_t polls);

/* Factor and invert (same results as selinv_factor + selinv_invert, up to
 * the order of floating-point atomic additions) with one persistent
 * work-queue launch per level and sweep.  d_valsA / d_sel as in
 * selinv_factor / selinv_invert.  use_graph = 1: the launch sequence is
 * captured into a HIP graph on the first call (and again whenever d_valsA,
 * d_sel, the schedule or the workspace change) and replayed on stream s.
 * Errors found on the device are reported by selinv_sync_status. */
selinv_status selinv_run(selinv_plan p, const double* d_valsA, double* d_sel, int32_t use_graph, hipStream_t s);

/* Autotuner: times selinv_run (no graph) on the given buffers for schedules
 * along each axis in turn (small_s 0/4/16, mb_tiles 0/8/64, order, bn_cap
 * 32/64/128, split_fill 0/512/4096, grid_mult 1/2/4), keeps the fastest and
 * leaves it set.  cache_path (may be NULL):
 * a JSON file of earlier choices keyed by device and block structure; a hit
 * skips the timing, a miss adds the choice.  On return d_sel holds the
 * selected inverse of d_valsA; *chosen and *best_ms (may be NULL) the
 * schedule and its time in ms.  Synchronises s. */
selinv_status selinv_tune(selinv_plan p, const double* d_valsA, double* d_sel, const char* cache_path,
                          selinv_sched* chosen, double* best_ms, hipStream_t s);

/* Device ceilings for the roofline, measured on the current device (not
 * part of the method): a sustained FP64 MFMA rate (every wave issuing
 * independent v_mfma_f64_16x16x4f64 back to back, best of four launches)
 * and a copy bandwidth (the first half of d_buf copied into the second,
 * bytes read + written over the kernel time, best of four after one
 * warm-up).  d_buf: caller-owned device scratch of `bytes` >= 64 MiB,
 * 256-byte aligned (its contents are overwritten; 2 GiB or more measures
 * HBM rather than cache).  Synchronises s.  SELINV_EINVAL for a bad
 * buffer. */
selinv_status selinv_measure_peaks(void* d_buf, size_t bytes, double* fp64_mfma_tflops, double* copy_gbs,
                                   hipStream_t s);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * ------------------------------------------------------------------------ */

/* Size of the library's static per-device scratch array (64 MiB): each GPU
 * the library runs on holds one copy until the process ends. */
#define SELINV_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* selinv_factor + selinv_invert (same results up to the order of
 * floating-point atomic additions) with the plan's whole workspace (tables,
 * factor, inverse panels) in the static scratch array instead of a bound
 * workspace: the call allocates nothing (no hipMalloc, no allocating
 * library routine).  The plan needs no selinv_bind_workspace and its bound
 * workspace, if any, is left untouched.  d_valsA: nnzA doubles as in
 * selinv_factor; d_sel: nnzL doubles as in selinv_invert (caller-owned).
 * The first call on a device looks up the array's device address; the
 * plan's tables are copied in (host to device, stream-ordered) whenever
 * the array last served another plan, so repeated calls with one plan
 * launch kernels only.  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other threads) race.  bad_col: NULL, or the call synchronises s
 * and reports a pivot failure as SELINV_EPIVOT with *bad_col = original
 * column (else -1).  SELINV_ENOMEM when selinv_workspace_size exceeds
 * SELINV_STATIC_SCRATCH_BYTES; SELINV_EINVAL for a plan with complex
 * values. */
selinv_status selinv_factor_invert_static(selinv_plan p, const double* d_valsA, double* d_sel, int64_t* bad_col,
                                          hipStream_t s);

/* Message for the last failing call on this thread. */
const char* selinv_last_error(void);

void selinv_destroy(selinv_plan p);

#ifdef __cplusplus
}
#endif
#endif /* SELINV_H */
