// Launch wrappers for the device kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <string>
#include <vector>

#include "plan.hpp"

namespace selinv {

// Device views of the workspace sub-arrays.
struct DevPtrs {
    double *Lp, *Ap, *Hp, *Wp, *Tp;
    double *Zb, *Hb, *Tb;  // adjoint arenas
    double* Zs;            // complex plans: partial products of the split diagonal step
    unsigned long long* status;
    const BlockDesc* blocks;
    const int32_t* crow;
    const int64_t *cbase, *rbase;
    const int64_t* cr2;  // (cbase, rbase) interleaved, for the gather loops
    const int32_t* rel;
    const int64_t *asm_off, *exp_off;
    const int32_t* colblk;     // column -> execution block
    const int64_t* colptrL;    // canonical column pointers of L
    const Task *t_diag, *t_ldlt, *t_panel, *t_schur, *t_gemm, *t_sdiag, *t_zero, *t_sb;
    const Task *t_rs1, *t_rs2, *t_rs3, *t_rf1a, *t_rf1b, *t_rf2;
    double* ck;             // checkpoint store of inverse panels
    const int64_t* ck_off;  // per block: its offset in the store (-1: not stored)
};

hipError_t kernels_init();
hipError_t launch_backward_init(Prof* P, const DevPtrs& D, int64_t arena, int64_t harena, const double* gsel,
                                int64_t nnzL, hipStream_t s);
// rs3_cuts[0..ncuts): the level's t_rs3 tasks in groups launched one after
// the other (colour groups of disjoint scatters in the deterministic mode)
hipError_t launch_revsel_level(Prof* P, const DevPtrs& D, int64_t a0, int64_t na, int64_t b0, int64_t nb,
                               const int64_t* rs3_cuts, int ncuts, hipStream_t s);
hipError_t launch_revfac_init(Prof* P, const DevPtrs& D, int64_t nblocks, int64_t arena, hipStream_t s);
hipError_t launch_revfac_level(Prof* P, const DevPtrs& D, int64_t a0, int64_t na, int64_t b0, int64_t nb, int64_t c0,
                               int64_t nc, int64_t d0, int64_t nd, hipStream_t s);
// set-up of the inversion: tasks t_zero[t0 .. t0+n)
hipError_t launch_zero_x(Prof* P, const DevPtrs& D, int64_t t0, int64_t n, hipStream_t s);
// inverse panels of the blocks listed by t_diag[0 .. ntasks) that have a
// checkpoint slot: dir 0 copies them to the store, dir 1 back
hipError_t launch_checkpoint(Prof* P, const DevPtrs& D, int64_t ntasks, int dir, hipStream_t s);
hipError_t launch_export_L(Prof* P, const DevPtrs& D, int64_t n, double* out, hipStream_t s);
hipError_t launch_status_reset(unsigned long long* status, hipStream_t s);
hipError_t launch_fill(Prof* P, int kind, double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_scatter_set(Prof* P, int kind, const double* src, const int64_t* off, int64_t n, double* dst,
                              hipStream_t s);
hipError_t launch_gather(Prof* P, int kind, const double* src, const int64_t* off, int64_t n, double* dst,
                         hipStream_t s);
// diagonal blocks with 1x1/2x2 (Bunch-Kaufman) pivots, T only; diag as for
// launch_ldlt_level (s <= 32, <= 64 and wider)
hipError_t launch_ldlt_bk(Prof* P, const DevPtrs& D, const int64_t diag[4], hipStream_t s);
// diag[0..3]: the level's diagonal-block tasks for s <= 32, <= 64 and wider
hipError_t launch_ldlt_level(Prof* P, const DevPtrs& D, const int64_t diag[4], int require_spd, hipStream_t s);
// panel_deep bit 0: whole-contraction panel kernel; bit 1: whole-contraction
// Schur kernel allowed for small groups (0 in the deterministic mode)
hipError_t launch_panel_level(Prof* P, const DevPtrs& D, int64_t panel0, int64_t npanel, int panel_deep, hipStream_t s);
// Schur colour groups [g0, g1) of a level, cuts as in schur_cuts
hipError_t launch_schur_groups(Prof* P, const DevPtrs& D, const int64_t* cuts, int g0, int g1, int panel_deep,
                               hipStream_t s);
// diagonal-step tasks t_sdiag[sdiag0 .. sdiag_cut) then [sdiag_cut .. sdiag1),
// as two launches
hipError_t launch_invert_level(Prof* P, const DevPtrs& D, int64_t gemm0, int64_t ngemm, int64_t sdiag0,
                               int64_t sdiag_cut, int64_t sdiag1, hipStream_t s);
// persistent work-queue kernels: resident work-groups per CU, and one
// level's launch over ntasks queue entries at q
hipError_t persist_occupancy(int occ[kNumVariants]);
hipError_t launch_fill_u32(Prof* P, int kind, unsigned* p, int64_t n, hipStream_t s);
hipError_t launch_persist_factor(Prof* P, const DevPtrs& D, const Task* q, int64_t ntasks, unsigned* head,
                                 unsigned* done, int grid, int variant, int require_spd, unsigned spin_limit,
                                 hipStream_t s);
hipError_t launch_persist_invert(Prof* P, const DevPtrs& D, const Task* q, int64_t ntasks, unsigned* head,
                                 unsigned* done, int grid, int variant, unsigned spin_limit, hipStream_t s);
// small-block path of one level (per-level launches)
hipError_t launch_sb_factor(Prof* P, const DevPtrs& D, int64_t sb0, int64_t nsb, int require_spd, hipStream_t s);
hipError_t launch_sb_invert(Prof* P, const DevPtrs& D, int64_t sb0, int64_t nsb, hipStream_t s);

// complex-symmetric path (zkernels.hip): values are (re, im) pairs; the level
// lists are those of the deterministic schedule (blocks of at most 64 columns)
hipError_t launch_zassemble(const double* vals, const int64_t* off, int64_t n, double* Lp, hipStream_t s);
hipError_t launch_zexport(const double* Ap, const int64_t* off, int64_t n, double* out, hipStream_t s);
hipError_t launch_zfactor_level(const DevPtrs& D, int64_t diag0, int64_t ndiag, int64_t panel0, int64_t npanel,
                                const int64_t* schur_cuts, int ncuts, hipStream_t s);
// inversion of one level: the gather-GEMM's whole tiles [gemm[0], gemm[1]),
// pieces of split tiles [gemm[1], gemm[2]) and their summing tasks
// [gemm[2], gemm[3]); then the diagonal step's tasks [sdiag0, sdiag_cut)
// (whole blocks and pieces) and summing tasks [sdiag_cut, sdiag1)
hipError_t launch_zinvert_level(const DevPtrs& D, const int64_t gemm[4], int64_t sdiag0, int64_t sdiag_cut,
                                int64_t sdiag1, hipStream_t s);

// Launch sequences and helpers of the C ABI (capi.cpp), shared with the
// static-scratch entry point.
DevPtrs dev_ptrs_at(const selinv_plan_s* P, char* ws, char* tr);
hipError_t upload_tables(selinv_plan_s* P, char* ws, hipStream_t s);
hipError_t factor_levels(selinv_plan_s* P, const DevPtrs& D, const double* d_valsA, hipStream_t s, Prof* prof);
hipError_t invert_level(selinv_plan_s* P, const DevPtrs& D, int l, hipStream_t s, Prof* prof);
hipError_t invert_levels(selinv_plan_s* P, const DevPtrs& D, double* d_sel, hipStream_t s, Prof* prof);
hipError_t rebuild_inverse(selinv_plan_s* P, const DevPtrs& D, hipStream_t s, Prof* prof);
selinv_status set_error(selinv_status st, const std::string& msg);

}  // namespace selinv
