// C ABI of the selected-inversion library (declared in include/selinv.h).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>

#include "kernels.hpp"
#include "plan.hpp"
#include "tiles.hpp"

using namespace selinv;

namespace {
thread_local std::string g_err;

selinv_status fail(selinv_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

selinv_status hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return SELINV_EHIP;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

void compute_layout(selinv_plan_s* P)
{
    DeviceLayout& L = P->lay;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return at;
    };
    // persistent part (complex values: two doubles per entry, no adjoint)
    const size_t w = P->opts.complex_values ? 2 : 1;
    L.lp = take(w * sizeof(double) * P->arena);
    L.hp = take(w * sizeof(double) * P->harena);
    L.wp = take(w * sizeof(double) * P->warena);
    L.tp = take(w * sizeof(double) * P->warena);
    L.status = take(2 * sizeof(unsigned long long));
    L.blocks = take(sizeof(BlockDesc) * P->blocks.size());
    L.crow = take(sizeof(int32_t) * P->crow.size());
    L.cbase = take(sizeof(int64_t) * P->cbase.size());
    L.cr2 = take(2 * sizeof(int64_t) * P->cbase.size());
    L.rbase = take(sizeof(int64_t) * P->rbase.size());
    L.rel = take(sizeof(int32_t) * P->rel.size());
    L.asm_off = take(sizeof(int64_t) * P->asm_off.size());
    L.exp_off = take(sizeof(int64_t) * P->exp_off.size());
    L.colblk = take(sizeof(int32_t) * P->colblk.size());
    L.colptrL = take(sizeof(int64_t) * P->colptrL.size());
    L.t_diag = take(sizeof(Task) * P->t_diag.tasks.size());
    L.t_ldlt = take(sizeof(Task) * P->t_ldlt.tasks.size());
    L.t_sb = take(sizeof(Task) * P->t_sb.tasks.size());
    L.t_panel = take(sizeof(Task) * P->t_panel.tasks.size());
    L.t_schur = take(sizeof(Task) * P->t_schur.tasks.size());
    L.t_gemm = take(sizeof(Task) * P->t_gemm.tasks.size());
    L.t_sdiag = take(sizeof(Task) * P->t_sdiag.tasks.size());
    L.t_zero = take(sizeof(Task) * P->t_zero.size());
    L.t_rs1 = take(sizeof(Task) * P->t_rs1.tasks.size());
    L.t_rs2 = take(sizeof(Task) * P->t_rs2.tasks.size());
    L.t_rs3 = take(sizeof(Task) * P->t_rs3.tasks.size());
    L.t_rf1a = take(sizeof(Task) * P->t_rf1a.tasks.size());
    L.t_rf1b = take(sizeof(Task) * P->t_rf1b.tasks.size());
    L.t_rf2 = take(sizeof(Task) * P->t_rf2.tasks.size());
    L.q_fac = take(sizeof(Task) * P->q_cap_fac);
    L.q_inv = take(sizeof(Task) * P->q_cap_inv);
    // completion counters (factor, inversion) per block, then the queue
    // heads (factor, inversion) per level
    const size_t nb = P->blocks.size(), nl = (size_t)std::max(P->exec.depth, 0);
    L.q_done = take(sizeof(unsigned) * 2 * (nb + nl));
    L.q_head = L.q_done + sizeof(unsigned) * 2 * nb;
    L.ck = take(sizeof(double) * (size_t)P->ck_size);
    L.ck_off = take(sizeof(int64_t) * P->ck_off.size());
    L.persist = o;
    // transient part
    o = 0;
    const size_t adj = P->opts.complex_values ? 0 : 1;
    L.ap = take(w * sizeof(double) * P->arena);
    L.zb = take(adj * sizeof(double) * P->arena);
    L.hb = take(adj * sizeof(double) * P->harena);
    L.tb = take(adj * sizeof(double) * P->warena);
    L.zsp = take(P->opts.complex_values ? sizeof(double) * kZSlotDoubles * (size_t)P->zsd_slots : 0);
    L.transient = o;
    L.total = L.persist + L.transient;
    P->info.workspace_bytes = (int64_t)L.total;
}

}  // namespace

namespace selinv {
DevPtrs dev_ptrs_at(const selinv_plan_s* P, char* w, char* t)
{
    const DeviceLayout& L = P->lay;
    // t may be null: then the transient arenas are unusable
    DevPtrs D;
    D.Lp = (double*)(w + L.lp);
    D.Ap = t ? (double*)(t + L.ap) : nullptr;
    D.Hp = (double*)(w + L.hp);
    D.Wp = (double*)(w + L.wp);
    D.Tp = (double*)(w + L.tp);
    D.status = (unsigned long long*)(w + L.status);
    D.blocks = (const BlockDesc*)(w + L.blocks);
    D.crow = (const int32_t*)(w + L.crow);
    D.cbase = (const int64_t*)(w + L.cbase);
    D.cr2 = (const int64_t*)(w + L.cr2);
    D.rbase = (const int64_t*)(w + L.rbase);
    D.rel = (const int32_t*)(w + L.rel);
    D.asm_off = (const int64_t*)(w + L.asm_off);
    D.exp_off = (const int64_t*)(w + L.exp_off);
    D.colblk = (const int32_t*)(w + L.colblk);
    D.colptrL = (const int64_t*)(w + L.colptrL);
    D.t_diag = (const Task*)(w + L.t_diag);
    D.t_ldlt = (const Task*)(w + L.t_ldlt);
    D.t_sb = (const Task*)(w + L.t_sb);
    D.t_panel = (const Task*)(w + L.t_panel);
    D.t_schur = (const Task*)(w + L.t_schur);
    D.t_gemm = (const Task*)(w + L.t_gemm);
    D.t_sdiag = (const Task*)(w + L.t_sdiag);
    D.t_zero = (const Task*)(w + L.t_zero);
    D.Zb = t ? (double*)(t + L.zb) : nullptr;
    D.Hb = t ? (double*)(t + L.hb) : nullptr;
    D.Tb = t ? (double*)(t + L.tb) : nullptr;
    D.Zs = t ? (double*)(t + L.zsp) : nullptr;
    D.ck = (double*)(w + L.ck);
    D.ck_off = (const int64_t*)(w + L.ck_off);
    D.t_rs1 = (const Task*)(w + L.t_rs1);
    D.t_rs2 = (const Task*)(w + L.t_rs2);
    D.t_rs3 = (const Task*)(w + L.t_rs3);
    D.t_rf1a = (const Task*)(w + L.t_rf1a);
    D.t_rf1b = (const Task*)(w + L.t_rf1b);
    D.t_rf2 = (const Task*)(w + L.t_rf2);
    return D;
}

template <class T>
static hipError_t upload(char* ws, size_t off, const std::vector<T>& v, hipStream_t s)
{
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(ws + off, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s);
}

// the plan's tables (block descriptors, index maps, task lists, queues,
// checkpoint offsets) into the persistent part at ws, on stream s
hipError_t upload_tables(selinv_plan_s* P, char* ws, hipStream_t s)
{
    const DeviceLayout& L = P->lay;
    P->cr2.resize(2 * P->cbase.size());
    for (size_t p = 0; p < P->cbase.size(); p++) {
        P->cr2[2 * p] = P->cbase[p];
        P->cr2[2 * p + 1] = P->rbase[p];
    }
    hipError_t e = upload(ws, L.blocks, P->blocks, s);
    if (!e) e = upload(ws, L.crow, P->crow, s);
    if (!e) e = upload(ws, L.cbase, P->cbase, s);
    if (!e) e = upload(ws, L.cr2, P->cr2, s);
    if (!e) e = upload(ws, L.rbase, P->rbase, s);
    if (!e) e = upload(ws, L.rel, P->rel, s);
    if (!e) e = upload(ws, L.asm_off, P->asm_off, s);
    if (!e) e = upload(ws, L.exp_off, P->exp_off, s);
    if (!e) e = upload(ws, L.colblk, P->colblk, s);
    if (!e) e = upload(ws, L.colptrL, P->colptrL, s);
    if (!e) e = upload(ws, L.t_diag, P->t_diag.tasks, s);
    if (!e) e = upload(ws, L.t_ldlt, P->t_ldlt.tasks, s);
    if (!e) e = upload(ws, L.t_sb, P->t_sb.tasks, s);
    if (!e) e = upload(ws, L.t_panel, P->t_panel.tasks, s);
    if (!e) e = upload(ws, L.t_schur, P->t_schur.tasks, s);
    if (!e) e = upload(ws, L.t_gemm, P->t_gemm.tasks, s);
    if (!e) e = upload(ws, L.t_sdiag, P->t_sdiag.tasks, s);
    if (!e) e = upload(ws, L.t_zero, P->t_zero, s);
    if (!e) e = upload(ws, L.t_rs1, P->t_rs1.tasks, s);
    if (!e) e = upload(ws, L.t_rs2, P->t_rs2.tasks, s);
    if (!e) e = upload(ws, L.t_rs3, P->t_rs3.tasks, s);
    if (!e) e = upload(ws, L.t_rf1a, P->t_rf1a.tasks, s);
    if (!e) e = upload(ws, L.t_rf1b, P->t_rf1b.tasks, s);
    if (!e) e = upload(ws, L.t_rf2, P->t_rf2.tasks, s);
    if (!e) e = upload(ws, L.q_fac, P->q_fac, s);
    if (!e) e = upload(ws, L.q_inv, P->q_inv, s);
    if (!e) e = upload(ws, L.ck_off, P->ck_off, s);
    return e;
}

selinv_status set_error(selinv_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}
}  // namespace selinv

namespace {
DevPtrs dev_ptrs(const selinv_plan_s* P) { return dev_ptrs_at(P, P->ws, P->tr); }
}  // namespace

extern "C" {

const char* selinv_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {
// Validate one matrix and run the host analysis into P (no schedule yet).
selinv_status analyze_one(int64_t n, const int64_t* colptr, const int32_t* rowind, const selinv_geom* geom,
                          const int32_t* perm_or_null, const selinv_opts& o, selinv_plan_s* P, std::string& err)
{
    if (n < 0 || n > INT32_MAX - 1) return err = "n out of range", SELINV_EINVAL;
    if (n > 0 && (!colptr || !rowind)) return err = "colptr/rowind is NULL", SELINV_EINVAL;
    if (n > 0) {
        if (colptr[0] != 0) return err = "colptr[0] must be 0", SELINV_EINVAL;
        for (int64_t j = 0; j < n; j++) {
            if (colptr[j + 1] < colptr[j]) return err = "colptr is not monotone", SELINV_EINVAL;
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                if (rowind[p] < j || rowind[p] >= n)
                    return err = "row index outside the lower triangle at column " + std::to_string(j), SELINV_EINVAL;
                if (p > colptr[j] && rowind[p] <= rowind[p - 1])
                    return err = "rows not strictly increasing in column " + std::to_string(j), SELINV_EINVAL;
            }
        }
    }
    if (geom && geom->ndim > 0) {
        if (geom->ndim > 3) return err = "geom.ndim must be 0..3", SELINV_EINVAL;
        int64_t pts = 1;
        for (int d = 0; d < geom->ndim; d++) {
            if (geom->dims[d] <= 0) return err = "geom.dims must be positive", SELINV_EINVAL;
            pts *= geom->dims[d];
        }
        int dofs = geom->dofs_per_point > 0 ? geom->dofs_per_point : 1;
        if (pts * dofs != n) return err = "geometry does not match n", SELINV_EINVAL;
    }
    P->n = n;
    P->opts = o;
    P->nnzA = n > 0 ? colptr[n] : 0;
    P->colptr.assign(colptr, colptr + (n > 0 ? n + 1 : 1));
    if (n == 0) P->colptr.assign(1, 0);
    if (P->nnzA > 0) P->rowind.assign(rowind, rowind + P->nnzA);
    return analyze(P, geom, perm_or_null, err);
}

selinv_status resolve_opts(const selinv_opts* opts, selinv_opts& o)
{
    o = selinv_opts{128, 1, 1, 0, 0, 0, 1, 0, 0, 0};
    if (opts) o = *opts;
    if (o.pivoting != 0 && o.pivoting != 1) return fail(SELINV_EINVAL, "pivoting must be 0 or 1");
    if (o.pivoting && o.require_spd) return fail(SELINV_EINVAL, "pivoting needs require_spd = 0");
    if (o.pivoting && o.complex_values)
        return fail(SELINV_EUNSUPPORTED, "pivoting is not supported for complex values");
    if (o.complex_values != 0 && o.complex_values != 1) return fail(SELINV_EINVAL, "complex_values must be 0 or 1");
    if (o.relaxed != 0 && o.relaxed != 1) return fail(SELINV_EINVAL, "relaxed must be 0 or 1");
    if (o.relaxed && !o.fuse_chains) return fail(SELINV_EINVAL, "relaxed supernodes need fuse_chains = 1");
    if (o.sep_order != 0 && o.sep_order != 1) return fail(SELINV_EINVAL, "sep_order must be 0 or 1");
    if (o.deterministic != 0 && o.deterministic != 1) return fail(SELINV_EINVAL, "deterministic must be 0 or 1");
    if (o.checkpoint_every < 1) o.checkpoint_every = 1;
    if (o.max_super <= 0) o.max_super = 128;
    // execution blocks default to <= 128 columns (the width the register
    // sweep of the diagonal block holds); the L pattern does not depend on
    // the partition, only the reported fundamental supernodes use max_super
    if (o.exec_cap <= 0) o.exec_cap = std::min(o.max_super, (int32_t)kLdsDiagMax);
    if (o.max_super > 256 || o.exec_cap > 256)
        return fail(SELINV_EUNSUPPORTED, "supernode width cap above 256 is not supported");
    if (o.complex_values) {
        // the complex kernels hold a whole diagonal block in registers (four
        // 16-row sub-blocks) and one 64 x 64 output tile per diagonal step, and
        // add without atomics: blocks of at most 64 columns, deterministic schedule
        o.exec_cap = std::min(o.exec_cap, (int32_t)kZMaxS);
        o.deterministic = 1;
    }
    // the pivoted diagonal kernel holds a whole block in registers
    if (o.pivoting) o.exec_cap = std::min(o.exec_cap, (int32_t)kLdsDiagMax);
    return SELINV_OK;
}

// queue-tile widths and split fills the schedule may take; the workspace
// reserves queue entries for the largest of them
constexpr int32_t kTuneOrders[] = {qoPlan, qoLpt, qoRoundRobin, qoTileLpt};
constexpr int32_t kTuneBn[] = {32, 64, 128};
constexpr int32_t kTuneFill[] = {0, 512, 4096};
constexpr int32_t kTuneGrid[] = {1, 2, 4};
constexpr int32_t kTuneSmall[] = {0, 4, 16};
constexpr int32_t kTuneMb[] = {0, 8, 64};
constexpr int32_t kSmallValues[] = {0, 1, 2, 4, 8, 16};  // the accepted small_s values

// per level: the persistent variant its queue needs (light when it holds
// only small-block tasks, else the class of its widest diagonal block or
// output tile)
void level_variants(const selinv_plan_s* P, const std::vector<Task>& q, const std::vector<int64_t>& off,
                    bool factor, std::vector<uint8_t>& var)
{
    const int sb_op = factor ? qSbFactor : qSbInvert;
    var.assign(off.empty() ? 0 : off.size() - 1, 0);
    for (size_t l = 0; l + 1 < off.size(); l++) {
        bool tiled = false;
        int widest = 0;
        for (int64_t k = off[l]; k < off[l + 1]; k++) {
            const int op = q[k].flags >> 8;
            if (op == sb_op) continue;
            tiled = true;
            if (op == qLdlt || op == qMbFactor) widest = std::max(widest, P->blocks[q[k].b].s);
            if (op == qGemm || op == qMbInvert) widest = std::max(widest, q[k].bn);
        }
        if (factor) var[l] = !tiled ? kLightFactor : widest <= 32 ? kFactor32 : widest <= 64 ? kFactor64 : kFactor128;
        else var[l] = !tiled ? kLightInvert : widest <= 32 ? kInvert32 : widest <= 64 ? kInvert64 : kInvert128;
    }
}

// per-level task lists, persistent queues for the default schedule, and
// the device layout
void finish_plan(selinv_plan_s* P)
{
    if (P->b_noff.empty()) {  // a single matrix: a batch of one
        P->blk_matrix.assign(P->blocks.size(), 0);
        P->b_noff = {0, P->n};
        P->b_aoff = {0, P->nnzA};
        P->b_loff = {0, P->colptrL.back()};
    }
    build_schedule(P);
    queue_bound(P, P->q_cap_fac, P->q_cap_inv);
    build_queues(P, P->sched, P->q_fac, P->q_fac_off, P->q_inv, P->q_inv_off);
    level_variants(P, P->q_fac, P->q_fac_off, true, P->q_var_fac);
    level_variants(P, P->q_inv, P->q_inv_off, false, P->q_var_inv);
    compute_layout(P);
}

void drop_graph(selinv_plan_s* P)
{
    if (P->graph_exec) (void)hipGraphExecDestroy(P->graph_exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->graph_exec = nullptr;
    P->graph = nullptr;
    P->graph_in = nullptr;
    P->graph_out = nullptr;
}
}  // namespace

namespace selinv {
// Factor, leaves first: assemble, then per level the small blocks and the
// tiled path (diagonal blocks, panels, Schur colour groups).
hipError_t factor_levels(selinv_plan_s* P, const DevPtrs& D, const double* d_valsA, hipStream_t s, Prof* prof)
{
    hipError_t e = launch_status_reset(D.status, s);
    if (!e) e = launch_fill(prof, kAssemble, D.Lp, P->arena, 0.0, s);
    if (!e) e = launch_scatter_set(prof, kAssemble, d_valsA, D.asm_off, P->nnzA, D.Lp, s);
    const int spd = P->opts.require_spd ? 1 : 0;
    const int deep_ok = P->opts.deterministic ? 0 : 3;
    for (int l = P->exec.depth - 1; l >= 0 && !e; l--) {
        const auto& q = P->t_sb.off;
        const auto& b = P->t_panel.off;
        const auto& a = P->t_ldlt.off;
        const auto& cut = P->schur_cuts[l];
        const int deep = P->panel_deep[l] & deep_ok;
        const int64_t dg[4] = {a[l], P->ldlt_cut[2 * l], P->ldlt_cut[2 * l + 1], a[l + 1]};
        e = launch_sb_factor(prof, D, q[l], q[l + 1] - q[l], spd, s);
        if (!e) e = P->opts.pivoting ? launch_ldlt_bk(prof, D, dg, s)
                                     : launch_ldlt_level(prof, D, dg, spd, s);
        if (!e) e = launch_panel_level(prof, D, b[l], b[l + 1] - b[l], deep, s);
        if (!e) e = launch_schur_groups(prof, D, cut.data(), 0, (int)cut.size() - 1, deep, s);
    }
    return e;
}

// One level of the inversion: small blocks, gather-GEMM, diagonal step (in
// two launches where the deterministic mode orders the half-products).
hipError_t invert_level(selinv_plan_s* P, const DevPtrs& D, int l, hipStream_t s, Prof* prof)
{
    const auto& q = P->t_sb.off;
    const auto& g = P->t_gemm.off;
    const auto& d = P->t_sdiag.off;
    hipError_t e = launch_sb_invert(prof, D, q[l], q[l + 1] - q[l], s);
    if (!e) e = launch_invert_level(prof, D, g[l], g[l + 1] - g[l], d[l], P->sdiag_cut[l], d[l + 1], s);
    return e;
}

// Inversion, root first, then the export to the canonical order.
hipError_t invert_levels(selinv_plan_s* P, const DevPtrs& D, double* d_sel, hipStream_t s, Prof* prof)
{
    hipError_t e = launch_zero_x(prof, D, 0, (int64_t)P->t_zero.size(), s);
    for (int l = 0; l < P->exec.depth && !e; l++) e = invert_level(P, D, l, s, prof);
    if (!e) e = launch_gather(prof, kExport, D.Ap, D.exp_off, P->colptrL.back(), d_sel, s);
    return e;
}

// The inverse panels from the checkpoint store (checkpointed levels) and by
// recomputation (the other levels, root first, each from its ancestors).
hipError_t rebuild_inverse(selinv_plan_s* P, const DevPtrs& D, hipStream_t s, Prof* prof)
{
    hipError_t e = launch_checkpoint(prof, D, (int64_t)P->t_diag.tasks.size(), 1, s);
    const int k = P->opts.checkpoint_every;
    for (int l = 0; l < P->exec.depth && !e; l++) {
        if (l % k == 0) continue;
        const int64_t z0 = P->t_zero_off[l], z1 = P->t_zero_off[l + 1];
        e = launch_zero_x(prof, D, z0, z1 - z0, s);
        if (!e) e = invert_level(P, D, l, s, prof);
    }
    return e;
}
}  // namespace selinv

selinv_plan_s::~selinv_plan_s()
{
    drop_graph(this);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

extern "C" {

selinv_status selinv_analyze(int64_t n, const int64_t* colptr, const int32_t* rowind, const selinv_geom* geom,
                             const int32_t* perm_or_null, const selinv_opts* opts, selinv_plan* out)
{
    if (!out) return fail(SELINV_EINVAL, "out is NULL");
    *out = nullptr;
    selinv_opts o;
    if (selinv_status st = resolve_opts(opts, o)) return st;
    selinv_plan_s* P = new (std::nothrow) selinv_plan_s();
    if (!P) return fail(SELINV_ENOMEM, "out of host memory");
    try {
        std::string err;
        selinv_status st = analyze_one(n, colptr, rowind, geom, perm_or_null, o, P, err);
        if (st != SELINV_OK) {
            delete P;
            return fail(st, err);
        }
        finish_plan(P);
    } catch (const std::bad_alloc&) {
        delete P;
        return fail(SELINV_ENOMEM, "out of host memory during analysis");
    }
    *out = P;
    return SELINV_OK;
}

selinv_status selinv_analyze_batch(int32_t count, const int64_t* ns, const int64_t* const* colptrs,
                                   const int32_t* const* rowinds, const selinv_geom* geoms, const selinv_opts* opts,
                                   selinv_plan* out)
{
    if (!out) return fail(SELINV_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 0) return fail(SELINV_EINVAL, "count must be >= 0");
    if (count > 0 && (!ns || !colptrs || !rowinds)) return fail(SELINV_EINVAL, "ns/colptrs/rowinds is NULL");
    selinv_opts o;
    if (selinv_status st = resolve_opts(opts, o)) return st;
    int64_t total = 0;
    for (int32_t m = 0; m < count; m++) {
        if (ns[m] < 0) return fail(SELINV_EINVAL, "matrix " + std::to_string(m) + ": n out of range");
        total += ns[m];
    }
    if (total > INT32_MAX - 1) return fail(SELINV_EINVAL, "batch too large: total order exceeds 2^31 - 2");
    std::vector<selinv_plan_s*> parts;
    selinv_plan_s* U = nullptr;
    auto cleanup = [&]() {
        for (selinv_plan_s* p : parts) delete p;
        parts.clear();
    };
    try {
        for (int32_t m = 0; m < count; m++) {
            selinv_plan_s* P = new selinv_plan_s();
            parts.push_back(P);
            std::string err;
            selinv_status st = analyze_one(ns[m], colptrs[m], rowinds[m], geoms ? geoms + m : nullptr, nullptr, o,
                                           P, err);
            if (st != SELINV_OK) {
                cleanup();
                return fail(st, "matrix " + std::to_string(m) + ": " + err);
            }
        }
        U = new selinv_plan_s();
        U->opts = o;
        merge_plans(parts, U);
        cleanup();
        finish_plan(U);
    } catch (const std::bad_alloc&) {
        cleanup();
        delete U;
        return fail(SELINV_ENOMEM, "out of host memory during batch analysis");
    }
    *out = U;
    return SELINV_OK;
}

selinv_status selinv_analyze_poles(int64_t n, const int64_t* colptr, const int32_t* rowind, const selinv_geom* geom,
                                   const int32_t* perm_or_null, const selinv_opts* opts, int32_t count,
                                   selinv_plan* out)
{
    if (!out) return fail(SELINV_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1) return fail(SELINV_EINVAL, "count must be >= 1");
    if ((int64_t)count * n > INT32_MAX - 1) return fail(SELINV_EINVAL, "batch too large: total order exceeds 2^31 - 2");
    selinv_opts o;
    if (selinv_status st = resolve_opts(opts, o)) return st;
    selinv_plan_s* one = new (std::nothrow) selinv_plan_s();
    if (!one) return fail(SELINV_ENOMEM, "out of host memory");
    selinv_plan_s* U = nullptr;
    try {
        std::string err;
        selinv_status st = analyze_one(n, colptr, rowind, geom, perm_or_null, o, one, err);
        if (st != SELINV_OK) {
            delete one;
            return fail(st, err);
        }
        // the one analysis, repeated: the union reads its parts only
        std::vector<selinv_plan_s*> parts((size_t)count, one);
        U = new selinv_plan_s();
        U->opts = o;
        merge_plans(parts, U);
        delete one;
        one = nullptr;
        finish_plan(U);
    } catch (const std::bad_alloc&) {
        delete one;
        delete U;
        return fail(SELINV_ENOMEM, "out of host memory during analysis");
    }
    *out = U;
    return SELINV_OK;
}

selinv_status selinv_batch_offsets(selinv_plan P, int32_t* count, int64_t* n_off, int64_t* nnzA_off,
                                   int64_t* nnzL_off)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (count) *count = (int32_t)P->b_noff.size() - 1;
    if (n_off) std::copy(P->b_noff.begin(), P->b_noff.end(), n_off);
    if (nnzA_off) std::copy(P->b_aoff.begin(), P->b_aoff.end(), nnzA_off);
    if (nnzL_off) std::copy(P->b_loff.begin(), P->b_loff.end(), nnzL_off);
    return SELINV_OK;
}

selinv_status selinv_workspace_size(selinv_plan P, size_t* bytes)
{
    if (!P || !bytes) return fail(SELINV_EINVAL, "NULL argument");
    *bytes = P->lay.total;
    return SELINV_OK;
}

selinv_status selinv_workspace_sizes(selinv_plan P, size_t* persistent, size_t* transient)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (persistent) *persistent = P->lay.persist;
    if (transient) *transient = P->lay.transient;
    return SELINV_OK;
}

selinv_status selinv_bind_transient(selinv_plan P, void* d_tr, size_t bytes)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (d_tr) {
        if (bytes < P->lay.transient) return fail(SELINV_ENOMEM, "transient buffer too small");
        if (((uintptr_t)d_tr & 255) != 0) return fail(SELINV_EINVAL, "transient buffer must be 256-byte aligned");
    }
    drop_graph(P);
    if (d_tr) {
        P->tr = (char*)d_tr;
        P->tr_separate = true;
    } else {
        P->tr = (P->ws && P->ws_bytes >= P->lay.total) ? P->ws + P->lay.persist : nullptr;
        P->tr_separate = false;
    }
    P->ap_valid = false;
    return SELINV_OK;
}

selinv_status selinv_generation(selinv_plan P, uint64_t* gen)
{
    if (!P || !gen) return fail(SELINV_EINVAL, "NULL argument");
    *gen = P->generation;
    return SELINV_OK;
}

selinv_status selinv_bind_workspace(selinv_plan P, void* d_ws, size_t bytes, hipStream_t s)
{
    if (!P || !d_ws) return fail(SELINV_EINVAL, "NULL argument");
    if (bytes < P->lay.persist) return fail(SELINV_ENOMEM, "workspace too small");
    if (((uintptr_t)d_ws & 255) != 0) return fail(SELINV_EINVAL, "workspace must be 256-byte aligned");
    drop_graph(P);
    P->ws = (char*)d_ws;
    P->ws_bytes = bytes;
    P->tr = bytes >= P->lay.total ? P->ws + P->lay.persist : nullptr;
    P->tr_separate = false;
    P->factored = false;
    P->inverted = false;
    P->ap_valid = false;
    P->queues_on_device = false;
    const hipError_t init = kernels_init();
    if (init != hipSuccess) return hip_fail(init, "kernel attributes");
    hipError_t e = hipSuccess;
    int dev = 0;
    hipDeviceProp_t prop;
    if (!e) e = hipGetDevice(&dev);
    if (!e) e = hipGetDeviceProperties(&prop, dev);
    if (!e) e = persist_occupancy(P->occ);
    if (e) {
        P->ws = nullptr;
        return hip_fail(e, "device query");
    }
    P->n_cu = prop.multiProcessorCount;
    P->dev_arch = prop.gcnArchName;
    if (!e) e = upload_tables(P, P->ws, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) {
        P->ws = nullptr;
        return hip_fail(e, "bind_workspace upload");
    }
    P->queues_on_device = true;
    return SELINV_OK;
}

selinv_status selinv_factor(selinv_plan P, const double* d_valsA, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (P->opts.complex_values) return fail(SELINV_EINVAL, "the plan holds complex values (selinv_*_complex)");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (P->nnzA > 0 && !d_valsA) return fail(SELINV_EINVAL, "d_valsA is NULL");
    P->generation++;
    P->factored = false;
    P->inverted = false;
    P->ap_valid = false;
    hipError_t e = factor_levels(P, dev_ptrs(P), d_valsA, s, &P->prof);
    if (e) return hip_fail(e, "factor launch");
    P->factored = true;
    return SELINV_OK;
}

selinv_status selinv_backward(selinv_plan P, const double* d_gsel, double* d_gA, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (P->opts.complex_values) return fail(SELINV_EINVAL, "the plan holds complex values (selinv_*_complex)");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (!P->inverted) return fail(SELINV_ESTATE, "backward needs factor and invert of the same values first");
    if (!P->tr) return fail(SELINV_ESTATE, "no transient memory bound (selinv_bind_transient)");
    const bool rebuild = P->opts.checkpoint_every > 1;
    if (!rebuild && !P->ap_valid)
        return fail(SELINV_ESTATE, "the inverse panels were released and checkpoint_every is 1: invert again");
    if ((P->colptrL.back() > 0 && !d_gsel) || (P->nnzA > 0 && !d_gA)) return fail(SELINV_EINVAL, "NULL buffer");
    for (const BlockDesc& d : P->blocks)
        if (d.s > kLdsDiagMax)
            return fail(SELINV_EUNSUPPORTED, "backward supports execution blocks of at most 128 columns");
    DevPtrs D = dev_ptrs(P);
    hipError_t e = hipSuccess;
    // checkpointed levels restored, the others recomputed root first: every
    // level's gathers read all of its ancestors' panels
    if (rebuild) e = rebuild_inverse(P, D, s, &P->prof);
    if (e) return hip_fail(e, "inverse rebuild");
    P->ap_valid = true;
    e = launch_backward_init(&P->prof, D, P->arena, P->harena, d_gsel, P->colptrL.back(), s);
    if (e) return hip_fail(e, "backward setup");
    const int depth = P->exec.depth;
    // reverse selected inversion: leaves first
    for (int l = depth - 1; l >= 0; l--) {
        const auto& a = P->t_rs1.off;
        const auto& b = P->t_rs2.off;
        const auto& cut = P->rs3_cuts[l];
        e = launch_revsel_level(&P->prof, D, a[l], a[l + 1] - a[l], b[l], b[l + 1] - b[l], cut.data(), (int)cut.size(),
                                s);
        if (e) return hip_fail(e, "reverse inversion launch");
    }
    e = launch_revfac_init(&P->prof, D, (int64_t)P->t_diag.tasks.size(), P->arena, s);
    if (e) return hip_fail(e, "reverse factor setup");
    // reverse factorization: root first
    for (int l = 0; l < depth; l++) {
        const auto& a = P->t_rf1a.off;
        const auto& b = P->t_rf1b.off;
        const auto& c = P->t_rf2.off;
        const auto& d = P->t_diag.off;
        e = launch_revfac_level(&P->prof, D, a[l], a[l + 1] - a[l], b[l], b[l + 1] - b[l], c[l], c[l + 1] - c[l],
                                d[l], d[l + 1] - d[l], s);
        if (e) return hip_fail(e, "reverse factor launch");
    }
    e = launch_gather(&P->prof, kRevFac, D.Zb, D.asm_off, P->nnzA, d_gA, s);
    if (e) return hip_fail(e, "gradient export");
    return SELINV_OK;
}

selinv_status selinv_invert(selinv_plan P, double* d_sel, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (P->opts.complex_values) return fail(SELINV_EINVAL, "the plan holds complex values (selinv_*_complex)");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (!P->factored) return fail(SELINV_ESTATE, "invert called before factor");
    if (!P->tr) return fail(SELINV_ESTATE, "no transient memory bound (selinv_bind_transient)");
    if (P->colptrL.back() > 0 && !d_sel) return fail(SELINV_EINVAL, "d_sel is NULL");
    DevPtrs D = dev_ptrs(P);
    hipError_t e = invert_levels(P, D, d_sel, s, &P->prof);
    if (!e && P->opts.checkpoint_every > 1) e = launch_checkpoint(&P->prof, D, (int64_t)P->t_diag.tasks.size(), 0, s);
    if (e) return hip_fail(e, "invert launch");
    P->inverted = true;
    P->ap_valid = true;
    return SELINV_OK;
}

selinv_status selinv_factor_complex(selinv_plan P, const double* d_valsA, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (!P->opts.complex_values) return fail(SELINV_EINVAL, "the plan holds real values (analyse with complex_values)");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (P->nnzA > 0 && !d_valsA) return fail(SELINV_EINVAL, "d_valsA is NULL");
    P->generation++;
    P->factored = P->inverted = P->ap_valid = false;
    const DevPtrs D = dev_ptrs(P);
    hipError_t e = launch_status_reset(D.status, s);
    if (!e) e = launch_fill(nullptr, kAssemble, D.Lp, 2 * P->arena, 0.0, s);
    if (!e) e = launch_zassemble(d_valsA, D.asm_off, P->nnzA, D.Lp, s);
    for (int l = P->exec.depth - 1; l >= 0 && !e; l--) {
        const auto& a = P->t_ldlt.off;
        const auto& b = P->t_panel.off;
        const auto& cut = P->schur_cuts[l];
        e = launch_zfactor_level(D, a[l], a[l + 1] - a[l], b[l], b[l + 1] - b[l], cut.data(), (int)cut.size(), s);
    }
    if (e) return hip_fail(e, "complex factor launch");
    P->factored = true;
    return SELINV_OK;
}

selinv_status selinv_invert_complex(selinv_plan P, double* d_sel, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (!P->opts.complex_values) return fail(SELINV_EINVAL, "the plan holds real values (analyse with complex_values)");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (!P->factored) return fail(SELINV_ESTATE, "invert called before factor");
    if (!P->tr) return fail(SELINV_ESTATE, "no transient memory bound (selinv_bind_transient)");
    if (P->colptrL.back() > 0 && !d_sel) return fail(SELINV_EINVAL, "d_sel is NULL");
    const DevPtrs D = dev_ptrs(P);
    hipError_t e = hipSuccess;
    for (int l = 0; l < P->exec.depth && !e; l++) {
        const auto& g = P->t_gemm.off;
        const auto& d = P->t_sdiag.off;
        const int64_t gc[4] = {g[l], P->zgemm_mid[l], P->zgemm_cut[l], g[l + 1]};
        e = launch_zinvert_level(D, gc, d[l], P->sdiag_cut[l], d[l + 1], s);
    }
    if (!e) e = launch_zexport(D.Ap, D.exp_off, P->colptrL.back(), d_sel, s);
    if (e) return hip_fail(e, "complex invert launch");
    P->inverted = true;
    P->ap_valid = true;
    return SELINV_OK;
}

selinv_status selinv_get_factor(selinv_plan P, double* d_L, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (P->opts.complex_values) return fail(SELINV_EINVAL, "the plan holds complex values (selinv_*_complex)");
    if (P->opts.pivoting) return fail(SELINV_EUNSUPPORTED, "with pivoting the diagonal blocks keep T only: no factor");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (!P->factored) return fail(SELINV_ESTATE, "no factor computed");
    DevPtrs D = dev_ptrs(P);
    hipError_t e = launch_export_L(&P->prof, D, P->n, d_L, s);
    if (e) return hip_fail(e, "export launch");
    return SELINV_OK;
}

selinv_status selinv_sync_status(selinv_plan P, hipStream_t s, int64_t* bad_col)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (bad_col) *bad_col = -1;
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    unsigned long long w[2] = {~0ull, 0ull};
    hipError_t e = hipMemcpyAsync(w, P->ws + P->lay.status, sizeof w, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return hip_fail(e, "sync_status");
    if (w[1] != 0)
        return fail(SELINV_EQUEUE, "a work-queue dependency wait exceeded its poll limit; results are invalid");
    const unsigned long long v = w[0];
    if (v != ~0ull) {
        int64_t col = (int64_t)v;
        int64_t orig = (col >= 0 && col < P->n) ? P->perm[col] : -1;
        if (bad_col) *bad_col = orig;
        return fail(SELINV_EPIVOT, "bad pivot at original column " + std::to_string(orig));
    }
    return SELINV_OK;
}

selinv_status selinv_get_info(selinv_plan P, selinv_info* out)
{
    if (!P || !out) return fail(SELINV_EINVAL, "NULL argument");
    *out = P->info;
    return SELINV_OK;
}

selinv_status selinv_get_pattern(selinv_plan P, int64_t* colptrL, int32_t* rowindL, int32_t* perm)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (colptrL) std::copy(P->colptrL.begin(), P->colptrL.end(), colptrL);
    if (rowindL) std::copy(P->rowindL.begin(), P->rowindL.end(), rowindL);
    if (perm) std::copy(P->perm.begin(), P->perm.end(), perm);
    return SELINV_OK;
}

selinv_status selinv_symbolic_sizes(selinv_plan P, int64_t* nsuper, int64_t* ncrows, int64_t* nrel)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    const Partition& F = P->fund;
    if (nsuper) *nsuper = F.nblocks();
    if (ncrows) *ncrows = (int64_t)F.crows.size();
    if (nrel) {
        std::vector<int64_t> rptr;
        std::vector<int32_t> rel;
        block_index_maps(F, rptr, rel);
        *nrel = (int64_t)rel.size();
    }
    return SELINV_OK;
}

selinv_status selinv_get_symbolic(selinv_plan P, int32_t* parent, int32_t* xsuper, int32_t* sparent, int32_t* level,
                                  int64_t* cptr, int32_t* crows, int64_t* rptr, int32_t* rel)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    const Partition& F = P->fund;
    if (parent) std::copy(P->parent.begin(), P->parent.end(), parent);
    if (xsuper) std::copy(F.xs.begin(), F.xs.end(), xsuper);
    if (sparent) std::copy(F.par.begin(), F.par.end(), sparent);
    if (level) std::copy(F.lev.begin(), F.lev.end(), level);
    if (cptr) std::copy(F.cptr.begin(), F.cptr.end(), cptr);
    if (crows) std::copy(F.crows.begin(), F.crows.end(), crows);
    if (rptr || rel) {
        std::vector<int64_t> rp;
        std::vector<int32_t> rl;
        block_index_maps(F, rp, rl);
        if (rptr) std::copy(rp.begin(), rp.end(), rptr);
        if (rel) std::copy(rl.begin(), rl.end(), rel);
    }
    return SELINV_OK;
}

selinv_status selinv_profile(selinv_plan P, int32_t enable)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    P->prof.on = enable != 0;
    return SELINV_OK;
}

selinv_status selinv_profile_read(selinv_plan P, double* ms, int64_t* launches)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    Prof& R = P->prof;
    for (int k = 0; k < kNumKinds; k++) {
        if (ms) ms[k] = 0.0;
        if (launches) launches[k] = 0;
    }
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < R.kinds.size() && !e; i++) {
        e = hipEventSynchronize(R.pool[2 * i + 1]);
        float t = 0.f;
        if (!e) e = hipEventElapsedTime(&t, R.pool[2 * i], R.pool[2 * i + 1]);
        if (!e) {
            if (ms) ms[R.kinds[i]] += t;
            if (launches) launches[R.kinds[i]] += 1;
        }
    }
    R.kinds.clear();
    R.used = 0;
    if (e) return hip_fail(e, "profile_read");
    return SELINV_OK;
}

selinv_status selinv_kernel_work(selinv_plan P, double* flops, double* bytes)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    for (int k = 0; k < kNumKinds; k++) {
        if (flops) flops[k] = P->work_flops[k];
        if (bytes) bytes[k] = P->work_bytes[k];
    }
    return SELINV_OK;
}

selinv_status selinv_get_arena(selinv_plan P, int32_t which, double* d_out, int64_t* count, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    size_t off;
    int64_t n;
    bool transient = false;
    switch (which) {
        case 0: off = P->lay.lp; n = P->arena; break;
        case 1: off = P->lay.ap; n = P->arena; transient = true; break;
        case 2: off = P->lay.hp; n = P->harena; break;
        case 3: off = P->lay.wp; n = P->warena; break;
        case 4: off = P->lay.tp; n = P->warena; break;
        case 5: off = P->lay.zb; n = P->arena; transient = true; break;
        case 6: off = P->lay.hb; n = P->harena; transient = true; break;
        case 7: off = P->lay.tb; n = P->warena; transient = true; break;
        default: return fail(SELINV_EINVAL, "unknown arena");
    }
    if (P->opts.complex_values) {
        // (re, im) pairs; a complex plan has no adjoint arenas
        if (which >= 5) return fail(SELINV_EINVAL, "a complex plan has no adjoint arenas");
        n *= 2;
    }
    if (count) *count = n;
    if (!d_out || n == 0) return SELINV_OK;
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    char* base = transient ? P->tr : P->ws;
    if (!base) return fail(SELINV_ESTATE, "no transient memory bound");
    hipError_t e = hipMemcpyAsync(d_out, base + off, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
    if (e) return hip_fail(e, "get_arena");
    return SELINV_OK;
}

selinv_status selinv_get_blocks(selinv_plan P, int32_t* first, int32_t* s, int32_t* c, int32_t* level,
                                int64_t* poff, int64_t* hoff, int64_t* woff, int64_t* crow_off)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    for (size_t b = 0; b < P->blocks.size(); b++) {
        const BlockDesc& d = P->blocks[b];
        if (first) first[b] = d.first;
        if (s) s[b] = d.s;
        if (c) c[b] = d.c;
        if (level) level[b] = d.level;
        if (poff) poff[b] = d.poff;
        if (hoff) hoff[b] = d.hoff;
        if (woff) woff[b] = d.woff;
        if (crow_off) crow_off[b] = d.coff;
    }
    return SELINV_OK;
}

selinv_status selinv_get_exec_rows(selinv_plan P, int32_t* rows)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (rows) std::copy(P->crow.begin(), P->crow.end(), rows);
    return SELINV_OK;
}

}  // extern "C"

namespace {
// One factor + inversion on the persistent kernels: assemble, one launch per
// level of the factor (leaves first) and of the inversion (root first),
// export.  Kernels only (fill kernels clear memory), so the sequence can be
// captured into a graph.
selinv_status run_persistent(selinv_plan_s* P, const double* d_valsA, double* d_sel, hipStream_t s, Prof* prof)
{
    DevPtrs D = dev_ptrs(P);
    const int64_t nb = (int64_t)P->blocks.size();
    const int depth = P->exec.depth;
    unsigned* done_f = (unsigned*)(P->ws + P->lay.q_done);
    unsigned* done_i = done_f + nb;
    unsigned* head_f = (unsigned*)(P->ws + P->lay.q_head);
    unsigned* head_i = head_f + depth;
    const Task* qf = (const Task*)(P->ws + P->lay.q_fac);
    const Task* qi = (const Task*)(P->ws + P->lay.q_inv);
    auto grid = [&](int variant) {
        // light (wave-granular) levels fill the occupancy; tiled levels take
        // grid_mult work-groups per CU, capped by it
        const int occ = std::max(1, P->occ[variant]);
        const bool light = variant == kLightFactor || variant == kLightInvert;
        return P->n_cu * (light ? occ : std::min(P->sched.grid_mult, occ));
    };
    hipError_t e = launch_status_reset(D.status, s);
    if (!e) e = launch_fill(prof, kAssemble, D.Lp, P->arena, 0.0, s);
    if (!e) e = launch_scatter_set(prof, kAssemble, d_valsA, D.asm_off, P->nnzA, D.Lp, s);
    if (!e) e = launch_fill_u32(prof, kAssemble, done_f, 2 * (nb + depth), s);
    for (int l = depth - 1; l >= 0 && !e; l--) {
        const int64_t a = P->q_fac_off[l], z = P->q_fac_off[l + 1];
        const int var = P->q_var_fac[l];
        e = launch_persist_factor(prof, D, qf + a, z - a, head_f + l, done_f, grid(var), var, P->opts.require_spd,
                                  P->spin_limit, s);
    }
    for (int l = 0; l < depth && !e; l++) {
        const int64_t a = P->q_inv_off[l], z = P->q_inv_off[l + 1];
        const int var = P->q_var_inv[l];
        e = launch_persist_invert(prof, D, qi + a, z - a, head_i + l, done_i, grid(var), var, P->spin_limit, s);
    }
    if (!e) e = launch_gather(prof, kExport, D.Ap, D.exp_off, P->colptrL.back(), d_sel, s);
    if (e) return hip_fail(e, "persistent launch");
    return SELINV_OK;
}

// What selinv_run launches: the persistent kernels, or in deterministic
// mode (no atomics) and with pivoting (the pivoted diagonal kernel) the
// per-level sequence, followed by the checkpoint copy when checkpointing is
// on.  Kernels only, so it can be captured.
selinv_status run_sequence(selinv_plan_s* P, const double* d_valsA, double* d_sel, hipStream_t s, Prof* prof)
{
    if (!P->opts.deterministic && !P->opts.pivoting) {
        if (selinv_status st = run_persistent(P, d_valsA, d_sel, s, prof)) return st;
    } else {
        const DevPtrs D = dev_ptrs(P);
        hipError_t e = factor_levels(P, D, d_valsA, s, prof);
        if (!e) e = invert_levels(P, D, d_sel, s, prof);
        if (e) return hip_fail(e, "per-level run launch");
    }
    if (P->opts.checkpoint_every > 1) {
        hipError_t e = launch_checkpoint(prof, dev_ptrs(P), (int64_t)P->t_diag.tasks.size(), 0, s);
        if (e) return hip_fail(e, "checkpoint launch");
    }
    return SELINV_OK;
}

selinv_status check_sched(const selinv_sched* sc)
{
    if (!sc) return fail(SELINV_EINVAL, "NULL schedule");
    if (sc->order < 0 || sc->order >= qoNumOrders) return fail(SELINV_EINVAL, "schedule order out of range");
    if (sc->bn_cap != 16 && sc->bn_cap != 32 && sc->bn_cap != 64 && sc->bn_cap != 128)
        return fail(SELINV_EINVAL, "bn_cap must be 16, 32, 64 or 128");
    if (sc->split_fill < 0 || sc->split_fill > 4096) return fail(SELINV_EINVAL, "split_fill must be 0..4096");
    if (sc->grid_mult < 1 || sc->grid_mult > 16) return fail(SELINV_EINVAL, "grid_mult must be 1..16");
    if (std::find(std::begin(kSmallValues), std::end(kSmallValues), sc->small_s) == std::end(kSmallValues))
        return fail(SELINV_EINVAL, "small_s must be 0, 1, 2, 4, 8 or 16");
    if (sc->mb_tiles < 0 || sc->mb_tiles > 4096) return fail(SELINV_EINVAL, "mb_tiles must be 0..4096");
    return SELINV_OK;
}

// 64-bit FNV-1a over the block structure: the autotuner cache key
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(uint64_t v)
    {
        for (int b = 0; b < 8; b++) {
            h ^= (v >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    }
};

std::string tune_key(const selinv_plan_s* P)
{
    Fnv f;
    f.add((uint64_t)P->n);
    f.add((uint64_t)P->colptrL.back());
    f.add((uint64_t)P->blocks.size());
    f.add((uint64_t)P->exec.depth);
    f.add((uint64_t)P->opts.require_spd);
    for (const BlockDesc& d : P->blocks) {
        f.add((uint64_t)d.s);
        f.add((uint64_t)d.c);
        f.add((uint64_t)d.level);
    }
    char buf[64];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)f.h);
    return "selinv/" + P->dev_arch + "/" + std::to_string(P->n_cu) + "cu/" + buf;
}

// Cache file: a JSON object with one entry per line,
//   "key": {"order": 1, "bn_cap": 128, "split_fill": 512, "grid_mult": 2, "small_s": 16, "mb_tiles": 8,
//           "ms": 1.5},   (one line per entry)
bool cache_lookup(const char* path, const std::string& key, selinv_sched& sc, double& ms)
{
    std::ifstream in(path);
    if (!in) return false;
    std::string line;
    const std::string tag = "\"" + key + "\":";
    while (std::getline(in, line)) {
        const size_t at = line.find(tag);
        if (at == std::string::npos) continue;
        auto num = [&](const char* name, double& v) {
            const std::string f = std::string("\"") + name + "\":";
            const size_t q = line.find(f, at + tag.size());
            if (q == std::string::npos) return false;
            v = std::strtod(line.c_str() + q + f.size(), nullptr);
            return true;
        };
        double o, b, fl, g, sm, mb;
        if (!num("order", o) || !num("bn_cap", b) || !num("split_fill", fl) || !num("grid_mult", g) ||
            !num("small_s", sm) || !num("mb_tiles", mb))
            return false;
        if (!num("ms", ms)) ms = 0.0;
        sc = selinv_sched{(int32_t)o, (int32_t)b, (int32_t)fl, (int32_t)g, (int32_t)sm, (int32_t)mb};
        return check_sched(&sc) == SELINV_OK;
    }
    return false;
}

bool cache_store(const char* path, const std::string& key, const selinv_sched& sc, double ms)
{
    std::vector<std::string> keep;
    {
        std::ifstream in(path);
        std::string line;
        const std::string tag = "\"" + key + "\":";
        while (in && std::getline(in, line)) {
            if (line.find("\": {") == std::string::npos || line.find(tag) != std::string::npos) continue;
            while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
            keep.push_back(line);
        }
    }
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "  \"%s\": {\"order\": %d, \"bn_cap\": %d, \"split_fill\": %d, \"grid_mult\": %d, "
                  "\"small_s\": %d, \"mb_tiles\": %d, \"ms\": %.6f}",
                  key.c_str(), sc.order, sc.bn_cap, sc.split_fill, sc.grid_mult, sc.small_s, sc.mb_tiles, ms);
    keep.push_back(buf);
    std::ofstream out(path, std::ios::trunc);
    if (!out) return false;
    out << "{\n";
    for (size_t i = 0; i < keep.size(); i++) out << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
    out << "}\n";
    return (bool)out;
}
}  // namespace

extern "C" {

selinv_status selinv_set_schedule(selinv_plan P, const selinv_sched* sc, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (selinv_status st = check_sched(sc)) return st;
    Sched next{sc->order, sc->bn_cap, sc->split_fill, sc->grid_mult, sc->small_s, sc->mb_tiles};
    std::vector<Task> qf, qi;
    std::vector<int64_t> of, oi;
    try {
        build_queues(P, next, qf, of, qi, oi);
    } catch (const std::bad_alloc&) {
        return fail(SELINV_ENOMEM, "out of host memory building the queues");
    }
    if ((int64_t)qf.size() > P->q_cap_fac || (int64_t)qi.size() > P->q_cap_inv)
        return fail(SELINV_EINVAL, "internal: queue longer than its bound");
    if (P->ws) {
        hipError_t e = upload(P->ws, P->lay.q_fac, qf, s);
        if (!e) e = upload(P->ws, P->lay.q_inv, qi, s);
        if (!e) e = hipStreamSynchronize(s);
        if (e) {
            P->queues_on_device = false;
            return hip_fail(e, "queue upload");
        }
    }
    drop_graph(P);
    P->sched = next;
    P->q_fac.swap(qf);
    P->q_inv.swap(qi);
    P->q_fac_off.swap(of);
    P->q_inv_off.swap(oi);
    level_variants(P, P->q_fac, P->q_fac_off, true, P->q_var_fac);
    level_variants(P, P->q_inv, P->q_inv_off, false, P->q_var_inv);
    return SELINV_OK;
}

selinv_status selinv_get_schedule(selinv_plan P, selinv_sched* sc)
{
    if (!P || !sc) return fail(SELINV_EINVAL, "NULL argument");
    *sc = selinv_sched{P->sched.order,     P->sched.bn_cap,  P->sched.split_fill,
                       P->sched.grid_mult, P->sched.small_s, P->sched.mb_tiles};
    return SELINV_OK;
}

selinv_status selinv_get_queue(selinv_plan P, int32_t sweep, int32_t level, int32_t* tasks, int64_t* count)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (sweep != 0 && sweep != 1) return fail(SELINV_EINVAL, "sweep must be 0 (factor) or 1 (inversion)");
    if (level < 1 || level > P->exec.depth) return fail(SELINV_EINVAL, "level out of range");
    const std::vector<Task>& q = sweep == 0 ? P->q_fac : P->q_inv;
    const std::vector<int64_t>& off = sweep == 0 ? P->q_fac_off : P->q_inv_off;
    const int64_t a = off[level - 1], z = off[level];
    if (count) *count = z - a;
    if (tasks) std::memcpy(tasks, q.data() + a, sizeof(Task) * (size_t)(z - a));
    return SELINV_OK;
}

selinv_status selinv_set_spin_limit(selinv_plan P, uint32_t polls)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    P->spin_limit = polls;
    drop_graph(P);
    return SELINV_OK;
}

selinv_status selinv_run(selinv_plan P, const double* d_valsA, double* d_sel, int32_t use_graph, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (P->opts.complex_values) return fail(SELINV_EINVAL, "the plan holds complex values (selinv_*_complex)");
    if (!P->ws || !P->queues_on_device) return fail(SELINV_ESTATE, "no workspace bound");
    if (!P->tr) return fail(SELINV_ESTATE, "no transient memory bound (selinv_bind_transient)");
    if ((P->nnzA > 0 && !d_valsA) || (P->colptrL.back() > 0 && !d_sel)) return fail(SELINV_EINVAL, "NULL buffer");
    P->generation++;
    P->factored = P->inverted = P->ap_valid = false;
    if (!use_graph) {
        if (selinv_status st = run_sequence(P, d_valsA, d_sel, s, &P->prof)) return st;
    } else {
        if (!P->graph_exec || P->graph_in != (const void*)d_valsA || P->graph_out != (void*)d_sel) {
            drop_graph(P);
            hipError_t e = hipSuccess;
            if (!P->cap_stream) e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
            if (e) return hip_fail(e, "capture stream");
            e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e) return hip_fail(e, "begin capture");
            selinv_status st = run_sequence(P, d_valsA, d_sel, P->cap_stream, nullptr);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(P->cap_stream, &g);
            if (st != SELINV_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e) return hip_fail(e, "end capture");
            P->graph = g;
            e = hipGraphInstantiate(&P->graph_exec, g, nullptr, nullptr, 0);
            if (e) {
                drop_graph(P);
                return hip_fail(e, "graph instantiate");
            }
            P->graph_in = d_valsA;
            P->graph_out = d_sel;
        }
        hipError_t e = hipGraphLaunch(P->graph_exec, s);
        if (e) return hip_fail(e, "graph launch");
    }
    P->factored = true;
    P->inverted = true;
    P->ap_valid = true;
    return SELINV_OK;
}

selinv_status selinv_tune(selinv_plan P, const double* d_valsA, double* d_sel, const char* cache_path,
                          selinv_sched* chosen, double* best_ms, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (P->opts.complex_values) return fail(SELINV_EINVAL, "the plan holds complex values (selinv_*_complex)");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (!P->tr) return fail(SELINV_ESTATE, "no transient memory bound (selinv_bind_transient)");
    if (P->opts.deterministic || P->opts.pivoting)
        return fail(SELINV_EUNSUPPORTED, "deterministic and pivoting plans run per-level launches: no schedule to tune");
    const std::string key = tune_key(P);
    selinv_sched best{};
    double ms = 0.0;
    if (cache_path && cache_lookup(cache_path, key, best, ms)) {
        if (selinv_status st = selinv_set_schedule(P, &best, s)) return st;
        if (chosen) *chosen = best;
        if (best_ms) *best_ms = ms;
        return SELINV_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (!he) he = hipEventCreate(&e1);
    if (he) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(he, "tune events");
    }
    const bool prof_was = P->prof.on;
    P->prof.on = false;
    // time one schedule: a warm-up run, then the best of three
    auto evaluate = [&](const selinv_sched& sc, double& t) -> selinv_status {
        if (selinv_status st = selinv_set_schedule(P, &sc, s)) return st;
        if (selinv_status st = run_persistent(P, d_valsA, d_sel, s, nullptr)) return st;
        t = 1e30;
        for (int r = 0; r < 3; r++) {
            hipError_t e = hipEventRecord(e0, s);
            if (e) return hip_fail(e, "tune timing");
            if (selinv_status st = run_persistent(P, d_valsA, d_sel, s, nullptr)) return st;
            e = hipEventRecord(e1, s);
            if (!e) e = hipEventSynchronize(e1);
            float dt = 0.f;
            if (!e) e = hipEventElapsedTime(&dt, e0, e1);
            if (e) return hip_fail(e, "tune timing");
            t = std::min(t, (double)dt);
        }
        int64_t bad = -1;
        return selinv_sync_status(P, s, &bad);
    };
    // coordinate descent over small-block width, medium-block size, queue
    // order, tile cap, split fill, grid size
    best = selinv_sched{P->sched.order,     P->sched.bn_cap,  P->sched.split_fill,
                        P->sched.grid_mult, P->sched.small_s, P->sched.mb_tiles};
    const selinv_sched start = best;
    double tbest = 0.0;
    selinv_status st = evaluate(best, tbest);
    for (int dim = 0; dim < 6 && st == SELINV_OK; dim++) {
        const int32_t* axes[] = {kTuneSmall, kTuneMb, kTuneOrders, kTuneBn, kTuneFill, kTuneGrid};
        const int32_t* vals = axes[dim];
        const int nv = dim == 2 ? 4 : 3;
        for (int v = 0; v < nv && st == SELINV_OK; v++) {
            selinv_sched c = best;
            int32_t* fields[] = {&c.small_s, &c.mb_tiles, &c.order, &c.bn_cap, &c.split_fill, &c.grid_mult};
            int32_t* field = fields[dim];
            if (*field == vals[v]) continue;
            *field = vals[v];
            double t = 0.0;
            st = evaluate(c, t);
            if (st == SELINV_OK && t < tbest) {
                tbest = t;
                best = c;
            }
        }
    }
    // every exit: events freed, timing flag restored, and the plan left on
    // the best schedule found (the starting one if none was timed)
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->prof.on = prof_was;
    if (st != SELINV_OK) {
        const std::string msg = g_err;
        const selinv_sched keep = tbest > 0.0 ? best : start;
        (void)selinv_set_schedule(P, &keep, s);
        g_err = msg;
        return st;
    }
    if ((st = selinv_set_schedule(P, &best, s))) return st;
    if (cache_path && !cache_store(cache_path, key, best, tbest))
        return fail(SELINV_EINVAL, std::string("cannot write the tuning cache ") + cache_path);
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = tbest;
    return SELINV_OK;
}

void selinv_destroy(selinv_plan P) { delete P; }

}  // extern "C"
