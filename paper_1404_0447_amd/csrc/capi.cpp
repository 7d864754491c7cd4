// C ABI of the selected-inversion library (declared in include/selinv.h).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
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
    L.lp = take(sizeof(double) * P->arena);
    L.ap = take(sizeof(double) * P->arena);
    L.hp = take(sizeof(double) * P->harena);
    L.wp = take(sizeof(double) * P->warena);
    L.tp = take(sizeof(double) * P->warena);
    L.status = take(sizeof(unsigned long long));
    L.blocks = take(sizeof(BlockDesc) * P->blocks.size());
    L.crow = take(sizeof(int32_t) * P->crow.size());
    L.cbase = take(sizeof(int64_t) * P->cbase.size());
    L.rbase = take(sizeof(int64_t) * P->rbase.size());
    L.rel = take(sizeof(int32_t) * P->rel.size());
    L.asm_off = take(sizeof(int64_t) * P->asm_off.size());
    L.exp_off = take(sizeof(int64_t) * P->exp_off.size());
    L.colblk = take(sizeof(int32_t) * P->colblk.size());
    L.colptrL = take(sizeof(int64_t) * P->colptrL.size());
    L.t_diag = take(sizeof(Task) * P->t_diag.tasks.size());
    L.t_panel = take(sizeof(Task) * P->t_panel.tasks.size());
    L.t_schur = take(sizeof(Task) * P->t_schur.tasks.size());
    L.t_gemm = take(sizeof(Task) * P->t_gemm.tasks.size());
    L.t_sdiag = take(sizeof(Task) * P->t_sdiag.tasks.size());
    L.t_zero = take(sizeof(Task) * P->t_zero.size());
    L.zb = take(sizeof(double) * P->arena);
    L.hb = take(sizeof(double) * P->harena);
    L.tb = take(sizeof(double) * P->warena);
    L.t_rs1 = take(sizeof(Task) * P->t_rs1.tasks.size());
    L.t_rs2 = take(sizeof(Task) * P->t_rs2.tasks.size());
    L.t_rs3 = take(sizeof(Task) * P->t_rs3.tasks.size());
    L.t_rf1a = take(sizeof(Task) * P->t_rf1a.tasks.size());
    L.t_rf1b = take(sizeof(Task) * P->t_rf1b.tasks.size());
    L.t_rf2 = take(sizeof(Task) * P->t_rf2.tasks.size());
    L.total = o;
    P->info.workspace_bytes = (int64_t)o;
}

DevPtrs dev_ptrs(const selinv_plan_s* P)
{
    const DeviceLayout& L = P->lay;
    char* w = P->ws;
    DevPtrs D;
    D.Lp = (double*)(w + L.lp);
    D.Ap = (double*)(w + L.ap);
    D.Hp = (double*)(w + L.hp);
    D.Wp = (double*)(w + L.wp);
    D.Tp = (double*)(w + L.tp);
    D.status = (unsigned long long*)(w + L.status);
    D.blocks = (const BlockDesc*)(w + L.blocks);
    D.crow = (const int32_t*)(w + L.crow);
    D.cbase = (const int64_t*)(w + L.cbase);
    D.rbase = (const int64_t*)(w + L.rbase);
    D.rel = (const int32_t*)(w + L.rel);
    D.asm_off = (const int64_t*)(w + L.asm_off);
    D.exp_off = (const int64_t*)(w + L.exp_off);
    D.colblk = (const int32_t*)(w + L.colblk);
    D.colptrL = (const int64_t*)(w + L.colptrL);
    D.t_diag = (const Task*)(w + L.t_diag);
    D.t_panel = (const Task*)(w + L.t_panel);
    D.t_schur = (const Task*)(w + L.t_schur);
    D.t_gemm = (const Task*)(w + L.t_gemm);
    D.t_sdiag = (const Task*)(w + L.t_sdiag);
    D.t_zero = (const Task*)(w + L.t_zero);
    D.Zb = (double*)(w + L.zb);
    D.Hb = (double*)(w + L.hb);
    D.Tb = (double*)(w + L.tb);
    D.t_rs1 = (const Task*)(w + L.t_rs1);
    D.t_rs2 = (const Task*)(w + L.t_rs2);
    D.t_rs3 = (const Task*)(w + L.t_rs3);
    D.t_rf1a = (const Task*)(w + L.t_rf1a);
    D.t_rf1b = (const Task*)(w + L.t_rf1b);
    D.t_rf2 = (const Task*)(w + L.t_rf2);
    return D;
}

template <class T>
hipError_t upload(char* ws, size_t off, const std::vector<T>& v, hipStream_t s)
{
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(ws + off, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s);
}
}  // namespace

extern "C" {

const char* selinv_last_error(void) { return g_err.c_str(); }

selinv_status selinv_analyze(int64_t n, const int64_t* colptr, const int32_t* rowind, const selinv_geom* geom,
                             const int32_t* perm_or_null, const selinv_opts* opts, selinv_plan* out)
{
    if (!out) return fail(SELINV_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 0 || n > INT32_MAX - 1) return fail(SELINV_EINVAL, "n out of range");
    if (n > 0 && (!colptr || !rowind)) return fail(SELINV_EINVAL, "colptr/rowind is NULL");
    selinv_opts o{128, 1, 1, 0};
    if (opts) o = *opts;
    if (o.max_super <= 0) o.max_super = 128;
    // execution blocks default to <= 128 columns (the width the register
    // sweep of the diagonal block holds); the L pattern does not depend on
    // the partition, only the reported fundamental supernodes use max_super
    if (o.exec_cap <= 0) o.exec_cap = std::min(o.max_super, (int32_t)kLdsDiagMax);
    if (o.max_super > 256 || o.exec_cap > 256)
        return fail(SELINV_EUNSUPPORTED, "supernode width cap above 256 is not supported");
    if (n > 0) {
        if (colptr[0] != 0) return fail(SELINV_EINVAL, "colptr[0] must be 0");
        for (int64_t j = 0; j < n; j++) {
            if (colptr[j + 1] < colptr[j]) return fail(SELINV_EINVAL, "colptr is not monotone");
            for (int64_t p = colptr[j]; p < colptr[j + 1]; p++) {
                if (rowind[p] < j || rowind[p] >= n)
                    return fail(SELINV_EINVAL, "row index outside the lower triangle at column " + std::to_string(j));
                if (p > colptr[j] && rowind[p] <= rowind[p - 1])
                    return fail(SELINV_EINVAL, "rows not strictly increasing in column " + std::to_string(j));
            }
        }
    }
    if (geom && geom->ndim > 0) {
        if (geom->ndim > 3) return fail(SELINV_EINVAL, "geom.ndim must be 0..3");
        int64_t pts = 1;
        for (int d = 0; d < geom->ndim; d++) {
            if (geom->dims[d] <= 0) return fail(SELINV_EINVAL, "geom.dims must be positive");
            pts *= geom->dims[d];
        }
        int dofs = geom->dofs_per_point > 0 ? geom->dofs_per_point : 1;
        if (pts * dofs != n) return fail(SELINV_EINVAL, "geometry does not match n");
    }
    selinv_plan_s* P = new (std::nothrow) selinv_plan_s();
    if (!P) return fail(SELINV_ENOMEM, "out of host memory");
    try {
        P->n = n;
        P->opts = o;
        P->nnzA = n > 0 ? colptr[n] : 0;
        P->colptr.assign(colptr, colptr + (n > 0 ? n + 1 : 1));
        if (n == 0) P->colptr.assign(1, 0);
        if (P->nnzA > 0) P->rowind.assign(rowind, rowind + P->nnzA);
        std::string err;
        selinv_status st = analyze(P, geom, perm_or_null, err);
        if (st != SELINV_OK) {
            delete P;
            return fail(st, err);
        }
        build_schedule(P);
        compute_layout(P);
    } catch (const std::bad_alloc&) {
        delete P;
        return fail(SELINV_ENOMEM, "out of host memory during analysis");
    }
    *out = P;
    return SELINV_OK;
}

selinv_status selinv_workspace_size(selinv_plan P, size_t* bytes)
{
    if (!P || !bytes) return fail(SELINV_EINVAL, "NULL argument");
    *bytes = P->lay.total;
    return SELINV_OK;
}

selinv_status selinv_bind_workspace(selinv_plan P, void* d_ws, size_t bytes, hipStream_t s)
{
    if (!P || !d_ws) return fail(SELINV_EINVAL, "NULL argument");
    if (bytes < P->lay.total) return fail(SELINV_ENOMEM, "workspace too small");
    if (((uintptr_t)d_ws & 255) != 0) return fail(SELINV_EINVAL, "workspace must be 256-byte aligned");
    P->ws = (char*)d_ws;
    P->ws_bytes = bytes;
    P->factored = false;
    const DeviceLayout& L = P->lay;
    static hipError_t init = kernels_init();
    if (init != hipSuccess) return hip_fail(init, "kernel attributes");
    hipError_t e = hipSuccess;
    if (!e) e = upload(P->ws, L.blocks, P->blocks, s);
    if (!e) e = upload(P->ws, L.crow, P->crow, s);
    if (!e) e = upload(P->ws, L.cbase, P->cbase, s);
    if (!e) e = upload(P->ws, L.rbase, P->rbase, s);
    if (!e) e = upload(P->ws, L.rel, P->rel, s);
    if (!e) e = upload(P->ws, L.asm_off, P->asm_off, s);
    if (!e) e = upload(P->ws, L.exp_off, P->exp_off, s);
    if (!e) e = upload(P->ws, L.colblk, P->colblk, s);
    if (!e) e = upload(P->ws, L.colptrL, P->colptrL, s);
    if (!e) e = upload(P->ws, L.t_diag, P->t_diag.tasks, s);
    if (!e) e = upload(P->ws, L.t_panel, P->t_panel.tasks, s);
    if (!e) e = upload(P->ws, L.t_schur, P->t_schur.tasks, s);
    if (!e) e = upload(P->ws, L.t_gemm, P->t_gemm.tasks, s);
    if (!e) e = upload(P->ws, L.t_sdiag, P->t_sdiag.tasks, s);
    if (!e) e = upload(P->ws, L.t_zero, P->t_zero, s);
    if (!e) e = upload(P->ws, L.t_rs1, P->t_rs1.tasks, s);
    if (!e) e = upload(P->ws, L.t_rs2, P->t_rs2.tasks, s);
    if (!e) e = upload(P->ws, L.t_rs3, P->t_rs3.tasks, s);
    if (!e) e = upload(P->ws, L.t_rf1a, P->t_rf1a.tasks, s);
    if (!e) e = upload(P->ws, L.t_rf1b, P->t_rf1b.tasks, s);
    if (!e) e = upload(P->ws, L.t_rf2, P->t_rf2.tasks, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) {
        P->ws = nullptr;
        return hip_fail(e, "bind_workspace upload");
    }
    return SELINV_OK;
}

selinv_status selinv_factor(selinv_plan P, const double* d_valsA, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (P->nnzA > 0 && !d_valsA) return fail(SELINV_EINVAL, "d_valsA is NULL");
    DevPtrs D = dev_ptrs(P);
    // status word := "no failure"; zero the factor arena; assemble A
    hipError_t e = launch_status_reset(D.status, s);
    if (!e) e = launch_fill(&P->prof, kAssemble, D.Lp, P->arena, 0.0, s);
    if (!e) e = launch_scatter_set(&P->prof, kAssemble, d_valsA, D.asm_off, P->nnzA, D.Lp, s);
    if (e) return hip_fail(e, "factor setup");
    const int depth = P->exec.depth;
    for (int l = depth - 1; l >= 0; l--) {
        const auto& a = P->t_diag.off;
        const auto& b = P->t_panel.off;
        const auto& c = P->t_schur.off;
        e = launch_factor_level(&P->prof, D, a[l], a[l + 1] - a[l], b[l], b[l + 1] - b[l], c[l], c[l + 1] - c[l],
                                P->opts.require_spd, s);
        if (e) return hip_fail(e, "factor level launch");
    }
    P->factored = true;
    P->inverted = false;
    return SELINV_OK;
}

selinv_status selinv_backward(selinv_plan P, const double* d_gsel, double* d_gA, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (!P->inverted) return fail(SELINV_ESTATE, "backward needs factor and invert of the same values first");
    if ((P->colptrL.back() > 0 && !d_gsel) || (P->nnzA > 0 && !d_gA)) return fail(SELINV_EINVAL, "NULL buffer");
    for (const BlockDesc& d : P->blocks)
        if (d.s > kLdsDiagMax)
            return fail(SELINV_EUNSUPPORTED, "backward supports execution blocks of at most 128 columns");
    DevPtrs D = dev_ptrs(P);
    hipError_t e = launch_backward_init(&P->prof, D, P->arena, P->harena, d_gsel, P->colptrL.back(), s);
    if (e) return hip_fail(e, "backward setup");
    const int depth = P->exec.depth;
    // reverse selected inversion: leaves first
    for (int l = depth - 1; l >= 0; l--) {
        const auto& a = P->t_rs1.off;
        const auto& b = P->t_rs2.off;
        const auto& c = P->t_rs3.off;
        e = launch_revsel_level(&P->prof, D, a[l], a[l + 1] - a[l], b[l], b[l + 1] - b[l], c[l], c[l + 1] - c[l], s);
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
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    if (!P->factored) return fail(SELINV_ESTATE, "invert called before factor");
    if (P->colptrL.back() > 0 && !d_sel) return fail(SELINV_EINVAL, "d_sel is NULL");
    DevPtrs D = dev_ptrs(P);
    hipError_t e = launch_zero_x(&P->prof, D, (int64_t)P->t_zero.size(), s);
    if (e) return hip_fail(e, "invert setup");
    const int depth = P->exec.depth;
    for (int l = 0; l < depth; l++) {
        const auto& g = P->t_gemm.off;
        const auto& d = P->t_sdiag.off;
        e = launch_invert_level(&P->prof, D, g[l], g[l + 1] - g[l], d[l], d[l + 1] - d[l], s);
        if (e) return hip_fail(e, "invert level launch");
    }
    e = launch_gather(&P->prof, kExport, D.Ap, D.exp_off, P->colptrL.back(), d_sel, s);
    if (e) return hip_fail(e, "export launch");
    P->inverted = true;
    return SELINV_OK;
}

selinv_status selinv_get_factor(selinv_plan P, double* d_L, hipStream_t s)
{
    if (!P) return fail(SELINV_EINVAL, "NULL plan");
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
    unsigned long long v = ~0ull;
    hipError_t e = hipMemcpyAsync(&v, P->ws + P->lay.status, sizeof v, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return hip_fail(e, "sync_status");
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
    switch (which) {
        case 0: off = P->lay.lp; n = P->arena; break;
        case 1: off = P->lay.ap; n = P->arena; break;
        case 2: off = P->lay.hp; n = P->harena; break;
        case 3: off = P->lay.wp; n = P->warena; break;
        case 4: off = P->lay.tp; n = P->warena; break;
        case 5: off = P->lay.zb; n = P->arena; break;
        case 6: off = P->lay.hb; n = P->harena; break;
        case 7: off = P->lay.tb; n = P->warena; break;
        default: return fail(SELINV_EINVAL, "unknown arena");
    }
    if (count) *count = n;
    if (!d_out || n == 0) return SELINV_OK;
    if (!P->ws) return fail(SELINV_ESTATE, "no workspace bound");
    hipError_t e = hipMemcpyAsync(d_out, P->ws + off, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
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

void selinv_destroy(selinv_plan P) { delete P; }

}  // extern "C"
