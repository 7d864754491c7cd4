// Batched form: many independent sparse matrices treated as the
// block-diagonal matrix they form together.  Its elimination tree is the
// forest of their trees, so the Algorithm 2 levels of all matrices line up
// (every root has priority 1) and one launch per level covers the whole
// batch.  Each matrix is analysed on its own; this file only concatenates
// the results, shifting column, block and arena offsets.
#include <algorithm>

#include "plan.hpp"

namespace selinv {

namespace {
template <class T>
void append(std::vector<T>& dst, const std::vector<T>& src, T shift, size_t skip_last = 0)
{
    const size_t n = src.size() - std::min(skip_last, src.size());
    for (size_t i = 0; i < n; i++) dst.push_back(src[i] + shift);
}

// tree parents: -1 stays a root
void append_parent(std::vector<int32_t>& dst, const std::vector<int32_t>& src, int32_t shift)
{
    for (int32_t p : src) dst.push_back(p >= 0 ? p + shift : -1);
}

void append_partition(Partition& U, const Partition& P, int32_t col0, int32_t blk0, int64_t row0)
{
    append(U.xs, P.xs, col0, 1);
    append(U.of, P.of, blk0);
    append_parent(U.par, P.par, blk0);
    append(U.lev, P.lev, 0);
    append(U.cptr, P.cptr, row0, 1);
    append(U.crows, P.crows, col0);
    U.depth = std::max(U.depth, P.depth);
}
}  // namespace

void merge_plans(const std::vector<selinv_plan_s*>& parts, selinv_plan_s* U)
{
    int64_t n0 = 0, a0 = 0, l0 = 0, ar0 = 0, h0 = 0, w0 = 0, rel0 = 0;
    int32_t f0 = 0, e0 = 0;
    int64_t fr0 = 0, er0 = 0;
    U->colptr.assign(1, 0);
    U->colptrL.assign(1, 0);
    U->b_noff.assign(1, 0);
    U->b_aoff.assign(1, 0);
    U->b_loff.assign(1, 0);
    selinv_info& I = U->info;
    I = selinv_info{};
    for (size_t m = 0; m < parts.size(); m++) {
        const selinv_plan_s* P = parts[m];
        const int32_t c0 = (int32_t)n0;
        // pattern of A and the ordering
        for (size_t j = 1; j < P->colptr.size(); j++) U->colptr.push_back(P->colptr[j] + a0);
        append(U->rowind, P->rowind, c0);
        append(U->perm, P->perm, c0);
        append(U->iperm, P->iperm, c0);
        append_parent(U->parent, P->parent, c0);
        append(U->cnt, P->cnt, 0);
        // supernodes and execution blocks
        append_partition(U->fund, P->fund, c0, f0, fr0);
        append_partition(U->exec, P->exec, c0, e0, er0);
        // canonical pattern of L
        for (size_t j = 1; j < P->colptrL.size(); j++) U->colptrL.push_back(P->colptrL[j] + l0);
        append(U->rowindL, P->rowindL, c0);
        // device tables
        for (const BlockDesc& d0 : P->blocks) {
            BlockDesc d = d0;
            d.poff += ar0;
            d.hoff += h0;
            d.woff += w0;
            d.coff += er0;
            d.first += c0;
            U->blocks.push_back(d);
            U->blk_matrix.push_back((int32_t)m);
        }
        append(U->crow, P->crow, c0);
        append(U->cbase, P->cbase, ar0);
        append(U->rbase, P->rbase, rel0);
        append(U->rel, P->rel, 0);
        append(U->asm_off, P->asm_off, ar0);
        append(U->exp_off, P->exp_off, ar0);
        append(U->colblk, P->colblk, e0);
        // counts
        I.nsuper += P->info.nsuper;
        I.depth = std::max(I.depth, P->info.depth);
        I.nblocks += P->info.nblocks;
        I.exec_depth = std::max(I.exec_depth, P->info.exec_depth);
        I.flops_factor += P->info.flops_factor;
        I.flops_gemm += P->info.flops_gemm;
        I.flops_selinv += P->info.flops_selinv;
        I.gather_bytes += P->info.gather_bytes;
        I.exec_flops_gemm += P->info.exec_flops_gemm;
        n0 += P->n;
        a0 += P->nnzA;
        l0 += P->colptrL.back();
        ar0 += P->arena;
        h0 += P->harena;
        w0 += P->warena;
        rel0 += (int64_t)P->rel.size();
        f0 += P->fund.nblocks();
        e0 += P->exec.nblocks();
        fr0 += (int64_t)P->fund.crows.size();
        er0 += (int64_t)P->exec.crows.size();
        U->b_noff.push_back(n0);
        U->b_aoff.push_back(a0);
        U->b_loff.push_back(l0);
    }
    U->fund.xs.push_back((int32_t)n0);
    U->fund.cptr.push_back(fr0);
    U->exec.xs.push_back((int32_t)n0);
    U->exec.cptr.push_back(er0);
    U->n = n0;
    U->nnzA = a0;
    U->arena = ar0;
    U->harena = h0;
    U->warena = w0;
    I.n = n0;
    I.nnzA = a0;
    I.nnzL = l0;
}

}  // namespace selinv
