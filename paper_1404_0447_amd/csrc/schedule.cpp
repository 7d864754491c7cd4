// Per-level task lists (Algorithm 2 priority levels): the factor runs the
// levels from the leaves up, the inversion from the root down; all blocks of
// one level are independent (Section 2.2), so each level is one launch per
// kernel kind with one work-group per task.
#include <algorithm>

#include "kernels.hpp"
#include "plan.hpp"
#include "tiles.hpp"

namespace selinv {

static void by_level(const selinv_plan_s* P, std::vector<std::vector<int>>& lv)
{
    lv.assign(P->exec.depth, {});
    for (int B = 0; B < P->exec.nblocks(); B++) lv[P->exec.lev[B] - 1].push_back(B);
}

void build_schedule(selinv_plan_s* P)
{
    std::vector<std::vector<int>> lv;
    by_level(P, lv);
    const int D = (int)lv.size();
    LevelTasks* all[] = {&P->t_diag, &P->t_panel, &P->t_schur, &P->t_gemm, &P->t_sdiag};
    for (LevelTasks* t : all) {
        t->tasks.clear();
        t->off.assign(D + 1, 0);
    }
    P->t_zero.clear();
    for (int l = 0; l < D; l++) {
        // tiles of X this level has without splitting the contraction over C
        int64_t base = 0, dbase = 0;
        for (int B : lv[l]) {
            const BlockDesc& d = P->blocks[B];
            base += (int64_t)((d.c + kTileM - 1) / kTileM) * ((d.s + tile_bn(d.s) - 1) / tile_bn(d.s));
            const int nd = (d.s + kDiagTile - 1) / kDiagTile;
            dbase += nd * (nd + 1) / 2;
        }
        const int64_t want = base > 0 && base < kFillTiles ? (kFillTiles + base - 1) / base : 1;
        const int64_t dwant = dbase > 0 && dbase < kFillTiles ? (kFillTiles + dbase - 1) / dbase : 1;
        for (int B : lv[l]) {
            const BlockDesc& d = P->blocks[B];
            const int bn = tile_bn(d.s);
            P->t_diag.tasks.push_back({B, 0, 0, 0, 0, 0, 0, 0});
            // contractions over C are split into pieces of >= kMinSplitK rows
            // when a level has too few tiles to fill the device
            const int nchunk = (d.c + 15) / 16;
            const int maxsplit = std::max(1, nchunk / (kMinSplitK / 16));
            const int split = (int)std::min<int64_t>(want, maxsplit);
            const int dsplit = (int)std::min<int64_t>(dwant, maxsplit);
            if (split > 1 || dsplit > 1) P->t_zero.push_back({B, 0, 0, 0, 0, 0, 0, 0});
            const int nd = (d.s + kDiagTile - 1) / kDiagTile;
            for (int I = 0; I < nd; I++)
                for (int J = 0; J <= I; J++)
                    for (int q = 0; q < dsplit; q++) {
                        const int kb = (int)((int64_t)nchunk * q / dsplit) * 16;
                        const int ke = std::min(d.c, (int)((int64_t)nchunk * (q + 1) / dsplit) * 16);
                        P->t_sdiag.tasks.push_back({B, I * kDiagTile, J * kDiagTile, 0, kb, ke, dsplit > 1, 0});
                    }
            for (int j = 0; j < d.s; j += bn)
                for (int r = 0; r < d.c; r += kTileM) {
                    P->t_panel.tasks.push_back({B, r, j, bn, 0, d.s, 0, 0});
                    for (int q = 0; q < split; q++) {
                        const int kb = (int)((int64_t)nchunk * q / split) * 16;
                        const int ke = std::min(d.c, (int)((int64_t)nchunk * (q + 1) / split) * 16);
                        P->t_gemm.tasks.push_back({B, r, j, bn, kb, ke, split > 1 ? 1 : 0, 0});
                    }
                }
            for (int k = 0; k < d.c; k += kSchurTile)
                for (int i = k; i < d.c; i += kSchurTile)
                    P->t_schur.tasks.push_back({B, i, k, kSchurTile, 0, d.s, 0, 0});
        }
        for (LevelTasks* t : all) t->off[l + 1] = (int64_t)t->tasks.size();
    }
    // algorithmic work of one factor / one invert call, per kernel kind
    P->work_flops.assign(kNumKinds, 0.0);
    P->work_bytes.assign(kNumKinds, 0.0);
    for (const BlockDesc& d : P->blocks) {
        const double s = d.s, c = d.c;
        P->work_flops[kLdlt] += s * s * s;              // LDL^T s^3/3, W s^3/3, T s^3/3
        P->work_bytes[kLdlt] += 8.0 * 3 * s * s;
        P->work_flops[kPanel] += 2.0 * c * s * s;       // L_hat = F(C,B) T
        P->work_bytes[kPanel] += 8.0 * (2 * c * s + s * s);
        P->work_flops[kSchur] += c * c * s;             // lower half of L D L^T
        P->work_bytes[kSchur] += 8.0 * (c * s + c * (c + 1) / 2);
        P->work_flops[kGemm] += 2.0 * c * c * s;        // X = -G L_hat
        P->work_bytes[kGemm] += 8.0 * (c * (c + 1) / 2 + 2 * c * s);
        P->work_flops[kSdiag] += 2.0 * c * s * s;       // Y = T - L_hat^T X
        P->work_bytes[kSdiag] += 8.0 * (2 * c * s + 2 * s * s);
    }
    const double nnzL = (double)P->colptrL.back(), nnzA = (double)P->nnzA;
    P->work_bytes[kAssemble] = 8.0 * P->arena + 24.0 * nnzA;
    P->work_bytes[kExport] = 24.0 * nnzL;
}

}  // namespace selinv
