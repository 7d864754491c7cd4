// Per-level task lists (Algorithm 2 priority levels): the factor runs the
// levels from the leaves up, the inversion from the root down; all blocks of
// one level are independent (Section 2.2), so each level is one launch per
// kernel kind with one work-group per task.
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
    for (int l = 0; l < D; l++) {
        for (int B : lv[l]) {
            const BlockDesc& d = P->blocks[B];
            P->t_diag.tasks.push_back({B, 0, 0, 0});
            P->t_sdiag.tasks.push_back({B, 0, 0, 0});
            for (int r = 0; r < d.c; r += kPanelRows) P->t_panel.tasks.push_back({B, r, 0, 0});
            for (int k = 0; k < d.c; k += kSchurTile)
                for (int i = k; i < d.c; i += kSchurTile) P->t_schur.tasks.push_back({B, i, k, 0});
            for (int j = 0; j < d.s; j += kGemmBN)
                for (int r = 0; r < d.c; r += kGemmBM) P->t_gemm.tasks.push_back({B, r, j, 0});
        }
        for (LevelTasks* t : all) t->off[l + 1] = (int64_t)t->tasks.size();
    }
}

}  // namespace selinv
