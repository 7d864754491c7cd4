// Per-level task lists (Algorithm 2 priority levels): the factor runs the
// levels from the leaves up, the inversion from the root down; all blocks of
// one level are independent (Section 2.2), so each level is one launch per
// kernel kind with one work-group per task.  The reverse sweep uses the same
// levels in the opposite orders.
#include <algorithm>
#include <functional>
#include <queue>
#include <unordered_map>

#include "kernels.hpp"
#include "plan.hpp"
#include "tiles.hpp"

namespace selinv {

static void by_level(const selinv_plan_s* P, std::vector<std::vector<int>>& lv)
{
    lv.assign(P->exec.depth, {});
    for (int B = 0; B < P->exec.nblocks(); B++) lv[P->exec.lev[B] - 1].push_back(B);
}

// contraction range [lo, hi) cut into `split` pieces aligned to 16 rows; an
// empty range still yields one (empty) piece, e.g. the diagonal block of a
// root (c = 0) whose inverse is T alone
template <class F>
static void pieces(int lo, int hi, int split, F emit)
{
    if (hi <= lo) {
        emit(lo, lo, 0);
        return;
    }
    const int n16 = (hi - lo + 15) / 16;
    for (int q = 0; q < split; q++) {
        const int kb = lo + (int)((int64_t)n16 * q / split) * 16;
        const int ke = std::min(hi, lo + (int)((int64_t)n16 * (q + 1) / split) * 16);
        if (kb < ke) emit(kb, ke, q);
    }
}

static int split_for(int64_t want, int len, int mink = kMinSplitK)
{
    const int maxsplit = std::max(1, ((len + 15) / 16) / (mink / 16));
    return (int)std::min<int64_t>(want, maxsplit);
}

// Tiles of one level with the same contraction length c and width weight w.
struct TileGroup {
    int64_t count;
    int c;
    int w;
};

// Split request for one level: every tile's contraction is cut into
// split_for(want, c) pieces, one work-group each; work-groups run in rounds
// on `slots` resident places, so a level whose count is just above a
// multiple of slots pays a nearly empty round.  Pick the request whose
// greedy list schedule (largest first onto the least loaded place; cost =
// (16-row chunks + ovh) times tile width) finishes first.  ovh is the fixed
// cost of one work-group in chunk times: the exposed latency of its first
// loads and its epilogue (atomic for a split contraction); on the gathered
// GEMM it measures at seven to twelve chunks, so splitting stops paying
// once the pieces get short.
static int64_t best_split(const std::vector<TileGroup>& groups, int64_t slots, double ovh, int maxwant = 32,
                          int mink = kMinSplitK)
{
    int64_t base = 0;
    for (const TileGroup& g : groups) base += g.count;
    if (base == 0 || base >= 4 * slots) return 1;
    int64_t best = 1;
    double best_t = -1.0;
    std::vector<double> cost;
    for (int64_t want = 1; want <= maxwant; want++) {
        cost.clear();
        for (const TileGroup& g : groups) {
            const int sp = split_for(want, g.c, mink), n16 = (g.c + 15) / 16;
            for (int q = 0; q < sp; q++) {
                const int len = (int)((int64_t)n16 * (q + 1) / sp - (int64_t)n16 * q / sp);
                for (int64_t k = 0; k < g.count; k++) cost.push_back((len + ovh) * g.w);
            }
        }
        std::sort(cost.begin(), cost.end(), std::greater<double>());
        std::priority_queue<double, std::vector<double>, std::greater<double>> load;
        for (int64_t k = 0; k < slots; k++) load.push(0.0);
        double t = 0.0;
        for (double x : cost) {
            const double y = load.top() + x;
            load.pop();
            load.push(y);
            t = std::max(t, y);
        }
        if (best_t < 0 || t < best_t * (1 - 1e-9)) {
            best_t = t;
            best = want;
        }
    }
    return best;
}

// Schur tiles of one level, [t0, end) of `tasks`, appended block by block.
// Two blocks update a common ancestor entry exactly when their C share a
// column, so a greedy colouring of the level's blocks (largest update
// first; colour = lowest one no block sharing a column has taken) gives
// groups whose updates are disjoint: each group runs as one launch with
// plain read-modify-write (flags bit 2).  Past 63 colours the rest keep
// FP64 atomics in a last group.  cuts receives the group boundaries.
static void schur_colours(const selinv_plan_s* P, std::vector<Task>& tasks, int64_t t0, std::vector<uint64_t>& mask,
                          std::vector<int64_t>& cuts)
{
    const std::vector<int32_t>& cr = P->crow;
    std::vector<int> bl;
    for (int64_t t = t0; t < (int64_t)tasks.size(); t++)
        if (bl.empty() || bl.back() != tasks[t].b) bl.push_back(tasks[t].b);
    std::vector<int> order = bl;
    auto work = [&](int B) {
        const BlockDesc& d = P->blocks[B];
        return (double)d.c * d.c * d.s;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    std::unordered_map<int, int> col;
    for (int B : order) {
        const BlockDesc& d = P->blocks[B];
        uint64_t used = 0;
        for (int r = 0; r < d.c; r++) used |= mask[cr[d.coff + r]];
        int k = 0;
        while (k < 63 && ((used >> k) & 1)) k++;
        col[B] = k;
        for (int r = 0; r < d.c; r++) mask[cr[d.coff + r]] |= uint64_t(1) << k;
    }
    for (int B : bl) {
        const BlockDesc& d = P->blocks[B];
        for (int r = 0; r < d.c; r++) mask[cr[d.coff + r]] = 0;
    }
    // more colours than kMaxSchurColours: one launch, FP64 atomics (blocks
    // found exclusive keep read-modify-write)
    int ncol = 0;
    for (const auto& kv : col) ncol = std::max(ncol, kv.second + 1);
    if (ncol > kMaxSchurColours) {
        cuts.assign({t0, (int64_t)tasks.size()});
        return;
    }
    std::stable_sort(tasks.begin() + t0, tasks.end(), [&](const Task& a, const Task& b) { return col[a.b] < col[b.b]; });
    cuts.assign(1, t0);
    for (int64_t t = t0; t < (int64_t)tasks.size(); t++) {
        const int k = col[tasks[t].b];
        tasks[t].flags = k < 63 ? (tasks[t].flags | 4) : (tasks[t].flags & ~4);
        if (t > t0 && k != col[tasks[t - 1].b]) cuts.push_back(t);
    }
    cuts.push_back((int64_t)tasks.size());
}

// Colours for the blocks `bl` of one level with no limit on their number
// (deterministic mode): blocks sharing a column of C get different colours;
// greedy passes, colour k taking every still uncoloured block (largest
// update first) whose columns no block of colour k has claimed.
static std::unordered_map<int, int> colour_unbounded(const selinv_plan_s* P, const std::vector<int>& bl,
                                                     std::vector<int32_t>& stamp)
{
    const std::vector<int32_t>& cr = P->crow;
    std::vector<int> order = bl;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const BlockDesc &x = P->blocks[a], &y = P->blocks[b];
        return (double)x.c * x.c * x.s > (double)y.c * y.c * y.s;
    });
    std::unordered_map<int, int> col;
    size_t left = order.size();
    for (int k = 0; left > 0; k++) {
        for (int B : order) {
            if (col.count(B)) continue;
            const BlockDesc& d = P->blocks[B];
            bool ok = true;
            for (int r = 0; r < d.c && ok; r++) ok = stamp[cr[d.coff + r]] != k;
            if (!ok) continue;
            col[B] = k;
            for (int r = 0; r < d.c; r++) stamp[cr[d.coff + r]] = k;
            left--;
        }
    }
    for (int B : bl) {
        const BlockDesc& d = P->blocks[B];
        for (int r = 0; r < d.c; r++) stamp[cr[d.coff + r]] = -1;
    }
    return col;
}

// Tasks [t0, end) of one level grouped by the colour of their block (stable
// within a colour), flags |= `bit` on every task, cuts = group boundaries.
static void group_by_colour(std::vector<Task>& tasks, int64_t t0, const std::unordered_map<int, int>& col, int bit,
                            std::vector<int64_t>& cuts)
{
    std::stable_sort(tasks.begin() + t0, tasks.end(),
                     [&](const Task& a, const Task& b) { return col.at(a.b) < col.at(b.b); });
    cuts.assign(1, t0);
    for (int64_t t = t0; t < (int64_t)tasks.size(); t++) {
        tasks[t].flags |= bit;
        if (t > t0 && col.at(tasks[t].b) != col.at(tasks[t - 1].b)) cuts.push_back(t);
    }
    cuts.push_back((int64_t)tasks.size());
}

// Blocks of one level whose Schur updates no other block of the level
// touches: two blocks update a common ancestor entry exactly when their row
// structures C share a column (the diagonal entry of that column), so a
// block is exclusive when every column of its C is in no other block's C.
// Exclusive blocks add their updates with plain read-modify-write instead
// of atomics.
static void exclusive_blocks(const selinv_plan_s* P, const std::vector<int>& bl, std::vector<int32_t>& touch,
                             std::vector<char>& excl)
{
    const std::vector<int32_t>& cr = P->crow;
    for (int B : bl) {
        const BlockDesc& d = P->blocks[B];
        for (int r = 0; r < d.c; r++) touch[cr[d.coff + r]]++;
    }
    for (int B : bl) {
        const BlockDesc& d = P->blocks[B];
        bool ok = true;
        for (int r = 0; r < d.c && ok; r++) ok = touch[cr[d.coff + r]] == 1;
        excl[B] = ok;
    }
    for (int B : bl) {
        const BlockDesc& d = P->blocks[B];
        for (int r = 0; r < d.c; r++) touch[cr[d.coff + r]] = 0;
    }
}

// small blocks of a level in groups of four (one per wave of a work-group)
static void push_sb_groups(const std::vector<int>& small, int op, std::vector<Task>& out)
{
    for (size_t q = 0; q < small.size(); q += kSbPerTask) {
        int id[kSbPerTask];
        for (int w = 0; w < kSbPerTask; w++) id[w] = q + w < small.size() ? small[q + w] : -1;
        out.push_back({id[0], id[1], id[2], id[3], 0, 0, q_flags(op, 0), 0});
    }
}

// Complex plans (deterministic schedule: every gather-GEMM tile and
// diagonal-step task contracts over all of C): a level with fewer than
// kZSplitFill / 2 tasks of one kind cuts each task's contraction into
// pieces of at least kZSplitRows rows (half that in a level of fewer than
// kZSplitFewTasks tasks; boundaries on 16-row chunks), about
// kZSplitFill pieces in all.  A piece (flags bit 5) writes its partial
// product over its rows of C to scratch slot `pad`; after the pieces, one
// task per split task (same block and tile origin, bn = pieces, kb = first
// slot, flags bit 6) sums them in piece order and writes the result.
// Unsplit tasks keep their form and do both.  Every sum has a fixed order,
// so the results stay bitwise repeatable.  The level's list becomes whole
// tasks, then pieces (from `mid`), then summing tasks (from `cut`); returns
// the slots used.
static int64_t zsplit_level(const selinv_plan_s* P, LevelTasks& lt, int l, int64_t& mid, int64_t& cut)
{
    std::vector<Task>& t = lt.tasks;
    const int64_t t0 = lt.off[l], n = (int64_t)t.size() - t0;
    mid = cut = (int64_t)t.size();
    if (n <= 0 || n >= kZSplitFill / 2) return 0;
    const int want = (int)((kZSplitFill + n - 1) / n);
    // levels with very few tasks (a single pole's) take shorter pieces
    const int rows = n < kZSplitFewTasks ? kZSplitRows / 2 : kZSplitRows;
    std::vector<Task> whole, pieces, sums;
    int64_t slot = 0;
    for (int64_t q = t0; q < (int64_t)t.size(); q++) {
        const Task k = t[q];
        const int c = P->blocks[k.b].c;
        const int np = std::max(1, std::min(want, c / rows));
        if (np == 1) {
            whole.push_back(k);
            continue;
        }
        for (int i = 0; i < np; i++) {
            const int kb = (int)((int64_t)c * i / np) & ~15;
            const int ke = i + 1 == np ? c : (int)((int64_t)c * (i + 1) / np) & ~15;
            pieces.push_back({k.b, k.i0, k.j0, k.bn, kb, ke, 32, (int32_t)(slot + i)});
        }
        sums.push_back({k.b, k.i0, k.j0, np, (int32_t)slot, 0, 64, 0});
        slot += np;
    }
    t.resize(t0);
    t.insert(t.end(), whole.begin(), whole.end());
    mid = (int64_t)t.size();
    t.insert(t.end(), pieces.begin(), pieces.end());
    cut = (int64_t)t.size();
    t.insert(t.end(), sums.begin(), sums.end());
    return slot;
}

void build_schedule(selinv_plan_s* P)
{
    std::vector<std::vector<int>> lv;
    by_level(P, lv);
    const int D = (int)lv.size();
    LevelTasks* all[] = {&P->t_diag, &P->t_ldlt, &P->t_panel, &P->t_schur, &P->t_gemm, &P->t_sdiag, &P->t_sb,
                         &P->t_rs1,  &P->t_rs2,  &P->t_rs3,   &P->t_rf1a,  &P->t_rf1b, &P->t_rf2};
    for (LevelTasks* t : all) {
        t->tasks.clear();
        t->off.assign(D + 1, 0);
    }
    P->t_zero.clear();
    P->t_zero_off.assign(D + 1, 0);
    P->ldlt_cut.assign(2 * D, 0);
    P->schur_cuts.assign(D, {});
    P->rs3_cuts.assign(D, {});
    P->sdiag_cut.assign(D, 0);
    P->panel_deep.assign(D, 0);
    P->zsd_slots = 0;
    P->zgemm_cut.assign(D, 0);
    P->zgemm_mid.assign(D, 0);
    // deterministic mode: no small-block kernels (their Schur updates use
    // atomics), no split contractions, no whole-contraction kernel variants
    const bool det = P->opts.deterministic != 0;
    // the small-block kernels factor without pivots: none with pivoting
    const bool piv = P->opts.pivoting != 0;
    auto small_block = [&](int s, int c) { return !det && !piv && is_small_level(s, c); };
    std::vector<uint64_t> colour_mask((size_t)P->n, 0);
    std::vector<int32_t> touch((size_t)P->n, 0), stamp((size_t)P->n, -1);
    std::vector<char> excl(P->blocks.size(), 0);
    for (int l = 0; l < D; l++) {
        exclusive_blocks(P, lv[l], touch, excl);
        // tiles this level has without splitting contractions over C: of the
        // tiled forward path, and of the reverse sweep (every block)
        int64_t base = 0, dbase = 0, rbase_ = 0, rdbase = 0;
        std::vector<int> small;
        for (int B : lv[l]) {
            const BlockDesc& d = P->blocks[B];
            const int64_t tiles = (int64_t)((d.c + kTileM - 1) / kTileM) * ((d.s + tile_bn(d.s) - 1) / tile_bn(d.s));
            const int nd = (d.s + kDiagTile - 1) / kDiagTile;
            rbase_ += tiles;
            rdbase += nd * (nd + 1) / 2;
            if (small_block(d.s, d.c)) {
                small.push_back(B);
                continue;
            }
            base += tiles;
            dbase += nd * (nd + 1) / 2;
        }
        push_sb_groups(small, qSbFactor, P->t_sb.tasks);
        auto fill_for = [](int64_t tiles) { return tiles > 0 && tiles < kFillTiles ? (kFillTiles + tiles - 1) / tiles : 1; };
        // forward splits from the round model; the reverse sweep fills kFillTiles
        std::vector<TileGroup> gg, dg;
        for (int B : lv[l]) {
            const BlockDesc& d = P->blocks[B];
            if (small_block(d.s, d.c) || d.c == 0) continue;
            const int bn = tile_bn(d.s), nd = (d.s + kDiagTile64 - 1) / kDiagTile64;
            gg.push_back({(int64_t)((d.c + kTileM - 1) / kTileM) * ((d.s + bn - 1) / bn), d.c, bn});
            // one 64 x 64 product per task: nd diagonal tiles, two halves per
            // off-diagonal tile
            dg.push_back({(int64_t)nd * nd, d.c, kDiagTile64});
        }
        const int64_t want = det ? 1 : best_split(gg, kGemmSlots, kGemmTaskOvh, 64);
        // a block has only nd (nd + 1) / 2 diagonal pairs: their contraction
        // may be cut finer to fill the device
        const int64_t dwant = det ? 1 : best_split(dg, kGemmSlots, kSdiagTaskOvh, 64, kMinSplitKDiag);
        const int64_t rwant = det ? 1 : fill_for(rbase_), rdwant = det ? 1 : fill_for(rdbase);
        (void)base;
        (void)dbase;
        // few panel tiles: at most 64 wide each, for the whole-contraction kernel
        int64_t npanel64 = 0;
        int smax = 0;
        for (int B : lv[l]) {
            const BlockDesc& d = P->blocks[B];
            if (small_block(d.s, d.c)) continue;
            const int pbn = std::min(tile_bn(d.s), 64);
            npanel64 += (int64_t)((d.c + kTileM - 1) / kTileM) * ((d.s + pbn - 1) / pbn);
            smax = std::max(smax, d.s);
        }
        // the whole-contraction kernels hold a contraction of at most kDeepK
        // (blocks wider than 128 columns exist only with exec_cap > 128)
        const bool deep_ok = !det && smax <= kDeepK;
        const bool deep = deep_ok && npanel64 <= kDeepMaxTiles;
        P->panel_deep[l] = (char)((deep ? 1 : 0) | (deep_ok ? 2 : 0));
        for (int B : lv[l]) {
            const BlockDesc& d = P->blocks[B];
            const int bn = tile_bn(d.s);
            const int pbn = deep ? std::min(bn, 64) : bn;
            const int s = d.s, c = d.c;
            P->t_diag.tasks.push_back({B, 0, 0, 0, 0, 0, 0, 0});
            // reverse sweep: every block, tiled
            const int nd = (s + kDiagTile - 1) / kDiagTile;
            const int rsplit = split_for(rdwant, c);
            for (int I = 0; I < nd; I++)
                for (int J = 0; J < nd; J++)
                    pieces(0, c, rsplit, [&](int kb, int ke, int) {
                        P->t_rf2.tasks.push_back({B, I * kDiagTile, J * kDiagTile, 0, kb, ke, rsplit > 1, 0});
                    });
            for (int j = 0; j < s; j += bn)
                for (int r = 0; r < c; r += kTileM) {
                    P->t_rs1.tasks.push_back({B, r, j, bn, 0, s, 0, 0});
                    const int rs = split_for(rwant, c);
                    pieces(0, c, rs, [&](int kb, int ke, int) {
                        P->t_rs2.tasks.push_back({B, r, j, bn, kb, ke, rs > 1, 0});
                    });
                    // reverse factor: Ubar is lower triangular, so row tile r
                    // contracts over [0, r+64) with Ubar and over [r, c) with Ubar^T
                    const int hi = std::min(c, r + kTileM);
                    const int sa = split_for(rwant, hi);
                    pieces(0, hi, sa, [&](int kb, int ke, int) {
                        P->t_rf1a.tasks.push_back({B, r, j, bn, kb, ke, sa > 1, 0});
                    });
                    const int sb = split_for(rwant, c - r);
                    pieces(r, c, sb, [&](int kb, int ke, int q) {
                        // piece 0 also adds L_hat_bar T
                        P->t_rf1b.tasks.push_back({B, r, j, bn, kb, ke, (sb > 1) | (q == 0 ? 2 : 0), 0});
                    });
                }
            for (int k = 0; k < c; k += kSchurTile)
                for (int i = k; i < c; i += kSchurTile) P->t_rs3.tasks.push_back({B, i, k, kSchurTile, 0, 2 * s, 0, 0});
            if (small_block(s, c)) continue;
            // forward, tiled path
            // contractions over C are split into pieces of >= kMinSplitK rows
            // when a level has too few tiles to fill the device
            const int split = split_for(want, c);
            const int dsplit = split_for(dwant, c, kMinSplitKDiag);
            const int nd64 = (s + kDiagTile64 - 1) / kDiagTile64;
            // Ainv(B,B) accumulates (from T) when a contraction is split or
            // the block has off-diagonal tiles; X only when the GEMM is split
            const bool acc = dsplit > 1 || nd64 > 1;
            // a task per kZeroCols columns: one work-group per block would
            // serialise the largest blocks' (s + c) x s columns
            if (split > 1 || acc)
                for (int j = 0; j < s; j += kZeroCols)
                    P->t_zero.push_back({B, 0, 0, 0, j, std::min(s, j + kZeroCols), split > 1, 0});
            // deterministic: the half-products add with plain read-modify-write
            // (flags bit 4), the second halves in a launch of their own
            for (int I = 0; I < nd64; I++)
                for (int J = 0; J <= I; J++)
                    for (int half = 0; half < (I == J ? 1 : 2); half++)
                        pieces(0, c, dsplit, [&](int kb, int ke, int) {
                            P->t_sdiag.tasks.push_back({B, I * kDiagTile64, J * kDiagTile64, 0, kb, ke,
                                                        (int)acc | (half << 3) | (det && I != J ? 16 : 0), 0});
                        });
            for (int j = 0; j < s; j += pbn)
                for (int r = 0; r < c; r += kTileM) P->t_panel.tasks.push_back({B, r, j, pbn, 0, s, 0, 0});
            for (int j = 0; j < s; j += bn)
                for (int r = 0; r < c; r += kTileM) {
                    pieces(0, c, split, [&](int kb, int ke, int) {
                        P->t_gemm.tasks.push_back({B, r, j, bn, kb, ke, split > 1, 0});
                    });
                }
            for (int k = 0; k < c; k += kSchurTile)
                for (int i = k; i < c; i += kSchurTile)
                    P->t_schur.tasks.push_back({B, i, k, kSchurTile, 0, s, excl[B] ? 4 : 0, 0});
        }
        if (det) {
            // every Schur update and adjoint scatter in colour groups, however many
            const auto col = colour_unbounded(P, lv[l], stamp);
            group_by_colour(P->t_schur.tasks, P->t_schur.off[l], col, 4, P->schur_cuts[l]);
            group_by_colour(P->t_rs3.tasks, P->t_rs3.off[l], col, 4, P->rs3_cuts[l]);
            std::stable_partition(P->t_sdiag.tasks.begin() + P->t_sdiag.off[l], P->t_sdiag.tasks.end(),
                                  [](const Task& t) { return (t.flags & 8) == 0; });
            P->sdiag_cut[l] = P->t_sdiag.off[l] +
                              std::count_if(P->t_sdiag.tasks.begin() + P->t_sdiag.off[l], P->t_sdiag.tasks.end(),
                                            [](const Task& t) { return (t.flags & 8) == 0; });
        } else {
            schur_colours(P, P->t_schur.tasks, P->t_schur.off[l], colour_mask, P->schur_cuts[l]);
            P->rs3_cuts[l] = {P->t_rs3.off[l], (int64_t)P->t_rs3.tasks.size()};
            P->sdiag_cut[l] = (int64_t)P->t_sdiag.tasks.size();
        }
        if (P->opts.complex_values) {
            // the two launches run one after the other: they share the slots
            int64_t mid = 0;
            const int64_t a = zsplit_level(P, P->t_gemm, l, P->zgemm_mid[l], P->zgemm_cut[l]);
            const int64_t b = zsplit_level(P, P->t_sdiag, l, mid, P->sdiag_cut[l]);
            P->zsd_slots = std::max(P->zsd_slots, std::max(a, b));
        }
        P->t_zero_off[l + 1] = (int64_t)P->t_zero.size();
        // diagonal blocks of the tiled path by width class (one launch each)
        const int64_t cls[] = {32, 64, 1 << 30};
        for (int k = 0; k < 3; k++) {
            for (int B : lv[l]) {
                const BlockDesc& d = P->blocks[B];
                if (small_block(d.s, d.c) || d.s > cls[k] || (k > 0 && d.s <= cls[k - 1])) continue;
                P->t_ldlt.tasks.push_back({B, 0, 0, 0, 0, 0, 0, 0});
            }
            if (k < 2) P->ldlt_cut[2 * l + k] = (int64_t)P->t_ldlt.tasks.size();
        }
        for (LevelTasks* t : all) t->off[l + 1] = (int64_t)t->tasks.size();
    }
    // algorithmic work of one factor / invert / backward call, per kernel kind
    P->work_flops.assign(kNumKinds, 0.0);
    P->work_bytes.assign(kNumKinds, 0.0);
    for (const BlockDesc& d : P->blocks) {
        const double s = d.s, c = d.c;
        const double fl[] = {s * s * s, 2.0 * c * s * s, c * c * s, 2.0 * c * c * s, 2.0 * c * s * s};
        const double by[] = {8.0 * 3 * s * s, 8.0 * (2 * c * s + s * s), 8.0 * (c * s + c * (c + 1) / 2),
                             8.0 * (c * (c + 1) / 2 + 2 * c * s), 8.0 * (2 * c * s + 2 * s * s)};
        // sweep: s pivots x s^2 updates; L_hat = F(C,B) T; lower half of
        // L_hat F^T; X = -G L_hat; Y = T - L_hat^T X
        if (small_block(d.s, d.c)) {
            P->work_flops[kSbFactor] += fl[0] + fl[1] + fl[2];
            P->work_bytes[kSbFactor] += by[0] + by[1] + by[2];
            P->work_flops[kSbInvert] += fl[3] + fl[4];
            P->work_bytes[kSbInvert] += by[3] + by[4];
        } else {
            const Kind k[] = {kLdlt, kPanel, kSchur, kGemm, kSdiag};
            for (int q = 0; q < 5; q++) {
                P->work_flops[k[q]] += fl[q];
                P->work_bytes[k[q]] += by[q];
            }
        }
        P->work_flops[kQFactor] += fl[0] + fl[1] + fl[2];
        P->work_bytes[kQFactor] += by[0] + by[1] + by[2];
        P->work_flops[kQInvert] += fl[3] + fl[4];
        P->work_bytes[kQInvert] += by[3] + by[4];
        // reverse selected inversion: Xbar (2cs^2), Lhat_bar (2c^2 s + 2cs^2),
        // symmetric scatter of -(Xbar L_hat^T + L_hat Xbar^T) (2c^2 s, lower half)
        P->work_flops[kRevSel] += 4.0 * c * c * s + 4.0 * c * s * s;
        P->work_bytes[kRevSel] += 8.0 * (c * (c + 1) + 6 * c * s + s * s);
        // reverse factor: Ubar F (c^2 s), Ubar^T L_hat + Lhat_bar T (c^2 s + 2cs^2),
        // F^T Lhat_bar (2cs^2), -T (Tbar + Tbar^T) T (4 s^3)
        P->work_flops[kRevFac] += 2.0 * c * c * s + 4.0 * c * s * s + 4.0 * s * s * s;
        P->work_bytes[kRevFac] += 8.0 * (c * (c + 1) + 6 * c * s + 4 * s * s);
    }
    const double nnzL = (double)P->colptrL.back(), nnzA = (double)P->nnzA;
    P->work_bytes[kAssemble] = 8.0 * P->arena + 24.0 * nnzA;
    P->work_bytes[kExport] = 24.0 * nnzL;
    // checkpoint slots: whole inverse panels of levels 1, 1 + k, 1 + 2k, ...
    const int k = std::max(1, (int)P->opts.checkpoint_every);
    P->ck_off.assign(P->blocks.size(), -1);
    P->ck_size = 0;
    if (k > 1)
        for (size_t B = 0; B < P->blocks.size(); B++) {
            const BlockDesc& d = P->blocks[B];
            if ((d.level - 1) % k != 0) continue;
            P->ck_off[B] = P->ck_size;
            P->ck_size += ((int64_t)d.s + d.c) * d.s;
        }
    P->work_bytes[kCheckpoint] = 16.0 * (double)P->ck_size;
}

// ---------------------------------------------------------------------------
// Work queues of the persistent level kernels.  One queue per level and
// sweep holds the level's tasks of every block (and, in a batch, of every
// matrix) in phase order; `pad` counts the earlier tasks of the same block
// that must have finished.  A work-group only ever waits on tasks with a
// smaller queue index, which were claimed before it by running work-groups,
// so the queue drains whatever the residency.
// ---------------------------------------------------------------------------
static double block_cost(const BlockDesc& d)
{
    const double s = d.s, c = d.c;
    return 2 * c * c * s + 2 * c * s * s + s * s * s;
}

// blocks of one level in the queue order of `order`
static void order_blocks(const selinv_plan_s* P, int order, std::vector<int>& bl)
{
    if (order == qoLpt || order == qoTileLpt) {
        std::stable_sort(bl.begin(), bl.end(),
                         [&](int a, int b) { return block_cost(P->blocks[a]) > block_cost(P->blocks[b]); });
    } else if (order == qoRoundRobin && !P->blk_matrix.empty()) {
        // i-th block of every matrix in turn
        std::vector<int> rank(bl.size());
        int last = -1, r = 0;
        for (size_t q = 0; q < bl.size(); q++) {  // bl is ascending, so matrix-major
            const int m = P->blk_matrix[bl[q]];
            r = (m == last) ? r + 1 : 0;
            last = m;
            rank[q] = r;
        }
        std::vector<size_t> idx(bl.size());
        for (size_t q = 0; q < idx.size(); q++) idx[q] = q;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return rank[a] < rank[b]; });
        std::vector<int> out(bl.size());
        for (size_t q = 0; q < idx.size(); q++) out[q] = bl[idx[q]];
        bl.swap(out);
    }
}

static double task_cost(const Task& t)
{
    const int op = t.flags >> 8;
    if (op == qSbFactor || op == qSbInvert) return 0.0;  // groups keep their block order
    if (op == qMbFactor || op == qMbInvert) return 1e30;  // whole blocks: before the tiles
    if (op == qSchur) return (double)t.ke * kSchurTile * kSchurTile;
    if (op == qSdiag) return 2.0 * (t.ke - t.kb) * kDiagTile * kDiagTile;
    return (double)(t.ke - t.kb) * t.bn * kTileM;
}

void build_queues(const selinv_plan_s* P, const Sched& sc, std::vector<Task>& qf, std::vector<int64_t>& qf_off,
                  std::vector<Task>& qi, std::vector<int64_t>& qi_off)
{
    std::vector<std::vector<int>> lv;
    by_level(P, lv);
    const int D = (int)lv.size();
    qf.clear();
    qi.clear();
    qf_off.assign(D + 1, 0);
    qi_off.assign(D + 1, 0);
    const int cap = std::max(16, std::min(128, sc.bn_cap));
    auto bn_of = [&](int s) { return std::min(tile_bn(s), cap); };
    std::vector<Task> ph[3];
    std::vector<int32_t> touch((size_t)P->n, 0);
    std::vector<char> excl(P->blocks.size(), 0);
    auto flush = [&](std::vector<Task>& q) {
        for (auto& p : ph) {
            if (sc.order == qoTileLpt)
                std::stable_sort(p.begin(), p.end(), [](const Task& a, const Task& b) { return task_cost(a) > task_cost(b); });
            q.insert(q.end(), p.begin(), p.end());
            p.clear();
        }
    };
    for (int l = 0; l < D; l++) {
        std::vector<int> bl = lv[l];
        order_blocks(P, sc.order, bl);
        exclusive_blocks(P, bl, touch, excl);
        std::vector<int> small, medium, big;
        for (int B : bl) {
            const BlockDesc& d = P->blocks[B];
            const int bn = bn_of(d.s);
            const int64_t tiles = (int64_t)((d.c + kTileM - 1) / kTileM) * ((d.s + bn - 1) / bn);
            if (is_small(d.s, d.c, sc.small_s)) small.push_back(B);
            else if (tiles <= sc.mb_tiles) medium.push_back(B);
            else big.push_back(B);
        }
        // factor: small blocks whole on a wave, medium ones whole on a
        // work-group; big ones as diagonal block, then L_hat tiles, then
        // Schur tiles
        push_sb_groups(small, qSbFactor, ph[0]);
        for (int B : medium)
            ph[0].push_back({B, 0, 0, bn_of(P->blocks[B].s), 0, 0, q_flags(qMbFactor, excl[B] ? 4 : 0), 0});
        for (int B : big) {
            const BlockDesc& d = P->blocks[B];
            const int bn = bn_of(d.s);
            const int npanel = ((d.c + kTileM - 1) / kTileM) * ((d.s + bn - 1) / bn);
            ph[0].push_back({B, 0, 0, 0, 0, 0, q_flags(qLdlt, npanel > 0 ? 2 : 0), 0});
            for (int j = 0; j < d.s; j += bn)
                for (int r = 0; r < d.c; r += kTileM) ph[1].push_back({B, r, j, bn, 0, d.s, q_flags(qPanel, 2), 1});
            for (int k = 0; k < d.c; k += kSchurTile)
                for (int i = k; i < d.c; i += kSchurTile)
                    ph[2].push_back({B, i, k, kSchurTile, 0, d.s, q_flags(qSchur, excl[B] ? 4 : 0), 1 + npanel});
        }
        flush(qf);
        qf_off[l + 1] = (int64_t)qf.size();
        // inversion: small blocks whole; big ones as zero X (split blocks),
        // then X tiles, then diagonal tiles
        int64_t base = 0, dbase = 0;
        for (int B : big) {
            const BlockDesc& d = P->blocks[B];
            base += (int64_t)((d.c + kTileM - 1) / kTileM) * ((d.s + bn_of(d.s) - 1) / bn_of(d.s));
            const int nd = (d.s + kDiagTile - 1) / kDiagTile;
            dbase += nd * (nd + 1) / 2;
        }
        const int64_t fill = sc.split_fill;
        const int64_t want = fill > 0 && base > 0 && base < fill ? (fill + base - 1) / base : 1;
        const int64_t dwant = fill > 0 && dbase > 0 && dbase < fill ? (fill + dbase - 1) / dbase : 1;
        push_sb_groups(small, qSbInvert, ph[0]);
        for (int B : medium) ph[0].push_back({B, 0, 0, bn_of(P->blocks[B].s), 0, 0, q_flags(qMbInvert, 0), 0});
        for (int B : big) {
            const BlockDesc& d = P->blocks[B];
            const int bn = bn_of(d.s);
            const int split = split_for(want, d.c);
            const int dsplit = split_for(dwant, d.c);
            const int nz = (split > 1 || dsplit > 1) ? 1 : 0;
            if (nz) ph[0].push_back({B, 0, 0, 0, 0, 0, q_flags(qZero, 2), 0});
            int ng = 0;
            for (int j = 0; j < d.s; j += bn)
                for (int r = 0; r < d.c; r += kTileM)
                    pieces(0, d.c, split, [&](int kb, int ke, int) {
                        ph[1].push_back({B, r, j, bn, kb, ke, q_flags(qGemm, (split > 1) | 2), nz});
                        ng++;
                    });
            const int nd = (d.s + kDiagTile - 1) / kDiagTile;
            for (int I = 0; I < nd; I++)
                for (int J = 0; J <= I; J++)
                    pieces(0, d.c, dsplit, [&](int kb, int ke, int) {
                        ph[2].push_back({B, I * kDiagTile, J * kDiagTile, 0, kb, ke, q_flags(qSdiag, dsplit > 1), nz + ng});
                    });
        }
        flush(qi);
        qi_off[l + 1] = (int64_t)qi.size();
    }
}

void queue_bound(const selinv_plan_s* P, int64_t& nfac, int64_t& ninv)
{
    // per block, whatever the schedule: one small-block, medium-block or
    // diagonal task; output tiles at most as many as with 16-column tiles;
    // each contraction in at most split_for's cap of pieces
    nfac = ninv = 0;
    for (const BlockDesc& d : P->blocks) {
        const int64_t rows = (d.c + kTileM - 1) / kTileM, nsc = (d.c + kSchurTile - 1) / kSchurTile;
        const int64_t tiles = rows * ((d.s + 15) / 16);
        const int64_t nd = (d.s + kDiagTile - 1) / kDiagTile;
        const int64_t ms = std::max(1, ((d.c + 15) / 16) / (kMinSplitK / 16));
        nfac += 1 + tiles + nsc * (nsc + 1) / 2;
        ninv += 1 + tiles * ms + nd * (nd + 1) / 2 * ms;
    }
}

}  // namespace selinv
