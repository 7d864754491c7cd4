// Host symbolic phase: ordering, elimination tree, column counts,
// fundamental supernodes, supernodal row structures, execution blocks,
// priority levels (Algorithm 2), block index maps and the assemble/export
// maps used by the device kernels.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "plan.hpp"

namespace selinv {

// ---------------------------------------------------------------------------
// Nested dissection of a grid box.  Boxes are split across their longest
// axis (ties to the lowest axis) at lo + floor(extent/2); the order is the
// left box, the right box, then the separator plane with points in
// lexicographic order (x fastest) or, with rim_last, its interior points
// first and then its rim (points with a coordinate along another axis of
// the grid, one of more than one point, at the box's first or last value),
// each lexicographic.  dofs unknowns per point stay
// together.  Implemented as an explicit post-order walk of the bisection
// tree.
// ---------------------------------------------------------------------------
namespace {
struct Box {
    int32_t lo[3], hi[3];
    bool empty() const { return hi[0] <= lo[0] || hi[1] <= lo[1] || hi[2] <= lo[2]; }
};
}  // namespace

void nd_order_box(int ndim, const int32_t dims[3], int dofs, int rim_last, std::vector<int32_t>& perm)
{
    int32_t full[3] = {1, 1, 1};
    for (int d = 0; d < ndim && d < 3; d++) full[d] = dims[d];
    int64_t npts = (int64_t)full[0] * full[1] * full[2];
    perm.clear();
    perm.reserve((size_t)(npts * dofs));
    struct Frame {
        Box b;
        int stage;  // 0: descend left, 1: descend right, 2: emit separator
        int axis, mid;
    };
    std::vector<Frame> st;
    Box root{{0, 0, 0}, {full[0], full[1], full[2]}};
    if (!root.empty()) st.push_back({root, 0, 0, 0});
    while (!st.empty()) {
        Frame& f = st.back();
        if (f.stage == 0) {
            int ax = 0;
            for (int d = 1; d < 3; d++)
                if (f.b.hi[d] - f.b.lo[d] > f.b.hi[ax] - f.b.lo[ax]) ax = d;
            f.axis = ax;
            f.mid = f.b.lo[ax] + (f.b.hi[ax] - f.b.lo[ax]) / 2;
            f.stage = 1;
            Box l = f.b;
            l.hi[ax] = f.mid;
            if (!l.empty()) { st.push_back({l, 0, 0, 0}); continue; }
        }
        if (f.stage == 1) {
            f.stage = 2;
            Box r = f.b;
            r.lo[f.axis] = f.mid + 1;
            if (!r.empty()) { st.push_back({r, 0, 0, 0}); continue; }
        }
        // stage 2: separator plane (pass 0 interior, pass 1 rim when rim_last)
        Box s = f.b;
        s.lo[f.axis] = f.mid;
        s.hi[f.axis] = f.mid + 1;
        const int ax = f.axis;
        for (int pass = rim_last ? 0 : 1; pass < 2; pass++)
            for (int32_t z = s.lo[2]; z < s.hi[2]; z++)
                for (int32_t y = s.lo[1]; y < s.hi[1]; y++)
                    for (int32_t x = s.lo[0]; x < s.hi[0]; x++) {
                        if (rim_last) {
                            const int32_t p3[3] = {x, y, z};
                            bool rim = false;
                            for (int d = 0; d < 3; d++)
                                if (d != ax && full[d] > 1 && (p3[d] == f.b.lo[d] || p3[d] == f.b.hi[d] - 1))
                                    rim = true;
                            if (rim != (pass == 1)) continue;
                        }
                        int64_t pt = x + (int64_t)full[0] * (y + (int64_t)full[1] * z);
                        for (int k = 0; k < dofs; k++) perm.push_back((int32_t)(pt * dofs + k));
                    }
        st.pop_back();
    }
}

// Priority numbers of Algorithm 2 for a block tree whose parents have larger
// indices: roots get 1, every other block its parent's number plus one.
static void priority_levels(Partition& P)
{
    int N = P.nblocks();
    P.lev.assign(N, 0);
    P.depth = 0;
    for (int K = N - 1; K >= 0; K--) {
        P.lev[K] = P.par[K] < 0 ? 1 : P.lev[P.par[K]] + 1;
        P.depth = std::max(P.depth, P.lev[K]);
    }
}

// Block index maps: for block K, each ancestor J met by C(K) (ascending), the
// positions of C(K)[a..c) inside rows(J) = cols(J) U C(J), by a merge of the
// two sorted lists.  Layout per segment: [J, a, pos...].
void block_index_maps(const Partition& P, std::vector<int64_t>& rptr, std::vector<int32_t>& rel)
{
    int N = P.nblocks();
    rptr.assign(N + 1, 0);
    for (int K = 0; K < N; K++) {
        const int32_t* C = P.C(K);
        int c = P.clen(K);
        int64_t tot = 0;
        int r = 0;
        while (r < c) {
            int J = P.of[C[r]];
            tot += 2 + (c - r);
            int e = r;
            while (e < c && C[e] < P.xs[J + 1]) e++;
            r = e;
        }
        rptr[K + 1] = rptr[K] + tot;
    }
    rel.assign((size_t)rptr[N], 0);
    for (int K = 0; K < N; K++) {
        const int32_t* C = P.C(K);
        int c = P.clen(K);
        int64_t q = rptr[K];
        int r = 0;
        while (r < c) {
            int J = P.of[C[r]];
            rel[q++] = J;
            rel[q++] = r;
            int fJ = P.xs[J], lJ = P.xs[J + 1];
            const int32_t* CJ = P.C(J);
            int cJ = P.clen(J), sJ = lJ - fJ;
            int u = 0;  // cursor in C(J)
            for (int t = r; t < c; t++) {
                int x = C[t];
                int pos;
                if (x < lJ) {
                    pos = x - fJ;
                } else {
                    while (u < cJ && CJ[u] < x) u++;
                    pos = (u < cJ && CJ[u] == x) ? sJ + u : -1;
                }
                rel[q++] = pos;
            }
            int e = r;
            while (e < c && C[e] < lJ) e++;
            r = e;
        }
    }
}

static int64_t pos_in_rows(const Partition& P, int K, int32_t x)
{
    int f = P.xs[K], l = P.xs[K + 1];
    if (x >= f && x < l) return x - f;
    const int32_t* C = P.C(K);
    int c = P.clen(K);
    const int32_t* it = std::lower_bound(C, C + c, x);
    if (it == C + c || *it != x) return -1;
    return (l - f) + (it - C);
}

selinv_status analyze(selinv_plan_s* P, const selinv_geom* geom, const int32_t* perm_or_null,
                      std::string& err)
{
    const int64_t n = P->n;
    const int32_t cap = P->opts.max_super > 0 ? P->opts.max_super : (int32_t)std::max<int64_t>(n, 1);
    const int32_t ecap = P->opts.exec_cap > 0 ? P->opts.exec_cap : cap;
    // ---- ordering
    if (perm_or_null) {
        P->perm.assign(perm_or_null, perm_or_null + n);
    } else if (geom && geom->ndim > 0) {
        int32_t d3[3] = {geom->dims[0], geom->ndim > 1 ? geom->dims[1] : 1, geom->ndim > 2 ? geom->dims[2] : 1};
        int dofs = geom->dofs_per_point > 0 ? geom->dofs_per_point : 1;
        nd_order_box(geom->ndim, d3, dofs, P->opts.sep_order, P->perm);
        if ((int64_t)P->perm.size() != n) {
            err = "geometry does not match n";
            return SELINV_EINVAL;
        }
    } else {
        P->perm.resize(n);
        std::iota(P->perm.begin(), P->perm.end(), 0);
    }
    P->iperm.assign(n, -1);
    for (int64_t k = 0; k < n; k++) {
        int32_t o = P->perm[k];
        if (o < 0 || o >= n || P->iperm[o] != -1) {
            err = "permutation is not a bijection";
            return SELINV_EINVAL;
        }
        P->iperm[o] = (int32_t)k;
    }
    // ---- permuted pattern: lower entries by column (collist) and by row (rowlist)
    std::vector<int64_t> cl_ptr(n + 1, 0), rl_ptr(n + 1, 0);
    const int64_t* cp = P->colptr.data();
    const int32_t* ri = P->rowind.data();
    for (int64_t j = 0; j < n; j++)
        for (int64_t p = cp[j]; p < cp[j + 1]; p++) {
            int32_t a = P->iperm[ri[p]], b = P->iperm[j];
            if (a == b) continue;
            int32_t lo = std::max(a, b), hi = std::min(a, b);
            cl_ptr[hi + 1]++;
            rl_ptr[lo + 1]++;
        }
    for (int64_t j = 0; j < n; j++) {
        cl_ptr[j + 1] += cl_ptr[j];
        rl_ptr[j + 1] += rl_ptr[j];
    }
    std::vector<int32_t> cl(cl_ptr[n]), rl(rl_ptr[n]);
    {
        std::vector<int64_t> fc(cl_ptr.begin(), cl_ptr.end() - 1), fr(rl_ptr.begin(), rl_ptr.end() - 1);
        for (int64_t j = 0; j < n; j++)
            for (int64_t p = cp[j]; p < cp[j + 1]; p++) {
                int32_t a = P->iperm[ri[p]], b = P->iperm[j];
                if (a == b) continue;
                int32_t lo = std::max(a, b), hi = std::min(a, b);
                cl[fc[hi]++] = lo;
                rl[fr[lo]++] = hi;
            }
    }
    // ---- elimination tree (Liu's algorithm with path compression)
    P->parent.assign(n, -1);
    {
        std::vector<int32_t> anc(n, -1);
        for (int64_t j = 0; j < n; j++)
            for (int64_t p = rl_ptr[j]; p < rl_ptr[j + 1]; p++) {
                int32_t r = rl[p];
                while (anc[r] != -1 && anc[r] != j) {
                    int32_t t = anc[r];
                    anc[r] = (int32_t)j;
                    r = t;
                }
                if (anc[r] == -1) {
                    anc[r] = (int32_t)j;
                    P->parent[r] = (int32_t)j;
                }
            }
    }
    // ---- column counts by row subtrees: L(i,k) != 0 iff k lies on a tree
    //      path from some j with B(i,j) != 0 up to i.
    P->cnt.assign(n, 0);
    {
        std::vector<int32_t> mark(n, -1);
        for (int64_t i = 0; i < n; i++) {
            mark[i] = (int32_t)i;
            for (int64_t p = rl_ptr[i]; p < rl_ptr[i + 1]; p++)
                for (int32_t k = rl[p]; k >= 0 && mark[k] != i; k = P->parent[k]) {
                    mark[k] = (int32_t)i;
                    P->cnt[k]++;
                }
        }
    }
    // ---- fundamental supernodes, split at `cap` columns
    std::vector<int32_t> nchild(n + 1, 0);
    for (int64_t j = 0; j < n; j++)
        if (P->parent[j] >= 0) nchild[P->parent[j]]++;
    Partition& F = P->fund;
    F.xs.clear();
    if (n > 0) F.xs.push_back(0);
    for (int64_t j = 0; j + 1 < n; j++) {
        bool join = P->parent[j] == j + 1 && nchild[j + 1] == 1 && P->cnt[j] == P->cnt[j + 1] + 1 &&
                    (j + 1 - F.xs.back()) < cap;
        if (!join) F.xs.push_back((int32_t)(j + 1));
    }
    F.xs.push_back((int32_t)n);
    int32_t N = F.nblocks();
    F.of.assign(n, 0);
    for (int K = 0; K < N; K++)
        for (int j = F.xs[K]; j < F.xs[K + 1]; j++) F.of[j] = K;
    F.par.assign(N, -1);
    for (int K = 0; K < N; K++) {
        int32_t p = P->parent[F.xs[K + 1] - 1];
        F.par[K] = p >= 0 ? F.of[p] : -1;
    }
    priority_levels(F);
    // ---- supernodal row structures: C(K) = rows of A below K U children's C
    {
        std::vector<int32_t> head(N, -1), next(N, -1);
        for (int K = 0; K < N; K++)
            if (F.par[K] >= 0) {
                next[K] = head[F.par[K]];
                head[F.par[K]] = K;
            }
        F.cptr.assign(N + 1, 0);
        for (int K = 0; K < N; K++) F.cptr[K + 1] = F.cptr[K] + P->cnt[F.xs[K + 1] - 1];
        F.crows.assign((size_t)F.cptr[N], 0);
        std::vector<int32_t> mark(n, -1), buf;
        for (int K = 0; K < N; K++) {
            int32_t last = F.xs[K + 1] - 1;
            buf.clear();
            for (int32_t j = F.xs[K]; j <= last; j++)
                for (int64_t p = cl_ptr[j]; p < cl_ptr[j + 1]; p++) {
                    int32_t x = cl[p];
                    if (x > last && mark[x] != K) { mark[x] = K; buf.push_back(x); }
                }
            for (int Q = head[K]; Q >= 0; Q = next[Q]) {
                const int32_t* CQ = F.C(Q);
                for (int t = 0; t < F.clen(Q); t++) {
                    int32_t x = CQ[t];
                    if (x > last && mark[x] != K) { mark[x] = K; buf.push_back(x); }
                }
            }
            std::sort(buf.begin(), buf.end());
            if ((int64_t)buf.size() != F.clen(K)) {
                err = "internal: supernode structure does not match column counts";
                return SELINV_EINVAL;
            }
            std::copy(buf.begin(), buf.end(), F.crows.begin() + F.cptr[K]);
        }
    }
    // ---- execution blocks.  Fundamental supernodes wider than ecap are cut
    //      into pieces of at most ecap columns (a piece is a supernode whose
    //      rows below are the rest of its supernode plus C(K)); then chains
    //      of single-child pieces run as one amalgamated block with
    //      rows(B) = cols(B) U C(top piece of the chain).
    Partition& E = P->exec;
    std::vector<int32_t> nsch(N, 0);
    for (int K = 0; K < N; K++)
        if (F.par[K] >= 0) nsch[F.par[K]]++;
    std::vector<int32_t> topK, topEnd;  // exec block -> top supernode, end column of its top piece
    E.xs.clear();
    for (int K = 0; K < N; K++) {
        const int32_t f = F.xs[K], l = F.xs[K + 1];
        for (int32_t a = f; a < l; a += ecap) {
            const int32_t b = std::min(l, a + ecap);
            // the previous piece is this piece's only child: within K always,
            // at K's first piece when K-1 is K's only child
            bool chain = a > f || (K > 0 && F.par[K - 1] == K && nsch[K] == 1);
            bool join = !E.xs.empty() && P->opts.fuse_chains && chain && (b - E.xs.back()) <= ecap;
            if (join) {
                topK.back() = K;
                topEnd.back() = b;
            } else {
                E.xs.push_back(a);
                topK.push_back(K);
                topEnd.push_back(b);
            }
        }
    }
    E.xs.push_back((int32_t)n);
    int32_t NB = E.nblocks();
    E.of.assign(n, 0);
    for (int B = 0; B < NB; B++)
        for (int j = E.xs[B]; j < E.xs[B + 1]; j++) E.of[j] = B;
    E.par.assign(NB, -1);
    E.cptr.assign(NB + 1, 0);
    for (int B = 0; B < NB; B++) {
        const int K = topK[B];
        const int32_t e = topEnd[B], l = F.xs[K + 1];
        if (e < l) E.par[B] = E.of[e];                          // next piece of the same supernode
        else E.par[B] = F.par[K] >= 0 ? E.of[F.xs[F.par[K]]] : -1;
        E.cptr[B + 1] = E.cptr[B] + (l - e) + F.clen(K);
    }
    E.crows.resize((size_t)E.cptr[NB]);
    for (int B = 0; B < NB; B++) {
        const int K = topK[B];
        int64_t q = E.cptr[B];
        for (int32_t x = topEnd[B]; x < F.xs[K + 1]; x++) E.crows[q++] = x;
        std::copy(F.C(K), F.C(K) + F.clen(K), E.crows.begin() + q);
    }
    priority_levels(E);
    // ---- the reported partition: the fundamental supernodes, or with
    //      `relaxed` the execution blocks themselves (their explicit zeros
    //      become part of the reported pattern)
    if (P->opts.relaxed) {
        F = E;
        N = F.nblocks();
    }
    // ---- canonical pattern: per column j of block K, j, the later columns
    //      of K, then C(K) (for fundamental supernodes: j and struct(j))
    P->colptrL.assign(n + 1, 0);
    for (int K = 0; K < N; K++)
        for (int32_t j = F.xs[K]; j < F.xs[K + 1]; j++)
            P->colptrL[j + 1] = (F.xs[K + 1] - j) + F.clen(K);
    for (int64_t j = 0; j < n; j++) P->colptrL[j + 1] += P->colptrL[j];
    P->rowindL.resize((size_t)P->colptrL[n]);
    for (int K = 0; K < N; K++) {
        int32_t f = F.xs[K], l = F.xs[K + 1];
        for (int32_t j = f; j < l; j++) {
            int64_t q = P->colptrL[j];
            for (int32_t i = j; i < l; i++) P->rowindL[q++] = i;
            for (int t = 0; t < F.clen(K); t++) P->rowindL[q++] = F.C(K)[t];
        }
    }
    // ---- execution-block device tables
    P->blocks.resize(NB);
    int64_t poff = 0, hoff = 0, woff = 0;
    for (int B = 0; B < NB; B++) {
        BlockDesc& d = P->blocks[B];
        d.first = E.xs[B];
        d.s = E.width(B);
        d.c = E.clen(B);
        d.level = E.lev[B];
        d.poff = poff;
        d.hoff = hoff;
        d.woff = woff;
        d.coff = E.cptr[B];
        poff += (int64_t)(d.s + d.c) * d.s;
        hoff += (int64_t)d.c * d.s;
        woff += (int64_t)d.s * d.s;
    }
    P->arena = poff;
    P->harena = hoff;
    P->warena = woff;
    P->crow = E.crows;
    {
        std::vector<int64_t> rptr;
        block_index_maps(E, rptr, P->rel);
        // compact the records: drop the [J, a] headers, keep positions only
        std::vector<int32_t> pos;
        pos.reserve(P->rel.size());
        P->cbase.assign(E.crows.size(), 0);
        P->rbase.assign(E.crows.size(), 0);
        for (int B = 0; B < NB; B++) {
            int c = E.clen(B);
            int64_t q = rptr[B];
            while (q < rptr[B + 1]) {
                int J = P->rel[q], a = P->rel[q + 1];
                int64_t start = (int64_t)pos.size();
                for (int t = a; t < c; t++) {
                    int32_t v = P->rel[q + 2 + (t - a)];
                    if (v < 0) {
                        err = "internal: block index map incomplete";
                        return SELINV_EINVAL;
                    }
                    pos.push_back(v);
                }
                q += 2 + (c - a);
                int lJ = E.xs[J + 1];
                const BlockDesc& dj = P->blocks[J];
                int64_t ldJ = dj.s + dj.c;
                for (int t = a; t < c && E.C(B)[t] < lJ; t++) {
                    int64_t cpos = E.cptr[B] + t;
                    P->cbase[cpos] = dj.poff + (int64_t)(E.C(B)[t] - dj.first) * ldJ;
                    P->rbase[cpos] = start - a;
                }
            }
        }
        P->rel.swap(pos);
    }
    // ---- assemble map: original CSC entry -> arena offset
    P->asm_off.resize((size_t)P->nnzA);
    for (int64_t j = 0; j < n; j++)
        for (int64_t p = cp[j]; p < cp[j + 1]; p++) {
            int32_t a = P->iperm[ri[p]], b = P->iperm[j];
            int32_t lo = std::max(a, b), hi = std::min(a, b);
            int B = E.of[hi];
            int64_t r = pos_in_rows(E, B, lo);
            if (r < 0) {
                err = "internal: entry of A outside the pattern of L";
                return SELINV_EINVAL;
            }
            const BlockDesc& d = P->blocks[B];
            P->asm_off[p] = d.poff + r + (int64_t)(hi - d.first) * (d.s + d.c);
        }
    P->colblk = E.of;
    // ---- export map: canonical entry of L -> arena offset
    P->exp_off.resize(P->rowindL.size());
    for (int64_t j = 0; j < n; j++) {
        int B = E.of[j];
        const BlockDesc& d = P->blocks[B];
        int64_t colbase = d.poff + (int64_t)(j - d.first) * (d.s + d.c);
        for (int64_t q = P->colptrL[j]; q < P->colptrL[j + 1]; q++) {
            int64_t r = pos_in_rows(E, B, P->rowindL[q]);
            if (r < 0) {
                err = "internal: entry of L outside its execution block";
                return SELINV_EINVAL;
            }
            P->exp_off[q] = colbase + r;
        }
    }
    // ---- every offset the kernels will dereference stays inside its arena
    for (int64_t v : P->asm_off)
        if (v < 0 || v >= P->arena) { err = "internal: assemble map out of range"; return SELINV_EINVAL; }
    for (int64_t v : P->exp_off)
        if (v < 0 || v >= P->arena) { err = "internal: export map out of range"; return SELINV_EINVAL; }
    for (int B = 0; B < NB; B++) {
        const BlockDesc& d = P->blocks[B];
        for (int k = 0; k < d.c; k++) {
            int64_t pk = d.coff + k;
            int64_t lo = P->rbase[pk] + k, hi = P->rbase[pk] + d.c - 1;
            if (lo < 0 || hi >= (int64_t)P->rel.size()) { err = "internal: index map range"; return SELINV_EINVAL; }
            int J = E.of[E.C(B)[k]];
            const BlockDesc& dj = P->blocks[J];
            if (P->cbase[pk] < dj.poff || P->cbase[pk] >= dj.poff + (int64_t)(dj.s + dj.c) * dj.s) {
                err = "internal: column base out of range";
                return SELINV_EINVAL;
            }
            for (int i = k; i < d.c; i++) {
                int32_t r = P->rel[P->rbase[pk] + i];
                if (r < 0 || r >= dj.s + dj.c) { err = "internal: relative row out of range"; return SELINV_EINVAL; }
            }
        }
    }
    // ---- work counts
    selinv_info& I = P->info;
    I = selinv_info{};
    I.n = n;
    I.nnzA = P->nnzA;
    I.nnzL = P->colptrL[n];
    I.nsuper = N;
    I.depth = F.depth;
    I.nblocks = NB;
    I.exec_depth = E.depth;
    for (int K = 0; K < N; K++) {
        double s = F.width(K), c = F.clen(K);
        I.flops_factor += c * c * s + c * s * s + s * s * s / 3.0;
        I.flops_gemm += 2 * c * c * s + 2 * c * s * s;
        I.flops_selinv += 2 * c * c * s + 3 * c * s * s + 2.0 / 3.0 * s * s * s;
        I.gather_bytes += 8.0 * c * (c + 1) / 2;
    }
    for (int B = 0; B < NB; B++) {
        double s = E.width(B), c = E.clen(B);
        I.exec_flops_gemm += 2 * c * c * s + 2 * c * s * s;
    }
    return SELINV_OK;
}

}  // namespace selinv
