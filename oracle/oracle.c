/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for supernodal selected inversion
 * (Jacquelin, Lin, Yang: "PSelInv -- a distributed memory parallel algorithm
 * for selected inversion: the symmetric case", ACM TOMS).  Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or table with the HIP
 * library: both sides only read the same generated matrices.
 *
 * Tiers:
 *   O1  orc_dense_inverse   -- A^{-1} by an LDL^T factorization and n
 *                              triangular solves (Section 2.1, the
 *                              "direct inversion" by triangular solves).
 *   O2  orc_selinv_columns  -- dense LDL^T then the scalar (column)
 *                              recurrence obtained from the 2x2 block form
 *                              (Section 2.1, the 2x2 block form of A^{-1}
 *                              with normalised factors).
 *   O3  orc_factor_selinv   -- supernodal LDL^T, then Algorithm 1 with the
 *                              symmetric simplifications of Section 2.1
 *                              (U_hat = L_hat^T, LDL^T diagonal term,
 *                              symmetrised diagonal block), root first.
 *   sym orc_symbolic        -- nested-dissection order (geometric reading),
 *                              column structures by definition, elimination
 *                              tree (Section 2.2), fundamental supernodes
 *                              capped in size (Section 2.1), priority
 *                              levels of Algorithm 2 and block index maps.
 *   grad orc_dense_grad     -- dense reference gradient of a weighted sum of
 *                              selected entries: -(A^{-1} S A^{-1}).
 *
 * Everything is FP64, round to nearest; no blocking or reordering beyond the
 * formulas.  OpenMP only splits independent loop iterations.
 *
 * Readings where the paper is silent:
 *   - ordering: recursive coordinate bisection of the grid box (longest axis,
 *     ties to the lowest axis, separator plane at lo + floor(ext/2); left
 *     half, right half, then the plane in lexicographic order, x fastest);
 *   - supernodes: fundamental (column j+1 joins j iff j is its only child and
 *     struct(j) = {j+1} U struct(j+1)), split when a supernode reaches `cap`;
 *   - D has 1x1 blocks, no pivoting (Section 4 uses none); a pivot that is
 *     zero, not finite, or (when SPD is required) not positive is reported.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;

/* Planted-mistake switch used only by the tests that show the pins catch
 * errors.  0 = correct code; the mistakes are listed where the tests plant
 * them (1-7 in the arithmetic and the symbolic phase, 8-9 in the export of
 * the factor, 10 in the complex tier, 11 in the pivoted tier). */
static int g_mut = 0;
void orc_set_mutation(int m) { g_mut = m; }
int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
/* threads of the following parallel regions (n > 0); returns the setting */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#endif
    return orc_get_threads();
}

/* ------------------------------------------------------------------ */
/* Nested dissection over a box of grid points                         */
/* ------------------------------------------------------------------ */
/* rim_last = 1 orders a separator plane's interior points before its rim
 * (the points with a coordinate along another grid axis of more than one
 * point at the box's first or last value), each part in lexicographic order */
static void nd_box(const int lo[3], const int hi[3], const int full[3], int dofs, int rim_last,
                   int* perm, i64* pos)
{
    int ext[3];
    for (int k = 0; k < 3; k++) ext[k] = hi[k] - lo[k];
    if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) return;
    int d = 0;
    for (int k = 1; k < 3; k++)
        if (ext[k] > ext[d]) d = k;
    int mid = lo[d] + ext[d] / 2;
    int l2[3], h2[3];
    memcpy(l2, lo, sizeof l2);
    memcpy(h2, hi, sizeof h2);
    h2[d] = mid;
    nd_box(l2, h2, full, dofs, rim_last, perm, pos);
    memcpy(h2, hi, sizeof h2);
    l2[d] = mid + 1;
    nd_box(l2, h2, full, dofs, rim_last, perm, pos);
    memcpy(l2, lo, sizeof l2);
    l2[d] = mid;
    h2[d] = mid + 1;
    for (int want_rim = 0; want_rim < 2; want_rim++) {
        if (!rim_last && want_rim == 0) continue;  /* one lexicographic pass */
        for (int z = l2[2]; z < h2[2]; z++)
            for (int y = l2[1]; y < h2[1]; y++)
                for (int x = l2[0]; x < h2[0]; x++) {
                    if (rim_last) {
                        int c3[3] = {x, y, z}, on_rim = 0;
                        for (int k = 0; k < 3; k++)
                            if (k != d && full[k] > 1 && (c3[k] == lo[k] || c3[k] == hi[k] - 1)) on_rim = 1;
                        if (on_rim != want_rim) continue;
                    }
                    i64 pt = (i64)x + (i64)full[0] * ((i64)y + (i64)full[1] * z);
                    for (int b = 0; b < dofs; b++) perm[(*pos)++] = (int)(pt * dofs + b);
                }
    }
}

/* perm[new] = old.  Returns the number of unknowns. */
i64 orc_nd_order_sep(int ndim, const int* dims, int dofs, int rim_last, int* perm)
{
    int full[3] = {1, 1, 1};
    for (int k = 0; k < ndim && k < 3; k++) full[k] = dims[k];
    int lo[3] = {0, 0, 0};
    i64 pos = 0;
    nd_box(lo, full, full, dofs, rim_last, perm, &pos);
    return pos;
}

i64 orc_nd_order(int ndim, const int* dims, int dofs, int* perm)
{
    return orc_nd_order_sep(ndim, dims, dofs, 0, perm);
}

/* ------------------------------------------------------------------ */
/* Symbolic analysis                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    int n, N, cap;
    int* perm;    /* new -> old */
    int* iperm;   /* old -> new */
    int* parent;  /* column elimination tree, -1 = root */
    i64* sptr;    /* struct(j) = srow[sptr[j] .. sptr[j+1]), rows > j, sorted */
    int* srow;
    int* xsuper;  /* supernode K = columns xsuper[K] .. xsuper[K+1]-1 */
    int* sn;      /* column -> supernode */
    int* sparent; /* supernodal tree */
    int* level;   /* priority number of Algorithm 2 (root = 1) */
    i64* poff;    /* panel offsets, panel K is (s+c) x s column-major */
    i64 arena;
    /* block index maps: per supernode a flat list of segments
     * [J, a, pos(C[a]), pos(C[a+1]), ..., pos(C[c-1])]; rptr[K] is where
     * K's list starts in the concatenation (the lists are built on demand,
     * map_build) */
    i64* rptr;
    int err;
} orc_sym;

static int cmp_int(const void* a, const void* b)
{
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

static inline int sn_s(const orc_sym* S, int K) { return S->xsuper[K + 1] - S->xsuper[K]; }
static inline const int* sn_C(const orc_sym* S, int K) { return S->srow + S->sptr[S->xsuper[K + 1] - 1]; }
static inline int sn_c(const orc_sym* S, int K)
{
    int j = S->xsuper[K + 1] - 1;
    return (int)(S->sptr[j + 1] - S->sptr[j]);
}

/* position of global row r in rows(J) = cols(J) U C(J); -1 if absent */
static int row_pos(const orc_sym* S, int J, int r)
{
    int f = S->xsuper[J], l = S->xsuper[J + 1];
    if (r >= f && r < l) return r - f;
    const int* C = sn_C(S, J);
    int c = sn_c(S, J);
    int lo = 0, hi = c;
    while (lo < hi) {
        int m = (lo + hi) / 2;
        if (C[m] < r) lo = m + 1; else hi = m;
    }
    if (lo < c && C[lo] == r) return (l - f) + lo;
    return -1;
}

/* first index q >= lo of the sorted array v[0..len) with v[q] >= r
 * (galloping from lo, then bisection) */
static int lower_from(const int* v, int len, int lo, int r)
{
    int step = 1, hi = lo;
    while (hi < len && v[hi] < r) { lo = hi + 1; hi += step; step *= 2; }
    if (hi > len) hi = len;
    while (lo < hi) {
        int m = (lo + hi) / 2;
        if (v[m] < r) lo = m + 1; else hi = m;
    }
    return lo;
}

/* Block index map of supernode K (Section 3.2, the relative indices of
 * C(K) inside each ancestor): for each ancestor J met in C(K), in ascending
 * order, the record [J, a, pos(C[a]), ..., pos(C[c-1])] with a the first
 * position of C(K) inside J's columns and pos(x) the row of x within
 * rows(J) = cols(J) U C(J).  Writes rptr[K+1] - rptr[K] ints to out. */
static void map_build(const orc_sym* S, int K, int* out)
{
    const int* C = sn_C(S, K);
    int c = sn_c(S, K);
    i64 q = 0;
    for (int r = 0; r < c;) {
        int J = S->sn[C[r]];
        int f = S->xsuper[J], l = S->xsuper[J + 1];
        const int* CJ = sn_C(S, J);
        int cJ = sn_c(S, J), lo = 0;
        out[q++] = J;
        out[q++] = r;
        for (int t = r; t < c; t++) {
            int x = C[t], p = -1;
            if (x >= f && x < l) {
                p = x - f;
            } else {
                lo = lower_from(CJ, cJ, lo, x);
                if (lo < cJ && CJ[lo] == x) p = (l - f) + lo;
            }
            out[q++] = p;
        }
        while (r < c && S->sn[C[r]] == J) r++;
    }
}

void orc_sym_free(orc_sym* S)
{
    if (!S) return;
    free(S->perm); free(S->iperm); free(S->parent); free(S->sptr); free(S->srow);
    free(S->xsuper); free(S->sn); free(S->sparent); free(S->level); free(S->poff);
    free(S->rptr);
    free(S);
}

/* Build the symbolic structure of L for the lower CSC pattern (colptr,
 * rowind) of A in original numbering, under perm (new -> old; NULL =
 * identity). */
static void relax_partition(orc_sym* S, int rcap);

/* As orc_symbolic; with rcap > 0 the supernodes are then relaxed (see
 * relax_partition) and every result (pattern, levels, maps, arena) refers to
 * the relaxed partition. */
orc_sym* orc_symbolic_relaxed(int n, const i64* colptr, const int* rowind, const int* perm, int cap, int rcap);

orc_sym* orc_symbolic(int n, const i64* colptr, const int* rowind, const int* perm, int cap)
{
    return orc_symbolic_relaxed(n, colptr, rowind, perm, cap, 0);
}

orc_sym* orc_symbolic_relaxed(int n, const i64* colptr, const int* rowind, const int* perm, int cap, int rcap)
{
    orc_sym* S = (orc_sym*)calloc(1, sizeof(orc_sym));
    S->n = n;
    S->cap = cap > 0 ? cap : n;
    S->perm = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    S->iperm = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int k = 0; k < n; k++) S->perm[k] = perm ? perm[k] : k;
    for (int k = 0; k < n; k++) S->iperm[k] = -1;
    for (int k = 0; k < n; k++) {
        int o = S->perm[k];
        if (o < 0 || o >= n || S->iperm[o] != -1) { S->err = 1; return S; }
        S->iperm[o] = k;
    }
    /* permuted off-diagonal lower pattern: adj[j] = {i > j : B_ij != 0} */
    i64 nnz = colptr[n];
    i64* acnt = (i64*)calloc((size_t)n + 1, sizeof(i64));
    for (int j = 0; j < n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            int i = rowind[p];
            if (i < j || i >= n) { S->err = 2; free(acnt); return S; }
            int a = S->iperm[i], b = S->iperm[j];
            if (a == b) continue;
            acnt[(a < b ? a : b) + 1]++;
        }
    for (int j = 0; j < n; j++) acnt[j + 1] += acnt[j];
    int* adj = (int*)malloc(sizeof(int) * (size_t)(acnt[n] + 1));
    i64* fill = (i64*)malloc(sizeof(i64) * ((size_t)n + 1));
    memcpy(fill, acnt, sizeof(i64) * ((size_t)n + 1));
    for (int j = 0; j < n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            int a = S->iperm[rowind[p]], b = S->iperm[j];
            if (a == b) continue;
            int lo = a < b ? a : b, hi = a < b ? b : a;
            adj[fill[lo]++] = hi;
        }
    free(fill);
    (void)nnz;

    /* column structures by definition (Section 2.2):
     * struct(j) = {i>j : B_ij != 0}  U  (U over children c of struct(c) \ {j}),
     * parent(j) = min struct(j). */
    S->parent = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    S->sptr = (i64*)malloc(sizeof(i64) * ((size_t)n + 1));
    i64 capw = (i64)acnt[n] * 2 + 16;
    S->srow = (int*)malloc(sizeof(int) * (size_t)capw);
    int* mark = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    int* buf = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    int* chead = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    int* cnext = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int j = 0; j < n; j++) { mark[j] = -1; chead[j] = -1; }
    S->sptr[0] = 0;
    for (int j = 0; j < n; j++) {
        int m = 0;
        for (i64 p = acnt[j]; p < acnt[j + 1]; p++) {
            int i = adj[p];
            if (mark[i] != j) { mark[i] = j; buf[m++] = i; }
        }
        if (g_mut != 7) {
            for (int ch = chead[j]; ch >= 0; ch = cnext[ch])
                for (i64 p = S->sptr[ch]; p < S->sptr[ch + 1]; p++) {
                    int i = S->srow[p];
                    if (i != j && mark[i] != j) { mark[i] = j; buf[m++] = i; }
                }
        }
        qsort(buf, (size_t)m, sizeof(int), cmp_int);
        if (S->sptr[j] + m > capw) {
            while (S->sptr[j] + m > capw) capw *= 2;
            S->srow = (int*)realloc(S->srow, sizeof(int) * (size_t)capw);
        }
        memcpy(S->srow + S->sptr[j], buf, sizeof(int) * (size_t)m);
        S->sptr[j + 1] = S->sptr[j] + m;
        S->parent[j] = m > 0 ? buf[0] : -1;
        if (m > 0) { cnext[j] = chead[buf[0]]; chead[buf[0]] = j; }
    }
    free(adj); free(acnt); free(mark); free(buf);

    /* fundamental supernodes, split at `cap` columns */
    int* nchild = (int*)calloc((size_t)n + 1, sizeof(int));
    for (int j = 0; j < n; j++)
        if (S->parent[j] >= 0) nchild[S->parent[j]]++;
    S->xsuper = (int*)malloc(sizeof(int) * ((size_t)n + 1));
    S->sn = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    int N = 0, start = 0;
    if (n > 0) S->xsuper[N++] = 0;
    for (int j = 0; j + 1 < n; j++) {
        int join = S->parent[j] == j + 1 && nchild[j + 1] == 1;
        if (join) {
            i64 cj = S->sptr[j + 1] - S->sptr[j], cn = S->sptr[j + 2] - S->sptr[j + 1];
            join = (cj == cn + 1) && S->srow[S->sptr[j]] == j + 1;
            for (i64 k = 1; join && k < cj; k++)
                if (S->srow[S->sptr[j] + k] != S->srow[S->sptr[j + 1] + k - 1]) join = 0;
        }
        if (join && (j + 1 - start) >= S->cap) join = 0;
        if (!join) { S->xsuper[N++] = j + 1; start = j + 1; }
    }
    S->xsuper[N] = n;
    S->N = N;
    free(nchild);
    for (int K = 0; K < N; K++)
        for (int j = S->xsuper[K]; j < S->xsuper[K + 1]; j++) S->sn[j] = K;
    S->sparent = (int*)malloc(sizeof(int) * (N > 0 ? N : 1));
    S->level = (int*)malloc(sizeof(int) * (N > 0 ? N : 1));
    for (int K = 0; K < N; K++) {
        int p = S->parent[S->xsuper[K + 1] - 1];
        S->sparent[K] = p >= 0 ? S->sn[p] : -1;
    }
    if (rcap > 0) {
        relax_partition(S, rcap);
        N = S->N;
    }
    /* Algorithm 2: sigma(root) = 1, sigma(I) = sigma(parent(I)) + 1 */
    for (int K = N - 1; K >= 0; K--)
        S->level[K] = S->sparent[K] < 0 ? 1 : S->level[S->sparent[K]] + 1;
    /* panel layout */
    S->poff = (i64*)malloc(sizeof(i64) * ((size_t)N + 1));
    S->poff[0] = 0;
    for (int K = 0; K < N; K++) {
        i64 s = sn_s(S, K), c = sn_c(S, K);
        S->poff[K + 1] = S->poff[K] + (s + c) * s;
    }
    S->arena = S->poff[N];
    /* sizes of the block index maps (the records are built per supernode,
     * on demand, by map_build) */
    S->rptr = (i64*)malloc(sizeof(i64) * ((size_t)N + 1));
    S->rptr[0] = 0;
    for (int K = 0; K < N; K++) {
        const int* C = sn_C(S, K);
        int c = sn_c(S, K);
        i64 tot = 0;
        for (int r = 0; r < c;) {
            int J = S->sn[C[r]];
            tot += 2 + (c - r);
            while (r < c && S->sn[C[r]] == J) r++;
        }
        S->rptr[K + 1] = S->rptr[K] + tot;
    }
    return S;
}

/* Relaxed supernodes (Section 2.1 relaxes supernodes within a column limit
 * and stores the explicit zeros this creates).  Reading used here: each
 * fundamental supernode is cut into pieces of at most rcap columns from its
 * first column; going through the pieces in column order, a piece joins the
 * block before it when it continues a chain -- it is not the first piece of
 * its supernode, or its supernode has exactly one child and that child is
 * the supernode just before it -- and the block then has at most rcap
 * columns.  The rows below a block are the structure of its last column,
 * which contains the structures of the columns below it (they form a
 * chain), so the block's other columns get explicit zeros there.  Replaces
 * xsuper, sn and sparent; levels and maps follow from them. */
static void relax_partition(orc_sym* S, int rcap)
{
    int n = S->n, N = S->N;
    int* nch = (int*)calloc((size_t)N + 1, sizeof(int));
    for (int K = 0; K < N; K++)
        if (S->sparent[K] >= 0) nch[S->sparent[K]]++;
    int* xs = (int*)malloc(sizeof(int) * ((size_t)n + 1));
    int M = 0;
    for (int K = 0; K < N; K++) {
        int f = S->xsuper[K], l = S->xsuper[K + 1];
        for (int a = f; a < l; a += rcap) {
            int b = a + rcap < l ? a + rcap : l;
            int chain = a > f || (K > 0 && S->sparent[K - 1] == K && nch[K] == 1);
            int fits = M > 0 && b - xs[M - 1] <= rcap;
            if (!(chain && fits)) xs[M++] = a;
        }
    }
    xs[M] = n;
    free(nch);
    free(S->xsuper);
    S->xsuper = xs;
    S->N = M;
    for (int K = 0; K < M; K++)
        for (int j = xs[K]; j < xs[K + 1]; j++) S->sn[j] = K;
    for (int K = 0; K < M; K++) {
        int p = S->parent[xs[K + 1] - 1];
        S->sparent[K] = p >= 0 ? S->sn[p] : -1;
    }
}

int orc_sym_error(const orc_sym* S) { return S->err; }
int orc_sym_nsuper(const orc_sym* S) { return S->N; }
/* entries of the pattern: per supernode, its dense lower diagonal block and
 * the rows below it in every column (for fundamental supernodes this is
 * n + sum |struct(j)|) */
i64 orc_sym_nnzL(const orc_sym* S)
{
    i64 q = 0;
    for (int K = 0; K < S->N; K++) {
        i64 s = sn_s(S, K), c = sn_c(S, K);
        q += s * (s + 1) / 2 + s * c;
    }
    return q;
}
i64 orc_sym_relsize(const orc_sym* S) { return S->rptr[S->N]; }
i64 orc_sym_arena(const orc_sym* S) { return S->arena; }

void orc_sym_get(const orc_sym* S, int* perm, int* parent, int* xsuper, int* sparent, int* level,
                 i64* cptr, int* crows)
{
    int n = S->n, N = S->N;
    if (perm) memcpy(perm, S->perm, sizeof(int) * (size_t)n);
    if (parent) memcpy(parent, S->parent, sizeof(int) * (size_t)n);
    if (xsuper) memcpy(xsuper, S->xsuper, sizeof(int) * ((size_t)N + 1));
    if (sparent) memcpy(sparent, S->sparent, sizeof(int) * (size_t)N);
    if (level) memcpy(level, S->level, sizeof(int) * (size_t)N);
    if (cptr) {
        cptr[0] = 0;
        for (int K = 0; K < N; K++) cptr[K + 1] = cptr[K] + sn_c(S, K);
        if (crows)
            for (int K = 0; K < N; K++) memcpy(crows + cptr[K], sn_C(S, K), sizeof(int) * (size_t)sn_c(S, K));
    }
}

void orc_sym_rel(const orc_sym* S, i64* rptr, int* rel)
{
    memcpy(rptr, S->rptr, sizeof(i64) * ((size_t)S->N + 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int K = 0; K < S->N; K++) map_build(S, K, rel + S->rptr[K]);
}

/* -1 entries in a map are rows missing from their ancestor (an error) */
int orc_sym_check_maps(const orc_sym* S)
{
    int bad = 0;
#pragma omp parallel
    {
        i64 cap = 0;
        int* buf = NULL;
#pragma omp for schedule(dynamic, 16) reduction(| : bad)
        for (int K = 0; K < S->N; K++) {
            i64 len = S->rptr[K + 1] - S->rptr[K];
            if (len > cap) { free(buf); cap = len; buf = (int*)malloc(sizeof(int) * (size_t)cap); }
            map_build(S, K, buf);
            for (i64 q = 0; q < len;) {
                int a = buf[q + 1], c = sn_c(S, K);
                for (int t = a; t < c; t++) bad |= buf[q + 2 + t - a] < 0;
                q += 2 + (c - a);
            }
        }
        free(buf);
    }
    return bad;
}

/* canonical lower pattern in permuted numbering: column j of supernode K
 * holds j, the later columns of K, then C(K), ascending (for fundamental
 * supernodes: j then struct(j)) */
void orc_sym_pattern(const orc_sym* S, i64* colptrL, int* rowindL)
{
    i64 q = 0;
    for (int K = 0; K < S->N; K++) {
        const int* C = sn_C(S, K);
        int c = sn_c(S, K), l = S->xsuper[K + 1];
        for (int j = S->xsuper[K]; j < l; j++) {
            colptrL[j] = q;
            for (int i = j; i < l; i++) rowindL[q++] = i;
            for (int t = 0; t < c; t++) rowindL[q++] = C[t];
        }
    }
    colptrL[S->n] = q;
}

/* work per supernode: gemm = 2c^2 s + 2 c s^2, factor = c^2 s + c s^2 + s^3/3 */
void orc_sym_flops(const orc_sym* S, double* gemm, double* factor)
{
    double g = 0, f = 0;
    for (int K = 0; K < S->N; K++) {
        double s = sn_s(S, K), c = sn_c(S, K);
        g += 2 * c * c * s + 2 * c * s * s;
        f += c * c * s + c * s * s + s * s * s / 3.0;
    }
    *gemm = g;
    *factor = f;
}

/* ------------------------------------------------------------------ */
/* O3: supernodal LDL^T and selected inversion                         */
/* ------------------------------------------------------------------ */

/* segment lookup in the block index map of supernode K (map, as written by
 * map_build): pointer to the positions of the segment containing position r
 * of C(K), that segment's ancestor J and start a */
static const int* seg_of(const int* map, i64 len, int c, int r, int* J, int* a)
{
    i64 q = 0;
    for (;;) {
        int JJ = map[q], aa = map[q + 1];
        i64 nq = q + 2 + (c - aa);
        int nexta = nq < len ? map[nq + 1] : c;
        if (r >= aa && r < nexta) { *J = JJ; *a = aa; return map + q + 2; }
        q = nq;
    }
}

/* Numerical supernodal LDL^T (leaves first), then Algorithm 1 (root first).
 * valsA: values in the original CSC order given to orc_symbolic.
 * sel:   nnz(L) values of A^{-1} on the canonical pattern (may be NULL).
 * Lout:  nnz(L) values of L on the canonical pattern, D on the diagonal
 *        (may be NULL).
 * Returns 0, -3 on a bad pivot with *bad_col = original column index, -4 when
 * out of memory, -5 when a block index map is inconsistent.
 *
 * Loop nests run along columns (contiguous in memory); every sum still runs
 * over its own index in ascending order, as the formulas are written, so the
 * order of the loops does not change a single rounding. */
int orc_factor_selinv(const orc_sym* S, const i64* colptr, const int* rowind, const double* valsA,
                      int require_spd, double* sel, double* Lout, i64* bad_col, double* t_factor,
                      double* t_selinv)
{
    int n = S->n, N = S->N;
    double* Lp = (double*)calloc((size_t)S->arena + 1, sizeof(double));
    double* Ai = (double*)calloc((size_t)S->arena + 1, sizeof(double));
    if (!Lp || !Ai) { free(Lp); free(Ai); return -4; }
    int bad = -1, maperr = 0;
    /* block index maps of every supernode (symbolic data: built before the
     * timed region); a -1 entry is a row missing from its ancestor's rows */
    int* maps = (int*)malloc(sizeof(int) * (size_t)(S->rptr[N] + 1));
    if (!maps) { free(Lp); free(Ai); return -4; }
#pragma omp parallel for schedule(dynamic, 16) reduction(| : maperr)
    for (int K = 0; K < N; K++) {
        map_build(S, K, maps + S->rptr[K]);
        for (i64 q = S->rptr[K]; q < S->rptr[K + 1]; q++) maperr |= maps[q] < 0;
    }
    if (maperr) { free(Lp); free(Ai); free(maps); return -5; }
    double t0 = 0;
#ifdef _OPENMP
    t0 = omp_get_wtime();
#endif
    /* assemble the permuted lower triangle into the panels */
    for (int j = 0; j < n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            int a = S->iperm[rowind[p]], b = S->iperm[j];
            int lo = a > b ? a : b, hi = a > b ? b : a;
            int K = S->sn[hi];
            i64 ld = sn_s(S, K) + sn_c(S, K);
            int r = row_pos(S, K, lo);
            Lp[S->poff[K] + r + (i64)(hi - S->xsuper[K]) * ld] += valsA[p];
        }
    /* factor, supernodes in increasing order (children before parents) */
    for (int K = 0; K < N && bad < 0; K++) {
        int s = sn_s(S, K), c = sn_c(S, K);
        i64 ld = s + c;
        double* F = Lp + S->poff[K];
        /* column LDL^T of the whole panel: for j, d_j = F(j,j) - sum_k L(j,k)^2 d_k
         * and L(i,j) = (F(i,j) - sum_k L(i,k) d_k L(j,k)) / d_j for rows i > j
         * (diagonal block and C(K) rows alike; the C rows give
         * L(C,K) = F(C,K) L_KK^{-T} D_K^{-1}). */
        for (int j = 0; j < s; j++) {
            double dj = F[j + j * ld];
            for (int k = 0; k < j; k++) dj -= F[j + k * ld] * F[j + k * ld] * F[k + k * ld];
            int ok = isfinite(dj) && dj != 0.0 && (!require_spd || dj > 0.0);
            if (!ok) { bad = S->xsuper[K] + j; break; }
            F[j + j * ld] = dj;
            double* Fj = F + (i64)j * ld;
            /* rows are independent: threads take runs of 256 rows */
#pragma omp parallel for schedule(static) if (ld > 2048)
            for (i64 i0 = j + 1; i0 < ld; i0 += 256) {
                i64 i1 = i0 + 256 < ld ? i0 + 256 : ld;
                for (int k = 0; k < j; k++) {
                    const double* Fk = F + (i64)k * ld;
                    double dk = Fk[k], ljk = Fk[j];
                    for (i64 i = i0; i < i1; i++) Fj[i] -= Fk[i] * dk * ljk;
                }
                for (i64 i = i0; i < i1; i++) Fj[i] = Fj[i] / dj;
            }
        }
        if (bad >= 0) break;
        if (c == 0) continue;
        const int* map = maps + S->rptr[K];
        i64 mlen = S->rptr[K + 1] - S->rptr[K];
        /* Schur complement update of the ancestors:
         * F(C,C) -= L(C,K) D_K L(C,K)^T, added into the owning panels.
         * Row r of L(C,K) is copied to LT(:,r), and row r of L(C,K) D_K
         * (the products L(r,t) d_t) to DT(:,r), so that each entry's sum over
         * t reads two contiguous vectors. */
        const int* C = sn_C(S, K);
        double* LT = (double*)malloc(sizeof(double) * (size_t)c * s);
        double* DT = (double*)malloc(sizeof(double) * (size_t)c * s);
#pragma omp parallel for schedule(static) if ((i64)c * s > 65536)
        for (int r = 0; r < c; r++)
            for (int t = 0; t < s; t++) {
                LT[t + (i64)r * s] = F[s + r + t * ld];
                DT[t + (i64)r * s] = F[s + r + t * ld] * F[t + t * ld];
            }
#pragma omp parallel for schedule(dynamic, 4) if (c > 64)
        for (int kk = 0; kk < c; kk++) {
            int J, a;
            const int* pos = seg_of(map, mlen, c, kk, &J, &a);
            i64 ldJ = sn_s(S, J) + sn_c(S, J);
            double* FJ = Lp + S->poff[J] + (i64)(C[kk] - S->xsuper[J]) * ldJ;
            const double* lk = LT + (i64)kk * s;
            int i0 = (g_mut == 5) ? kk + 1 : kk;
            for (int ii = i0; ii < c; ii++) {
                const double* di = DT + (i64)ii * s;
                double u = 0;
                for (int t = 0; t < s; t++) u += di[t] * lk[t];
                FJ[pos[ii - a]] -= u;
            }
        }
        free(LT);
        free(DT);
    }
    double t1 = 0;
#ifdef _OPENMP
    t1 = omp_get_wtime();
#endif
    if (bad >= 0) {
        if (bad_col) *bad_col = S->perm[bad];
        free(Lp); free(Ai); free(maps);
        return -3;
    }
    /* Algorithm 1, K = N .. 1 (root first; parents have larger indices) */
    for (int K = N - 1; K >= 0; K--) {
        int s = sn_s(S, K), c = sn_c(S, K);
        i64 ld = s + c;
        const double* F = Lp + S->poff[K];
        double* X = Ai + S->poff[K];
        const int* C = sn_C(S, K);
        double* Lh = (double*)malloc(sizeof(double) * ((size_t)c * s + 1));
        /* step 2: L_hat(C,K) = L(C,K) L_KK^{-1}, i.e. L_hat L_KK = L(C,K),
         * solved for the columns of L_hat from the last one back */
        /* rows are independent: threads take runs of 256 rows */
#pragma omp parallel for schedule(static) if ((i64)c * s > 65536)
        for (int r0 = 0; r0 < c; r0 += 256) {
            int r1 = r0 + 256 < c ? r0 + 256 : c;
            for (int j = s - 1; j >= 0; j--) {
                double* Hj = Lh + (i64)j * c;
                for (int r = r0; r < r1; r++) Hj[r] = F[s + r + (i64)j * ld];
                if (g_mut != 3)
                    for (int k = j + 1; k < s; k++) {
                        const double* Hk = Lh + (i64)k * c;
                        double lkj = F[k + (i64)j * ld];
                        for (int r = r0; r < r1; r++) Hj[r] -= Hk[r] * lkj;
                    }
            }
        }
        if (c > 0) {
            const int* map = maps + S->rptr[K];
            i64 mlen = S->rptr[K + 1] - S->rptr[K];
            /* step 1 + gather: G = Ainv(C,C) from the stored lower entries */
            double* G = (double*)malloc(sizeof(double) * (size_t)c * c);
#pragma omp parallel for schedule(dynamic, 4) if (c > 64)
            for (int kk = 0; kk < c; kk++) {
                int J, a;
                const int* pos = seg_of(map, mlen, c, kk, &J, &a);
                i64 ldJ = sn_s(S, J) + sn_c(S, J);
                const double* AJ = Ai + S->poff[J] + (i64)(C[kk] - S->xsuper[J]) * ldJ;
                for (int ii = kk; ii < c; ii++) G[ii + (i64)kk * c] = AJ[pos[ii - a]];
            }
            /* the entries above the diagonal by symmetry, G(k,i) = G(i,k),
             * copied in 64 x 64 tiles so that both sides stay in cache */
#pragma omp parallel for schedule(dynamic, 1) if (c > 64)
            for (int kb = 0; kb < c; kb += 64)
                for (int ib = kb; ib < c; ib += 64)
                    for (int kk = kb; kk < kb + 64 && kk < c; kk++)
                        for (int ii = (ib > kk + 1 ? ib : kk + 1); ii < ib + 64 && ii < c; ii++)
                            G[kk + (i64)ii * c] = (g_mut == 4) ? 0.0 : G[ii + (i64)kk * c];
            /* step 3: Ainv(C,K) = -Ainv(C,C) L_hat(C,K).  G is symmetric, so
             * row r of G is read as its column r (G(r,k) = G(k,r)); with L_hat
             * transposed, the s sums of row r advance together over k. */
            double* HT = (double*)malloc(sizeof(double) * (size_t)c * s);
            for (int j = 0; j < s; j++)
                for (int k = 0; k < c; k++) HT[j + (i64)k * s] = Lh[k + (i64)j * c];
#pragma omp parallel if (c > 64)
            {
                double* v = (double*)malloc(sizeof(double) * (size_t)s);
#pragma omp for schedule(static)
                for (int r = 0; r < c; r++) {
                    const double* Gr = G + (i64)r * c;
                    for (int j = 0; j < s; j++) v[j] = 0;
                    for (int k = 0; k < c; k++) {
                        const double g = Gr[k];
                        const double* h = HT + (i64)k * s;
                        for (int j = 0; j < s; j++) v[j] += g * h[j];
                    }
                    for (int j = 0; j < s; j++) X[s + r + (i64)j * ld] = (g_mut == 1) ? v[j] : -v[j];
                }
                free(v);
            }
            free(HT);
            free(G);
        }
        /* step 4: Ainv(K,K) = U_KK^{-1} L_KK^{-1} - U_hat(K,C) Ainv(C,K),
         * with U = D L^T and U_hat = L_hat^T.  T(:,j) solves L D L^T x = e_j. */
        double* Y = (double*)malloc(sizeof(double) * (size_t)s * s);
#pragma omp parallel if (s > 16)
        {
            double* y = (double*)malloc(sizeof(double) * (size_t)s);
#pragma omp for schedule(static)
            for (int j = 0; j < s; j++) {
                for (int i = 0; i < s; i++) y[i] = (i == j) ? 1.0 : 0.0;
                for (int i = 0; i < s; i++)
                    for (int k = 0; k < i; k++) y[i] -= F[i + (i64)k * ld] * y[k];
                for (int i = 0; i < s; i++)
                    y[i] = (g_mut == 6) ? y[i] * F[i + (i64)i * ld] : y[i] / F[i + (i64)i * ld];
                for (int i = s - 1; i >= 0; i--)
                    for (int k = i + 1; k < s; k++) y[i] -= F[k + (i64)i * ld] * y[k];
                for (int i = 0; i < s; i++) Y[i + (i64)j * s] = (g_mut == 2) ? 0.0 : y[i];
            }
            free(y);
#pragma omp for schedule(static)
            for (int j = 0; j < s; j++)
                for (int i = 0; i < s; i++) {
                    double v = 0;
                    for (int r = 0; r < c; r++) v += Lh[r + (i64)i * c] * X[s + r + (i64)j * ld];
                    Y[i + (i64)j * s] -= v;
                }
        }
        /* symmetrise the diagonal block */
        for (int j = 0; j < s; j++)
            for (int i = 0; i < s; i++)
                X[i + (i64)j * ld] = 0.5 * (Y[i + (i64)j * s] + Y[j + (i64)i * s]);
        free(Y); free(Lh);
    }
    free(maps);
    double t2 = 0;
#ifdef _OPENMP
    t2 = omp_get_wtime();
#endif
    if (t_factor) *t_factor = t1 - t0;
    if (t_selinv) *t_selinv = t2 - t1;
    /* export on the canonical pattern */
    i64 q = 0;
    for (int K = 0; K < N; K++) {
        int s = sn_s(S, K), c = sn_c(S, K);
        i64 ld = s + c;
        for (int j = 0; j < s; j++)
            for (i64 i = j; i < ld; i++) {
                i64 o = S->poff[K] + i + (i64)j * ld;
                if (sel) sel[q] = Ai[o];
                if (Lout) {
                    double v = Lp[o];
                    if (g_mut == 8 && i > j) v *= Lp[S->poff[K] + j + (i64)j * ld]; /* L D, not L */
                    if (g_mut == 9 && i == j) v = 1.0 / v;                         /* D^{-1}, not D */
                    Lout[q] = v;
                }
                q++;
            }
    }
    free(Lp); free(Ai);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Dense tiers                                                          */
/* ------------------------------------------------------------------ */

/* in-place dense LDL^T of a symmetric n x n column-major matrix: on exit the
 * strict lower triangle holds L (unit diagonal implied), the diagonal holds D.
 * Returns the first bad column or -1. */
static int dense_ldlt(int n, double* A)
{
    for (int j = 0; j < n; j++) {
        double dj = A[j + (i64)j * n];
        for (int k = 0; k < j; k++) dj -= A[j + (i64)k * n] * A[j + (i64)k * n] * A[k + (i64)k * n];
        if (!isfinite(dj) || dj == 0.0) return j;
        A[j + (i64)j * n] = dj;
#pragma omp parallel for schedule(static) if (n > 256)
        for (int i = j + 1; i < n; i++) {
            double v = A[i + (i64)j * n];
            for (int k = 0; k < j; k++) v -= A[i + (i64)k * n] * A[k + (i64)k * n] * A[j + (i64)k * n];
            A[i + (i64)j * n] = v / dj;
        }
    }
    return -1;
}

/* O1's factor alone: the dense LDL^T of a symmetric n x n column-major A
 * (strict lower triangle L, diagonal D, upper triangle left as given).
 * Returns 0 or -3 on a zero pivot. */
int orc_dense_ldlt(int n, const double* A, double* F)
{
    memcpy(F, A, sizeof(double) * (size_t)n * n);
    return dense_ldlt(n, F) >= 0 ? -3 : 0;
}

/* O1: A^{-1} by LDL^T and n triangular solves L y = e_j, D z = y, L^T x = z. */
int orc_dense_inverse(int n, const double* A, double* Ainv)
{
    double* F = (double*)malloc(sizeof(double) * (size_t)n * n);
    memcpy(F, A, sizeof(double) * (size_t)n * n);
    int bad = dense_ldlt(n, F);
    if (bad >= 0) { free(F); return -3; }
#pragma omp parallel for schedule(dynamic, 8)
    for (int j = 0; j < n; j++) {
        double* x = Ainv + (i64)j * n;
        for (int i = 0; i < n; i++) x[i] = (i == j) ? 1.0 : 0.0;
        for (int i = 0; i < n; i++)
            for (int k = 0; k < i; k++) x[i] -= F[i + (i64)k * n] * x[k];
        for (int i = 0; i < n; i++) x[i] /= F[i + (i64)i * n];
        for (int i = n - 1; i >= 0; i--)
            for (int k = i + 1; k < n; k++) x[i] -= F[k + (i64)i * n] * x[k];
    }
    free(F);
    return 0;
}

/* O2: scalar recurrence on the pattern of L (canonical lower CSC, rows
 * sorted, diagonal first) for a dense, already permuted A:
 *   Ainv(C,j) = -Ainv(C,C) L(C,j),   Ainv(j,j) = 1/d_j - L(C,j)^T Ainv(C,j),
 * for j = n-1 .. 0, C = struct(L(:,j)). */
int orc_selinv_columns(int n, const double* A, const i64* colptrL, const int* rowindL, double* sel)
{
    double* F = (double*)malloc(sizeof(double) * (size_t)n * n);
    memcpy(F, A, sizeof(double) * (size_t)n * n);
    int bad = dense_ldlt(n, F);
    if (bad >= 0) { free(F); return -3; }
    double* Z = (double*)calloc((size_t)n * n, sizeof(double));
    double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
    for (int j = n - 1; j >= 0; j--) {
        i64 p0 = colptrL[j] + 1, p1 = colptrL[j + 1];
        for (i64 p = p0; p < p1; p++) {
            int i = rowindL[p];
            double v = 0;
            for (i64 q = p0; q < p1; q++) {
                int k = rowindL[q];
                v += Z[i + (i64)k * n] * F[k + (i64)j * n];
            }
            tmp[p - p0] = -v;
        }
        double d = 1.0 / F[j + (i64)j * n];
        for (i64 p = p0; p < p1; p++) {
            int i = rowindL[p];
            Z[i + (i64)j * n] = tmp[p - p0];
            Z[j + (i64)i * n] = tmp[p - p0];
            d -= F[i + (i64)j * n] * tmp[p - p0];
        }
        Z[j + (i64)j * n] = d;
    }
    for (int j = 0; j < n; j++)
        for (i64 p = colptrL[j]; p < colptrL[j + 1]; p++) sel[p] = Z[rowindL[p] + (i64)j * n];
    free(F); free(Z); free(tmp);
    return 0;
}

/* Dense reference gradient.  f = sum over the lower pattern of L of
 * w_ij Ainv_ij; S = W + W^T (so S_ii = 2 w_ii).  An off-diagonal parameter
 * a_ij drives A_ij and A_ji, so df/da_ij = -(Ainv S Ainv)_ij for i != j and
 * -(1/2)(Ainv S Ainv)_ii on the diagonal.  Ainv: dense n x n (permuted
 * numbering), W on (colptrL, rowindL); g on A's lower pattern given in the
 * same numbering as (colptrA, rowindA). */
void orc_dense_grad(int n, const double* Ainv, const i64* colptrL, const int* rowindL, const double* w,
                    const i64* colptrA, const int* rowindA, double* g)
{
    double* Sm = (double*)calloc((size_t)n * n, sizeof(double));
    for (int j = 0; j < n; j++)
        for (i64 p = colptrL[j]; p < colptrL[j + 1]; p++) {
            int i = rowindL[p];
            Sm[i + (i64)j * n] += w[p];
            Sm[j + (i64)i * n] += w[p];
        }
    double* T = (double*)calloc((size_t)n * n, sizeof(double));
    /* T = S Ainv */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; j++)
        for (int k = 0; k < n; k++) {
            double b = Ainv[k + (i64)j * n];
            if (b == 0.0) continue;
            for (int i = 0; i < n; i++) T[i + (i64)j * n] += Sm[i + (i64)k * n] * b;
        }
    for (int j = 0; j < n; j++)
        for (i64 p = colptrA[j]; p < colptrA[j + 1]; p++) {
            int i = rowindA[p];
            double m = 0;
            for (int k = 0; k < n; k++) m += Ainv[i + (i64)k * n] * T[k + (i64)j * n];
            g[p] = (i == j) ? -0.5 * m : -m;
        }
    free(Sm); free(T);
}

/* ------------------------------------------------------------------ */
/* Complex symmetric matrices A(z) = H - z S (Section 4.3: the pole     */
/* expansion inverts such matrices, symmetric but not Hermitian).       */
/* The same LDL^T and Algorithm 1 with complex numbers: transposes are  */
/* plain transposes, never conjugates.  Values are interleaved (re, im).*/
/* ------------------------------------------------------------------ */
#include <complex.h>

typedef double complex zc;

/* O3 for complex values: valsA and sel hold 2 doubles per entry.  A pivot
 * that is zero or not finite is reported (there is no sign condition).
 * Returns 0, -3 (bad pivot, *bad_col = original column), -4 (memory) or -5
 * (inconsistent index map). */
int orc_factor_selinv_z(const orc_sym* S, const i64* colptr, const int* rowind, const double* valsA, double* sel,
                        i64* bad_col)
{
    int n = S->n, N = S->N;
    zc* Lp = (zc*)calloc((size_t)S->arena + 1, sizeof(zc));
    zc* Ai = (zc*)calloc((size_t)S->arena + 1, sizeof(zc));
    int* maps = (int*)malloc(sizeof(int) * (size_t)(S->rptr[N] + 1));
    if (!Lp || !Ai || !maps) { free(Lp); free(Ai); free(maps); return -4; }
    int bad = -1, maperr = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : maperr)
    for (int K = 0; K < N; K++) {
        map_build(S, K, maps + S->rptr[K]);
        for (i64 q = S->rptr[K]; q < S->rptr[K + 1]; q++) maperr |= maps[q] < 0;
    }
    if (maperr) { free(Lp); free(Ai); free(maps); return -5; }
    for (int j = 0; j < n; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            int a = S->iperm[rowind[p]], b = S->iperm[j];
            int lo = a > b ? a : b, hi = a > b ? b : a;
            int K = S->sn[hi];
            i64 ld = sn_s(S, K) + sn_c(S, K);
            int r = row_pos(S, K, lo);
            Lp[S->poff[K] + r + (i64)(hi - S->xsuper[K]) * ld] += valsA[2 * p] + I * valsA[2 * p + 1];
        }
    /* factor: column LDL^T of each panel, then the Schur update of the ancestors */
    for (int K = 0; K < N && bad < 0; K++) {
        int s = sn_s(S, K), c = sn_c(S, K);
        i64 ld = s + c;
        zc* F = Lp + S->poff[K];
        for (int j = 0; j < s; j++) {
            zc dj = F[j + j * ld];
            for (int k = 0; k < j; k++) dj -= F[j + k * ld] * F[j + k * ld] * F[k + k * ld];
            if (dj == 0 || !isfinite(creal(dj)) || !isfinite(cimag(dj))) { bad = S->xsuper[K] + j; break; }
            F[j + j * ld] = dj;
            zc* Fj = F + (i64)j * ld;
            for (int k = 0; k < j; k++) {
                const zc* Fk = F + (i64)k * ld;
                zc dk = Fk[k], ljk = Fk[j];
                for (i64 i = j + 1; i < ld; i++) Fj[i] -= Fk[i] * dk * ljk;
            }
            for (i64 i = j + 1; i < ld; i++) Fj[i] = Fj[i] / dj;
        }
        if (bad >= 0 || c == 0) continue;
        const int* map = maps + S->rptr[K];
        i64 mlen = S->rptr[K + 1] - S->rptr[K];
        const int* C = sn_C(S, K);
#pragma omp parallel for schedule(dynamic, 4) if (c > 64)
        for (int kk = 0; kk < c; kk++) {
            int J, a;
            const int* pos = seg_of(map, mlen, c, kk, &J, &a);
            i64 ldJ = sn_s(S, J) + sn_c(S, J);
            zc* FJ = Lp + S->poff[J] + (i64)(C[kk] - S->xsuper[J]) * ldJ;
            for (int ii = kk; ii < c; ii++) {
                zc u = 0;
                for (int t = 0; t < s; t++) u += F[s + ii + t * ld] * F[t + t * ld] * F[s + kk + t * ld];
                FJ[pos[ii - a]] -= u;
            }
        }
    }
    if (bad >= 0) {
        if (bad_col) *bad_col = S->perm[bad];
        free(Lp); free(Ai); free(maps);
        return -3;
    }
    /* Algorithm 1, root first */
    for (int K = N - 1; K >= 0; K--) {
        int s = sn_s(S, K), c = sn_c(S, K);
        i64 ld = s + c;
        const zc* F = Lp + S->poff[K];
        zc* X = Ai + S->poff[K];
        const int* C = sn_C(S, K);
        zc* Lh = (zc*)malloc(sizeof(zc) * ((size_t)c * s + 1));
        /* step 2: L_hat L_KK = L(C,K), columns from the last one back */
        for (int j = s - 1; j >= 0; j--) {
            zc* Hj = Lh + (i64)j * c;
            for (int r = 0; r < c; r++) Hj[r] = F[s + r + (i64)j * ld];
            for (int k = j + 1; k < s; k++) {
                const zc* Hk = Lh + (i64)k * c;
                zc lkj = F[k + (i64)j * ld];
                for (int r = 0; r < c; r++) Hj[r] -= Hk[r] * lkj;
            }
        }
        if (c > 0) {
            const int* map = maps + S->rptr[K];
            i64 mlen = S->rptr[K + 1] - S->rptr[K];
            /* gather G = Ainv(C,C) (symmetric: the upper entries mirror the lower) */
            zc* G = (zc*)malloc(sizeof(zc) * (size_t)c * c);
#pragma omp parallel for schedule(dynamic, 4) if (c > 64)
            for (int kk = 0; kk < c; kk++) {
                int J, a;
                const int* pos = seg_of(map, mlen, c, kk, &J, &a);
                i64 ldJ = sn_s(S, J) + sn_c(S, J);
                const zc* AJ = Ai + S->poff[J] + (i64)(C[kk] - S->xsuper[J]) * ldJ;
                for (int ii = kk; ii < c; ii++) {
                    G[ii + (i64)kk * c] = AJ[pos[ii - a]];
                    /* planted mistake 10: a Hermitian mirror (conjugate) */
                    G[kk + (i64)ii * c] = (g_mut == 10 && ii != kk) ? conj(AJ[pos[ii - a]]) : AJ[pos[ii - a]];
                }
            }
            /* step 3: Ainv(C,K) = -G L_hat */
#pragma omp parallel for schedule(static) if (c > 64)
            for (int r = 0; r < c; r++)
                for (int j = 0; j < s; j++) {
                    zc v = 0;
                    for (int k = 0; k < c; k++) v += G[k + (i64)r * c] * Lh[k + (i64)j * c];
                    X[s + r + (i64)j * ld] = -v;
                }
            free(G);
        }
        /* step 4: Ainv(K,K) = L_KK^{-T} D^{-1} L_KK^{-1} - L_hat^T Ainv(C,K), symmetrised */
        zc* Y = (zc*)malloc(sizeof(zc) * (size_t)s * s);
        zc* y = (zc*)malloc(sizeof(zc) * (size_t)s);
        for (int j = 0; j < s; j++) {
            for (int i = 0; i < s; i++) y[i] = (i == j) ? 1.0 : 0.0;
            for (int i = 0; i < s; i++)
                for (int k = 0; k < i; k++) y[i] -= F[i + (i64)k * ld] * y[k];
            for (int i = 0; i < s; i++) y[i] = y[i] / F[i + (i64)i * ld];
            for (int i = s - 1; i >= 0; i--)
                for (int k = i + 1; k < s; k++) y[i] -= F[k + (i64)i * ld] * y[k];
            for (int i = 0; i < s; i++) Y[i + (i64)j * s] = y[i];
        }
        for (int j = 0; j < s; j++)
            for (int i = 0; i < s; i++) {
                zc v = 0;
                for (int r = 0; r < c; r++) v += Lh[r + (i64)i * c] * X[s + r + (i64)j * ld];
                Y[i + (i64)j * s] -= v;
            }
        for (int j = 0; j < s; j++)
            for (int i = 0; i < s; i++) X[i + (i64)j * ld] = 0.5 * (Y[i + (i64)j * s] + Y[j + (i64)i * s]);
        free(Y); free(y); free(Lh);
    }
    i64 q = 0;
    for (int K = 0; K < N; K++) {
        int s = sn_s(S, K), c = sn_c(S, K);
        i64 ld = s + c;
        for (int j = 0; j < s; j++)
            for (i64 i = j; i < ld; i++) {
                zc v = Ai[S->poff[K] + i + (i64)j * ld];
                sel[2 * q] = creal(v);
                sel[2 * q + 1] = cimag(v);
                q++;
            }
    }
    free(Lp); free(Ai); free(maps);
    return 0;
}

/* O1 for complex symmetric A (column-major, interleaved re/im): dense LDL^T
 * without conjugation, then n triangular solves.  Returns 0 or -3. */
int orc_dense_inverse_z(int n, const double* A, double* Ainv)
{
    zc* F = (zc*)malloc(sizeof(zc) * (size_t)n * n);
    for (i64 e = 0; e < (i64)n * n; e++) F[e] = A[2 * e] + I * A[2 * e + 1];
    for (int j = 0; j < n; j++) {
        zc dj = F[j + (i64)j * n];
        for (int k = 0; k < j; k++) dj -= F[j + (i64)k * n] * F[j + (i64)k * n] * F[k + (i64)k * n];
        if (dj == 0 || !isfinite(creal(dj)) || !isfinite(cimag(dj))) { free(F); return -3; }
        F[j + (i64)j * n] = dj;
        for (int i = j + 1; i < n; i++) {
            zc v = F[i + (i64)j * n];
            for (int k = 0; k < j; k++) v -= F[i + (i64)k * n] * F[k + (i64)k * n] * F[j + (i64)k * n];
            F[i + (i64)j * n] = v / dj;
        }
    }
#pragma omp parallel for schedule(dynamic, 8)
    for (int j = 0; j < n; j++) {
        zc* x = (zc*)malloc(sizeof(zc) * (size_t)n);
        for (int i = 0; i < n; i++) x[i] = (i == j) ? 1.0 : 0.0;
        for (int i = 0; i < n; i++)
            for (int k = 0; k < i; k++) x[i] -= F[i + (i64)k * n] * x[k];
        for (int i = 0; i < n; i++) x[i] /= F[i + (i64)i * n];
        for (int i = n - 1; i >= 0; i--)
            for (int k = i + 1; k < n; k++) x[i] -= F[k + (i64)i * n] * x[k];
        for (int i = 0; i < n; i++) {
            Ainv[2 * (i + (i64)j * n)] = creal(x[i]);
            Ainv[2 * (i + (i64)j * n) + 1] = cimag(x[i]);
        }
        free(x);
    }
    free(F);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Symmetric indefinite matrices: LDL^T with 1x1 and 2x2 pivots         */
/* (Section 2.1: D may have 2x2 blocks), chosen by the Bunch-Kaufman    */
/* rule inside each supernode's diagonal block.  The rest of the method */
/* needs the diagonal block only through its inverse T = F_KK^{-1}      */
/* (L_hat = F(C,K) T, the Schur update L_hat F(C,K)^T and Algorithm 1). */
/* ------------------------------------------------------------------ */

/* Bunch-Kaufman factorization of the symmetric s x s matrix M (column
 * major, both triangles): P M P^T = L D L^T with L unit lower and D of 1x1
 * and 2x2 blocks.  On return M's strict lower part holds L, piv[k] the row
 * swapped with k at step k, bs[k] = 1 or 2 the size of the pivot starting at
 * k (0 for the second column of a 2x2 pivot), and the D blocks stay on M's
 * diagonal / first subdiagonal.  Returns 0, or -1 for a singular block. */
static int bk_factor(int s, double* M, int* piv, int* bs)
{
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
#define AT(i, j) M[(i) + (i64)(j) * s]
    int k = 0;
    while (k < s) {
        double lambda = 0.0;
        int r = k;
        for (int i = k + 1; i < s; i++)
            if (fabs(AT(i, k)) > lambda) { lambda = fabs(AT(i, k)); r = i; }
        int size = 1, swap = k;
        if (lambda == 0.0) {
            if (AT(k, k) == 0.0) return -1;
        } else if (fabs(AT(k, k)) < alpha * lambda) {
            double sigma = 0.0;
            for (int j = k; j < s; j++)
                if (j != r && fabs(AT(r, j)) > sigma) sigma = fabs(AT(r, j));
            if (fabs(AT(k, k)) * sigma >= alpha * lambda * lambda) {
                size = 1;
            } else if (fabs(AT(r, r)) >= alpha * sigma) {
                size = 1;
                swap = r;
            } else {
                size = 2;
                swap = r;
            }
        }
        if (g_mut == 11 && size == 2) { size = 1; swap = k; } /* planted mistake: no 2x2 pivots */
        /* symmetric interchange of row/column kp with `swap` (both triangles) */
        int kp = (size == 2) ? k + 1 : k;
        if (swap != kp) {
            for (int j = 0; j < s; j++) { double t = AT(kp, j); AT(kp, j) = AT(swap, j); AT(swap, j) = t; }
            for (int i = 0; i < s; i++) { double t = AT(i, kp); AT(i, kp) = AT(i, swap); AT(i, swap) = t; }
        }
        piv[kp] = swap;
        if (size == 2) piv[k] = k;
        if (size == 1) {
            double d = AT(k, k);
            if (d == 0.0 || !isfinite(d)) return -1;
            for (int i = k + 1; i < s; i++) AT(i, k) /= d;           /* L(:,k) */
            for (int j = k + 1; j < s; j++)                          /* trailing update, both triangles */
                for (int i = k + 1; i < s; i++) AT(i, j) -= AT(i, k) * d * AT(j, k);
            for (int j = k + 1; j < s; j++) AT(k, j) = AT(j, k);     /* keep the row consistent (unused) */
            bs[k] = 1;
            k += 1;
        } else {
            double a = AT(k, k), b = AT(k + 1, k), c = AT(k + 1, k + 1);
            double det = a * c - b * b;
            if (det == 0.0 || !isfinite(det)) return -1;
            /* rows i > k+1: [L(i,k) L(i,k+1)] = [M(i,k) M(i,k+1)] D^{-1} */
            for (int i = k + 2; i < s; i++) {
                double u = AT(i, k), v = AT(i, k + 1);
                AT(i, k) = (u * c - v * b) / det;
                AT(i, k + 1) = (v * a - u * b) / det;
            }
            for (int j = k + 2; j < s; j++)
                for (int i = k + 2; i < s; i++)
                    AT(i, j) -= AT(i, k) * (a * AT(j, k) + b * AT(j, k + 1)) + AT(i, k + 1) * (b * AT(j, k) + c * AT(j, k + 1));
            bs[k] = 2;
            bs[k + 1] = 0;
            k += 2;
        }
    }
    return 0;
#undef AT
}

/* T = M^{-1} from the factorization: T(:,j) = P^T L^{-T} D^{-1} L^{-1} P e_j,
 * the interchanges applied in order and undone in reverse order */
static void bk_inverse(int s, const double* F, const int* piv, const int* bs, double* T)
{
#define AT(i, j) F[(i) + (i64)(j) * s]
    double* x = (double*)malloc(sizeof(double) * (size_t)s);
    for (int j = 0; j < s; j++) {
        for (int i = 0; i < s; i++) x[i] = (i == j) ? 1.0 : 0.0;
        for (int k = 0; k < s; k++) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
        for (int k = 0; k < s; k++) {                          /* L y = P e_j */
            if (bs[k] == 0) continue;
            int w = bs[k];
            for (int i = k + w; i < s; i++) {
                x[i] -= AT(i, k) * x[k];
                if (w == 2) x[i] -= AT(i, k + 1) * x[k + 1];
            }
        }
        for (int k = 0; k < s; k++) {                          /* D z = y */
            if (bs[k] == 1) x[k] /= AT(k, k);
            else if (bs[k] == 2) {
                double a = AT(k, k), b = AT(k + 1, k), c = AT(k + 1, k + 1), det = a * c - b * b;
                double u = x[k], v = x[k + 1];
                x[k] = (c * u - b * v) / det;
                x[k + 1] = (a * v - b * u) / det;
            }
        }
        for (int k = s - 1; k >= 0; k--) {                     /* L^T w = z */
            if (bs[k] == 0) continue;
            int w = bs[k];
            for (int i = k + w; i < s; i++) {
                x[k] -= AT(i, k) * x[i];
                if (w == 2) x[k + 1] -= AT(i, k + 1) * x[i];
            }
        }
        for (int k = s - 1; k >= 0; k--) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
        for (int i = 0; i < s; i++) T[i + (i64)j * s] = x[i];
    }
    free(x);
#undef AT
}

/* O3 with 1x1/2x2 pivots inside the diagonal blocks.  Per supernode K, leaves
 * first: T = F_KK^{-1} (Bunch-Kaufman), L_hat(C,K) = F(C,K) T, and the Schur
 * update F(C,C) -= L_hat F(C,K)^T into the ancestors; then Algorithm 1 root
 * first with that L_hat and T.  Returns 0, -3 (singular diagonal block,
 * *bad_col = original index of its first column), -4 or -5 as
 * orc_factor_selinv. */
int orc_factor_selinv_bk(const orc_sym* S, const i64* colptr, const int* rowind, const double* valsA, double* sel,
                         i64* bad_col)
{
    int n = S->n, N = S->N;
    double* Lp = (double*)calloc((size_t)S->arena + 1, sizeof(double));
    double* Ai = (double*)calloc((size_t)S->arena + 1, sizeof(double));
    i64* hoff = (i64*)malloc(sizeof(i64) * ((size_t)N + 1));
    i64* toff = (i64*)malloc(sizeof(i64) * ((size_t)N + 1));
    hoff[0] = toff[0] = 0;
    for (int K = 0; K < N; K++) {
        hoff[K + 1] = hoff[K] + (i64)sn_c(S, K) * sn_s(S, K);
        toff[K + 1] = toff[K] + (i64)sn_s(S, K) * sn_s(S, K);
    }
    double* Lh = (double*)malloc(sizeof(double) * (size_t)(hoff[N] + 1));
    double* Tt = (double*)malloc(sizeof(double) * (size_t)(toff[N] + 1));
    int* maps = (int*)malloc(sizeof(int) * (size_t)(S->rptr[N] + 1));
    if (!Lp || !Ai || !Lh || !Tt || !maps) { free(Lp); free(Ai); free(Lh); free(Tt); free(maps); free(hoff); free(toff); return -4; }
    int maperr = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : maperr)
    for (int K = 0; K < N; K++) {
        map_build(S, K, maps + S->rptr[K]);
        for (i64 q = S->rptr[K]; q < S->rptr[K + 1]; q++) maperr |= maps[q] < 0;
    }
    int status = maperr ? -5 : 0;
    for (int j = 0; j < n && !status; j++)
        for (i64 p = colptr[j]; p < colptr[j + 1]; p++) {
            int a = S->iperm[rowind[p]], b = S->iperm[j];
            int lo = a > b ? a : b, hi = a > b ? b : a;
            int K = S->sn[hi];
            i64 ld = sn_s(S, K) + sn_c(S, K);
            Lp[S->poff[K] + row_pos(S, K, lo) + (i64)(hi - S->xsuper[K]) * ld] += valsA[p];
        }
    for (int K = 0; K < N && !status; K++) {
        int s = sn_s(S, K), c = sn_c(S, K);
        i64 ld = s + c;
        double* F = Lp + S->poff[K];
        /* the diagonal block, both triangles */
        double* M = (double*)malloc(sizeof(double) * (size_t)s * s);
        int* piv = (int*)malloc(sizeof(int) * (size_t)s);
        int* bs = (int*)malloc(sizeof(int) * (size_t)s);
        for (int j = 0; j < s; j++)
            for (int i = j; i < s; i++) M[i + (i64)j * s] = M[j + (i64)i * s] = F[i + (i64)j * ld];
        if (bk_factor(s, M, piv, bs)) {
            if (bad_col) *bad_col = S->perm[S->xsuper[K]];
            status = -3;
        } else {
            double* T = Tt + toff[K];
            bk_inverse(s, M, piv, bs, T);
            double* H = Lh + hoff[K];
            /* L_hat(C,K) = F(C,K) T */
            for (int r = 0; r < c; r++)
                for (int j = 0; j < s; j++) {
                    double v = 0;
                    for (int k = 0; k < s; k++) v += F[s + r + (i64)k * ld] * T[k + (i64)j * s];
                    H[r + (i64)j * c] = v;
                }
            if (c > 0) {
                const int* map = maps + S->rptr[K];
                i64 mlen = S->rptr[K + 1] - S->rptr[K];
                const int* C = sn_C(S, K);
#pragma omp parallel for schedule(dynamic, 4) if (c > 64)
                for (int kk = 0; kk < c; kk++) {
                    int J, a;
                    const int* pos = seg_of(map, mlen, c, kk, &J, &a);
                    i64 ldJ = sn_s(S, J) + sn_c(S, J);
                    double* FJ = Lp + S->poff[J] + (i64)(C[kk] - S->xsuper[J]) * ldJ;
                    for (int ii = kk; ii < c; ii++) {
                        double u = 0;
                        for (int t = 0; t < s; t++) u += H[ii + (i64)t * c] * F[s + kk + (i64)t * ld];
                        FJ[pos[ii - a]] -= u;
                    }
                }
            }
        }
        free(M); free(piv); free(bs);
    }
    /* Algorithm 1, root first, with the stored L_hat and T */
    for (int K = N - 1; K >= 0 && !status; K--) {
        int s = sn_s(S, K), c = sn_c(S, K);
        i64 ld = s + c;
        double* X = Ai + S->poff[K];
        const double* H = Lh + hoff[K];
        const double* T = Tt + toff[K];
        const int* C = sn_C(S, K);
        if (c > 0) {
            const int* map = maps + S->rptr[K];
            i64 mlen = S->rptr[K + 1] - S->rptr[K];
            double* G = (double*)malloc(sizeof(double) * (size_t)c * c);
#pragma omp parallel for schedule(dynamic, 4) if (c > 64)
            for (int kk = 0; kk < c; kk++) {
                int J, a;
                const int* pos = seg_of(map, mlen, c, kk, &J, &a);
                i64 ldJ = sn_s(S, J) + sn_c(S, J);
                const double* AJ = Ai + S->poff[J] + (i64)(C[kk] - S->xsuper[J]) * ldJ;
                for (int ii = kk; ii < c; ii++) G[ii + (i64)kk * c] = G[kk + (i64)ii * c] = AJ[pos[ii - a]];
            }
#pragma omp parallel for schedule(static) if (c > 64)
            for (int r = 0; r < c; r++)
                for (int j = 0; j < s; j++) {
                    double v = 0;
                    for (int k = 0; k < c; k++) v += G[k + (i64)r * c] * H[k + (i64)j * c];
                    X[s + r + (i64)j * ld] = -v;
                }
            free(G);
        }
        for (int j = 0; j < s; j++)
            for (int i = 0; i < s; i++) {
                double v = T[i + (i64)j * s], w = T[j + (i64)i * s];
                for (int r = 0; r < c; r++) {
                    v -= H[r + (i64)i * c] * X[s + r + (i64)j * ld];
                    w -= H[r + (i64)j * c] * X[s + r + (i64)i * ld];
                }
                X[i + (i64)j * ld] = 0.5 * (v + w);
            }
    }
    if (!status) {
        i64 q = 0;
        for (int K = 0; K < N; K++) {
            int s = sn_s(S, K), c = sn_c(S, K);
            i64 ld = s + c;
            for (int j = 0; j < s; j++)
                for (i64 i = j; i < ld; i++) sel[q++] = Ai[S->poff[K] + i + (i64)j * ld];
        }
    }
    free(Lp); free(Ai); free(Lh); free(Tt); free(maps); free(hoff); free(toff);
    return status;
}
