// Complex-symmetric path: the same supernodal LDL^T and selected inversion
// (Algorithm 1) for A(z) = H - z S, the matrices of the pole expansion
// (Section 4.3).  Values are complex (re, im interleaved, 16 bytes each);
// every transpose is a plain transpose, never a conjugate.  Blocks are at
// most 64 columns wide; the plan's level schedule is the deterministic one
// (Schur updates in colour groups; a diagonal step's long contraction may be
// cut into pieces, summed afterwards in a fixed order), so no kernel here
// needs atomics.  Products run on FP64 MFMA: a 64 x 64 complex output
// tile per work-group, real and imaginary parts as separate accumulators,
// operands staged through LDS in 16-deep chunks.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"
#include "plan.hpp"
#include "tiles.hpp"

namespace selinv {
namespace {

typedef double z2 __attribute__((ext_vector_type(2)));  // (re, im)

__device__ __forceinline__ z2 zmul(z2 a, z2 b) { return z2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

constexpr int kZT = 64;  // output tile edge
constexpr int kZK = 16;  // contraction chunk

// ---------------------------------------------------------------------------
// A 64 x 64 complex product tile on FP64 MFMA: real and imaginary parts in
// separate LDS planes, four waves of 32 x 32 (2 x 2 MFMA tiles each), and
// per 4-deep step four real products per output tile:
//   C_re += A_re B_re - A_im B_im,  C_im += A_re B_im + A_im B_re.
// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16]; result
// element (l/16 + 4 v, l%16) in register v.  Operands of the next chunk are
// loaded into registers while the current one's products run.
// ---------------------------------------------------------------------------
typedef double zd4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ zd4 zmfma(double a, double b, zd4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kZP = kZT + 4;  // padded LDS row

struct ZLdsM {
    double ar[kZK][kZP], ai[kZK][kZP], br[kZK][kZP], bi[kZK][kZP];
};

struct ZAcc {
    zd4 re[2][2], im[2][2];
};

struct ZNoHook {
    __device__ void operator()() const {}
};

// after_first: loads of the caller's own, issued once the first chunk's
// operand loads are in flight (they may then wait under the products)
template <class LA, class LB, class AF = ZNoHook>
__device__ __forceinline__ void ztile_mfma(ZLdsM& L, int K, ZAcc& acc, LA loadA, LB loadB, AF after_first = AF())
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm0 = (wave & 1) * 32, wn0 = (wave >> 1) * 32;
    constexpr int NQ = (kZK * kZT) / kThreads;
    z2 ra[NQ], rb[NQ];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = t + q * kThreads, kk = e / kZT, i = e % kZT;
            ra[q] = loadA(k0 + kk, i);
            rb[q] = loadB(k0 + kk, i);
        }
    };
    if (K > 0) fetch(0);
    after_first();
    for (int k0 = 0; k0 < K; k0 += kZK) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = t + q * kThreads, kk = e / kZT, i = e % kZT;
            L.ar[kk][i] = ra[q].x;
            L.ai[kk][i] = ra[q].y;
            L.br[kk][i] = rb[q].x;
            L.bi[kk][i] = rb[q].y;
        }
        __syncthreads();
        if (k0 + kZK < K) fetch(k0 + kZK);
#pragma unroll
        for (int ks = 0; ks < kZK / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            double xr[2], xi[2], yr[2], yi[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                xr[m] = L.ar[kr][wm0 + 16 * m + (lane & 15)];
                xi[m] = L.ai[kr][wm0 + 16 * m + (lane & 15)];
                yr[m] = L.br[kr][wn0 + 16 * m + (lane & 15)];
                yi[m] = L.bi[kr][wn0 + 16 * m + (lane & 15)];
            }
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n) {
                    acc.re[m][n] = zmfma(xr[m], yr[n], acc.re[m][n]);
                    acc.re[m][n] = zmfma(-xi[m], yi[n], acc.re[m][n]);
                    acc.im[m][n] = zmfma(xr[m], yi[n], acc.im[m][n]);
                    acc.im[m][n] = zmfma(xi[m], yr[n], acc.im[m][n]);
                }
        }
        __syncthreads();
    }
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 15\n\ts_nop 15\n\ts_nop 15\n\ts_nop 15" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// f(i, j, value) for every element of the tile (tile-local i, j)
template <class F>
__device__ __forceinline__ void zvisit(const ZAcc& acc, F f)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave & 1) * 32, wn0 = (wave >> 1) * 32;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                f(wm0 + 16 * m + (lane >> 4) + 4 * v, wn0 + 16 * n + (lane & 15), z2{acc.re[m][n][v], acc.im[m][n][v]});
}

__device__ __forceinline__ z2 zload(const double* p, int64_t e) { return *reinterpret_cast<const z2*>(p + 2 * e); }
__device__ __forceinline__ void zstore(double* p, int64_t e, z2 v) { *reinterpret_cast<z2*>(p + 2 * e) = v; }

// 1 / b: the hardware reciprocal of |b|^2 refined by two Newton steps
// (each doubles the correct bits of the ~23-bit estimate), then b's
// conjugate scaled by it
__device__ __forceinline__ z2 zrecip(z2 b)
{
    const double den = b.x * b.x + b.y * b.y;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    return z2{b.x * r, -b.y * r};
}

// ---------------------------------------------------------------------------
// Diagonal block by the symmetric sweep (Gauss-Jordan) in registers: pivot p
// in natural order (d = M(p,p), c = column p) sets M(i,j) -= c_i c_j / d,
// M(i,p) = c_i / d, M(p,p) = -1/d, plain (not conjugate) products, so after
// all s pivots M = -F_KK^{-1} = -T_K; only T leaves the kernel.  Thread
// (tx, ty) holds the lower 16 x 16 sub-blocks' entries (tx + 16a, ty + 16b),
// a >= b; a pivot's column goes through LDS (two alternating slots, one
// barrier per pivot).  Row and column p are cleared by lane masks and the
// pivot's own entries of the update vectors set to -1/d (rows) and -1
// (columns), so one rank-1 pass also writes the new row and column p.  Per
// pivot the slots holding the next pivot's column are updated first and the
// column published; the rest follow the barrier, while that column's LDS
// reads are in flight.  s <= 64, one work-group per block; a zero or
// non-finite pivot latches its column.
// ---------------------------------------------------------------------------
template <int N, class Fn>
__device__ __forceinline__ void zfor(Fn&& f)
{
    if constexpr (N > 0) {
        zfor<N - 1>(f);
        f(std::integral_constant<int, N - 1>{});
    }
}

__device__ __forceinline__ z2 zuniform(z2 v)
{
    const double x = v.x, y = v.y;
    const int a = __builtin_amdgcn_readfirstlane(__double2loint(x)), b = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    const int c = __builtin_amdgcn_readfirstlane(__double2loint(y)), e = __builtin_amdgcn_readfirstlane(__double2hiint(y));
    return z2{__hiloint2double(b, a), __hiloint2double(e, c)};
}

__global__ __launch_bounds__(kThreads) void k_zdiag(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                    double* __restrict__ Lp, double* __restrict__ Tp,
                                                    unsigned long long* __restrict__ status)
{
    constexpr int NB = kZT / 16;
    constexpr int NS = NB * (NB + 1) / 2;
    __shared__ z2 cb[2][kZT];
    const BlockDesc d = blk[tasks[blockIdx.x].b];
    const int s = d.s, tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t ld = (int64_t)d.s + d.c;
    auto slot = [](int a, int b) { return a * (a + 1) / 2 + b; };
    z2 M[NS];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tx + 16 * a, k = ty + 16 * b;
            z2 v = {0.0, 0.0};
            if (i < s && k < s) v = i >= k ? zload(Lp, d.poff + i + (int64_t)k * ld) : zload(Lp, d.poff + k + (int64_t)i * ld);
            M[slot(a, b)] = v;
        }
    // column p into col: rows at and below p's sub-block row from the
    // column's owners, the rows above from the owners of row p
    auto publish = [&](int p, z2* col) {
        const int pt = p & 15, pb = p >> 4;
        zfor<NB>([&](auto c) {
            constexpr int b0 = decltype(c)::value;
            if (pb == b0) {
                if (ty == pt) {
#pragma unroll
                    for (int a = b0; a < NB; ++a) col[tx + 16 * a] = M[slot(a, b0)];
                }
                if (tx == pt) {
#pragma unroll
                    for (int b = 0; b < b0; ++b) col[ty + 16 * b] = M[slot(b0, b)];
                }
            }
        });
    };
    if (s > 0) publish(0, cb[0]);
    __syncthreads();
    // column p as read from LDS: rows tx + 16a, rows ty + 16b, the pivot
    z2 ri[NB], rk[NB], dp;
    auto read_col = [&](int p) {
        const z2* col = cb[p & 1];
#pragma unroll
        for (int a = 0; a < NB; ++a) ri[a] = col[tx + 16 * a];
#pragma unroll
        for (int b = 0; b < NB; ++b) rk[b] = col[ty + 16 * b];
        dp = zuniform(col[p]);
    };
    if (s > 0) read_col(0);
    int bad = -1;
    for (int p = 0; p < s; ++p) {
        if (!((dp.x != 0.0 || dp.y != 0.0) && isfinite(dp.x) && isfinite(dp.y))) {
            bad = p;
            break;
        }
        const z2 inv = zrecip(dp);
        bool rz[NB], cz[NB];
        z2 si[NB], sk[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            rz[a] = tx + 16 * a == p;
            si[a] = rz[a] ? -inv : zmul(ri[a], inv);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            cz[b] = ty + 16 * b == p;
            sk[b] = cz[b] ? z2{-1.0, 0.0} : rk[b];
        }
        auto upd = [&](int a, int b) {
            const z2 m = (rz[a] || cz[b]) ? z2{0.0, 0.0} : M[slot(a, b)];
            M[slot(a, b)] = m - zmul(si[a], sk[b]);
        };
        // the slots of the next pivot's sub-block column and row first, so
        // that its column is published (and read) while the rest update
        const int q = p + 1, qb = q >> 4;
        if (qb >= NB) {  // the last pivot of a full block
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) upd(a, b);
        }
        zfor<NB>([&](auto cc) {
            constexpr int b0 = decltype(cc)::value;
            if (qb == b0) {
#pragma unroll
                for (int a = b0; a < NB; ++a) upd(a, b0);
#pragma unroll
                for (int b = 0; b < b0; ++b) upd(b0, b);
                if (q < s) publish(q, cb[q & 1]);
                __syncthreads();
                if (q < s) read_col(q);
#pragma unroll
                for (int a = 0; a < NB; ++a)
#pragma unroll
                    for (int b = 0; b <= a; ++b)
                        if (a != b0 && b != b0) upd(a, b);
            }
        });
    }
    if (bad >= 0) {  // every thread took the same branch
        if (tid == 0) atomicMin(status, (unsigned long long)(d.first + bad));
        return;
    }
    // T = -M from the lower triangle (exactly symmetric)
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tx + 16 * a, j = ty + 16 * b;
            if (i < s && j < s && i >= j) {
                zstore(Tp, d.woff + i + (int64_t)j * s, -M[slot(a, b)]);
                zstore(Tp, d.woff + j + (int64_t)i * s, -M[slot(a, b)]);
            }
        }
}

// L_hat(C,K) rows [r0, r0+64) = F(C,K) T_K
__global__ __launch_bounds__(kThreads) void k_zpanel(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                     const double* __restrict__ Lp, double* __restrict__ Hp,
                                                     const double* __restrict__ Tp)
{
    const Task tk = tasks[blockIdx.x];
    const BlockDesc d = blk[tk.b];
    const int s = d.s, c = d.c, r0 = tk.i0;
    const int64_t ld = (int64_t)s + c;
    auto la = [&](int k, int i) { return (k < s && r0 + i < c) ? zload(Lp, d.poff + s + r0 + i + (int64_t)k * ld) : z2{0, 0}; };
    auto lb = [&](int k, int j) { return (k < s && j < s) ? zload(Tp, d.woff + k + (int64_t)j * s) : z2{0, 0}; };
    auto out = [&](int ti, int j, z2 v) {
        const int i = r0 + ti;
        if (i < c && j < s) zstore(Hp, d.hoff + i + (int64_t)j * c, v);
    };
    __shared__ ZLdsM L;
    ZAcc acc = {};
    ztile_mfma(L, s, acc, la, lb);
    zvisit(acc, out);
}

// Schur update of one 64 x 64 lower tile (rows i0.., columns k0.. of C):
// F(C[i], C[k]) -= sum_t L_hat(i, t) F(C[k], t), scattered into the owning
// ancestor panels; the tasks of one launch touch disjoint entries.  The
// scatter targets do not depend on the product: their (cbase, rbase) pairs
// are loaded before the products and the rel entries under them, and the
// epilogue reads every target before it writes the first.
__global__ __launch_bounds__(kThreads) void k_zschur(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                     double* __restrict__ Lp, const double* __restrict__ Hp,
                                                     const int64_t* __restrict__ cr2, const int32_t* __restrict__ rel)
{
    typedef int64_t i64v2 __attribute__((ext_vector_type(2)));
    const Task tk = tasks[blockIdx.x];
    const BlockDesc d = blk[tk.b];
    const int s = d.s, c = d.c, i0 = tk.i0, k0 = tk.j0;
    const int64_t ld = (int64_t)s + c;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave & 1) * 32, wn0 = (wave >> 1) * 32;
    // this thread's outputs (as zvisit visits them): rows i0 + wm0 + 16m +
    // lane / 16 + 4v, columns k0 + wn0 + 16n + lane % 16
    auto row_of = [&](int m, int v) { return i0 + wm0 + 16 * m + (lane >> 4) + 4 * v; };
    auto col_of = [&](int n) { return k0 + wn0 + 16 * n + (lane & 15); };
    auto live = [&](int m, int n, int v) {
        const int ii = row_of(m, v), kk = col_of(n);
        return ii < c && kk < c && ii >= kk;
    };
    int64_t cb[2], rb[2];
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int kk = col_of(n);
        const i64v2 cr = *reinterpret_cast<const i64v2*>(cr2 + 2 * (d.coff + (kk < c ? kk : 0)));
        cb[n] = cr.x;
        rb[n] = cr.y;
    }
    int32_t ro[2][2][4];
    auto prefetch = [&]() {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int v = 0; v < 4; ++v) ro[m][n][v] = rel[rb[n] + (live(m, n, v) ? row_of(m, v) : 0)];
    };
    auto la = [&](int t, int i) { return (t < s && i0 + i < c) ? zload(Hp, d.hoff + i0 + i + (int64_t)t * c) : z2{0, 0}; };
    auto lb = [&](int t, int k) { return (t < s && k0 + k < c) ? zload(Lp, d.poff + s + k0 + k + (int64_t)t * ld) : z2{0, 0}; };
    __shared__ ZLdsM L;
    ZAcc acc = {};
    ztile_mfma(L, s, acc, la, lb, prefetch);
    z2 old[2][2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                old[m][n][v] = live(m, n, v) ? zload(Lp, cb[n] + ro[m][n][v]) : z2{0.0, 0.0};
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (live(m, n, v))
                    zstore(Lp, cb[n] + ro[m][n][v], old[m][n][v] - z2{acc.re[m][n][v], acc.im[m][n][v]});
}

// Ainv(C,K) rows [r0, r0+64) = -G L_hat with G = Ainv(C,C) gathered from the
// ancestors' inverse panels: G(i,k) = Ainv[cbase[p] + rel[rbase[p] + q]] with
// p = min(i,k), q = max(i,k) (lower entries; the upper ones by symmetry).
// Each element's address is a chain of three dependent loads, so the loop is
// pipelined over four chunks, one stage a chunk apart: (cbase, rbase) pairs
// of chunk n+3, rel entries of chunk n+2, values of chunk n+1 (G and L_hat),
// the LDS planes of chunk n feeding the MFMAs.  Chunks entirely above the
// diagonal band (every k past the tile's rows, p = i) are read along k, so
// sixteen lanes walk one row of an ancestor panel; the others along i.
// Loads are unconditional (a padding element reads an in-bounds stand-in and
// is zeroed by its mask at the LDS store), so no wait sits behind a branch.
// Three work-groups per CU (registers capped at 168, a few spilled) measured
// faster than two: 39.1 vs 39.8 ms for the 32-pole batch.  kPiece (kernel
// k_zgemm_piece): the contraction runs over rows [kb, ke) of C (kb on a
// 16-row chunk boundary) and the tile's G L_hat goes to scratch slot `pad`
// (row-major 64 x 64 complex), for k_zgemm_sum to complete.  The two are
// separate kernels: with the piece's extra argument and range the whole-tile
// kernel spilled 13 registers instead of 3 and ran the batch 5 % slower.
template <bool kPiece>
__device__ __forceinline__ void zgemm_body(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                    double* __restrict__ Ap, const double* __restrict__ Hp,
                                                    const int64_t* __restrict__ cr2, const int32_t* __restrict__ rel,
                                                    double* __restrict__ Zs)
{
    typedef int64_t i64v2 __attribute__((ext_vector_type(2)));
    const Task tk = tasks[blockIdx.x];
    const BlockDesc d = blk[tk.b];
    const int s = d.s, c = d.c, r0 = tk.i0;
    const int64_t ld = (int64_t)s + c;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm0 = (wave & 1) * 32, wn0 = (wave >> 1) * 32;
    constexpr int NQ = (kZK * kZT) / kThreads;  // elements of each operand per thread and chunk
    // kb is a multiple of kZK: the chunks from ch0 on start at row kb
    const int ke = kPiece ? tk.ke : c, ch0 = kPiece ? tk.kb / kZK : 0, nch = (ke + kZK - 1) / kZK;
    const double* Lh = Hp + 2 * d.hoff;
    auto along_of = [&](int ch) { return ch * kZK >= r0 + kZT; };
    // stage M: (cbase, rbase) of p and q (-1: padding); stage R: cbase and
    // the rel entry; stage V: the values
    int64_t m_cb[NQ], m_rb[NQ];
    int m_q[NQ];
    int64_t r_cb[NQ];
    int32_t r_rel[NQ];
    bool r_ok[NQ];
    z2 v_a[NQ], v_b[NQ];
    bool v_ok[NQ], v_bok[NQ], v_al = false;
    auto stage_m = [&](int ch) {
        const bool al = along_of(ch);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = t + q * kThreads;
            const int k = ch * kZK + (al ? (e & 15) : (e >> 6)), i = r0 + (al ? (e >> 4) : (e & 63));
            const bool ok = ch < nch && k < ke && i < c;
            const int64_t p = d.coff + (ok ? (i >= k ? k : i) : 0);
            const i64v2 cr = *reinterpret_cast<const i64v2*>(cr2 + 2 * p);
            m_cb[q] = cr.x;
            m_rb[q] = cr.y;
            m_q[q] = ok ? (i >= k ? i : k) : -1;
        }
    };
    auto stage_r = [&]() {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            r_ok[q] = m_q[q] >= 0;
            r_rel[q] = rel[m_rb[q] + (r_ok[q] ? m_q[q] : 0)];
            r_cb[q] = m_cb[q];
        }
    };
    auto stage_v = [&](int ch) {
        v_al = along_of(ch);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            v_a[q] = zload(Ap, r_cb[q] + r_rel[q]);
            v_ok[q] = r_ok[q];
            // L_hat(k, j) along k (contiguous), a stand-in past the ends
            const int e = t + q * kThreads;
            const int k = ch * kZK + (e & 15), j = e >> 4;
            v_bok[q] = k < ke && j < s;
            v_b[q] = zload(Lh, v_bok[q] ? k + (int64_t)j * c : 0);
        }
    };
    __shared__ ZLdsM L;
    auto stage_store = [&]() {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = t + q * kThreads;
            const int kk = v_al ? (e & 15) : (e >> 6), i = v_al ? (e >> 4) : (e & 63);
            const z2 x = v_ok[q] ? v_a[q] : z2{0.0, 0.0};
            L.ar[kk][i] = x.x;
            L.ai[kk][i] = x.y;
            const z2 y = v_bok[q] ? v_b[q] : z2{0.0, 0.0};
            L.br[e & 15][e >> 4] = y.x;
            L.bi[e & 15][e >> 4] = y.y;
        }
    };
    ZAcc acc = {};
    stage_m(ch0);
    stage_r();
    stage_v(ch0);
    stage_m(ch0 + 1);
    stage_r();
    stage_m(ch0 + 2);
    // registers now: values of the first chunk, rel entries of the second,
    // pairs of the third
    for (int ch = ch0; ch < nch; ++ch) {
        stage_store();
        __syncthreads();
        stage_v(ch + 1);
        stage_r();
        stage_m(ch + 3);
#pragma unroll
        for (int ks = 0; ks < kZK / 4; ++ks) {
            const int kr = 4 * ks + (lane >> 4);
            double xr[2], xi[2], yr[2], yi[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                xr[m] = L.ar[kr][wm0 + 16 * m + (lane & 15)];
                xi[m] = L.ai[kr][wm0 + 16 * m + (lane & 15)];
                yr[m] = L.br[kr][wn0 + 16 * m + (lane & 15)];
                yi[m] = L.bi[kr][wn0 + 16 * m + (lane & 15)];
            }
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n) {
                    acc.re[m][n] = zmfma(xr[m], yr[n], acc.re[m][n]);
                    acc.re[m][n] = zmfma(-xi[m], yi[n], acc.re[m][n]);
                    acc.im[m][n] = zmfma(xr[m], yi[n], acc.im[m][n]);
                    acc.im[m][n] = zmfma(xi[m], yr[n], acc.im[m][n]);
                }
        }
        __syncthreads();
    }
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 15\n\ts_nop 15\n\ts_nop 15\n\ts_nop 15" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (kPiece) {
        double* z = Zs + (int64_t)tk.pad * kZSlotDoubles;
        zvisit(acc, [&](int ti, int j, z2 v) { zstore(z, (int64_t)ti * kZT + j, v); });
    } else {
        zvisit(acc, [&](int ti, int j, z2 v) {
            const int i = r0 + ti;
            if (i < c && j < s) zstore(Ap, d.poff + s + i + (int64_t)j * ld, -v);
        });
    }
}

__global__ __launch_bounds__(kThreads, 3) void k_zgemm(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                    double* __restrict__ Ap, const double* __restrict__ Hp,
                                                    const int64_t* __restrict__ cr2, const int32_t* __restrict__ rel)
{
    zgemm_body<false>(tasks, blk, Ap, Hp, cr2, rel, nullptr);
}
__global__ __launch_bounds__(kThreads, 3) void k_zgemm_piece(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                    double* __restrict__ Ap, const double* __restrict__ Hp,
                                                    const int64_t* __restrict__ cr2, const int32_t* __restrict__ rel,
                                                    double* __restrict__ Zs)
{
    zgemm_body<true>(tasks, blk, Ap, Hp, cr2, rel, Zs);
}

// The sum of a split task's pieces (slots kb .. kb + bn - 1) at element e of
// the row-major 64 x 64 tile: four running sums over the pieces q = 4m + r,
// combined in a fixed order, so that four loads are in flight at a time.
__device__ __forceinline__ z2 zslot_sum(const double* __restrict__ z0, int np, int e)
{
    z2 a[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    int q = 0;
    for (; q + 4 <= np; q += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] += zload(z0 + (int64_t)(q + r) * kZSlotDoubles, e);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
        if (q + r < np) a[r] += zload(z0 + (int64_t)(q + r) * kZSlotDoubles, e);
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// Rows of a 64 x 64 summing tile one work-group handles (one element per
// thread); a summing task takes kZT / kZSumRows work-groups (blockIdx.y), so
// the reads of its pieces spread over that many CUs.
constexpr int kZSumRows = kThreads / kZT;

// A split gather-GEMM tile: the sum of its pieces' G L_hat, stored negated
// as Ainv(C,K) rows [r0, r0+64); this work-group's rows ti0 .. ti0 + 3.
__global__ __launch_bounds__(kThreads) void k_zgemm_sum(const Task* __restrict__ tasks,
                                                        const BlockDesc* __restrict__ blk, double* __restrict__ Ap,
                                                        const double* __restrict__ Zs)
{
    const Task tk = tasks[blockIdx.x];
    const BlockDesc d = blk[tk.b];
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int ti = blockIdx.y * kZSumRows + threadIdx.x / kZT, j = threadIdx.x % kZT, i = tk.i0 + ti;
    if (i >= c || j >= s) return;
    const z2 x = zslot_sum(Zs + (int64_t)tk.kb * kZSlotDoubles, tk.bn, ti * kZT + j);
    zstore(Ap, d.poff + s + i + (int64_t)j * ld, -x);
}

// Ainv(K,K) = T - (P + P^T) / 2 with P = L_hat^T Ainv(C,K) (lower triangle),
// the contraction over rows [kb, ke) of C.  A piece of a split block (flags
// bit 5) stores its P to scratch slot `pad` (row-major, kZMaxS x kZMaxS
// complex) instead; k_zsdiag_sum completes the block.
static_assert(kZT == kZMaxS, "one output tile holds a whole diagonal block");
__global__ __launch_bounds__(kThreads) void k_zsdiag(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                     double* __restrict__ Ap, const double* __restrict__ Hp,
                                                     const double* __restrict__ Tp, double* __restrict__ Zs)
{
    // the product's operand planes, then P for the transpose (the tile loop
    // ends with a barrier, so P may reuse the space)
    __shared__ union {
        ZLdsM L;
        z2 P[kZT][kZT + 1];
    } U;
    auto& P = U.P;
    const Task tk = tasks[blockIdx.x];
    const BlockDesc d = blk[tk.b];
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int kb = tk.kb, ke = tk.ke;
    auto la = [&](int r, int i) {
        r += kb;
        return (r < ke && i < s) ? zload(Hp, d.hoff + r + (int64_t)i * c) : z2{0, 0};
    };
    auto lb = [&](int r, int j) {
        r += kb;
        return (r < ke && j < s) ? zload(Ap, d.poff + s + r + (int64_t)j * ld) : z2{0, 0};
    };
    ZAcc acc = {};
    ztile_mfma(U.L, ke - kb, acc, la, lb);
    if (tk.flags & 32) {
        double* z = Zs + (int64_t)tk.pad * kZSlotDoubles;
        zvisit(acc, [&](int i, int j, z2 v) { zstore(z, (int64_t)i * kZT + j, v); });
        return;
    }
    zvisit(acc, [&](int i, int j, z2 v) { P[i][j] = v; });
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 4 * tx + u, j = 4 * ty + v;
            if (i < s && j < s && i >= j) {
                const z2 p = 0.5 * (P[i][j] + P[j][i]);
                zstore(Ap, d.poff + i + (int64_t)j * ld, zload(Tp, d.woff + i + (int64_t)j * s) - p);
            }
        }
}

// A split block's diagonal step: P = the sum of its pieces' partial
// products, then Ainv(K,K) = T - (P + P^T) / 2 on the lower triangle; this
// work-group's rows i0 .. i0 + 3 (P(i,j) and P(j,i) summed separately, each
// in the fixed order of zslot_sum).
__global__ __launch_bounds__(kThreads) void k_zsdiag_sum(const Task* __restrict__ tasks,
                                                         const BlockDesc* __restrict__ blk, double* __restrict__ Ap,
                                                         const double* __restrict__ Tp, const double* __restrict__ Zs)
{
    const Task tk = tasks[blockIdx.x];
    const BlockDesc d = blk[tk.b];
    const int s = d.s;
    const int64_t ld = (int64_t)s + d.c;
    const int i = blockIdx.y * kZSumRows + threadIdx.x / kZT, j = threadIdx.x % kZT;
    if (i >= s || j > i) return;
    const double* z0 = Zs + (int64_t)tk.kb * kZSlotDoubles;
    const z2 pij = zslot_sum(z0, tk.bn, i * kZT + j), pji = zslot_sum(z0, tk.bn, j * kZT + i);
    zstore(Ap, d.poff + i + (int64_t)j * ld, zload(Tp, d.woff + i + (int64_t)j * s) - 0.5 * (pij + pji));
}

// assemble: panel entry off[q] (a complex element) := value q; export: out
// entry q := panel entry off[q]
__global__ void k_zscatter(const double* __restrict__ src, const int64_t* __restrict__ off, int64_t n,
                           double* __restrict__ dst)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        zstore(dst, off[q], zload(src, q));
}

__global__ void k_zgather(const double* __restrict__ src, const int64_t* __restrict__ off, int64_t n,
                          double* __restrict__ dst)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        zstore(dst, q, zload(src, off[q]));
}

unsigned zgrid(int64_t n)
{
    int64_t g = (n + kThreads - 1) / kThreads;
    return (unsigned)(g < 1 ? 1 : g > 65536 ? 65536 : g);
}
}  // namespace

hipError_t launch_zassemble(const double* vals, const int64_t* off, int64_t n, double* Lp, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_zscatter, dim3(zgrid(n)), dim3(kThreads), 0, s, vals, off, n, Lp);
    return hipGetLastError();
}

hipError_t launch_zexport(const double* Ap, const int64_t* off, int64_t n, double* out, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_zgather, dim3(zgrid(n)), dim3(kThreads), 0, s, Ap, off, n, out);
    return hipGetLastError();
}

hipError_t launch_zfactor_level(const DevPtrs& D, int64_t diag0, int64_t ndiag, int64_t panel0, int64_t npanel,
                                const int64_t* schur_cuts, int ncuts, hipStream_t s)
{
    if (ndiag > 0)
        hipLaunchKernelGGL(k_zdiag, dim3((unsigned)ndiag), dim3(kThreads), 0, s, D.t_ldlt + diag0, D.blocks, D.Lp,
                           D.Tp, D.status);
    if (npanel > 0)
        hipLaunchKernelGGL(k_zpanel, dim3((unsigned)npanel), dim3(kThreads), 0, s, D.t_panel + panel0, D.blocks,
                           (const double*)D.Lp, D.Hp, (const double*)D.Tp);
    for (int g = 0; g + 1 < ncuts; g++) {
        const int64_t n = schur_cuts[g + 1] - schur_cuts[g];
        if (n > 0)
            hipLaunchKernelGGL(k_zschur, dim3((unsigned)n), dim3(kThreads), 0, s, D.t_schur + schur_cuts[g], D.blocks,
                               D.Lp, (const double*)D.Hp, D.cr2, D.rel);
    }
    return hipGetLastError();
}

hipError_t launch_zinvert_level(const DevPtrs& D, const int64_t gemm[4], int64_t sdiag0, int64_t sdiag_cut,
                                int64_t sdiag1, hipStream_t s)
{
    if (gemm[1] > gemm[0])
        hipLaunchKernelGGL(k_zgemm, dim3((unsigned)(gemm[1] - gemm[0])), dim3(kThreads), 0, s,
                           D.t_gemm + gemm[0], D.blocks, D.Ap, (const double*)D.Hp, D.cr2, D.rel);
    if (gemm[2] > gemm[1])
        hipLaunchKernelGGL(k_zgemm_piece, dim3((unsigned)(gemm[2] - gemm[1])), dim3(kThreads), 0, s,
                           D.t_gemm + gemm[1], D.blocks, D.Ap, (const double*)D.Hp, D.cr2, D.rel, D.Zs);
    if (gemm[3] > gemm[2])
        hipLaunchKernelGGL(k_zgemm_sum, dim3((unsigned)(gemm[3] - gemm[2]), kZT / kZSumRows), dim3(kThreads), 0, s,
                           D.t_gemm + gemm[2], D.blocks, D.Ap, (const double*)D.Zs);
    if (sdiag_cut > sdiag0)
        hipLaunchKernelGGL(k_zsdiag, dim3((unsigned)(sdiag_cut - sdiag0)), dim3(kThreads), 0, s, D.t_sdiag + sdiag0,
                           D.blocks, D.Ap, (const double*)D.Hp, (const double*)D.Tp, D.Zs);
    if (sdiag1 > sdiag_cut)
        hipLaunchKernelGGL(k_zsdiag_sum, dim3((unsigned)(sdiag1 - sdiag_cut), kZT / kZSumRows), dim3(kThreads), 0, s,
                           D.t_sdiag + sdiag_cut, D.blocks, D.Ap, (const double*)D.Tp, (const double*)D.Zs);
    return hipGetLastError();
}

}  // namespace selinv
