// Device kernels for the supernodal LDL^T and the selected inversion.
//
// Data layout (all FP64, in one caller-bound workspace):
//   Lp  panels of the factor: block B is an (s+c) x s column-major panel,
//       ld = s+c; rows = cols(B) then C(B).  Holds A, then L (D on the
//       diagonal of the s x s block).
//   Ap  same layout, holds the selected entries of A^{-1}.
//   Hp  L_hat(C,B) = L(C,B) L_BB^{-1}, c x s column-major (ld = c).
//   Wp  W = L_BB^{-1} (s x s); Tp  T = L_BB^{-T} D_B^{-1} L_BB^{-1} (s x s).
// Block index maps: for position r of C(B), cbase[r] is the arena offset of
// column C[r] inside its owning block J, and rel[rbase[r] + i] the row of
// C[i] (i >= r's segment start) inside rows(J).  So the entry
// A^{-1}(C[i], C[k]), i >= k, lives at cbase[k] + rel[rbase[k] + i].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "plan.hpp"
#include "tiles.hpp"

namespace selinv {

__global__ void k_fill(double* __restrict__ p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_status_reset(unsigned long long* status)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = ~0ull;
}

__global__ void k_scatter_set(const double* __restrict__ src, const int64_t* __restrict__ off, int64_t n,
                              double* __restrict__ dst)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[off[i]] = src[i];
}

__global__ void k_gather(const double* __restrict__ src, const int64_t* __restrict__ off, int64_t n,
                         double* __restrict__ dst)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[off[i]];
}

// ---------------------------------------------------------------------------
// Factor, diagonal block: F_BB = L_BB D_B L_BB^T in place (right-looking, no
// pivoting), then W = L_BB^{-1} and T = W^T D^{-1} W.  One work-group per
// block.  A pivot that is zero, not finite, or (require_spd) not positive is
// latched as the smallest failing permuted column.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_ldlt_diag(const Task* __restrict__ tasks,
                                                        const BlockDesc* __restrict__ blk, double* __restrict__ Lp,
                                                        double* __restrict__ Wp, double* __restrict__ Tp,
                                                        unsigned long long* __restrict__ status, int require_spd)
{
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    const int s = d.s;
    const int64_t ld = (int64_t)d.s + d.c;
    double* F = Lp + d.poff;
    double* W = Wp + d.woff;
    double* T = Tp + d.woff;
    const int tid = threadIdx.x;
    for (int j = 0; j < s; ++j) {
        __syncthreads();
        const double dj = F[j + j * ld];
        const bool ok = isfinite(dj) && dj != 0.0 && (!require_spd || dj > 0.0);
        if (!ok && tid == 0) atomicMin(status, (unsigned long long)(d.first + j));
        const int m = s - j - 1;
        // L(i,j) for i > j inside the block: keep F(i,j) for the update first
        for (int e = tid; e < m * m; e += kThreads) {
            const int ii = e % m, kk = e / m;
            if (ii >= kk) {
                const int i = j + 1 + ii, k = j + 1 + kk;
                F[i + k * ld] -= F[i + j * ld] * F[k + j * ld] / dj;
            }
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < s; i += kThreads) F[i + j * ld] /= dj;
    }
    __syncthreads();
    // W = L^{-1}: column j by forward substitution (one thread per column)
    for (int j = tid; j < s; j += kThreads) {
        for (int i = 0; i < j; ++i) W[i + j * s] = 0.0;
        W[j + j * s] = 1.0;
        for (int i = j + 1; i < s; ++i) {
            double v = 0.0;
            for (int k = j; k < i; ++k) v += F[i + k * ld] * W[k + j * s];
            W[i + j * s] = -v;
        }
    }
    __syncthreads();
    // T(i,j) = sum_{k >= max(i,j)} W(k,i) W(k,j) / d_k
    for (int e = tid; e < s * s; e += kThreads) {
        const int i = e % s, j = e / s;
        const int m = i > j ? i : j;
        double v = 0.0;
        for (int k = m; k < s; ++k) v += W[k + i * s] * W[k + j * s] / F[k + k * ld];
        T[e] = v;
    }
}

// ---------------------------------------------------------------------------
// Factor, panel: L(C,B) = F(C,B) W^T D^{-1} (in place) and, fused,
// the normalised panel L_hat(C,B) = L(C,B) W = F(C,B) T (Algorithm 1 step 2).
// One work-group per kPanelRows rows of C(B).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_panel(const Task* __restrict__ tasks,
                                                    const BlockDesc* __restrict__ blk, double* __restrict__ Lp,
                                                    double* __restrict__ Hp, const double* __restrict__ Wp,
                                                    const double* __restrict__ Tp)
{
    __shared__ double Fs[kPanelRows][kMaxS + 1];
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    double* F = Lp + d.poff;
    const double* W = Wp + d.woff;
    const double* T = Tp + d.woff;
    const int r0 = t.i0;
    const int nr = min(kPanelRows, c - r0);
    for (int e = threadIdx.x; e < kPanelRows * s; e += kThreads) {
        const int rr = e % kPanelRows, k = e / kPanelRows;
        Fs[rr][k] = rr < nr ? F[s + r0 + rr + k * ld] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kPanelRows * s; e += kThreads) {
        const int rr = e % kPanelRows, j = e / kPanelRows;
        if (rr >= nr) continue;
        double v = 0.0;
        for (int k = 0; k <= j; ++k) v += Fs[rr][k] * W[j + k * s];
        double h = 0.0;
        for (int k = 0; k < s; ++k) h += Fs[rr][k] * T[k + j * s];
        F[s + r0 + rr + j * ld] = v / F[j + j * ld];
        Hp[d.hoff + r0 + rr + (int64_t)j * c] = h;
    }
}

// ---------------------------------------------------------------------------
// Factor, Schur update: F(C,C) -= L(C,B) D_B L(C,B)^T, lower half, added into
// the ancestor panels through the block index maps (FP64 atomics: sibling
// blocks of one level may update the same ancestor entry).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_schur(const Task* __restrict__ tasks,
                                                    const BlockDesc* __restrict__ blk, double* __restrict__ Lp,
                                                    const int64_t* __restrict__ cbase,
                                                    const int64_t* __restrict__ rbase,
                                                    const int32_t* __restrict__ rel)
{
    constexpr int TS = kSchurTile;
    __shared__ double As[TS][TS + 1];
    __shared__ double Bs[TS][TS + 1];
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const double* F = Lp + d.poff;
    const int i0 = t.i0, k0 = t.j0;
    const int ii = threadIdx.x % TS, kq = threadIdx.x / TS;  // kq in 0..7, 4 columns each
    double acc[4] = {0, 0, 0, 0};
    for (int t0 = 0; t0 < s; t0 += TS) {
        for (int e = threadIdx.x; e < TS * TS; e += kThreads) {
            const int r = e % TS, tt = e / TS;
            const int col = t0 + tt;
            double a = 0.0, b = 0.0;
            if (col < s) {
                const double dc = F[col + col * ld];
                if (i0 + r < c) a = F[s + i0 + r + col * ld] * dc;
                if (k0 + r < c) b = F[s + k0 + r + col * ld];
            }
            As[r][tt] = a;
            Bs[r][tt] = b;
        }
        __syncthreads();
#pragma unroll 4
        for (int tt = 0; tt < TS; ++tt) {
            const double a = As[ii][tt];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += a * Bs[kq * 4 + q][tt];
        }
        __syncthreads();
    }
    const int i = i0 + ii;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = k0 + kq * 4 + q;
        if (i < c && k < c && i >= k) {
            const int64_t pk = d.coff + k;
            unsafeAtomicAdd(Lp + cbase[pk] + rel[rbase[pk] + i], -acc[q]);
        }
    }
}

// ---------------------------------------------------------------------------
// Selected inversion, step 3: X = Ainv(C,B) = -Ainv(C,C) L_hat(C,B).
// Ainv(C,C) is gathered from the ancestors' panels (lower entries directly,
// upper entries through symmetry) into LDS tiles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_gemm(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                   double* __restrict__ Ap, const double* __restrict__ Hp,
                                                   const int64_t* __restrict__ cbase,
                                                   const int64_t* __restrict__ rbase,
                                                   const int32_t* __restrict__ rel)
{
    constexpr int BM = kGemmBM, BN = kGemmBN, BK = kGemmBK;
    __shared__ double Gs[BK][BM + 1];
    __shared__ double Ls[BK][BN + 1];
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int r0 = t.i0, n0 = t.j0;
    const int rr = threadIdx.x % BM, nq = threadIdx.x / BM;  // 8 groups of 4 columns
    const double* H = Hp + d.hoff;
    double acc[4] = {0, 0, 0, 0};
    for (int k0 = 0; k0 < c; k0 += BK) {
        for (int e = threadIdx.x; e < BM * BK; e += kThreads) {
            const int r = e % BM, kk = e / BM;
            const int i = r0 + r, k = k0 + kk;
            double g = 0.0;
            if (i < c && k < c) {
                if (i >= k) {
                    const int64_t pk = d.coff + k;
                    g = Ap[cbase[pk] + rel[rbase[pk] + i]];
                } else {
                    const int64_t pi = d.coff + i;
                    g = Ap[cbase[pi] + rel[rbase[pi] + k]];
                }
            }
            Gs[kk][r] = g;
        }
        for (int e = threadIdx.x; e < BK * BN; e += kThreads) {
            const int kk = e % BK, nn = e / BK;
            const int k = k0 + kk, j = n0 + nn;
            Ls[kk][nn] = (k < c && j < s) ? H[k + (int64_t)j * c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            const double g = Gs[kk][rr];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += g * Ls[kk][nq * 4 + q];
        }
        __syncthreads();
    }
    const int i = r0 + rr;
    if (i < c) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = n0 + nq * 4 + q;
            if (j < s) Ap[d.poff + s + i + (int64_t)j * ld] = -acc[q];
        }
    }
}

// ---------------------------------------------------------------------------
// Selected inversion, step 4 + symmetrisation:
// Y = T - L_hat^T X, Ainv(B,B) = (Y + Y^T)/2.  One work-group per block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_sdiag(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                    double* __restrict__ Ap, const double* __restrict__ Hp,
                                                    const double* __restrict__ Tp)
{
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    double* A = Ap + d.poff;
    const double* H = Hp + d.hoff;
    const double* T = Tp + d.woff;
    for (int e = threadIdx.x; e < s * s; e += kThreads) {
        const int i = e % s, j = e / s;
        double v = 0.0;
        for (int r = 0; r < c; ++r) v += H[r + (int64_t)i * c] * A[s + r + j * ld];
        A[i + j * ld] = T[e] - v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < s * s; e += kThreads) {
        const int i = e % s, j = e / s;
        if (i > j) {
            const double m = 0.5 * (A[i + j * ld] + A[j + i * ld]);
            A[i + j * ld] = m;
            A[j + i * ld] = m;
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n)
{
    int64_t g = (n + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_status_reset(unsigned long long* status, hipStream_t s)
{
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, s, status);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_scatter_set(const double* src, const int64_t* off, int64_t n, double* dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_set, dim3(grid_for(n)), dim3(kThreads), 0, s, src, off, n, dst);
    return hipGetLastError();
}

hipError_t launch_gather(const double* src, const int64_t* off, int64_t n, double* dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kThreads), 0, s, src, off, n, dst);
    return hipGetLastError();
}

hipError_t launch_factor_level(const DevPtrs& D, int64_t diag0, int64_t ndiag, int64_t panel0, int64_t npanel,
                               int64_t schur0, int64_t nschur, int require_spd, hipStream_t s)
{
    if (ndiag > 0)
        hipLaunchKernelGGL(k_ldlt_diag, dim3((unsigned)ndiag), dim3(kThreads), 0, s, D.t_diag + diag0, D.blocks,
                           D.Lp, D.Wp, D.Tp, D.status, require_spd);
    if (npanel > 0)
        hipLaunchKernelGGL(k_panel, dim3((unsigned)npanel), dim3(kThreads), 0, s, D.t_panel + panel0, D.blocks,
                           D.Lp, D.Hp, D.Wp, D.Tp);
    if (nschur > 0)
        hipLaunchKernelGGL(k_schur, dim3((unsigned)nschur), dim3(kThreads), 0, s, D.t_schur + schur0, D.blocks,
                           D.Lp, D.cbase, D.rbase, D.rel);
    return hipGetLastError();
}

hipError_t launch_invert_level(const DevPtrs& D, int64_t gemm0, int64_t ngemm, int64_t sdiag0, int64_t nsdiag,
                               hipStream_t s)
{
    if (ngemm > 0)
        hipLaunchKernelGGL(k_gemm, dim3((unsigned)ngemm), dim3(kThreads), 0, s, D.t_gemm + gemm0, D.blocks, D.Ap,
                           D.Hp, D.cbase, D.rbase, D.rel);
    if (nsdiag > 0)
        hipLaunchKernelGGL(k_sdiag, dim3((unsigned)nsdiag), dim3(kThreads), 0, s, D.t_sdiag + sdiag0, D.blocks,
                           D.Ap, D.Hp, D.Tp);
    return hipGetLastError();
}

}  // namespace selinv
