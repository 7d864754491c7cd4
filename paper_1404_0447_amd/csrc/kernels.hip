// Device kernels for the supernodal LDL^T and the selected inversion.
//
// Data layout (all FP64, in one caller-bound workspace):
//   Lp  panels of the factor: block B is an (s+c) x s column-major panel,
//       ld = s+c; rows = cols(B) then C(B).  The s x s block holds L_BB
//       (unit diagonal implied, D on the diagonal; with 2x2 pivots it keeps
//       the assembled F_BB, whose inverse goes to Tp alone); the C rows hold
//       F(C,B), the assembled and updated entries of A (L(C,B) is
//       F(C,B) L_BB^{-T} D^{-1} and is formed only on export).
//   Ap  same layout, holds the selected entries of A^{-1}.
//   Hp  L_hat(C,B) = L(C,B) L_BB^{-1} = F(C,B) T, c x s column-major (ld c).
//   Wp  W = L_BB^{-1} (s x s); Tp  T = L_BB^{-T} D_B^{-1} L_BB^{-1} (s x s).
// Block index maps: for position r of C(B), cbase[r] is the arena offset of
// column C[r] inside its owning block J, and rel[rbase[r] + i] the row of
// C[i] (i >= r's segment start) inside rows(J).  So the entry
// A^{-1}(C[i], C[k]), i >= k, lives at cbase[k] + rel[rbase[k] + i].
//
// Dense products use v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; the 16x16 result element (l/16 + 4v, l%16) sits in
// register v of lane l.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <atomic>
#include <type_traits>
#include <utility>

#include "kernels.hpp"
#include "plan.hpp"
#include "tiles.hpp"

namespace selinv {

typedef double d4 __attribute__((ext_vector_type(4)));
// two doubles read with one load from an 8-byte aligned address
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
// (cbase, rbase) of one position, one 16-byte load
typedef int64_t i64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Wait states after the last MFMA of a loop, before its accumulators are
// read by ordinary vector instructions (the scheduler may not move anything
// across the barrier).
__device__ __forceinline__ void mfma_drain()
{
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 15\n\ts_nop 15\n\ts_nop 15\n\ts_nop 15" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Instruction interleaving for a software-pipelined MFMA loop body: NM
// slots, each one MFMA followed by its share of the other instructions of
// the body (DS reads, DS writes, global loads, VALU), so that a wave issues
// its address arithmetic and memory operations while its own MFMAs run
// instead of in a block of its own.  A prologue slot holds the DS reads the
// first MFMA needs.  Counts are hints to the scheduler: what does not fit
// the pattern is scheduled freely.
template <int NM, int NDR0, int NDR, int NDW, int NVM, int NVALU, int I>
__device__ __forceinline__ void sgb_slot()
{
    constexpr int kMfma = 0x008, kValu = 0x002, kVmemRead = 0x020, kDsRead = 0x100, kDsWrite = 0x200;
    __builtin_amdgcn_sched_group_barrier(kMfma, 1, 0);
    if constexpr ((I + 1) * NDR / NM > I * NDR / NM) __builtin_amdgcn_sched_group_barrier(kDsRead, 1, 0);
    if constexpr ((I + 1) * NDW / NM > I * NDW / NM) __builtin_amdgcn_sched_group_barrier(kDsWrite, 1, 0);
    if constexpr ((I + 1) * NVM / NM > I * NVM / NM) __builtin_amdgcn_sched_group_barrier(kVmemRead, 1, 0);
    if constexpr (NVALU > 0) __builtin_amdgcn_sched_group_barrier(kValu, NVALU, 0);
}
template <int NM, int NDR0, int NDR, int NDW, int NVM, int NVALU, int... I>
__device__ __forceinline__ void sgb_body(std::integer_sequence<int, I...>)
{
    if constexpr (NDR0 > 0) __builtin_amdgcn_sched_group_barrier(0x100, NDR0, 0);
    (sgb_slot<NM, NDR0, NDR, NDW, NVM, NVALU, I>(), ...);
}
template <int NM, int NDR0, int NDR, int NDW, int NVM, int NVALU>
__device__ __forceinline__ void sgb_interleave()
{
    sgb_body<NM, NDR0, NDR, NDW, NVM, NVALU>(std::make_integer_sequence<int, NM>{});
}

// LDS written by some lanes of a wave, then read by others
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// status[0]: smallest failing pivot column (~0 = none); status[1]: error
// flags of the persistent work queues (0 = none)
__global__ void k_status_reset(unsigned long long* status)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        status[0] = ~0ull;
        status[1] = 0ull;
    }
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

// Blocks whose products accumulate over several work-groups start from
// the lower triangle of Ainv(B,B) := T and, when the gather-GEMM is split
// (zx), X = Ainv(C,B) := 0.  One wave per column, lanes along its rows.
__device__ __forceinline__ void zero_task(const BlockDesc d, double* __restrict__ Ap, const double* __restrict__ Tp,
                                          bool zx = true, int j0 = 0, int j1 = 1 << 30)
{
    const int64_t ld = (int64_t)d.s + d.c;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    j1 = min(j1, d.s);
    for (int j = j0 + wave; j < j1; j += kThreads / 64) {
        double* col = Ap + d.poff + (int64_t)j * ld;
        const double* tcol = Tp + d.woff + (int64_t)j * d.s;
        for (int i = j + lane; i < d.s; i += 64) col[i] = tcol[i];
        if (zx)
            for (int i = lane; i < d.c; i += 64) col[d.s + i] = 0.0;
    }
}

__global__ __launch_bounds__(kThreads) void k_zero_x(const Task* __restrict__ tasks,
                                                     const BlockDesc* __restrict__ blk, double* __restrict__ Ap,
                                                     const double* __restrict__ Tp)
{
    const Task t = tasks[blockIdx.x];
    zero_task(blk[t.b], Ap, Tp, t.flags & 1, t.kb, t.ke);  // columns [kb, ke)
}

// Checkpoint copy of whole inverse panels ((s + c) x s, contiguous): dir 0
// panel -> store, dir 1 store -> panel; blocks without a slot are skipped.
__global__ __launch_bounds__(kThreads) void k_ck_copy(const Task* __restrict__ tasks,
                                                      const BlockDesc* __restrict__ blk,
                                                      const int64_t* __restrict__ ck_off, double* __restrict__ Ap,
                                                      double* __restrict__ ck, int dir)
{
    const int b = tasks[blockIdx.x].b;
    const int64_t o = ck_off[b];
    if (o < 0) return;
    const BlockDesc d = blk[b];
    const int64_t n = ((int64_t)d.s + d.c) * d.s;
    double* panel = Ap + d.poff;
    double* slot = ck + o;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
        if (dir == 0) slot[i] = panel[i];
        else panel[i] = slot[i];
    }
}

// L on the canonical pattern: diagonal-block entries are stored; an entry in
// C(B) rows is L(r,j) = sum_{k>=j} L_hat(r,k) L_BB(k,j).  One thread per column.
__global__ void k_export_L(const BlockDesc* __restrict__ blk, const int32_t* __restrict__ colblk,
                           const int64_t* __restrict__ colptrL, const int64_t* __restrict__ off, int64_t n,
                           const double* __restrict__ Lp, const double* __restrict__ Hp, double* __restrict__ out)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const BlockDesc d = blk[colblk[j]];
        const int64_t ld = (int64_t)d.s + d.c;
        for (int64_t q = colptrL[j]; q < colptrL[j + 1]; ++q) {
            const int64_t o = off[q] - d.poff;
            const int row = (int)(o % ld), col = (int)(o / ld);
            double v;
            if (row < d.s) {
                v = Lp[off[q]];
            } else {
                const int r = row - d.s;
                v = Hp[d.hoff + r + (int64_t)col * d.c];
                for (int k = col + 1; k < d.s; ++k)
                    v += Hp[d.hoff + r + (int64_t)k * d.c] * Lp[d.poff + k + (int64_t)col * ld];
            }
            out[q] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Generic 64 x BN MFMA tile: acc += A(64 x K) B(K x BN), K streamed in
// chunks of 16 through LDS, accumulated transposed (read it with
// tile_epilogue_t).  loadA(k0, kk, i) -> A(i, k0+kk) and
// loadB(k0, kk, j) -> B(k0+kk, j).  The A loads run with consecutive threads
// along i, or along kk for chunks where chunkAlongK(k0) holds (contiguous
// in k).  Four waves: BN >= 64 -> 2 x 2 waves of 32 x BN/2, else 4 x 1 waves
// of 16 x BN.
// ---------------------------------------------------------------------------
constexpr int TBM = 64, TBK = 16, TPAD = 4;

struct TileLds {
    double A[TBK][TBM + TPAD];
    double B[TBK][128 + TPAD];
};

template <int BN>
struct TileShape {
    static constexpr int WM = BN >= 64 ? 2 : 4;
    static constexpr int WN = 4 / WM;
    static constexpr int MT = TBM / WM / 16;
    static constexpr int NT = BN / WN / 16;
};

template <int BN, class FA, class FB, class FAK>
__device__ __forceinline__ void tile_mma(TileLds& L, int Kb, int Ke, d4 (&acc)[2][4], FA loadA, FB loadB,
                                         FAK chunkAlongK)
{
    using SH = TileShape<BN>;
    constexpr int NB = BN / 16;  // B elements per thread per chunk
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave % SH::WM) * (TBM / SH::WM), wn0 = (wave / SH::WM) * (BN / SH::WN);
    // the next chunk is fetched into registers while the current one feeds
    // the MFMAs, so gather latency overlaps the products
    double ra[4], rb[NB];
    bool along = false;
    auto fetch = [&](int k0) {
        along = chunkAlongK(k0);
        if (along) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = threadIdx.x + q * kThreads;
                ra[q] = loadA(k0, e & 15, e >> 4);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = threadIdx.x + q * kThreads;
                ra[q] = loadA(k0, e >> 6, e & 63);
            }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = threadIdx.x + q * kThreads;
            rb[q] = loadB(k0, e & 15, e >> 4);
        }
    };
    if (Kb < Ke) fetch(Kb);
    for (int k0 = Kb; k0 < Ke; k0 += TBK) {
        if (along) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = threadIdx.x + q * kThreads;
                L.A[e & 15][e >> 4] = ra[q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = threadIdx.x + q * kThreads;
                L.A[e >> 6][e & 63] = ra[q];
            }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = threadIdx.x + q * kThreads;
            L.B[e & 15][e >> 4] = rb[q];
        }
        __syncthreads();
        if (k0 + TBK < Ke) fetch(k0 + TBK);
#pragma unroll
        for (int ks = 0; ks < TBK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double a[SH::MT], b[SH::NT];
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt) a[mt] = L.A[kr][wm0 + mt * 16 + (lane & 15)];
#pragma unroll
            for (int nt = 0; nt < SH::NT; ++nt) b[nt] = L.B[kr][wn0 + nt * 16 + (lane & 15)];
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < SH::NT; ++nt) acc[mt][nt] = mfma(b[nt], a[mt], acc[mt][nt]);
        }
        __syncthreads();
    }
    mfma_drain();
}

// Visit every element f(i, j, value) (tile-local i, j) of a tile whose
// MFMAs ran with their operands swapped: mfma(b, a) forms the transposed
// 16 x 16 product, and register v of lane l holds row l / 16 + 4 v, column
// l % 16 of whatever product it forms, so here lane l holds row i = l % 16.
// Sixteen lanes then cover sixteen consecutive rows of one column, which
// makes the stores (and atomics) into a column-major output contiguous.
template <int BN, class F>
__device__ __forceinline__ void tile_epilogue_t(const d4 (&acc)[2][4], F f)
{
    using SH = TileShape<BN>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave % SH::WM) * (TBM / SH::WM), wn0 = (wave / SH::WM) * (BN / SH::WN);
#pragma unroll
    for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                f(wm0 + mt * 16 + (lane & 15), wn0 + nt * 16 + (lane >> 4) + 4 * v, acc[mt][nt][v]);
}

// ---------------------------------------------------------------------------
// Pipelined 64 x BN MFMA tile: acc += A(64 x K) B(K x BN) over 16-deep
// chunks, LDS double-buffered with one barrier per chunk.  While the MFMAs
// consume chunk n, chunk n+1's values (loaded an iteration earlier) go to
// the other buffer, chunk n+2's values are loaded from the addresses found
// an iteration earlier, and chunk n+3's addresses are formed.  Loads are
// unconditional: addrA(k0, kk, ii, ok) / addrB(k0, kk, j, ok) return an
// in-bounds stand-in when !ok, and the mask is applied at the LDS store.
// A chunk is read along k (contiguous in k) where alongA(k0) holds, else
// along i; B along j (kBJ: B(k, j) contiguous in j) or along k.
// ---------------------------------------------------------------------------
struct GemmLds {
    double A[2][TBK][TBM + TPAD];
    double B[2][TBK][128 + TPAD];
};

template <int BN, bool kBJ, bool kT, bool kPairK = false, class FA, class FB, class FAK, class FH>
__device__ __forceinline__ void tile_mma2(GemmLds& L, int Kb, int Ke, d4 (&acc)[2][4], FA addrA, FB addrB,
                                          FAK alongA, FH afterPrologue)
{
    using SH = TileShape<BN>;
    constexpr int NB = BN / 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % SH::WM) * (TBM / SH::WM), wn0 = (wave / SH::WM) * (BN / SH::WN);
    const int nch = Ke > Kb ? (Ke - Kb + TBK - 1) / TBK : 0;
    const double *pa[4], *pb[NB];  // stage ADDR
    bool oka[4], okb[NB], ala = false;
    double va[4], vb[NB];          // stage VAL
    bool vka[4], vkb[NB], vla = false;
    // kPairK (both operands read along k, kBJ false, every chunk along k):
    // rows k, k+1 of one column per load, the caller guaranteeing that a
    // pair never straddles the end of the contraction
    auto stage_addr = [&](int ch) {
        const int k0 = Kb + ch * TBK;
        const bool past = ch >= nch;
        ala = alongA(k0);
        if constexpr (kPairK) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = tid + q * kThreads;
                pa[q] = addrA(k0, 2 * (e & 7), e >> 3, oka[q]);
                oka[q] = oka[q] && !past;
            }
#pragma unroll
            for (int q = 0; q < NB / 2; ++q) {
                const int e = tid + q * kThreads;
                pb[q] = addrB(k0, 2 * (e & 7), e >> 3, okb[q]);
                okb[q] = okb[q] && !past;
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * kThreads;
            const int kk = ala ? (e & 15) : (e >> 6), ii = ala ? (e >> 4) : (e & 63);
            pa[q] = addrA(k0, kk, ii, oka[q]);
            oka[q] = oka[q] && !past;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + q * kThreads;
            const int kk = kBJ ? e / BN : (e & 15), j = kBJ ? e % BN : (e >> 4);
            pb[q] = addrB(k0, kk, j, okb[q]);
            okb[q] = okb[q] && !past;
        }
    };
    auto stage_val = [&]() {
        vla = ala;
        if constexpr (kPairK) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const d2u x = *reinterpret_cast<const d2u*>(pa[q]);
                va[2 * q] = x.x;
                va[2 * q + 1] = x.y;
                vka[q] = oka[q];
            }
#pragma unroll
            for (int q = 0; q < NB / 2; ++q) {
                const d2u x = *reinterpret_cast<const d2u*>(pb[q]);
                vb[2 * q] = x.x;
                vb[2 * q + 1] = x.y;
                vkb[q] = okb[q];
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            va[q] = *pa[q];
            vka[q] = oka[q];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            vb[q] = *pb[q];
            vkb[q] = okb[q];
        }
    };
    auto stage_store = [&](int buf) {
        if constexpr (kPairK) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = tid + q * kThreads;
                L.A[buf][2 * (e & 7)][e >> 3] = vka[q] ? va[2 * q] : 0.0;
                L.A[buf][2 * (e & 7) + 1][e >> 3] = vka[q] ? va[2 * q + 1] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < NB / 2; ++q) {
                const int e = tid + q * kThreads;
                L.B[buf][2 * (e & 7)][e >> 3] = vkb[q] ? vb[2 * q] : 0.0;
                L.B[buf][2 * (e & 7) + 1][e >> 3] = vkb[q] ? vb[2 * q + 1] : 0.0;
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * kThreads;
            const int kk = vla ? (e & 15) : (e >> 6), ii = vla ? (e >> 4) : (e & 63);
            L.A[buf][kk][ii] = vka[q] ? va[q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + q * kThreads;
            const int kk = kBJ ? e / BN : (e & 15), j = kBJ ? e % BN : (e >> 4);
            L.B[buf][kk][j] = vkb[q] ? vb[q] : 0.0;
        }
    };
    stage_addr(0);
    stage_val();
    stage_store(0);
    stage_addr(1);
    stage_val();
    stage_addr(2);
    afterPrologue();  // loads of the caller's own that may run under the main loop
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
#pragma unroll
        for (int ks = 0; ks < TBK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double a[SH::MT], b[SH::NT];
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt) a[mt] = L.A[buf][kr][wm0 + mt * 16 + (lane & 15)];
#pragma unroll
            for (int nt = 0; nt < SH::NT; ++nt) b[nt] = L.B[buf][kr][wn0 + nt * 16 + (lane & 15)];
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < SH::NT; ++nt)
                    acc[mt][nt] = kT ? mfma(b[nt], a[mt], acc[mt][nt]) : mfma(a[mt], b[nt], acc[mt][nt]);
        }
        stage_store(buf ^ 1);
        stage_val();
        stage_addr(ch + 3);
        __syncthreads();
    }
    mfma_drain();
}

// ---------------------------------------------------------------------------
// The same 64 x BN product for a contraction of at most NCH chunks of 16
// (NCH <= 8: at most 128), for levels with few tiles, where a tile's time is
// its latency: every chunk's loads are issued before the first product, so
// the global-memory latency is paid once instead of once per chunk.  The
// loads of all NCH chunks are unconditional (past the contraction the
// address callbacks return an in-bounds stand-in and a false mask), which
// keeps them in one straight run: with a branch per chunk the wait before
// the first product would have to cover every path, i.e. all loads.  A read
// along i, B as in tile_mma2 (kBJ), operands swapped when kT; masks kept as
// bits.  BN <= 64 (at most 8 values per thread a chunk).
// ---------------------------------------------------------------------------
template <int BN, int NCH, bool kBJ, bool kT, class FA, class FB, class FH>
__device__ __forceinline__ void tile_mma_deep(GemmLds& L, int Kb, int Ke, d4 (&acc)[2][4], FA addrA, FB addrB,
                                              FH afterPrologue)
{
    static_assert(BN <= 64 && NCH * TBK <= kDeepK, "at most 8 chunks of 8 values in registers");
    using SH = TileShape<BN>;
    constexpr int NB = BN / 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % SH::WM) * (TBM / SH::WM), wn0 = (wave / SH::WM) * (BN / SH::WN);
    const int nch = Ke > Kb ? (Ke - Kb + TBK - 1) / TBK : 0;
    double va[NCH][4], vb[NCH][NB];
    uint32_t oka = 0, okb = 0;  // bit 4 ch + q (A), NB ch + q (B)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int k0 = Kb + ch * TBK;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * kThreads;
            bool ok;
            va[ch][q] = *addrA(k0, e >> 6, e & 63, ok);
            oka |= (uint32_t)ok << (4 * ch + q);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + q * kThreads;
            const int kk = kBJ ? e / BN : (e & 15), j = kBJ ? e % BN : (e >> 4);
            bool ok;
            vb[ch][q] = *addrB(k0, kk, j, ok);
            okb |= (uint32_t)ok << (NB * ch + q);
        }
    }
    afterPrologue();
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        if (ch >= nch) break;
        const int buf = ch & 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * kThreads;
            L.A[buf][e >> 6][e & 63] = (oka >> (4 * ch + q)) & 1 ? va[ch][q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + q * kThreads;
            const int kk = kBJ ? e / BN : (e & 15), j = kBJ ? e % BN : (e >> 4);
            L.B[buf][kk][j] = (okb >> (NB * ch + q)) & 1 ? vb[ch][q] : 0.0;
        }
        // chunk ch - 1 was read from the other buffer before every wave
        // passed the previous barrier; this buffer was last read two chunks ago
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TBK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double a[SH::MT], b[SH::NT];
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt) a[mt] = L.A[buf][kr][wm0 + mt * 16 + (lane & 15)];
#pragma unroll
            for (int nt = 0; nt < SH::NT; ++nt) b[nt] = L.B[buf][kr][wn0 + nt * 16 + (lane & 15)];
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < SH::NT; ++nt)
                    acc[mt][nt] = kT ? mfma(b[nt], a[mt], acc[mt][nt]) : mfma(a[mt], b[nt], acc[mt][nt]);
        }
    }
    mfma_drain();
}

#define SELINV_BN_DISPATCH(bn, CALL) \
    switch (bn) {                    \
        case 16: CALL(16); break;    \
        case 32: CALL(32); break;    \
        case 64: CALL(64); break;    \
        default: CALL(128); break;   \
    }

// ---------------------------------------------------------------------------
// Selected inversion, step 3: X = Ainv(C,B) = -Ainv(C,C) L_hat(C,B) for rows
// [i0, i0+64) and columns [j0, j0+BN) of X.  Ainv(C,C) is gathered from the
// ancestors' panels: entries with i >= k directly, the others by symmetry.
//
// The gather G(i,k) = Ap[cbase[p] + rel[rbase[p] + q]] (p, q = k, i when
// i >= k, else i, k) is a chain of three dependent loads, so the main loop
// is a software pipeline over 16-deep chunks of the contraction: while the
// MFMAs consume chunk n from one LDS buffer, the values of chunk n+1 are
// stored to the other, the values of chunk n+2 are loaded from the offsets
// found one iteration earlier, the rel entries of chunk n+3 and the
// (cbase, rbase) pairs of chunk n+4 are loaded: every load has a whole
// iteration of MFMAs to arrive, and there is one barrier per chunk.
// ---------------------------------------------------------------------------
// The pipelined gather-GEMM loop, shared by the forward gather-GEMM and the
// reverse sweep: acc += A B over the contraction [Kb, Ke) for tile rows
// [r0, r0+64) and columns [n0, n0+BN), accumulated transposed, with
//   A(i, k) = S[cbase[p] + rel[rbase[p] + q]],  p = min(i, k), q = max(i, k)
// (an arena gathered through the block index maps; kTri = 1 keeps k <= i
// only, 2 keeps k >= i only, 0 all) and B(k, j) = Bm[k + (n0 + j) ldb].
template <int BN, bool kPair, int kTri>
__device__ __forceinline__ void gather_mma(GemmLds& L, const BlockDesc d, const int r0, const int n0, const int Kb,
                                           const int Ke, const double* __restrict__ S, const double* __restrict__ Bm,
                                           const int64_t ldb, const int64_t* __restrict__ cr2,
                                           const int32_t* __restrict__ rel, d4 (&acc)[2][4])
{
    using SH = TileShape<BN>;
    constexpr int NB = BN / 16;  // B elements per thread per chunk
    const int s = d.s, c = d.c;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % SH::WM) * (TBM / SH::WM), wn0 = (wave / SH::WM) * (BN / SH::WN);
    const int nch = Ke > Kb ? (Ke - Kb + TBK - 1) / TBK : 0;
    // chunks entirely above the diagonal band are read along k (contiguous)
    auto along_of = [&](int ch) { return Kb + ch * TBK >= r0 + TBM; };
    // element q of this thread in chunk ch: (kk, ii) = along ? (e & 15, e >> 4) : (e >> 6, e & 63)
    auto elem = [&](int ch, int q, int& i, int& k) {
        const int e = tid + q * kThreads;
        const bool al = along_of(ch);
        i = r0 + (al ? e >> 4 : e & 63);
        k = Kb + ch * TBK + (al ? e & 15 : e >> 6);
        if (ch >= nch) k = c;  // past the end: padding
    };
    // Loads are unconditional and every stage only issues loads into raw
    // registers; whatever consumes a loaded value (the offset sums, the
    // padding masks) runs in the next stage, an iteration later, so no wait
    // falls right behind its own load.  A padding element reads an in-bounds
    // stand-in (position 0 of the block's maps, its own L_hat) and is zeroed
    // by its mask.
    int64_t m_cb[4], m_rb[4];  // stage M: cbase[p], rbase[p] as loaded
    int m_q[4];                // stage M: q (the second index), -1 for padding
    int64_t r_cb[4];           // stage R: cbase[p]
    int32_t r_rel[4];          // stage R: rel[rbase[p] + q] as loaded
    bool r_ok[4];
    double v_a[4], v_b[NB];    // stage V: values as loaded
    bool v_ok[4];
    bool av = false;           // stage V chunk is read along k
    auto stage_m = [&](int ch) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int i, k;
            elem(ch, q, i, k);
            const bool ok = i < c && k < c && (kTri == 0 || (kTri == 1 ? k <= i : k >= i));
            const int64_t p = d.coff + (ok ? (i >= k ? k : i) : 0);
            const i64x2 cr = *reinterpret_cast<const i64x2*>(cr2 + 2 * p);  // (cbase[p], rbase[p])
            m_cb[q] = cr.x;
            m_rb[q] = cr.y;
            m_q[q] = ok ? (i >= k ? i : k) : -1;
        }
    };
    auto stage_r = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            r_ok[q] = m_q[q] >= 0;
            r_rel[q] = rel[m_rb[q] + (r_ok[q] ? m_q[q] : 0)];
            r_cb[q] = m_cb[q];
        }
    };
    auto stage_v = [&](int ch) {
        av = along_of(ch);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v_a[q] = S[r_cb[q] + r_rel[q]];
            v_ok[q] = r_ok[q];
        }
        // L_hat needs no mask: where k >= c the gathered A is zero, and
        // columns past s are never written; a stand-in keeps the read in bounds
        const int k0 = Kb + ch * TBK;
        if constexpr (kPair) {
            // rows k, k+1 of one column per load (c even: a pair never
            // crosses the column's end)
#pragma unroll
            for (int q = 0; q < NB / 2; ++q) {
                const int e = tid + q * kThreads;
                const int k = k0 + 2 * (e & 7), jj = n0 + (e >> 3);
                const bool ok = k < c && jj < s;
                const d2u pr = *reinterpret_cast<const d2u*>(Bm + (ok ? k + (int64_t)jj * ldb : 0));
                v_b[2 * q] = pr.x;
                v_b[2 * q + 1] = pr.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int e = tid + q * kThreads;
                const int k = k0 + (e & 15), jj = n0 + (e >> 4);
                v_b[q] = Bm[(k < c && jj < s) ? k + (int64_t)jj * ldb : 0];
            }
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * kThreads;
            const double x = v_ok[q] ? v_a[q] : 0.0;
            const int row = av ? (e & 15) : (e >> 6), col = av ? (e >> 4) : (e & 63);
            L.A[buf][row][col] = x;
        }
        if constexpr (kPair) {
#pragma unroll
            for (int q = 0; q < NB / 2; ++q) {
                const int e = tid + q * kThreads;
                L.B[buf][2 * (e & 7)][e >> 3] = v_b[2 * q];
                L.B[buf][2 * (e & 7) + 1][e >> 3] = v_b[2 * q + 1];
            }
        } else {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int e = tid + q * kThreads;
                L.B[buf][e & 15][e >> 4] = v_b[q];
            }
        }
    };
    // prologue: chunk 0 in LDS, chunk 1 values, chunk 2 offsets, chunk 3
    // (cbase, rbase).  Chunks past the end are all padding: the stages run
    // for them anyway, so the loop body has no branches.
    stage_m(0);
    stage_r();
    stage_v(0);
    stage_store(0);
    stage_m(1);
    stage_r();
    stage_v(1);
    stage_m(2);
    stage_r();
    stage_m(3);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
#pragma unroll
        for (int ks = 0; ks < TBK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double a[SH::MT], b[SH::NT];
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt) a[mt] = L.A[buf][kr][wm0 + mt * 16 + (lane & 15)];
#pragma unroll
            for (int nt = 0; nt < SH::NT; ++nt) b[nt] = L.B[buf][kr][wn0 + nt * 16 + (lane & 15)];
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < SH::NT; ++nt) acc[mt][nt] = mfma(b[nt], a[mt], acc[mt][nt]);
        }
        stage_store(buf ^ 1);
        stage_v(ch + 2);
        stage_r();
        stage_m(ch + 4);
        {
            // one MFMA, then about five VALU and a share of the DS and
            // global-memory operations (swept 3, 5, 8: 5 fastest, 22.85 ->
            // 22.3 ms of gather-GEMM at 64^3)
            constexpr int nm = (TBK / 4) * SH::MT * SH::NT, nr = (TBK / 4) * (SH::MT + SH::NT) / 2;
            constexpr int nw = 4 + NB, nv = 12 + (kPair ? NB / 2 : NB);
            sgb_interleave<nm, (SH::MT + SH::NT) / 2, nr - (SH::MT + SH::NT) / 2, nw, nv, 5>();
        }
        __syncthreads();
    }
    mfma_drain();
}

template <int BN, bool kPair = false>
__device__ __forceinline__ void gemm_task(GemmLds& L, const Task t, const BlockDesc d, double* __restrict__ Ap,
                          const double* __restrict__ Hp, const int64_t* __restrict__ cr2, const int32_t* __restrict__ rel)
{
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int r0 = t.i0, n0 = t.j0;
    d4 acc[2][4] = {};
    gather_mma<BN, kPair, 0>(L, d, r0, n0, t.kb, t.ke, Ap, Hp + d.hoff, c, cr2, rel, acc);
    // transposed accumulation: stores and atomics run down the columns of X
    tile_epilogue_t<BN>(acc, [&](int i, int j, double v) {
        const int ii = r0 + i, jj = n0 + j;
        if (ii < c && jj < s) {
            double* x = Ap + d.poff + s + ii + (int64_t)jj * ld;
            if (t.flags & 1) unsafeAtomicAdd(x, -v); else *x = -v;
        }
    });
}

__global__ __launch_bounds__(kThreads) void k_gemm(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                   double* __restrict__ Ap, const double* __restrict__ Hp,
                                                   const int64_t* __restrict__ cr2,
                                                   const int32_t* __restrict__ rel)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    // even |C|: L_hat read two rows per load
#define SELINV_CALL(BN)                                                \
    if (BN >= 32 && (d.c & 1) == 0) gemm_task<BN, BN >= 32>(L, t, d, Ap, Hp, cr2, rel); \
    else gemm_task<BN, false>(L, t, d, Ap, Hp, cr2, rel)
    SELINV_BN_DISPATCH(t.bn, SELINV_CALL)
#undef SELINV_CALL
}

// ---------------------------------------------------------------------------
// Factor panel (Algorithm 1 step 2, fused into the factorization):
// L_hat(C,B) = F(C,B) T for rows [i0, i0+64), columns [j0, j0+BN).
// ---------------------------------------------------------------------------
template <int BN, bool kDeep = false>
__device__ __forceinline__ void panel_task(GemmLds& L, const Task t, const BlockDesc d, const double* __restrict__ Lp,
                           double* __restrict__ Hp, const double* __restrict__ Tp)
{
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int r0 = t.i0, n0 = t.j0;
    d4 acc[2][4] = {};
    const double* F = Lp + d.poff + s;
    const double* T = Tp + d.woff;
    auto addrA = [&](int k0, int kk, int ii, bool& ok) -> const double* {
        const int i = r0 + ii, k = k0 + kk;
        ok = i < c && k < s;
        return ok ? F + i + (int64_t)k * ld : F;
    };
    auto addrB = [&](int k0, int kk, int j, bool& ok) -> const double* {
        const int k = k0 + kk, jj = n0 + j;
        ok = k < s && jj < s;
        return ok ? T + k + (int64_t)jj * s : T;
    };
    if constexpr (kDeep) {
        // chunks of 16 the contraction s needs: 1, 2, 4 or 8 (s <= 128)
        if (s <= 16) tile_mma_deep<BN, 1, false, true>(L, 0, s, acc, addrA, addrB, [] {});
        else if (s <= 32) tile_mma_deep<BN, 2, false, true>(L, 0, s, acc, addrA, addrB, [] {});
        else if (s <= 64) tile_mma_deep<BN, 4, false, true>(L, 0, s, acc, addrA, addrB, [] {});
        else if (s <= kDeepK) tile_mma_deep<BN, 8, false, true>(L, 0, s, acc, addrA, addrB, [] {});
        else tile_mma2<BN, false, true>(L, 0, s, acc, addrA, addrB, [](int) { return false; }, [] {});
    } else {
        tile_mma2<BN, false, true>(L, 0, s, acc, addrA, addrB, [](int) { return false; }, [] {});
    }
    tile_epilogue_t<BN>(acc, [&](int i, int j, double v) {
        const int ii = r0 + i, jj = n0 + j;
        if (ii < c && jj < s) Hp[d.hoff + ii + (int64_t)jj * c] = v;
    });
}

__global__ __launch_bounds__(kThreads) void k_panel(const Task* __restrict__ tasks,
                                                    const BlockDesc* __restrict__ blk, const double* __restrict__ Lp,
                                                    double* __restrict__ Hp, const double* __restrict__ Tp)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
#define SELINV_CALL(BN) panel_task<BN>(L, t, d, Lp, Hp, Tp)
    SELINV_BN_DISPATCH(t.bn, SELINV_CALL)
#undef SELINV_CALL
}

// levels with few panel tiles (width <= 64 each): the contraction (s <= 128)
// loaded up front
__global__ __launch_bounds__(kThreads) void k_panel_deep(const Task* __restrict__ tasks,
                                                         const BlockDesc* __restrict__ blk,
                                                         const double* __restrict__ Lp, double* __restrict__ Hp,
                                                         const double* __restrict__ Tp)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    switch (t.bn) {
        case 16: panel_task<16, true>(L, t, d, Lp, Hp, Tp); break;
        case 32: panel_task<32, true>(L, t, d, Lp, Hp, Tp); break;
        default: panel_task<64, true>(L, t, d, Lp, Hp, Tp); break;
    }
}

// ---------------------------------------------------------------------------
// Factor, Schur update: F(C,C) -= L(C,B) D_B L(C,B)^T = L_hat(C,B) F(C,B)^T,
// lower half, tile rows [i0, i0+64) x columns [k0, k0+64), added into the
// ancestor panels through the block index maps.  FP64 atomics where sibling
// blocks of the level may update the same ancestor entry; plain
// read-modify-write for blocks the host found exclusive (flags bit 2).
//
// The tile is formed transposed, as F(k0.., :) L_hat(i0.., :)^T, so that the
// sixteen lanes of an MFMA output row hold sixteen consecutive rows ii of one
// target column kk: rows of one ancestor column are contiguous in its panel,
// so each group of sixteen lanes updates one run of memory instead of
// sixteen columns.  The scatter targets do not depend on the product: their
// (cbase, rbase) pairs are loaded before the main loop and the rel entries
// right after its prologue, so the epilogue issues only the updates.
// ---------------------------------------------------------------------------
template <bool kDeep = false>
__device__ __forceinline__ void schur_task(GemmLds& L, const Task t, const BlockDesc d, double* __restrict__ Lp,
                           const double* __restrict__ Hp, const int64_t* __restrict__ cbase,
                           const int64_t* __restrict__ rbase, const int32_t* __restrict__ rel)
{
    using SH = TileShape<64>;
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int i0 = t.i0, k0c = t.j0;
    const double* H = Hp + d.hoff;
    const double* F = Lp + d.poff + s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave % SH::WM) * (TBM / SH::WM), wn0 = (wave / SH::WM) * (64 / SH::WN);
    // this thread's outputs (mt, nt, v): target column kk = k0 + wm0 + 16 mt +
    // lane / 16 + 4 v, row ii = i0 + wn0 + 16 nt + lane % 16
    auto col_of = [&](int mt, int v) { return k0c + wm0 + mt * 16 + (lane >> 4) + 4 * v; };
    auto row_of = [&](int nt) { return i0 + wn0 + nt * 16 + (lane & 15); };
    int64_t cb[SH::MT][4], rb[SH::MT][4];
#pragma unroll
    for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = col_of(mt, v);
            const int64_t pk = d.coff + (kk < c ? kk : 0);
            cb[mt][v] = cbase[pk];
            rb[mt][v] = rbase[pk];
        }
    int32_t ro[SH::MT][SH::NT][4];
    auto live = [&](int mt, int nt, int v) {
        const int ii = row_of(nt), kk = col_of(mt, v);
        return ii < c && kk < c && ii >= kk;
    };
    auto prefetch = [&]() {
#pragma unroll
        for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) ro[mt][nt][v] = rel[rb[mt][v] + (live(mt, nt, v) ? row_of(nt) : 0)];
    };
    d4 acc[2][4] = {};
    // A(kk, t) = F(k0 + kk, t): contiguous along the tile rows
    auto addrA = [&](int t0, int tt, int kk, bool& ok) -> const double* {
        const int k = k0c + kk, col = t0 + tt;
        ok = k < c && col < s;
        return ok ? F + k + (int64_t)col * ld : F;
    };
    // B(t, ii) = L_hat(i0 + ii, t): contiguous in ii
    auto addrB = [&](int t0, int tt, int ii, bool& ok) -> const double* {
        const int i = i0 + ii, k = t0 + tt;
        ok = i < c && k < s;
        return ok ? H + i + (int64_t)k * c : H;
    };
    if constexpr (kDeep) {
        if (s <= 16) tile_mma_deep<64, 1, true, false>(L, 0, s, acc, addrA, addrB, prefetch);
        else if (s <= 32) tile_mma_deep<64, 2, true, false>(L, 0, s, acc, addrA, addrB, prefetch);
        else if (s <= 64) tile_mma_deep<64, 4, true, false>(L, 0, s, acc, addrA, addrB, prefetch);
        else if (s <= kDeepK) tile_mma_deep<64, 8, true, false>(L, 0, s, acc, addrA, addrB, prefetch);
        else tile_mma2<64, true, false>(L, 0, s, acc, addrA, addrB, [](int) { return false; }, prefetch);
    } else {
        tile_mma2<64, true, false>(L, 0, s, acc, addrA, addrB, [](int) { return false; }, prefetch);
    }
    auto target = [&](int mt, int nt, int v) { return Lp + cb[mt][v] + ro[mt][nt][v]; };
    // a tile strictly below the diagonal and inside C has every entry live:
    // its updates are issued without per-entry branches, which would put a
    // wait on all outstanding memory operations in front of every store
    const bool full = i0 > k0c && i0 + TBM <= c;
    if (t.flags & 4) {
        // no other block of the level updates these entries: plain
        // read-modify-write, all reads issued before the first write (the
        // targets of one thread are distinct entries)
        double old[SH::MT][SH::NT][4];
        if (full) {
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) old[mt][nt][v] = *target(mt, nt, v);
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) *target(mt, nt, v) = old[mt][nt][v] - acc[mt][nt][v];
        } else {
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) old[mt][nt][v] = live(mt, nt, v) ? *target(mt, nt, v) : 0.0;
#pragma unroll
            for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (live(mt, nt, v)) *target(mt, nt, v) = old[mt][nt][v] - acc[mt][nt][v];
        }
    } else if (full) {
#pragma unroll
        for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) unsafeAtomicAdd(target(mt, nt, v), -acc[mt][nt][v]);
    } else {
#pragma unroll
        for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (live(mt, nt, v)) unsafeAtomicAdd(target(mt, nt, v), -acc[mt][nt][v]);
    }
}

__global__ __launch_bounds__(kThreads) void k_schur(const Task* __restrict__ tasks,
                                                    const BlockDesc* __restrict__ blk, double* __restrict__ Lp,
                                                    const double* __restrict__ Hp,
                                                    const int64_t* __restrict__ cbase,
                                                    const int64_t* __restrict__ rbase,
                                                    const int32_t* __restrict__ rel)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    schur_task(L, t, blk[t.b], Lp, Hp, cbase, rbase, rel);
}

// colour groups with few tiles: the contraction (s <= 128) loaded up front
__global__ __launch_bounds__(kThreads) void k_schur_deep(const Task* __restrict__ tasks,
                                                         const BlockDesc* __restrict__ blk, double* __restrict__ Lp,
                                                         const double* __restrict__ Hp,
                                                         const int64_t* __restrict__ cbase,
                                                         const int64_t* __restrict__ rbase,
                                                         const int32_t* __restrict__ rel)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    schur_task<true>(L, t, blk[t.b], Lp, Hp, cbase, rbase, rel);
}

// ---------------------------------------------------------------------------
// Selected inversion, step 4 + symmetrisation, one pair of 32 x 32 tiles
// (I, J), I >= J, of the diagonal block per work-group:
//   Y(I,J) = T(I,J) - L_hat(:,I)^T X(:,J),  Y(J,I) = T(J,I) - L_hat(:,J)^T X(:,I)
//   Ainv(I,J) = Ainv(J,I)^T = (Y(I,J) + Y(J,I)^T) / 2.
// ---------------------------------------------------------------------------
constexpr int SDT = 32;

struct SdiagLds {
    double LI[16][SDT + 1], LJ[16][SDT + 1], XI[16][SDT + 1], XJ[16][SDT + 1];
    double Sx[SDT][SDT + 1];
};

__device__ __forceinline__ void sdiag_task(SdiagLds& S, const Task t, const BlockDesc d, double* __restrict__ Ap,
                           const double* __restrict__ Hp, const double* __restrict__ Tp)
{
    auto& LI = S.LI;
    auto& LJ = S.LJ;
    auto& XI = S.XI;
    auto& XJ = S.XJ;
    auto& Sx = S.Sx;
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int I0 = t.i0, J0 = t.j0;
    double* A = Ap + d.poff;
    const double* H = Hp + d.hoff;
    const double* T = Tp + d.woff;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fm = (wave & 1) * 16, fn = (wave >> 1) * 16;
    d4 accIJ = {0, 0, 0, 0}, accJI = {0, 0, 0, 0};
    // Branch-free body: a diagonal tile (I == J) simply recomputes its own
    // product as the partner.  Control flow between an FP64 MFMA and a read
    // of its accumulator let the compiler place the read too early.
    const int rend = min(c, t.ke);
    for (int r0 = t.kb; r0 < rend; r0 += 16) {
#pragma unroll
        for (int q = 0; q < (16 * SDT) / kThreads; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int kk = e & 15, col = e >> 4;
            const int r = r0 + kk;
            const bool okr = r < rend;
            const int ci = I0 + col, cj = J0 + col;
            const double li = (okr && ci < s) ? H[r + (int64_t)ci * c] : 0.0;
            const double lj = (okr && cj < s) ? H[r + (int64_t)cj * c] : 0.0;
            const double xi = (okr && ci < s) ? A[s + r + ci * ld] : 0.0;
            const double xj = (okr && cj < s) ? A[s + r + cj * ld] : 0.0;
            LI[kk][col] = li;
            LJ[kk][col] = lj;
            XI[kk][col] = xi;
            XJ[kk][col] = xj;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            accIJ = mfma(LI[kr][fm + (lane & 15)], XJ[kr][fn + (lane & 15)], accIJ);
            accJI = mfma(LJ[kr][fm + (lane & 15)], XI[kr][fn + (lane & 15)], accJI);
        }
        __syncthreads();
    }
    mfma_drain();
    // Only the lower triangle of Ainv(B,B) is kept (it is all that the
    // gathers and the export read).  A whole contraction writes
    // (Y(I,J) + Y(J,I)^T)/2 there; a split piece adds its share
    // -(P(I,J) + P(J,I)^T)/2 to the T written beforehand (the average is
    // linear, so the pieces may arrive in any order).
    const bool split = t.flags & 1;
    // Sx[b][a] = element (a, b) of the partner tile
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = fm + (lane >> 4) + 4 * v, j = fn + (lane & 15);
        const double tji = (!split && J0 + i < s && I0 + j < s) ? T[(J0 + i) + (I0 + j) * s] : 0.0;
        Sx[j][i] = tji - accJI[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = fm + (lane >> 4) + 4 * v, j = fn + (lane & 15);
        const int gi = I0 + i, gj = J0 + j;
        if (gi < s && gj < s && gi >= gj) {
            if (split) {
                unsafeAtomicAdd(A + gi + gj * ld, 0.5 * (Sx[i][j] - accIJ[v]));
            } else {
                A[gi + gj * ld] = 0.5 * ((T[gi + gj * s] - accIJ[v]) + Sx[i][j]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Selected inversion, step 4 + symmetrisation, per-level path, on 64 x 64
// tiles of the diagonal block, with P = L_hat^T X (so Y = T - P) and
// Ainv(i,j) = T(i,j) - (P(i,j) + P(j,i)) / 2 for i >= j:
//  * diagonal tile I: P(I,I) on the pipelined MFMA tile; the transpose
//    reaches the thread holding P(i,j) through LDS; stored as T - (P + P^T)/2,
//    or with a split contraction added as -(P + P^T)/2 (atomics) to the T
//    written beforehand;
//  * tile (I,J), I > J: two tasks, one per half, each adding -1/2 of its
//    product to Ainv(I,J) with atomics (T written beforehand):
//    L_hat(:,I)^T X(:,J) (flags bit 3 clear) and X(:,I)^T L_hat(:,J) =
//    P(J,I)^T (bit 3 set).  One product per task keeps the longest task of a
//    level short.
// Products accumulate transposed (lane l holds tile row l % 16), so stores
// and atomics run down the columns of the panel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sdiag64_task(GemmLds& L, const Task t, const BlockDesc d, double* __restrict__ Ap,
                                             const double* __restrict__ Hp, const double* __restrict__ Tp)
{
    using SH = TileShape<64>;
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int I0 = t.i0, J0 = t.j0;
    const int kb = t.kb, ke = min(t.ke, c);
    const double* H = Hp + d.hoff;       // L_hat(r, j) at H[r + j c]
    const double* X = Ap + d.poff + s;   // X(r, j) at X[r + j ld]
    const bool diag = I0 == J0, second = t.flags & 8;
    // A(i, r) = U(r, I0 + i), B(r, j) = V(r, J0 + j): both contiguous in r
    const double* U = second ? X : H;
    const double* V = second ? H : X;
    const int64_t ldu = second ? ld : c, ldv = second ? c : ld;
    d4 acc[2][4] = {};
    auto addrA = [&](int k0, int kk, int ii, bool& ok) -> const double* {
        const int r = k0 + kk, col = I0 + ii;
        ok = r < ke && col < s;
        return ok ? U + r + (int64_t)col * ldu : U;
    };
    auto addrB = [&](int k0, int kk, int j, bool& ok) -> const double* {
        const int r = k0 + kk, col = J0 + j;
        ok = r < ke && col < s;
        return ok ? V + r + (int64_t)col * ldv : V;
    };
    // pairs of rows never straddle the end of the contraction when c and kb are even
    if ((c & 1) == 0 && (kb & 1) == 0)
        tile_mma2<64, false, true, true>(L, kb, ke, acc, addrA, addrB, [](int) { return true; }, [] {});
    else
        tile_mma2<64, false, true>(L, kb, ke, acc, addrA, addrB, [](int) { return true; }, [] {});
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm0 = (wave % SH::WM) * (TBM / SH::WM), wn0 = (wave / SH::WM) * (64 / SH::WN);
    const double* T = Tp + d.woff;
    double* A = Ap + d.poff;
    if (!diag) {
#pragma unroll
        for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int gi = I0 + wm0 + mt * 16 + (lane & 15), gj = J0 + wn0 + nt * 16 + (lane >> 4) + 4 * v;
                    if (gi < s && gj < s) {
                        double* a = A + gi + (int64_t)gj * ld;
                        if (t.flags & 16) *a -= 0.5 * acc[mt][nt][v];  // the only writer of its launch
                        else unsafeAtomicAdd(a, -0.5 * acc[mt][nt][v]);
                    }
                }
        return;
    }
    // diagonal tile: the loop ended on a barrier, the LDS tile is free
    double(*S)[TBM + 1] = reinterpret_cast<double(*)[TBM + 1]>(&L);
    static_assert(sizeof(double) * TBM * (TBM + 1) <= sizeof(GemmLds), "exchange tile fits the LDS tile");
    static_assert(sizeof(TileLds) <= sizeof(GemmLds), "the one-stage tile fits the LDS tile");
#pragma unroll
    for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = wm0 + mt * 16 + (lane & 15), j = wn0 + nt * 16 + (lane >> 4) + 4 * v;
                S[j][i] = acc[mt][nt][v];  // S[a][b] = P(b, a)
            }
    __syncthreads();
    const bool split = t.flags & 1;
#pragma unroll
    for (int mt = 0; mt < SH::MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < SH::NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = wm0 + mt * 16 + (lane & 15), j = wn0 + nt * 16 + (lane >> 4) + 4 * v;
                const int gi = I0 + i, gj = J0 + j;
                if (gi < s && gj < s && gi >= gj) {
                    const double p = 0.5 * (acc[mt][nt][v] + S[i][j]);
                    if (split) unsafeAtomicAdd(A + gi + (int64_t)gj * ld, -p);
                    else A[gi + (int64_t)gj * ld] = T[gi + (int64_t)gj * s] - p;
                }
            }
}

__global__ __launch_bounds__(kThreads) void k_sdiag64(const Task* __restrict__ tasks,
                                                      const BlockDesc* __restrict__ blk, double* __restrict__ Ap,
                                                      const double* __restrict__ Hp, const double* __restrict__ Tp)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    sdiag64_task(L, t, blk[t.b], Ap, Hp, Tp);
}

// ---------------------------------------------------------------------------
// Factor, diagonal block wider than the register sweeps hold (s > 128, only
// with exec_cap above 128), on global memory: right-looking LDL^T without
// pivoting in place of F_BB, then W = L_BB^{-1} column by column (forward
// substitution, one thread a column) and T = W^T D^{-1} W.  A pivot that is
// zero, not finite, or (require_spd) not positive is latched as the smallest
// failing column.
// ---------------------------------------------------------------------------
__device__ void ldlt_global(const BlockDesc d, double* __restrict__ Lp, double* __restrict__ Wp,
                            double* __restrict__ Tp, unsigned long long* __restrict__ status, int require_spd)
{
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
    for (int e = tid; e < s * s; e += kThreads) {
        const int i = e % s, j = e / s;
        const int m = i > j ? i : j;
        double v = 0.0;
        for (int k = m; k < s; ++k) v += W[k + i * s] * W[k + j * s] / F[k + k * ld];
        T[e] = v;
    }
}

// Diagonal block, s <= 16 NB (NB = 2, 4, 8), by symmetric Gauss-Jordan
// sweeps held in registers.  Sweeping pivot j (M(j,j) = d_j, c = M(:,j)):
//   M(i,k) -= c_i c_k / d_j  (i, k != j),  M(i,j) = M(j,i) = c_i / d_j,
//   M(j,j) = -1 / d_j.
// After all pivots M = -F_BB^{-1} = -T.  Before its own sweep, column j
// below the diagonal holds the Schur-complement column, so the multipliers
// c_i / d_j (i > j) are L_BB(i,j) and d_j is D's entry: both are written
// out as they appear.
//
// M stays symmetric, so only its lower 16 x 16 sub-blocks are held: thread
// (tx, ty) = (tid % 16, tid / 16) owns M(tx + 16a, ty + 16b) for a >= b
// (a diagonal sub-block whole).  Column j is then spread over two groups of
// threads: ty == j % 16 holds rows >= 16 (j / 16) in sub-blocks (a, j / 16),
// tx == j % 16 holds the rows above as row j of sub-blocks (j / 16, b).
// The sweep is latency-bound (one pivot after the other), so each pivot
// first forms the next pivot's column and publishes it in LDS (two
// alternating slots, one barrier per pivot), then issues the LDS reads of
// that column, and only then updates the rest of its registers while the
// reads are in flight.
template <int NB>
__device__ __forceinline__ void ldlt_sweep(const BlockDesc d, double* __restrict__ Lp, double* __restrict__ Tp,
                           unsigned long long* __restrict__ status, int require_spd, double (*colbuf)[kLdsDiagMax])
{
    constexpr int NS = NB * (NB + 1) / 2;
    const int s = d.s;
    const int64_t ld = (int64_t)d.s + d.c;
    double* F = Lp + d.poff;
    double* T = Tp + d.woff;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    auto slot = [](int a, int b) { return a * (a + 1) / 2 + b; };
    auto read_col = [&](const double* col, double (&v)[NB], int r0) {
#pragma unroll
        for (int a = 0; a < NB; ++a) v[a] = col[r0 + 16 * a];
    };
    double M[NS];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tx + 16 * a, k = ty + 16 * b;
            double v = 0.0;
            if (i < s && k < s) v = i >= k ? F[i + k * ld] : F[k + i * ld];
            M[slot(a, b)] = v;
        }
    // column 0 to slot 0; its reads
    if (ty == 0) {
#pragma unroll
        for (int a = 0; a < NB; ++a) colbuf[0][tx + 16 * a] = M[slot(a, 0)];
    }
    __syncthreads();
    double ri_[NB], rk_[NB], rd;  // the pivot column as read: rows tx + 16a, ty + 16b, and d_j
    read_col(colbuf[0], ri_, tx);
    read_col(colbuf[0], rk_, ty);
    rd = colbuf[0][0];
    // A thread records the column of L_BB (and D's entry) of the one pivot
    // per group of 16 that it owns, and stores them when the group ends:
    // a store inside the pivot loop would make every later write of its
    // data register wait for the store to complete, a full memory round
    // trip per pivot.
    double lc[NB], dd = 0.0;
#pragma unroll
    for (int a = 0; a < NB; ++a) lc[a] = 0.0;
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
        const int jt_end = min(16, s - 16 * jb);
        for (int jt = 0; jt < jt_end; ++jt) {
            const int j = 16 * jb + jt;
            const double dj = rd;
            // 1 / d_j: hardware reciprocal and two Newton steps (each squares
            // the relative error; the first estimate is good to about 2^-26)
            double inv = __builtin_amdgcn_rcp(dj);
            inv = fma(inv, fma(-dj, inv, 1.0), inv);
            inv = fma(inv, fma(-dj, inv, 1.0), inv);
            double ci[NB], ck[NB];
#pragma unroll
            for (int a = 0; a < NB; ++a) ci[a] = ri_[a] * inv;  // c_i / d_j
#pragma unroll
            for (int b = 0; b < NB; ++b) ck[b] = rk_[b];
            if (tid == 0) {
                const bool ok = isfinite(dj) && dj != 0.0 && (!require_spd || dj > 0.0);
                if (!ok) atomicMin(status, (unsigned long long)(d.first + j));
            }
            if (ty == jt) {  // column j of L_BB and D, stored after this group of 16 pivots
#pragma unroll
                for (int a = jb; a < NB; ++a) lc[a] = ci[a];
                dd = dj;
            }
            // M(tx + 16a, ty + 16b) after this pivot (a, b known at compile time)
            auto after = [&](int a, int b) {
                const bool ri = a == jb && tx == jt, rk = b == jb && ty == jt;
                const double upd = M[slot(a, b)] - ci[a] * ck[b];
                return (ri && rk) ? -inv : (ri ? ck[b] * inv : (rk ? ci[a] : upd));
            };
            // the next pivot's column, published before the bulk update
            const bool more = j + 1 < s;
            double* nb = colbuf[(j + 1) & 1];
            if (more) {
                if (jt + 1 < 16) {
                    if (ty == jt + 1) {
#pragma unroll
                        for (int a = jb; a < NB; ++a) nb[tx + 16 * a] = after(a, jb);
                    }
                    if (tx == jt + 1) {
#pragma unroll
                        for (int b = 0; b < jb; ++b) nb[ty + 16 * b] = after(jb, b);
                    }
                } else if (jb + 1 < NB) {
                    if (ty == 0) {
#pragma unroll
                        for (int a = jb + 1; a < NB; ++a) nb[tx + 16 * a] = after(a, jb + 1);
                    }
                    if (tx == 0) {
#pragma unroll
                        for (int b = 0; b < jb + 1; ++b) nb[ty + 16 * b] = after(jb + 1, b);
                    }
                }
            }
            __syncthreads();
            if (more) {
                read_col(nb, ri_, tx);
                read_col(nb, rk_, ty);
                rd = nb[j + 1];
            }
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b) M[slot(a, b)] = after(a, b);
        }
        const int jo = 16 * jb + ty;  // the pivot this thread recorded
        if (jo < s) {
#pragma unroll
            for (int a = jb; a < NB; ++a) {
                const int i = tx + 16 * a;
                if (i > jo && i < s) F[i + (int64_t)jo * ld] = lc[a];
            }
            if (tx == 0) F[jo + (int64_t)jo * ld] = dd;
        }
    }
    // T = -M, made exactly symmetric from the lower triangle
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tx + 16 * a, k = ty + 16 * b;
            if (i < s && k < s && i >= k) {
                T[i + (int64_t)k * s] = -M[slot(a, b)];
                T[k + (int64_t)i * s] = -M[slot(a, b)];
            }
        }
}

// f(integral_constant<int, I>) for I = I0 .. N - 1, each call with its own
// compile-time index (register arrays indexed by it stay in registers)
template <int I0, int N>
struct StaticFor {
    template <class Fn>
    __device__ __forceinline__ static void run(Fn&& f)
    {
        f(std::integral_constant<int, I0>{});
        StaticFor<I0 + 1, N>::run(f);
    }
};
template <int N>
struct StaticFor<N, N> {
    template <class Fn>
    __device__ __forceinline__ static void run(Fn&&)
    {
    }
};

// 1 / d: hardware reciprocal and two Newton steps (each squares the relative
// error; the first estimate is good to about 2^-26)
__device__ __forceinline__ double recip(double d)
{
    double inv = __builtin_amdgcn_rcp(d);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    return inv;
}

// The same sweep (same thread ownership of M, same arithmetic per entry) for
// a work-group that has the LDS to itself: every pivot's column is kept,
// lds[j W + i] = M(i, j) when pivot j is swept (W = 16 NB), and 1 / d_j in
// invd[j].  Rows below j of that column are the Schur-complement column, so
// L_BB and D are written from LDS after the sweep (coalesced, no store inside
// the pivot loop); T then goes through the same LDS, as a (W + 1)-strided
// square, to be stored column by column.  Per pivot, the entries of the next
// pivot's column are updated first and published, then, while the reads of
// that column are in flight, the rest; the two register sets of the pivot
// column alternate between pivots, so no copies are made.
template <int NB>
__device__ __forceinline__ void ldlt_sweep_cols(const BlockDesc d, double* __restrict__ Lp, double* __restrict__ Tp,
                                                unsigned long long* __restrict__ status, int require_spd,
                                                double* lds, double* invd)
{
    constexpr int NS = NB * (NB + 1) / 2;
    constexpr int W = 16 * NB;
    const int s = d.s;
    const int64_t ld = (int64_t)d.s + d.c;
    double* F = Lp + d.poff;
    double* T = Tp + d.woff;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    auto slot = [](int a, int b) { return a * (a + 1) / 2 + b; };
    double M[NS];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tx + 16 * a, k = ty + 16 * b;
            double v = 0.0;
            if (i < s && k < s) v = i >= k ? F[i + k * ld] : F[k + i * ld];
            M[slot(a, b)] = v;
        }
    if (ty == 0) {
#pragma unroll
        for (int a = 0; a < NB; ++a) lds[tx + 16 * a] = M[slot(a, 0)];
    }
    __syncthreads();
    // Column j of the LDS array.  Its offset is made opaque to the compiler:
    // folded into the instruction it would exceed the 16-bit immediate offset
    // of LDS instructions past 64 KiB, and every access would need an add.
    auto col_at = [&](int j) {
        int o = j * W;
        asm volatile("" : "+s"(o));
        return lds + o;
    };
    // the pivot column as read (rows tx + 16a, rows ty + 16b, d_j), in two sets
    double riA[NB], rkA[NB], rdA, riB[NB], rkB[NB], rdB;
    auto read_col = [&](int j, double (&ri)[NB], double (&rk)[NB], double& rd) {
        const double* col = col_at(j);
#pragma unroll
        for (int a = 0; a < NB; ++a) ri[a] = col[tx + 16 * a];
#pragma unroll
        for (int b = 0; b < NB; ++b) rk[b] = col[ty + 16 * b];
        rd = col[j];
    };
    read_col(0, riA, rkA, rdA);

    // Pivot j = 16 jb + jt.  `last`: jt = 15 with a next group, whose first
    // column lies in sub-block column jb + 1.
    auto pivot = [&](const int jb, const int jt, const bool last, const double (&ri)[NB], const double (&rk)[NB],
                     const double rd, double (&rin)[NB], double (&rkn)[NB], double& rdn) {
        const int j = 16 * jb + jt;
        const double dj = rd;
        const double inv = recip(dj);
        double ci[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) ci[a] = ri[a] * inv;  // c_i / d_j
        // the slots that hold the next pivot's column
        const int nb = last ? jb + 1 : jb;
        auto in_next = [&](int a, int b) { return (b == nb && a >= nb) || (a == nb && b < nb); };
        // M(i, k) -= c_i c_k / d_j for every slot of one phase, then row and
        // column j overwritten by the lanes that hold them (a, b known at
        // compile time; jb too, so only the slots of sub-block row / column
        // jb take part)
        auto update = [&](bool first) {
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    if (in_next(a, b) == first) M[slot(a, b)] = fma(-ci[a], rk[b], M[slot(a, b)]);
            if (ty == jt) {  // column j: c_i / d_j, and -1 / d_j on the diagonal
#pragma unroll
                for (int a = jb; a < NB; ++a)
                    if (in_next(a, jb) == first) M[slot(a, jb)] = (a == jb && tx == jt) ? -inv : ci[a];
            }
            if (tx == jt) {  // row j
#pragma unroll
                for (int b = 0; b <= jb; ++b)
                    if (in_next(jb, b) == first) M[slot(jb, b)] = (b == jb && ty == jt) ? -inv : rk[b] * inv;
            }
        };
        update(true);
        const bool more = j + 1 < s;
        const int nt = last ? 0 : jt + 1;  // the next pivot within sub-block nb
        if (more) {
            double* col = col_at(j + 1);
            if (ty == nt) {
#pragma unroll
                for (int a = nb; a < NB; ++a) col[tx + 16 * a] = M[slot(a, nb)];
            }
            if (tx == nt) {
#pragma unroll
                for (int b = 0; b < nb; ++b) col[ty + 16 * b] = M[slot(nb, b)];
            }
        }
        __syncthreads();
        if (more) read_col(j + 1, rin, rkn, rdn);
        update(false);
        // keeps this pivot's updates inside it, where they hide the latency
        // of the column reads (the compiler would sink them past the next
        // pivot's barrier)
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b)
                if (!in_next(a, b)) asm volatile("" : "+v"(M[slot(a, b)]));
    };
    auto copy_BA = [&]() {
#pragma unroll
        for (int a = 0; a < NB; ++a) riA[a] = riB[a], rkA[a] = rkB[a];
        rdA = rdB;
    };
    StaticFor<0, NB>::run([&](auto jbc) {
        constexpr int jb = decltype(jbc)::value;
        const int jt_end = min(16, s - 16 * jb);
        const bool handover = jt_end == 16 && 16 * (jb + 1) < s;
        const int nplain = handover ? 15 : jt_end;
        int jt = 0;
        for (; jt + 1 < nplain; jt += 2) {
            pivot(jb, jt, false, riA, rkA, rdA, riB, rkB, rdB);
            pivot(jb, jt + 1, false, riB, rkB, rdB, riA, rkA, rdA);
        }
        if (jt < nplain) {
            pivot(jb, jt, false, riA, rkA, rdA, riB, rkB, rdB);
            copy_BA();
        }
        if (handover) {
            pivot(jb, 15, true, riA, rkA, rdA, riB, rkB, rdB);
            copy_BA();
        }
    });
    // d_j is column j's diagonal entry: the pivot check (the first failing
    // pivot wins the atomic minimum) and 1 / d_j as the sweep formed it
    if (tid < s) {
        const double dj = lds[tid * W + tid];
        const bool ok = isfinite(dj) && dj != 0.0 && (!require_spd || dj > 0.0);
        if (!ok) atomicMin(status, (unsigned long long)(d.first + tid));
        invd[tid] = recip(dj);
    }
    __syncthreads();
    // L_BB(i, j) = c_i / d_j below the diagonal, D on it; eight columns per
    // thread at a time, their LDS reads issued together
    constexpr int kCols = kThreads / W;  // columns per pass
    constexpr int kU = 8;
    const int i = tid % W;
    for (int j0 = tid / W; j0 < s; j0 += kCols * kU) {
        double v[kU], r[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int j = min(j0 + u * kCols, W - 1);
            v[u] = lds[j * W + i];
            r[u] = invd[j];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int j = j0 + u * kCols;
            if (j < s && i >= j && i < s) F[i + (int64_t)j * ld] = i == j ? v[u] : v[u] * r[u];
        }
    }
    __syncthreads();  // column history read
    // T = -M, made exactly symmetric from the lower triangle
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int r = tx + 16 * a, k = ty + 16 * b;
            if (r >= k) {
                lds[r + k * (W + 1)] = -M[slot(a, b)];
                lds[k + r * (W + 1)] = -M[slot(a, b)];
            }
        }
    __syncthreads();
    for (int k0 = tid / W; k0 < s; k0 += kCols * kU) {
        double v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = lds[i + min(k0 + u * kCols, W - 1) * (W + 1)];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int k = k0 + u * kCols;
            if (k < s && i < s) T[i + (int64_t)k * s] = v[u];
        }
    }
}

// one launch per width class: NB = 2, 4, 8 for s <= 32, 64, 128; wider
// blocks take ldlt_global
template <int NB>
__global__ __launch_bounds__(kThreads) void k_ldlt_diag(const Task* __restrict__ tasks,
                                                        const BlockDesc* __restrict__ blk, double* __restrict__ Lp,
                                                        double* __restrict__ Wp, double* __restrict__ Tp,
                                                        unsigned long long* __restrict__ status, int require_spd)
{
    static_assert(kThreads % (16 * NB) == 0, "rows of a column split evenly over the work-group");
    __shared__ __align__(16) double lds[16 * NB * (16 * NB + 1)];
    __shared__ double invd[16 * NB];
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    if (d.s > 16 * NB) ldlt_global(d, Lp, Wp, Tp, status, require_spd);
    else ldlt_sweep_cols<NB>(d, Lp, Tp, status, require_spd, lds, invd);
}

// ---------------------------------------------------------------------------
// Diagonal block of a symmetric indefinite matrix: T_K = F_KK^{-1} with 1x1
// and 2x2 pivots chosen by the Bunch-Kaufman rule (Section 2.1: D may have
// 2x2 blocks; Bunch and Kaufman 1977 for the rule).  The rest of the method
// needs the diagonal block only through T (L_hat = F(C,K) T, the Schur update
// L_hat F(C,K)^T, Algorithm 1 and the adjoint), so the block is inverted
// directly by the symmetric sweep (Gauss-Jordan with diagonal pivots), which
// accepts the pivots in any order: a pivot on index p (d = M(p,p), c = column
// p) sets M(i,j) -= c_i c_j / d, M(i,p) = c_i / d, M(p,p) = -1/d; a 2x2 pivot
// on b = {p, r} does the same with E = M(b,b): M -= M(:,b) E^{-1} M(b,:),
// M(:,b) = M(:,b) E^{-1}, M(b,b) = -E^{-1}.  After every index is swept, M =
// -F_KK^{-1}.  The unswept part of M is the Schur complement the pivoted
// LDL^T would hold, so the rule is applied to it unchanged; an interchange
// only reorders the list of unswept indices (ord[position] = index), and no
// data moves.  The block lives in registers with the ownership of the
// positive definite sweep (lower 16 x 16 sub-blocks, thread (tx, ty) holds
// rows tx + 16a, columns ty + 16b); a pivot's column goes through LDS, where
// every wave reads it and takes the rule's decisions itself (the same values
// give every wave the same decision, so no decision is broadcast).  One
// work-group per block, NB = 2, 4, 8 for s <= 32, 64, 128.  A singular 1x1 or
// 2x2 pivot latches the block's first column in the status word.
// ---------------------------------------------------------------------------

// a value every lane holds alike, made known to the compiler as uniform
__device__ __forceinline__ double uniform_f64(double x)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(x), __double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(x), __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// largest x over the wave (NaN lanes ignored): within each row of 16 lanes
// by DPP (exchange within quads, then rotations by 4 and 8), then across
// the four rows
__device__ __forceinline__ double wave_max_f64(double x)
{
    x = fmax(x, dpp_f64<0xB1>(x));   // quad_perm [1,0,3,2]
    x = fmax(x, dpp_f64<0x4E>(x));   // quad_perm [2,3,0,1]
    x = fmax(x, dpp_f64<0x124>(x));  // row_ror:4
    x = fmax(x, dpp_f64<0x128>(x));  // row_ror:8
    return fmax(fmax(readlane_f64(x, 0), readlane_f64(x, 16)), fmax(readlane_f64(x, 32), readlane_f64(x, 48)));
}

// f(integral_constant<int, pb>) for the one pb in [0, NB) equal to the
// uniform value v
template <int NB, class Fn>
__device__ __forceinline__ void with_subblock(int v, Fn&& f)
{
    StaticFor<0, NB>::run([&](auto c) {
        if (v == decltype(c)::value) f(c);
    });
}

template <int NB>
__global__ __launch_bounds__(kThreads) void k_ldlt_bk(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                      const double* __restrict__ Lp, double* __restrict__ Tp,
                                                      unsigned long long* __restrict__ status)
{
    constexpr int NS = NB * (NB + 1) / 2;
    constexpr int W = 16 * NB;
    constexpr int NH = (W + 63) / 64;  // positions per lane in a search
    // columns of the pivots: [0], [1] alternate as the next candidate's
    // column, [2] holds the second candidate's (the row searched for sigma)
    __shared__ double cb[3][W];
    const BlockDesc d = blk[tasks[blockIdx.x].b];
    const int s = d.s;
    if (s > W) {  // the launch groups blocks by width, so this does not happen
        if (threadIdx.x == 0) atomicMin(status, (unsigned long long)d.first);
        return;
    }
    const int64_t ld = (int64_t)s + d.c;
    const double* F = Lp + d.poff;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4, lane = tid & 63;
    const double alpha = (1.0 + sqrt(17.0)) / 8.0;
    auto slot = [](int a, int b) { return a * (a + 1) / 2 + b; };
    double M[NS];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tx + 16 * a, k = ty + 16 * b;
            double v = 0.0;
            if (i < s && k < s) v = i >= k ? F[i + k * ld] : F[k + i * ld];
            M[slot(a, b)] = v;
        }
    // ord[q] for the positions q = lane + 64h this lane stands for in searches
    int ordq[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) ordq[h] = lane + 64 * h;
    auto ord_at = [&](int q) {
        int v = ordq[0];
        if (NH > 1 && q >= 64) v = ordq[NH - 1];
        return __builtin_amdgcn_readlane(v, q & 63);
    };
    auto swap_positions = [&](int q0, int q1) {
        const int v0 = ord_at(q0), v1 = ord_at(q1);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int q = lane + 64 * h;
            ordq[h] = q == q0 ? v1 : (q == q1 ? v0 : ordq[h]);
        }
    };
    // column p of M into col: rows at and below p's sub-block row from the
    // column's owners, rows above it from the owners of row p
    auto publish = [&](int p, double* col) {
        const int pt = p & 15;
        with_subblock<NB>(p >> 4, [&](auto pbc) {
            constexpr int pb = decltype(pbc)::value;
            if (ty == pt) {
#pragma unroll
                for (int a = pb; a < NB; ++a) col[tx + 16 * a] = M[slot(a, pb)];
            }
            if (tx == pt) {
#pragma unroll
                for (int b = 0; b < pb; ++b) col[ty + 16 * b] = M[slot(pb, b)];
            }
        });
    };
    // largest |col[ord[q]]| over positions q in [q0, s), q != skip, and the
    // smallest position holding it (-1 if none): the LDS reads, then the
    // reduction (split so that other reads can be issued in between)
    auto search_load = [&](const double* col, int q0, int skip, double (&v)[NH]) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int q = lane + 64 * h;
            const bool in = q >= q0 && q < s && q != skip;
            const double x = col[in ? ordq[h] : 0];
            v[h] = in ? fabs(x) : -1.0;
        }
    };
    auto search_reduce = [&](const double (&v)[NH], double& best, int& arg) {
        double m = -1.0;
#pragma unroll
        for (int h = 0; h < NH; ++h) m = fmax(m, v[h]);
        m = wave_max_f64(m);
        int a = -1;
        if (m >= 0.0) {
            const unsigned long long b0 = __ballot(v[0] == m);
            if (b0) a = __builtin_ctzll(b0);
            else if (NH > 1) a = 64 + __builtin_ctzll(__ballot(v[NH - 1] == m));
        }
        best = m;
        arg = a;
    };
    // pivot column values at this thread's rows (ri) and columns (rk)
    auto read_col = [&](const double* col, double (&ri)[NB], double (&rk)[NB]) {
#pragma unroll
        for (int a = 0; a < NB; ++a) ri[a] = col[tx + 16 * a];
#pragma unroll
        for (int b = 0; b < NB; ++b) rk[b] = col[ty + 16 * b];
    };
    // Lanes holding row p (rows tx + 16a) and column p (columns ty + 16b).
    // Row and column p are cleared and the pivot's own entries of the update
    // vectors set (row side at p to -1/d, column side at p to -1); the
    // update M(i,j) -= g_i x_j then writes the new row and column p too:
    // g_i where M(i,p) = 0, x_p = -1; x_j / d where M(p,j) = 0; -1/d at (p,p).
    auto hits = [&](int p, bool (&rz)[NB], bool (&cz)[NB]) {
#pragma unroll
        for (int a = 0; a < NB; ++a) rz[a] = tx + 16 * a == p;
#pragma unroll
        for (int b = 0; b < NB; ++b) cz[b] = ty + 16 * b == p;
    };

    publish(0, cb[0]);
    __syncthreads();
    int cur = 0;
    bool bad = false;
    double ri0[NB], rk0[NB], ri1[NB], rk1[NB];
    for (int k = 0; k < s;) {
        const int pk = ord_at(k);
        // the candidate's diagonal and the search first (they decide the
        // step), then its column for the update
        const double akk_raw = cb[cur][pk];
        double v[NH];
        search_load(cb[cur], k + 1, -1, v);
        read_col(cb[cur], ri0, rk0);
        double lam;
        int rq;
        search_reduce(v, lam, rq);
        const double akk_s = uniform_f64(akk_raw), akk = fabs(akk_s);
        int size = 1, sq = k;
        bool on_r = false;   // 1x1 pivot on the second candidate
        double rr_s = 0.0;   // M(r, r), signed
        double e01 = 0.0;    // M(r, k), signed
        if (rq < 0 || !(lam > 0.0)) {
            bad = akk == 0.0;
        } else if (akk < alpha * lam) {
            const int pr = ord_at(rq);
            const double e01_raw = cb[cur][pr];
            publish(pr, cb[2]);
            __syncthreads();
            const double rr_raw = cb[2][pr];
            search_load(cb[2], k, rq, v);
            double sig;
            int unused;
            search_reduce(v, sig, unused);
            rr_s = uniform_f64(rr_raw);
            e01 = uniform_f64(e01_raw);
            if (akk * sig >= alpha * lam * lam) {
                // 1x1 pivot on the first candidate
            } else if (fabs(rr_s) >= alpha * sig) {
                on_r = true;
                sq = rq;
            } else {
                size = 2;
                sq = rq;
            }
        }
        if (bad) break;
        const int kp = size == 2 ? k + 1 : k;
        if (sq != kp) swap_positions(kp, sq);
        const int p0 = ord_at(k);
        bool rz[NB], cz[NB];
        hits(p0, rz, cz);
        if (size == 1) {
            if (on_r) read_col(cb[2], ri0, rk0);
            const double dd = on_r ? rr_s : akk_s;
            if (dd == 0.0 || !isfinite(dd)) {
                bad = true;
                break;
            }
            const double inv = recip(dd);
            // g = c / d (rows), x = c (columns), the pivot's entries as above
#pragma unroll
            for (int a = 0; a < NB; ++a) ri0[a] = rz[a] ? -inv : ri0[a] * inv;
#pragma unroll
            for (int b = 0; b < NB; ++b) rk0[b] = cz[b] ? -1.0 : rk0[b];
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    M[slot(a, b)] = fma(-ri0[a], rk0[b], (rz[a] || cz[b]) ? 0.0 : M[slot(a, b)]);
        } else {
            const int p1 = ord_at(k + 1);
            bool rz1[NB], cz1[NB];
            hits(p1, rz1, cz1);
            read_col(cb[2], ri1, rk1);
            const double e00 = akk_s, e11 = rr_s;
            const double det = e00 * e11 - e01 * e01;
            if (det == 0.0 || !isfinite(det)) {
                bad = true;
                break;
            }
            const double rdet = recip(det);
            const double i00 = e11 * rdet, i01 = -e01 * rdet, i11 = e00 * rdet;
            // rows: (g0, g1) = M(i, b) E^{-1}, and -E^{-1}'s rows at p0, p1;
            // columns: (x0, x1) = M(b, j), and -(1, 0), -(0, 1) at p0, p1.
            // With rows and columns p0, p1 cleared, M(i,j) -= g0_i x0_j +
            // g1_i x1_j gives M(:,b) E^{-1} in those columns, E^{-1} M(b,:)
            // in those rows and -E^{-1} on the block.
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                const double x = ri0[a], y = ri1[a];
                ri0[a] = rz[a] ? -i00 : (rz1[a] ? -i01 : x * i00 + y * i01);
                ri1[a] = rz[a] ? -i01 : (rz1[a] ? -i11 : x * i01 + y * i11);
                rz[a] = rz[a] || rz1[a];
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                rk0[b] = cz[b] ? -1.0 : (cz1[b] ? 0.0 : rk0[b]);
                rk1[b] = cz[b] ? 0.0 : (cz1[b] ? -1.0 : rk1[b]);
                cz[b] = cz[b] || cz1[b];
            }
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    M[slot(a, b)] = fma(-ri0[a], rk0[b],
                                        fma(-ri1[a], rk1[b], (rz[a] || cz[b]) ? 0.0 : M[slot(a, b)]));
        }
        k += size;
        if (k < s) publish(ord_at(k), cb[cur ^ 1]);
        __syncthreads();
        cur ^= 1;
    }
    if (bad) {  // every thread took the same decisions
        if (tid == 0) atomicMin(status, (unsigned long long)d.first);
        return;
    }
    // T = -M from the lower triangle (exactly symmetric)
    double* T = Tp + d.woff;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = tx + 16 * a, j = ty + 16 * b;
            if (i < s && j < s && i >= j) {
                T[i + (int64_t)j * s] = -M[slot(a, b)];
                T[j + (int64_t)i * s] = -M[slot(a, b)];
            }
        }
}

// ===========================================================================
// Small blocks (s <= 16, c <= 256): one wave runs a whole block, every phase
// in turn, on 16 x 16 FP64 MFMA tiles (output rows in groups of 16, the
// contraction in steps of 4), so a block needs no other wave and no
// work-group barrier.  Per wave, LDS holds the s x s diagonal block during
// its sweep (then T = -M) and one 16 x 16 tile for transposition.
//   factor:  sweep F_BB -> L_BB, D, T;  per row group I of C: L_hat(I,:) =
//            F(I,B) T, then for every row group K <= I the Schur tile
//            -L_hat(I,:) F(K,:)^T added into the ancestors (lower part);
//   invert:  per row group I: X(I,:) = -G(I,:) L_hat, written to Ainv(C,B),
//            and P += L_hat(I,:)^T X(I,:) straight from the accumulators;
//            then Ainv(B,B) = ((T - P) + (T - P)^T) / 2 on the lower triangle.
// ===========================================================================
struct SbLds {
    double M[16][17];
    double L[16][17];
};

__device__ void sb_factor(const BlockDesc d, double* __restrict__ Lp, double* __restrict__ Hp,
                          double* __restrict__ Tp, const int64_t* __restrict__ cbase,
                          const int64_t* __restrict__ rbase, const int32_t* __restrict__ rel,
                          unsigned long long* __restrict__ status, int require_spd, SbLds& S)
{
    const int lane = threadIdx.x & 63;
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    double* F = Lp + d.poff;
    // diagonal block: symmetric Gauss-Jordan sweep (as in ldlt_sweep), lane
    // holds entries (e & 15, e >> 4) for e = lane + 64 q
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q, i = e & 15, k = e >> 4;
        S.M[i][k] = (i < s && k < s) ? (i >= k ? F[i + k * ld] : F[k + i * ld]) : 0.0;
    }
    wave_sync();
    for (int j = 0; j < s; ++j) {
        const double dj = S.M[j][j];
        const double inv = 1.0 / dj;
        double nv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = lane + 64 * q, i = e & 15, k = e >> 4;
            const double ci = S.M[i][j], ck = S.M[k][j], m = S.M[i][k];
            nv[q] = (i == j && k == j) ? -inv : (i == j ? ck * inv : (k == j ? ci * inv : m - ci * ck * inv));
        }
        const double cl = S.M[lane & 15][j];  // Schur-complement column j
        wave_sync();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = lane + 64 * q, i = e & 15, k = e >> 4;
            if (i < s && k < s) S.M[i][k] = nv[q];
        }
        if (lane < s && lane > j) F[lane + j * ld] = cl * inv;  // L_BB(i, j)
        if (lane == j) F[j + j * ld] = dj;                      // D_j
        if (lane == 0 && !(isfinite(dj) && dj != 0.0 && (!require_spd || dj > 0.0)))
            atomicMin(status, (unsigned long long)(d.first + j));
        wave_sync();
    }
    // T = -M (the sweep keeps M exactly symmetric)
    double* T = Tp + d.woff;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q, i = e & 15, k = e >> 4;
        if (i < s && k < s) T[i + (int64_t)k * s] = -S.M[i][k];
    }
    const double* FC = F + s;  // F(C,B)(i, k) = FC[i + k ld]
    double* H = Hp + d.hoff;
    const int m16 = lane & 15, q4 = lane >> 4;
    for (int r0 = 0; r0 < c; r0 += 16) {
        // L_hat(I,:) = F(I,B) T
        d4 acc = {0, 0, 0, 0};
        for (int k0 = 0; k0 < s; k0 += 4) {
            const int kk = k0 + q4;
            const double a = (r0 + m16 < c && kk < s) ? FC[(r0 + m16) + (int64_t)kk * ld] : 0.0;
            const double b = (kk < s && m16 < s) ? -S.M[kk][m16] : 0.0;
            acc = mfma(a, b, acc);
        }
        mfma_drain();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = r0 + q4 + 4 * v;
            if (row < c && m16 < s) H[row + (int64_t)m16 * c] = acc[v];
            S.L[q4 + 4 * v][m16] = acc[v];
        }
        wave_sync();
        // Schur tiles (I, K), K <= I: F(C,C) -= L_hat(I,:) F(K,:)^T, lower part
        for (int k0c = 0; k0c <= r0; k0c += 16) {
            d4 u = {0, 0, 0, 0};
            for (int t0 = 0; t0 < s; t0 += 4) {
                const int kk = t0 + q4;
                const double a = kk < s ? S.L[m16][kk] : 0.0;
                const double b = (k0c + m16 < c && kk < s) ? FC[(k0c + m16) + (int64_t)kk * ld] : 0.0;
                u = mfma(a, b, u);
            }
            mfma_drain();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ii = r0 + q4 + 4 * v, kk = k0c + m16;
                if (ii < c && kk < c && ii >= kk) {
                    const int64_t pk = d.coff + kk;
                    unsafeAtomicAdd(Lp + cbase[pk] + rel[rbase[pk] + ii], -u[v]);
                }
            }
        }
        wave_sync();
    }
}

__device__ void sb_invert(const BlockDesc d, double* __restrict__ Ap, const double* __restrict__ Hp,
                          const double* __restrict__ Tp, const int64_t* __restrict__ cbase,
                          const int64_t* __restrict__ rbase, const int32_t* __restrict__ rel, SbLds& S)
{
    const int lane = threadIdx.x & 63;
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const double* H = Hp + d.hoff;
    const double* T = Tp + d.woff;
    double* A = Ap + d.poff;
    const int m16 = lane & 15, q4 = lane >> 4;
    d4 p = {0, 0, 0, 0};  // P = L_hat^T X
    for (int r0 = 0; r0 < c; r0 += 16) {
        const int i = r0 + m16;
        d4 acc = {0, 0, 0, 0};
        for (int k0 = 0; k0 < c; k0 += 4) {
            const int kk = k0 + q4;
            double g = 0.0;
            if (i < c && kk < c) {
                const int64_t pc = d.coff + (i >= kk ? kk : i);
                g = Ap[cbase[pc] + rel[rbase[pc] + (i >= kk ? i : kk)]];
            }
            const double b = (kk < c && m16 < s) ? H[kk + (int64_t)m16 * c] : 0.0;
            acc = mfma(g, b, acc);
        }
        mfma_drain();
        // acc[v] = (G L_hat)(r0 + q4 + 4v, m16): X = -acc
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = r0 + q4 + 4 * v;
            if (row < c && m16 < s) A[s + row + (int64_t)m16 * ld] = -acc[v];
        }
        // P += L_hat(I,:)^T X(I,:): B(kk, n) = X(r0 + 4t + kk, n) is -acc[t] of this lane
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = r0 + 4 * t + q4;
            const double a = (row < c && m16 < s) ? H[row + (int64_t)m16 * c] : 0.0;
            p = mfma(a, -acc[t], p);
        }
    }
    mfma_drain();
#pragma unroll
    for (int v = 0; v < 4; ++v) S.M[q4 + 4 * v][m16] = p[v];
    wave_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q, ii = e & 15, jj = e >> 4;
        if (ii < s && jj < s && ii >= jj)
            A[ii + (int64_t)jj * ld] = 0.5 * ((T[ii + (int64_t)jj * s] - S.M[ii][jj]) + (T[jj + (int64_t)ii * s] - S.M[jj][ii]));
    }
    wave_sync();
}

// Per-level launches of the small-block path: task q holds up to four block
// ids (b, i0, j0, bn; -1 = none), one per wave.
__device__ __forceinline__ int sb_block_of(const Task& t)
{
    const int w = threadIdx.x >> 6;
    return w == 0 ? t.b : w == 1 ? t.i0 : w == 2 ? t.j0 : t.bn;
}

__global__ __launch_bounds__(kThreads) void k_sb_factor(const Task* __restrict__ tasks,
                                                        const BlockDesc* __restrict__ blk, double* __restrict__ Lp,
                                                        double* __restrict__ Hp, double* __restrict__ Tp,
                                                        const int64_t* __restrict__ cbase,
                                                        const int64_t* __restrict__ rbase,
                                                        const int32_t* __restrict__ rel,
                                                        unsigned long long* __restrict__ status, int require_spd)
{
    __shared__ SbLds S[kThreads / 64];
    const int b = sb_block_of(tasks[blockIdx.x]);
    if (b >= 0) sb_factor(blk[b], Lp, Hp, Tp, cbase, rbase, rel, status, require_spd, S[threadIdx.x >> 6]);
}

__global__ __launch_bounds__(kThreads) void k_sb_invert(const Task* __restrict__ tasks,
                                                        const BlockDesc* __restrict__ blk, double* __restrict__ Ap,
                                                        const double* __restrict__ Hp, const double* __restrict__ Tp,
                                                        const int64_t* __restrict__ cbase,
                                                        const int64_t* __restrict__ rbase,
                                                        const int32_t* __restrict__ rel)
{
    __shared__ SbLds S[kThreads / 64];
    const int b = sb_block_of(tasks[blockIdx.x]);
    if (b >= 0) sb_invert(blk[b], Ap, Hp, Tp, cbase, rbase, rel, S[threadIdx.x >> 6]);
}

// ===========================================================================
// Persistent level kernels (batched form).  One launch per tree level runs
// every task of the level, across all blocks of all matrices of a batch,
// from a work queue: a work-group claims the next index with an atomic add
// on the level's queue head until the queue is empty.  Tasks of one block
// depend on the block's earlier phases (factor: diagonal block -> L_hat
// tiles -> Schur tiles; inversion: zero X -> X tiles -> diagonal tiles); a
// task waits until its block's completion counter reaches task.pad.  Waits
// are on smaller queue indices only, which running work-groups hold, so
// every wait ends; a wait that exceeds spin_limit polls latches status[1]
// and the task proceeds, so the kernel always drains.
// ===========================================================================
union PersistLds {
    TileLds tile;
    GemmLds gemm;
    SdiagLds sd;
    alignas(16) double colbuf[2][kLdsDiagMax];
    SbLds sb[kThreads / 64];
};


struct QueueArgs {
    const Task* q;
    int64_t ntasks;
    unsigned* head;   // this level's queue head
    unsigned* done;   // per-block completion counters of this sweep
    unsigned long long* status;
    int require_spd;
    unsigned spin_limit;
};

// The claimed index is the same in every thread; readfirstlane makes it a
// wave-uniform (scalar) value, so the compiler sees a uniform loop whose
// barriers every thread reaches together.
__device__ __forceinline__ int claim(const QueueArgs& a, int* s_idx)
{
    if (threadIdx.x == 0) *s_idx = (int)__hip_atomic_fetch_add(a.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(*s_idx);
    __syncthreads();
    return idx;
}

__device__ __forceinline__ Task uniform_task(const Task* q, int idx)
{
    const Task r = q[idx];
    Task t;
    t.b = __builtin_amdgcn_readfirstlane(r.b);
    t.i0 = __builtin_amdgcn_readfirstlane(r.i0);
    t.j0 = __builtin_amdgcn_readfirstlane(r.j0);
    t.bn = __builtin_amdgcn_readfirstlane(r.bn);
    t.kb = __builtin_amdgcn_readfirstlane(r.kb);
    t.ke = __builtin_amdgcn_readfirstlane(r.ke);
    t.flags = __builtin_amdgcn_readfirstlane(r.flags);
    t.pad = __builtin_amdgcn_readfirstlane(r.pad);
    return t;
}

// Thread 0 polls the block's counter (relaxed loads; one acquire fence for
// the whole work-group once the count is reached).  A wait gives up after
// spin_limit polls, or at once when another wait has already given up, so
// a run ends within about one poll limit whatever happens.
__device__ __forceinline__ void wait_deps(const QueueArgs& a, const Task& t)
{
    if (t.pad > 0 && threadIdx.x == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(a.done + t.b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)t.pad) {
            const bool gave_up =
                (spins & 255u) == 0 && __hip_atomic_load(a.status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            if (gave_up || ++spins > a.spin_limit) {
                atomicOr(a.status + 1, 1ull);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void signal_done(const QueueArgs& a, const Task& t)
{
    __threadfence();  // every thread's results reach device scope first
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(a.done + t.b, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// diagonal block of a tiled level: the host keeps s <= 16 NB, or NB = 8
template <int NB>
__device__ __forceinline__ void diag_block(const BlockDesc& d, double* Lp, double* Wp, double* Tp,
                                           unsigned long long* status, int require_spd, double (*colbuf)[kLdsDiagMax])
{
    if constexpr (NB == 8) {
        if (d.s > kLdsDiagMax) {
            ldlt_global(d, Lp, Wp, Tp, status, require_spd);
            return;
        }
    }
    ldlt_sweep<NB>(d, Lp, Tp, status, require_spd, colbuf);
}

// L_hat tile; tiles are at most as wide as the level's widest block
template <int NB>
__device__ __forceinline__ void panel_bounded(GemmLds& L, const Task& t, const BlockDesc& d, const double* Lp,
                                              double* Hp, const double* Tp)
{
    if (t.bn <= 16) {
        panel_task<16>(L, t, d, Lp, Hp, Tp);
    } else if (t.bn <= 32) {
        panel_task<32>(L, t, d, Lp, Hp, Tp);
    } else if constexpr (NB >= 4) {
        if (t.bn <= 64) panel_task<64>(L, t, d, Lp, Hp, Tp);
        else if constexpr (NB >= 8) panel_task<128>(L, t, d, Lp, Hp, Tp);
    }
}

// gather-GEMM tile; the host keeps t.bn <= BNMAX in this variant's levels
template <int BNMAX>
__device__ __forceinline__ void gemm_bounded(GemmLds& L, const Task& t, const BlockDesc& d, double* Ap,
                                             const double* Hp, const int64_t* cr2,
                                             const int32_t* rel)
{
    if (t.bn <= 16) {
        gemm_task<16>(L, t, d, Ap, Hp, cr2, rel);
    } else if (t.bn <= 32) {
        gemm_task<32>(L, t, d, Ap, Hp, cr2, rel);
    } else if constexpr (BNMAX >= 64) {
        if (t.bn <= 64) gemm_task<64>(L, t, d, Ap, Hp, cr2, rel);
        else if constexpr (BNMAX >= 128) gemm_task<128>(L, t, d, Ap, Hp, cr2, rel);
    }
}

// Levels with tiled blocks; NB bounds the diagonal sweep (s <= 16 NB, wider
// blocks take ldlt_global) and so the kernel's registers.
template <int NB>
__global__ __launch_bounds__(kThreads, NB < 8 ? 2 : 1) void k_persist_factor(const QueueArgs a, const BlockDesc* __restrict__ blk,
                                                             double* __restrict__ Lp, double* __restrict__ Wp,
                                                             double* __restrict__ Hp, double* __restrict__ Tp,
                                                             const int64_t* __restrict__ cbase,
                                                             const int64_t* __restrict__ rbase,
                                                             const int32_t* __restrict__ rel)
{
    __shared__ PersistLds sm;
    __shared__ int s_idx;
    // a work-group cannot claim more than ntasks entries: the bound only
    // makes termination evident
    for (int64_t it = 0; it < a.ntasks; ++it) {
        const int idx = claim(a, &s_idx);
        if (idx >= a.ntasks) break;
        const Task t = uniform_task(a.q, idx);
        const int op = t.flags >> 8;
        if (op == qSbFactor) {
            const int b = sb_block_of(t);
            if (b >= 0)
                sb_factor(blk[b], Lp, Hp, Tp, cbase, rbase, rel, a.status, a.require_spd, sm.sb[threadIdx.x >> 6]);
            __syncthreads();  // the LDS union is reused by the next task
            continue;
        }
        const BlockDesc d = blk[t.b];
        // a medium block runs its diagonal block, L_hat tiles and Schur tiles
        // here in turn (one call site per routine keeps registers down)
        const bool whole = op == qMbFactor;
        if (!whole) wait_deps(a, t);
        const int nrow = (d.c + kTileM - 1) / kTileM, ncol = whole ? (d.s + t.bn - 1) / t.bn : 0;
        const int nsc = (d.c + kSchurTile - 1) / kSchurTile;
        const int steps = whole ? 1 + nrow * ncol + nsc * (nsc + 1) / 2 : 1;
        int pr = 0, pj = 0, si = 0, sk = 0;  // next panel tile (row, column), Schur tile (row, column)
        for (int st = 0; st < steps; ++st) {
            int o = op;
            Task u = t;
            if (whole) {
                if (st == 0) {
                    o = qLdlt;
                } else if (st <= nrow * ncol) {
                    o = qPanel;
                    u = Task{t.b, pr * kTileM, pj * t.bn, t.bn, 0, d.s, 0, 0};
                    if (++pr == nrow) pr = 0, ++pj;
                } else {
                    o = qSchur;
                    u = Task{t.b, si * kSchurTile, sk * kSchurTile, kSchurTile, 0, d.s, t.flags & 4, 0};
                    if (++si == nsc) si = ++sk;
                }
            }
            switch (o) {
                case qLdlt:
                    diag_block<NB>(d, Lp, Wp, Tp, a.status, a.require_spd, sm.colbuf);
                    break;
                case qPanel:
                    panel_bounded<NB>(sm.gemm, u, d, Lp, Hp, Tp);
                    break;
                default:
                    schur_task(sm.gemm, u, d, Lp, Hp, cbase, rbase, rel);
                    break;
            }
            if (whole) __syncthreads();
        }
        if (!whole && (t.flags & 2)) signal_done(a, t);
        else __syncthreads();
    }
}

// Levels with tiled blocks; BNMAX bounds the gather-GEMM tile width and so
// the kernel's registers.
template <int BNMAX>
__global__ __launch_bounds__(kThreads, 2) void k_persist_invert(const QueueArgs a, const BlockDesc* __restrict__ blk,
                                                                double* __restrict__ Ap, const double* __restrict__ Hp,
                                                                const double* __restrict__ Tp,
                                                                const int64_t* __restrict__ cbase,
                                                                const int64_t* __restrict__ rbase,
                                                                const int32_t* __restrict__ rel,
                                                                const int64_t* __restrict__ cr2)
{
    __shared__ PersistLds sm;
    __shared__ int s_idx;
    for (int64_t it = 0; it < a.ntasks; ++it) {
        const int idx = claim(a, &s_idx);
        if (idx >= a.ntasks) break;
        const Task t = uniform_task(a.q, idx);
        const int op = t.flags >> 8;
        if (op == qSbInvert) {
            const int b = sb_block_of(t);
            if (b >= 0) sb_invert(blk[b], Ap, Hp, Tp, cbase, rbase, rel, sm.sb[threadIdx.x >> 6]);
            __syncthreads();
            continue;
        }
        const BlockDesc d = blk[t.b];
        // a medium block runs its X tiles (whole contractions) and then its
        // diagonal tiles here in turn
        const bool whole = op == qMbInvert;
        if (!whole) wait_deps(a, t);
        const int nrow = (d.c + kTileM - 1) / kTileM, ncol = whole ? (d.s + t.bn - 1) / t.bn : 0;
        const int nd = (d.s + kDiagTile - 1) / kDiagTile;
        const int steps = whole ? nrow * ncol + nd * (nd + 1) / 2 : 1;
        int gr = 0, gj = 0, di = 0, dj = 0;  // next X tile (row, column), diagonal tile pair (I, J)
        for (int st = 0; st < steps; ++st) {
            int o = op;
            Task u = t;
            if (whole) {
                if (st < nrow * ncol) {
                    o = qGemm;
                    u = Task{t.b, gr * kTileM, gj * t.bn, t.bn, 0, d.c, 0, 0};
                    if (++gr == nrow) gr = 0, ++gj;
                } else {
                    o = qSdiag;
                    u = Task{t.b, di * kDiagTile, dj * kDiagTile, 0, 0, d.c, 0, 0};
                    if (++dj > di) dj = 0, ++di;
                }
            }
            switch (o) {
                case qZero:
                    zero_task(d, Ap, Tp);
                    break;
                case qGemm:
                    gemm_bounded<BNMAX>(sm.gemm, u, d, Ap, Hp, cr2, rel);
                    break;
                default:
                    sdiag_task(sm.sd, u, d, Ap, Hp, Tp);
                    break;
            }
            if (whole) __syncthreads();
        }
        if (!whole && (t.flags & 2)) signal_done(a, t);
        else __syncthreads();
    }
}

// Levels made only of small blocks: no dependencies, so no queue head
// either.  Wave g of W takes slots g, g + W, g + 2W, ... (slot = 4 task +
// wave field) of the level's cost-ordered list, so every wave gets a like
// mix; no atomics, no work-group barrier.
__device__ __forceinline__ int slot_block(const QueueArgs& a, int64_t slot)
{
    const int32_t* ids = reinterpret_cast<const int32_t*>(a.q + slot / kSbPerTask);
    return __builtin_amdgcn_readfirstlane(ids[slot % kSbPerTask]);
}

__global__ __launch_bounds__(kThreads) void k_light_factor(const QueueArgs a, const BlockDesc* __restrict__ blk,
                                                           double* __restrict__ Lp, double* __restrict__ Hp,
                                                           double* __restrict__ Tp, const int64_t* __restrict__ cbase,
                                                           const int64_t* __restrict__ rbase,
                                                           const int32_t* __restrict__ rel)
{
    __shared__ SbLds S[kThreads / 64];
    const int64_t nslots = a.ntasks * kSbPerTask;
    const int64_t nw = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t slot = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); slot < nslots; slot += nw) {
        const int b = slot_block(a, slot);
        if (b >= 0) sb_factor(blk[b], Lp, Hp, Tp, cbase, rbase, rel, a.status, a.require_spd, S[threadIdx.x >> 6]);
    }
}

__global__ __launch_bounds__(kThreads) void k_light_invert(const QueueArgs a, const BlockDesc* __restrict__ blk,
                                                           double* __restrict__ Ap, const double* __restrict__ Hp,
                                                           const double* __restrict__ Tp,
                                                           const int64_t* __restrict__ cbase,
                                                           const int64_t* __restrict__ rbase,
                                                           const int32_t* __restrict__ rel,
                                                                const int64_t* __restrict__ cr2)
{
    __shared__ SbLds S[kThreads / 64];
    const int64_t nslots = a.ntasks * kSbPerTask;
    const int64_t nw = (int64_t)gridDim.x * (kThreads / 64);
    for (int64_t slot = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); slot < nslots; slot += nw) {
        const int b = slot_block(a, slot);
        if (b >= 0) sb_invert(blk[b], Ap, Hp, Tp, cbase, rbase, rel, S[threadIdx.x >> 6]);
    }
}

__global__ void k_fill_u32(unsigned* __restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ===========================================================================
// Reverse sweep: adjoint of the factorization and of the selected inversion.
// Adjoints are those of the stored values: an entry of a diagonal block's
// lower triangle stands for both (i,j) and (j,i), an entry of the C rows for
// itself.  Zb holds the adjoint of Ainv during the reverse selected
// inversion (leaves first) and the adjoint of F during the reverse
// factorization (root first), in the panel layout; Hb is the adjoint of
// L_hat and Tb that of T.  Per block, with Zbar the adjoint of its panel:
//   Ybar = (Zbar_BB + Zbar_BB^T)/2,  Xbar = Zbar(C,B) - L_hat Ybar,
//   Lhat_bar = -X Ybar - G Xbar,  Tbar = Ybar,
//   ancestors' Zbar(C,C) += -(Xbar L_hat^T + L_hat Xbar^T)  (stored lower);
// then, root first, with Ubar(i,k) = -Fbar(C[i],C[k]) (i >= k) from the
// ancestors: Lhat_bar += Ubar F(C,B), Fbar(C,B) = Ubar^T L_hat + Lhat_bar T,
// Tbar += F(C,B)^T Lhat_bar, Fbar_BB = -T (Tbar + Tbar^T) T (stored lower).
// The gradient of A's entries is Fbar at their positions.
// ===========================================================================
__device__ __forceinline__ double ybar_at(const double* __restrict__ Zd, int64_t ld, int t, int j)
{
    if (t == j) return Zd[t + (int64_t)t * ld];
    const int a = t > j ? t : j, b = t > j ? j : t;
    return 0.5 * Zd[a + (int64_t)b * ld];
}

template <int BN>
__device__ void rs1_task(TileLds& L, const Task t, const BlockDesc d, double* __restrict__ Zb,
                         const double* __restrict__ Hp)
{
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int r0 = t.i0, n0 = t.j0;
    const double* Zd = Zb + d.poff;
    d4 acc[2][4] = {};
    auto loadA = [&](int k0, int kk, int ii) -> double {
        const int i = r0 + ii, k = k0 + kk;
        return (i < c && k < s) ? Hp[d.hoff + i + (int64_t)k * c] : 0.0;
    };
    auto loadB = [&](int k0, int kk, int j) -> double {
        const int k = k0 + kk, jj = n0 + j;
        return (k < s && jj < s) ? ybar_at(Zd, ld, k, jj) : 0.0;
    };
    tile_mma<BN>(L, 0, s, acc, loadA, loadB, [](int) { return false; });
    tile_epilogue_t<BN>(acc, [&](int i, int j, double v) {
        const int ii = r0 + i, jj = n0 + j;
        if (ii < c && jj < s) Zb[d.poff + s + ii + (int64_t)jj * ld] -= v;
    });
}

__global__ __launch_bounds__(kThreads) void k_rs1(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                  double* __restrict__ Zb, const double* __restrict__ Hp)
{
    __shared__ TileLds L;
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
#define SELINV_CALL(BN) rs1_task<BN>(L, t, d, Zb, Hp)
    SELINV_BN_DISPATCH(t.bn, SELINV_CALL)
#undef SELINV_CALL
}

template <int BN, bool kPair>
__device__ void rs2_task(GemmLds& L, const Task t, const BlockDesc d, const double* __restrict__ Ap,
                         const double* __restrict__ Zb, double* __restrict__ Hb, const int64_t* __restrict__ cr2, const int32_t* __restrict__ rel)
{
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int r0 = t.i0, n0 = t.j0;
    const double* Zd = Zb + d.poff;
    d4 acc[2][4] = {};
    // G Xbar: G gathered from the inverse panels, Xbar = Zbar(C,B)
    gather_mma<BN, kPair, 0>(L, d, r0, n0, t.kb, t.ke, Ap, Zb + d.poff + s, ld, cr2, rel, acc);
    if (t.kb == 0) {  // -X Ybar, once per tile
        auto loadX = [&](int k0, int kk, int ii) -> double {
            const int i = r0 + ii, k = k0 + kk;
            return (i < c && k < s) ? Ap[d.poff + s + i + (int64_t)k * ld] : 0.0;
        };
        auto loadY = [&](int k0, int kk, int j) -> double {
            const int k = k0 + kk, jj = n0 + j;
            return (k < s && jj < s) ? ybar_at(Zd, ld, k, jj) : 0.0;
        };
        tile_mma<BN>(reinterpret_cast<TileLds&>(L), 0, s, acc, loadX, loadY, [](int) { return false; });
    }
    tile_epilogue_t<BN>(acc, [&](int i, int j, double v) {
        const int ii = r0 + i, jj = n0 + j;
        if (ii < c && jj < s) {
            double* p = Hb + d.hoff + ii + (int64_t)jj * c;
            if (t.flags & 1) unsafeAtomicAdd(p, -v); else *p = -v;
        }
    });
}

__global__ __launch_bounds__(kThreads) void k_rs2(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                  const double* __restrict__ Ap, const double* __restrict__ Zb,
                                                  double* __restrict__ Hb, const int64_t* __restrict__ cr2, const int32_t* __restrict__ rel)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
#define SELINV_CALL(BN)                                                                        \
    if (BN >= 32 && (d.c & 1) == 0) rs2_task<BN, BN >= 32>(L, t, d, Ap, Zb, Hb, cr2, rel); \
    else rs2_task<BN, false>(L, t, d, Ap, Zb, Hb, cr2, rel)
    SELINV_BN_DISPATCH(t.bn, SELINV_CALL)
#undef SELINV_CALL
}

// ancestors' Zbar += -(Xbar L_hat^T + L_hat Xbar^T): lower tile rows
// [i0, i0+64) x columns [k0, k0+64), contraction over [Xbar | L_hat]
__global__ __launch_bounds__(kThreads) void k_rs3(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                  double* __restrict__ Zb, const double* __restrict__ Hp,
                                                  const int64_t* __restrict__ cbase,
                                                  const int64_t* __restrict__ rbase, const int32_t* __restrict__ rel)
{
    __shared__ TileLds L;
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int i0 = t.i0, k0c = t.j0;
    const double* Xb = Zb + d.poff + s;
    const double* H = Hp + d.hoff;
    d4 acc[2][4] = {};
    auto loadA = [&](int q0, int qq, int ii) -> double {
        const int i = i0 + ii, q = q0 + qq;
        if (i >= c || q >= 2 * s) return 0.0;
        return q < s ? Xb[i + (int64_t)q * ld] : H[i + (int64_t)(q - s) * c];
    };
    auto loadB = [&](int q0, int qq, int j) -> double {
        const int k = k0c + j, q = q0 + qq;
        if (k >= c || q >= 2 * s) return 0.0;
        return q < s ? H[k + (int64_t)q * c] : Xb[k + (int64_t)(q - s) * ld];
    };
    tile_mma<64>(L, 0, 2 * s, acc, loadA, loadB, [](int) { return false; });
    tile_epilogue_t<64>(acc, [&](int i, int j, double v) {
        const int ii = i0 + i, kk = k0c + j;
        if (ii < c && kk < c && ii >= kk) {
            const int64_t pk = d.coff + kk;
            double* z = Zb + cbase[pk] + rel[rbase[pk] + ii];
            const double u = ii == kk ? -0.5 * v : -v;
            if (t.flags & 4) *z += u;  // colour group: no other writer in this launch
            else unsafeAtomicAdd(z, u);
        }
    });
}

// Tbar := Ybar for every block, once the reverse selected inversion is done
__global__ void k_tbar_init(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                            const double* __restrict__ Zb, double* __restrict__ Tb)
{
    const BlockDesc d = blk[tasks[blockIdx.x].b];
    const int64_t ld = (int64_t)d.s + d.c;
    for (int e = threadIdx.x; e < d.s * d.s; e += blockDim.x)
        Tb[d.woff + e] = ybar_at(Zb + d.poff, ld, e % d.s, e / d.s);
}

// Lhat_bar += Ubar F(C,B), Ubar(i,k) = -Fbar(C[i],C[k]) for i >= k
template <int BN, bool kPair>
__device__ void rf1a_task(GemmLds& L, const Task t, const BlockDesc d, const double* __restrict__ Zb,
                          const double* __restrict__ Lp, double* __restrict__ Hb, const int64_t* __restrict__ cr2, const int32_t* __restrict__ rel)
{
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int r0 = t.i0, n0 = t.j0;
    d4 acc[2][4] = {};
    // Ubar(i,k) = -Fbar(C[i],C[k]) for k <= i, gathered from the adjoint panels; B = F(C,B)
    gather_mma<BN, kPair, 1>(L, d, r0, n0, t.kb, t.ke, Zb, Lp + d.poff + s, ld, cr2, rel, acc);
    tile_epilogue_t<BN>(acc, [&](int i, int j, double v) {
        const int ii = r0 + i, jj = n0 + j;
        if (ii < c && jj < s) {
            double* p = Hb + d.hoff + ii + (int64_t)jj * c;
            if (t.flags & 1) unsafeAtomicAdd(p, -v); else *p -= v;
        }
    });
}

__global__ __launch_bounds__(kThreads) void k_rf1a(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                   const double* __restrict__ Zb, const double* __restrict__ Lp,
                                                   double* __restrict__ Hb, const int64_t* __restrict__ cr2,
                                                   const int32_t* __restrict__ rel)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
#define SELINV_CALL(BN)                                                                         \
    if (BN >= 32 && (d.c & 1) == 0) rf1a_task<BN, BN >= 32>(L, t, d, Zb, Lp, Hb, cr2, rel); \
    else rf1a_task<BN, false>(L, t, d, Zb, Lp, Hb, cr2, rel)
    SELINV_BN_DISPATCH(t.bn, SELINV_CALL)
#undef SELINV_CALL
}

// Fbar(C,B) = Ubar^T L_hat (+ Lhat_bar T on piece 0), Ubar^T(i,k) = -Fbar(C[k],C[i]) for k >= i
template <int BN, bool kPair>
__device__ void rf1b_task(GemmLds& L, const Task t, const BlockDesc d, double* __restrict__ Zb,
                          const double* __restrict__ Hp, const double* __restrict__ Hb, const double* __restrict__ Tp,
                          const int64_t* __restrict__ cr2,
                          const int32_t* __restrict__ rel)
{
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int r0 = t.i0, n0 = t.j0;
    d4 acc[2][4] = {};
    // -Ubar^T L_hat: Fbar(C[k],C[i]) for k >= i, gathered from the adjoint panels
    gather_mma<BN, kPair, 2>(L, d, r0, n0, t.kb, t.ke, Zb, Hp + d.hoff, c, cr2, rel, acc);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = -acc[mt][nt];
    if (t.flags & 2) {
        auto loadA2 = [&](int k0, int kk, int ii) -> double {
            const int i = r0 + ii, k = k0 + kk;
            return (i < c && k < s) ? Hb[d.hoff + i + (int64_t)k * c] : 0.0;
        };
        auto loadB2 = [&](int k0, int kk, int j) -> double {
            const int k = k0 + kk, jj = n0 + j;
            return (k < s && jj < s) ? Tp[d.woff + k + (int64_t)jj * s] : 0.0;
        };
        tile_mma<BN>(reinterpret_cast<TileLds&>(L), 0, s, acc, loadA2, loadB2, [](int) { return false; });
    }
    tile_epilogue_t<BN>(acc, [&](int i, int j, double v) {
        const int ii = r0 + i, jj = n0 + j;
        if (ii < c && jj < s) {
            double* p = Zb + d.poff + s + ii + (int64_t)jj * ld;
            if (t.flags & 1) unsafeAtomicAdd(p, v); else *p = v;
        }
    });
}

__global__ __launch_bounds__(kThreads) void k_rf1b(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                   double* __restrict__ Zb, const double* __restrict__ Hp,
                                                   const double* __restrict__ Hb, const double* __restrict__ Tp,
                                                   const int64_t* __restrict__ cr2,
                                                   const int32_t* __restrict__ rel)
{
    __shared__ GemmLds L;
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
#define SELINV_CALL(BN)                                                                             \
    if (BN >= 32 && (d.c & 1) == 0) rf1b_task<BN, BN >= 32>(L, t, d, Zb, Hp, Hb, Tp, cr2, rel); \
    else rf1b_task<BN, false>(L, t, d, Zb, Hp, Hb, Tp, cr2, rel)
    SELINV_BN_DISPATCH(t.bn, SELINV_CALL)
#undef SELINV_CALL
}

// Tbar(I,J) += F(C,B)^T Lhat_bar over rows [kb, ke) of C, one 32 x 32 tile
__global__ __launch_bounds__(kThreads) void k_rf2(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                  const double* __restrict__ Lp, const double* __restrict__ Hb,
                                                  double* __restrict__ Tb)
{
    __shared__ double FI[16][SDT + 1], HJ[16][SDT + 1];
    const Task t = tasks[blockIdx.x];
    const BlockDesc d = blk[t.b];
    const int s = d.s, c = d.c;
    const int64_t ld = (int64_t)s + c;
    const int I0 = t.i0, J0 = t.j0;
    const double* F = Lp + d.poff + s;
    const double* H = Hb + d.hoff;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int fm = (wave & 1) * 16, fn = (wave >> 1) * 16;
    d4 acc = {0, 0, 0, 0};
    const int rend = min(c, t.ke);
    for (int r0 = t.kb; r0 < rend; r0 += 16) {
#pragma unroll
        for (int q = 0; q < (16 * SDT) / kThreads; ++q) {
            const int e = threadIdx.x + q * kThreads;
            const int kk = e & 15, col = e >> 4;
            const int r = r0 + kk;
            const bool okr = r < rend;
            const int ci = I0 + col, cj = J0 + col;
            const double f = (okr && ci < s) ? F[r + (int64_t)ci * ld] : 0.0;
            const double h = (okr && cj < s) ? H[r + (int64_t)cj * c] : 0.0;
            FI[kk][col] = f;
            HJ[kk][col] = h;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            acc = mfma(FI[kr][fm + (lane & 15)], HJ[kr][fn + (lane & 15)], acc);
        }
        __syncthreads();
    }
    mfma_drain();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int gi = I0 + fm + (lane >> 4) + 4 * v, gj = J0 + fn + (lane & 15);
        if (gi < s && gj < s) {
            double* p = Tb + d.woff + gi + (int64_t)gj * s;
            if (t.flags & 1) unsafeAtomicAdd(p, acc[v]); else *p += acc[v];
        }
    }
}

// Fbar(B,B) stored lower = -T (Tbar + Tbar^T) T with the diagonal halved; one
// work-group per block, Q = (Tbar + Tbar^T) T held in LDS (s <= 128).
__global__ __launch_bounds__(kThreads) void k_rf3(const Task* __restrict__ tasks, const BlockDesc* __restrict__ blk,
                                                  const double* __restrict__ Tp, const double* __restrict__ Tb,
                                                  double* __restrict__ Zb)
{
    extern __shared__ double Q[];
    const BlockDesc d = blk[tasks[blockIdx.x].b];
    const int s = d.s;
    const int64_t ld = (int64_t)d.s + d.c;
    const int ls = s + 1;
    const double* T = Tp + d.woff;
    const double* Tbar = Tb + d.woff;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nt = (s + 15) / 16;
    for (int p = wave; p < nt * nt; p += kThreads / 64) {
        const int i0 = (p / nt) * 16, j0 = (p % nt) * 16;
        d4 acc = {0, 0, 0, 0};
        for (int k4 = 0; k4 < s; k4 += 4) {
            const int k = k4 + (lane >> 4), i = i0 + (lane & 15), j = j0 + (lane & 15);
            const double a = (i < s && k < s) ? Tbar[i + (int64_t)k * s] + Tbar[k + (int64_t)i * s] : 0.0;
            const double b = (k < s && j < s) ? T[k + (int64_t)j * s] : 0.0;
            acc = mfma(a, b, acc);
        }
        mfma_drain();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ii = i0 + (lane >> 4) + 4 * v, jj = j0 + (lane & 15);
            if (ii < s && jj < s) Q[ii * ls + jj] = acc[v];
        }
    }
    __syncthreads();
    for (int p = wave; p < nt * (nt + 1) / 2; p += kThreads / 64) {
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= p) ++I;
        const int J = p - I * (I + 1) / 2;
        const int i0 = I * 16, j0 = J * 16;
        d4 acc = {0, 0, 0, 0};
        for (int k4 = 0; k4 < s; k4 += 4) {
            const int k = k4 + (lane >> 4), i = i0 + (lane & 15), j = j0 + (lane & 15);
            const double a = (i < s && k < s) ? T[i + (int64_t)k * s] : 0.0;
            const double b = (k < s && j < s) ? Q[k * ls + j] : 0.0;
            acc = mfma(a, b, acc);
        }
        mfma_drain();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ii = i0 + (lane >> 4) + 4 * v, jj = j0 + (lane & 15);
            if (ii < s && jj < s && ii >= jj) Zb[d.poff + ii + (int64_t)jj * ld] = ii == jj ? -0.5 * acc[v] : -acc[v];
        }
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipEvent_t Prof::next()
{
    if (used == pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        pool.push_back(e);
    }
    return pool[used++];
}

Prof::~Prof()
{
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

template <class Kern, class... Args>
static void launch(Prof* P, int kind, Kern kern, dim3 grid, size_t shmem, hipStream_t s, Args... args)
{
    if (P && P->on) {
        hipEvent_t a = P->next(), z = P->next();
        if (a && z) {
            hipExtLaunchKernelGGL(kern, grid, dim3(kThreads), (uint32_t)shmem, s, a, z, 0, args...);
            P->kinds.push_back(kind);
            return;
        }
    }
    hipLaunchKernelGGL(kern, grid, dim3(kThreads), shmem, s, args...);
}

static inline unsigned grid_for(int64_t n)
{
    int64_t g = (n + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t kernels_init()
{
    // the reverse diagonal step needs more than the default 64 KB of LDS;
    // set once per process (a failure is not remembered: the next call tries again)
    static std::atomic<bool> done{false};
    if (done.load()) return hipSuccess;
    const hipError_t e =
        hipFuncSetAttribute((const void*)k_rf3, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsDiagBytes);
    if (e == hipSuccess) done.store(true);
    return e;
}

hipError_t launch_backward_init(Prof* P, const DevPtrs& D, int64_t arena, int64_t harena, const double* gsel,
                                int64_t nnzL, hipStream_t s)
{
    hipError_t e = launch_fill(P, kRevSel, D.Zb, arena, 0.0, s);
    if (!e) e = launch_fill(P, kRevSel, D.Hb, harena, 0.0, s);
    if (!e) e = launch_scatter_set(P, kRevSel, gsel, D.exp_off, nnzL, D.Zb, s);
    return e;
}

hipError_t launch_revsel_level(Prof* P, const DevPtrs& D, int64_t a0, int64_t na, int64_t b0, int64_t nb,
                               const int64_t* rs3_cuts, int ncuts, hipStream_t s)
{
    if (na > 0) launch(P, kRevSel, k_rs1, dim3((unsigned)na), 0, s, D.t_rs1 + a0, D.blocks, D.Zb, (const double*)D.Hp);
    if (nb > 0)
        launch(P, kRevSel, k_rs2, dim3((unsigned)nb), 0, s, D.t_rs2 + b0, D.blocks, (const double*)D.Ap,
               (const double*)D.Zb, D.Hb, D.cr2, D.rel);
    for (int g = 0; g + 1 < ncuts; g++) {
        const int64_t n = rs3_cuts[g + 1] - rs3_cuts[g];
        if (n > 0)
            launch(P, kRevSel, k_rs3, dim3((unsigned)n), 0, s, D.t_rs3 + rs3_cuts[g], D.blocks, D.Zb,
                   (const double*)D.Hp, D.cbase, D.rbase, D.rel);
    }
    return hipGetLastError();
}

hipError_t launch_revfac_init(Prof* P, const DevPtrs& D, int64_t nblocks, int64_t arena, hipStream_t s)
{
    if (nblocks > 0)
        launch(P, kRevFac, k_tbar_init, dim3((unsigned)nblocks), 0, s, D.t_diag, D.blocks, (const double*)D.Zb, D.Tb);
    return launch_fill(P, kRevFac, D.Zb, arena, 0.0, s);
}

hipError_t launch_revfac_level(Prof* P, const DevPtrs& D, int64_t a0, int64_t na, int64_t b0, int64_t nb, int64_t c0,
                               int64_t nc, int64_t d0, int64_t nd, hipStream_t s)
{
    if (na > 0)
        launch(P, kRevFac, k_rf1a, dim3((unsigned)na), 0, s, D.t_rf1a + a0, D.blocks, (const double*)D.Zb,
               (const double*)D.Lp, D.Hb, D.cr2, D.rel);
    if (nb > 0)
        launch(P, kRevFac, k_rf1b, dim3((unsigned)nb), 0, s, D.t_rf1b + b0, D.blocks, D.Zb, (const double*)D.Hp,
               (const double*)D.Hb, (const double*)D.Tp, D.cr2, D.rel);
    if (nc > 0)
        launch(P, kRevFac, k_rf2, dim3((unsigned)nc), 0, s, D.t_rf2 + c0, D.blocks, (const double*)D.Lp,
               (const double*)D.Hb, D.Tb);
    if (nd > 0)
        launch(P, kRevFac, k_rf3, dim3((unsigned)nd), kLdsDiagBytes, s, D.t_diag + d0, D.blocks, (const double*)D.Tp,
               (const double*)D.Tb, D.Zb);
    return hipGetLastError();
}

hipError_t launch_status_reset(unsigned long long* status, hipStream_t s)
{
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, s, status);
    return hipGetLastError();
}

hipError_t launch_fill(Prof* P, int kind, double* p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    launch(P, kind, k_fill, dim3(grid_for(n)), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_scatter_set(Prof* P, int kind, const double* src, const int64_t* off, int64_t n, double* dst,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    launch(P, kind, k_scatter_set, dim3(grid_for(n)), 0, s, src, off, n, dst);
    return hipGetLastError();
}

hipError_t launch_gather(Prof* P, int kind, const double* src, const int64_t* off, int64_t n, double* dst,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    launch(P, kind, k_gather, dim3(grid_for(n)), 0, s, src, off, n, dst);
    return hipGetLastError();
}

hipError_t launch_zero_x(Prof* P, const DevPtrs& D, int64_t t0, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    launch(P, kGemm, k_zero_x, dim3((unsigned)n), 0, s, D.t_zero + t0, D.blocks, D.Ap, (const double*)D.Tp);
    return hipGetLastError();
}

hipError_t launch_checkpoint(Prof* P, const DevPtrs& D, int64_t ntasks, int dir, hipStream_t s)
{
    if (ntasks <= 0) return hipSuccess;
    launch(P, kCheckpoint, k_ck_copy, dim3((unsigned)ntasks), 0, s, D.t_diag, D.blocks, D.ck_off, D.Ap, D.ck, dir);
    return hipGetLastError();
}

hipError_t launch_export_L(Prof* P, const DevPtrs& D, int64_t n, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    launch(P, kExport, k_export_L, dim3(grid_for(n)), 0, s, D.blocks, D.colblk, D.colptrL, D.exp_off, n,
           (const double*)D.Lp, (const double*)D.Hp, out);
    return hipGetLastError();
}

hipError_t launch_sb_factor(Prof* P, const DevPtrs& D, int64_t sb0, int64_t nsb, int require_spd, hipStream_t s)
{
    if (nsb > 0)
        launch(P, kSbFactor, k_sb_factor, dim3((unsigned)nsb), 0, s, D.t_sb + sb0, D.blocks, D.Lp, D.Hp, D.Tp, D.cbase,
               D.rbase, D.rel, D.status, require_spd);
    return hipGetLastError();
}

hipError_t launch_sb_invert(Prof* P, const DevPtrs& D, int64_t sb0, int64_t nsb, hipStream_t s)
{
    if (nsb > 0)
        launch(P, kSbInvert, k_sb_invert, dim3((unsigned)nsb), 0, s, D.t_sb + sb0, D.blocks, D.Ap, (const double*)D.Hp,
               (const double*)D.Tp, D.cbase, D.rbase, D.rel);
    return hipGetLastError();
}

hipError_t launch_ldlt_bk(Prof* P, const DevPtrs& D, const int64_t diag[4], hipStream_t s)
{
    // by width class: [diag[0], diag[1]) s <= 32, then <= 64, then <= 128
    if (diag[1] > diag[0])
        launch(P, kLdlt, k_ldlt_bk<2>, dim3((unsigned)(diag[1] - diag[0])), 0, s, D.t_ldlt + diag[0], D.blocks,
               (const double*)D.Lp, D.Tp, D.status);
    if (diag[2] > diag[1])
        launch(P, kLdlt, k_ldlt_bk<4>, dim3((unsigned)(diag[2] - diag[1])), 0, s, D.t_ldlt + diag[1], D.blocks,
               (const double*)D.Lp, D.Tp, D.status);
    if (diag[3] > diag[2])
        launch(P, kLdlt, k_ldlt_bk<8>, dim3((unsigned)(diag[3] - diag[2])), 0, s, D.t_ldlt + diag[2], D.blocks,
               (const double*)D.Lp, D.Tp, D.status);
    return hipGetLastError();
}

hipError_t launch_ldlt_level(Prof* P, const DevPtrs& D, const int64_t diag[4], int require_spd, hipStream_t s)
{
    // diagonal blocks by width class: [diag[0], diag[1]) s <= 32, then <= 64,
    // then wider
    if (diag[1] > diag[0])
        launch(P, kLdlt, k_ldlt_diag<2>, dim3((unsigned)(diag[1] - diag[0])), 0, s, D.t_ldlt + diag[0], D.blocks,
               D.Lp, D.Wp, D.Tp, D.status, require_spd);
    if (diag[2] > diag[1])
        launch(P, kLdlt, k_ldlt_diag<4>, dim3((unsigned)(diag[2] - diag[1])), 0, s, D.t_ldlt + diag[1], D.blocks,
               D.Lp, D.Wp, D.Tp, D.status, require_spd);
    if (diag[3] > diag[2])
        launch(P, kLdlt, k_ldlt_diag<8>, dim3((unsigned)(diag[3] - diag[2])), 0, s, D.t_ldlt + diag[2], D.blocks,
               D.Lp, D.Wp, D.Tp, D.status, require_spd);
    return hipGetLastError();
}

hipError_t launch_panel_level(Prof* P, const DevPtrs& D, int64_t panel0, int64_t npanel, int panel_deep, hipStream_t s)
{
    // panel_deep: bit 0 the level's panel tiles take the whole-contraction
    // kernel; bit 1 its blocks are narrow enough for it (s <= kDeepK)
    if (npanel > 0)
        launch(P, kPanel, (panel_deep & 1) ? k_panel_deep : k_panel, dim3((unsigned)npanel), 0, s,
               D.t_panel + panel0, D.blocks, (const double*)D.Lp, D.Hp, (const double*)D.Tp);
    return hipGetLastError();
}

hipError_t launch_schur_groups(Prof* P, const DevPtrs& D, const int64_t* cuts, int g0, int g1, int panel_deep,
                               hipStream_t s)
{
    // one launch per colour group (groups update disjoint entries)
    for (int g = g0; g < g1; g++) {
        const int64_t n = cuts[g + 1] - cuts[g];
        if (n > 0)
            launch(P, kSchur, (panel_deep & 2) && n <= kDeepMaxTiles ? k_schur_deep : k_schur, dim3((unsigned)n), 0, s,
                   D.t_schur + cuts[g], D.blocks, D.Lp, (const double*)D.Hp, D.cbase, D.rbase, D.rel);
    }
    return hipGetLastError();
}

hipError_t launch_invert_level(Prof* P, const DevPtrs& D, int64_t gemm0, int64_t ngemm, int64_t sdiag0,
                               int64_t sdiag_cut, int64_t sdiag1, hipStream_t s)
{
    if (ngemm > 0)
        launch(P, kGemm, k_gemm, dim3((unsigned)ngemm), 0, s, D.t_gemm + gemm0, D.blocks, D.Ap,
               (const double*)D.Hp, D.cr2, D.rel);
    if (sdiag_cut > sdiag0)
        launch(P, kSdiag, k_sdiag64, dim3((unsigned)(sdiag_cut - sdiag0)), 0, s, D.t_sdiag + sdiag0, D.blocks, D.Ap,
               (const double*)D.Hp, (const double*)D.Tp);
    if (sdiag1 > sdiag_cut)
        launch(P, kSdiag, k_sdiag64, dim3((unsigned)(sdiag1 - sdiag_cut)), 0, s, D.t_sdiag + sdiag_cut, D.blocks,
               D.Ap, (const double*)D.Hp, (const double*)D.Tp);
    return hipGetLastError();
}


// resident work-groups per CU of each persistent variant, in the order of
// selinv::PersistVariant
hipError_t persist_occupancy(int occ[kNumVariants])
{
    const void* k[kNumVariants] = {(const void*)k_light_factor,       (const void*)k_persist_factor<2>,
                                   (const void*)k_persist_factor<4>,  (const void*)k_persist_factor<8>,
                                   (const void*)k_light_invert,       (const void*)k_persist_invert<32>,
                                   (const void*)k_persist_invert<64>, (const void*)k_persist_invert<128>};
    hipError_t e = hipSuccess;
    for (int v = 0; v < kNumVariants && !e; v++) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(occ + v, k[v], kThreads, 0);
    return e;
}

hipError_t launch_fill_u32(Prof* P, int kind, unsigned* p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    launch(P, kind, k_fill_u32, dim3(grid_for(n)), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_persist_factor(Prof* P, const DevPtrs& D, const Task* q, int64_t ntasks, unsigned* head,
                                 unsigned* done, int grid, int variant, int require_spd, unsigned spin_limit,
                                 hipStream_t s)
{
    if (ntasks <= 0) return hipSuccess;
    const QueueArgs a{q, ntasks, head, done, D.status, require_spd, spin_limit};
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid, ntasks));
#define SELINV_PF(K) launch(P, kQFactor, K, dim3(g), 0, s, a, D.blocks, D.Lp, D.Wp, D.Hp, D.Tp, D.cbase, D.rbase, D.rel)
    switch (variant) {
        case kLightFactor:
            launch(P, kQFactor, k_light_factor, dim3(g), 0, s, a, D.blocks, D.Lp, D.Hp, D.Tp, D.cbase, D.rbase, D.rel);
            break;
        case kFactor32: SELINV_PF(k_persist_factor<2>); break;
        case kFactor64: SELINV_PF(k_persist_factor<4>); break;
        default: SELINV_PF(k_persist_factor<8>); break;
    }
#undef SELINV_PF
    return hipGetLastError();
}

hipError_t launch_persist_invert(Prof* P, const DevPtrs& D, const Task* q, int64_t ntasks, unsigned* head,
                                 unsigned* done, int grid, int variant, unsigned spin_limit, hipStream_t s)
{
    if (ntasks <= 0) return hipSuccess;
    const QueueArgs a{q, ntasks, head, done, D.status, 0, spin_limit};
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(grid, ntasks));
#define SELINV_PI(K)                                                                                              \
    launch(P, kQInvert, K, dim3(g), 0, s, a, D.blocks, D.Ap, (const double*)D.Hp, (const double*)D.Tp, D.cbase, \
           D.rbase, D.rel, D.cr2)
    switch (variant) {
        case kLightInvert: SELINV_PI(k_light_invert); break;
        case kInvert32: SELINV_PI(k_persist_invert<32>); break;
        case kInvert64: SELINV_PI(k_persist_invert<64>); break;
        default: SELINV_PI(k_persist_invert<128>); break;
    }
#undef SELINV_PI
    return hipGetLastError();
}

}  // namespace selinv
