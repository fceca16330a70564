// Principal-shared contraction on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
//   Y[:, c] (+)= sum_g scale_g sum_k coef_g[cell(c), k] * A_{g,k} X_g[:, c]
//
// Every cell (column c; cell = c mod ncells) combines the same few principal
// operators A_{g,k} with its own coefficients (paper Remark 7: the ROM
// operators of eqs. (48), (49), Algorithm 3 and eq. (46a) as sums over the
// principal cells), so all cells become one dense contraction.
//
// Kernels (each principal operator is copied once into MFMA-fragment order, so
// a wave reads one coalesced 16-byte unit per lane per MFMA group):
//  * pc64_tile — operators resident in L2 (the dual/primal blocks of the
//    bank): NW waves share one output tile, split the (principal, inner step)
//    sequence round-robin and sum their partial tiles through LDS by a fixed
//    pairwise tree;
//  * k_pc64_big — tall operators (the stacked local inverses of eq. (46a)):
//    waves own distinct row tiles and run the whole sequence;
//  * k_pclp_tile / k_pclp_big — the same two shapes for the precision form
//    (FP32 16x16x4 or BF16 16x16x32 MFMAs, FP32 accumulation).
// The cell vectors of a tile's columns are staged in LDS (plain columns, or
// gathered from the interface multipliers through the jump codes) and scaled
// by the cell's coefficient of the current principal as they are fed.
// The 16x16 f64 MFMA returns D with lane l, register i -> row 4*i + l/16,
// column l % 16; the f32 / bf16 ones row 4*(l/16) + i (checked on gfx950).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include <hip/hip_ext.h>

#include <rocblas/rocblas.h>

#include "common.hpp"

namespace ifeti {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

struct GemmArgsDev {
    const double *A[2];
    const double *X[2];
    const double *coef[2];
    int Kd[2], ldx[2], K[2];
    long long xbs[2];
    double scale[2];
    int ngroups;
    double *Y;
    long long ybs;
    int ldy, M, ncols, ncells, accumulate;
};


typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- fragment-ordered FP64 path
// For operators that stay resident in L2 (the dual/primal blocks of the
// principal bank), A_k is copied once into MFMA-fragment order: for row tile
// mt (16 rows) and pair q of 4-deep k-steps, lane l holds rows mt*16 + l%16
// and inner indices (2q + j)*4 + l/16, j = 0, 1, as one 16-byte pair, so a
// coalesced 1 KB wave load feeds two MFMAs.
__global__ void k_to_frag(const double *__restrict__ A, int M, int Kd, int K, int MT, int KT2,
                          double *__restrict__ F) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)K * MT * KT2 * 128;
    if (t >= total) return;
    const int j = (int)(t & 1), lane = (int)((t >> 1) & 63);
    long long rest = t >> 7;
    const int q = (int)(rest % KT2);
    rest /= KT2;
    const int mt = (int)(rest % MT), k = (int)(rest / MT);
    const int row = mt * 16 + (lane & 15), inner = (2 * q + j) * 4 + (lane >> 4);
    F[t] = (row < M && inner < Kd) ? A[(size_t)k * M * Kd + (size_t)row * Kd + inner] : 0.0;
}

struct GemmArgsFrag {
    const double *Af[2];
    const double *X[2];
    const double *coef[2];
    const int *gcodes[2];
    const double *gw[2];
    int Kd[2], ldx[2], K[2], KT2[2];
    long long xbs[2];
    double scale[2];
    int ngroups;
    double *Y;
    long long ybs;
    int ldy, M, MT, ncols, ncells, accumulate;
    int ksplit;    // >1: inner range split over blockIdx.z, partials to `part` ([z][col][M])
    double *part;
};

constexpr int FKC = 128;      // inner rows of the cell vectors staged per chunk
constexpr int FXS = FKC + 2;  // LDS row stride (doubles): conflict-free B-fragment reads
constexpr int kMaxCoefK = 40;

// Stages the cell vectors of columns [col0, col0 + NC), inner rows [kk, kk + kc) into
// Xs[col][row] (row stride XST), zero-padded to KC rows: plain strided columns, or the
// fused (weighted) jump transpose from the signed multiplier rows in `gcodes`.  Entries
// are taken in batches of up to SBMAX per thread with every load of a batch (codes, then
// multiplier rows and weights) issued before the first is consumed.
template <int NC, int KC, int NT, int XST, int SBMAX, typename G, typename XT>
__device__ __forceinline__ void stage_chunk(const G &g, const double *__restrict__ X,
                                            const int *__restrict__ gcodes, const double *__restrict__ gw, int Kd,
                                            int ldx, long long xbs, int col0, int kk, int kc, XT *__restrict__ Xs,
                                            int tid) {
    constexpr int PER = (NC * KC + NT - 1) / NT;
    constexpr int SB = PER < SBMAX ? PER : SBMAX;
#pragma unroll 1
    for (int i0 = 0; i0 < PER; i0 += SB) {
        int2 cd[SB];
        double v[SB];
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int e = tid + (i0 + i) * NT, cc = e / KC, r = e % KC, col = col0 + cc;
            cd[i] = int2{0, 0};
            v[i] = 0.0;
            if (e < NC * KC && col < g.ncols && r < kc) {
                const int cell = col % g.ncells;
                if (gcodes)
                    cd[i] = *reinterpret_cast<const int2 *>(gcodes + ((size_t)cell * Kd + kk + r) * 2);
                else
                    v[i] = X[(long long)(col / g.ncells) * xbs + (size_t)cell * ldx + kk + r];
            }
        }
        if (gcodes) {
            double x0[SB], x1[SB];
#pragma unroll
            for (int i = 0; i < SB; ++i) {
                const int col = col0 + (tid + (i0 + i) * NT) / KC;
                const double *lam = X + (long long)(col / g.ncells) * xbs;
                const int r0 = abs(cd[i].x) - 1, r1 = abs(cd[i].y) - 1;
                x0[i] = cd[i].x ? lam[r0] : 0.0;
                x1[i] = cd[i].y ? lam[r1] : 0.0;
                if (gw) {
                    x0[i] *= cd[i].x ? gw[r0] : 0.0;
                    x1[i] *= cd[i].y ? gw[r1] : 0.0;
                }
            }
#pragma unroll
            for (int i = 0; i < SB; ++i)
                v[i] = (cd[i].x >= 0 ? x0[i] : -x0[i]) + (cd[i].y >= 0 ? x1[i] : -x1[i]);
        }
#pragma unroll
        for (int i = 0; i < SB; ++i) {
            const int e = tid + (i0 + i) * NT;
            if (e < NC * KC) Xs[(e / KC) * XST + e % KC] = (XT)v[i];
        }
    }
}

// Workgroup = NW waves sharing one output tile of RT row tiles x CB column
// blocks (16 x 16 each).  The cell vectors of the tile's 16*CB columns and
// their coefficients are staged in LDS; the (principal, k-step pair) sequence
// is dealt round-robin to the NW waves, each streaming its A fragments from L2
// PF pairs ahead; partial tiles are summed through LDS by a fixed pairwise
// tree, so every column's result is independent of the launch shape and of
// the other columns (bitwise reproducible).
template <int RT, int CB, int NW>
struct Pc64Lds {
    static constexpr int NC = 16 * CB;
    static constexpr int XW = NC * FXS;
    static constexpr int RED = (NW / 2) * RT * CB * 256;
    static constexpr int SX = XW > RED ? XW : RED;
    static constexpr int SC = kMaxCoefK * NC;
};

template <int RT, int CB, int PF, int NW>
__device__ __forceinline__ void pc64_tile(const GemmArgsFrag &g, int bx, int by, double *__restrict__ Xs,
                                          double *__restrict__ Cs) {
    static_assert((NW & (NW - 1)) == 0, "NW must be a power of two");
    constexpr int NT = 64 * NW;
    constexpr int NC = 16 * CB;
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const int mt0 = by * RT, col0 = bx * NC;
    v4d acc[RT][CB];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = v4d{0.0, 0.0, 0.0, 0.0};

    for (int gi = 0; gi < g.ngroups; ++gi) {
        const double *__restrict__ Af = g.Af[gi];
        const double *__restrict__ X = g.X[gi];
        const double *__restrict__ coef = g.coef[gi];
        const int *__restrict__ gcodes = g.gcodes[gi];
        const double *__restrict__ gw = g.gw[gi];
        const int Kd = g.Kd[gi], K = g.K[gi], KT2 = g.KT2[gi], ldx = g.ldx[gi];
        const long long xbs = g.xbs[gi];
        const double scale = g.scale[gi];
        for (int kk = 0; kk < Kd; kk += FKC) {
            const int kc = min(FKC, Kd - kk);
            const int np = (kc + 7) / 8;  // fragment pairs of this chunk
            const int q0 = kk / 8;
            const int total = K * np;
            const int ns = wave < total ? (total - wave + NW - 1) / NW : 0;  // steps s = wave + NW i
            // fragment loads of step i (clamped to the last step: the ring is refilled unconditionally, so
            // the loop has no join points and each step waits only for the load issued PF steps earlier)
            auto load = [&](int i, double2 (&dst)[RT]) {
                const int s = wave + NW * min(i, ns - 1), k = s / np, q = s % np;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const int mt = min(mt0 + rt, g.MT - 1);  // rows beyond M: in-bounds, result dropped
                    dst[rt] = reinterpret_cast<const double2 *>(Af + (((size_t)k * g.MT + mt) * KT2 + q0 + q) * 128)[lane];
                }
            };
            __syncthreads();  // previous chunk fully consumed
            // the first operator fragments do not depend on the staged columns: their loads are in
            // flight while the columns and coefficients are staged
            // ring of PF + 1 fragment slots: step i reads slot i mod (PF + 1) while the load of step i + PF
            // goes to another slot, so no slot is copied or waited for early (the loop is unrolled by the
            // ring size and every slot is a fixed register set)
            constexpr int S = PF + 1;
            double2 ab[S][RT];
            if (ns > 0) {
#pragma unroll
                for (int u = 0; u < PF; ++u) load(u, ab[u]);
            }
            stage_chunk<NC, FKC, NT, FXS, 4>(g, X, gcodes, gw, Kd, ldx, xbs, col0, kk, kc, Xs, tid);
            for (int e = tid; e < K * NC; e += NT) {
                const int k = e / NC, cc = e % NC, col = col0 + cc;
                double v = 0.0;
                if (col < g.ncols) v = scale * (coef ? coef[(size_t)(col % g.ncells) * K + k] : 1.0);
                Cs[e] = v;
            }
            __syncthreads();
            if (ns == 0) continue;  // wave-uniform
            // B operands of step i: the staged rows of its fragment pair scaled by its principal's coefficient
            // of each column; steps padded to a multiple of the ring size repeat the last step with zero
            // operands, which leaves the accumulators unchanged
            auto bops = [&](int i, double (&bo)[2][CB]) {
                const double live = i < ns ? 1.0 : 0.0;
                const int s = wave + NW * min(i, ns - 1), k = s / np, q = s % np;
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const double cf = Cs[k * NC + cb * 16 + lr] * live;
#pragma unroll
                    for (int j = 0; j < 2; ++j) bo[j][cb] = Xs[(cb * 16 + lr) * FXS + 4 * (2 * q + j) + lk] * cf;
                }
            };
            // the B operands of the next step are read from LDS while this step's MFMAs run
            double bb[S][2][CB];
            bops(0, bb[0]);
            const int nsp = (ns + S - 1) / S * S;
            for (int i0 = 0; i0 < nsp; i0 += S) {
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    const int i = i0 + u;
                    load(i + PF, ab[(u + PF) % S]);
                    const double2 *a = ab[u];
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb)
                                acc[rt][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(j ? a[rt].y : a[rt].x, bb[u][j][cb],
                                                                                   acc[rt][cb], 0, 0, 0);
                    bops(i + 1, bb[(u + 1) % S]);
                }
            }
        }
    }
    // pairwise tree over the waves: wave w += wave w + h, h = NW/2, NW/4, ..., 1
#pragma unroll
    for (int h = NW / 2; h >= 1; h >>= 1) {
        __syncthreads();
        if (wave >= h && wave < 2 * h)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        Xs[(((wave - h) * RT + rt) * CB + cb) * 256 + i * 64 + lane] = acc[rt][cb][i];
        __syncthreads();
        if (wave < h)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[rt][cb][i] += Xs[((wave * RT + rt) * CB + cb) * 256 + i * 64 + lane];
    }
    if (wave != 0) return;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int mt = mt0 + rt, col = col0 + cb * 16 + lr;
            if (mt >= g.MT || col >= g.ncols) continue;
            double *ycol = g.Y + (long long)(col / g.ncells) * g.ybs + (size_t)(col % g.ncells) * g.ldy;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = mt * 16 + 4 * i + lk;
                if (row < g.M) ycol[row] = g.accumulate ? ycol[row] + acc[rt][cb][i] : acc[rt][cb][i];
            }
        }
}

template <int RT, int CB, int PF, int NW>
__global__ __launch_bounds__(64 * NW) void k_pc64(GemmArgsFrag g) {
    using L = Pc64Lds<RT, CB, NW>;
    __shared__ double Xs[L::SX];
    __shared__ double Cs[L::SC];
    pc64_tile<RT, CB, PF, NW>(g, blockIdx.x, blockIdx.y, Xs, Cs);
}


// Large-M variant (operators that do not stay in L2, e.g. the stacked local
// inverses of (46a)): the NW waves of a workgroup own distinct row tiles
// (RTW each) of one 16*CB-column block and all of them run the full
// (principal, k-step pair) sequence, with the column chunk (KCB inner rows)
// and coefficients shared through LDS; no cross-wave reduction.
template <int RTW, int CB, int NW, int KCB, int PF>
__global__ __launch_bounds__(64 * NW) void k_pc64_big(GemmArgsFrag g) {
    constexpr int NT = 64 * NW;
    constexpr int NC = 16 * CB;
    constexpr int XSB = KCB + 2;
    static_assert(KCB % 8 == 0, "chunk must hold whole fragment pairs");
    __shared__ double Xs[NC * XSB];
    __shared__ double Cs[kMaxCoefK * NC];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const int mt0 = (blockIdx.y * NW + wave) * RTW, col0 = blockIdx.x * NC;
    v4d acc[RTW][CB];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = v4d{0.0, 0.0, 0.0, 0.0};
    bool rtv[RTW];
    bool any = false;
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt) {
        rtv[rt] = mt0 + rt < g.MT;
        any = any || rtv[rt];
    }
    for (int gi = 0; gi < g.ngroups; ++gi) {
        const double *__restrict__ Af = g.Af[gi];
        const double *__restrict__ X = g.X[gi];
        const double *__restrict__ coef = g.coef[gi];
        const int *__restrict__ gcodes = g.gcodes[gi];
        const double *__restrict__ gw = g.gw[gi];
        const int Kd = g.Kd[gi], K = g.K[gi], KT2 = g.KT2[gi], ldx = g.ldx[gi];
        const long long xbs = g.xbs[gi];
        const double scale = g.scale[gi];
        // inner range of this split (whole chunks), all of it when ksplit = 1
        const int nsplit = g.ksplit > 1 ? g.ksplit : 1;
        const int per = ((Kd + KCB * nsplit - 1) / (KCB * nsplit)) * KCB;
        const int kbeg = blockIdx.z * per, kend = min(Kd, kbeg + per);
        for (int kk = kbeg; kk < kend; kk += KCB) {
            const int kc = min(KCB, kend - kk);
            __syncthreads();
            // one entry at a time: the chunk loop repeats often and occupancy hides the latency
            stage_chunk<NC, KCB, NT, XSB, 1>(g, X, gcodes, gw, Kd, ldx, xbs, col0, kk, kc, Xs, tid);
            for (int e = tid; e < K * NC; e += NT) {
                const int k = e / NC, cc = e % NC, col = col0 + cc;
                double v = 0.0;
                if (col < g.ncols) v = scale * (coef ? coef[(size_t)(col % g.ncells) * K + k] : 1.0);
                Cs[e] = v;
            }
            __syncthreads();
            if (!any) continue;  // wave-uniform: this wave's row tiles lie beyond M
            const int np = (kc + 7) / 8, q0 = kk / 8, ns = K * np;
            // fragment loads of step s clamped to the last step, rows beyond M clamped to the last row
            // tile (in bounds; their results are dropped): the ring is refilled unconditionally and the
            // loop has no join points, so each step waits only for the load issued PF steps earlier
            auto load = [&](int s, double2 (&dst)[RTW]) {
                const int sc = min(s, ns - 1), k = sc / np, q = sc % np;
#pragma unroll
                for (int rt = 0; rt < RTW; ++rt) {
                    const int mt = min(mt0 + rt, g.MT - 1);
                    dst[rt] = reinterpret_cast<const double2 *>(Af + (((size_t)k * g.MT + mt) * KT2 + q0 + q) * 128)[lane];
                }
            };
            constexpr int S = PF + 1;  // ring of fragment slots (see pc64_tile)
            double2 ab[S][RTW];
#pragma unroll
            for (int u = 0; u < PF; ++u) load(u, ab[u]);
            const int nsp = (ns + S - 1) / S * S;  // padded steps carry a zero coefficient
            for (int s0 = 0; s0 < nsp; s0 += S) {
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    const int s = s0 + u;
                    load(s + PF, ab[(u + PF) % S]);
                    const double2 *a = ab[u];
                    const bool live = s < ns;
                    const int sc = min(s, ns - 1), k = sc / np, q = sc % np;
                    double cf[CB];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) cf[cb] = live ? Cs[k * NC + cb * 16 + lr] : 0.0;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int r = 4 * (2 * q + j) + lk;
                        double b[CB];
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) b[cb] = Xs[(cb * 16 + lr) * XSB + r] * cf[cb];
#pragma unroll
                        for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb)
                                acc[rt][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(j ? a[rt].y : a[rt].x, b[cb],
                                                                                   acc[rt][cb], 0, 0, 0);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int mt = mt0 + rt, col = col0 + cb * 16 + lr;
            if (mt >= g.MT || col >= g.ncols) continue;
            if (g.part) {
                double *pcol = g.part + ((size_t)blockIdx.z * g.ncols + col) * g.M;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = mt * 16 + 4 * i + lk;
                    if (row < g.M) pcol[row] = acc[rt][cb][i];
                }
                continue;
            }
            double *ycol = g.Y + (long long)(col / g.ncells) * g.ybs + (size_t)(col % g.ncells) * g.ldy;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = mt * 16 + 4 * i + lk;
                if (row < g.M) ycol[row] = g.accumulate ? ycol[row] + acc[rt][cb][i] : acc[rt][cb][i];
            }
        }
}

// sum of the split-K partials in split order, into Y
__global__ __launch_bounds__(256) void k_split_reduce(const double *__restrict__ part, int ksplit, int ncols, int M,
                                                      int ncells, double *__restrict__ Y, long long ybs, int ldy,
                                                      int accumulate) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)ncols * M) return;
    const int col = (int)(t / M), row = (int)(t % M);
    double v = part[t];
    for (int z = 1; z < ksplit; ++z) v += part[(size_t)z * ncols * M + t];
    double *y = Y + (long long)(col / ncells) * ybs + (size_t)(col % ncells) * ldy + row;
    *y = accumulate ? *y + v : v;
}

// ---------------------------------------------------------------- precision form, large M
// FP32 / BF16 counterpart of k_pc64_big.  The operator is copied once into
// 16-byte fragment units: FP32 — lane l holds rows mt*16 + l%16 and inner
// indices (4u + j)*4 + l/16, j = 0..3 (four 16x16x4 MFMAs); BF16 — inner
// indices 32u + 8(l/16) + e, e = 0..7 (one 16x16x32 MFMA).  Cell vectors are
// staged in LDS as FP32 and scaled by the coefficients as they are fed;
// accumulation in FP32, result written in FP64.
template <typename T>
struct LpUnit;
template <>
struct LpUnit<float> {
    static constexpr int KPF = 16, U = 4;
};
template <>
struct LpUnit<__bf16> {
    static constexpr int KPF = 32, U = 8;
};

template <typename T>
__global__ void k_to_frag_lp(const double *__restrict__ A, int M, int Kd, int K, int MT, int QU, T *__restrict__ F) {
    constexpr int U = LpUnit<T>::U;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)K * MT * QU * 64 * U;
    if (t >= total) return;
    const int u = (int)(t % U), lane = (int)((t / U) % 64);
    long long rest = t / (U * 64);
    const int qu = (int)(rest % QU);
    rest /= QU;
    const int mt = (int)(rest % MT), k = (int)(rest / MT);
    const int row = mt * 16 + (lane & 15);
    const int inner = U == 4 ? (4 * qu + u) * 4 + (lane >> 4) : 32 * qu + 8 * (lane >> 4) + u;
    F[t] = (row < M && inner < Kd) ? (T)(float)A[(size_t)k * M * Kd + (size_t)row * Kd + inner] : (T)0.f;
}

struct GemmArgsFragLP {
    int ksplit;    // inner-range splits over blockIdx.z (0/1: none)
    const void *Af[2];
    const double *X[2];
    const double *coef[2];
    const int *gcodes[2];
    const double *gw[2];
    int Kd[2], ldx[2], K[2], QU[2];
    long long xbs[2];
    double scale[2];
    int ngroups;
    double *Y;
    long long ybs;
    int ldy, M, MT, ncols, ncells, accumulate;
};

template <typename T, int RTW, int CB, int NW, int KCB>
__global__ __launch_bounds__(64 * NW) void k_pclp_big(GemmArgsFragLP g) {
    constexpr bool BF = sizeof(T) == 2;
    constexpr int KPF = LpUnit<T>::KPF, U = LpUnit<T>::U;
    constexpr int NT = 64 * NW, NC = 16 * CB, XS = KCB + 4, PF = 2;
    static_assert(KCB % KPF == 0, "chunk must hold whole fragment units");
    __shared__ __attribute__((aligned(16))) float Xs[NC * XS];
    __shared__ float Cs[kMaxCoefK * NC];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const int mt0 = (blockIdx.y * NW + wave) * RTW, col0 = blockIdx.x * NC;
    v4f acc[RTW][CB];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = v4f{0.f, 0.f, 0.f, 0.f};
    bool rtv[RTW];
    bool any = false;
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt) {
        rtv[rt] = mt0 + rt < g.MT;
        any = any || rtv[rt];
    }
    for (int gi = 0; gi < g.ngroups; ++gi) {
        const T *__restrict__ Af = reinterpret_cast<const T *>(g.Af[gi]);
        const double *__restrict__ X = g.X[gi];
        const double *__restrict__ coef = g.coef[gi];
        const int *__restrict__ gcodes = g.gcodes[gi];
        const double *__restrict__ gw = g.gw[gi];
        const int Kd = g.Kd[gi], K = g.K[gi], QU = g.QU[gi], ldx = g.ldx[gi];
        const long long xbs = g.xbs[gi];
        const double scale = g.scale[gi];
        // inner range of this split (whole chunks), all of it when ksplit = 1
        const int nsplit = g.ksplit > 1 ? g.ksplit : 1;
        const int per = ((Kd + KCB * nsplit - 1) / (KCB * nsplit)) * KCB;
        const int kbeg = blockIdx.z * per, kend = min(Kd, kbeg + per);
        for (int kk = kbeg; kk < kend; kk += KCB) {
            const int kc = min(KCB, kend - kk);
            __syncthreads();
            for (int e = tid; e < NC * KCB; e += NT) {
                const int cc = e / KCB, r = e % KCB, col = col0 + cc;
                double v = 0.0;
                if (col < g.ncols && r < kc) {
                    const int cell = col % g.ncells;
                    const long long rhs = col / g.ncells;
                    if (gcodes) {
                        const double *lam = X + rhs * xbs;
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            const int code = gcodes[((size_t)cell * Kd + kk + r) * 2 + u];
                            if (code == 0) continue;
                            const int row = (code > 0 ? code : -code) - 1;
                            const double x = gw ? lam[row] * gw[row] : lam[row];
                            v += code > 0 ? x : -x;
                        }
                    } else {
                        v = X[rhs * xbs + (size_t)cell * ldx + kk + r];
                    }
                }
                Xs[cc * XS + r] = (float)v;
            }
            for (int e = tid; e < K * NC; e += NT) {
                const int k = e / NC, cc = e % NC, col = col0 + cc;
                double v = 0.0;
                if (col < g.ncols) v = scale * (coef ? coef[(size_t)(col % g.ncells) * K + k] : 1.0);
                Cs[e] = (float)v;
            }
            __syncthreads();
            if (!any) continue;
            const int np = (kc + KPF - 1) / KPF, q0 = kk / KPF, ns = K * np;
            // ring of PF + 1 fragment slots with clamped loads and zero-operand padding, as in pc64_tile
            auto load = [&](int s, uint4 (&dst)[RTW]) {
                const int sc = min(s, ns - 1), k = sc / np, q = sc % np;
#pragma unroll
                for (int rt = 0; rt < RTW; ++rt) {
                    const int mt = min(mt0 + rt, g.MT - 1);
                    dst[rt] = reinterpret_cast<const uint4 *>(Af + ((((size_t)k * g.MT + mt) * QU + q0 + q) * 64 + lane) * U)[0];
                }
            };
            constexpr int S = PF + 1;
            uint4 ab[S][RTW];
#pragma unroll
            for (int u = 0; u < PF; ++u) load(u, ab[u]);
            const int nsp = (ns + S - 1) / S * S;
            for (int s0 = 0; s0 < nsp; s0 += S) {
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    const int s = s0 + u;
                    load(s + PF, ab[(u + PF) % S]);
                    const uint4 *a = ab[u];
                    const float live = s < ns ? 1.f : 0.f;
                    const int sc = min(s, ns - 1), k = sc / np, q = sc % np;
                    float cf[CB];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) cf[cb] = Cs[k * NC + cb * 16 + lr] * live;
                    if constexpr (BF) {
                        v8bf b[CB];
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) {
                            const float *xr = Xs + (cb * 16 + lr) * XS + q * KPF + 8 * lk;
#pragma unroll
                            for (int e = 0; e < 8; ++e) b[cb][e] = (__bf16)(xr[e] * cf[cb]);
                        }
#pragma unroll
                        for (int rt = 0; rt < RTW; ++rt) {
                            const v8bf av = __builtin_bit_cast(v8bf, a[rt]);
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb)
                                acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[cb], acc[rt][cb], 0, 0, 0);
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int r = q * KPF + 4 * j + lk;
                            float b[CB];
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb) b[cb] = Xs[(cb * 16 + lr) * XS + r] * cf[cb];
#pragma unroll
                            for (int rt = 0; rt < RTW; ++rt) {
                                const uint32_t aw = j == 0 ? a[rt].x : j == 1 ? a[rt].y : j == 2 ? a[rt].z : a[rt].w;
                                const float av = __builtin_bit_cast(float, aw);
#pragma unroll
                                for (int cb = 0; cb < CB; ++cb)
                                    acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b[cb], acc[rt][cb], 0, 0, 0);
                            }
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int mt = mt0 + rt, col = col0 + cb * 16 + lr;
            if (mt >= g.MT || col >= g.ncols) continue;
            double *ycol = g.Y + (long long)(col / g.ncells) * g.ybs + (size_t)(col % g.ncells) * g.ldy;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = mt * 16 + 4 * lk + i;
                if (row < g.M) ycol[row] = g.accumulate ? ycol[row] + (double)acc[rt][cb][i] : (double)acc[rt][cb][i];
            }
        }
}

// ---------------------------------------------------------------- precision form, small M
// FP32 / BF16 counterpart of pc64_tile for operators that stay in L2: NW waves
// share one output tile of RT row tiles x CB column blocks; the cell vectors of
// the tile's columns are staged in LDS as FP32 (gathered from the multipliers
// when jump codes are given) and the (principal, fragment unit) sequence is
// dealt round-robin to the waves; partial tiles are summed in FP32 by a fixed
// pairwise tree, so each column's result does not depend on the launch shape.
constexpr int LKC = 128;      // inner rows staged per chunk
constexpr int LXS = LKC + 4;  // LDS row stride (floats)

template <int RT, int CB, int NW>
struct PclpLds {
    static constexpr int NC = 16 * CB;
    static constexpr int XW = NC * LXS;
    static constexpr int RED = (NW / 2) * RT * CB * 256;
    static constexpr int SX = XW > RED ? XW : RED;
};

template <typename T, int RT, int CB, int NW>
__global__ __launch_bounds__(64 * NW) void k_pclp_tile(GemmArgsFragLP g) {
    static_assert((NW & (NW - 1)) == 0, "NW must be a power of two");
    constexpr bool BF = sizeof(T) == 2;
    constexpr int KPF = LpUnit<T>::KPF, U = LpUnit<T>::U, PF = 2;
    constexpr int NT = 64 * NW, NC = 16 * CB;
    using L = PclpLds<RT, CB, NW>;
    __shared__ __attribute__((aligned(16))) float Xs[L::SX];
    __shared__ float Cs[kMaxCoefK * NC];
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lk = lane >> 4;
    const int mt0 = blockIdx.y * RT, col0 = blockIdx.x * NC;
    v4f acc[RT][CB];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rt][cb] = v4f{0.f, 0.f, 0.f, 0.f};
    bool rtv[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) rtv[rt] = mt0 + rt < g.MT;

    for (int gi = 0; gi < g.ngroups; ++gi) {
        const T *__restrict__ Af = reinterpret_cast<const T *>(g.Af[gi]);
        const double *__restrict__ X = g.X[gi];
        const double *__restrict__ coef = g.coef[gi];
        const int *__restrict__ gcodes = g.gcodes[gi];
        const double *__restrict__ gw = g.gw[gi];
        const int Kd = g.Kd[gi], K = g.K[gi], QU = g.QU[gi], ldx = g.ldx[gi];
        const long long xbs = g.xbs[gi];
        const double scale = g.scale[gi];
        for (int kk = 0; kk < Kd; kk += LKC) {
            const int kc = min(LKC, Kd - kk);
            __syncthreads();  // previous chunk fully consumed
            stage_chunk<NC, LKC, NT, LXS, 4>(g, X, gcodes, gw, Kd, ldx, xbs, col0, kk, kc, Xs, tid);
            for (int e = tid; e < K * NC; e += NT) {
                const int k = e / NC, cc = e % NC, col = col0 + cc;
                double v = 0.0;
                if (col < g.ncols) v = scale * (coef ? coef[(size_t)(col % g.ncells) * K + k] : 1.0);
                Cs[e] = (float)v;
            }
            __syncthreads();
            const int np = (kc + KPF - 1) / KPF, q0 = kk / KPF, total = K * np;
            const int ns = wave < total ? (total - wave + NW - 1) / NW : 0;  // steps s = wave + NW i
            if (ns == 0) continue;  // wave-uniform
            // ring of PF + 1 fragment slots with clamped loads and zero-operand padding, as in pc64_tile
            auto load = [&](int i, uint4 (&dst)[RT]) {
                const int s = wave + NW * min(i, ns - 1), k = s / np, q = s % np;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const int mt = min(mt0 + rt, g.MT - 1);
                    dst[rt] = reinterpret_cast<const uint4 *>(Af + ((((size_t)k * g.MT + mt) * QU + q0 + q) * 64 + lane) * U)[0];
                }
            };
            constexpr int S = PF + 1;
            uint4 ab[S][RT];
#pragma unroll
            for (int u = 0; u < PF; ++u) load(u, ab[u]);
            const int nsp = (ns + S - 1) / S * S;
            for (int i0 = 0; i0 < nsp; i0 += S) {
#pragma unroll
                for (int u = 0; u < S; ++u) {
                    const int i = i0 + u;
                    load(i + PF, ab[(u + PF) % S]);
                    const uint4 *a = ab[u];
                    const float live = i < ns ? 1.f : 0.f;
                    const int s = wave + NW * min(i, ns - 1), k = s / np, q = s % np;
                    float cf[CB];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) cf[cb] = Cs[k * NC + cb * 16 + lr] * live;
                    if constexpr (BF) {
                        v8bf b[CB];
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) {
                            const float *xr = Xs + (cb * 16 + lr) * LXS + q * KPF + 8 * lk;
#pragma unroll
                            for (int e = 0; e < 8; ++e) b[cb][e] = (__bf16)(xr[e] * cf[cb]);
                        }
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt) {
                            const v8bf av = __builtin_bit_cast(v8bf, a[rt]);
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb)
                                acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[cb], acc[rt][cb], 0, 0, 0);
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int r = q * KPF + 4 * j + lk;
                            float b[CB];
#pragma unroll
                            for (int cb = 0; cb < CB; ++cb) b[cb] = Xs[(cb * 16 + lr) * LXS + r] * cf[cb];
#pragma unroll
                            for (int rt = 0; rt < RT; ++rt) {
                                const uint32_t aw = j == 0 ? a[rt].x : j == 1 ? a[rt].y : j == 2 ? a[rt].z : a[rt].w;
                                const float av = __builtin_bit_cast(float, aw);
#pragma unroll
                                for (int cb = 0; cb < CB; ++cb)
                                    acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b[cb], acc[rt][cb], 0, 0, 0);
                            }
                        }
                    }
                }
            }
        }
    }
    // pairwise tree over the waves: wave w += wave w + h, h = NW/2, NW/4, ..., 1
#pragma unroll
    for (int h = NW / 2; h >= 1; h >>= 1) {
        __syncthreads();
        if (wave >= h && wave < 2 * h)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        Xs[(((wave - h) * RT + rt) * CB + cb) * 256 + i * 64 + lane] = acc[rt][cb][i];
        __syncthreads();
        if (wave < h)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[rt][cb][i] += Xs[((wave * RT + rt) * CB + cb) * 256 + i * 64 + lane];
    }
    if (wave != 0) return;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int mt = mt0 + rt, col = col0 + cb * 16 + lr;
            if (mt >= g.MT || col >= g.ncols) continue;
            double *ycol = g.Y + (long long)(col / g.ncells) * g.ybs + (size_t)(col % g.ncells) * g.ldy;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = mt * 16 + 4 * lk + i;
                if (row < g.M) ycol[row] = g.accumulate ? ycol[row] + (double)acc[rt][cb][i] : (double)acc[rt][cb][i];
            }
        }
}

template <int RTW, int CB, int NW, int KCB, int PF = 2>
void launch_big(const GemmArgsFrag &a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    dim3 grid((unsigned)((a.ncols + 16 * CB - 1) / (16 * CB)), (unsigned)((a.MT + RTW * NW - 1) / (RTW * NW)),
              (unsigned)std::max(1, a.ksplit));
    if (t0)
        hipExtLaunchKernelGGL((k_pc64_big<RTW, CB, NW, KCB, PF>), grid, dim3(64 * NW), 0, s, t0, t1, 0, a);
    else
        hipLaunchKernelGGL((k_pc64_big<RTW, CB, NW, KCB, PF>), grid, dim3(64 * NW), 0, s, a);
}

template <int RT, int CB, int PF, int NW>
void launch_frag(const GemmArgsFrag &a, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    dim3 grid((unsigned)((a.ncols + 16 * CB - 1) / (16 * CB)), (unsigned)((a.MT + RT - 1) / RT));
    if (t0)
        hipExtLaunchKernelGGL((k_pc64<RT, CB, PF, NW>), grid, dim3(64 * NW), 0, s, t0, t1, 0, a);
    else
        hipLaunchKernelGGL((k_pc64<RT, CB, PF, NW>), grid, dim3(64 * NW), 0, s, a);
}


}  // namespace

// fp32/bf16 copies of the principal operators used by the precision form
// ---------------------------------------------------------------- tile autotuner
// Candidate tile shapes of the two FP64 fragment kernels.  With options.autotune on, the first
// launch of each (shape, column count) times every candidate of its family in place (the output
// is overwritten, so only non-accumulating launches are tuned) and keeps the fastest; otherwise
// the defaults below are used (chosen by sweeps on gfx950).  Candidates differ in the order of
// the fixed-order sums, so results agree to rounding, not bitwise, across candidates.
using FragLauncher = void (*)(const GemmArgsFrag &, hipStream_t, hipEvent_t, hipEvent_t);
const FragLauncher kSmallCandidates[] = {launch_frag<4, 2, 2, 8>, launch_frag<2, 4, 4, 8>, launch_frag<2, 2, 4, 8>,
                                         launch_frag<4, 1, 4, 4>, launch_frag<1, 1, 2, 16>, launch_frag<2, 2, 2, 4>,
                                         launch_frag<4, 2, 3, 8>, launch_frag<2, 2, 3, 8>};
const FragLauncher kBigCandidates[] = {launch_big<2, 4, 4, 64>, launch_big<4, 2, 4, 64>, launch_big<2, 2, 8, 64>,
                                       launch_big<1, 4, 4, 64>, launch_big<2, 4, 4, 128>};
constexpr int kNSmall = sizeof(kSmallCandidates) / sizeof(kSmallCandidates[0]);
constexpr int kNBig = sizeof(kBigCandidates) / sizeof(kBigCandidates[0]);

static FragLauncher choose_launcher(ifeti_ctx *c, const GemmArgsFrag &f, bool big, int def, bool tunable) {
    const FragLauncher *cand = big ? kBigCandidates : kSmallCandidates;
    const int n = big ? kNBig : kNSmall;
    if (c->opt.tile_candidate >= 0) return cand[c->opt.tile_candidate % n];
    if (!c->opt.autotune || !tunable || c->capturing) return cand[def];
    std::vector<long long> key = {big ? 1 : 0, f.M, f.ncols, f.ngroups};
    for (int i = 0; i < f.ngroups; ++i) key.insert(key.end(), {f.Kd[i], f.K[i], f.gcodes[i] ? 1 : 0});
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) return cand[it->second];
    if (c->no_alloc) return cand[def];  // timing the candidates needs events
    hipEvent_t e0, e1;
    IFETI_HIP(hipEventCreate(&e0));
    IFETI_HIP(hipEventCreate(&e1));
    int best = def;
    float best_ms = 1e30f;
    for (int i = 0; i < n; ++i) {
        cand[i](f, c->stream, nullptr, nullptr);  // warm-up
        float tot = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
            cand[i](f, c->stream, e0, e1);
            IFETI_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            IFETI_HIP(hipEventElapsedTime(&ms, e0, e1));
            tot += ms;
        }
        if (tot < best_ms) {
            best_ms = tot;
            best = i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tuned[key] = best;
    if (std::getenv("IFETI_TUNE_VERBOSE"))
        std::fprintf(stderr, "[ifeti tune] %s M=%d ncols=%d Kd=%d K=%d -> candidate %d\n", big ? "big" : "small", f.M,
                     f.ncols, f.Kd[0], f.K[0], best);
    return cand[best];
}

template <typename T, int RTW, int CB, int NW, int KCB>
void launch_lp_big(const GemmArgsFragLP &f, hipStream_t s) {
    dim3 grid((unsigned)((f.ncols + 16 * CB - 1) / (16 * CB)), (unsigned)((f.MT + RTW * NW - 1) / (RTW * NW)));
    hipLaunchKernelGGL((k_pclp_big<T, RTW, CB, NW, KCB>), grid, dim3(64 * NW), 0, s, f);
}
template <typename T, int RT, int CB, int NW>
void launch_lp_tile(const GemmArgsFragLP &f, hipStream_t s) {
    dim3 grid((unsigned)((f.ncols + 16 * CB - 1) / (16 * CB)), (unsigned)((f.MT + RT - 1) / RT));
    hipLaunchKernelGGL((k_pclp_tile<T, RT, CB, NW>), grid, dim3(64 * NW), 0, s, f);
}
using LpLauncher = void (*)(const GemmArgsFragLP &, hipStream_t);
constexpr int kNLp = 4;
// [precision][shape][candidate]: FP32 / BF16; row-owning waves (large M) / shared tiles (small M)
const LpLauncher kLpCandidates[2][2][kNLp] = {
    {{launch_lp_big<float, 2, 4, 4, 64>, launch_lp_big<float, 4, 2, 4, 64>, launch_lp_big<float, 2, 2, 8, 64>,
      launch_lp_big<float, 2, 4, 4, 128>},
     {launch_lp_tile<float, 4, 2, 8>, launch_lp_tile<float, 2, 4, 4>, launch_lp_tile<float, 2, 2, 4>,
      launch_lp_tile<float, 1, 2, 8>}},
    {{launch_lp_big<__bf16, 2, 4, 4, 64>, launch_lp_big<__bf16, 4, 2, 4, 64>, launch_lp_big<__bf16, 2, 2, 8, 64>,
      launch_lp_big<__bf16, 2, 4, 4, 128>},
     {launch_lp_tile<__bf16, 4, 2, 8>, launch_lp_tile<__bf16, 2, 4, 4>, launch_lp_tile<__bf16, 2, 2, 4>,
      launch_lp_tile<__bf16, 1, 2, 8>}}};

static LpLauncher choose_lp_launcher(ifeti_ctx *c, const GemmArgsFragLP &f, bool bf, bool big, bool tunable) {
    const LpLauncher *cand = kLpCandidates[bf ? 1 : 0][big ? 0 : 1];
    if (c->opt.tile_candidate >= 0) return cand[c->opt.tile_candidate % kNLp];
    if (!c->opt.autotune || !tunable || c->capturing) return cand[big ? 2 : 0];  // the tuner's usual choice
    std::vector<long long> key = {bf ? 3 : 2, big ? 1 : 0, f.M, f.ncols, f.ngroups};
    for (int i = 0; i < f.ngroups; ++i) key.insert(key.end(), {f.Kd[i], f.K[i], f.gcodes[i] ? 1 : 0});
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) return cand[it->second];
    if (c->no_alloc) return cand[big ? 2 : 0];
    hipEvent_t e0, e1;
    IFETI_HIP(hipEventCreate(&e0));
    IFETI_HIP(hipEventCreate(&e1));
    int best = 0;
    float best_ms = 1e30f;
    for (int i = 0; i < kNLp; ++i) {
        cand[i](f, c->stream);  // warm-up
        IFETI_HIP(hipEventRecord(e0, c->stream));
        for (int rep = 0; rep < 3; ++rep) cand[i](f, c->stream);
        IFETI_HIP(hipEventRecord(e1, c->stream));
        IFETI_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        IFETI_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tuned[key] = best;
    if (std::getenv("IFETI_TUNE_VERBOSE"))
        std::fprintf(stderr, "[ifeti tune] %s %s M=%d ncols=%d Kd=%d K=%d -> candidate %d\n", bf ? "bf16" : "fp32",
                     big ? "big" : "tile", f.M, f.ncols, f.Kd[0], f.K[0], best);
    return cand[best];
}

// fragment-ordered copy of A viewed as K stacked M x Kd operators (built on first use)
static const double *frag_copy(ifeti_ctx *c, const double *A, int M, int Kd, int K) {
    for (auto &cp : c->frag)
        if (cp.src == A && cp.M == M && cp.Kd == Kd && cp.K == K && cp.kind == IFETI_FP64)
            return (const double *)cp.frag;
    IFETI_REQUIRE(!c->no_alloc, IFETI_EINVAL,
                  "allocation-free call: the fragment-order copy of an operator is not built (ifeti_apply_F "
                  "builds it)");
    const int MT = (M + 15) / 16, KT2 = (Kd + 7) / 8;
    const long long n = (long long)K * MT * KT2 * 128;
    ifeti_ctx::FragCopy cp;
    cp.src = A;
    cp.M = M;
    cp.Kd = Kd;
    cp.K = K;
    cp.kind = IFETI_FP64;
    IFETI_HIP(hipMalloc(&cp.frag, n * sizeof(double)));
    hipLaunchKernelGGL(k_to_frag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, A, M, Kd, K, MT, KT2,
                       (double *)cp.frag);
    IFETI_HIP(hipGetLastError());
    c->frag.push_back(cp);
    return (const double *)cp.frag;
}

// FP32 / BF16 fragment-unit copy of A (precision form, large M), built on first use
static const void *frag_copy_lp(ifeti_ctx *c, const double *A, int M, int Kd, int K, int kind) {
    for (auto &cp : c->frag)
        if (cp.src == A && cp.M == M && cp.Kd == Kd && cp.K == K && cp.kind == kind) return cp.frag;
    IFETI_REQUIRE(!c->no_alloc, IFETI_EINVAL,
                  "allocation-free call: the FP32/BF16 copy of an operator is not built (the first ifeti_apply_F "
                  "in that precision builds it)");
    const bool bf = kind == IFETI_BF16_LOCAL;
    const int MT = (M + 15) / 16, QU = (Kd + (bf ? 31 : 15)) / (bf ? 32 : 16), U = bf ? 8 : 4;
    const long long n = (long long)K * MT * QU * 64 * U;
    ifeti_ctx::FragCopy cp;
    cp.src = A;
    cp.M = M;
    cp.Kd = Kd;
    cp.K = K;
    cp.kind = kind;
    IFETI_HIP(hipMalloc(&cp.frag, n * (bf ? 2 : 4)));
    if (bf)
        hipLaunchKernelGGL(k_to_frag_lp<__bf16>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, A, M, Kd,
                           K, MT, QU, (__bf16 *)cp.frag);
    else
        hipLaunchKernelGGL(k_to_frag_lp<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, A, M, Kd,
                           K, MT, QU, (float *)cp.frag);
    IFETI_HIP(hipGetLastError());
    c->frag.push_back(cp);
    return cp.frag;
}

// Precision form: the sum sum_k c_sk A_k of a cell loses every digit to cancellation when the
// principal operators are nearly dependent and the coefficients large with opposite signs (the
// coefficient systems (41) are then ill-conditioned).  In a basis of the bank that is orthonormal in
// the Frobenius inner product, A'_j = sum_k A_k T_kj with T = V diag(lambda)^(-1/2) from the Gram matrix
// G_kl = <A_k, A_l>_F = V diag(lambda) V^T, the same sum has coefficients c'_s = diag(lambda)^(1/2) V^T c_s
// whose size is that of the sum itself, so the narrow operands round relative to the result.  The
// transformation is exact in FP64 (directions with lambda <= 1e-14 lambda_max carry no Frobenius mass
// and are dropped); only the narrow copies and the narrow-precision contractions use it.
void jacobi_eigen(std::vector<double> &A, int n, std::vector<double> &V, std::vector<double> &w) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {  // A <- J^T A J
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = cs * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = cs * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = cs * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

static const ifeti_ctx::RebasedBank &rebased_bank(ifeti_ctx *c, const double *A, const double *coef, int M, int Kd,
                                                 int K, int ncells) {
    for (auto &rb : c->rebased)
        if (rb.src == A && rb.coef == coef && rb.M == M && rb.Kd == Kd && rb.K == K && rb.ncells == ncells) return rb;
    IFETI_REQUIRE(!c->no_alloc, IFETI_EINVAL,
                  "allocation-free call: the precision form's re-based bank is not built (the first ifeti_apply_F "
                  "in that precision builds it)");
    const size_t me = (size_t)M * Kd;
    std::vector<double> hA((size_t)K * me), hc((size_t)ncells * K);
    IFETI_HIP(hipMemcpyAsync(hA.data(), A, hA.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipMemcpyAsync(hc.data(), coef, hc.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipStreamSynchronize(c->stream));
    std::vector<double> G((size_t)K * K, 0.0);
    for (int k = 0; k < K; ++k)
        for (int l = 0; l <= k; ++l) {
            const double *a = &hA[(size_t)k * me], *b = &hA[(size_t)l * me];
            double s = 0.0;
            for (size_t e = 0; e < me; ++e) s += a[e] * b[e];
            G[(size_t)k * K + l] = G[(size_t)l * K + k] = s;
        }
    std::vector<double> V, lam;
    jacobi_eigen(G, K, V, lam);
    double lmax = 0.0;
    for (double x : lam) lmax = std::max(lmax, x);
    std::vector<int> keep;
    for (int j = 0; j < K; ++j)
        if (lam[j] > 1e-14 * lmax) keep.push_back(j);
    const int Kp = (int)keep.size();
    IFETI_REQUIRE(Kp >= 1, IFETI_EINVAL, "precision form: the principal bank has no Frobenius mass");
    std::vector<double> Ap((size_t)Kp * me, 0.0), cp((size_t)ncells * Kp, 0.0);
    for (int jj = 0; jj < Kp; ++jj) {
        const int j = keep[jj];
        const double is = 1.0 / std::sqrt(lam[j]), sq = std::sqrt(lam[j]);
        double *dst = &Ap[(size_t)jj * me];
        for (int k = 0; k < K; ++k) {
            const double t = V[(size_t)k * K + j] * is;  // T_kj
            const double *a = &hA[(size_t)k * me];
            for (size_t e = 0; e < me; ++e) dst[e] += t * a[e];
        }
        for (int s = 0; s < ncells; ++s) {
            double v = 0.0;
            for (int k = 0; k < K; ++k) v += V[(size_t)k * K + j] * hc[(size_t)s * K + k];
            cp[(size_t)s * Kp + jj] = sq * v;
        }
    }
    ifeti_ctx::RebasedBank rb;
    rb.src = A;
    rb.coef = coef;
    rb.M = M;
    rb.Kd = Kd;
    rb.K = K;
    rb.Kp = Kp;
    rb.ncells = ncells;
    IFETI_HIP(hipMalloc(&rb.bank, Ap.size() * sizeof(double)));
    IFETI_HIP(hipMalloc(&rb.cf, cp.size() * sizeof(double)));
    IFETI_HIP(hipMemcpyAsync(rb.bank, Ap.data(), Ap.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    IFETI_HIP(hipMemcpyAsync(rb.cf, cp.data(), cp.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    IFETI_HIP(hipStreamSynchronize(c->stream));  // host staging goes out of scope
    c->rebased.push_back(rb);
    return c->rebased.back();
}

void prepare_operator_copies(ifeti_ctx *c) {
    if (c->K < 1) return;
    (void)frag_copy(c, c->Fdd.p, c->n_d, c->n_d, c->K);  // F̊ (48)
    (void)frag_copy(c, c->Sdd.p, c->n_d, c->n_d, c->K);  // M̊_D^-1 (49)
    if (c->n_p > 0) {  // the coarse restriction and prolongation of F̊ in principal form
        (void)frag_copy(c, c->WT.p, c->n_p, c->n_d, c->K);
        (void)frag_copy(c, c->W.p, c->n_d, c->n_p, c->K);
    }
}

void release_blas(void *handle) {
    if (handle) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(handle));
}

// Principal-weighted products with one small side (M <= 16 rows, or Kd <= 16 inputs: the restrictions
// and prolongations between the r block and the primal corners) for a block of load cases: one
// workgroup per cell forms the cell's combined operator sum_k coef_k A_k once and applies it to every
// load case, instead of K products per column on 16-row MFMA tiles of which the small side fills half.
// Rows: the combined M x Kd operator in LDS, one wave per load case, lanes over the Kd inputs and a
// wave reduction per row.  Columns: each thread keeps its rows' Kd combined entries in registers.
template <int MMAX>
__global__ __launch_bounds__(256) void k_small_rows(const double *__restrict__ A, const double *__restrict__ coef, int K,
                                                    int M, int Kd, const double *__restrict__ X, int ldx, long long xbs,
                                                    int ncells, int nrhs, double scale, double *__restrict__ Y, int ldy,
                                                    long long ybs, int accumulate) {
    extern __shared__ double Cl[];  // [M][Kd]
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t mk = (size_t)M * Kd;
    for (size_t e = tid; e < mk; e += 256) {
        double v = 0.0;
        for (int k = 0; k < K; ++k) v += coef[(size_t)s * K + k] * A[(size_t)k * mk + e];
        Cl[e] = v;
    }
    __syncthreads();
    for (int rhs = wave; rhs < nrhs; rhs += 4) {  // no barrier below: any trip count per wave
        const double *x = X + rhs * xbs + (size_t)s * ldx;
        double acc[MMAX];
#pragma unroll
        for (int m = 0; m < MMAX; ++m) acc[m] = 0.0;
        for (int j = lane; j < Kd; j += 64) {
            const double xv = x[j];
#pragma unroll
            for (int m = 0; m < MMAX; ++m)
                if (m < M) acc[m] += Cl[(size_t)m * Kd + j] * xv;
        }
        double *y = Y + rhs * ybs + (size_t)s * ldy;
#pragma unroll
        for (int m = 0; m < MMAX; ++m) {
            double v = acc[m];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0 && m < M) y[m] = accumulate ? y[m] + scale * v : scale * v;
        }
    }
}

template <int KMAX>
__global__ __launch_bounds__(256) void k_small_cols(const double *__restrict__ A, const double *__restrict__ coef, int K,
                                                    int M, int Kd, const double *__restrict__ X, int ldx, long long xbs,
                                                    int ncells, int nrhs, double scale, double *__restrict__ Y, int ldy,
                                                    long long ybs, int accumulate) {
    const int s = blockIdx.x;
    const size_t mk = (size_t)M * Kd;
    for (int m = threadIdx.x; m < M; m += 256) {
        double cr[KMAX];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) cr[j] = 0.0;
        for (int k = 0; k < K; ++k) {
            const double ck = coef[(size_t)s * K + k];
            const double *a = A + (size_t)k * mk + (size_t)m * Kd;
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < Kd) cr[j] += ck * a[j];
        }
        for (int rhs = 0; rhs < nrhs; ++rhs) {
            const double *x = X + rhs * xbs + (size_t)s * ldx;
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < Kd) v += cr[j] * x[j];
            double *y = Y + rhs * ybs + (size_t)s * ldy + m;
            *y = accumulate ? *y + scale * v : scale * v;
        }
    }
}

static bool small_side_gemm(ifeti_ctx *c, const GemmGroup &g, double *Y, int ldy, long long ybs, int M, int ncols,
                            int ncells, bool accumulate, const char *tag) {
    if (!g.coef || g.gcodes || g.gw || ncols % ncells != 0 || ncols / ncells < 4 || c->opt.tile_candidate >= 0)
        return false;
    const int nrhs = ncols / ncells;
    const long long xbs = g.xbs ? g.xbs : (long long)ncells * g.ldx;
    const long long ys = ybs ? ybs : (long long)ncells * ldy;
    const double cols = (double)ncols;
    if (M <= 8 && (size_t)M * g.Kd * sizeof(double) <= 64 * 1024) {
        const size_t lds = (size_t)M * g.Kd * sizeof(double);
        Prof prof(c, tag, 2.0 * M * cols * g.Kd + 2.0 * g.K * M * (double)g.Kd * ncells,
                  8.0 * ((double)g.K * M * g.Kd + cols * g.Kd + cols * M * (accumulate ? 2 : 1)));
        IFETI_HIP(hipFuncSetAttribute((const void *)k_small_rows<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
        hipLaunchKernelGGL(k_small_rows<8>, dim3(ncells), dim3(256), lds, c->stream, g.A, g.coef, g.K, M, g.Kd, g.X,
                           g.ldx, xbs, ncells, nrhs, g.scale, Y, ldy, ys, accumulate ? 1 : 0);
        IFETI_HIP(hipGetLastError());
        return true;
    }
    if (g.Kd <= 8) {
        Prof prof(c, tag, 2.0 * M * cols * g.Kd + 2.0 * g.K * M * (double)g.Kd * ncells,
                  8.0 * ((double)g.K * M * g.Kd + cols * g.Kd + cols * M * (accumulate ? 2 : 1)));
        hipLaunchKernelGGL(k_small_cols<8>, dim3(ncells), dim3(256), 0, c->stream, g.A, g.coef, g.K, M, g.Kd, g.X,
                           g.ldx, xbs, ncells, nrhs, g.scale, Y, ldy, ys, accumulate ? 1 : 0);
        IFETI_HIP(hipGetLastError());
        return true;
    }
    return false;
}

// A plain product (one operator, no principal coefficients, no fused gather) with many rows in FP64:
// the stacked principal inverses of (46a) applied to every cell vector.  rocBLAS's DGEMM runs it at
// 0.87 of the FP64 matrix peak on the c2 shape (7680 x 640 times 640 x 4096), against 0.51 for the
// principal-shared kernel, whose LDS staging is built for the coefficient-weighted sums.  Few columns
// (the coarse solve of a block of load cases: 8320 x 8320 times 32 columns) stay with the own kernels,
// where the library runs at a quarter of their rate.  A forced tile candidate keeps the own kernel
// (its parity tests force every candidate), and so does an allocation-free call.
static bool library_gemm(ifeti_ctx *c, const GemmGroup &g, double *Y, int ldy, long long ybs, int M, int ncols,
                         int ncells, bool accumulate, const char *tag) {
    if (g.K != 1 || g.coef || g.gcodes || g.gw || g.scale != 1.0 || accumulate || M < 512 || ncols < 1024 ||
        c->no_alloc || c->opt.tile_candidate >= 0 || ncols % ncells != 0)
        return false;
    if (!c->blas) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return false;
        c->blas = h;
    }
    rocblas_handle h = static_cast<rocblas_handle>(c->blas);
    const int nrhs = ncols / ncells;
    const long long xbs = g.xbs ? g.xbs : (long long)ncells * g.ldx;
    const long long ys = ybs ? ybs : (long long)ncells * ldy;
    IFETI_REQUIRE(rocblas_set_stream(h, c->stream) == rocblas_status_success, IFETI_EHIP, "rocblas_set_stream");
    const double one = 1.0, zero = 0.0;
    Prof prof(c, tag, 2.0 * M * (double)ncols * g.Kd,
              8.0 * ((double)M * g.Kd + (double)ncols * g.Kd + (double)ncols * M));
    // Y (M x ncells per load case, column-major, ld ldy) = A (M x Kd, row-major = transposed
    // column-major) times X (Kd x ncells, ld ldx)
    const rocblas_status st = rocblas_dgemm_strided_batched(
        h, rocblas_operation_transpose, rocblas_operation_none, M, ncells, g.Kd, &one, g.A, g.Kd, 0, g.X, g.ldx,
        xbs, &zero, Y, ldy, ys, nrhs);
    IFETI_REQUIRE(st == rocblas_status_success, IFETI_EHIP,
                  std::string("rocblas_dgemm_strided_batched: ") + rocblas_status_to_string(st));
    return true;
}

// narrow copies for the library: A row-major in FP32 or BF16 (cached with the fragment copies, kind
// 100 + precision), X cast column by column
template <typename T>
__global__ __launch_bounds__(256) void k_cast_cols(const double *__restrict__ X, int ldx, long long xbs, int Kd,
                                                   int ncells, int nrhs, T *__restrict__ Y) {
    const long long n = (long long)Kd * ncells * nrhs;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const long long col = e / Kd;
    const int k = (int)(e % Kd), r = (int)(col / ncells), s = (int)(col % ncells);
    Y[e] = (T)X[r * xbs + (long long)s * ldx + k];
}

static const void *plain_copy_narrow(ifeti_ctx *c, const double *A, int M, int Kd, int kind) {
    const int key = 100 + kind;
    for (auto &cp : c->frag)
        if (cp.src == A && cp.M == M && cp.Kd == Kd && cp.K == 1 && cp.kind == key) return cp.frag;
    const bool bf = kind == IFETI_BF16_LOCAL;
    const long long n = (long long)M * Kd;
    ifeti_ctx::FragCopy cp;
    cp.src = A;
    cp.M = M;
    cp.Kd = Kd;
    cp.K = 1;
    cp.kind = key;
    IFETI_HIP(hipMalloc(&cp.frag, n * (bf ? 2 : 4)));
    if (bf)
        hipLaunchKernelGGL(k_cast_cols<__bf16>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, A, Kd,
                           0LL, Kd, M, 1, (__bf16 *)cp.frag);
    else
        hipLaunchKernelGGL(k_cast_cols<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, A, Kd, 0LL,
                           Kd, M, 1, (float *)cp.frag);
    IFETI_HIP(hipGetLastError());
    c->frag.push_back(cp);
    return cp.frag;
}

bool library_gemm_narrow(ifeti_ctx *c, const double *A, int M, int Kd, const double *X, int ldx, long long xbs,
                         int ncells, int nrhs, int kind, float *Y32, const char *tag) {
    if ((kind != IFETI_FP32_LOCAL && kind != IFETI_BF16_LOCAL) || c->no_alloc || c->opt.tile_candidate >= 0 ||
        (long long)ncells * nrhs < 1024)
        return false;
    if (!c->blas) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return false;
        c->blas = h;
    }
    rocblas_handle h = static_cast<rocblas_handle>(c->blas);
    const bool bf = kind == IFETI_BF16_LOCAL;
    const void *An = plain_copy_narrow(c, A, M, Kd, kind);
    const long long nx = (long long)Kd * ncells * nrhs;
    c->w_v16.ensure((size_t)nx * (bf ? 1 : 2), c->stream);
    if (bf)
        hipLaunchKernelGGL(k_cast_cols<__bf16>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, c->stream, X, ldx,
                           xbs, Kd, ncells, nrhs, (__bf16 *)c->w_v16.p);
    else
        hipLaunchKernelGGL(k_cast_cols<float>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, c->stream, X, ldx, xbs,
                           Kd, ncells, nrhs, (float *)c->w_v16.p);
    IFETI_HIP(hipGetLastError());
    IFETI_REQUIRE(rocblas_set_stream(h, c->stream) == rocblas_status_success, IFETI_EHIP, "rocblas_set_stream");
    const double cols = (double)ncells * nrhs;
    Prof prof(c, tag, 2.0 * M * cols * Kd, (bf ? 2.0 : 4.0) * ((double)M * Kd + cols * Kd) + 4.0 * cols * M);
    const float one = 1.0f, zero = 0.0f;
    const rocblas_int n = ncells * nrhs;  // the narrow copy of X is one contiguous Kd x n matrix
    rocblas_status st;
    if (bf)
        st = rocblas_gemm_ex(h, rocblas_operation_transpose, rocblas_operation_none, M, n, Kd, &one, An,
                             rocblas_datatype_bf16_r, Kd, c->w_v16.p, rocblas_datatype_bf16_r, Kd, &zero, Y32,
                             rocblas_datatype_f32_r, M, Y32, rocblas_datatype_f32_r, M, rocblas_datatype_f32_r,
                             rocblas_gemm_algo_standard, 0, 0);
    else
        st = rocblas_sgemm(h, rocblas_operation_transpose, rocblas_operation_none, M, n, Kd, &one, (const float *)An, Kd,
                           (const float *)c->w_v16.p, Kd, &zero, Y32, M);
    IFETI_REQUIRE(st == rocblas_status_success, IFETI_EHIP,
                  std::string("rocBLAS narrow product: ") + rocblas_status_to_string(st));
    return true;
}

void gemm(ifeti_ctx *c, const GemmGroup *groups, int ngroups, double *Y, int ldy, long long ybs, int M, int ncols,
          bool accumulate, int ncells, const char *tag, bool lp_ok) {
    IFETI_REQUIRE(ngroups >= 1 && ngroups <= 2, IFETI_EINVAL, "gemm: 1 or 2 groups");
    for (int i = 0; i < ngroups; ++i)
        IFETI_REQUIRE(groups[i].K >= 1 && groups[i].K <= kMaxCoefK, IFETI_EINVAL, "gemm: 1 to 40 principal operators");
    if (ncols <= 0 || M <= 0) return;
    GemmArgsDev a{};
    a.ncells = ncells > 0 ? ncells : c->N;
    int Kmax = 0, Kdmax = 0;
    for (int i = 0; i < ngroups; ++i) {
        Kdmax = std::max(Kdmax, groups[i].Kd);
        a.A[i] = groups[i].A;
        a.X[i] = groups[i].X;
        a.coef[i] = groups[i].coef;
        a.Kd[i] = groups[i].Kd;
        a.ldx[i] = groups[i].ldx;
        a.xbs[i] = groups[i].xbs ? groups[i].xbs : (long long)a.ncells * groups[i].ldx;
        a.K[i] = groups[i].K;
        a.scale[i] = groups[i].scale;
        Kmax = std::max(Kmax, groups[i].K);
    }
    a.ngroups = ngroups;
    a.Y = Y;
    a.ldy = ldy;
    a.ybs = ybs ? ybs : (long long)a.ncells * ldy;
    a.M = M;
    a.ncols = ncols;
    a.accumulate = accumulate ? 1 : 0;
    // algorithmic work: 2*M*ncols*sum_g K_g*Kd_g flops; operators, cell vectors and results moved once
    double flops = 0.0, bytes = 8.0 * (double)ncols * M * (accumulate ? 2 : 1);
    for (int i = 0; i < ngroups; ++i) {
        flops += 2.0 * M * (double)ncols * groups[i].K * groups[i].Kd;
        bytes += 8.0 * ((double)groups[i].K * M * groups[i].Kd + (groups[i].coef ? (double)a.ncells * groups[i].K : 0.0));
        if (groups[i].gcodes) {  // gathered staging: multipliers (+ weights) once, two int32 codes per slot
            const double nr = (double)ncols / a.ncells;
            bytes += 8.0 * (double)groups[i].xbs * nr * (groups[i].gw ? 2.0 : 1.0) + 8.0 * (double)a.ncells * groups[i].Kd;
        } else {
            bytes += 8.0 * (double)ncols * groups[i].Kd;
        }
    }
    double abytes = 0.0;
    for (int i = 0; i < ngroups; ++i) abytes += 8.0 * (double)groups[i].K * M * groups[i].Kd;
    const int prec = c->prec_override >= 0 ? c->prec_override : c->opt.precision;
    const bool lp_path = lp_ok && prec != IFETI_FP64 && M > 16 && Kdmax > 16;
    if (!lp_path && ngroups == 1 && library_gemm(c, groups[0], Y, ldy, a.ybs, M, ncols, a.ncells, accumulate, tag))
        return;
    if (!lp_path && ngroups == 1 &&
        small_side_gemm(c, groups[0], Y, ldy, a.ybs, M, ncols, a.ncells, accumulate, tag))
        return;
    const bool frag_small = abytes <= 4.0 * 1024 * 1024;  // operators that stay resident in L2
    const bool frag_big = !frag_small && M >= 512;         // many row tiles: waves own rows
    // large operators, or many columns (a block of load cases): row-owning waves, fragment units
    const bool lp_big = lp_path && ((!frag_small && M >= 512) || (M >= 64 && ncols >= 16384));
    if (lp_path) {
        GemmArgsFragLP f{};
        const int kind = prec;
        const bool bf = kind == IFETI_BF16_LOCAL;
        for (int i = 0; i < ngroups; ++i) {
            // summed principal operators: the re-based bank and its coefficients (no cancellation in the
            // narrow operands)
            const double *Ai = groups[i].A, *ci = a.coef[i];
            int Ki = groups[i].K;
            if (ci && Ki > 1) {
                const auto &rb = rebased_bank(c, Ai, ci, M, groups[i].Kd, Ki, a.ncells);
                Ai = rb.bank;
                ci = rb.cf;
                Ki = rb.Kp;
            }
            f.Af[i] = frag_copy_lp(c, Ai, M, groups[i].Kd, Ki, kind);
            f.X[i] = a.X[i];
            f.coef[i] = ci;
            f.gcodes[i] = groups[i].gcodes;
            f.gw[i] = groups[i].gw;
            f.Kd[i] = a.Kd[i];
            f.ldx[i] = a.ldx[i];
            f.K[i] = Ki;
            f.QU[i] = (a.Kd[i] + (bf ? 31 : 15)) / (bf ? 32 : 16);
            f.xbs[i] = a.xbs[i];
            f.scale[i] = a.scale[i];
        }
        f.ngroups = ngroups;
        f.Y = Y;
        f.ybs = a.ybs;
        f.ldy = ldy;
        f.M = M;
        f.MT = (M + 15) / 16;
        f.ncols = ncols;
        f.ncells = a.ncells;
        f.accumulate = a.accumulate;
        // as the FP64 count, with the operators moved in the narrow type
        const double lbytes = bytes - (8.0 - (bf ? 2.0 : 4.0)) * abytes / 8.0;
        Prof prof(c, tag, flops, lbytes);
        LpLauncher launch_fn = choose_lp_launcher(c, f, bf, lp_big, !accumulate);
        launch_fn(f, c->stream);
        IFETI_HIP(hipGetLastError());
        return;
    }
    // FP64: L2-resident operators (a few MB per XCD) take the fragment-ordered path
    {
        GemmArgsFrag f{};
        for (int i = 0; i < ngroups; ++i) {
            f.Af[i] = frag_copy(c, groups[i].A, M, groups[i].Kd, groups[i].K);
            f.X[i] = a.X[i];
            f.coef[i] = a.coef[i];
            f.gcodes[i] = groups[i].gcodes;
            f.gw[i] = groups[i].gw;
            f.Kd[i] = a.Kd[i];
            f.ldx[i] = a.ldx[i];
            f.K[i] = a.K[i];
            f.KT2[i] = (a.Kd[i] + 7) / 8;
            f.xbs[i] = a.xbs[i];
            f.scale[i] = a.scale[i];
        }
        f.ngroups = ngroups;
        f.Y = Y;
        f.ybs = a.ybs;
        f.ldy = ldy;
        f.M = M;
        f.MT = (M + 15) / 16;
        f.ncols = ncols;
        f.ncells = a.ncells;
        f.accumulate = a.accumulate;
        Prof prof(c, tag, flops, bytes, true);
        // shapes tuned on gfx950: few rows -> many waves per tile; few inner steps -> tall tiles
        if (frag_big && ncols <= 128 && ngroups == 1) {
            // tall operator, few columns (coarse solve of a block of load cases): 64-row tiles, inner range
            // split 8 ways over blockIdx.z, partials summed in split order
            f.ksplit = 8;
            IFETI_REQUIRE(!c->no_alloc || c->w_split.n >= (size_t)f.ksplit * ncols * M, IFETI_EINVAL,
                          "allocation-free call: the split-K partial buffer is too small (ifeti_apply_F grows it)");
            c->w_split.ensure((size_t)f.ksplit * ncols * M, c->stream);
            f.part = c->w_split.p;
            launch_big<1, 2, 4, 128, 8>(f, c->stream, prof.start(), prof.stop());  // 8 pairs in flight per wave
            const long long n = (long long)ncols * M;
            hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                               c->w_split.p, f.ksplit, ncols, M, f.ncells, Y, f.ybs, ldy, f.accumulate);
        } else {
            // defaults = the autotuner's usual choice on gfx950 (2D and 3D lattices).  Beside a concurrent
            // branch, the one-workgroup-per-CU 64-row tile (173 VGPRs, two waves per SIMD) instead of the
            // fastest tile alone (two workgroups per CU, which fill the register files and hold the branch
            // back until the contraction ends); such launches are not autotuned (timed alone)
            const int def = frag_big ? 2 : (f.MT <= 2 ? 4 : (Kdmax <= 16 ? 3 : 7));
            FragLauncher launch_fn = choose_launcher(c, f, frag_big, def, !accumulate);
            launch_fn(f, c->stream, prof.start(), prof.stop());
        }
        IFETI_HIP(hipGetLastError());
        return;
    }
}


}  // namespace ifeti
