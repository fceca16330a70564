// Online operators of the ROM-based inexact FETI-DP preconditioner (paper
// Sec. 3.2): jump gather/scatter (eq. (15)), primal assembly (eq. (18)), coarse
// solve (Sec. 3.2.1), F̊ (48), M̊_D^-1 (49), Ů / Ůᵀ (Algorithm 3), K̊^-ROM
// (eqs. (45)-(46), Algorithm 2), the true saddle operator (16), and the
// vector kernels of the Krylov solvers.
//
// Cell vectors are cell-major: column c = rhs*N + s holds cell s of load case
// rhs.  Scatters are pull-based (every multiplier row reads its at most two
// signed endpoints, every primal dof its at most 2^d cell corners), so results
// are bitwise reproducible and no floating-point atomics are used.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace ifeti {
namespace {

// Workgroup b of a cell-batched launch -> (cell s, load case rhs).  Workgroups go to the eight XCDs in
// turn; with several load cases, b takes cell (b mod 8) + 8 (j / nrhs) and load case j mod nrhs,
// j = b / 8, so the load cases of a cell run together on one XCD and its L2 serves them the cell's
// data (the grid is padded to 8 ceil(N/8) cells; false for a padding workgroup, which exits whole).
// One load case: the identity.
__device__ __forceinline__ bool cell_of_block(int b, int N, int nrhs, int &s, int &rhs) {
    if (nrhs <= 1) {
        s = b;
        rhs = 0;
        return true;
    }
    const int j = b >> 3;
    s = (b & 7) + 8 * (j / nrhs);
    rhs = j % nrhs;
    return s < N;
}

constexpr int kB = 256;
inline unsigned nblocks(long long n, int b = kB) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------------ B_d^T, B_d
__global__ __launch_bounds__(kB) void k_gather(const int *__restrict__ gl, const double *__restrict__ Dw,
                                               const double *__restrict__ lam, long long lam_rs,
                                               double *__restrict__ out, int N, int n_d, int nrhs, int weights) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long per = (long long)N * n_d;
    if (t >= per * nrhs) return;
    int rhs = (int)(t / per);
    long long sj = t % per;
    const double *l = lam + rhs * lam_rs;
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        int code = gl[sj * 2 + u];
        if (code == 0) continue;
        int row = (code > 0 ? code : -code) - 1;
        double x = l[row] * (weights ? Dw[row] : 1.0);
        v += code > 0 ? x : -x;
    }
    out[t] = v;
}

__global__ __launch_bounds__(kB) void k_scatter(const int *__restrict__ sl, const double *__restrict__ Dw,
                                                const double *__restrict__ Y, int y_ld, int y_off, long long y_rs,
                                                double *__restrict__ out, long long out_rs, int L, int n_d, int nrhs,
                                                int weights) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)L * nrhs) return;
    int rhs = (int)(t / L), l = (int)(t % L);
    const double *y = Y + rhs * y_rs;
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        int code = sl[(size_t)l * 2 + u];
        if (code == 0) continue;
        int e = (code > 0 ? code : -code) - 1;
        int s = e / n_d, j = e % n_d;
        double x = y[(size_t)s * y_ld + y_off + j];
        v += code > 0 ? x : -x;
    }
    out[rhs * out_rs + l] = weights ? v * Dw[l] : v;
}

// B_d (and D-scaling) with the PCG dot product fused: grid (nblk, nrhs), block b
// owns the contiguous chunk b of the L multipliers of its load case and writes
// its partial sum of out . w (tree-reduced in a fixed order).
__global__ __launch_bounds__(kB) void k_scatter_dot(const int *__restrict__ sl, const double *__restrict__ Dw,
                                                    const double *__restrict__ Y, const double *__restrict__ Y2,
                                                    int y_ld, int y_off, long long y_rs,
                                                    double *__restrict__ out, long long out_rs, int L, int n_d,
                                                    int weights, const double *__restrict__ w, int nblk,
                                                    double *__restrict__ part) {
    __shared__ double sh[kB];
    const int b = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x;
    const int chunk = (L + nblk - 1) / nblk;
    const int i0 = b * chunk, i1 = min(L, i0 + chunk);
    const double *y = Y + rhs * y_rs;
    const double *y2 = Y2 ? Y2 + rhs * y_rs : nullptr;
    double acc = 0.0;
    for (int l = i0 + tid; l < i1; l += kB) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            int code = sl[(size_t)l * 2 + u];
            if (code == 0) continue;
            int e = (code > 0 ? code : -code) - 1;
            int s = e / n_d, j = e % n_d;
            const size_t at = (size_t)s * y_ld + y_off + j;
            double x = y2 ? y[at] + y2[at] : y[at];
            v += code > 0 ? x : -x;
        }
        if (weights) v *= Dw[l];
        out[rhs * out_rs + l] = v;
        if (w) acc += v * w[rhs * out_rs + l];
    }
    if (!part) return;  // uniform
    // a butterfly within each wave, then the wave sums in wave order (fixed order)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kB / 64; ++w) t += sh[w];
        part[(size_t)rhs * nblk + b] = t;
    }
}

// ------------------------------------------------------------------ coarse maps of F̊ (48)
// The coarse restriction and prolongation of F̊ use, per cell, the same
// n_p x n_d matrix C_s = sum_k pi_sk (T_dr U_rp^(k))^T.  It depends only on the
// coefficients, so it is combined once per reduced basis and both maps become
// streaming per-cell products instead of small-M contractions.
__global__ __launch_bounds__(kB) void k_combine_wt(const double *__restrict__ pi, const double *__restrict__ WT,
                                                   int N, int K, int npd, double *__restrict__ C) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)N * npd) return;
    const int s = (int)(t / npd), e = (int)(t % npd);
    double v = 0.0;
    for (int k = 0; k < K; ++k) v += pi[(size_t)s * K + k] * WT[(size_t)k * npd + e];
    C[t] = v;
}

constexpr int kMaxNp = 24;  // primal (corner) dofs per cell: 4 x 2 in 2D, 8 x 3 in 3D

// c_s = C_s B_d^T lam for column (rhs, s): one workgroup of NWC waves per column;
// wave w takes the 64-row chunks w, w + NWC, ... of the cell's dual dofs (lanes
// gather the signed multipliers), reduces its n_p sums across the wave, and the
// NWC partial vectors are added in wave order through LDS.
template <int NPM, int NWC>
__global__ __launch_bounds__(64 * NWC) void k_restrict_c(const double *__restrict__ C, const int *__restrict__ gl,
                                                          const double *__restrict__ lam, long long lam_rs, int N,
                                                          int n_d, int n_p, int ncols, double *__restrict__ out) {
    __shared__ double part[NWC][NPM];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int s, rhs;
    if (!cell_of_block(blockIdx.x, N, ncols / N, s, rhs)) return;  // whole workgroup, before any barrier
    const int col = rhs * N + s;
    const double *l = lam + rhs * lam_rs;
    const double *Cs = C + (size_t)s * n_p * n_d;
    double acc[NPM];
#pragma unroll
    for (int i = 0; i < NPM; ++i) acc[i] = 0.0;
    for (int j = 64 * wave + lane; j < n_d; j += 64 * NWC) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int code = gl[((size_t)s * n_d + j) * 2 + u];
            if (code == 0) continue;
            const double x = l[(code > 0 ? code : -code) - 1];
            v += code > 0 ? x : -x;
        }
#pragma unroll
        for (int i = 0; i < NPM; ++i)
            if (i < n_p) acc[i] += Cs[(size_t)i * n_d + j] * v;
    }
#pragma unroll
    for (int i = 0; i < NPM; ++i) {
        if (i < n_p) {  // uniform over the workgroup
            double v = acc[i];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) part[wave][i] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < n_p) {
        double v = part[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < NWC; ++w) v += part[w][threadIdx.x];
        out[(size_t)col * n_p + threadIdx.x] = v;
    }
}

// the same with one wave per column and n_p <= 8: the 8 per-lane partial sums go through LDS, lane
// (i, g) adds the partials of row i held by lanes 8g..8g+7, and three butterfly steps over g finish
template <int NPM>
__global__ __launch_bounds__(64) void k_restrict_c1(const double *__restrict__ C, const int *__restrict__ gl,
                                                    const double *__restrict__ lam, long long lam_rs, int N, int n_d,
                                                    int n_p, int ncols, double *__restrict__ out) {
    static_assert(NPM == 8, "one row per group of 8 lanes");
    __shared__ double part[64][NPM + 1];
    const int lane = threadIdx.x;
    int s, rhs;
    if (!cell_of_block(blockIdx.x, N, ncols / N, s, rhs)) return;  // whole workgroup, before any barrier
    const int col = rhs * N + s;
    const double *l = lam + rhs * lam_rs;
    const double *Cs = C + (size_t)s * n_p * n_d;
    double acc[NPM];
#pragma unroll
    for (int i = 0; i < NPM; ++i) acc[i] = 0.0;
    for (int j = lane; j < n_d; j += 64) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int code = gl[((size_t)s * n_d + j) * 2 + u];
            if (code == 0) continue;
            const double x = l[(code > 0 ? code : -code) - 1];
            v += code > 0 ? x : -x;
        }
#pragma unroll
        for (int i = 0; i < NPM; ++i)
            if (i < n_p) acc[i] += Cs[(size_t)i * n_d + j] * v;
    }
#pragma unroll
    for (int i = 0; i < NPM; ++i) part[lane][i] = acc[i];
    __syncthreads();
    const int i = lane >> 3, g = lane & 7;
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t) v += part[8 * g + t][i];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    if (g == 0 && i < n_p) out[(size_t)col * n_p + i] = v;
}

// The same restriction for a block of load cases, one workgroup of four waves per cell: each wave
// loads the cell's C_s and jump codes once (two dual rows per lane, n_d <= 128) and takes every fourth
// load case, so C_s is read once per cell instead of once per load case.  Per load case the eight
// partial sums are reduced as in k_restrict_c1 (LDS, then three butterflies).
template <int NPM>
__global__ __launch_bounds__(256) void k_restrict_cm(const double *__restrict__ C, const int *__restrict__ gl,
                                                     const double *__restrict__ lam, long long lam_rs, int N, int n_d,
                                                     int n_p, int nrhs, double *__restrict__ out) {
    static_assert(NPM == 8, "one row per group of 8 lanes");
    __shared__ double part[4][64][NPM + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int s = blockIdx.x;
    const double *Cs = C + (size_t)s * n_p * n_d;
    double cv[2][NPM];
    int code[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = lane + 64 * h;
        const bool in = j < n_d;
#pragma unroll
        for (int i = 0; i < NPM; ++i) cv[h][i] = (in && i < n_p) ? Cs[(size_t)i * n_d + j] : 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u) code[h][u] = in ? gl[((size_t)s * n_d + j) * 2 + u] : 0;
    }
    for (int r0 = 0; r0 < nrhs; r0 += 4) {  // the same trip count in every wave: barriers below
        const int rhs = r0 + wave;
        const bool act = rhs < nrhs;
        const double *l = lam + (act ? rhs : 0) * lam_rs;
        double acc[NPM];
#pragma unroll
        for (int i = 0; i < NPM; ++i) acc[i] = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int cd = act ? code[h][u] : 0;
                if (cd == 0) continue;
                const double x = l[(cd > 0 ? cd : -cd) - 1];
                v += cd > 0 ? x : -x;
            }
#pragma unroll
            for (int i = 0; i < NPM; ++i) acc[i] += cv[h][i] * v;
        }
#pragma unroll
        for (int i = 0; i < NPM; ++i) part[wave][lane][i] = acc[i];
        __syncthreads();
        const int i = lane >> 3, g = lane & 7;
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < 8; ++t) v += part[wave][8 * g + t][i];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        if (act && g == 0 && i < n_p) out[((size_t)rhs * N + s) * n_p + i] = v;
        __syncthreads();  // the partials are read before the next load cases overwrite them
    }
}

// Y_s (+)= C_s^T y_P[A_p(s)] for a block of load cases: one workgroup of n_d threads (n_d <= 256) per
// cell, each thread's column of C_s loaded once and used for every load case
template <int NPM>
__global__ __launch_bounds__(256) void k_prolong_cm(const double *__restrict__ C, const int *__restrict__ Ap,
                                                    const double *__restrict__ yP, long long yP_rs, int N, int n_d,
                                                    int n_p, int nrhs, double *__restrict__ Y, int accumulate) {
    const int s = blockIdx.x, j = threadIdx.x;
    const bool in = j < n_d;
    const double *Cs = C + (size_t)s * n_p * n_d;
    double cv[NPM];
    int P[NPM];
#pragma unroll
    for (int i = 0; i < NPM; ++i) {
        cv[i] = (in && i < n_p) ? Cs[(size_t)i * n_d + j] : 0.0;
        P[i] = i < n_p ? Ap[(size_t)s * n_p + i] : -1;
    }
    for (int rhs = 0; rhs < nrhs; ++rhs) {
        const double *zP = yP + rhs * yP_rs;
        double *Yc = Y + ((size_t)rhs * N + s) * n_d;
        double v = (in && accumulate) ? Yc[j] : 0.0;
#pragma unroll
        for (int i = 0; i < NPM; ++i)
            if (P[i] >= 0) v += cv[i] * zP[P[i]];
        if (in) Yc[j] = v;
    }
}

// Y_s (+)= C_s^T y_P[A_p(s)] for column (rhs, s): one workgroup of NWC waves per
// column, lanes over the cell's dual rows (coalesced rows of C_s); the n_p
// primal values of the cell are uniform.
template <int NPM, int NWC>
__global__ __launch_bounds__(64 * NWC) void k_prolong_c(const double *__restrict__ C, const int *__restrict__ Ap,
                                                         const double *__restrict__ yP, long long yP_rs, int N,
                                                         int n_d, int n_p, int ncols, double *__restrict__ Y,
                                                         int accumulate) {
    int s, rhs;
    if (!cell_of_block(blockIdx.x, N, ncols / N, s, rhs)) return;  // whole workgroup
    const int col = rhs * N + s;
    const double *zP = yP + rhs * yP_rs;
    const double *Cs = C + (size_t)s * n_p * n_d;
    double *Yc = Y + (size_t)col * n_d;
    if (n_d <= 64 * NWC) {  // one row per thread: its C column and Y entry are loaded before the primal values
        const int j = threadIdx.x;
        const bool in = j < n_d;
        double cv[NPM];
#pragma unroll
        for (int i = 0; i < NPM; ++i) cv[i] = (in && i < n_p) ? Cs[(size_t)i * n_d + j] : 0.0;
        double v = (in && accumulate) ? Yc[j] : 0.0;
        double ypv[NPM];
#pragma unroll
        for (int i = 0; i < NPM; ++i) {
            ypv[i] = 0.0;
            if (i < n_p) {
                const int P = Ap[(size_t)s * n_p + i];
                if (P >= 0) ypv[i] = zP[P];
            }
        }
#pragma unroll
        for (int i = 0; i < NPM; ++i)
            if (i < n_p) v += cv[i] * ypv[i];
        if (in) Yc[j] = v;
        return;
    }
    double yp[NPM];
#pragma unroll
    for (int i = 0; i < NPM; ++i) {
        yp[i] = 0.0;
        if (i < n_p) {
            const int P = Ap[(size_t)s * n_p + i];
            if (P >= 0) yp[i] = zP[P];
        }
    }
    for (int j = threadIdx.x; j < n_d; j += 64 * NWC) {
        double v = accumulate ? Yc[j] : 0.0;
#pragma unroll
        for (int i = 0; i < NPM; ++i)
            if (i < n_p) v += Cs[(size_t)i * n_d + j] * yp[i];
        Yc[j] = v;
    }
}

// ------------------------------------------------------------------ A_p, A_p^T
__global__ __launch_bounds__(kB) void k_assemble_primal(const int *__restrict__ pull, int maxc,
                                                        const double *__restrict__ cp, int N, int n_p,
                                                        const double *__restrict__ base, long long b_rs, double sgn,
                                                        double *__restrict__ zP, long long z_rs, int nP, int nrhs) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)nP * nrhs) return;
    int rhs = (int)(t / nP), P = (int)(t % nP);
    double v = 0.0;
    for (int u = 0; u < maxc; ++u) {
        int e = pull[(size_t)P * maxc + u];
        if (e < 0) break;
        v += cp[((size_t)rhs * N) * n_p + e];
    }
    double b = base ? base[rhs * b_rs + P] : 0.0;
    zP[rhs * z_rs + P] = b + sgn * v;
}

// the same for a fixed number of contributions per primal dof (2^dim): every pull entry and every
// contribution is loaded before the first is added (two dependent loads per thread instead of
// 2 MAXC), the sum taken in the same order; one wave per block spreads the few rows over more CUs
template <int MAXC>
__global__ __launch_bounds__(64) void k_assemble_primal_t(const int *__restrict__ pull, const double *__restrict__ cp,
                                                          int N, int n_p, const double *__restrict__ base,
                                                          long long b_rs, double sgn, double *__restrict__ zP,
                                                          long long z_rs, int nP, int nrhs) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)nP * nrhs) return;
    int rhs = (int)(t / nP), P = (int)(t % nP);
    int e[MAXC];
#pragma unroll
    for (int u = 0; u < MAXC; ++u) e[u] = pull[(size_t)P * MAXC + u];
    bool live[MAXC];
    double x[MAXC];
#pragma unroll
    for (int u = 0; u < MAXC; ++u) {
        live[u] = e[u] >= 0 && (u == 0 || live[u - 1]);  // a list ends at its first negative entry
        x[u] = live[u] ? cp[((size_t)rhs * N) * n_p + e[u]] : 0.0;
    }
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < MAXC; ++u)
        if (live[u]) v += x[u];
    double b = base ? base[rhs * b_rs + P] : 0.0;
    zP[rhs * z_rs + P] = b + sgn * v;
}

__global__ __launch_bounds__(kB) void k_restrict_primal(const int *__restrict__ Ap, const double *__restrict__ xP,
                                                        long long x_rs, double *__restrict__ xp, int N, int n_p,
                                                        int nrhs) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long per = (long long)N * n_p;
    if (t >= per * nrhs) return;
    int rhs = (int)(t / per);
    int P = Ap[t % per];
    xp[t] = P >= 0 ? xP[rhs * x_rs + P] : 0.0;
}

// ------------------------------------------------------------------ coarse solve, symmetric tiles
typedef double v2d __attribute__((ext_vector_type(2)));

// y = scale * S z with S = S̊_PP^-1 stored as its lower-triangle 64x64 tiles.
// Pass 1, one workgroup per tile (I, J), streamed with non-temporal loads so
// the L2-resident principal operators of the concurrent contraction stay
// cached: each thread owns 4 rows x 4 columns; the row partial S_IJ z_J and,
// off the diagonal, the column partial S_IJ^T z_I are reduced with lane
// shuffles and LDS in a fixed order and written per tile.  Pass 2 sums, for every row of block I, the row partials
// of tiles (I, 0..I) and the column partials of tiles (I+1..nT-1, I) in that
// fixed order (bitwise reproducible, no atomics).
template <int NR>
__global__ __launch_bounds__(256) void k_sym_tiles(const double *__restrict__ T, const int *__restrict__ tiles, int n,
                                                   const double *__restrict__ z, long long z_rs,
                                                   double *__restrict__ P) {
    __shared__ double red[NR][4][64];
    const int tile = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int I = tiles[2 * tile], J = tiles[2 * tile + 1];
    // thread owns rows 4a + i and columns cidx(j) = 2b + (j & 1) + 32 (j >> 1): each
    // 16-byte load instruction covers 4 rows x 256 contiguous bytes per wave
    const int a = tid >> 4, b = tid & 15;
    double S[4][4];
    const double *src = T + (size_t)tile * 4096;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const v2d v0 = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(src + (4 * a + i) * 64 + 2 * b));
        const v2d v1 = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(src + (4 * a + i) * 64 + 32 + 2 * b));
        S[i][0] = v0.x;
        S[i][1] = v0.y;
        S[i][2] = v1.x;
        S[i][3] = v1.y;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const double *zq = z + q * z_rs;
        double zJ[4], zI[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cJ = J * 64 + 2 * b + (j & 1) + 32 * (j >> 1), rI = I * 64 + 4 * a + j;
            zJ[j] = cJ < n ? zq[cJ] : 0.0;
            zI[j] = rI < n ? zq[rI] : 0.0;
        }
        double pr[4], pc[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            pr[i] = ((S[i][0] * zJ[0] + S[i][1] * zJ[1]) + S[i][2] * zJ[2]) + S[i][3] * zJ[3];
            pc[i] = ((S[0][i] * zI[0] + S[1][i] * zI[1]) + S[2][i] * zI[2]) + S[3][i] * zI[3];
        }
        // row partials: sum over the 16 column groups b (lanes of one 16-lane row)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1)
#pragma unroll
            for (int i = 0; i < 4; ++i) pr[i] += __shfl_xor(pr[i], off);
        double *Pt = P + ((size_t)tile * NR + q) * 128;
        if (b == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) Pt[4 * a + i] = pr[i];
        if (I != J) {
            // column partials: sum over the 16 row groups a (4 per wave, then the 4 waves)
#pragma unroll
            for (int off = 16; off < 64; off <<= 1)
#pragma unroll
                for (int j = 0; j < 4; ++j) pc[j] += __shfl_xor(pc[j], off);
            if (lane < 16)
#pragma unroll
                for (int j = 0; j < 4; ++j) red[q][wave][2 * b + (j & 1) + 32 * (j >> 1)] = pc[j];
        }
    }
    if (I == J) return;  // uniform per workgroup
    __syncthreads();
    if (tid < 64)
#pragma unroll
        for (int q = 0; q < NR; ++q)
            P[((size_t)tile * NR + q) * 128 + 64 + tid] =
                ((red[q][0][tid] + red[q][1][tid]) + red[q][2][tid]) + red[q][3][tid];
}

// Partitioned coarse solve, one phase: row w < nrows (WPR waves per row, 256/(64 WPR) rows per
// workgroup) computes R = rows[w],
//   y[q][R.out] = alpha * dot,  y2[q][R.out] = alpha2 * dot (if y2),  dot = M[R.off + c] x[q][R.xlo + c]
// summed over c < R.len (thread t of the row takes c = t mod 64 WPR in increasing c, then a fixed
// butterfly within each wave and the waves in order), for NR load cases at once.  The operator rows
// are read with ordinary loads: nothing runs beside these phases, and the three phases' rows (about
// 80 MB on the 2D 64x64-cell lattice) then stay in the last-level cache from one F̊ apply to the next
// (c2 solve 111.3 -> 108.7 ms against non-temporal loads).  Rows w >= nrows copy cz to cw (ncopy
// entries per load case), which phase 1 uses to assemble the phase-3 input.
template <int NR, int WPR>
__global__ __launch_bounds__(256) void k_coarse_rows(const double *__restrict__ M, const CoarseRow *__restrict__ rows,
                                                     int nrows, const double *__restrict__ x, long long x_rs,
                                                     double alpha, double *__restrict__ y, long long y_rs,
                                                     double alpha2, double *__restrict__ y2, long long y2_rs,
                                                     const double *__restrict__ cz, long long cz_rs,
                                                     double *__restrict__ cw, long long cw_rs, int ncopy) {
    constexpr int RT = 64 * WPR;        // threads per row
    constexpr int RPB = 256 / RT;       // rows per workgroup
    __shared__ double red[4][NR];
    const int w = blockIdx.x * RPB + threadIdx.x / RT, t = threadIdx.x % RT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool dot = w < nrows;  // uniform per row (whole waves)
    if (!dot) {
        const long long e = (long long)(w - nrows) * RT + t;
        if (e < ncopy)
#pragma unroll
            for (int q = 0; q < NR; ++q) cw[q * cw_rs + e] = cz[q * cz_rs + e];
    }
    const CoarseRow R = dot ? rows[w] : CoarseRow{0, 0, 0, 0, 0};
    const double *m = M + R.off;
    double acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = 0.0;
    // batches of 8 predicated loads per thread, all issued before the first is used
    for (int c = t; c < R.len; c += 8 * RT) {
        double a[8], xv[8][NR];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int cc = c + RT * u;
            a[u] = cc < R.len ? m[cc] : 0.0;
#pragma unroll
            for (int q = 0; q < NR; ++q) xv[u][q] = cc < R.len ? x[q * x_rs + R.xlo + cc] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < NR; ++q) acc[q] += a[u] * xv[u][q];
    }
#pragma unroll
    for (int q = 0; q < NR; ++q)
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
    if constexpr (WPR > 1) {
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < NR; ++q) red[wave][q] = acc[q];
        __syncthreads();  // reached by every thread of the workgroup (no early exits above)
        if (!dot || t != 0) return;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            double s = red[wave][q];
#pragma unroll
            for (int v = 1; v < WPR; ++v) s += red[wave + v][q];
            acc[q] = s;
        }
    } else if (!dot || lane != 0) {
        return;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        y[q * y_rs + R.out] = alpha * acc[q];
        if (y2) y2[q * y2_rs + R.out] = alpha2 * acc[q];
    }
}

typedef double v4d __attribute__((ext_vector_type(4)));

// The same phase rows for a block of load cases, as FP64 MFMA tiles: one workgroup of four waves per
// tile of up to 16 rows sharing their input range, output [16 rows] x [16 NT load cases]; the waves
// take every fourth 16-column step of the range (a phase has only about a hundred tiles, each a few
// hundred KB of rows) and their partial tiles are added in wave order through LDS.  The k index of the
// 16x16x4 product is assigned so that lane (lr, lk) of step t takes column c + 4 lk + t: each lane then
// walks four consecutive entries of its row of M and of its load case's input.  Workgroups past the
// tiles copy cz into cw (ncopy entries per load case) as the row form does.
template <int NT>
__global__ __launch_bounds__(256) void k_coarse_tiles(const double *__restrict__ M, const CoarseRow *__restrict__ rows,
                                                      const CoarseTile *__restrict__ tiles, int ntiles,
                                                      const double *__restrict__ x, long long x_rs, double alpha,
                                                      double *__restrict__ y, long long y_rs, double alpha2,
                                                      double *__restrict__ y2, long long y2_rs,
                                                      const double *__restrict__ cz, long long cz_rs,
                                                      double *__restrict__ cw, long long cw_rs, int ncopy, int nrhs) {
    constexpr int WPT = 4;
    __shared__ double part[WPT][NT][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((int)blockIdx.x >= ntiles) {  // the copy: whole workgroups, before any barrier
        const long long e = (long long)(blockIdx.x - ntiles) * 256 + threadIdx.x;
        if (e < (long long)ncopy * nrhs) {
            const int q = (int)(e / ncopy);
            const long long i = e % ncopy;
            cw[q * cw_rs + i] = cz[q * cz_rs + i];
        }
        return;
    }
    const CoarseTile T = tiles[blockIdx.x];
    const CoarseRow R0 = rows[T.row0];
    const int lr = lane & 15, lk = lane >> 4;
    const bool rowok = lr < T.nrows;
    const double *m = M + R0.off + (size_t)(rowok ? lr : 0) * R0.len;
    const double *xb = x + R0.xlo;
    v4d acc[NT];
    bool qok[NT];
    const double *xq[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
        const int q = 16 * j + lr;
        qok[j] = q < nrhs;
        xq[j] = xb + (size_t)(qok[j] ? q : 0) * x_rs;
    }
    const int len = R0.len;
    for (int c = 16 * wave; c < len; c += 16 * WPT) {  // uniform per wave: the MFMA needs all 64 lanes
        double a[4], b[NT][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int cc = c + 4 * lk + t;
            const bool in = cc < len;
            a[t] = rowok && in ? m[cc] : 0.0;
#pragma unroll
            for (int j = 0; j < NT; ++j) b[j][t] = qok[j] && in ? xq[j][cc] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[j][t], acc[j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) part[wave][j][i][lane] = acc[j][i];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = 4 * i + lk;
        if (row >= T.nrows) continue;
        const int out = rows[T.row0 + row].out;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int q = 16 * j + lr;
            if (q >= nrhs) continue;
            double sum = part[0][j][i][lane];
#pragma unroll
            for (int w = 1; w < WPT; ++w) sum += part[w][j][i][lane];
            y[q * y_rs + out] = alpha * sum;
            if (y2) y2[q * y2_rs + out] = alpha2 * sum;
        }
    }
}

// one workgroup per (block row I, load case): thread (part, r) sums the
// contributions J = part, part + 16, ... of row r; the 16 parts are added in
// order through LDS
__global__ __launch_bounds__(1024) void k_sym_reduce(const double *__restrict__ P, int n, int nT, int NR,
                                                     double *__restrict__ y, long long y_rs, double scale) {
    __shared__ double part_s[16][64];
    const int I = blockIdx.x, q = blockIdx.y, tid = threadIdx.x;
    const int r = tid & 63, part = tid >> 6;
    const size_t base = (size_t)I * (I + 1) / 2;
    double s = 0.0;
#pragma unroll 4
    for (int J = part; J < nT; J += 16) {
        const size_t off = J <= I ? ((base + J) * NR + q) * 128 + r
                                  : (((size_t)J * (J + 1) / 2 + I) * NR + q) * 128 + 64 + r;
        s += P[off];
    }
    part_s[part][r] = s;
    __syncthreads();
    const int row = I * 64 + tid;
    if (tid < 64 && row < n) {
        double t = part_s[0][tid];
#pragma unroll
        for (int p = 1; p < 16; ++p) t += part_s[p][tid];
        y[q * y_rs + row] = scale * t;
    }
}


// ------------------------------------------------------------------ reduced local solve (46)
// Column c = rhs*N + s.  R_c holds the K reduced-basis vectors
// K_rr^(sigma_k)^-1 v as [r][k] (the K values of one row contiguous).  The Gram matrix
// G = R^T K_rr^(s) R uses the cell's own stencil values; G c = R^T v is solved
// by Cholesky (symmetric pseudo-inverse with a 1e-13 relative cut if a pivot
// fails) and x = R c is written.

// (46b) step 1: H_c = K_rr^(s) R for a chunk of KCOL reduced-basis vectors.
// One workgroup per column c; the chunk of R (n_r x KCOL, from the [r][k] layout) is staged in LDS
// (row-major with an odd row stride, plus a zero row that primal dofs map to) with
// the dof -> r-row map; one thread per control point a accumulates the
// d x KCOL block of H for the rows of a.  The stencil offsets are unrolled
// and branch-free: an out-of-range neighbour is clamped onto a itself, whose
// stencil value for that offset is stored as zero, so every stencil load
// (layout [o][i][k][a], coalesced over a) is in bounds and independent.
constexpr int kRomHB = 1024;

template <int D, int KCOL>
__global__ __launch_bounds__(kRomHB) void k_rom_H(const double *__restrict__ R, const double *__restrict__ Kst,
                                                  const int *__restrict__ r_of_dof, int N, int K, int k0, int n_r,
                                                  int nc, int n_ctrl, double *__restrict__ H) {
    constexpr int P = 2;                   // quadratic B-splines: neighbours within +-2
    constexpr int W = 2 * P + 1;
    constexpr int NOFF = D == 2 ? W * W : W * W * W;
    constexpr int KP = KCOL | 1;           // odd row stride: lanes reading neighbouring rows hit distinct banks
    extern __shared__ double Rl[];         // [n_r + 1][KP], then int rmap[n_ctrl * D]
    const int col = blockIdx.x, s = col % N, tid = threadIdx.x, nt = blockDim.x;
    int *rmap = reinterpret_cast<int *>(Rl + (size_t)(n_r + 1) * KP);
    const double *Rc = R + (size_t)col * K * n_r;
    const int kc = min(KCOL, K - k0);
    for (int e = tid; e < (n_r + 1) * KCOL; e += nt) {
        const int r = e / KCOL, kk = e % KCOL;
        Rl[r * KP + kk] = (kk < kc && r < n_r) ? Rc[(size_t)r * K + k0 + kk] : 0.0;
    }
    for (int e = tid; e < n_ctrl * D; e += nt) {
        const int rr = r_of_dof[e];
        rmap[e] = rr >= 0 ? rr : n_r;
    }
    __syncthreads();
    const double *Ks = Kst + (size_t)s * n_ctrl * NOFF * D * D;
    double *Hc = H + (size_t)col * K * n_r;
    double hsave[D][KCOL];
    int arow = -1;
    for (int a = tid; a < n_ctrl; a += nt) {  // one control point per thread (blockDim >= n_ctrl)
        int ma[D], stride[D];
        {
            int ta = a, st = 1;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                ma[j] = ta % nc;
                ta /= nc;
                stride[j] = st;
                st *= nc;
            }
        }
        double h[D][KCOL];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int q = 0; q < KCOL; ++q) h[i][q] = 0.0;
#pragma unroll W
        for (int o = 0; o < NOFF; ++o) {
            int b = a;
            bool ok = true;
            {
                int to = o;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int d = to % W - P;
                    to /= W;
                    const int m = ma[j] + d;
                    ok = ok && m >= 0 && m < nc;
                    b += d * stride[j];
                }
            }
            if (!ok) b = a;  // stencil value stored as zero for this offset
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double *row = Rl + rmap[b * D + k] * KP;
                double kv[D];
#pragma unroll
                for (int i = 0; i < D; ++i) kv[i] = Ks[(((size_t)o * D + i) * D + k) * n_ctrl + a];
#pragma unroll
                for (int q = 0; q < KCOL; ++q) {
                    const double rq = row[q];
#pragma unroll
                    for (int i = 0; i < D; ++i) h[i][q] += kv[i] * rq;
                }
            }
        }
        // park this control point's rows until every thread has finished reading R
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int q = 0; q < KCOL; ++q) hsave[i][q] = h[i][q];
        arow = a;
    }
    __syncthreads();  // R no longer needed: reuse its LDS rows for H ([r][KP])
    if (arow >= 0)
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int ri = r_of_dof[arow * D + i];
            if (ri < 0) continue;
#pragma unroll
            for (int q = 0; q < KCOL; ++q) Rl[ri * KP + q] = hsave[i][q];
        }
    __syncthreads();
    for (int e = tid; e < n_r * KCOL; e += nt) {  // coalesced: [r][k0 .. k0+kc) of H
        const int r = e / KCOL, kk = e % KCOL;
        if (kk < kc) Hc[(size_t)r * K + k0 + kk] = Rl[r * KP + kk];
    }
}

// Cholesky A = L L^T of a symmetric K x K matrix (row-major) by one lane; false at the first
// pivot that is not positive.
__device__ bool small_chol(const double *A, double *Lm, int K) {
    for (int j = 0; j < K; ++j) {
        double sj = A[j * K + j];
        for (int k = 0; k < j; ++k) sj -= Lm[j * K + k] * Lm[j * K + k];
        if (!(sj > 0.0)) return false;
        double l = sqrt(sj);
        Lm[j * K + j] = l;
        for (int i = j + 1; i < K; ++i) {
            double t = A[i * K + j];
            for (int k = 0; k < j; ++k) t -= Lm[i * K + k] * Lm[j * K + k];
            Lm[i * K + j] = t / l;
        }
    }
    return true;
}

// Cyclic Jacobi eigen-decomposition by one lane: A is diagonalised in place (eigenvalues on the
// diagonal), V holds the eigenvectors as columns.
__device__ void small_sym_jacobi(double *A, double *V, int K) {
    for (int i = 0; i < K * K; ++i) V[i] = 0.0;
    for (int i = 0; i < K; ++i) V[i * K + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j) {
                double a = A[i * K + j];
                tot += a * a;
                if (i != j) off += a * a;
            }
        if (off <= 1e-30 * tot) break;
        for (int pp = 0; pp < K; ++pp)
            for (int q = pp + 1; q < K; ++q) {
                double apq = A[pp * K + q];
                if (apq == 0.0) continue;
                double th = (A[q * K + q] - A[pp * K + pp]) / (2.0 * apq);
                double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < K; ++k) {
                    double akp = A[k * K + pp], akq = A[k * K + q];
                    A[k * K + pp] = cs * akp - sn * akq;
                    A[k * K + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < K; ++k) {
                    double apk = A[pp * K + k], aqk = A[q * K + k];
                    A[pp * K + k] = cs * apk - sn * aqk;
                    A[q * K + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < K; ++k) {
                    double vkp = V[k * K + pp], vkq = V[k * K + q];
                    V[k * K + pp] = cs * vkp - sn * vkq;
                    V[k * K + q] = sn * vkp + cs * vkq;
                }
            }
    }
}

// Small dense solve by one lane: x = A^-1 b for symmetric A (K x K, row-major).
// Cholesky; if a pivot is not positive, a cyclic Jacobi eigen-decomposition
// gives the pseudo-inverse with a 1e-13 relative cut.
__device__ void small_sym_solve(double *A, double *Lm, double *V, const double *b, double *x, int K) {
    if (small_chol(A, Lm, K)) {
        for (int i = 0; i < K; ++i) {
            double t = b[i];
            for (int k = 0; k < i; ++k) t -= Lm[i * K + k] * x[k];
            x[i] = t / Lm[i * K + i];
        }
        for (int i = K - 1; i >= 0; --i) {
            double t = x[i];
            for (int k = i + 1; k < K; ++k) t -= Lm[k * K + i] * x[k];
            x[i] = t / Lm[i * K + i];
        }
        return;
    }
    small_sym_jacobi(A, V, K);
    double wmax = 0.0;
    for (int i = 0; i < K; ++i) wmax = fmax(wmax, A[i * K + i]);
    for (int i = 0; i < K; ++i) x[i] = 0.0;
    for (int k = 0; k < K; ++k) {
        double wk = A[k * K + k];
        if (!(wk > 1e-13 * wmax)) continue;
        double proj = 0.0;
        for (int i = 0; i < K; ++i) proj += V[i * K + k] * b[i];
        proj /= wk;
        for (int i = 0; i < K; ++i) x[i] += proj * V[i * K + k];
    }
}

constexpr int kMaxK = 40;

// (46b) step 2, one wave64 per column c: [G | g] = R^T [H | v] on the FP64 MFMA
// (A fragment R^T: lane l -> basis vector l%16, rows 4t + l/16; B fragment
// [H | v]: rows 4t + l/16, column l%16), then G c = g by lane 0 and x = R c.
// G is symmetric up to rounding; its upper triangle is mirrored.  KB =
// 16-blocks of the padded (K + 1) dimension, WPB = waves per workgroup; each
// wave owns 3K^2 + 2K doubles of dynamic LDS (G, Cholesky factor, eigenvector
// scratch, right-hand side, coefficients).
template <int KB, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_rom_gram(const double *__restrict__ vR, long long v_rs,
                                                       const double *__restrict__ R, const double *__restrict__ H,
                                                       int N, int ncols, int K, int n_r, double *__restrict__ xR,
                                                       long long x_rs) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = blockIdx.x * WPB + wave;
    const bool active = col < ncols;
    const int rhs = col / N, s = col % N;
    const int lr = lane & 15, lk = lane >> 4;
    const double *Rc = R + (size_t)col * K * n_r;
    const double *Hc = H + (size_t)col * K * n_r;
    double *A = lds + (size_t)wave * (3 * K * K + 2 * K);
    double *Lm = A + K * K, *Vm = Lm + K * K, *rhsb = Vm + K * K, *cv = rhsb + K;
    if (active) {
        const double *v = vR + rhs * v_rs + (size_t)s * n_r;
        v4d acc[KB][KB];
#pragma unroll
        for (int a = 0; a < KB; ++a)
#pragma unroll
            for (int b = 0; b < KB; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
        const int nt4 = (n_r + 3) / 4;
        for (int t = 0; t < nt4; ++t) {  // uniform trip count: the MFMA needs all 64 lanes
            const int r = 4 * t + lk;
            const bool rin = r < n_r;
            double af[KB], bf[KB];
#pragma unroll
            for (int a = 0; a < KB; ++a) {
                const int k1 = 16 * a + lr;
                af[a] = (rin && k1 < K) ? Rc[(size_t)r * K + k1] : 0.0;
                bf[a] = !rin ? 0.0 : (k1 < K ? Hc[(size_t)r * K + k1] : (k1 == K ? v[r] : 0.0));
            }
#pragma unroll
            for (int a = 0; a < KB; ++a)
#pragma unroll
                for (int b = 0; b < KB; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < KB; ++a)
#pragma unroll
            for (int b = 0; b < KB; ++b)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * a + 4 * i + lk, cc = 16 * b + lr;
                    if (row >= K) continue;
                    if (cc == K) rhsb[row] = acc[a][b][i];
                    else if (row <= cc && cc < K) {
                        A[row * K + cc] = acc[a][b][i];
                        A[cc * K + row] = acc[a][b][i];
                    }
                }
    }
    __syncthreads();
    if (active && lane == 0) small_sym_solve(A, Lm, Vm, rhsb, cv, K);
    __syncthreads();
    if (active) {
        double *x = xR + rhs * x_rs + (size_t)s * n_r;
        for (int r = lane; r < n_r; r += 64) {
            double t = 0.0;
            for (int k = 0; k < K; ++k) t += Rc[(size_t)r * K + k] * cv[k];
            x[r] = t;
        }
    }
}

// (46b) fused, one workgroup per column (cell s, load case): H = K_rr^(s) R is formed chunk by chunk
// in LDS and never stored; as each chunk of H appears, the waves add its share of
// [G | g] = R^T [H | v] on the FP64 MFMA (rows of R split across waves, partial tiles summed in wave
// order), then the block solves G c = g and writes x = R c.  H takes the place of the staged chunk of R,
// so the Gram product and the combination read R again (from L2 or the last-level cache); keeping both
// resident halves the workgroups per CU and measured slower.  K <= 16, one 16 x 16 tile of [G | g]:
// a chunk has at most 15 columns, so column kc of the first chunk carries R^T v.
template <typename TR, int D, int KCOL>
__global__ __launch_bounds__(kRomHB) void k_rom_local(const TR *__restrict__ R, const double *__restrict__ Kst,
                                                      const int *__restrict__ r_of_dof,
                                                      const double *__restrict__ vR, long long v_rs, int N,
                                                      int nrhs, int K, int n_r, int nc, int n_ctrl,
                                                      double *__restrict__ xR, long long x_rs) {
    constexpr int P = 2;  // quadratic B-splines: neighbours within +-2
    constexpr int W = 2 * P + 1;
    constexpr int NOFF = D == 2 ? W * W : W * W * W;
    constexpr int KP = KCOL | 1;  // odd row stride: lanes reading neighbouring rows hit distinct banks
    static_assert(KCOL <= 15, "column KCOL of the Gram tile carries R^T v");
    extern __shared__ double lds[];
    // the load cases of a cell together on one XCD, whose L2 serves them the cell's stencil
    int s, rhs;
    if (!cell_of_block(blockIdx.x, N, nrhs, s, rhs)) return;  // whole workgroup, before any barrier
    const int col = rhs * N + s, tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    // [D n_ctrl + 1][KP] a chunk of R in R's own precision (FP32 in the precision form: half the LDS
    // reads of the stencil loop), its rows component-major (slot k n_ctrl + a for component k of control
    // point a, the last slot zero): the lanes of the stencil loop, consecutive control points, then read
    // rows KP apart, an odd number of banks (with the dof order they were D KP apart and hit each bank
    // twice); then H of the chunk over the same bytes in the order of R, also in R's precision (FP32 in
    // the precision form: half the LDS of a workgroup, three workgroups per CU in 2D instead of two),
    // then the wave partials in FP64
    const int zslot = D * n_ctrl;
    const size_t rows = (size_t)(zslot + 1) * KP;
    TR *Rl = reinterpret_cast<TR *>(lds);
    TR *Hl = Rl;
    double *G = reinterpret_cast<double *>(reinterpret_cast<char *>(lds) + ((rows * sizeof(TR) + 15) & ~(size_t)15));
    // G: [K][K], a copy of it, two [K][K+1] work arrays, g [K], c [K]
    double *G0 = G + K * K, *W1 = G0 + K * K, *W2 = W1 + K * (K + 1), *gb = W2 + K * (K + 1), *cv = gb + K;
    int *rmap = reinterpret_cast<int *>(cv + K);  // [n_ctrl][D]: row of R, or n_r for none
    int *rslot = rmap + n_ctrl * D;               // [n_r + 1]: LDS slot of each row of R, the zero row last
    const TR *Rc = R + (size_t)col * K * n_r;
    const double *v = vR + (size_t)rhs * v_rs + (size_t)s * n_r;
    const double *Ks = Kst + (size_t)s * n_ctrl * NOFF * D * D;
    for (int e = tid; e < n_ctrl * D; e += nt) {
        const int rr = r_of_dof[e];
        rmap[e] = rr >= 0 ? rr : n_r;
        if (rr >= 0) rslot[rr] = (e % D) * n_ctrl + e / D;
    }
    if (tid == 0) rslot[n_r] = zslot;
    __syncthreads();
    for (int k0 = 0; k0 < K; k0 += KCOL) {
        const int kc = min(KCOL, K - k0);
        const int tot = (n_r + 1) * KCOL;
        // four loads in flight per thread, then the stores (c2: 661 us against 705 with one; the Gram loop
        // below unrolled the same way ran out of registers and slowed to 774 us)
        constexpr int SU = 4;
        for (int e0 = tid; e0 < tot; e0 += SU * nt) {
            TR tmp[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int e = e0 + u * nt, r = e / KCOL, kk = e % KCOL;
                tmp[u] = (e < tot && kk < kc && r < n_r) ? Rc[(size_t)r * K + k0 + kk] : (TR)0;
            }
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int e = e0 + u * nt;
                if (e < tot) Rl[rslot[e / KCOL] * KP + e % KCOL] = tmp[u];
            }
        }
        __syncthreads();
        double h[D][KCOL];
        const int a = tid;  // one control point per thread (blockDim >= n_ctrl)
        if (a < n_ctrl) {
            int ma[D], stride[D];
            {
                int ta = a, st = 1;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    ma[j] = ta % nc;
                    ta /= nc;
                    stride[j] = st;
                    st *= nc;
                }
            }
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int q = 0; q < KCOL; ++q) h[i][q] = 0.0;
#pragma unroll W
            for (int o = 0; o < NOFF; ++o) {
                int b = a;
                bool ok = true;
                {
                    int to = o;
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        const int d = to % W - P;
                        to /= W;
                        const int m = ma[j] + d;
                        ok = ok && m >= 0 && m < nc;
                        b += d * stride[j];
                    }
                }
                if (!ok) b = a;  // stencil value stored as zero for this offset
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const TR *row = Rl + (rmap[b * D + k] < n_r ? k * n_ctrl + b : zslot) * KP;
                    double kv[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) kv[i] = Ks[(((size_t)o * D + i) * D + k) * n_ctrl + a];
#pragma unroll
                    for (int q = 0; q < KCOL; ++q) {
                        const double rq = (double)row[q];
#pragma unroll
                        for (int i = 0; i < D; ++i) h[i][q] += kv[i] * rq;
                    }
                }
            }
        }
        __syncthreads();  // every thread has read the chunk of R before H takes its place
        if (a < n_ctrl)
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int ri = rmap[a * D + i];
                if (ri < n_r)
#pragma unroll
                    for (int q = 0; q < KCOL; ++q) Hl[ri * KP + q] = (TR)h[i][q];
            }
        __syncthreads();
        // this chunk's columns of [G | g]: rows k = 4 i + lk, column q = lr (q == kc: R^T v, first chunk)
        v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
        const int nt4 = (n_r + 3) / 4;
        for (int t = wave; t < nt4; t += nw) {  // uniform per wave: the MFMA needs all 64 lanes
            const int r = 4 * t + lk;
            const bool rin = r < n_r;
            const double af = (rin && lr < K) ? (double)Rc[(size_t)r * K + lr] : 0.0;
            const double bf = !rin ? 0.0 : (lr < kc ? (double)Hl[r * KP + lr] : (lr == kc && k0 == 0 ? v[r] : 0.0));
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, acc, 0, 0, 0);
        }
        __syncthreads();  // H read by every wave: its rows take the partial tiles
        double *part = lds;
#pragma unroll
        for (int i = 0; i < 4; ++i) part[(size_t)(wave * 4 + i) * 64 + lane] = acc[i];
        __syncthreads();
        if (tid < 256) {
            const int i = tid >> 6, l = tid & 63;
            const int k = 4 * i + (l >> 4), q = l & 15;
            double sum = 0.0;
            for (int w = 0; w < nw; ++w) sum += part[(size_t)(w * 4 + i) * 64 + l];
            if (k < K) {
                if (q < kc) G[k * K + k0 + q] = sum;
                else if (q == kc && k0 == 0) gb[k] = sum;
            }
        }
        __syncthreads();  // partials consumed before the next chunk is staged
    }
    for (int e = tid; e < K * K; e += nt) {  // the upper triangle, mirrored; a copy for the fallback
        const int i = e / K, j = e % K;
        G0[e] = G[e] = j < i ? G[j * K + i] : G[e];
    }
    __syncthreads();
    // G c = g by Gauss-Jordan elimination of [G | g] spread over the block, one thread per entry and
    // one barrier per pivot (the pivots of a symmetric positive definite matrix need no exchange; a
    // Cholesky factorisation with its two substitutions took four times the barriers, a one-lane solve
    // leaves the CU idle for tens of microseconds per column).  A pivot that is not positive hands the
    // copy to the one-lane solve with its eigen-decomposition fallback.
    const int K1 = K + 1;
    for (int e = tid; e < K * K1; e += nt) {
        const int i = e / K1, m = e % K1;
        W1[e] = m < K ? G[i * K + m] : gb[i];
    }
    __syncthreads();
    bool spd = true;
    double *src = W1, *dst = W2;
    for (int j = 0; j < K; ++j) {
        const double piv = src[j * K1 + j];  // the same value in every thread: a uniform branch
        if (!(piv > 0.0)) {
            spd = false;
            break;
        }
        for (int e = tid; e < K * K1; e += nt) {
            const int i = e / K1, m = e % K1;
            dst[e] = i == j ? src[e] / piv : src[e] - src[i * K1 + j] * (src[j * K1 + m] / piv);
        }
        __syncthreads();
        double *t = src;
        src = dst;
        dst = t;
    }
    if (spd) {
        if (tid < K) cv[tid] = src[tid * K1 + K];
    } else if (tid == 0) {
        small_sym_solve(G0, W1, W2, gb, cv, K);  // W1, W2: K x K workspaces of the fallback
    }
    __syncthreads();
    double *x = xR + (size_t)rhs * x_rs + (size_t)s * n_r;
    for (int r = tid; r < n_r; r += nt) {
        double t = 0.0;
        for (int k = 0; k < K; ++k) t += (double)Rc[(size_t)r * K + k] * cv[k];
        x[r] = t;
    }
}

// ------------------------------------------------------------------ K̊^-MPCG (Remark 6)
// Multi-preconditioned CG for the local problems K_rr^(s) x = v with the principal inverses as the K
// preconditioners.  Each iteration's block Z = [K_rr^(σk)-1 r]_k is whitened, Ẑ = Z T with
// Ẑᵀ K_rr^(s) Ẑ = I on the range of G = Zᵀ K_rr^(s) Z, so the energy minimisation is
// x += Ẑ Ẑᵀ r, r -= K Ẑ Ẑᵀ r (that is Z G^-1 Zᵀ r) and the conjugation of a later block against it
// is Z -= Ẑ (K Ẑ)ᵀ Z (that is P G^-1 (K P)ᵀ Z).  Cholesky gives T = L^-T; a pivot that is not positive
// switches to the Jacobi eigen-decomposition, T = V diag(w^-1/2) over the eigenvalues above 1e-13 of
// the largest (the pseudo-inverse of the reduced solve).

// T (K x K, row-major) with Tᵀ A T = I on the range of A; A is overwritten.  One lane.
__device__ void small_sym_whiten(double *A, double *Lm, double *V, double *T, int K) {
    if (small_chol(A, Lm, K)) {
        for (int i = 0; i < K * K; ++i) T[i] = 0.0;
        for (int j = 0; j < K; ++j) {  // column j of L^-1 is row j of T = L^-T
            T[j * K + j] = 1.0 / Lm[j * K + j];
            for (int i = j + 1; i < K; ++i) {
                double t = 0.0;
                for (int k = j; k < i; ++k) t += Lm[i * K + k] * T[j * K + k];
                T[j * K + i] = -t / Lm[i * K + i];
            }
        }
        return;
    }
    small_sym_jacobi(A, V, K);
    double wmax = 0.0;
    for (int i = 0; i < K; ++i) wmax = fmax(wmax, A[i * K + i]);
    for (int k = 0; k < K; ++k) {
        const double wk = A[k * K + k];
        const double sc = wk > 1e-13 * wmax ? 1.0 / sqrt(wk) : 0.0;
        for (int i = 0; i < K; ++i) T[i * K + k] = V[i * K + k] * sc;
    }
}

// acc = Aᵀ [B | b] over the n_r rows of one column (A, B: [r][k] with K columns; b optional), on the
// FP64 MFMA; the K x K block and the extra column are left in LDS (M row-major, m).
template <int KB>
__device__ __forceinline__ void col_gram(const double *__restrict__ Ac, const double *__restrict__ Bc,
                                         const double *__restrict__ bv, int K, int n_r, int lane, double *M,
                                         double *m) {
    const int lr = lane & 15, lk = lane >> 4;
    v4d acc[KB][KB];
#pragma unroll
    for (int a = 0; a < KB; ++a)
#pragma unroll
        for (int b = 0; b < KB; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    const int nt4 = (n_r + 3) / 4;
    for (int t = 0; t < nt4; ++t) {  // uniform trip count: the MFMA needs all 64 lanes
        const int r = 4 * t + lk;
        const bool rin = r < n_r;
        double af[KB], bf[KB];
#pragma unroll
        for (int a = 0; a < KB; ++a) {
            const int k1 = 16 * a + lr;
            af[a] = (rin && k1 < K) ? Ac[(size_t)r * K + k1] : 0.0;
            bf[a] = !rin ? 0.0 : (k1 < K ? Bc[(size_t)r * K + k1] : (k1 == K && bv ? bv[r] : 0.0));
        }
#pragma unroll
        for (int a = 0; a < KB; ++a)
#pragma unroll
            for (int b = 0; b < KB; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < KB; ++a)
#pragma unroll
        for (int b = 0; b < KB; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * a + 4 * i + lk, cc = 16 * b + lr;
                if (row >= K) continue;
                if (cc == K) m[row] = acc[a][b][i];
                else if (cc < K) M[row * K + cc] = acc[a][b][i];
            }
}

// One MPCG step per column (one wave each): G = Zᵀ KZ, g = Zᵀ r, T from G, â = Tᵀ g;
// P = Z T, KP = KZ T (stored for later conjugations), x (+)= P â, r -= KP â.
template <int KB, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_mpcg_step(const double *__restrict__ Z, const double *__restrict__ KZ,
                                                        double *__restrict__ r, double *__restrict__ xR,
                                                        long long x_rs, int first, double *__restrict__ P,
                                                        double *__restrict__ KP, int N, int ncols, int K,
                                                        int n_r) {
    constexpr int KM = 16 * KB;
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = blockIdx.x * WPB + wave;
    const bool active = col < ncols;
    const int rhs = col / N, s = col % N;
    double *G = lds + (size_t)wave * (4 * K * K + 2 * K);
    double *Lm = G + K * K, *Vm = Lm + K * K, *T = Vm + K * K, *g = T + K * K, *ah = g + K;
    const double *Zc = Z + (size_t)col * K * n_r, *KZc = KZ + (size_t)col * K * n_r;
    double *rc = r + (size_t)col * n_r;
    if (active) col_gram<KB>(Zc, KZc, rc, K, n_r, lane, G, g);
    __syncthreads();
    if (active && lane == 0) {
        for (int i = 0; i < K; ++i)  // symmetric from the upper triangle
            for (int j = i + 1; j < K; ++j) G[j * K + i] = G[i * K + j];
        small_sym_whiten(G, Lm, Vm, T, K);
        for (int b = 0; b < K; ++b) {
            double t = 0.0;
            for (int a = 0; a < K; ++a) t += T[a * K + b] * g[a];
            ah[b] = t;
        }
    }
    __syncthreads();
    if (!active) return;
    double *x = xR + rhs * x_rs + (size_t)s * n_r;
    double *Pc = P + (size_t)col * K * n_r, *KPc = KP + (size_t)col * K * n_r;
    for (int row = lane; row < n_r; row += 64) {
        double zh[KM], kh[KM];
#pragma unroll
        for (int b = 0; b < KM; ++b) zh[b] = kh[b] = 0.0;
        for (int a = 0; a < K; ++a) {
            const double za = Zc[(size_t)row * K + a], ka = KZc[(size_t)row * K + a];
#pragma unroll
            for (int b = 0; b < KM; ++b) {
                const double t = b < K ? T[a * K + b] : 0.0;
                zh[b] += za * t;
                kh[b] += ka * t;
            }
        }
        double xu = 0.0, ru = 0.0;
#pragma unroll
        for (int b = 0; b < KM; ++b) {
            if (b < K) {
                Pc[(size_t)row * K + b] = zh[b];
                KPc[(size_t)row * K + b] = kh[b];
                xu += zh[b] * ah[b];
                ru += kh[b] * ah[b];
            }
        }
        x[row] = first ? xu : x[row] + xu;
        rc[row] -= ru;
    }
}

// Conjugation of a new block against a stored whitened one: Z -= P (KPᵀ Z), one wave per column.
template <int KB, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_mpcg_conj(double *__restrict__ Z, const double *__restrict__ P,
                                                        const double *__restrict__ KP, int ncols, int K, int n_r) {
    constexpr int KM = 16 * KB;
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = blockIdx.x * WPB + wave;
    const bool active = col < ncols;
    double *C = lds + (size_t)wave * (K * K + K);
    double *Zc = Z + (size_t)col * K * n_r;
    const double *Pc = P + (size_t)col * K * n_r, *KPc = KP + (size_t)col * K * n_r;
    if (active) col_gram<KB>(KPc, Zc, nullptr, K, n_r, lane, C, C + K * K);
    __syncthreads();
    if (!active) return;
    for (int row = lane; row < n_r; row += 64) {
        double d[KM];
#pragma unroll
        for (int b = 0; b < KM; ++b) d[b] = 0.0;
        for (int a = 0; a < K; ++a) {
            const double pa = Pc[(size_t)row * K + a];
#pragma unroll
            for (int b = 0; b < KM; ++b) d[b] += pa * (b < K ? C[a * K + b] : 0.0);
        }
#pragma unroll
        for (int b = 0; b < KM; ++b)
            if (b < K) Zc[(size_t)row * K + b] -= d[b];
    }
}

// ------------------------------------------------------------------ true cell operator (16)
// y_R = K_rr u_r + K_rp u_p + B_r^T lam ;  yp (per cell) = K_pr u_r + K_pp u_p
template <int D, int NRB>
__global__ __launch_bounds__(kB) void k_true_K(const double *__restrict__ Kst, const double *__restrict__ x,
                                               long long x_rs, long long nU, const int *__restrict__ Ap,
                                               const int *__restrict__ idx_r, const int *__restrict__ idx_p,
                                               const int *__restrict__ r_of_dof, const int *__restrict__ p_of_dof,
                                               const int *__restrict__ gl, int N, int n_r, int n_p, int n_i,
                                               int n_d, int nc, int n_ctrl, int n_off, int p,
                                               double *__restrict__ y, long long y_rs,
                                               double *__restrict__ yp_cells, int nrhs) {
    extern __shared__ double uloc[];  // [NRB][n_dof]
    // NRB load cases per workgroup share every stencil value they read; the groups of a cell run
    // together on one XCD, whose L2 serves them the cell's stencil
    const int ngroups = (nrhs + NRB - 1) / NRB;
    int s, grp;
    if (!cell_of_block(blockIdx.x, N, ngroups, s, grp)) return;  // whole workgroup, before any barrier
    const int r0 = grp * NRB, nq = min(NRB, nrhs - r0);
    const int tid = threadIdx.x;
    const int n_dof = n_ctrl * D;
    for (int q = 0; q < nq; ++q) {
        const double *u = x + (r0 + q) * x_rs;
        double *ul = uloc + (size_t)q * n_dof;
        for (int i = tid; i < n_r; i += kB) ul[idx_r[i]] = u[(size_t)s * n_r + i];
        for (int j = tid; j < n_p; j += kB) {
            int P = Ap[(size_t)s * n_p + j];
            ul[idx_p[j]] = P >= 0 ? u[(size_t)N * n_r + P] : 0.0;
        }
    }
    __syncthreads();
    const int w = 2 * p + 1;
    const double *Ks = Kst + (size_t)s * n_ctrl * n_off * D * D;
    for (int t = tid; t < n_dof; t += kB) {
        const int i = t / n_ctrl, a = t % n_ctrl;
        const int row = a * D + i;
        int ma[D];
        int ta = a;
        for (int j = 0; j < D; ++j) {
            ma[j] = ta % nc;
            ta /= nc;
        }
        double acc[NRB];
#pragma unroll
        for (int q = 0; q < NRB; ++q) acc[q] = 0.0;
        for (int o = 0; o < n_off; ++o) {
            int to = o, b = 0;
            bool ok = true;
            int mb[D];
            for (int j = 0; j < D; ++j) {
                mb[j] = ma[j] + (to % w) - p;
                to /= w;
                if (mb[j] < 0 || mb[j] >= nc) ok = false;
            }
            if (!ok) continue;
            for (int j = D - 1; j >= 0; --j) b = b * nc + mb[j];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double kv = Ks[(((size_t)o * D + i) * D + k) * n_ctrl + a];
#pragma unroll
                for (int q = 0; q < NRB; ++q)
                    if (NRB == 1 || q < nq) acc[q] += kv * uloc[(size_t)q * n_dof + b * D + k];
            }
        }
        const int rp = r_of_dof[row];
        for (int q = 0; q < nq; ++q) {
            const int rhs = r0 + q, col = rhs * N + s;
            double v = acc[q];
            if (rp >= 0) {
                if (rp >= n_i) {  // dual dof: add B_d^T lam
                    const double *lam = x + rhs * x_rs + nU;
                    int j = rp - n_i;
#pragma unroll
                    for (int t2 = 0; t2 < 2; ++t2) {
                        int code = gl[((size_t)s * n_d + j) * 2 + t2];
                        if (code == 0) continue;
                        double lv = lam[(code > 0 ? code : -code) - 1];
                        v += code > 0 ? lv : -lv;
                    }
                }
                y[rhs * y_rs + (size_t)s * n_r + rp] = v;
            } else {
                yp_cells[(size_t)col * n_p + p_of_dof[row]] = v;
            }
        }
    }
}

// y_s = K^(s) x_s over all n_dof rows of every cell (stencil values; one workgroup per cell)
template <int D>
__global__ __launch_bounds__(kB) void k_cell_matvec_full(const double *__restrict__ Kst, const double *__restrict__ x,
                                                         int nc, int n_ctrl, int n_off, int p,
                                                         double *__restrict__ y) {
    const int s = blockIdx.x;
    const int n_dof = n_ctrl * D, w = 2 * p + 1;
    const double *xs = x + (size_t)s * n_dof;
    const double *Ks = Kst + (size_t)s * n_ctrl * n_off * D * D;
    for (int t = threadIdx.x; t < n_dof; t += kB) {
        const int i = t / n_ctrl, a = t % n_ctrl;
        int ma[D];
        int ta = a;
        for (int j = 0; j < D; ++j) {
            ma[j] = ta % nc;
            ta /= nc;
        }
        double acc = 0.0;
        for (int o = 0; o < n_off; ++o) {
            int to = o, b = 0;
            bool ok = true;
            int mb[D];
            for (int j = 0; j < D; ++j) {
                mb[j] = ma[j] + (to % w) - p;
                to /= w;
                if (mb[j] < 0 || mb[j] >= nc) ok = false;
            }
            if (!ok) continue;
            for (int j = D - 1; j >= 0; --j) b = b * nc + mb[j];
#pragma unroll
            for (int k = 0; k < D; ++k) acc += Ks[(((size_t)o * D + i) * D + k) * n_ctrl + a] * xs[b * D + k];
        }
        y[(size_t)s * n_dof + a * D + i] = acc;
    }
}

// ------------------------------------------------------------------ matrix-free true cell operator
// K^(s) u without the assembled values (Sec. 4.2.1, Remark 9): the stiffness is linear in the
// pulled-back tensor Ĉ^(s) at the quadrature points (eq. (52)), so per element E and point q
//   G_kl = sum_b u_{b,k} dN_{b,l}(q),  sigma_ij = w_q sum_kl Ĉ_ijkl(q) G_kl,
//   y_{a,i} += sum_j dN_{a,j}(q) sigma_ij.
// dN is a tensor product of the shared 1D B-spline tables (values v, derivatives d per element
// and Gauss point), so both G and the outputs are taken one direction at a time (sum
// factorisation: three-term contractions through LDS instead of 3^d x 3^d products).  Elements
// are taken in 3^d colours (e_j mod 3 per direction): two elements of one colour share no control
// point (quadratic supports span 3), so each colour's outputs are added into the LDS result
// without conflicts, and every output is summed over its elements in one fixed order.
constexpr int kMfB = 256;

template <int D>
__global__ __launch_bounds__(kMfB) void k_true_K_mf(const double *__restrict__ snap, const double *__restrict__ tab1,
                                                    const double *__restrict__ x, long long x_rs, long long nU,
                                                    const int *__restrict__ Ap, const int *__restrict__ idx_r,
                                                    const int *__restrict__ idx_p, const int *__restrict__ r_of_dof,
                                                    const int *__restrict__ p_of_dof, const int *__restrict__ gl,
                                                    int N, int n_r, int n_p, int n_i, int n_d, int n_el, int eb,
                                                    double *__restrict__ y, long long y_rs,
                                                    double *__restrict__ yp_cells) {
    constexpr int NQ = D == 2 ? 9 : 27, DD = D * D, D4 = DD * DD;
    extern __shared__ double sm[];
    const int nc = n_el + 2;
    int n_ctrl = 1, n_elem = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        n_ctrl *= nc;
        n_elem *= n_el;
    }
    const int n_dof = n_ctrl * D, nt1 = n_el * 9;
    double *ul = sm, *yl = ul + n_dof, *bA = yl + n_dof, *bB = bA + (size_t)eb * NQ * DD, *tv = bB + (size_t)eb * NQ * DD,
           *td = tv + nt1, *tw = td + nt1;
    const int col = blockIdx.x, rhs = col / N, s = col % N, tid = threadIdx.x;
    const double *u = x + rhs * x_rs;
    const double *lam = u + nU;
    for (int i = tid; i < n_r; i += kMfB) ul[idx_r[i]] = u[(size_t)s * n_r + i];
    for (int j = tid; j < n_p; j += kMfB) {
        const int P = Ap[(size_t)s * n_p + j];
        ul[idx_p[j]] = P >= 0 ? u[(size_t)N * n_r + P] : 0.0;
    }
    for (int i = tid; i < n_dof; i += kMfB) yl[i] = 0.0;
    for (int i = tid; i < 2 * nt1 + n_el * 3; i += kMfB) tv[i] = tab1[i];
    __syncthreads();
    const double *Cs = snap + (size_t)s * n_elem * NQ * D4;
    // 1D tables of element e: V(e, g, b) = tv[(3e + g) * 3 + b], derivative td, weight tw[3e + g]
    int ncolour = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) ncolour *= 3;
    for (int cl = 0; cl < ncolour; ++cl) {
        int c0[D], cnt[D], ncl = 1;
#pragma unroll
        for (int j = 0, t = cl; j < D; ++j, t /= 3) {
            c0[j] = t % 3;
            cnt[j] = c0[j] < n_el ? (n_el - c0[j] + 2) / 3 : 0;
            ncl *= cnt[j];
        }
        for (int bb = 0; bb < ncl; bb += eb) {
            const int nb = min(eb, ncl - bb);
            auto elem = [&](int ie, int (&e)[D]) {
                int r = bb + ie;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    e[j] = c0[j] + 3 * (r % cnt[j]);
                    r /= cnt[j];
                }
            };
            if constexpr (D == 3) {
                // 1: T0[ie][k][b2][b1][g0] = (sum_b0 v u, sum_b0 d u)
                for (int t = tid; t < nb * 81; t += kMfB) {
                    const int g0 = t % 3, b1 = (t / 3) % 3, b2 = (t / 9) % 3, k = (t / 27) % 3, ie = t / 81;
                    int e[3];
                    elem(ie, e);
                    const int nb0 = (e[0] + nc * ((e[1] + b1) + nc * (e[2] + b2))) * 3 + k;
                    const double *V = tv + (3 * e[0] + g0) * 3, *Dv = td + (3 * e[0] + g0) * 3;
                    double v = 0.0, d = 0.0;
#pragma unroll
                    for (int b0 = 0; b0 < 3; ++b0) {
                        const double uu = ul[nb0 + 3 * b0];
                        v += V[b0] * uu;
                        d += Dv[b0] * uu;
                    }
                    bA[2 * t] = v;
                    bA[2 * t + 1] = d;
                }
                __syncthreads();
                // 2: T1[ie][k][b2][g1][g0] = (vv, vd, dv) over b1
                for (int t = tid; t < nb * 81; t += kMfB) {
                    const int g0 = t % 3, g1 = (t / 3) % 3, b2 = (t / 9) % 3, k = (t / 27) % 3, ie = t / 81;
                    int e[3];
                    elem(ie, e);
                    const double *V = tv + (3 * e[1] + g1) * 3, *Dv = td + (3 * e[1] + g1) * 3;
                    const double *T = bA + (size_t)((((ie * 3 + k) * 3 + b2) * 3) * 3 + g0) * 2;
                    double vv = 0.0, vd = 0.0, dv = 0.0;
#pragma unroll
                    for (int b1 = 0; b1 < 3; ++b1) {
                        const double tvv = T[b1 * 6], tdd = T[b1 * 6 + 1];
                        vv += V[b1] * tvv;
                        vd += Dv[b1] * tvv;
                        dv += V[b1] * tdd;
                    }
                    bB[3 * t] = vv;
                    bB[3 * t + 1] = vd;
                    bB[3 * t + 2] = dv;
                }
                __syncthreads();
                // 3: G[ie][q][k][l] over b2
                for (int t = tid; t < nb * 81; t += kMfB) {
                    const int g0 = t % 3, g1 = (t / 3) % 3, g2 = (t / 9) % 3, k = (t / 27) % 3, ie = t / 81;
                    int e[3];
                    elem(ie, e);
                    const double *V = tv + (3 * e[2] + g2) * 3, *Dv = td + (3 * e[2] + g2) * 3;
                    const double *T = bB + (size_t)(((ie * 3 + k) * 3) * 3 * 3 + g1 * 3 + g0) * 3;
                    double G0 = 0.0, G1 = 0.0, G2 = 0.0;
#pragma unroll
                    for (int b2 = 0; b2 < 3; ++b2) {
                        const double *Tb = T + b2 * 27;
                        G0 += V[b2] * Tb[2];
                        G1 += V[b2] * Tb[1];
                        G2 += Dv[b2] * Tb[0];
                    }
                    double *Gq = bA + ((size_t)(ie * 27 + g0 + 3 * g1 + 9 * g2) * 3 + k) * 3;
                    Gq[0] = G0;
                    Gq[1] = G1;
                    Gq[2] = G2;
                }
                __syncthreads();
                // 4: sigma[ie][q][i][j] = w_q sum_kl C_ijkl G_kl
                for (int t = tid; t < nb * 81; t += kMfB) {
                    const int i = t % 3, q = (t / 3) % 27, ie = t / 81;
                    int e[3];
                    elem(ie, e);
                    const int g0 = q % 3, g1 = (q / 3) % 3, g2 = q / 9;
                    const int E = e[0] + n_el * (e[1] + n_el * e[2]);
                    const double w = tw[3 * e[0] + g0] * tw[3 * e[1] + g1] * tw[3 * e[2] + g2];
                    const double *C = Cs + ((size_t)E * 27 + q) * 81 + i * 27;
                    const double *G = bA + (size_t)(ie * 27 + q) * 9;
                    double sg[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int j = 0; j < 3; ++j)
#pragma unroll
                        for (int kl = 0; kl < 9; ++kl) sg[j] += C[j * 9 + kl] * G[kl];
                    double *S = bB + (size_t)(ie * 27 + q) * 9 + i * 3;
#pragma unroll
                    for (int j = 0; j < 3; ++j) S[j] = w * sg[j];
                }
                __syncthreads();
                // 5: A[ie][i][b2][g1][g0] over g2: (v Z0, v Z1, d Z2)
                for (int t = tid; t < nb * 81; t += kMfB) {
                    const int g0 = t % 3, g1 = (t / 3) % 3, b2 = (t / 9) % 3, i = (t / 27) % 3, ie = t / 81;
                    int e[3];
                    elem(ie, e);
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
                    for (int g2 = 0; g2 < 3; ++g2) {
                        const double v = tv[(3 * e[2] + g2) * 3 + b2], d = td[(3 * e[2] + g2) * 3 + b2];
                        const double *Z = bB + (size_t)(ie * 27 + g0 + 3 * g1 + 9 * g2) * 9 + i * 3;
                        a0 += v * Z[0];
                        a1 += v * Z[1];
                        a2 += d * Z[2];
                    }
                    bA[3 * t] = a0;
                    bA[3 * t + 1] = a1;
                    bA[3 * t + 2] = a2;
                }
                __syncthreads();
                // 6: B[ie][i][b2][b1][g0] over g1: (v A0, d A1 + v A2)
                for (int t = tid; t < nb * 81; t += kMfB) {
                    const int g0 = t % 3, b1 = (t / 3) % 3, b2 = (t / 9) % 3, i = (t / 27) % 3, ie = t / 81;
                    int e[3];
                    elem(ie, e);
                    const double *A = bA + (size_t)((((ie * 3 + i) * 3 + b2) * 3) * 3 + g0) * 3;
                    double pp = 0.0, qq = 0.0;
#pragma unroll
                    for (int g1 = 0; g1 < 3; ++g1) {
                        const double v = tv[(3 * e[1] + g1) * 3 + b1], d = td[(3 * e[1] + g1) * 3 + b1];
                        const double *Ag = A + g1 * 9;
                        pp += v * Ag[0];
                        qq += d * Ag[1] + v * Ag[2];
                    }
                    bB[2 * t] = pp;
                    bB[2 * t + 1] = qq;
                }
                __syncthreads();
                // 7: y over g0, added at the element's control points (disjoint within a colour)
                for (int t = tid; t < nb * 81; t += kMfB) {
                    const int b0 = t % 3, b1 = (t / 3) % 3, b2 = (t / 9) % 3, i = (t / 27) % 3, ie = t / 81;
                    int e[3];
                    elem(ie, e);
                    const double *B = bB + (size_t)((((ie * 3 + i) * 3 + b2) * 3 + b1) * 3) * 2;
                    double acc = 0.0;
#pragma unroll
                    for (int g0 = 0; g0 < 3; ++g0)
                        acc += td[(3 * e[0] + g0) * 3 + b0] * B[2 * g0] + tv[(3 * e[0] + g0) * 3 + b0] * B[2 * g0 + 1];
                    yl[((e[0] + b0) + nc * ((e[1] + b1) + nc * (e[2] + b2))) * 3 + i] += acc;
                }
                __syncthreads();
            } else {
                // 1: T0[ie][k][b1][g0] = (sum_b0 v u, sum_b0 d u)
                for (int t = tid; t < nb * 18; t += kMfB) {
                    const int g0 = t % 3, b1 = (t / 3) % 3, k = (t / 9) % 2, ie = t / 18;
                    int e[2];
                    elem(ie, e);
                    const int nb0 = (e[0] + nc * (e[1] + b1)) * 2 + k;
                    const double *V = tv + (3 * e[0] + g0) * 3, *Dv = td + (3 * e[0] + g0) * 3;
                    double v = 0.0, d = 0.0;
#pragma unroll
                    for (int b0 = 0; b0 < 3; ++b0) {
                        const double uu = ul[nb0 + 2 * b0];
                        v += V[b0] * uu;
                        d += Dv[b0] * uu;
                    }
                    bA[2 * t] = v;
                    bA[2 * t + 1] = d;
                }
                __syncthreads();
                // 2: G[ie][q][k][l] over b1
                for (int t = tid; t < nb * 18; t += kMfB) {
                    const int g0 = t % 3, g1 = (t / 3) % 3, k = (t / 9) % 2, ie = t / 18;
                    int e[2];
                    elem(ie, e);
                    const double *V = tv + (3 * e[1] + g1) * 3, *Dv = td + (3 * e[1] + g1) * 3;
                    const double *T = bA + (size_t)((ie * 2 + k) * 9 + g0) * 2;
                    double G0 = 0.0, G1 = 0.0;
#pragma unroll
                    for (int b1 = 0; b1 < 3; ++b1) {
                        G0 += V[b1] * T[b1 * 6 + 1];
                        G1 += Dv[b1] * T[b1 * 6];
                    }
                    double *Gq = bB + ((size_t)(ie * 9 + g0 + 3 * g1) * 2 + k) * 2;
                    Gq[0] = G0;
                    Gq[1] = G1;
                }
                __syncthreads();
                // 3: sigma[ie][q][i][j] = w_q sum_kl C_ijkl G_kl
                for (int t = tid; t < nb * 18; t += kMfB) {
                    const int i = t % 2, q = (t / 2) % 9, ie = t / 18;
                    int e[2];
                    elem(ie, e);
                    const int g0 = q % 3, g1 = q / 3;
                    const int E = e[0] + n_el * e[1];
                    const double w = tw[3 * e[0] + g0] * tw[3 * e[1] + g1];
                    const double *C = Cs + ((size_t)E * 9 + q) * 16 + i * 8;
                    const double *G = bB + (size_t)(ie * 9 + q) * 4;
                    double s0 = 0.0, s1 = 0.0;
#pragma unroll
                    for (int kl = 0; kl < 4; ++kl) {
                        s0 += C[kl] * G[kl];
                        s1 += C[4 + kl] * G[kl];
                    }
                    double *S = bA + (size_t)(ie * 9 + q) * 4 + i * 2;
                    S[0] = w * s0;
                    S[1] = w * s1;
                }
                __syncthreads();
                // 4: B[ie][i][b1][g0] over g1: (v Z0, d Z1)
                for (int t = tid; t < nb * 18; t += kMfB) {
                    const int g0 = t % 3, b1 = (t / 3) % 3, i = (t / 9) % 2, ie = t / 18;
                    int e[2];
                    elem(ie, e);
                    double pp = 0.0, qq = 0.0;
#pragma unroll
                    for (int g1 = 0; g1 < 3; ++g1) {
                        const double *Z = bA + (size_t)(ie * 9 + g0 + 3 * g1) * 4 + i * 2;
                        pp += tv[(3 * e[1] + g1) * 3 + b1] * Z[0];
                        qq += td[(3 * e[1] + g1) * 3 + b1] * Z[1];
                    }
                    bB[2 * t] = pp;
                    bB[2 * t + 1] = qq;
                }
                __syncthreads();
                // 5: y over g0, added at the element's control points (disjoint within a colour)
                for (int t = tid; t < nb * 18; t += kMfB) {
                    const int b0 = t % 3, b1 = (t / 3) % 3, i = (t / 9) % 2, ie = t / 18;
                    int e[2];
                    elem(ie, e);
                    const double *B = bB + (size_t)(((ie * 2 + i) * 3 + b1) * 3) * 2;
                    double acc = 0.0;
#pragma unroll
                    for (int g0 = 0; g0 < 3; ++g0)
                        acc += td[(3 * e[0] + g0) * 3 + b0] * B[2 * g0] + tv[(3 * e[0] + g0) * 3 + b0] * B[2 * g0 + 1];
                    yl[((e[0] + b0) + nc * (e[1] + b1)) * 2 + i] += acc;
                }
                __syncthreads();
            }
        }
    }
    double *yr = y + rhs * y_rs + (size_t)s * n_r;
    for (int row = tid; row < n_dof; row += kMfB) {
        double acc = yl[row];
        const int rp = r_of_dof[row];
        if (rp >= 0) {
            if (rp >= n_i) {  // dual dof: add B_d^T lam
                const int j = rp - n_i;
#pragma unroll
                for (int t2 = 0; t2 < 2; ++t2) {
                    const int code = gl[((size_t)s * n_d + j) * 2 + t2];
                    if (code == 0) continue;
                    const double lv = lam[(code > 0 ? code : -code) - 1];
                    acc += code > 0 ? lv : -lv;
                }
            }
            yr[rp] = acc;
        } else {
            yp_cells[(size_t)col * n_p + p_of_dof[row]] = acc;
        }
    }
}

// ------------------------------------------------------------------ reductions (deterministic)
// a butterfly within each wave, then the wave sums in wave order (fixed order, one barrier pair)
__device__ inline double block_reduce(double v, double *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// partial[(rhs*nv + i)*nblk + b] = sum over block b's chunk of V_i . w (per rhs).  The vectors
// are taken G at a time so each pass reads w once beside G vector streams; per thread the
// elements are summed in increasing order, then a fixed butterfly per wave and the 4 waves in
// order.
template <int G>
__global__ __launch_bounds__(256) void k_multidot_partial(const double *__restrict__ V, long long vstride,
                                                          const double *const *__restrict__ Vp, int nv,
                                                          const double *__restrict__ w, long long n, long long rs,
                                                          int nblk, double *__restrict__ partial) {
    __shared__ double sh[4][G];
    const int b = blockIdx.x, rhs = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long chunk = (n + nblk - 1) / nblk;
    const long long i0 = b * chunk, i1 = min(n, i0 + chunk);
    const double *wr = w + rhs * rs;
    for (int g0 = 0; g0 < nv; g0 += G) {
        const int ng = min(G, nv - g0);
        const double *vp[G];
        double acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            vp[g] = g < ng ? (Vp ? Vp[g0 + g] : V + (g0 + g) * vstride) + rhs * rs : wr;
            acc[g] = 0.0;
        }
        for (long long t = i0 + threadIdx.x; t < i1; t += 256) {
            const double x = wr[t];
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (g < ng) acc[g] += vp[g][t] * x;
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            for (int off = 32; off > 0; off >>= 1) acc[g] += __shfl_xor(acc[g], off);
        if (lane == 0)
#pragma unroll
            for (int g = 0; g < G; ++g) sh[wave][g] = acc[g];
        __syncthreads();
        if ((int)threadIdx.x < ng)
            partial[((size_t)rhs * nv + g0 + threadIdx.x) * nblk + b] =
                ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kB) void k_reduce_partials(const double *__restrict__ partial, int nblk,
                                                        double *__restrict__ out) {
    __shared__ double sh[kB];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kB) acc += partial[(size_t)blockIdx.x * nblk + b];
    acc = block_reduce(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// w[rhs] = a*w[rhs] + sum_i coef[rhs*nv + i] * V_i[rhs]
__global__ __launch_bounds__(kB) void k_multiaxpy(const double *__restrict__ V, long long vstride,
                                                  const double *const *__restrict__ Vp, int nv,
                                                  const double *__restrict__ coef, double a, double *__restrict__ w,
                                                  long long n, long long rs, int nrhs, double cscale) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    int rhs = (int)(t / n);
    long long i = t % n;
    double acc = a * w[rhs * rs + i];
    for (int k = 0; k < nv; ++k)
        acc += (cscale * coef[rhs * nv + k]) * (Vp ? Vp[k] : V + k * vstride)[rhs * rs + i];
    w[rhs * rs + i] = acc;
}

// w[rhs] += cscale * sum_i coef[rhs*nv + i] V_i[rhs] (the terms of k_multiaxpy with a = 1, in its order),
// written back, and in the same pass the partial sums of the updated w with every V_i (NORM = false:
// those of k_multidot_partial) or with itself (NORM = true: one per load case).  The chunks, the
// per-thread order and the reduction are those of k_multidot_partial, so the results equal those of
// the separate passes bitwise while the vectors are read once instead of twice.
template <int NVMAX, bool NORM>
__global__ __launch_bounds__(256) void k_axpy_dot(const double *const *__restrict__ Vp, int nv,
                                                  const double *__restrict__ coef, double cscale,
                                                  double *__restrict__ w, long long n, long long rs, int nblk,
                                                  double *__restrict__ partial) {
    constexpr int NP = NORM ? 1 : NVMAX;
    __shared__ double sh[4][NP];
    const int b = blockIdx.x, rhs = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long chunk = (n + nblk - 1) / nblk;
    const long long i0 = b * chunk, i1 = min(n, i0 + chunk);
    double *wr = w + rhs * rs;
    const double *vp[NVMAX];
    double cf[NVMAX], acc[NP];
#pragma unroll
    for (int g = 0; g < NVMAX; ++g) {
        vp[g] = g < nv ? Vp[g] + rhs * rs : wr;
        cf[g] = g < nv ? cscale * coef[rhs * nv + g] : 0.0;
    }
#pragma unroll
    for (int g = 0; g < NP; ++g) acc[g] = 0.0;
    for (long long t = i0 + threadIdx.x; t < i1; t += 256) {
        double v[NVMAX];
#pragma unroll
        for (int g = 0; g < NVMAX; ++g) v[g] = g < nv ? vp[g][t] : 0.0;
        double x = wr[t];
#pragma unroll
        for (int g = 0; g < NVMAX; ++g)
            if (g < nv) x += cf[g] * v[g];
        wr[t] = x;
        if constexpr (NORM) {
            acc[0] += x * x;
        } else {
#pragma unroll
            for (int g = 0; g < NVMAX; ++g)
                if (g < nv) acc[g] += v[g] * x;
        }
    }
    const int np = NORM ? 1 : nv;
#pragma unroll
    for (int g = 0; g < NP; ++g)
        for (int off = 32; off > 0; off >>= 1) acc[g] += __shfl_xor(acc[g], off);
    if (lane == 0)
#pragma unroll
        for (int g = 0; g < NP; ++g) sh[wave][g] = acc[g];
    __syncthreads();
    if ((int)threadIdx.x < np)
        partial[((size_t)rhs * np + threadIdx.x) * nblk + b] =
            ((sh[0][threadIdx.x] + sh[1][threadIdx.x]) + sh[2][threadIdx.x]) + sh[3][threadIdx.x];
}

// sc[r] = 1 / sqrt(h[r]) (0 for a zero norm)
__global__ void k_inv_sqrt(const double *__restrict__ h, double *__restrict__ sc, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) sc[t] = h[t] > 0.0 ? 1.0 / sqrt(h[t]) : 0.0;
}

__global__ __launch_bounds__(kB) void k_scale_copy(const double *__restrict__ x, long long n, long long rs,
                                                   const double *__restrict__ sc, double *__restrict__ y, int nrhs) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    int rhs = (int)(t / n);
    long long i = t % n;
    y[rhs * rs + i] = sc[rhs] * x[rhs * rs + i];
}

}  // namespace

// ================================================================== host wrappers
// grid of a cell-batched launch whose workgroups map to cells through cell_of_block
static unsigned cell_grid(int N, int nrhs) {
    return nrhs <= 1 ? (unsigned)N : 8u * (unsigned)((N + 7) / 8) * (unsigned)nrhs;
}

// Work enqueued inside a SideStream scope goes to the context's second stream
// (default priority); it starts after everything queued so far on the main
// stream, and join_side() makes the main stream wait for it.
SideStream::SideStream(ifeti_ctx *c) : c_(c), main_(c->stream) {
    if (!c->side_stream) {
        IFETI_HIP(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
        // device-local hand-offs only: no system-scope (host-visibility) fence on these markers
        IFETI_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming | hipEventDisableSystemFence));
        IFETI_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming | hipEventDisableSystemFence));
    }
    IFETI_HIP(hipEventRecord(c->ev_fork, main_));
    IFETI_HIP(hipStreamWaitEvent(c->side_stream, c->ev_fork, 0));
    c->stream = c->side_stream;
}

SideStream::~SideStream() {
    (void)hipEventRecord(c_->ev_join, c_->side_stream);
    c_->stream = main_;
    c_->side_pending = true;
}

void join_side(ifeti_ctx *c) {
    if (!c->side_pending) return;
    IFETI_HIP(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    c->side_pending = false;
}

void ensure_work(ifeti_ctx *c, int nrhs) {
    size_t cols = (size_t)c->N * nrhs;
    hipStream_t s = c->stream;
    c->w_Lam.ensure(cols * std::max(c->n_d, c->n_p), s);
    c->w_Y.ensure(cols * c->n_d, s);
    c->w_Yc.ensure(cols * c->n_d, s);
    c->w_c.ensure(cols * c->n_p, s);
    c->w_yp.ensure(cols * c->n_p, s);
    c->w_zP.ensure((size_t)std::max(c->nP, 1) * nrhs, s);
    c->w_yP.ensure((size_t)std::max(c->nP, 1) * nrhs, s);
    if (c->K > 0) {
        c->w_R.ensure(cols * c->K * c->n_r, s);
        c->w_H.ensure(cols * c->K * c->n_r, s);
    }
    c->w_red.ensure((size_t)2048 * 64 * nrhs + 1024, s);
}

void op_gather(ifeti_ctx *c, const double *lam, long long lam_rs, double *Lam, int nrhs, bool weights) {
    long long n = (long long)c->N * c->n_d * nrhs;
    Prof prof(c, "gather", 0.0, 8.0 * (double)n + 8.0 * (double)c->L * nrhs + 8.0 * (double)c->N * c->n_d);
    hipLaunchKernelGGL(k_gather, dim3(nblocks(n)), dim3(kB), 0, c->stream, c->g_gather.p, c->g_Dw.p, lam, lam_rs,
                       Lam, c->N, c->n_d, nrhs, weights ? 1 : 0);
}

// blocks of 512 entries for the interface-vector kernels: enough workgroups to keep the gathers and
// streams in flight, few enough partial sums for every block of the next kernel to add them up
int dot_blocks(long long n) { return (int)std::max<long long>(1, std::min<long long>(2048, (n + 511) / 512)); }

void op_scatter(ifeti_ctx *c, const double *Y, int y_ld, int y_off, long long y_rs, double *out, long long out_rs,
                int nrhs, bool weights, const double *dot_w, double *dot_part, const double *Y2) {
    long long n = (long long)c->L * nrhs;
    if (dot_w || Y2) {
        const int nblk = dot_blocks(c->L);
        Prof prof(c, "scatter_dot", 2.0 * (double)n,
                  16.0 * (double)n + 8.0 * (double)c->N * c->n_d * nrhs + 8.0 * (double)c->L);
        hipLaunchKernelGGL(k_scatter_dot, dim3(nblk, nrhs), dim3(kB), 0, c->stream, c->g_scatter.p, c->g_Dw.p, Y,
                           Y2, y_ld, y_off, y_rs, out, out_rs, c->L, c->n_d, weights ? 1 : 0, dot_w, nblk,
                           dot_w ? dot_part : nullptr);
        return;
    }
    Prof prof(c, "scatter", 0.0, 8.0 * (double)n + 8.0 * (double)c->N * c->n_d * nrhs + 8.0 * (double)c->L);
    hipLaunchKernelGGL(k_scatter, dim3(nblocks(n)), dim3(kB), 0, c->stream, c->g_scatter.p, c->g_Dw.p, Y, y_ld,
                       y_off, y_rs, out, out_rs, c->L, c->n_d, nrhs, weights ? 1 : 0);
}

void op_assemble_primal(ifeti_ctx *c, const double *cp, const double *base, long long b_rs, double sgn, double *zP,
                        long long z_rs, int nrhs) {
    long long n = (long long)c->nP * nrhs;
    if (n == 0) return;
    Prof prof(c, "assemble_primal", 0.0,
              8.0 * ((double)c->N * c->n_p * nrhs + (double)n * (base ? 2 : 1)) + 4.0 * (double)c->nP * c->maxc);
    const unsigned nb64 = (unsigned)((n + 63) / 64);
    if (c->maxc == 4)
        hipLaunchKernelGGL(k_assemble_primal_t<4>, dim3(nb64), dim3(64), 0, c->stream, c->g_Ppull.p, cp, c->N, c->n_p,
                           base, b_rs, sgn, zP, z_rs, c->nP, nrhs);
    else if (c->maxc == 8)
        hipLaunchKernelGGL(k_assemble_primal_t<8>, dim3(nb64), dim3(64), 0, c->stream, c->g_Ppull.p, cp, c->N, c->n_p,
                           base, b_rs, sgn, zP, z_rs, c->nP, nrhs);
    else
        hipLaunchKernelGGL(k_assemble_primal, dim3(nblocks(n)), dim3(kB), 0, c->stream, c->g_Ppull.p, c->maxc, cp,
                           c->N, c->n_p, base, b_rs, sgn, zP, z_rs, c->nP, nrhs);
}

void op_restrict_primal(ifeti_ctx *c, const double *xP, long long x_rs, double *xp, int nrhs) {
    long long n = (long long)c->N * c->n_p * nrhs;
    Prof prof(c, "restrict_primal", 0.0, 8.0 * (double)n + 8.0 * (double)c->nP * nrhs + 4.0 * (double)c->N * c->n_p);
    hipLaunchKernelGGL(k_restrict_primal, dim3(nblocks(n)), dim3(kB), 0, c->stream, c->g_Ap.p, xP, x_rs, xp, c->N,
                       c->n_p, nrhs);
}

void coarse_reduce(ifeti_ctx *c, const CoarseSolver &co, double *y, long long y_rs, int nrhs, double scale) {
    const double n = (double)c->nP, nt = (double)co.nT * (co.nT + 1) / 2;
    Prof prof(c, "coarse_reduce", (double)nrhs * nt * 128.0, 8.0 * (nt * 128.0 + n) * nrhs);
    hipLaunchKernelGGL(k_sym_reduce, dim3(co.nT, nrhs), dim3(1024), 0, c->stream, co.w_symP.p, c->nP, co.nT, nrhs, y,
                       y_rs, scale);
}

template <int NR, int WPR>
void coarse_rows(ifeti_ctx *c, const double *M, const CoarseRow *rows, int nrows, const double *x, long long x_rs,
                 double alpha, double *y, long long y_rs, double alpha2, double *y2, long long y2_rs,
                 const double *cz, long long cz_rs, double *cw, long long cw_rs, int ncopy) {
    constexpr int RPB = 4 / WPR;
    const long long total_rows = (long long)nrows + (ncopy + 64 * WPR - 1) / (64 * WPR);
    hipLaunchKernelGGL((k_coarse_rows<NR, WPR>), dim3((unsigned)((total_rows + RPB - 1) / RPB)), dim3(256), 0,
                       c->stream, M, rows, nrows, x, x_rs, alpha, y, y_rs, alpha2, y2, y2_rs, cz, cz_rs, cw, cw_rs,
                       ncopy);
    IFETI_HIP(hipGetLastError());
}

// the phases for a block of load cases (up to 32 a pass): the tile form, each row of the phase matrices
// read once per 32 load cases
static void coarse_partitioned_tiles(ifeti_ctx *c, CoarseSolver &co, const double *z, long long z_rs, double *y,
                                     long long y_rs, int nrhs, double scale) {
    const int n = c->nP, ns = co.cp_ns;
    const int nb = std::min(nrhs, 32);
    co.w_cg.ensure((size_t)ns * nb, c->stream);
    co.w_cw.ensure((size_t)n * nb, c->stream);
    for (int r0 = 0; r0 < nrhs; r0 += 32) {
        const int nr = std::min(32, nrhs - r0);
        const double *zz = z + (size_t)r0 * z_rs;
        double *yy = y + (size_t)r0 * y_rs;
        auto launch = [&](const double *M, const CoarseRow *rows, const CoarseTile *tiles, int ntiles,
                          const double *x, long long x_rs, double alpha, double *yo, long long yo_rs, double alpha2,
                          double *y2, long long y2_rs, const double *cz, int ncopy) {
            const unsigned blocks = (unsigned)(ntiles + ((long long)ncopy * nr + 255) / 256);
            if (nr <= 16)
                hipLaunchKernelGGL(k_coarse_tiles<1>, dim3(blocks), dim3(256), 0, c->stream, M, rows, tiles, ntiles, x,
                                   x_rs, alpha, yo, yo_rs, alpha2, y2, y2_rs, cz, z_rs, co.w_cw.p, (long long)n,
                                   ncopy, nr);
            else
                hipLaunchKernelGGL(k_coarse_tiles<2>, dim3(blocks), dim3(256), 0, c->stream, M, rows, tiles, ntiles, x,
                                   x_rs, alpha, yo, yo_rs, alpha2, y2, y2_rs, cz, z_rs, co.w_cw.p, (long long)n,
                                   ncopy, nr);
            IFETI_HIP(hipGetLastError());
        };
        {
            Prof prof(c, "coarse_sep_rhs", 2.0 * (double)co.cp_M1.n * nr,
                      8.0 * ((double)co.cp_M1.n + (double)ns * nr + 2.0 * n * nr) + 24.0 * ns);
            launch(co.cp_M1.p, co.cp_R1.p, co.cp_T1.p, (int)co.cp_T1.n, zz, z_rs, -1.0, co.w_cg.p, ns, 0.0, nullptr, 0,
                   zz, n);
        }
        {
            Prof prof(c, "coarse_sep_solve", 2.0 * (double)ns * ns * nr,
                      8.0 * ((double)ns * ns + 3.0 * ns * nr) + 24.0 * ns);
            launch(co.cp_M2.p, co.cp_R2.p, co.cp_T2.p, (int)co.cp_T2.n, co.w_cg.p, ns, 1.0, co.w_cw.p, n, scale, yy,
                   y_rs, nullptr, 0);
        }
        {
            Prof prof(c, "coarse_interior", 2.0 * (double)co.cp_M3.n * nr,
                      8.0 * ((double)co.cp_M3.n + 2.0 * (double)n * nr) + 24.0 * (n - ns));
            launch(co.cp_M3.p, co.cp_R3.p, co.cp_T3.p, (int)co.cp_T3.n, co.w_cw.p, n, scale, yy, y_rs, 0.0, nullptr, 0,
                   nullptr, 0);
        }
    }
}

// y = scale * S̊_PP^-1 z through the three phases of the partitioned solve (1 to 3 load cases)
void coarse_partitioned(ifeti_ctx *c, CoarseSolver &co, const double *z, long long z_rs, double *y, long long y_rs,
                        int nrhs, double scale) {
    const int n = c->nP, ns = co.cp_ns, nI = n - ns;
    // separator phases have few rows (one workgroup per row keeps enough loads in flight); the
    // interior phase has many (two waves per row)
    auto launch = [&](auto wpr, const double *M, const CoarseRow *rows, int nrows, const double *x, long long x_rs,
                      double alpha, double *yy, long long yy_rs, double alpha2, double *y2, long long y2_rs,
                      const double *cz, int ncopy) {
        constexpr int W = decltype(wpr)::value;
        if (nrhs == 1)
            coarse_rows<1, W>(c, M, rows, nrows, x, x_rs, alpha, yy, yy_rs, alpha2, y2, y2_rs, cz, z_rs, co.w_cw.p,
                              n, ncopy);
        else if (nrhs == 2)
            coarse_rows<2, W>(c, M, rows, nrows, x, x_rs, alpha, yy, yy_rs, alpha2, y2, y2_rs, cz, z_rs, co.w_cw.p,
                              n, ncopy);
        else
            coarse_rows<3, W>(c, M, rows, nrows, x, x_rs, alpha, yy, yy_rs, alpha2, y2, y2_rs, cz, z_rs, co.w_cw.p,
                              n, ncopy);
    };
    using Sep = std::integral_constant<int, 4>;
    using Int = std::integral_constant<int, 2>;
    {
        Prof prof(c, "coarse_sep_rhs", 2.0 * (double)co.cp_M1.n * nrhs,
                  8.0 * ((double)co.cp_M1.n + (double)ns * nrhs + 2.0 * n * nrhs) + 24.0 * ns);
        launch(Sep{}, co.cp_M1.p, co.cp_R1.p, ns, z, z_rs, -1.0, co.w_cg.p, ns, 0.0, nullptr, 0, z, n);
    }
    {
        Prof prof(c, "coarse_sep_solve", 2.0 * (double)ns * ns * nrhs,
                  8.0 * ((double)ns * ns + 3.0 * ns * nrhs) + 24.0 * ns);
        launch(Sep{}, co.cp_M2.p, co.cp_R2.p, ns, co.w_cg.p, ns, 1.0, co.w_cw.p, n, scale, y, y_rs, nullptr, 0);
    }
    {
        Prof prof(c, "coarse_interior", 2.0 * (double)co.cp_M3.n * nrhs,
                  8.0 * ((double)co.cp_M3.n + (double)n * nrhs + (double)nI * nrhs) + 24.0 * nI);
        launch(Int{}, co.cp_M3.p, co.cp_R3.p, nI, co.w_cw.p, n, scale, y, y_rs, 0.0, nullptr, 0, nullptr, 0);
    }
}

void coarse_solve(ifeti_ctx *c, CoarseSolver &co, const double *z, long long z_rs, double *y, long long y_rs,
                  int nrhs, double scale) {
    if (c->nP == 0) return;
    if (co.ap_B > 0) {  // block-Jacobi approximation: one phase of independent rows, up to 3 load cases a pass
        const int n = c->nP;
        for (int r0 = 0; r0 < nrhs; r0 += 3) {
            const int nr = std::min(3, nrhs - r0);
            Prof prof(c, "coarse_approx", 2.0 * (double)co.ap_M.n * nr, 8.0 * ((double)co.ap_M.n + 2.0 * n * nr) + 24.0 * n);
            const double *zz = z + (size_t)r0 * z_rs;
            double *yy = y + (size_t)r0 * y_rs;
            if (nr == 1)
                coarse_rows<1, 2>(c, co.ap_M.p, co.ap_R.p, n, zz, z_rs, scale, yy, y_rs, 0.0, nullptr, 0, nullptr, 0,
                                  nullptr, 0, 0);
            else if (nr == 2)
                coarse_rows<2, 2>(c, co.ap_M.p, co.ap_R.p, n, zz, z_rs, scale, yy, y_rs, 0.0, nullptr, 0, nullptr, 0,
                                  nullptr, 0, 0);
            else
                coarse_rows<3, 2>(c, co.ap_M.p, co.ap_R.p, n, zz, z_rs, scale, yy, y_rs, 0.0, nullptr, 0, nullptr, 0,
                                  nullptr, 0, 0);
        }
        return;
    }
    if (nrhs < 4 && co.cp_p >= 2) {
        coarse_partitioned(c, co, z, z_rs, y, y_rs, nrhs, scale);
        return;
    }
    if (co.cp_p >= 2 && !c->no_alloc) {
        coarse_partitioned_tiles(c, co, z, z_rs, y, y_rs, nrhs, scale);
        return;
    }
    ensure_coarse_inverse(c, co);
    if (nrhs < 4) {
        const double n = (double)c->nP, nt = (double)co.nT * (co.nT + 1) / 2;
        {
            // algorithmic: the symmetric operator's n(n+1)/2 entries read once, the vectors, the partials
            Prof prof(c, "coarse_symv", 2.0 * n * n * nrhs,
                      8.0 * (n * (n + 1) / 2 + 2.0 * n * nrhs + nt * 128.0 * nrhs));
            const unsigned ntiles = (unsigned)nt;
            if (nrhs == 1)
                hipLaunchKernelGGL(k_sym_tiles<1>, dim3(ntiles), dim3(256), 0, c->stream, co.SPPt.p,
                                   co.sym_tiles.p, c->nP, z, z_rs, co.w_symP.p);
            else if (nrhs == 2)
                hipLaunchKernelGGL(k_sym_tiles<2>, dim3(ntiles), dim3(256), 0, c->stream, co.SPPt.p,
                                   co.sym_tiles.p, c->nP, z, z_rs, co.w_symP.p);
            else
                hipLaunchKernelGGL(k_sym_tiles<3>, dim3(ntiles), dim3(256), 0, c->stream, co.SPPt.p,
                                   co.sym_tiles.p, c->nP, z, z_rs, co.w_symP.p);
            IFETI_HIP(hipGetLastError());
        }
        coarse_reduce(c, co, y, y_rs, nrhs, scale);
    } else {
        GemmGroup g;
        g.A = co.SPPinv.p;
        g.X = z;
        g.Kd = c->nP;
        g.ldx = (int)z_rs;
        g.xbs = (long long)nrhs * z_rs;
        g.K = 1;
        g.scale = scale;
        gemm(c, &g, 1, y, (int)y_rs, (long long)nrhs * y_rs, c->nP, nrhs, false, nrhs, "coarse_gemm", false);
    }
}

void op_coarse_solve(ifeti_ctx *c, const double *z, long long z_rs, double *y, long long y_rs, int nrhs,
                     double scale) {
    coarse_solve(c, c->co, z, z_rs, y, y_rs, nrhs, scale);
}

// ------------------------------------------------------------------ F̊ (48)
// Lambda = B_d^T lam; c_s = (T_dr Ů_rp^(s))^T Lambda_s, assembled and sent through the
// coarse solve; the dominant contraction sum_k delta_k F_dd^(k) Lambda; the coarse correction
// (T_dr Ů_rp^(s)) A_p^T y_P is added as B_d scatters.
void combine_coarse_maps(ifeti_ctx *c) {
    const int npd = c->n_p * c->n_d;
    IFETI_REQUIRE(c->n_p <= kMaxNp, IFETI_EINVAL, "too many primal dofs per cell");
    c->Wc.alloc((size_t)c->N * npd);
    hipLaunchKernelGGL(k_combine_wt, dim3(nblocks((long long)c->N * npd)), dim3(kB), 0, c->stream, c->pi.p, c->WT.p,
                       c->N, c->K, npd, c->Wc.p);
    IFETI_HIP(hipGetLastError());
}

// c_s = C_s B_d^(s)T lam for every column (rhs, s); C is [s][n_p][n_d]
void op_restrict_cells(ifeti_ctx *c, const double *C, const double *lam, long long lam_rs, double *out, int nrhs,
                       const char *tag) {
    const int N = c->N, nd = c->n_d, np = c->n_p, cols = N * nrhs;
    Prof prof(c, tag, 2.0 * (double)cols * np * nd,
              8.0 * (double)N * np * nd + 8.0 * ((double)c->L * nrhs + (double)cols * np) + 8.0 * (double)N * nd);
    if (np <= 8 && nd <= 128 && nrhs >= 4)
        // a block of load cases: C_s and the codes read once per cell
        hipLaunchKernelGGL((k_restrict_cm<8>), dim3(N), dim3(256), 0, c->stream, C, c->g_gather.p, lam, lam_rs, N, nd,
                           np, nrhs, out);
    else if (np <= 8)
        // 2D: one wave per cell; its partial sums are reduced through LDS rather than by eight
        // butterflies, which compete for the LDS pipe with the contraction running beside it
        hipLaunchKernelGGL((k_restrict_c1<8>), dim3(cell_grid(N, nrhs)), dim3(64), 0, c->stream, C, c->g_gather.p, lam, lam_rs,
                           N, nd, np, cols, out);
    else if (nrhs < 4)
        // 3D, in order on one stream: four waves per cell keep the 166 KB of C_s per cell streaming
        hipLaunchKernelGGL((k_restrict_c<kMaxNp, 4>), dim3(cell_grid(N, nrhs)), dim3(256), 0, c->stream, C, c->g_gather.p,
                           lam, lam_rs, N, nd, np, cols, out);
    else
        // 3D beside the contraction on the second stream: one wave per cell keeps the coarse branch from
        // crowding it
        hipLaunchKernelGGL((k_restrict_c<kMaxNp, 1>), dim3(cell_grid(N, nrhs)), dim3(64), 0, c->stream, C, c->g_gather.p, lam,
                           lam_rs, N, nd, np, cols, out);
    IFETI_HIP(hipGetLastError());
}

// Y_s (+)= C_s^T yP[A_p(s)] for every column (rhs, s); Y is [col][n_d]
void op_prolong_cells(ifeti_ctx *c, const double *C, const double *yP, long long yP_rs, double *Y, int nrhs,
                      bool accumulate, const char *tag) {
    const int N = c->N, nd = c->n_d, np = c->n_p, cols = N * nrhs;
    Prof prof(c, tag, 2.0 * (double)cols * np * nd, 8.0 * (double)N * np * nd + 8.0 * (double)cols * nd);
    if (np <= 8 && nd <= 256 && nrhs >= 4)
        hipLaunchKernelGGL((k_prolong_cm<8>), dim3(N), dim3((nd + 63) / 64 * 64), 0, c->stream, C, c->g_Ap.p, yP, yP_rs,
                           N, nd, np, nrhs, Y, accumulate ? 1 : 0);
    else if (np <= 8)
        hipLaunchKernelGGL((k_prolong_c<8, 2>), dim3(cell_grid(N, nrhs)), dim3(128), 0, c->stream, C, c->g_Ap.p, yP, yP_rs, N, nd,
                           np, cols, Y, accumulate ? 1 : 0);
    else if (nrhs < 4)
        hipLaunchKernelGGL((k_prolong_c<kMaxNp, 4>), dim3(cell_grid(N, nrhs)), dim3(256), 0, c->stream, C, c->g_Ap.p, yP,
                           yP_rs, N, nd, np, cols, Y, accumulate ? 1 : 0);
    else
        hipLaunchKernelGGL((k_prolong_c<kMaxNp, 1>), dim3(cell_grid(N, nrhs)), dim3(64), 0, c->stream, C, c->g_Ap.p, yP, yP_rs, N,
                           nd, np, cols, Y, accumulate ? 1 : 0);
    IFETI_HIP(hipGetLastError());
}

// F̊ lam = B_d [sum_k delta_k F_dd^(k) B_d^T lam + C^T A_p S̊_PP^-1 A_p^T C B_d^T lam]:
// the coarse branch (restriction, assembly, symmetric coarse solve) runs on the
// side stream while the main stream runs the dominant contraction; the
// prolongation is folded into the final scatter.
void apply_F_into(ifeti_ctx *c, const double *lam, double *out, int nrhs, double *Y, double *Yc, double *cb,
                  double *zP, double *yP, const double *dot_w, double *dot_part) {
    const int N = c->N, nd = c->n_d, K = c->K;
    const int cols = N * nrhs;
    GemmGroup g1;  // B_d^T lam fused into the staging
    g1.A = c->Fdd.p; g1.X = lam; g1.xbs = c->L; g1.gcodes = c->g_gather.p; g1.coef = c->delta.p; g1.Kd = nd;
    g1.K = K;
    // Up to three load cases everything runs in order on one stream: the coarse branch beside the
    // contraction on a second stream measured slower on c2 (each cross-stream wait costs about 15 us on
    // the host and leaves a gap of that order on the GPU, more than the overlap gains).  With a block
    // of load cases both branches take hundreds of microseconds and the contraction runs on the second
    // stream beside the coarse branch, after the restriction.
    const bool side = nrhs >= 4 && !c->no_alloc;
    const bool bank_streamed = 8.0 * K * nd * nd > 4.0 * 1024 * 1024 && nd >= 512;  // the F_dd bank exceeds L2
    const int prec = c->prec_override >= 0 ? c->prec_override : c->opt.precision;
    if (!side && bank_streamed && prec != IFETI_BF16_LOCAL) {
        // Principal form of the coarse branch: the restriction c_s = sum_k pi_sk (T_dr U_rp^(k))^T Lambda_s
        // is a small contraction over the principal maps (L2-resident) with the jump gather fused, and the
        // prolongation sum_k pi_sk (T_dr U_rp^(k)) y_P[A_p(s)] is a second group of the dominant
        // contraction (its cell vectors gathered from y_P through A_p): neither streams the per-cell
        // combined maps (340 MB on the 3D c3 lattice), and the prolongation needs no launch of its own.
        // Where the bank streams from HBM the extra group adds n_p / n_d of the contraction's steps (c3:
        // restriction 136 -> 72 us, prolongation 107 us -> +62 us in the contraction); where the bank
        // stays in L2 the contraction is short and the extra group's latency is not hidden (c2: +12.7 us
        // against a 7.5 us prolongation, the restriction unchanged), so the combined maps serve there.  In
        // the FP32 precision form both maps run in FP32 with the contraction (the coarse solve stays FP64;
        // c3 FP32 local 2.47 -> 2.16 s); in BF16 they slowed the outer iteration (c3: 26 -> 44 outer
        // iterations), so the BF16 form keeps the FP64 combined maps.
        const int np = c->n_p;
        GemmGroup gr;
        gr.A = c->WT.p; gr.X = lam; gr.xbs = c->L; gr.gcodes = c->g_gather.p; gr.coef = c->pi.p; gr.Kd = nd;
        gr.K = K;
        gemm(c, &gr, 1, cb, np, 0, np, cols, false, 0, "F_restrict");
        op_assemble_primal(c, cb, nullptr, 0, 1.0, zP, c->nP, nrhs);
        op_coarse_solve(c, zP, c->nP, yP, c->nP, nrhs, 1.0);
        GemmGroup g2[2];
        g2[0] = g1;
        g2[1].A = c->W.p; g2[1].X = yP; g2[1].xbs = c->nP; g2[1].gcodes = c->g_Apc.p; g2[1].coef = c->pi.p;
        g2[1].Kd = np; g2[1].K = K;
        gemm(c, g2, 2, Y, nd, 0, nd, cols, false, 0, "F_gemm");
        op_scatter(c, Y, nd, 0, (long long)N * nd, out, c->L, nrhs, false, dot_w, dot_part);
        c->applies[IFETI_OP_F] += nrhs;
        IFETI_HIP(hipGetLastError());
        return;
    }
    op_restrict_cells(c, c->Wc.p, lam, c->L, cb, nrhs, "F_restrict");
    if (side) {
        SideStream ss(c);
        gemm(c, &g1, 1, Y, nd, 0, nd, cols, false, 0, "F_gemm");
    } else {
        gemm(c, &g1, 1, Y, nd, 0, nd, cols, false, 0, "F_gemm");
    }
    op_assemble_primal(c, cb, nullptr, 0, 1.0, zP, c->nP, nrhs);
    op_coarse_solve(c, zP, c->nP, yP, c->nP, nrhs, 1.0);
    op_prolong_cells(c, c->Wc.p, yP, c->nP, Yc, nrhs, false, "F_prolong");
    if (side) join_side(c);
    op_scatter(c, Y, nd, 0, (long long)N * nd, out, c->L, nrhs, false, dot_w, dot_part, Yc);
    c->applies[IFETI_OP_F] += nrhs;
    IFETI_HIP(hipGetLastError());
}

void apply_F(ifeti_ctx *c, const double *lam, double *out, int nrhs, const double *dot_w, double *dot_part) {
    ensure_work(c, nrhs);
    apply_F_into(c, lam, out, nrhs, c->w_Y.p, c->w_Yc.p, c->w_c.p, c->w_zP.p, c->w_yP.p, dot_w, dot_part);
}

// ------------------------------------------------------------------ M̊_D^-1 (49)
void apply_MD(ifeti_ctx *c, const double *r, double *out, int nrhs, const double *dot_w, double *dot_part) {
    ensure_work(c, nrhs);
    const int N = c->N, nd = c->n_d, K = c->K;
    GemmGroup g;  // D-scaled B_d^T r fused into the staging
    g.A = c->Sdd.p; g.X = r; g.xbs = c->L; g.gcodes = c->g_gather.p; g.gw = c->g_Dw.p; g.coef = c->alpha.p;
    g.Kd = nd; g.K = K;
    {
        // the preconditioner's own precision, if set (restored also when the contraction throws)
        struct Scope {
            ifeti_ctx *c;
            ~Scope() { c->prec_override = -1; }
        } scope{c};
        c->prec_override = c->opt.md_precision;
        gemm(c, &g, 1, c->w_Y.p, nd, 0, nd, N * nrhs, false, 0, "MD_gemm");
    }
    op_scatter(c, c->w_Y.p, nd, 0, (long long)N * nd, out, c->L, nrhs, true, dot_w, dot_part);
    c->applies[IFETI_OP_MD] += nrhs;
    IFETI_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ Ů (Algorithm 3)
void apply_U(ifeti_ctx *c, const double *v, double *z, int nrhs) {
    ensure_work(c, nrhs);
    const int N = c->N, nd = c->n_d, np = c->n_p, nr = c->n_r, K = c->K;
    const int cols = N * nrhs;
    const long long nU = c->nU;
    GemmGroup g0;  // t_s = Ů_rp^T v_r
    g0.A = c->UrpT.p; g0.X = v; g0.coef = c->pi.p; g0.Kd = nr; g0.ldx = nr; g0.xbs = nU; g0.K = K;
    gemm(c, &g0, 1, c->w_c.p, np, 0, np, cols, false, 0, "U_restrict_gemm");
    // v̄_P = v_P - Ů_RP^T v_R
    op_assemble_primal(c, c->w_c.p, v + (size_t)N * nr, nU, -1.0, c->w_zP.p, c->nP, nrhs);
    op_coarse_solve(c, c->w_zP.p, c->nP, c->w_yP.p, c->nP, nrhs, 1.0);
    op_restrict_primal(c, c->w_yP.p, c->nP, c->w_yp.p, nrhs);
    GemmGroup g[2];  // Y = Ů_rd^T v_r - T_dr Ů_rp z_p
    g[0].A = c->UrdT.p; g[0].X = v; g[0].coef = c->delta.p; g[0].Kd = nr; g[0].ldx = nr; g[0].xbs = nU; g[0].K = K;
    g[1].A = c->W.p; g[1].X = c->w_yp.p; g[1].coef = c->pi.p; g[1].Kd = np; g[1].ldx = np; g[1].K = K;
    g[1].scale = -1.0;
    gemm(c, g, 2, c->w_Y.p, nd, 0, nd, cols, false, 0, "U_gemm");
    op_scatter(c, c->w_Y.p, nd, 0, (long long)N * nd, z, c->L, nrhs, false);
    c->applies[IFETI_OP_U] += nrhs;
    IFETI_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ Ůᵀ (transpose of Algorithm 3)
void apply_Ut(ifeti_ctx *c, const double *y, double *x, int nrhs) {
    ensure_work(c, nrhs);
    const int N = c->N, nd = c->n_d, np = c->n_p, nr = c->n_r, K = c->K;
    const int cols = N * nrhs;
    const long long nU = c->nU;
    op_gather(c, y, c->L, c->w_Lam.p, nrhs, false);
    GemmGroup g0;
    g0.A = c->WT.p; g0.X = c->w_Lam.p; g0.coef = c->pi.p; g0.Kd = nd; g0.ldx = nd; g0.K = K;
    gemm(c, &g0, 1, c->w_c.p, np, 0, np, cols, false, 0, "Ut_restrict_gemm");
    op_assemble_primal(c, c->w_c.p, nullptr, 0, 1.0, c->w_zP.p, c->nP, nrhs);
    double *xP = x + (size_t)N * nr;
    op_coarse_solve(c, c->w_zP.p, c->nP, xP, nU, nrhs, -1.0);  // x_P = -S̊^-1 Ů_RP^T B_R^T y
    op_restrict_primal(c, xP, nU, c->w_yp.p, nrhs);
    GemmGroup g[2];  // x_r = Ů_rd B_d^T y - Ů_rp A_p^T x_P
    g[0].A = c->Urd.p; g[0].X = c->w_Lam.p; g[0].coef = c->delta.p; g[0].Kd = nd; g[0].ldx = nd; g[0].K = K;
    g[1].A = c->Urp.p; g[1].X = c->w_yp.p; g[1].coef = c->pi.p; g[1].Kd = np; g[1].ldx = np; g[1].K = K;
    g[1].scale = -1.0;
    gemm(c, g, 2, x, nr, nU, nr, cols, false, 0, "Ut_gemm");
    c->applies[IFETI_OP_UT] += nrhs;
    IFETI_HIP(hipGetLastError());
}

// (46b) H = K_rr^(s) R for the K columns of R (work buffers w_R -> w_H) of `cols` cell columns,
// in LDS-staged column chunks
static void launch_rom_H(ifeti_ctx *c, int cols) {
    const RefTables &R = c->ref;
    const int N = c->N, nr = c->n_r, K = c->K;
    const double colsd = (double)cols;
    {
        int kcol = 4;
        for (int cand : {8, 12, 16})
            if ((size_t)(nr + 1) * (cand | 1) * 8 <= 100 * 1024 && kcol < K) kcol = cand;
        const int nthr = (R.n_ctrl + 63) / 64 * 64;
        IFETI_REQUIRE(nthr <= kRomHB, IFETI_EINVAL, "reduced local solve: too many control points per cell");
        const size_t lds = (size_t)(nr + 1) * (kcol | 1) * sizeof(double) + (size_t)R.n_ctrl * c->dim * sizeof(int);
        IFETI_REQUIRE(lds <= 160 * 1024, IFETI_EINVAL, "cell too large for the LDS-staged reduced local solve");
        const double chunks = (double)((K + kcol - 1) / kcol);
        Prof prof(c, "rom_H", colsd * 2.0 * K * c->nnz_rr,
                  colsd * 8.0 * (2.0 * K * nr + chunks * (double)R.n_ctrl * R.n_off * c->dim * c->dim));
        for (int k0 = 0; k0 < K; k0 += kcol) {
#define IFETI_ROM_H(DD, KC)                                                                                       \
    do {                                                                                                          \
    (void)hipFuncSetAttribute((const void *)k_rom_H<DD, KC>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    (void)hipGetLastError();                                                                                      \
    hipLaunchKernelGGL((k_rom_H<DD, KC>), dim3(cols), dim3(nthr), lds, c->stream, c->w_R.p, c->Kst.p,             \
                       c->r_of_dof.p, N, K, k0, nr, R.nc, R.n_ctrl, c->w_H.p);               \
    } while (0)
            if (c->dim == 2) {
                if (kcol == 4) IFETI_ROM_H(2, 4);
                else if (kcol == 8) IFETI_ROM_H(2, 8);
                else if (kcol == 12) IFETI_ROM_H(2, 12);
                else IFETI_ROM_H(2, 16);
            } else {
                if (kcol == 4) IFETI_ROM_H(3, 4);
                else if (kcol == 8) IFETI_ROM_H(3, 8);
                else if (kcol == 12) IFETI_ROM_H(3, 12);
                else IFETI_ROM_H(3, 16);
            }
#undef IFETI_ROM_H
            IFETI_HIP(hipGetLastError());
        }
    }
}

// cell r-vectors of every column into one contiguous block: out[col][n_r], col = rhs*N + s
__global__ __launch_bounds__(kB) void k_cells_contiguous(const double *__restrict__ v, long long v_rs, int N, int n_r,
                                                         long long total, double *__restrict__ out) {
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t >= total) return;
    const long long col = t / n_r;
    out[t] = v[(col / N) * v_rs + (col % N) * n_r + t % n_r];
}

// K̊^-MPCG (Remark 6): opt.local_iters multi-preconditioned CG iterations per cell, the first of which
// is the reduced solve (46); the whitened blocks of earlier iterations are kept for the conjugations
static void op_mpcg_local(ifeti_ctx *c, const double *vR, long long v_rs, double *xR, long long x_rs, int nrhs) {
    const int N = c->N, nr = c->n_r, K = c->K, iters = c->opt.local_iters;
    const int cols = N * nrhs;
    const size_t blk = (size_t)cols * K * nr;
    hipStream_t s = c->stream;
    c->mp_r.ensure((size_t)cols * nr, s);
    while ((int)c->mp_P.size() < iters) {
        c->mp_P.emplace_back(new DevBuf<double>());
        c->mp_KP.emplace_back(new DevBuf<double>());
    }
    for (int j = 0; j < iters; ++j) {
        c->mp_P[j]->ensure(blk, s);
        c->mp_KP[j]->ensure(blk, s);
    }
    const long long total = (long long)cols * nr;
    hipLaunchKernelGGL(k_cells_contiguous, dim3((unsigned)((total + kB - 1) / kB)), dim3(kB), 0, s, vR, v_rs, N, nr,
                       total, c->mp_r.p);
    const int kb = (K + 1 + 15) / 16, wpb = kb == 3 ? 2 : 4;
    const dim3 grid((cols + wpb - 1) / wpb), block(64 * wpb);
    const size_t lds_step = (size_t)wpb * (4 * K * K + 2 * K) * sizeof(double);
    const size_t lds_conj = (size_t)wpb * (K * K + K) * sizeof(double);
    const double colsd = (double)cols;
    for (int it = 0; it < iters; ++it) {
        GemmGroup g;  // Z = [K_rr^(σk)-1 r]_k
        g.A = c->Kinv.p; g.X = c->mp_r.p; g.Kd = nr; g.ldx = nr; g.xbs = (long long)N * nr; g.K = 1;
        gemm(c, &g, 1, c->w_R.p, K * nr, 0, K * nr, cols, false, 0, "rom_R_gemm");
        for (int j = 0; j < it; ++j) {
            Prof prof(c, "mpcg_conj", colsd * 4.0 * K * K * nr, colsd * 8.0 * 4.0 * K * nr);
            const double *P = c->mp_P[j]->p, *KP = c->mp_KP[j]->p;
            if (kb == 1)
                hipLaunchKernelGGL((k_mpcg_conj<1, 4>), grid, block, lds_conj, s, c->w_R.p, P, KP, cols, K, nr);
            else if (kb == 2)
                hipLaunchKernelGGL((k_mpcg_conj<2, 4>), grid, block, lds_conj, s, c->w_R.p, P, KP, cols, K, nr);
            else
                hipLaunchKernelGGL((k_mpcg_conj<3, 2>), grid, block, lds_conj, s, c->w_R.p, P, KP, cols, K, nr);
            IFETI_HIP(hipGetLastError());
        }
        launch_rom_H(c, cols);
        {
            Prof prof(c, "mpcg_step", colsd * (2.0 * (K + 1.0) * K * nr + 4.0 * K * K * nr),
                      colsd * 8.0 * (6.0 * K * nr + 3.0 * nr));
            double *P = c->mp_P[it]->p, *KP = c->mp_KP[it]->p;
            if (kb == 1)
                hipLaunchKernelGGL((k_mpcg_step<1, 4>), grid, block, lds_step, s, c->w_R.p, c->w_H.p, c->mp_r.p, xR,
                                   x_rs, it == 0 ? 1 : 0, P, KP, N, cols, K, nr);
            else if (kb == 2)
                hipLaunchKernelGGL((k_mpcg_step<2, 4>), grid, block, lds_step, s, c->w_R.p, c->w_H.p, c->mp_r.p, xR,
                                   x_rs, it == 0 ? 1 : 0, P, KP, N, cols, K, nr);
            else
                hipLaunchKernelGGL((k_mpcg_step<3, 2>), grid, block, lds_step, s, c->w_R.p, c->w_H.p, c->mp_r.p, xR,
                                   x_rs, it == 0 ? 1 : 0, P, KP, N, cols, K, nr);
            IFETI_HIP(hipGetLastError());
        }
    }
}

// (46b) in one pass when the cell and K allow it (K <= 16, the LDS footprint below 160 KB): the variant
// (0: 2D, 12 columns a chunk; 1: 2D, 8; 2: 3D, 8) and its LDS bytes, or -1 for the two-kernel form
// LDS bytes of k_rom_local with chunks of kcol columns and R (and H) in elements of esize bytes, or a
// huge value when the FP64 wave partials do not fit in the chunk's bytes
static size_t rom_local_lds(ifeti_ctx *c, int kcol, size_t esize) {
    const RefTables &R = c->ref;
    const int K = c->K, D = c->dim;
    const int nthr = (R.n_ctrl + 63) / 64 * 64;
    const size_t rbytes = ((size_t)(D * R.n_ctrl + 1) * (kcol | 1) * esize + 15) & ~(size_t)15;
    if ((size_t)(nthr / 64) * 256 * sizeof(double) > rbytes) return (size_t)1 << 30;
    return rbytes + (size_t)(4 * K * K + 4 * K) * sizeof(double) + ((size_t)R.n_ctrl * D + c->n_r + 1) * sizeof(int);
}

static int rom_local_mode(ifeti_ctx *c) {
    const RefTables &R = c->ref;
    const int K = c->K, D = c->dim;
    if (K > 16 || R.p != 2 || (D != 2 && D != 3)) return -1;
    const int nthr = (R.n_ctrl + 63) / 64 * 64;
    if (nthr > kRomHB) return -1;
    constexpr size_t kLds = 160 * 1024;
    // c2: 661 us, against 790 us for the two-kernel form
    int mode = -1;
    if (D == 2 && K <= 12 && rom_local_lds(c, 12, sizeof(double)) <= kLds) mode = 0;
    else if (D == 2 && rom_local_lds(c, 8, sizeof(double)) <= kLds) mode = 1;
    else if (D == 3 && rom_local_lds(c, 8, sizeof(double)) <= kLds) mode = 2;
    return mode;
}

// R: [col][n_r][K] in FP64, or in FP32 (the precision form's narrow product)
template <typename TR>
static void launch_rom_local(ifeti_ctx *c, int mode, const TR *Rp, const double *vR, long long v_rs,
                             double *xR, long long x_rs, int cols) {
    const size_t lds = rom_local_lds(c, mode == 0 ? 12 : 8, sizeof(TR));
    const RefTables &R = c->ref;
    const int nr = c->n_r, K = c->K, D = c->dim;
    const int nthr = (R.n_ctrl + 63) / 64 * 64;
    const int nrhs = cols / c->N;
    const unsigned grid = cell_grid(c->N, nrhs);
    const double colsd = (double)cols, chunks = mode == 0 ? 1.0 : (double)((K + 7) / 8);
    // algorithmic: the stencil of the column's cell once per chunk, R, v and x once
    Prof prof(c, "rom_local", colsd * (2.0 * K * c->nnz_rr + 2.0 * (K + 1.0) * K * nr + 2.0 * K * nr),
              colsd * (8.0 * chunks * (double)R.n_ctrl * R.n_off * D * D + (double)sizeof(TR) * K * nr + 16.0 * nr));
#define IFETI_ROM_LOCAL(DD, KC)                                                                                   \
    do {                                                                                                          \
        IFETI_HIP(hipFuncSetAttribute((const void *)k_rom_local<TR, DD, KC>,                                \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));                     \
        hipLaunchKernelGGL((k_rom_local<TR, DD, KC>), dim3(grid), dim3(nthr), lds, c->stream, Rp, c->Kst.p,      \
                           c->r_of_dof.p, vR, v_rs, c->N, nrhs, K, nr, R.nc, R.n_ctrl, xR, x_rs);               \
    } while (0)
    if (mode == 0) IFETI_ROM_LOCAL(2, 12);
    else if (mode == 1) IFETI_ROM_LOCAL(2, 8);
    else IFETI_ROM_LOCAL(3, 8);
#undef IFETI_ROM_LOCAL
    IFETI_HIP(hipGetLastError());
}

void op_rom_local(ifeti_ctx *c, const double *vR, long long v_rs, double *xR, long long x_rs, int nrhs,
                  const double *bank, const char *rtag) {
    const int N = c->N, nr = c->n_r, K = c->K;
    IFETI_REQUIRE(K <= kMaxK, IFETI_EINVAL, "reduced local solve supports at most 40 principal cells");
    if (c->opt.local_iters > 1 && !bank) {
        op_mpcg_local(c, vR, v_rs, xR, x_rs, nrhs);
        return;
    }
    // (46a) R = [K_rr^(sigma_k)-1 v]_k : one GEMM with the row-interleaved explicit inverses, so each
    // column comes out as [r][k] (or the zero-padded interior inverses of (47))
    const int cols = N * nrhs;
    const int mode = rom_local_mode(c);
    const int prec = c->prec_override >= 0 ? c->prec_override : c->opt.precision;
    if (mode >= 0 && prec != IFETI_FP64) {
        // precision form: the narrow product by the library into an FP32 R, read as such by (46b)
        c->w_R32.ensure((size_t)cols * K * nr, c->stream);
        if (library_gemm_narrow(c, bank ? bank : c->Kinv.p, K * nr, nr, vR, nr, v_rs, N, nrhs, prec, c->w_R32.p,
                                rtag)) {
            launch_rom_local(c, mode, c->w_R32.p, vR, v_rs, xR, x_rs, cols);
            return;
        }
    }
    GemmGroup g;
    g.A = bank ? bank : c->Kinv.p; g.X = vR; g.Kd = nr; g.ldx = nr; g.xbs = v_rs; g.K = 1;
    gemm(c, &g, 1, c->w_R.p, K * nr, 0, K * nr, N * nrhs, false, 0, rtag);
    // (46b) H = K_rr^(s) R in column chunks, then the per-cell Gram system and combination
    const double colsd = (double)cols;
    if (mode >= 0) {
        launch_rom_local(c, mode, (const double *)c->w_R.p, vR, v_rs, xR, x_rs, cols);
        return;
    }
    launch_rom_H(c, cols);
    {
        Prof prof(c, "rom_gram", colsd * (2.0 * (K + 1.0) * K * nr + 2.0 * K * nr),
                  colsd * 8.0 * (3.0 * K * nr + 2.0 * nr));
        const int kb = (K + 1 + 15) / 16;
        const int wpb = kb == 3 ? 2 : 4;
        const size_t lds = (size_t)wpb * (3 * K * K + 2 * K) * sizeof(double);
        const dim3 grid((cols + wpb - 1) / wpb), block(64 * wpb);
        if (kb == 1)
            hipLaunchKernelGGL((k_rom_gram<1, 4>), grid, block, lds, c->stream, vR, v_rs, c->w_R.p, c->w_H.p, N, cols,
                               K, nr, xR, x_rs);
        else if (kb == 2)
            hipLaunchKernelGGL((k_rom_gram<2, 4>), grid, block, lds, c->stream, vR, v_rs, c->w_R.p, c->w_H.p, N, cols,
                               K, nr, xR, x_rs);
        else
            hipLaunchKernelGGL((k_rom_gram<3, 2>), grid, block, lds, c->stream, vR, v_rs, c->w_R.p, c->w_H.p, N, cols,
                               K, nr, xR, x_rs);
        IFETI_HIP(hipGetLastError());
    }
}

// ------------------------------------------------------------------ K̊^-ROM (45), Algorithm 2
void apply_Kinv_rom(ifeti_ctx *c, const double *v, double *x, int nrhs, bool local_done) {
    ensure_work(c, nrhs);
    const int N = c->N, np = c->n_p, nr = c->n_r, K = c->K;
    const int cols = N * nrhs;
    const long long nU = c->nU;
    GemmGroup g0;
    g0.A = c->UrpT.p; g0.X = v; g0.coef = c->pi.p; g0.Kd = nr; g0.ldx = nr; g0.xbs = nU; g0.K = K;
    gemm(c, &g0, 1, c->w_c.p, np, 0, np, cols, false, 0, "Kinv_restrict_gemm");
    op_assemble_primal(c, c->w_c.p, v + (size_t)N * nr, nU, -1.0, c->w_zP.p, c->nP, nrhs);
    double *xP = x + (size_t)N * nr;
    op_coarse_solve(c, c->w_zP.p, c->nP, xP, nU, nrhs, 1.0);
    if (!local_done) op_rom_local(c, v, nU, x, nU, nrhs);      // x_R = K̊_RR^-ROM v_R (unless already there)
    op_restrict_primal(c, xP, nU, c->w_yp.p, nrhs);
    GemmGroup g;                                                 // x_R -= Ů_RP x_P
    g.A = c->Urp.p; g.X = c->w_yp.p; g.coef = c->pi.p; g.Kd = np; g.ldx = np; g.K = K; g.scale = -1.0;
    gemm(c, &g, 1, x, nr, nU, nr, cols, true, 0, "Kinv_prolong_gemm");
    c->applies[IFETI_OP_KINV_ROM] += nrhs;
    IFETI_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ true saddle operator (16)
// per-cell part of (16) on packed saddle vectors (stride nU + L): y_R = K_rr u_r + K_rp u_p + B_r^T lam,
// and the cells' primal rows K_pr u_r + K_pp u_p into w_c (stencil values or matrix-free, by option)
static void op_cell_K(ifeti_ctx *c, const double *x, double *y, int nrhs) {
    const int N = c->N, nr = c->n_r, np = c->n_p;
    const long long nU = c->nU, rs = nU + c->L;
    const RefTables &R = c->ref;
    size_t shmem = (size_t)R.n_dof * sizeof(double);
    if (c->opt.true_operator == 1) {
        IFETI_REQUIRE(c->snap_valid, IFETI_EINVAL, "matrix-free true operator: pulled-back tensor not available");
        IFETI_REQUIRE(R.p == 2, IFETI_EINVAL, "matrix-free true operator: quadratic B-splines only");
        // two stage buffers of up to 2048 doubles each (whole colours of the c2/c3 cells in one batch)
        const int DD = c->dim * c->dim;
        const int eb = std::max(1, 2048 / (R.nq * DD));
        const size_t lds = (size_t)(2 * R.n_dof + 2 * eb * R.nq * DD + 2 * R.n_el * 9 + R.n_el * 3) * sizeof(double);
        IFETI_REQUIRE(lds <= 160 * 1024, IFETI_EINVAL, "matrix-free true operator: cell too large for LDS");
        const double colsd = (double)N * nrhs;
        // flops of the definition: per element and point, G (2 D^2 nloc), sigma (2 D^4), outputs (2 D^2 nloc)
        const double fl = colsd * R.n_elem * R.nq * (4.0 * DD * R.nloc + 2.0 * DD * DD);
        Prof prof(c, "true_K_mf", fl, 8.0 * (double)N * R.n_snap + colsd * 8.0 * 2.0 * R.n_dof);
        if (c->dim == 2) {
            IFETI_HIP(hipFuncSetAttribute((const void *)k_true_K_mf<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds));
            hipLaunchKernelGGL(k_true_K_mf<2>, dim3(N * nrhs), dim3(kMfB), lds, c->stream, c->snap.p,
                               c->g_tables_1d.p, x, rs, nU, c->g_Ap.p, c->g_idx_r.p, c->g_idx_p.p, c->r_of_dof.p,
                               c->p_of_dof.p, c->g_gather.p, N, nr, np, c->n_i, c->n_d, R.n_el, eb, y, rs, c->w_c.p);
        } else {
            IFETI_HIP(hipFuncSetAttribute((const void *)k_true_K_mf<3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds));
            hipLaunchKernelGGL(k_true_K_mf<3>, dim3(N * nrhs), dim3(kMfB), lds, c->stream, c->snap.p,
                               c->g_tables_1d.p, x, rs, nU, c->g_Ap.p, c->g_idx_r.p, c->g_idx_p.p, c->r_of_dof.p,
                               c->p_of_dof.p, c->g_gather.p, N, nr, np, c->n_i, c->n_d, R.n_el, eb, y, rs, c->w_c.p);
        }
    } else {
    const double colsd = (double)N * nrhs;
    Prof prof(c, "true_K", colsd * 2.0 * c->nnz_full,
              8.0 * (double)N * R.n_ctrl * R.n_off * c->dim * c->dim + colsd * 8.0 * 2.0 * R.n_dof);
    // four load cases a workgroup for a block of them (each stencil value read once for the four)
    const int nrb = nrhs >= 4 ? 4 : 1;
    const unsigned grid = cell_grid(N, (nrhs + nrb - 1) / nrb);
    const size_t shm = shmem * nrb;
#define IFETI_TRUE_K(DD, NB)                                                                                      \
    hipLaunchKernelGGL((k_true_K<DD, NB>), dim3(grid), dim3(kB), shm, c->stream, c->Kst.p, x, rs, nU, c->g_Ap.p,   \
                       c->g_idx_r.p, c->g_idx_p.p, c->r_of_dof.p, c->p_of_dof.p, c->g_gather.p, N, nr, np, c->n_i, \
                       c->n_d, R.nc, R.n_ctrl, R.n_off, R.p, y, rs, c->w_c.p, nrhs)
    if (c->dim == 2) {
        if (nrb == 4) IFETI_TRUE_K(2, 4);
        else IFETI_TRUE_K(2, 1);
    } else {
        if (nrb == 4) IFETI_TRUE_K(3, 4);
        else IFETI_TRUE_K(3, 1);
    }
#undef IFETI_TRUE_K
    }
}

void apply_A(ifeti_ctx *c, const double *x, double *y, int nrhs) {
    ensure_work(c, nrhs);
    const int N = c->N, nr = c->n_r;
    const long long nU = c->nU, rs = nU + c->L;
    op_cell_K(c, x, y, nrhs);
    op_assemble_primal(c, c->w_c.p, nullptr, 0, 1.0, y + (size_t)N * nr, rs, nrhs);
    op_scatter(c, x, nr, c->n_i, rs, y + nU, rs, nrhs, false);  // B u
    c->applies[IFETI_OP_A] += nrhs;
    IFETI_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ M̊_D^-ROM (47)
// Principal interior inverses from the stacked K_rr^-1 (rows interleaved [r][k][n_r]) and S_dd by
// block inversion: with A = K_rr^-1, A_dd = S_dd^-1 and K_ii^-1 = A_ii - A_id S_dd A_di.  One
// workgroup per (interior row i, principal k); written zero-padded to n_r x n_r in the same
// interleaved layout, so the reduced solve of (46) takes it in place of K_rr^-1.
__global__ __launch_bounds__(256) void k_kii_inverse(const double *__restrict__ Kinv, const double *__restrict__ Sdd,
                                                     int K, int n_r, int n_i, int n_d, double *__restrict__ out) {
    extern __shared__ double sh[];  // a_d[n_d], t[n_d]
    const int i = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
    double *ad = sh, *t = sh + n_d;
    const double *Ai = Kinv + ((size_t)i * K + k) * n_r;  // row i of A_k
    for (int b = tid; b < n_d; b += 256) ad[b] = Ai[n_i + b];
    __syncthreads();
    const double *S = Sdd + (size_t)k * n_d * n_d;
    for (int a = tid; a < n_d; a += 256) {  // t = A_id(i,:) S (S symmetric: column a = row a)
        double acc = 0.0;
        for (int b = 0; b < n_d; ++b) acc += ad[b] * S[(size_t)a * n_d + b];
        t[a] = acc;
    }
    __syncthreads();
    double *o = out + ((size_t)i * K + k) * n_r;
    for (int j = tid; j < n_r; j += 256) {
        double v = 0.0;
        if (j < n_i) {
            double acc = 0.0;
            for (int a = 0; a < n_d; ++a) acc += t[a] * Kinv[((size_t)(n_i + a) * K + k) * n_r + j];
            v = Ai[j] - acc;
        }
        o[j] = v;
    }
}

// zero rows of the padded bank beyond the interior
__global__ __launch_bounds__(256) void k_zero_rows(double *__restrict__ out, long long from, long long n) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) out[from + t] = 0.0;
}

// packed saddle vectors (stride rs) for the cell operator: u_r^(s) = [-x_i^(s); Lam_s] (x null: zero
// interior), u_P = 0, lam = 0
__global__ __launch_bounds__(kB) void k_mdrom_saddle(const double *__restrict__ Lam, const double *__restrict__ xr,
                                                     int N, int n_r, int n_i, int n_d, long long rs,
                                                     double *__restrict__ X, int nrhs) {
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t >= rs * nrhs) return;
    const int rhs = (int)(t / rs);
    const long long e = t % rs;
    double v = 0.0;
    if (e < (long long)N * n_r) {
        const int s = (int)(e / n_r), j = (int)(e % n_r);
        const size_t col = (size_t)rhs * N + s;
        v = j >= n_i ? Lam[col * n_d + (j - n_i)] : (xr ? -xr[col * n_r + j] : 0.0);
    }
    X[t] = v;
}

// interior part of the cells' r rows of packed saddle vectors, dual part zero: out [rhs][s][n_r]
__global__ __launch_bounds__(kB) void k_r_interior(const double *__restrict__ Y, long long rs, int N, int n_r,
                                                   int n_i, double *__restrict__ out, int nrhs) {
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    const long long per = (long long)N * n_r;
    if (t >= per * nrhs) return;
    const int rhs = (int)(t / per);
    const long long e = t % per;
    out[t] = (int)(e % n_r) < n_i ? Y[rhs * rs + e] : 0.0;
}

static void build_kii_bank(ifeti_ctx *c) {
    if (c->kii_gen == c->bank_gen && c->Kii_pad.p) return;
    const int K = c->K, nr = c->n_r, ni = c->n_i, nd = c->n_d;
    c->Kii_pad.alloc((size_t)K * nr * nr);
    if (ni > 0) {
        const size_t lds = (size_t)2 * nd * sizeof(double);
        IFETI_REQUIRE(lds <= 160 * 1024, IFETI_EINVAL, "M_D^-ROM: dual block too large for LDS");
        if (lds > 64 * 1024)
            IFETI_HIP(hipFuncSetAttribute((const void *)k_kii_inverse, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)lds));
        hipLaunchKernelGGL(k_kii_inverse, dim3(ni, K), dim3(256), lds, c->stream, c->Kinv.p, c->Sdd.p, K, nr, ni, nd,
                           c->Kii_pad.p);
        IFETI_HIP(hipGetLastError());
    }
    const long long from = (long long)ni * K * nr, n = (long long)(nr - ni) * K * nr;
    if (n > 0) hipLaunchKernelGGL(k_zero_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->Kii_pad.p, from, n);
    IFETI_HIP(hipGetLastError());
    c->kii_gen = c->bank_gen;
}

// out = sum_s D B_d^(s) S̃_dd^(s) B_d^(s)T D r with S̃_dd = K_dd - K_di x(w), w = K_id Lam_s and x(w) the
// reduced interior solve of (46) with the principal K_ii^-1 (eq. (47)):
//   1. Lam = D-weighted gather; u_r = [0; Lam]; w_r = interior rows of K_rr u_r (cell operator)
//   2. x = R (Rᵀ K_ii R)^-1 Rᵀ w, R = [K_ii^(σk)-1 w]_k (the reduced local solve on the padded bank)
//   3. y = dual rows of K_rr [-x_i; Lam] (cell operator); out = D-weighted scatter of y
void apply_MD_rom(ifeti_ctx *c, const double *r, double *out, int nrhs) {
    ensure_work(c, nrhs);
    build_kii_bank(c);
    const int N = c->N, nr = c->n_r;
    const long long rs = c->nU + c->L, per = (long long)N * nr;
    hipStream_t s = c->stream;
    c->mdr_X.ensure((size_t)rs * nrhs, s);
    c->mdr_Y.ensure((size_t)rs * nrhs, s);
    c->mdr_v.ensure((size_t)per * nrhs, s);
    c->mdr_x.ensure((size_t)per * nrhs, s);
    op_gather(c, r, c->L, c->w_Lam.p, nrhs, true);
    const unsigned gX = (unsigned)((rs * nrhs + kB - 1) / kB), gR = (unsigned)((per * nrhs + kB - 1) / kB);
    hipLaunchKernelGGL(k_mdrom_saddle, dim3(gX), dim3(kB), 0, s, c->w_Lam.p, nullptr, N, nr, c->n_i, c->n_d, rs,
                       c->mdr_X.p, nrhs);
    op_cell_K(c, c->mdr_X.p, c->mdr_Y.p, nrhs);
    hipLaunchKernelGGL(k_r_interior, dim3(gR), dim3(kB), 0, s, c->mdr_Y.p, rs, N, nr, c->n_i, c->mdr_v.p, nrhs);
    op_rom_local(c, c->mdr_v.p, per, c->mdr_x.p, per, nrhs, c->Kii_pad.p, "mdrom_R_gemm");
    hipLaunchKernelGGL(k_mdrom_saddle, dim3(gX), dim3(kB), 0, s, c->w_Lam.p, c->mdr_x.p, N, nr, c->n_i, c->n_d, rs,
                       c->mdr_X.p, nrhs);
    op_cell_K(c, c->mdr_X.p, c->mdr_Y.p, nrhs);
    op_scatter(c, c->mdr_Y.p, nr, c->n_i, rs, out, c->L, nrhs, true);
    IFETI_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ per-cell displacement view
// out[rhs][s][e] for every local dof e of every cell (node-major, components interleaved): the r
// entries of u_r^(s), the primal entries from u_P through A_p, zero at clamped corners
__global__ __launch_bounds__(kB) void k_cell_view(const double *__restrict__ u, long long nU, int N, int n_r, int n_p,
                                                  int n_dof, const int *__restrict__ r_of_dof,
                                                  const int *__restrict__ p_of_dof, const int *__restrict__ Ap,
                                                  const double *__restrict__ up_dir, double *__restrict__ out,
                                                  long long total) {
    const long long t = (long long)blockIdx.x * kB + threadIdx.x;
    if (t >= total) return;
    const int e = (int)(t % n_dof);
    const long long col = t / n_dof;
    const int s = (int)(col % N);
    const double *ur = u + (col / N) * nU;
    const int rp = r_of_dof[e];
    double v = 0.0;
    if (rp >= 0) {
        v = ur[(size_t)s * n_r + rp];
    } else {
        const int j = p_of_dof[e];
        const int P = Ap[(size_t)s * n_p + j];
        v = P >= 0 ? ur[(size_t)N * n_r + P] : (up_dir ? up_dir[(size_t)s * n_p + j] : 0.0);
    }
    out[t] = v;
}

void cell_matvec_full(ifeti_ctx *c, const double *x, double *y) {
    const RefTables &R = c->ref;
    if (c->dim == 2)
        hipLaunchKernelGGL(k_cell_matvec_full<2>, dim3(c->N), dim3(kB), 0, c->stream, c->Kst.p, x, R.nc, R.n_ctrl,
                           R.n_off, R.p, y);
    else
        hipLaunchKernelGGL(k_cell_matvec_full<3>, dim3(c->N), dim3(kB), 0, c->stream, c->Kst.p, x, R.nc, R.n_ctrl,
                           R.n_off, R.p, y);
    IFETI_HIP(hipGetLastError());
}

void cell_displacements(ifeti_ctx *c, const double *u, double *out, int nrhs) {
    const long long total = (long long)nrhs * c->N * c->ref.n_dof;
    if (total == 0) return;
    hipLaunchKernelGGL(k_cell_view, dim3((unsigned)((total + kB - 1) / kB)), dim3(kB), 0, c->stream, u, c->nU, c->N,
                       c->n_r, c->n_p, c->ref.n_dof, c->r_of_dof.p, c->p_of_dof.p, c->g_Ap.p,
                       c->g_up_dir.n ? c->g_up_dir.p : nullptr, out, total);
    IFETI_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ vector helpers

// out_dev[rhs*nv + i] = V_i[rhs] . w[rhs]
void multidot(ifeti_ctx *c, const double *V, long long vstride, int nv, const double *w, long long n, long long rs,
              int nrhs, double *out_dev, const double *const *Vp) {
    // enough workgroups to keep the vector streams in flight (about 2K elements per workgroup)
    const int nblk = (int)std::max<long long>(1, std::min<long long>(2048, (n + 2047) / 2048));
    size_t need = (size_t)nblk * nv * nrhs;
    c->w_red.ensure(need, c->stream);
    Prof prof(c, "gmres_vec", 2.0 * n * nv * nrhs, 8.0 * (double)n * (nv + 1) * nrhs);
    hipLaunchKernelGGL(k_multidot_partial<8>, dim3(nblk, nrhs), dim3(256), 0, c->stream, V, vstride, Vp, nv, w, n, rs,
                       nblk, c->w_red.p);
    hipLaunchKernelGGL(k_reduce_partials, dim3(nv * nrhs), dim3(kB), 0, c->stream, c->w_red.p, nblk, out_dev);
    IFETI_HIP(hipGetLastError());
}

void multiaxpy(ifeti_ctx *c, const double *V, long long vstride, int nv, const double *coef_dev, double a, double *w,
               long long n, long long rs, int nrhs, const double *const *Vp, double cscale) {
    Prof prof(c, "gmres_vec", 2.0 * n * nv * nrhs, 8.0 * (double)n * (nv + 2) * nrhs);
    hipLaunchKernelGGL(k_multiaxpy, dim3(nblocks(n * nrhs)), dim3(kB), 0, c->stream, V, vstride, Vp, nv, coef_dev, a, w,
                       n, rs, nrhs, cscale);
    IFETI_HIP(hipGetLastError());
}

bool axpy_dot(ifeti_ctx *c, int nv, const double *coef_dev, double cscale, double *w, long long n, long long rs,
              int nrhs, const double *const *Vp, bool norm, double *out_dev) {
    constexpr int kMax = kAxpyDotMax;
    if (nv < 1 || nv > kMax || !Vp) return false;
    const int nblk = (int)std::max<long long>(1, std::min<long long>(2048, (n + 2047) / 2048));  // as multidot
    const int np = norm ? 1 : nv;
    c->w_red.ensure((size_t)nblk * np * nrhs, c->stream);
    Prof prof(c, "gmres_vec", 2.0 * n * nv * nrhs + 2.0 * n * np * nrhs, 8.0 * (double)n * (nv + 2) * nrhs);
    if (norm)
        hipLaunchKernelGGL((k_axpy_dot<kMax, true>), dim3(nblk, nrhs), dim3(256), 0, c->stream, Vp, nv, coef_dev, cscale,
                           w, n, rs, nblk, c->w_red.p);
    else
        hipLaunchKernelGGL((k_axpy_dot<kMax, false>), dim3(nblk, nrhs), dim3(256), 0, c->stream, Vp, nv, coef_dev,
                           cscale, w, n, rs, nblk, c->w_red.p);
    hipLaunchKernelGGL(k_reduce_partials, dim3(np * nrhs), dim3(kB), 0, c->stream, c->w_red.p, nblk, out_dev);
    IFETI_HIP(hipGetLastError());
    return true;
}

void inv_sqrt(ifeti_ctx *c, const double *h, double *sc, int n) {
    hipLaunchKernelGGL(k_inv_sqrt, dim3((n + 255) / 256), dim3(256), 0, c->stream, h, sc, n);
    IFETI_HIP(hipGetLastError());
}

void scale_copy(ifeti_ctx *c, const double *x, long long n, long long rs, const double *sc_dev, double *y, int nrhs) {
    Prof prof(c, "gmres_vec", (double)n * nrhs, 16.0 * (double)n * nrhs);
    hipLaunchKernelGGL(k_scale_copy, dim3(nblocks(n * nrhs)), dim3(kB), 0, c->stream, x, n, rs, sc_dev, y, nrhs);
    IFETI_HIP(hipGetLastError());
}

}  // namespace ifeti
