// Standard (exact) FETI-DP on the GPU: the comparator of the ROM solver (Sec. 2.2.4, Tables 1-2).
//
// Every cell's K_rr^(s) is factorised.  The factorisation runs batched over cells on an
// augmented dense matrix per cell, rows and columns ordered
//
//     [ r (n_r: interior, then dual) | p (n_p) | q (n_d) ]
//     [ K_rr   K_rp   E ]
//     [ K_pr   K_pp   0 ]        E = the n_r x n_d selection of the dual rows
//     [ E^T    0      0 ]
//
// by a right-looking blocked Cholesky of the first n_r columns only.  The trailing (p, q)
// block then holds the Schur complement
//
//     [ S_pp^(s)   -U_d^T ]       S_pp = K_pp - K_pr K_rr^-1 K_rp   (eq. (22))
//     [ -U_d      -F_dd   ]       U_d = E^T K_rr^-1 K_rp (dual rows of U_rp, eq. (29)),
//                                 F_dd = E^T K_rr^-1 E  (eq. (27))
//
// and the trailing dual block just before the dual columns are eliminated is the Dirichlet
// Schur complement S_dd^(s) = K_dd - K_di K_ii^-1 K_id (eq. (30)).  The first n_r columns hold
// the Cholesky factor of K_rr^(s), kept for the right-hand side (25) and the recovery
// (20)-(21).  The assembled S_PP gets its own coarse solver.  The online operators are the
// exact F of (24) and M_D of (30): per-cell dense products (HBM-bound: each apply streams all
// N n_d^2 operator entries, against K n_d^2 for the ROM contraction), with the coarse branch
// and the jump gather/scatter shared with the ROM path.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace ifeti {
namespace {

constexpr int XB = 64;      // panel width of the blocked factorisation
constexpr int kExMaxNp = 24;  // primal dofs per cell handled by the recovery kernel
typedef double v4d __attribute__((ext_vector_type(4)));

// entry K^(s)[u][v] of the cell matrix from its stencil values [o][i][k][a]
template <int D>
__device__ __forceinline__ double stencil_entry(const double *__restrict__ Ks, int u, int v, int nc, int n_ctrl,
                                                int p) {
    const int a = u / D, i = u % D, b = v / D, k = v % D;
    const int w = 2 * p + 1;
    int o = 0, ta = a, tb = b, scale = 1;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int d = tb % nc - ta % nc;
        if (d < -p || d > p) return 0.0;
        o += (d + p) * scale;
        scale *= w;
        ta /= nc;
        tb /= nc;
    }
    return Ks[(((size_t)o * D + i) * D + k) * n_ctrl + a];
}

// Lower triangle of the augmented matrix of list entries k = k0 + blockIdx.y (cell cells[k], or k
// without a list), column-major with leading dimension lda, one wave per column.  The q block
// selects the r rows [q_lo, q_lo + n_q).  K_pr and K_pp (lower) of each entry are written on the side.
template <int D>
__global__ __launch_bounds__(256) void k_ex_densify(const double *__restrict__ Kst, const int *__restrict__ cells,
                                                    int k0, int n_r, int n_p, int q_lo, int n_a, int lda,
                                                    const int *__restrict__ idx_r, const int *__restrict__ idx_p,
                                                    int nc, int n_ctrl, int n_off, int p, double *__restrict__ A,
                                                    double *__restrict__ Kpr, double *__restrict__ Kpp) {
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (col >= n_a) return;
    const int k = k0 + blockIdx.y, s = cells ? cells[k] : k;
    const double *Ks = Kst + (size_t)s * n_ctrl * n_off * D * D;
    double *M = A + (size_t)blockIdx.y * lda * n_a;
    const int nrp = n_r + n_p;
    const int v = col < n_r ? idx_r[col] : (col < nrp ? idx_p[col - n_r] : -1);
    for (int row = col + lane; row < n_a; row += 64) {
        double val;
        if (row < nrp) {
            const int u = row < n_r ? idx_r[row] : idx_p[row - n_r];
            val = stencil_entry<D>(Ks, u, v, nc, n_ctrl, p);
            if (row >= n_r && col < n_r) Kpr[((size_t)k * n_p + (row - n_r)) * n_r + col] = val;
            if (row >= n_r && col >= n_r && Kpp) Kpp[((size_t)k * n_p + (row - n_r)) * n_p + (col - n_r)] = val;
        } else {
            val = (col == q_lo + (row - nrp)) ? 1.0 : 0.0;  // E^T; zero against p and q
        }
        M[(size_t)col * lda + row] = val;
    }
}

// S_dd^(s): the trailing dual block when the interior columns are eliminated (full n_d x n_d)
__global__ __launch_bounds__(256) void k_ex_snap_sdd(const double *__restrict__ A, int lda, int n_a, int n_i,
                                                     int n_d, int s0, double *__restrict__ Sdd) {
    const double *M = A + (size_t)blockIdx.x * lda * n_a;
    double *S = Sdd + (size_t)(s0 + blockIdx.x) * n_d * n_d;
    for (int e = threadIdx.x; e < n_d * n_d; e += 256) {
        const int i = e / n_d, j = e % n_d, hi = max(i, j), lo = min(i, j);
        S[e] = M[(size_t)(n_i + lo) * lda + n_i + hi];
    }
}

// Panel [j0, j0+nb) of every cell of the batch: Cholesky of the diagonal block L11 in LDS, its
// inverse (one column per thread), then the rows below, L21 = A21 L11^-T, as an FP64 MFMA product
// (wave w takes 16-row blocks w, w+4, ...).  Beyond nb the block is padded with the identity.
// A pivot <= 0 (or not finite) marks the cell in bad[] and continues with 1.
__global__ __launch_bounds__(256) void k_ex_panel(double *__restrict__ A, int lda, int n_a, int j0, int nb, int s0,
                                                  int *__restrict__ bad) {
    __shared__ double Ld[XB][XB + 1];
    __shared__ double Li[XB][XB + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *M = A + (size_t)blockIdx.x * lda * n_a;
    for (int e = tid; e < XB * XB; e += 256) {
        const int i = e / XB, j = e % XB;
        double v = (i == j) ? 1.0 : 0.0;
        if (i < nb && j < nb && i >= j) v = M[(size_t)(j0 + j) * lda + j0 + i];
        Ld[i][j] = v;
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (tid == 0) {
            double d = Ld[k][k];
            if (!(d > 0.0) || !isfinite(d)) {
                bad[s0 + blockIdx.x] = 1;
                d = 1.0;
            }
            Ld[k][k] = sqrt(d);
        }
        __syncthreads();
        const double dk = Ld[k][k];
        for (int i = k + 1 + tid; i < nb; i += 256) Ld[i][k] /= dk;
        __syncthreads();
        const int m = nb - k - 1;  // trailing order
        for (int e = tid; e < m * m; e += 256) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j <= i) Ld[i][j] -= Ld[i][k] * Ld[j][k];
        }
        __syncthreads();
    }
    // L11^-1 by forward substitution, column j by thread j
    if (tid < XB) {
        const int j = tid;
        for (int i = 0; i < XB; ++i) {
            double v = (i == j) ? 1.0 : 0.0;
            for (int m = j; m < i; ++m) v -= Ld[i][m] * Li[m][j];
            Li[i][j] = i < j ? 0.0 : v / Ld[i][i];
        }
    }
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e / nb, j = e % nb;
        if (i >= j) M[(size_t)(j0 + j) * lda + j0 + i] = Ld[i][j];
    }
    __syncthreads();
    // L21 = A21 L11^-T: D[row][k] = sum_m A21[row][m] Linv[k][m]
    const int lr = lane & 15, lk = lane >> 4;
    for (int r0 = j0 + nb + 16 * wave; r0 < n_a; r0 += 64) {
        const int ra = r0 + lr;
        double a[XB / 4];
#pragma unroll
        for (int s = 0; s < XB / 4; ++s) {
            const int m = 4 * s + lk;
            a[s] = (m < nb && ra < n_a) ? M[(size_t)(j0 + m) * lda + ra] : 0.0;
        }
        v4d acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < XB / 4; ++s)
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], Li[16 * cb + lr][4 * s + lk], acc[cb], 0, 0, 0);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = r0 + 4 * i + lk, k = 16 * cb + lr;
                if (row < n_a && k < nb) M[(size_t)(j0 + k) * lda + row] = acc[cb][i];
            }
    }
}

// Trailing update A22 -= L21 L21^T on the lower 64x64 tiles of rows/columns >= t0, FP64 MFMA.
// Tile x of the batch's cell blockIdx.y: I(I+1)/2 + J = x, I >= J.  Wave w owns rows 16w..16w+15
// of the tile and its four 16-column blocks.
__global__ __launch_bounds__(256) void k_ex_syrk(double *__restrict__ A, int lda, int n_a, int j0, int nb, int t0) {
    const long long x = blockIdx.x;
    int I = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while ((long long)(I + 1) * (I + 2) / 2 <= x) ++I;
    while ((long long)I * (I + 1) / 2 > x) --I;
    const int J = (int)(x - (long long)I * (I + 1) / 2);
    double *M = A + (size_t)blockIdx.y * lda * n_a;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int rbase = t0 + 64 * I + 16 * wave, col0 = t0 + 64 * J;
    const int row_a = rbase + lr;
    v4d acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rbase + 4 * i + lk, col = col0 + 16 * cb + lr;
            acc[cb][i] = (row < n_a && col < n_a) ? M[(size_t)col * lda + row] : 0.0;
        }
    for (int k0 = 0; k0 < nb; k0 += 4) {
        const bool kin = k0 + lk < nb;
        const size_t kc = (size_t)(j0 + k0 + lk) * lda;
        const double a = (kin && row_a < n_a) ? -M[kc + row_a] : 0.0;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int cc = col0 + 16 * cb + lr;
            const double b = (kin && cc < n_a) ? M[kc + cc] : 0.0;
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rbase + 4 * i + lk, col = col0 + 16 * cb + lr;
            if (row < n_a && col < n_a) M[(size_t)col * lda + row] = acc[cb][i];
        }
}

// Fq = -A[q,q] = E^T K_rr^-1 E (full, from the lower triangle), S_pp = A[p,p], UqT = -A[q,p]^T
// (the q rows of U_rp, transposed: [n_p][n_q]), L = the first n_r columns (lower; skipped if null)
__global__ __launch_bounds__(256) void k_ex_extract(const double *__restrict__ A, int lda, int n_a, int n_r,
                                                    int n_p, int n_q, int k0, double *__restrict__ Fq,
                                                    double *__restrict__ Spp, double *__restrict__ UqT,
                                                    double *__restrict__ L) {
    const double *M = A + (size_t)blockIdx.x * lda * n_a;
    const int k = k0 + blockIdx.x, q0 = n_r + n_p;
    double *F = Fq + (size_t)k * n_q * n_q;
    for (long long e = threadIdx.x; e < (long long)n_q * n_q; e += 256) {
        const int i = (int)(e / n_q), j = (int)(e % n_q), hi = max(i, j), lo = min(i, j);
        F[e] = -M[(size_t)(q0 + lo) * lda + q0 + hi];
    }
    double *S = Spp + (size_t)k * n_p * n_p;
    for (int e = threadIdx.x; e < n_p * n_p; e += 256) {
        const int a = e / n_p, b = e % n_p, hi = max(a, b), lo = min(a, b);
        S[e] = M[(size_t)(n_r + lo) * lda + n_r + hi];
    }
    double *Cs = UqT + (size_t)k * n_p * n_q;
    for (int e = threadIdx.x; e < n_p * n_q; e += 256) {
        const int a = e / n_q, j = e % n_q;
        Cs[e] = -M[(size_t)(n_r + a) * lda + q0 + j];
    }
    if (!L) return;
    double *Ls = L + (size_t)k * n_r * n_r;
    for (int col = threadIdx.x >> 6; col < n_r; col += 4)
        for (int row = col + (threadIdx.x & 63); row < n_r; row += 64)
            Ls[(size_t)col * n_r + row] = M[(size_t)col * lda + row];
}

// x <- K_rr^(s)^-1 x with the stored factor (lower, column-major, leading dimension n_r), one
// workgroup per (cell, load case): blocks of 64, each diagonal block solved by one wave with
// shuffles, the remaining rows updated by the workgroup.
__global__ __launch_bounds__(256) void k_ex_trsv(const double *__restrict__ L, int n_r, int N,
                                                 double *__restrict__ X, long long x_rs) {
    extern __shared__ double xs[];  // n_r values, then 4 x 64 partials
    double *part = xs + n_r;
    const int s = blockIdx.x, rhs = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double *Ls = L + (size_t)s * n_r * n_r;
    double *x = X + rhs * x_rs + (size_t)s * n_r;
    for (int i = tid; i < n_r; i += 256) xs[i] = x[i];
    __syncthreads();
    // forward: L y = b
    for (int j0 = 0; j0 < n_r; j0 += 64) {
        const int nb = min(64, n_r - j0);
        if (wave == 0) {
            double v = lane < nb ? xs[j0 + lane] : 0.0;
            for (int m = 0; m < nb; ++m) {
                const double ym = __shfl(v, m) / Ls[(size_t)(j0 + m) * n_r + j0 + m];
                if (lane == m) v = ym;
                if (lane > m && lane < nb) v -= Ls[(size_t)(j0 + m) * n_r + j0 + lane] * ym;
            }
            if (lane < nb) xs[j0 + lane] = v;
        }
        __syncthreads();
        for (int r = j0 + nb + tid; r < n_r; r += 256) {
            double acc = 0.0;
            for (int m = 0; m < nb; ++m) acc += Ls[(size_t)(j0 + m) * n_r + r] * xs[j0 + m];
            xs[r] -= acc;
        }
        __syncthreads();
    }
    // backward: L^T x = y
    for (int j0 = ((n_r - 1) / 64) * 64; j0 >= 0; j0 -= 64) {
        const int nb = min(64, n_r - j0);
        // t_j = sum over rows below the block of L[r][j0+j] x_r: wave w takes columns w, w+4, ...
        for (int j = wave; j < nb; j += 4) {
            double acc = 0.0;
            for (int r = j0 + nb + lane; r < n_r; r += 64) acc += Ls[(size_t)(j0 + j) * n_r + r] * xs[r];
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if (lane == 0) part[j] = acc;
        }
        __syncthreads();
        if (wave == 0) {
            double v = lane < nb ? xs[j0 + lane] - part[lane] : 0.0;
            for (int m = nb - 1; m >= 0; --m) {
                const double xm = __shfl(v, m) / Ls[(size_t)(j0 + m) * n_r + j0 + m];
                if (lane == m) v = xm;
                if (lane < m) v -= Ls[(size_t)(j0 + lane) * n_r + j0 + m] * xm;
            }
            if (lane < nb) xs[j0 + lane] = v;
        }
        __syncthreads();
    }
    for (int i = tid; i < n_r; i += 256) x[i] = xs[i];
}

// Y[col] = A_s Lambda_s for column col = rhs*N + s: Lambda_s = (D-weighted) B_d^(s)T lam gathered into
// LDS, A_s the cell's n_d x n_d operator (row-major), rows by waves, a fixed butterfly per row.
__global__ __launch_bounds__(256) void k_ex_cell_gemv(const double *__restrict__ Mops, const int *__restrict__ gl,
                                                      const double *__restrict__ gw, const double *__restrict__ lam,
                                                      long long lam_rs, int N, int n_d, double *__restrict__ Y) {
    extern __shared__ double xs[];
    const int col = blockIdx.x, rhs = col / N, s = col % N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double *l = lam + rhs * lam_rs;
    for (int j = tid; j < n_d; j += 256) {
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int code = gl[((size_t)s * n_d + j) * 2 + u];
            if (code == 0) continue;
            const int row = (code > 0 ? code : -code) - 1;
            const double x = gw ? l[row] * gw[row] : l[row];
            v += code > 0 ? x : -x;
        }
        xs[j] = v;
    }
    __syncthreads();
    const double *Ms = Mops + (size_t)s * n_d * n_d;
    double *y = Y + (size_t)col * n_d;
    // four rows per wave at a time, so each lane keeps several row loads in flight
    for (int r0 = 4 * wave; r0 < n_d; r0 += 16) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c = lane; c < n_d; c += 64) {
            double m[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) m[q] = r0 + q < n_d ? __builtin_nontemporal_load(Ms + (size_t)(r0 + q) * n_d + c) : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += m[q] * xs[c];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (r0 + q < n_d) y[r0 + q] = acc[q];
    }
}

// out[col][a] = K_pr^(s)[a] . x_r^(s)  (col = rhs*N + s; x cell-major with load-case stride x_rs)
__global__ __launch_bounds__(256) void k_ex_kpr_mv(const double *__restrict__ Kpr, const double *__restrict__ x,
                                                   long long x_rs, int N, int n_r, int n_p,
                                                   double *__restrict__ out) {
    const int col = blockIdx.x, rhs = col / N, s = col % N, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double *xs = x + rhs * x_rs + (size_t)s * n_r;
    for (int a = wave; a < n_p; a += 4) {
        const double *k = Kpr + ((size_t)s * n_p + a) * n_r;
        double acc = 0.0;
        for (int j = lane; j < n_r; j += 64) acc += k[j] * xs[j];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) out[(size_t)col * n_p + a] = acc;
    }
}

// W[col][j] = X_r^(s)[n_i + j] + Yc[col][j]  (the dual part of a cell vector plus a correction)
__global__ __launch_bounds__(256) void k_ex_dual_plus(const double *__restrict__ X, long long x_rs,
                                                      const double *__restrict__ Yc, int N, int n_r, int n_i,
                                                      int n_d, int nrhs, double *__restrict__ W) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)N * nrhs * n_d) return;
    const long long col = t / n_d;
    const int j = (int)(t % n_d), rhs = (int)(col / N), s = (int)(col % N);
    W[t] = X[rhs * x_rs + (size_t)s * n_r + n_i + j] + Yc[t];
}

// u_r^(s) = f_r^(s) - K_rp^(s) u_p^(s) - B_d^(s)T lam, the right-hand side of (20) before K_rr^-1
__global__ __launch_bounds__(256) void k_ex_rhs_u(const double *__restrict__ f, long long f_rs,
                                                  const double *__restrict__ Kpr, const int *__restrict__ Ap,
                                                  const int *__restrict__ gl, const double *__restrict__ lam,
                                                  long long lam_rs, int N, int n_r, int n_p, int n_i, int n_d,
                                                  double *__restrict__ u, long long u_rs) {
    __shared__ double up[kExMaxNp];
    const int col = blockIdx.x, rhs = col / N, s = col % N;
    double *ur = u + rhs * u_rs;
    const double *uP = ur + (size_t)N * n_r;
    if (threadIdx.x < n_p) {
        const int P = Ap[(size_t)s * n_p + threadIdx.x];
        up[threadIdx.x] = P >= 0 ? uP[P] : 0.0;
    }
    __syncthreads();
    const double *fr = f + rhs * f_rs + (size_t)s * n_r;
    const double *l = lam + rhs * lam_rs;
    for (int j = threadIdx.x; j < n_r; j += 256) {
        double v = fr[j];
        for (int a = 0; a < n_p; ++a) v -= Kpr[((size_t)s * n_p + a) * n_r + j] * up[a];
        if (j >= n_i) {
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                const int code = gl[((size_t)s * n_d + (j - n_i)) * 2 + w];
                if (code == 0) continue;
                const double x = l[(code > 0 ? code : -code) - 1];
                v -= code > 0 ? x : -x;
            }
        }
        ur[(size_t)s * n_r + j] = v;
    }
}

// dense lower (column-major) from the symmetric band band[i][i-j] (width bw+1); zero outside the band
__global__ __launch_bounds__(256) void k_band_to_dense(const double *__restrict__ band, int n, int bw,
                                                       double *__restrict__ A) {
    const int col = blockIdx.x;
    for (int row = col + threadIdx.x; row < n; row += 256)
        A[(size_t)col * n + row] = row - col <= bw ? band[(size_t)row * (bw + 1) + (row - col)] : 0.0;
}

// band[i][i-j] = L[i][j] for j >= i - bw, from the dense lower factor
__global__ __launch_bounds__(256) void k_dense_to_band(const double *__restrict__ A, int n, int bw,
                                                       double *__restrict__ band) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)n * (bw + 1)) return;
    const int i = (int)(t / (bw + 1)), d = (int)(t % (bw + 1)), j = i - d;
    band[t] = j >= 0 ? A[(size_t)j * n + i] : 0.0;
}

// out = a + sb * b per load case
__global__ __launch_bounds__(256) void k_ex_axpy(const double *__restrict__ a, const double *__restrict__ b,
                                                 double *__restrict__ out, long long n, double sb) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) out[t] = a[t] + sb * b[t];
}

int nblk(long long n) { return (int)((n + 255) / 256); }

void trsv_cells(ifeti_ctx *c, double *X, long long x_rs, int nrhs) {
    const int nr = c->n_r;
    Prof prof(c, "exact_trsv", 2.0 * (double)c->N * nr * nr * nrhs, 8.0 * (double)c->N * nr * nr * 2.0 * nrhs);
    hipLaunchKernelGGL(k_ex_trsv, dim3(c->N, nrhs), dim3(256), (size_t)(nr + 256) * sizeof(double), c->stream,
                       c->ex_L.p, nr, c->N, X, x_rs);
    IFETI_HIP(hipGetLastError());
}

void cell_gemv(ifeti_ctx *c, const double *Mops, const double *lam, bool weights, double *Y, int nrhs,
               const char *tag) {
    const int N = c->N, nd = c->n_d;
    Prof prof(c, tag, 2.0 * (double)N * nd * nd * nrhs,
              8.0 * ((double)N * nd * nd * nrhs + (double)N * nd * nrhs + (double)c->L * nrhs) +
                  8.0 * (double)N * nd);
    hipLaunchKernelGGL(k_ex_cell_gemv, dim3(N * nrhs), dim3(256), (size_t)nd * sizeof(double), c->stream, Mops,
                       c->g_gather.p, weights ? c->g_Dw.p : nullptr, lam, (long long)c->L, N, nd, Y);
    IFETI_HIP(hipGetLastError());
}

}  // namespace

// Batched factorisation of the augmented matrices of ncell list entries (cells[k], or k when cells
// is null), q block = the r rows [q_lo, q_lo + n_q); outputs per list entry (see FactorOut).
void factor_cells(ifeti_ctx *c, const int *cells, int ncell, int q_lo, int n_q, const FactorOut &o) {
    const int nr = c->n_r, np = c->n_p, ni = c->n_i, nd = c->n_d, dim = c->dim;
    const RefTables &R = c->ref;
    const int na = nr + np + n_q, lda = na;
    const size_t cell_elems = (size_t)lda * na;
    // batch of entries whose augmented matrices fit a fixed workspace
    const size_t budget = (size_t)6 << 30;
    const int batch =
        (int)std::max<size_t>(1, std::min<size_t>((size_t)ncell, budget / (cell_elems * sizeof(double))));
    DevBuf<double> A;
    A.alloc(cell_elems * batch);
    DevBuf<int> bad;
    bad.alloc(ncell);
    IFETI_HIP(hipMemsetAsync(bad.p, 0, (size_t)ncell * sizeof(int), c->stream));
    for (int k0 = 0; k0 < ncell; k0 += batch) {
        const int nb_cells = std::min(batch, ncell - k0);
        {
            Prof prof(c, "exact_densify", 0.0, 8.0 * (double)nb_cells * na * (na + 1) / 2);
            const dim3 grid((na + 3) / 4, nb_cells);
            if (dim == 2)
                hipLaunchKernelGGL(k_ex_densify<2>, grid, dim3(256), 0, c->stream, c->Kst.p, cells, k0, nr, np, q_lo,
                                   na, lda, c->g_idx_r.p, c->g_idx_p.p, R.nc, R.n_ctrl, R.n_off, R.p, A.p, o.Kpr,
                                   o.Kpp);
            else
                hipLaunchKernelGGL(k_ex_densify<3>, grid, dim3(256), 0, c->stream, c->Kst.p, cells, k0, nr, np, q_lo,
                                   na, lda, c->g_idx_r.p, c->g_idx_p.p, R.nc, R.n_ctrl, R.n_off, R.p, A.p, o.Kpr,
                                   o.Kpp);
            IFETI_HIP(hipGetLastError());
        }
        for (int j0 = 0; j0 < nr;) {
            const int j1 = std::min(j0 + XB, j0 < ni ? ni : nr);
            const int nbp = j1 - j0;
            if (j0 == ni && o.Sdd) {
                hipLaunchKernelGGL(k_ex_snap_sdd, dim3(nb_cells), dim3(256), 0, c->stream, A.p, lda, na, ni, nd, k0,
                                   o.Sdd);
                IFETI_HIP(hipGetLastError());
            }
            {
                Prof prof(c, "exact_panel", (double)nb_cells * ((double)nbp * nbp * nbp / 3.0 +
                                                                 (double)(na - j1) * nbp * nbp),
                          16.0 * (double)nb_cells * (na - j0) * nbp);
                hipLaunchKernelGGL(k_ex_panel, dim3(nb_cells), dim3(256), 0, c->stream, A.p, lda, na, j0, nbp, k0,
                                   bad.p);
                IFETI_HIP(hipGetLastError());
            }
            if (j1 < na) {
                const long long t = na - j1, T = (t + 63) / 64, tiles = T * (T + 1) / 2;
                Prof prof(c, "exact_syrk", (double)nb_cells * (double)t * (t + 1) * nbp,
                          16.0 * (double)nb_cells * ((double)t * (t + 1) / 2 + (double)t * nbp));
                hipLaunchKernelGGL(k_ex_syrk, dim3((unsigned)tiles, nb_cells), dim3(256), 0, c->stream, A.p, lda, na,
                                   j0, nbp, (int)j1);
                IFETI_HIP(hipGetLastError());
            }
            j0 = j1;
        }
        hipLaunchKernelGGL(k_ex_extract, dim3(nb_cells), dim3(256), 0, c->stream, A.p, lda, na, nr, np, n_q, k0, o.Fq,
                           o.Spp, o.UqT, o.L);
        IFETI_HIP(hipGetLastError());
    }
    std::vector<int> hbad(ncell);
    IFETI_HIP(hipMemcpyAsync(hbad.data(), bad.p, (size_t)ncell * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipStreamSynchronize(c->stream));
    for (int k = 0; k < ncell; ++k) IFETI_REQUIRE(!hbad[k], IFETI_ENOTSPD, "a cell's K_rr is not positive definite");
}

// Cholesky factor of a symmetric positive definite band matrix on the GPU: the band is expanded
// to a dense lower matrix and eliminated with the blocked panel and trailing-update kernels of the
// cell factorisations; the factor keeps the band, which is returned in the same band form.
std::vector<double> band_cholesky_device(ifeti_ctx *c, const std::vector<double> &band, int n, int bw) {
    std::vector<double> out;
    if (n == 0) return out;
    DevBuf<double> db, A;
    DevBuf<int> bad;
    db.upload(band, c->stream);
    A.alloc((size_t)n * n);
    bad.alloc(1);
    bad.zero(c->stream);
    hipLaunchKernelGGL(k_band_to_dense, dim3(n), dim3(256), 0, c->stream, db.p, n, bw, A.p);
    IFETI_HIP(hipGetLastError());
    for (int j0 = 0; j0 < n; j0 += XB) {
        const int j1 = std::min(n, j0 + XB), nbp = j1 - j0;
        hipLaunchKernelGGL(k_ex_panel, dim3(1), dim3(256), 0, c->stream, A.p, n, n, j0, nbp, 0, bad.p);
        if (j1 < n) {
            const long long t = n - j1, T = (t + 63) / 64, tiles = T * (T + 1) / 2;
            hipLaunchKernelGGL(k_ex_syrk, dim3((unsigned)tiles, 1), dim3(256), 0, c->stream, A.p, n, n, j0, nbp,
                               (int)j1);
        }
        IFETI_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_dense_to_band, dim3(nblk((long long)n * (bw + 1))), dim3(256), 0, c->stream, A.p, n, bw,
                       db.p);
    IFETI_HIP(hipGetLastError());
    db.download(out, c->stream);
    int hbad = 0;
    IFETI_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipStreamSynchronize(c->stream));
    IFETI_REQUIRE(!hbad, IFETI_ENOTSPD, "coarse matrix S_PP is not positive definite");
    return out;
}

void build_exact(ifeti_ctx *c) {
    const int N = c->N, nr = c->n_r, np = c->n_p, nd = c->n_d;
    IFETI_REQUIRE(np <= kExMaxNp, IFETI_EINVAL, "too many primal dofs per cell");
    c->ex_L.alloc((size_t)N * nr * nr);
    c->ex_Fdd.alloc((size_t)N * nd * nd);
    c->ex_Sdd.alloc((size_t)N * nd * nd);
    c->ex_C.alloc((size_t)N * np * nd);
    c->ex_Spp.alloc((size_t)N * np * np);
    c->ex_Kpr.alloc((size_t)N * np * nr);
    FactorOut o;
    o.L = c->ex_L.p;
    o.Fq = c->ex_Fdd.p;
    o.Sdd = c->ex_Sdd.p;
    o.UqT = c->ex_C.p;
    o.Spp = c->ex_Spp.p;
    o.Kpr = c->ex_Kpr.p;
    factor_cells(c, nullptr, N, c->n_i, nd, o);
    std::vector<double> Spp((size_t)N * np * np);
    IFETI_HIP(hipMemcpyAsync(Spp.data(), c->ex_Spp.p, Spp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipStreamSynchronize(c->stream));
    // assembled S_PP (eq. (22)) in band form, then its own coarse solver
    const int nP = c->nP;
    int bw = 0;
    for (int s = 0; s < N; ++s)
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
                const int I = c->h_Ap[(size_t)s * np + a], J = c->h_Ap[(size_t)s * np + b];
                if (I >= 0 && J >= 0) bw = std::max(bw, std::abs(I - J));
            }
    std::vector<double> band((size_t)nP * (bw + 1), 0.0);
    for (int s = 0; s < N; ++s) {
        const double *X = &Spp[(size_t)s * np * np];
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
                const int I = c->h_Ap[(size_t)s * np + a], J = c->h_Ap[(size_t)s * np + b];
                if (I < 0 || J < 0 || J > I) continue;
                band[(size_t)I * (bw + 1) + (I - J)] += 0.5 * (X[a * np + b] + X[b * np + a]);
            }
    }
    c->co_ex.h_Sband = band;
    c->co_ex.bw = bw;
    if (nP > 0) {
        c->co_ex.h_bandL = band_cholesky_device(c, band, nP, bw);  // explicit inverse on first use
        c->co_ex.inv_ready = false;
        build_coarse_partition(c, c->co_ex);
    }
    IFETI_HIP(hipStreamSynchronize(c->stream));
    c->ex_built = true;
}

void apply_F_exact(ifeti_ctx *c, const double *lam, double *out, int nrhs, const double *dot_w, double *dot_part) {
    ensure_work(c, nrhs);
    const int N = c->N, nd = c->n_d;
    {
        // the per-cell products run beside the coarse branch, into their own buffer
        SideStream side(c);
        cell_gemv(c, c->ex_Fdd.p, lam, false, c->w_Y.p, nrhs, "exact_F_cells");
    }
    op_restrict_cells(c, c->ex_C.p, lam, c->L, c->w_c.p, nrhs, "exact_restrict");
    op_assemble_primal(c, c->w_c.p, nullptr, 0, 1.0, c->w_zP.p, c->nP, nrhs);
    coarse_solve(c, c->co_ex, c->w_zP.p, c->nP, c->w_yP.p, c->nP, nrhs, 1.0);
    op_prolong_cells(c, c->ex_C.p, c->w_yP.p, c->nP, c->w_Yc.p, nrhs, false, "exact_prolong");
    join_side(c);
    op_scatter(c, c->w_Y.p, nd, 0, (long long)N * nd, out, c->L, nrhs, false, dot_w, dot_part, c->w_Yc.p);
    c->applies[IFETI_OP_F] += nrhs;
}

void apply_MD_exact(ifeti_ctx *c, const double *r, double *out, int nrhs, const double *dot_w, double *dot_part) {
    ensure_work(c, nrhs);
    const int N = c->N, nd = c->n_d;
    cell_gemv(c, c->ex_Sdd.p, r, true, c->w_Y.p, nrhs, "exact_MD_cells");
    op_scatter(c, c->w_Y.p, nd, 0, (long long)N * nd, out, c->L, nrhs, true, dot_w, dot_part);
    c->applies[IFETI_OP_MD] += nrhs;
}

// Standard FETI-DP solve (Sec. 2.2.4): d̄ of (25), interface PCG on F (24) with M_D (30), then
// u_P from (21) and u_R from (20).
int solve_exact(ifeti_ctx *c, const double *f, const double *d, double *u, double *lam, int nrhs, double tol,
                int maxit, int *iters, double *relres) {
    ensure_work(c, nrhs);
    const int N = c->N, nr = c->n_r, np = c->n_p, ni = c->n_i, nd = c->n_d, nP = c->nP;
    const long long nU = c->nU, L = c->L, NR = (long long)N * nr;
    hipStream_t s = c->stream;
    c->ex_w.ensure((size_t)NR * nrhs, s);
    c->ex_g.ensure((size_t)std::max(nP, 1) * nrhs, s);
    c->ex_z.ensure((size_t)std::max(nP, 1) * nrhs, s);
    c->ex_d.ensure((size_t)L * nrhs, s);
    // K_RR^-1 f_R
    IFETI_HIP(hipMemcpy2DAsync(c->ex_w.p, NR * sizeof(double), f, nU * sizeof(double), NR * sizeof(double), nrhs,
                               hipMemcpyDeviceToDevice, s));
    trsv_cells(c, c->ex_w.p, NR, nrhs);
    // g = f_P - A_p^T K_pr K_RR^-1 f_R
    hipLaunchKernelGGL(k_ex_kpr_mv, dim3(N * nrhs), dim3(256), 0, s, c->ex_Kpr.p, c->ex_w.p, NR, N, nr, np, c->w_c.p);
    op_assemble_primal(c, c->w_c.p, f + NR, nU, -1.0, c->ex_g.p, nP, nrhs);
    // d̄ = B_R (K_RR^-1 f_R - K_RR^-1 K_RP S_PP^-1 g) - d, dual rows only
    coarse_solve(c, c->co_ex, c->ex_g.p, nP, c->ex_z.p, nP, nrhs, -1.0);
    op_prolong_cells(c, c->ex_C.p, c->ex_z.p, nP, c->w_Yc.p, nrhs, false, "exact_prolong");
    hipLaunchKernelGGL(k_ex_dual_plus, dim3(nblk((long long)N * nrhs * nd)), dim3(256), 0, s, c->ex_w.p, NR,
                       c->w_Yc.p, N, nr, ni, nd, nrhs, c->w_Y.p);
    op_scatter(c, c->w_Y.p, nd, 0, (long long)N * nd, c->ex_d.p, L, nrhs, false);
    hipLaunchKernelGGL(k_ex_axpy, dim3(nblk(L * nrhs)), dim3(256), 0, s, c->ex_d.p, d, c->ex_d.p, L * nrhs, -1.0);
    IFETI_HIP(hipGetLastError());
    const int st = solve_interface(c, c->ex_d.p, lam, nrhs, tol, maxit, iters, relres, true);
    if (st != IFETI_OK && st != IFETI_EMAXIT) return st;
    // u_P = S_PP^-1 (g + A_p^T U_d^T B_d^T lam)      (21)
    op_restrict_cells(c, c->ex_C.p, lam, L, c->w_c.p, nrhs, "exact_restrict");
    op_assemble_primal(c, c->w_c.p, c->ex_g.p, nP, 1.0, c->ex_z.p, nP, nrhs);
    coarse_solve(c, c->co_ex, c->ex_z.p, nP, u + NR, nU, nrhs, 1.0);
    // u_R = K_RR^-1 (f_R - K_RP u_P - B_R^T lam)       (20)
    hipLaunchKernelGGL(k_ex_rhs_u, dim3(N * nrhs), dim3(256), 0, s, f, nU, c->ex_Kpr.p, c->g_Ap.p, c->g_gather.p, lam,
                       L, N, nr, np, ni, nd, u, nU);
    IFETI_HIP(hipGetLastError());
    trsv_cells(c, u, nU, nrhs);
    IFETI_HIP(hipStreamSynchronize(s));
    return st;
}

}  // namespace ifeti
