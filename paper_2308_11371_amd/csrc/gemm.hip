// Principal-shared contraction on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
//   Y[:, c] (+)= sum_g scale_g sum_k coef_g[cell(c), k] * A_{g,k} X_g[:, c]
//
// Every cell (column c; cell = c mod N) combines the same few principal
// operators A_{g,k} with its own coefficients (paper Remark 7: the ROM
// operators of eqs. (48), (49), Algorithm 3 and eq. (46a) as sums over the
// principal cells), so all cells become one dense GEMM whose B operand is
// the cell vectors scaled by the coefficients while being staged.
//
// Tiling: 256 threads = 4 wave64, a TM x TN output tile, wave grid WM x WN;
// each wave owns (TM/WM) x (TN/WN) made of 16x16 MFMA blocks.  A chunk of the
// principal operator (TM x KC) and of the cell vectors (TN x KC) are staged in
// LDS (rows padded by one double against bank conflicts); the coefficient
// scaling is applied when the B fragment is read from LDS.
#include "common.hpp"

namespace ifeti {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

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

template <int TM, int TN, int WM, int WN, int KC>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgsDev g) {
    constexpr int WTM = TM / WM, WTN = TN / WN;
    constexpr int BM = WTM / 16, BN = WTN / 16;
    static_assert(WM * WN == 4, "four waves");
    static_assert(BM >= 1 && BN >= 1, "wave tile >= 16x16");
    __shared__ double As[TM][KC + 1];
    __shared__ double Xs[TN][KC + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int m0 = blockIdx.y * TM, c0 = blockIdx.x * TN;
    const int lr = lane & 15, lk = lane >> 4;

    v4d acc[BM][BN];
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    for (int gi = 0; gi < g.ngroups; ++gi) {
        const double *__restrict__ A = g.A[gi];
        const double *__restrict__ X = g.X[gi];
        const double *__restrict__ coef = g.coef[gi];
        const int Kd = g.Kd[gi], ldx = g.ldx[gi], K = g.K[gi];
        const long long xbs = g.xbs[gi];
        const double scale = g.scale[gi];
        const long long strideA = (long long)g.M * Kd;
        // per-lane cell of each of its B blocks
        int cell[BN];
        bool cvalid[BN];
#pragma unroll
        for (int bn = 0; bn < BN; ++bn) {
            int col = c0 + wn * WTN + bn * 16 + lr;
            cvalid[bn] = col < g.ncols;
            cell[bn] = cvalid[bn] ? col % g.ncells : 0;
        }
        for (int kk = 0; kk < Kd; kk += KC) {
            __syncthreads();
            for (int idx = tid; idx < TN * KC; idx += 256) {
                int n = idx / KC, kc = idx % KC;
                int col = c0 + n, kx = kk + kc;
                Xs[n][kc] = (col < g.ncols && kx < Kd)
                                ? X[(col / g.ncells) * xbs + (size_t)(col % g.ncells) * ldx + kx]
                                : 0.0;
            }
            for (int k = 0; k < K; ++k) {
                __syncthreads();
                const double *__restrict__ Ak = A + (size_t)k * strideA;
                for (int idx = tid; idx < TM * KC; idx += 256) {
                    int m = idx / KC, kc = idx % KC;
                    int row = m0 + m, kx = kk + kc;
                    As[m][kc] = (row < g.M && kx < Kd) ? Ak[(size_t)row * Kd + kx] : 0.0;
                }
                __syncthreads();
                double cf[BN];
#pragma unroll
                for (int bn = 0; bn < BN; ++bn)
                    cf[bn] = scale * (coef ? (cvalid[bn] ? coef[(size_t)cell[bn] * K + k] : 0.0) : 1.0);
#pragma unroll
                for (int kc = 0; kc < KC; kc += 4) {
                    double a[BM], b[BN];
#pragma unroll
                    for (int bm = 0; bm < BM; ++bm) a[bm] = As[wm * WTM + bm * 16 + lr][kc + lk];
#pragma unroll
                    for (int bn = 0; bn < BN; ++bn) b[bn] = Xs[wn * WTN + bn * 16 + lr][kc + lk] * cf[bn];
#pragma unroll
                    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
                        for (int bn = 0; bn < BN; ++bn)
                            acc[bm][bn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bm], b[bn], acc[bm][bn], 0, 0, 0);
                }
            }
        }
    }
    // D layout of the 16x16 f64 MFMA (checked on gfx950): lane l, register i -> row 4*i + l/16, column l % 16
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn) {
            int col = c0 + wn * WTN + bn * 16 + lr;
            if (col >= g.ncols) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int row = m0 + wm * WTM + bm * 16 + 4 * i + lk;
                if (row >= g.M) continue;
                double *y = g.Y + (col / g.ncells) * g.ybs + (size_t)(col % g.ncells) * g.ldy + row;
                *y = g.accumulate ? *y + acc[bm][bn][i] : acc[bm][bn][i];
            }
        }
}

template <int TM, int TN, int WM, int WN, int KC>
void launch(const GemmArgsDev &a, hipStream_t s) {
    dim3 grid((a.ncols + TN - 1) / TN, (a.M + TM - 1) / TM);
    hipLaunchKernelGGL((k_gemm_f64<TM, TN, WM, WN, KC>), grid, dim3(256), 0, s, a);
}

}  // namespace

void gemm(ifeti_ctx *c, const GemmGroup *groups, int ngroups, double *Y, int ldy, long long ybs, int M, int ncols,
          bool accumulate, int ncells, const char *tag) {
    IFETI_REQUIRE(ngroups >= 1 && ngroups <= 2, IFETI_EINVAL, "gemm: 1 or 2 groups");
    if (ncols <= 0 || M <= 0) return;
    GemmArgsDev a{};
    a.ncells = ncells > 0 ? ncells : c->N;
    for (int i = 0; i < ngroups; ++i) {
        a.A[i] = groups[i].A;
        a.X[i] = groups[i].X;
        a.coef[i] = groups[i].coef;
        a.Kd[i] = groups[i].Kd;
        a.ldx[i] = groups[i].ldx;
        a.xbs[i] = groups[i].xbs ? groups[i].xbs : (long long)a.ncells * groups[i].ldx;
        a.K[i] = groups[i].K;
        a.scale[i] = groups[i].scale;
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
        bytes += 8.0 * ((double)groups[i].K * M * groups[i].Kd + (double)ncols * groups[i].Kd +
                        (groups[i].coef ? (double)a.ncells * groups[i].K : 0.0));
    }
    Prof prof(c, tag, flops, bytes);
    // tile choice: keep >= 256 workgroups where the shape allows it
    long long tiles64 = (long long)((ncols + 63) / 64) * ((M + 63) / 64);
    if (M <= 16)
        launch<16, 64, 1, 4, 32>(a, c->stream);
    else if (M <= 32)
        launch<32, 64, 2, 2, 32>(a, c->stream);
    else if (tiles64 >= 512)
        launch<64, 64, 2, 2, 32>(a, c->stream);
    else
        launch<64, 32, 2, 2, 32>(a, c->stream);
    IFETI_HIP(hipGetLastError());
}

}  // namespace ifeti
