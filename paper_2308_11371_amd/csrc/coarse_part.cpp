// Partitioned direct solve of the assembled coarse problem S̊_PP y = z (Sec. 3.2.1).
//
// The paper factorises S̊_PP once and applies it by forward and backward
// substitution.  On the GPU the substitutions are a chain of n dependent steps,
// and the explicit inverse streams n^2/2 doubles per apply.  In the
// lexicographic vertex order S̊_PP is banded (half-bandwidth bw), so any bw
// consecutive rows separate the rows before them from the rows after them.
// The rows are cut into p interior blocks I_i with a separator S_j of bw rows
// between blocks j and j+1.  Block elimination of the interiors gives, exactly
// (up to rounding):
//
//   E_i   = A_{S,I_i} A_{I_i}^-1                       (bw x m_i for each adjacent separator)
//   S_ss  = A_{SS} - sum_i E_i A_{I_i,S}                (separator Schur complement)
//   g_j   = z_{S_j} - E_j^R z_{I_j} - E_{j+1}^L z_{I_{j+1}}                   (phase 1)
//   u     = S_ss^-1 g,        y_S = u                                          (phase 2)
//   y_I_i = A_{I_i}^-1 z_{I_i} - (E_i^L)^T u_{S_{i-1}} - (E_i^R)^T u_{S_i}     (phase 3)
//
// Each phase is a set of independent dense rows (one dot product per output
// row over a contiguous range of its input), stored row-major with a row
// descriptor, so an apply streams sum_j bw (m_j + bw + m_{j+1}) + ns^2 +
// sum_i m_i (m_i + 2 bw) doubles instead of n^2/2.  p is chosen to minimise
// those bytes; for bands too wide to gain (3D lexicographic orders), the
// symmetric-tile inverse stays in use.
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

namespace ifeti {
namespace {

template <class F>
void par_for(int n, F f) {
    unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    int nt = std::min<int>(n, (int)hw);
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int i = t; i < n; i += nt) f(i);
        });
    for (auto &x : th) x.join();
}

// entry (i, j) of the symmetric band matrix stored as its lower band [i][i-j]
struct Band {
    const std::vector<double> &b;
    int n, bw;
    double operator()(int i, int j) const {
        if (i < j) std::swap(i, j);
        const int d = i - j;
        return d > bw ? 0.0 : b[(size_t)i * (bw + 1) + d];
    }
};

// Banded Cholesky of rows [lo, lo+m) of the band matrix: L[i][i-j] (local indices).
std::vector<double> band_chol(const Band &A, int lo, int m) {
    const int bw = A.bw;
    std::vector<double> L((size_t)m * (bw + 1), 0.0);
    for (int i = 0; i < m; ++i)
        for (int d = 0; d <= std::min(bw, i); ++d) L[(size_t)i * (bw + 1) + d] = A(lo + i, lo + i - d);
    for (int j = 0; j < m; ++j) {
        double s = L[(size_t)j * (bw + 1)];
        for (int k = std::max(0, j - bw); k < j; ++k) {
            const double l = L[(size_t)j * (bw + 1) + (j - k)];
            s -= l * l;
        }
        IFETI_REQUIRE(s > 0.0, IFETI_ENOTSPD, "coarse block is not positive definite");
        const double ljj = std::sqrt(s);
        L[(size_t)j * (bw + 1)] = ljj;
        for (int i = j + 1; i <= std::min(m - 1, j + bw); ++i) {
            double t = L[(size_t)i * (bw + 1) + (i - j)];
            for (int k = std::max(0, i - bw); k < j; ++k)
                t -= L[(size_t)i * (bw + 1) + (i - k)] * L[(size_t)j * (bw + 1) + (j - k)];
            L[(size_t)i * (bw + 1) + (i - j)] = t / ljj;
        }
    }
    return L;
}

struct Layout {
    int p = 0, ns = 0;
    std::vector<int> lo, hi;  // interior block i = [lo, hi); separator j = [hi[j], lo[j+1])
    double bytes = 0.0;
};

Layout layout(int n, int bw, int p) {
    Layout L;
    L.p = p;
    L.ns = (p - 1) * bw;
    const int rest = n - L.ns;
    if (p < 2 || rest < 2 * p) return L;  // too many blocks for the band: unusable
    int at = 0;
    for (int i = 0; i < p; ++i) {
        const int m = rest / p + (i < rest % p ? 1 : 0);
        L.lo.push_back(at);
        L.hi.push_back(at + m);
        at += m + (i + 1 < p ? bw : 0);
    }
    double d = (double)L.ns * L.ns;
    for (int j = 0; j + 1 < p; ++j) d += (double)bw * ((L.hi[j] - L.lo[j]) + bw + (L.hi[j + 1] - L.lo[j + 1]));
    for (int i = 0; i < p; ++i) {
        const int m = L.hi[i] - L.lo[i];
        d += (double)m * (m + (i > 0 ? bw : 0) + (i + 1 < p ? bw : 0));
    }
    L.bytes = 8.0 * d;
    return L;
}

}  // namespace

// Block-Jacobi approximation of S̊_PP^-1 (the approximative coarse solvers of Sec. 3.2.1): the inverse
// of each diagonal block of B consecutive rows, every row of it one output row of a single streamed
// phase (n B doubles per apply instead of the partitioned solve's three dependent phases).
void build_coarse_approx(ifeti_ctx *c, CoarseSolver &co) {
    IFETI_HIP(hipStreamSynchronize(c->stream));
    release_graph(c);  // a captured PCG iteration may hold the previous tables
    ++c->rom_gen;
    co.ap_B = 0;
    const int n = c->nP, bw = co.bw, B = c->opt.coarse_approx;
    if (B <= 0 || n == 0) {
        co.ap_M.release();
        co.ap_R.release();
        return;
    }
    const Band A{co.h_Sband, n, bw};
    std::vector<double> M;
    std::vector<CoarseRow> R;
    for (int lo = 0; lo < n; lo += B) {
        const int m = std::min(B, n - lo);
        const std::vector<double> inv = band_inverse_device(c, band_chol(A, lo, m), m, bw);
        for (int q = 0; q < m; ++q) {
            R.push_back(CoarseRow{(long long)M.size(), lo, m, lo + q, 0});
            for (int t = 0; t < m; ++t)  // symmetrised
                M.push_back(0.5 * (inv[(size_t)q * m + t] + inv[(size_t)t * m + q]));
        }
    }
    co.ap_M.upload(M, c->stream);
    co.ap_R.upload(R, c->stream);
    IFETI_HIP(hipStreamSynchronize(c->stream));
    co.ap_B = B;
}

std::vector<double> band_cholesky(const std::vector<double> &band, int n, int bw) {
    const Band A{band, n, bw};
    return band_chol(A, 0, n);
}

void build_coarse_partition(ifeti_ctx *c, CoarseSolver &co) {
    // a captured PCG iteration holds the partition's buffers and row counts: drop it
    IFETI_HIP(hipStreamSynchronize(c->stream));
    release_graph(c);
    ++c->rom_gen;
    co.cp_p = 0;
    co.cp_ns = 0;
    const int n = c->nP, bw = co.bw;
    if (n == 0 || c->opt.coarse_parts == 1) return;
    Layout best;
    if (c->opt.coarse_parts >= 2) {
        best = layout(n, bw, c->opt.coarse_parts);
        IFETI_REQUIRE(!best.lo.empty(), IFETI_EINVAL, "coarse_parts too large for the coarse band");
    } else {
        // automatic: fewest streamed bytes, and clearly below the symmetric-tile inverse (which also
        // gets by with one pass and a short reduction)
        for (int p = 2; p <= 64; ++p) {
            Layout l = layout(n, bw, p);
            if (!l.lo.empty() && (best.lo.empty() || l.bytes < best.bytes)) best = l;
        }
        const double sym = 8.0 * (double)n * (n + 1) / 2;
        if (best.lo.empty() || best.bytes > 0.6 * sym) return;
    }
    const int p = best.p, ns = best.ns;
    const Band A{co.h_Sband, n, bw};
    // interior inverses and their couplings to the adjacent separators
    std::vector<std::vector<double>> Ainv(p), EL(p), ER(p);
    for (int i = 0; i < p; ++i) {
        const int lo = best.lo[i], m = best.hi[i] - lo;
        std::vector<double> &X = Ainv[i];
        X = band_inverse_device(c, band_chol(A, lo, m), m, bw);
        for (int r = 0; r < m; ++r)  // symmetrise
            for (int q = r + 1; q < m; ++q) {
                const double v = 0.5 * (X[(size_t)r * m + q] + X[(size_t)q * m + r]);
                X[(size_t)r * m + q] = X[(size_t)q * m + r] = v;
            }
        // E^L = A_{S_{i-1}, I_i} A^-1: separator row lo-bw+t couples to interior columns k <= t
        if (i > 0) {
            EL[i].assign((size_t)bw * m, 0.0);
            par_for(bw, [&](int t) {
                for (int k = 0; k <= std::min(t, m - 1); ++k) {
                    const double a = A(lo - bw + t, lo + k);
                    if (a == 0.0) continue;
                    for (int q = 0; q < m; ++q) EL[i][(size_t)t * m + q] += a * X[(size_t)k * m + q];
                }
            });
        }
        // E^R = A_{S_i, I_i} A^-1: separator row hi+t couples to interior columns k >= m+t-bw
        if (i + 1 < p) {
            ER[i].assign((size_t)bw * m, 0.0);
            par_for(bw, [&](int t) {
                for (int k = std::max(0, m + t - bw); k < m; ++k) {
                    const double a = A(lo + m + t, lo + k);
                    if (a == 0.0) continue;
                    for (int q = 0; q < m; ++q) ER[i][(size_t)t * m + q] += a * X[(size_t)k * m + q];
                }
            });
        }
    }
    // separator Schur complement S_ss = A_SS - sum_i E_i A_{I_i,S}; separator row (j, t) -> j*bw + t
    auto grow = [&](int s) { return best.hi[s / bw] + s % bw; };
    std::vector<double> S((size_t)ns * ns, 0.0);
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) S[(size_t)a * ns + b] = A(grow(a), grow(b));
    for (int i = 0; i < p; ++i) {
        const int lo = best.lo[i], m = best.hi[i] - lo;
        // (E_x A_{I,Sy})[t][t2] = sum_k E_x[t][k] A(lo+k, row of Sy t2)
        auto sub = [&](const std::vector<double> &E, int jx, int jy) {
            par_for(bw, [&](int t) {
                for (int t2 = 0; t2 < bw; ++t2) {
                    const int r2 = best.hi[jy] + t2;
                    double s = 0.0;
                    for (int k = std::max(0, r2 - lo - bw); k <= std::min(m - 1, r2 - lo + bw); ++k)
                        s += E[(size_t)t * m + k] * A(lo + k, r2);
                    S[(size_t)(jx * bw + t) * ns + jy * bw + t2] -= s;
                }
            });
        };
        if (i > 0) sub(EL[i], i - 1, i - 1);
        if (i + 1 < p) sub(ER[i], i, i);
        if (i > 0 && i + 1 < p) {
            sub(EL[i], i - 1, i);
            sub(ER[i], i, i - 1);
        }
    }
    for (int a = 0; a < ns; ++a)  // symmetrise
        for (int b = a + 1; b < ns; ++b) {
            const double v = 0.5 * (S[(size_t)a * ns + b] + S[(size_t)b * ns + a]);
            S[(size_t)a * ns + b] = S[(size_t)b * ns + a] = v;
        }
    // S_ss is block tridiagonal (bandwidth < 2 bw): banded factor, inverse by columns
    std::vector<double> Sb((size_t)ns * (2 * bw + 1), 0.0);
    const int sbw = 2 * bw;
    for (int a = 0; a < ns; ++a)
        for (int d = 0; d <= std::min(sbw, a); ++d) Sb[(size_t)a * (sbw + 1) + d] = S[(size_t)a * ns + a - d];
    const Band SB{Sb, ns, sbw};
    std::vector<double> Sinv = band_inverse_device(c, band_chol(SB, 0, ns), ns, sbw);
    for (int a = 0; a < ns; ++a)
        for (int b = a + 1; b < ns; ++b) {
            const double v = 0.5 * (Sinv[(size_t)a * ns + b] + Sinv[(size_t)b * ns + a]);
            Sinv[(size_t)a * ns + b] = Sinv[(size_t)b * ns + a] = v;
        }
    // phase rows
    std::vector<double> M1, M3;
    std::vector<CoarseRow> R1, R2, R3;
    for (int j = 0; j + 1 < p; ++j) {
        const int m0 = best.hi[j] - best.lo[j], m1 = best.hi[j + 1] - best.lo[j + 1];
        for (int t = 0; t < bw; ++t) {
            CoarseRow r{(long long)M1.size(), best.lo[j], m0 + bw + m1, j * bw + t, 0};
            M1.insert(M1.end(), &ER[j][(size_t)t * m0], &ER[j][(size_t)(t + 1) * m0]);
            for (int q = 0; q < bw; ++q) M1.push_back(q == t ? -1.0 : 0.0);
            M1.insert(M1.end(), &EL[j + 1][(size_t)t * m1], &EL[j + 1][(size_t)(t + 1) * m1]);
            R1.push_back(r);
        }
    }
    for (int s = 0; s < ns; ++s) R2.push_back(CoarseRow{(long long)s * ns, 0, ns, grow(s), 0});
    for (int i = 0; i < p; ++i) {
        const int lo = best.lo[i], m = best.hi[i] - lo;
        const int bl = i > 0 ? bw : 0, br = i + 1 < p ? bw : 0;
        for (int q = 0; q < m; ++q) {
            R3.push_back(CoarseRow{(long long)M3.size(), lo - bl, bl + m + br, lo + q, 0});
            for (int t = 0; t < bl; ++t) M3.push_back(-EL[i][(size_t)t * m + q]);
            M3.insert(M3.end(), &Ainv[i][(size_t)q * m], &Ainv[i][(size_t)(q + 1) * m]);
            for (int t = 0; t < br; ++t) M3.push_back(-ER[i][(size_t)t * m + q]);
        }
    }
    // tiles of up to 16 consecutive rows with one input range (one MFMA row tile each)
    auto tiles = [](const std::vector<CoarseRow> &R) {
        std::vector<CoarseTile> T;
        for (int i = 0; i < (int)R.size();) {
            int j = i + 1;
            while (j < (int)R.size() && j - i < 16 && R[j].xlo == R[i].xlo && R[j].len == R[i].len &&
                   R[j].off == R[j - 1].off + R[i].len)
                ++j;
            T.push_back(CoarseTile{i, j - i});
            i = j;
        }
        return T;
    };
    co.cp_M1.upload(M1, c->stream);
    co.cp_M2.upload(Sinv, c->stream);
    co.cp_M3.upload(M3, c->stream);
    co.cp_R1.upload(R1, c->stream);
    co.cp_R2.upload(R2, c->stream);
    co.cp_R3.upload(R3, c->stream);
    const std::vector<CoarseTile> T1 = tiles(R1), T2 = tiles(R2), T3 = tiles(R3);  // live until the sync below
    co.cp_T1.upload(T1, c->stream);
    co.cp_T2.upload(T2, c->stream);
    co.cp_T3.upload(T3, c->stream);
    co.w_cg.alloc((size_t)ns * 3);
    co.w_cw.alloc((size_t)n * 3);
    IFETI_HIP(hipStreamSynchronize(c->stream));
    co.cp_p = p;
    co.cp_ns = ns;
}

}  // namespace ifeti
