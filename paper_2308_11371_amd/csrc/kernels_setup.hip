// Device kernels of the offline phase: pulled-back material tensor and cell
// stiffness (Sec. 4.2.1, eq. (52)), greedy sweeps (Algorithm 4), explicit
// coarse inverse from the banded Cholesky factor (Sec. 3.2.1).
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace ifeti {
namespace {

constexpr int kBlock = 256;

__device__ inline double seg_dist2d(double x, double y, double ax, double ay, double bx, double by) {
    double ux = bx - ax, uy = by - ay;
    double t = ((x - ax) * ux + (y - ay) * uy) / (ux * ux + uy * uy);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    double dx = x - (ax + t * ux), dy = y - (ay + t * uy);
    return sqrt(dx * dx + dy * dy);
}

// Distance from a reference point to the nearest strut axis.  2D: the four
// cell edges and both diagonals (Euclidean); 3D: the twelve cube edges
// (Chebyshev distance across the edge).
template <int D>
__device__ double strut_distance(const double *xi) {
    if constexpr (D == 2) {
        double x = xi[0], y = xi[1];
        double d = seg_dist2d(x, y, 0, 0, 1, 0);
        d = fmin(d, seg_dist2d(x, y, 1, 0, 1, 1));
        d = fmin(d, seg_dist2d(x, y, 1, 1, 0, 1));
        d = fmin(d, seg_dist2d(x, y, 0, 1, 0, 0));
        d = fmin(d, seg_dist2d(x, y, 0, 0, 1, 1));
        d = fmin(d, seg_dist2d(x, y, 1, 0, 0, 1));
        return d;
    } else {
        double best = 1e300;
        for (int axis = 0; axis < 3; ++axis) {
            int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
            for (int c1 = 0; c1 < 2; ++c1)
                for (int c2 = 0; c2 < 2; ++c2) {
                    double d = fmax(fabs(xi[o1] - c1), fabs(xi[o2] - c2));
                    best = fmin(best, d);
                }
        }
        return best;
    }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_pulled_back(const double *__restrict__ ctrl,
                                                        const double *__restrict__ widths,
                                                        const double *__restrict__ xi,
                                                        const double *__restrict__ dN,
                                                        const int *__restrict__ elem_ctrl, int N, int nE, int nq,
                                                        int nloc, int n_ctrl, double E_in, double E_out, double nu,
                                                        double eps, double h, double *__restrict__ snap,
                                                        int *__restrict__ bad) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long total = (long long)N * nE * nq;
    if (t >= total) return;
    int q = (int)(t % nq);
    int E = (int)((t / nq) % nE);
    int s = (int)(t / ((long long)nq * nE));
    double J[D][D];
#pragma unroll
    for (int m = 0; m < D; ++m)
#pragma unroll
        for (int j = 0; j < D; ++j) J[m][j] = 0.0;
    const double *dNq = dN + (size_t)(E * nq + q) * nloc * D;
    for (int l = 0; l < nloc; ++l) {
        int a = elem_ctrl[E * nloc + l];
        const double *P = ctrl + ((size_t)s * n_ctrl + a) * D;
#pragma unroll
        for (int m = 0; m < D; ++m)
#pragma unroll
            for (int j = 0; j < D; ++j) J[m][j] += P[m] * dNq[l * D + j];
    }
    double det, G[D][D];  // G = J^-1, G[j][m]
    if constexpr (D == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        G[0][0] = J[1][1] / det;
        G[0][1] = -J[0][1] / det;
        G[1][0] = -J[1][0] / det;
        G[1][1] = J[0][0] / det;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        G[0][0] = c00 / det;
        G[1][0] = c01 / det;
        G[2][0] = c02 / det;
        G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    if (!(det > 0.0)) atomicOr(bad, 1);
    // ersatz material: E_in inside the struts, E_out elsewhere (optionally tanh-smoothed)
    double dist = strut_distance<D>(xi + (size_t)(E * nq + q) * D) * h;
    double half = 0.5 * widths[s];
    double Ey;
    if (eps > 0.0)
        Ey = E_out + (E_in - E_out) * 0.5 * (1.0 + tanh((half - dist) / eps));
    else
        Ey = dist < half ? E_in : E_out;
    double lam = Ey * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double mu = Ey / (2.0 * (1.0 + nu));
    double *out = snap + (size_t)t * D * D * D * D;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j)
#pragma unroll
            for (int k = 0; k < D; ++k)
#pragma unroll
                for (int l = 0; l < D; ++l) {
                    double gg = 0.0;
#pragma unroll
                    for (int m = 0; m < D; ++m) gg += G[j][m] * G[l][m];
                    double v = lam * G[j][i] * G[l][k] + mu * ((i == k ? gg : 0.0) + G[j][k] * G[l][i]);
                    out[((i * D + j) * D + k) * D + l] = det * v;
                }
}

// Stiffness block (a, b = a + offset) of every cell, gathered over the
// elements shared by the supports of N_a and N_b (no atomics).
template <int D>
__global__ __launch_bounds__(kBlock) void k_stiffness(const double *__restrict__ snap,
                                                      const double *__restrict__ wq,
                                                      const double *__restrict__ dN, int N, int n_el, int p,
                                                      int nc, int nq, int nloc, int n_off,
                                                      double *__restrict__ Kst) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int n_ctrl = 1;
    for (int j = 0; j < D; ++j) n_ctrl *= nc;
    long long total = (long long)N * n_ctrl * n_off;
    if (t >= total) return;
    int o = (int)(t % n_off);
    int a = (int)((t / n_off) % n_ctrl);
    int s = (int)(t / ((long long)n_off * n_ctrl));
    int ma[D], mb[D], lo[D], hi[D];
    int w = 2 * p + 1;
    bool valid = true;
    {
        int ta = a, to = o;
        for (int j = 0; j < D; ++j) {
            ma[j] = ta % nc;
            ta /= nc;
            mb[j] = ma[j] + (to % w) - p;
            to /= w;
            if (mb[j] < 0 || mb[j] >= nc) valid = false;
            lo[j] = max(max(ma[j], mb[j]) - p, 0);
            hi[j] = min(min(ma[j], mb[j]), n_el - 1);
            if (lo[j] > hi[j]) valid = false;
        }
    }
    double Kb[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) Kb[i][k] = 0.0;
    int nE = 1;
    for (int j = 0; j < D; ++j) nE *= n_el;
    if (valid) {
        int e[D];
        for (int j = 0; j < D; ++j) e[j] = lo[j];
        while (true) {
            int E = 0, la = 0, lb = 0;
            for (int j = D - 1; j >= 0; --j) {
                E = E * n_el + e[j];
                la = la * (p + 1) + (ma[j] - e[j]);
                lb = lb * (p + 1) + (mb[j] - e[j]);
            }
            for (int q = 0; q < nq; ++q) {
                const double *dNa = dN + ((size_t)(E * nq + q) * nloc + la) * D;
                const double *dNb = dN + ((size_t)(E * nq + q) * nloc + lb) * D;
                const double *C = snap + ((size_t)((long long)s * nE + E) * nq + q) * D * D * D * D;
                double wv = wq[E * nq + q];
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        double acc = 0.0;
#pragma unroll
                        for (int j = 0; j < D; ++j)
#pragma unroll
                            for (int l = 0; l < D; ++l) acc += dNa[j] * C[((i * D + j) * D + k) * D + l] * dNb[l];
                        Kb[i][k] += wv * acc;
                    }
            }
            int j = 0;
            for (; j < D; ++j) {
                if (++e[j] <= hi[j]) break;
                e[j] = lo[j];
            }
            if (j == D) break;
        }
    }
    // layout [s][o][i][k][a]: consecutive control points adjacent (coalesced cell mat-vecs)
    double *out = Kst + (size_t)s * n_off * D * D * n_ctrl;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) out[(((size_t)o * D + i) * D + k) * n_ctrl + a] = Kb[i][k];
}

// -------------------------------------------------------------- greedy sweeps
__device__ inline double block_sum(double v, double *sh) {
    int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off) sh[tid] += sh[tid + off];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__device__ inline double block_max(double v, double *sh) {
    int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off) sh[tid] = fmax(sh[tid], sh[tid + off]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// norms[s] = ||A_s||_2, then A_s /= norms[s]; absmax[s] = ||A_s||_inf afterwards.
__global__ __launch_bounds__(kBlock) void k_normalise_rows(double *__restrict__ A, long long n,
                                                           double *__restrict__ norms, double *__restrict__ absmax) {
    __shared__ double sh[kBlock];
    double *row = A + (size_t)blockIdx.x * n;
    double s2 = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) s2 += row[i] * row[i];
    double nrm = sqrt(block_sum(s2, sh));
    double inv = 1.0 / nrm;
    double mx = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        double v = row[i] * inv;
        row[i] = v;
        mx = fmax(mx, fabs(v));
    }
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) {
        norms[blockIdx.x] = nrm;
        absmax[blockIdx.x] = mx;
    }
}

// zeta = A_sigma / ||A_sigma||
__global__ __launch_bounds__(kBlock) void k_make_zeta(const double *__restrict__ A, long long n, int sigma,
                                                      double *__restrict__ z) {
    __shared__ double sh[kBlock];
    const double *row = A + (size_t)sigma * n;
    double s2 = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) s2 += row[i] * row[i];
    double inv = 1.0 / sqrt(block_sum(s2, sh));
    for (long long i = threadIdx.x; i < n; i += blockDim.x) z[i] = row[i] * inv;
}

// beta_s = Delta_s . zeta; Delta_s -= beta_s zeta; absmax_s = ||Delta_s||_inf
__global__ __launch_bounds__(kBlock) void k_gs_update(double *__restrict__ A, long long n,
                                                      const double *__restrict__ z, double *__restrict__ beta,
                                                      double *__restrict__ absmax) {
    __shared__ double sh[kBlock];
    double *row = A + (size_t)blockIdx.x * n;
    double dot = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) dot += row[i] * z[i];
    double b = block_sum(dot, sh);
    double mx = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        double v = row[i] - b * z[i];
        row[i] = v;
        mx = fmax(mx, fabs(v));
    }
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) {
        beta[blockIdx.x] = b;
        absmax[blockIdx.x] = mx;
    }
}

// Columns of (L L^T)^-1 for a banded lower factor band[i*(bw+1) + (i-k)] = L[i][k]: one wave per
// CPW = 64/S consecutive columns j, S lanes per column splitting the band dot product of each
// substitution step (fixed butterfly over the S lanes), the column's last bw entries in an LDS ring
// of W > bw slots.  Forward L y = e_j from row j0 of the wave's first column (entries above a
// column's own j stay zero), then backward L^T x = y over all rows.  Entries are stored as rows of
// X (X[i][j]; the inverse is symmetric), so the lanes of a step write contiguous entries.
template <int S>
__global__ __launch_bounds__(64) void k_band_inverse(const double *__restrict__ band, int n, int bw, int W,
                                                     double *__restrict__ X) {
    constexpr int CPW = 64 / S;
    extern __shared__ double ring_all[];
    const int lane = threadIdx.x, cl = lane / S, sl = lane % S;
    const int j0 = blockIdx.x * CPW, j = j0 + cl;
    const bool valid = j < n;
    double *ring = ring_all + (size_t)cl * W;
    const int ld = bw + 1;
    for (int e = sl; e < W; e += S) ring[e] = 0.0;
    __syncthreads();
    for (int i = j0; i < n; ++i) {  // forward
        const double *Li = band + (size_t)i * ld;
        const int klo = max(0, i - bw) + sl;
        int pos = klo % W;
        double t = 0.0;
#pragma unroll 8
        for (int k = klo; k < i; k += S) {  // unrolled: the band loads of several terms in flight
            t += Li[i - k] * ring[pos];
            pos += S;
            if (pos >= W) pos -= W;
        }
#pragma unroll
        for (int off = S / 2; off > 0; off >>= 1) t += __shfl_xor(t, off);
        const double v = ((valid && i == j ? 1.0 : 0.0) - t) / Li[0];
        __syncthreads();  // every lane has read the ring for this step
        if (sl == 0) {
            ring[i % W] = v;
            if (valid) X[(size_t)i * n + j] = v;
        }
        __syncthreads();
    }
    for (int e = sl; e < W; e += S) ring[e] = 0.0;
    __syncthreads();
    for (int i = n - 1; i >= 0; --i) {  // backward
        const int khi = min(n - 1, i + bw);
        int pos = (i + 1 + sl) % W;
        double t = 0.0;
#pragma unroll 8
        for (int k = i + 1 + sl; k <= khi; k += S) {
            t += band[(size_t)k * ld + (k - i)] * ring[pos];
            pos += S;
            if (pos >= W) pos -= W;
        }
#pragma unroll
        for (int off = S / 2; off > 0; off >>= 1) t += __shfl_xor(t, off);
        const double y = (valid && i >= j) ? X[(size_t)i * n + j] : 0.0;  // zero above j (not written forward)
        const double v = (y - t) / band[(size_t)i * ld];
        __syncthreads();
        if (sl == 0) {
            ring[i % W] = v;
            if (valid) X[(size_t)i * n + j] = v;
        }
        __syncthreads();
    }
}

// Trace tables of eq. (42) at quadrature point eq = blockIdx.x (the lookup-table form of eqs. (52)-(54)).
// With the gradients at the point of the principal fields, G_p[(k,ab)][a] = sum_l dN_l[j] U_rp^(k)[r(l,i)][a]
// and G_d[(k,ab)][c] = sum_l dN_l[j] K_rr^(k)-1[r(l,i)][n_i + c] (ab = i d + j, r(l,i) the r position of
// local dof (l,i)), and the primal unit fields ge[ab][a] = sum_l dN_l[j] [p(l,i) = a]:
//   Psi[t][eq][ab][cd]         = w_q G_p[(i,ab)] . G_p[(j,cd)]     (A pairs t = (i <= j))
//   Psi[npair + t][eq][ab][cd] = w_q G_d[(i,ab)] . G_d[(j,cd)]     (M pairs)
//   Psi[2 npair + i][eq][ab][cd] = w_q G_p[(i,ab)] . ge[cd]          (b)
// G_d is built in LDS in chunks of NC dual columns; each thread accumulates up to MAXE M entries per
// pass in registers (fixed column order: bitwise reproducible).
template <int D>
__global__ __launch_bounds__(256) void k_trace_tables(const double *__restrict__ Kinv, const double *__restrict__ UqT,
                                                      const double *__restrict__ dN, const double *__restrict__ wts,
                                                      const int *__restrict__ elem_ctrl,
                                                      const int *__restrict__ r_of_dof,
                                                      const int *__restrict__ p_of_dof,
                                                      const int *__restrict__ pair_i, const int *__restrict__ pair_j,
                                                      int K, int n_r, int n_p, int n_i, int n_d, int nq, int nloc,
                                                      long long nsnap, double *__restrict__ Psi) {
    constexpr int D2 = D * D, D4 = D2 * D2, NC = 16, NCS = NC + 1, MAXE = 48;
    extern __shared__ double sm[];
    const int eq = blockIdx.x, E = eq / nq, tid = threadIdx.x;
    const int KD2 = K * D2, npair = K * (K + 1) / 2, nld = nloc * D;
    double *Gp = sm;
    double *ge = Gp + (size_t)KD2 * n_p;
    double *Gd = ge + (size_t)D2 * n_p;
    double *dn = Gd + (size_t)KD2 * NCS;
    int *rpl = (int *)(dn + nld);
    int *ppl = rpl + nld;
    for (int e = tid; e < nld; e += 256) {
        const int l = e / D, i1 = e % D;
        const int dof = elem_ctrl[(size_t)E * nloc + l] * D + i1;
        rpl[e] = r_of_dof[dof];
        ppl[e] = p_of_dof[dof];
        dn[e] = dN[((size_t)eq * nloc + l) * D + i1];  // dn[l*D + j] = dN_l[j]
    }
    __syncthreads();
    for (int e = tid; e < KD2 * n_p; e += 256) {
        const int row = e / n_p, a = e % n_p, k = row / D2, ab = row % D2, i1 = ab / D, j1 = ab % D;
        double s = 0.0;
        for (int l = 0; l < nloc; ++l) {
            const int rp = rpl[l * D + i1];
            if (rp >= 0) s += dn[l * D + j1] * UqT[((size_t)k * n_p + a) * n_r + rp];
        }
        Gp[e] = s;
    }
    for (int e = tid; e < D2 * n_p; e += 256) {
        const int ab = e / n_p, a = e % n_p, i1 = ab / D, j1 = ab % D;
        double s = 0.0;
        for (int l = 0; l < nloc; ++l)
            if (ppl[l * D + i1] == a) s += dn[l * D + j1];
        ge[e] = s;
    }
    __syncthreads();
    const double w = wts[eq];
    const size_t base = (size_t)eq * D4;
    for (int e = tid; e < npair * D4; e += 256) {
        const int t = e / D4, rem = e % D4, ab = rem / D2, cd = rem % D2;
        const double *u = Gp + (size_t)(pair_i[t] * D2 + ab) * n_p, *v = Gp + (size_t)(pair_j[t] * D2 + cd) * n_p;
        double s = 0.0;
        for (int a = 0; a < n_p; ++a) s += u[a] * v[a];
        Psi[(size_t)t * nsnap + base + rem] = w * s;
    }
    for (int e = tid; e < K * D4; e += 256) {
        const int i = e / D4, rem = e % D4, ab = rem / D2, cd = rem % D2;
        const double *u = Gp + (size_t)(i * D2 + ab) * n_p, *v = ge + (size_t)cd * n_p;
        double s = 0.0;
        for (int a = 0; a < n_p; ++a) s += u[a] * v[a];
        Psi[(size_t)(2 * npair + i) * nsnap + base + rem] = w * s;
    }
    const int nM = npair * D4;
    for (int e0 = 0; e0 < nM; e0 += 256 * MAXE) {
        double acc[MAXE];
#pragma unroll
        for (int m = 0; m < MAXE; ++m) acc[m] = 0.0;
        for (int c0 = 0; c0 < n_d; c0 += NC) {
            __syncthreads();  // the previous chunk is consumed
            for (int e = tid; e < KD2 * NC; e += 256) {
                const int row = e / NC, cc = e % NC, col = c0 + cc;
                const int k = row / D2, ab = row % D2, i1 = ab / D, j1 = ab % D;
                double s = 0.0;
                if (col < n_d)
                    for (int l = 0; l < nloc; ++l) {
                        const int rp = rpl[l * D + i1];
                        if (rp >= 0) s += dn[l * D + j1] * Kinv[((size_t)k * n_r + rp) * n_r + n_i + col];
                    }
                Gd[(size_t)row * NCS + cc] = s;
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < MAXE; ++m) {
                const int e = e0 + tid + 256 * m;
                if (e < nM) {
                    const int t = e / D4, rem = e % D4, ab = rem / D2, cd = rem % D2;
                    const double *u = Gd + (size_t)(pair_i[t] * D2 + ab) * NCS;
                    const double *v = Gd + (size_t)(pair_j[t] * D2 + cd) * NCS;
                    double s = 0.0;
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc) s += u[cc] * v[cc];
                    acc[m] += s;
                }
            }
        }
#pragma unroll
        for (int m = 0; m < MAXE; ++m) {
            const int e = e0 + tid + 256 * m;
            if (e < nM) Psi[(size_t)(npair + e / D4) * nsnap + base + e % D4] = w * acc[m];
        }
    }
}

inline unsigned blocks_for(long long n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_pulled_back(ifeti_ctx *c) {
    const RefTables &R = c->ref;
    DevBuf<int> bad;
    bad.alloc(1);
    bad.zero(c->stream);
    long long total = (long long)c->N * R.n_elem * R.nq;
    const auto &d = c->desc;
    if (c->dim == 2)
        hipLaunchKernelGGL(k_pulled_back<2>, dim3(blocks_for(total)), dim3(kBlock), 0, c->stream, c->ctrl.p,
                           c->widths.p, c->g_tables_xi.p, c->g_tables_dN.p, c->g_tables_ctrl.p, c->N, R.n_elem,
                           R.nq, R.nloc, R.n_ctrl, d.E_in, d.E_out, d.nu, d.smooth_eps, d.h, c->snap.p, bad.p);
    else
        hipLaunchKernelGGL(k_pulled_back<3>, dim3(blocks_for(total)), dim3(kBlock), 0, c->stream, c->ctrl.p,
                           c->widths.p, c->g_tables_xi.p, c->g_tables_dN.p, c->g_tables_ctrl.p, c->N, R.n_elem,
                           R.nq, R.nloc, R.n_ctrl, d.E_in, d.E_out, d.nu, d.smooth_eps, d.h, c->snap.p, bad.p);
    IFETI_HIP(hipGetLastError());
    int hbad = 0;
    IFETI_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipStreamSynchronize(c->stream));
    IFETI_REQUIRE(hbad == 0, IFETI_EINVAL, "a cell map has a non-positive Jacobian determinant");
}

void launch_stiffness(ifeti_ctx *c) {
    const RefTables &R = c->ref;
    long long total = (long long)c->N * R.n_ctrl * R.n_off;
    if (c->dim == 2)
        hipLaunchKernelGGL(k_stiffness<2>, dim3(blocks_for(total)), dim3(kBlock), 0, c->stream, c->snap.p,
                           c->g_tables_w.p, c->g_tables_dN.p, c->N, R.n_el, R.p, R.nc, R.nq, R.nloc, R.n_off,
                           c->Kst.p);
    else
        hipLaunchKernelGGL(k_stiffness<3>, dim3(blocks_for(total)), dim3(kBlock), 0, c->stream, c->snap.p,
                           c->g_tables_w.p, c->g_tables_dN.p, c->N, R.n_el, R.p, R.nc, R.nq, R.nloc, R.n_off,
                           c->Kst.p);
    IFETI_HIP(hipGetLastError());
}

// Algorithm 4 on the snapshots held in c->snap (overwritten by the residuals).
int greedy_device(ifeti_ctx *c, int n_principal, double tol_rb, const int *principal_in, std::vector<int> &sigma,
                  std::vector<double> &beta, std::vector<double> &norms) {
    const int N = c->N;
    const long long n = c->ref.n_snap;
    DevBuf<double> d_norm, d_absmax, d_beta, d_z;
    d_norm.alloc(N);
    d_absmax.alloc(N);
    d_beta.alloc(N);
    d_z.alloc(n);
    hipLaunchKernelGGL(k_normalise_rows, dim3(N), dim3(kBlock), 0, c->stream, c->snap.p, n, d_norm.p, d_absmax.p);
    IFETI_HIP(hipGetLastError());
    norms.assign(N, 0.0);
    std::vector<double> absmax(N), b(N);
    IFETI_HIP(hipMemcpyAsync(norms.data(), d_norm.p, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    std::vector<std::vector<double>> betas;
    sigma.clear();
    for (int i = 0; i < n_principal; ++i) {
        IFETI_HIP(hipMemcpyAsync(absmax.data(), d_absmax.p, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        IFETI_HIP(hipStreamSynchronize(c->stream));
        int s;
        if (principal_in) {
            s = principal_in[i];
            IFETI_REQUIRE(s >= 0 && s < N, IFETI_EINVAL, "principal cell index out of range");
        } else {
            double mx = *std::max_element(absmax.begin(), absmax.end());
            if (!(mx > tol_rb)) break;
            s = -1;
            for (int t = 0; t < N; ++t)
                if (absmax[t] >= mx * (1.0 - 1e-12)) {
                    s = t;
                    break;
                }
        }
        hipLaunchKernelGGL(k_make_zeta, dim3(1), dim3(kBlock), 0, c->stream, c->snap.p, n, s, d_z.p);
        hipLaunchKernelGGL(k_gs_update, dim3(N), dim3(kBlock), 0, c->stream, c->snap.p, n, d_z.p, d_beta.p,
                           d_absmax.p);
        IFETI_HIP(hipGetLastError());
        IFETI_HIP(hipMemcpyAsync(b.data(), d_beta.p, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        IFETI_HIP(hipStreamSynchronize(c->stream));
        sigma.push_back(s);
        betas.push_back(b);
    }
    const int K = (int)sigma.size();
    IFETI_REQUIRE(K > 0, IFETI_EINVAL, "greedy selected no principal cell");
    beta.assign((size_t)N * K, 0.0);
    for (int k = 0; k < K; ++k)
        for (int s = 0; s < N; ++s) beta[(size_t)s * K + k] = betas[k][s];
    return K;
}

// lower-triangle tiles of the explicit coarse inverse (one workgroup per tile,
// tiles with J > I exit), zero-padded beyond nP
__global__ __launch_bounds__(kBlock) void k_sym_pack(const double *__restrict__ S, int n, double *__restrict__ T) {
    const int I = blockIdx.y, J = blockIdx.x;
    if (J > I) return;
    double *dst = T + ((size_t)I * (I + 1) / 2 + J) * 4096;
    for (int e = threadIdx.x; e < 4096; e += kBlock) {
        const int r = I * 64 + e / 64, cc = J * 64 + e % 64;
        dst[e] = (r < n && cc < n) ? S[(size_t)r * n + cc] : 0.0;
    }
}

void trace_tables_device(ifeti_ctx *c, int K, const double *Kinv, const double *UqT, double *Psi) {
    const RefTables &R = c->ref;
    const int npair = K * (K + 1) / 2, d2 = R.dim * R.dim, nld = R.nloc * R.dim;
    std::vector<int> pi((size_t)npair), pj((size_t)npair);
    for (int i = 0, t = 0; i < K; ++i)
        for (int j = i; j < K; ++j, ++t) {
            pi[t] = i;
            pj[t] = j;
        }
    DevBuf<int> dpi, dpj;
    dpi.upload(pi, c->stream);
    dpj.upload(pj, c->stream);
    const size_t lds = sizeof(double) * ((size_t)K * d2 * c->n_p + (size_t)d2 * c->n_p + (size_t)K * d2 * 17 + nld) +
                       sizeof(int) * 2 * (size_t)nld;
    IFETI_REQUIRE(lds <= 160 * 1024, IFETI_EINVAL, "too many principal cells for the trace tables");
    const int nqp = R.n_elem * R.nq;
    auto launch = [&](auto kern) {
        IFETI_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(nqp), dim3(256), lds, c->stream, Kinv, UqT, c->g_tables_dN.p, c->g_tables_w.p,
                           c->g_tables_ctrl.p, c->r_of_dof.p, c->p_of_dof.p, dpi.p, dpj.p, K, c->n_r, c->n_p,
                           c->n_i, c->n_d, R.nq, R.nloc, (long long)R.n_snap, Psi);
    };
    if (R.dim == 2)
        launch(k_trace_tables<2>);
    else
        launch(k_trace_tables<3>);
    IFETI_HIP(hipGetLastError());
    IFETI_HIP(hipStreamSynchronize(c->stream));  // the pair tables are released on return
}

// (L L^T)^-1 into X [n][n] from a banded lower factor on the device
static void launch_band_inverse(ifeti_ctx *c, const double *band, int n, int bw, double *X) {
    constexpr int S = 16, CPW = 64 / S;  // ~n/4 single-wave workgroups: several per compute unit
    const int W = std::max(bw + 1, S + 1) | 1;  // ring slots: more than the band and than S, odd
    const size_t lds = (size_t)CPW * W * sizeof(double);
    IFETI_REQUIRE(lds <= 160 * 1024, IFETI_EINVAL, "band too wide for the LDS of the band inverse");
    IFETI_HIP(hipFuncSetAttribute((const void *)k_band_inverse<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
    hipLaunchKernelGGL(k_band_inverse<S>, dim3((n + CPW - 1) / CPW), dim3(64), lds, c->stream, band, n, bw, W, X);
    IFETI_HIP(hipGetLastError());
}

std::vector<double> band_inverse_device(ifeti_ctx *c, const std::vector<double> &band_L, int n, int bw) {
    std::vector<double> out;
    if (n == 0) return out;
    DevBuf<double> band, X;
    band.upload(band_L, c->stream);
    X.alloc((size_t)n * n);
    launch_band_inverse(c, band.p, n, bw, X.p);
    X.download(out, c->stream);
    IFETI_HIP(hipStreamSynchronize(c->stream));
    return out;
}

void coarse_inverse_device(ifeti_ctx *c, CoarseSolver &co, const std::vector<double> &band_L, int bw) {
    DevBuf<double> band;
    band.upload(band_L, c->stream);
    co.SPPinv.alloc((size_t)c->nP * c->nP);
    // the inverse is rewritten in place: fragment copies made from an earlier one are stale
    c->drop_copies(co.SPPinv.p);
    launch_band_inverse(c, band.p, c->nP, bw, co.SPPinv.p);
    const int nT = (c->nP + 63) / 64;
    const size_t ntiles = (size_t)nT * (nT + 1) / 2;
    co.nT = nT;
    co.SPPt.alloc(ntiles * 4096);
    hipLaunchKernelGGL(k_sym_pack, dim3(nT, nT), dim3(kBlock), 0, c->stream, co.SPPinv.p, c->nP, co.SPPt.p);
    IFETI_HIP(hipGetLastError());
    std::vector<int> tl(2 * ntiles);
    for (int I = 0; I < nT; ++I)
        for (int J = 0; J <= I; ++J) {
            const size_t t = (size_t)I * (I + 1) / 2 + J;
            tl[2 * t] = I;
            tl[2 * t + 1] = J;
        }
    co.sym_tiles.upload(tl, c->stream);
    co.w_symP.alloc(ntiles * 3 * 128);  // up to 3 load cases per pass
    IFETI_HIP(hipStreamSynchronize(c->stream));
    co.inv_ready = true;
}

// The explicit inverse serves the symmetric-tile solve and the many-load-case contraction only; the
// partitioned solve needs the band alone, so the inverse is built the first time a path reads it.
void ensure_coarse_inverse(ifeti_ctx *c, CoarseSolver &co) {
    if (co.inv_ready) return;
    IFETI_REQUIRE(!c->capturing, IFETI_EINVAL, "coarse inverse must exist before graph capture");
    IFETI_REQUIRE(!c->no_alloc, IFETI_EINVAL, "allocation-free call: the explicit coarse inverse is not built");
    coarse_inverse_device(c, co, co.h_bandL, co.bw);
}

}  // namespace ifeti
