// Compliance and its strut-width gradient (differentiation form).
//
// c = f^T u for the solution u of (16); the loads do not depend on the widths
// and the system is self-adjoint, so dc/dw_s = -u_s^T (dK^(s)/dw_s) u_s.  The
// cell stiffness of eq. (52) is linear in the pulled-back tensor Ĉ, which is
// linear in the Young modulus, so dĈ/dw_s = (dE/dw_s / E) Ĉ and
//   dc/dw_s = -sum_q w_q (dE/dw_s / E)(x_q) grad(u_s)(x_q) : Ĉ_q : grad(u_s)(x_q),
// one workgroup per cell reading the cell's snapshot Ĉ (kept on the device).
#include <cmath>

#include "common.hpp"

namespace ifeti {
namespace {

constexpr int kB = 256;

__device__ inline double seg_dist(double x, double y, double ax, double ay, double bx, double by) {
    double ux = bx - ax, uy = by - ay;
    double t = ((x - ax) * ux + (y - ay) * uy) / (ux * ux + uy * uy);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    double dx = x - (ax + t * ux), dy = y - (ay + t * uy);
    return sqrt(dx * dx + dy * dy);
}

template <int D>
__device__ double strut_dist(const double *xi) {
    if constexpr (D == 2) {
        double x = xi[0], y = xi[1];
        double d = seg_dist(x, y, 0, 0, 1, 0);
        d = fmin(d, seg_dist(x, y, 1, 0, 1, 1));
        d = fmin(d, seg_dist(x, y, 1, 1, 0, 1));
        d = fmin(d, seg_dist(x, y, 0, 1, 0, 0));
        d = fmin(d, seg_dist(x, y, 0, 0, 1, 1));
        d = fmin(d, seg_dist(x, y, 1, 0, 0, 1));
        return d;
    } else {
        double best = 1e300;
        for (int axis = 0; axis < 3; ++axis) {
            int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
            for (int c1 = 0; c1 < 2; ++c1)
                for (int c2 = 0; c2 < 2; ++c2) best = fmin(best, fmax(fabs(xi[o1] - c1), fabs(xi[o2] - c2)));
        }
        return best;
    }
}

template <int D>
__global__ __launch_bounds__(kB) void k_compliance_grad(const double *__restrict__ u, long long nU,
                                                        const int *__restrict__ Ap, const int *__restrict__ idx_r,
                                                        const int *__restrict__ idx_p, const double *__restrict__ snap,
                                                        const double *__restrict__ widths,
                                                        const double *__restrict__ wq,
                                                        const double *__restrict__ xi,
                                                        const double *__restrict__ dN,
                                                        const int *__restrict__ elem_ctrl, int N, int n_r, int n_p,
                                                        int n_dof, int nE, int nq, int nloc, double E_in,
                                                        double E_out, double eps, double h,
                                                        double *__restrict__ grad) {
    extern __shared__ double sm[];
    double *uloc = sm;               // n_dof
    double *red = sm + n_dof;        // kB
    const int col = blockIdx.x, rhs = col / N, s = col % N, tid = threadIdx.x;
    const double *ur = u + (long long)rhs * nU;
    for (int i = tid; i < n_r; i += kB) uloc[idx_r[i]] = ur[(size_t)s * n_r + i];
    for (int j = tid; j < n_p; j += kB) {
        int P = Ap[(size_t)s * n_p + j];
        uloc[idx_p[j]] = P >= 0 ? ur[(size_t)N * n_r + P] : 0.0;
    }
    __syncthreads();
    const double half = 0.5 * widths[s];
    double acc = 0.0;
    if (eps > 0.0) {
        for (int eq = tid; eq < nE * nq; eq += kB) {
            const int E = eq / nq;
            const double dist = strut_dist<D>(xi + (size_t)eq * D) * h;
            const double t = tanh((half - dist) / eps);
            const double Ey = E_out + (E_in - E_out) * 0.5 * (1.0 + t);
            const double dE = (E_in - E_out) * 0.5 * (1.0 - t * t) * (0.5 / eps);
            double G[D][D];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) G[i][j] = 0.0;
            for (int l = 0; l < nloc; ++l) {
                const int a = elem_ctrl[E * nloc + l];
                const double *g = dN + ((size_t)eq * nloc + l) * D;
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < D; ++j) G[i][j] += uloc[a * D + i] * g[j];
            }
            const double *C = snap + ((size_t)s * nE * nq + eq) * D * D * D * D;
            double e = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j)
#pragma unroll
                    for (int k = 0; k < D; ++k)
#pragma unroll
                        for (int l = 0; l < D; ++l) e += G[i][j] * C[((i * D + j) * D + k) * D + l] * G[k][l];
            acc += wq[eq] * (dE / Ey) * e;
        }
    }
    red[tid] = acc;
    __syncthreads();
    for (int off = kB / 2; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) grad[col] = -red[0];
}

}  // namespace

void compliance_grad(ifeti_ctx *c, const double *f, const double *u, double *grad, double *comp_host, int nrhs) {
    IFETI_REQUIRE(c->snap_valid, IFETI_EINVAL, "snapshots not available");
    const RefTables &R = c->ref;
    const int N = c->N;
    const double colsd = (double)N * nrhs;
    const size_t shmem = (size_t)(R.n_dof + kB) * sizeof(double);
    {
        Prof prof(c, "compliance_grad", colsd * (double)R.n_elem * R.nq * (2.0 * R.nloc * c->dim * c->dim +
                                                                              3.0 * R.n_snap / ((double)R.n_elem * R.nq)),
                  colsd * 8.0 * ((double)R.n_snap + R.n_dof));
        if (c->dim == 2)
            hipLaunchKernelGGL(k_compliance_grad<2>, dim3(N * nrhs), dim3(kB), shmem, c->stream, u, c->nU, c->g_Ap.p,
                               c->g_idx_r.p, c->g_idx_p.p, c->snap.p, c->widths.p, c->g_tables_w.p, c->g_tables_xi.p,
                               c->g_tables_dN.p, c->g_tables_ctrl.p, N, c->n_r, c->n_p, R.n_dof, R.n_elem, R.nq,
                               R.nloc, c->desc.E_in, c->desc.E_out, c->desc.smooth_eps, c->desc.h, grad);
        else
            hipLaunchKernelGGL(k_compliance_grad<3>, dim3(N * nrhs), dim3(kB), shmem, c->stream, u, c->nU, c->g_Ap.p,
                               c->g_idx_r.p, c->g_idx_p.p, c->snap.p, c->widths.p, c->g_tables_w.p, c->g_tables_xi.p,
                               c->g_tables_dN.p, c->g_tables_ctrl.p, N, c->n_r, c->n_p, R.n_dof, R.n_elem, R.nq,
                               R.nloc, c->desc.E_in, c->desc.E_out, c->desc.smooth_eps, c->desc.h, grad);
        IFETI_HIP(hipGetLastError());
    }
    if (comp_host) {
        DevBuf<double> cd;
        cd.alloc(nrhs);
        multidot(c, f, 0, 1, u, c->nU, c->nU, nrhs, cd.p);
        IFETI_HIP(hipMemcpyAsync(comp_host, cd.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        IFETI_HIP(hipStreamSynchronize(c->stream));
    }
}

}  // namespace ifeti
