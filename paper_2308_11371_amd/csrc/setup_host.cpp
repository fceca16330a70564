// Host side of the offline phase: reference tables, decomposition bookkeeping,
// loads, principal bank, coefficient systems and the coarse matrix.
//
// Paper: Sec. 2.2 (eqs. (6), (12)-(18), (22), (27)-(30)), Sec. 3.1 (eqs. (38)-(43)),
// Sec. 3.2.1 (coarse problem), Sec. 4.2 (eqs. (52), (56), Algorithm 4).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include <chrono>
#include <cstdio>
#include <cstdlib>

#include "common.hpp"

namespace ifeti {

// ------------------------------------------------------------------ splines
namespace {

std::vector<double> knot_vector(int n_el, int p) {
    std::vector<double> U;
    for (int i = 0; i <= p; ++i) U.push_back(0.0);
    for (int i = 1; i < n_el; ++i) U.push_back(double(i) / n_el);
    for (int i = 0; i <= p; ++i) U.push_back(1.0);
    return U;
}

// Non-zero B-splines of degree p on knot span `span` at u (triangular
// recurrence of the Cox-de Boor relation); out[r] is function span-p+r.
void span_basis(const std::vector<double> &U, int span, double u, int p, double *out) {
    std::vector<double> left(p + 1), right(p + 1);
    out[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = u - U[span + 1 - j];
        right[j] = U[span + j] - u;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double tmp = out[r] / (right[r + 1] + left[j - r]);
            out[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        out[j] = saved;
    }
}

// Values and first derivatives of the p+1 non-zero functions on `span`.
void span_basis_ders(const std::vector<double> &U, int span, double u, int p, double *val, double *der) {
    span_basis(U, span, u, p, val);
    if (p == 0) {
        der[0] = 0.0;
        return;
    }
    std::vector<double> low(p);
    span_basis(U, span, u, p - 1, low.data());  // functions span-p+1 .. span of degree p-1
    for (int r = 0; r <= p; ++r) {
        int g = span - p + r;
        double a = 0.0, b = 0.0;
        if (r >= 1) {
            double den = U[g + p] - U[g];
            if (den > 0) a = low[r - 1] / den;
        }
        if (r <= p - 1) {
            double den = U[g + p + 1] - U[g + 1];
            if (den > 0) b = low[r] / den;
        }
        der[r] = p * (a - b);
    }
}

// n-point Gauss-Legendre rule on [0,1] by Newton iteration on P_n.
void gauss_rule(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // final derivative for the weight
                double q0 = 1.0, q1 = 0.0;
                for (int k = 1; k <= n; ++k) {
                    double q2 = q1;
                    q1 = q0;
                    q0 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q2) / k;
                }
                dp = n * (z * q0 - q1) / (z * z - 1.0);
                break;
            }
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) scaled by 1/2
    }
    // ascending order
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
    std::vector<double> xs(n), ws(n);
    for (int i = 0; i < n; ++i) {
        xs[i] = x[idx[i]];
        ws[i] = w[idx[i]];
    }
    x = xs;
    w = ws;
}

inline void multi_index(int a, int n, int dim, int *out) {
    for (int j = 0; j < dim; ++j) {
        out[j] = a % n;
        a /= n;
    }
}

}  // namespace

void build_reference_tables(ifeti_ctx *c) {
    RefTables &R = c->ref;
    const int dim = c->dim, p = c->desc.degree, n_el = c->desc.n_el;
    R.dim = dim;
    R.n_el = n_el;
    R.p = p;
    R.nc = n_el + p;
    R.n_ctrl = 1;
    for (int j = 0; j < dim; ++j) R.n_ctrl *= R.nc;
    R.n_dof = R.n_ctrl * dim;
    R.nq1 = p + 1;
    R.nq = 1;
    R.n_elem = 1;
    R.nloc = 1;
    R.n_off = 1;
    for (int j = 0; j < dim; ++j) {
        R.nq *= R.nq1;
        R.n_elem *= n_el;
        R.nloc *= p + 1;
        R.n_off *= 2 * p + 1;
    }
    int d4 = dim * dim * dim * dim;
    R.n_snap = R.n_elem * R.nq * d4;
    std::vector<double> U = knot_vector(n_el, p);
    std::vector<double> gx, gw;
    gauss_rule(R.nq1, gx, gw);
    // 1D tables per element e and point g: values/derivatives of local functions
    std::vector<double> v1(n_el * R.nq1 * (p + 1)), d1(n_el * R.nq1 * (p + 1)), x1(n_el * R.nq1),
        w1(n_el * R.nq1);
    for (int e = 0; e < n_el; ++e)
        for (int g = 0; g < R.nq1; ++g) {
            double u = (e + gx[g]) / n_el;
            x1[e * R.nq1 + g] = u;
            w1[e * R.nq1 + g] = gw[g] / n_el;
            span_basis_ders(U, e + p, u, p, &v1[(e * R.nq1 + g) * (p + 1)], &d1[(e * R.nq1 + g) * (p + 1)]);
        }
    R.tab1.assign(v1.begin(), v1.end());
    R.tab1.insert(R.tab1.end(), d1.begin(), d1.end());
    R.tab1.insert(R.tab1.end(), w1.begin(), w1.end());
    R.w.assign(R.n_elem * R.nq, 0.0);
    R.xi.assign(R.n_elem * R.nq * dim, 0.0);
    R.dN.assign((size_t)R.n_elem * R.nq * R.nloc * dim, 0.0);
    R.elem_ctrl.assign(R.n_elem * R.nloc, 0);
    int e_idx[3], g_idx[3], l_idx[3];
    for (int E = 0; E < R.n_elem; ++E) {
        multi_index(E, n_el, dim, e_idx);
        for (int l = 0; l < R.nloc; ++l) {
            multi_index(l, p + 1, dim, l_idx);
            int a = 0;
            for (int j = dim - 1; j >= 0; --j) a = a * R.nc + (e_idx[j] + l_idx[j]);
            R.elem_ctrl[E * R.nloc + l] = a;
        }
        for (int q = 0; q < R.nq; ++q) {
            multi_index(q, R.nq1, dim, g_idx);
            double wq = 1.0;
            for (int j = 0; j < dim; ++j) {
                wq *= w1[e_idx[j] * R.nq1 + g_idx[j]];
                R.xi[(E * R.nq + q) * dim + j] = x1[e_idx[j] * R.nq1 + g_idx[j]];
            }
            R.w[E * R.nq + q] = wq;
            for (int l = 0; l < R.nloc; ++l) {
                multi_index(l, p + 1, dim, l_idx);
                for (int jd = 0; jd < dim; ++jd) {
                    double prod = 1.0;
                    for (int j = 0; j < dim; ++j) {
                        size_t o = (e_idx[j] * R.nq1 + g_idx[j]) * (p + 1) + l_idx[j];
                        prod *= (j == jd) ? d1[o] : v1[o];
                    }
                    R.dN[((size_t)(E * R.nq + q) * R.nloc + l) * dim + jd] = prod;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ partition (12)
void build_partition(ifeti_ctx *c) {
    const RefTables &R = c->ref;
    const int dim = c->dim, nc = R.nc;
    c->idx_i.clear();
    c->idx_d.clear();
    c->idx_p.clear();
    int mi[3];
    for (int a = 0; a < R.n_ctrl; ++a) {
        multi_index(a, nc, dim, mi);
        int nb = 0;
        for (int j = 0; j < dim; ++j) nb += (mi[j] == 0 || mi[j] == nc - 1);
        std::vector<int> *dst = (nb == dim) ? &c->idx_p : (nb > 0 ? &c->idx_d : &c->idx_i);
        for (int k = 0; k < dim; ++k) dst->push_back(a * dim + k);
    }
    c->n_i = (int)c->idx_i.size();
    c->n_d = (int)c->idx_d.size();
    c->n_p = (int)c->idx_p.size();
    c->n_r = c->n_i + c->n_d;
    c->idx_r = c->idx_i;
    c->idx_r.insert(c->idx_r.end(), c->idx_d.begin(), c->idx_d.end());
    std::vector<int> rpos(R.n_dof, -1), ppos(R.n_dof, -1);
    for (int i = 0; i < c->n_r; ++i) rpos[c->idx_r[i]] = i;
    for (int i = 0; i < c->n_p; ++i) ppos[c->idx_p[i]] = i;
    c->r_of_dof.upload(rpos, c->stream);
    c->p_of_dof.upload(ppos, c->stream);
    // non-zeros of the shared stencil (full cell matrix and its r-r block)
    const int w = 2 * R.p + 1;
    c->nnz_rr = c->nnz_full = 0;
    int mb[3];
    for (int a = 0; a < R.n_ctrl; ++a) {
        multi_index(a, nc, dim, mi);
        for (int o = 0; o < R.n_off; ++o) {
            int t = o, b = 0;
            bool ok = true;
            for (int j = 0; j < dim; ++j) {
                mb[j] = mi[j] + (t % w) - R.p;
                t /= w;
                if (mb[j] < 0 || mb[j] >= nc) ok = false;
            }
            if (!ok) continue;
            for (int j = dim - 1; j >= 0; --j) b = b * nc + mb[j];
            for (int i = 0; i < dim; ++i)
                for (int k = 0; k < dim; ++k) {
                    c->nnz_full += 1;
                    if (rpos[a * dim + i] >= 0 && rpos[b * dim + k] >= 0) c->nnz_rr += 1;
                }
        }
    }
}

// ------------------------------------------------------------------ B, D, A_p (14)-(18), (30)
void build_decomposition(ifeti_ctx *c) {
    const RefTables &R = c->ref;
    const int dim = c->dim, nc = R.nc, N = c->N;
    int G[3] = {1, 1, 1}, V[3] = {1, 1, 1};
    for (int j = 0; j < dim; ++j) {
        G[j] = c->shape[j] * (nc - 1) + 1;
        V[j] = c->shape[j] + 1;
    }
    auto cell_coord = [&](int s, int *cc) {
        cc[0] = s % c->shape[0];
        cc[1] = (s / c->shape[0]) % c->shape[1];
        cc[2] = s / (c->shape[0] * c->shape[1]);
    };
    auto on_dirichlet = [&](const int *gp, const int *ext) {
        for (int f = 0; f < 2 * dim; ++f)
            if (c->desc.dirichlet_mask & (1 << f)) {
                int axis = f / 2, side = f % 2;
                if (gp[axis] == (side ? ext[axis] - 1 : 0)) return true;
            }
        return false;
    };
    // dual control points of the reference cell
    std::vector<int> dual_ctrl;
    for (size_t t = 0; t < c->idx_d.size(); t += dim) dual_ctrl.push_back(c->idx_d[t] / dim);
    const int ndc = (int)dual_ctrl.size();
    struct Entry {
        long long g;
        int s, t;
        bool dir;
    };
    std::vector<Entry> ent;
    ent.reserve((size_t)N * ndc);
    int cc[3], mi[3], gp[3];
    for (int s = 0; s < N; ++s) {
        cell_coord(s, cc);
        for (int t = 0; t < ndc; ++t) {
            multi_index(dual_ctrl[t], nc, dim, mi);
            long long g = 0;
            for (int j = dim - 1; j >= 0; --j) {
                gp[j] = cc[j] * (nc - 1) + mi[j];
                g = g * G[j] + gp[j];
            }
            ent.push_back({g, s, t, on_dirichlet(gp, G)});
        }
    }
    std::sort(ent.begin(), ent.end(), [](const Entry &a, const Entry &b) {
        return a.g != b.g ? a.g < b.g : a.s < b.s;
    });
    // rows: interface (chained pairs), then Dirichlet (every copy); both by (g, comp, position)
    std::vector<int> row_e1, row_e2, row_comp;  // entry indices (e2 = -1 for Dirichlet rows)
    std::vector<int> dir_e, dir_comp;
    size_t i0 = 0;
    while (i0 < ent.size()) {
        size_t i1 = i0;
        while (i1 < ent.size() && ent[i1].g == ent[i0].g) ++i1;
        if (ent[i0].dir) {
            for (int k = 0; k < dim; ++k)
                for (size_t e = i0; e < i1; ++e) {
                    dir_e.push_back((int)e);
                    dir_comp.push_back(k);
                }
        } else {
            for (int k = 0; k < dim; ++k)
                for (size_t e = i0; e + 1 < i1; ++e) {
                    row_e1.push_back((int)e);
                    row_e2.push_back((int)e + 1);
                    row_comp.push_back(k);
                }
        }
        i0 = i1;
    }
    c->L_int = (int)row_e1.size();
    c->L = c->L_int + (int)dir_e.size();
    const int L = c->L, n_d = c->n_d;
    std::vector<int> gat((size_t)N * n_d * 2, 0), sca((size_t)L * 2, 0);
    std::vector<double> Dw(L, 1.0);
    auto add_gather = [&](int s, int j, int row, int sign) {
        size_t base = ((size_t)s * n_d + j) * 2;
        if (gat[base] == 0)
            gat[base] = sign * (row + 1);
        else if (gat[base + 1] == 0)
            gat[base + 1] = sign * (row + 1);
        else
            throw Error{IFETI_EINVAL, "more than two multipliers on one dual dof"};
    };
    for (int r = 0; r < c->L_int; ++r) {
        const Entry &a = ent[row_e1[r]], &b = ent[row_e2[r]];
        int k = row_comp[r];
        int ja = a.t * dim + k, jb = b.t * dim + k;
        add_gather(a.s, ja, r, +1);
        add_gather(b.s, jb, r, -1);
        sca[2 * r] = +(a.s * n_d + ja + 1);
        sca[2 * r + 1] = -(b.s * n_d + jb + 1);
        Dw[r] = 0.5;
    }
    for (size_t q = 0; q < dir_e.size(); ++q) {
        int r = c->L_int + (int)q;
        const Entry &a = ent[dir_e[q]];
        int j = a.t * dim + dir_comp[q];
        add_gather(a.s, j, r, +1);
        sca[2 * r] = a.s * n_d + j + 1;
        Dw[r] = 1.0;
    }
    c->g_gather.upload(gat, c->stream);
    c->g_scatter.upload(sca, c->stream);
    c->h_sca = sca;
    c->g_Dw.upload(Dw, c->stream);
    c->h_d.assign(L, 0.0);

    // primal assembly A_p (18): free lattice vertices in lexicographic order
    long long nV = (long long)V[0] * V[1] * V[2];
    std::vector<int> vnum(nV, -1);
    int nfree = 0;
    for (long long v = 0; v < nV; ++v) {
        int vp[3] = {(int)(v % V[0]), (int)((v / V[0]) % V[1]), (int)(v / ((long long)V[0] * V[1]))};
        if (!on_dirichlet(vp, V)) vnum[v] = nfree++;
    }
    c->n_vert_free = nfree;
    c->nP = nfree * dim;
    c->nU = (long long)N * c->n_r + c->nP;
    const int n_p = c->n_p, ncorner = n_p / dim;
    c->h_Ap.assign((size_t)N * n_p, -1);
    std::vector<int> corner_ctrl;
    for (int t = 0; t < n_p; t += dim) corner_ctrl.push_back(c->idx_p[t] / dim);
    for (int s = 0; s < N; ++s) {
        cell_coord(s, cc);
        for (int q = 0; q < ncorner; ++q) {
            multi_index(corner_ctrl[q], nc, dim, mi);
            long long v = 0;
            for (int j = dim - 1; j >= 0; --j) v = v * V[j] + (cc[j] + mi[j] / (nc - 1));
            int num = vnum[v];
            for (int k = 0; k < dim; ++k) c->h_Ap[(size_t)s * n_p + q * dim + k] = num < 0 ? -1 : num * dim + k;
        }
    }
    c->g_Ap.upload(c->h_Ap, c->stream);
    {
        std::vector<int> codes(2 * c->h_Ap.size(), 0);
        for (size_t i = 0; i < c->h_Ap.size(); ++i) codes[2 * i] = c->h_Ap[i] < 0 ? 0 : c->h_Ap[i] + 1;
        c->g_Apc.upload(codes, c->stream);
    }
    c->maxc = 1 << dim;
    std::vector<int> pull((size_t)c->nP * c->maxc, -1), cnt(c->nP, 0);
    for (int s = 0; s < N; ++s)
        for (int j = 0; j < n_p; ++j) {
            int P = c->h_Ap[(size_t)s * n_p + j];
            if (P < 0) continue;
            IFETI_REQUIRE(cnt[P] < c->maxc, IFETI_EINVAL, "primal dof shared by too many cells");
            pull[(size_t)P * c->maxc + cnt[P]++] = s * n_p + j;
        }
    c->g_Ppull.upload(pull, c->stream);
}

bool has_dirichlet_data(const ifeti_ctx *c) {
    for (int i = 0; i < c->dim * c->dim; ++i)
        if (c->desc.u0_grad[i] != 0.0) return true;
    return false;
}

// Dirichlet data u0(x) = G x (3c) at the control points of the Dirichlet faces: d of (14) on the
// Dirichlet rows, and the values of the eliminated primal corners, lifted into the cell loads
// (f_s -= K^(s) u0 on those columns) so that (16) holds for the remaining unknowns.
static void apply_dirichlet_data(ifeti_ctx *c, std::vector<double> &fc) {
    const RefTables &R = c->ref;
    const int dim = c->dim, N = c->N, n_dof = R.n_dof, n_p = c->n_p, n_d = c->n_d;
    c->h_d.assign(c->L, 0.0);
    c->g_up_dir.release();
    if (!has_dirichlet_data(c)) return;
    const double *G = c->desc.u0_grad;
    std::vector<double> P((size_t)N * R.n_ctrl * dim);
    IFETI_HIP(hipMemcpyAsync(P.data(), c->ctrl.p, P.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipStreamSynchronize(c->stream));
    auto u0 = [&](int s, int a, int comp) {
        double v = 0.0;
        for (int m = 0; m < dim; ++m) v += G[comp * dim + m] * P[((size_t)s * R.n_ctrl + a) * dim + m];
        return v;
    };
    for (int r = c->L_int; r < c->L; ++r) {  // Dirichlet rows: one +1 entry at a cell's dual dof
        const int e = c->h_sca[2 * (size_t)r] - 1, s = e / n_d, j = e % n_d, dof = c->idx_d[j];
        c->h_d[r] = u0(s, dof / dim, dof % dim);
    }
    std::vector<double> up((size_t)N * n_p, 0.0), uD((size_t)N * n_dof, 0.0);
    bool any = false;
    for (int s = 0; s < N; ++s)
        for (int j = 0; j < n_p; ++j) {
            if (c->h_Ap[(size_t)s * n_p + j] >= 0) continue;  // a free lattice vertex
            const int dof = c->idx_p[j];
            const double v = u0(s, dof / dim, dof % dim);
            up[(size_t)s * n_p + j] = v;
            uD[(size_t)s * n_dof + dof] = v;
            any = any || v != 0.0;
        }
    c->g_up_dir.upload(up, c->stream);
    if (!any) return;
    DevBuf<double> dx, dy;
    dx.upload(uD, c->stream);
    dy.alloc(uD.size());
    cell_matvec_full(c, dx.p, dy.p);
    std::vector<double> KuD(uD.size());
    IFETI_HIP(hipMemcpyAsync(KuD.data(), dy.p, KuD.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    IFETI_HIP(hipStreamSynchronize(c->stream));
    for (int r = 0; r < c->nrhs; ++r)
        for (size_t t = 0; t < KuD.size(); ++t) fc[(size_t)r * N * n_dof + t] -= KuD[t];
}

// ------------------------------------------------------------------ loads (5b)
void build_loads(ifeti_ctx *c) {
    const RefTables &R = c->ref;
    const int dim = c->dim, nc = R.nc, N = c->N, p = R.p, nrhs = c->nrhs;
    const int n_dof = R.n_dof;
    std::vector<double> fc((size_t)nrhs * N * n_dof, 0.0);
    int face = c->desc.load_face;
    if (face >= 0) {
        std::vector<double> P((size_t)N * R.n_ctrl * dim);
        IFETI_HIP(hipMemcpyAsync(P.data(), c->ctrl.p, P.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        IFETI_HIP(hipStreamSynchronize(c->stream));
        const int axis = face / 2, side = face % 2;
        int tang[2], nt = 0;
        for (int j = 0; j < dim; ++j)
            if (j != axis) tang[nt++] = j;
        std::vector<double> U = knot_vector(R.n_el, p), gx, gw;
        gauss_rule(R.nq1, gx, gw);
        const int nf1 = R.n_el * R.nq1;  // 1D face points
        std::vector<double> fv(nf1 * (p + 1)), fd(nf1 * (p + 1)), fw(nf1);
        std::vector<int> ffirst(nf1);
        for (int e = 0; e < R.n_el; ++e)
            for (int g = 0; g < R.nq1; ++g) {
                int i = e * R.nq1 + g;
                span_basis_ders(U, e + p, (e + gx[g]) / R.n_el, p, &fv[i * (p + 1)], &fd[i * (p + 1)]);
                fw[i] = gw[g] / R.n_el;
                ffirst[i] = e;
            }
        const int a_norm = side ? nc - 1 : 0;  // the only function non-zero on the face
        int npts = (dim == 2) ? nf1 : nf1 * nf1;
        int nlf = (dim == 2) ? (p + 1) : (p + 1) * (p + 1);
        int cc[3];
        for (int s = 0; s < N; ++s) {
            cc[0] = s % c->shape[0];
            cc[1] = (s / c->shape[0]) % c->shape[1];
            cc[2] = s / (c->shape[0] * c->shape[1]);
            if (cc[axis] != (side ? c->shape[axis] - 1 : 0)) continue;
            const double *Ps = &P[(size_t)s * R.n_ctrl * dim];
            for (int ip = 0; ip < npts; ++ip) {
                int i0 = ip % nf1, i1 = (dim == 3) ? ip / nf1 : 0;
                double T[2][3] = {{0, 0, 0}, {0, 0, 0}};
                std::vector<int> ctrl_ids(nlf);
                std::vector<double> Nv(nlf);
                for (int l = 0; l < nlf; ++l) {
                    int l0 = l % (p + 1), l1 = l / (p + 1);
                    int t0 = ffirst[i0] + l0, t1 = (dim == 3) ? ffirst[i1] + l1 : 0;
                    int mi[3];
                    mi[axis] = a_norm;
                    mi[tang[0]] = t0;
                    if (dim == 3) mi[tang[1]] = t1;
                    int a = 0;
                    for (int j = dim - 1; j >= 0; --j) a = a * nc + mi[j];
                    ctrl_ids[l] = a;
                    double v0 = fv[i0 * (p + 1) + l0], d0 = fd[i0 * (p + 1) + l0];
                    double v1 = (dim == 3) ? fv[i1 * (p + 1) + l1] : 1.0;
                    double d1 = (dim == 3) ? fd[i1 * (p + 1) + l1] : 0.0;
                    Nv[l] = v0 * v1;
                    for (int m = 0; m < dim; ++m) {
                        T[0][m] += Ps[a * dim + m] * d0 * v1;
                        if (dim == 3) T[1][m] += Ps[a * dim + m] * v0 * d1;
                    }
                }
                double meas;
                if (dim == 2) {
                    meas = std::hypot(T[0][0], T[0][1]);
                } else {
                    double cx = T[0][1] * T[1][2] - T[0][2] * T[1][1];
                    double cy = T[0][2] * T[1][0] - T[0][0] * T[1][2];
                    double cz = T[0][0] * T[1][1] - T[0][1] * T[1][0];
                    meas = std::sqrt(cx * cx + cy * cy + cz * cz);
                }
                double wq = fw[i0] * ((dim == 3) ? fw[i1] : 1.0) * meas;
                for (int l = 0; l < nlf; ++l)
                    for (int r = 0; r < nrhs; ++r)
                        for (int m = 0; m < dim; ++m)
                            fc[((size_t)r * N + s) * n_dof + ctrl_ids[l] * dim + m] +=
                                wq * Nv[l] * c->tractions[r * dim + m];
            }
        }
    }
    apply_dirichlet_data(c, fc);
    c->f_cells.upload(fc, c->stream);
    // f of (16): f_R per cell, f_P assembled (18)
    std::vector<double> fv((size_t)nrhs * c->nU, 0.0);
    for (int r = 0; r < nrhs; ++r)
        for (int s = 0; s < N; ++s) {
            const double *fs = &fc[((size_t)r * N + s) * n_dof];
            double *fR = &fv[(size_t)r * c->nU + (size_t)s * c->n_r];
            for (int i = 0; i < c->n_r; ++i) fR[i] = fs[c->idx_r[i]];
            for (int j = 0; j < c->n_p; ++j) {
                int P = c->h_Ap[(size_t)s * c->n_p + j];
                if (P >= 0) fv[(size_t)r * c->nU + (size_t)N * c->n_r + P] += fs[c->idx_p[j]];
            }
        }
    c->f_vec.upload(fv, c->stream);
    std::vector<double> dv((size_t)nrhs * c->L, 0.0);
    for (int r = 0; r < nrhs; ++r) std::copy(c->h_d.begin(), c->h_d.end(), dv.begin() + (size_t)r * c->L);
    c->d_vec.upload(dv, c->stream);
}

// ------------------------------------------------------------------ dense helpers
namespace {

// In-place lower Cholesky of a row-major n x n SPD matrix; false on a pivot <= 0.
bool cholesky(std::vector<double> &A, int n) {
    for (int j = 0; j < n; ++j) {
        double *Aj = &A[(size_t)j * n];
        double s = Aj[j];
        for (int k = 0; k < j; ++k) s -= Aj[k] * Aj[k];
        if (!(s > 0.0)) return false;
        double ljj = std::sqrt(s);
        Aj[j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double *Ai = &A[(size_t)i * n];
            double t = Ai[j];
            for (int k = 0; k < j; ++k) t -= Ai[k] * Aj[k];
            Ai[j] = t / ljj;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = 0.0;
    return true;
}

// X (n x m, row-major) <- (L L^T)^-1 X.
void chol_solve(const std::vector<double> &Lf, int n, std::vector<double> &X, int m) {
    for (int i = 0; i < n; ++i) {
        double *Xi = &X[(size_t)i * m];
        const double *Li = &Lf[(size_t)i * n];
        for (int k = 0; k < i; ++k) {
            double l = Li[k];
            if (l == 0.0) continue;
            const double *Xk = &X[(size_t)k * m];
            for (int c = 0; c < m; ++c) Xi[c] -= l * Xk[c];
        }
        double inv = 1.0 / Li[i];
        for (int c = 0; c < m; ++c) Xi[c] *= inv;
    }
    for (int i = n - 1; i >= 0; --i) {
        double *Xi = &X[(size_t)i * m];
        for (int k = i + 1; k < n; ++k) {
            double l = Lf[(size_t)k * n + i];
            if (l == 0.0) continue;
            const double *Xk = &X[(size_t)k * m];
            for (int c = 0; c < m; ++c) Xi[c] -= l * Xk[c];
        }
        double inv = 1.0 / Lf[(size_t)i * n + i];
        for (int c = 0; c < m; ++c) Xi[c] *= inv;
    }
}

// Cyclic Jacobi eigen-decomposition of a small symmetric matrix (row-major).
void jacobi_eig(std::vector<double> A, int n, std::vector<double> &w, std::vector<double> &V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = cs * akp - sn * akq;
                    A[k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = cs * apk - sn * aqk;
                    A[q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = cs * vkp - sn * vkq;
                    V[k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// x = A^-1 b for a small SPD A: Cholesky, or a symmetric pseudo-inverse cutting
// eigenvalues below 1e-13 of the largest when the factorisation fails.
std::vector<double> small_spd_solve(const std::vector<double> &A, int n, const std::vector<double> &b) {
    std::vector<double> Lf = A;
    bool ok = cholesky(Lf, n);
    if (ok)
        for (int i = 0; i < n * n; ++i) ok = ok && std::isfinite(Lf[i]);
    if (ok) {
        std::vector<double> x = b;
        chol_solve(Lf, n, x, 1);
        return x;
    }
    std::vector<double> S(n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) S[i * n + j] = 0.5 * (A[i * n + j] + A[j * n + i]);
    std::vector<double> w, V;
    jacobi_eig(S, n, w, V);
    double wmax = 0.0;
    for (double v : w) wmax = std::max(wmax, v);
    std::vector<double> x(n, 0.0);
    for (int k = 0; k < n; ++k) {
        if (!(w[k] > 1e-13 * wmax)) continue;
        double proj = 0.0;
        for (int i = 0; i < n; ++i) proj += V[i * n + k] * b[i];
        proj /= w[k];
        for (int i = 0; i < n; ++i) x[i] += proj * V[i * n + k];
    }
    return x;
}

// Principal-cell operators on the host (eqs. (22), (27)-(30), (39)), from the batched GPU
// factorisation of the principal cells.
struct Principal {
    std::vector<double> Krp, Kpp;             // dense blocks, n_r x n_p and n_p x n_p (row-major)
    std::vector<double> Kinv, Urp, Fdd, Sdd;  // n_r x n_r, n_r x n_p, n_d x n_d, n_d x n_d
};

template <class F>
void parallel_for(int n, F f) {
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

}  // namespace

// ------------------------------------------------------------------ offline phase
// IFETI_SETUP_VERBOSE=1 prints the wall time of each offline stage (the stream is synchronised at
// each mark, so the times include the device work of the stage)
struct StageClock {
    ifeti_ctx *c;
    bool on;
    std::chrono::steady_clock::time_point t;
    explicit StageClock(ifeti_ctx *cc) : c(cc), on(std::getenv("IFETI_SETUP_VERBOSE") != nullptr) {
        t = std::chrono::steady_clock::now();
    }
    void mark(const char *what) {
        if (!on) return;
        IFETI_HIP(hipStreamSynchronize(c->stream));
        const auto n = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[ifeti setup] %-28s %8.1f ms\n", what,
                     std::chrono::duration<double, std::milli>(n - t).count());
        t = n;
    }
};

void build_reduced_basis(ifeti_ctx *c, int n_principal, double tol_rb, const int *principal_in) {
    StageClock clk(c);
    const RefTables &R = c->ref;
    const int N = c->N, nr = c->n_r, np = c->n_p, nd = c->n_d, ni = c->n_i;
    // 1. greedy (Algorithm 4) on the device; affine coordinates (56) on the host
    std::vector<int> sigma;
    std::vector<double> beta, norms;
    int K = greedy_device(c, n_principal, tol_rb, principal_in, sigma, beta, norms);
    std::vector<double> alpha((size_t)N * K, 0.0);
    {
        std::vector<double> U((size_t)K * K, 0.0);  // U[i][j] = ||A^(sigma_j)|| beta_i^(sigma_j), i <= j
        for (int j = 0; j < K; ++j)
            for (int i = 0; i <= j; ++i) U[i * K + j] = norms[sigma[j]] * beta[(size_t)sigma[j] * K + i];
        for (int s = 0; s < N; ++s) {
            double *a = &alpha[(size_t)s * K];
            for (int i = K - 1; i >= 0; --i) {
                double t = norms[s] * beta[(size_t)s * K + i];
                for (int j = i + 1; j < K; ++j) t -= U[i * K + j] * a[j];
                a[i] = t / U[i * K + i];
            }
        }
    }
    clk.mark("greedy + affine coordinates");
    // 2. principal bank (eqs. (22), (27)-(30), (39)): the principal cells' augmented matrices
    //    [K_rr K_rp I; K_pr K_pp 0; I 0 0] factorised on the GPU (the batched elimination of the
    //    standard FETI-DP form with every r row selected), giving K_rr^-1, U_rp, S_pp, S_dd, K_pr, K_pp
    std::vector<Principal> bank(K);
    DevBuf<double> dFq, dUqT;  // K_rr^-1 and U_rp^T of the principals, also used by the trace tables
    {
        DevBuf<int> dsig;
        dsig.upload(sigma, c->stream);
        DevBuf<double> dSdd, dSpp, dKpr, dKpp;
        dFq.alloc((size_t)K * nr * nr);
        dSdd.alloc((size_t)K * nd * nd);
        dUqT.alloc((size_t)K * np * nr);
        dSpp.alloc((size_t)K * np * np);
        dKpr.alloc((size_t)K * np * nr);
        dKpp.alloc((size_t)K * np * np);
        FactorOut o;
        o.Fq = dFq.p;
        o.Sdd = dSdd.p;
        o.UqT = dUqT.p;
        o.Spp = dSpp.p;
        o.Kpr = dKpr.p;
        o.Kpp = dKpp.p;
        factor_cells(c, dsig.p, K, 0, nr, o);
        std::vector<double> hFq(dFq.n), hSdd(dSdd.n), hUqT(dUqT.n), hKpr(dKpr.n), hKpp(dKpp.n);
        dFq.download(hFq, c->stream);
        dSdd.download(hSdd, c->stream);
        dUqT.download(hUqT, c->stream);
        dKpr.download(hKpr, c->stream);
        dKpp.download(hKpp, c->stream);
        IFETI_HIP(hipStreamSynchronize(c->stream));
        parallel_for(K, [&](int k) {
            Principal &P = bank[k];
            P.Kinv.assign(&hFq[(size_t)k * nr * nr], &hFq[(size_t)(k + 1) * nr * nr]);
            P.Sdd.assign(&hSdd[(size_t)k * nd * nd], &hSdd[(size_t)(k + 1) * nd * nd]);
            P.Urp.assign((size_t)nr * np, 0.0);
            P.Krp.assign((size_t)nr * np, 0.0);
            for (int r = 0; r < nr; ++r)
                for (int a = 0; a < np; ++a) {
                    P.Urp[(size_t)r * np + a] = hUqT[((size_t)k * np + a) * nr + r];
                    P.Krp[(size_t)r * np + a] = hKpr[((size_t)k * np + a) * nr + r];
                }
            P.Kpp.assign((size_t)np * np, 0.0);
            for (int a = 0; a < np; ++a)
                for (int b = 0; b <= a; ++b)
                    P.Kpp[(size_t)a * np + b] = P.Kpp[(size_t)b * np + a] = hKpp[((size_t)k * np + a) * np + b];
            P.Fdd.assign((size_t)nd * nd, 0.0);
            for (int i = 0; i < nd; ++i)
                for (int j = 0; j < nd; ++j) P.Fdd[(size_t)i * nd + j] = P.Kinv[(size_t)(ni + i) * nr + ni + j];
        });
    }
    clk.mark("principal bank");
    // 3. traces of eq. (42) with every cell's own operator K^(s).  K^(s) is linear in the cell's
    //    pulled-back tensor at the quadrature points (eq. (52)), so each trace tr(U^T K^(s) V) is the
    //    dot product of the cell snapshot with a table Psi[q][ab][cd] = w_q sum_col (grad U)_ab (grad V)_cd
    //    built once from the principal fields (the lookup-table idea of Sec. 4.2.1, Remark 9); all cells
    //    then need one GEMM against their snapshots.
    const int npair = K * (K + 1) / 2;
    const int ncoef = 2 * npair + K;  // A pairs, M pairs, b
    std::vector<int> pi_i(npair), pi_j(npair);
    {
        int t = 0;
        for (int i = 0; i < K; ++i)
            for (int j = i; j < K; ++j) {
                pi_i[t] = i;
                pi_j[t] = j;
                ++t;
            }
    }
    const size_t nsnap = (size_t)R.n_snap;
    DevBuf<double> dPsi;
    dPsi.alloc((size_t)ncoef * nsnap);
    trace_tables_device(c, K, dFq.p, dUqT.p, dPsi.p);
    std::vector<double> dv(K);
    for (int m = 0; m < K; ++m) {
        double tr = 0.0;
        for (int q = 0; q < nd; ++q) tr += bank[m].Fdd[(size_t)q * nd + q];
        dv[m] = tr;
    }
    // the greedy overwrote the snapshots with its residuals: rebuild them, then contract on the device
    launch_pulled_back(c);
    std::vector<double> traces((size_t)N * ncoef);
    {
        DevBuf<double> dOut;
        dOut.alloc((size_t)N * ncoef);
        GemmGroup g;
        g.A = dPsi.p;
        g.X = c->snap.p;
        g.Kd = (int)nsnap;
        g.ldx = (int)nsnap;
        g.K = 1;
        gemm(c, &g, 1, dOut.p, ncoef, 0, ncoef, N, false, 0, "coef_traces_gemm", false);
        IFETI_HIP(hipMemcpyAsync(traces.data(), dOut.p, traces.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        IFETI_HIP(hipStreamSynchronize(c->stream));
    }
    c->snap_valid = true;
    clk.mark("trace tables + snapshot GEMM");
    // 4. per-cell pi, delta (41)
    std::vector<double> pi((size_t)N * K), delta((size_t)N * K);
    parallel_for(N, [&](int s) {
        std::vector<double> A((size_t)K * K, 0.0), M((size_t)K * K, 0.0), b(K, 0.0);
        const double *tr = &traces[(size_t)s * ncoef];
        for (int t = 0; t < npair; ++t) {
            const int i = pi_i[t], j = pi_j[t];
            A[i * K + j] = A[j * K + i] = tr[t];
            M[i * K + j] = M[j * K + i] = tr[npair + t];
        }
        for (int i = 0; i < K; ++i) b[i] = tr[2 * npair + i];
        std::vector<double> x = small_spd_solve(A, K, b), y = small_spd_solve(M, K, dv);
        std::copy(x.begin(), x.end(), &pi[(size_t)s * K]);
        std::copy(y.begin(), y.end(), &delta[(size_t)s * K]);
    });
    clk.mark("pi, delta systems");
    // 5. S̊_pp^(s) = sym(K̊_pp - K̊_rp^T Ů_rp) (43) and the coarse matrix (Sec. 3.2.1)
    std::vector<double> Q((size_t)K * K * np * np);  // Q[m][k] = K_rp^(m)T U_rp^(k)
    parallel_for(K, [&](int m) {
        for (int k = 0; k < K; ++k)
            for (int a = 0; a < np; ++a)
                for (int b = 0; b < np; ++b) {
                    double s = 0.0;
                    for (int r = 0; r < nr; ++r) s += bank[m].Krp[(size_t)r * np + a] * bank[k].Urp[(size_t)r * np + b];
                    Q[(((size_t)m * K + k) * np + a) * np + b] = s;
                }
    });
    const int nP = c->nP;
    int bw = 0;
    for (int s = 0; s < N; ++s)
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
                int A1 = c->h_Ap[(size_t)s * np + a], B1 = c->h_Ap[(size_t)s * np + b];
                if (A1 >= 0 && B1 >= 0) bw = std::max(bw, std::abs(A1 - B1));
            }
    std::vector<double> band((size_t)nP * (bw + 1), 0.0);  // band[i][i-j] for j <= i
    std::vector<double> Xs((size_t)N * np * np, 0.0);     // per-cell S̊_pp, in parallel
    parallel_for(N, [&](int s) {
        const double *a = &alpha[(size_t)s * K], *pk = &pi[(size_t)s * K];
        double *X = &Xs[(size_t)s * np * np];
        for (int m = 0; m < K; ++m) {
            for (int t = 0; t < np * np; ++t) X[t] += a[m] * bank[m].Kpp[t];
            for (int k = 0; k < K; ++k) {
                double w = a[m] * pk[k];
                const double *q = &Q[((size_t)m * K + k) * np * np];
                for (int t = 0; t < np * np; ++t) X[t] -= w * q[t];
            }
        }
    });
    for (int s = 0; s < N; ++s) {  // assembly in cell order (fixed summation order)
        const double *X = &Xs[(size_t)s * np * np];
        for (int i = 0; i < np; ++i)
            for (int j = 0; j < np; ++j) {
                int I = c->h_Ap[(size_t)s * np + i], J = c->h_Ap[(size_t)s * np + j];
                if (I < 0 || J < 0 || J > I) continue;
                band[(size_t)I * (bw + 1) + (I - J)] += 0.5 * (X[i * np + j] + X[j * np + i]);
            }
    }
    c->co.h_Sband = band;
    c->co.bw = bw;
    // banded Cholesky factor L[i][j] -> band[i][i-j], on the GPU
    clk.mark("coarse matrix assembly");
    band = band_cholesky_device(c, band, nP, bw);
    clk.mark("coarse factor");
    // 6. upload the bank and the coefficients
    c->K = K;
    c->sigma = sigma;
    c->h_alpha = alpha;
    c->h_pi = pi;
    c->h_delta = delta;
    c->alpha.upload(alpha, c->stream);
    c->pi.upload(pi, c->stream);
    c->delta.upload(delta, c->stream);
    std::vector<double> Fdd((size_t)K * nd * nd), Sdd((size_t)K * nd * nd), W((size_t)K * nd * np),
        WT((size_t)K * np * nd), UrdT((size_t)K * nd * nr), Urd((size_t)K * nr * nd), Urp((size_t)K * nr * np),
        UrpT((size_t)K * np * nr), Kinv((size_t)K * nr * nr);
    parallel_for(K, [&](int k) {  // each principal fills its own slices
        const Principal &P = bank[k];
        std::copy(P.Fdd.begin(), P.Fdd.end(), &Fdd[(size_t)k * nd * nd]);
        std::copy(P.Sdd.begin(), P.Sdd.end(), &Sdd[(size_t)k * nd * nd]);
        for (int r = 0; r < nr; ++r)  // interleaved rows r*K + k: reduced bases come out as [r][k]
            std::copy(&P.Kinv[(size_t)r * nr], &P.Kinv[(size_t)(r + 1) * nr], &Kinv[((size_t)r * K + k) * nr]);
        std::copy(P.Urp.begin(), P.Urp.end(), &Urp[(size_t)k * nr * np]);
        for (int q = 0; q < nd; ++q)
            for (int a = 0; a < np; ++a) {
                double v = P.Urp[(size_t)(ni + q) * np + a];
                W[((size_t)k * nd + q) * np + a] = v;
                WT[((size_t)k * np + a) * nd + q] = v;
            }
        for (int r = 0; r < nr; ++r) {
            for (int q = 0; q < nd; ++q) {
                double v = P.Kinv[(size_t)r * nr + ni + q];
                Urd[((size_t)k * nr + r) * nd + q] = v;
                UrdT[((size_t)k * nd + q) * nr + r] = v;
            }
            for (int a = 0; a < np; ++a) UrpT[((size_t)k * np + a) * nr + r] = P.Urp[(size_t)r * np + a];
        }
    });
    c->Fdd.upload(Fdd, c->stream);
    c->Sdd.upload(Sdd, c->stream);
    c->W.upload(W, c->stream);
    c->WT.upload(WT, c->stream);
    c->UrdT.upload(UrdT, c->stream);
    c->Urd.upload(Urd, c->stream);
    c->Urp.upload(Urp, c->stream);
    c->UrpT.upload(UrpT, c->stream);
    c->Kinv.upload(Kinv, c->stream);
    combine_coarse_maps(c);
    IFETI_HIP(hipStreamSynchronize(c->stream));
    c->free_copies();  // the bank was (re)built: every fragment-ordered copy is stale
    clk.mark("bank upload");
    // 7. coarse solve: the band factor is kept; the explicit inverse S̊_PP^-1 follows on first use
    c->co.h_bandL = band;  // the explicit inverse is built on first use
    c->co.inv_ready = false;
    build_coarse_partition(c, c->co);
    // the coarse solve of 1-3 load cases reads the explicit inverse when no partition pays
    if (c->co.cp_p < 2 && c->nP > 0) ensure_coarse_inverse(c, c->co);
    build_coarse_approx(c, c->co);
    prepare_operator_copies(c);
    clk.mark("coarse partition");
    IFETI_HIP(hipStreamSynchronize(c->stream));
    c->rom_built = true;
}

}  // namespace ifeti
