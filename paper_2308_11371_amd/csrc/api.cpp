#include <algorithm>
// extern "C" entry points of libifeti (see include/ifeti.h).
#include <cmath>
#include <cstring>
#include <new>

#include "common.hpp"

namespace ifeti {
static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }
}  // namespace ifeti

using namespace ifeti;

template <class F>
static int guarded(F f) {
    try {
        return f();
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return IFETI_ENOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return IFETI_EINVAL;
    }
}

#define REQ(cond, msg) IFETI_REQUIRE(cond, IFETI_EINVAL, msg)

extern "C" {

const char *ifeti_last_error(void) { return g_last_error.c_str(); }

int ifeti_create(ifeti_ctx **out, const ifeti_lattice_desc *d, void *stream) {
    return guarded([&]() {
        REQ(out && d, "null argument");
        *out = nullptr;
        REQ(d->dim == 2 || d->dim == 3, "dim must be 2 or 3");
        REQ(d->nx >= 1 && d->ny >= 1 && d->nz >= 1, "cell counts must be >= 1");
        REQ(d->dim == 3 || d->nz == 1, "nz must be 1 in 2D");
        REQ(d->n_el >= 1, "n_el must be >= 1");
        REQ(d->degree == 2, "only quadratic splines (degree 2) are supported");
        REQ(d->h > 0 && d->E_in > 0, "h and E_in must be positive");
        REQ(d->E_out >= 0, "E_out must be >= 0");
        for (int i = 0; i < 9; ++i) REQ(std::isfinite(d->u0_grad[i]), "u0_grad must be finite");
        REQ(d->nu > -1.0 && d->nu < 0.5, "Poisson ratio must lie in (-1, 0.5)");
        REQ(d->smooth_eps >= 0, "smooth_eps must be >= 0");
        REQ(d->dirichlet_mask != 0 && (d->dirichlet_mask >> (2 * d->dim)) == 0, "dirichlet_mask must name faces");
        REQ(d->load_face >= -1 && d->load_face < 2 * d->dim, "load_face out of range");
        auto *c = new ifeti_ctx();
        c->desc = *d;
        c->dim = d->dim;
        c->shape[0] = d->nx;
        c->shape[1] = d->ny;
        c->shape[2] = d->dim == 3 ? d->nz : 1;
        c->N = c->shape[0] * c->shape[1] * c->shape[2];
        c->stream = (hipStream_t)stream;
        try {
            build_reference_tables(c);
            build_partition(c);
            build_decomposition(c);
            const RefTables &R = c->ref;
            c->g_tables_w.upload(R.w, c->stream);
            c->g_tables_xi.upload(R.xi, c->stream);
            c->g_tables_dN.upload(R.dN, c->stream);
            c->g_tables_1d.upload(R.tab1, c->stream);
            c->g_tables_ctrl.upload(R.elem_ctrl, c->stream);
            c->g_idx_r.upload(c->idx_r, c->stream);
            c->g_idx_p.upload(c->idx_p, c->stream);
            IFETI_HIP(hipStreamSynchronize(c->stream));
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
        return IFETI_OK;
    });
}

void ifeti_destroy(ifeti_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->local_stream) (void)hipStreamSynchronize(c->local_stream);
    release_events(c);
    if (c->local_stream) {
        (void)hipStreamDestroy(c->local_stream);
        (void)hipEventDestroy(c->ev_local_fork);
        (void)hipEventDestroy(c->ev_local_join);
    }
    if (c->side_stream) {
        (void)hipStreamSynchronize(c->side_stream);
        (void)hipStreamDestroy(c->side_stream);
        (void)hipEventDestroy(c->ev_fork);
        (void)hipEventDestroy(c->ev_join);
    }
    release_graph(c);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    if (c->ev_poll) (void)hipEventDestroy(c->ev_poll);
    for (int i = 0; i < 2; ++i) {
        if (c->h_poll[i]) (void)hipHostFree(c->h_poll[i]);
        if (c->ev_pollv[i]) (void)hipEventDestroy(c->ev_pollv[i]);
    }
    if (c->own_stream) {
        (void)hipStreamSynchronize(c->own_stream);
        (void)hipStreamDestroy(c->own_stream);
        (void)hipEventDestroy(c->ev_own_in);
        (void)hipEventDestroy(c->ev_own_out);
    }
    delete c;
}

int ifeti_get_stats(ifeti_ctx *c, ifeti_stats *o) {
    return guarded([&]() {
        REQ(c && o, "null argument");
        flush_events(c);
        std::memset(o, 0, sizeof(*o));
        for (int i = 0; i < IFETI_OP_COUNT; ++i) o->applies[i] = c->applies[i];
        o->pcg_iterations = c->pcg_its;
        o->fgmres_iterations = c->fgmres_its;
        int n = 0;
        for (const auto &k : c->kstats) {
            if (n >= 32) break;
            ifeti_kernel_stat &d = o->kernels[n++];
            std::strncpy(d.name, k.name.c_str(), sizeof(d.name) - 1);
            d.launches = k.launches;
            d.timed = k.timed;
            d.total_ms = k.ms;
            d.flops = k.flops;
            d.bytes = k.bytes;
        }
        o->n_kernels = n;
        return IFETI_OK;
    });
}

int ifeti_reset_stats(ifeti_ctx *c) {
    return guarded([&]() {
        REQ(c, "null argument");
        flush_events(c);
        for (auto &x : c->applies) x = 0;
        c->pcg_its = c->fgmres_its = 0;
        c->kstats.clear();
        return IFETI_OK;
    });
}

int ifeti_get_sizes(const ifeti_ctx *c, ifeti_sizes *o) {
    return guarded([&]() {
        REQ(c && o, "null argument");
        o->N = c->N;
        o->dim = c->dim;
        o->n_ctrl = c->ref.n_ctrl;
        o->n_dof = c->ref.n_dof;
        o->n_i = c->n_i;
        o->n_d = c->n_d;
        o->n_p = c->n_p;
        o->n_r = c->n_r;
        o->L = c->L;
        o->L_interface = c->L_int;
        o->nP = c->nP;
        o->nU = c->nU;
        o->K = c->K;
        o->nrhs = c->nrhs;
        return IFETI_OK;
    });
}

int ifeti_set_options(ifeti_ctx *c, const ifeti_options *opt) {
    return guarded([&]() {
        REQ(c && opt, "null argument");
        REQ(opt->precision == IFETI_FP64 || opt->precision == IFETI_FP32_LOCAL || opt->precision == IFETI_BF16_LOCAL,
            "precision must be IFETI_FP64, IFETI_FP32_LOCAL or IFETI_BF16_LOCAL");
        REQ(opt->pcg_check_every >= 1, "pcg_check_every must be >= 1");
        REQ(opt->fgmres_restart >= 1, "fgmres_restart must be >= 1");
        REQ(opt->pcg_maxit >= 1, "pcg_maxit must be >= 1");
        c->opt.pcg_maxit = opt->pcg_maxit;
        c->opt.precision = opt->precision;
        c->opt.pcg_check_every = opt->pcg_check_every;
        c->opt.fgmres_restart = opt->fgmres_restart;
        if (!opt->timing) flush_events(c);
        c->opt.timing = opt->timing ? 1 : 0;
        c->opt.timing_filter.assign(opt->timing_filter, strnlen(opt->timing_filter, sizeof(opt->timing_filter)));
        c->opt.timing_every = std::max(1, opt->timing_every);
        c->opt.use_graph = opt->use_graph ? 1 : 0;
        c->opt.autotune = opt->autotune ? 1 : 0;
        REQ(opt->interface_block >= 0 && opt->interface_block <= 2, "interface_block must be 0, 1 or 2");
        c->opt.interface_block = opt->interface_block;
        c->opt.overlap_local = opt->overlap_local ? 1 : 0;
        REQ(opt->md_precision >= -1 && opt->md_precision <= IFETI_BF16_LOCAL, "md_precision must be -1, 0, 1 or 2");
        c->opt.md_precision = opt->md_precision;
        REQ(opt->local_iters >= 1 && opt->local_iters <= 8, "local_iters must be in [1, 8]");
        c->opt.local_iters = opt->local_iters;
        REQ(opt->true_operator == 0 || opt->true_operator == 1, "true_operator must be 0 or 1");
        REQ(opt->true_operator == 0 || c->ref.p == 2, "the matrix-free true operator needs quadratic B-splines");
        c->opt.true_operator = opt->true_operator;
        REQ(opt->tile_candidate >= -1, "tile_candidate must be >= -1");
        c->opt.tile_candidate = opt->tile_candidate;
        REQ(opt->block_cg == 0 || opt->block_cg == 1, "block_cg must be 0 or 1");
        c->opt.block_cg = opt->block_cg;
        REQ(opt->coarse_approx >= 0, "coarse_approx must be >= 0");
        if (opt->coarse_approx != c->opt.coarse_approx) {
            c->opt.coarse_approx = opt->coarse_approx;
            if (c->rom_built) build_coarse_approx(c, c->co);
        }
        REQ(opt->coarse_parts >= 0, "coarse_parts must be >= 0");
        if (opt->coarse_parts != c->opt.coarse_parts) {
            c->opt.coarse_parts = opt->coarse_parts;
            if (c->rom_built) build_coarse_partition(c, c->co);
            if (c->ex_built) build_coarse_partition(c, c->co_ex);
        }
        return IFETI_OK;
    });
}

int ifeti_get_options(const ifeti_ctx *c, ifeti_options *o) {
    return guarded([&]() {
        REQ(c && o, "null argument");
        std::memset(o, 0, sizeof(*o));
        const Options &p = c->opt;
        o->precision = p.precision;
        o->pcg_check_every = p.pcg_check_every;
        o->fgmres_restart = p.fgmres_restart;
        o->pcg_maxit = p.pcg_maxit;
        o->timing = p.timing;
        std::strncpy(o->timing_filter, p.timing_filter.c_str(), sizeof(o->timing_filter) - 1);
        o->timing_every = p.timing_every;
        o->use_graph = p.use_graph;
        o->autotune = p.autotune;
        o->coarse_parts = p.coarse_parts;
        o->true_operator = p.true_operator;
        o->interface_block = p.interface_block;
        o->overlap_local = p.overlap_local;
        o->local_iters = p.local_iters;
        o->md_precision = p.md_precision;
        o->tile_candidate = p.tile_candidate;
        o->coarse_approx = p.coarse_approx;
        o->block_cg = p.block_cg;
        return IFETI_OK;
    });
}

int ifeti_build_cells(ifeti_ctx *c, const double *ctrl_pts, const double *widths, const double *tractions,
                      int nrhs) {
    return guarded([&]() {
        REQ(c && ctrl_pts && widths, "null argument");
        REQ(nrhs >= 1, "nrhs must be >= 1");
        REQ(tractions || c->desc.load_face < 0, "tractions required when a load face is set");
        const RefTables &R = c->ref;
        const int N = c->N;
        c->ctrl.alloc((size_t)N * R.n_ctrl * c->dim);
        IFETI_HIP(hipMemcpyAsync(c->ctrl.p, ctrl_pts, c->ctrl.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        c->widths.alloc(N);
        IFETI_HIP(hipMemcpyAsync(c->widths.p, widths, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        std::vector<double> hw(N);
        IFETI_HIP(hipMemcpyAsync(hw.data(), widths, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        IFETI_HIP(hipStreamSynchronize(c->stream));
        for (double w : hw) REQ(std::isfinite(w) && w > 0.0, "strut widths must be positive and finite");
        c->nrhs = nrhs;
        c->tractions.assign((size_t)nrhs * c->dim, 0.0);
        if (tractions) std::memcpy(c->tractions.data(), tractions, c->tractions.size() * sizeof(double));
        c->snap.alloc((size_t)N * R.n_snap);
        c->Kst.alloc((size_t)N * R.n_ctrl * R.n_off * c->dim * c->dim);
        launch_pulled_back(c);
        launch_stiffness(c);
        build_loads(c);
        IFETI_HIP(hipStreamSynchronize(c->stream));
        c->cells_built = true;
        c->snap_valid = true;
        c->rom_built = false;
        c->ex_built = false;  // the exact factorisation belongs to the previous cells
        ++c->rom_gen;
        return IFETI_OK;
    });
}

int ifeti_get_rhs(ifeti_ctx *c, double *f, double *d) {
    return guarded([&]() {
        REQ(c && c->cells_built, "cells not built");
        if (f)
            IFETI_HIP(hipMemcpyAsync(f, c->f_vec.p, c->f_vec.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        if (d)
            IFETI_HIP(hipMemcpyAsync(d, c->d_vec.p, c->d_vec.n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        return IFETI_OK;
    });
}

int ifeti_build_reduced_basis(ifeti_ctx *c, int n_principal, double tol_rb, const int *principal_in,
                              int *principal_out, double *theta_out) {
    return guarded([&]() {
        REQ(c && c->cells_built, "cells not built");
        REQ(n_principal >= 1 && n_principal <= c->N, "n_principal must be in [1, N]");
        REQ(n_principal <= 40, "at most 40 principal cells are supported");
        REQ(tol_rb >= 0.0, "tol_rb must be >= 0");
        if (!c->snap_valid) launch_pulled_back(c);  // the greedy consumes the snapshots
        c->snap_valid = false;
        c->rom_built = false;
        build_reduced_basis(c, n_principal, tol_rb, principal_in);
        if (principal_out)
            for (int k = 0; k < c->K; ++k) principal_out[k] = c->sigma[k];
        if (theta_out)
            IFETI_HIP(hipMemcpyAsync(theta_out, c->alpha.p, c->alpha.n * sizeof(double), hipMemcpyDeviceToDevice,
                                     c->stream));
        ensure_work(c, 1);
        IFETI_HIP(hipStreamSynchronize(c->stream));
        return IFETI_OK;
    });
}

int ifeti_get_coefficients(ifeti_ctx *c, double *alpha, double *pi, double *delta) {
    return guarded([&]() {
        REQ(c && c->rom_built, "reduced basis not built");
        if (alpha) std::memcpy(alpha, c->h_alpha.data(), c->h_alpha.size() * sizeof(double));
        if (pi) std::memcpy(pi, c->h_pi.data(), c->h_pi.size() * sizeof(double));
        if (delta) std::memcpy(delta, c->h_delta.data(), c->h_delta.size() * sizeof(double));
        return IFETI_OK;
    });
}

#define ROM_READY(c, nrhs)                                                        \
    REQ(c && c->rom_built, "reduced basis not built");                           \
    REQ((nrhs) >= 1 && (long long)c->N * (nrhs) < (1LL << 31), "nrhs out of range")

int ifeti_apply_F(ifeti_ctx *c, const double *lam, double *out, int nrhs) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(lam && out && lam != out, "bad pointers");
        apply_F(c, lam, out, nrhs);
        return IFETI_OK;
    });
}

int ifeti_apply_MD(ifeti_ctx *c, const double *r, double *out, int nrhs) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(r && out && r != out, "bad pointers");
        apply_MD(c, r, out, nrhs);
        return IFETI_OK;
    });
}

int ifeti_apply_MD_rom(ifeti_ctx *c, const double *r, double *out, int nrhs) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(r && out && r != out, "bad pointers");
        apply_MD_rom(c, r, out, nrhs);
        return IFETI_OK;
    });
}

int ifeti_cell_displacements(ifeti_ctx *c, const double *u, double *out, int nrhs) {
    return guarded([&]() {
        REQ(c && c->cells_built, "cells not built");
        REQ(nrhs >= 1 && (long long)c->N * c->ref.n_dof * nrhs < (1LL << 40), "nrhs out of range");
        REQ(u && out && u != out, "bad pointers");
        cell_displacements(c, u, out, nrhs);
        return IFETI_OK;
    });
}

int ifeti_apply_U(ifeti_ctx *c, const double *v, double *z, int nrhs) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(v && z, "bad pointers");
        apply_U(c, v, z, nrhs);
        return IFETI_OK;
    });
}

int ifeti_apply_Ut(ifeti_ctx *c, const double *y, double *x, int nrhs) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(y && x, "bad pointers");
        apply_Ut(c, y, x, nrhs);
        return IFETI_OK;
    });
}

int ifeti_apply_Kinv_rom(ifeti_ctx *c, const double *v, double *x, int nrhs) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(v && x && v != x, "bad pointers");
        apply_Kinv_rom(c, v, x, nrhs);
        return IFETI_OK;
    });
}

int ifeti_apply_A(ifeti_ctx *c, const double *x, double *y, int nrhs) {
    return guarded([&]() {
        REQ(c && c->cells_built, "cells not built");
        REQ(nrhs >= 1, "nrhs must be >= 1");
        REQ(x && y && x != y, "bad pointers");
        apply_A(c, x, y, nrhs);
        return IFETI_OK;
    });
}

int ifeti_solve_interface(ifeti_ctx *c, const double *rhs, double *lam, int nrhs, double tol, int maxit,
                          int *iters_out, double *relres_out) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(rhs && lam && rhs != lam, "bad pointers");
        REQ(tol > 0 && maxit >= 1, "tol must be > 0 and maxit >= 1");
        return solve_interface(c, rhs, lam, nrhs, tol, maxit, iters_out, relres_out);
    });
}

int ifeti_recover_displacement(ifeti_ctx *c, const double *v, const double *y, double *u, int nrhs) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(v && y && u && v != u, "bad pointers");
        DevBuf<double> t;
        t.alloc((size_t)c->nU * nrhs);
        apply_Kinv_rom(c, v, u, nrhs);
        apply_Ut(c, y, t.p, nrhs);
        // u -= Ůᵀ y
        std::vector<double> m1(nrhs, -1.0);
        DevBuf<double> coef;
        coef.upload(m1, c->stream);
        multiaxpy(c, t.p, 0, 1, coef.p, 1.0, u, c->nU, c->nU, nrhs);
        IFETI_HIP(hipStreamSynchronize(c->stream));
        return IFETI_OK;
    });
}

int ifeti_solve(ifeti_ctx *c, const double *f, const double *d, double *u, double *lam, int nrhs, double tol,
                int maxit, double inner_tol, int *outer_iters, int *inner_iters_total, double *relres) {
    return guarded([&]() {
        ROM_READY(c, nrhs);
        REQ(f && d && u && lam, "bad pointers");
        REQ(tol > 0 && inner_tol > 0 && maxit >= 1, "tolerances must be > 0 and maxit >= 1");
        return solve_fgmres(c, f, d, u, lam, nrhs, tol, maxit, inner_tol, outer_iters, inner_iters_total, relres);
    });
}

int ifeti_compliance_grad(ifeti_ctx *c, const double *f, const double *u, double *grad, double *compliance,
                          int nrhs) {
    return guarded([&]() {
        REQ(c && c->cells_built, "cells not built");
        REQ(f && u && grad, "bad pointers");
        REQ(nrhs >= 1, "nrhs must be >= 1");
        REQ(c->desc.smooth_eps > 0.0,
            "the width gradient needs a smoothed strut indicator (smooth_eps > 0): with the sharp one the cell "
            "operators are piecewise constant in the widths");
        ensure_work(c, nrhs);
        compliance_grad(c, f, u, grad, compliance, nrhs);
        return IFETI_OK;
    });
}

int ifeti_update_widths(ifeti_ctx *c, const double *widths) {
    return guarded([&]() {
        REQ(c && c->cells_built, "cells not built");
        REQ(widths, "bad pointer");
        const int N = c->N;
        std::vector<double> hw(N);
        IFETI_HIP(hipMemcpyAsync(hw.data(), widths, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        IFETI_HIP(hipStreamSynchronize(c->stream));
        for (double w : hw) REQ(std::isfinite(w) && w > 0.0, "strut widths must be positive and finite");
        IFETI_HIP(hipMemcpyAsync(c->widths.p, widths, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        launch_pulled_back(c);
        launch_stiffness(c);
        if (has_dirichlet_data(c)) build_loads(c);  // the lifting of the Dirichlet corners uses K
        IFETI_HIP(hipStreamSynchronize(c->stream));
        c->snap_valid = true;
        ++c->rom_gen;
        c->ex_built = false;  // the exact factorisation belongs to the previous widths
        return IFETI_OK;
    });
}

#define EXACT_READY(c, nrhs)                                                      \
    REQ(c && c->ex_built, "exact FETI-DP not built (ifeti_build_exact)");        \
    REQ((nrhs) >= 1 && (long long)c->N * (nrhs) < (1LL << 31), "nrhs out of range")

int ifeti_build_exact(ifeti_ctx *c) {
    return guarded([&]() {
        REQ(c && c->cells_built, "cells not built");
        c->ex_built = false;
        build_exact(c);
        return IFETI_OK;
    });
}

int ifeti_exact_apply_F(ifeti_ctx *c, const double *lam, double *out, int nrhs) {
    return guarded([&]() {
        EXACT_READY(c, nrhs);
        REQ(lam && out && lam != out, "bad pointers");
        apply_F_exact(c, lam, out, nrhs);
        return IFETI_OK;
    });
}

int ifeti_exact_apply_MD(ifeti_ctx *c, const double *r, double *out, int nrhs) {
    return guarded([&]() {
        EXACT_READY(c, nrhs);
        REQ(r && out && r != out, "bad pointers");
        apply_MD_exact(c, r, out, nrhs);
        return IFETI_OK;
    });
}

int ifeti_exact_solve(ifeti_ctx *c, const double *f, const double *d, double *u, double *lam, int nrhs, double tol,
                      int maxit, int *iters, double *relres) {
    return guarded([&]() {
        EXACT_READY(c, nrhs);
        REQ(f && d && u && lam, "bad pointers");
        REQ(tol > 0 && maxit >= 1, "tol must be > 0 and maxit >= 1");
        const int st = solve_exact(c, f, d, u, lam, nrhs, tol, maxit, iters, relres);
        if (st == IFETI_EMAXIT) set_last_error("PCG reached the iteration limit");
        return st;
    });
}

int ifeti_exact_cell_blocks(ifeti_ctx *c, int s, double *Fdd, double *Sdd, double *Spp, double *Ud,
                            long long *device_bytes) {
    return guarded([&]() {
        REQ(c && c->ex_built, "exact FETI-DP not built (ifeti_build_exact)");
        REQ(s >= 0 && s < c->N, "cell index out of range");
        const size_t nd = c->n_d, np = c->n_p;
        IFETI_HIP(hipStreamSynchronize(c->stream));
        if (Fdd) IFETI_HIP(hipMemcpy(Fdd, c->ex_Fdd.p + s * nd * nd, nd * nd * sizeof(double), hipMemcpyDeviceToHost));
        if (Sdd) IFETI_HIP(hipMemcpy(Sdd, c->ex_Sdd.p + s * nd * nd, nd * nd * sizeof(double), hipMemcpyDeviceToHost));
        if (Spp) IFETI_HIP(hipMemcpy(Spp, c->ex_Spp.p + s * np * np, np * np * sizeof(double), hipMemcpyDeviceToHost));
        if (Ud) {
            std::vector<double> C(np * nd);
            IFETI_HIP(hipMemcpy(C.data(), c->ex_C.p + s * np * nd, C.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (size_t j = 0; j < nd; ++j)
                for (size_t a = 0; a < np; ++a) Ud[j * np + a] = C[a * nd + j];
        }
        if (device_bytes) {
            const CoarseSolver &co = c->co_ex;
            long long b = 0;
            for (size_t n : {c->ex_L.n, c->ex_Fdd.n, c->ex_Sdd.n, c->ex_C.n, c->ex_Spp.n, c->ex_Kpr.n, co.SPPinv.n,
                             co.SPPt.n, co.cp_M1.n, co.cp_M2.n, co.cp_M3.n})
                b += (long long)n * 8;
            *device_bytes = b;
        }
        return IFETI_OK;
    });
}

}  // extern "C"
