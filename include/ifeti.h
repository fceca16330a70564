/*
 * ifeti.h -- C ABI of the MI355X (gfx950) ROM-based inexact FETI-DP library.
 *
 * Method: T. Hirschler, R. Bouclier, P. Antolin, A. Buffa, "Reduced Order
 * Modeling based Inexact FETI-DP solver for lattice structures".  Every cell
 * of a lattice is one subdomain (Sec. 2.1, eq. (1)); every cell space is the
 * push-forward of one reference quadratic B-spline space (eq. (6)); corners
 * are primal, the other cell-boundary control points dual (Sec. 2.2.2); the
 * saddle system (16) is solved by flexible GMRES preconditioned by the block
 * preconditioner (44) whose sub-blocks are built from a few principal cells
 * chosen by the greedy of Algorithm 4 (Sec. 3, 4.2).
 *
 * Conventions (all calls):
 *  - Every call returns an ifeti_status (0 = success) and never throws; on
 *    failure a message is kept per thread and returned by ifeti_last_error().
 *  - "dev" pointers are device (HIP) memory owned by the caller; "host"
 *    pointers are host memory owned by the caller.  No call keeps a caller
 *    pointer after it returns.  The context owns all of its internal
 *    buffers (cell operators, principal bank, coefficients, coarse inverse).
 *  - Work is enqueued on the stream given to ifeti_create; calls return
 *    without a device synchronisation unless they write host outputs
 *    (iteration counts, residuals, principal lists), which synchronise.
 *  - Vectors are float64.  Multi-RHS vectors are rhs-major: right-hand side
 *    r occupies [r*n, (r+1)*n).
 *  - Displacement layout u = (u_r^(1), ..., u_r^(N), u_P) (eq. (13)):
 *    u_r^(s) holds the n_r = n_i + n_d non-primal dofs of cell s, interior
 *    dofs first then dual dofs, each in ascending local dof order with local
 *    dof = dim*a + component and control point a = ax + nc*(ay + nc*az);
 *    u_P holds the primal (corner) dofs of the lattice vertices not on a
 *    Dirichlet face, vertex-major in lexicographic (x fastest) order.
 *  - Multipliers lambda in R^L (eqs. (14)-(16)): one row per matching dual
 *    dof pair (chained by ascending cell index where more than two cells share
 *    a dof, +1 on the lower cell, -1 on the higher) and one +1 row per cell
 *    copy of a dual dof on a Dirichlet face; interface rows sorted by
 *    (global control point, component, chain position), then the Dirichlet
 *    rows in the same key order.
 *  - Cells: s = ix + nx*(iy + ny*iz).
 */
#ifndef IFETI_H
#define IFETI_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ifeti_ctx ifeti_ctx;

typedef enum {
    IFETI_OK = 0,
    IFETI_EINVAL = -1,      /* bad argument, shape or call order            */
    IFETI_ENOMEM = -2,      /* device or host allocation failed             */
    IFETI_ENOTSPD = -3,     /* a Cholesky factorisation met a pivot <= 0    */
    IFETI_EBREAKDOWN = -4,  /* PCG p^T F p <= 0 or non-finite               */
    IFETI_EMAXIT = -5,      /* iteration limit reached (partial result kept)*/
    IFETI_EHIP = -6         /* a HIP runtime call failed                    */
} ifeti_status;

typedef enum {
    IFETI_FP64 = 0,         /* every contraction in float64                 */
    IFETI_FP32_LOCAL = 1,   /* principal contractions fp32 operands/accum   */
    IFETI_BF16_LOCAL = 2    /* principal contractions bf16 operands, fp32 accum */
} ifeti_precision;

/* Lattice description (paper Sec. 2.2.1 and 4.1).  Geometry enters through
 * the control points passed to ifeti_build_cells. */
typedef struct {
    int dim;                /* 2 (plane strain) or 3                         */
    int nx, ny, nz;         /* cells per direction (nz = 1 in 2D)            */
    int n_el;               /* elements per direction per cell               */
    int degree;             /* spline degree; 2 is supported                 */
    double h;               /* cell size of the reference lattice            */
    double E_in, E_out;     /* Young modulus inside (> 0) / outside (>= 0; 0 leaves voids, whose cells
                               may be singular: ENOTSPD from the factorisations) the struts */
    double nu;              /* Poisson ratio                                 */
    double smooth_eps;      /* 0: sharp strut indicator; > 0: tanh width     */
    int dirichlet_mask;     /* bit f set: face f carries Dirichlet data u = u0;
                               faces 0:X=0 1:X=Lx 2:Y=0 3:Y=Ly 4:Z=0 5:Z=Lz   */
    int load_face;          /* face carrying the constant traction, -1: none */
    double u0_grad[9];      /* Dirichlet data (3c): u0(x) = G x at the control points of the Dirichlet
                               faces, G row-major dim x dim (first dim*dim entries); all zero: clamped.
                               Dual dofs on the faces take u0 through their +1 rows of B (d of eq. (14));
                               primal corners on the faces are eliminated from u_P and their values
                               lifted into f (f -= K u0 on those columns) by ifeti_build_cells */
} ifeti_lattice_desc;

typedef struct {
    int N, dim, n_ctrl, n_dof;  /* cells; dofs per cell = dim*n_ctrl        */
    int n_i, n_d, n_p, n_r;     /* local partition (eq. (12))               */
    int L, L_interface;         /* multipliers; interface rows come first    */
    int nP;                     /* assembled primal dofs                     */
    long long nU;               /* N*n_r + nP (eq. (13))                     */
    int K;                      /* principal cells (after the greedy)        */
    int nrhs;                   /* load cases given to ifeti_build_cells     */
} ifeti_sizes;

typedef struct {
    int precision;          /* ifeti_precision of the principal contractions */
    int pcg_check_every;    /* PCG host convergence check interval (>= 1; default 2) */
    int fgmres_restart;     /* maximum Krylov dimension of the outer solver */
    int pcg_maxit;          /* iteration cap of the interface PCG inside the preconditioner */
    int timing;             /* 1: time kernel launches with HIP events       */
    char timing_filter[256]; /* "" : every kernel family; else a comma-separated list of families
                                (NUL-terminated; longer lists are the caller's error) */
    int timing_every;       /* time one launch in this many of each family (<= 1: every launch) */
    int use_graph;          /* 1: the interface PCG runs its first iteration eagerly, captures the
                               second in a HIP graph (both streams) and replays it for the rest;
                               results are bitwise those of the eager loop; kernel timing is off
                               for the replayed iterations */
    int autotune;           /* 1: the first launch of each contraction shape times the candidate tile
                               shapes and keeps the fastest for the context's lifetime (results then
                               agree with the default tiles to rounding, not bitwise) */
    int coarse_parts;       /* coarse solve S̊_PP^-1 for 1-3 load cases: 0 automatic (fewest bytes per
                               apply), 1 the explicit inverse in symmetric tiles, p >= 2 the partitioned
                               solve with p interior blocks (EINVAL if the band does not allow p) */
    int true_operator;      /* cell operator K^(s) in the true operator (16) (ifeti_apply_A, the outer
                               solver, the displacement recovery): 0 the assembled stencil values,
                               1 matrix-free (Sec. 4.2.1, Remark 9): from the pulled-back tensor at the
                               quadrature points and the shared 1D B-spline tables, element by element
                               in 3^dim colours (quadratic B-splines only, EINVAL otherwise); both
                               are deterministic */
    int interface_block;    /* interface block of the preconditioner (Alg. 1): 0 F̊^-pcg (PCG on (48)
                               preconditioned by (49)); 1 one application of M̊_D^-1 (49); 2 one
                               application of M̊_D^-ROM (47), the Dirichlet preconditioner with
                               reduced interior solves (Sec. 3.2.3).  1 and 2 make the preconditioner
                               cheaper and the outer FGMRES longer */
    int overlap_local;      /* 1: inside the preconditioner, the reduced local solves of (46) on v
                               run on a third stream while Ů v and the interface PCG run on the main
                               stream (they share no buffers); results are bitwise those of 0.  The
                               solve gains about 1 % on c2 while the interface contractions that meet
                               the local solve's contraction slow down; 0 by default.  Ignored with
                               use_graph = 1 or interface_block != 0 */
    int local_iters;        /* 1: the reduced local solves of (46); 2..8: K̊^-MPCG of Remark 6, that
                               many multi-preconditioned CG iterations per cell with the principal
                               inverses as the preconditioners (the first iteration is (46); later
                               blocks are made K_rr^(s)-conjugate to all earlier ones) */
    int md_precision;       /* precision of the M̊_D^-1 contraction (49), an ifeti_precision, or -1 for
                               the value of `precision`: e.g. FP32 operators with a BF16 preconditioner
                               (PCG only needs the preconditioner to stay symmetric positive definite) */
    int tile_candidate;     /* -1: tile shapes of the principal contractions by default or by the autotuner;
                               i >= 0: candidate i of each contraction's family (modulo the family's
                               size), for every launch; the autotuner is bypassed.  Each candidate sums
                               in its own fixed order (results agree across candidates to rounding) */
    int coarse_approx;      /* 0: the coarse problem S̊_PP^-1 solved exactly (Sec. 3.2.1); B >= 1: the
                               approximate coarse solve Sec. 3.2.1 allows in the inexact method, block
                               Jacobi over consecutive blocks of B primal dofs (inverse of each diagonal
                               block of S̊_PP; one streamed pass per apply).  Applies to the ROM operators
                               F̊, Ů, Ůᵀ and K̊^-ROM; it stays linear and symmetric positive definite, so the
                               interface PCG stays valid and the outer FGMRES still converges to the
                               solution of (16).  B >= nP gives the exact solve */
    int block_cg;           /* 0: several load cases of the interface problem run as independent PCG
                               recurrences sharing each operator application; 1: O'Leary's block PCG on
                               them (the block Krylov space of all load cases; breakdown-free form: the
                               search block is orthonormalised each step and linearly dependent
                               directions dropped, so dependent load cases cost no operator columns).
                               Single load cases and the standard FETI-DP solve are unaffected */
} ifeti_options;

/* Per-kernel-family statistics.  flops and bytes are the algorithmic counts
 * (operations the method needs, minimum HBM traffic of the launch), summed
 * over launches; total_ms is the sum of the HIP-event durations of the `timed`
 * launches (0 unless options.timing = 1); the average launch time is
 * total_ms / timed. */
typedef struct {
    char name[32];
    long long launches;
    double total_ms;
    double flops;
    double bytes;
    long long timed;
} ifeti_kernel_stat;

enum { IFETI_OP_F = 0, IFETI_OP_MD, IFETI_OP_U, IFETI_OP_UT, IFETI_OP_KINV_ROM, IFETI_OP_A, IFETI_OP_COUNT };

typedef struct {
    long long applies[IFETI_OP_COUNT];  /* operator applications times load cases */
    long long pcg_iterations;           /* interface PCG iterations, summed over load cases */
    long long fgmres_iterations;        /* outer iterations, summed over load cases */
    int n_kernels;
    ifeti_kernel_stat kernels[32];
} ifeti_stats;

/* Statistics since the last reset (synchronises the stream when timing is on). */
int ifeti_get_stats(ifeti_ctx *ctx, ifeti_stats *out);
int ifeti_reset_stats(ifeti_ctx *ctx);

/* Create a context for the lattice `desc`; work goes to `hip_stream`
 * (hipStream_t, may be NULL for the default stream).  EINVAL for an
 * unsupported description. */
int ifeti_create(ifeti_ctx **ctx, const ifeti_lattice_desc *desc, void *hip_stream);
void ifeti_destroy(ifeti_ctx *ctx);
const char *ifeti_last_error(void);
int ifeti_get_sizes(const ifeti_ctx *ctx, ifeti_sizes *out);
int ifeti_set_options(ifeti_ctx *ctx, const ifeti_options *opt);
/* Current options of the context (all fields), e.g. to change one field and set them back. */
int ifeti_get_options(const ifeti_ctx *ctx, ifeti_options *out);

/* Assemble every cell (Sec. 4.2.1, eq. (52)): pulled-back material tensor at
 * the 3^d Gauss points of each element (the greedy snapshots), cell
 * stiffness on the shared stencil, consistent tractions (eq. (5b)), and the
 * decomposition bookkeeping B, D, A_p (eqs. (14)-(18), (30)).
 *   ctrl_pts  dev  N x n_ctrl x dim control points of the cell maps
 *   widths    dev  N strut widths
 *   tractions host nrhs x dim constant traction per load case on load_face
 * EINVAL on a non-positive width or a non-invertible cell map. */
int ifeti_build_cells(ifeti_ctx *ctx, const double *ctrl_pts, const double *widths,
                      const double *tractions, int nrhs);

/* Right-hand side of (16): f (dev, nU x nrhs) and d (dev, L x nrhs); with Dirichlet data u0 != 0
 * f includes the lifting of the Dirichlet corners and d holds u0 on the Dirichlet rows. */
int ifeti_get_rhs(ifeti_ctx *ctx, double *f, double *d);

/* Offline phase (Sec. 3.1, 3.2.1, 4.2.2): greedy of Algorithm 4 (stops after
 * n_principal picks or when the residual max-norm falls to tol_rb), principal
 * bank (eqs. (22), (27)-(30), (39)), coefficients pi, delta (eqs. (40)-(42)),
 * ROM operators (43) and the coarse matrix with its explicit inverse.
 *   principal_in  host, nullable: n_principal cell indices used instead of the greedy picks
 *   principal_out host, nullable: receives the K chosen cells (room for n_principal)
 *   theta_out     dev,  nullable: N x K affine coordinates alpha (eq. (38), (56))
 * ENOTSPD if a principal K_rr or the coarse matrix is not positive definite. */
int ifeti_build_reduced_basis(ifeti_ctx *ctx, int n_principal, double tol_rb,
                              const int *principal_in, int *principal_out, double *theta_out);

/* Host copies of the per-cell coefficients, each N x K row-major
 * (alpha eq. (38); pi, delta eq. (41)).  Any pointer may be NULL. */
int ifeti_get_coefficients(ifeti_ctx *ctx, double *alpha, double *pi, double *delta);

/* out = F̊ lam, the ROM dual operator of eq. (48), lam/out dev L x nrhs. */
int ifeti_apply_F(ifeti_ctx *ctx, const double *lam, double *out, int nrhs);
/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops that
 * forbid hipMalloc): out = F̊ lam exactly as ifeti_apply_F computes it (bitwise the same values), with
 * its work buffers in a device array the library holds for the life of the process, 32 MiB on each
 * GPU it runs on; the call makes no device or host allocation.  All work goes to the context stream
 * (no second stream).  Limits: 1 to 3 load cases, and 8 * (N nrhs (2 n_d + n_p) + 2 nP nrhs) bytes
 * (each part rounded up to 256 B) at most 32 MiB (c2: one to three load cases), EINVAL otherwise.
 * Needs the copies ifeti_build_reduced_basis makes (FP64 operators); in the FP32/BF16 precision form
 * the narrow copies are made by the first ifeti_apply_F in that precision (EINVAL before).  Calls
 * share each GPU's array: calls that overlap on one GPU (other streams, other threads, other
 * contexts) race and give wrong results.  No statistics are recorded for these calls. */
int ifeti_apply_F_noalloc(ifeti_ctx *ctx, const double *lam, double *out, int nrhs);
/* out = M̊_D^-1 r, the ROM Dirichlet preconditioner of eq. (49). */
int ifeti_apply_MD(ifeti_ctx *ctx, const double *r, double *out, int nrhs);

/* Per-cell view of a displacement in the layout of eq. (13): out[rhs][s][e] for every local dof e of
 * cell s in the cell's own order (control points in lexicographic order, components interleaved):
 * the r entries from u_r^(s), the primal entries from u_P through the cell's primal map, zero at
 * clamped corners.  u: device, nrhs vectors of length nU; out: device, nrhs * N * n_dof doubles.
 * Needs ifeti_build_cells; EINVAL on null or aliased pointers or nrhs < 1. */
int ifeti_cell_displacements(ifeti_ctx *ctx, const double *u, double *out, int nrhs);

/* M̊_D^-ROM of eq. (47) (Sec. 3.2.3): out = sum_s D B_d^(s) S̃_dd^(s) B_d^(s)T D r with
 * S̃_dd^(s) = K_dd - K_di K̊_ii^-ROM K_id, where K̊_ii^-ROM w = R (Rᵀ K_ii^(s) R)^-1 Rᵀ w and
 * R = [K_ii^(σk)-1 w]_k is the reduced solve of eq. (46) on the interior block.  r and out: device,
 * nrhs contiguous vectors of length L.  The principal interior inverses K_ii^(σk)-1 (K n_r^2 doubles,
 * zero-padded) are built on the first call after ifeti_build_reduced_basis and kept.  Positively
 * homogeneous, not linear (the projection space depends on r).  EINVAL before the reduced basis. */
int ifeti_apply_MD_rom(ifeti_ctx *ctx, const double *r, double *out, int nrhs);
/* z = Ů v (Algorithm 3), v dev nU x nrhs, z dev L x nrhs. */
int ifeti_apply_U(ifeti_ctx *ctx, const double *v, double *z, int nrhs);
/* x = Ůᵀ y, y dev L x nrhs, x dev nU x nrhs. */
int ifeti_apply_Ut(ifeti_ctx *ctx, const double *y, double *x, int nrhs);
/* x = K̊^-ROM v (eq. (45), Algorithm 2, reduced local solves eq. (46)). */
int ifeti_apply_Kinv_rom(ifeti_ctx *ctx, const double *v, double *x, int nrhs);
/* y = [[K, B^T], [B, 0]] x, the true saddle operator of eq. (16);
 * x, y dev (nU + L) x nrhs with u first then lambda for each rhs. */
int ifeti_apply_A(ifeti_ctx *ctx, const double *x, double *y, int nrhs);

/* Interface problem F̊ lam = rhs by PCG preconditioned with M̊_D^-1
 * (Sec. 3.2.3), lam_0 = 0, stop when ||r_k||/||r_0|| <= tol for every rhs.
 * iters_out/relres_out host arrays of nrhs (nullable).  EMAXIT keeps the
 * last iterate; EBREAKDOWN if p^T F̊ p <= 0 or non-finite. */
int ifeti_solve_interface(ifeti_ctx *ctx, const double *rhs, double *lam, int nrhs,
                          double tol, int maxit, int *iters_out, double *relres_out);

/* x = K̊^-ROM v - Ůᵀ y: the recovery step of Algorithm 1. */
int ifeti_recover_displacement(ifeti_ctx *ctx, const double *v, const double *y, double *u, int nrhs);

/* Solve (16) by right-preconditioned flexible GMRES with the block
 * preconditioner (44) (Algorithm 1), x_0 = 0, until ||b - A x|| <= tol ||b||
 * for every rhs.  f dev nU x nrhs, d dev L x nrhs, u dev nU x nrhs,
 * lam dev L x nrhs.  inner_tol: relative tolerance of the interface PCG.
 * outer_iters/inner_iters_total/relres host arrays of nrhs (nullable). */
int ifeti_solve(ifeti_ctx *ctx, const double *f, const double *d, double *u, double *lam, int nrhs,
                double tol, int maxit, double inner_tol, int *outer_iters, int *inner_iters_total,
                double *relres);

/* Differentiation form.  Compliance c = f^T u and its gradient with respect
 * to every cell's strut width, dc/dw_s = -u_s^T (dK^(s)/dw_s) u_s (the system
 * (16) is self-adjoint and f does not depend on the widths), evaluated by
 * quadrature of the width derivative of eq. (52).  Needs a smoothed strut
 * indicator (smooth_eps > 0): with the sharp one the derivative vanishes almost
 * everywhere and the call returns IFETI_EINVAL.
 *   f, u        dev nU x nrhs (u: a converged solution of ifeti_solve)
 *   grad        dev N x nrhs (rhs-major)
 *   compliance  host nrhs, nullable. */
int ifeti_compliance_grad(ifeti_ctx *ctx, const double *f, const double *u, double *grad,
                          double *compliance, int nrhs);

/* Replace the strut widths (dev N) and re-assemble the cells (snapshots and
 * stiffness) while keeping the reduced basis, coefficients and coarse inverse
 * of the last ifeti_build_reduced_basis: the preconditioner is then that of the
 * previous widths, the outer iteration uses the new operator, so ifeti_solve
 * converges to the solution for the new widths.  EINVAL on a non-positive width. */
int ifeti_update_widths(ifeti_ctx *ctx, const double *widths);

/* ---- Standard (exact) FETI-DP, the paper's comparator (Sec. 2.2.4) ----
 * Factorise every cell's K_rr^(s) (batched blocked Cholesky on the GPU) and keep, per cell, the
 * factor, F_dd = [K_rr^-1]_dd (eq. (27)), the Dirichlet Schur complement S_dd (eq. (30)), the
 * dual rows of U_rp = K_rr^-1 K_rp (eq. (29)), S_pp (eq. (22)) and K_pr; assemble the exact
 * S_PP and build its coarse solver.  Needs ifeti_build_cells (not the reduced basis); device
 * memory grows by N (n_r^2 + 2 n_d^2 + n_p (n_d + n_p + n_r)) doubles plus the coarse solver
 * (c2: 14 GB), and a 6 GB workspace during the call.  ifeti_update_widths invalidates it.
 * ENOTSPD if a cell's K_rr is not positive definite. */
int ifeti_build_exact(ifeti_ctx *ctx);

/* out = F lam, the exact dual operator of eq. (24) (B_R K_RR^-1 B_R^T plus the coarse term with
 * the exact S_PP), lam/out dev L x nrhs. */
int ifeti_exact_apply_F(ifeti_ctx *ctx, const double *lam, double *out, int nrhs);

/* out = M_D^-1 r = sum_s D B_d^(s) S_dd^(s) B_d^(s)T D r, the exact Dirichlet preconditioner
 * (eq. (30)), r/out dev L x nrhs. */
int ifeti_exact_apply_MD(ifeti_ctx *ctx, const double *r, double *out, int nrhs);

/* Standard FETI-DP solve of (16): the right-hand side d̄ of eq. (25), PCG on F with M_D^-1 from
 * lam_0 = 0 to ||r|| <= tol ||d̄||, then u_P by eq. (21) and u_R by eq. (20).
 *   f dev nU x nrhs, d dev L x nrhs, u dev nU x nrhs (eq. (13) order), lam dev L x nrhs;
 *   iters, relres host arrays of nrhs (nullable).  EMAXIT keeps the last iterate. */
int ifeti_exact_solve(ifeti_ctx *ctx, const double *f, const double *d, double *u, double *lam, int nrhs,
                      double tol, int maxit, int *iters, double *relres);

/* Host copies of cell s's exact blocks (any pointer may be NULL): Fdd, Sdd n_d x n_d, Spp
 * n_p x n_p, Ud n_d x n_p (row-major), and the device bytes the exact form holds. */
int ifeti_exact_cell_blocks(ifeti_ctx *ctx, int s, double *Fdd, double *Sdd, double *Spp, double *Ud,
                            long long *device_bytes);

#ifdef __cplusplus
}
#endif
#endif /* IFETI_H */
