// Internal declarations of the ROM-based inexact FETI-DP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <map>
#include <memory>
#include <vector>

#include "ifeti.h"

namespace ifeti {

struct Error {
    int code;
    std::string msg;
};

void set_last_error(const std::string &msg);

#define IFETI_HIP(x)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess)                                                                \
            throw ::ifeti::Error{IFETI_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define IFETI_REQUIRE(cond, code, msg)                                \
    do {                                                              \
        if (!(cond)) throw ::ifeti::Error{(code), std::string(msg)};  \
    } while (0)

// Owned device buffer.
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        if (count == n && p) return;
        release();
        if (count) {
            hipError_t e = hipMalloc(&p, count * sizeof(T));
            if (e != hipSuccess) {
                p = nullptr;
                throw Error{IFETI_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
            }
        }
        n = count;
    }
    // grow-only allocation for work buffers (waits for queued work before freeing)
    void ensure(size_t count, hipStream_t s) {
        if (count <= n && p) return;
        if (p) (void)hipStreamSynchronize(s);
        alloc(count);
    }
    void upload(const std::vector<T> &h, hipStream_t s) {
        alloc(h.size());
        if (n) IFETI_HIP(hipMemcpyAsync(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void zero(hipStream_t s) {
        if (n) IFETI_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s));
    }
    // asynchronous copy to a host vector of size n (the caller synchronises the stream)
    void download(std::vector<T> &h, hipStream_t s) const {
        h.resize(n);
        if (n) IFETI_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
    }
};

// Reference-cell tables (eq. (6)): identical for every cell.
struct RefTables {
    int dim = 0, n_el = 0, p = 0, nc = 0, n_ctrl = 0, n_dof = 0;
    int nq1 = 0, nq = 0, n_elem = 0, nloc = 0, n_off = 0, n_snap = 0;
    std::vector<double> w;        // [E][q] quadrature weight (reference measure)
    std::vector<double> xi;       // [E][q][dim] reference coordinates
    std::vector<double> dN;       // [E][q][l][dim] gradients of the local functions
    std::vector<int> elem_ctrl;   // [E][l] local control point index
    std::vector<double> tab1;     // 1D tables: values [e][g][l], derivatives [e][g][l], weights [e][g]
};

// One group of the principal-combined contraction:
//   Y[:, c] (+)= scale * sum_k coef[cell(c), k] * A_k X[:, c]
struct GemmGroup {
    const double *A = nullptr;  // K blocks, each M x Kd row-major, consecutive
    const double *X = nullptr;  // column c at X + c*ldx, Kd entries
    const double *coef = nullptr;  // [cell*K + k], or null for 1
    int Kd = 0, ldx = 0, K = 1;
    long long xbs = 0;          // stride between right-hand sides (0: ncells*ldx)
    double scale = 1.0;
    // optional fused B_d^T: X is then a multiplier vector (load case stride xbs) and
    // column c = cell s takes entry j from the signed rows gcodes[(s*Kd + j)*2 + u],
    // each multiplied by gw[row] when gw is set (the scaled jump operator)
    const int *gcodes = nullptr;
    const double *gw = nullptr;
};

struct Options {
    int precision = IFETI_FP64;
    int pcg_check_every = 2;
    int fgmres_restart = 60;
    int pcg_maxit = 1000;
    int timing = 0;
    std::string timing_filter;  // empty: time every kernel family; else a comma-separated list
    int timing_every = 1;       // time one launch in this many of each family
    int use_graph = 0;          // replay captured interface-PCG iterations (HIP graph)
    int autotune = 0;           // time the candidate tile shapes on first use of each contraction shape
    int coarse_parts = 0;       // coarse solve: 0 automatic, 1 symmetric-tile inverse, >= 2 that many blocks
    int true_operator = 0;      // K^(s) in (16): 0 stencil values, 1 matrix-free from the pulled-back tensor
    int interface_block = 0;    // Alg. 1 interface block: 0 PCG on (48), 1 one M̊_D^-1 (49), 2 one M̊_D^-ROM (47)
    int overlap_local = 0;      // reduced local solves of (46) on a third stream beside Ů v and the PCG
    int local_iters = 1;        // > 1: K̊^-MPCG, multi-preconditioned CG local solves (Remark 6)
    int md_precision = -1;      // precision of the M̊_D^-1 contraction (49); -1: as `precision`
    int tile_candidate = -1;    // >= 0: force this candidate of every contraction family's tile shapes
    int coarse_approx = 0;      // > 0: block-Jacobi coarse solve with blocks of this many primal dofs
    int block_cg = 0;           // 1: O'Leary block PCG for several load cases of the interface problem
};

// One row of a partitioned coarse-solve phase: out[out] = alpha * M[off .. off+len) . x[xlo .. xlo+len)
struct CoarseRow {
    long long off;
    int xlo, len, out, pad;
};
// up to 16 consecutive rows of one phase that share their input range (stored one after another)
struct CoarseTile {
    int row0, nrows;
};

// Direct solver of an assembled coarse problem S_PP (banded in the lexicographic vertex order).
struct CoarseSolver {
    std::vector<double> h_Sband;  // lower band before factorisation, [i][i-j], width bw+1
    std::vector<double> h_bandL;  // its Cholesky factor in the same band form
    int bw = 0;
    bool inv_ready = false;       // explicit inverse built (on first use by a path that reads it)
    DevBuf<double> SPPinv;        // [nP][nP] explicit inverse
    DevBuf<double> SPPt;          // its lower-triangle 64x64 tiles, tile (I, J), I >= J, at I(I+1)/2 + J, row-major
    DevBuf<int> sym_tiles;        // [tile] -> (I, J)
    DevBuf<double> w_symP;        // [tile][rhs][row partial 64 | column partial 64]
    int nT = 0;
    // partitioned form (interior blocks separated by bandwidth-wide separators): phase 1 the
    // separator right-hand side, phase 2 the separator Schur-complement inverse, phase 3 the interiors
    int cp_p = 0, cp_ns = 0;      // interior blocks (0: not built), separator rows
    DevBuf<double> cp_M1, cp_M2, cp_M3;
    DevBuf<CoarseRow> cp_R1, cp_R2, cp_R3;
    DevBuf<CoarseTile> cp_T1, cp_T2, cp_T3;  // the same rows in tiles (blocks of load cases)
    DevBuf<double> w_cg, w_cw;    // separator rhs [rhs][ns], assembled input [rhs][nP]
    // approximate solve (block Jacobi): the inverse of each diagonal block of B rows, one row per output
    int ap_B = 0;
    DevBuf<double> ap_M;
    DevBuf<CoarseRow> ap_R;
};

// Kernel statistics: algorithmic flops/bytes per launch and, when timing is
// enabled, HIP-event durations recorded on the context stream.
struct KernelStat {
    std::string name;
    long long launches = 0, timed = 0;
    double ms = 0.0, flops = 0.0, bytes = 0.0;
};
struct PendingEvent {
    int id;
    hipEvent_t a, b;
};

void release_blas(void *handle);  // destroys a rocBLAS handle (null: nothing)

}  // namespace ifeti

struct ifeti_ctx {
    // ---- description
    ifeti_lattice_desc desc{};
    int dim = 0, shape[3] = {1, 1, 1}, N = 0;
    hipStream_t stream = nullptr;        // stream work is enqueued on (the caller's, except inside a SideStream)
    hipStream_t side_stream = nullptr;   // second stream for the coarse path
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool side_pending = false;
    int prec_override = -1;              // >= 0: precision of the contractions issued in the current scope
    hipStream_t local_stream = nullptr;  // third stream: reduced local solves beside the interface PCG
    hipEvent_t ev_local_fork = nullptr, ev_local_join = nullptr;
    ifeti::Options opt;
    ifeti::RefTables ref;

    // ---- partition (eq. (12)), host
    int n_i = 0, n_d = 0, n_p = 0, n_r = 0;
    std::vector<int> idx_i, idx_d, idx_p, idx_r;
    long long nnz_rr = 0, nnz_full = 0;  // stencil non-zeros of K_rr and of the full cell matrix
    // ---- multipliers and primal assembly, host + device
    int L = 0, L_int = 0, nP = 0, n_vert_free = 0;
    long long nU = 0;
    ifeti::DevBuf<int> g_gather;     // [(s*n_d + j)*2 + t]: sign*(row+1), 0 none
    ifeti::DevBuf<int> g_scatter;    // [l*2 + t]: sign*(s*n_d + j + 1), 0 none
    ifeti::DevBuf<double> g_Dw;      // [L] multiplicity weights
    ifeti::DevBuf<int> g_Ap;         // [s*n_p + j] global primal dof or -1
    ifeti::DevBuf<int> g_Apc;        // [(s*n_p + j)*2 + t]: A_p as gather codes (t = 0: dof + 1, 0 none; t = 1: 0)
    ifeti::DevBuf<double> g_up_dir;  // [s*n_p + j] u0 at primal corners on a Dirichlet face (0 elsewhere)
    ifeti::DevBuf<int> g_Ppull;      // [P*maxc + t]: s*n_p + j, -1 none
    int maxc = 0;
    std::vector<int> h_Ap;
    std::vector<int> h_sca;          // host copy of g_scatter (Dirichlet rows name their cell dof)
    std::vector<double> h_d;         // Dirichlet data d of (14) (zero on clamped faces)

    // ---- cells (device)
    int nrhs = 0;
    std::vector<double> tractions;
    ifeti::DevBuf<double> ctrl;      // [s][a][dim]
    ifeti::DevBuf<double> widths;    // [s]
    ifeti::DevBuf<double> snap;      // [s][E][q][dim^4] pulled-back tensor (greedy snapshots)
    ifeti::DevBuf<double> Kst;       // [s][o][i][k][a] stencil stiffness values (offset o, comps i,k)
    ifeti::DevBuf<double> f_cells;   // [rhs][s][n_dof]
    ifeti::DevBuf<double> f_vec;     // [rhs][nU]
    ifeti::DevBuf<double> d_vec;     // [rhs][L]
    ifeti::DevBuf<int> r_of_dof;     // [n_dof] r position or -1
    ifeti::DevBuf<int> p_of_dof;     // [n_dof] p position or -1
    ifeti::DevBuf<int> g_tables_ctrl;  // ref elem_ctrl
    ifeti::DevBuf<int> g_idx_r, g_idx_p;  // local dof of each r / p position
    ifeti::DevBuf<double> g_tables_w, g_tables_xi, g_tables_dN, g_tables_1d;
    bool cells_built = false;
    bool snap_valid = false;         // snapshots not yet consumed by a greedy

    // ---- reduced basis (device unless noted)
    int K = 0;
    std::vector<int> sigma;
    std::vector<double> h_alpha, h_pi, h_delta;   // [s*K + k]
    ifeti::DevBuf<double> alpha, pi, delta;
    ifeti::DevBuf<double> Fdd, Sdd;     // [k][n_d][n_d]
    ifeti::DevBuf<double> W;            // [k][n_d][n_p]   T_dr U_rp
    ifeti::DevBuf<double> WT;           // [k][n_p][n_d]
    ifeti::DevBuf<double> UrdT;         // [k][n_d][n_r]
    ifeti::DevBuf<double> Urd;          // [k][n_r][n_d]
    ifeti::DevBuf<double> Urp;          // [k][n_r][n_p]
    ifeti::DevBuf<double> UrpT;         // [k][n_p][n_r]
    ifeti::DevBuf<double> Wc;           // [s][n_p][n_d] per-cell sum_k pi_sk (T_dr U_rp^(k))^T
    ifeti::DevBuf<double> Kinv;         // [n_r][k][n_r]: row r*K + k is row r of K_rr^(sigma_k)^-1
    ifeti::CoarseSolver co;             // S̊_PP of the ROM operators (Sec. 3.2.1)
    // standard (exact) FETI-DP (Sec. 2.2.4): factor of every K_rr^(s) [s][n_r][n_r] (lower,
    // column-major), F_dd and S_dd [s][n_d][n_d], U_d^T [s][n_p][n_d], S_pp [s][n_p][n_p],
    // K_pr [s][n_p][n_r]; the exact S_PP and its solver; work vectors of the exact solve
    bool ex_built = false;
    ifeti::DevBuf<double> ex_L, ex_Fdd, ex_Sdd, ex_C, ex_Spp, ex_Kpr;
    ifeti::CoarseSolver co_ex;
    ifeti::DevBuf<double> ex_w, ex_g, ex_z, ex_d;
    bool rom_built = false;
    bool capturing = false;             // a HIP graph capture is in progress on `stream`
    bool no_alloc = false;              // inside an allocation-free call: anything that would allocate
                                        // (copies, inverses, work buffers, timing events) is an EINVAL
    hipStream_t own_stream = nullptr;   // non-blocking stream of the graph form (default priority)
    void *h_pin = nullptr;              // pinned host staging for convergence reads (hipHostMalloc)
    size_t h_pin_bytes = 0;
    hipEvent_t ev_poll = nullptr;
    // FGMRES storage kept across solves (grow-only, no allocation inside a warm solve): Krylov
    // blocks V_j and Z_j, their device pointer tables (with host mirrors) and work vectors
    std::vector<std::unique_ptr<ifeti::DevBuf<double>>> fg_V, fg_Z;
    ifeti::DevBuf<const double *> fg_dV, fg_dZ;
    std::vector<const double *> fg_hV, fg_hZ;
    ifeti::DevBuf<double> fg_w, fg_coef, fg_tu, fg_tL, fg_tL2, fg_tu2, fg_hdev, fg_hall, fg_scd, fg_xs;
    void *h_poll[2] = {nullptr, nullptr};  // pinned slots of the look-ahead convergence polls
    size_t h_poll_bytes = 0;
    hipEvent_t ev_pollv[2] = {nullptr, nullptr};
    hipGraph_t g_graph = nullptr;       // cached captured PCG iteration and its key / counters
    hipGraphExec_t g_exec = nullptr;
    std::vector<uintptr_t> g_key;
    std::vector<ifeti::KernelStat> g_delta;
    long long g_dap[IFETI_OP_COUNT] = {};
    long long rom_gen = 0;              // bumped whenever the reduced basis / cell data change
    std::map<std::vector<long long>, int> tuned;  // contraction shape -> chosen tile candidate
    hipEvent_t ev_own_in = nullptr, ev_own_out = nullptr;
    struct FragCopy {                   // a bank array in MFMA-fragment order, per (M, Kd, K, element type) view
        const double *src = nullptr;
        int M = 0, Kd = 0, K = 0, kind = 0;  // kind: IFETI_FP64 / IFETI_FP32_LOCAL / IFETI_BF16_LOCAL
        void *frag = nullptr;
    };
    std::vector<FragCopy> frag;
    struct RebasedBank {                // a principal bank in a Frobenius-orthonormal basis (precision form)
        const double *src = nullptr, *coef = nullptr;  // original operators [K][M][Kd] and coefficients [cell][K]
        int M = 0, Kd = 0, K = 0, Kp = 0, ncells = 0;  // Kp: directions kept
        double *bank = nullptr;         // [Kp][M][Kd]
        double *cf = nullptr;           // [cell][Kp]
    };
    std::vector<RebasedBank> rebased;
    // M̊_D^-ROM (47): principal interior inverses K_ii^(σk)-1 zero-padded to n_r x n_r, rows interleaved
    // [r][k][n_r] like the stacked K_rr^-1 (built on first use for the current bank), and work vectors
    ifeti::DevBuf<double> Kii_pad, mdr_X, mdr_Y, mdr_v, mdr_x;
    // K̊^-MPCG: residuals of the local problems and the whitened blocks of each iteration
    ifeti::DevBuf<double> mp_r;
    std::vector<std::unique_ptr<ifeti::DevBuf<double>>> mp_P, mp_KP;
    long long bank_gen = 0, kii_gen = -1;
    void free_copies() {
        ++rom_gen;
        ++bank_gen;
        for (auto &cp : frag)
            if (cp.frag) (void)hipFree(cp.frag);
        frag.clear();
        for (auto &rb : rebased) {
            if (rb.bank) (void)hipFree(rb.bank);
            if (rb.cf) (void)hipFree(rb.cf);
        }
        rebased.clear();
    }
    // drop the fragment-order copies of one source array whose contents are rewritten in place
    // (the copies are keyed by the source pointer); also invalidates a cached graph
    void drop_copies(const void *src) {
        ++rom_gen;
        for (auto &cp : frag)
            if (cp.src == src && cp.frag) {
                (void)hipStreamSynchronize(stream);  // queued work may still read the copy
                (void)hipFree(cp.frag);
                cp.frag = nullptr;
            }
        frag.erase(std::remove_if(frag.begin(), frag.end(), [](const FragCopy &cp) { return !cp.frag; }),
                   frag.end());
    }
    void *blas = nullptr;               // rocBLAS handle of the plain FP64 products (created on first use)
    ~ifeti_ctx() {
        free_copies();
        ifeti::release_blas(blas);
    }

    // ---- statistics
    long long applies[IFETI_OP_COUNT] = {0, 0, 0, 0, 0, 0};
    long long pcg_its = 0, fgmres_its = 0;
    std::vector<ifeti::KernelStat> kstats;
    std::vector<ifeti::PendingEvent> pending;
    std::vector<hipEvent_t> event_pool;

    // ---- work buffers
    ifeti::DevBuf<double> w_Lam, w_Y, w_c, w_zP, w_yP, w_yp, w_R, w_H, w_Yc, w_split, w_x, w_tmpL, w_tmpU;
    ifeti::DevBuf<float> w_R32;          // precision form: R of (46a) in FP32 (the library's narrow product)
    ifeti::DevBuf<unsigned short> w_v16; // the narrow copy of v (FP32 as two halves, or BF16)
    ifeti::DevBuf<double> w_red;        // reduction partials
    ifeti::DevBuf<double> pcg_r, pcg_z, pcg_p, pcg_q, pcg_st, pcg_pa, pcg_pb, pcg_pc;  // interface PCG state
    ifeti::DevBuf<int> pcg_ist;
    ifeti::DevBuf<double> w_scal;       // PCG scalars
    ifeti::DevBuf<double> bcg_part, bcg_G, bcg_C;  // block PCG: Gram partial sums, Gram matrices, coefficients
    ifeti::DevBuf<int> w_iflag;
};

namespace ifeti {
// stats.cpp: RAII timing of one launch (flops/bytes always counted)
// Counts one launch of a kernel family (algorithmic flops / bytes) and, when
// timing is on for that family, brackets it with HIP events.  With
// in_packet = true the launcher passes start() / stop() to
// hipExtLaunchKernelGGL, so the events are stamped by the kernel's own
// dispatch packet (kernel duration without the marker-packet latency).
class Prof {
   public:
    Prof(ifeti_ctx *c, const char *name, double flops, double bytes, bool in_packet = false);
    ~Prof();
    hipEvent_t start() const { return a_; }
    hipEvent_t stop() const { return b_; }

   private:
    ifeti_ctx *c_;
    int id_;
    bool in_packet_ = false;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};
void flush_events(ifeti_ctx *c);
void release_events(ifeti_ctx *c);

// setup_host.cpp
void build_reference_tables(ifeti_ctx *c);
void build_partition(ifeti_ctx *c);
void build_decomposition(ifeti_ctx *c);
void build_loads(ifeti_ctx *c);
bool has_dirichlet_data(const ifeti_ctx *c);  // u0 != 0 on the Dirichlet faces
void build_reduced_basis(ifeti_ctx *c, int n_principal, double tol_rb, const int *principal_in);

// kernels_setup.hip
void launch_pulled_back(ifeti_ctx *c);
void launch_stiffness(ifeti_ctx *c);
int greedy_device(ifeti_ctx *c, int n_principal, double tol_rb, const int *principal_in,
                  std::vector<int> &sigma, std::vector<double> &beta, std::vector<double> &norms);
void coarse_inverse_device(ifeti_ctx *c, CoarseSolver &co, const std::vector<double> &band_L, int bw);
void ensure_coarse_inverse(ifeti_ctx *c, CoarseSolver &co);
// (L L^T)^-1 as a dense row-major n x n host array, from a banded lower factor L[i][i-j] (width bw+1)
std::vector<double> band_inverse_device(ifeti_ctx *c, const std::vector<double> &band_L, int n, int bw);
void build_coarse_partition(ifeti_ctx *c, CoarseSolver &co);
// block-Jacobi approximation of the coarse solve with blocks of opt.coarse_approx rows (0: none)
void build_coarse_approx(ifeti_ctx *c, CoarseSolver &co);
// trace tables Psi [2 npair + K][n_snap] of eq. (42) from the principal K_rr^-1 [k][n_r][n_r] and
// U_rp^T [k][n_p][n_r] on the device
void trace_tables_device(ifeti_ctx *c, int K, const double *Kinv, const double *UqT, double *Psi);
// lower-band Cholesky factor L[i][i-j] of the symmetric band matrix band[i][i-j] (ENOTSPD if not SPD)
std::vector<double> band_cholesky(const std::vector<double> &band, int n, int bw);

// gemm.hip
// eigenpairs of a small symmetric matrix (cyclic Jacobi; A is overwritten): A = V diag(w) V^T, V row-major
void jacobi_eigen(std::vector<double> &A, int n, std::vector<double> &V, std::vector<double> &w);
// fragment-order FP64 copies of the operators the interface operators contract with (built at setup)
void prepare_operator_copies(ifeti_ctx *c);
// Y column c at Y + (c / ncells)*ybs + (c % ncells)*ldy (ybs 0: ncells*ldy; ncells 0: N)
void gemm(ifeti_ctx *c, const GemmGroup *groups, int ngroups, double *Y, int ldy, long long ybs, int M, int ncols,
          bool accumulate, int ncells = 0, const char *tag = "gemm", bool lp_ok = true);
// The plain product Y32 = A X (A M x Kd row-major, column s of load case r at X + r*xbs + s*ldx) with
// narrow operands (kind IFETI_FP32_LOCAL or IFETI_BF16_LOCAL, FP32 accumulation and FP32 result) by the
// library: Y32 column r*ncells + s at Y32 + (r*ncells + s)*M.  False when it does not apply (the caller
// then runs the own kernels).
bool library_gemm_narrow(ifeti_ctx *c, const double *A, int M, int Kd, const double *X, int ldx, long long xbs,
                         int ncells, int nrhs, int kind, float *Y32, const char *tag);

// ops.hip
class SideStream {
   public:
    explicit SideStream(ifeti_ctx *c);
    ~SideStream();

   private:
    ifeti_ctx *c_;
    hipStream_t main_;
};
void join_side(ifeti_ctx *c);
void ensure_work(ifeti_ctx *c, int nrhs);
void op_gather(ifeti_ctx *c, const double *lam, long long lam_rs, double *Lam, int nrhs, bool weights);
void op_scatter(ifeti_ctx *c, const double *Y, int y_ld, int y_off, long long y_rs, double *out, long long out_rs,
                int nrhs, bool weights, const double *dot_w = nullptr, double *dot_part = nullptr,
                const double *Y2 = nullptr);
void op_assemble_primal(ifeti_ctx *c, const double *cp, const double *base, long long b_rs, double sgn, double *zP,
                        long long z_rs, int nrhs);
void op_restrict_primal(ifeti_ctx *c, const double *xP, long long x_rs, double *xp, int nrhs);
// c_s = C_s B_d^(s)T lam (C [s][n_p][n_d], gather fused); Y_s (+)= C_s^T yP[A_p(s)] (Y [col][n_d])
void op_restrict_cells(ifeti_ctx *c, const double *C, const double *lam, long long lam_rs, double *out, int nrhs,
                       const char *tag);
void op_prolong_cells(ifeti_ctx *c, const double *C, const double *yP, long long yP_rs, double *Y, int nrhs,
                      bool accumulate, const char *tag);
void op_coarse_solve(ifeti_ctx *c, const double *z, long long z_rs, double *y, long long y_rs, int nrhs,
                     double scale);
// the same with an explicit coarse solver (the exact FETI-DP operators carry their own)
void coarse_solve(ifeti_ctx *c, CoarseSolver &co, const double *z, long long z_rs, double *y, long long y_rs,
                  int nrhs, double scale);
void op_rom_local(ifeti_ctx *c, const double *vR, long long v_rs, double *xR, long long x_rs, int nrhs,
                  const double *bank = nullptr, const char *rtag = "rom_R_gemm");
void apply_MD_rom(ifeti_ctx *c, const double *r, double *out, int nrhs);
void cell_displacements(ifeti_ctx *c, const double *u, double *out, int nrhs);
// y_s = K^(s) x_s for every cell from the stencil values; x, y device [N][n_dof] (setup use)
void cell_matvec_full(ifeti_ctx *c, const double *x, double *y);
// dot_w / dot_part (optional): the final scatter also writes the per-block partial
// sums of out . dot_w, dot_blocks(L) per load case (consumed by the PCG kernels)
void combine_coarse_maps(ifeti_ctx *c);
void release_graph(ifeti_ctx *c);
// copy `bytes` from device memory to pinned host staging on the context stream and wait for it by
// spinning on an event (no blocking stream synchronisation); returns the staging pointer
const void *read_back(ifeti_ctx *c, const void *dev, size_t bytes);
void coarse_reduce(ifeti_ctx *c, const CoarseSolver &co, double *y, long long y_rs, int nrhs, double scale);
void apply_F(ifeti_ctx *c, const double *lam, double *out, int nrhs, const double *dot_w = nullptr,
             double *dot_part = nullptr);
// F̊ lam with explicit work buffers: Y, Yc [N*nrhs][n_d], cb [N*nrhs][n_p], zP, yP [nrhs][nP]
void apply_F_into(ifeti_ctx *c, const double *lam, double *out, int nrhs, double *Y, double *Yc, double *cb,
                  double *zP, double *yP, const double *dot_w, double *dot_part);
void apply_MD(ifeti_ctx *c, const double *r, double *out, int nrhs, const double *dot_w = nullptr,
              double *dot_part = nullptr);
int dot_blocks(long long n);
void apply_U(ifeti_ctx *c, const double *v, double *z, int nrhs);
void apply_Ut(ifeti_ctx *c, const double *y, double *x, int nrhs);
void apply_Kinv_rom(ifeti_ctx *c, const double *v, double *x, int nrhs, bool local_done = false);
void apply_A(ifeti_ctx *c, const double *x, double *y, int nrhs);
// V_i = Vp[i] when a device pointer table is given, else V + i*vstride
void multidot(ifeti_ctx *c, const double *V, long long vstride, int nv, const double *w, long long n, long long rs,
              int nrhs, double *out_dev, const double *const *Vp = nullptr);
// w = a w + cscale * sum_k coef_k V_k (per load case)
void multiaxpy(ifeti_ctx *c, const double *V, long long vstride, int nv, const double *coef_dev, double a, double *w,
               long long n, long long rs, int nrhs, const double *const *Vp = nullptr, double cscale = 1.0);
// w += cscale * V coef (a pointer array of nv <= kAxpyDotMax vectors) and, in the same pass, the dot products of
// the updated w with the nv vectors (norm = false) or with itself (norm = true) into out_dev, equal
// bitwise to multiaxpy followed by multidot; false (nothing done) for more than kAxpyDotMax vectors
constexpr int kAxpyDotMax = 16;
bool axpy_dot(ifeti_ctx *c, int nv, const double *coef_dev, double cscale, double *w, long long n, long long rs,
              int nrhs, const double *const *Vp, bool norm, double *out_dev);
void inv_sqrt(ifeti_ctx *c, const double *h, double *sc, int n);
void scale_copy(ifeti_ctx *c, const double *x, long long n, long long rs, const double *sc_dev, double *y, int nrhs);

// gradient.hip
void compliance_grad(ifeti_ctx *c, const double *f, const double *u, double *grad, double *comp_host, int nrhs);

// solver.hip (exact: the standard FETI-DP operators F and M_D instead of F̊ and M̊_D^-1)
int solve_interface(ifeti_ctx *c, const double *rhs, double *lam, int nrhs, double tol, int maxit, int *iters,
                    double *relres, bool exact = false);

// exact.hip: standard FETI-DP (Sec. 2.2.4) and the batched factorisation it shares with the
// principal bank.  Outputs per list entry k (any may be null except Fq, Spp, UqT, Kpr):
struct FactorOut {
    double *L = nullptr;    // [k][n_r][n_r] Cholesky factor of K_rr (lower, column-major)
    double *Fq = nullptr;   // [k][n_q][n_q] E^T K_rr^-1 E for the selected rows
    double *Sdd = nullptr;  // [k][n_d][n_d] Dirichlet Schur complement (30)
    double *UqT = nullptr;  // [k][n_p][n_q] selected rows of U_rp = K_rr^-1 K_rp, transposed
    double *Spp = nullptr;  // [k][n_p][n_p] S_pp (22)
    double *Kpr = nullptr;  // [k][n_p][n_r]
    double *Kpp = nullptr;  // [k][n_p][n_p] (lower triangle)
};
void factor_cells(ifeti_ctx *c, const int *cells, int ncell, int q_lo, int n_q, const FactorOut &o);
// lower-band Cholesky factor of an SPD band matrix band[i][i-j] computed on the GPU (ENOTSPD if not SPD)
std::vector<double> band_cholesky_device(ifeti_ctx *c, const std::vector<double> &band, int n, int bw);
void build_exact(ifeti_ctx *c);
void apply_F_exact(ifeti_ctx *c, const double *lam, double *out, int nrhs, const double *dot_w = nullptr,
                   double *dot_part = nullptr);
void apply_MD_exact(ifeti_ctx *c, const double *r, double *out, int nrhs, const double *dot_w = nullptr,
                    double *dot_part = nullptr);
int solve_exact(ifeti_ctx *c, const double *f, const double *d, double *u, double *lam, int nrhs, double tol,
                int maxit, int *iters, double *relres);
int solve_fgmres(ifeti_ctx *c, const double *f, const double *d, double *u, double *lam, int nrhs, double tol,
                 int maxit, double inner_tol, int *outer, int *inner_total, double *relres);
}  // namespace ifeti
