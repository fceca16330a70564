// Krylov drivers: interface PCG on F̊ preconditioned by M̊_D^-1 (paper
// Sec. 3.2.3, eqs. (48)-(49)) and right-preconditioned flexible GMRES on the
// saddle system (16) with the block preconditioner (44) (Algorithm 1).
//
// Several load cases run as independent recurrences that share every operator
// application (one batched F̊ / M̊_D^-1 / K̊^-ROM per step); a load case that has
// converged is frozen (zero step length) so each one follows exactly its
// single-load-case iteration.  All PCG scalars live on the device; the host
// only polls the convergence flags every `pcg_check_every` iterations.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "common.hpp"

namespace ifeti {
namespace {

constexpr int kB = 256;
inline unsigned nblocks(long long n) { return (unsigned)((n + kB - 1) / kB); }

// PCG state per load case (doubles): rho, r0, relres, alpha, beta
enum { S_RHO = 0, S_R0, S_REL, S_ALPHA, S_BETA, S_N };
// ints: active, iterations when last active, breakdown, iterations executed (all load cases)
enum { I_ACT = 0, I_IT, I_BRK, I_ITER, I_N };

// Block sum in a fixed order: a butterfly within each wave (lane i adds lane i ^ 32, ^ 16, ..., ^ 1; every
// lane ends with the same bits), then the wave sums in wave order from LDS: one barrier pair instead of
// a barrier per tree level.
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

// partial[rhs*nblk + b] = x . y over block b's chunk
__global__ __launch_bounds__(kB) void k_dot_partial(const double *__restrict__ x, const double *__restrict__ y,
                                                    long long n, long long rs, int nblk, double *__restrict__ part) {
    __shared__ double sh[kB];
    int b = blockIdx.x, rhs = blockIdx.y;
    long long chunk = (n + nblk - 1) / nblk;
    long long i0 = b * chunk, i1 = min(n, i0 + chunk);
    const double *xr = x + rhs * rs, *yr = y + rhs * rs;
    double acc = 0.0;
    for (long long t = i0 + threadIdx.x; t < i1; t += kB) acc += xr[t] * yr[t];
    acc = block_reduce(acc, sh);
    if (threadIdx.x == 0) part[(size_t)rhs * nblk + b] = acc;
}

__device__ inline double sum_partials(const double *part, int nblk, double *sh) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kB) acc += part[b];
    return block_reduce(acc, sh);
}

// two sums of partials through one reduction (the same order per sum as sum_partials, half the
// barriers); both partial sets are loaded before the first addition
__device__ inline void sum_partials2(const double *pa, const double *pb, int nblk, double *sh2, double &a,
                                     double &b) {
    double x = 0.0, y = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kB) {
        const double u = pa[k], v = pb[k];
        x += u;
        y += v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off);
        y += __shfl_xor(y, off);
    }
    constexpr int nw = kB / 64;
    if ((threadIdx.x & 63) == 0) {
        sh2[threadIdx.x >> 6] = x;
        sh2[nw + (threadIdx.x >> 6)] = y;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int w = 0; w < nw; ++w) {
        a += sh2[w];
        b += sh2[nw + w];
    }
    __syncthreads();
}

// stage 0: r0 = ||r||, rho = r.z
__global__ __launch_bounds__(kB) void k_pcg_init(const double *__restrict__ p_rr, const double *__restrict__ p_rz,
                                                 int nblk, double *__restrict__ st, int *__restrict__ ist) {
    __shared__ double sh[kB];
    int rhs = blockIdx.x;
    double rr = sum_partials(p_rr + (size_t)rhs * nblk, nblk, sh);
    double rz = sum_partials(p_rz + (size_t)rhs * nblk, nblk, sh);
    if (threadIdx.x == 0) {
        double r0 = sqrt(rr);
        // a non-finite right-hand side (or preconditioned residual) is a breakdown, not convergence
        const bool bad = !isfinite(rr) || !isfinite(rz);
        st[rhs * S_N + S_RHO] = rz;
        st[rhs * S_N + S_R0] = r0;
        st[rhs * S_N + S_REL] = r0 > 0.0 ? 1.0 : 0.0;
        st[rhs * S_N + S_ALPHA] = 0.0;
        st[rhs * S_N + S_BETA] = 0.0;
        ist[rhs * I_N + I_ACT] = (!bad && r0 > 0.0) ? 1 : 0;
        ist[rhs * I_N + I_IT] = 0;
        ist[rhs * I_N + I_ITER] = 0;
        ist[rhs * I_N + I_BRK] = bad ? 1 : 0;
    }
}

// ---- fused PCG step kernels.  The scalar state is double-buffered: slot 0
// holds the state between iterations, slot 1 the state after the update.
// Every block recomputes the scalars it needs from the partial sums (fixed
// order, so all blocks agree bitwise) and reads only the slot the kernel does
// not write; block (0, rhs) writes the other slot.

// alpha = rho / p.q (breakdown if p.q <= 0 or not finite); lam += alpha p,
// r -= alpha q; partial ||r||^2.  Reads slot 0, writes slot 1.
constexpr int kPre = 2;  // interface-vector entries per thread loaded ahead of the partial sums

__global__ __launch_bounds__(kB) void k_pcg_step(double *__restrict__ lam, double *__restrict__ r,
                                                 const double *__restrict__ p, const double *__restrict__ q,
                                                 long long n, long long rs, int nrhs, double *__restrict__ st,
                                                 int *__restrict__ ist, const double *__restrict__ p_pq, int nblk,
                                                 double *__restrict__ p_rr) {
    __shared__ double sh[kB];
    const int b = blockIdx.x, rhs = blockIdx.y;
    const double *s0 = st + (size_t)rhs * S_N;
    const int *i0s = ist + (size_t)rhs * I_N;
    double *s1 = st + ((size_t)nrhs + rhs) * S_N;
    int *i1s = ist + ((size_t)nrhs + rhs) * I_N;
    const long long chunk = (n + nblk - 1) / nblk;
    const long long j0 = b * chunk, j1 = min(n, j0 + chunk);
    const size_t base = (size_t)rhs * rs;
    // the thread's first kPre entries are loaded before the partial sums are reduced (they do not
    // depend on them), the rest in the loop below; every entry takes the same operations in order
    double pr[kPre], pp[kPre], pqv[kPre], pl[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const long long t = j0 + threadIdx.x + (long long)u * kB;
        const bool in = t < j1;
        pr[u] = in ? r[base + t] : 0.0;
        pp[u] = in ? p[base + t] : 0.0;
        pqv[u] = in ? q[base + t] : 0.0;
        pl[u] = in ? lam[base + t] : 0.0;
    }
    const double pq = sum_partials(p_pq + (size_t)rhs * nblk, nblk, sh);
    int act = i0s[I_ACT], brk = i0s[I_BRK];
    double a = 0.0;
    if (act) {
        if (!(pq > 0.0) || !isfinite(pq)) {
            brk = 1;
            act = 0;
        } else {
            a = s0[S_RHO] / pq;
        }
    }
    if (b == 0 && threadIdx.x == 0) {
        for (int k = 0; k < S_N; ++k) s1[k] = s0[k];
        s1[S_ALPHA] = a;
        i1s[I_ACT] = act;
        i1s[I_IT] = i0s[I_IT];
        i1s[I_ITER] = i0s[I_ITER];
        i1s[I_BRK] = brk;
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const long long t = j0 + threadIdx.x + (long long)u * kB;
        if (t < j1) {
            double rv = pr[u];
            if (a != 0.0) {
                lam[base + t] = pl[u] + a * pp[u];
                rv -= a * pqv[u];
                r[base + t] = rv;
            }
            acc += rv * rv;
        }
    }
    for (long long t = j0 + threadIdx.x + (long long)kPre * kB; t < j1; t += kB) {
        double rv = r[base + t];
        if (a != 0.0) {
            lam[base + t] += a * p[base + t];
            rv -= a * q[base + t];
            r[base + t] = rv;
        }
        acc += rv * rv;
    }
    acc = block_reduce(acc, sh);
    if (threadIdx.x == 0) p_rr[(size_t)rhs * nblk + b] = acc;
}

// relres from ||r||^2 (stop at tol), beta = r.z / rho, p = z + beta p for the
// load cases still active.  Reads slot 1, writes slot 0.
__global__ __launch_bounds__(kB) void k_pcg_next(double *__restrict__ p, const double *__restrict__ z, long long n,
                                                 long long rs, int nrhs, double *__restrict__ st,
                                                 int *__restrict__ ist, const double *__restrict__ p_rr,
                                                 const double *__restrict__ p_rz, int nblk, double tol) {
    __shared__ double sh[2 * kB];
    const int b = blockIdx.x, rhs = blockIdx.y;
    double *s0 = st + (size_t)rhs * S_N;
    int *i0s = ist + (size_t)rhs * I_N;
    const double *s1 = st + ((size_t)nrhs + rhs) * S_N;
    const int *i1s = ist + ((size_t)nrhs + rhs) * I_N;
    const long long chunk = (n + nblk - 1) / nblk;
    const long long j0 = b * chunk, j1 = min(n, j0 + chunk);
    const size_t base = (size_t)rhs * rs;
    double pz[kPre], pp[kPre];  // the thread's first kPre entries, loaded before the partial sums
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const long long t = j0 + threadIdx.x + (long long)u * kB;
        const bool in = t < j1;
        pz[u] = in ? z[base + t] : 0.0;
        pp[u] = in ? p[base + t] : 0.0;
    }
    double rr, rz;
    sum_partials2(p_rr + (size_t)rhs * nblk, p_rz + (size_t)rhs * nblk, nblk, sh, rr, rz);
    const int it = i1s[I_ITER] + 1;  // this iteration's number, kept on the device (graph replays)
    int act = i1s[I_ACT], its = i1s[I_IT];
    double rel = s1[S_REL], rho = s1[S_RHO], beta = 0.0;
    if (act) {
        rel = sqrt(rr) / s1[S_R0];
        its = it;
        if (rel <= tol) act = 0;
    }
    if (act) {
        beta = rz / rho;
        rho = rz;
    }
    if (b == 0 && threadIdx.x == 0) {
        for (int k = 0; k < S_N; ++k) s0[k] = s1[k];
        s0[S_REL] = rel;
        s0[S_RHO] = rho;
        s0[S_BETA] = beta;
        i0s[I_ACT] = act;
        i0s[I_IT] = its;
        i0s[I_ITER] = it;
        i0s[I_BRK] = i1s[I_BRK];
    }
    if (!act) return;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
        const long long t = j0 + threadIdx.x + (long long)u * kB;
        if (t < j1) p[base + t] = pz[u] + beta * pp[u];
    }
    for (long long t = j0 + threadIdx.x + (long long)kPre * kB; t < j1; t += kB)
        p[base + t] = z[base + t] + beta * p[base + t];
}

__global__ __launch_bounds__(kB) void k_copy(const double *__restrict__ x, double *__restrict__ y, long long n) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = x[t];
}

__global__ __launch_bounds__(kB) void k_fill(double *__restrict__ y, long long n, double v) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) y[t] = v;
}

// out[rhs*n + i] = in1 segment followed by in2 segment (saddle vector packing)
__global__ __launch_bounds__(kB) void k_pack(const double *__restrict__ a, long long na,
                                             const double *__restrict__ b, long long nb, double *__restrict__ out,
                                             int nrhs) {
    long long n = na + nb;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    int rhs = (int)(t / n);
    long long i = t % n;
    out[t] = i < na ? a[rhs * na + i] : b[rhs * nb + (i - na)];
}

__global__ __launch_bounds__(kB) void k_unpack(const double *__restrict__ x, long long na, long long nb,
                                               double *__restrict__ a, double *__restrict__ b, int nrhs) {
    long long n = na + nb;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    int rhs = (int)(t / n);
    long long i = t % n;
    if (i < na)
        a[rhs * na + i] = x[t];
    else
        b[rhs * nb + (i - na)] = x[t];
}

// x = a - b (per element) on a strided sub-vector set
__global__ __launch_bounds__(kB) void k_sub(const double *__restrict__ a, long long a_rs, const double *__restrict__ b,
                                            long long b_rs, double *__restrict__ out, long long o_rs, long long n,
                                            int nrhs, double sb) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    int rhs = (int)(t / n);
    long long i = t % n;
    out[rhs * o_rs + i] = a[rhs * a_rs + i] + sb * b[rhs * b_rs + i];
}

// ---- block PCG (O'Leary), breakdown-free form: tall-skinny Gram matrices and block combinations.
// Gram G = U^T V of a <= 32 and b <= 32 columns (column i of U at U + i*urs): one workgroup per chunk of
// kGramRows rows stages the chunk of every column in LDS (rows padded by one against bank conflicts)
// and writes its a x b partial sums; k_gram_reduce adds the chunks in order (bitwise repeatable).
constexpr int kGramRows = 256;
constexpr int kGramStride = kGramRows + 1;
constexpr int kBlockMax = 32;

__global__ __launch_bounds__(kB) void k_gram_partial(const double *__restrict__ U, long long urs, int a,
                                                     const double *__restrict__ V, long long vrs, int b, long long n,
                                                     double *__restrict__ part) {
    extern __shared__ double gsh[];  // (a + b) x kGramStride
    const long long r0 = (long long)blockIdx.x * kGramRows;
    const int rows = (int)min((long long)kGramRows, n - r0);
    for (int e = threadIdx.x; e < (a + b) * kGramRows; e += kB) {
        const int col = e / kGramRows, r = e % kGramRows;
        double v = 0.0;
        if (r < rows) v = col < a ? U[col * urs + r0 + r] : V[(col - a) * vrs + r0 + r];
        gsh[col * kGramStride + r] = v;
    }
    __syncthreads();
    // 2 x 2 blocks of (i, j) per thread
    const int ai = (a + 1) / 2, bj = (b + 1) / 2;
    for (int t = threadIdx.x; t < ai * bj; t += kB) {
        const int i = 2 * (t / bj), j = 2 * (t % bj);
        const double *u0 = gsh + i * kGramStride, *u1 = gsh + min(i + 1, a - 1) * kGramStride;
        const double *v0 = gsh + (a + j) * kGramStride, *v1 = gsh + (a + min(j + 1, b - 1)) * kGramStride;
        double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
        for (int r = 0; r < kGramRows; ++r) {
            const double x0 = u0[r], x1 = u1[r], y0 = v0[r], y1 = v1[r];
            s00 += x0 * y0;
            s01 += x0 * y1;
            s10 += x1 * y0;
            s11 += x1 * y1;
        }
        double *p = part + (size_t)blockIdx.x * a * b;
        p[i * b + j] = s00;
        if (j + 1 < b) p[i * b + j + 1] = s01;
        if (i + 1 < a) p[(i + 1) * b + j] = s10;
        if (i + 1 < a && j + 1 < b) p[(i + 1) * b + j + 1] = s11;
    }
}

__global__ __launch_bounds__(kB) void k_gram_reduce(const double *__restrict__ part, int nchunk, int ab,
                                                    double *__restrict__ G) {
    const int t = blockIdx.x * kB + threadIdx.x;
    if (t >= ab) return;
    double s = 0.0;
    for (int k = 0; k < nchunk; ++k) s += part[(size_t)k * ab + t];
    G[t] = s;
}

// Y_j = alpha Y_j + sum_i C[i][j] X_i for j < b (row-parallel; C is a x b row-major, staged in LDS)
__global__ __launch_bounds__(kB) void k_block_combine(double *__restrict__ Y, long long yrs, int b, double alpha,
                                                      const double *__restrict__ X, long long xrs, int a,
                                                      const double *__restrict__ Cm, long long n) {
    __shared__ double cs[kBlockMax * kBlockMax];
    for (int e = threadIdx.x; e < a * b; e += kB) cs[e] = Cm[e];
    __syncthreads();
    const long long l = (long long)blockIdx.x * kB + threadIdx.x;
    if (l >= n) return;
    double x[kBlockMax];
#pragma unroll
    for (int i = 0; i < kBlockMax; ++i) x[i] = i < a ? X[i * xrs + l] : 0.0;
    for (int j = 0; j < b; ++j) {
        double v = alpha == 0.0 ? 0.0 : alpha * Y[j * yrs + l];
#pragma unroll
        for (int i = 0; i < kBlockMax; ++i)
            if (i < a) v += cs[i * b + j] * x[i];
        Y[j * yrs + l] = v;
    }
}

// One captured PCG iteration (both streams, joined through the fork/join events), instantiated
// and kept in the context while its key (every buffer the iteration touches, load cases,
// tolerance, precision, reduced-basis generation) is unchanged; the statistics of the
// captured iteration are re-applied per replay.
struct GraphIteration {
    static void release(ifeti_ctx *c) {
        if (c->g_exec) (void)hipGraphExecDestroy(c->g_exec);
        if (c->g_graph) (void)hipGraphDestroy(c->g_graph);
        c->g_exec = nullptr;
        c->g_graph = nullptr;
        c->g_key.clear();
        c->g_delta.clear();
    }
    template <typename F>
    static void capture(ifeti_ctx *c, const std::vector<uintptr_t> &key, F &&body) {
        release(c);
        std::vector<KernelStat> ks0 = c->kstats;
        long long ap0[IFETI_OP_COUNT];
        for (int i = 0; i < IFETI_OP_COUNT; ++i) ap0[i] = c->applies[i];
        IFETI_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        c->capturing = true;
        try {
            body();
        } catch (...) {
            c->capturing = false;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(c->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        c->capturing = false;
        IFETI_HIP(hipStreamEndCapture(c->stream, &c->g_graph));
        IFETI_HIP(hipGraphInstantiate(&c->g_exec, c->g_graph, nullptr, nullptr, 0));
        // nothing ran during the capture: keep the per-iteration increments, restore the counters
        for (size_t i = 0; i < c->kstats.size(); ++i) {
            KernelStat d = c->kstats[i];
            if (i < ks0.size()) {
                d.launches -= ks0[i].launches;
                d.flops -= ks0[i].flops;
                d.bytes -= ks0[i].bytes;
                c->kstats[i] = ks0[i];
            } else {
                c->kstats[i].launches = 0;
                c->kstats[i].flops = c->kstats[i].bytes = 0.0;
            }
            c->g_delta.push_back(d);
        }
        for (int i = 0; i < IFETI_OP_COUNT; ++i) {
            c->g_dap[i] = c->applies[i] - ap0[i];
            c->applies[i] = ap0[i];
        }
        c->g_key = key;
    }
    static void launch(ifeti_ctx *c) {
        IFETI_HIP(hipGraphLaunch(c->g_exec, c->stream));
        for (size_t i = 0; i < c->g_delta.size() && i < c->kstats.size(); ++i) {
            c->kstats[i].launches += c->g_delta[i].launches;
            c->kstats[i].flops += c->g_delta[i].flops;
            c->kstats[i].bytes += c->g_delta[i].bytes;
        }
        for (int i = 0; i < IFETI_OP_COUNT; ++i) c->applies[i] += c->g_dap[i];
    }
};

}  // namespace

// ------------------------------------------------------------------ interface PCG
// One iteration = F̊ p (its final scatter also yields the p.q partials),
// k_pcg_step, M̊_D^-1 r (its scatter yields the r.z partials), k_pcg_next.
// Runs the enclosed work on the context's own non-blocking stream (capturable, unlike a caller's
// legacy default stream), ordered after and before the caller's stream by events.
class OwnStream {
   public:
    OwnStream(ifeti_ctx *c, bool on) : c_(c), caller_(c->stream), on_(on) {
        if (!on_) return;
        if (!c->own_stream) {
            IFETI_HIP(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
            IFETI_HIP(hipEventCreateWithFlags(&c->ev_own_in, hipEventDisableTiming));
            IFETI_HIP(hipEventCreateWithFlags(&c->ev_own_out, hipEventDisableTiming));
        }
        IFETI_HIP(hipEventRecord(c->ev_own_in, caller_));
        IFETI_HIP(hipStreamWaitEvent(c->own_stream, c->ev_own_in, 0));
        c->stream = c->own_stream;
    }
    ~OwnStream() {
        if (!on_) return;
        (void)hipEventRecord(c_->ev_own_out, c_->own_stream);
        (void)hipStreamWaitEvent(caller_, c_->ev_own_out, 0);
        c_->stream = caller_;
    }

   private:
    ifeti_ctx *c_;
    hipStream_t caller_;
    bool on_;
};

void release_graph(ifeti_ctx *c) { GraphIteration::release(c); }

// ------------------------------------------------------------------ block PCG (O'Leary)
// The load cases' interface problems F̊ Lam = R_0 solved together in the block Krylov space of all of
// them: Q = F̊ P, alpha = (P^T Q)^-1 P^T R, Lam += P alpha, R -= Q alpha, Z = M̊_D^-1 R,
// beta = -(P^T Q)^-1 Q^T Z, P = orth(Z + P beta).  Breakdown-free form: orth() takes the eigenvectors of
// the Gram matrix of Z + P beta and drops directions of relative eigenvalue <= 1e-12, so linearly
// dependent load cases (the c4 tractions span two directions) cost no operator columns.  The k x k
// algebra runs on the host from the Gram matrices (three reads per iteration).
static void gram(ifeti_ctx *c, const double *U, long long urs, int a, const double *V, long long vrs, int b,
                 long long n, double *G) {
    const int nchunk = (int)((n + kGramRows - 1) / kGramRows);
    c->bcg_part.ensure((size_t)nchunk * a * b, c->stream);
    const size_t lds = (size_t)(a + b) * kGramStride * sizeof(double);
    IFETI_HIP(hipFuncSetAttribute((const void *)k_gram_partial, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
    Prof prof(c, "bcg_gram", 2.0 * a * b * (double)n, 8.0 * (a + b) * (double)n);
    hipLaunchKernelGGL(k_gram_partial, dim3(nchunk), dim3(kB), lds, c->stream, U, urs, a, V, vrs, b, n,
                       c->bcg_part.p);
    hipLaunchKernelGGL(k_gram_reduce, dim3((a * b + kB - 1) / kB), dim3(kB), 0, c->stream, c->bcg_part.p, nchunk,
                       a * b, G);
    IFETI_HIP(hipGetLastError());
}

static void combine(ifeti_ctx *c, double *Y, long long yrs, int b, double alpha, const double *X, long long xrs,
                    int a, const std::vector<double> &Cm, long long n) {
    if (b == 0) return;
    IFETI_HIP(hipMemcpyAsync(c->bcg_C.p, Cm.data(), Cm.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    Prof prof(c, "bcg_combine", 2.0 * a * b * (double)n, 8.0 * (a + b + (alpha != 0.0 ? b : 0)) * (double)n);
    hipLaunchKernelGGL(k_block_combine, dim3(nblocks(n)), dim3(kB), 0, c->stream, Y, yrs, b, alpha, X, xrs, a,
                       c->bcg_C.p, n);
    IFETI_HIP(hipGetLastError());
}

// X = G^-1 B (G k x k symmetric, B k x s) through the eigenpairs of G; false if G is not positive definite
static bool spd_solve_eig(std::vector<double> G, int k, const std::vector<double> &B, int s, std::vector<double> &X) {
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) G[(size_t)i * k + j] = G[(size_t)j * k + i] = 0.5 * (G[(size_t)i * k + j] + G[(size_t)j * k + i]);
    for (double v : G)
        if (!std::isfinite(v)) return false;
    std::vector<double> V, w;
    jacobi_eigen(G, k, V, w);
    double wmax = 0.0;
    for (double x : w) wmax = std::max(wmax, x);
    for (double x : w)
        if (!(x > 1e-14 * wmax)) return false;
    X.assign((size_t)k * s, 0.0);
    for (int m = 0; m < k; ++m)
        for (int j = 0; j < s; ++j) {
            double t = 0.0;
            for (int i = 0; i < k; ++i) t += V[(size_t)i * k + m] * B[(size_t)i * s + j];
            t /= w[m];
            for (int i = 0; i < k; ++i) X[(size_t)i * s + j] += V[(size_t)i * k + m] * t;
        }
    return true;
}

static int solve_interface_block(ifeti_ctx *c, const double *rhs, double *lam, int s, double tol, int maxit,
                                 int *iters, double *relres) {
    IFETI_REQUIRE(s <= kBlockMax, IFETI_EINVAL, "block PCG takes at most 32 load cases");
    const long long L = c->L, n = L * s;
    hipStream_t st = c->stream;
    c->pcg_r.ensure(n, st);
    c->pcg_z.ensure(n, st);
    c->pcg_p.ensure(n, st);
    c->pcg_q.ensure(n, st);
    c->bcg_G.ensure(5 * kBlockMax * kBlockMax, st);
    c->bcg_C.ensure(kBlockMax * kBlockMax, st);
    double *R = c->pcg_r.p, *Z = c->pcg_z.p, *P = c->pcg_p.p, *Q = c->pcg_q.p, *G = c->bcg_G.p;
    double *G1 = G, *G2 = G + 1024, *Grr = G + 2048, *G3 = G + 3072, *G4 = G + 4096;
    hipLaunchKernelGGL(k_copy, dim3(nblocks(n)), dim3(kB), 0, st, rhs, R, n);
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kB), 0, st, lam, n, 0.0);
    auto fetch = [&](const double *dev, size_t count) {
        const double *h = (const double *)read_back(c, dev, count * sizeof(double));
        return std::vector<double>(h, h + count);
    };
    gram(c, R, L, s, R, L, s, L, Grr);
    std::vector<double> nb(s);
    {
        const auto g = fetch(Grr, (size_t)s * s);
        for (int j = 0; j < s; ++j) nb[j] = std::sqrt(std::max(g[(size_t)j * s + j], 0.0));
    }
    for (double v : nb)
        if (!std::isfinite(v)) {
            set_last_error("PCG breakdown: non-finite right-hand side");
            return IFETI_EBREAKDOWN;
        }
    std::vector<double> rel(s, 0.0);
    for (int j = 0; j < s; ++j) rel[j] = nb[j] > 0.0 ? 1.0 : 0.0;
    // P = orth(W) from the Gram matrix of W (s columns at W) scaled to unit column norms (zero columns
    // stay zero), so that only linear dependence drops a direction: the new block's coefficients T (s x k)
    auto orth = [&](const double *W) {
        gram(c, W, L, s, W, L, s, L, G4);
        std::vector<double> g4 = fetch(G4, (size_t)s * s), V, w, D(s);
        for (int i = 0; i < s; ++i) {
            const double dg = g4[(size_t)i * s + i];
            D[i] = dg > 0.0 && std::isfinite(dg) ? 1.0 / std::sqrt(dg) : 0.0;
        }
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) g4[(size_t)i * s + j] *= D[i] * D[j];
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < i; ++j)
                g4[(size_t)i * s + j] = g4[(size_t)j * s + i] = 0.5 * (g4[(size_t)i * s + j] + g4[(size_t)j * s + i]);
        jacobi_eigen(g4, s, V, w);
        double wmax = 0.0;
        for (double x : w) wmax = std::max(wmax, x);
        std::vector<int> keep;
        for (int m = 0; m < s; ++m)
            if (w[m] > 1e-12 * wmax && std::isfinite(w[m])) keep.push_back(m);
        const int k = (int)keep.size();
        std::vector<double> T((size_t)s * k);
        for (int i = 0; i < s; ++i)
            for (int m = 0; m < k; ++m)
                T[(size_t)i * k + m] = D[i] * V[(size_t)i * s + keep[m]] / std::sqrt(w[keep[m]]);
        combine(c, P, L, k, 0.0, W, L, s, T, L);
        return k;
    };
    int it = 0, status = IFETI_OK;
    bool done = *std::max_element(nb.begin(), nb.end()) == 0.0;
    int k = 0;
    if (!done) {
        apply_MD(c, R, Z, s);
        k = orth(Z);
    }
    while (!done && k > 0 && it < maxit) {
        apply_F(c, P, Q, k);                                   // Q = F̊ P
        gram(c, P, L, k, Q, L, k, L, G1);                      // P^T Q
        gram(c, P, L, k, R, L, s, L, G2);                      // P^T R
        const std::vector<double> g12 = fetch(G1, 2048);  // P^T Q and P^T R in one read
        const std::vector<double> g1(g12.begin(), g12.begin() + (size_t)k * k);
        const std::vector<double> g2(g12.begin() + 1024, g12.begin() + 1024 + (size_t)k * s);
        std::vector<double> alpha, beta;
        if (!spd_solve_eig(g1, k, g2, s, alpha)) {
            set_last_error("PCG breakdown: P^T F P not positive definite or non-finite");
            status = IFETI_EBREAKDOWN;
            break;
        }
        combine(c, lam, L, s, 1.0, P, L, k, alpha, L);         // Lam += P alpha
        std::vector<double> malpha(alpha);
        for (double &v : malpha) v = -v;
        combine(c, R, L, s, 1.0, Q, L, k, malpha, L);          // R -= Q alpha
        ++it;
        apply_MD(c, R, Z, s);                                   // Z = M̊_D^-1 R
        gram(c, R, L, s, R, L, s, L, Grr);                      // R^T R (convergence)
        gram(c, Q, L, k, Z, L, s, L, G3);                       // Q^T Z
        const std::vector<double> g33 = fetch(Grr, 2048);  // R^T R and Q^T Z in one read
        {
            const auto &g = g33;
            done = true;
            for (int j = 0; j < s; ++j) {
                rel[j] = nb[j] > 0.0 ? std::sqrt(std::max(g[(size_t)j * s + j], 0.0)) / nb[j] : 0.0;
                done = done && rel[j] <= tol;
            }
        }
        if (done) break;
        const std::vector<double> g3(g33.begin() + 1024, g33.begin() + 1024 + (size_t)k * s);
        if (!spd_solve_eig(g1, k, g3, s, beta)) {
            set_last_error("PCG breakdown: P^T F P not positive definite or non-finite");
            status = IFETI_EBREAKDOWN;
            break;
        }
        for (double &v : beta) v = -v;
        combine(c, Z, L, s, 1.0, P, L, k, beta, L);            // W = Z + P beta (in Z)
        k = orth(Z);                                            // P = orth(W)
    }
    int live = 0;
    for (int j = 0; j < s; ++j) {
        live += nb[j] > 0.0 ? 1 : 0;
        if (iters) iters[j] = nb[j] > 0.0 ? it : 0;
        if (relres) relres[j] = rel[j];
    }
    c->pcg_its += (long long)it * live;
    if (status != IFETI_OK) return status;
    if (!done) {
        set_last_error("PCG reached the iteration limit");
        return IFETI_EMAXIT;
    }
    return IFETI_OK;
}

int solve_interface(ifeti_ctx *c, const double *rhs, double *lam, int nrhs, double tol, int maxit, int *iters,
                    double *relres, bool exact) {
    if (c->opt.block_cg && nrhs > 1 && !exact) return solve_interface_block(c, rhs, lam, nrhs, tol, maxit, iters, relres);
    auto opF = exact ? apply_F_exact : apply_F;
    auto opMD = exact ? apply_MD_exact : apply_MD;
    OwnStream own(c, c->opt.use_graph != 0);
    const long long L = c->L;
    const long long n = L * nrhs;
    hipStream_t s = c->stream;
    const int nblk = dot_blocks(L);
    c->pcg_r.ensure(n, s);
    c->pcg_z.ensure(n, s);
    c->pcg_p.ensure(n, s);
    c->pcg_q.ensure(n, s);
    c->pcg_st.ensure((size_t)2 * S_N * nrhs, s);
    c->pcg_ist.ensure((size_t)2 * I_N * nrhs, s);
    c->pcg_pa.ensure((size_t)nblk * nrhs, s);
    c->pcg_pb.ensure((size_t)nblk * nrhs, s);
    c->pcg_pc.ensure((size_t)nblk * nrhs, s);
    double *r = c->pcg_r.p, *z = c->pcg_z.p, *p = c->pcg_p.p, *q = c->pcg_q.p, *st = c->pcg_st.p;
    double *pa = c->pcg_pa.p, *pb = c->pcg_pb.p, *pc = c->pcg_pc.p;
    int *ist = c->pcg_ist.p;
    hipLaunchKernelGGL(k_copy, dim3(nblocks(n)), dim3(kB), 0, s, rhs, r, n);
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kB), 0, s, lam, n, 0.0);
    opMD(c, r, z, nrhs, r, pb);                                       // z = M r, partials of r.z
    hipLaunchKernelGGL(k_dot_partial, dim3(nblk, nrhs), dim3(kB), 0, s, r, r, L, L, nblk, pa);
    hipLaunchKernelGGL(k_pcg_init, dim3(nrhs), dim3(kB), 0, s, pa, pb, nblk, st, ist);
    hipLaunchKernelGGL(k_copy, dim3(nblocks(n)), dim3(kB), 0, s, z, p, n);
    IFETI_HIP(hipGetLastError());
    std::vector<int> hist((size_t)I_N * nrhs);
    auto any_active = [&]() {  // slot 0 holds the state between iterations
        const int *hp = (const int *)read_back(c, ist, hist.size() * sizeof(int));
        std::copy(hp, hp + hist.size(), hist.begin());
        bool act = false, brk = false;
        for (int r2 = 0; r2 < nrhs; ++r2) {
            act |= hist[r2 * I_N + I_ACT] != 0;
            brk |= hist[r2 * I_N + I_BRK] != 0;
        }
        return std::make_pair(act, brk);
    };
    auto st0 = any_active();
    const int every = std::max(1, c->opt.pcg_check_every);
    const double Ld = (double)L * nrhs;
    auto iteration = [&]() {
        opF(c, p, q, nrhs, p, pa);                                    // q = F p, partials of p.q
        {
            Prof prof(c, "pcg_step", 5.0 * Ld, 48.0 * Ld);            // read lam, p, q, r; write lam, r
            hipLaunchKernelGGL(k_pcg_step, dim3(nblk, nrhs), dim3(kB), 0, s, lam, r, p, q, L, L, nrhs, st, ist, pa,
                               nblk, pb);
        }
        opMD(c, r, z, nrhs, r, pc);                                   // z = M r, partials of r.z
        {
            Prof prof(c, "pcg_next", 2.0 * Ld, 24.0 * Ld);
            hipLaunchKernelGGL(k_pcg_next, dim3(nblk, nrhs), dim3(kB), 0, s, p, z, L, L, nrhs, st, ist, pb, pc,
                               nblk, tol);
        }
        IFETI_HIP(hipGetLastError());
    };
    // Graph form: with a cached graph of this exact configuration every iteration is a replay;
    // otherwise the first iteration runs eagerly (work buffers and operator copies exist
    // afterwards) and the second is captured.
    std::vector<uintptr_t> key;
    if (c->opt.use_graph) {
        const void *bufs[] = {lam, r, z, p, q, st, ist, pa, pb, pc, c->w_Y.p, c->w_Yc.p, c->w_c.p, c->w_zP.p,
                              c->w_yP.p, c->co.w_symP.p, c->w_split.p, c->w_Lam.p, c->side_stream, c->stream};
        for (const void *b : bufs) key.push_back((uintptr_t)b);
        for (long long v : {(long long)nrhs, (long long)c->opt.precision, (long long)c->opt.md_precision, c->rom_gen,
                            (long long)nblk,
                            (long long)exact})
            key.push_back((uintptr_t)v);
        double tv = tol;
        uintptr_t tb = 0;
        std::memcpy(&tb, &tv, sizeof(tv));
        key.push_back(tb);
    }
    // Convergence polls with look-ahead: the poll after chunk k (every `every` iterations) is read
    // while chunk k+1 already runs, unless the residual trend of the last two polls predicts the
    // end within the next two chunks, in which case it is read at once.  Iterations after a load
    // case has converged leave its state unchanged, so a look-ahead chunk changes no result.
    const size_t ib = hist.size() * sizeof(int), sb = (size_t)S_N * nrhs * sizeof(double);
    const size_t soff = (ib + 15) / 16 * 16;
    if (soff + sb > c->h_poll_bytes) {
        IFETI_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < 2; ++i) {
            if (c->h_poll[i]) (void)hipHostFree(c->h_poll[i]);
            c->h_poll[i] = nullptr;
        }
        c->h_poll_bytes = 0;
        const size_t want = std::max<size_t>(soff + sb, 1 << 12);
        for (int i = 0; i < 2; ++i) IFETI_HIP(hipHostMalloc(&c->h_poll[i], want, hipHostMallocDefault));
        c->h_poll_bytes = want;
    }
    for (int i = 0; i < 2; ++i)
        if (!c->ev_pollv[i]) IFETI_HIP(hipEventCreateWithFlags(&c->ev_pollv[i], hipEventDisableTiming));
    auto poll_issue = [&](int slot) {
        IFETI_HIP(hipMemcpyAsync(c->h_poll[slot], ist, ib, hipMemcpyDeviceToHost, s));
        IFETI_HIP(hipMemcpyAsync((char *)c->h_poll[slot] + soff, st, sb, hipMemcpyDeviceToHost, s));
        IFETI_HIP(hipEventRecord(c->ev_pollv[slot], s));
    };
    struct Poll {
        bool act, brk;
        int it;
        double rel;  // largest relative residual over the active load cases
    };
    auto poll_wait = [&](int slot, int it) {
        for (;;) {
            const hipError_t e = hipEventQuery(c->ev_pollv[slot]);
            if (e == hipSuccess) break;
            if (e != hipErrorNotReady) IFETI_HIP(e);
        }
        const int *hi = (const int *)c->h_poll[slot];
        const double *hs = (const double *)((const char *)c->h_poll[slot] + soff);
        Poll P{false, false, it, 0.0};
        for (int r2 = 0; r2 < nrhs; ++r2) {
            const bool a = hi[r2 * I_N + I_ACT] != 0;
            P.act |= a;
            P.brk |= hi[r2 * I_N + I_BRK] != 0;
            if (a) P.rel = std::max(P.rel, hs[r2 * S_N + S_REL]);
        }
        return P;
    };
    Poll prev{true, false, 0, 1.0}, last{true, false, 0, 1.0};
    int pending = -1, pending_it = 0, slot = 0;
    auto near_end = [&]() {  // iterations left predicted from the last two polls
        if (last.it <= prev.it || !(last.rel > 0.0) || !(prev.rel > last.rel)) return true;
        const double rate = std::log(prev.rel / last.rel) / (last.it - prev.it);
        const double left = std::log(last.rel / tol) / rate;
        return left <= 2.0 * every;
    };
    for (int it = 1; it <= maxit && st0.first && !st0.second; ++it) {
        if (c->opt.use_graph && (c->g_exec && c->g_key == key)) {
            GraphIteration::launch(c);
        } else if (c->opt.use_graph && it >= 2) {
            GraphIteration::capture(c, key, iteration);
            GraphIteration::launch(c);
        } else {
            iteration();
        }
        if (it % every == 0 || it == maxit) {
            poll_issue(slot);
            if (pending >= 0) {  // the previous chunk's poll, read while this chunk runs
                prev = last;
                last = poll_wait(pending, pending_it);
                pending = -1;
                if (!last.act || last.brk) {
                    st0 = {last.act, last.brk};
                    break;
                }
            }
            if (near_end() || it == maxit) {
                prev = last;
                last = poll_wait(slot, it);
                st0 = {last.act, last.brk};
            } else {
                pending = slot;
                pending_it = it;
            }
            slot ^= 1;
        }
    }
    // final state: flags, counts and residuals in one pinned read
    poll_issue(slot);
    (void)poll_wait(slot, 0);
    {
        const int *hi = (const int *)c->h_poll[slot];
        const double *hs = (const double *)((const char *)c->h_poll[slot] + soff);
        std::copy(hi, hi + hist.size(), hist.begin());
        st0 = {false, false};
        for (int r2 = 0; r2 < nrhs; ++r2) {
            st0.first |= hist[r2 * I_N + I_ACT] != 0;
            st0.second |= hist[r2 * I_N + I_BRK] != 0;
            c->pcg_its += hist[r2 * I_N + I_IT];
            if (iters) iters[r2] = hist[r2 * I_N + I_IT];
            if (relres) relres[r2] = hs[r2 * S_N + S_REL];
        }
    }
    if (st0.second) {
        set_last_error("PCG breakdown: p^T F p <= 0 or non-finite");
        return IFETI_EBREAKDOWN;
    }
    if (st0.first) {
        set_last_error("PCG reached the iteration limit");
        return IFETI_EMAXIT;
    }
    return IFETI_OK;
}

// ------------------------------------------------------------------ Algorithm 1 / (44)
// x = (v, w) -> (x_u, y):  w̄ = w - Ů v;  y = -F̊^-pcg w̄;  x_u = K̊^-ROM v - Ůᵀ y
// (option interface_block: F̊^-pcg replaced by one application of M̊_D^-1 (49) or M̊_D^-ROM (47))
static int apply_prec(ifeti_ctx *c, const double *in, double *out, int nrhs, double inner_tol, int inner_maxit,
                      std::vector<long long> &inner_total, DevBuf<double> &t_u, DevBuf<double> &t_L, DevBuf<double> &t_L2,
                      DevBuf<double> &t_u2) {
    const long long nU = c->nU, L = c->L, ns = nU + L;
    hipStream_t s = c->stream;
    // split the packed saddle vector (rhs-major, u then lambda)
    t_u.ensure((size_t)nU * nrhs, s);
    t_u2.ensure((size_t)nU * nrhs, s);
    t_L.ensure((size_t)L * nrhs, s);
    t_L2.ensure((size_t)L * nrhs, s);
    hipLaunchKernelGGL(k_unpack, dim3(nblocks(ns * nrhs)), dim3(kB), 0, s, in, nU, L, t_u.p, t_L.p, nrhs);
    // the reduced local solves of (46) depend on v alone: with overlap_local they run on a third
    // stream (into the r rows of x_u) while Ů v and the interface PCG run here; they touch only
    // their own work buffers (R, H), which nothing on this stream uses
    const bool overlap = c->opt.overlap_local && !c->opt.use_graph && c->opt.interface_block == 0;
    if (overlap) {
        ensure_work(c, nrhs);  // no reallocation while the third stream runs
        if (!c->local_stream) {
            IFETI_HIP(hipStreamCreateWithFlags(&c->local_stream, hipStreamNonBlocking));
            IFETI_HIP(hipEventCreateWithFlags(&c->ev_local_fork, hipEventDisableTiming | hipEventDisableSystemFence));
            IFETI_HIP(hipEventCreateWithFlags(&c->ev_local_join, hipEventDisableTiming | hipEventDisableSystemFence));
        }
        IFETI_HIP(hipEventRecord(c->ev_local_fork, s));
        IFETI_HIP(hipStreamWaitEvent(c->local_stream, c->ev_local_fork, 0));
        struct Scope {  // the main stream is restored also when the local solve throws
            ifeti_ctx *c;
            hipStream_t s;
            ~Scope() { c->stream = s; }
        } scope{c, s};
        c->stream = c->local_stream;
        op_rom_local(c, t_u.p, nU, t_u2.p, nU, nrhs);
        IFETI_HIP(hipEventRecord(c->ev_local_join, c->local_stream));
    }
    apply_U(c, t_u.p, t_L2.p, nrhs);                                      // Ů v
    hipLaunchKernelGGL(k_sub, dim3(nblocks(L * nrhs)), dim3(kB), 0, s, t_L.p, L, t_L2.p, L, t_L.p, L, L, nrhs,
                       -1.0);                                            // w̄ = w - Ů v
    if (c->opt.interface_block == 1) {
        apply_MD(c, t_L.p, t_L2.p, nrhs);      // lambda = M̊_D^-1 w̄ (49), no inner iteration
    } else if (c->opt.interface_block == 2) {
        apply_MD_rom(c, t_L.p, t_L2.p, nrhs);  // lambda = M̊_D^-ROM w̄ (47)
    } else {
        std::vector<int> its(nrhs);
        int st = solve_interface(c, t_L.p, t_L2.p, nrhs, inner_tol, inner_maxit, its.data(), nullptr);
        for (int r = 0; r < nrhs; ++r) inner_total[r] += its[r];
        if (st != IFETI_OK && st != IFETI_EMAXIT) {
            if (overlap) IFETI_HIP(hipStreamWaitEvent(s, c->ev_local_join, 0));
            return st;
        }
    }
    // y = -lambda; x_u = K̊^-ROM v + Ůᵀ lambda
    if (overlap) IFETI_HIP(hipStreamWaitEvent(s, c->ev_local_join, 0));
    apply_Kinv_rom(c, t_u.p, t_u2.p, nrhs, overlap);
    apply_Ut(c, t_L2.p, t_u.p, nrhs);
    hipLaunchKernelGGL(k_sub, dim3(nblocks(nU * nrhs)), dim3(kB), 0, s, t_u2.p, nU, t_u.p, nU, t_u2.p, nU, nU,
                       nrhs, 1.0);
    hipLaunchKernelGGL(k_fill, dim3(nblocks(L * nrhs)), dim3(kB), 0, s, t_L.p, L * nrhs, 0.0);
    hipLaunchKernelGGL(k_sub, dim3(nblocks(L * nrhs)), dim3(kB), 0, s, t_L.p, L, t_L2.p, L, t_L.p, L, L, nrhs,
                       -1.0);                                            // y = -lambda
    hipLaunchKernelGGL(k_pack, dim3(nblocks(ns * nrhs)), dim3(kB), 0, s, t_u2.p, nU, t_L.p, L, out, nrhs);
    IFETI_HIP(hipGetLastError());
    return IFETI_OK;
}

// ------------------------------------------------------------------ flexible GMRES on (16)
int solve_fgmres(ifeti_ctx *c, const double *f, const double *d, double *u, double *lam, int nrhs, double tol,
                 int maxit, double inner_tol, int *outer, int *inner_total, double *relres) {
    const long long nU = c->nU, L = c->L, ns = nU + L;
    const int m = std::max(1, std::min(maxit, c->opt.fgmres_restart));
    hipStream_t s = c->stream;
    // Krylov blocks come from a pool kept in the context: allocated the first time an iteration
    // count is reached, reused by later solves (memory ~ iterations used x load cases)
    const size_t nblk_elems = (size_t)ns * nrhs;
    // device tables of block pointers: growing one reallocates it without its entries, so the host
    // mirrors are cleared with it and every block pointer is uploaded again on first use
    if (c->fg_dV.n < (size_t)m + 1) {
        c->fg_dV.ensure(m + 1, s);
        std::fill(c->fg_hV.begin(), c->fg_hV.end(), nullptr);
    }
    if (c->fg_dZ.n < (size_t)m + 1) {
        c->fg_dZ.ensure(m + 1, s);
        std::fill(c->fg_hZ.begin(), c->fg_hZ.end(), nullptr);
    }
    if (c->fg_hV.size() < (size_t)m + 1) c->fg_hV.resize(m + 1, nullptr);
    if (c->fg_hZ.size() < (size_t)m + 1) c->fg_hZ.resize(m + 1, nullptr);
    int nV = 0, nZ = 0;
    auto new_block = [&](std::vector<std::unique_ptr<DevBuf<double>>> &pool, std::vector<const double *> &hp,
                         DevBuf<const double *> &dp, int &k) {
        if ((size_t)k == pool.size()) pool.emplace_back(new DevBuf<double>());
        DevBuf<double> &b = *pool[k];
        if (b.n < nblk_elems) {
            IFETI_HIP(hipStreamSynchronize(s));  // earlier work may still read the old block
            b.alloc(nblk_elems);
        }
        if (hp[k] != b.p) {  // the device table changes only when a block is (re)allocated
            hp[k] = b.p;
            IFETI_HIP(hipMemcpyAsync(dp.p + k, hp.data() + k, sizeof(double *), hipMemcpyHostToDevice, s));
        }
        return pool[k++]->p;
    };
    DevBuf<double> &w = c->fg_w, &coef = c->fg_coef, &hdev = c->fg_hdev, &hall = c->fg_hall, &scd = c->fg_scd;
    DevBuf<double> &tu = c->fg_tu, &tL = c->fg_tL, &tL2 = c->fg_tL2, &tu2 = c->fg_tu2;
    DevBuf<const double *> &dVp = c->fg_dV, &dZp = c->fg_dZ;
    w.ensure((size_t)ns * nrhs, s);
    hdev.ensure((size_t)(m + 1) * nrhs + 16, s);
    coef.ensure((size_t)(m + 1) * nrhs + 16, s);
    const size_t hstride = (size_t)(m + 1) * nrhs;
    hall.ensure(2 * hstride + nrhs, s);  // [h pass 1 | h pass 2 | ||w||^2]
    scd.ensure(nrhs, s);
    double *V0 = new_block(c->fg_V, c->fg_hV, dVp, nV);
    // b = (f, d) packed into V_0 (unnormalised)
    hipLaunchKernelGGL(k_pack, dim3(nblocks(ns * nrhs)), dim3(kB), 0, s, f, nU, d, L, V0, nrhs);
    multidot(c, V0, 0, 1, V0, ns, ns, nrhs, hdev.p);
    std::vector<double> bn(nrhs);
    {
        const double *hp = (const double *)read_back(c, hdev.p, nrhs * sizeof(double));
        std::copy(hp, hp + nrhs, bn.begin());
    }
    std::vector<double> beta(nrhs), inv(nrhs);
    for (int r = 0; r < nrhs; ++r) {
        beta[r] = std::sqrt(bn[r]);
        inv[r] = beta[r] > 0 ? 1.0 / beta[r] : 0.0;
    }
    IFETI_HIP(hipMemcpyAsync(coef.p, inv.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, s));
    scale_copy(c, V0, ns, ns, coef.p, V0, nrhs);
    // per-load-case Hessenberg and Givens data on the host
    std::vector<std::vector<double>> H(nrhs, std::vector<double>((size_t)(m + 1) * m, 0.0));
    std::vector<std::vector<double>> cs(nrhs, std::vector<double>(m)), sn(nrhs, std::vector<double>(m));
    std::vector<std::vector<double>> g(nrhs, std::vector<double>(m + 1, 0.0));
    std::vector<int> kdim(nrhs, 0), done(nrhs, 0);
    for (int r = 0; r < nrhs; ++r) {
        g[r][0] = beta[r];
        if (beta[r] == 0.0) done[r] = 1;
    }
    std::vector<long long> inner(nrhs, 0);
    int status = IFETI_OK;
    std::vector<double> h1((size_t)(m + 1) * nrhs), h2((size_t)(m + 1) * nrhs), hn(nrhs);
    int j = 0;
    for (; j < m; ++j) {
        bool all = true;
        for (int r = 0; r < nrhs; ++r) all = all && done[r];
        if (all) break;
        double *Vj = c->fg_V[j]->p;
        double *Zj = new_block(c->fg_Z, c->fg_hZ, dZp, nZ);
        int st = apply_prec(c, Vj, Zj, nrhs, inner_tol, c->opt.pcg_maxit, inner, tu, tL, tL2, tu2);
        if (st != IFETI_OK) {
            status = st;
            break;
        }
        apply_A(c, Zj, w.p, nrhs);
        // classical Gram-Schmidt, twice, with the projections kept on the device; the next basis
        // vector is normalised on the device and the host reads the Hessenberg column once
        // (the subtraction of each pass fused with the dot products that follow it: the basis is read
        // three times per step instead of four, with the same results)
        multidot(c, nullptr, 0, j + 1, w.p, ns, ns, nrhs, hall.p, dVp.p);
        if (j + 1 <= kAxpyDotMax) {
            axpy_dot(c, j + 1, hall.p, -1.0, w.p, ns, ns, nrhs, dVp.p, false, hall.p + hstride);
            axpy_dot(c, j + 1, hall.p + hstride, -1.0, w.p, ns, ns, nrhs, dVp.p, true, hall.p + 2 * hstride);
        } else {
            multiaxpy(c, nullptr, 0, j + 1, hall.p, 1.0, w.p, ns, ns, nrhs, dVp.p, -1.0);
            multidot(c, nullptr, 0, j + 1, w.p, ns, ns, nrhs, hall.p + hstride, dVp.p);
            multiaxpy(c, nullptr, 0, j + 1, hall.p + hstride, 1.0, w.p, ns, ns, nrhs, dVp.p, -1.0);
            multidot(c, w.p, 0, 1, w.p, ns, ns, nrhs, hall.p + 2 * hstride);
        }
        inv_sqrt(c, hall.p + 2 * hstride, scd.p, nrhs);
        double *Vn = new_block(c->fg_V, c->fg_hV, dVp, nV);
        scale_copy(c, w.p, ns, ns, scd.p, Vn, nrhs);
        {  // one read of [h pass 1 | h pass 2 | ||w||^2]
            const double *hp = (const double *)read_back(c, hall.p, (2 * hstride + nrhs) * sizeof(double));
            std::copy(hp, hp + (size_t)(j + 1) * nrhs, h1.begin());
            std::copy(hp + hstride, hp + hstride + (size_t)(j + 1) * nrhs, h2.begin());
            std::copy(hp + 2 * hstride, hp + 2 * hstride + nrhs, hn.begin());
        }
        for (int r = 0; r < nrhs; ++r) {
            double hj1 = std::sqrt(hn[r]);
            if (done[r]) continue;
            std::vector<double> &Hr = H[r];
            for (int i = 0; i <= j; ++i) Hr[(size_t)i * m + j] = h1[(size_t)r * (j + 1) + i] + h2[(size_t)r * (j + 1) + i];
            Hr[(size_t)(j + 1) * m + j] = hj1;
            for (int i = 0; i < j; ++i) {
                double a = Hr[(size_t)i * m + j], b = Hr[(size_t)(i + 1) * m + j];
                Hr[(size_t)i * m + j] = cs[r][i] * a + sn[r][i] * b;
                Hr[(size_t)(i + 1) * m + j] = -sn[r][i] * a + cs[r][i] * b;
            }
            double a = Hr[(size_t)j * m + j], b = Hr[(size_t)(j + 1) * m + j];
            double den = std::hypot(a, b);
            cs[r][j] = a / den;
            sn[r][j] = b / den;
            Hr[(size_t)j * m + j] = den;
            Hr[(size_t)(j + 1) * m + j] = 0.0;
            g[r][j + 1] = -sn[r][j] * g[r][j];
            g[r][j] = cs[r][j] * g[r][j];
            kdim[r] = j + 1;
            if (std::fabs(g[r][j + 1]) <= tol * beta[r] || hj1 == 0.0) done[r] = 1;
        }
    }
    // x = sum_i y_i Z_i per load case
    int kmax = 0;
    for (int r = 0; r < nrhs; ++r) {
        int k = kdim[r];
        kmax = std::max(kmax, k);
        std::vector<double> y(k, 0.0);
        for (int i = k - 1; i >= 0; --i) {
            double t = g[r][i];
            for (int l = i + 1; l < k; ++l) t -= H[r][(size_t)i * m + l] * y[l];
            y[i] = t / H[r][(size_t)i * m + i];
        }
        for (int i = 0; i < k; ++i) g[r][i] = y[i];  // keep the solution coefficients
    }
    std::vector<double> yc((size_t)std::max(kmax, 1) * nrhs, 0.0);
    for (int r = 0; r < nrhs; ++r)
        for (int i = 0; i < kdim[r]; ++i) yc[(size_t)r * kmax + i] = g[r][i];
    DevBuf<double> &xs = c->fg_xs;
    xs.ensure((size_t)ns * nrhs, s);
    hipLaunchKernelGGL(k_fill, dim3(nblocks(ns * nrhs)), dim3(kB), 0, s, xs.p, ns * nrhs, 0.0);
    if (kmax > 0) {
        IFETI_HIP(hipMemcpyAsync(coef.p, yc.data(), yc.size() * sizeof(double), hipMemcpyHostToDevice, s));
        multiaxpy(c, nullptr, 0, kmax, coef.p, 1.0, xs.p, ns, ns, nrhs, dZp.p);
    }
    hipLaunchKernelGGL(k_unpack, dim3(nblocks(ns * nrhs)), dim3(kB), 0, s, xs.p, nU, L, u, lam, nrhs);
    // true residual ||b - A x|| / ||b||
    apply_A(c, xs.p, w.p, nrhs);
    hipLaunchKernelGGL(k_pack, dim3(nblocks(ns * nrhs)), dim3(kB), 0, s, f, nU, d, L, xs.p, nrhs);
    hipLaunchKernelGGL(k_sub, dim3(nblocks(ns * nrhs)), dim3(kB), 0, s, xs.p, ns, w.p, ns, xs.p, ns, ns, nrhs, -1.0);
    multidot(c, xs.p, 0, 1, xs.p, ns, ns, nrhs, hdev.p);
    {
        const double *hp = (const double *)read_back(c, hdev.p, nrhs * sizeof(double));
        std::copy(hp, hp + nrhs, hn.begin());
    }
    bool conv = true;
    for (int r = 0; r < nrhs; ++r) {
        double rel = beta[r] > 0 ? std::sqrt(hn[r]) / beta[r] : 0.0;
        if (relres) relres[r] = rel;
        if (outer) outer[r] = kdim[r];
        c->fgmres_its += kdim[r];
        conv = conv && done[r];
    }
    if (inner_total)
        for (int r = 0; r < nrhs; ++r) inner_total[r] = (int)inner[r];
    if (status != IFETI_OK) return status;
    if (!conv) {
        set_last_error("FGMRES reached the iteration limit");
        return IFETI_EMAXIT;
    }
    return IFETI_OK;
}

}  // namespace ifeti
