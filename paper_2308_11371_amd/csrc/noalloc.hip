// Allocation-free variant of the F̊ apply (eq. (48)) for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).  Its work buffers (the contraction output, the
// coarse correction, the restricted cell vectors and the coarse right-hand side and solution) live in
// one file-scope device array; each GPU holds its own copy for the life of the process.
#include <mutex>

#include "common.hpp"

namespace {

// 4 Mi doubles (32 MiB) per GPU: one c2 load case needs 1.1 Mi, three need 3.3 Mi
constexpr size_t kScratchDoubles = (size_t)4 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

// the array's address on the current device (taken once per device): host code may not pass the
// symbol itself to a kernel, only this address
double *scratch_on_current_device() {
    int dev = 0;
    IFETI_HIP(hipGetDevice(&dev));
    IFETI_REQUIRE(dev >= 0 && dev < kMaxDevices, IFETI_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw ifeti::Error{IFETI_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch[dev] = static_cast<double *>(p);
    }
    return g_scratch[dev];
}

inline size_t round_up(size_t n) { return (n + 31) / 32 * 32; }  // 256-byte segments

struct NoAllocScope {
    ifeti_ctx *c;
    explicit NoAllocScope(ifeti_ctx *cc) : c(cc) { c->no_alloc = true; }
    ~NoAllocScope() { c->no_alloc = false; }
};

}  // namespace

using namespace ifeti;

extern "C" int ifeti_apply_F_noalloc(ifeti_ctx *c, const double *lam, double *out, int nrhs) {
    try {
        IFETI_REQUIRE(c && c->rom_built, IFETI_EINVAL, "reduced basis not built");
        IFETI_REQUIRE(lam && out && lam != out, IFETI_EINVAL, "bad pointers");
        IFETI_REQUIRE(nrhs >= 1 && nrhs <= 3, IFETI_EINVAL,
                      "ifeti_apply_F_noalloc takes 1 to 3 load cases (the coarse solve's preallocated buffers)");
        const size_t cols = (size_t)c->N * nrhs;
        const size_t nY = round_up(cols * c->n_d), nC = round_up(cols * c->n_p);
        const size_t nPv = round_up((size_t)std::max(c->nP, 1) * nrhs);
        const size_t need = 2 * nY + nC + 2 * nPv;
        if (need > kScratchDoubles)
            throw Error{IFETI_EINVAL, "ifeti_apply_F_noalloc needs " + std::to_string(need * 8) +
                                          " bytes of scratch; the maximum is " + std::to_string(kScratchDoubles * 8)};
        double *base = scratch_on_current_device();
        double *Y = base, *Yc = Y + nY, *cb = Yc + nY, *zP = cb + nC, *yP = zP + nPv;
        NoAllocScope scope(c);
        apply_F_into(c, lam, out, nrhs, Y, Yc, cb, zP, yP, nullptr, nullptr);
        IFETI_HIP(hipGetLastError());
        return IFETI_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return IFETI_EINVAL;
    }
}
