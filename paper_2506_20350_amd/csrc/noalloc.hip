// MLFFT product for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation): the
// spectral workspaces of the product come from a fixed array in the library's
// own device memory instead of the context's allocator.
#include <mutex>

#include "lib.h"

using namespace mlfft;

namespace {

// Two spectral workspaces of kScratchHalf bytes each.  Every device the library
// runs on holds its own copy until the process ends.
constexpr size_t kScratchHalf = size_t(64) << 20;
constexpr size_t kScratchBytes = 2 * kScratchHalf;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};      // device address of `scratch` on each device

}  // namespace

namespace mlfft {

// Look up the device address of the scratch array on `device` (which must be
// the current device) once per device.  The array's name is a host-side
// stand-in: host code passes only the address found here to kernels.
hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[device] = p;
    return hipSuccess;
}

}  // namespace mlfft

extern "C" mlfft_status mlfft_matvec_noalloc(mlfft_ctx ctx, int array_id, int W, const void* x, void* y,
                                             mlfft_prec prec) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (W < 0) return c->fail(MLFFT_E_ARG, "W must be >= 0");
    if (prec < MLFFT_FP64 || prec > MLFFT_FP32_BF16GEMM) return c->fail(MLFFT_E_ARG, "invalid precision");
    if (W == 0) return MLFFT_OK;
    if (!x || !y) return c->fail(MLFFT_E_ARG, "x or y is NULL");
    const size_t vb = a->Nt() * W * prec_elem_bytes(prec);
    if ((const char*)x < (const char*)y + vb && (const char*)y < (const char*)x + vb)
        return c->fail(MLFFT_E_ARG, "x and y overlap");
    const size_t need = ((size_t)a->K * a->b * W * prec_elem_bytes(prec) + 255) / 256 * 256;
    if (need > kScratchHalf)
        return c->fail(MLFFT_E_ARG,
                       "product needs two spectral workspaces of %zu bytes; the fixed scratch holds two of %zu "
                       "(4 Nx Ny b W x %d bytes each)",
                       need, kScratchHalf, prec_elem_bytes(prec));
    void* base = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch[c->device] : nullptr;
    if (!base) return c->fail(MLFFT_E_STATE, "scratch of device %d was not set up", c->device);
    std::vector<MatvecItem> items(1);
    items[0] = MatvecItem{a, W, x, y, nullptr, 1.0, 0.0};
    // profiling records create events; this entry point runs unprofiled
    const bool prof = c->prof;
    c->prof = false;
    const mlfft_status st = c->matvec_group(items, prec, base, (char*)base + kScratchHalf, kScratchHalf);
    c->prof = prof;
    return st;
}
