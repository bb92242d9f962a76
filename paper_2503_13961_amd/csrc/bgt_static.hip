// The photometric loss pass with its workspace in a fixed device array, for
// callers that cannot allocate device memory (code under stream capture,
// serving loops, harnesses that forbid hipMalloc): bgt_loss_noalloc.
//
// The workspace (three float maps per pixel and channel, then the
// per-workgroup partial sums) lives in `scratch`, a file-scope device array
// of kScratchBytes.  Every device the library runs on holds its own copy
// until the process ends.  In host code `scratch` only names the symbol;
// its device address on each GPU is fetched once per device, with that
// device current, when a context is created (bgt_create), and only that
// address is ever passed to kernels.  Every call on one GPU shares the
// array: calls that overlap on a GPU (two streams, or two host threads)
// race on it.  The loss kernels write every map entry and partial sum they
// read, so nothing needs clearing between calls.
#include <mutex>
#include <string>

#include "bgt_internal.h"

namespace bgt {

static __device__ __align__(256) unsigned char scratch[size_t(64) << 20];

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB: about 1.86 M pixels of views
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

static_assert(sizeof(scratch) == kScratchBytes, "static workspace size");

}  // namespace

hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the calling thread's current device
    if (e != hipSuccess) return e;
    g_scratch[device] = p;
    return hipSuccess;
}

size_t static_scratch_bytes() { return kScratchBytes; }

void *static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_scratch[device];
}

}  // namespace bgt

extern "C" bgt_status bgt_loss_noalloc(bgt_ctx *ctx, const bgt_views *views, const float *images,
                                       const float *targets, float lambda, float *loss, float *grad_images,
                                       void *stream) {
    using namespace bgt;
    if (!ctx) return BGT_E_INVALID;
    size_t need = 0;
    if (bgt_loss_workspace_size(views, &need) != BGT_OK)
        return ctx_fail(ctx, BGT_E_INVALID, "invalid views");
    if (need > kScratchBytes) {
        const std::string msg = "loss workspace of " + std::to_string(need) + " bytes exceeds the " +
                                std::to_string(kScratchBytes) + "-byte static workspace of bgt_loss_noalloc";
        return ctx_fail(ctx, BGT_E_NOMEM, msg.c_str());
    }
    void *ws = static_scratch(ctx_device(ctx));
    if (!ws) return ctx_fail(ctx, BGT_E_INVALID, "no static workspace on this context's device");
    return bgt_loss(ctx, views, images, targets, lambda, loss, grad_images, ws, kScratchBytes, stream);
}
