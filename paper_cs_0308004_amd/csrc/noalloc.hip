// dpg_retrieve_noalloc: record retrieval whose workspace is a static device
// array of the library instead of caller memory, for callers that cannot
// allocate device memory.
//
// `scratch` below is a device variable.  Its name, used in host code, is a
// host-side stand-in registered with the HIP runtime, not a device address:
// the device address is looked up once per device (hipGetSymbolAddress, with
// that device current, when a context is created on it) and only that
// address is handed to kernels.  Every device the library runs on holds its
// own copy of the array until the process ends.
#include <mutex>

#include "dpg_internal.h"

namespace dpg {

static __device__ __align__(256) unsigned char scratch[DPG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_done[kMaxDevices];
void *g_addr[kMaxDevices];  // device address of `scratch` on each device (null if the lookup failed)
}  // namespace

void scratch_init(dpg_ctx *ctx) {
    ctx->scratch = nullptr;
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[ctx->device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_addr[ctx->device] = (e == hipSuccess) ? ptr : nullptr;
        g_done[ctx->device] = true;
    }
    ctx->scratch = g_addr[ctx->device];
}

}  // namespace dpg

extern "C" dpg_status dpg_retrieve_noalloc(dpg_ctx *ctx, const void *src, int64_t n_src, int32_t rec_bytes,
                                           const int32_t *rids, int64_t n_rids, void *dst, dpg_algo algo,
                                           int check_rids, hipStream_t stream) {
    if (!ctx) return DPG_ERR_INVALID_ARG;
    const size_t need = dpg_retrieve_workspace_bytes(ctx, n_src, rec_bytes, n_rids, algo);
    if (need > DPG_NOALLOC_SCRATCH_BYTES) return DPG_ERR_WORKSPACE_TOO_SMALL;
    if (n_rids > 0 && !ctx->scratch) return DPG_ERR_HIP;
    // the same validation, plan and kernels as dpg_retrieve; none of them
    // allocates, and none needs the workspace cleared beforehand
    return dpg_retrieve(ctx, src, n_src, rec_bytes, rids, n_rids, dst, ctx->scratch, DPG_NOALLOC_SCRATCH_BYTES,
                        algo, check_rids, stream);
}
