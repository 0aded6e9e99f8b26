// Allocation-free solve: tpf_solve_timeseries with the scratch its kernels use (the atomic
// column queue of the persistent sweep kernels) in a file-scope device array instead of a
// caller workspace, for callers that cannot allocate.
#include "tpf_internal.h"

namespace {

// Bytes of the per-GPU scratch array; a request whose workspace exceeds it is refused.
constexpr size_t kScratchBytes = 4096;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per HIP device, looked up once per device with that device
// current (each GPU holds its own copy of the array).  Fixed-size table: no allocation.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return tpf::fail(TPF_ERR_DEVICE, "hipGetDevice failed (no GPU?)");
    if (dev < 0 || dev >= kMaxDevices) return tpf::fail(TPF_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return tpf::fail(TPF_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TPF_OK;
}

}  // namespace

extern "C" int tpf_solve_timeseries_noalloc(tpf_network net, const void *S, int32_t dtype, int64_t T, double tol,
                                            int32_t max_iter, const tpf_options *opts, void *V_out,
                                            int32_t *iters_out, int8_t *status_out, void *stream) {
    tpf::clear_error();
    if (!net) return tpf::fail(TPF_ERR_INVALID_ARG, "net is NULL");
    if (T < 0) return tpf::fail(TPF_ERR_INVALID_ARG, "T must be >= 0");
    const size_t need = tpf_workspace_bytes(net, T, opts);
    if (need > kScratchBytes)
        return tpf::fail(TPF_ERR_UNSUPPORTED, "this solve needs " + std::to_string(need) +
                                                  " bytes of workspace; the allocation-free entry point holds " +
                                                  std::to_string(kScratchBytes) +
                                                  " (large networks' per-sweep path and warm starts need "
                                                  "tpf_solve_timeseries)");
    void *ws = nullptr;
    int rc = scratch_for_current_device(&ws);
    if (rc != TPF_OK) return rc;
    return tpf::solve_impl(net, S, dtype, T, tol, max_iter, opts, V_out, iters_out, status_out, ws, kScratchBytes,
                           stream, true);
}
