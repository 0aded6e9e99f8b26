// C ABI entry points: argument checks, workspace carving and kernel dispatch.
#include <cmath>

#include "tpf_internal.h"

using namespace tpf;

namespace {

constexpr size_t kQueueBytes = 256;  // atomic column queue (+ padding to 256 B)

bool valid_dtype(int32_t d) { return d == TPF_C64 || d == TPF_C128; }

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TPF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return TPF_OK;
}

}  // namespace

namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

bool is_tree(int mode) { return mode == TPF_MODE_TREE_FP64 || mode == TPF_MODE_TREE_FP32; }

// Workspace of the sweeps alone: the atomic column queue, or the per-sweep path's state.
size_t base_workspace(const tpf_network_s &net, int64_t tau, int mode) {
    if (!is_tree(mode) && uses_large_path(net.n, mode)) return large_workspace_bytes(net.n, tau, mode);
    return kQueueBytes;
}

// Workspace for the V0 a learned start writes before the sweeps (complex128 assumed: the
// larger of the two dtypes) and for its inference scratch.
size_t warm_workspace(const tpf_network_s &net, int64_t tau, tpf_mlp mlp) {
    if (!mlp) return 0;
    return align256((size_t)tau * net.n * 16) + align256(mlp_predict_scratch_bytes(mlp, tau));
}

}  // namespace

extern "C" size_t tpf_workspace_bytes(tpf_network net, int64_t tau, const tpf_options *opts) {
    if (!net || tau < 0) return kQueueBytes;
    const int mode = opts ? opts->mode : TPF_MODE_FP64;
    const size_t base = base_workspace(*net, tau, mode);
    const size_t warm = warm_workspace(*net, tau, opts ? opts->warm_start : nullptr);
    return warm ? align256(base) + warm : base;
}

namespace tpf {

int solve_impl(tpf_network net, const void *S, int32_t dtype, int64_t T, double tol, int32_t max_iter,
               const tpf_options *opts, void *V_out, int32_t *iters_out, int8_t *status_out, void *workspace,
               size_t workspace_bytes, void *stream, bool resident_only) {
    if (!net) return fail(TPF_ERR_INVALID_ARG, "net is NULL");
    if (!valid_dtype(dtype)) return fail(TPF_ERR_INVALID_ARG, "dtype must be TPF_C64 or TPF_C128");
    if (T < 0) return fail(TPF_ERR_INVALID_ARG, "T must be >= 0");
    if (!(tol >= 0.0)) return fail(TPF_ERR_INVALID_ARG, "tol must be >= 0 (and not NaN)");
    if (max_iter < 0) return fail(TPF_ERR_INVALID_ARG, "max_iter must be >= 0");
    const int mode = opts ? opts->mode : TPF_MODE_FP64;
    if (mode < TPF_MODE_FP64 || mode > TPF_MODE_TREE_FP32) return fail(TPF_ERR_INVALID_ARG, "unknown mode");
    if (mode != TPF_MODE_FP64 && mode != TPF_MODE_TREE_FP64 && tol < 5e-7)
        return fail(TPF_ERR_INVALID_ARG, "tol below the FP32 state floor (5e-7 pu) in a reduced-precision mode");
    const void *V0 = opts ? opts->V0 : nullptr;
    tpf_mlp mlp = opts ? opts->warm_start : nullptr;
    if (V0 && mlp) return fail(TPF_ERR_INVALID_ARG, "give either V0 or a warm-start network, not both");
    if (T == 0) return TPF_OK;
    if (!S || !V_out || !iters_out || !status_out) return fail(TPF_ERR_INVALID_ARG, "array pointer is NULL");
    const int n = net->n;
    if (T > (int64_t)1 << 40 || (int64_t)n * T > ((int64_t)1 << 50)) return fail(TPF_ERR_INVALID_ARG, "T too large");
    if (!workspace || workspace_bytes < tpf_workspace_bytes(net, T, opts))
        return fail(TPF_ERR_INVALID_ARG, "workspace missing or smaller than tpf_workspace_bytes()");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(TPF_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    DeviceNet *dn = nullptr;
    int rc = resident_only ? device_net_resident(net, &dn) : device_net(net, &dn);
    if (rc != TPF_OK) return rc;
    double *mismatch_out = opts ? opts->mismatch_out : nullptr;
    const int64_t *t_index = opts ? opts->t_index : nullptr;
    if (mlp) {  // the learned start: its inference writes V0 into the workspace, past the sweeps' part
        const size_t off = align256(base_workspace(*net, T, mode));
        void *v0buf = static_cast<char *>(workspace) + off;
        void *scratch = static_cast<char *>(v0buf) + align256((size_t)T * n * 16);
        rc = mlp_predict_into(mlp, S, dtype, t_index, T, v0buf, scratch, st);
        if (rc != TPF_OK) return rc;
        V0 = v0buf;
    }
    if (max_iter == 0) {
        rc = launch_start_only(n, V0, dtype, T, V_out, iters_out, status_out, st);
    } else if (is_tree(mode)) {
        rc = launch_fpi_tree(*net, *dn, mode, S, dtype, T, tol, max_iter, V0, V_out, iters_out, status_out, st);
    } else if (uses_large_path(n, mode)) {
        rc = launch_fpi_large(*net, *dn, mode, S, dtype, T, tol, max_iter, V0, V_out, iters_out, status_out,
                              workspace, st);
    } else if (n <= 8 * kMaxSmallTiles) {
        auto *queue = reinterpret_cast<unsigned long long *>(workspace);
        rc = launch_zero_u64(queue, 1, st);
        if (rc == TPF_OK) rc = check_launch("queue reset");
        if (rc == TPF_OK && mode == TPF_MODE_FP64) {
            rc = launch_fpi_small_f64(*net, *dn, S, dtype, T, tol, max_iter, V0, V_out, iters_out, status_out,
                                      queue, st);
        }
        else if (rc == TPF_OK) {
            rc = launch_fpi_mixed(*net, *dn, mode, S, dtype, T, tol, max_iter, V0, V_out, iters_out, status_out,
                                  queue, st);
        }
    } else {
        return fail(TPF_ERR_UNSUPPORTED, "no sweep path for this network size and mode");
    }
    if (rc != TPF_OK) return rc;
    rc = check_launch("sweep kernel launch");
    if (rc != TPF_OK) return rc;
    if (mismatch_out) {  // FP64 check of the returned voltages, as its own pass
        rc = launch_mismatch_f64(*net, *dn, S, V_out, dtype, T, mismatch_out, st);
        if (rc == TPF_OK) rc = check_launch("mismatch kernel launch");
    }
    return rc;
}

}  // namespace tpf

extern "C" int tpf_solve_timeseries(tpf_network net, const void *S, int32_t dtype, int64_t T, double tol,
                                    int32_t max_iter, const tpf_options *opts, void *V_out, int32_t *iters_out,
                                    int8_t *status_out, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    return solve_impl(net, S, dtype, T, tol, max_iter, opts, V_out, iters_out, status_out, workspace,
                      workspace_bytes, stream, false);
}

extern "C" int tpf_solve_tensor(tpf_network net, const void *S, int32_t dtype, int64_t n_scen, int64_t T, double tol,
                                int32_t max_iter, const tpf_options *opts, void *V_out, int32_t *iters_out,
                                int8_t *status_out, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (n_scen < 0 || T < 0) return fail(TPF_ERR_INVALID_ARG, "n_scen and T must be >= 0");
    if (T > 0 && n_scen > (((int64_t)1 << 40) / T)) return fail(TPF_ERR_INVALID_ARG, "n_scen * T too large");
    // Sec. IV-A: [P][T][n] is contiguous-reshaped to [P*T][n]; no iterate changes.
    return tpf_solve_timeseries(net, S, dtype, n_scen * T, tol, max_iter, opts, V_out, iters_out, status_out,
                                workspace, workspace_bytes, stream);
}

extern "C" int tpf_mismatch(tpf_network net, const void *S, const void *V, int32_t dtype, int64_t tau, double *out,
                            void *stream) {
    clear_error();
    if (!net) return fail(TPF_ERR_INVALID_ARG, "net is NULL");
    if (!valid_dtype(dtype)) return fail(TPF_ERR_INVALID_ARG, "dtype must be TPF_C64 or TPF_C128");
    if (tau < 0) return fail(TPF_ERR_INVALID_ARG, "tau must be >= 0");
    if (tau == 0) return TPF_OK;
    if (!S || !V || !out) return fail(TPF_ERR_INVALID_ARG, "array pointer is NULL");
    DeviceNet *dn = nullptr;
    int rc = device_net(net, &dn);
    if (rc != TPF_OK) return rc;
    rc = launch_mismatch_f64(*net, *dn, S, V, dtype, tau, out, reinterpret_cast<hipStream_t>(stream));
    if (rc != TPF_OK) return rc;
    return check_launch("mismatch kernel launch");
}
