// Internal declarations shared by the host and device sources of libtpf.so.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpf.h"

namespace tpf {

using cd = std::complex<double>;

// Register-resident sweep kernels keep one 16-row MFMA tile per 8 PQ buses in
// registers; MT = ceil(n / 8) tiles, n <= 8 * kMaxSmallTiles.
constexpr int kMaxSmallTiles = 40;

// Workgroup shape of the register-resident kernels for MT row tiles: NW waves,
// each owning at most TPW tiles (tile t belongs to wave role t % NW).
inline void rows_config(int MT, int &NW, int &TPW) {
    NW = MT <= 4 ? 4 : 8;
    TPW = (MT + NW - 1) / NW;
}
// Floor of |V|^2 in the FP32 injections conj(S) V / |V|^2: an iterate passing through
// V = 0 (an infeasible load's orbit can) then gives a large finite injection,
// |I| <= |S| 1e15, instead of inf, so a column with finite inputs stays finite and ends
// MAX_ITER, never NONFINITE.  Every feasible iterate has |V|^2 far above it.
constexpr float kMinV2 = 1e-30f;
// The FP64 fragment array carries this many zero k-steps past the end so that the
// k-loop's prefetch ring never needs a bounds branch.
constexpr int kFragPadSteps = 4;

// Device copies of a network, made on first use on each device.
struct DeviceNet {
    int device = -1;
    int MT = 0;                  // 16-row tiles of the real-block operator (small-n kernels)
    int NW = 0, TPW = 0;         // workgroup shape (rows_config)
    double *A64 = nullptr;       // FP64 MFMA A fragments, [NW roles][4*MT+pad k-steps][TPW tiles][64 lanes]
    double *w64 = nullptr;       // [2][8*MT]: Re w then Im w per bus (padding buses: 1, 0)
    // FP32-family kernels (FP32 and mixed modes), n <= 128.  Rows/cols use the order
    // of the FP32/BF16/FP16 MFMA output (lane group g holds tile rows 4g..4g+3):
    // row 16 t + 2 (q % 8) + part for PQ bus q = 8 t + (q % 8).
    int KTL = 0;                 // 32-wide k-steps of the 16-bit products (K padded to 32 KTL)
    int sZ = 0;                  // power-of-two scale of Z in the FP16 operands
    float *A32 = nullptr;        // FP32 fragments, [NW][4*MT+pad][TPW][64]
    uint16_t *Abf = nullptr;     // BF16 fragments, [NW][TPW][KTL][64][8]
    uint16_t *Ah = nullptr;      // FP16 fragments of Z 2^sZ, [NW][TPW][KTL][64][8]
    uint16_t *Al = nullptr;      // FP16 residual Z 2^sZ - Ah, same layout
    // Large-network path (fpi_large.hip): operator [MPL][KPL] row-major, K interleaved
    // Re/Im per bus; FP64 rows in 16-row tiles of 8 buses (Re rows 0-7, Im rows 8-15),
    // FP32-family rows interleaved (2 q + part).  wl = w as [n][2].  The 16-bit
    // operands (BF16 Z, FP16 Z 2^sZ) have K padded to KPL16, a multiple of 32.
    int MPL64 = 0, MPL32 = 0, KPL = 0, KPL16 = 0;
    double *AL64 = nullptr;
    float *AL32 = nullptr;
    uint16_t *ALbf = nullptr, *ALh = nullptr;
    double *wl = nullptr;
    // Large path: a pinned host word, mapped for the device (done_dev), to which a sweep
    // that finds no active column posts its solve's sequence number; the host loop that
    // queues the sweeps reads it without waiting and stops queueing once it matches.
    int *done_host = nullptr, *done_dev = nullptr;
    mutable std::atomic<int> solve_seq{0};
    // Sparse Y_dd (CSR) and c = Y_ds v_s for the FP64 mismatch.
    int32_t *rowptr = nullptr;   // [n+1]
    int32_t *colidx = nullptr;   // [nnz]
    double *yval = nullptr;      // [nnz][2]
    double *cval = nullptr;      // [n][2]
    // ZIP load shares per PQ bus (Eq. (2)); NULL for constant-power loads.
    // Radial networks, tree operator (fpi_tree.hip): breadth-first positions 0..n_bus-1
    // (0 = slack).  tree_i = [pq bus][parent][first child][end of children] per position
    // (4 n_bus int32) then the level starts (tree_levels + 2 int32); tree_z = per position
    // the branch impedance (phases x phases complex) then w of its phases, as doubles.
    int tree_levels = 0;
    int tree_phases = 1;
    int32_t *tree_i = nullptr;
    double *tree_z = nullptr;
    double *aI = nullptr, *aP = nullptr;  // [n] each
    double *aZ = nullptr;                 // [n], only when some alpha_Z != 0
    float zscale = 1.0f;                  // max_b |alpha_P| + |alpha_I| + |alpha_Z| (bounds |I| / |S| with |V|)
    std::vector<void *> owned;   // every allocation above, freed with the network
};

// Inference into V0 (device [rows][n], dtype of S), as tpf_mlp_predict, for the solve
// calls' warm start when the fused kernel does not apply; `t_index` may be NULL (t =
// column index).  `scratch` holds at least mlp_predict_scratch_bytes(mlp, rows) bytes.
size_t mlp_predict_scratch_bytes(tpf_mlp mlp, int64_t rows);
int mlp_predict_into(tpf_mlp mlp, const void *S, int dtype, const int64_t *t_index, int64_t rows, void *V0,
                     void *scratch, hipStream_t stream);

// Sparse Y_dd and c = Y_ds v_s on the device, for the FP64 power-balance mismatch
// (Eq. (1)); `out` is NULL when no mismatch is requested.
}  // namespace tpf

struct tpf_network_s {
    int n_bus = 0;
    int phases = 1;  // 3 for tpf_build_network_3ph: demand node 3 k + p is phase p of PQ bus k
    int n = 0;  // demand nodes (PQ buses x phases)
    int slack = 0;
    tpf::cd vs;
    std::vector<tpf::cd> Z;  // [n][n], Z = -Y_dd^-1
    std::vector<tpf::cd> w;  // [n]
    // CSR of Y_dd in PQ order and c = Y_ds v_s.
    std::vector<int32_t> rowptr, colidx;
    std::vector<tpf::cd> yval;
    std::vector<tpf::cd> c;
    // ZIP loads (Eq. (2)): shares of constant current and constant power per PQ bus; empty
    // for constant-power loads.  alpha_z (constant impedance) is empty unless some share
    // is non-zero: the tree operator then eliminates B = diag(alpha_Z s*) + Y_dd per column
    // along the tree, the dense forms carry the current alpha_Z conj(S) V in the injection.
    bool zip = false;
    std::vector<double> alpha_i, alpha_p, alpha_z;
    // Breadth-first tree of a radial single-phase network (empty otherwise): per position
    // p = 0..n (0 = slack) the PQ index, parent position, children range and the impedance
    // of the branch from the parent; level starts.  Children of a position are
    // contiguous, and each level is a contiguous range of positions.
    std::vector<int32_t> tree_pq, tree_parent, tree_c0, tree_c1, tree_level_start;
    std::vector<tpf::cd> tree_z;  // phases x phases per position
    int tree_phases = 1;
    std::mutex mu;
    std::vector<tpf::DeviceNet *> dev;  // indexed by HIP device id
};

namespace tpf {

// Thread-local error text + return code helper.
int fail(int code, const std::string &msg);
void clear_error();

// Returns the device copies of `net` on the current device, uploading on first use.
int device_net(tpf_network net, DeviceNet **out);
// The same when the copies already exist on the current device; TPF_ERR_UNSUPPORTED
// otherwise (allocates nothing).
int device_net_resident(tpf_network net, DeviceNet **out);
// tpf_solve_timeseries's body; resident_only: the network must already be on the device.
int solve_impl(tpf_network net, const void *S, int32_t dtype, int64_t T, double tol, int32_t max_iter,
               const tpf_options *opts, void *V_out, int32_t *iters_out, int8_t *status_out, void *workspace,
               size_t workspace_bytes, void *stream, bool resident_only);

// Launchers (device code in fpi_small.hip / mismatch.hip).  All asynchronous on `stream`.
int launch_fpi_small_f64(const tpf_network_s &net, const DeviceNet &dn, const void *S, int dtype,
                         int64_t tau, double tol, int max_iter, const void *V0, void *V,
                         int32_t *iters, int8_t *status, unsigned long long *queue, hipStream_t stream);
int launch_fpi_tree(const tpf_network_s &net, const DeviceNet &dn, int mode, const void *S, int dtype, int64_t tau,
                    double tol, int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                    hipStream_t stream);
int launch_fpi_mixed(const tpf_network_s &net, const DeviceNet &dn, int mode, const void *S, int dtype,
                     int64_t tau, double tol, int max_iter, const void *V0, void *V, int32_t *iters,
                     int8_t *status, unsigned long long *queue, hipStream_t stream);
int launch_fpi_large(const tpf_network_s &net, const DeviceNet &dn, int mode, const void *S, int dtype,
                     int64_t tau, double tol, int max_iter, const void *V0, void *V, int32_t *iters,
                     int8_t *status, void *workspace, hipStream_t stream);
size_t large_workspace_bytes(int n, int64_t tau, int mode);
// The register-resident kernels cover FP64 up to 8 * kMaxSmallTiles PQ buses and the
// FP32/mixed ones up to 128; larger networks use the large path (FP64, FP32).
inline bool uses_large_path(int n, int mode) { return mode == TPF_MODE_FP64 ? n > 8 * kMaxSmallTiles : n > 128; }
int launch_start_only(int n, const void *V0, int dtype, int64_t tau, void *V, int32_t *iters,
                      int8_t *status, hipStream_t stream);
int launch_mismatch_f64(const tpf_network_s &net, const DeviceNet &dn, const void *S, const void *V,
                        int dtype, int64_t tau, double *out, hipStream_t stream);
int launch_zero_u64(unsigned long long *p, int count, hipStream_t stream);

}  // namespace tpf
