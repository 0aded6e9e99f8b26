// FP64 power-balance mismatch of a batch of voltage solutions.
//
// Eq. (1) of the paper gives -i_d = Y_ds v_s + Y_dd v for the demand nodes, so a
// load drawing S must satisfy S = v .* conj(i_d), i.e.
//     m = S + V .* conj(Y_ds v_s + Y_dd V) = 0.
// One wavefront handles one column at a time: its lanes walk the buses (coalesced
// reads of S and V), multiply the sparse row of Y_dd (a radial feeder has about
// three nonzeros per row), and the wave reduces max |m_i| with NaN propagation.
// The kernel is bandwidth-bound: S and V are read once.
#include "tpf_internal.h"

namespace tpf {

__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

template <typename IO>
__global__ __launch_bounds__(256) void mismatch_f64_kernel(const IO *__restrict__ S, const IO *__restrict__ V,
                                                           int n, long long tau, const int32_t *__restrict__ rowptr,
                                                           const int32_t *__restrict__ colidx,
                                                           const double *__restrict__ yv,
                                                           const double *__restrict__ cv, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const long long wid = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const long long nw = (long long)gridDim.x * 4;
    for (long long c = wid; c < tau; c += nw) {
        const IO *vc = V + 2 * c * n;
        const IO *sc = S + 2 * c * n;
        double worst = 0.0;
        const MismatchArgs mm{rowptr, colidx, yv, cv, out, 0, 0};
        for (int i = lane; i < n; i += 64) {
            worst = nanmax(worst, bus_mismatch(mm, i, (double)sc[2 * i], (double)sc[2 * i + 1], (double)vc[2 * i],
                                               (double)vc[2 * i + 1], [&](int k, double &xr, double &xi) {
                                                   xr = (double)vc[2 * k];
                                                   xi = (double)vc[2 * k + 1];
                                               }));
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) worst = nanmax(worst, __shfl_xor(worst, off));
        if (lane == 0) out[c] = worst;
    }
}

int launch_mismatch_f64(const tpf_network_s &net, const DeviceNet &dn, const void *S, const void *V, int dtype,
                        int64_t tau, double *out, hipStream_t stream) {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long blocks = std::max<long long>(1, std::min<long long>((long long)cus * 16, (tau + 3) / 4));
    if (dtype == TPF_C128)
        hipLaunchKernelGGL(mismatch_f64_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const double *)S, (const double *)V, net.n, (long long)tau, dn.rowptr, dn.colidx,
                           dn.yval, dn.cval, out);
    else
        hipLaunchKernelGGL(mismatch_f64_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const float *)S, (const float *)V, net.n, (long long)tau, dn.rowptr, dn.colidx,
                           dn.yval, dn.cval, out);
    return TPF_OK;
}

}  // namespace tpf
