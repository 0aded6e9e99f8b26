// Persistent FP64 sweep kernel for networks with up to 320 PQ buses.
//
// Algorithm 1 (Sec. IV-A) evaluates V <- Z conj(S ./ V) + w for every power flow
// (column) of the reshaped load matrix until the voltage step of that column
// falls below the tolerance.  Here each wavefront is an independent worker that
// owns 16 column slots.  Per sweep it
//   1. forms the current injection conj(S./V) = conj(S) V / |V|^2 (Eq. (3)) of the
//      slot's buses straight into its MFMA B operand (never stored to memory),
//   2. multiplies by Z as one real product [Zr -Zi; Zi Zr] [Ir; Ii] on the
//      16x16x4 FP64 matrix cores, with Z streamed from L2 in fragment order,
//   3. adds w, measures max_i |V'_i - V_i| per column with lane shuffles, and
//   4. retires converged columns (writes V, sweep count and status) and refills
//      their slots from a global atomic column queue, so the 16-wide MFMA tiles
//      stay full while columns finish after different numbers of sweeps.
//
// Register layout.  The real-block operator is arranged in 16-row tiles of 8
// buses: tile rows 0-7 hold the real parts, 8-15 the imaginary parts.  The FP64
// MFMA leaves tile row g + 4r of output column j in lane 16g + j, register r, so
// a lane holds Re/Im of buses 8mt+g and 8mt+g+4 of its column.  The K index of
// the B operand uses the same order, and for k-step 4mt + r lane 16g + j must
// supply B[16mt + 4r + g][j], which is exactly the value it holds in register r
// of tile mt: the injection never leaves the lane.
#include "tpf_internal.h"

namespace tpf {

typedef double d4 __attribute__((ext_vector_type(4)));

template <typename IO>
__device__ __forceinline__ void ld_c(const IO *p, double &re, double &im) {
    re = (double)p[0];
    im = (double)p[1];
}

template <typename IO>
__device__ __forceinline__ void st_c(IO *p, double re, double im) {
    p[0] = (IO)re;
    p[1] = (IO)im;
}

// One workgroup of NW waves owns 16 column slots; wave w computes the output row
// tiles t = w' + NW q (w' its rotated role) of all 16 columns.  Per lane and
// owned tile q: v[q] = {Re V(8t+g), Re V(8t+g+4), Im V(8t+g), Im V(8t+g+4)} of the
// slot's column, s[q] the loads in the same order.  The injections conj(S./V)
// (B operand) of all buses live in LDS as Ib[16*MT rows][16 columns]; the lane
// that holds tile-row g + 4r of tile t writes row 16t + g + 4r, and k-step kt
// reads row 4kt + g, so both access patterns are contiguous 512-byte spans.
template <int TPW>
struct SlotState {
    d4 v[TPW], s[TPW];
};

// Writes the injection conj(S./V) of the lane's two buses 8t+g and 8t+g+4; for ZIP loads
// (Eq. (2)) alpha_P conj(S./V) + alpha_I conj(S) + alpha_Z conj(S) V, with the shares
// staged in LDS as zl[3][8 MT] (alpha_P, alpha_I, alpha_Z).
template <bool ZIP>
__device__ __forceinline__ void put_injection(double *Ib, int t, int lane, const d4 &vv, const d4 &ss,
                                              const double *zl, int MT) {
    const int g = lane >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double vr = vv[h], vi = vv[h + 2], sr = ss[h], si = ss[h + 2];
        const double inv = 1.0 / (vr * vr + vi * vi);
        double ir = (sr * vr + si * vi) * inv, ii = (sr * vi - si * vr) * inv;  // conj(S/V)
        if constexpr (ZIP) {
            const int b = 8 * t + g + 4 * h;
            const double ap = zl[b], ai = zl[8 * MT + b], az = zl[16 * MT + b];
            ir = ap * ir + ai * sr + az * (sr * vr + si * vi);
            ii = ap * ii - ai * si + az * (sr * vi - si * vr);
        }
        Ib[256 * t + 64 * h + lane] = ir;        // Re, row 16t+g+4h
        Ib[256 * t + 64 * (h + 2) + lane] = ii;  // Im, row 16t+g+8+4h
    }
}

// acc[q] += A(tile t_q, k-step kt) * B(k-step kt) over all k-steps, NV owned tiles.
// A fragments stream from L2 through a 4-deep register ring (loads issued three
// k-steps ahead of their MFMA); KT = 4 MT is a multiple of 4.  Aw points at this
// wave role's fragments, laid out [KT + pad][TPW][64].
template <int TPW, int NV>
__device__ __forceinline__ void sweep_product(d4 (&acc)[TPW], const double *__restrict__ Aw, const double *Ib,
                                              int MT, int lane) {
    const int KT = 4 * MT;
    constexpr int ST = TPW * 64;  // doubles per k-step
    // Uniform (scalar) fragment pointers, lane offset added last: the loads use a
    // scalar base and a 32-bit lane offset instead of per-lane 64-bit addresses.
    double r0[NV], r1[NV], r2[NV], r3[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        r0[q] = Aw[q * 64 + lane];
        r1[q] = Aw[ST + q * 64 + lane];
        r2[q] = Aw[2 * ST + q * 64 + lane];
    }
#pragma unroll 1
    for (int kt = 0; kt < KT; kt += 4) {
        const double *A3 = Aw + (size_t)(kt + 3) * ST;
#pragma unroll
        for (int q = 0; q < NV; ++q) r3[q] = A3[q * 64 + lane];
        const double b0 = Ib[kt * 64 + lane];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(r0[q], b0, acc[q], 0, 0, 0);
        {  // the fragment array is padded with zero k-steps: no bounds branch
            const double *A4 = Aw + (size_t)(kt + 4) * ST;
#pragma unroll
            for (int q = 0; q < NV; ++q) r0[q] = A4[q * 64 + lane];
        }
        const double b1 = Ib[(kt + 1) * 64 + lane];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(r1[q], b1, acc[q], 0, 0, 0);
        {
            const double *A5 = Aw + (size_t)(kt + 5) * ST;
#pragma unroll
            for (int q = 0; q < NV; ++q) r1[q] = A5[q * 64 + lane];
        }
        const double b2 = Ib[(kt + 2) * 64 + lane];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(r2[q], b2, acc[q], 0, 0, 0);
        {
            const double *A6 = Aw + (size_t)(kt + 6) * ST;
#pragma unroll
            for (int q = 0; q < NV; ++q) r2[q] = A6[q * 64 + lane];
        }
        const double b3 = Ib[(kt + 3) * 64 + lane];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(r3[q], b3, acc[q], 0, 0, 0);
    }
}

template <int TPW, int NW, bool ZIP, typename IO>
__global__ __launch_bounds__(NW * 64) void fpi_f64_kernel(
    const IO *__restrict__ S, IO *__restrict__ Vout, int32_t *__restrict__ iters_out,
    int8_t *__restrict__ status_out, const IO *__restrict__ V0, const double *__restrict__ A,
    const double *__restrict__ wv, int n, int MT, long long tau, double tol, int max_iter,
    unsigned long long *__restrict__ queue, const double *__restrict__ aP, const double *__restrict__ aI,
    const double *__restrict__ aZ) {
    extern __shared__ double lds[];
    double *Ib = lds;                                 // [16*MT][16]
    double *part = lds + 256 * MT;                    // [NW][16] partial max |dV|^2
    int *flag = reinterpret_cast<int *>(part + NW * 16);  // [NW][16] partial non-finite / guard flags
    unsigned long long *qb = reinterpret_cast<unsigned long long *>(flag + NW * 16);
    double *wl = reinterpret_cast<double *>(qb + 2);   // [2][8*MT] w staged once
    double *zl = wl + 16 * MT;                         // [3][8*MT] ZIP shares (ZIP only)

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int g = lane >> 4, j = lane & 15;
    const int tw = (wave + blockIdx.x) % NW;  // rotated role: balances tiles over SIMDs
    const int nv = (MT - tw + NW - 1) / NW;   // tiles owned by this wave (0..TPW)
    const double *Aw = A + (size_t)tw * (4 * MT + kFragPadSteps) * TPW * 64;

    SlotState<TPW> st;
    long long col = -1;
    int it = 0;
    bool exhausted = false;

    // Loads column c into the lanes of the slots with `take` (c < 0: empty slot),
    // writes their injections, and applies the warm-start guard across the workgroup.
    auto load_slots = [&](bool take, long long c) {
        int ok = 1;
        const bool real = take && c >= 0;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int t = tw + NW * q;
            if (q < nv && take) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int b = 8 * t + g + 4 * h;
                    double sr = 0.0, si = 0.0, vr = 1.0, vi = 0.0;
                    if (real && b < n) {
                        ld_c(S + 2 * (c * n + b), sr, si);
                        if (V0) {
                            ld_c(V0 + 2 * (c * n + b), vr, vi);
                            const double m2 = vr * vr + vi * vi;
                            ok &= (m2 >= 0.25 && m2 <= 2.25) ? 1 : 0;
                        }
                    }
                    st.s[q][h] = sr;
                    st.s[q][h + 2] = si;
                    st.v[q][h] = vr;
                    st.v[q][h + 2] = vi;
                }
            }
        }
        if (V0) {  // uniform: a warm start is kept only if every bus of the column passes
            ok &= __shfl_xor(ok, 16);
            ok &= __shfl_xor(ok, 32);
            if (g == 0) flag[wave * 16 + j] = ok;
            __syncthreads();
            int all = 1;
            for (int w = 0; w < NW; ++w) all &= flag[w * 16 + j];
            __syncthreads();
            if (real && !all) {
#pragma unroll
                for (int q = 0; q < TPW; ++q) st.v[q] = d4{1.0, 1.0, 0.0, 0.0};
            }
        }
        if (take) {
            col = c;
            it = 0;
#pragma unroll
            for (int q = 0; q < TPW; ++q)
                if (q < nv) put_injection<ZIP>(Ib, tw + NW * q, lane, st.v[q], st.s[q], zl, MT);
        }
    };

    for (int e = threadIdx.x; e < 16 * MT; e += NW * 64) wl[e] = wv[e];
    if constexpr (ZIP) {  // padding buses: no load, share 0
        for (int e = threadIdx.x; e < 8 * MT; e += NW * 64) {
            zl[e] = e < n ? aP[e] : 0.0;
            zl[8 * MT + e] = e < n ? aI[e] : 0.0;
            zl[16 * MT + e] = e < n && aZ ? aZ[e] : 0.0;
        }
    }
    // Initial fill: 16 consecutive queue entries per workgroup.
    if (threadIdx.x == 0) *qb = atomicAdd(queue, 16ull);
    __syncthreads();
    {
        const unsigned long long base = *qb;
        if (base + 16 >= (unsigned long long)tau) exhausted = true;
        const long long c = (long long)base + j;
        load_slots(true, c < tau ? c : -1);
    }
    __syncthreads();

    while (__ballot(col >= 0)) {
        // ---- product [Zr -Zi; Zi Zr] [Ir; Ii] for the owned row tiles
        d4 acc[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
        switch (nv) {
#define TPF_NV(k) \
    case k: if constexpr (k <= TPW) sweep_product<TPW, k>(acc, Aw, Ib, MT, lane); break;
            TPF_NV(1) TPF_NV(2) TPF_NV(3) TPF_NV(4) TPF_NV(5) TPF_NV(6)
#undef TPF_NV
            default: break;
        }
        __syncthreads();  // every wave has read Ib
        // ---- epilogue: V' = acc + w, partial max |V' - V|^2, next injections
        double dmax = 0.0;
        int bad = 0;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            if (q < nv) {
                const int t = tw + NW * q;
                const int b0 = 8 * t + g;
                const double w0r = wl[b0], w1r = wl[b0 + 4];
                const double w0i = wl[8 * MT + b0], w1i = wl[8 * MT + b0 + 4];
                const double n0r = acc[q][0] + w0r, n1r = acc[q][1] + w1r;
                const double n0i = acc[q][2] + w0i, n1i = acc[q][3] + w1i;
                const double d0r = n0r - st.v[q][0], d0i = n0i - st.v[q][2];
                const double d1r = n1r - st.v[q][1], d1i = n1i - st.v[q][3];
                const double e0 = d0r * d0r + d0i * d0i, e1 = d1r * d1r + d1i * d1i;
                bad |= !(e0 < HUGE_VAL) | !(e1 < HUGE_VAL);
                dmax = e0 > dmax ? e0 : dmax;
                dmax = e1 > dmax ? e1 : dmax;
                st.v[q] = d4{n0r, n1r, n0i, n1i};
                put_injection<ZIP>(Ib, t, lane, st.v[q], st.s[q], zl, MT);
            }
        }
        dmax = fmax(dmax, __shfl_xor(dmax, 16));
        dmax = fmax(dmax, __shfl_xor(dmax, 32));
        bad |= __shfl_xor(bad, 16);
        bad |= __shfl_xor(bad, 32);
        if (g == 0) {
            part[wave * 16 + j] = dmax;
            flag[wave * 16 + j] = bad;
        }
        __syncthreads();
        dmax = 0.0;
        bad = 0;
        for (int w = 0; w < NW; ++w) {
            dmax = fmax(dmax, part[w * 16 + j]);
            bad |= flag[w * 16 + j];
        }
        ++it;
        const bool conv = !bad && sqrt(dmax) < tol;
        const bool done = col >= 0 && (bad || conv || it >= max_iter);
        const unsigned long long dm = __ballot(done && g == 0);  // same in every wave
        if (dm) {
            if (done) {
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    if (q < nv) {
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int b = 8 * (tw + NW * q) + g + 4 * h;
                            if (b < n) st_c(Vout + 2 * (col * n + b), st.v[q][h], st.v[q][h + 2]);
                        }
                    }
                }
                if (wave == 0 && g == 0) {
                    iters_out[col] = it;
                    status_out[col] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
                }
            }
            const int cnt = __popcll(dm);
            if (threadIdx.x == 0) *qb = exhausted ? (unsigned long long)tau : atomicAdd(queue, (unsigned long long)cnt);
            __syncthreads();
            const unsigned long long base = *qb;
            if (base + cnt >= (unsigned long long)tau) exhausted = true;
            const int rank = __popcll(dm & ((1ull << j) - 1ull));
            const long long c = (long long)base + rank;
            load_slots(done, c < tau ? c : -1);
            __syncthreads();  // refilled injections visible; qb free again
        }
    }
}

// max_iter == 0: return the start voltages (guarded warm start or flat).
template <typename IO>
__global__ void start_only_kernel(int n, const IO *__restrict__ V0, long long tau, IO *__restrict__ V,
                                  int32_t *__restrict__ iters, int8_t *__restrict__ status) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < tau;
         c += (long long)gridDim.x * blockDim.x) {
        bool ok = V0 != nullptr;
        if (V0)
            for (int b = 0; b < n; ++b) {
                const double vr = (double)V0[2 * (c * n + b)], vi = (double)V0[2 * (c * n + b) + 1];
                const double m2 = vr * vr + vi * vi;
                ok = ok && (m2 >= 0.25 && m2 <= 2.25);
            }
        for (int b = 0; b < n; ++b) {
            V[2 * (c * n + b)] = ok ? V0[2 * (c * n + b)] : (IO)1;
            V[2 * (c * n + b) + 1] = ok ? V0[2 * (c * n + b) + 1] : (IO)0;
        }
        iters[c] = 0;
        status[c] = TPF_ST_MAX_ITER;
    }
}

__global__ void zero_u64_kernel(unsigned long long *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

static int num_cus() {
    static int cached[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) dev = 0;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 1;
        cached[dev] = v;
    }
    return cached[dev];
}

template <int TPW, int NW, bool ZIP, typename IO>
static int launch_rows_as(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                          int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                          unsigned long long *queue, hipStream_t stream) {
    const int MT = dn.MT;
    const size_t lds = (size_t)256 * MT * sizeof(double) + (size_t)NW * 16 * (sizeof(double) + sizeof(int)) + 16 +
                       (size_t)(ZIP ? 40 : 16) * MT * sizeof(double);
    auto kern = fpi_f64_kernel<TPW, NW, ZIP, IO>;
    if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NW * 64, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const long long blocks = std::min<long long>((long long)num_cus() * per_cu, (tau + 15) / 16);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), lds, stream, (const IO *)S, (IO *)V, iters,
                       status, (const IO *)V0, dn.A64, dn.w64, net.n, MT, (long long)tau, tol, max_iter, queue,
                       (const double *)dn.aP, (const double *)dn.aI, (const double *)dn.aZ);
    return TPF_OK;
}

template <int TPW, int NW, typename IO>
static int launch_rows(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                       int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                       unsigned long long *queue, hipStream_t stream) {
    if (dn.aP)
        return launch_rows_as<TPW, NW, true, IO>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
    return launch_rows_as<TPW, NW, false, IO>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
}

template <typename IO>
static int dispatch_rows(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                         int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                         unsigned long long *queue, hipStream_t stream) {
#define TPF_GO(T, W)                                                                                      \
    if (dn.TPW == T && dn.NW == W)                                                                        \
        return launch_rows<T, W, IO>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
    TPF_GO(1, 4) TPF_GO(1, 8) TPF_GO(2, 8) TPF_GO(3, 8) TPF_GO(4, 8) TPF_GO(5, 8)
#undef TPF_GO
    return fail(TPF_ERR_UNSUPPORTED, "register-resident sweep kernel: no instance for this network size");
}

int launch_fpi_small_f64(const tpf_network_s &net, const DeviceNet &dn, const void *S, int dtype, int64_t tau,
                         double tol, int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                         unsigned long long *queue, hipStream_t stream) {
    if (dtype == TPF_C128)
        return dispatch_rows<double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
    return dispatch_rows<float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
}

int launch_start_only(int n, const void *V0, int dtype, int64_t tau, void *V, int32_t *iters, int8_t *status,
                      hipStream_t stream) {
    const long long blocks = std::min<long long>(4096, (tau + 255) / 256);
    if (dtype == TPF_C128)
        hipLaunchKernelGGL(start_only_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, stream, n,
                           (const double *)V0, (long long)tau, (double *)V, iters, status);
    else
        hipLaunchKernelGGL(start_only_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, stream, n,
                           (const float *)V0, (long long)tau, (float *)V, iters, status);
    return TPF_OK;
}

int launch_zero_u64(unsigned long long *p, int count, hipStream_t stream) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3((count + 63) / 64), dim3(64), 0, stream, p, count);
    return TPF_OK;
}

}  // namespace tpf
