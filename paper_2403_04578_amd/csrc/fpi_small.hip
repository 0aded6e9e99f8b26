// Persistent FP64 sweep kernel for networks with up to 128 PQ buses.
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

// Per lane: v[mt] = {Re V(8mt+g), Re V(8mt+g+4), Im V(8mt+g), Im V(8mt+g+4)} of the
// slot's column, s[mt] the loads in the same order, acc[mt] the MFMA output.  The
// injections conj(S./V) (the B operand) go to a lane-private LDS array
// [4*MT k-steps][64 lanes] so that the k-loop can index them at run time.
template <int MT, typename IO>
__device__ __forceinline__ void put_injection(double *iL, int lane, int mt, const d4 &vv, const d4 &ss) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double vr = vv[h], vi = vv[h + 2], sr = ss[h], si = ss[h + 2];
        const double inv = 1.0 / (vr * vr + vi * vi);
        iL[(4 * mt + h) * 64 + lane] = (sr * vr + si * vi) * inv;      // Re conj(S/V)
        iL[(4 * mt + h + 2) * 64 + lane] = (sr * vi - si * vr) * inv;  // Im conj(S/V)
    }
}

template <int MT, typename IO>
__global__ __launch_bounds__(256, 1) void fpi_small_f64_kernel(
    const IO *__restrict__ S, IO *__restrict__ Vout, int32_t *__restrict__ iters_out,
    int8_t *__restrict__ status_out, const IO *__restrict__ V0, const double *__restrict__ A,
    const double *__restrict__ wv, int n, long long tau, double tol, int max_iter,
    unsigned long long *__restrict__ queue) {
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, j = lane & 15;
    double *iL = lds + (size_t)wave * (MT * 4 * 64);
    constexpr int KT = 4 * MT;

    d4 v[MT], s[MT];
    long long col = -1;
    int it = 0;
    bool exhausted = false;

    // Slot (re)fill: lanes with `take` load column c (c < 0: leave the slot empty).
    auto load_slot = [&](bool take, long long c) {
        bool ok = true;
        const bool real = take && c >= 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int b = 8 * mt + g + 4 * h;
                double sr = 0.0, si = 0.0, vr = 1.0, vi = 0.0;
                if (real && b < n) {
                    ld_c(S + 2 * (c * n + b), sr, si);
                    if (V0) {
                        ld_c(V0 + 2 * (c * n + b), vr, vi);
                        const double m2 = vr * vr + vi * vi;
                        ok = ok && (m2 >= 0.25 && m2 <= 2.25);
                    }
                }
                if (take) {
                    s[mt][h] = sr;
                    s[mt][h + 2] = si;
                    v[mt][h] = vr;
                    v[mt][h + 2] = vi;
                }
            }
        }
        // A warm start is used only if every bus of the column passes the guard.
        int okc = ok ? 1 : 0;
        okc &= __shfl_xor(okc, 16);
        okc &= __shfl_xor(okc, 32);
        if (real && V0 && !okc) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) v[mt] = d4{1.0, 1.0, 0.0, 0.0};
        }
        if (take) {
            col = c;
            it = 0;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) put_injection<MT, IO>(iL, lane, mt, v[mt], s[mt]);
        }
    };

    // Initial fill: 16 consecutive queue entries per wave.
    {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(queue, 16ull);
        base = __shfl(base, 0);
        if (base + 16 >= (unsigned long long)tau) exhausted = true;
        const long long c = (long long)base + j;
        load_slot(true, c < tau ? c : -1);
    }

    while (__ballot(col >= 0)) {
        // ---- sweep: acc = [Zr -Zi; Zi Zr] [Ir; Ii], A fragments prefetched one k-step ahead
        d4 acc[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) acc[mt] = d4{0.0, 0.0, 0.0, 0.0};
        double a0[MT], a1[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a0[mt] = A[mt * 64 + lane];
#pragma unroll 1
        for (int kt = 0; kt < KT; kt += 2) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a1[mt] = A[((kt + 1) * MT + mt) * 64 + lane];
            const double b0 = iL[kt * 64 + lane];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[mt], b0, acc[mt], 0, 0, 0);
            if (kt + 2 < KT) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a0[mt] = A[((kt + 2) * MT + mt) * 64 + lane];
            }
            const double b1 = iL[(kt + 1) * 64 + lane];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[mt], b1, acc[mt], 0, 0, 0);
        }
        // ---- epilogue: V' = acc + w, per-column max |V' - V|, next injections
        double dmax = 0.0;
        int bad = 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int b0 = 8 * mt + g;
            const double w0r = wv[b0], w1r = wv[b0 + 4];
            const double w0i = wv[8 * MT + b0], w1i = wv[8 * MT + b0 + 4];
            const double n0r = acc[mt][0] + w0r, n1r = acc[mt][1] + w1r;
            const double n0i = acc[mt][2] + w0i, n1i = acc[mt][3] + w1i;
            const double d0r = n0r - v[mt][0], d0i = n0i - v[mt][2];
            const double d1r = n1r - v[mt][1], d1i = n1i - v[mt][3];
            const double e0 = d0r * d0r + d0i * d0i, e1 = d1r * d1r + d1i * d1i;
            bad |= !(e0 < HUGE_VAL) | !(e1 < HUGE_VAL);
            dmax = e0 > dmax ? e0 : dmax;
            dmax = e1 > dmax ? e1 : dmax;
            v[mt] = d4{n0r, n1r, n0i, n1i};
            put_injection<MT, IO>(iL, lane, mt, v[mt], s[mt]);
        }
        dmax = fmax(dmax, __shfl_xor(dmax, 16));
        dmax = fmax(dmax, __shfl_xor(dmax, 32));
        bad |= __shfl_xor(bad, 16);
        bad |= __shfl_xor(bad, 32);
        ++it;
        const bool conv = !bad && sqrt(dmax) < tol;
        const bool done = col >= 0 && (bad || conv || it >= max_iter);

        const unsigned long long dm = __ballot(done && g == 0);
        if (dm) {
            if (done) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int b = 8 * mt + g + 4 * h;
                        if (b < n) st_c(Vout + 2 * (col * n + b), v[mt][h], v[mt][h + 2]);
                    }
                if (g == 0) {
                    iters_out[col] = it;
                    status_out[col] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
                }
            }
            const int cnt = __popcll(dm);
            unsigned long long base = (unsigned long long)tau;
            if (!exhausted) {
                if (lane == 0) base = atomicAdd(queue, (unsigned long long)cnt);
                base = __shfl(base, 0);
                if (base + cnt >= (unsigned long long)tau) exhausted = true;
            }
            const int rank = __popcll(dm & ((1ull << j) - 1ull));
            const long long c = (long long)base + rank;
            load_slot(done, c < tau ? c : -1);
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

template <int MT, typename IO>
static int launch_mt(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                     int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                     unsigned long long *queue, hipStream_t stream) {
    const size_t lds = (size_t)4 * MT * 4 * 64 * sizeof(double);
    static bool attr_set = false;
    if (!attr_set) {
        if (hipFuncSetAttribute((const void *)fpi_small_f64_kernel<MT, IO>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
        attr_set = true;
    }
    const long long waves_needed = (tau + 15) / 16;
    const long long blocks = std::min<long long>((long long)num_cus(), (waves_needed + 3) / 4);
    hipLaunchKernelGGL((fpi_small_f64_kernel<MT, IO>), dim3((unsigned)blocks), dim3(256), lds, stream,
                       (const IO *)S, (IO *)V, iters, status, (const IO *)V0, dn.A64, dn.w64, net.n,
                       (long long)tau, tol, max_iter, queue);
    return TPF_OK;
}

template <typename IO>
static int dispatch_mt(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                       int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                       unsigned long long *queue, hipStream_t stream) {
#define TPF_CASE(M) \
    case M: return launch_mt<M, IO>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
    switch (dn.MT) {
        TPF_CASE(1) TPF_CASE(2) TPF_CASE(3) TPF_CASE(4) TPF_CASE(5) TPF_CASE(6) TPF_CASE(7) TPF_CASE(8)
        TPF_CASE(9) TPF_CASE(10) TPF_CASE(11) TPF_CASE(12) TPF_CASE(13) TPF_CASE(14) TPF_CASE(15) TPF_CASE(16)
        default: return fail(TPF_ERR_UNSUPPORTED, "small-network kernel: tile count out of range");
    }
#undef TPF_CASE
}

int launch_fpi_small_f64(const tpf_network_s &net, const DeviceNet &dn, const void *S, int dtype, int64_t tau,
                         double tol, int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                         unsigned long long *queue, hipStream_t stream) {
    if (dtype == TPF_C128)
        return dispatch_mt<double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
    return dispatch_mt<float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
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
