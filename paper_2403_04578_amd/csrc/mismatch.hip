// FP64 power-balance mismatch of a batch of voltage solutions.
//
// Eq. (1) of the paper gives -i_d = Y_ds v_s + Y_dd v for the demand nodes, so a
// load drawing S must satisfy S = v .* conj(i_d), i.e.
//     m = S + V .* conj(Y_ds v_s + Y_dd V) = 0,
// reported per column as max_i |m_i| (NaN if any term is NaN).  ZIP loads of Eq. (2)
// draw S (alpha_P + alpha_I V + alpha_Z |V|^2) in place of S.
//
// Tiled kernel: a workgroup takes CB columns at a time (their V are contiguous),
// copies their V into LDS with coalesced loads, and then TPC = 256 / CB consecutive
// threads share a column's buses, walking the sparse row of Y_dd (a radial feeder has
// about three nonzeros per row, kept in LDS) against the LDS copy of V; the column's
// maximum is a shuffle reduction over those lanes.  Only S and V cross HBM, once.
// Complex values move through LDS as one 16-byte access each (two 8-byte accesses at a
// 16-byte stride doubled the bank conflicts, which took about half of the LDS time), and
// the reduction runs over |m|^2 with one square root per column (a column whose
// mismatch exceeds 1e154 pu would read inf).
// Networks whose CSR or columns do not fit LDS use one wavefront per column with the
// CSR in global memory.
#include "tpf_internal.h"

namespace tpf {

namespace {

struct MismatchArgs {
    const int32_t *rowptr;
    const int32_t *colidx;
    const double *yval;  // [nnz][2]
    const double *cval;  // [n][2]
    const double *aI, *aP;  // ZIP shares [n], or NULL for constant-power loads
    const double *aZ;       // constant-impedance share [n], or NULL
    double *out;         // [tau]
};

// The power a load draws: S for constant power, S (alpha_P + alpha_I V + alpha_Z |V|^2)
// for ZIP loads (the constant-impedance current alpha_Z S* V draws alpha_Z S |V|^2).
__device__ __forceinline__ void load_power(const MismatchArgs &mm, int b, double sr, double si, double vr, double vi,
                                           double &lr, double &li) {
    lr = sr;
    li = si;
    if (mm.aP) {
        double ap = mm.aP[b];
        const double ai = mm.aI[b];
        if (mm.aZ) ap += mm.aZ[b] * (vr * vr + vi * vi);
        lr = sr * ap + ai * (sr * vr - si * vi);
        li = si * ap + ai * (sr * vi + si * vr);
    }
}

__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// |m_b| = |S_b + V_b conj(c_b + sum_k (Y_dd)_bk V_k)| for one bus; `vk(k, re, im)` fetches V_k.
template <typename F>
__device__ __forceinline__ double bus_mismatch(const MismatchArgs &mm, int b, double sr, double si, double vr,
                                               double vi, F vk) {
    double ar = mm.cval[2 * b], ai = mm.cval[2 * b + 1];
    for (int e = mm.rowptr[b]; e < mm.rowptr[b + 1]; ++e) {
        double xr, xi;
        vk(mm.colidx[e], xr, xi);
        const double yr = mm.yval[2 * e], yi = mm.yval[2 * e + 1];
        ar += yr * xr - yi * xi;
        ai += yr * xi + yi * xr;
    }
    double lr, li;
    load_power(mm, b, sr, si, vr, vi, lr, li);
    const double mr = lr + vr * ar + vi * ai;
    const double mi = li + vi * ar - vr * ai;
    return sqrt(mr * mr + mi * mi);
}

// Complex pairs as clang vectors: S and V stream through once (nontemporal loads).
template <typename IO>
struct Pair2 {
    typedef IO T __attribute__((ext_vector_type(2)));
};

constexpr int kCsrLdsCap = 96 * 1024;  // three-phase Y_dd has ~9x the nonzeros of a single-phase one
constexpr int kTileVBytes = 64 * 1024;  // LDS for the tile's copy of V
constexpr int kBatch = 8;               // independent loads issued before their data is used

inline size_t csr_lds_bytes(int n, int nnz) {
    return ((size_t)16 * nnz + 16 * (size_t)n + 4 * (size_t)(n + 1) + 4 * (size_t)nnz + 15) / 16 * 16;
}

// Columns per tile: 16 (16 threads per column) up to 256 buses, 8 up to 512, 4 up to 1024.
inline int tile_columns(int n) { return n <= 256 ? 16 : n <= 512 ? 8 : n <= 1024 ? 4 : 0; }

typedef double d2 __attribute__((ext_vector_type(2)));  // (Re, Im) in one LDS access

// LONG: rows of Y_dd long enough (a three-phase network's 3x3 blocks: about nine nonzeros
// per row) that the walk is unrolled by four, so that the dependent LDS loads of the column
// index and then the voltage overlap across nonzeros (3.0 -> 2.4 ms for a 100-bus
// three-phase year; the three nonzeros of a single-phase row keep the plain loop, which
// the unrolled one slowed from 0.28 to 0.32 ms).
template <typename IO, int CB, bool LONG>
__global__ __launch_bounds__(256) void mismatch_tile_kernel(const IO *__restrict__ S, const IO *__restrict__ V, int n,
                                                            long long tau, int nnz, const MismatchArgs mm) {
    typedef typename Pair2<IO>::T P2;
    constexpr int TPC = 256 / CB;  // threads per column: consecutive lanes of one wavefront
    extern __shared__ double smem[];
    double *Vs = smem;                            // [CB n][2]
    double *yv = Vs + 2 * (size_t)CB * n;         // [nnz][2]
    double *cv = yv + 2 * nnz;                    // [n][2]
    int32_t *rp = reinterpret_cast<int32_t *>(cv + 2 * n);  // [n+1]
    int32_t *ci = rp + n + 1;                     // [nnz]
    const int tid = threadIdx.x;
    for (int i = tid; i < 2 * nnz; i += 256) yv[i] = mm.yval[i];
    for (int i = tid; i < 2 * n; i += 256) cv[i] = mm.cval[i];
    for (int i = tid; i <= n; i += 256) rp[i] = mm.rowptr[i];
    for (int i = tid; i < nnz; i += 256) ci[i] = mm.colidx[i];
    const int cl = tid / TPC, part = tid - cl * TPC;
    for (long long c0 = (long long)blockIdx.x * CB; c0 < tau; c0 += (long long)gridDim.x * CB) {
        const int cols = (int)((tau - c0) < CB ? (tau - c0) : CB);
        const int total = cols * n;
        const P2 *Vg = reinterpret_cast<const P2 *>(V) + c0 * n;
        __syncthreads();  // the previous tile's readers are done with Vs
        for (int e0 = tid; e0 < total; e0 += 256 * kBatch) {
            P2 v[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int e = e0 + 256 * u;
                if (e < total) v[u] = __builtin_nontemporal_load(Vg + e);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int e = e0 + 256 * u;
                if (e < total) reinterpret_cast<d2 *>(Vs)[e] = d2{(double)v[u].x, (double)v[u].y};
            }
        }
        __syncthreads();
        // thread (column cl, part) takes buses part, part + TPC, ...
        double worst = 0.0;
        if (cl < cols) {
            const P2 *Sc = reinterpret_cast<const P2 *>(S) + (c0 + cl) * n;
            const double *vc = Vs + 2 * (size_t)cl * n;
            for (int b0 = part; b0 < n; b0 += TPC * kBatch) {
                P2 s[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int b = b0 + TPC * u;
                    if (b < n) s[u] = __builtin_nontemporal_load(Sc + b);
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int b = b0 + TPC * u;
                    if (b < n) {
                        const d2 c = reinterpret_cast<const d2 *>(cv)[b];
                        double ar = c.x, ai = c.y;
                        const int k1 = rp[b + 1];
                        int k = rp[b];
                        if constexpr (LONG) {  // four nonzeros' loads in flight at once
                            for (; k + 4 <= k1; k += 4) {
                                int q[4];
                                d2 y[4], x[4];
#pragma unroll
                                for (int u = 0; u < 4; ++u) q[u] = ci[k + u];
#pragma unroll
                                for (int u = 0; u < 4; ++u) {
                                    y[u] = reinterpret_cast<const d2 *>(yv)[k + u];
                                    x[u] = reinterpret_cast<const d2 *>(vc)[q[u]];
                                }
#pragma unroll
                                for (int u = 0; u < 4; ++u) {
                                    ar += y[u].x * x[u].x - y[u].y * x[u].y;
                                    ai += y[u].x * x[u].y + y[u].y * x[u].x;
                                }
                            }
                        }
                        for (; k < k1; ++k) {
                            const int q = ci[k];
                            const d2 y = reinterpret_cast<const d2 *>(yv)[k], x = reinterpret_cast<const d2 *>(vc)[q];
                            ar += y.x * x.x - y.y * x.y;
                            ai += y.x * x.y + y.y * x.x;
                        }
                        const d2 v = reinterpret_cast<const d2 *>(vc)[b];
                        const double vr = v.x, vi = v.y;
                        double lr, li;
                        load_power(mm, b, (double)s[u].x, (double)s[u].y, vr, vi, lr, li);
                        const double mr = lr + vr * ar + vi * ai;
                        const double mi = li + vi * ar - vr * ai;
                        worst = nanmax(worst, mr * mr + mi * mi);
                    }
                }
            }
        }
#pragma unroll
        for (int off = TPC / 2; off > 0; off >>= 1) worst = nanmax(worst, __shfl_xor(worst, off));
        if (part == 0 && cl < cols) mm.out[c0 + cl] = sqrt(worst);
    }
}

template <typename IO>
__global__ __launch_bounds__(256) void mismatch_wave_kernel(const IO *__restrict__ S, const IO *__restrict__ V, int n,
                                                            long long tau, const MismatchArgs mm) {
    const int lane = threadIdx.x & 63;
    const long long wid = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const long long nw = (long long)gridDim.x * 4;
    for (long long c = wid; c < tau; c += nw) {
        const IO *vc = V + 2 * c * n;
        const IO *sc = S + 2 * c * n;
        double worst = 0.0;
        for (int i = lane; i < n; i += 64) {
            worst = nanmax(worst, bus_mismatch(mm, i, (double)sc[2 * i], (double)sc[2 * i + 1], (double)vc[2 * i],
                                               (double)vc[2 * i + 1], [&](int k, double &xr, double &xi) {
                                                   xr = (double)vc[2 * k];
                                                   xi = (double)vc[2 * k + 1];
                                               }));
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) worst = nanmax(worst, __shfl_xor(worst, off));
        if (lane == 0) mm.out[c] = worst;
    }
}

template <typename IO, int CB>
int launch_tile(const MismatchArgs &mm, int nnz, size_t csr, const void *S, const void *V, int n, int64_t tau,
                int cus, hipStream_t st) {
    const size_t lds = (size_t)CB * n * 16 + csr;
    auto k = nnz >= 6 * n ? mismatch_tile_kernel<IO, CB, true> : mismatch_tile_kernel<IO, CB, false>;
    if (hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    const long long blocks = std::max<long long>(1, std::min<long long>((long long)cus * per_cu, (tau + CB - 1) / CB));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), lds, st, (const IO *)S, (const IO *)V, n, (long long)tau,
                       nnz, mm);
    return TPF_OK;
}

template <typename IO>
int launch_io(const MismatchArgs &mm, int nnz, const void *S, const void *V, int n, int64_t tau, hipStream_t st) {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t csr = csr_lds_bytes(n, nnz);
    const int CB = tile_columns(n);
    if (CB && csr <= (size_t)kCsrLdsCap && (size_t)CB * n * 16 <= (size_t)kTileVBytes) {
        if (CB == 16) return launch_tile<IO, 16>(mm, nnz, csr, S, V, n, tau, cus, st);
        if (CB == 8) return launch_tile<IO, 8>(mm, nnz, csr, S, V, n, tau, cus, st);
        return launch_tile<IO, 4>(mm, nnz, csr, S, V, n, tau, cus, st);
    }
    const long long blocks = std::max<long long>(1, std::min<long long>((long long)cus * 16, (tau + 3) / 4));
    hipLaunchKernelGGL(mismatch_wave_kernel<IO>, dim3((unsigned)blocks), dim3(256), 0, st, (const IO *)S,
                       (const IO *)V, n, (long long)tau, mm);
    return TPF_OK;
}

}  // namespace

int launch_mismatch_f64(const tpf_network_s &net, const DeviceNet &dn, const void *S, const void *V, int dtype,
                        int64_t tau, double *out, hipStream_t stream) {
    const MismatchArgs mm{dn.rowptr, dn.colidx, dn.yval, dn.cval, dn.aI, dn.aP, dn.aZ, out};
    const int nnz = (int)net.colidx.size();
    if (dtype == TPF_C128) return launch_io<double>(mm, nnz, S, V, net.n, tau, stream);
    return launch_io<float>(mm, nnz, S, V, net.n, tau, stream);
}

}  // namespace tpf
