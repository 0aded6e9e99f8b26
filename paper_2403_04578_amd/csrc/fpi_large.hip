// Sweep path for networks too large for the register-resident kernels (the dense
// operator no longer fits one workgroup): every sweep of Algorithm 1 runs as
//   inject  I = conj(S./V) for the active columns (Eq. (3)), written as the B operand
//           [active][K] with K = interleaved Re/Im per bus;
//   gemm    V' = Z I + w on MFMA (64 x 64 output tiles, K staged through LDS), whose
//           epilogue updates the state in place and reduces max |V' - V| per column
//           with atomics;
//   finish  chunks of 256 active columns: sweep count, stopping rule, retirement to the
//           output, compaction of the active list for the next sweep and the next
//           sweep's injection (the first sweep's comes from its own kernel).
// FP64 mode keeps the state V in FP64; FP32 mode keeps the FP32 drop U = V - w.  Every
// sweep is queued without waiting on the device: the active counts stay there.
#include "tpf_internal.h"

#include <algorithm>

namespace tpf {

typedef double d4x __attribute__((ext_vector_type(4)));
typedef float f4x __attribute__((ext_vector_type(4)));

namespace {

template <typename T>
struct Acc;
template <>
struct Acc<double> {
    typedef d4x v4;
    __device__ static v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // FP64 16x16x4 output: lane group g holds tile rows g + 4 r
    __device__ static int row(int g, int r) { return g + 4 * r; }
};
template <>
struct Acc<float> {
    typedef f4x v4;
    __device__ static v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // FP32 16x16x4 output: lane group g holds tile rows 4 g + r
    __device__ static int row(int g, int r) { return 4 * g + r; }
};

// Row r of the operator (output order) -> (bus, part).  FP64: 16-row tiles of 8 buses,
// Re in rows 0-7, Im in rows 8-15 (so a lane holds both parts of a bus); FP32:
// interleaved Re/Im.  The K order is always interleaved.
template <typename T>
__device__ __forceinline__ void row_bus(int r, int &bus, int &part) {
    if constexpr (sizeof(T) == 8) {
        bus = 8 * (r >> 4) + (r & 7);
        part = (r >> 3) & 1;
    } else {
        bus = r >> 1;
        part = r & 1;
    }
}

// State x[col][2 n]: FP64 mode holds V, FP32 mode holds U = V - w.
template <typename T, typename IO>
__global__ void init_kernel(const IO *__restrict__ V0, const double *__restrict__ w, int n, long long tau, T *x,
                            int32_t *iters, long long *act, int *na, unsigned long long *dmax) {
    const long long c = blockIdx.x * 4LL + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= tau) return;
    int ok = V0 != nullptr;
    if (V0)
        for (int b = lane; b < n; b += 64) {
            const double vr = (double)V0[2 * (c * n + b)], vi = (double)V0[2 * (c * n + b) + 1];
            const double m2 = vr * vr + vi * vi;
            ok &= (m2 >= 0.25 && m2 <= 2.25) ? 1 : 0;
        }
    for (int off = 32; off > 0; off >>= 1) ok &= __shfl_xor(ok, off);
    for (int b = lane; b < n; b += 64) {
        double vr = 1.0, vi = 0.0;
        if (ok) vr = (double)V0[2 * (c * n + b)], vi = (double)V0[2 * (c * n + b) + 1];
        if constexpr (sizeof(T) == 8) {
            x[2 * (c * n + b)] = vr;
            x[2 * (c * n + b) + 1] = vi;
        } else {
            x[2 * (c * n + b)] = (T)(vr - w[2 * b]);
            x[2 * (c * n + b) + 1] = (T)(vi - w[2 * b + 1]);
        }
    }
    if (lane == 0) {
        iters[c] = 0;
        act[c] = c;
        dmax[c] = 0ull;
        if (c == 0) na[0] = (int)tau;
    }
}

// ZIP shares of Eq. (2) per PQ bus: all NULL for constant-power loads; aZ NULL when no
// bus has a constant-impedance share.
struct ZipShares {
    const double *aP, *aI, *aZ;
};

// I = conj(S./V), or for ZIP loads alpha_P conj(S./V) + alpha_I conj(S) + alpha_Z conj(S) V
// (the constant-impedance current, carried in the injection: the same fixed point as
// eliminating diag(alpha_Z s*) into Y_dd), at bus b of column c; zero on the K padding.
template <typename T, typename IO>
__device__ __forceinline__ void injection_at(const IO *__restrict__ S, const T *__restrict__ x,
                                             const double *__restrict__ w, int n, long long c, int b,
                                             const ZipShares zs, T &ir, T &ii) {
    ir = 0, ii = 0;
    if (b >= n) return;
    const double sr = (double)S[2 * (c * n + b)], si = (double)S[2 * (c * n + b) + 1];
    double vr = (double)x[2 * (c * n + b)], vi = (double)x[2 * (c * n + b) + 1];
    if constexpr (sizeof(T) == 4) vr += w[2 * b], vi += w[2 * b + 1];
    const double inv = 1.0 / (vr * vr + vi * vi);
    double jr = (sr * vr + si * vi) * inv, ji = (sr * vi - si * vr) * inv;
    if (zs.aP) {
        const double ap = zs.aP[b], ai = zs.aI[b];
        jr = ap * jr + ai * sr;
        ji = ap * ji - ai * si;
        if (zs.aZ) {
            const double az = zs.aZ[b];
            jr += az * (sr * vr + si * vi);
            ji += az * (sr * vi - si * vr);
        }
    }
    ir = (T)jr;
    ii = (T)ji;
}

// The first sweep's B operand [rows][KP]: row a = injection of column act[a] (zero past na).
template <typename T, typename IO>
__global__ void inject_kernel(const IO *__restrict__ S, const T *__restrict__ x, const double *__restrict__ w, int n,
                              int KP, const long long *__restrict__ act, const int *__restrict__ na, int rows,
                              const ZipShares zs, T *__restrict__ B) {
    const long long total = (long long)rows * KP;
    const int nact = *na;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total / 2;
         e += (long long)gridDim.x * blockDim.x) {
        const long long a = e / (KP / 2);
        const int b = (int)(e - a * (KP / 2));
        T ir = 0, ii = 0;
        if (a < nact) injection_at<T, IO>(S, x, w, n, act[a], b, zs, ir, ii);
        B[a * KP + 2 * b] = ir;
        B[a * KP + 2 * b + 1] = ii;
    }
}

// C tile [64 rows][64 active columns] = A[rows][K] B[cols][K]^T; epilogue on the state.
template <typename T>
__global__ __launch_bounds__(256) void gemm_kernel(const T *__restrict__ A, int KP, const T *__restrict__ B,
                                                   const long long *__restrict__ act, const int *__restrict__ na,
                                                   int row_blocks, const double *__restrict__ w, int n,
                                                   T *__restrict__ x, unsigned long long *__restrict__ dmax,
                                                   int *__restrict__ badf) {
    using Ops = Acc<T>;
    typedef typename Ops::v4 v4;
    const int nact = *na;
    const int ct = (nact + 63) / 64;
    __shared__ T As[2][64][17];  // two buffers: the next k-slab lands while this one is used
    __shared__ T Bs[2][64][17];
    __shared__ double red[2][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    // A fixed grid walks the tiles of the active columns (none once every column is done).
    // With A small enough to stay in L2 the row blocks of a column tile run back to back
    // (its B slab is fetched from HBM about once); otherwise column tiles run fastest and
    // the resident blocks share A's row block.
    const bool rows_fast = (size_t)row_blocks * 64 * KP * sizeof(T) <= ((size_t)2 << 20);
    for (int t = blockIdx.x; t < ct * row_blocks; t += gridDim.x) {
        const int c0 = (rows_fast ? t / row_blocks : t % ct) * 64;
        const int r0 = (rows_fast ? t % row_blocks : t / ct) * 64;
        v4 acc[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) acc[a][b] = v4{0, 0, 0, 0};
        const int rr = tid >> 2, kk = (tid & 3) * 4;
        const T *Ap = A + (size_t)(r0 + rr) * KP + kk, *Bp = B + (size_t)(c0 + rr) * KP + kk;
        // the next k-slab is fetched into registers while the current one is multiplied
        T pa0 = Ap[0], pa1 = Ap[1], pa2 = Ap[2], pa3 = Ap[3];
        T pb0 = Bp[0], pb1 = Bp[1], pb2 = Bp[2], pb3 = Bp[3];
        As[0][rr][kk] = pa0, As[0][rr][kk + 1] = pa1, As[0][rr][kk + 2] = pa2, As[0][rr][kk + 3] = pa3;
        Bs[0][rr][kk] = pb0, Bs[0][rr][kk + 1] = pb1, Bs[0][rr][kk + 2] = pb2, Bs[0][rr][kk + 3] = pb3;
        __syncthreads();
        int buf = 0;
        for (int k0 = 0; k0 < KP; k0 += 16) {
            const bool more = k0 + 16 < KP;
            if (more) {
                const int o = k0 + 16;
                pa0 = Ap[o], pa1 = Ap[o + 1], pa2 = Ap[o + 2], pa3 = Ap[o + 3];
                pb0 = Bp[o], pb1 = Bp[o + 1], pb2 = Bp[o + 2], pb3 = Bp[o + 3];
            }
    #pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                T af[2], bf[2];
    #pragma unroll
                for (int a = 0; a < 2; ++a) af[a] = As[buf][wr + 16 * a + j][4 * ks + g];
    #pragma unroll
                for (int b = 0; b < 2; ++b) bf[b] = Bs[buf][wc + 16 * b + j][4 * ks + g];
    #pragma unroll
                for (int a = 0; a < 2; ++a)
    #pragma unroll
                    for (int b = 0; b < 2; ++b) acc[a][b] = Ops::mma(af[a], bf[b], acc[a][b]);
            }
            if (more) {  // the other buffer: its last readers passed the previous barrier
                T *as = &As[buf ^ 1][rr][kk], *bs = &Bs[buf ^ 1][rr][kk];
                as[0] = pa0, as[1] = pa1, as[2] = pa2, as[3] = pa3;
                bs[0] = pb0, bs[1] = pb1, bs[2] = pb2, bs[3] = pb3;
            }
            __syncthreads();
            buf ^= 1;
        }
        // epilogue: each lane holds both parts of two buses (FP64 layout) or of two buses
        // (FP32 interleaved layout: rows 4g..4g+3 = Re/Im of two buses) of column j
    #pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int ac = c0 + wc + 16 * b + j;
            double emax = 0.0;
            int bad = 0;
            const bool live = ac < nact;
            const long long c = live ? act[ac] : 0;
    #pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int tile0 = r0 + wr + 16 * a;
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    // the two registers holding Re and Im of one bus
                    const int rre = sizeof(T) == 8 ? h : 2 * h, rim = sizeof(T) == 8 ? h + 2 : 2 * h + 1;
                    int bus, part;
                    row_bus<T>(tile0 + Ops::row(g, rre), bus, part);
                    if (live && bus < n) {
                        const double nr = (double)acc[a][b][rre] + (sizeof(T) == 8 ? w[2 * bus] : 0.0);
                        const double ni = (double)acc[a][b][rim] + (sizeof(T) == 8 ? w[2 * bus + 1] : 0.0);
                        T *xp = x + 2 * (c * n + bus);
                        const double dr = nr - (double)xp[0], di = ni - (double)xp[1];
                        const double e2 = dr * dr + di * di;
                        bad |= !(e2 < HUGE_VAL);
                        emax = e2 > emax ? e2 : emax;
                        xp[0] = (T)nr;
                        xp[1] = (T)ni;
                    }
                }
            }
            emax = fmax(emax, __shfl_xor(emax, 16));
            emax = fmax(emax, __shfl_xor(emax, 32));
            bad |= __shfl_xor(bad, 16);
            bad |= __shfl_xor(bad, 32);
            if (g == 0) {
                red[wave >> 1][wc + 16 * b + j] = emax;
                if (live && bad) atomicOr(badf + c, 1);
            }
        }
        __syncthreads();
        if (tid < 64 && c0 + tid < nact) {  // non-negative doubles order like their bit patterns
            const double e = fmax(red[0][tid], red[1][tid]);
            atomicMax(dmax + act[c0 + tid], (unsigned long long)__double_as_longlong(e));
        }
    }
}

// Tells the host that queues the sweeps that none is left to do (a store to pinned host
// memory, visible to the host without any wait on the device).
__device__ __forceinline__ void post_done(int *done_flag, int seq) {
    if (done_flag) __hip_atomic_store(done_flag, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Places of the staying columns of a chunk in the next list: a rank from the
// block's ballots and one atomic per chunk (a counter shared by every column of the sweep
// would serialise a million atomics).  Returns the slot, or -1 when `stay` is false.
__device__ __forceinline__ int chunk_slot(bool stay, int *counter, int *wsum, int *base) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long m = __ballot(stay);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    if (tid == 0) {
        const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        *base = tot ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    int off = *base;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    return stay ? off + rank : -1;
}

// Chunks of cpb active columns (a power of two, 4 to 256: fewer for wider networks, so
// that the per-column work of the second phase spreads over enough wavefronts): one
// thread per column for the convergence test (Eq. (3))
// and retirement, the staying columns' places in the next list, then one wave per column
// for the outputs of a retired one or the next sweep's B row (injection) of a staying
// one.  `cnt_next` was cleared a sweep earlier; `cnt_clear` (the count two sweeps back,
// read by no kernel still to run) is cleared for the sweep after next.
template <typename T, typename IO>
__global__ __launch_bounds__(256) void finish_kernel(
    const long long *__restrict__ act, const int *__restrict__ cnt, int *cnt_clear, const IO *__restrict__ S,
    const T *__restrict__ x, const double *__restrict__ w, int n, int KP, const ZipShares zs, double tol,
    int max_iter, unsigned long long *__restrict__ dmax,
    const int *__restrict__ badf, int32_t *iters, int8_t *status, IO *__restrict__ V,
    long long *__restrict__ act_next, int *cnt_next, T *__restrict__ B, int *done_flag, int seq, int cpb) {
    __shared__ long long col_s[256];
    __shared__ int slot_s[256];
    __shared__ int wsum[4], base_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nact = *cnt;
    if (blockIdx.x == 0 && tid == 0) {
        *cnt_clear = 0;
        if (nact == 0) post_done(done_flag, seq);
    }
    for (long long c0 = blockIdx.x * (long long)cpb; c0 < nact; c0 += (long long)gridDim.x * cpb) {  // block-uniform
        const long long a = c0 + tid;
        long long c = -1;
        bool stay = false;
        if (tid < cpb && a < nact) {
            c = act[a];
            const double e = __longlong_as_double((long long)dmax[c]);
            const int bad = badf[c];
            const int it = iters[c] + 1;
            const bool conv = !bad && sqrt(e) < tol;
            const bool done = bad || conv || it >= max_iter;
            iters[c] = it;
            dmax[c] = 0ull;
            if (done) status[c] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
            stay = !done;
        }
        const int slot = chunk_slot(stay, cnt_next, wsum, &base_s);
        if (stay) act_next[slot] = c;
        col_s[tid] = c;
        slot_s[tid] = slot;
        __syncthreads();
        for (int k = wave; k < cpb; k += 4) {
            const long long cc = col_s[k];
            if (cc < 0) break;  // past the active columns (wave-uniform)
            const int sl = slot_s[k];
            if (sl < 0) {
                for (int b = lane; b < n; b += 64) {
                    double vr = (double)x[2 * (cc * n + b)], vi = (double)x[2 * (cc * n + b) + 1];
                    if constexpr (sizeof(T) == 4) vr += w[2 * b], vi += w[2 * b + 1];
                    V[2 * (cc * n + b)] = (IO)vr;
                    V[2 * (cc * n + b) + 1] = (IO)vi;
                }
            } else {
                T *Br = B + (long long)sl * KP;
                for (int b = lane; b < KP / 2; b += 64) {
                    T ir, ii;
                    injection_at<T, IO>(S, x, w, n, cc, b, zs, ir, ii);
                    Br[2 * b] = ir;
                    Br[2 * b + 1] = ii;
                }
            }
        }
        __syncthreads();  // the chunk's tables are reused
    }
}

__global__ void zero_i32_kernel(int *p, long long count) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---- mixed precision (BF16 / FP16 operands) for large networks
//
// Each column follows the schedule of the register-resident mixed kernel: full
// low-precision sweeps U' = Z I until its step reaches the low-precision floor or
// stalls; one FP32 sweep (refine) that makes U = Z I_prev FP32-accurate; then
// low-precision sweeps on the change of the injection, U' = U + Z (I - I_prev), with a
// new refine once the distance they travelled makes their rounding matter.  Columns
// are kept in two lists per sweep, refine and low, each with its own product.

struct MixState {
    int it, ph, want;            // sweeps done; 0 = full low sweeps, 1 = difference sweeps; refine wanted
    float dprev, sumd, uref;     // previous step, steps since the last refine, max |U| seen
    float ks, inv;               // B scale 2^sB and product unscale 2^-(sB + sZ) (FP16); 1, 1 (BF16)
};

typedef short s8x __attribute__((ext_vector_type(8)));
typedef __bf16 bf8x __attribute__((ext_vector_type(8)));
typedef _Float16 h8x __attribute__((ext_vector_type(8)));

template <int MODE>
struct Low16;
template <>
struct Low16<TPF_MODE_MIXED_BF16> {
    static constexpr float u = 0.00390625f;  // 2^-8
    __device__ static uint32_t enc2(float a, float b) {
        return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)a) |
               ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)b) << 16);
    }
    __device__ static f4x mma(const uint4 &a, const uint4 &b, const f4x &c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8x, a), __builtin_bit_cast(bf8x, b), c,
                                                       0, 0, 0);
    }
};
template <>
struct Low16<TPF_MODE_MIXED_FP16> {
    static constexpr float u = 0.00048828125f;  // 2^-11
    __device__ static uint32_t enc2(float a, float b) {
        a = __builtin_amdgcn_fmed3f(a, -65504.f, 65504.f);
        b = __builtin_amdgcn_fmed3f(b, -65504.f, 65504.f);
        return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)a) |
               ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)b) << 16);
    }
    __device__ static f4x mma(const uint4 &a, const uint4 &b, const f4x &c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8x, a), __builtin_bit_cast(h8x, b), c, 0,
                                                      0, 0);
    }
};

// One wave per column: FP16 scale from max |S| (times zscale = max |alpha_P| + |alpha_I| +
// |alpha_Z| for ZIP loads) and the initial schedule state.
template <int MODE, typename IO>
__global__ void init_mix_kernel(const IO *__restrict__ S, int n, long long tau, int sZ, float zscale, MixState *ms,
                                unsigned *umax) {
    const long long c = blockIdx.x * 4LL + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= tau) return;
    float sm = 0.f;
    int sbad = 0;
    for (int b = lane; b < n; b += 64) {
        const double sr = fabs((double)S[2 * (c * n + b)]), si = fabs((double)S[2 * (c * n + b) + 1]);
        sbad |= !(sr + si < HUGE_VAL);
        sm = fmaxf(sm, (float)fmax(sr, si));
    }
    sm *= zscale;
    for (int off = 32; off > 0; off >>= 1) {
        sm = fmaxf(sm, __shfl_xor(sm, off));
        sbad |= __shfl_xor(sbad, off);
    }
    if (lane == 0) {
        int sB = 0;
        if (MODE == TPF_MODE_MIXED_FP16) {
            int e = 0;
            (void)frexpf(sm > 0.f && sm < 1e30f ? sm : 1.0f, &e);
            sB = 12 - e;  // max |S| 2^sB < 2^12: |I| 2^sB < 2^15 while |V| > 1/4
        }
        MixState m;
        m.it = m.ph = m.want = 0;
        m.dprev = m.sumd = m.uref = 0.f;
        m.ks = ldexpf(1.0f, sB);
        m.inv = ldexpf(1.0f, -(sB + (MODE == TPF_MODE_MIXED_FP16 ? sZ : 0)));
        // the FP16 saturation would clip a non-finite load; the unscale carries it into
        // the iterate instead, so the column ends NONFINITE
        if (sbad) m.inv = __builtin_nanf("");
        ms[c] = m;
        umax[c] = 0u;
    }
}

// alpha_P conj(S./V) + alpha_I conj(S) + alpha_Z conj(S) V for ZIP loads, else conj(S./V)
// (given as ir, ii).
__device__ __forceinline__ float2 zip_injection(float ir, float ii, float sr, float si, float vr, float vi,
                                                const ZipShares &zs, int b) {
    if (!zs.aP) return make_float2(ir, ii);
    const float ap = (float)zs.aP[b], ai = (float)zs.aI[b];
    float2 o = make_float2(ap * ir + ai * sr, ap * ii - ai * si);
    if (zs.aZ) {
        const float az = (float)zs.aZ[b];
        o.x += az * (sr * vr + si * vi);
        o.y += az * (sr * vi - si * vr);
    }
    return o;
}

// FP32 injection of column c at bus b (o = 2 (c n + b)) from U = V - w.
template <typename IO>
__device__ __forceinline__ float2 injection32(const IO *__restrict__ S, const float *__restrict__ U,
                                              const double *__restrict__ w, long long o, int b,
                                              const ZipShares &zs) {
    const float sr = (float)S[o], si = (float)S[o + 1];
    const float vr = (float)w[2 * b] + U[o], vi = (float)w[2 * b + 1] + U[o + 1];
    const float r = 1.0f / fmaxf(vr * vr + vi * vi, kMinV2);
    return zip_injection((sr * vr + si * vi) * r, (sr * vi - si * vr) * r, sr, si, vr, vi, zs, b);
}

// 16-bit B entry of a low-list column: I 2^sB on a full sweep (ph = 0), (I - I_prev) 2^sB
// on a difference sweep; I_prev <- I.
template <int MODE>
__device__ __forceinline__ uint32_t low_entry(float2 iz, float2 *ip, int ph, float ks) {
    float br = iz.x, bi = iz.y;
    if (ph) {
        const float2 p = *ip;
        br -= p.x;
        bi -= p.y;
    }
    *ip = iz;
    return Low16<MODE>::enc2(br * ks, bi * ks);
}

// The first sweep's B16 [rows][KP16] for the low list act[0..na).
template <int MODE, typename IO>
__global__ void inject_low_kernel(const IO *__restrict__ S, const float *__restrict__ U,
                                  const double *__restrict__ w, float *__restrict__ Ip,
                                  const MixState *__restrict__ ms, int n, int KP16,
                                  const long long *__restrict__ act, const int *__restrict__ na, int rows,
                                  const ZipShares zs,
                                  uint32_t *__restrict__ B) {
    const int nact = *na;
    const int half = KP16 / 2;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)rows * half;
         e += (long long)gridDim.x * blockDim.x) {
        const long long a = e / half;
        const int b = (int)(e - a * half);
        uint32_t out = 0u;
        if (a < nact && b < n) {
            const long long c = act[a], o = 2 * (c * n + b);
            out = low_entry<MODE>(injection32(S, U, w, o, b, zs), reinterpret_cast<float2 *>(Ip + o), ms[c].ph,
                                  ms[c].ks);
        }
        B[a * half + b] = out;
    }
}

// C tile [128 rows][128 active columns] = A16[rows][K] B16[cols][K]^T on 16x16x32 MFMA;
// epilogue U' = C inv (full) or U + C inv (difference), step and max |U'| per column.
template <int MODE>
__global__ __launch_bounds__(256) void gemm_low_kernel(const uint16_t *__restrict__ A, int KP16,
                                                       const uint16_t *__restrict__ B,
                                                       const long long *__restrict__ act, const int *__restrict__ na,
                                                       const MixState *__restrict__ ms, int n, float *__restrict__ U,
                                                       unsigned long long *__restrict__ dmax,
                                                       unsigned *__restrict__ umax, int *__restrict__ badf,
                                                       int row_blocks) {
    const int nact = *na;
    const int ct = (nact + 127) / 128;
    __shared__ uint4 As[2][128][5];  // 32 K values per row + one pad quad against bank conflicts;
    __shared__ uint4 Bs[2][128][5];  // two buffers: the next k-slab lands while this one is used
    __shared__ float redd[2][128], redu[2][128];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    // a fixed grid walks the tiles of the active columns, ordered as in gemm_kernel
    const bool rows_fast = (size_t)row_blocks * 128 * KP16 * 2 <= ((size_t)2 << 20);
    for (int t = blockIdx.x; t < ct * row_blocks; t += gridDim.x) {
        const int c0 = (rows_fast ? t / row_blocks : t % ct) * 128;
        const int r0 = (rows_fast ? t % row_blocks : t / ct) * 128;
        f4x acc[4][4];
    #pragma unroll
        for (int a = 0; a < 4; ++a)
    #pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = f4x{0.f, 0.f, 0.f, 0.f};
        // thread tid moves quads (row tid / 4, q) and (row 64 + tid / 4, q) of both operands
        const int lrow = tid >> 2, lq = tid & 3;
        const uint4 *Ap = reinterpret_cast<const uint4 *>(A + (size_t)(r0 + lrow) * KP16 + 8 * lq);
        const uint4 *Bp = reinterpret_cast<const uint4 *>(B + (size_t)(c0 + lrow) * KP16 + 8 * lq);
        const size_t half = (size_t)64 * KP16 / 8;  // 64 rows further, in quads
        // the next k-slab is fetched into registers while the current one is multiplied
        uint4 pa0 = Ap[0], pa1 = Ap[half], pb0 = Bp[0], pb1 = Bp[half];
        As[0][lrow][lq] = pa0;
        As[0][64 + lrow][lq] = pa1;
        Bs[0][lrow][lq] = pb0;
        Bs[0][64 + lrow][lq] = pb1;
        __syncthreads();
        int buf = 0;
        for (int k0 = 0; k0 < KP16; k0 += 32) {
            const bool more = k0 + 32 < KP16;
            if (more) {
                const int o = (k0 + 32) / 8;
                pa0 = Ap[o];
                pa1 = Ap[half + o];
                pb0 = Bp[o];
                pb1 = Bp[half + o];
            }
            uint4 af[4], bf[4];
    #pragma unroll
            for (int a = 0; a < 4; ++a) af[a] = As[buf][wr + 16 * a + j][g];
    #pragma unroll
            for (int b = 0; b < 4; ++b) bf[b] = Bs[buf][wc + 16 * b + j][g];
    #pragma unroll
            for (int a = 0; a < 4; ++a)
    #pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = Low16<MODE>::mma(af[a], bf[b], acc[a][b]);
            if (more) {  // the other buffer: its last readers passed the previous barrier
                As[buf ^ 1][lrow][lq] = pa0;
                As[buf ^ 1][64 + lrow][lq] = pa1;
                Bs[buf ^ 1][lrow][lq] = pb0;
                Bs[buf ^ 1][64 + lrow][lq] = pb1;
            }
            __syncthreads();
            buf ^= 1;
        }
        // lane group g holds rows 4g..4g+3 of each 16-row tile: Re/Im of two buses.  All of
        // the lane's state loads are issued before its first store: behind stores to
        // addresses the compiler cannot tell apart they would go out one at a time.
        long long cb[4];
        int phb[4];
        float invb[4];
        float2 oldv[4][4][2];
    #pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int ac = c0 + wc + 16 * b + j;
            const bool live = ac < nact;
            cb[b] = live ? act[ac] : -1;
            phb[b] = 0;
            invb[b] = 1.f;
            if (live) {
                phb[b] = ms[cb[b]].ph;
                invb[b] = ms[cb[b]].inv;
            }
    #pragma unroll
            for (int a = 0; a < 4; ++a)
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int bus = (r0 + wr + 16 * a + 4 * g + 2 * h) >> 1;
                    oldv[b][a][h] = make_float2(0.f, 0.f);
                    if (live && bus < n) oldv[b][a][h] = *reinterpret_cast<const float2 *>(U + 2 * (cb[b] * n + bus));
                }
        }
    #pragma unroll
        for (int b = 0; b < 4; ++b) {
            const bool live = cb[b] >= 0;
            const long long c = live ? cb[b] : 0;
            const int ph = phb[b];
            const float inv = invb[b];
            float emax = 0.f, umx = 0.f;
            int bad = 0;
    #pragma unroll
            for (int a = 0; a < 4; ++a) {
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int bus = (r0 + wr + 16 * a + 4 * g + 2 * h) >> 1;
                    if (live && bus < n) {
                        const float2 old = oldv[b][a][h];
                        const float pr = acc[a][b][2 * h] * inv, pi = acc[a][b][2 * h + 1] * inv;
                        const float nr = ph ? old.x + pr : pr, ni = ph ? old.y + pi : pi;
                        const float dr = nr - old.x, di = ni - old.y;
                        const float e2 = dr * dr + di * di;
                        bad |= !(e2 < HUGE_VALF);
                        emax = e2 > emax ? e2 : emax;
                        umx = fmaxf(umx, fmaxf(fabsf(nr), fabsf(ni)));
                        *reinterpret_cast<float2 *>(U + 2 * (c * n + bus)) = make_float2(nr, ni);
                    }
                }
            }
            emax = fmaxf(emax, __shfl_xor(emax, 16));
            emax = fmaxf(emax, __shfl_xor(emax, 32));
            umx = fmaxf(umx, __shfl_xor(umx, 16));
            umx = fmaxf(umx, __shfl_xor(umx, 32));
            bad |= __shfl_xor(bad, 16);
            bad |= __shfl_xor(bad, 32);
            if (g == 0) {
                redd[wave >> 1][wc + 16 * b + j] = emax;
                redu[wave >> 1][wc + 16 * b + j] = umx;
                if (live && bad) atomicOr(badf + c, 1);
            }
        }
        __syncthreads();
        if (tid < 128 && c0 + tid < nact) {  // non-negative values order like their bit patterns
            const long long c = act[c0 + tid];
            const double e = (double)fmaxf(redd[0][tid], redd[1][tid]);
            atomicMax(dmax + c, (unsigned long long)__double_as_longlong(e));
            atomicMax(umax + c, __float_as_uint(fmaxf(redu[0][tid], redu[1][tid])));
        }
    }
}

// Chunks of cpb columns (as finish_kernel) of the refine list (first) and the low list: one thread per
// column for the schedule update and retirement and the staying columns' places in the
// next refine or low list (chunk_slot), then one wave per column for the outputs of a
// retired one or its injection into the next sweep's B32 row (I) or B16 row (as
// low_entry), I_prev <- I.  cnt = {low, refine} counts of this sweep; cnt_next was cleared
// a sweep earlier; cnt_clear (the pair two sweeps back) is cleared for the sweep after next.
template <int MODE, typename IO>
__global__ __launch_bounds__(256) void finish_mixed_kernel(
    const long long *__restrict__ actR, const long long *__restrict__ actL, const int *__restrict__ cnt,
    int *cnt_clear, const IO *__restrict__ S, const float *__restrict__ U, const double *__restrict__ w, int n,
    int KP, int KP16, const ZipShares zs, float tol, int max_iter,
    unsigned long long *__restrict__ dmax, unsigned *__restrict__ umax, const int *__restrict__ badf,
    MixState *__restrict__ ms, int32_t *iters, int8_t *status, IO *__restrict__ V, float *__restrict__ Ip,
    long long *__restrict__ nextR, long long *__restrict__ nextL, int *cnt_next, float *__restrict__ B32,
    uint32_t *__restrict__ B16, int *done_flag, int seq, int cpb) {
    __shared__ long long col_s[256];
    __shared__ int slot_s[256];  // -1: retired; else the slot in the list kind_s names
    __shared__ int kind_s[256];  // 0: refine next, 1: low next
    __shared__ int ph_s[256];
    __shared__ float ks_s[256];
    __shared__ int wsum[4], base_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nl = cnt[0], nr = cnt[1];
    const long long total = (long long)nr + nl;
    if (blockIdx.x == 0 && tid < 2) cnt_clear[tid] = 0;
    if (blockIdx.x == 0 && tid == 0 && total == 0) post_done(done_flag, seq);
    constexpr float u = Low16<MODE>::u;
    const float theta = 4.0f * u, refresh = 6.7e-8f / u, margin = 1.0f + 8.0f * u;
    for (long long c0 = blockIdx.x * (long long)cpb; c0 < total; c0 += (long long)gridDim.x * cpb) {  // block-uniform
        const long long a = c0 + tid;
        long long c = -1;
        bool stay = false, want = false;
        MixState m{};
        if (tid < cpb && a < total) {
            const bool refine = a < nr;
            c = refine ? actR[a] : actL[a - nr];
            m = ms[c];
            const float d = (float)sqrt(__longlong_as_double((long long)dmax[c]));
            const float um = __uint_as_float(umax[c]);
            const int bad = badf[c];
            m.it += 1;
            bool conv = false;
            if (refine) {
                conv = d < tol;
                m.ph = 1;
                m.want = 0;
                m.sumd = 0.f;
            } else if (m.ph == 0) {
                m.uref = fmaxf(m.uref, um);
                if (!m.want && (d <= theta * m.uref || (m.it >= 2 && d > 0.5f * m.dprev))) m.want = 1;
            } else {
                conv = d * margin < tol;
                m.sumd += d;
                if (!m.want && m.sumd > refresh) m.want = 1;
            }
            m.dprev = d;
            const bool done = bad || conv || m.it >= max_iter;
            iters[c] = m.it;
            dmax[c] = 0ull;
            umax[c] = 0u;
            ms[c] = m;
            if (done) status[c] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
            stay = !done;
            want = m.want != 0;
        }
        const int sr = chunk_slot(stay && want, cnt_next + 1, wsum, &base_s);
        __syncthreads();  // wsum and base_s are reused
        const int sl = chunk_slot(stay && !want, cnt_next, wsum, &base_s);
        if (sr >= 0) nextR[sr] = c;
        if (sl >= 0) nextL[sl] = c;
        col_s[tid] = c;
        slot_s[tid] = sr >= 0 ? sr : sl;
        kind_s[tid] = sr >= 0 ? 0 : 1;
        ph_s[tid] = m.ph;
        ks_s[tid] = m.ks;
        __syncthreads();
        for (int k = wave; k < cpb; k += 4) {
            const long long cc = col_s[k];
            if (cc < 0) break;  // past the active columns (wave-uniform)
            const int slot = slot_s[k];
            if (slot < 0) {
                for (int b = lane; b < n; b += 64) {
                    V[2 * (cc * n + b)] = (IO)(w[2 * b] + (double)U[2 * (cc * n + b)]);
                    V[2 * (cc * n + b) + 1] = (IO)(w[2 * b + 1] + (double)U[2 * (cc * n + b) + 1]);
                }
            } else if (kind_s[k] == 0) {
                float2 *Br = reinterpret_cast<float2 *>(B32 + (long long)slot * KP);
                for (int b = lane; b < KP / 2; b += 64) {
                    float2 iz = make_float2(0.f, 0.f);
                    if (b < n) {
                        const long long o = 2 * (cc * n + b);
                        iz = injection32(S, U, w, o, b, zs);
                        *reinterpret_cast<float2 *>(Ip + o) = iz;
                    }
                    Br[b] = iz;
                }
            } else {
                const int ph = ph_s[k];
                const float kss = ks_s[k];
                uint32_t *Br = B16 + (long long)slot * (KP16 / 2);
                for (int b = lane; b < KP16 / 2; b += 64) {
                    uint32_t out = 0u;
                    if (b < n) {
                        const long long o = 2 * (cc * n + b);
                        out = low_entry<MODE>(injection32(S, U, w, o, b, zs), reinterpret_cast<float2 *>(Ip + o),
                                              ph, kss);
                    }
                    Br[b] = out;
                }
            }
        }
        __syncthreads();  // the chunk's tables are reused
    }
}

}  // namespace

// Whether a sweep of solve `seq` already found every column retired: the sweeps queued
// after it would all exit at once, so the host queues no more.  A read of pinned host
// memory; it never waits for the device.
static bool all_retired(const DeviceNet &dn, int seq) {
    return dn.done_host && __atomic_load_n(dn.done_host, __ATOMIC_ACQUIRE) == seq;
}

// Columns per finish chunk: about 16,384 buses' worth, a power of two in [4, 256] (one
// atomic per chunk keeps a million-column sweep from serialising on the list counter,
// and small chunks keep a few wide columns spread over many wavefronts).
static int finish_chunk(int n) {
    int c = 4;
    while (c < 256 && 2 * c * n <= 16384) c *= 2;
    return c;
}

// Fixed grids of the queued sweeps: enough blocks to fill the chip, few enough that a
// sweep with nothing left to do costs little.
constexpr int64_t kGemmGrid = 1024, kFinishGrid = 1024;

// Grid of a persistent GEMM: at most kGemmGrid blocks and no more than are resident at
// once (CUs x blocks per CU).  Its blocks share the tiles evenly, so blocks beyond the
// resident ones would start only after others had finished all of theirs and run the
// kernel's second half at a fraction of the occupancy (the 16-bit GEMM, three blocks per
// CU for its 43 KB of LDS, took twice as long with 1,024 blocks).
template <typename Kernel>
static int64_t gemm_grid(Kernel kernel, int64_t tiles) {
    int dev = 0, cus = 256, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kernel, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return std::max<int64_t>(1, std::min<int64_t>({kGemmGrid, (int64_t)cus * per_cu, tiles}));
}

// Workspace of the large path: state [tau][2n] (T), B operand [tau rounded to 64][KP] (T),
// dmax [tau] (u64), bad flags [tau] (int), two active lists [tau] (i64), counters.
// Mixed modes add I_prev [tau][2n] (FP32), the 16-bit B operand [tau rounded to 128][KP16],
// per-column schedule state and max |U| [tau], and two more active lists.
size_t large_workspace_bytes(int n, int64_t tau, int mode) {
    const size_t ts = mode == TPF_MODE_FP64 ? 8 : 4;
    const size_t KP = (size_t)(2 * n + 15) / 16 * 16;
    const size_t rows = (size_t)(tau + 63) / 64 * 64;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t bytes = al((size_t)tau * 2 * n * ts) + al(rows * KP * ts) + al((size_t)tau * 8) + al((size_t)tau * 4) +
                   2 * al((size_t)tau * 8) + 256;
    if (mode == TPF_MODE_MIXED_BF16 || mode == TPF_MODE_MIXED_FP16) {
        const size_t K16 = (size_t)(2 * n + 31) / 32 * 32, rows16 = (size_t)(tau + 127) / 128 * 128;
        bytes += al((size_t)tau * 2 * n * 4) + al(rows16 * K16 * 2) + al((size_t)tau * sizeof(MixState)) +
                 al((size_t)tau * 4) + 2 * al((size_t)tau * 8);
    }
    return bytes;
}

template <typename T, typename IO>
static int run_large(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                     int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status, void *ws,
                     hipStream_t st) {
    const int n = net.n;
    const int KP = (2 * n + 15) / 16 * 16;
    const int64_t rows = (tau + 63) / 64 * 64;
    const int MP = sizeof(T) == 8 ? dn.MPL64 : dn.MPL32;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    char *p = static_cast<char *>(ws);
    T *x = reinterpret_cast<T *>(p);
    p += al((size_t)tau * 2 * n * sizeof(T));
    T *B = reinterpret_cast<T *>(p);
    p += al((size_t)rows * KP * sizeof(T));
    auto *dmax = reinterpret_cast<unsigned long long *>(p);
    p += al((size_t)tau * 8);
    int *badf = reinterpret_cast<int *>(p);
    p += al((size_t)tau * 4);
    long long *act[2];
    act[0] = reinterpret_cast<long long *>(p);
    p += al((size_t)tau * 8);
    act[1] = reinterpret_cast<long long *>(p);
    p += al((size_t)tau * 8);
    int *cnt = reinterpret_cast<int *>(p);  // three active counts in rotation
    const T *A = sizeof(T) == 8 ? (const T *)(const void *)dn.AL64 : (const T *)(const void *)dn.AL32;
    const double *w = dn.wl;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)std::min<int64_t>(65536, (tau + 255) / 256)), dim3(256), 0, st,
                       badf, (long long)tau);
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, cnt, 3LL);
    hipLaunchKernelGGL((init_kernel<T, IO>), dim3((unsigned)((tau + 3) / 4)), dim3(256), 0, st, (const IO *)V0, w, n,
                       (long long)tau, x, iters, act[0], cnt, dmax);
    hipLaunchKernelGGL((inject_kernel<T, IO>), dim3((unsigned)std::min<long long>(65536, (rows * KP / 2 + 255) / 256)),
                       dim3(256), 0, st, (const IO *)S, x, w, n, KP, act[0], cnt, (int)rows, ZipShares{dn.aP, dn.aI, dn.aZ}, B);
    // Every sweep is queued without waiting, with grids fixed from tau: the active counts
    // stay on the device (three of them in rotation: read, appended, cleared) and the
    // kernels of a sweep with no active column exit at once.  Queueing stops early when
    // the device has already posted that none is left (all_retired).
    const int row_blocks = MP / 64;
    const unsigned g_mm = (unsigned)gemm_grid(gemm_kernel<T>, (int64_t)row_blocks * (rows / 64));
    const int cpb = finish_chunk(n);
    const unsigned g_fin = (unsigned)std::min<int64_t>(kFinishGrid, (tau + cpb - 1) / cpb);
    const int seq = ++dn.solve_seq;
    for (int sweep = 0; sweep < max_iter; ++sweep) {
        if (all_retired(dn, seq)) break;
        const int cur = sweep & 1;
        int *cr = cnt + sweep % 3, *cn = cnt + (sweep + 1) % 3, *cz = cnt + (sweep + 2) % 3;
        hipLaunchKernelGGL((gemm_kernel<T>), dim3(g_mm), dim3(256), 0, st, A, KP, B, act[cur], cr, row_blocks, w, n, x,
                           dmax, badf);
        hipLaunchKernelGGL((finish_kernel<T, IO>), dim3(g_fin), dim3(256), 0, st, act[cur], cr, cz, (const IO *)S, x, w,
                           n, KP, ZipShares{dn.aP, dn.aI, dn.aZ}, tol, max_iter, dmax, badf, iters, status, (IO *)V, act[cur ^ 1], cn,
                           B, dn.done_dev, seq, cpb);
    }
    return TPF_OK;
}

template <int MODE, typename IO>
static int run_large_mixed(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                           int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status, void *ws,
                           hipStream_t st) {
    const int n = net.n;
    const int KP = (2 * n + 15) / 16 * 16, K16 = (2 * n + 31) / 32 * 32;
    const int64_t rows = (tau + 63) / 64 * 64, rows16 = (tau + 127) / 128 * 128;
    const int MP = dn.MPL32;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    // same carve as large_workspace_bytes: the FP32 part first, then the mixed additions
    char *p = static_cast<char *>(ws);
    float *U = reinterpret_cast<float *>(p);
    p += al((size_t)tau * 2 * n * 4);
    float *B32 = reinterpret_cast<float *>(p);
    p += al((size_t)rows * KP * 4);
    auto *dmax = reinterpret_cast<unsigned long long *>(p);
    p += al((size_t)tau * 8);
    int *badf = reinterpret_cast<int *>(p);
    p += al((size_t)tau * 4);
    long long *actL[2], *actR[2];
    actL[0] = reinterpret_cast<long long *>(p);
    p += al((size_t)tau * 8);
    actL[1] = reinterpret_cast<long long *>(p);
    p += al((size_t)tau * 8);
    int *cnt = reinterpret_cast<int *>(p);  // [3 pairs in rotation][0: low, 1: refine]
    p += 256;
    float *Ip = reinterpret_cast<float *>(p);
    p += al((size_t)tau * 2 * n * 4);
    uint16_t *B16 = reinterpret_cast<uint16_t *>(p);
    p += al((size_t)rows16 * K16 * 2);
    MixState *ms = reinterpret_cast<MixState *>(p);
    p += al((size_t)tau * sizeof(MixState));
    unsigned *umax = reinterpret_cast<unsigned *>(p);
    p += al((size_t)tau * 4);
    actR[0] = reinterpret_cast<long long *>(p);
    p += al((size_t)tau * 8);
    actR[1] = reinterpret_cast<long long *>(p);
    const double *w = dn.wl;
    const uint16_t *A16 = MODE == TPF_MODE_MIXED_FP16 ? dn.ALh : dn.ALbf;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)std::min<int64_t>(65536, (tau + 255) / 256)), dim3(256), 0, st,
                       badf, (long long)tau);
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, cnt, 6LL);
    hipLaunchKernelGGL((init_kernel<float, IO>), dim3((unsigned)((tau + 3) / 4)), dim3(256), 0, st, (const IO *)V0, w,
                       n, (long long)tau, U, iters, actL[0], cnt, dmax);
    hipLaunchKernelGGL((init_mix_kernel<MODE, IO>), dim3((unsigned)((tau + 3) / 4)), dim3(256), 0, st, (const IO *)S,
                       n, (long long)tau, dn.sZ, dn.aP ? dn.zscale : 1.0f, ms, umax);
    hipLaunchKernelGGL((inject_low_kernel<MODE, IO>),
                       dim3((unsigned)std::min<long long>(65536, (rows16 * K16 / 2 + 255) / 256)), dim3(256), 0, st,
                       (const IO *)S, U, w, Ip, ms, n, K16, actL[0], cnt, (int)rows16, ZipShares{dn.aP, dn.aI, dn.aZ},
                       reinterpret_cast<uint32_t *>(B16));
    // Queued at once as in run_large; counts in pairs {low, refine}, three pairs in rotation.
    const unsigned g_r = (unsigned)gemm_grid(gemm_kernel<float>, (int64_t)(MP / 64) * (rows / 64));
    const unsigned g_l = (unsigned)gemm_grid(gemm_low_kernel<MODE>, (int64_t)(MP / 128) * (rows16 / 128));
    const int cpb = finish_chunk(n);
    const unsigned g_fin = (unsigned)std::min<int64_t>(kFinishGrid, (tau + cpb - 1) / cpb);
    const int seq = ++dn.solve_seq;
    for (int sweep = 0; sweep < max_iter; ++sweep) {
        if (all_retired(dn, seq)) break;
        const int cur = sweep & 1;
        int *cc = cnt + 2 * (sweep % 3), *cn = cnt + 2 * ((sweep + 1) % 3), *cz = cnt + 2 * ((sweep + 2) % 3);
        if (sweep > 0)  // the first sweep has no refine list
            hipLaunchKernelGGL((gemm_kernel<float>), dim3(g_r), dim3(256), 0, st, dn.AL32, KP, B32, actR[cur], cc + 1,
                               MP / 64, w, n, U, dmax, badf);
        hipLaunchKernelGGL((gemm_low_kernel<MODE>), dim3(g_l), dim3(256), 0, st, A16, K16, B16, actL[cur], cc, ms, n,
                           U, dmax, umax, badf, MP / 128);
        hipLaunchKernelGGL((finish_mixed_kernel<MODE, IO>), dim3(g_fin), dim3(256), 0, st, actR[cur], actL[cur], cc, cz,
                           (const IO *)S, U, w, n, KP, K16, ZipShares{dn.aP, dn.aI, dn.aZ}, (float)tol, max_iter, dmax, umax, badf, ms,
                           iters, status, (IO *)V, Ip, actR[cur ^ 1], actL[cur ^ 1], cn, B32,
                           reinterpret_cast<uint32_t *>(B16), dn.done_dev, seq, cpb);
    }
    return TPF_OK;
}

int launch_fpi_large(const tpf_network_s &net, const DeviceNet &dn, int mode, const void *S, int dtype, int64_t tau,
                     double tol, int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status, void *ws,
                     hipStream_t st) {
    if (!dn.AL64) return fail(TPF_ERR_UNSUPPORTED, "large-network operator not staged");
    if (mode == TPF_MODE_FP64)
        return dtype == TPF_C128 ? run_large<double, double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, ws, st)
                                 : run_large<double, float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, ws, st);
    if (mode == TPF_MODE_FP32)
        return dtype == TPF_C128 ? run_large<float, double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, ws, st)
                                 : run_large<float, float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, ws, st);
    if (!dn.ALbf) return fail(TPF_ERR_UNSUPPORTED, "16-bit large-network operator not staged");
    if (mode == TPF_MODE_MIXED_BF16)
        return dtype == TPF_C128
                   ? run_large_mixed<TPF_MODE_MIXED_BF16, double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, ws, st)
                   : run_large_mixed<TPF_MODE_MIXED_BF16, float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, ws, st);
    return dtype == TPF_C128
               ? run_large_mixed<TPF_MODE_MIXED_FP16, double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, ws, st)
               : run_large_mixed<TPF_MODE_MIXED_FP16, float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, ws, st);
}

}  // namespace tpf
