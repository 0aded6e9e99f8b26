// FP32 and mixed-precision sweep kernels for networks with up to 128 PQ buses.
//
// The iteration is Algorithm 1's V <- Z conj(S./V) + w (Sec. IV-A), carried in
// FP32 as the drop U = V - w, so that the state keeps ~1e-9 pu of absolute
// precision while |V| ~ 1.  Three forms share this kernel:
//
//   TPF_MODE_FP32        every sweep: U' = Z I on 16x16x4 FP32 MFMA;
//   TPF_MODE_MIXED_BF16  low sweeps on 16x16x32 BF16 MFMA (FP32 accumulation),
//                        refine sweeps on FP32 MFMA;
//   TPF_MODE_MIXED_FP16  low sweeps on 16x16x32 FP16 MFMA with a power-of-two
//                        scale per column, refine sweeps as the three-term FP16
//                        split Zh Ih + Zh Il + Zl Ih (~22-bit products).
//
// A mixed column goes through (i) full low-precision sweeps U' = Z I until its
// step size reaches the low-precision floor, (ii) one refine sweep that makes
// U = Z I_prev hold to FP32 accuracy, then (iii) low-precision sweeps on the
// change of the injection, U' = U + Z (I - I_prev).  These compute the same
// iterates as (i) -- Z I = Z I_prev + Z (I - I_prev) -- but the rounding error
// of a low-precision product is now relative to the step, so the contraction of
// the map refines the iterate down to FP32 accuracy.  Convergence (d < tol) is
// only declared on a refine sweep or a difference sweep.  A refine sweep is
// repeated when the distance travelled by difference sweeps grows large enough
// for their rounding to matter.
//
// Workgroup: 8 waves own 16 column slots as a batch.  Wave role tw multiplies
// output row tiles tw + 8 q.  The 16-bit A fragments of its tiles stay in
// registers for the whole kernel; FP32 A fragments stream from L2 through a
// register ring.  B operands live in LDS as [16 columns][K], written by the
// epilogue lanes (4 consecutive K rows per lane) and read as MFMA fragments.
// Columns retire individually; the batch is refilled when all 16 are done, so
// that one refine sweep serves the whole batch.
#include "tpf_internal.h"

namespace tpf {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));

template <typename IO>
__device__ __forceinline__ void ldc(const IO *p, double &re, double &im) {
    re = (double)p[0];
    im = (double)p[1];
}

template <int MODE>
struct LowOps;
template <>
struct LowOps<TPF_MODE_MIXED_BF16> {
    typedef b8 frag;
    typedef b4 quad;
    static constexpr float u = 0.00390625f;  // 2^-8
    __device__ static f4 mma(const frag &a, const frag &b, const f4 &c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static quad cvt(const f4 &x) { return quad{(__bf16)x[0], (__bf16)x[1], (__bf16)x[2], (__bf16)x[3]}; }
};
template <>
struct LowOps<TPF_MODE_MIXED_FP16> {
    typedef h8 frag;
    typedef h4 quad;
    static constexpr float u = 0.00048828125f;  // 2^-11
    __device__ static f4 mma(const frag &a, const frag &b, const f4 &c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    __device__ static quad cvt(const f4 &x) {
        return quad{(_Float16)x[0], (_Float16)x[1], (_Float16)x[2], (_Float16)x[3]};
    }
};
template <>
struct LowOps<TPF_MODE_FP32> : LowOps<TPF_MODE_MIXED_BF16> {};

// conj(S./V) = conj(S) V / |V|^2 for the two buses (Re, Im, Re, Im) of a lane's tile.
__device__ __forceinline__ f4 injection(const f4 &s, float w0r, float w0i, float w1r, float w1i, const f4 &u) {
    const float v0r = w0r + u[0], v0i = w0i + u[1], v1r = w1r + u[2], v1i = w1i + u[3];
    const float i0 = 1.0f / (v0r * v0r + v0i * v0i), i1 = 1.0f / (v1r * v1r + v1i * v1i);
    return f4{(s[0] * v0r + s[1] * v0i) * i0, (s[0] * v0i - s[1] * v0r) * i0,
              (s[2] * v1r + s[3] * v1i) * i1, (s[2] * v1i - s[3] * v1r) * i1};
}

__device__ __forceinline__ float amax4(const f4 &x) {
    return fmaxf(fmaxf(fabsf(x[0]), fabsf(x[1])), fmaxf(fabsf(x[2]), fabsf(x[3])));
}

template <int TPW, int NW, int KTL, int MODE, typename IO>
__global__ __launch_bounds__(NW * 64) void fpi_mixed_kernel(
    const IO *__restrict__ S, IO *__restrict__ Vout, int32_t *__restrict__ iters_out,
    int8_t *__restrict__ status_out, const IO *__restrict__ V0, const float *__restrict__ A32,
    const uint16_t *__restrict__ Alow, const uint16_t *__restrict__ Alo, const double *__restrict__ wv, int n,
    int MT, int sZ, long long tau, float tol, int max_iter, unsigned long long *__restrict__ queue) {
    using L = LowOps<MODE>;
    typedef typename L::frag frag;
    typedef typename L::quad quad;
    constexpr bool kMixed = MODE != TPF_MODE_FP32;
    constexpr bool kSplit = MODE == TPF_MODE_MIXED_FP16;
    constexpr bool kF32Refine = !kSplit;
    constexpr int KPL = 32 * KTL + 8;  // 16-bit B row stride (halves)
    const int KP32 = 16 * MT + 4;      // FP32 B row stride (floats)

    extern __shared__ __align__(16) unsigned char smem[];
    float *B32 = reinterpret_cast<float *>(smem);                             // [16][KP32]
    uint16_t *Bh = reinterpret_cast<uint16_t *>(B32 + (kF32Refine ? 16 * KP32 : 0));  // [16][KPL]
    uint16_t *Bl = Bh + 16 * KPL;                                             // [16][KPL] (FP16 split)
    float *pd = reinterpret_cast<float *>(Bl + (kSplit ? 16 * KPL : 0));      // [NW][16] max |dU|^2
    float *pu = pd + NW * 16;                                                 // [NW][16] max |U|
    float *pm = pu + NW * 16;                                                 // [NW][16] max |B|
    int *pb = reinterpret_cast<int *>(pm + NW * 16);                          // [NW][16] flags
    float *wl = reinterpret_cast<float *>(pb + NW * 16);                      // [2][8 MT]
    unsigned long long *qb = reinterpret_cast<unsigned long long *>(wl + 16 * MT + 2);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, j = lane & 15;
    const int tw = (wave + blockIdx.x) % NW;
    const int nv = (MT - tw + NW - 1) / NW;

    // zero the B operands once (K padding rows stay zero), stage w as FP32
    for (int e = threadIdx.x; e < (kF32Refine ? 16 * KP32 : 0); e += NW * 64) B32[e] = 0.0f;
    for (int e = threadIdx.x; e < 16 * KPL * (kSplit ? 2 : 1); e += NW * 64) Bh[e] = 0;
    for (int e = threadIdx.x; e < 16 * MT; e += NW * 64) wl[e] = (float)wv[e];

    // 16-bit A fragments of the owned tiles, resident for the whole kernel.
    frag Af[TPW][KTL], Ag[kSplit ? TPW : 1][kSplit ? KTL : 1];
    if constexpr (kMixed) {
#pragma unroll
        for (int q = 0; q < TPW; ++q)
#pragma unroll
            for (int kt = 0; kt < KTL; ++kt) {
                if (q < nv) {
                    const size_t idx = ((((size_t)tw * TPW + q) * KTL + kt) * 64 + lane) * 8;
                    Af[q][kt] = *reinterpret_cast<const frag *>(Alow + idx);
                    if constexpr (kSplit) Ag[q][kt] = *reinterpret_cast<const frag *>(Alo + idx);
                }
            }
    }
    const float *Aw = A32 + (size_t)tw * (4 * MT + kFragPadSteps) * TPW * 64;

    f4 U[TPW], Sv[TPW], Ip[TPW], In[TPW];
    long long col = -1;
    int it = 0, ph = 0, want = 0, wait = 0;  // ph: 0 full low sweeps, 1 difference sweeps
    float dprev = 0.f, sumd = 0.f, uref = 0.f;
    int sB = 0;          // power-of-two scale exponent of this column's B operand
    bool precise = !kMixed;  // kind of the next sweep (workgroup-uniform)
    bool exhausted = false;
    const float theta_k = 4.0f * L::u;                       // switch when d < theta_k max|U|
    const float refresh = 6.7e-8f / L::u;                    // distance budget of difference sweeps
    const float margin = 1.0f + 8.0f * L::u;
    __syncthreads();

    auto wbus = [&](int t, float &w0r, float &w0i, float &w1r, float &w1i) {
        const int b0 = 8 * t + 2 * g;
        w0r = wl[b0];
        w1r = wl[b0 + 1];
        w0i = wl[8 * MT + b0];
        w1i = wl[8 * MT + b0 + 1];
    };

    // Batch (re)fill: all 16 slots from the queue.  Returns false when the queue is empty.
    auto refill = [&]() -> bool {
        if (threadIdx.x == 0) *qb = exhausted ? (unsigned long long)tau : atomicAdd(queue, 16ull);
        __syncthreads();
        const unsigned long long base = *qb;
        __syncthreads();
        if (base >= (unsigned long long)tau) {
            exhausted = true;
            return false;
        }
        if (base + 16 >= (unsigned long long)tau) exhausted = true;
        const long long c = (long long)base + j;
        col = c < tau ? c : -1;
        int ok = 1;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            double s[4] = {0, 0, 0, 0}, v[4] = {1, 0, 1, 0};
            if (q < nv && col >= 0) {
                const int t = tw + NW * q;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int b = 8 * t + 2 * g + h;
                    if (b < n) {
                        ldc(S + 2 * (col * n + b), s[2 * h], s[2 * h + 1]);
                        if (V0) {
                            ldc(V0 + 2 * (col * n + b), v[2 * h], v[2 * h + 1]);
                            const double m2 = v[2 * h] * v[2 * h] + v[2 * h + 1] * v[2 * h + 1];
                            ok &= (m2 >= 0.25 && m2 <= 2.25) ? 1 : 0;
                        }
                    }
                }
            }
            Sv[q] = f4{(float)s[0], (float)s[1], (float)s[2], (float)s[3]};
            if (q < nv) {
                const int t = tw + NW * q, b0 = 8 * t + 2 * g;
                U[q] = f4{(float)(v[0] - wv[b0]), (float)(v[1] - wv[8 * MT + b0]), (float)(v[2] - wv[b0 + 1]),
                          (float)(v[3] - wv[8 * MT + b0 + 1])};
            } else {
                U[q] = f4{0, 0, 0, 0};
            }
        }
        if (V0) {  // a warm start is kept only if every bus of the column passes the guard
            ok &= __shfl_xor(ok, 16);
            ok &= __shfl_xor(ok, 32);
            if (g == 0) pb[wave * 16 + j] = ok;
            __syncthreads();
            int all = 1;
            for (int w = 0; w < NW; ++w) all &= pb[w * 16 + j];
            __syncthreads();
            if (!all) {  // flat start V = 1 + j0
#pragma unroll
                for (int q = 0; q < TPW; ++q)
                    if (q < nv) {
                        const int t = tw + NW * q, b0 = 8 * t + 2 * g;
                        U[q] = f4{(float)(1.0 - wv[b0]), (float)(-wv[8 * MT + b0]), (float)(1.0 - wv[b0 + 1]),
                                  (float)(-wv[8 * MT + b0 + 1])};
                    }
            }
        }
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            float w0r = 1, w0i = 0, w1r = 1, w1i = 0;
            if (q < nv) wbus(tw + NW * q, w0r, w0i, w1r, w1i);
            In[q] = injection(Sv[q], w0r, w0i, w1r, w1i, U[q]);
            Ip[q] = In[q];
        }
        it = 0;
        ph = 0;
        want = 0;
        wait = 0;
        dprev = 0.f;
        sumd = 0.f;
        uref = 0.f;
        precise = !kMixed;
        return true;
    };

    // Writes the B operand of the next sweep from In (full form) or In - Ip (difference form).
    auto prepare_b = [&](bool diff) {
        f4 Bv[TPW];
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            Bv[q] = diff ? In[q] - Ip[q] : In[q];
            if (q < nv) m = fmaxf(m, amax4(Bv[q]));
            Ip[q] = In[q];
        }
        if (precise && kF32Refine) {
#pragma unroll
            for (int q = 0; q < TPW; ++q)
                if (q < nv)
                    *reinterpret_cast<f4 *>(B32 + j * KP32 + 16 * (tw + NW * q) + 4 * g) = Bv[q];
            return;
        }
        if constexpr (MODE == TPF_MODE_MIXED_FP16) {
            // per-column power of two putting max |B| just below 2^14
            m = fmaxf(m, __shfl_xor(m, 16));
            m = fmaxf(m, __shfl_xor(m, 32));
            if (g == 0) pm[wave * 16 + j] = m;
            __syncthreads();
            float mm = 0.f;
            for (int w = 0; w < NW; ++w) mm = fmaxf(mm, pm[w * 16 + j]);
            int e = 0;
            (void)frexpf(mm > 0.f ? mm : 1.0f, &e);
            sB = 14 - e;
        } else {
            sB = 0;
        }
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            if (q < nv) {
                const f4 x = f4{ldexpf(Bv[q][0], sB), ldexpf(Bv[q][1], sB), ldexpf(Bv[q][2], sB),
                                ldexpf(Bv[q][3], sB)};
                const quad hq = L::cvt(x);
                const int off = j * KPL + 16 * (tw + NW * q) + 4 * g;
                *reinterpret_cast<quad *>(Bh + off) = hq;
                if constexpr (kSplit) {
                    const f4 r = x - f4{(float)hq[0], (float)hq[1], (float)hq[2], (float)hq[3]};
                    *reinterpret_cast<quad *>(Bl + off) = L::cvt(r);
                }
            }
        }
    };

    if (!refill()) return;
    prepare_b(false);
    __syncthreads();

    while (true) {
        // ---- product
        f4 acc[TPW];
#pragma unroll
        for (int q = 0; q < TPW; ++q) acc[q] = f4{0, 0, 0, 0};
        if (precise && kF32Refine) {
            const int KT = 4 * MT;
            constexpr int ST = TPW * 64;
            float r0[TPW], r1[TPW];
#pragma unroll
            for (int q = 0; q < TPW; ++q) r0[q] = Aw[q * 64 + lane];
#pragma unroll 1
            for (int kt = 0; kt < KT; kt += 2) {
#pragma unroll
                for (int q = 0; q < TPW; ++q) r1[q] = Aw[(size_t)(kt + 1) * ST + q * 64 + lane];
                const float b0 = B32[j * KP32 + 4 * kt + g];
#pragma unroll
                for (int q = 0; q < TPW; ++q)
                    if (q < nv) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(r0[q], b0, acc[q], 0, 0, 0);
#pragma unroll
                for (int q = 0; q < TPW; ++q) r0[q] = Aw[(size_t)(kt + 2) * ST + q * 64 + lane];
                const float b1 = B32[j * KP32 + 4 * (kt + 1) + g];
#pragma unroll
                for (int q = 0; q < TPW; ++q)
                    if (q < nv) acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(r1[q], b1, acc[q], 0, 0, 0);
            }
        } else if constexpr (kMixed) {
#pragma unroll
            for (int kt = 0; kt < KTL; ++kt) {
                const frag bh = *reinterpret_cast<const frag *>(Bh + j * KPL + 32 * kt + 8 * g);
#pragma unroll
                for (int q = 0; q < TPW; ++q)
                    if (q < nv) acc[q] = L::mma(Af[q][kt], bh, acc[q]);
                if constexpr (kSplit) {
                    if (precise) {
                        const frag bl = *reinterpret_cast<const frag *>(Bl + j * KPL + 32 * kt + 8 * g);
#pragma unroll
                        for (int q = 0; q < TPW; ++q)
                            if (q < nv) {
                                acc[q] = L::mma(Af[q][kt], bl, acc[q]);
                                acc[q] = L::mma(Ag[q][kt], bh, acc[q]);
                            }
                    }
                }
            }
        }
        // ---- epilogue: new drop, step size, next injection
        const bool full = precise || ph == 0;
        const float inv = (precise && kF32Refine) ? 1.0f : ldexpf(1.0f, -(sB + (kSplit ? sZ : 0)));
        float dmax = 0.f, umax = 0.f;
        int bad = 0;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            if (q < nv) {
                const f4 p = acc[q] * inv;
                const f4 un = full ? p : U[q] + p;
                const f4 dd = un - U[q];
                const float e0 = dd[0] * dd[0] + dd[1] * dd[1], e1 = dd[2] * dd[2] + dd[3] * dd[3];
                bad |= !(e0 < INFINITY) | !(e1 < INFINITY);
                dmax = fmaxf(dmax, fmaxf(e0, e1));
                umax = fmaxf(umax, amax4(un));
                U[q] = un;
                float w0r, w0i, w1r, w1i;
                wbus(tw + NW * q, w0r, w0i, w1r, w1i);
                In[q] = injection(Sv[q], w0r, w0i, w1r, w1i, un);
            }
        }
        dmax = fmaxf(dmax, __shfl_xor(dmax, 16));
        dmax = fmaxf(dmax, __shfl_xor(dmax, 32));
        umax = fmaxf(umax, __shfl_xor(umax, 16));
        umax = fmaxf(umax, __shfl_xor(umax, 32));
        bad |= __shfl_xor(bad, 16);
        bad |= __shfl_xor(bad, 32);
        if (g == 0) {
            pd[wave * 16 + j] = dmax;
            pu[wave * 16 + j] = umax;
            pb[wave * 16 + j] = bad;
        }
        __syncthreads();
        dmax = 0.f;
        umax = 0.f;
        bad = 0;
        for (int w = 0; w < NW; ++w) {
            dmax = fmaxf(dmax, pd[w * 16 + j]);
            umax = fmaxf(umax, pu[w * 16 + j]);
            bad |= pb[w * 16 + j];
        }
        // ---- per-column decisions (identical in every wave)
        bool done = false, conv = false;
        if (col >= 0) {
            ++it;
            const float d = sqrtf(dmax);
            if (!kMixed || precise) {
                conv = d < tol;
                if (kMixed && (want || ph == 1)) {
                    ph = 1;
                    want = 0;
                    wait = 0;
                    sumd = 0.f;
                }
            } else if (ph == 0) {
                if (it == 1) uref = umax;
                uref = fmaxf(uref, umax);
                if (!want && (d < theta_k * uref || (it >= 2 && d > 0.5f * dprev))) want = 1;
            } else {
                conv = d * margin < tol;
                sumd += d;
                if (!want && sumd > refresh) want = 1;
            }
            if (want) ++wait;
            dprev = d;
            done = bad || conv || it >= max_iter;
            if (done) {
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    if (q < nv) {
                        const int t = tw + NW * q;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int b = 8 * t + 2 * g + h;
                            if (b < n) {
                                IO *o = Vout + 2 * (col * n + b);
                                o[0] = (IO)(wv[b] + (double)U[q][2 * h]);
                                o[1] = (IO)(wv[8 * MT + b] + (double)U[q][2 * h + 1]);
                            }
                        }
                    }
                }
                if (wave == 0 && g == 0) {
                    iters_out[col] = it;
                    status_out[col] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
                }
                col = -1;
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    Sv[q] = f4{0, 0, 0, 0};
                    In[q] = f4{0, 0, 0, 0};
                    Ip[q] = f4{0, 0, 0, 0};
                }
                want = 0;
                ph = 0;
            }
        }
        const unsigned long long act = __ballot(col >= 0 && g == 0);
        if (!act) {
            if (!refill()) break;
            prepare_b(false);
            __syncthreads();
            continue;
        }
        // ---- next sweep kind: refine when every low-phase column is ready, or one waited long
        if (kMixed) {
            const unsigned long long lowcols = __ballot(col >= 0 && g == 0 && ph == 0);
            const unsigned long long wants = __ballot(col >= 0 && g == 0 && want);
            const unsigned long long stale = __ballot(col >= 0 && g == 0 && wait >= 3);
            precise = wants != 0 && (((lowcols & ~wants) == 0) || stale != 0);
        }
        prepare_b(!precise && ph == 1 && col >= 0);
        __syncthreads();
    }
}

template <int TPW, int NW, int KTL, int MODE, typename IO>
static int launch_one(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                      int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                      unsigned long long *queue, hipStream_t stream) {
    const int MT = dn.MT;
    const bool f32r = MODE != TPF_MODE_MIXED_FP16;
    const size_t KPL = 32 * KTL + 8, KP32 = 16 * MT + 4;
    const size_t lds = (f32r ? 16 * KP32 * 4 : 0) + 16 * KPL * 2 * (MODE == TPF_MODE_MIXED_FP16 ? 2 : 1) +
                       (size_t)NW * 16 * 16 + (16 * MT + 2) * 4 + 16 + 16;
    auto kern = fpi_mixed_kernel<TPW, NW, KTL, MODE, IO>;
    if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NW * 64, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long blocks = std::min<long long>((long long)cus * per_cu, (tau + 15) / 16);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), lds, stream, (const IO *)S, (IO *)V, iters,
                       status, (const IO *)V0, dn.A32, MODE == TPF_MODE_MIXED_BF16 ? dn.Abf : dn.Ah, dn.Al,
                       dn.w64, net.n, MT, dn.sZ, (long long)tau, (float)tol, max_iter, queue);
    return TPF_OK;
}

template <int MODE, typename IO>
static int dispatch(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                    int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                    unsigned long long *queue, hipStream_t stream) {
#define TPF_GO(T, W, K)                                                                                      \
    if (dn.TPW == T && dn.NW == W && dn.KTL == K)                                                            \
        return launch_one<T, W, K, MODE, IO>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);
    TPF_GO(1, 4, 1) TPF_GO(1, 4, 2) TPF_GO(1, 8, 3) TPF_GO(1, 8, 4)
    TPF_GO(2, 8, 5) TPF_GO(2, 8, 6) TPF_GO(2, 8, 7) TPF_GO(2, 8, 8)
#undef TPF_GO
    return fail(TPF_ERR_UNSUPPORTED, "FP32/mixed sweep kernels support up to 128 PQ buses");
}

int launch_fpi_mixed(const tpf_network_s &net, const DeviceNet &dn, int mode, const void *S, int dtype, int64_t tau,
                     double tol, int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                     unsigned long long *queue, hipStream_t stream) {
    if (!dn.A32) return fail(TPF_ERR_UNSUPPORTED, "FP32/mixed sweep kernels support up to 128 PQ buses");
#define TPF_MODE_CASE(M)                                                                                      \
    if (mode == M) {                                                                                         \
        if (dtype == TPF_C128)                                                                               \
            return dispatch<M, double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream); \
        return dispatch<M, float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, queue, stream);      \
    }
    TPF_MODE_CASE(TPF_MODE_FP32)
    TPF_MODE_CASE(TPF_MODE_MIXED_BF16)
    TPF_MODE_CASE(TPF_MODE_MIXED_FP16)
#undef TPF_MODE_CASE
    return fail(TPF_ERR_INVALID_ARG, "unknown mode");
}

}  // namespace tpf
