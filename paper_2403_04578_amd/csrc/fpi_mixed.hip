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

#ifndef TPF_MIXED_CG
#define TPF_MIXED_CG 2
#endif

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
    const float i0 = 1.0f / fmaxf(v0r * v0r + v0i * v0i, kMinV2), i1 = 1.0f / fmaxf(v1r * v1r + v1i * v1i, kMinV2);
    return f4{(s[0] * v0r + s[1] * v0i) * i0, (s[0] * v0i - s[1] * v0r) * i0,
              (s[2] * v1r + s[3] * v1i) * i1, (s[2] * v1i - s[3] * v1r) * i1};
}

__device__ __forceinline__ float amax4(const f4 &x) {
    return fmaxf(fmaxf(fabsf(x[0]), fabsf(x[1])), fmaxf(fabsf(x[2]), fabsf(x[3])));
}

// Per-column state of a batch, double-buffered in LDS by sweep parity.  Every
// wave evaluates the same update for the columns of its lanes; wave 0 stores it.
struct ColState {
    long long col;  // -1 when the slot is idle
    float dprev, sumd, uref;
    int it, ph, want, wait;
};

// PF (FP16 form only): 1 = the rows of S of each batch are staged in LDS, the next batch's
// copied while the current one sweeps; 2 = the rows of V0 as well.  ZIP: loads of Eq. (2)
// with constant-power, constant-current and constant-impedance shares (aP, aI, aZ per bus,
// aZ possibly NULL; zscale = max_b |alpha_P| + |alpha_I| + |alpha_Z| bounds the injection
// for the FP16 column scale while 1/4 < |V| < 4).
template <int TPW, int NW, int KTL, int MODE, int CG, int PF, bool ZIP, typename IO>
__global__ __launch_bounds__(NW * 64) void fpi_mixed_kernel(
    const IO *__restrict__ S, IO *__restrict__ Vout, int32_t *__restrict__ iters_out,
    int8_t *__restrict__ status_out, const IO *__restrict__ V0, const float *__restrict__ A32,
    const uint16_t *__restrict__ Alow, const uint16_t *__restrict__ Alo, const double *__restrict__ wv, int n,
    int MT, int sZ, long long tau, float tol, int max_iter, unsigned long long *__restrict__ queue,
    const double *__restrict__ aP, const double *__restrict__ aI, const double *__restrict__ aZ, float zscale) {
    using L = LowOps<MODE>;
    typedef typename L::frag frag;
    typedef typename L::quad quad;
    constexpr bool kMixed = MODE != TPF_MODE_FP32;
    constexpr bool kSplit = MODE == TPF_MODE_MIXED_FP16;
    constexpr bool kF32Refine = !kSplit;
    constexpr bool kScaled = MODE == TPF_MODE_MIXED_FP16;  // FP16 operands need a power-of-two scale
    constexpr int NC = 16 * CG;
    constexpr bool kPfS = kSplit && PF >= 1, kPfV = kSplit && PF >= 2;
    constexpr int NT = NW * 64;
    constexpr int KPL = 32 * KTL + 8;
    const int KP32 = 16 * MT + 4;

    extern __shared__ __align__(16) unsigned char smem[];
    float *B32 = reinterpret_cast<float *>(smem);                                     // [NC][KP32] (FP32 refine)
    uint16_t *Bh = reinterpret_cast<uint16_t *>(B32 + (kF32Refine ? NC * KP32 : 0));  // [NC][KPL]
    uint16_t *Bl = Bh + (kMixed ? NC * KPL : 0);                                      // [NC][KPL]
    f4 *Sx = reinterpret_cast<f4 *>(Bl + (kSplit ? NC * KPL : 0));                    // [CG][MT][64]
    float *rmax = reinterpret_cast<float *>(Sx + CG * MT * 64);                       // [2][2][NC]
    int *rbad = reinterpret_cast<int *>(rmax + 4 * NC);                               // [2][NC]
    float *rsm = reinterpret_cast<float *>(rbad + 2 * NC);                            // [NC] max |S|
    int *rok = reinterpret_cast<int *>(rsm + NC);                                     // [NC] guard
    ColState *cs = reinterpret_cast<ColState *>(rok + NC);                            // [2][NC]
    unsigned long long *qb = reinterpret_cast<unsigned long long *>(cs + 2 * NC);     // [3] batch claims
    double *wl = reinterpret_cast<double *>(qb + 4);                                  // [2][8 MT] w
    // S (and V0) of the next batch, copied from HBM into LDS (no registers) while this
    // batch sweeps
    IO *Spf = reinterpret_cast<IO *>(wl + 16 * MT);                                   // [NC][n][2]
    IO *Vpf = Spf + (size_t)NC * n * 2;                                               // [NC][n][2]
    // ZIP shares [3][8 MT] (alpha_P, alpha_I, alpha_Z; padding buses 0), after the row copies
    float *zl = reinterpret_cast<float *>(Spf + (size_t)NC * n * 2 * (kSplit ? PF : 0));

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, j = lane & 15;
    const int tw = (wave + blockIdx.x) % NW;
    const int nv = (MT - tw + NW - 1) / NW;

    for (int e = tid; e < (kF32Refine ? NC * KP32 : 0); e += NT) B32[e] = 0.0f;
    for (int e = tid; e < (kMixed ? NC * KPL * (kSplit ? 2 : 1) : 0); e += NT) Bh[e] = 0;
    for (int e = tid; e < 4 * NC; e += NT) rmax[e] = 0.0f;
    for (int e = tid; e < 2 * NC; e += NT) rbad[e] = 0;
    for (int e = tid; e < 16 * MT; e += NT) wl[e] = wv[e];
    if constexpr (ZIP) {
        for (int e = tid; e < 8 * MT; e += NT) {
            zl[e] = e < n ? (float)aP[e] : 0.0f;
            zl[8 * MT + e] = e < n ? (float)aI[e] : 0.0f;
            zl[16 * MT + e] = e < n && aZ ? (float)aZ[e] : 0.0f;
        }
    }

    frag Af[TPW][KTL], Ag[kSplit ? TPW : 1][kSplit ? KTL : 1];
    f4 Wq[TPW];  // w of the lane's two buses per tile, FP32, (Re, Im, Re, Im)
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        Wq[q] = f4{1, 0, 1, 0};
        if (q < nv) {
            const int b0 = 8 * (tw + NW * q) + 2 * g;
            Wq[q] = f4{(float)wv[b0], (float)wv[8 * MT + b0], (float)wv[b0 + 1], (float)wv[8 * MT + b0 + 1]};
        }
        if constexpr (kMixed) {
#pragma unroll
            for (int kt = 0; kt < KTL; ++kt) {
                if (q < nv) {
                    const size_t idx = ((((size_t)tw * TPW + q) * KTL + kt) * 64 + lane) * 8;
                    Af[q][kt] = *reinterpret_cast<const frag *>(Alow + idx);
                    if constexpr (kSplit) Ag[q][kt] = *reinterpret_cast<const frag *>(Alo + idx);
                }
            }
        }
    }
    const float *Aw = A32 + (size_t)tw * (4 * MT + kFragPadSteps) * TPW * 64;

    f4 U[CG][TPW], Ip[CG][TPW];
    long long col[CG];
    float ks[CG], inv[CG];  // B scale 2^sB and product unscale 2^-(sB + sZ) per group
    bool dif[CG];
    bool precise = !kMixed;
    int par = 0;
    const float theta_k = 4.0f * L::u;
    const float refresh = 6.7e-8f / L::u;
    const float margin = 1.0f + 8.0f * L::u;

    // conj(S./V) 2^sB for the lane's two buses of tile q (rcp: ~1 ulp, far below the FP32 state floor)
    auto inject = [&](const f4 &sv, const f4 &w, const f4 &u, float k) -> f4 {
        const f4 v = w + u;
        const float r0 = __builtin_amdgcn_rcpf(fmaxf(v[0] * v[0] + v[1] * v[1], kMinV2)) * k;
        const float r1 = __builtin_amdgcn_rcpf(fmaxf(v[2] * v[2] + v[3] * v[3], kMinV2)) * k;
        return f4{(sv[0] * v[0] + sv[1] * v[1]) * r0, (sv[0] * v[1] - sv[1] * v[0]) * r0,
                  (sv[2] * v[2] + sv[3] * v[3]) * r1, (sv[2] * v[3] - sv[3] * v[2]) * r1};
    };

    // Forms the injections of every group from the current drops (Eq. (3), scaled by the
    // column's 2^sB), writes the B operand of the next sweep and rotates Ip.
    auto prepare_b = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int c = 0; c < CG; ++c) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                const f4 sv = q < nv ? Sx[(c * MT + tw + NW * q) * 64 + lane] : f4{0, 0, 0, 0};
                f4 In = inject(sv, Wq[q], U[c][q], ks[c]);
                if (ZIP && q < nv) {
                    // alpha_P conj(S./V) + alpha_I conj(S) + alpha_Z conj(S) V, all scaled
                    const int b0 = 8 * (tw + NW * q) + 2 * g;
                    const float p0 = zl[b0], p1 = zl[b0 + 1];
                    const float i0 = zl[8 * MT + b0] * ks[c], i1 = zl[8 * MT + b0 + 1] * ks[c];
                    const float z0 = zl[16 * MT + b0] * ks[c], z1 = zl[16 * MT + b0 + 1] * ks[c];
                    const f4 v = Wq[q] + U[c][q];
                    In = f4{p0 * In[0] + i0 * sv[0] + z0 * (sv[0] * v[0] + sv[1] * v[1]),
                            p0 * In[1] - i0 * sv[1] + z0 * (sv[0] * v[1] - sv[1] * v[0]),
                            p1 * In[2] + i1 * sv[2] + z1 * (sv[2] * v[2] + sv[3] * v[3]),
                            p1 * In[3] - i1 * sv[3] + z1 * (sv[2] * v[3] - sv[3] * v[2])};
                }
                if (q < nv) {
                    const f4 bv = dif[c] ? In - Ip[c][q] : In;
                    const int t = tw + NW * q;
                    if (precise && kF32Refine) {
                        *reinterpret_cast<f4 *>(B32 + (16 * c + j) * KP32 + 16 * t + 4 * g) = bv;
                    } else if constexpr (kMixed) {
                        // The column scale keeps |B| < 2^14 while |V| > 1/4 pu; a diverging
                        // (infeasible) column may leave that range: saturate instead of
                        // overflowing to inf, so it ends as MAX_ITER, not NONFINITE.
                        const f4 bc = kScaled ? f4{__builtin_amdgcn_fmed3f(bv[0], -65504.f, 65504.f),
                                                   __builtin_amdgcn_fmed3f(bv[1], -65504.f, 65504.f),
                                                   __builtin_amdgcn_fmed3f(bv[2], -65504.f, 65504.f),
                                                   __builtin_amdgcn_fmed3f(bv[3], -65504.f, 65504.f)}
                                              : bv;
                        const quad hq = L::cvt(bc);
                        const int off = (16 * c + j) * KPL + 16 * t + 4 * g;
                        *reinterpret_cast<quad *>(Bh + off) = hq;
                        if constexpr (kSplit) {
                            if (precise) {
                                const f4 r = bc - f4{(float)hq[0], (float)hq[1], (float)hq[2], (float)hq[3]};
                                *reinterpret_cast<quad *>(Bl + off) = L::cvt(r);
                            }
                        }
                    }
                }
                Ip[c][q] = In;
            }
        }
    };

    // Starts copying the S rows of batch `nb` (NC consecutive columns, contiguous in HBM)
    // into Spf, and its V0 rows into Vpf when kPfV: each wavefront moves 1 KB per
    // instruction straight into LDS.  Only whole batches are copied (a multiple of 16
    // bytes); a partial last batch reads HBM directly.
    auto prefetch = [&](unsigned long long nb) {
        if (nb + NC > (unsigned long long)tau) return;
        const long long bytes = (long long)NC * n * 2 * (long long)sizeof(IO);
#pragma unroll
        for (int arr = 0; arr < 2; ++arr) {
            if (arr == 1 && !kPfV) break;
            const char *src = reinterpret_cast<const char *>((arr ? V0 : S) + 2 * (long long)nb * n);
            char *dst = reinterpret_cast<char *>(arr ? Vpf : Spf);
            for (long long off = (long long)wave * 1024; off < bytes; off += (long long)NW * 1024) {
                if (off + 16 * lane < bytes)
                    __builtin_amdgcn_global_load_lds(src + off + 16 * lane,
                                                     (__attribute__((address_space(3))) void *)(dst + off), 16, 0, 0);
            }
        }
    };
    bool from_pf = false;  // this refill's batch was claimed ahead and its rows copied
    int slot = 1;          // qb[slot]: the batch whose rows are being copied
    auto refill = [&]() -> bool {
        if (tid < NC) {
            rsm[tid] = 0.0f;
            rok[tid] = 0;
        }
        if (tid == 0 && !from_pf) qb[0] = atomicAdd(queue, (unsigned long long)NC);
        if (from_pf) __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wavefront's copies landed
        __syncthreads();
        const unsigned long long base = from_pf ? qb[slot] : qb[0];
        if (base >= (unsigned long long)tau) return false;
        if constexpr (kPfS) {
            if (!(from_pf && base + NC <= (unsigned long long)tau)) {
                // the first batch and a partial last one were not copied ahead: copy their
                // rows now (8-byte units, coalesced), so that every batch reads LDS below
                const long long cols = (long long)tau - (long long)base < NC ? (long long)tau - (long long)base : NC;
                const long long units = cols * n * 2 * (long long)sizeof(IO) / 8;
#pragma unroll
                for (int arr = 0; arr < (kPfV ? 2 : 1); ++arr) {
                    const unsigned long long *src =
                        reinterpret_cast<const unsigned long long *>((arr ? V0 : S) + 2 * (long long)base * n);
                    unsigned long long *dst = reinterpret_cast<unsigned long long *>(arr ? Vpf : Spf);
                    for (long long e = tid; e < units; e += NT) dst[e] = src[e];
                }
                __syncthreads();
            }
        }
        // claim the batch after this one now; the atomic's latency overlaps the loads below
        unsigned long long next = (unsigned long long)tau;
        if (kPfS && tid == 0 && base + NC < (unsigned long long)tau)
            next = atomicAdd(queue, (unsigned long long)NC);
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            const long long cc = (long long)base + 16 * c + j;
            col[c] = cc < tau ? cc : -1;
            float sm = 0.0f;
            int bad = 0, sbad = 0;
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                double s[4] = {0, 0, 0, 0}, v[4] = {1, 0, 1, 0};
                if (q < nv && col[c] >= 0) {
                    const int b0 = 8 * (tw + NW * q) + 2 * g;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (b0 + h < n) {
                            if constexpr (kPfS)
                                ldc(Spf + 2 * ((16 * c + j) * n + b0 + h), s[2 * h], s[2 * h + 1]);
                            else
                                ldc(S + 2 * (col[c] * n + b0 + h), s[2 * h], s[2 * h + 1]);
                            if (V0) {
                                if constexpr (kPfV)
                                    ldc(Vpf + 2 * ((16 * c + j) * n + b0 + h), v[2 * h], v[2 * h + 1]);
                                else
                                    ldc(V0 + 2 * (col[c] * n + b0 + h), v[2 * h], v[2 * h + 1]);
                                const double m2 = v[2 * h] * v[2 * h] + v[2 * h + 1] * v[2 * h + 1];
                                bad |= (m2 >= 0.25 && m2 <= 2.25) ? 0 : 1;
                            }
                        }
                    }
                }
                const f4 sv = f4{(float)s[0], (float)s[1], (float)s[2], (float)s[3]};
                sbad |= !(fabs(s[0]) + fabs(s[1]) + fabs(s[2]) + fabs(s[3]) < HUGE_VAL);
                if (q < nv) Sx[(c * MT + tw + NW * q) * 64 + lane] = sv;
                sm = fmaxf(sm, amax4(sv));
                U[c][q] = f4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]} - Wq[q];
            }
            if constexpr (ZIP) sm *= zscale;
            sm = fmaxf(sm, __shfl_xor(sm, 16));
            sm = fmaxf(sm, __shfl_xor(sm, 32));
            bad |= __shfl_xor(bad, 16);
            bad |= __shfl_xor(bad, 32);
            sbad |= __shfl_xor(sbad, 16);
            sbad |= __shfl_xor(sbad, 32);
            if (g == 0) {
                atomicMax(reinterpret_cast<int *>(rsm) + 16 * c + j, __float_as_int(sm));  // sm >= 0: int order
                if (bad | sbad) atomicOr(rok + 16 * c + j, bad | (sbad << 1));
            }
        }
        // The other slot: qb[slot] may still be read by a wavefront that has not passed the
        // barrier above; the slot written here is next read after two more barriers.
        if (kPfS && tid == 0) qb[3 - slot] = next;
        __syncthreads();  // column reductions complete; every wavefront is done with Spf and Vpf
        if (kPfS) {
            slot = 3 - slot;
            prefetch(qb[slot]);
            from_pf = true;
        }
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            if (V0 && (rok[16 * c + j] & 1)) {  // guard failed somewhere in the column: flat start
#pragma unroll
                for (int q = 0; q < TPW; ++q) U[c][q] = f4{1, 0, 1, 0} - Wq[q];
            }
            int sB = 0;
            if constexpr (kScaled) {
                int e = 0;
                const float sm = rsm[16 * c + j];
                (void)frexpf(sm > 0.f ? sm : 1.0f, &e);
                sB = 12 - e;  // max |S| 2^sB < 2^12: |I| 2^sB < 2^14 while |V| > 1/4
            }
            ks[c] = ldexpf(1.0f, sB);
            inv[c] = ldexpf(1.0f, -(sB + (kScaled ? sZ : 0)));
            // A non-finite load would be clipped by the FP16 saturation; the product's
            // unscale carries it into the iterate instead, so the column ends NONFINITE.
            if (rok[16 * c + j] & 2) inv[c] = __builtin_nanf("");
            dif[c] = false;
            if (wave == 0 && g == 0) {
                ColState st;
                st.col = col[c];
                st.dprev = st.sumd = st.uref = 0.f;
                st.it = st.ph = st.want = st.wait = 0;
                // A warm start that passed the guard is already near the FP16 floor: the
                // column skips the full FP16 sweeps and begins with the accurate one.
                if (kMixed && V0 && !(rok[16 * c + j] & 1)) st.want = 1;
                cs[par * NC + 16 * c + j] = st;
            }
        }
        precise = !kMixed || V0 != nullptr;
        prepare_b();
        return true;
    };

    if (!refill()) return;
    __syncthreads();

    while (true) {
        // ---- products and epilogues
        auto epilogue = [&](int c, const f4(&acc)[TPW], bool full) {
            float emax = 0.f, esum = 0.f, umax = 0.f;
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (q < nv) {
                    const f4 p = acc[q] * inv[c];
                    const f4 un = full ? p : U[c][q] + p;
                    const f4 dd = un - U[c][q];
                    const float e0 = dd[0] * dd[0] + dd[1] * dd[1], e1 = dd[2] * dd[2] + dd[3] * dd[3];
                    esum += e0 + e1;
                    emax = fmaxf(emax, fmaxf(e0, e1));
                    umax = fmaxf(umax, amax4(un));
                    U[c][q] = un;
                }
            }
            emax = fmaxf(emax, __shfl_xor(emax, 16));
            emax = fmaxf(emax, __shfl_xor(emax, 32));
            umax = fmaxf(umax, __shfl_xor(umax, 16));
            umax = fmaxf(umax, __shfl_xor(umax, 32));
            int bad = !(esum < INFINITY);
            bad |= __shfl_xor(bad, 16);
            bad |= __shfl_xor(bad, 32);
            if (g == 0) {
                const int k = 16 * c + j;
                atomicMax(reinterpret_cast<int *>(rmax) + par * 2 * NC + k, __float_as_int(emax));
                atomicMax(reinterpret_cast<int *>(rmax) + par * 2 * NC + NC + k, __float_as_int(umax));
                if (bad) atomicOr(rbad + par * NC + k, 1);
            }
        };
        if (precise && kF32Refine) {
            f4 acc[CG][TPW];
#pragma unroll
            for (int c = 0; c < CG; ++c)
#pragma unroll
                for (int q = 0; q < TPW; ++q) acc[c][q] = f4{0, 0, 0, 0};
            const int KT = 4 * MT;
            constexpr int ST = TPW * 64;
            float r0[TPW], r1[TPW], r2[TPW], r3[TPW];
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                r0[q] = Aw[q * 64 + lane];
                r1[q] = Aw[ST + q * 64 + lane];
                r2[q] = Aw[2 * ST + q * 64 + lane];
            }
            auto step = [&](int kt, float(&r)[TPW]) {
#pragma unroll
                for (int c = 0; c < CG; ++c) {
                    const float b = B32[(16 * c + j) * KP32 + 4 * kt + g];
#pragma unroll
                    for (int q = 0; q < TPW; ++q)
                        if (q < nv) acc[c][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[q], b, acc[c][q], 0, 0, 0);
                }
            };
#pragma unroll 1
            for (int kt = 0; kt < KT; kt += 4) {
                const float *Ak = Aw + (size_t)kt * ST + lane;
#pragma unroll
                for (int q = 0; q < TPW; ++q) r3[q] = Ak[3 * ST + q * 64];
                step(kt, r0);
#pragma unroll
                for (int q = 0; q < TPW; ++q) r0[q] = Ak[4 * ST + q * 64];
                step(kt + 1, r1);
#pragma unroll
                for (int q = 0; q < TPW; ++q) r1[q] = Ak[5 * ST + q * 64];
                step(kt + 2, r2);
#pragma unroll
                for (int q = 0; q < TPW; ++q) r2[q] = Ak[6 * ST + q * 64];
                step(kt + 3, r3);
            }
#pragma unroll
            for (int c = 0; c < CG; ++c) epilogue(c, acc[c], true);
        } else if constexpr (kMixed) {
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                f4 acc[TPW];
#pragma unroll
                for (int q = 0; q < TPW; ++q) acc[q] = f4{0, 0, 0, 0};
#pragma unroll
                for (int kt = 0; kt < KTL; ++kt) {
                    const frag bh = *reinterpret_cast<const frag *>(Bh + (16 * c + j) * KPL + 32 * kt + 8 * g);
#pragma unroll
                    for (int q = 0; q < TPW; ++q)
                        if (q < nv) acc[q] = L::mma(Af[q][kt], bh, acc[q]);
                    if constexpr (kSplit) {
                        if (precise) {
                            const frag bl =
                                *reinterpret_cast<const frag *>(Bl + (16 * c + j) * KPL + 32 * kt + 8 * g);
#pragma unroll
                            for (int q = 0; q < TPW; ++q)
                                if (q < nv) {
                                    acc[q] = L::mma(Af[q][kt], bl, acc[q]);
                                    acc[q] = L::mma(Ag[q][kt], bh, acc[q]);
                                }
                        }
                    }
                }
                epilogue(c, acc, !dif[c]);
            }
        }
        __syncthreads();
        // ---- decisions, evaluated identically by every wave
        if (tid < NC) {  // clear the reductions of the next sweep
            rmax[(par ^ 1) * 2 * NC + tid] = 0.f;
            rmax[(par ^ 1) * 2 * NC + NC + tid] = 0.f;
            rbad[(par ^ 1) * NC + tid] = 0;
        }
        long long rcol[CG];
        bool want_any = false, low_unready = false, stale = false, active = false;
        int ph_next[CG];
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            const int k = 16 * c + j;
            const ColState st = cs[par * NC + k];
            ColState nx = st;
            rcol[c] = -1;
            if (st.col >= 0) {
                const float d = sqrtf(rmax[par * 2 * NC + k]);
                const float um = rmax[par * 2 * NC + NC + k];
                const int bad = rbad[par * NC + k];
                nx.it = st.it + 1;
                bool conv = false;
                if (!kMixed || precise) {
                    conv = d < tol;
                    if (kMixed && (st.want || st.ph == 1)) {
                        nx.ph = 1;
                        nx.want = 0;
                        nx.wait = 0;
                        nx.sumd = 0.f;
                    }
                } else if (st.ph == 0) {
                    nx.uref = fmaxf(st.uref, um);
                    if (!st.want && (d <= theta_k * nx.uref || (nx.it >= 2 && d > 0.5f * st.dprev))) nx.want = 1;
                } else {
                    conv = d * margin < tol;
                    nx.sumd = st.sumd + d;
                    if (!st.want && nx.sumd > refresh) nx.want = 1;
                }
                nx.wait = nx.want ? nx.wait + 1 : 0;
                nx.dprev = d;
                if (bad || conv || nx.it >= max_iter) {
                    if (wave == 0 && g == 0) {
                        iters_out[st.col] = nx.it;
                        status_out[st.col] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
                    }
                    rcol[c] = st.col;
                    nx.col = -1;
                    nx.want = 0;
                    nx.ph = 0;
                }
            }
            if (wave == 0 && g == 0) cs[(par ^ 1) * NC + k] = nx;
            col[c] = nx.col;
            ph_next[c] = nx.ph;
            const bool live = nx.col >= 0;
            want_any |= live && nx.want;
            low_unready |= live && nx.ph == 0 && !nx.want;
            stale |= live && nx.wait >= 3;
            active |= live;
        }
        // workgroup-uniform: every wave holds all NC columns in its lanes
        want_any = __ballot(want_any) != 0;
        low_unready = __ballot(low_unready) != 0;
        stale = __ballot(stale) != 0;
        active = __ballot(active) != 0;
        precise = !kMixed || (want_any && (!low_unready || stale));
        // ---- retire finished columns
#pragma unroll
        for (int c = 0; c < CG; ++c) {
            if (rcol[c] >= 0) {
#pragma unroll
                for (int q = 0; q < TPW; ++q) {
                    if (q < nv) {
                        const int b0 = 8 * (tw + NW * q) + 2 * g;
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int b = b0 + h;
                            if (b < n) {
                                IO *o = Vout + 2 * (rcol[c] * n + b);
                                o[0] = (IO)(wl[b] + (double)U[c][q][2 * h]);
                                o[1] = (IO)(wl[8 * MT + b] + (double)U[c][q][2 * h + 1]);
                            }
                        }
                        Sx[(c * MT + tw + NW * q) * 64 + lane] = f4{0, 0, 0, 0};  // idle slot: zero injection
                    }
                }
            }
            dif[c] = !precise && ph_next[c] == 1;
        }
        par ^= 1;
        if (!active) {
            __syncthreads();
            if (!refill()) break;
            __syncthreads();
            continue;
        }
        prepare_b();
        __syncthreads();
    }
}

template <int TPW, int NW, int KTL, int MODE, typename IO>
static int launch_one(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                      int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                      unsigned long long *queue, hipStream_t stream) {
    // column groups per workgroup: as many as the registers hold without spilling
    constexpr int CG = (MODE == TPF_MODE_FP32 || TPW == 1) ? 4 : TPF_MIXED_CG;
    const int MT = dn.MT;
    constexpr bool mixed = MODE != TPF_MODE_FP32, split = MODE == TPF_MODE_MIXED_FP16;
    const size_t NC = 16 * CG;
    const size_t KPL = 32 * KTL + 8, KP32 = 16 * MT + 4;
    const bool zip = dn.aP != nullptr;
    const size_t lds0 = (split ? 0 : NC * KP32 * 4) + (mixed ? NC * KPL * 2 * (split ? 2 : 1) : 0) +
                        (size_t)CG * MT * 64 * 16 + NC * (16 + 8 + 8) + 2 * NC * sizeof(ColState) + 32 +
                        (size_t)16 * MT * 8 + (zip ? (size_t)24 * MT * 4 : 0);
    // The next batch's S is prefetched into LDS when it fits beside the rest, and its V0
    // too when that also fits (the copies write exactly the rows' bytes).
    // (measured: it pays in the FP16 form, not in the BF16 one, whose registers it raises)
    const size_t spf = (size_t)NC * net.n * 2 * sizeof(IO);
    const size_t cap = (size_t)160 * 1024;
    int pf = split && lds0 + spf <= cap ? 1 : 0;
    if (pf && V0 && lds0 + 2 * spf <= cap) pf = 2;
    const size_t lds = lds0 + (size_t)pf * spf;
    auto kern = zip ? fpi_mixed_kernel<TPW, NW, KTL, MODE, CG, 0, true, IO>
                    : fpi_mixed_kernel<TPW, NW, KTL, MODE, CG, 0, false, IO>;
    if constexpr (split) {
        if (pf == 1)
            kern = zip ? fpi_mixed_kernel<TPW, NW, KTL, MODE, CG, 1, true, IO>
                       : fpi_mixed_kernel<TPW, NW, KTL, MODE, CG, 1, false, IO>;
        if (pf == 2)
            kern = zip ? fpi_mixed_kernel<TPW, NW, KTL, MODE, CG, 2, true, IO>
                       : fpi_mixed_kernel<TPW, NW, KTL, MODE, CG, 2, false, IO>;
    }
    if (hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NW * 64, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long blocks = std::min<long long>((long long)cus * per_cu, (tau + (long long)NC - 1) / (long long)NC);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(NW * 64), lds, stream, (const IO *)S, (IO *)V, iters,
                       status, (const IO *)V0, dn.A32, MODE == TPF_MODE_MIXED_BF16 ? dn.Abf : dn.Ah, dn.Al,
                       dn.w64, net.n, MT, dn.sZ, (long long)tau, (float)tol, max_iter, queue, dn.aP, dn.aI,
                       dn.aZ, dn.zscale);
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
