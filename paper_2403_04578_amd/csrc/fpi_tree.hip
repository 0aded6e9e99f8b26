// Sweeps with the tree operator, for radial (tree) networks, single- or three-phase, in
// FP64 or with the FP32 drop state V - w.
//
// On a radial feeder without shunts, Z = -Y_dd^-1 is minus the path-impedance matrix:
// (Y_dd^-1)_ij is the sum of the impedances of the branches shared by the paths from the
// slack to i and to j.  So the product Z I of Algorithm 1 (Sec. IV-A) needs no matrix:
//   backward pass  J_b = I_b + sum of J over the children of b   (current of the branch
//                  into b: the injections of b's subtree),
//   forward pass   D_b = D_parent(b) + z_b J_b, D_slack = 0       (drop from the slack),
// and Z I = -D.  This is O(n) work per column instead of the dense 8 n^2, with the same
// iterates up to rounding.
//
// A wavefront carries CPW power flows (columns) side by side, 64 / CPW lanes each: lane
// l of a column owns the breadth-first positions 1 + l + (64 / CPW) r (r < B) and keeps
// their S and V in registers.  The passes run level by level over a per-column LDS array
// of n + 1 complex values (J, then D in place); within a level the positions are spread
// over the column's lanes, and a wavefront's LDS accesses complete in order, so no
// workgroup barrier is needed.  Columns are dealt to the slots round robin.  Per sweep
// each column reads and writes only LDS and registers; S, V0 and the result cross HBM
// once.
#include "tpf_internal.h"

namespace tpf {

// Orders the LDS accesses of a wavefront's lanes around a point where they exchange values:
// the wave barrier is only a convergence and scheduling point, so wavefront-scope release and
// acquire fences on either side make the cross-lane reads see the writes before it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

namespace {

constexpr int kTreeWaves = 4;

template <typename IO, int CPW, int B, int ZM>
__global__ __launch_bounds__(kTreeWaves * 64) void fpi_tree_kernel(
    const IO *__restrict__ S, IO *__restrict__ Vout, int32_t *__restrict__ iters_out,
    int8_t *__restrict__ status_out, const IO *__restrict__ V0, const int32_t *__restrict__ tree_i,
    const double *__restrict__ tree_z, int n, int levels, long long tau, double tol, int max_iter,
    const double *__restrict__ aP, const double *__restrict__ aI, const double *__restrict__ aZ, double vs_re,
    double vs_im) {
    constexpr int LPC = 64 / CPW;  // lanes per column
    constexpr int NZ = ZM == 0 ? 0 : ZM + 1;  // ZIP shares per position
    extern __shared__ double lds[];
    const int np = n + 1;
    double *tz = lds;                                        // [np][4]: z, w per position
    double *za = tz + 4 * np;                                // [np][NZ]: alpha_P, alpha_I (, alpha_Z)
    double *Jw = za + NZ * np;                               // [waves][CPW][np][2]
    double *Gw = Jw + kTreeWaves * CPW * 2 * np;             // ZM == 2: G' per column, as Jw
    int32_t *ti = reinterpret_cast<int32_t *>(Gw + (ZM == 2 ? kTreeWaves * CPW * 2 * np : 0));  // [np][4], levels
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int slot = lane / LPC, sl = lane % LPC;  // column slot of the wavefront, lane within it
    for (int e = threadIdx.x; e < 4 * np; e += kTreeWaves * 64) tz[e] = tree_z[e];
    for (int e = threadIdx.x; e < 4 * np + levels + 2; e += kTreeWaves * 64) ti[e] = tree_i[e];
    if constexpr (ZM >= 1) {
        for (int p = threadIdx.x; p < np; p += kTreeWaves * 64) {
            const int q = tree_i[4 * p];
            za[NZ * p] = q >= 0 ? aP[q] : 0.0;
            za[NZ * p + 1] = q >= 0 ? aI[q] : 0.0;
            if constexpr (ZM == 2) za[NZ * p + 2] = q >= 0 ? aZ[q] : 0.0;
        }
    }
    __syncthreads();
    double *J = Jw + (wave * CPW + slot) * 2 * np;
    double *G = Gw + (wave * CPW + slot) * 2 * np;
    bool fresh = true;  // the slot's column is new: its G' still to be formed (ZM == 2)
    const int32_t *ls = ti + 4 * np;  // level L = positions [ls[L], ls[L+1])
    if (sl == 0) J[0] = J[1] = 0.0;   // the slack's drop

    // Column slots take columns round robin; a slot that finishes a column loads its next
    // one at once, so the slots of a wavefront may be at different sweeps.
    const long long nslots = (long long)gridDim.x * kTreeWaves * CPW;
    long long c = ((long long)blockIdx.x * kTreeWaves + wave) * CPW + slot;
    double sr[B], si[B], vr[B], vi[B];
    int it = 0;
    auto load = [&]() __attribute__((always_inline)) {
        int ok = 1;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            sr[r] = si[r] = vi[r] = 0.0;
            vr[r] = 1.0;
            if (c < tau && p <= n) {
                const long long o = 2 * (c * n + ti[4 * p]);
                sr[r] = (double)S[o];
                si[r] = (double)S[o + 1];
                if (V0) {
                    vr[r] = (double)V0[o];
                    vi[r] = (double)V0[o + 1];
                    const double m2 = vr[r] * vr[r] + vi[r] * vi[r];
                    ok &= (m2 >= 0.25 && m2 <= 2.25) ? 1 : 0;
                }
            }
        }
        if (V0) {  // the guard failed somewhere in the column: flat start
#pragma unroll
            for (int off = LPC / 2; off > 0; off >>= 1) ok &= __shfl_xor(ok, off);
            if (!ok) {
#pragma unroll
                for (int r = 0; r < B; ++r) vr[r] = 1.0, vi[r] = 0.0;
            }
        }
        it = 0;
        fresh = true;
    };
    load();
    while (__ballot(c < tau)) {
        const bool live = c < tau;
        // injections conj(S./V) (ZIP: alpha_P conj(S./V) + alpha_I conj(S)) into J
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            if (p <= n) {
                const double inv = 1.0 / (vr[r] * vr[r] + vi[r] * vi[r]);
                double ir = (sr[r] * vr[r] + si[r] * vi[r]) * inv, ii = (sr[r] * vi[r] - si[r] * vr[r]) * inv;
                if constexpr (ZM >= 1) {
                    const double ap = za[NZ * p], ai = za[NZ * p + 1];
                    ir = ap * ir + ai * sr[r];
                    ii = ap * ii - ai * si[r];
                }
                J[2 * p] = ir;
                J[2 * p + 1] = ii;
                if (ZM == 2 && fresh) {  // y_b = alpha_Z s_b*, the start of G_b
                    const double az = za[NZ * p + 2];
                    G[2 * p] = az * sr[r];
                    G[2 * p + 1] = -az * si[r];
                }
            }
        }
        wave_sync();
        // backward pass, deepest level first: J_b += J of b's children.  ZM == 2: a
        // constant-impedance share (Eq. (2), B = diag(alpha_Z s*) + Y_dd) makes each subtree
        // a Norton load G x + J seen from its parent, with G_b = y_b + sum of the
        // children's G'_c and G'_b = G_b / (1 + z_b G_b), which depend on the column's s
        // only: formed in the first sweep of a column and kept.  The branch current's
        // source part is J'_b = k_b (I_b + sum of the children's J'), k_b = 1 / (1 + z_b G_b)
        // = 1 - z_b G'_b.
        for (int L = levels; L >= 1; --L) {
            for (int p = ls[L] + sl; p < ls[L + 1]; p += LPC) {
                double jr = J[2 * p], ji = J[2 * p + 1];
                for (int ch = ti[4 * p + 2]; ch < ti[4 * p + 3]; ++ch) {
                    jr += J[2 * ch];
                    ji += J[2 * ch + 1];
                }
                if constexpr (ZM == 2) {
                    if (fresh) {
                        double gr = G[2 * p], gi = G[2 * p + 1];
                        for (int ch = ti[4 * p + 2]; ch < ti[4 * p + 3]; ++ch) {
                            gr += G[2 * ch];
                            gi += G[2 * ch + 1];
                        }
                        const double dr = 1.0 + tz[4 * p] * gr - tz[4 * p + 1] * gi;
                        const double di = tz[4 * p] * gi + tz[4 * p + 1] * gr;
                        const double dd = 1.0 / (dr * dr + di * di);
                        G[2 * p] = (gr * dr + gi * di) * dd;
                        G[2 * p + 1] = (gi * dr - gr * di) * dd;
                    }
                    const double kr = 1.0 - (tz[4 * p] * G[2 * p] - tz[4 * p + 1] * G[2 * p + 1]);
                    const double ki = -(tz[4 * p] * G[2 * p + 1] + tz[4 * p + 1] * G[2 * p]);
                    const double tr = kr * jr - ki * ji;
                    ji = kr * ji + ki * jr;
                    jr = tr;
                }
                J[2 * p] = jr;
                J[2 * p + 1] = ji;
            }
            wave_sync();
        }
        // forward pass, level 1 first: D_b = D_parent + z_b J_b (in place of J_b); ZM == 2:
        // x_b = k_b x_parent - z_b J'_b, so with D = v_s - x,
        // D_b = k_b D_parent + z_b (J'_b + G'_b v_s)
        for (int L = 1; L <= levels; ++L) {
            for (int p = ls[L] + sl; p < ls[L + 1]; p += LPC) {
                const int par = ti[4 * p + 1];
                const double zr = tz[4 * p], zi = tz[4 * p + 1];
                double jr = J[2 * p], ji = J[2 * p + 1], pr = J[2 * par], pi = J[2 * par + 1];
                if constexpr (ZM == 2) {
                    const double gr = G[2 * p], gi = G[2 * p + 1];
                    const double kr = 1.0 - (zr * gr - zi * gi), ki = -(zr * gi + zi * gr);
                    jr += gr * vs_re - gi * vs_im;
                    ji += gr * vs_im + gi * vs_re;
                    const double tr = kr * pr - ki * pi;
                    pi = kr * pi + ki * pr;
                    pr = tr;
                }
                J[2 * p] = pr + zr * jr - zi * ji;
                J[2 * p + 1] = pi + zr * ji + zi * jr;
            }
            wave_sync();
        }
        fresh = false;
        // V' = w + Z I = w - D (ZM == 2: v_s - D); step max |V' - V| per column
        double dmax = 0.0;
        int bad = 0;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            if (p <= n) {
                const double wr = ZM == 2 ? vs_re : tz[4 * p + 2], wi = ZM == 2 ? vs_im : tz[4 * p + 3];
                const double nr = wr - J[2 * p], ni = wi - J[2 * p + 1];
                const double er = nr - vr[r], ei = ni - vi[r];
                const double e = er * er + ei * ei;
                bad |= !(e < HUGE_VAL);
                dmax = e > dmax ? e : dmax;
                vr[r] = nr;
                vi[r] = ni;
            }
        }
#pragma unroll
        for (int off = LPC / 2; off > 0; off >>= 1) {
            dmax = fmax(dmax, __shfl_xor(dmax, off));
            bad |= __shfl_xor(bad, off);
        }
        ++it;
        const bool conv = !bad && sqrt(dmax) < tol;
        if (live && (bad || conv || it >= max_iter)) {
#pragma unroll
            for (int r = 0; r < B; ++r) {
                const int p = 1 + sl + LPC * r;
                if (p <= n) {
                    const long long o = 2 * (c * n + ti[4 * p]);
                    Vout[o] = (IO)vr[r];
                    Vout[o + 1] = (IO)vi[r];
                }
            }
            if (sl == 0) {
                iters_out[c] = it;
                status_out[c] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
            }
            c += nslots;
            load();
        }
        wave_sync();
    }
}

// FP32 form of the tree operator (single-phase): the state is the drop U = V - w in FP32
// (as in the FP32 sweep kernels), and since V' = w - D the new state is simply U' = -D.
// The injection uses V = w + U; w is added back in FP64 for the output.  The passes run
// in FP32 (|D| ~ 1e-2 pu keeps their rounding near 1e-9 pu).
template <typename IO, int CPW, int B, int ZM>
__global__ __launch_bounds__(kTreeWaves * 64) void fpi_tree32_kernel(
    const IO *__restrict__ S, IO *__restrict__ Vout, int32_t *__restrict__ iters_out,
    int8_t *__restrict__ status_out, const IO *__restrict__ V0, const int32_t *__restrict__ tree_i,
    const double *__restrict__ tree_z, int n, int levels, long long tau, float tol, int max_iter,
    const double *__restrict__ aP, const double *__restrict__ aI, const double *__restrict__ aZ, double vs_re,
    double vs_im) {
    constexpr int LPC = 64 / CPW;
    constexpr int NZ = ZM == 0 ? 0 : ZM + 1;
    extern __shared__ double lds[];
    const int np = n + 1;
    double *wd = lds;                                        // [np][2] w in FP64 (outputs); ZM == 2: v_s
    float *tz = reinterpret_cast<float *>(wd + 2 * np);      // [np][4]: z, w in FP32
    float *za = tz + 4 * np;                                 // [np][NZ]: alpha_P, alpha_I (, alpha_Z)
    float *Jw = za + NZ * np;                                // [waves][CPW][np][2]
    float *Gw = Jw + kTreeWaves * CPW * 2 * np;              // ZM == 2: G' per column, as Jw
    int32_t *ti = reinterpret_cast<int32_t *>(Gw + (ZM == 2 ? kTreeWaves * CPW * 2 * np : 0));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int slot = lane / LPC, sl = lane % LPC;
    // the state is the drop U = V - w; with a constant-impedance share w differs per column
    // (w = -B^-1 c), so the drop is taken from the slack voltage instead
    for (int p = threadIdx.x; p < np; p += kTreeWaves * 64) {
        wd[2 * p] = ZM == 2 ? vs_re : tree_z[4 * p + 2];
        wd[2 * p + 1] = ZM == 2 ? vs_im : tree_z[4 * p + 3];
    }
    for (int e = threadIdx.x; e < 4 * np; e += kTreeWaves * 64)
        tz[e] = (ZM == 2 && (e & 3) >= 2) ? (float)((e & 1) ? vs_im : vs_re) : (float)tree_z[e];
    for (int e = threadIdx.x; e < 4 * np + levels + 2; e += kTreeWaves * 64) ti[e] = tree_i[e];
    if constexpr (ZM >= 1) {
        for (int p = threadIdx.x; p < np; p += kTreeWaves * 64) {
            const int q = tree_i[4 * p];
            za[NZ * p] = q >= 0 ? (float)aP[q] : 0.0f;
            za[NZ * p + 1] = q >= 0 ? (float)aI[q] : 0.0f;
            if constexpr (ZM == 2) za[NZ * p + 2] = q >= 0 ? (float)aZ[q] : 0.0f;
        }
    }
    __syncthreads();
    float *J = Jw + (wave * CPW + slot) * 2 * np;
    float *G = Gw + (wave * CPW + slot) * 2 * np;
    bool fresh = true;
    const float vsr = (float)vs_re, vsi = (float)vs_im;
    const int32_t *ls = ti + 4 * np;
    if (sl == 0) J[0] = J[1] = 0.0f;

    const long long nslots = (long long)gridDim.x * kTreeWaves * CPW;
    long long c = ((long long)blockIdx.x * kTreeWaves + wave) * CPW + slot;
    float sr[B], si[B], ur[B], ui[B];
    int it = 0;
    auto load = [&]() __attribute__((always_inline)) {
        int ok = 1;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            sr[r] = si[r] = 0.0f;
            ur[r] = ui[r] = 0.0f;
            if (c < tau && p <= n) {
                const long long o = 2 * (c * n + ti[4 * p]);
                sr[r] = (float)S[o];
                si[r] = (float)S[o + 1];
                double vr = 1.0, vi = 0.0;
                if (V0) {
                    vr = (double)V0[o];
                    vi = (double)V0[o + 1];
                    const double m2 = vr * vr + vi * vi;
                    ok &= (m2 >= 0.25 && m2 <= 2.25) ? 1 : 0;
                }
                ur[r] = (float)(vr - wd[2 * p]);
                ui[r] = (float)(vi - wd[2 * p + 1]);
            }
        }
        if (V0) {
#pragma unroll
            for (int off = LPC / 2; off > 0; off >>= 1) ok &= __shfl_xor(ok, off);
            if (!ok) {
#pragma unroll
                for (int r = 0; r < B; ++r) {
                    const int p = 1 + sl + LPC * r;
                    if (p <= n) {
                        ur[r] = (float)(1.0 - wd[2 * p]);
                        ui[r] = (float)(0.0 - wd[2 * p + 1]);
                    }
                }
            }
        }
        it = 0;
        fresh = true;
    };
    load();
    while (__ballot(c < tau)) {
        const bool live = c < tau;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            if (p <= n) {
                const float vr = tz[4 * p + 2] + ur[r], vi = tz[4 * p + 3] + ui[r];
                const float inv = 1.0f / fmaxf(vr * vr + vi * vi, kMinV2);
                float ir = (sr[r] * vr + si[r] * vi) * inv, ii = (sr[r] * vi - si[r] * vr) * inv;
                if constexpr (ZM >= 1) {
                    const float ap = za[NZ * p], ai = za[NZ * p + 1];
                    ir = ap * ir + ai * sr[r];
                    ii = ap * ii - ai * si[r];
                }
                J[2 * p] = ir;
                J[2 * p + 1] = ii;
                if (ZM == 2 && fresh) {
                    const float az = za[NZ * p + 2];
                    G[2 * p] = az * sr[r];
                    G[2 * p + 1] = -az * si[r];
                }
            }
        }
        wave_sync();
        for (int L = levels; L >= 1; --L) {  // as in fpi_tree_kernel
            for (int p = ls[L] + sl; p < ls[L + 1]; p += LPC) {
                float jr = J[2 * p], ji = J[2 * p + 1];
                for (int ch = ti[4 * p + 2]; ch < ti[4 * p + 3]; ++ch) {
                    jr += J[2 * ch];
                    ji += J[2 * ch + 1];
                }
                if constexpr (ZM == 2) {
                    if (fresh) {
                        float gr = G[2 * p], gi = G[2 * p + 1];
                        for (int ch = ti[4 * p + 2]; ch < ti[4 * p + 3]; ++ch) {
                            gr += G[2 * ch];
                            gi += G[2 * ch + 1];
                        }
                        const float dr = 1.0f + tz[4 * p] * gr - tz[4 * p + 1] * gi;
                        const float di = tz[4 * p] * gi + tz[4 * p + 1] * gr;
                        const float dd = 1.0f / (dr * dr + di * di);
                        G[2 * p] = (gr * dr + gi * di) * dd;
                        G[2 * p + 1] = (gi * dr - gr * di) * dd;
                    }
                    const float kr = 1.0f - (tz[4 * p] * G[2 * p] - tz[4 * p + 1] * G[2 * p + 1]);
                    const float ki = -(tz[4 * p] * G[2 * p + 1] + tz[4 * p + 1] * G[2 * p]);
                    const float tr = kr * jr - ki * ji;
                    ji = kr * ji + ki * jr;
                    jr = tr;
                }
                J[2 * p] = jr;
                J[2 * p + 1] = ji;
            }
            wave_sync();
        }
        for (int L = 1; L <= levels; ++L) {
            for (int p = ls[L] + sl; p < ls[L + 1]; p += LPC) {
                const int par = ti[4 * p + 1];
                const float zr = tz[4 * p], zi = tz[4 * p + 1];
                float jr = J[2 * p], ji = J[2 * p + 1], pr = J[2 * par], pi = J[2 * par + 1];
                if constexpr (ZM == 2) {
                    const float gr = G[2 * p], gi = G[2 * p + 1];
                    const float kr = 1.0f - (zr * gr - zi * gi), ki = -(zr * gi + zi * gr);
                    jr += gr * vsr - gi * vsi;
                    ji += gr * vsi + gi * vsr;
                    const float tr = kr * pr - ki * pi;
                    pi = kr * pi + ki * pr;
                    pr = tr;
                }
                J[2 * p] = pr + zr * jr - zi * ji;
                J[2 * p + 1] = pi + zr * ji + zi * jr;
            }
            wave_sync();
        }
        fresh = false;
        float dmax = 0.0f;
        int bad = 0;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            if (p <= n) {
                const float nr = -J[2 * p], ni = -J[2 * p + 1];  // U' = V' - w = -D
                const float er = nr - ur[r], ei = ni - ui[r];
                const float e = er * er + ei * ei;
                bad |= !(e < INFINITY);
                dmax = e > dmax ? e : dmax;
                ur[r] = nr;
                ui[r] = ni;
            }
        }
#pragma unroll
        for (int off = LPC / 2; off > 0; off >>= 1) {
            dmax = fmaxf(dmax, __shfl_xor(dmax, off));
            bad |= __shfl_xor(bad, off);
        }
        ++it;
        const bool conv = !bad && sqrtf(dmax) < tol;
        if (live && (bad || conv || it >= max_iter)) {
#pragma unroll
            for (int r = 0; r < B; ++r) {
                const int p = 1 + sl + LPC * r;
                if (p <= n) {
                    const long long o = 2 * (c * n + ti[4 * p]);
                    Vout[o] = (IO)(wd[2 * p] + (double)ur[r]);
                    Vout[o + 1] = (IO)(wd[2 * p + 1] + (double)ui[r]);
                }
            }
            if (sl == 0) {
                iters_out[c] = it;
                status_out[c] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
            }
            c += nslots;
            load();
        }
        wave_sync();
    }
}

template <typename IO, int CPW, int B, int ZM>
int launch32_as(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol, int max_iter,
                const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    const int n = net.n, np = n + 1, levels = dn.tree_levels;
    const size_t lds = (size_t)2 * np * 8 + (size_t)4 * np * 4 + (size_t)(ZM ? ZM + 1 : 0) * np * 4 +
                       (size_t)(ZM == 2 ? 2 : 1) * kTreeWaves * CPW * 2 * np * 4 + (size_t)(4 * np + levels + 2) * 4;
    if (lds > (size_t)160 * 1024) return fail(TPF_ERR_UNSUPPORTED, "tree operator: network too large for LDS");
    auto k = fpi_tree32_kernel<IO, CPW, B, ZM>;
    if (hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kTreeWaves * 64, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long per_block = (long long)kTreeWaves * CPW;
    const long long blocks =
        std::max<long long>(1, std::min<long long>((long long)cus * per_cu, (tau + per_block - 1) / per_block));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kTreeWaves * 64), lds, st, (const IO *)S, (IO *)V, iters,
                       status, (const IO *)V0, dn.tree_i, dn.tree_z, n, levels, (long long)tau, (float)tol, max_iter,
                       (const double *)dn.aP, (const double *)dn.aI, (const double *)dn.aZ, net.vs.real(),
                       net.vs.imag());
    return TPF_OK;
}

template <typename IO, int CPW, int B>
int launch32_b(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol, int max_iter,
               const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    // (the FP32 state is half the size: the shape of launch_b's halving measured slower here,
    // 1.19 against 1.02 ms on the 100-bus year)
    if (dn.aZ) return launch32_as<IO, CPW, B, 2>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (dn.aP) return launch32_as<IO, CPW, B, 1>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    return launch32_as<IO, CPW, B, 0>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
}

// The FP32 form takes 4 columns of 16 lanes up to 128 PQ buses: with half the FP64
// kernel's registers per position, the wider column group measured fastest there
// (8 columns of 8 lanes, the FP64 choice, ran the 100-bus year 16 % slower).
template <typename IO>
int launch32_io(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol, int max_iter,
                const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    const int n = net.n;
    if (n <= 64) return launch32_b<IO, 8, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (n <= 128) return launch32_b<IO, 4, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (n <= 256) return launch32_b<IO, 2, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (n <= 512) return launch32_b<IO, 1, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (n <= 1024) return launch32_b<IO, 1, 16>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    return fail(TPF_ERR_UNSUPPORTED, "tree operator: up to 1,024 PQ buses");
}

// Three-phase networks: the same passes with three phase nodes per position; a branch
// carries a 3x3 impedance matrix, so the forward pass is D_b = D_parent + Z_abc,b J_b.
// Position p's node f is demand node 3 pq(p) + f.  tz: per position Z_abc (9 complex)
// then w of the three phases; J: per column [np][3] complex.
template <typename IO, int CPW, int B>
__global__ __launch_bounds__(kTreeWaves * 64) void fpi_tree3_kernel(
    const IO *__restrict__ S, IO *__restrict__ Vout, int32_t *__restrict__ iters_out,
    int8_t *__restrict__ status_out, const IO *__restrict__ V0, const int32_t *__restrict__ tree_i,
    const double *__restrict__ tree_z, int nb, int levels, long long tau, double tol, int max_iter) {
    constexpr int LPC = 64 / CPW;
    constexpr int TZ = 24;  // doubles per position in tz
    extern __shared__ double lds[];
    const int np = nb + 1;   // positions (buses)
    const int n = 3 * nb;    // demand nodes per column
    double *tz = lds;                                        // [np][24]
    double *Jw = tz + TZ * np;                               // [waves][CPW][np][6]
    int32_t *ti = reinterpret_cast<int32_t *>(Jw + kTreeWaves * CPW * 6 * np);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int slot = lane / LPC, sl = lane % LPC;
    for (int e = threadIdx.x; e < TZ * np; e += kTreeWaves * 64) tz[e] = tree_z[e];
    for (int e = threadIdx.x; e < 4 * np + levels + 2; e += kTreeWaves * 64) ti[e] = tree_i[e];
    __syncthreads();
    double *J = Jw + (wave * CPW + slot) * 6 * np;
    const int32_t *ls = ti + 4 * np;
    if (sl == 0)
        for (int e = 0; e < 6; ++e) J[e] = 0.0;  // the slack's drop

    const long long nslots = (long long)gridDim.x * kTreeWaves * CPW;
    long long c = ((long long)blockIdx.x * kTreeWaves + wave) * CPW + slot;
    double sr[B][3], si[B][3], vr[B][3], vi[B][3];
    int it = 0;
    auto load = [&]() __attribute__((always_inline)) {
        int ok = 1;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                sr[r][f] = si[r][f] = vi[r][f] = 0.0;
                vr[r][f] = 1.0;
                if (c < tau && p <= nb) {
                    const long long o = 2 * (c * n + 3 * ti[4 * p] + f);
                    sr[r][f] = (double)S[o];
                    si[r][f] = (double)S[o + 1];
                    if (V0) {
                        vr[r][f] = (double)V0[o];
                        vi[r][f] = (double)V0[o + 1];
                        const double m2 = vr[r][f] * vr[r][f] + vi[r][f] * vi[r][f];
                        ok &= (m2 >= 0.25 && m2 <= 2.25) ? 1 : 0;
                    }
                }
            }
        }
        if (V0) {
#pragma unroll
            for (int off = LPC / 2; off > 0; off >>= 1) ok &= __shfl_xor(ok, off);
            if (!ok) {
#pragma unroll
                for (int r = 0; r < B; ++r)
#pragma unroll
                    for (int f = 0; f < 3; ++f) vr[r][f] = 1.0, vi[r][f] = 0.0;
            }
        }
        it = 0;
    };
    load();
    while (__ballot(c < tau)) {
        const bool live = c < tau;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            if (p <= nb) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const double inv = 1.0 / (vr[r][f] * vr[r][f] + vi[r][f] * vi[r][f]);
                    J[6 * p + 2 * f] = (sr[r][f] * vr[r][f] + si[r][f] * vi[r][f]) * inv;
                    J[6 * p + 2 * f + 1] = (sr[r][f] * vi[r][f] - si[r][f] * vr[r][f]) * inv;
                }
            }
        }
        wave_sync();
        for (int L = levels; L >= 1; --L) {
            for (int p = ls[L] + sl; p < ls[L + 1]; p += LPC) {
                double j[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) j[e] = J[6 * p + e];
                for (int ch = ti[4 * p + 2]; ch < ti[4 * p + 3]; ++ch) {
#pragma unroll
                    for (int e = 0; e < 6; ++e) j[e] += J[6 * ch + e];
                }
#pragma unroll
                for (int e = 0; e < 6; ++e) J[6 * p + e] = j[e];
            }
            wave_sync();
        }
        for (int L = 1; L <= levels; ++L) {
            for (int p = ls[L] + sl; p < ls[L + 1]; p += LPC) {
                const int par = ti[4 * p + 1];
                double j[6], d[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) j[e] = J[6 * p + e], d[e] = J[6 * par + e];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const double zr = tz[TZ * p + 2 * (3 * a + b)], zi = tz[TZ * p + 2 * (3 * a + b) + 1];
                        d[2 * a] += zr * j[2 * b] - zi * j[2 * b + 1];
                        d[2 * a + 1] += zr * j[2 * b + 1] + zi * j[2 * b];
                    }
                }
#pragma unroll
                for (int e = 0; e < 6; ++e) J[6 * p + e] = d[e];
            }
            wave_sync();
        }
        double dmax = 0.0;
        int bad = 0;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            if (p <= nb) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const double nr = tz[TZ * p + 18 + 2 * f] - J[6 * p + 2 * f];
                    const double ni = tz[TZ * p + 19 + 2 * f] - J[6 * p + 2 * f + 1];
                    const double er = nr - vr[r][f], ei = ni - vi[r][f];
                    const double e = er * er + ei * ei;
                    bad |= !(e < HUGE_VAL);
                    dmax = e > dmax ? e : dmax;
                    vr[r][f] = nr;
                    vi[r][f] = ni;
                }
            }
        }
#pragma unroll
        for (int off = LPC / 2; off > 0; off >>= 1) {
            dmax = fmax(dmax, __shfl_xor(dmax, off));
            bad |= __shfl_xor(bad, off);
        }
        ++it;
        const bool conv = !bad && sqrt(dmax) < tol;
        if (live && (bad || conv || it >= max_iter)) {
#pragma unroll
            for (int r = 0; r < B; ++r) {
                const int p = 1 + sl + LPC * r;
                if (p <= nb) {
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const long long o = 2 * (c * n + 3 * ti[4 * p] + f);
                        Vout[o] = (IO)vr[r][f];
                        Vout[o + 1] = (IO)vi[r][f];
                    }
                }
            }
            if (sl == 0) {
                iters_out[c] = it;
                status_out[c] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
            }
            c += nslots;
            load();
        }
        wave_sync();
    }
}

// Three-phase FP32 form: the state is the FP32 drop U = V - w per phase node and U' = -D,
// as in the single-phase FP32 kernel; the 3x3 blocks and w are staged in FP32 (w also in
// FP64 for the output).
template <typename IO, int CPW, int B>
__global__ __launch_bounds__(kTreeWaves * 64) void fpi_tree3_32_kernel(
    const IO *__restrict__ S, IO *__restrict__ Vout, int32_t *__restrict__ iters_out,
    int8_t *__restrict__ status_out, const IO *__restrict__ V0, const int32_t *__restrict__ tree_i,
    const double *__restrict__ tree_z, int nb, int levels, long long tau, float tol, int max_iter) {
    constexpr int LPC = 64 / CPW;
    constexpr int TZ = 24;
    extern __shared__ double lds[];
    const int np = nb + 1;
    const int n = 3 * nb;
    double *wd = lds;                                        // [np][6] w in FP64
    float *tz = reinterpret_cast<float *>(wd + 6 * np);      // [np][24]
    float *Jw = tz + TZ * np;                                // [waves][CPW][np][6]
    int32_t *ti = reinterpret_cast<int32_t *>(Jw + kTreeWaves * CPW * 6 * np);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int slot = lane / LPC, sl = lane % LPC;
    for (int e = threadIdx.x; e < TZ * np; e += kTreeWaves * 64) tz[e] = (float)tree_z[e];
    for (int p = threadIdx.x; p < np; p += kTreeWaves * 64)
        for (int e = 0; e < 6; ++e) wd[6 * p + e] = tree_z[TZ * p + 18 + e];
    for (int e = threadIdx.x; e < 4 * np + levels + 2; e += kTreeWaves * 64) ti[e] = tree_i[e];
    __syncthreads();
    float *J = Jw + (wave * CPW + slot) * 6 * np;
    const int32_t *ls = ti + 4 * np;
    if (sl == 0)
        for (int e = 0; e < 6; ++e) J[e] = 0.0f;

    const long long nslots = (long long)gridDim.x * kTreeWaves * CPW;
    long long c = ((long long)blockIdx.x * kTreeWaves + wave) * CPW + slot;
    float sr[B][3], si[B][3], ur[B][3], ui[B][3];
    int it = 0;
    auto load = [&]() __attribute__((always_inline)) {
        int ok = 1;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                sr[r][f] = si[r][f] = ur[r][f] = ui[r][f] = 0.0f;
                if (c < tau && p <= nb) {
                    const long long o = 2 * (c * n + 3 * ti[4 * p] + f);
                    sr[r][f] = (float)S[o];
                    si[r][f] = (float)S[o + 1];
                    double vr = 1.0, vi = 0.0;
                    if (V0) {
                        vr = (double)V0[o];
                        vi = (double)V0[o + 1];
                        const double m2 = vr * vr + vi * vi;
                        ok &= (m2 >= 0.25 && m2 <= 2.25) ? 1 : 0;
                    }
                    ur[r][f] = (float)(vr - wd[6 * p + 2 * f]);
                    ui[r][f] = (float)(vi - wd[6 * p + 2 * f + 1]);
                }
            }
        }
        if (V0) {
#pragma unroll
            for (int off = LPC / 2; off > 0; off >>= 1) ok &= __shfl_xor(ok, off);
            if (!ok) {
#pragma unroll
                for (int r = 0; r < B; ++r) {
                    const int p = 1 + sl + LPC * r;
                    if (p <= nb) {
#pragma unroll
                        for (int f = 0; f < 3; ++f) {
                            ur[r][f] = (float)(1.0 - wd[6 * p + 2 * f]);
                            ui[r][f] = (float)(0.0 - wd[6 * p + 2 * f + 1]);
                        }
                    }
                }
            }
        }
        it = 0;
    };
    load();
    while (__ballot(c < tau)) {
        const bool live = c < tau;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            if (p <= nb) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const float vr = tz[TZ * p + 18 + 2 * f] + ur[r][f], vi = tz[TZ * p + 19 + 2 * f] + ui[r][f];
                    const float inv = 1.0f / fmaxf(vr * vr + vi * vi, kMinV2);
                    J[6 * p + 2 * f] = (sr[r][f] * vr + si[r][f] * vi) * inv;
                    J[6 * p + 2 * f + 1] = (sr[r][f] * vi - si[r][f] * vr) * inv;
                }
            }
        }
        wave_sync();
        for (int L = levels; L >= 1; --L) {
            for (int p = ls[L] + sl; p < ls[L + 1]; p += LPC) {
                float j[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) j[e] = J[6 * p + e];
                for (int ch = ti[4 * p + 2]; ch < ti[4 * p + 3]; ++ch) {
#pragma unroll
                    for (int e = 0; e < 6; ++e) j[e] += J[6 * ch + e];
                }
#pragma unroll
                for (int e = 0; e < 6; ++e) J[6 * p + e] = j[e];
            }
            wave_sync();
        }
        for (int L = 1; L <= levels; ++L) {
            for (int p = ls[L] + sl; p < ls[L + 1]; p += LPC) {
                const int par = ti[4 * p + 1];
                float j[6], d[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) j[e] = J[6 * p + e], d[e] = J[6 * par + e];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const float zr = tz[TZ * p + 2 * (3 * a + b)], zi = tz[TZ * p + 2 * (3 * a + b) + 1];
                        d[2 * a] += zr * j[2 * b] - zi * j[2 * b + 1];
                        d[2 * a + 1] += zr * j[2 * b + 1] + zi * j[2 * b];
                    }
                }
#pragma unroll
                for (int e = 0; e < 6; ++e) J[6 * p + e] = d[e];
            }
            wave_sync();
        }
        float dmax = 0.0f;
        int bad = 0;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int p = 1 + sl + LPC * r;
            if (p <= nb) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const float nr = -J[6 * p + 2 * f], ni = -J[6 * p + 2 * f + 1];
                    const float er = nr - ur[r][f], ei = ni - ui[r][f];
                    const float e = er * er + ei * ei;
                    bad |= !(e < INFINITY);
                    dmax = e > dmax ? e : dmax;
                    ur[r][f] = nr;
                    ui[r][f] = ni;
                }
            }
        }
#pragma unroll
        for (int off = LPC / 2; off > 0; off >>= 1) {
            dmax = fmaxf(dmax, __shfl_xor(dmax, off));
            bad |= __shfl_xor(bad, off);
        }
        ++it;
        const bool conv = !bad && sqrtf(dmax) < tol;
        if (live && (bad || conv || it >= max_iter)) {
#pragma unroll
            for (int r = 0; r < B; ++r) {
                const int p = 1 + sl + LPC * r;
                if (p <= nb) {
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const long long o = 2 * (c * n + 3 * ti[4 * p] + f);
                        Vout[o] = (IO)(wd[6 * p + 2 * f] + (double)ur[r][f]);
                        Vout[o + 1] = (IO)(wd[6 * p + 2 * f + 1] + (double)ui[r][f]);
                    }
                }
            }
            if (sl == 0) {
                iters_out[c] = it;
                status_out[c] = bad ? TPF_ST_NONFINITE : (conv ? TPF_ST_CONVERGED : TPF_ST_MAX_ITER);
            }
            c += nslots;
            load();
        }
        wave_sync();
    }
}

template <typename IO, int CPW, int B>
int launch3_32_as(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                  int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    const int nb = net.n / 3, np = nb + 1, levels = dn.tree_levels;
    const size_t lds = (size_t)6 * np * 8 + (size_t)24 * np * 4 + (size_t)kTreeWaves * CPW * 6 * np * 4 +
                       (size_t)(4 * np + levels + 2) * 4;
    if (lds > (size_t)160 * 1024) return fail(TPF_ERR_UNSUPPORTED, "tree operator: network too large for LDS");
    auto k = fpi_tree3_32_kernel<IO, CPW, B>;
    if (hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kTreeWaves * 64, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long per_block = (long long)kTreeWaves * CPW;
    const long long blocks =
        std::max<long long>(1, std::min<long long>((long long)cus * per_cu, (tau + per_block - 1) / per_block));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kTreeWaves * 64), lds, st, (const IO *)S, (IO *)V, iters,
                       status, (const IO *)V0, dn.tree_i, dn.tree_z, nb, levels, (long long)tau, (float)tol,
                       max_iter);
    return TPF_OK;
}

template <typename IO>
int launch3_32_io(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol,
                  int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    const int nb = net.n / 3;
    if (nb <= 128) return launch3_32_as<IO, 2, 4>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (nb <= 256) return launch3_32_as<IO, 1, 4>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (nb <= 512) return launch3_32_as<IO, 1, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    return fail(TPF_ERR_UNSUPPORTED, "tree operator: up to 512 three-phase buses");
}

template <typename IO, int CPW, int B>
int launch3_as(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol, int max_iter,
               const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    const int nb = net.n / 3, np = nb + 1, levels = dn.tree_levels;
    const size_t lds = (size_t)24 * np * 8 + (size_t)kTreeWaves * CPW * 6 * np * 8 + (size_t)(4 * np + levels + 2) * 4;
    if (lds > (size_t)160 * 1024) return fail(TPF_ERR_UNSUPPORTED, "tree operator: network too large for LDS");
    auto k = fpi_tree3_kernel<IO, CPW, B>;
    if (hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kTreeWaves * 64, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long per_block = (long long)kTreeWaves * CPW;
    const long long blocks =
        std::max<long long>(1, std::min<long long>((long long)cus * per_cu, (tau + per_block - 1) / per_block));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kTreeWaves * 64), lds, st, (const IO *)S, (IO *)V, iters,
                       status, (const IO *)V0, dn.tree_i, dn.tree_z, nb, levels, (long long)tau, tol, max_iter);
    return TPF_OK;
}

// Three-phase FP64: 2 columns per wavefront up to 128 buses, then 1, as far as the LDS holds
// the per-position state (3x3 blocks, w and the per-column drops: 400 bytes per position
// with 4 wavefronts, so up to 408 buses); larger networks return TPF_ERR_UNSUPPORTED from
// the launch (the FP32 form reaches 512).
template <typename IO>
int launch3_io(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol, int max_iter,
               const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    const int nb = net.n / 3;
    if (nb <= 128) return launch3_as<IO, 2, 4>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (nb <= 256) return launch3_as<IO, 1, 4>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (nb <= 512) return launch3_as<IO, 1, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    return fail(TPF_ERR_UNSUPPORTED, "tree operator: up to 512 three-phase buses");
}

template <typename IO, int CPW, int B, int ZM>
int launch_as(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol, int max_iter,
              const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    const int n = net.n, np = n + 1, levels = dn.tree_levels;
    const size_t lds = (size_t)4 * np * 8 + (size_t)(ZM ? ZM + 1 : 0) * np * 8 +
                       (size_t)(ZM == 2 ? 2 : 1) * kTreeWaves * CPW * 2 * np * 8 + (size_t)(4 * np + levels + 2) * 4;
    if (lds > (size_t)160 * 1024) return fail(TPF_ERR_UNSUPPORTED, "tree operator: network too large for LDS");
    auto k = fpi_tree_kernel<IO, CPW, B, ZM>;
    if (hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(TPF_ERR_DEVICE, "hipFuncSetAttribute failed");
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kTreeWaves * 64, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long per_block = (long long)kTreeWaves * CPW;
    const long long blocks =
        std::max<long long>(1, std::min<long long>((long long)cus * per_cu, (tau + per_block - 1) / per_block));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(kTreeWaves * 64), lds, st, (const IO *)S, (IO *)V, iters,
                       status, (const IO *)V0, dn.tree_i, dn.tree_z, n, levels, (long long)tau, tol, max_iter,
                       (const double *)dn.aP, (const double *)dn.aI, (const double *)dn.aZ, net.vs.real(),
                       net.vs.imag());
    return TPF_OK;
}

template <typename IO, int CPW, int B>
int launch_b(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol, int max_iter,
             const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    // a constant-impedance share doubles the per-column LDS state (G' beside J): half the
    // columns per wavefront, each over twice the lanes, keeps the workgroups per CU (100-bus
    // year with alpha_Z: 2.00 ms against 2.74 ms with the constant-power shape)
    if (dn.aZ) {
        if constexpr (CPW >= 2)
            return launch_as<IO, CPW / 2, B / 2, 2>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
        else
            return launch_as<IO, CPW, B, 2>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    }
    if (dn.aP) return launch_as<IO, CPW, B, 1>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    return launch_as<IO, CPW, B, 0>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
}

// Columns per wavefront: 8 (8 lanes each) up to 128 buses, 2 up to 256, then 1.  (At 99
// buses: 1.40 ms per year with 8 columns, 1.51 with 4, 2.48 with 1.)
template <typename IO>
int launch_io(const tpf_network_s &net, const DeviceNet &dn, const void *S, int64_t tau, double tol, int max_iter,
              const void *V0, void *V, int32_t *iters, int8_t *status, hipStream_t st) {
    const int n = net.n;
    if (n <= 64) return launch_b<IO, 8, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (n <= 128) return launch_b<IO, 8, 16>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (n <= 256) return launch_b<IO, 2, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (n <= 512) return launch_b<IO, 1, 8>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    if (n <= 1024) return launch_b<IO, 1, 16>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, st);
    return fail(TPF_ERR_UNSUPPORTED, "tree operator: up to 1,024 PQ buses");
}

}  // namespace

int launch_fpi_tree(const tpf_network_s &net, const DeviceNet &dn, int mode, const void *S, int dtype, int64_t tau,
                    double tol, int max_iter, const void *V0, void *V, int32_t *iters, int8_t *status,
                    hipStream_t stream) {
    if (!dn.tree_i) return fail(TPF_ERR_UNSUPPORTED, "the tree operator needs a radial network (n_bus - 1 branches)");
    if (mode == TPF_MODE_TREE_FP32) {
        if (dn.tree_phases == 3) {
            if (dtype == TPF_C128)
                return launch3_32_io<double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, stream);
            return launch3_32_io<float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, stream);
        }
        if (dtype == TPF_C128)
            return launch32_io<double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, stream);
        return launch32_io<float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, stream);
    }
    if (dn.tree_phases == 3) {
        if (dtype == TPF_C128)
            return launch3_io<double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, stream);
        return launch3_io<float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, stream);
    }
    if (dtype == TPF_C128)
        return launch_io<double>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, stream);
    return launch_io<float>(net, dn, S, tau, tol, max_iter, V0, V, iters, status, stream);
}

}  // namespace tpf
