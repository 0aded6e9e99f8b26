// Network build (host, FP64) and per-device staging of the sweep operator.
//
// Sec. II Eq. (1): nodal admittance Y from the series branches, partitioned into
// the slack block and the demand block; Eq. (2) with constant-power loads:
// Z = -Y_dd^-1 and w = -Y_dd^-1 Y_ds v_s, computed once per network (the paper
// notes F and w stay constant through the iteration).  Y_dd is factorised here
// by LU with partial pivoting; the solve kernels never see Y_dd except through
// the FP64 mismatch check.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <queue>

#include "tpf_internal.h"

namespace tpf {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}
void clear_error() { g_err.clear(); }

// In-place LU with partial pivoting of a dense n x n complex matrix (row-major);
// returns false when a pivot is negligible against the matrix scale.
static bool lu_factor(std::vector<cd> &a, std::vector<int> &piv, int n) {
    double scale = 0.0;
    for (const cd &v : a) scale = std::max(scale, std::abs(v));
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::abs(a[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = std::abs(a[(size_t)i * n + k]);
            if (v > best) best = v, p = i;
        }
        if (!(best > 1e-13 * scale)) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(a[(size_t)k * n + j], a[(size_t)p * n + j]);
        const cd inv = 1.0 / a[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            cd f = a[(size_t)i * n + k] * inv;
            a[(size_t)i * n + k] = f;
            if (f == 0.0) continue;
            for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= f * a[(size_t)k * n + j];
        }
    }
    return true;
}

// Solves LU x = b in place (b length n).
static void lu_solve(const std::vector<cd> &lu, const std::vector<int> &piv, int n, cd *b) {
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int i = 1; i < n; ++i) {
        cd s = b[i];
        for (int j = 0; j < i; ++j) s -= lu[(size_t)i * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        cd s = b[i];
        for (int j = i + 1; j < n; ++j) s -= lu[(size_t)i * n + j] * b[j];
        b[i] = s / lu[(size_t)i * n + i];
    }
}

// Row/column position of (PQ bus q, part) inside the real-block operator used by
// the small-network kernels: each 16-row tile holds 8 buses, real parts in rows
// 0-7 and imaginary parts in rows 8-15, so that the FP64 MFMA output layout
// (lane group g holds tile rows g, g+4, g+8, g+12) keeps Re and Im of a bus in
// one lane.
static inline int blk_pos(int q, int part) { return 16 * (q / 8) + 8 * part + (q % 8); }

// Order of the FP32-family kernels: Re/Im of a bus on adjacent tile rows so that
// the 16x16 output layout (rows 4g..4g+3 in lane group g) keeps a bus in one lane.
static inline int blk_pos32(int q, int part) { return 16 * (q / 8) + 2 * (q % 8) + part; }

static uint16_t to_bf16(float f) {  // round to nearest even
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static uint16_t to_f16(float f) {
    _Float16 h = (_Float16)f;
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}
static float from_f16(uint16_t u) {
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return (float)h;
}

static int upload(tpf_network_s &net, DeviceNet &dn) {
    const int n = net.n;
    auto dalloc = [&](void **p, size_t bytes) -> bool {
        if (hipMalloc(p, bytes) != hipSuccess) return false;
        dn.owned.push_back(*p);
        return true;
    };
    auto h2d = [&](void *dst, const void *src, size_t bytes) -> bool {
        return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    // ---- small-network FP64 fragments
    if (n <= 8 * kMaxSmallTiles) {
        const int MT = (n + 7) / 8, M = 16 * MT, KT = 4 * MT;
        dn.MT = MT;
        std::vector<double> Ab((size_t)M * M, 0.0);  // real-block operator, permuted rows/cols
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                const cd z = net.Z[(size_t)i * n + k];
                Ab[(size_t)blk_pos(i, 0) * M + blk_pos(k, 0)] = z.real();
                Ab[(size_t)blk_pos(i, 0) * M + blk_pos(k, 1)] = -z.imag();
                Ab[(size_t)blk_pos(i, 1) * M + blk_pos(k, 0)] = z.imag();
                Ab[(size_t)blk_pos(i, 1) * M + blk_pos(k, 1)] = z.real();
            }
        // 16x16x4 FP64 MFMA A operand: lane 16*kk + ii holds A[16*mt + ii][4*kt + kk].  Grouped
        // by the wave role that multiplies tile mt (mt % NW), so that one wave's fragments
        // of a k-step are contiguous.
        int NW = 0, TPW = 0;
        rows_config(MT, NW, TPW);
        dn.NW = NW;
        dn.TPW = TPW;
        const int KP = KT + kFragPadSteps;
        std::vector<double> frag((size_t)NW * KP * TPW * 64, 0.0);
        for (int tw = 0; tw < NW; ++tw)
            for (int kt = 0; kt < KT; ++kt)
                for (int q = 0; q < TPW; ++q) {
                    const int mt = tw + NW * q;
                    if (mt >= MT) continue;
                    for (int l = 0; l < 64; ++l)
                        frag[(((size_t)tw * KP + kt) * TPW + q) * 64 + l] =
                            Ab[(size_t)(16 * mt + (l % 16)) * M + 4 * kt + l / 16];
                }
        std::vector<double> wv(2 * 8 * MT);
        for (int q = 0; q < 8 * MT; ++q) {
            wv[q] = q < n ? net.w[q].real() : 1.0;
            wv[8 * MT + q] = q < n ? net.w[q].imag() : 0.0;
        }
        if (!dalloc((void **)&dn.A64, frag.size() * 8) || !dalloc((void **)&dn.w64, wv.size() * 8))
            return fail(TPF_ERR_OOM, "device allocation failed (network staging)");
        if (!h2d(dn.A64, frag.data(), frag.size() * 8) || !h2d(dn.w64, wv.data(), wv.size() * 8))
            return fail(TPF_ERR_DEVICE, "host-to-device copy failed (network staging)");
    }
    // ---- FP32-family fragments (FP32 and mixed modes)
    if (n <= 8 * 16) {
        const int MT = dn.MT, M = 16 * MT, KT = 4 * MT, NW = dn.NW, TPW = dn.TPW;
        const int KTL = (MT + 1) / 2, KL = 32 * KTL;
        dn.KTL = KTL;
        std::vector<double> Ab((size_t)M * KL, 0.0);
        double zmax = 0.0;
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) {
                const cd z = net.Z[(size_t)i * n + k];
                Ab[(size_t)blk_pos32(i, 0) * KL + blk_pos32(k, 0)] = z.real();
                Ab[(size_t)blk_pos32(i, 0) * KL + blk_pos32(k, 1)] = -z.imag();
                Ab[(size_t)blk_pos32(i, 1) * KL + blk_pos32(k, 0)] = z.imag();
                Ab[(size_t)blk_pos32(i, 1) * KL + blk_pos32(k, 1)] = z.real();
                zmax = std::max(zmax, std::max(std::abs(z.real()), std::abs(z.imag())));
            }
        // FP16 operands carry Z 2^sZ with the largest entry just below 2^14.
        int e = 0;
        (void)std::frexp(zmax > 0 ? zmax : 1.0, &e);
        dn.sZ = 14 - e;
        const int KP = KT + kFragPadSteps;
        std::vector<float> f32((size_t)NW * KP * TPW * 64, 0.0f);
        const size_t nl = (size_t)NW * TPW * KTL * 64 * 8;
        std::vector<uint16_t> fbf(nl, 0), fh(nl, 0), fl(nl, 0);
        for (int tw = 0; tw < NW; ++tw)
            for (int q = 0; q < TPW; ++q) {
                const int mt = tw + NW * q;
                if (mt >= MT) continue;
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * mt + (l % 16), kk = l / 16;
                    for (int kt = 0; kt < KT; ++kt)
                        f32[(((size_t)tw * KP + kt) * TPW + q) * 64 + l] = (float)Ab[(size_t)row * KL + 4 * kt + kk];
                    for (int kt = 0; kt < KTL; ++kt)
                        for (int x = 0; x < 8; ++x) {
                            const double a = Ab[(size_t)row * KL + 32 * kt + 8 * kk + x];
                            const size_t idx = ((((size_t)tw * TPW + q) * KTL + kt) * 64 + l) * 8 + x;
                            fbf[idx] = to_bf16((float)a);
                            const float as = (float)std::ldexp(a, dn.sZ);
                            fh[idx] = to_f16(as);
                            fl[idx] = to_f16(as - from_f16(fh[idx]));
                        }
                }
            }
        if (!dalloc((void **)&dn.A32, f32.size() * 4) || !dalloc((void **)&dn.Abf, nl * 2) ||
            !dalloc((void **)&dn.Ah, nl * 2) || !dalloc((void **)&dn.Al, nl * 2))
            return fail(TPF_ERR_OOM, "device allocation failed (network staging)");
        if (!h2d(dn.A32, f32.data(), f32.size() * 4) || !h2d(dn.Abf, fbf.data(), nl * 2) ||
            !h2d(dn.Ah, fh.data(), nl * 2) || !h2d(dn.Al, fl.data(), nl * 2))
            return fail(TPF_ERR_DEVICE, "host-to-device copy failed (network staging)");
    }
    // ---- large-network operator (FP64 beyond the register kernels, FP32 beyond 128 buses)
    if (n > 128) {
        const int KP = (2 * n + 15) / 16 * 16, K16 = (2 * n + 31) / 32 * 32;
        const int M64 = (16 * ((n + 7) / 8) + 63) / 64 * 64, M32 = (2 * n + 127) / 128 * 128;
        dn.KPL = KP;
        dn.KPL16 = K16;
        dn.MPL64 = M64;
        dn.MPL32 = M32;
        double zmax = 0.0;
        for (size_t i = 0; i < (size_t)n * n; ++i)
            zmax = std::max(zmax, std::max(std::abs(net.Z[i].real()), std::abs(net.Z[i].imag())));
        int e = 0;
        (void)std::frexp(zmax > 0 ? zmax : 1.0, &e);
        dn.sZ = 14 - e;  // FP16 operand Z 2^sZ: largest entry just below 2^14
        if (hipHostMalloc((void **)&dn.done_host, 256, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            dn.done_host = nullptr;
            return fail(TPF_ERR_OOM, "pinned host allocation failed (network staging)");
        }
        *dn.done_host = 0;
        if (hipHostGetDevicePointer((void **)&dn.done_dev, dn.done_host, 0) != hipSuccess)
            return fail(TPF_ERR_DEVICE, "pinned host word not mapped (network staging)");
        std::vector<double> a64((size_t)M64 * KP, 0.0);
        std::vector<float> a32((size_t)M32 * KP, 0.0f);
        std::vector<uint16_t> abf((size_t)M32 * K16, 0), ah((size_t)M32 * K16, 0);
        std::vector<double> wn(2 * n);
        for (int i = 0; i < n; ++i) {
            wn[2 * i] = net.w[i].real();
            wn[2 * i + 1] = net.w[i].imag();
            for (int k = 0; k < n; ++k) {
                const cd z = net.Z[(size_t)i * n + k];
                const double blk[2][2] = {{z.real(), -z.imag()}, {z.imag(), z.real()}};
                for (int pi = 0; pi < 2; ++pi)
                    for (int pk = 0; pk < 2; ++pk) {
                        a64[(size_t)blk_pos(i, pi) * KP + 2 * k + pk] = blk[pi][pk];
                        a32[(size_t)(2 * i + pi) * KP + 2 * k + pk] = (float)blk[pi][pk];
                        abf[(size_t)(2 * i + pi) * K16 + 2 * k + pk] = to_bf16((float)blk[pi][pk]);
                        ah[(size_t)(2 * i + pi) * K16 + 2 * k + pk] = to_f16((float)std::ldexp(blk[pi][pk], dn.sZ));
                    }
            }
        }
        if (!dalloc((void **)&dn.AL64, a64.size() * 8) || !dalloc((void **)&dn.AL32, a32.size() * 4) ||
            !dalloc((void **)&dn.ALbf, abf.size() * 2) || !dalloc((void **)&dn.ALh, ah.size() * 2) ||
            !dalloc((void **)&dn.wl, wn.size() * 8))
            return fail(TPF_ERR_OOM, "device allocation failed (network staging)");
        if (!h2d(dn.AL64, a64.data(), a64.size() * 8) || !h2d(dn.AL32, a32.data(), a32.size() * 4) ||
            !h2d(dn.ALbf, abf.data(), abf.size() * 2) || !h2d(dn.ALh, ah.data(), ah.size() * 2) ||
            !h2d(dn.wl, wn.data(), wn.size() * 8))
            return fail(TPF_ERR_DEVICE, "host-to-device copy failed (network staging)");
    }
    // ---- CSR Y_dd and c = Y_ds v_s (FP64 mismatch)
    {
        const size_t nnz = net.colidx.size();
        std::vector<double> yv(2 * nnz), cv(2 * n);
        for (size_t e = 0; e < nnz; ++e) yv[2 * e] = net.yval[e].real(), yv[2 * e + 1] = net.yval[e].imag();
        for (int i = 0; i < n; ++i) cv[2 * i] = net.c[i].real(), cv[2 * i + 1] = net.c[i].imag();
        if (!dalloc((void **)&dn.rowptr, (n + 1) * 4) || !dalloc((void **)&dn.colidx, nnz * 4) ||
            !dalloc((void **)&dn.yval, nnz * 16) || !dalloc((void **)&dn.cval, n * 16))
            return fail(TPF_ERR_OOM, "device allocation failed (network staging)");
        if (!h2d(dn.rowptr, net.rowptr.data(), (n + 1) * 4) || !h2d(dn.colidx, net.colidx.data(), nnz * 4) ||
            !h2d(dn.yval, yv.data(), nnz * 16) || !h2d(dn.cval, cv.data(), n * 16))
            return fail(TPF_ERR_DEVICE, "host-to-device copy failed (network staging)");
    }
    // ---- breadth-first tree (radial networks): per position the branch impedance
    // (phases x phases) and w of its phases, as doubles
    if (!net.tree_pq.empty()) {
        const int levels = (int)net.tree_level_start.size() - 2;
        const int np = (int)net.tree_pq.size(), ph = net.tree_phases, pp = ph * ph, stride = 2 * (pp + ph);
        std::vector<int32_t> ti(4 * np + levels + 2);
        std::vector<double> tz((size_t)stride * np);
        for (int p = 0; p < np; ++p) {
            ti[4 * p] = net.tree_pq[p];
            ti[4 * p + 1] = net.tree_parent[p];
            ti[4 * p + 2] = net.tree_c0[p];
            ti[4 * p + 3] = net.tree_c1[p];
            for (int e = 0; e < pp; ++e) {
                tz[(size_t)stride * p + 2 * e] = net.tree_z[(size_t)pp * p + e].real();
                tz[(size_t)stride * p + 2 * e + 1] = net.tree_z[(size_t)pp * p + e].imag();
            }
            for (int f = 0; f < ph; ++f) {
                const tpf::cd wq = p > 0 ? net.w[ph * net.tree_pq[p] + f] : tpf::cd(0.0);
                tz[(size_t)stride * p + 2 * pp + 2 * f] = wq.real();
                tz[(size_t)stride * p + 2 * pp + 2 * f + 1] = wq.imag();
            }
        }
        for (int L = 0; L < levels + 2; ++L) ti[4 * np + L] = net.tree_level_start[L];
        if (!dalloc((void **)&dn.tree_i, ti.size() * 4) || !dalloc((void **)&dn.tree_z, tz.size() * 8))
            return fail(TPF_ERR_OOM, "device allocation failed (tree)");
        if (!h2d(dn.tree_i, ti.data(), ti.size() * 4) || !h2d(dn.tree_z, tz.data(), tz.size() * 8))
            return fail(TPF_ERR_DEVICE, "host-to-device copy failed (tree)");
        dn.tree_levels = levels;
        dn.tree_phases = ph;
    }
    // ---- ZIP shares
    if (net.zip) {
        if (!dalloc((void **)&dn.aI, n * 8) || !dalloc((void **)&dn.aP, n * 8))
            return fail(TPF_ERR_OOM, "device allocation failed (ZIP shares)");
        if (!h2d(dn.aI, net.alpha_i.data(), n * 8) || !h2d(dn.aP, net.alpha_p.data(), n * 8))
            return fail(TPF_ERR_DEVICE, "host-to-device copy failed (ZIP shares)");
        double zs = 0.0;
        for (int q = 0; q < n; ++q)
            zs = std::max(zs, std::fabs(net.alpha_p[q]) + std::fabs(net.alpha_i[q]) +
                                  (net.alpha_z.empty() ? 0.0 : std::fabs(net.alpha_z[q])));
        dn.zscale = (float)zs;
        if (!net.alpha_z.empty()) {
            if (!dalloc((void **)&dn.aZ, n * 8)) return fail(TPF_ERR_OOM, "device allocation failed (ZIP shares)");
            if (!h2d(dn.aZ, net.alpha_z.data(), n * 8))
                return fail(TPF_ERR_DEVICE, "host-to-device copy failed (ZIP shares)");
        }
    }
    return TPF_OK;
}

int device_net(tpf_network net, DeviceNet **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TPF_ERR_DEVICE, "hipGetDevice failed (no GPU?)");
    std::lock_guard<std::mutex> lock(net->mu);
    if ((int)net->dev.size() <= dev) net->dev.resize(dev + 1, nullptr);
    if (!net->dev[dev]) {
        auto *dn = new (std::nothrow) DeviceNet();
        if (!dn) return fail(TPF_ERR_OOM, "host allocation failed");
        dn->device = dev;
        int rc = upload(*net, *dn);
        if (rc != TPF_OK) {
            for (void *p : dn->owned) (void)hipFree(p);
            if (dn->done_host) (void)hipHostFree(dn->done_host);
            delete dn;
            return rc;
        }
        net->dev[dev] = dn;
    }
    *out = net->dev[dev];
    return TPF_OK;
}

int device_net_resident(tpf_network net, DeviceNet **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TPF_ERR_DEVICE, "hipGetDevice failed (no GPU?)");
    std::lock_guard<std::mutex> lock(net->mu);
    if ((int)net->dev.size() <= dev || !net->dev[dev])
        return fail(TPF_ERR_UNSUPPORTED, "the network is not yet resident on this device (a first tpf_solve_timeseries, "
                                         "tpf_solve_tensor or tpf_mismatch call with it uploads it)");
    *out = net->dev[dev];
    return TPF_OK;
}

}  // namespace tpf

using namespace tpf;

// Checks of the bus-level topology shared by the builders: indices, self loops, and that
// every bus reaches the slack (else Y_dd is singular).
static int check_topology(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                          int32_t slack_bus) {
    if (n_bus < 2) return fail(TPF_ERR_INVALID_ARG, "n_bus must be >= 2");
    if (n_branch < 1) return fail(TPF_ERR_INVALID_ARG, "n_branch must be >= 1");
    if (!from || !to) return fail(TPF_ERR_INVALID_ARG, "branch arrays must not be NULL");
    if (slack_bus < 0 || slack_bus >= n_bus) return fail(TPF_ERR_INVALID_ARG, "slack_bus out of range");
    for (int k = 0; k < n_branch; ++k) {
        if (from[k] < 0 || from[k] >= n_bus || to[k] < 0 || to[k] >= n_bus)
            return fail(TPF_ERR_INVALID_ARG, "branch " + std::to_string(k) + ": bus index out of range");
        if (from[k] == to[k]) return fail(TPF_ERR_INVALID_ARG, "branch " + std::to_string(k) + ": from == to");
    }
    std::vector<std::vector<int>> adj(n_bus);
    for (int k = 0; k < n_branch; ++k) adj[from[k]].push_back(to[k]), adj[to[k]].push_back(from[k]);
    std::vector<char> seen(n_bus, 0);
    std::queue<int> q;
    q.push(slack_bus);
    seen[slack_bus] = 1;
    int cnt = 1;
    while (!q.empty()) {
        int u = q.front();
        q.pop();
        for (int v : adj[u])
            if (!seen[v]) seen[v] = 1, ++cnt, q.push(v);
    }
    if (cnt != n_bus) return fail(TPF_ERR_SINGULAR, "network is not connected: some bus cannot reach the slack");
    return TPF_OK;
}

// Branches of a radial network (n_bus - 1 branches, connected), for its tree layout and
// its factorisation-free Z.
struct TreeBranches {
    int32_t n_branch;
    const int32_t *from, *to;
    std::vector<cd> zbr;  // phases x phases per branch, row-major
    int phases;
};

static void build_tree(tpf_network_s &net, int32_t n_branch, const int32_t *from, const int32_t *to,
                       const std::vector<cd> &zbr, int phases);

// Eq. (2) for a radial network with series branches only: Y_dd = A^T diag(y_b) A with A
// the square branch-bus incidence of the tree, whose inverse marks the branches on each
// bus's path from the slack.  So Y_dd^-1 between demand nodes of buses p and q is the sum
// of the impedance blocks of the branches their two paths share, and Z = -Y_dd^-1 follows
// in O(n^2) from the tree layout: the row of bus p is its parent's row, with the columns
// of p's subtree set to p's own path impedance.
static void tree_inverse(tpf_network_s &net) {
    const int N = net.n_bus, P = net.tree_phases, n = net.n, pp = P * P;
    const auto &par = net.tree_parent, &c0 = net.tree_c0, &c1 = net.tree_c1;
    // path impedance per position (positions are breadth-first: parents come first)
    std::vector<cd> zp((size_t)N * pp, 0.0);
    for (int p = 1; p < N; ++p)
        for (int e = 0; e < pp; ++e) zp[(size_t)p * pp + e] = zp[(size_t)par[p] * pp + e] + net.tree_z[(size_t)p * pp + e];
    // depth-first preorder: each subtree is the contiguous range [pre[p], pre[p] + size[p])
    std::vector<int> pre(N), size(N, 1), dfs;
    dfs.reserve(N);
    std::vector<int> stack = {0};
    while (!stack.empty()) {
        const int u = stack.back();
        stack.pop_back();
        pre[u] = (int)dfs.size();
        dfs.push_back(u);
        for (int v = c1[u] - 1; v >= c0[u]; --v) stack.push_back(v);
    }
    for (int p = N - 1; p >= 1; --p) size[par[p]] += size[p];
    net.Z.assign((size_t)n * n, 0.0);
    for (int i = 1; i < N; ++i) {  // preorder: the parent's rows are already complete
        const int p = dfs[i], k = net.tree_pq[p], pa = par[p];
        for (int a = 0; a < P; ++a) {
            cd *row = &net.Z[(size_t)(P * k + a) * n];
            if (pa > 0) std::copy_n(&net.Z[(size_t)(P * net.tree_pq[pa] + a) * n], n, row);
            for (int j = pre[p]; j < pre[p] + size[p]; ++j) {
                const int m = net.tree_pq[dfs[j]];
                for (int b = 0; b < P; ++b) row[P * m + b] = -zp[(size_t)p * pp + a * P + b];
            }
        }
    }
}

// Sec. II Eqs. (1)-(2) from a node-level admittance matrix Y [Nn][Nn]: the slack nodes
// (with their voltages) against the demand nodes in ascending node order; CSR of Y_dd,
// c = Y_ds v_s, Z = -Y_dd^-1 (LU with partial pivoting, or the path sums of tree_inverse
// for a radial network given its branches), w = Z c.
static int finish_network(const std::vector<cd> &Y, int Nn, const std::vector<int> &slack_nodes,
                          const std::vector<cd> &vs_nodes, int n_bus, int slack_bus, const TreeBranches *tree,
                          tpf_network *out) {
    auto *net = new (std::nothrow) tpf_network_s();
    if (!net) return fail(TPF_ERR_OOM, "host allocation failed");
    try {
        const int n = Nn - (int)slack_nodes.size();
        net->n_bus = n_bus;
        net->n = n;
        net->slack = slack_bus;
        net->vs = vs_nodes[0];
        std::vector<char> is_slack(Nn, 0);
        for (int sn : slack_nodes) is_slack[sn] = 1;
        std::vector<int> pq;
        for (int b = 0; b < Nn; ++b)
            if (!is_slack[b]) pq.push_back(b);
        net->c.assign(n, 0.0);
        for (int i = 0; i < n; ++i)
            for (size_t p = 0; p < slack_nodes.size(); ++p)
                net->c[i] += Y[(size_t)pq[i] * Nn + slack_nodes[p]] * vs_nodes[p];
        net->rowptr.assign(1, 0);
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                const cd y = Y[(size_t)pq[i] * Nn + pq[j]];
                if (y != 0.0) net->colidx.push_back(j), net->yval.push_back(y);
            }
            net->rowptr.push_back((int32_t)net->colidx.size());
        }
        if (tree) {
            net->phases = tree->phases;
            build_tree(*net, tree->n_branch, tree->from, tree->to, tree->zbr, tree->phases);
            tree_inverse(*net);
        } else {
            // Eq. (2): Z = -Y_dd^-1 (column by column from the LU factors)
            std::vector<int> piv;
            std::vector<cd> lu((size_t)n * n);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) lu[(size_t)i * n + j] = Y[(size_t)pq[i] * Nn + pq[j]];
            if (!lu_factor(lu, piv, n)) {
                delete net;
                return fail(TPF_ERR_SINGULAR, "Y_dd is numerically singular");
            }
            net->Z.assign((size_t)n * n, 0.0);
            std::vector<cd> col(n);
            for (int j = 0; j < n; ++j) {
                std::fill(col.begin(), col.end(), cd(0.0));
                col[j] = -1.0;
                lu_solve(lu, piv, n, col.data());
                for (int i = 0; i < n; ++i) net->Z[(size_t)i * n + j] = col[i];
            }
        }
        // w = Z (Y_ds v_s)
        net->w.assign(n, 0.0);
        for (int i = 0; i < n; ++i) {
            cd acc = 0.0;
            for (int j = 0; j < n; ++j) acc += net->Z[(size_t)i * n + j] * net->c[j];
            net->w[i] = acc;
        }
    } catch (const std::bad_alloc &) {
        delete net;
        return fail(TPF_ERR_OOM, "host allocation failed");
    }
    *out = net;
    return TPF_OK;
}

// Breadth-first layout of a connected network with n_bus - 1 branches (a tree): the
// positions (buses), parents, children ranges, levels and branch impedances (phases x
// phases per branch, row-major, in zbr) the tree operator walks.  Host work once per
// network.
static void build_tree(tpf_network_s &net, int32_t n_branch, const int32_t *from, const int32_t *to,
                       const std::vector<cd> &zbr, int phases) {
    const int N = net.n_bus, slack = net.slack;
    std::vector<std::vector<std::pair<int, int>>> adj(N);  // (neighbour, branch)
    for (int k = 0; k < n_branch; ++k) adj[from[k]].push_back({to[k], k}), adj[to[k]].push_back({from[k], k});
    std::vector<int> pos(N, -1), order, lev;
    std::vector<int32_t> par, c0, c1;
    const int pp = phases * phases;
    std::vector<cd> zb(pp, 0.0);
    order.push_back(slack);
    pos[slack] = 0;
    par.push_back(-1);
    lev.push_back(0);
    for (size_t h = 0; h < order.size(); ++h) {
        const int u = order[h];
        c0.push_back((int32_t)order.size());
        for (auto [v, k] : adj[u]) {
            if (pos[v] >= 0) continue;
            pos[v] = (int)order.size();
            order.push_back(v);
            par.push_back((int32_t)h);
            lev.push_back(lev[h] + 1);
            zb.insert(zb.end(), zbr.begin() + (size_t)pp * k, zbr.begin() + (size_t)pp * (k + 1));
        }
        c1.push_back((int32_t)order.size());
    }
    const int n = N - 1;  // positions 1..n are the non-slack buses
    net.tree_phases = phases;
    net.tree_pq.assign(n + 1, -1);
    for (int p = 1; p <= n; ++p) net.tree_pq[p] = order[p] < slack ? order[p] : order[p] - 1;
    net.tree_parent = par;
    net.tree_c0 = c0;
    net.tree_c1 = c1;
    net.tree_z = zb;
    net.tree_level_start.clear();
    for (int p = 0; p <= n; ++p)
        if (p == 0 || lev[p] != lev[p - 1]) net.tree_level_start.push_back(p);
    net.tree_level_start.push_back(n + 1);
}

extern "C" int tpf_build_network(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                                 const double *r, const double *x, int32_t slack_bus, double vs_re,
                                 double vs_im, tpf_network *out) {
    clear_error();
    if (!out) return fail(TPF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_topology(n_bus, n_branch, from, to, slack_bus);
    if (rc != TPF_OK) return rc;
    if (!r || !x) return fail(TPF_ERR_INVALID_ARG, "branch arrays must not be NULL");
    if (!std::isfinite(vs_re) || !std::isfinite(vs_im)) return fail(TPF_ERR_INVALID_ARG, "slack voltage not finite");
    for (int k = 0; k < n_branch; ++k) {
        if (!std::isfinite(r[k]) || !std::isfinite(x[k]))
            return fail(TPF_ERR_INVALID_ARG, "branch " + std::to_string(k) + ": impedance not finite");
        if (r[k] == 0.0 && x[k] == 0.0)
            return fail(TPF_ERR_INVALID_ARG, "branch " + std::to_string(k) + ": zero impedance");
    }
    const int N = n_bus;
    std::vector<cd> Y;
    try {
        // Eq. (1): branch admittances stamped into Y.
        Y.assign((size_t)N * N, 0.0);
        for (int k = 0; k < n_branch; ++k) {
            const cd y = 1.0 / cd(r[k], x[k]);
            const int f = from[k], t = to[k];
            Y[(size_t)f * N + f] += y;
            Y[(size_t)t * N + t] += y;
            Y[(size_t)f * N + t] -= y;
            Y[(size_t)t * N + f] -= y;
        }
    } catch (const std::bad_alloc &) {
        return fail(TPF_ERR_OOM, "host allocation failed");
    }
    TreeBranches tb{n_branch, from, to, {}, 1};
    const bool radial = n_branch == n_bus - 1;  // connected (checked) with n_bus - 1 branches
    try {
        if (radial) {
            tb.zbr.resize(n_branch);
            for (int k = 0; k < n_branch; ++k) tb.zbr[k] = cd(r[k], x[k]);
        }
    } catch (const std::bad_alloc &) {
        return fail(TPF_ERR_OOM, "host allocation failed");
    }
    return finish_network(Y, N, {slack_bus}, {cd(vs_re, vs_im)}, n_bus, slack_bus, radial ? &tb : nullptr, out);
}

extern "C" int tpf_build_network_3ph(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                                     const double *zabc, int32_t slack_bus, const double *vs_abc,
                                     tpf_network *out) {
    clear_error();
    if (!out) return fail(TPF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_topology(n_bus, n_branch, from, to, slack_bus);
    if (rc != TPF_OK) return rc;
    if (!zabc || !vs_abc) return fail(TPF_ERR_INVALID_ARG, "zabc and vs_abc must not be NULL");
    for (int i = 0; i < 6; ++i)
        if (!std::isfinite(vs_abc[i])) return fail(TPF_ERR_INVALID_ARG, "slack voltage not finite");
    const int Nn = 3 * n_bus;
    std::vector<cd> Y;
    try {
        Y.assign((size_t)Nn * Nn, 0.0);
        std::vector<cd> zb(9), yb(9), col(3);
        std::vector<int> piv;
        for (int k = 0; k < n_branch; ++k) {
            for (int e = 0; e < 9; ++e) {
                zb[e] = cd(zabc[18 * (size_t)k + 2 * e], zabc[18 * (size_t)k + 2 * e + 1]);
                if (!std::isfinite(zb[e].real()) || !std::isfinite(zb[e].imag()))
                    return fail(TPF_ERR_INVALID_ARG, "branch " + std::to_string(k) + ": impedance not finite");
            }
            // branch admittance matrix Y_b = Z_abc^-1
            if (!lu_factor(zb, piv, 3))
                return fail(TPF_ERR_INVALID_ARG, "branch " + std::to_string(k) + ": singular impedance matrix");
            for (int j = 0; j < 3; ++j) {
                col = {0.0, 0.0, 0.0};
                col[j] = 1.0;
                lu_solve(zb, piv, 3, col.data());
                for (int i = 0; i < 3; ++i) yb[3 * i + j] = col[i];
            }
            // Eq. (1) with 3x3 blocks: node 3 b + p is phase p of bus b
            const int f = 3 * from[k], t = 3 * to[k];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const cd y = yb[3 * i + j];
                    Y[(size_t)(f + i) * Nn + f + j] += y;
                    Y[(size_t)(t + i) * Nn + t + j] += y;
                    Y[(size_t)(f + i) * Nn + t + j] -= y;
                    Y[(size_t)(t + i) * Nn + f + j] -= y;
                }
        }
    } catch (const std::bad_alloc &) {
        return fail(TPF_ERR_OOM, "host allocation failed");
    }
    const std::vector<int> sn = {3 * slack_bus, 3 * slack_bus + 1, 3 * slack_bus + 2};
    const std::vector<cd> vs = {cd(vs_abc[0], vs_abc[1]), cd(vs_abc[2], vs_abc[3]), cd(vs_abc[4], vs_abc[5])};
    TreeBranches tb{n_branch, from, to, {}, 3};
    const bool radial = n_branch == n_bus - 1;
    try {
        if (radial) {
            tb.zbr.resize((size_t)9 * n_branch);
            for (size_t e = 0; e < tb.zbr.size(); ++e) tb.zbr[e] = cd(zabc[2 * e], zabc[2 * e + 1]);
        }
    } catch (const std::bad_alloc &) {
        return fail(TPF_ERR_OOM, "host allocation failed");
    }
    rc = finish_network(Y, Nn, sn, vs, n_bus, slack_bus, radial ? &tb : nullptr, out);
    if (rc == TPF_OK) (*out)->phases = 3;
    return rc;
}

extern "C" void tpf_free_network(tpf_network net) {
    if (!net) return;
    for (DeviceNet *dn : net->dev) {
        if (!dn) continue;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(dn->device);
        for (void *p : dn->owned) (void)hipFree(p);
        if (dn->done_host) (void)hipHostFree(dn->done_host);
        (void)hipSetDevice(cur);
        delete dn;
    }
    delete net;
}

extern "C" int tpf_network_n_pq(tpf_network net) { return net ? net->n : fail(TPF_ERR_INVALID_ARG, "net is NULL"); }

extern "C" int tpf_network_get_zw(tpf_network net, double *Z_out, double *w_out) {
    clear_error();
    if (!net) return fail(TPF_ERR_INVALID_ARG, "net is NULL");
    if (Z_out) std::memcpy(Z_out, net->Z.data(), net->Z.size() * sizeof(cd));
    if (w_out) std::memcpy(w_out, net->w.data(), net->w.size() * sizeof(cd));
    return TPF_OK;
}

extern "C" const char *tpf_last_error(void) { return tpf::g_err.c_str(); }

extern "C" int tpf_build_network_zip(int32_t n_bus, int32_t n_branch, const int32_t *from, const int32_t *to,
                                     const double *r, const double *x, int32_t slack_bus, double vs_re,
                                     double vs_im, const double *alpha_z, const double *alpha_i,
                                     const double *alpha_p, tpf_network *out) {
    clear_error();
    if (!out) return fail(TPF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_bus < 2) return fail(TPF_ERR_INVALID_ARG, "n_bus must be >= 2");
    if (!alpha_i || !alpha_p) return fail(TPF_ERR_INVALID_ARG, "alpha_i and alpha_p must not be NULL");
    const int n = n_bus - 1;
    bool any_z = false;
    for (int q = 0; q < n; ++q) {
        if (!std::isfinite(alpha_i[q]) || !std::isfinite(alpha_p[q]) || (alpha_z && !std::isfinite(alpha_z[q])))
            return fail(TPF_ERR_INVALID_ARG, "ZIP share of PQ bus " + std::to_string(q) + " not finite");
        any_z |= alpha_z && alpha_z[q] != 0.0;
    }
    tpf_network net = nullptr;
    const int rc = tpf_build_network(n_bus, n_branch, from, to, r, x, slack_bus, vs_re, vs_im, &net);
    if (rc != TPF_OK) return rc;
    try {
        net->alpha_i.assign(alpha_i, alpha_i + n);
        net->alpha_p.assign(alpha_p, alpha_p + n);
        if (any_z) net->alpha_z.assign(alpha_z, alpha_z + n);
    } catch (...) {
        tpf_free_network(net);
        return fail(TPF_ERR_OOM, "host allocation failed");
    }
    net->zip = true;
    *out = net;
    return TPF_OK;
}
