"""GPU parity of the FP32 and mixed-precision sweep forms against the FP64 oracle.

Contract for the fast forms: every returned voltage within 1e-6 pu of the oracle's
solution converged to 1e-10 pu, with the FP64 mismatch within its bound.  The fast
forms compute in FP32 (state) and 16-bit products, so their iterates are not
compared sweep by sweep; what is compared is the solution they stop at.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_04578_amd as tpf
from paper_2403_04578_amd import workloads as W

pytestmark = pytest.mark.gpu

FAST_BOUND = 1e-6
MODES = ["fp32", "mixed_bf16", "mixed_fp16"]


def _dev(S, gpu, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(S)).to(gpu).to(dtype).contiguous()


def _mismatch_bound(onet, tol=1e-6):
    """FP64 mismatch of a solution that is within dv of the fixed point and stopped at
    step d: about |Y_dd row|_1 dv + |S| d / |V|.  With the drop kept in FP32
    (|V - w| <= 0.1 pu, ulp 7.5e-9) dv is at most a few 1e-9."""
    return np.abs(onet.Ydd).sum(axis=1).max() * 1e-8 + 1e-7 + tol * 0.1


def _check(onet, S, V, it, st, bound=FAST_BOUND, ref=None):
    if ref is None:
        ref = oracle.fpi(onet, S, 1e-10, 200)
    Vg = V.cpu().numpy().astype(np.complex128)
    err = np.abs(Vg - ref.V).max(axis=1)
    ok = st.cpu().numpy() == tpf.ST_CONVERGED
    assert ok.all(), f"{np.sum(~ok)} columns did not converge"
    assert err.max() <= bound, f"max error {err.max():.3e}"
    return err.max()


@pytest.fixture(scope="module")
def feeder100():
    f = W.make_feeder(100)
    return f, tpf.Network.from_feeder(f), oracle.build_feeder(f)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("T", [1, 16, 17, 3001])
def test_fast_forms_match_oracle(gpu, feeder100, mode, T):
    f, net, onet = feeder100
    S = W.profile_minute_year(f, steps=T, t0=2024)
    V, it, st, mm = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=100, mode=mode, mismatch=True)
    _check(onet, S, V, it, st)
    assert float(mm.max()) < _mismatch_bound(onet)


@pytest.mark.parametrize("mode", MODES)
def test_fast_forms_complex64(gpu, feeder100, mode):
    f, net, onet = feeder100
    S = W.profile_minute_year(f, steps=2000, t0=77, dtype=np.complex64)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu, torch.complex64), tol=1e-6, max_iter=100, mode=mode)
    assert V.dtype == torch.complex64
    _check(onet, S.astype(np.complex128), V, it, st, bound=FAST_BOUND + 2e-7)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n_bus", [2, 9, 33, 64, 65, 100, 129])
def test_fast_forms_sizes(gpu, mode, n_bus):
    f = W.make_feeder(n_bus, seed=100 + n_bus)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=250, seed=n_bus + 1)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=100, mode=mode)
    _check(onet, S, V, it, st)


@pytest.mark.parametrize("mode", MODES)
def test_fast_forms_heavy_load(gpu, mode):
    # slower contraction (rho ~ 0.2): the difference sweeps travel further
    f = W.make_feeder(100, seed=5, load_scale=4.0)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=1000, seed=9)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=200, mode=mode)
    _check(onet, S, V, it, st)


@pytest.mark.parametrize("mode", MODES + ["tree_fp32"])
def test_fast_forms_edge_columns(gpu, mode):
    f = W.make_star_feeder(np.array([1.0 + 0.5j]))
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = np.array([[0.18 + 0.11j], [0.25 + 0.15j], [np.nan + 0j], [0.0 + 0j]])
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=300, mode=mode)
    st = st.cpu().numpy()
    # Column 1 has no solution (Eq. (11) violated): the map is not a contraction and its
    # orbit is chaotic, so a reduced-precision run may leave the oracle's orbit and even
    # pass through V = 0, where the injection's |V|^2 is floored: a finite load ends
    # MAX_ITER, never converged and never non-finite (the FP64 form reproduces the
    # oracle's MAX_ITER exactly: FP64 tests); a NaN load ends NONFINITE.
    assert st[1] == tpf.ST_MAX_ITER
    assert [st[0], st[2], st[3]] == [tpf.ST_CONVERGED, tpf.ST_NONFINITE, tpf.ST_CONVERGED]
    ref = oracle.fpi(onet, S[[0, 3]], 1e-12, 1000)
    assert np.abs(V.cpu().numpy()[[0, 3]] - ref.V).max() < 2e-6  # k = 0.61: bound k/(1-k) tol


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("mode", MODES)
def test_fast_forms_warm_start(gpu, feeder100, mode, dtype):
    """Guarded warm starts in the first batch of a workgroup (read from HBM), in later
    batches (copied into LDS ahead of time in the FP16 form) and in the partial last one."""
    f, net, onet = feeder100
    S = W.profile_minute_year(f, steps=700, t0=5)
    if dtype == torch.complex64:
        S = S.astype(np.complex64).astype(np.complex128)
    ref = oracle.fpi(onet, S, 1e-10, 200)
    rng = np.random.default_rng(2)
    V0 = ref.V + 3e-5 * (rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape))
    V0[10, 3] = np.nan  # guarded: these columns start flat
    V0[333, 50] = 3.0
    V0[690, 98] = 0.1
    Vw, iw, sw = tpf.solve_timeseries(net, _dev(S, gpu, dtype), tol=1e-6, max_iter=100, mode=mode,
                                      V0=_dev(V0, gpu, dtype))
    _check(onet, S, Vw, iw, sw, bound=FAST_BOUND + (1e-7 if dtype == torch.complex64 else 0.0), ref=ref)
    Vf, i_f, sf = tpf.solve_timeseries(net, _dev(S, gpu, dtype), tol=1e-6, max_iter=100, mode=mode)
    iw, i_f = iw.cpu().numpy(), i_f.cpu().numpy()
    assert iw.mean() < i_f.mean()
    if mode == "fp32":  # a guarded column runs exactly as from the flat start
        for c in (10, 333, 690):
            assert iw[c] == i_f[c], c


@pytest.mark.parametrize("mode", MODES)
def test_fast_forms_reject_tol_below_fp32_floor(gpu, feeder100, mode):
    f, net, _ = feeder100
    S = _dev(W.profile_minute_year(f, steps=10), gpu)
    with pytest.raises(tpf.TpfError) as e:
        tpf.solve_timeseries(net, S, tol=1e-8, max_iter=10, mode=mode)
    assert e.value.code == tpf.TPF_ERR_INVALID_ARG


def test_fast_forms_full_year_sampled(gpu, feeder100):
    f, net, onet = feeder100
    S = W.profile_minute_year(f)
    Sd = _dev(S, gpu)
    rng = np.random.default_rng(12)
    idx = np.sort(rng.choice(S.shape[0], 3000, replace=False))
    ref = oracle.fpi(onet, S[idx], 1e-10, 200)
    ti = torch.from_numpy(idx).to(gpu)
    for mode in MODES:
        V, it, st, mm = tpf.solve_timeseries(net, Sd, tol=1e-6, max_iter=100, mode=mode, mismatch=True)
        torch.cuda.synchronize()
        assert int(st.max()) == tpf.ST_CONVERGED, mode
        _check(onet, S[idx], V[ti], it[ti], st[ti], ref=ref)
        assert float(mm.max()) < _mismatch_bound(onet), mode
