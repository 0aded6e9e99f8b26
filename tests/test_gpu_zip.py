"""GPU parity of the ZIP load model of Eq. (2) (constant-impedance share zero) against
the oracle's per-column F and w: the FP64 register-resident kernel (99 and 299 PQ buses)
and per-sweep path (399), the FP32 and mixed forms (register-resident at 99, per-sweep at
299, with warm starts), complex128 and complex64 loads, the constant-power and
constant-current limits, and the ZIP power-balance mismatch.

Bounds: the FP64 contract, 1e-9 pu, on columns with the oracle's sweep count (a column
whose last step sits on the tolerance may stop one sweep apart and is re-run on the
oracle with that count); complex64 output adds its rounding (<= 8.5e-8).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_04578_amd as tpf
from paper_2403_04578_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-9


def _dev(S, gpu, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(S)).to(gpu).to(dtype).contiguous()


def _shares(n, seed):
    """Seeded per-bus shares: constant current in [0, 0.6], the rest constant power."""
    ai = np.random.default_rng(seed).uniform(0.0, 0.6, n)
    return ai, 1.0 - ai


def _compare(onet, S, ai, ap, V, it, st, tol, max_iter, bound):
    ref = oracle.fpi_zip(onet, S, ai, ap, tol, max_iter)
    Vg = V.cpu().numpy().astype(np.complex128).reshape(ref.V.shape)
    ig, sg = it.cpu().numpy(), st.cpu().numpy()
    same = ig == ref.iters
    assert np.sum(~same) <= max(2, 0.002 * len(same)), f"sweep counts differ on {np.sum(~same)} columns"
    assert np.array_equal(sg[same], ref.status[same])
    err = np.abs(Vg[same] - ref.V[same]).max(initial=0.0)
    assert err <= bound, f"max |dV| = {err:.3e}"
    for c in np.nonzero(~same)[0]:
        assert abs(int(ig[c]) - int(ref.iters[c])) <= 1
        r2 = oracle.fpi_zip(onet, S[c:c + 1], ai, ap, 0.0, int(ig[c]))
        assert np.abs(Vg[c] - r2.V[0]).max() <= bound
    return Vg


@pytest.mark.parametrize("n_bus,T", [(100, 700), (300, 257), (400, 130)])
def test_zip_fp64_every_column(gpu, n_bus, T):
    f = W.make_feeder(n_bus)
    ai, ap = _shares(n_bus - 1, 11)
    net, onet = tpf.Network.from_feeder(f, alpha_i=ai, alpha_p=ap), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=T, t0=321)
    V, it, st, mm = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-9, max_iter=100, mismatch=True)
    assert int(st.max()) == tpf.ST_CONVERGED
    Vg = _compare(onet, S, ai, ap, V, it, st, 1e-9, 100, TOL_FP64)
    # the ZIP balance of the returned voltages, against the oracle's (rounding-level values)
    ref_mm = oracle.mismatch_zip(onet, S, Vg, ai, ap)
    scale = 16 * 2.0 ** -52 * float(np.abs(onet.Ydd).sum(axis=1).max())
    assert np.all(np.abs(mm.cpu().numpy() - ref_mm) <= scale + 1e-9 * ref_mm)
    # and the loads really follow the ZIP model: the constant-power solution is elsewhere
    Vc, _, _ = tpf.solve_timeseries(tpf.Network.from_feeder(f), _dev(S, gpu), tol=1e-9, max_iter=100)
    assert float((Vc - V).abs().max()) > 1e-6


def test_zip_mismatch_away_from_solution(gpu):
    """tpf_mismatch of a ZIP network on perturbed voltages (mismatch ~1e-3) equals the
    oracle's ZIP balance to rounding, for both dtypes."""
    f = W.make_feeder(100)
    ai, ap = _shares(99, 4)
    net, onet = tpf.Network.from_feeder(f, alpha_i=ai, alpha_p=ap), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=333, t0=9)
    rng = np.random.default_rng(8)
    Vp = 1.0 + 0.02 * (rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape))
    for dt in (torch.complex128, torch.complex64):
        Sd, Vd = _dev(S, gpu, dt), _dev(Vp, gpu, dt)
        g = tpf.mismatch(net, Sd, Vd).cpu().numpy()
        ref = oracle.mismatch_zip(onet, Sd.cpu().numpy().astype(np.complex128), Vd.cpu().numpy().astype(np.complex128),
                                  ai, ap)
        assert np.allclose(g, ref, rtol=1e-12, atol=1e-15)


def test_zip_limits(gpu):
    """alpha_P = 1, alpha_I = 0 through the ZIP kernels reproduces the constant-power
    kernels bit for bit; alpha_P = 0 (constant current) converges in two sweeps to the
    linear solve."""
    f = W.make_feeder(100)
    S = W.profile_minute_year(f, steps=200, t0=77)
    Sd = _dev(S, gpu)
    Vc, ic, sc = tpf.solve_timeseries(tpf.Network.from_feeder(f), Sd, tol=1e-9, max_iter=100)
    Vz, iz, sz = tpf.solve_timeseries(tpf.Network.from_feeder(f, alpha_i=0.0, alpha_p=1.0), Sd, tol=1e-9, max_iter=100)
    assert torch.equal(Vc, Vz) and torch.equal(ic, iz) and torch.equal(sc, sz)
    onet = oracle.build_feeder(f)
    Vi, ii, si = tpf.solve_timeseries(tpf.Network.from_feeder(f, alpha_i=1.0, alpha_p=0.0), Sd, tol=1e-12,
                                      max_iter=10)
    assert int(ii.min()) == 2 and int(ii.max()) == 2 and int(si.max()) == tpf.ST_CONVERGED
    rhs = -(onet.Yds[None, :] * onet.vs + np.conj(S))
    Vs = np.linalg.solve(onet.Ydd, rhs.T).T
    assert np.abs(Vi.cpu().numpy() - Vs).max() < 1e-12


@pytest.mark.parametrize("n_bus", [100, 400])
def test_zip_complex64_and_edges(gpu, n_bus):
    f = W.make_feeder(n_bus)
    ai, ap = _shares(n_bus - 1, 5)
    net, onet = tpf.Network.from_feeder(f, alpha_i=ai, alpha_p=ap), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=130, t0=4000, dtype=np.complex64).astype(np.complex128)
    S[3, 7] = np.nan
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu, torch.complex64), tol=1e-6, max_iter=100)
    assert V.dtype == torch.complex64
    stn = st.cpu().numpy()
    assert stn[3] == tpf.ST_NONFINITE and int(it[3]) == 1
    good = np.arange(130) != 3
    ref = oracle.fpi_zip(onet, S[good], ai, ap, 1e-6, 100)
    same = it.cpu().numpy()[good] == ref.iters
    assert same.mean() > 0.99
    assert np.abs(V.cpu().numpy()[good][same].astype(np.complex128) - ref.V[same]).max() < 2e-7
    assert np.all(stn[good] == tpf.ST_CONVERGED)


@pytest.mark.parametrize("mode", ["fp32", "mixed_bf16", "mixed_fp16"])
@pytest.mark.parametrize("n_bus,dtype", [(100, torch.complex128), (100, torch.complex64), (300, torch.complex128)])
def test_zip_fast_forms(gpu, mode, n_bus, dtype):
    """The reduced-precision forms with ZIP loads: register-resident kernels at 99 PQ
    buses, the per-sweep path at 299; warm starts at 99 (staged in LDS in the FP16 form).
    Bound: the fast-form contract, 1e-6 pu against a tol-1e-10 oracle solution."""
    f = W.make_feeder(n_bus)
    ai, ap = _shares(n_bus - 1, 13)
    net, onet = tpf.Network.from_feeder(f, alpha_i=ai, alpha_p=ap), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=600, t0=55)
    if dtype == torch.complex64:
        S = S.astype(np.complex64).astype(np.complex128)
    ref = oracle.fpi_zip(onet, S, ai, ap, 1e-10, 200)
    bound = 1e-6 + (1e-7 if dtype == torch.complex64 else 0.0)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu, dtype), tol=1e-6, max_iter=100, mode=mode)
    assert int(st.max()) == tpf.ST_CONVERGED
    assert np.abs(V.cpu().numpy().astype(np.complex128) - ref.V).max() <= bound
    if n_bus == 100:
        rng = np.random.default_rng(3)
        V0 = ref.V + 2e-4 * (rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape))
        Vw, iw, sw = tpf.solve_timeseries(net, _dev(S, gpu, dtype), tol=1e-6, max_iter=100, mode=mode,
                                          V0=_dev(V0, gpu, dtype))
        assert int(sw.max()) == tpf.ST_CONVERGED
        assert np.abs(Vw.cpu().numpy().astype(np.complex128) - ref.V).max() <= bound
        assert float(iw.float().mean()) < float(it.float().mean())


def test_zip_large_shares_keep_fp16_in_range(gpu):
    """Shares far from a partition of unity (alpha_P = 3, alpha_I = 2) enlarge the
    injection; the FP16 column scale accounts for them, so the form still converges to
    the oracle's solution."""
    f = W.make_feeder(100)
    net, onet = tpf.Network.from_feeder(f, alpha_i=2.0, alpha_p=3.0), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=128, t0=600) * 0.2
    ref = oracle.fpi_zip(onet, S, 2.0, 3.0, 1e-10, 200)
    for mode in ("mixed_fp16", "mixed_bf16"):
        V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=100, mode=mode)
        assert int(st.max()) == tpf.ST_CONVERGED
        assert np.abs(V.cpu().numpy() - ref.V).max() <= 1e-6
