"""GPU parity of the tree operator (TPF_MODE_TREE_FP64) against the dense CPU oracle of
Algorithm 1: on a radial feeder without shunts, Z I equals minus the subtree-current /
path-drop passes, so the iterates agree up to rounding.  Every register width of the
kernel (1, 2, 4, 8, 16 positions per lane: 30, 99, 199, 399 and 999 PQ buses), both
dtypes, fixed sweep counts, edge columns, warm starts, ZIP loads, and the networks the
operator refuses.

Bounds: 1e-9 pu on columns with the oracle's sweep count (a column whose last step sits
on the tolerance may stop one sweep apart and is re-run on the oracle with that count);
complex64 output adds its rounding (<= 8.5e-8); fixed sweep counts 1e-12.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_04578_amd as tpf
from paper_2403_04578_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(S, gpu, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(S)).to(gpu).to(dtype).contiguous()


def _compare(onet, S, V, it, st, tol, max_iter, bound, V0=None, ref=None):
    if ref is None:
        ref = oracle.fpi(onet, S, tol, max_iter, V0)
    Vg = V.cpu().numpy().astype(np.complex128).reshape(ref.V.shape)
    ig, sg = it.cpu().numpy().reshape(-1), st.cpu().numpy().reshape(-1)
    same = ig == ref.iters
    assert np.sum(~same) <= max(2, 0.002 * len(same)), f"sweep counts differ on {np.sum(~same)} columns"
    assert np.array_equal(sg[same], ref.status[same])
    err = np.abs(Vg[same] - ref.V[same]).max(initial=0.0)
    assert err <= bound, f"max |dV| = {err:.3e}"
    for c in np.nonzero(~same)[0]:
        assert abs(int(ig[c]) - int(ref.iters[c])) <= 1
        r2 = oracle.fpi(onet, S[c:c + 1], 0.0, int(ig[c]), None if V0 is None else V0[c:c + 1])
        assert np.abs(Vg[c] - r2.V[0]).max() <= bound


@pytest.mark.parametrize("n_bus,T", [(31, 500), (100, 700), (200, 300), (400, 200), (1000, 120)])
def test_tree_every_column(gpu, n_bus, T):
    f = W.make_feeder(n_bus)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=T, t0=4321)
    V, it, st, mm = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-9, max_iter=100, mode="tree_fp64", mismatch=True)
    assert int(st.max()) == tpf.ST_CONVERGED
    _compare(onet, S, V, it, st, 1e-9, 100, 1e-9)
    # the dense FP64 form on the same columns: same sweeps, same voltages to rounding
    Vd, idn, _ = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-9, max_iter=100)
    assert float((Vd - V).abs().max()) < 1e-9
    assert float((idn != it).float().mean()) < 0.01


def test_tree_complex64_and_fixed_sweeps(gpu):
    f = W.make_feeder(100)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=300, t0=77, dtype=np.complex64).astype(np.complex128)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu, torch.complex64), tol=1e-6, max_iter=100, mode="tree_fp64")
    assert V.dtype == torch.complex64
    _compare(onet, S, V, it, st, 1e-6, 100, 2e-7)
    for k in (1, 2, 5):
        V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=0.0, max_iter=k, mode="tree_fp64")
        assert int(it.min()) == k == int(it.max()) and int(st.min()) == tpf.ST_MAX_ITER
        ref = oracle.fpi(onet, S, 0.0, k)
        assert np.abs(V.cpu().numpy() - ref.V).max() < 1e-12


def test_tree_edge_columns_and_warm_start(gpu):
    """Non-finite loads retire NONFINITE after one sweep, zero load converges to w in one
    sweep, a warm start from the solution converges at once, a bad V0 column starts flat."""
    f = W.make_feeder(100)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=6, t0=300)
    S[1, 17] = np.nan
    S[2] = 0.0
    S[3, 50] = np.inf
    sol = oracle.fpi(onet, S[[0]], 1e-12, 200).V[0]
    V0 = np.ones_like(S)
    V0[4] = sol
    V0[5] = sol
    S[4] = S[0]
    S[5] = S[0]
    V0[5, 3] = 3.0
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-9, max_iter=100, mode="tree_fp64", V0=_dev(V0, gpu))
    st, it = st.cpu().numpy(), it.cpu().numpy()
    assert list(st) == [0, 2, 0, 2, 0, 0]
    assert it[1] == 1 and it[3] == 1 and it[2] == 1
    assert it[4] <= 2 and it[5] == it[0]
    good = [0, 2, 4, 5]
    V0g = V0[good].copy()
    V0g[3] = 1.0
    _compare(onet, S[good], V[good], torch.from_numpy(it[good]), torch.from_numpy(st[good]), 1e-9, 100, 1e-9,
             V0=V0g)


def test_tree_year_sampled(gpu):
    """The 100-bus year (525,600 columns) in the launch configuration the benchmark uses,
    checked on sampled columns and by the FP64 mismatch of every column."""
    f = W.make_feeder(100)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f)
    V, it, st, mm = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=100, mode="tree_fp64", mismatch=True)
    torch.cuda.synchronize()
    assert int(st.max()) == tpf.ST_CONVERGED
    idx = np.unique(np.concatenate([np.random.default_rng(3).integers(0, len(S), 400), [0, len(S) - 1]]))
    Vs = V[torch.from_numpy(idx).to(gpu)]
    _compare(onet, S[idx], Vs, it[torch.from_numpy(idx).to(gpu)], st[torch.from_numpy(idx).to(gpu)], 1e-6, 100,
             1e-9)
    ymax = np.abs(onet.Ydd).sum(axis=1).max()
    assert float(mm.max()) < ymax * 1.2e-7 + 1e-7


def test_tree_zip_loads(gpu):
    f = W.make_feeder(100)
    ai, ap = W.zip_shares(99)
    net, onet = tpf.Network.from_feeder(f, alpha_i=ai, alpha_p=ap), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=400, t0=9)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-9, max_iter=100, mode="tree_fp64")
    assert int(st.max()) == tpf.ST_CONVERGED
    _compare(onet, S, V, it, st, 1e-9, 100, 1e-9, ref=oracle.fpi_zip(onet, S, ai, ap, 1e-9, 100))


def test_tree_refuses_meshed(gpu):
    meshed = tpf.Network(4, [0, 1, 2, 0], [1, 2, 3, 3], [0.01] * 4, [0.02] * 4)
    S = _dev(np.full((3, 3), 0.01 + 0.005j), gpu)
    with pytest.raises(tpf.TpfError) as e:
        tpf.solve_timeseries(meshed, S, tol=1e-9, max_iter=10, mode="tree_fp64")
    assert e.value.code == tpf.TPF_ERR_UNSUPPORTED


def test_tree_two_bus_network(gpu):
    z = 0.05 + 0.08j
    net = tpf.Network(2, [0], [1], [z.real], [z.imag])
    onet = oracle.build_network(2, [0], [1], [z.real], [z.imag])
    S = np.array([[0.5 + 0.2j], [0.0], [1.0 + 0.3j]])
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-12, max_iter=200, mode="tree_fp64")
    _compare(onet, S, V, it, st, 1e-12, 200, 1e-12)


@pytest.mark.parametrize("n_bus,T,dtype", [(31, 300, torch.complex128), (100, 700, torch.complex128),
                                           (100, 300, torch.complex64), (200, 300, torch.complex128),
                                           (400, 200, torch.complex128), (1000, 100, torch.complex128)])
def test_tree_fp32_form(gpu, n_bus, T, dtype):
    """The FP32 tree form (state as the FP32 drop V - w) to the fast-form contract: 1e-6
    pu against a tol-1e-10 oracle solution, every register width of its kernel."""
    f = W.make_feeder(n_bus)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=T, t0=50)
    if dtype == torch.complex64:
        S = S.astype(np.complex64).astype(np.complex128)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu, dtype), tol=1e-6, max_iter=100, mode="tree_fp32")
    assert int(st.max()) == tpf.ST_CONVERGED
    ref = oracle.fpi(onet, S, 1e-10, 200)
    bound = 1e-6 + (1e-7 if dtype == torch.complex64 else 0.0)
    assert np.abs(V.cpu().numpy().astype(np.complex128) - ref.V).max() <= bound


def test_tree_fp32_zip_edges_and_refusals(gpu):
    f = W.make_feeder(100)
    ai, ap = W.zip_shares(99)
    net, onet = tpf.Network.from_feeder(f, alpha_i=ai, alpha_p=ap), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=200, t0=3)
    S[5, 7] = np.nan
    S[6] = 0.0
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=100, mode="tree_fp32")
    st = st.cpu().numpy()
    assert st[5] == tpf.ST_NONFINITE and int(it[5]) == 1
    good = np.arange(200) != 5
    assert np.all(st[good] == tpf.ST_CONVERGED)
    ref = oracle.fpi_zip(onet, S[good], ai, ap, 1e-10, 200)
    assert np.abs(V.cpu().numpy()[good] - ref.V).max() <= 1e-6
    # warm start from the solution: converges at once
    V0 = np.ones_like(S)
    V0[good] = ref.V
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=100, mode="tree_fp32", V0=_dev(V0, gpu))
    assert int(it.cpu().numpy()[good].max()) == 1
    with pytest.raises(tpf.TpfError) as e:  # below the FP32 state floor
        tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-8, max_iter=10, mode="tree_fp32")
    assert e.value.code == tpf.TPF_ERR_INVALID_ARG


@pytest.mark.parametrize("mode", ["tree_fp64", "tree_fp32"])
@pytest.mark.parametrize("T", [1, 5, 33])
def test_tree_few_columns(gpu, mode, T):
    """Fewer columns than the slots of one workgroup, and a ragged last round."""
    f = W.make_feeder(100)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=T, t0=999)
    tol = 1e-9 if mode == "tree_fp64" else 1e-6
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=tol, max_iter=100, mode=mode)
    assert V.shape == (T, 99) and int(st.max()) == tpf.ST_CONVERGED
    ref = oracle.fpi(onet, S, 1e-10, 200)
    assert np.abs(V.cpu().numpy() - ref.V).max() <= (1e-9 if mode == "tree_fp64" else 1e-6)
