"""GPU parity on three-phase (unbalanced, mutually coupled) feeders against the CPU
oracle: the sweep kernels see n = 3 (n_bus - 1) demand nodes, so the 100-bus three-phase
feeder (297 nodes) runs the register-resident FP64 kernel and the per-sweep path in the
reduced-precision forms, and the 40-bus one (117 nodes) the register-resident kernels of
every form.

Bounds: FP64 1e-9 pu on columns with the oracle's sweep count; the fast forms 1e-6 pu
against a tol-1e-10 oracle solution; mismatch at rounding level.
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


@pytest.fixture(scope="module", params=[100, 40])
def feeder3(request):
    f = W.make_feeder_3ph(request.param)
    return f, tpf.Network.from_feeder_3ph(f), oracle.build_feeder_3ph(f)


def test_three_phase_fp64_every_column(gpu, feeder3):
    f, net, onet = feeder3
    S = W.profile_minute_year(f, steps=300, t0=1234)
    V, it, st, mm = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-9, max_iter=100, mismatch=True)
    ref = oracle.fpi(onet, S, 1e-9, 100)
    ig = it.cpu().numpy()
    same = ig == ref.iters
    assert same.mean() > 0.99 and int(st.max()) == tpf.ST_CONVERGED
    Vg = V.cpu().numpy()
    assert np.abs(Vg[same] - ref.V[same]).max() < 1e-9
    for c in np.nonzero(~same)[0]:
        r2 = oracle.fpi(onet, S[c:c + 1], 0.0, int(ig[c]))
        assert np.abs(Vg[c] - r2.V[0]).max() < 1e-9
    ref_mm = oracle.mismatch(onet, S, Vg)
    scale = 16 * 2.0 ** -52 * float(np.abs(onet.Ydd).sum(axis=1).max())
    assert np.all(np.abs(mm.cpu().numpy() - ref_mm) <= scale + 1e-9 * ref_mm)
    # phase sequence a, b, c: phase b lags phase a by about 120 degrees at every bus
    lag = np.angle(Vg[:, 0::3] / Vg[:, 1::3], deg=True)
    assert np.abs(lag - 120.0).max() < 5.0


@pytest.mark.parametrize("mode", ["fp32", "mixed_bf16", "mixed_fp16"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_three_phase_fast_forms(gpu, feeder3, mode, dtype):
    f, net, onet = feeder3
    S = W.profile_minute_year(f, steps=257, t0=99)
    if dtype == torch.complex64:
        S = S.astype(np.complex64).astype(np.complex128)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu, dtype), tol=1e-6, max_iter=100, mode=mode)
    assert int(st.max()) == tpf.ST_CONVERGED
    ref = oracle.fpi(onet, S, 1e-10, 200)
    bound = 1e-6 + (1e-7 if dtype == torch.complex64 else 0.0)
    assert np.abs(V.cpu().numpy().astype(np.complex128) - ref.V).max() <= bound


def test_three_phase_tensor_and_warm_start(gpu):
    """[scenario, time, node] tensor in FP64 with a guarded warm start from the solution
    of a neighbouring scenario."""
    f = W.make_feeder_3ph(100)
    net, onet = tpf.Network.from_feeder_3ph(f), oracle.build_feeder_3ph(f)
    S = W.profile_minute_year(f, steps=2 * 96, t0=10).reshape(2, 96, -1)
    S[1] *= 1.1
    V1, _, _ = tpf.solve_tensor(net, _dev(S[:1], gpu), tol=1e-9, max_iter=100)
    V0 = torch.cat([V1, V1])
    V, it, st = tpf.solve_tensor(net, _dev(S, gpu), tol=1e-9, max_iter=100, V0=V0)
    assert V.shape == (2, 96, 297)
    ref = oracle.fpi(onet, S.reshape(-1, 297), 1e-9, 100, V0=V0.cpu().numpy().reshape(-1, 297))
    same = it.cpu().numpy().reshape(-1) == ref.iters
    assert same.mean() > 0.99
    assert np.abs(V.cpu().numpy().reshape(-1, 297)[same] - ref.V[same]).max() < 1e-9
    assert int(it[0].max()) == 1  # scenario 0 starts at its own solution


def test_three_phase_tree_operator(gpu, feeder3):
    """The tree operator with 3x3 branch blocks: the FP64 iterates up to rounding."""
    f, net, onet = feeder3
    S = W.profile_minute_year(f, steps=300, t0=2222)
    for dt in (torch.complex128, torch.complex64):
        Sd = _dev(S, gpu, dt)
        V, it, st = tpf.solve_timeseries(net, Sd, tol=1e-9, max_iter=100, mode="tree_fp64")
        Sh = Sd.cpu().numpy().astype(np.complex128)
        ref = oracle.fpi(onet, Sh, 1e-9, 100)
        ig = it.cpu().numpy()
        same = ig == ref.iters
        assert same.mean() > 0.99 and int(st.max()) == tpf.ST_CONVERGED
        bound = 1e-9 if dt == torch.complex128 else 2e-7
        assert np.abs(V.cpu().numpy().astype(np.complex128)[same] - ref.V[same]).max() < bound
    # with a warm start from the solution, one sweep
    V0 = torch.from_numpy(ref.V).to(gpu)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-8, max_iter=100, mode="tree_fp64", V0=V0)
    assert int(it.max()) == 1


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_three_phase_tree_fp32(gpu, feeder3, dtype):
    """The FP32 tree form with 3x3 branch blocks: 1e-6 pu from a tol-1e-10 oracle
    solution over a ragged column count (not a multiple of the columns per workgroup);
    a warm start whose column holds a modulus outside [0.5, 1.5] starts flat."""
    f, net, onet = feeder3
    S = W.profile_minute_year(f, steps=203, t0=4444)
    if dtype == torch.complex64:
        S = S.astype(np.complex64).astype(np.complex128)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu, dtype), tol=1e-6, max_iter=100, mode="tree_fp32")
    assert int(st.max()) == tpf.ST_CONVERGED
    ref = oracle.fpi(onet, S, 1e-10, 200)
    bound = 1e-6 + (1e-7 if dtype == torch.complex64 else 0.0)
    assert np.abs(V.cpu().numpy().astype(np.complex128) - ref.V).max() <= bound
    V0 = ref.V.copy()
    V0[7, 5] = 3.0
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu, dtype), tol=1e-6, max_iter=100, mode="tree_fp32",
                                     V0=_dev(V0, gpu, dtype))
    it = it.cpu().numpy()
    assert it[0] <= 2 and it[7] >= 3
    assert np.abs(V.cpu().numpy().astype(np.complex128) - ref.V).max() <= bound


@pytest.mark.parametrize("n_bus", [200, 300])
def test_three_phase_tree_wide_feeders(gpu, n_bus):
    """The tree kernels' one-column-per-wavefront shapes (4 and 8 positions per lane)
    on 199 and 299 three-phase buses, over a ragged column count: FP64 iterates up to
    rounding, the FP32 drop state within 1e-6 pu of a tol-1e-10 oracle solution."""
    f = W.make_feeder_3ph(n_bus)
    net, onet = tpf.Network.from_feeder_3ph(f), oracle.build_feeder_3ph(f)
    S = W.profile_minute_year(f, steps=37, t0=777)
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-9, max_iter=100, mode="tree_fp64")
    ref = oracle.fpi(onet, S, 1e-9, 100)
    ig = it.cpu().numpy()
    same = ig == ref.iters
    assert same.mean() > 0.9 and int(st.max()) == tpf.ST_CONVERGED
    Vg = V.cpu().numpy()
    assert np.abs(Vg[same] - ref.V[same]).max() < 1e-9
    for c in np.nonzero(~same)[0]:
        r2 = oracle.fpi(onet, S[c:c + 1], 0.0, int(ig[c]))
        assert np.abs(Vg[c] - r2.V[0]).max() < 1e-9
    V, it, st = tpf.solve_timeseries(net, _dev(S, gpu), tol=1e-6, max_iter=100, mode="tree_fp32")
    assert int(st.max()) == tpf.ST_CONVERGED
    ref = oracle.fpi(onet, S, 1e-10, 200)
    assert np.abs(V.cpu().numpy() - ref.V).max() <= 1e-6


def test_three_phase_tree_fp64_lds_limit(gpu):
    """The FP64 three-phase tree kernel keeps 400 bytes of state per bus in LDS: 408 PQ buses
    run, 409 return TPF_ERR_UNSUPPORTED, where the FP32 form (240 bytes per bus) still runs."""
    S_by_size = {}
    for n_bus in (409, 410):
        f = W.make_feeder_3ph(n_bus)
        net = tpf.Network.from_feeder_3ph(f)
        S = _dev(W.profile_minute_year(f, steps=20, t0=99), gpu)
        S_by_size[n_bus] = (f, net, S)
    f, net, S = S_by_size[409]
    V64, it64, st64 = tpf.solve_timeseries(net, S, tol=1e-9, max_iter=100, mode="tree_fp64")
    V32, it32, st32 = tpf.solve_timeseries(net, S, tol=1e-6, max_iter=100, mode="tree_fp32")
    assert int(st64.max()) == tpf.ST_CONVERGED and int(st32.max()) == tpf.ST_CONVERGED
    assert float((V64 - V32).abs().max()) < 1e-6
    f, net, S = S_by_size[410]
    with pytest.raises(tpf.TpfError) as e:
        tpf.solve_timeseries(net, S, tol=1e-9, max_iter=100, mode="tree_fp64")
    assert e.value.code == tpf.TPF_ERR_UNSUPPORTED
    V, it, st = tpf.solve_timeseries(net, S, tol=1e-6, max_iter=100, mode="tree_fp32")
    onet = oracle.build_feeder_3ph(f)
    ref = oracle.fpi(onet, S[:4].cpu().numpy(), 1e-10, 200)
    assert int(st.max()) == tpf.ST_CONVERGED
    assert np.abs(V[:4].cpu().numpy() - ref.V).max() <= 1e-6
