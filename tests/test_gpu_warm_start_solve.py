"""GPU checks of a solve that evaluates the learned warm start itself (tpf_options.warm_start).

The solve runs the network's inference on S into its workspace and starts every column from
it, guarded like a given V0.  In every mode the result must equal, bit for bit, the solve given
the separately predicted V0, and it must match the FP64 oracle (Algorithm 1 at tol 1e-10) to
the mode's contract.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_04578_amd as tpf
from paper_2403_04578_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(gpu):
    f = W.make_feeder(100)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    # a warm start trained briefly on solved minutes spread over a separately seeded year
    ntr = 6000
    t_tr = np.arange(ntr, dtype=np.int64) * 87 % W.MINUTES_PER_YEAR
    S_year_tr = W.profile_minute_year(f, steps=W.MINUTES_PER_YEAR, seed=W.SEED_TRAIN)
    S_tr = torch.from_numpy(S_year_tr[t_tr]).to(gpu)
    del S_year_tr
    V_tr, _, _ = tpf.solve_timeseries(net, S_tr, 1e-10, 100)
    mlp = tpf.WarmStart(99, params=W.mlp_init_params(W.mlp_sizes(99)))
    mlp.fit(S_tr, torch.from_numpy(t_tr).to(gpu), V_tr, epochs=30, batch=500, lr=2e-3, seed=1)
    # the year's first 3,000 minutes and 17 more
    T = 3017
    S = W.profile_minute_year(f, steps=T)
    ref = oracle.fpi(onet, S, 1e-10, 200)
    return f, net, onet, mlp, S, ref


def _run(net, S, mlp, mode="mixed_fp16", t_index=None, mismatch=True, tol=1e-6):
    return tpf.solve_timeseries(net, S, tol, 100, mode=mode, mismatch=mismatch, warm_start=mlp, t_index=t_index)


@pytest.mark.parametrize("mode", ["fp64", "mixed_fp16", "mixed_bf16", "fp32", "tree_fp32"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_warm_start_solve_equals_solve_from_predicted_start(setup, mode, dtype):
    f, net, onet, mlp, S, ref = setup
    dev = torch.device("cuda:0")
    Sd = torch.from_numpy(S).to(dtype).to(dev)
    tol = 1e-9 if mode == "fp64" and dtype == torch.complex128 else 1e-6
    t = torch.arange(S.shape[0], dtype=torch.int64, device=dev) + 1000
    V, it, st, mm = _run(net, Sd, mlp, mode=mode, tol=tol, t_index=t)
    V0 = mlp.predict(Sd, t)
    V2, it2, st2, mm2 = tpf.solve_timeseries(net, Sd, tol, 100, mode=mode, V0=V0, mismatch=True)
    assert torch.equal(V, V2) and torch.equal(it, it2) and torch.equal(st, st2) and torch.equal(mm, mm2)
    assert int(st.max()) == tpf.ST_CONVERGED
    bound = (1e-8 if mode == "fp64" else 1e-6) if dtype == torch.complex128 else 1e-6
    assert np.abs(V.cpu().numpy().astype(np.complex128) - ref.V).max() < bound
    # the learned start saves sweeps against the flat start
    _, it_flat, _ = tpf.solve_timeseries(net, Sd, tol, 100, mode=mode)
    assert float(it.float().mean()) < float(it_flat.float().mean()) - 0.5


def test_warm_start_default_minute_index(setup):
    f, net, onet, mlp, S, ref = setup
    dev = torch.device("cuda:0")
    Sd = torch.from_numpy(S[:500]).to(dev)
    a = _run(net, Sd, mlp)
    b = _run(net, Sd, mlp, t_index=torch.arange(500, dtype=torch.int64, device=dev))
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    # other minute indices change the calendar features, hence the start
    c = _run(net, Sd, mlp, t_index=torch.arange(500, dtype=torch.int64, device=dev) + 200_000)
    assert not torch.equal(a[0], c[0])


def test_warm_start_guard_falls_back_to_flat_start(setup):
    """A network with non-finite parameters fails the start guard in every column: the solve
    then runs exactly the schedule of a solve given a non-finite V0."""
    f, net, onet, mlp, S, ref = setup
    dev = torch.device("cuda:0")
    bad = tpf.WarmStart(99, params=np.full(mlp.num_params, np.nan, np.float32))
    Sd = torch.from_numpy(S[:500]).to(dev)
    V, it, st, mm = _run(net, Sd, bad)
    V0 = torch.full_like(Sd, float("nan"))
    V2, it2, st2, mm2 = tpf.solve_timeseries(net, Sd, 1e-6, 100, mode="mixed_fp16", V0=V0, mismatch=True)
    assert torch.equal(V, V2) and torch.equal(it, it2) and torch.equal(st, st2) and torch.equal(mm, mm2)


def test_warm_start_zero_sweeps_returns_the_guarded_start(setup):
    f, net, onet, mlp, S, ref = setup
    dev = torch.device("cuda:0")
    Sd = torch.from_numpy(S[:300]).to(dev)
    V, it, st = tpf.solve_timeseries(net, Sd, 1e-6, 0, mode="mixed_fp16", warm_start=mlp)
    V0 = mlp.predict(Sd, torch.arange(300, dtype=torch.int64, device=dev))
    assert torch.equal(V, V0) and int(it.max()) == 0 and int(st.min()) == tpf.ST_MAX_ITER


def test_warm_start_and_v0_together_is_an_error(setup):
    f, net, onet, mlp, S, ref = setup
    dev = torch.device("cuda:0")
    Sd = torch.from_numpy(S[:10]).to(dev)
    with pytest.raises(tpf.TpfError):
        tpf.solve_timeseries(net, Sd, 1e-6, 100, mode="mixed_fp16", V0=Sd.clone(), warm_start=mlp)


@pytest.mark.parametrize("mode", ["mixed_fp16", "fp64"])
def test_warm_start_full_year_sampled(setup, mode):
    """The headline launch: the 525,600-minute year of the 100-bus feeder in one call that
    evaluates the learned start itself (complex128 S, tol 1e-6, max 100 sweeps, FP64
    mismatch), checked on 3,000 sampled minutes against the oracle (Algorithm 1 from a flat
    start at tol 1e-10), with every column converged, the start saving sweeps against the
    flat start, and the mismatch of every column at the tolerance level."""
    f, net, onet, mlp, _, _ = setup
    dev = torch.device("cuda:0")
    S = W.profile_minute_year(f)
    Sd = torch.from_numpy(S).to(dev)
    t = torch.arange(S.shape[0], dtype=torch.int64, device=dev)
    V, it, st, mm = _run(net, Sd, mlp, mode=mode, t_index=t)
    torch.cuda.synchronize()
    assert int(st.max()) == tpf.ST_CONVERGED and int((st == tpf.ST_CONVERGED).sum()) == S.shape[0]
    idx = np.sort(np.random.default_rng(31).choice(S.shape[0], 3000, replace=False))
    ref = oracle.fpi(onet, S[idx], 1e-10, 200)
    err = np.abs(V[torch.from_numpy(idx).to(dev)].cpu().numpy() - ref.V).max()
    assert err < (1e-8 if mode == "fp64" else 1e-6), err
    _, it_flat, _ = tpf.solve_timeseries(net, Sd, 1e-6, 100, mode=mode)
    assert float(it.float().mean()) < float(it_flat.float().mean()) - 0.5
    # FP64 mismatch of a solution dv from the fixed point that stopped at step d < tol: about
    # |Y_dd row|_1 dv + |S| d / |V|; dv is FP64 rounding in the FP64 form and at most a few
    # 1e-9 with the drop kept in FP32 (|V - w| <= 0.1 pu, ulp 7.5e-9)
    dv = 1e-12 if mode == "fp64" else 1e-8
    assert float(mm.max()) < np.abs(onet.Ydd).sum(axis=1).max() * dv + 1e-7 + 1e-6 * 0.1
