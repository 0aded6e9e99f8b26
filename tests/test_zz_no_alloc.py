"""GPU checks of the allocation-free entry point tpf_solve_timeseries_noalloc.

It runs the same kernels as tpf_solve_timeseries with the column queue in the library's
static device scratch instead of a workspace, so its results must equal the regular entry
point's bit for bit -- on two calls in a row (the second on fewer columns, after the scratch
holds the first call's queue state) -- and it must refuse what needs more than its scratch.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_04578_amd as tpf
from paper_2403_04578_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def feeder(gpu):
    f = W.make_feeder(100)
    S = torch.from_numpy(W.profile_minute_year(f, steps=4000)).to(gpu)
    return f, S


@pytest.mark.parametrize("mode", ["fp64", "mixed_fp16", "mixed_bf16", "fp32", "tree_fp32"])
def test_noalloc_equals_regular_solve_on_two_calls(feeder, mode):
    f, S = feeder
    net = tpf.Network.from_feeder(f)
    tol = 1e-9 if mode == "fp64" else 1e-6
    ref1 = tpf.solve_timeseries(net, S, tol, 100, mode=mode, mismatch=True)  # also uploads the network
    a1 = tpf.solve_timeseries_noalloc(net, S, tol, 100, mode=mode, mismatch=True)
    S2 = S[1000:1777].contiguous()  # a second, smaller call: the scratch holds the first call's queue
    a2 = tpf.solve_timeseries_noalloc(net, S2, tol, 100, mode=mode, mismatch=True)
    ref2 = tpf.solve_timeseries(net, S2, tol, 100, mode=mode, mismatch=True)
    for x, y in zip(a1, ref1):
        assert torch.equal(x, y)
    for x, y in zip(a2, ref2):
        assert torch.equal(x, y)
    assert int(a1[2].max()) == tpf.ST_CONVERGED and int(a2[2].max()) == tpf.ST_CONVERGED


def test_noalloc_matches_oracle(feeder):
    f, S = feeder
    net = tpf.Network.from_feeder(f)
    tpf.mismatch(net, S[:1], S[:1])  # uploads the network
    Sd = S[:300].contiguous()
    V, it, st = tpf.solve_timeseries_noalloc(net, Sd, 1e-10, 100)
    ref = oracle.fpi(oracle.build_feeder(f), Sd.cpu().numpy(), 1e-10, 100)
    assert np.abs(V.cpu().numpy() - ref.V).max() < 1e-9
    assert np.array_equal(it.cpu().numpy(), ref.iters)


def test_noalloc_refuses_what_it_cannot_hold(feeder, gpu):
    f, S = feeder
    net = tpf.Network.from_feeder(f)
    # not yet resident on the device: uploading would allocate
    with pytest.raises(tpf.TpfError) as e:
        tpf.solve_timeseries_noalloc(net, S[:10].contiguous(), 1e-6, 100)
    assert e.value.code == tpf.TPF_ERR_UNSUPPORTED
    # a 400-bus feeder in FP64 takes the per-sweep path, whose workspace exceeds the scratch
    big = W.make_feeder(400)
    bnet = tpf.Network.from_feeder(big)
    Sb = torch.from_numpy(W.profile_minute_year(big, steps=64)).to(gpu)
    tpf.solve_timeseries(bnet, Sb, 1e-6, 100)
    with pytest.raises(tpf.TpfError) as e:
        tpf.solve_timeseries_noalloc(bnet, Sb, 1e-6, 100)
    assert e.value.code == tpf.TPF_ERR_UNSUPPORTED
    # the same network in the tree form needs no workspace beyond the scratch
    V, it, st = tpf.solve_timeseries_noalloc(bnet, Sb, 1e-6, 100, mode="tree_fp64")
    Vr, itr, str_ = tpf.solve_timeseries(bnet, Sb, 1e-6, 100, mode="tree_fp64")
    assert torch.equal(V, Vr) and torch.equal(it, itr)
