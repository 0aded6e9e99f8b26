"""GPU FP64 power-balance mismatch (Eq. (1)) against the oracle's, on every tile shape
of the kernel: 16 columns per tile up to 256 PQ buses, 8 up to 512, 4 up to 1,024,
and one wavefront per column beyond; ragged column counts; non-finite voltages."""
import numpy as np
import pytest
import torch

import oracle
import paper_2403_04578_amd as tpf
from paper_2403_04578_amd import workloads as W

pytestmark = pytest.mark.gpu


def _rounding(onet):
    # terms Y_bk V_k cancel from rowsum |Y_dd| down to the mismatch: a few units of 2^-52 of it
    return 16 * 2.0 ** -52 * float(np.abs(onet.Ydd).sum(axis=1).max())


@pytest.mark.parametrize("n_bus,T", [(2, 33), (100, 1), (100, 17), (100, 1001), (300, 37), (700, 9), (1200, 5)])
def test_mismatch_matches_oracle(gpu, n_bus, T):
    f = W.make_feeder(n_bus)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=T, t0=1234)
    # voltages near (not at) the solution, so that the mismatch is well above rounding
    V = oracle.fpi(onet, S, 1e-3, 100).V
    m = tpf.mismatch(net, torch.from_numpy(S).to(gpu), torch.from_numpy(V).to(gpu)).cpu().numpy()
    ref = oracle.mismatch(onet, S, V)
    assert ref.min() > 0
    assert np.all(np.abs(m - ref) <= 1e-12 * ref + _rounding(onet))


def test_mismatch_complex64_and_nonfinite(gpu):
    f = W.make_feeder(100)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=40, t0=99).astype(np.complex64)
    V = oracle.fpi(onet, S.astype(np.complex128), 1e-4, 100).V.astype(np.complex64)
    V[3, 7] = np.nan
    V[20, 98] = np.inf
    m = tpf.mismatch(net, torch.from_numpy(S).to(gpu), torch.from_numpy(V).to(gpu)).cpu().numpy()
    ref = oracle.mismatch(onet, S.astype(np.complex128), V.astype(np.complex128))
    bad = [3, 20]
    # a non-finite voltage gives a non-finite mismatch (inf or NaN, by arithmetic order)
    assert not np.isfinite(m[bad]).any() and not np.isfinite(ref[bad]).any()
    ok = np.setdiff1d(np.arange(40), bad)
    assert np.all(np.abs(m[ok] - ref[ok]) <= 1e-12 * ref[ok] + _rounding(onet))
