"""GPU checks of the learned warm start against the FP64 reference (oracle/mlp_ref.py).

The GPU network computes its products in BF16 with FP32 accumulation and keeps
FP32 master parameters.  The reference is evaluated with the parameters and the
input features rounded to BF16 exactly as the GPU stores them, so what remains
is the BF16 rounding of the hidden activations and of the back-propagated
gradients (unit roundoff 2^-9 each).  Gradients are compared element by element
against a bound built from the reference's own absolute-value products (see
``_grad_bound``).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp_ref as M
import paper_2403_04578_amd as tpf
from paper_2403_04578_amd import workloads as W

pytestmark = pytest.mark.gpu


def bf16_round(a):
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).to(torch.float32)
    return t.numpy().astype(np.float64)


def _ref_params(params, sizes):
    """Weights rounded to BF16 (as the GPU copies are), biases kept FP32."""
    out = np.array(params, np.float64)
    o = 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        out[o:o + a * b] = bf16_round(params[o:o + a * b])
        o += a * b + b
    return out


def _grad_bound(params, sizes, x, tgt, c=8.0):
    """Element-wise error allowance of the BF16 gradient, flat like the parameters.

    Weight (o, i) of layer l: c 2^-8 sum_r |dZ_l[r, o]| |H_{l-1}[r, i]|; bias o:
    c 2^-8 sum_r |dZ_l[r, o]|, with dZ and H the reference's own output gradients and
    layer inputs.  Each summed product carries the BF16 roundings of its two factors
    (2^-9 relative each), and dZ carries those of the deeper layers it came through.  At
    the output the GPU's y itself is off by the rounding of the last hidden layer, up to
    2^-8 (|H_L| |W|^T + |b|), so |y - t| is widened by that amount (it may be small after
    training).  A model of these rounding points on the host puts the worst element of
    the 99-bus network at 2.2 x 2^-8 of its allowance before the factor c; c = 8 leaves
    a margin of 3.6 while a gradient entry that is lost or misplaced (a padding column,
    a transposed tile) still exceeds its allowance."""
    y, cache = M.forward(params, sizes, x)
    layers = M.unpack(np.asarray(params, np.float64), sizes)
    N = y.size
    h_last, _ = cache[-1]
    W_last, b_last = layers[-1]
    y_abs = np.abs(h_last) @ np.abs(W_last).T + np.abs(b_last)
    dz = 2.0 * (y - tgt) / N
    out = []
    for l in range(len(layers) - 1, -1, -1):
        hin, _ = cache[l]
        W_l, _ = layers[l]
        da = np.abs(dz) if l < len(layers) - 1 else 2.0 * (np.abs(y - tgt) + 2.0 ** -8 * y_abs) / N
        out.append(((da.T @ np.abs(hin)).ravel(), da.sum(axis=0)))
        if l > 0:
            dz = (dz @ W_l) * M.gelu_grad(cache[l - 1][1])
    out.reverse()
    return c * 2.0 ** -8 * np.concatenate([np.concatenate(p) for p in out])


@pytest.fixture(scope="module")
def data(gpu):
    f = W.make_feeder(100)
    net, onet = tpf.Network.from_feeder(f), oracle.build_feeder(f)
    T = 6000
    S = W.profile_minute_year(f, steps=T, seed=W.SEED_TRAIN)
    t = np.arange(T, dtype=np.int64) * 83 % W.MINUTES_PER_YEAR
    Sd = torch.from_numpy(S).to(gpu)
    V, it, st = tpf.solve_timeseries(net, Sd, tol=1e-10, max_iter=100)
    return f, net, onet, S, t, Sd, torch.from_numpy(t).to(gpu), V


@pytest.mark.parametrize("seed", [11, 12])
def test_loss_and_gradient_match_reference(data, seed):
    """Every entry of the gradient (all four weight matrices and bias vectors, the
    calendar-feature columns of W_1 and the 202 -> 256 padding edge included) within its
    element-wise BF16 allowance of the FP64 reference."""
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    p0 = W.mlp_init_params(sizes, seed=seed)
    mlp = tpf.WarmStart(99, params=p0)
    rows = 200
    loss, grad = mlp.loss_grad(Sd[:rows].contiguous(), td[:rows].contiguous(), V[:rows].contiguous())
    g = grad.cpu().numpy().astype(np.float64)
    x = bf16_round(M.features(S[:rows], t[:rows]))
    tgt = M.targets(V[:rows].cpu().numpy())
    pr = _ref_params(p0, sizes)
    lref, gref = M.loss_and_grad(pr, sizes, x, tgt)
    assert abs(float(loss) - lref) <= 1e-2 * lref
    bound = _grad_bound(pr, sizes, x, tgt)
    excess = np.abs(g - gref) / bound
    worst = int(np.argmax(excess))
    assert excess.max() <= 1.0, (worst, g[worst], gref[worst], bound[worst])
    assert np.linalg.norm(g - gref) / np.linalg.norm(gref) < 2e-2


def test_adamw_step_matches_reference(data):
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    p0 = W.mlp_init_params(sizes, seed=12)
    mlp = tpf.WarmStart(99, params=p0)
    Sb, tb, Vb = Sd[:256].contiguous(), td[:256].contiguous(), V[:256].contiguous()
    _, grad = mlp.loss_grad(Sb, tb, Vb)
    mlp.train_step(Sb, tb, Vb, lr=1e-3, weight_decay=1e-2)
    p1 = mlp.get_params().astype(np.float64)
    ref, _, _ = M.adamw_step(p0.astype(np.float64), grad.cpu().numpy().astype(np.float64),
                             np.zeros(p0.size), np.zeros(p0.size), 1, lr=1e-3, wd=1e-2)
    assert np.abs(p1 - ref).max() < 2e-6


def test_adamw_five_steps_match_reference(data):
    """Five AdamW steps on a fixed batch: the moments carried from step to step and the
    bias corrections of steps 2-5 match the reference fed with the same gradients."""
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    p0 = W.mlp_init_params(sizes, seed=14)
    mlp = tpf.WarmStart(99, params=p0)
    Sb, tb, Vb = Sd[1000:1256].contiguous(), td[1000:1256].contiguous(), V[1000:1256].contiguous()
    p_ref, m, v = p0.astype(np.float64), np.zeros(p0.size), np.zeros(p0.size)
    for k in range(1, 6):
        _, grad = mlp.loss_grad(Sb, tb, Vb)  # the gradient the step below computes again
        lr = 1e-3 * (1.0 - 0.15 * k)
        mlp.train_step(Sb, tb, Vb, lr=lr, weight_decay=1e-2)
        p_ref, m, v = M.adamw_step(p_ref, grad.cpu().numpy().astype(np.float64), m, v, k, lr=lr, wd=1e-2)
        err = np.abs(mlp.get_params().astype(np.float64) - p_ref).max()
        assert err < 2e-6 * k, (k, err)


def test_train_full_batch_follows_cosine_schedule(data):
    """tpf_mlp_train with one batch of all rows per epoch equals AdamW steps on the whole
    set at the cosine schedule's rates (the gathered batch is a permutation of the rows,
    so only the order of the gradient sums differs)."""
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    p0 = W.mlp_init_params(sizes, seed=15)
    rows, epochs, lr, lr_min = 512, 3, 1e-3, 1e-4
    Sb, tb, Vb = Sd[:rows].contiguous(), td[:rows].contiguous(), V[:rows].contiguous()
    a = tpf.WarmStart(99, params=p0)
    hist = a.fit(Sb, tb, Vb, epochs=epochs, batch=rows, lr=lr, lr_min=lr_min, weight_decay=1e-3, seed=5)
    b = tpf.WarmStart(99, params=p0)
    for k in range(epochs):
        rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * k / (epochs - 1)))
        loss = b.train_step(Sb, tb, Vb, lr=rate, weight_decay=1e-3)
        assert abs(hist[k] - float(loss)) <= 1e-4 * float(loss), (k, hist[k], float(loss))
    assert np.abs(a.get_params() - b.get_params()).max() < 3e-5


def test_train_epoch_visits_every_row_once(data):
    """With zero learning rates nothing moves, and an epoch's mean batch loss is the loss
    of the whole set exactly when the epoch's order is a permutation of the rows."""
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    p0 = W.mlp_init_params(sizes, seed=16)
    rows = 1000
    Sb, tb, Vb = Sd[:rows].contiguous(), td[:rows].contiguous(), V[:rows].contiguous()
    mlp = tpf.WarmStart(99, params=p0)
    full, _ = mlp.loss_grad(Sb, tb, Vb)
    for batch, seed in ((100, 1), (125, 2), (250, 3)):
        hist = mlp.fit(Sb, tb, Vb, epochs=2, batch=batch, lr=0.0, lr_min=0.0, seed=seed)
        for h in hist:
            assert abs(h - float(full)) <= 2e-5 * float(full), (batch, seed, h, float(full))
    assert np.array_equal(mlp.get_params(), p0)


def test_train_resume_from_file_is_bitwise(data, tmp_path):
    """Two epochs, save (parameters, AdamW moments and step count), load, two more epochs:
    the same parameters bit for bit as four epochs in one call."""
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    p0 = W.mlp_init_params(sizes, seed=17)
    rows = 1000
    Sb, tb, Vb = Sd[:rows].contiguous(), td[:rows].contiguous(), V[:rows].contiguous()
    kw = dict(batch=128, lr=2e-3, lr_min=1e-5, weight_decay=1e-4, seed=9, total_epochs=4)
    a = tpf.WarmStart(99, params=p0)
    a.fit(Sb, tb, Vb, epochs=4, **kw)
    b = tpf.WarmStart(99, params=p0)
    b.fit(Sb, tb, Vb, epochs=2, first_epoch=0, **kw)
    path = str(tmp_path / "half.bin")
    b.save(path)
    c = tpf.WarmStart.load(path)
    assert np.array_equal(c.get_params(), b.get_params())
    c.fit(Sb, tb, Vb, epochs=2, first_epoch=2, **kw)
    pa, pc = a.get_params(), c.get_params()
    assert np.array_equal(pa, pc), np.abs(pa - pc).max()
    # a restart without the moments (what a parameters-only checkpoint would give) differs
    d = tpf.WarmStart(99, params=b.get_params())
    d.fit(Sb, tb, Vb, epochs=2, first_epoch=2, **kw)
    assert not np.array_equal(d.get_params(), pa)


def _predict_tol(y):
    """Allowed start-voltage error of the inference kernel, in pu.

    The reference takes the BF16-rounded weights and features, so what remains is the BF16
    rounding of the three hidden layers' activations (2^-9 relative each, random in sign)
    and the kernel's GELU polynomial (below 1.3e-5 |z|).  Together they leave about 2^-8 of
    the output's scale max |y| (measured 4e-3 max |y| for two random initialisations at 130
    and 2,000 rows); the bound 2^-6 max |y| keeps a factor 4 over that, while a wrong GELU
    coefficient or a misplaced tile errs by a sizeable fraction of |y|.  y is in the
    network's output units (OUT_SCALE x the voltage)."""
    return 2.0 ** -6 * np.abs(y).max() / M.OUT_SCALE


def test_prediction_matches_reference_forward(data):
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    p0 = W.mlp_init_params(sizes, seed=13)
    mlp = tpf.WarmStart(99, params=p0)
    rows = 130  # not a multiple of the 64-row tile
    V0 = mlp.predict(Sd[:rows].contiguous(), td[:rows].contiguous())
    y, _ = M.forward(_ref_params(p0, sizes), sizes, bf16_round(M.features(S[:rows], t[:rows])))
    ref = M.to_voltage(y)
    err = np.abs(V0.cpu().numpy() - ref).max()
    assert err < _predict_tol(y), (err, _predict_tol(y))


def test_training_reduces_sweeps_and_keeps_results(data, tmp_path):
    """What the trained network gains: fewer sweeps from its start than from a flat
    start, to the same solution."""
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    mlp = tpf.WarmStart(99, params=W.mlp_init_params(sizes))
    ntr = 5000
    hist = mlp.fit(Sd[:ntr].contiguous(), td[:ntr].contiguous(), V[:ntr].contiguous(), epochs=30, batch=500,
                   lr=2e-3)
    assert hist[-1] < 0.05 * hist[0], hist
    Sv, tv = Sd[ntr:].contiguous(), td[ntr:].contiguous()
    V0 = mlp.predict(Sv, tv)
    start_err = float((V0 - V[ntr:]).abs().max())
    assert start_err < 5e-3
    for mode in ("fp64", "mixed_fp16"):
        tol = 1e-6
        Vw, iw, sw = tpf.solve_timeseries(net, Sv, tol, 100, mode=mode, V0=V0)
        Vf, i_f, sf = tpf.solve_timeseries(net, Sv, tol, 100, mode=mode)
        assert int(sw.max()) == tpf.ST_CONVERGED
        assert float(iw.float().mean()) < float(i_f.float().mean()) - 0.5, mode
        assert float((Vw - V[ntr:]).abs().max()) < 1e-6
    # save / load round trip keeps the parameters and the prediction
    path = str(tmp_path / "ws.bin")
    mlp.save(path)
    m2 = tpf.WarmStart.load(path)
    assert np.array_equal(m2.get_params(), mlp.get_params())
    assert torch.equal(m2.predict(Sv, tv), V0)


def test_nonfinite_parameters_fall_back_to_flat_start(data):
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    bad = np.full(M.num_params(sizes), np.nan, np.float32)
    mlp = tpf.WarmStart(99, params=bad)
    Sv, tv = Sd[:300].contiguous(), td[:300].contiguous()
    V0 = mlp.predict(Sv, tv)
    assert torch.isnan(V0).all()
    Vw, iw, sw = tpf.solve_timeseries(net, Sv, 1e-8, 100, V0=V0)
    Vf, i_f, sf = tpf.solve_timeseries(net, Sv, 1e-8, 100)
    assert torch.equal(Vw, Vf) and torch.equal(iw, i_f)


@pytest.mark.parametrize("rows", [1, 47, 48, 49, 95, 96, 97, 128, 1000])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_fused_prediction_ragged_rows_and_dtypes(data, rows, dtype):
    """The inference kernel works on 96-row tiles whose outputs leave in two 48-row
    halves: partial last tiles and halves, both complex dtypes, and rows far apart in the
    year (calendar features) all match the reference."""
    f, net, onet, S, t, Sd, td, V = data
    sizes = W.mlp_sizes(99)
    p0 = W.mlp_init_params(sizes, seed=21)
    mlp = tpf.WarmStart(99, params=p0)
    Sx = Sd[-rows:].to(dtype).contiguous()
    V0 = mlp.predict(Sx, td[-rows:].contiguous())
    assert V0.dtype == dtype and V0.shape == Sx.shape
    Sh = Sx.cpu().numpy().astype(np.complex128)
    y, _ = M.forward(_ref_params(p0, sizes), sizes, bf16_round(M.features(Sh, t[-rows:])))
    err = np.abs(V0.cpu().numpy().astype(np.complex128) - M.to_voltage(y)).max()
    assert err < _predict_tol(y) + (1e-7 if dtype == torch.complex64 else 0.0), err
