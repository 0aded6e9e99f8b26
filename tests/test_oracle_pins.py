"""Pins of the CPU oracle to facts fixed by the paper and by the mathematics.

Each test checks the oracle against something other than itself: the paper's
two-bus worked example (Sec. III, Fig. 1) through the closed form of the
two-bus power flow, the star-feeder reduction to independent two-bus problems,
the path-impedance structure of Y_dd^-1 on radial feeders, the zero-load case,
an independent dense Newton-Raphson, the exact mismatch identity of one sweep,
the contraction behaviour (Sec. II, Eqs. (4)-(6)), the robustness claim of
Fig. 3, the feasibility region of Eq. (11), and the critical-loading conic of
Eq. (10) in its corrected form.  A dropped term, a wrong sign or a transposed
operand in the oracle breaks at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2403_04578_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_twobus():
    vals = {}
    with open(os.path.join(GOLDEN, "twobus_fig1.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return complex(vals["z_s_re"], vals["z_s_im"]), vals["v0_abs"], complex(vals["p_l"], vals["q_l"])


def twobus_roots(z, vs, s):
    """Both roots of the two-bus power flow V = vs - z conj(s / V).

    Multiplying by conj(V): |V|^2 = vs conj(V) - z conj(s), whose modulus gives
    |V|^4 - (|vs|^2 - 2 Re(z conj(s))) |V|^2 + |z|^2 |s|^2 = 0; then
    V = (|V|^2 + conj(z) s) / conj(vs).  Returns (V_high, V_low).
    """
    a = abs(vs) ** 2 - 2.0 * (z.real * s.real + z.imag * s.imag)
    disc = a * a - 4.0 * abs(z) ** 2 * abs(s) ** 2
    r = math.sqrt(disc)
    hi, lo = (a + r) / 2.0, (a - r) / 2.0
    return (hi + np.conj(z) * s) / np.conj(vs), (lo + np.conj(z) * s) / np.conj(vs)


def _twobus_net(z, vs=1.0 + 0.0j):
    return oracle.build_network(2, [0], [1], [z.real], [z.imag], 0, vs)


# ----------------------------------------------------------------------------- Sec. III

def test_paper_twobus_example_high_root():
    z, v0, s = _golden_twobus()
    net = _twobus_net(z, v0)
    res = oracle.fpi(net, np.array([[s]]), 1e-14, 500)
    vh, vl = twobus_roots(z, v0, s)
    assert res.status[0] == oracle.ST_CONVERGED
    # a posteriori bound of the contraction: |V - V*| <= k/(1-k) d, k = 0.611 here
    assert abs(res.V[0, 0] - vh) < 1e-13
    # values derived from the printed example
    assert abs(vh - (0.620830459736 + 0.02j)) < 1e-11
    assert abs(vl - (0.379169540264 + 0.02j)) < 1e-11
    # Sec. III: s_l = (r_l + j x_l) |v0|^2 / |z_s + z_l|^2 for the equivalent load impedance
    zl = abs(res.V[0, 0]) ** 2 / np.conj(s)
    assert abs(zl * v0 ** 2 / abs(z + zl) ** 2 - s) < 1e-12
    # the operational root lies outside the |z_s| circle, the other inside (Sec. III)
    zl_low = abs(vl) ** 2 / np.conj(s)
    assert abs(zl) > abs(z) > abs(zl_low)
    # Eq. (6): k = |z_jj| / |z_l| < 1 only for the high-impedance root
    assert abs(z) / abs(zl) < 1.0 < abs(z) / abs(zl_low)
    assert abs(abs(z) / abs(zl) - 0.611) < 1e-3


def test_fpi_reaches_high_root_from_any_start():
    # Fig. 3: FPI converges to the operational point whatever the initial voltage
    z, v0, s = _golden_twobus()
    net = _twobus_net(z, v0)
    rng = np.random.default_rng(0)
    mag = rng.uniform(0.05, 2.0, 2000)
    ang = rng.uniform(-math.pi, math.pi, 2000)
    V0 = (mag * np.exp(1j * ang))[:, None]
    S = np.full((2000, 1), s)
    res = oracle.fpi(net, S, 1e-13, 1000, V0)
    vh, _ = twobus_roots(z, v0, s)
    assert np.all(res.status == oracle.ST_CONVERGED)
    assert np.abs(res.V[:, 0] - vh).max() < 1e-11
    # consistent iteration counts over the start region
    assert res.iters.max() - res.iters.min() < 40


def test_infeasible_load_never_converges():
    # Eq. (11) violated and no real root: |v0|^2 < 4 |s| |z|
    z = 1.0 + 0.5j
    s = 0.25 + 0.15j
    assert 1.0 < 4 * abs(s) * abs(z)
    a = 1.0 - 2.0 * (z.real * s.real + z.imag * s.imag)
    assert a * a - 4 * abs(z) ** 2 * abs(s) ** 2 < 0
    res = oracle.fpi(_twobus_net(z), np.array([[s]]), 1e-6, 100)
    assert res.status[0] == oracle.ST_MAX_ITER and res.iters[0] == 100
    steps = [oracle.fpi(_twobus_net(z), np.array([[s]]), 0.0, k).d[0] for k in range(2, 101, 7)]
    assert min(steps) > 0.05


def test_feasibility_region_eq11_implies_convergence():
    # any two-bus load inside |v0|^2 >= 4|s||z| has a solution that FPI finds
    rng = np.random.default_rng(1)
    for _ in range(300):
        z = complex(*rng.uniform(0.01, 1.0, 2))
        ang = rng.uniform(-math.pi / 2, math.pi / 2)
        smax = 1.0 / (4.0 * abs(z))
        s = rng.uniform(0.01, 0.95) * smax * complex(math.cos(ang), math.sin(ang))
        res = oracle.fpi(_twobus_net(z), np.array([[s]]), 1e-12, 5000)
        assert res.status[0] == oracle.ST_CONVERGED
        assert abs(res.V[0, 0] - twobus_roots(z, 1.0, s)[0]) < 1e-9


def test_corrected_critical_conic_eq10():
    # Along s = t (0.18 + j0.11) on z_s = 1 + j0.5 the two roots merge where the
    # discriminant vanishes; the corrected Eq. (10) is zero exactly there.
    z, v0, s_dir = _golden_twobus()
    rs, xs = z.real, z.imag
    lo, hi = 0.5, 2.0
    for _ in range(200):
        t = 0.5 * (lo + hi)
        s = t * s_dir
        a = v0 ** 2 - 2.0 * (rs * s.real + xs * s.imag)
        if a * a - 4 * abs(z) ** 2 * abs(s) ** 2 > 0:
            lo = t
        else:
            hi = t
    s = lo * s_dir
    p, q = s.real, s.imag
    G, H, I, J, K, L = rs ** 2, -2 * rs * xs, xs ** 2, v0 ** 2 * xs, v0 ** 2 * rs, -v0 ** 4 / 4
    assert abs(G * q * q + H * p * q + I * p * p + J * q + K * p + L) < 1e-12
    assert abs(H * H - 4 * G * I) < 1e-15  # parabola
    # the coefficients as printed do not vanish on the critical load
    Gp, Hp, Ip, Jp, Kp, Lp = rs ** 2, -2 * rs * xs, v0 ** 2 * xs, xs ** 2, v0 ** 2 * rs, -v0 ** 2 / 4
    assert abs(Gp * q * q + Hp * p * q + Ip * p * p + Jp * q + Kp * p + Lp) > 1e-3
    # near the critical point the contraction factor approaches 1: many more sweeps
    slow = oracle.fpi(_twobus_net(z), np.array([[0.999 * s]]), 1e-9, 100000)
    fast = oracle.fpi(_twobus_net(z), np.array([[0.5 * s]]), 1e-9, 100000)
    assert slow.status[0] == oracle.ST_CONVERGED and slow.iters[0] > 5 * fast.iters[0]


# ----------------------------------------------------------------------------- Sec. II

def _paths(feeder):
    parent = {int(t): (int(f), k) for k, (f, t) in enumerate(zip(feeder.frm, feeder.to))}
    paths = {}
    for b in range(1, feeder.n_bus):
        br = set()
        u = b
        while u != 0:
            p, k = parent[u]
            br.add(k)
            u = p
        paths[b] = br
    return paths


@pytest.mark.parametrize("n_bus", [2, 10, 37, 100])
def test_zbus_is_path_impedance(n_bus):
    # For a shunt-free radial feeder, (Y_dd^-1)[i, j] is the sum of the impedances of
    # the branches shared by the slack->i and slack->j paths; the diagonal is the
    # Thevenin impedance of Eq. (6).
    f = W.make_feeder(n_bus, seed=7)
    net = oracle.build_feeder(f)
    z = f.r + 1j * f.x
    paths = _paths(f)
    n = n_bus - 1
    expect = np.zeros((n, n), complex)
    for i in range(n):
        for j in range(n):
            expect[i, j] = sum(z[k] for k in paths[i + 1] & paths[j + 1])
    assert np.abs(-net.Z - expect).max() <= 1e-13 * np.abs(expect).max()


def test_w_equals_slack_voltage_without_shunts():
    # rows of a shunt-free Y sum to zero: Y_ds = -Y_dd 1, hence w = v_s 1
    f = W.make_feeder(60, seed=3)
    vs = 1.02 * np.exp(1j * math.radians(5.0))
    net = oracle.build_network(f.n_bus, f.frm, f.to, f.r, f.x, 0, vs)
    assert np.abs(net.w - vs).max() < 1e-13


def test_zero_load_gives_slack_voltage_after_one_sweep():
    f = W.make_feeder(50, seed=9)
    net = oracle.build_feeder(f)
    res = oracle.fpi(net, np.zeros((3, 49)), 1e-12, 50)
    assert np.all(res.iters == 1) and np.all(res.status == oracle.ST_CONVERGED)
    assert np.abs(res.V - 1.0).max() < 1e-13


def test_star_feeder_is_independent_twobus():
    rng = np.random.default_rng(4)
    z = rng.uniform(0.01, 0.1, 25) + 1j * rng.uniform(0.01, 0.1, 25)
    f = W.make_star_feeder(z)
    net = oracle.build_feeder(f)
    S = rng.uniform(0.1, 1.0, (40, 25)) + 1j * rng.uniform(0.0, 0.5, (40, 25))  # 4|s||z| < 1
    res = oracle.fpi(net, S, 1e-14, 2000)
    expect = np.array([[twobus_roots(z[i], 1.0, S[c, i])[0] for i in range(25)] for c in range(40)])
    assert np.abs(res.V - expect).max() < 1e-12


def _nr_dense(feeder, S, tol=1e-13, max_iter=50):
    """Rectangular Newton-Raphson on m(V) = S + V conj(Y_ds v_s + Y_dd V) = 0 from a flat start."""
    N, n = feeder.n_bus, feeder.n_bus - 1
    Y = np.zeros((N, N), complex)
    for f, t, r, x in zip(feeder.frm, feeder.to, feeder.r, feeder.x):
        y = 1.0 / complex(r, x)
        Y[f, f] += y
        Y[t, t] += y
        Y[f, t] -= y
        Y[t, f] -= y
    Ydd, c = Y[1:, 1:], Y[1:, 0] * feeder.vs
    out = []
    for s in S:
        V = np.ones(n, complex)
        for _ in range(max_iter):
            a = c + Ydd @ V
            m = s + V * np.conj(a)
            if np.abs(m).max() < tol:
                break
            J1 = np.diag(np.conj(a)) + np.diag(V) @ np.conj(Ydd)
            J2 = 1j * (np.diag(np.conj(a)) - np.diag(V) @ np.conj(Ydd))
            Jr = np.block([[J1.real, J2.real], [J1.imag, J2.imag]])
            dx = np.linalg.solve(Jr, -np.concatenate([m.real, m.imag]))
            V = V + dx[:n] + 1j * dx[n:]
        out.append(V)
    return np.array(out)


@pytest.mark.parametrize("n_bus,seed", [(5, 1), (12, 2), (20, 3), (31, 4)])
def test_fpi_agrees_with_dense_newton_raphson(n_bus, seed):
    f = W.make_feeder(n_bus, seed=seed)
    S = W.profile_minute_year(f, steps=25, seed=seed, t0=1000 * seed) * 3.0
    net = oracle.build_feeder(f)
    res = oracle.fpi(net, S, 1e-13, 500)
    assert np.all(res.status == oracle.ST_CONVERGED)
    Vnr = _nr_dense(f, S)
    assert np.abs(res.V - Vnr).max() < 1e-11
    assert np.abs(Vnr).min() > 0.5  # the operational (high-voltage) root


def test_mismatch_identity_of_one_sweep():
    # After V(n) = Z conj(S./V(n-1)) + w:  Y_ds v_s + Y_dd V(n) = -conj(S./V(n-1)), so
    # m(V(n)) = S .* (V(n-1) - V(n)) ./ V(n-1) exactly (up to rounding).
    f = W.make_feeder(40, seed=11)
    net = oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=30, seed=5) * 2.0
    for k in (1, 2, 4):
        prev = oracle.fpi(net, S, 0.0, k - 1).V
        cur = oracle.fpi(net, S, 0.0, k).V
        expect = np.abs(S * (prev - cur) / prev).max(axis=1)
        got = oracle.mismatch(net, S, cur)
        assert np.all(np.abs(got - expect) <= 1e-13 + 1e-9 * expect)
    # and the converged solution balances power
    res = oracle.fpi(net, S, 1e-12, 100)
    assert oracle.mismatch(net, S, res.V).max() < 1e-12


def test_step_sizes_contract_geometrically():
    # Banach (Eqs. (4)-(6)): with k < 1 the steps shrink by a roughly constant factor
    f = W.make_feeder(100)
    net = oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=8, t0=600)
    d = np.array([oracle.fpi(net, S, 0.0, k).d for k in range(1, 8)])
    ratio = d[1:] / d[:-1]
    assert np.all(ratio[:5] < 0.2)
    # a posteriori error bound |V_k - V*| <= rho/(1-rho) d_k
    vstar = oracle.fpi(net, S, 1e-15, 200).V
    for k in range(2, 6):
        vk = oracle.fpi(net, S, 0.0, k).V
        rho = ratio[:, :].max()
        assert np.all(np.abs(vk - vstar).max(axis=1) <= rho / (1 - rho) * d[k - 1] * 1.5 + 1e-15)


# ----------------------------------------------------------------------------- Algorithm 1 semantics

def test_stopping_rule_is_first_step_below_tol():
    f = W.make_feeder(30, seed=2)
    net = oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=50, seed=8)
    res = oracle.fpi(net, S, 1e-8, 100)
    for c in range(50):
        k = res.iters[c]
        fixed = oracle.fpi(net, S[c:c + 1], 0.0, k)
        assert np.array_equal(fixed.V[0], res.V[c])
        assert fixed.d[0] < 1e-8
        before = oracle.fpi(net, S[c:c + 1], 0.0, k - 1)
        assert before.d[0] >= 1e-8


def test_zero_iterations_and_nonfinite():
    f = W.make_feeder(8, seed=2)
    net = oracle.build_feeder(f)
    S = W.profile_daily96(f)[:3].copy()
    r0 = oracle.fpi(net, S, 1e-6, 0)
    assert np.all(r0.V == 1.0) and np.all(r0.iters == 0) and np.all(r0.status == oracle.ST_MAX_ITER)
    S[1, 3] = np.nan
    r = oracle.fpi(net, S, 1e-10, 100)
    assert list(r.status) == [oracle.ST_CONVERGED, oracle.ST_NONFINITE, oracle.ST_CONVERGED]
    assert r.iters[1] == 1


def test_columns_are_independent():
    f = W.make_feeder(25, seed=6)
    net = oracle.build_feeder(f)
    S = W.profile_minute_year(f, steps=64, seed=3)
    all_ = oracle.fpi(net, S, 1e-9, 100)
    one = oracle.fpi(net, S[17:18], 1e-9, 100)
    assert np.array_equal(all_.V[17], one.V[0]) and all_.iters[17] == one.iters[0]


def test_singular_and_invalid_networks():
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_network(4, [0, 2], [1, 3], [0.01, 0.01], [0.01, 0.01])
    assert e.value.code == -2
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_network(3, [0, 1], [1, 2], [0.01, 0.0], [0.01, 0.0])
    assert e.value.code == -1


# ----------------------------------------------------------------------------- Eq. (2), ZIP loads

def _zip_numpy_balance(net, S, V, ai, ap):
    """Power balance of ZIP loads written independently of the oracle: a load draws
    s (alpha_P + alpha_I v), the network delivers -v conj(Y_ds v_s + Y_dd v)."""
    inj = net.Yds[None, :] * net.vs + V @ net.Ydd.T
    return np.abs(S * (ap + ai * V) + V * np.conj(inj)).max(axis=1)


def test_zip_constant_power_reduces_to_algorithm1():
    f = W.make_feeder(30)
    net = oracle.build_feeder(f)
    S = W.profile_daily96(f)
    a = oracle.fpi(net, S, 1e-12, 100)
    b = oracle.fpi_zip(net, S, 0.0, 1.0, 1e-12, 100)
    assert np.array_equal(a.iters, b.iters) and np.array_equal(a.status, b.status)
    assert np.abs(a.V - b.V).max() < 1e-13


def test_zip_constant_current_is_one_linear_solve():
    """alpha_P = 0: F = 0, the map is constant, so the first sweep lands on
    v = -Y_dd^-1 (Y_ds v_s + alpha_I s*) (a library solve, not the oracle's inverse)
    and the second sweep does not move."""
    f = W.make_feeder(40)
    net = oracle.build_feeder(f)
    S = W.profile_daily96(f, steps=8)
    res = oracle.fpi_zip(net, S, 1.0, 0.0, 1e-12, 10)
    assert np.all(res.iters == 2) and np.all(res.status == oracle.ST_CONVERGED)
    rhs = -(net.Yds[None, :] * net.vs + np.conj(S))
    Vs = np.linalg.solve(net.Ydd, rhs.T).T
    assert np.abs(res.V - Vs).max() < 1e-12
    assert _zip_numpy_balance(net, S, res.V, 1.0, 0.0).max() < 1e-11


def test_zip_twobus_closed_form():
    """One PQ bus behind z: v = v_s - z (alpha_P s*/v* + alpha_I s*).  Multiplying by v*
    gives the constant-power two-bus problem with source u = v_s - z alpha_I s* and load
    alpha_P s, whose high root is closed-form."""
    z, vs = 0.05 + 0.08j, 1.02 + 0.01j
    net = _twobus_net(z, vs)
    for s, ai, ap in [(0.9 + 0.4j, 0.3, 0.7), (1.5 + 0.2j, 0.8, 0.2), (0.6 - 0.3j, 0.5, 0.5)]:
        res = oracle.fpi_zip(net, np.array([[s]]), ai, ap, 1e-14, 500)
        assert res.status[0] == oracle.ST_CONVERGED
        u = vs - z * ai * np.conj(s)
        vh, _ = twobus_roots(z, u, ap * s)
        assert abs(res.V[0, 0] - vh) < 1e-12, (s, ai, ap)


@pytest.mark.parametrize("seed", [0, 1])
def test_zip_mixed_shares_satisfy_power_balance(seed):
    f = W.make_feeder(60, load_scale=3.0)
    net = oracle.build_feeder(f)
    S = W.profile_daily96(f, steps=12)
    rng = np.random.default_rng(seed)
    ai = rng.uniform(0.0, 1.0, net.n)
    ap = 1.0 - ai
    res = oracle.fpi_zip(net, S, ai, ap, 1e-13, 200)
    assert np.all(res.status == oracle.ST_CONVERGED)
    bal = _zip_numpy_balance(net, S, res.V, ai, ap)
    assert bal.max() < 1e-11
    assert oracle.mismatch_zip(net, S, res.V, ai, ap).max() < 1e-11
    # away from the solution the two formulas agree to rounding
    Vp = res.V + 1e-3 * (rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape))
    assert np.allclose(oracle.mismatch_zip(net, S, Vp, ai, ap), _zip_numpy_balance(net, S, Vp, ai, ap),
                       rtol=1e-10, atol=1e-13)
    # the constant-current share moves the solution, and the constant-power mismatch sees it
    cp = oracle.fpi(net, S, 1e-13, 200)
    assert np.abs(cp.V - res.V).max() > 1e-5
    assert oracle.mismatch(net, S, res.V).max() > 1e-6


def _zipz_numpy_balance(net, S, V, az, ai, ap):
    """Power balance with a constant-impedance share too, written independently of the
    oracle: the load current alpha_Z s* v draws alpha_Z s |v|^2."""
    inj = net.Yds[None, :] * net.vs + V @ net.Ydd.T
    return np.abs(S * (ap + ai * V + az * np.abs(V) ** 2) + V * np.conj(inj)).max(axis=1)


def test_zipz_twobus_closed_form():
    """One PQ bus behind z with all three shares: (y + alpha_Z s*) v = y v_s - alpha_I s*
    - alpha_P s*/v*, i.e. v = v_s' - z' alpha_P s*/v* with v_s' = (v_s - z alpha_I s*) /
    (1 + z alpha_Z s*) and z' = z / (1 + z alpha_Z s*): the constant-power two-bus problem
    again, whose high root is closed-form."""
    z, vs = 0.05 + 0.08j, 1.02 + 0.01j
    net = _twobus_net(z, vs)
    for s, az, ai, ap in [(0.9 + 0.4j, 0.3, 0.3, 0.4), (1.2 - 0.2j, 0.6, 0.1, 0.3), (0.7 + 0.7j, 0.2, 0.0, 0.8),
                          (1.5 + 0.5j, 1.0, 0.0, 0.0)]:
        res = oracle.fpi_zip(net, np.array([[s]]), ai, ap, 1e-14, 500, alpha_z=az)
        assert res.status[0] == oracle.ST_CONVERGED
        k = 1.0 + z * az * np.conj(s)
        vs2, z2 = (vs - z * ai * np.conj(s)) / k, z / k
        vh = twobus_roots(z2, vs2, ap * s)[0] if ap > 0 else vs2
        assert abs(res.V[0, 0] - vh) < 1e-12, (s, az, ai, ap)
        assert _zipz_numpy_balance(net, np.array([[s]]), res.V, az, ai, ap)[0] < 1e-12


def test_zipz_impedance_only_is_one_linear_solve():
    """alpha_P = 0: F = 0 and the first sweep lands on v = -(diag(alpha_Z s*) + Y_dd)^-1
    (Y_ds v_s + alpha_I s*), a library solve per column; the second sweep does not move."""
    f = W.make_feeder(25)
    net = oracle.build_feeder(f)
    S = W.profile_daily96(f, steps=6)
    rng = np.random.default_rng(4)
    az = rng.uniform(0.2, 1.0, net.n)
    ai = 1.0 - az
    res = oracle.fpi_zip(net, S, ai, 0.0, 1e-12, 10, alpha_z=az)
    assert np.all(res.iters == 2) and np.all(res.status == oracle.ST_CONVERGED)
    for c in range(S.shape[0]):
        B = net.Ydd + np.diag(az * np.conj(S[c]))
        v = np.linalg.solve(B, -(net.Yds * net.vs + ai * np.conj(S[c])))
        assert np.abs(res.V[c] - v).max() < 1e-12
    assert _zipz_numpy_balance(net, S, res.V, az, ai, 0.0).max() < 1e-11


def test_zipz_zero_share_is_the_alpha_z_free_iteration():
    f = W.make_feeder(30)
    net = oracle.build_feeder(f)
    S = W.profile_daily96(f, steps=10)
    a = oracle.fpi_zip(net, S, 0.3, 0.7, 1e-12, 100)
    b = oracle.fpi_zip(net, S, 0.3, 0.7, 1e-12, 100, alpha_z=0.0)
    assert np.array_equal(a.iters, b.iters) and np.array_equal(a.status, b.status)
    assert np.abs(a.V - b.V).max() < 1e-13


@pytest.mark.parametrize("seed", [0, 1])
def test_zipz_mixed_shares_satisfy_power_balance(seed):
    f = W.make_feeder(60, load_scale=3.0)
    net = oracle.build_feeder(f)
    S = W.profile_daily96(f, steps=12)
    rng = np.random.default_rng(seed)
    sh = rng.dirichlet([1.0, 1.0, 1.0], net.n)
    az, ai, ap = sh[:, 0], sh[:, 1], sh[:, 2]
    res = oracle.fpi_zip(net, S, ai, ap, 1e-13, 200, alpha_z=az)
    assert np.all(res.status == oracle.ST_CONVERGED)
    assert _zipz_numpy_balance(net, S, res.V, az, ai, ap).max() < 1e-11
    assert oracle.mismatch_zip(net, S, res.V, ai, ap, alpha_z=az).max() < 1e-11
    Vp = res.V + 1e-3 * (rng.standard_normal(S.shape) + 1j * rng.standard_normal(S.shape))
    assert np.allclose(oracle.mismatch_zip(net, S, Vp, ai, ap, alpha_z=az),
                       _zipz_numpy_balance(net, S, Vp, az, ai, ap), rtol=1e-10, atol=1e-13)
    # the constant-impedance share moves the solution, and the alpha_Z-free balance sees it
    nz = oracle.fpi_zip(net, S, ai + az, ap, 1e-13, 200)
    assert np.abs(nz.V - res.V).max() > 1e-5
    assert oracle.mismatch_zip(net, S, res.V, ai + az, ap).max() > 1e-6


# ----------------------------------------------------------------------------- three phases

def _a2():
    return np.exp(-2j * math.pi / 3.0)


def test_3ph_zbus_is_path_impedance_blocks():
    """Radial three-phase feeder: block (i, j) of Y_dd^-1 is the sum of the branch
    impedance matrices shared by the slack->i and slack->j paths; w = v_s per phase."""
    f = W.make_feeder_3ph(30, seed=7)
    net = oracle.build_feeder_3ph(f)
    paths = _paths(f)
    n = f.n_bus - 1
    expect = np.zeros((3 * n, 3 * n), complex)
    for i in range(n):
        for j in range(n):
            for k in paths[i + 1] & paths[j + 1]:
                expect[3 * i:3 * i + 3, 3 * j:3 * j + 3] += f.zabc[k]
    assert np.abs(-net.Z - expect).max() <= 1e-13 * np.abs(expect).max()
    assert np.abs(net.w - np.tile(f.vs_abc, n)).max() < 1e-13


def test_3ph_uncoupled_phases_are_three_single_phase_feeders():
    f1 = W.make_feeder(40, seed=2)
    z = f1.r + 1j * f1.x
    scale = (1.0, 1.3, 0.7)
    zabc = np.zeros((len(z), 3, 3), complex)
    for p in range(3):
        zabc[:, p, p] = z * scale[p]
    vs = W.balanced_slack() * 1.01
    net = oracle.build_network_3ph(f1.n_bus, f1.frm, f1.to, zabc, 0, vs)
    S1 = W.profile_daily96(f1, steps=20)
    S = np.stack([S1 * (0.8 + 0.2 * p) for p in range(3)], axis=2).reshape(20, -1)
    res = oracle.fpi(net, S, 1e-13, 200)
    for p in range(3):
        zp = z * scale[p]
        single = oracle.build_network(f1.n_bus, f1.frm, f1.to, zp.real, zp.imag, 0, vs[p])
        assert np.abs(net.Z[p::3, p::3] - single.Z).max() < 1e-14
        other = [q for q in range(3) if q != p]
        assert np.abs(net.Z[p::3][:, other[0]::3]).max() == 0.0
        r1 = oracle.fpi(single, S1 * (0.8 + 0.2 * p), 1e-13, 200)
        assert np.abs(res.V[:, p::3] - r1.V).max() < 1e-12


def test_3ph_balanced_transposed_line_is_its_positive_sequence():
    """Equal self and equal mutual impedances, a balanced source and balanced loads: the
    solution is a positive-sequence set whose phase a solves the single-phase feeder
    with z1 = z_self - z_mutual (I_a + I_b + I_c = 0 cancels the coupling)."""
    f1 = W.make_feeder(35, seed=4, load_scale=4.0)
    zs = f1.r + 1j * f1.x
    zm = 0.4 * zs
    zabc = zm[:, None, None] * np.ones((3, 3)) + (zs - zm)[:, None, None] * np.eye(3)
    net = oracle.build_network_3ph(f1.n_bus, f1.frm, f1.to, zabc)
    S1 = W.profile_daily96(f1, steps=16)
    S = np.repeat(S1, 3, axis=1)
    res = oracle.fpi(net, S, 1e-13, 200)
    z1 = zs - zm
    single = oracle.build_network(f1.n_bus, f1.frm, f1.to, z1.real, z1.imag)
    r1 = oracle.fpi(single, S1, 1e-13, 200)
    assert np.all(res.status == oracle.ST_CONVERGED)
    a2 = _a2()
    assert np.abs(res.V[:, 0::3] - r1.V).max() < 1e-12
    assert np.abs(res.V[:, 1::3] - a2 * r1.V).max() < 1e-12
    assert np.abs(res.V[:, 2::3] - np.conj(a2) * r1.V).max() < 1e-12
    # the coupling matters: the same loads on uncoupled phases with z_self land elsewhere
    loose = oracle.build_network(f1.n_bus, f1.frm, f1.to, zs.real, zs.imag)
    assert np.abs(oracle.fpi(loose, S1, 1e-13, 200).V - r1.V).max() > 1e-4


@pytest.mark.parametrize("seed", [0, 1])
def test_zipz_injection_splitting_has_the_same_fixed_point(seed):
    """The dense forms keep the shared Z and w and carry the constant-impedance current in
    the injection, V <- Z (alpha_P conj(S./V) + alpha_I conj(S) + alpha_Z conj(S) V) + w,
    instead of eliminating diag(alpha_Z s*) into B per column.  Written out here with plain
    numpy from a flat start, that iteration lands on the oracle's per-column-B solution
    (other iterates, the same fixed point), at three times the base load."""
    f = W.make_feeder(60, load_scale=3.0)
    net = oracle.build_feeder(f)
    S = W.profile_daily96(f, steps=12)
    sh = np.random.default_rng(seed).dirichlet([1.0, 1.0, 1.0], net.n)
    az, ai, ap = sh[:, 0], sh[:, 1], sh[:, 2]
    ref = oracle.fpi_zip(net, S, ai, ap, 1e-13, 200, alpha_z=az)
    assert np.all(ref.status == oracle.ST_CONVERGED)
    V = np.ones_like(S)
    for _ in range(200):
        inj = ap * np.conj(S / V) + ai * np.conj(S) + az * np.conj(S) * V
        Vn = inj @ net.Z.T + net.w
        step, V = np.abs(Vn - V).max(), Vn
        if step < 1e-14:
            break
    assert step < 1e-14
    assert np.abs(V - ref.V).max() < 1e-11
