"""Seeded synthetic workloads: radial feeders and load profiles.

This module only *draws inputs*.  It holds none of the power-flow arithmetic
(no admittance matrix, no inversion, no iteration), so both the GPU path and
the CPU oracle can be fed from it without sharing any of the method's code.

Feeders follow the paper's experimental set-up (Sec. V-A): radial networks
grown as a k-ary tree with a random number of children between 1 and 5 per
node.  The paper's load scenarios come from a copula fitted to smart-meter
data that is not available; the seeded sinusoid-plus-noise profiles below stand
in for them with the same shapes (time x bus, scenario x time x bus).

Sign convention (Sec. II, Eq. (1)): the demand-node current enters the
admittance relation with a minus sign, so S > 0 is consumption and a PV
injection is a negative S.

Seeds: feeder 1, load 2, training set 3, PV 4 (numpy PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_FEEDER = 1
SEED_LOAD = 2
SEED_TRAIN = 3
SEED_PV = 4
SEED_ZIP = 5

MINUTES_PER_YEAR = 525_600
HOURS_PER_YEAR = 8_760


@dataclass
class Feeder:
    """A radial feeder: branch list plus per-bus base load.

    Bus 0 is the slack (substation) bus.  ``frm[k] -> to[k]`` is branch k with
    series impedance ``r[k] + j x[k]`` pu.  ``p_base``/``q_base`` are the base
    active/reactive loads of the PQ buses 1..n_bus-1 (index 0 of the arrays is
    bus 1), in pu.
    """

    n_bus: int
    frm: np.ndarray  # int32 [n_branch]
    to: np.ndarray  # int32 [n_branch]
    r: np.ndarray  # float64 [n_branch]
    x: np.ndarray  # float64 [n_branch]
    p_base: np.ndarray  # float64 [n_bus-1]
    q_base: np.ndarray  # float64 [n_bus-1]
    vs: complex = 1.0 + 0.0j

    @property
    def n_pq(self) -> int:
        return self.n_bus - 1

    @property
    def s_base(self) -> np.ndarray:
        return self.p_base + 1j * self.q_base


def make_feeder(n_bus: int, seed: int = SEED_FEEDER, load_scale: float = 1.0) -> Feeder:
    """Random radial feeder grown breadth-first as a k-ary tree, k ~ U{1..5}.

    Line impedance r ~ U(0.005, 0.02) pu, x = r * U(0.5, 2).  Base load
    P ~ U(0.005, 0.02) pu with a lagging power factor pf ~ U(0.9, 1.0), times
    ``load_scale``.
    """
    if n_bus < 2:
        raise ValueError("a feeder needs the slack bus and at least one PQ bus")
    rng = np.random.Generator(np.random.PCG64(seed))
    frm, to = [], []
    queue = [0]
    nxt = 1
    head = 0
    while nxt < n_bus:
        parent = queue[head]
        head += 1
        k = int(rng.integers(1, 6))
        for _ in range(k):
            if nxt >= n_bus:
                break
            frm.append(parent)
            to.append(nxt)
            queue.append(nxt)
            nxt += 1
    nb = len(frm)
    r = rng.uniform(0.005, 0.02, nb)
    x = r * rng.uniform(0.5, 2.0, nb)
    p = rng.uniform(0.005, 0.02, n_bus - 1) * load_scale
    pf = rng.uniform(0.9, 1.0, n_bus - 1)
    q = p * np.tan(np.arccos(pf))
    return Feeder(n_bus, np.asarray(frm, np.int32), np.asarray(to, np.int32),
                  r.astype(np.float64), x.astype(np.float64), p, q)


def make_star_feeder(z: np.ndarray, vs: complex = 1.0 + 0.0j) -> Feeder:
    """Star feeder: PQ bus i (1-based) hangs on its own line z[i-1] from the slack."""
    z = np.asarray(z, np.complex128)
    n = len(z)
    return Feeder(n + 1, np.zeros(n, np.int32), np.arange(1, n + 1, dtype=np.int32),
                  z.real.copy(), z.imag.copy(), np.zeros(n), np.zeros(n), vs)


def make_chain_feeder(z: np.ndarray, vs: complex = 1.0 + 0.0j) -> Feeder:
    """Chain (path) feeder 0-1-2-...-n with branch impedances z."""
    z = np.asarray(z, np.complex128)
    n = len(z)
    return Feeder(n + 1, np.arange(0, n, dtype=np.int32), np.arange(1, n + 1, dtype=np.int32),
                  z.real.copy(), z.imag.copy(), np.zeros(n), np.zeros(n), vs)


@dataclass
class Feeder3ph:
    """A three-phase radial feeder: the bus tree of :func:`make_feeder` with a 3x3 series
    impedance matrix per branch and per-phase base loads.  Demand node 3 k + p is phase p
    of PQ bus k + 1; ``s_base`` and ``n_pq`` count demand nodes, so the profile
    generators below apply unchanged."""

    n_bus: int
    frm: np.ndarray  # int32 [n_branch]
    to: np.ndarray  # int32 [n_branch]
    zabc: np.ndarray  # complex128 [n_branch, 3, 3]
    s_base: np.ndarray  # complex128 [3 (n_bus - 1)]
    vs_abc: np.ndarray  # complex128 [3]

    @property
    def n_pq(self) -> int:
        return 3 * (self.n_bus - 1)


def balanced_slack() -> np.ndarray:
    """Phase voltages 1, e^{-j 2 pi/3}, e^{+j 2 pi/3} (phase sequence a, b, c)."""
    return np.exp(-2j * math.pi / 3.0 * np.arange(3))


def make_feeder_3ph(n_bus: int, seed: int = SEED_FEEDER, load_scale: float = 1.0) -> Feeder3ph:
    """Three-phase version of :func:`make_feeder` (same tree and self impedances).

    Per branch the self impedance z = r + jx of each phase is scaled by U(0.9, 1.1), and
    every phase pair couples with a mutual impedance z U(0.3, 0.45) (a symmetric, not
    transposed, matrix).  Each phase of a bus carries a third of the single-phase base
    load times an imbalance factor U(0.6, 1.4).
    """
    f = make_feeder(n_bus, seed, load_scale)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    nb = len(f.frm)
    z = f.r + 1j * f.x
    zabc = np.zeros((nb, 3, 3), np.complex128)
    for p in range(3):
        zabc[:, p, p] = z * rng.uniform(0.9, 1.1, nb)
    for p, q in ((0, 1), (0, 2), (1, 2)):
        m = z * rng.uniform(0.3, 0.45, nb)
        zabc[:, p, q] = m
        zabc[:, q, p] = m
    imb = rng.uniform(0.6, 1.4, (n_bus - 1, 3))
    s_base = (f.s_base[:, None] / 3.0 * imb).reshape(-1)
    return Feeder3ph(n_bus, f.frm, f.to, zabc, s_base, balanced_slack())


# ----------------------------------------------------------------------------- profiles

def profile_daily96(feeder: Feeder, seed: int = SEED_LOAD, steps: int = 96) -> np.ndarray:
    """Daily 96-step profile: m = max(0, 0.6 + 0.4 sin(2 pi t/96 - pi/2) + N(0, 0.05^2)).

    Returns S as complex128 [steps, n_pq].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.arange(steps, dtype=np.float64)[:, None]
    m = 0.6 + 0.4 * np.sin(2.0 * math.pi * t / 96.0 - math.pi / 2.0)
    m = m + rng.normal(0.0, 0.05, (steps, feeder.n_pq))
    m = np.maximum(m, 0.0)
    return m * feeder.s_base[None, :]


def _phases(rng: np.random.Generator, n: int):
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    psi = rng.uniform(0.0, 2.0 * math.pi, n)
    return phi, psi


def profile_minute_year(feeder: Feeder, steps: int = MINUTES_PER_YEAR, seed: int = SEED_LOAD,
                        t0: int = 0, dtype=np.complex128, chunk: int = 65_536) -> np.ndarray:
    """Per-bus one-minute profile over ``steps`` minutes starting at minute ``t0``.

    m(t, b) = (0.6 + 0.25 sin(2 pi t/1440 + phi_b) + 0.15 sin(2 pi t/10080 + psi_b))
              * exp(N(0, 0.2^2)),   phi_b, psi_b ~ U(0, 2 pi).
    Returns S = m * (P_b + j Q_b) as [steps, n_pq] of ``dtype``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = feeder.n_pq
    phi, psi = _phases(rng, n)
    out = np.empty((steps, n), dtype=dtype)
    sb = feeder.s_base
    for a in range(0, steps, chunk):
        b = min(steps, a + chunk)
        t = (t0 + np.arange(a, b, dtype=np.float64))[:, None]
        m = 0.6 + 0.25 * np.sin(2.0 * math.pi * t / 1440.0 + phi) \
            + 0.15 * np.sin(2.0 * math.pi * t / 10080.0 + psi)
        m = m * np.exp(rng.normal(0.0, 0.2, (b - a, n)))
        out[a:b] = m * sb
    return out


@dataclass
class ScenarioLoads:
    """[scenario, hour, bus] loads kept factored: S[s,h,b] = c[s] * L[h,b] - PV[h,b].

    The full tensor of the 300-bus case is 21 GB in complex64, so it is built on
    the device from these small factors; any single element can be recomputed
    on the host with :meth:`element`.
    """

    c: np.ndarray  # float64 [P]   per-scenario load scale ~ N(1, 0.15) clipped at 0
    L: np.ndarray  # complex128 [T, n] per-bus hourly load
    PV: np.ndarray  # float64 [T, n] PV injection (unity power factor), >= 0

    def element(self, s: np.ndarray, h: np.ndarray, dtype=np.complex64) -> np.ndarray:
        """Rows S[s, h, :] for index arrays s, h, rounded through ``dtype`` exactly
        as :meth:`dense` rounds them."""
        L = self.L.astype(dtype)
        pv = self.PV.astype(np.float32 if dtype == np.complex64 else np.float64)
        c = self.c.astype(np.float32 if dtype == np.complex64 else np.float64)
        return (c[s][:, None] * L[h] - pv[h]).astype(dtype)

    def dense(self, dtype=np.complex64) -> np.ndarray:
        """The full [P, T, n] tensor on the host (small cases only)."""
        P = len(self.c)
        s = np.repeat(np.arange(P), self.L.shape[0])
        h = np.tile(np.arange(self.L.shape[0]), P)
        return self.element(s, h, dtype).reshape(P, self.L.shape[0], -1)


def scenario_loads(feeder: Feeder, n_scen: int = 1000, hours: int = HOURS_PER_YEAR,
                   seed: int = SEED_LOAD, seed_pv: int = SEED_PV,
                   pv_share: float = 0.3) -> ScenarioLoads:
    """Scenario x hourly-year loads with PV on a seeded 30 % of the buses.

    Scenario scale c_s ~ N(1, 0.15) clipped >= 0.  Hourly profile: the minute
    profile's form with 24 h and 168 h periods.  PV: U_b(0, 0.02) pu times the
    clear-sky bell max(0, sin(pi (h_day - 6)/12)) for 6 <= h_day <= 18, unity pf.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = feeder.n_pq
    phi, psi = _phases(rng, n)
    t = np.arange(hours, dtype=np.float64)[:, None]
    m = 0.6 + 0.25 * np.sin(2.0 * math.pi * t / 24.0 + phi) \
        + 0.15 * np.sin(2.0 * math.pi * t / 168.0 + psi)
    m = m * np.exp(rng.normal(0.0, 0.2, (hours, n)))
    L = m * feeder.s_base[None, :]
    c = np.maximum(rng.normal(1.0, 0.15, n_scen), 0.0)
    prng = np.random.Generator(np.random.PCG64(seed_pv))
    has_pv = np.zeros(n, bool)
    has_pv[prng.choice(n, int(round(pv_share * n)), replace=False)] = True
    cap = np.where(has_pv, prng.uniform(0.0, 0.02, n), 0.0)
    hday = (np.arange(hours) % 24).astype(np.float64)
    bell = np.where((hday >= 6) & (hday <= 18), np.maximum(0.0, np.sin(math.pi * (hday - 6.0) / 12.0)), 0.0)
    PV = bell[:, None] * cap[None, :]
    return ScenarioLoads(c, L, PV)


def zip_shares(n_pq: int, seed: int = SEED_ZIP, max_current: float = 0.6):
    """Seeded ZIP shares per PQ bus for Eq. (2)'s load model: constant-current share
    alpha_I ~ U(0, max_current), constant-power share alpha_P = 1 - alpha_I, no
    constant-impedance share."""
    ai = np.random.default_rng(seed).uniform(0.0, max_current, n_pq)
    return ai, 1.0 - ai


def zipz_shares(n_pq: int, seed: int = SEED_ZIP, max_impedance: float = 0.4, max_current: float = 0.4):
    """Seeded ZIP shares with a constant-impedance part: alpha_Z ~ U(0, max_impedance),
    alpha_I ~ U(0, max_current), alpha_P = 1 - alpha_Z - alpha_I per PQ bus."""
    rng = np.random.default_rng(seed + 1)
    az = rng.uniform(0.0, max_impedance, n_pq)
    ai = rng.uniform(0.0, max_current, n_pq)
    return az, ai, 1.0 - az - ai


def mlp_sizes(n_pq: int, hidden: int = 256, layers: int = 3):
    """Layer widths of the warm-start network: 2 n + 4 inputs, `layers` hidden layers, 2 n outputs."""
    return [2 * n_pq + 4] + [hidden] * layers + [2 * n_pq]


def mlp_init_params(sizes, seed: int = SEED_TRAIN) -> np.ndarray:
    """Seeded initial parameters, flat [W_1 (out x in), b_1, W_2, b_2, ...] in float32:
    W ~ N(0, 1/fan_in), b = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append(rng.normal(0.0, 1.0 / math.sqrt(a), (b, a)).ravel())
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)
