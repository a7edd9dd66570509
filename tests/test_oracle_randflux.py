"""Pins of the oracle's random concentration flux Q^R (Eqs. 9-10).

Eq. (10) ties the random flux amplitude to the Fickian coefficient,
eps_ij^2 = m_s^2 kappa_ij rho (C_i + C_j), with w_RC = w_DC^(1/2).  For one
isolated pair under the Fickian flux (Eq. 8) and Q^R alone, the total
C_i + C_j is conserved (zeta_ij = -zeta_ji) and the difference
D = C_i - C_j obeys

    dD = -2 kappa w_DC D dt + 2 eps w_RC dW,

an Ornstein-Uhlenbeck process.  Its stationary variance is
(2 eps w_RC)^2 / (2 * 2 kappa w_DC) = eps^2 / kappa = m_s^2 rho (C_i + C_j):
the pairing makes the size of the concentration fluctuations independent of
kappa and of the pair distance.  The velocity-Verlet update of C (half kicks
around each evaluation, reading C9) advances the half-step difference
D' = D + dt/2 Q_D exactly as the AR(1) recursion
D'_{n+1} = (1 - theta dt) D'_n + 2 eps w_RC sqrt(dt) zeta_n with
theta = 2 kappa w_DC, whose stationary variance is

    Var(D') = m_s^2 rho (C_i + C_j) / (1 - kappa w_DC dt).

A dropped rho, a missing square root in eps, a wrong exponent of w_RC or a
symmetric zeta each break this (by a constant factor, by a dependence on
C_i + C_j, on the distance, or by losing conservation)."""
import numpy as np
import pytest

from oracle import Oracle, TERM
from paper_1611_06163_amd import inputs as I

M_S = 0.2
KAPPA = 10.0


def _pairs_cfg(n_side=10, spacing=3.0, seed=31):
    """n_side^3 isolated pairs on a cubic lattice (spacing 3 > r_cc + the
    largest pair distance, so no flux crosses between pairs), separations in
    [0.3, 0.9] along random directions, concentrations C_i = C_j = c_p with
    c_p in [0.2, 2]."""
    rng = np.random.default_rng(seed)
    L = n_side * spacing
    npair = n_side ** 3
    g = np.stack(np.meshgrid(*[np.arange(n_side)] * 3, indexing="ij"), -1).reshape(-1, 3)
    base = (g + 0.5) * spacing
    r = rng.uniform(0.3, 0.9, npair)
    u = rng.normal(size=(npair, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    pos = np.empty((2 * npair, 3))
    pos[0::2] = base - 0.5 * r[:, None] * u
    pos[1::2] = base + 0.5 * r[:, None] * u
    cfg = I.make_fluid(box=(L, L, L), n=2 * npair, seed=seed, rho=3.0)
    cfg.pos = pos.astype(np.float32)
    cfg.vel[:] = 0.0
    cp = rng.uniform(0.2, 2.0, npair)
    cfg.conc = np.repeat(cp, 2)[:, None].astype(np.float32)
    cfg.m_s = M_S
    cfg.kappa[:] = KAPPA
    return cfg


def _wdc(cfg):
    p = cfg.pos.astype(np.float64)
    r = np.linalg.norm(p[1::2] - p[0::2], axis=1)
    return np.maximum(1.0 - r / cfg.rcc, 0.0) ** cfg.sc_exp, r


def test_random_flux_single_evaluation():
    """Per evaluation: Q^R_i = -Q^R_j exactly, zero mean, and variance
    eps^2 w_RC^2 / dt over step counters."""
    cfg = _pairs_cfg(n_side=4)
    o = Oracle(cfg, terms=TERM["frand"])
    c = cfg.conc[:, 0].astype(np.float64)
    wdc, _ = _wdc(cfg)
    eps2 = M_S ** 2 * KAPPA * cfg.rho * (c[0::2] + c[1::2])
    expect = eps2 * wdc / cfg.dt
    qs = []
    for k in range(400):
        Q = o.forces(cfg.pos, cfg.vel, cfg.conc, k=k)["Q"][:, 0]
        assert np.array_equal(Q[0::2], -Q[1::2])
        qs.append(Q[1::2])
    qs = np.array(qs)  # [k, pair]
    z = qs / np.sqrt(expect)  # unit normals if the amplitude is right
    assert abs(z.mean()) < 5.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 0.03


@pytest.mark.parametrize("seed", [31])
def test_random_flux_stationary_variance(seed):
    """Fickian + random flux on isolated pairs: the half-step concentration
    difference reaches the stationary variance m_s^2 rho (C_i + C_j) /
    (1 - kappa w_DC dt) (module docstring), for every pair distance and
    every pair total; the pair total is conserved."""
    cfg = _pairs_cfg(seed=seed)
    o = Oracle(cfg, terms=TERM["fick"] | TERM["frand"])
    st = o.init_state()
    tot0 = st["conc"][0::2, 0] + st["conc"][1::2, 0]
    wdc, r = _wdc(cfg)
    h = 0.5 * cfg.dt
    burn, nstep = 150, 2150
    dh = []
    for k in range(1, nstep + 1):
        # D' of step k is the difference after its first half kick
        c = st["conc"][:, 0] + h * st["Q"][:, 0]
        if k > burn:
            dh.append(c[0::2] - c[1::2])
        assert o.step(st, k) == 0
    tot = st["conc"][0::2, 0] + st["conc"][1::2, 0]
    assert np.abs(tot - tot0).max() <= 1e-12 * np.abs(tot0).max() * nstep
    assert np.abs(st["pos"] - cfg.pos.astype(np.float64)).max() == 0.0
    dh = np.array(dh)
    expect = M_S ** 2 * cfg.rho * tot0 / (1.0 - KAPPA * wdc * cfg.dt)
    ratio = (dh ** 2).mean(axis=0) / expect  # zero-mean process
    print("stationary variance ratio: mean", ratio.mean(), "per-pair sd", ratio.std())
    assert abs(ratio.mean() - 1.0) < 0.03
    # no residual dependence on the pair distance or on the pair total
    for key in (r, tot0):
        q = np.quantile(key, [0.0, 0.25, 0.5, 0.75, 1.0])
        for a, b in zip(q[:-1], q[1:]):
            sel = (key >= a) & (key <= b)
            assert abs(ratio[sel].mean() - 1.0) < 0.06, (a, b, ratio[sel].mean())
