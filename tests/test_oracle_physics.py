"""Pins of the oracle's time integration against what the method fixes:
Fickian decay of a concentration mode at the rate that Eq. (8) gives in
expectation over uniformly placed particles (long-wave limit Eq. 12), recovery
of kT from the force fluctuation-dissipation pair (Eq. 6), energy conservation
of the conservative dynamics, momentum bookkeeping with a body force, and the
wall reflection."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import Oracle, TERM, TERMS_ALL
from paper_1611_06163_amd import inputs as I


def fickian_rate(kappa, rho, rcc, sc, k):
    """Decay rate of C = A sin(k x) under Eq. (8) with uniform particles:
    kappa rho 4 pi int_0^rcc r^2 w_DC(r) (1 - sin(kr)/(kr)) dr."""
    f = lambda r: r * r * (1 - r / rcc) ** sc * (1 - math.sin(k * r) / (k * r))
    return kappa * rho * 4 * math.pi * integrate.quad(f, 1e-12, rcc, epsabs=1e-14)[0]


def test_fickian_rate_formula_long_wave_limit():
    # D^F k^2 with D^F from Eq. (12) at g = 1 is the k -> 0 limit
    kap, rho, rcc, sc = 1.0, 4.0, 1.58, 2.0
    DF = 2 * math.pi * kap * rho / 3 * rcc ** 5 * math.gamma(5) * math.gamma(sc + 1) / math.gamma(sc + 6)
    assert abs(DF - 2 * math.pi * kap * rho * rcc ** 5 / 315) < 1e-12
    for k in (1e-2, 3e-2):
        assert abs(fickian_rate(kap, rho, rcc, sc, k) / (DF * k * k) - 1) < 1e-3


def _mode_setup(seed, sc, L=10.0):
    cfg = I.make_fluid(box=(L, L, L), rho=4.0, seed=seed)
    cfg.sc_exp = sc
    k = 2 * math.pi / L
    x = cfg.pos[:, 0].astype(np.float64)
    s = np.sin(k * x)
    cfg.conc = (0.5 + 0.3 * s).astype(np.float32)[:, None]
    cfg.vel[:] = 0
    return cfg, k, s


def _amp(c, s):
    return np.dot(c - c.mean(), s) / np.dot(s, s)


@pytest.mark.parametrize("sc", [2.0, 1.0])
def test_fickian_mode_decay(sc):
    """Rate of decay of C = 1/2 + A sin(kx): the expectation over uniform
    placements is the closed form; one placement scatters by about 3 %, so
    the initial rate is averaged over 16 placements (standard error ~0.8 %)."""
    rates = []
    for seed in range(100, 116):
        cfg, k, s = _mode_setup(seed, sc)
        o = Oracle(cfg, terms=TERM["fick"])
        Q = o.forces(cfg.pos, cfg.vel, cfg.conc)["Q"][:, 0]
        rates.append(-np.dot(Q, s) / np.dot(s, s) / _amp(cfg.conc[:, 0].astype(np.float64), s))
    lam_th = fickian_rate(1.0, 4.0, cfg.rcc, sc, k)
    assert abs(np.mean(rates) / lam_th - 1) < 0.025, (np.mean(rates), lam_th)


def test_fickian_integration_matches_rate():
    """Integrated over a few steps (particles at rest), the mode decays at the
    configuration's own instantaneous rate; positions and total C are kept."""
    cfg, k, s = _mode_setup(21, 2.0)
    o = Oracle(cfg, terms=TERM["fick"])
    st = o.init_state()
    a0 = _amp(st["conc"][:, 0], s)
    rate0 = -np.dot(st["Q"][:, 0], s) / np.dot(s, s) / a0
    nsteps = 3
    for n in range(1, nsteps + 1):
        o.step(st, n)
    lam = -math.log(_amp(st["conc"][:, 0], s) / a0) / (nsteps * cfg.dt)
    assert abs(lam / rate0 - 1) < 0.01, (lam, rate0)
    assert np.array_equal(st["pos"], cfg.pos.astype(np.float64))
    assert abs(st["conc"].sum() - cfg.conc.astype(np.float64).sum()) < 1e-10


@pytest.mark.parametrize("alpha", [25.0, 0.0])
def test_kT_recovery(alpha):
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), rho=4.0, seed=31)
    cfg.alpha[:] = alpha
    o = Oracle(cfg, terms=TERM["cons"] | TERM["diss"] | TERM["rand"])
    st = o.init_state()
    kts = []
    for n in range(1, 1301):
        o.step(st, n)
        if n > 300:
            kts.append(o.diag(st["vel"], st["conc"])["kT"])
    kt = float(np.mean(kts))
    assert abs(kt - 1.0) < 0.02, kt


def _pair_energy(o, cfg, pos):
    p, _ = o.pairs(pos.astype(np.float32), 0)
    d = pos[p[:, 1]] - pos[p[:, 0]]
    L = np.asarray(cfg.box)
    d -= L * np.round(d / L)
    r = np.linalg.norm(d, axis=1)
    return float(np.sum(cfg.alpha[0, 0] * cfg.rc / 2 * (1 - r / cfg.rc) ** 2))


def test_conservative_dynamics_conserve_energy():
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), rho=3.0, seed=41)
    cfg.dt = 0.005
    o = Oracle(cfg, terms=TERM["cons"])
    st = o.init_state()
    for n in range(1, 201):  # settle the random start
        o.step(st, n)
    e = []
    for n in range(201, 401):
        o.step(st, n)
        e.append(0.5 * np.sum(st["vel"] ** 2) + _pair_energy(o, cfg, st["pos"]))
    e = np.array(e)
    ke = 0.5 * np.sum(st["vel"] ** 2)
    assert (e.max() - e.min()) / ke < 2e-3


def test_body_force_momentum_bookkeeping():
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), rho=3.0, seed=51)
    cfg.body_force = (0.02, 0.0, -0.01)
    o = Oracle(cfg)
    st = o.init_state()
    p0 = o.diag(st["vel"], st["conc"])["P"]
    nsteps = 20
    for n in range(1, nsteps + 1):
        o.step(st, n)
    p1 = o.diag(st["vel"], st["conc"])["P"]
    expect = p0 + cfg.n * np.array(cfg.body_force) * cfg.dt * nsteps
    assert np.abs(p1 - expect).max() < 1e-9
    c0 = cfg.conc.astype(np.float64).sum()
    assert abs(st["conc"].sum() - c0) < 1e-10 * abs(c0)


def test_walls_reflect_and_frozen_stay_put():
    cfg = I.c3(scale=0.25, n_cells=0)
    cfg.steps = 0
    o = Oracle(cfg)
    st = o.init_state()
    frozen = (cfg.flags & I.FLAG_FROZEN) != 0
    mob0 = ~frozen
    # start every mobile particle inside the fluid slab
    assert np.all((cfg.pos[mob0, 1] >= cfg.wall_w) & (cfg.pos[mob0, 1] <= 32 - cfg.wall_w))
    for n in range(1, 31):
        o.step(st, n)
    y = st["pos"][mob0, 1]
    assert np.all((y >= cfg.wall_w) & (y <= 32 - cfg.wall_w))
    assert np.array_equal(st["pos"][frozen], cfg.pos[frozen].astype(np.float64))
    assert np.all(st["vel"][frozen] == 0)


def test_membrane_thermostat_recovers_kT():
    """An isolated cell with only its membrane terms: the bond viscosity
    (Eq. 15) and its random partner (Eq. 16, reading C13) form a thermostat,
    so the kinetic temperature of the vertices (centre-of-mass motion
    removed) relaxes to kT.  Checks the normalisation of the random bond
    force against the dissipative one."""
    MEM = TERM["bond"] | TERM["bvisc"] | TERM["brand"] | TERM["area"] | TERM["vol"] | TERM["bend"]
    cfg = I._suspension("isolated_cell", (20.0, 20.0, 20.0), 0.0, 1, 21, n_species=1,
                        permeability=(1.0,))
    assert cfg.n == cfg.mesh_xyz.shape[0]
    o = Oracle(cfg, terms=MEM)
    st = o.init_state()
    kts = []
    for k in range(1, 3001):
        o.step(st, k)
        if k > 600 and k % 10 == 0:
            kts.append(o.diag(st["vel"], st["conc"])["kT"])
    kt = float(np.mean(kts))
    print("membrane thermostat kT", kt, flush=True)
    assert abs(kt - cfg.kT) < 0.03 * cfg.kT
