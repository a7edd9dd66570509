"""Pins of the oracle's source term and Dirichlet boundaries (Eq. 7; the
transport validation of Section 4):

- Q^S (reading: a zero-order source a less a first-order decay k C per
  species and particle type) on a uniform system, where every flux vanishes:
  velocity Verlet for C (set-up evaluation at C_0) samples the forcing at
  the half-step values C_h(n) = C_(n-1) + dt/2 Q_(n-1), which therefore
  follow C_h(n+1) = C_h(n) + dt (a - k C_h(n)) from C_h(1) - a/k =
  (1 - k dt/2)(C_0 - a/k); so C_h(n) - a/k = (1 - k dt/2)(1 - k dt)^(n-1)
  (C_0 - a/k), and the full-step values C_n - a/k = (1 - k dt/2)^2
  (1 - k dt)^(n-1) (C_0 - a/k) tend to the exact exponential at first order
  in dt.  Frozen particles keep their concentration.
- Dirichlet walls: frozen wall particles hold C_D and exchange the Fickian
  flux of Eq. (8) with the fluid.  A fluid particle at distance d from a
  planar wall, the fluid at C = 0, receives in expectation over uniform
  placements kappa rho (C_D - 0) 2 pi int_d^rcc w_DC(r) r (r - d) dr (the
  weight integrated over the part of the cutoff sphere behind the wall).
- The cylindrical wall: a mobile particle that ends a drift at distance
  r > R from the axis is mirrored to 2R - r along its radius with its
  velocity reversed, so every mobile particle stays inside the tube.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import TERM, Oracle
from paper_1611_06163_amd import inputs as I


def _uniform_reacting(dt, seed=31):
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), rho=3.0, seed=seed, n_species=2)
    cfg.dt = dt
    cfg.conc[:, 0] = 0.1
    cfg.conc[:, 1] = 0.9
    # a few frozen particles: no Q at all, C held
    frozen = np.arange(0, cfg.n, 50)
    cfg.flags[frozen] = I.T_WALL | I.FLAG_FROZEN
    cfg.vel[frozen] = 0.0
    cfg.kappa[:, I.T_WALL, :] = 0.0   # no exchange with them, so the mobile
    cfg.kappa[:, :, I.T_WALL] = 0.0   # particles stay uniform
    cfg.source = np.zeros((2, 3))
    cfg.decay = np.zeros((2, 3))
    cfg.source[0, I.T_SOLVENT] = 0.7   # species 0: source and decay, c* = 0.35
    cfg.decay[0, I.T_SOLVENT] = 2.0
    cfg.decay[1, I.T_SOLVENT] = 0.5    # species 1: decay only, c* = 0
    return cfg, frozen


def _run(cfg, nsteps):
    o = Oracle(cfg, terms=TERM["fick"])
    st = o.init_state()
    for n in range(1, nsteps + 1):
        o.step(st, n)
    return st


def test_source_decay_follows_the_integrator_closed_form():
    dt, nsteps = 0.01, 200
    cfg, frozen = _uniform_reacting(dt)
    st = _run(cfg, nsteps)
    mobile = np.ones(cfg.n, bool)
    mobile[frozen] = False
    for sp, (a, k, c0) in enumerate([(0.7, 2.0, 0.1), (0.0, 0.5, 0.9)]):
        c0 = float(np.float32(c0))  # the state is handed over in FP32
        cs = a / k
        g = (1 - 0.5 * k * dt) * (1 - k * dt) ** (nsteps - 1)
        want = cs + (1 - 0.5 * k * dt) * g * (c0 - cs)
        got = st["conc"][mobile, sp]
        assert np.max(np.abs(got - want)) < 1e-12, (sp, got[:3], want)
        # Q at the end is the forcing at the last half-step value
        ch = cs + g * (c0 - cs)
        assert np.max(np.abs(st["Q"][mobile, sp] - (a - k * ch))) < 1e-12
        # frozen particles: C held, Q = 0
        assert np.all(st["conc"][frozen, sp] == c0)
        assert np.all(st["Q"][frozen, sp] == 0)


def test_source_decay_converges_to_the_exponential():
    """First order in dt: the deficit error is below k t * k dt and halves
    with dt."""
    t, errs = 2.0, []
    for dt in (0.02, 0.01):
        n = int(round(t / dt))
        cfg, frozen = _uniform_reacting(dt)
        st = _run(cfg, n)
        i = 1 if frozen[0] != 1 else 2
        k, c0 = 2.0, 0.1
        cs = 0.35
        exact = cs + math.exp(-k * t) * (c0 - cs)
        rel = abs(st["conc"][i, 0] - exact) / abs(exact - cs)
        assert rel < k * t * k * dt, (dt, rel)
        errs.append(rel)
    assert 1.7 < errs[0] / errs[1] < 2.3, errs


def _wall_weight(d, rcc, sc):
    """2 pi int_d^rcc w_DC(r) r (r - d) dr."""
    f = lambda r: (1 - r / rcc) ** sc * r * (r - d)
    return 2 * math.pi * integrate.quad(f, d, rcc, epsabs=1e-14)[0]


def test_dirichlet_wall_flux_in_expectation():
    """Fluid at C = 0 between two planar slabs of frozen particles held at
    C_D = 1 (kappa to the wall as in the fluid): the flux into each fluid
    particle against kappa rho C_D times the weight behind the wall, summed
    over the particles within the cutoff of a wall (8 placements), and in
    four bins of the distance."""
    kap, rho, w, ly = 1.0, 4.0, 2.0, 16.0
    got_tot = want_tot = 0.0
    bins = np.linspace(0.0, 1.58, 5)
    got_b = np.zeros(4)
    want_b = np.zeros(4)
    far_max = 0.0
    for seed in range(200, 208):
        cfg = I.make_fluid(box=(6.0, ly, 6.0), rho=rho, seed=seed)
        y = cfg.pos[:, 1].astype(np.float64)
        wall = (y < w) | (y > ly - w)
        cfg.flags[wall] = I.T_WALL | I.FLAG_FROZEN
        cfg.conc[:, 0] = np.where(wall, 1.0, 0.0).astype(np.float32)
        cfg.kappa[:] = kap
        cfg.wall_axis, cfg.wall_w = 1, w
        o = Oracle(cfg, terms=TERM["fick"])
        Q = o.forces(cfg.pos, cfg.vel, cfg.conc)["Q"][:, 0]
        d = np.minimum(y - w, ly - w - y)
        near = (~wall) & (d < cfg.rcc)
        far = (~wall) & (d >= cfg.rcc)
        far_max = max(far_max, float(np.max(np.abs(Q[far]))))
        want = np.array([kap * rho * _wall_weight(di, cfg.rcc, cfg.sc_exp) for di in d[near]])
        got_tot += Q[near].sum()
        want_tot += want.sum()
        idx = np.digitize(d[near], bins) - 1
        for b in range(4):
            got_b[b] += Q[near][idx == b].sum()
            want_b[b] += want[idx == b].sum()
        assert np.all(Q[wall] == 0)
    assert far_max == 0.0  # beyond the cutoff the walls do not reach
    assert abs(got_tot / want_tot - 1) < 0.03, (got_tot, want_tot)
    for b in range(3):  # the last bin holds little weight
        assert abs(got_b[b] / want_b[b] - 1) < 0.08, (b, got_b, want_b)


def test_cylinder_reflection_geometry():
    """Hand-set crossings of the cylinder: the particle is mirrored along its
    radius to 2R - r and its velocity reversed; one inside drifts freely."""
    R = 5.0
    cfg = I.cylinder(radius=R, length=6.0, rho=3.0, seed=4)
    c = 0.5 * cfg.box[1]
    mob = np.flatnonzero((cfg.flags & I.FLAG_FROZEN) == 0)
    i, j, m = int(mob[0]), int(mob[1]), int(mob[2])
    cfg.pos[i] = (1.0, c + 4.995, c)            # leaves along +y
    cfg.vel[i] = (0.0, 2.0, 0.0)
    cfg.pos[j] = (2.0, c - 3.0, c - 3.99)       # r = 4.990..., leaves along -z
    cfg.vel[j] = (0.5, 0.0, -2.0)
    cfg.pos[m] = (3.0, c, c + 1.0)              # stays inside
    cfg.vel[m] = (0.0, 1.0, 1.0)
    o = Oracle(cfg, terms=0)                    # no forces: v constant
    st = o.init_state()
    p0 = st["pos"].copy()
    v0 = st["vel"].copy()
    o.step(st, 1)
    for q in (i, j):
        p = p0[q] + cfg.dt * v0[q]
        dy, dz = p[1] - c, p[2] - c
        r = math.sqrt(dy * dy + dz * dz)
        assert r > R                            # the drift left the tube
        f = (2 * R - r) / r
        assert abs(st["pos"][q, 0] - p[0]) < 1e-12
        assert abs(st["pos"][q, 1] - (c + dy * f)) < 1e-12
        assert abs(st["pos"][q, 2] - (c + dz * f)) < 1e-12
        assert abs(math.hypot(st["pos"][q, 1] - c, st["pos"][q, 2] - c) - (2 * R - r)) < 1e-12
        assert np.array_equal(st["vel"][q], -v0[q])
    # i moved along +y only: y = c + 4.995 + 0.02 -> c + 5 - 0.015 (float32 input)
    assert abs(st["pos"][i, 1] - (c + 2 * R - (p0[i, 1] - c + 0.02))) < 1e-12
    assert abs(st["pos"][i, 2] - p0[i, 2]) < 1e-12
    np.testing.assert_allclose(st["pos"][m], p0[m] + cfg.dt * v0[m], atol=1e-12, rtol=0)
    assert np.array_equal(st["vel"][m], v0[m])


def test_cylinder_keeps_the_fluid_inside():
    cfg = I.cylinder(radius=5.0, length=6.0, rho=3.0, seed=5)
    o = Oracle(cfg)
    st = o.init_state()
    mob = (cfg.flags & I.FLAG_FROZEN) == 0
    c = 0.5 * cfg.box[1]
    speed0 = np.linalg.norm(st["vel"][mob], axis=1)
    for n in range(1, 41):
        o.step(st, n)
        r = np.hypot(st["pos"][mob, 1] - c, st["pos"][mob, 2] - c)
        assert np.all(r <= 5.0 + 1e-12)
    assert np.array_equal(st["pos"][~mob], cfg.pos[~mob].astype(np.float64))
    assert np.all(np.isfinite(speed0))
