"""Pins of the oracle's pair forces and fluxes (Section 2.1): momentum and
concentration conservation, Galilean invariance, axis-permutation symmetry,
and the physical sign of each term."""
import numpy as np

from oracle import Oracle, TERM, TERMS_ALL
from paper_1611_06163_amd import inputs as I


def _abs_sum(F):
    return np.abs(F).sum()


def test_total_force_and_flux_vanish_fluid():
    cfg = I.c1()
    cfg.m_s = 0.05  # exercise the random flux as well
    o = Oracle(cfg)
    r = o.forces(cfg.pos, cfg.vel, cfg.conc, k=5)
    assert r["err"] == 0
    F, Q = r["F"], r["Q"]
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * _abs_sum(F)
    assert np.abs(Q.sum(axis=0)).max() <= 1e-12 * np.abs(Q).sum()
    assert np.abs(Q).sum() > 0


def test_total_force_vanishes_with_membrane():
    cfg = I.small_suspension(n_cells=1, box=(12.0, 12.0, 12.0))
    o = Oracle(cfg)
    o.set_terms(TERMS_ALL & ~TERM["body"])
    r = o.forces(cfg.pos, cfg.vel, cfg.conc, k=3)
    F = r["F"]
    assert np.abs(F.sum(axis=0)).max() <= 1e-11 * _abs_sum(F)
    assert np.abs(r["Q"].sum(axis=0)).max() <= 1e-11 * np.abs(r["Q"]).sum()


def test_galilean_invariance():
    cfg = I.c1()
    o = Oracle(cfg)
    a = o.forces(cfg.pos, cfg.vel, cfg.conc, k=1)["F"]
    b = o.forces(cfg.pos, cfg.vel.astype(np.float64) + np.array([0.375, -1.25, 2.0]),
                 cfg.conc, k=1)["F"]
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()


def test_axis_permutation_symmetry():
    cfg = I.make_fluid(box=(7.0, 7.0, 7.0), rho=4.0, seed=9)
    o = Oracle(cfg)
    r1 = o.forces(cfg.pos, cfg.vel, cfg.conc, k=2)
    perm = [1, 2, 0]
    r2 = o.forces(cfg.pos[:, perm], cfg.vel[:, perm], cfg.conc, k=2)
    assert np.abs(r1["F"][:, perm] - r2["F"]).max() <= 1e-12 * np.abs(r1["F"]).max()
    assert np.abs(r1["Q"] - r2["Q"]).max() <= 1e-12 * np.abs(r1["Q"]).max()


def _two(x1, v1=(0, 0, 0), c=(0.0, 0.0)):
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), n=2, seed=0)
    cfg.pos = np.array([[3.0, 3.0, 3.0], x1], dtype=np.float32)
    cfg.vel = np.array([[0, 0, 0], v1], dtype=np.float32)
    cfg.conc = np.array([[c[0]], [c[1]]], dtype=np.float32)
    return cfg


def test_term_signs_two_particles():
    # conservative: repulsive, pushes particle 0 away from particle 1
    cfg = _two((3.6, 3.0, 3.0))
    o = Oracle(cfg, terms=TERM["cons"])
    F = o.forces(cfg.pos, cfg.vel, cfg.conc)["F"]
    assert F[0, 0] < 0 < F[1, 0] and abs(F[0, 1]) == 0
    # dissipative: opposes the relative velocity along the line of centres
    cfg = _two((3.6, 3.0, 3.0), v1=(-1.0, 0.0, 0.0))  # approaching
    o = Oracle(cfg, terms=TERM["diss"])
    F = o.forces(cfg.pos, cfg.vel, cfg.conc)["F"]
    assert F[1, 0] > 0 > F[0, 0]
    # transverse relative velocity gives no dissipative force
    cfg = _two((3.6, 3.0, 3.0), v1=(0.0, 1.0, 0.0))
    o = Oracle(cfg, terms=TERM["diss"])
    assert np.abs(o.forces(cfg.pos, cfg.vel, cfg.conc)["F"]).max() == 0
    # Fickian flux runs from high to low concentration
    cfg = _two((4.2, 3.0, 3.0), c=(1.0, 0.0))
    o = Oracle(cfg, terms=TERM["fick"])
    Q = o.forces(cfg.pos, cfg.vel, cfg.conc)["Q"]
    assert Q[0, 0] < 0 < Q[1, 0] and Q[0, 0] == -Q[1, 0]
    # beyond r_cc: nothing
    cfg = _two((4.6, 3.0, 3.0), c=(1.0, 0.0))
    o = Oracle(cfg, terms=TERMS_ALL & ~TERM["body"])
    r = o.forces(cfg.pos, cfg.vel, cfg.conc)
    assert np.abs(r["F"]).max() == 0 and np.abs(r["Q"]).max() == 0


def test_random_force_antisymmetric_and_scaled():
    # the random pair force on 0 and 1 is equal and opposite, and over many
    # steps its variance along e_ij is sigma^2 w_R^2 / dt (Eq. 5)
    cfg = _two((3.5, 3.0, 3.0))
    o = Oracle(cfg, terms=TERM["rand"])
    xs = []
    for k in range(4000):
        F = o.forces(cfg.pos, cfg.vel, cfg.conc, k=k)["F"]
        assert F[0, 0] == -F[1, 0]
        xs.append(F[1, 0])
    xs = np.array(xs)
    w = 1.0 - 0.5 / cfg.rc
    expect = cfg.sigma[0, 0] ** 2 * w ** cfg.s_exp / cfg.dt
    assert abs(xs.var() / expect - 1.0) < 0.1
    assert abs(xs.mean()) < 5 * np.sqrt(expect / xs.size)


def _many_species(n_species, seed=21):
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), rho=3.0, n_species=n_species, seed=seed)
    for sp in range(n_species):
        cfg.kappa[sp] *= 1.0 + 0.25 * sp
    return cfg


def test_many_species_independent_linear_and_conserved():
    """Ten species (the paper's many-species regime, Eqs. 7-10): a species'
    flux depends only on its own concentrations and kappa, so the first two
    equal a two-species run on the same particles; with equal concentrations
    the fluxes scale with kappa; every species' total vanishes; the forces
    do not depend on the species count."""
    c10 = _many_species(10)
    c2 = _many_species(2)
    c2.pos, c2.vel, c2.conc = c10.pos.copy(), c10.vel.copy(), c10.conc[:, :2].copy()
    r10 = Oracle(c10).forces(c10.pos, c10.vel, c10.conc, k=4)
    r2 = Oracle(c2).forces(c2.pos, c2.vel, c2.conc, k=4)
    assert r10["err"] == 0 and r2["err"] == 0
    assert np.array_equal(r10["F"], r2["F"])
    scale = np.abs(r2["Q"]).max()
    assert np.abs(r10["Q"][:, :2] - r2["Q"]).max() <= 1e-13 * scale
    assert np.abs(r10["Q"].sum(axis=0)).max() <= 1e-12 * np.abs(r10["Q"]).sum()
    # the same concentrations in every species: Q_s = (1 + s/4) Q_0
    conc = np.repeat(c10.conc[:, :1], 10, axis=1)
    q = Oracle(c10).forces(c10.pos, c10.vel, conc, k=4)["Q"]
    for sp in range(10):
        assert np.allclose(q[:, sp], (1.0 + 0.25 * sp) * q[:, 0], rtol=1e-12, atol=1e-14 * scale)
