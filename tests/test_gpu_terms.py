"""GPU parity of single terms and of the step's bookkeeping against the
oracle: each membrane term alone (Eqs. 13-19), the FP64 diagnostics, and
the wall reflection of reading C20 in one teacher-forced step."""
import numpy as np
import pytest

from gpu_helpers import TOL_MEM, compare_forces, gpu_system, near_cutoff
from oracle import Oracle, TERM
from paper_1611_06163_amd import inputs as I
from paper_1611_06163_amd import tdpd

pytestmark = pytest.mark.gpu

MEMBRANE_TERMS = {
    "bond": TERM["bond"],            # Eqs. (13)-(14)
    "viscous": TERM["bvisc"],        # Eq. (15)
    "random": TERM["brand"],         # Eq. (16)
    "area": TERM["area"],            # Eq. (17)
    "volume": TERM["vol"],           # Eq. (18)
    "bending": TERM["bend"],         # Eq. (19)
}


@pytest.mark.parametrize("name", list(MEMBRANE_TERMS))
def test_membrane_term_alone(name):
    """One membrane term at a time on the single-cell box (vertex forces
    only, every other term off on both sides), teacher-forced at a state
    20 steps into a run: each vertex within TOL_MEM (about 50 FP32 ulps) of
    that term's magnitude sum."""
    cfg = I.c2()
    run = gpu_system(cfg)
    run.step(20)
    run.sync()
    pos, vel, conc = run.get_state()
    run.close()
    terms = MEMBRANE_TERMS[name]
    cfg.pos, cfg.vel, cfg.conc = pos, vel, conc
    sysg = gpu_system(cfg, terms=terms)
    k = 21
    sysg.compute_forces(k)
    F, Q = sysg.get_forces()
    o = Oracle(cfg, terms=terms)
    ref = o.forces(pos, vel, conc, k=k)
    assert ref["err"] == 0
    g0, nv = cfg.rbc_first_gid[0], cfg.mesh_xyz.shape[0]
    which = np.zeros(cfg.n, np.uint8)
    which[g0:g0 + nv] = 1
    rep = compare_forces(F, Q, ref, which=which, label=f"membrane {name}")
    assert rep["badF"] == 0
    fm = ref["Fmabs"][g0:g0 + nv]
    print(f"{name}: median bound {np.median(TOL_MEM * fm):.3e}, median |F| "
          f"{np.median(np.linalg.norm(ref['F'][g0:g0 + nv], axis=1)):.3e}", flush=True)
    # solvent particles feel none of it
    assert np.all(F[:g0] == 0)


@pytest.mark.parametrize("name", ["c1", "c3_small", "c2"])
def test_diagnostics_match_oracle(name):
    """tdpd_diagnostics (FP64 sums over the FP32 state: momentum of mobile
    particles, kT, total concentration per species) equals the oracle's
    orc_diag on the same state up to FP64 summation order."""
    cfg = {"c1": I.c1(), "c2": I.c2(), "c3_small": I.c3(scale=0.25, n_cells=2)}[name]
    sysg = gpu_system(cfg)
    sysg.step(5)
    sysg.sync()
    pos, vel, conc = sysg.get_state()
    d = sysg.diagnostics()
    ref = Oracle(cfg).diag(vel, conc)
    mob = (cfg.flags & I.FLAG_FROZEN) == 0
    vabs = np.abs(vel[mob].astype(np.float64)).sum()
    print(name, "P", d["P"], ref["P"], "kT", d["kT"], ref["kT"], "C", d["C"], ref["C"], flush=True)
    assert np.abs(d["P"] - ref["P"]).max() <= 1e-12 * vabs
    assert abs(d["kT"] - ref["kT"]) <= 1e-12 * ref["kT"]
    assert np.allclose(d["C"], ref["C"], rtol=1e-12, atol=0)


def test_wall_reflection_matches_oracle():
    """One teacher-forced step of the channel with frozen walls (reading
    C20): from the GPU's state and forces, the oracle's kick, drift,
    reflection and wrap give the GPU's positions to FP32 rounding, and the
    particles it reflects are those the GPU reflects, with the half-step
    velocity reversed."""
    cfg = I.c3(scale=0.25, n_cells=2)
    sysg = gpu_system(cfg)
    sysg.step(30)
    sysg.sync()
    x0, v0, c0 = sysg.get_state()
    F0, Q0 = sysg.get_forces()
    sysg.step(1)
    sysg.sync()
    x1, v1, c1 = sysg.get_state()
    F1, Q1 = sysg.get_forces()
    k = sysg.step_counter
    o = Oracle(cfg)
    st = dict(pos=x0.astype(np.float64), vel=v0.astype(np.float64), conc=c0.astype(np.float64),
              F=F0.astype(np.float64), Q=Q0.astype(np.float64))
    assert o.step(st, k) == 0
    L = np.asarray(cfg.box)
    dx = x1 - st["pos"]
    dx -= L * np.round(dx / L)
    assert np.abs(dx).max() < 2e-5, np.abs(dx).max()
    # which particles were reflected: the drift from x0 would leave the fluid slab
    h = 0.5 * cfg.dt
    mob = (cfg.flags & I.FLAG_FROZEN) == 0
    y = x0[:, 1].astype(np.float64) + cfg.dt * (v0[:, 1] + h * F0[:, 1])
    refl = mob & ((y < cfg.wall_w) | (y > L[1] - cfg.wall_w))
    print("reflected particles:", int(refl.sum()), flush=True)
    assert refl.sum() > 0
    # half-step velocities: GPU v1 - h F1, oracle vel - h F (its own F at the new state)
    vh_g = v1.astype(np.float64) - h * F1
    vh_o = st["vel"] - h * st["F"]
    vpre = v0.astype(np.float64) + h * F0
    assert np.abs(vh_g[refl] + vpre[refl]).max() < 1e-5
    assert np.abs(vh_o[refl] + vpre[refl]).max() < 1e-5
    ok = mob & ~refl
    assert np.abs(vh_g[ok] - vpre[ok]).max() < 1e-5
    # reflected particles stay inside the slab
    assert np.all((x1[mob, 1] >= cfg.wall_w) & (x1[mob, 1] <= L[1] - cfg.wall_w))
    # frozen particles do not move and keep their concentrations
    fz = ~mob
    assert np.array_equal(x1[fz], x0[fz]) and np.array_equal(c1[fz], c0[fz])
