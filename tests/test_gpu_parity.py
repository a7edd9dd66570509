"""GPU parity tests: the HIP library, called through its C ABI, against the
FP64 CPU oracle on the same seeded inputs.

Pair sets must agree bit for bit.  Forces and concentration rates must agree
per particle within 1e-5 of the particle's sum of term magnitudes (the scale
of FP32 summation error), except particles whose force is ill-conditioned in
FP32: a pair so close to r_c that the weight (1 - r/r_c)^(s/2) turns the
rounding of r into more than a third of the tolerance (gpu_helpers); those
are counted, reported and bounded.
"""
import numpy as np
import pytest

from gpu_helpers import compare_forces, flux_sensitivity, gpu_system, near_cutoff
from oracle import Oracle
from paper_1611_06163_amd import inputs as I
from paper_1611_06163_amd import tdpd

pytestmark = pytest.mark.gpu


def _sorted_pairs(p):
    p = np.asarray(p)
    if p.size == 0:
        return p.reshape(0, 2)
    p = np.sort(p, axis=1)
    return p[np.lexsort((p[:, 1], p[:, 0]))]


def _cluster_cfg():
    """300 particles packed into a 1.2^3 corner of a 6^3 box: one cell holds
    more than 64 particles and its stencil more than 256 candidates."""
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), n=500, seed=13)
    rng = np.random.default_rng(14)
    cfg.pos[:300] = (5.5 + rng.random((300, 3)) * 1.2).astype(np.float32) % np.float32(6.0)
    cfg.pos[300] = cfg.pos[301]  # a coincident pair
    return cfg


def _cases():
    c1 = I.c1()
    tiny = I.make_fluid(box=(4.8, 5.0, 6.3), n=300, seed=3)
    return {"c1": c1, "tiny": tiny, "cluster": _cluster_cfg()}


@pytest.mark.parametrize("name", ["c1", "tiny", "cluster"])
@pytest.mark.parametrize("which", [0, 1])
def test_pair_sets_bit_exact(name, which):
    cfg = _cases()[name]
    sysg = gpu_system(cfg)
    sysg.compute_forces(0)
    got = _sorted_pairs(sysg.pairs(which))
    pos, _, _ = sysg.get_state()
    o = Oracle(cfg)
    ref, _ = o.pairs(pos, which, brute=cfg.n <= 2000)
    print(name, which, len(got), len(ref), flush=True)
    assert np.array_equal(got, _sorted_pairs(ref))


# (waves, chunks, workgroups per cell) of every built tile shape
_SHAPES = [(4, 2, 1), (4, 1, 1), (4, 3, 1), (2, 2, 1), (2, 3, 1), (2, 4, 1), (4, 2, 2), (4, 1, 2),
           (2, 2, 2), (2, 3, 2), (2, 4, 2), (2, 2, 4), (2, 3, 4), (4, 1, 4), (4, 2, 4)]


def _ordered_sorted(p):
    p = np.asarray(p).reshape(-1, 2)
    return p[np.lexsort((p[:, 1], p[:, 0]))]


@pytest.mark.parametrize("filt", [0, 1])
@pytest.mark.parametrize("name", ["c1", "tiny", "cluster", "dense", "walls", "sheared"])
def test_tiled_candidate_path_pair_sets_bit_exact(name, filt):
    """The default tiled kernel's own candidate path (stencil, filter on and
    off, periodic and sheared lifts, the FP32 distance test) lists, for every
    mobile home, exactly the partners of the brute-force (or pinned
    cell-bucket) pair set, at every built tile shape (Section 3.1)."""
    k = 0
    if name == "dense":  # stencils beyond the filter's list: the whole stencil is tested
        cfg = I.make_fluid(box=(6.0, 6.0, 6.0), n=1000, seed=17)
    elif name == "walls":  # frozen wall slabs: frozen homes are skipped
        cfg = I.c3(scale=0.25)
    elif name == "sheared":
        cfg = I.make_fluid(box=(8.0, 7.0, 6.5), rho=4.0, seed=3, shear_rate=0.4)
        k = 37
    else:
        cfg = _cases()[name]
    sysg = gpu_system(cfg, kernel=1)
    sysg.compute_forces(k)
    pos, _, _ = sysg.get_state()
    o = Oracle(cfg)
    mobile = (cfg.flags & I.FLAG_FROZEN) == 0
    refs = {}
    for which in (0, 1):
        ref, _ = o.pairs(pos, which, brute=cfg.n <= 2000, k=k)
        both = np.concatenate([ref, ref[:, ::-1]])
        refs[which] = _ordered_sorted(both[mobile[both[:, 0]]])
    for (wv, ch, sp) in _SHAPES:
        sysg.tile = (wv, ch, sp, filt)
        for which in (0, 1):
            got = _ordered_sorted(sysg.pairs(2 + which))
            print(name, (wv, ch, sp, filt), which, len(got), len(refs[which]), flush=True)
            assert np.array_equal(got, refs[which])
    sysg.close()


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("name", ["c1", "cluster", "c1_randflux", "c2", "c2_randflux",
                                  "three_randflux", "c3_small", "c3_cells"])
def test_teacher_forced_forces(kernel, name):
    """Forces and fluxes of one evaluation against the oracle at the GPU's
    own state; with the random flux of Eqs. (9)-(10) (m_s > 0) the tiled
    kernel runs its queued-flux build: one, two (with a cell body, whose
    vertex pairs exchange flux but no pair force) and three species (the
    third from the second Philox stream's other word pair)."""
    if name == "c1":
        cfg = I.c1()
    elif name == "cluster":
        cfg = _cluster_cfg()
    elif name == "c1_randflux":
        cfg = I.c1()
        cfg.m_s = 0.05
    elif name == "c2_randflux":
        cfg = I.c2()
        cfg.m_s = 0.05
    elif name == "three_randflux":
        cfg = I.make_fluid(box=(8.0, 8.0, 8.0), rho=3.0, n_species=3, seed=29)
        cfg.m_s = 0.08
    elif name == "c2":
        cfg = I.c2()
    elif name == "c3_cells":  # twenty cells
        cfg = I.c3(scale=0.25, n_cells=20)
    else:
        cfg = I.c3(scale=0.25, n_cells=2)
    sysg = gpu_system(cfg, kernel=kernel)
    k = 7
    sysg.compute_forces(k)
    F, Q = sysg.get_forces()
    pos, vel, conc = sysg.get_state()
    o = Oracle(cfg)
    ref = o.forces(pos, vel, conc, k=k)
    assert ref["err"] == 0
    excl, sens = near_cutoff(o, cfg, pos, vel, ref, k)
    rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, label=f"{name}/k{kernel}")
    assert rep["badF"] == 0 and rep["badQ"] == 0
    # a few percent of particles have a force pair close enough to r_c
    assert rep["excluded"] <= 5 + cfg.n // 20
    if cfg.mesh_xyz is not None and len(cfg.rbc_first_gid):
        d = sysg.diagnostics()
        # per-cell FP64 area/volume sums of FP32 triangle terms
        assert np.allclose(d["av"], ref["av"], rtol=2e-6, atol=0)
    if name == "cluster":
        assert sysg.coincident_pairs == 2 == ref["nzero"]


@pytest.mark.parametrize("name", ["c1", "c2", "c3_small"])
def test_ten_steps_teacher_forced(name):
    """Free-running GPU steps; after each, the oracle re-evaluates the forces
    at the GPU's own state (half-step velocity v - dt/2 F) with the same
    counter and checks the kick-drift update of positions."""
    cfg = {"c1": I.c1(), "c2": I.c2(), "c3_small": I.c3(scale=0.25, n_cells=2)}[name]
    sysg = gpu_system(cfg)
    o = Oracle(cfg)
    sysg.compute_forces(0)
    x0, v0, c0 = sysg.get_state()
    F0, Q0 = sysg.get_forces()
    frozen = (cfg.flags & I.FLAG_FROZEN) != 0
    h = 0.5 * cfg.dt
    L = np.asarray(cfg.box)
    for n in range(1, 11):
        sysg.step(1)
        sysg.sync()
        x, v, c = sysg.get_state()
        F, Q = sysg.get_forces()
        # drift: x_n = x_{n-1} + dt (v_{n-1} + dt/2 F_{n-1}), up to wall reflection
        pred = x0.astype(np.float64) + cfg.dt * (v0 + h * F0)
        dx = x.astype(np.float64) - pred
        dx -= L * np.round(dx / L)
        if cfg.wall_axis >= 0:
            w = cfg.wall_w
            y = pred[:, cfg.wall_axis] % L[cfg.wall_axis]
            refl = (y < w) | (y > L[cfg.wall_axis] - w)
            dx[refl] = 0.0
        dx[frozen] = 0.0
        assert np.abs(dx).max() < 2e-5, (n, np.abs(dx).max())
        vh = v.astype(np.float64) - h * F
        ch = c.astype(np.float64) - h * Q
        vh[frozen] = 0.0
        ch[frozen] = c[frozen]
        ref = o.forces(x, vh, ch, k=n)
        excl, sens = near_cutoff(o, cfg, x, vh, ref, n)
        rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, label=f"{name}/step{n}")
        assert rep["badF"] == 0 and rep["badQ"] == 0
        x0, v0, c0, F0, Q0 = x, v, c, F, Q


def test_free_running_trajectory_error_reported():
    cfg = I.c1()
    sysg = gpu_system(cfg)
    sysg.step(10)
    sysg.sync()
    x, v, c = sysg.get_state()
    o = Oracle(cfg)
    st = o.init_state()
    for n in range(1, 11):
        o.step(st, n)
    L = np.asarray(cfg.box)
    dx = x - st["pos"]
    dx -= L * np.round(dx / L)
    err = np.linalg.norm(dx, axis=1)
    ev = np.linalg.norm(v - st["vel"], axis=1)
    ec = np.abs(c - st["conc"]).max(axis=1)
    print("free-running 10 steps: |dx| max %.3e p99 %.3e, |dv| max %.3e p99 %.3e, "
          "|dC| max %.3e p99 %.3e" % (err.max(), np.quantile(err, 0.99), ev.max(),
                                     np.quantile(ev, 0.99), ec.max(), np.quantile(ec, 0.99)),
          flush=True)
    # FP32 trajectories separate from the FP64 ones only through rounding,
    # amplified where a pair sits at the force cutoff (a pair counted on one
    # side only moves its particles' velocities by up to dt/2 times the
    # cutoff noise force): bounds on the bulk (99th percentile) and the worst
    assert np.quantile(err, 0.99) < 1e-4
    assert err.max() < 1e-2
    assert np.quantile(ev, 0.99) < 1e-3
    assert ev.max() < 0.5
    assert np.quantile(ec, 0.99) < 1e-4
    assert ec.max() < 1e-2


def test_conservation_on_gpu():
    """Pair terms are exactly antisymmetric, so total momentum and total
    concentration change only by FP32 rounding of each particle's sum:
    per step at most about eps32 * sum_i sum_j |F_ij| * dt (and the same for
    C); the bound allows twice that, accumulated linearly."""
    cfg = I.c1()
    sysg = gpu_system(cfg)
    d0 = sysg.diagnostics()
    ref = Oracle(cfg).forces(cfg.pos, cfg.vel, cfg.conc, k=0)
    nsteps = 100
    eps = float(np.finfo(np.float32).eps)
    boundP = 2 * nsteps * cfg.dt * eps * ref["Fabs"].sum()
    boundC = 2 * nsteps * cfg.dt * eps * ref["Qabs"].sum() + 4 * eps * cfg.n
    sysg.step(nsteps)
    d1 = sysg.diagnostics()
    print("P0", d0["P"], "P100", d1["P"], "boundP", boundP, "C", d0["C"], d1["C"], "boundC",
          boundC, "kT", d1["kT"], flush=True)
    assert abs(d1["C"][0] - d0["C"][0]) < boundC
    assert np.abs(d1["P"] - d0["P"]).max() < boundP


def test_bitwise_deterministic():
    cfg = I.c2()
    outs = []
    for _ in range(2):
        s = gpu_system(cfg)
        s.step(20)
        outs.append(s.get_state() + s.get_forces())
        s.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["c2", "cluster"])
def test_binning_and_graph_modes_bitwise_equal(name):
    """The counting binning must reproduce the stable radix sort's order, and
    a captured graph must replay exactly the directly launched step."""
    cfg = I.c2() if name == "c2" else _cluster_cfg()
    outs = {}
    for mode in [dict(TDPD_BIN=1, TDPD_GRAPH=0), dict(TDPD_BIN=0, TDPD_GRAPH=0),
                 dict(TDPD_BIN=0, TDPD_GRAPH=1)]:
        s = gpu_system(cfg, env=mode)
        s.step(7)
        s.step(5)
        outs[str(mode)] = s.get_state() + s.get_forces()
        assert s.step_counter == 12
        s.close()
    ref = list(outs.values())[0]
    for key, val in outs.items():
        for a, b in zip(ref, val):
            assert np.array_equal(a, b), key


def test_empty_and_single_particle():
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), n=0)
    s = gpu_system(cfg)
    s.step(3)
    s.sync()
    assert s.get_state()[0].shape == (0, 3)
    cfg = I.make_fluid(box=(6.0, 6.0, 6.0), n=1)
    s = gpu_system(cfg)
    s.step(3)
    F, Q = s.get_forces()
    assert np.all(F == 0) and np.all(Q == 0)


def test_membrane_in_pair_kernel_equals_separate_kernel():
    """By default the membrane terms ride along in the binning scan's launch
    (K-Gather, bond forces) and the tiled pair kernel's (per-vertex terms);
    the separate membrane kernel on the second stream gives the same forces
    up to the order of the FP64 cell sums, and both runs step alike."""
    cfg = I.c3(scale=0.25, n_cells=20)
    out = []
    for fuse in ("1", "0"):
        s = gpu_system(cfg, kernel=1, env={"TDPD_FUSE_MEMBRANE": fuse})
        s.tile = (2, 2, 1, 0)
        s.compute_forces(5)
        F, Q = s.get_forces()
        d = s.diagnostics()
        s.step(3)
        x, _, _ = s.get_state()
        out.append((F, Q, d["av"], x))
        s.close()
    (F1, Q1, av1, x1), (F0, Q0, av0, x0) = out
    scale = np.abs(F0).max()
    assert np.abs(F1 - F0).max() <= 1e-5 * scale
    assert np.array_equal(Q1, Q0)
    assert np.allclose(av1, av0, rtol=1e-12, atol=0)
    assert np.abs(x1.astype(np.float64) - x0).max() < 1e-4


def test_full_size_sampled_c3():
    cfg = I.c3()
    rng = np.random.default_rng(0)
    which = np.zeros(cfg.n, np.uint8)
    which[rng.choice(cfg.n, 3000, replace=False)] = 1
    which[cfg.rbc_first_gid[0]:cfg.rbc_first_gid[0] + 500] = 1
    o = Oracle(cfg)
    for kernel in (1, 0):
        sysg = gpu_system(cfg, kernel=kernel)
        sysg.compute_forces(3)
        F, Q = sysg.get_forces()
        pos, vel, conc = sysg.get_state()
        ref = o.forces(pos, vel, conc, k=3, which=which)
        excl, sens = near_cutoff(o, cfg, pos, vel, ref, 3)
        rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, which=which, label=f"c3-full/k{kernel}")
        assert rep["badF"] == 0 and rep["badQ"] == 0
        sysg.close()


def test_full_size_sampled_c5():
    """The 1000-cell suspension at its full size (2,490,656 particles), in
    the launch configuration bench.py times (the tiled kernel at tile
    (2, 3, 1, 1), the membrane kernel on the second stream): forces and
    fluxes of 3000 sampled particles and of one cell's 500 vertices against
    the oracle, particle by particle (near-cutoff bounds from the sample's
    own pairs; the flux checked against the rounding bound of its weight
    near r_cc, flux_sensitivity, which at this size meets solvent particles
    whose species-1 flux is a few vertex pairs near the flux cutoff)."""
    cfg = I.c5()
    rng = np.random.default_rng(0)
    which = np.zeros(cfg.n, np.uint8)
    which[rng.choice(cfg.n, 3000, replace=False)] = 1
    which[cfg.rbc_first_gid[0]:cfg.rbc_first_gid[0] + 500] = 1
    print("c5 sampled: generated", flush=True)
    sysg = gpu_system(cfg, kernel=1)
    sysg.tile = (2, 3, 1, 1)
    sysg.compute_forces(3)
    F, Q = sysg.get_forces()
    pos, vel, conc = sysg.get_state()
    sysg.close()
    o = Oracle(cfg)
    ref = o.forces(pos, vel, conc, k=3, which=which)
    excl, sens = near_cutoff(o, cfg, pos, vel, ref, 3, which=which)
    sens_q = flux_sensitivity(cfg, pos, conc, which)
    rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, which=which, label="c5-full",
                         sens_q=sens_q)
    print(rep, flush=True)
    assert rep["n"] > 3000
    assert rep["badF"] == 0 and rep["badQ"] == 0


def test_checkpoint_resume_bitwise(tmp_path):
    """A run resumed from a checkpoint equals the uninterrupted run bit for
    bit (same cell order, step counter and centroids)."""
    cfg = I.small_suspension(seed=31, box=(14.0, 14.0, 14.0), n_cells=1)
    a = gpu_system(cfg)
    a.step(7)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    pairs7 = _sorted_pairs(a.pairs(1))
    a.step(8)
    ref = a.get_state() + a.get_forces()
    b = gpu_system(cfg)
    b.load(path)
    assert b.step_counter == 7
    # the cells of the last binning come back too: pairs listed right away
    assert np.array_equal(_sorted_pairs(b.pairs(1)), pairs7)
    b.step(8)
    got = b.get_state() + b.get_forces()
    for name, x, y in zip(("pos", "vel", "conc", "F", "Q"), got, ref):
        assert np.array_equal(x, y), name
    # a checkpoint of another system is refused
    with pytest.raises(tdpd.TdpdError):
        gpu_system(I.c1()).load(path)


@pytest.mark.parametrize("tile", [(4, 1, 1, 1), (4, 3, 1, 0), (2, 2, 1, 1), (2, 4, 1, 0),
                                  (4, 2, 2, 1), (2, 2, 4, 0), (2, 3, 1, 1), (4, 2, 1, 0)])
@pytest.mark.parametrize("name", ["cluster", "c2", "dense", "cluster_randflux", "c2_randflux"])
def test_tile_shapes_match_oracle(tile, name):
    """Every tile shape of the cell-tiled kernel, with and without the
    stencil filter, gives forces and fluxes within tolerance of the oracle
    (cluster: cells above 64 particles and stencils above 256 candidates;
    c2: one cell body in solvent; dense: stencils of 1000 candidates, beyond
    the filter's list, which then tests the whole stencil; *_randflux: the
    queued-flux build with the random flux, m_s = 0.05)."""
    if name.startswith("cluster"):
        cfg = _cluster_cfg()
    elif name == "dense":
        cfg = I.make_fluid(box=(6.0, 6.0, 6.0), n=1000, seed=17)
    else:
        cfg = I.c2()
    if name.endswith("randflux"):
        cfg.m_s = 0.05
    sysg = gpu_system(cfg, kernel=1)
    sysg.tile = tile
    assert sysg.tile == tile
    k = 3
    sysg.compute_forces(k)
    F, Q = sysg.get_forces()
    pos, vel, conc = sysg.get_state()
    o = Oracle(cfg)
    ref = o.forces(pos, vel, conc, k=k)
    excl, sens = near_cutoff(o, cfg, pos, vel, ref, k)
    rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, label=f"{name}/tile{tile}")
    assert rep["badF"] == 0 and rep["badQ"] == 0
    assert rep["excluded"] <= 5 + cfg.n // 20


def _ten_species(ns=10):
    cfg = I.make_fluid(box=(8.0, 8.0, 8.0), rho=3.0, n_species=ns, seed=23)
    for sp in range(ns):
        cfg.kappa[sp] *= 1.0 + 0.25 * sp
    return cfg


@pytest.mark.parametrize("ns", [10, 6])
@pytest.mark.parametrize("kernel,tile", [(0, None), (1, (4, 2, 1, 1)), (1, (4, 1, 2, 0)),
                                         (1, (2, 2, 1, 0)), (1, (4, 2, 4, 1))])
def test_ten_species_match_oracle(kernel, tile, ns):
    """Ten species (the 10-species build of the tiled kernel, two register
    chunks at most) and six (the 8-species build), both with the flux
    queued: forces and all fluxes against the oracle."""
    cfg = _ten_species(ns)
    sysg = gpu_system(cfg, kernel=kernel)
    if tile is not None:
        sysg.tile = tile
    k = 6
    sysg.compute_forces(k)
    F, Q = sysg.get_forces()
    assert Q.shape == (cfg.n, ns)
    pos, vel, conc = sysg.get_state()
    o = Oracle(cfg)
    ref = o.forces(pos, vel, conc, k=k)
    excl, sens = near_cutoff(o, cfg, pos, vel, ref, k)
    rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, label=f"{ns} species/k{kernel}/{tile}")
    assert rep["badF"] == 0 and rep["badQ"] == 0
    assert rep["excluded"] <= 5 + cfg.n // 20


@pytest.mark.parametrize("tile", [(4, 2, 1, 1), (2, 2, 2, 0)])
@pytest.mark.parametrize("ns", [3, 12, 16])
def test_species_builds_match_oracle(ns, tile):
    """The other species builds of the tiled kernel: three (the 4-species
    build, flux in place), twelve and sixteen (queued flux, partner
    concentrations from L2): forces and all fluxes against the oracle."""
    cfg = _ten_species(ns)
    sysg = gpu_system(cfg, kernel=1)
    sysg.tile = tile
    k = 4
    sysg.compute_forces(k)
    F, Q = sysg.get_forces()
    assert Q.shape == (cfg.n, ns)
    pos, vel, conc = sysg.get_state()
    o = Oracle(cfg)
    ref = o.forces(pos, vel, conc, k=k)
    excl, sens = near_cutoff(o, cfg, pos, vel, ref, k)
    rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, label=f"{ns} species/{tile}")
    assert rep["badF"] == 0 and rep["badQ"] == 0
    assert rep["excluded"] <= 5 + cfg.n // 20


def test_ten_species_refuses_three_chunk_shapes_and_tunes():
    sysg = gpu_system(_ten_species(), kernel=1)
    with pytest.raises(tdpd.TdpdError):
        sysg.tile = (4, 3, 1, 0)
    sysg.step(2)
    sysg.autotune(reps=2)
    assert sysg.tile[1] <= 2
    sysg.step(3)
    sysg.sync()


def test_autotune_picks_a_built_shape_and_caches(tmp_path):
    cfg = I.c2()
    a = gpu_system(cfg, kernel=1)
    a.step(3)
    path = str(tmp_path / "tiles.txt")
    ms = a.autotune(path, reps=3)
    assert ms > 0.0
    chosen = a.tile
    text = open(path).read()
    assert text.count("|") == 1 and text.strip().endswith(f"{ms:.6f}")
    # forces after tuning are those of the chosen shape at the same state
    F1, Q1 = a.get_forces()
    b = gpu_system(cfg, kernel=1)
    b.step(3)
    b.tile = chosen
    b.compute_forces(3)
    F2, Q2 = b.get_forces()
    assert np.array_equal(F1, F2) and np.array_equal(Q1, Q2)
    # a second system of the same workload takes the cached shape without timing
    c = gpu_system(cfg, kernel=1)
    c.autotune(path, reps=3)
    assert c.tile == chosen and open(path).read() == text
    with pytest.raises(tdpd.TdpdError):
        c.tile = (3, 3, 3, 1)
    with pytest.raises(tdpd.TdpdError):
        c.tile = (4, 2, 1, 2)
