"""GPU parity of Lees-Edwards sheared boxes (reading C21) against the oracle:
pair sets bit for bit, teacher-forced forces with both pair kernels, steps
with particles crossing the sheared boundary, a cell across the boundary,
and a sheared batch whose boxes follow their solo trajectories."""
import math

import numpy as np
import pytest

from gpu_helpers import compare_forces, gpu_system, near_cutoff
from oracle import Oracle
from paper_1611_06163_amd import inputs as I

pytestmark = pytest.mark.gpu


def _sheared(seed=3, n=None, box=(8.0, 7.0, 6.5), shear=0.4, rho=4.0):
    return I.make_fluid(box=box, rho=rho, n=n, seed=seed, shear_rate=shear)


def _delta(cfg, k):
    a = float(np.float32(cfg.shear_rate)) * float(np.float32(cfg.box[1]))
    b = k * float(np.float32(cfg.dt))
    return float(np.float32(math.fmod(a * b, float(np.float32(cfg.box[0]))))), float(np.float32(a))


def _sorted(p):
    p = np.sort(np.asarray(p), axis=1)
    return p[np.lexsort((p[:, 1], p[:, 0]))]


@pytest.mark.parametrize("k", [0, 37, 500])
@pytest.mark.parametrize("which", [0, 1])
def test_pair_sets_bit_exact(k, which):
    cfg = _sheared()
    g = gpu_system(cfg)
    g.compute_forces(k)
    pos, _, _ = g.get_state()
    ref, _ = Oracle(cfg).pairs(pos, which, k=k)
    got = g.pairs(which)
    print("k", k, "pairs", len(got), len(ref), flush=True)
    assert np.array_equal(_sorted(got), _sorted(ref))


@pytest.mark.parametrize("kernel", [0, 1])
def test_teacher_forced_forces(kernel):
    cfg = _sheared(seed=5)
    g = gpu_system(cfg, kernel=kernel)
    k = 41
    g.compute_forces(k)
    F, Q = g.get_forces()
    pos, vel, conc = g.get_state()
    o = Oracle(cfg)
    ref = o.forces(pos, vel, conc, k=k)
    excl, sens = near_cutoff(o, cfg, pos, vel, ref, k)
    rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, label=f"shear/k{kernel}")
    assert rep["badF"] == 0 and rep["badQ"] == 0
    assert rep["excluded"] <= 5 + cfg.n // 20


def test_steps_across_the_sheared_boundary():
    """Ten free GPU steps of a strongly sheared box; after each the oracle
    re-evaluates at the GPU's state, and the drift of every particle,
    including those that crossed y = 0 or y = L_y (x shifted by delta_n), is
    checked."""
    cfg = _sheared(seed=7, shear=0.5)
    g = gpu_system(cfg)
    o = Oracle(cfg)
    g.compute_forces(0)
    x0, v0, _ = g.get_state()
    F0, _ = g.get_forces()
    h = 0.5 * cfg.dt
    L = np.asarray(cfg.box)
    crossed = 0
    for n in range(1, 11):
        g.step(1)
        x, v, c = g.get_state()
        F, Q = g.get_forces()
        delta, u = _delta(cfg, n)
        pred = x0.astype(np.float64) + cfg.dt * (v0 + h * F0)
        up, down = pred[:, 1] >= L[1], pred[:, 1] < 0
        pred[up, 1] -= L[1]
        pred[up, 0] -= delta
        pred[down, 1] += L[1]
        pred[down, 0] += delta
        crossed += int(up.sum() + down.sum())
        dx = x.astype(np.float64) - pred
        dx -= L * np.round(dx / L)
        assert np.abs(dx).max() < 2e-5, (n, np.abs(dx).max())
        vh = v.astype(np.float64) - h * F
        ref = o.forces(x, vh, c.astype(np.float64) - h * Q, k=n)
        excl, sens = near_cutoff(o, cfg, x, vh, ref, n)
        rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, label=f"shear step {n}")
        assert rep["badF"] == 0 and rep["badQ"] == 0
        x0, v0, F0 = x, v, F
    assert crossed > 0


def test_cell_across_the_sheared_boundary():
    k = 20
    cfg = I.small_suspension(seed=51, box=(16.0, 16.0, 16.0), n_cells=1)
    cfg.shear_rate = 0.35
    delta, _ = _delta(cfg, k)
    L = np.asarray(cfg.box)
    nv = cfg.mesh_xyz.shape[0]
    g0 = cfg.rbc_first_gid[0]
    # move the cell so that it straddles y = 0, with the sheared image of
    # its lower part at this step counter
    verts = cfg.pos[g0:g0 + nv].astype(np.float64)
    c = verts.mean(axis=0)
    new = verts + np.array([0.0, L[1] + 0.5 - c[1], 0.0])  # centred at y = L_y + 0.5
    up = new[:, 1] >= L[1]
    new[up, 1] -= L[1]
    new[up, 0] -= delta
    new[:, 0] %= L[0]
    pos = cfg.pos.copy()
    pos[g0:g0 + nv] = new.astype(np.float32)
    # solvent overlapping the moved cell is harmless for the comparison
    cfg.pos = pos
    assert up.any() and (~up).any()
    g = gpu_system(cfg)
    g.compute_forces(k)
    F, Q = g.get_forces()
    p, v, cc = g.get_state()
    o = Oracle(cfg)
    ref = o.forces(p, v, cc, k=k)
    excl, sens = near_cutoff(o, cfg, p, v, ref, k)
    rep = compare_forces(F, Q, ref, exclude=excl, sens=sens, label="cell across the sheared boundary")
    assert rep["badF"] == 0 and rep["badQ"] == 0
    d = g.diagnostics()
    assert np.allclose(d["av"], ref["av"], rtol=2e-6, atol=0)


def test_sheared_batch_equals_solo_and_oracle():
    boxes = I.ensemble(n_boxes=5, seed=12, lo=2500, hi=9000, shear_max=0.5)
    assert all(b.shear_rate > 0 for b in boxes)
    bs = gpu_system(boxes)
    bs.step(8)
    pos, vel, conc = bs.get_state()
    F, Q = bs.get_forces()
    off = bs.box_offset
    for b, cfg in enumerate(boxes):
        solo = gpu_system(cfg)
        solo.step(8)
        sl = slice(off[b], off[b + 1])
        got = solo.get_state() + solo.get_forces()
        for name, a, r in zip(("pos", "vel", "conc", "F", "Q"), (pos, vel, conc, F, Q), got):
            assert np.array_equal(a[sl], r), (b, name)
        solo.close()
    bs.compute_forces(9)
    pos, vel, conc = bs.get_state()
    F, Q = bs.get_forces()
    for b, cfg in enumerate(boxes):
        sl = slice(off[b], off[b + 1])
        o = Oracle(cfg)
        ref = o.forces(pos[sl], vel[sl], conc[sl], k=9)
        excl, sens = near_cutoff(o, cfg, pos[sl], vel[sl], ref, 9)
        rep = compare_forces(F[sl], Q[sl], ref, exclude=excl, sens=sens, label=f"sheared box {b}")
        assert rep["badF"] == 0 and rep["badQ"] == 0
