"""Batched ensemble on the GPU: many independent periodic boxes of uneven
size in one system (one launch per phase).  A box in the batch must follow
the same trajectory as the box alone, bit for bit, and each box must match
the oracle of that box."""
import numpy as np
import pytest

from gpu_helpers import compare_forces, gpu_system, near_cutoff
from oracle import Oracle
from paper_1611_06163_amd import inputs as I

pytestmark = pytest.mark.gpu


def _boxes():
    """Five ensemble boxes of 2500-9000 particles plus a 14^3 box with one
    red cell, so that membrane work is batched too."""
    boxes = I.ensemble(n_boxes=5, seed=11, lo=2500, hi=9000, shear_max=0.0)
    c = I._suspension("batch_cell", (14.0, 14.0, 14.0), 3.0, 1, 1099, n_species=1,
                      permeability=(1.0,))
    c.box_id = len(boxes)
    return boxes + [c]


def test_batch_box_equals_solo_bitwise():
    boxes = _boxes()
    bs = gpu_system(boxes)
    bs.step(10)
    pos, vel, conc = bs.get_state()
    F, Q = bs.get_forces()
    off = bs.box_offset
    for b, cfg in enumerate(boxes):
        solo = gpu_system(cfg)
        solo.step(10)
        p1, v1, c1 = solo.get_state()
        F1, Q1 = solo.get_forces()
        sl = slice(off[b], off[b + 1])
        for name, a, r in [("pos", pos[sl], p1), ("vel", vel[sl], v1), ("conc", conc[sl], c1),
                           ("F", F[sl], F1), ("Q", Q[sl], Q1)]:
            assert np.array_equal(a, r), (b, name)
        solo.close()


def test_batch_forces_match_oracle_per_box():
    boxes = _boxes()
    bs = gpu_system(boxes)
    bs.compute_forces(5)
    pos, vel, conc = bs.get_state()
    F, Q = bs.get_forces()
    off = bs.box_offset
    for b, cfg in enumerate(boxes):
        sl = slice(off[b], off[b + 1])
        o = Oracle(cfg)
        ref = o.forces(pos[sl], vel[sl], conc[sl], k=5)
        excl, sens = near_cutoff(o, cfg, pos[sl], vel[sl], ref, 5)
        rep = compare_forces(F[sl], Q[sl], ref, exclude=excl, sens=sens, label=f"batch box {b}")
        assert rep["badF"] == 0 and rep["badQ"] == 0
        assert rep["excluded"] <= 5 + cfg.n // 20
