"""Pins of the oracle's pair enumeration: the cell-bucket search against the
O(N^2) scan on tiny periodic boxes (bit-exact sets), and hand-checked cases
at the cutoff, across the periodic boundary and for coincident particles."""
import numpy as np
import pytest

from oracle import Oracle
from paper_1611_06163_amd import inputs as I


def _sorted(p):
    p = np.asarray(p)
    if p.size == 0:
        return p.reshape(0, 2)
    return p[np.lexsort((p[:, 1], p[:, 0]))]


def _tiny(box, n, seed, rc=1.0, rcc=1.58):
    cfg = I.make_fluid(box=box, n=n, seed=seed)
    cfg.rc, cfg.rcc = rc, rcc
    return cfg


@pytest.mark.parametrize("box,n,seed", [((4.8, 4.8, 4.8), 300, 1), ((5.0, 6.3, 4.9), 500, 2),
                                        ((6.0, 6.0, 6.0), 50, 3), ((7.3, 4.8, 9.1), 400, 4)])
@pytest.mark.parametrize("which", [0, 1])
def test_cells_equal_bruteforce(box, n, seed, which):
    cfg = _tiny(box, n, seed)
    o = Oracle(cfg)
    a, _ = o.pairs(cfg.pos, which)
    b, _ = o.pairs(cfg.pos, which, brute=True)
    assert np.array_equal(_sorted(a), _sorted(b))


def test_adversarial_positions_bruteforce_equal():
    rng = np.random.default_rng(11)
    L = np.float32(6.4)
    h = np.float32(L / 4)
    pts = []
    for a in range(3):  # on cell faces and box faces
        for v in (0.0, float(h), float(2 * h), float(np.nextafter(L, 0)),
                  float(np.nextafter(h, 0))):
            p = rng.random(3).astype(np.float32) * L
            p[a] = v
            pts.append(p)
    base = np.float32([3.0, 3.0, 3.0])
    for r in (1.0, 1.58):
        for dr in (np.nextafter(np.float32(r), 0), np.float32(r), np.nextafter(np.float32(r), 2)):
            pts.append(base)
            pts.append(base + np.float32([dr, 0, 0]))
    pts.append(np.float32([2.0, 2.0, 2.0]))
    pts.append(np.float32([2.0, 2.0, 2.0]))  # coincident pair
    pts = np.array(pts, dtype=np.float32)
    pts = np.concatenate([pts, rng.random((200, 3)).astype(np.float32) * L])
    cfg = _tiny((6.4, 6.4, 6.4), pts.shape[0], 0)
    cfg.pos = pts
    o = Oracle(cfg)
    for which in (0, 1):
        a, za = o.pairs(pts, which)
        b, zb = o.pairs(pts, which, brute=True)
        assert np.array_equal(_sorted(a), _sorted(b))
        assert za == zb >= 2


def test_hand_checked_cutoff_and_wrap():
    L = 8.0
    one_minus = float(np.nextafter(np.float32(1.0), 0))
    pts = np.array([
        [1.0, 1.0, 0.0],            # 0
        [1.5, 1.0, 0.0],            # 1: d = 0.5 from 0 -> pair
        [1.0, 2.0, 0.0],            # 2: d = 1.0 exactly from 0 -> not a pair (strict)
        [1.0, 1.0, one_minus],      # 3: d = 1 - ulp from 0 -> pair
        [7.8, 1.0, 0.0],            # 4: 1.2 from 0 through the x boundary -> no pair
        [0.3, 5.0, 5.0],            # 5
        [7.9, 5.0, 5.0],            # 6: across boundary from 5, d = 0.4 -> pair
    ], dtype=np.float32)
    cfg = _tiny((L, L, L), pts.shape[0], 0)
    cfg.pos = pts
    o = Oracle(cfg)
    a, _ = o.pairs(pts, 0, brute=True)
    got = {tuple(x) for x in _sorted(a).tolist()}
    # (1,3): |(0.5, 0, 1-ulp)| > 1, absent; (0,4): 1.2 through the boundary
    assert got == {(0, 1), (0, 3), (5, 6)}


def test_displacement_antisymmetric_across_boundaries():
    """The FP32 displacement rule lifts the coordinate nearer 0 of a pair
    across the periodic boundary, so both orientations round the same value:
    d_ji = -d_ij and d2_ji = d2_ij bit for bit."""
    rng = np.random.default_rng(5)
    L = np.float32(17.3)
    cfg = _tiny((float(L), float(L), float(L)), 2, 0)
    o = Oracle(cfg)
    n_wrapped = 0
    for _ in range(4000):
        a = (rng.random(3) * L).astype(np.float32)
        b = (a + rng.normal(scale=1.0, size=3)).astype(np.float32)
        b = np.where(b < 0, b + L, np.where(b >= L, b - L, b)).astype(np.float32)
        b[b >= L] = 0
        dab, qab = o.disp(a, b)
        dba, qba = o.disp(b, a)
        assert np.array_equal(dab, -dba) and qab == qba
        n_wrapped += int(np.any(np.abs(b - a) > L / 2))
    assert n_wrapped > 200
