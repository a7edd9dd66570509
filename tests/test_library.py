"""Host-side checks of the C-ABI library (no GPU needed): it loads, it
exports every entry point include/tdpd.h declares, and parameter validation
rejects bad inputs without touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1611_06163_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdpd.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tdpd_[a-z_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("tdpd_create", "tdpd_set_state", "tdpd_step", "tdpd_get_state",
              "tdpd_get_pairs", "tdpd_add_mesh", "tdpd_add_rbc", "tdpd_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1611_06163_amd import tdpd
    L = tdpd.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def _create(cfg, **over):
    from paper_1611_06163_amd import tdpd
    p = tdpd.params_from_config(cfg)
    for k, v in over.items():
        setattr(p, k, v)
    h = C.c_void_p()
    rc = tdpd.lib().tdpd_create(C.byref(p), None, tdpd.ALLOC_FN(), tdpd.FREE_FN(), None,
                                C.byref(h))
    return rc, h


def test_create_validates_parameters_on_host():
    from paper_1611_06163_amd import tdpd
    cfg = I.c1()
    rc, h = _create(cfg)
    assert rc == 0
    tdpd.lib().tdpd_destroy(h)
    assert _create(cfg, rc=0.0)[0] == -1
    assert _create(cfg, n_species=0)[0] == -1
    assert _create(cfg, n_types=9)[0] == -1
    p = tdpd.params_from_config(cfg)
    p.sigma[0] = 2.0  # breaks sigma^2 = 2 kT gamma (Eq. 6)
    h = C.c_void_p()
    assert tdpd.lib().tdpd_create(C.byref(p), None, tdpd.ALLOC_FN(), tdpd.FREE_FN(), None,
                                  C.byref(h)) == -1
    small = I.make_fluid(box=(4.0, 10.0, 10.0), n=10)
    assert _create(small)[0] == -2  # 4 / 1.58 < 3 cells


def test_set_state_and_mesh_validation_on_host():
    from paper_1611_06163_amd import tdpd
    L = tdpd.lib()
    cfg = I.c1()
    rc, h = _create(cfg)
    assert rc == 0
    n = 10
    pos = np.zeros((n, 3), np.float32)
    vel = np.zeros((n, 3), np.float32)
    conc = np.zeros((n, 1), np.float32)
    flags = np.zeros(n, np.uint32)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    bad = flags.copy()
    bad[3] = 7  # type index >= n_types
    assert L.tdpd_set_state(h, n, ptr(pos), ptr(vel), ptr(conc), ptr(bad)) == -1
    pos[2, 1] = np.nan
    assert L.tdpd_set_state(h, n, ptr(pos), ptr(vel), ptr(conc), ptr(flags)) == -5
    pos[2, 1] = 1.0
    assert L.tdpd_set_state(h, n, ptr(pos), ptr(vel), ptr(conc), ptr(flags)) == 0
    # an open surface is rejected
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float64)
    tri = np.array([[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]], np.int32)  # inconsistent
    mp = tdpd.tdpd_mesh_params(p=0.02, x0=0.45, m_pow=2, kb=1, theta0=0, kg=1, kl=1, kv=1,
                               gamma_t=1, gamma_c=1)
    mid = C.c_int32()
    assert L.tdpd_add_mesh(h, 4, ptr(xyz), 4, ptr(tri), C.byref(mp), C.byref(mid)) == -1
    xyz, tri = I.tetra_mesh()
    tri = np.ascontiguousarray(tri, np.int32)
    xyz = np.ascontiguousarray(xyz * 0.5, np.float64)
    assert L.tdpd_add_mesh(h, 4, ptr(xyz), 4, ptr(tri), C.byref(mp), C.byref(mid)) == 0
    rid = C.c_int32()
    assert L.tdpd_add_rbc(h, mid.value, 8, C.byref(rid)) == -1   # runs past n
    assert L.tdpd_add_rbc(h, mid.value, 2, C.byref(rid)) == 0
    assert L.tdpd_add_rbc(h, mid.value, 4, C.byref(rid)) == -1   # overlaps the first
    L.tdpd_destroy(h)


def test_set_verlet_validation_on_host():
    """Neighbour-list settings: checked and applied before any upload."""
    from paper_1611_06163_amd import tdpd
    L = tdpd.lib()
    L.tdpd_set_verlet.argtypes = [C.c_void_p, C.c_float, C.c_int32, C.c_int32]
    L.tdpd_get_verlet.argtypes = [C.c_void_p] + [C.c_void_p] * 3
    cfg = I.c1()  # 10^3 box, r_max = 1.58
    rc, h = _create(cfg)
    assert rc == 0
    assert L.tdpd_set_verlet(h, -0.1, 5, 0) == -1
    assert L.tdpd_set_verlet(h, float("nan"), 5, 0) == -1
    assert L.tdpd_set_verlet(h, 0.3, -1, 0) == -1
    assert L.tdpd_set_verlet(h, 0.3, 5, 5000) == -1
    # 10 / (1.58 + 2.0) < 3 cells of the list radius
    assert L.tdpd_set_verlet(h, 2.0, 5, 0) == -2
    assert L.tdpd_set_verlet(h, 0.3, 5, 0) == 0
    sk, ev, cap = C.c_float(), C.c_int32(), C.c_int32()
    assert L.tdpd_get_verlet(h, C.byref(sk), C.byref(ev), C.byref(cap)) == 0
    assert abs(sk.value - 0.3) < 1e-7 and ev.value == 5
    # three times the mean count within 1.88 at rho = 4, plus 128, to a multiple of 32
    mean = 4.0 / 3.0 * np.pi * np.float32(1.88) ** 3 * 4.0
    assert cap.value == (int(3 * mean) + 128 + 31) // 32 * 32
    assert L.tdpd_set_verlet(h, 0.0, 0, 0) == 0  # back to per-step cells
    assert L.tdpd_get_verlet(h, C.byref(sk), C.byref(ev), C.byref(cap)) == 0
    assert ev.value == 0 and cap.value == 0
    L.tdpd_destroy(h)
    # sheared boxes and the random flux are not taken
    cfgs = I.c1()
    cfgs.shear_rate = 0.5
    rc, h = _create(cfgs, shear_rate=0.5)
    assert rc == 0
    assert L.tdpd_set_verlet(h, 0.3, 5, 0) == -8
    L.tdpd_destroy(h)
    rc, h = _create(cfg, m_s=0.05)
    assert rc == 0
    assert L.tdpd_set_verlet(h, 0.3, 5, 0) == -8
    L.tdpd_destroy(h)
