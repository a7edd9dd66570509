"""Pins of the oracle's membrane terms (Section 2.2, Eqs. 13-19): closed-form
area, volume and dihedral angle of regular polyhedra, stress-free rest shape,
forces equal to minus the gradient of the energies (central differences),
zero net force and torque, rotation covariance, unwrapping across the
periodic boundary."""
import math

import numpy as np
import pytest

from oracle import Oracle, TERM
from paper_1611_06163_amd import inputs as I

CONS = TERM["bond"] | TERM["area"] | TERM["vol"] | TERM["bend"]


def _mesh_cfg(xyz, tri, box=(30.0, 30.0, 30.0), shift=(15.0, 15.0, 15.0), mp=None):
    cfg = I.make_fluid(box=box, n=xyz.shape[0], seed=0)
    pos = xyz + np.asarray(shift)
    cfg.pos = np.mod(pos, np.asarray(box)).astype(np.float32)
    cfg.vel[:] = 0
    cfg.flags[:] = I.T_MEMBRANE
    cfg.mesh_xyz, cfg.mesh_tri = xyz, tri
    cfg.rbc_first_gid = [0]
    if mp is not None:
        cfg.mesh_params = mp
    return cfg


def test_icosahedron_closed_forms():
    a = 1.3
    xyz, tri = I.icosahedron_mesh(a)
    o = Oracle(_mesh_cfg(xyz, tri))
    info = o.mesh_info()
    assert info["nedge"] == 30 and info["ndih"] == 30 and info["ntri"] == 20
    assert abs(info["A0"] - 5 * math.sqrt(3) * a * a) < 1e-12
    assert abs(info["V0"] - 5.0 / 12.0 * (3 + math.sqrt(5)) * a ** 3) < 1e-12
    # angle between adjacent face normals = pi - interior dihedral = acos(sqrt5/3)
    assert abs(info["theta0"] - math.acos(math.sqrt(5) / 3)) < 1e-12


def test_tetrahedron_closed_forms():
    xyz, tri = I.tetra_mesh()  # edge 2*sqrt(2)
    o = Oracle(_mesh_cfg(xyz, tri))
    info = o.mesh_info()
    e = 2 * math.sqrt(2)
    assert abs(info["A0"] - math.sqrt(3) * e * e) < 1e-12
    assert abs(info["V0"] - e ** 3 / (6 * math.sqrt(2))) < 1e-12
    assert abs(info["theta0"] - (math.pi - math.acos(1.0 / 3.0))) < 1e-12


def test_area_volume_unwrapped_across_boundary():
    a = 1.1
    xyz, tri = I.icosahedron_mesh(a)
    cfg = _mesh_cfg(xyz, tri, box=(8.0, 8.0, 8.0), shift=(0.1, 7.9, 0.05))
    o = Oracle(cfg)
    m = o.membrane(cfg.pos.astype(np.float64))
    A, V = m["av"][0]
    assert abs(A - 5 * math.sqrt(3) * a * a) < 1e-5
    assert abs(V - 5.0 / 12.0 * (3 + math.sqrt(5)) * a ** 3) < 1e-5


def test_rest_shape_stress_free():
    xyz, tri = I.rbc_template()
    cfg = _mesh_cfg(xyz, tri)
    o = Oracle(cfg, terms=TERM["bond"] | TERM["area"] | TERM["vol"])
    F = o.membrane(cfg.mesh_xyz + 15.0)["F"]
    assert np.abs(F).max() < 1e-9
    # a regular icosahedron is also free of bending stress
    xyz, tri = I.icosahedron_mesh(0.9)
    c2 = _mesh_cfg(xyz, tri)
    o2 = Oracle(c2, terms=CONS)
    assert np.abs(o2.membrane(xyz + 15.0)["F"]).max() < 1e-9


def _perturbed_rbc(seed=0, amp=0.06):
    xyz, tri = I.rbc_template()
    cfg = _mesh_cfg(xyz, tri)
    rng = np.random.default_rng(seed)
    pos = xyz + 15.0 + rng.normal(scale=amp, size=xyz.shape)
    return cfg, pos


@pytest.mark.parametrize("term,idx", [("bond", 0), ("area", 1), ("vol", 2), ("bend", 3)])
def test_forces_are_minus_energy_gradient(term, idx):
    cfg, pos = _perturbed_rbc()
    cfg.mesh_params = I.MeshParams(kg=500.0, kv=500.0)
    o = Oracle(cfg, terms=TERM[term])
    F = o.membrane(pos)["F"]
    rng = np.random.default_rng(1)
    h = 1e-6
    for v in rng.choice(pos.shape[0], 12, replace=False):
        for a in range(3):
            p1 = pos.copy(); p1[v, a] += h
            p2 = pos.copy(); p2[v, a] -= h
            e1 = o.membrane(p1)["energy"][idx]
            e2 = o.membrane(p2)["energy"][idx]
            fd = -(e1 - e2) / (2 * h)
            scale = max(np.abs(F).max(), 1e-3)
            roundoff = 50 * 1.1e-16 * abs(e1) / h
            assert abs(fd - F[v, a]) <= 1e-6 * scale + roundoff, (term, v, a, fd, F[v, a])


def test_net_force_and_torque_vanish():
    cfg, pos = _perturbed_rbc(2)
    o = Oracle(cfg, terms=CONS)
    F = o.membrane(pos)["F"]
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * scale
    c = pos.mean(axis=0)
    tau = np.cross(pos - c, F).sum(axis=0)
    assert np.abs(tau).max() < 1e-11 * scale
    # the viscous and random bond forces are pairwise: zero net force
    o2 = Oracle(cfg, terms=TERM["bvisc"] | TERM["brand"])
    vel = np.random.default_rng(3).normal(size=pos.shape)
    F2 = o2.membrane(pos, vel, k=4)["F"]
    assert np.abs(F2.sum(axis=0)).max() < 1e-11 * np.abs(F2).sum()


def test_rotation_covariance():
    cfg, pos = _perturbed_rbc(4)
    o = Oracle(cfg, terms=CONS)
    F = o.membrane(pos)["F"]
    R = I.random_rotation(np.random.default_rng(5))
    c = np.array([15.0, 15.0, 15.0])
    posr = (pos - c) @ R.T + c
    Fr = o.membrane(posr)["F"]
    assert np.abs(Fr - F @ R.T).max() < 1e-9 * np.abs(F).max()


def test_bond_sign_stretch_and_compress():
    cfg, _ = _perturbed_rbc()
    o = Oracle(cfg, terms=TERM["bond"])
    xyz = cfg.mesh_xyz + 15.0
    e, _ = o.mesh_topology()
    a, b = e[0]
    for s, sign in ((1.05, 1.0), (0.95, -1.0)):
        p = xyz.copy()
        p[b] = p[a] + s * (xyz[b] - xyz[a])
        F = o.membrane(p)["F"]
        # stretched: a is pulled toward b; compressed: pushed away
        assert sign * np.dot(F[a], xyz[b] - xyz[a]) > 0


def test_reference_dihedral_mean_positive_for_convex_cell():
    xyz, tri = I.rbc_template()
    o = Oracle(_mesh_cfg(xyz, tri))
    assert o.mesh_info()["theta0"] > 0
