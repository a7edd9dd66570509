"""Pins of the surrogate oracle (oracle/surrogate.py) against what
mathematics and library routines fix: bfloat16 rounding against torch's
conversion, the gradient against central differences, Adam's first step in
closed form, the features of a regular icosahedron in closed form, and the
invariance of the features under rigid motions."""
import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S
from paper_1611_06163_amd import inputs as I


def test_bf16_matches_torch_including_ties():
    rng = np.random.default_rng(0)
    x = (rng.normal(size=20000) * 10.0 ** rng.integers(-6, 6, 20000)).astype(np.float32)
    # exact ties: low 16 bits = 0x8000 with even and odd kept parts
    t = (rng.integers(0, 2 ** 15, 2000, dtype=np.uint32) << 16) | 0x8000
    x = np.concatenate([x, t.astype(np.uint32).view(np.float32)])
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(x), ref)


def test_parameter_count():
    assert S.N_PARAMS == 36099


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = S.init_params(rng).astype(np.float64)
    X = rng.normal(size=(7, S.N_IN))
    T = rng.normal(size=(7, S.N_OUT))
    loss, g = S.loss_and_grad(p, X, T, rounding=False)
    idx = np.concatenate([rng.choice(S.N_PARAMS, 40, replace=False),
                          np.arange(S.N_PARAMS - 3, S.N_PARAMS)])  # output biases too
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (S.loss_and_grad(pp, X, T, rounding=False)[0] -
              S.loss_and_grad(pm, X, T, rounding=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, g[i])


def test_rounded_gradient_close_to_exact():
    rng = np.random.default_rng(2)
    p = S.init_params(rng).astype(np.float64)
    X = rng.normal(size=(64, S.N_IN))
    T = rng.normal(size=(64, S.N_OUT))
    _, g0 = S.loss_and_grad(p, X, T, rounding=False)
    _, g1 = S.loss_and_grad(p, X, T, rounding=True)
    assert np.linalg.norm(g1 - g0) < 2e-2 * np.linalg.norm(g0)


def test_adam_first_step_closed_form_and_convergence():
    rng = np.random.default_rng(3)
    g = rng.normal(size=50)
    w0 = rng.normal(size=50)
    w1, m, v = S.adam(w0, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-8)
    # bias-corrected m = g and v = g^2 after one step
    assert np.allclose(w1 - w0, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # minimises a diagonal quadratic
    a = rng.uniform(0.5, 5.0, 50)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 3001):
        w, m, v = S.adam(w, a * w, m, v, t, lr=0.01)
    assert np.abs(w).max() < 1e-2


def test_icosahedron_features_closed_form():
    xyz, tri = I.icosahedron_mesh(edge=1.0)
    rg = S.rings(tri, 12)
    assert all(r is not None and len(r) == 5 for r in rg)
    X, R, ok = S.features(xyz + 50.0, (100.0, 100.0, 100.0), rg, 1.0, 1.0, 1.0, 1.0, 1.0, 100.0)
    assert ok.all()
    rho = np.linalg.norm(xyz[0])
    phi = math.acos(1.0 / math.sqrt(5.0))  # angle between neighbouring vertex directions
    ref = np.array([[rho * math.sin(phi) * math.cos(2 * math.pi * k / 5),
                     rho * math.sin(phi) * math.sin(2 * math.pi * k / 5),
                     rho * (math.cos(phi) - 1.0)] for k in range(5)]).ravel()
    for v in range(12):
        assert np.allclose(X[v, :15], ref, atol=1e-12)
        assert np.allclose(X[v, 15:], 0.0)
        # the normal is the outward radial direction
        assert np.allclose(R[v, 2], xyz[v] / rho, atol=1e-12)


def test_features_invariant_under_rigid_motion():
    xyz, tri = I.rbc_template(500, 7.8)
    rg = S.rings(tri, xyz.shape[0])
    assert all(r is not None for r in rg)
    deg = np.array([len(r) for r in rg])
    assert deg.sum() == 3 * tri.shape[0]
    box = (30.0, 30.0, 30.0)
    X0, R0, ok0 = S.features(xyz + 15.0, box, rg, 130.0, 132.0, 91.0, 92.0, 0.55, 100.0)
    Q = I.random_rotation(np.random.default_rng(4))
    moved = (xyz @ Q.T) + np.array([29.0, 0.5, 14.0])   # crosses the periodic boundary
    moved = np.mod(moved, 30.0)
    X1, R1, ok1 = S.features(moved, box, rg, 130.0, 132.0, 91.0, 92.0, 0.55, 100.0)
    assert np.array_equal(ok0, ok1)
    assert np.allclose(X0, X1, atol=1e-10)
    assert np.allclose(R1, R0 @ Q.T, atol=1e-10)
    # outward orientation: the frame normal points away from the centre
    assert np.all(np.einsum("ni,ni->n", R0[:, 2], xyz) > 0)
    assert set(np.unique(deg)) <= {4, 5, 6, 7, 8}
    assert ok0.sum() == np.isin(deg, (5, 6)).sum()


def test_surrogate_forces_rotate_with_the_cell():
    rng = np.random.default_rng(5)
    p = S.init_params(rng)
    xyz, tri = I.rbc_template(500, 7.8)
    rg = S.rings(tri, xyz.shape[0])
    box = (30.0, 30.0, 30.0)
    X0, R0, _ = S.features(xyz + 15.0, box, rg, 130.0, 132.0, 91.0, 92.0, 0.55, 100.0)
    Q = I.random_rotation(rng)
    X1, R1, _ = S.features(xyz @ Q.T + 15.0, box, rg, 130.0, 132.0, 91.0, 92.0, 0.55, 100.0)
    F0 = S.surrogate_forces(p, X0, R0, 2.0, rounding=False)
    F1 = S.surrogate_forces(p, X1, R1, 2.0, rounding=False)
    assert np.allclose(F1, F0 @ Q.T, atol=1e-8)
