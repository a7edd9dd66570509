"""Shared helpers of the GPU parity tests."""
import os

import numpy as np

from oracle import Oracle, pair_normals_batch
from paper_1611_06163_amd import tdpd

TOL = 1e-5          # per-particle force / flux tolerance, relative to sum_j |term_ij|
# the membrane terms' share of that sum (bonds, area, volume, bending; each a
# handful of FP32 operations on vertex-relative vectors, the global area and
# volume totals exact in FP64) is held to about 50 FP32 ulps instead
TOL_MEM = 3e-6


def gpu_system(cfg, kernel=None, terms=tdpd.TERMS_ALL, env=None):
    """Create a GPU system; `kernel` picks the pair kernel (0 simple, 1 tiled)
    and `env` sets other library switches (TDPD_BIN, TDPD_GRAPH) for it."""
    env = dict(env or {})
    if kernel is not None:
        env["TDPD_PAIR_KERNEL"] = str(kernel)
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return tdpd.System(cfg, terms=terms)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _ulp32(x):
    x = np.abs(np.asarray(x, dtype=np.float32))
    return (np.nextafter(x, np.float32(np.inf)) - x).astype(np.float64)


def _pairs_of_sample(cfg, pos, which):
    """Ordered pairs (i, j), i in the sample, |d| below r_c (1 + 1e-4) under
    the minimum image (periodic k-d tree; no shear): a superset of the
    sample's pairs whose distances could round across r_c."""
    from scipy.spatial import cKDTree
    assert float(getattr(cfg, "shear_rate", 0.0)) == 0.0
    L = np.asarray(cfg.box, dtype=np.float64)
    x = np.mod(pos.astype(np.float64), L)
    x[x >= L] = 0.0
    tree = cKDTree(x, boxsize=L)
    idx = np.flatnonzero(which)
    nb = tree.query_ball_point(x[idx], r=cfg.rc * (1.0 + 1e-4))  # (superset)
    pi = np.concatenate([np.full(len(b), i, np.int64) for i, b in zip(idx, nb)])
    pj = np.concatenate([np.asarray(b, np.int64) for b in nb])
    keep = pi != pj
    return np.stack([pi[keep], pj[keep]], axis=1)


def flux_sensitivity(cfg, pos, conc, which):
    """Per sampled particle and species, a bound on how far the FP32
    rounding of its pair distances and of the flux weight can move its
    Fickian flux (Eq. 8).  w = 1 - r/r_cc loses relative precision as r
    nears r_cc, where a flux made of a few such pairs of one sign (a solvent
    particle at C = 0 beside a cell's vertices) is then resolved to no better
    than the pair's own weight error: per pair |dw| <= dr/r_cc + 2^-23 (dr
    the rounding of r, as in near_cutoff_sensitivity; one rounding of the
    fused 1 - r/r_cc and of 1/r_cc), and the flux term moves by at most
    kappa_ij |C_j - C_i| (2 w_hi |dw| + dw^2) for the exponent 2 weight."""
    from scipy.spatial import cKDTree
    assert float(getattr(cfg, "shear_rate", 0.0)) == 0.0 and float(cfg.sc_exp) == 2.0
    L = np.asarray(cfg.box, dtype=np.float64)
    x = np.mod(pos.astype(np.float64), L)
    x[x >= L] = 0.0
    tree = cKDTree(x, boxsize=L)
    idx = np.flatnonzero(which)
    nb = tree.query_ball_point(x[idx], r=cfg.rcc * (1.0 + 1e-4))
    pi = np.concatenate([np.full(len(b), i, np.int64) for i, b in zip(idx, nb)])
    pj = np.concatenate([np.asarray(b, np.int64) for b in nb])
    keep = pi != pj
    pi, pj = pi[keep], pj[keep]
    d = pos[pj].astype(np.float64) - pos[pi]
    shift = -L * np.round(d / L)
    d += shift
    r = np.linalg.norm(d, axis=1)
    # across the boundary the lifted coordinate (below 2 L) rounds to half an
    # ulp of 2 L; the difference rounds to half an ulp of d
    dd = np.where(shift != 0.0, 0.5 * _ulp32(2.0 * L)[None, :], 0.0) + 0.5 * _ulp32(d)
    dr = (np.abs(d) / np.maximum(r, 1e-30)[:, None] * dd).sum(axis=1) + 3.0 * _ulp32(r)
    dw = dr / cfg.rcc + 2.0 ** -23
    whi = np.clip(1.0 - (r - dr) / cfg.rcc, 0.0, 1.0)
    inside = r - dr < cfg.rcc
    kap = np.asarray(cfg.kappa, dtype=np.float64)            # [species][type i][type j]
    ti, tj = cfg.flags[pi] & 0xFF, cfg.flags[pj] & 0xFF       # flags: bits 0-7 the type
    kp = kap[:, ti, tj].T                                     # [pair][species]
    dC = np.abs(conc[pj].astype(np.float64) - conc[pi])
    per = np.where(inside, 2.0 * whi * dw + dw * dw, 0.0)[:, None] * kp * dC
    out = np.zeros((pos.shape[0], cfg.n_species))
    np.add.at(out, pi, per)
    return out


def near_cutoff_sensitivity(o, cfg, pos, vel, k, which=None):
    """Per particle, a bound on how far the FP32 rounding of the pair
    distances can move its force.

    Near r_c the weights w_R = w^(s/2) and w_D = w^s (w = 1 - r/r_c) turn a
    rounding of r into an unbounded relative change.  That rounding is bounded
    per pair from the specified arithmetic: for a pair across the periodic
    boundary the coordinate nearer 0 is lifted by +L, which rounds to half an
    ulp of the lifted value, and the difference with the other coordinate is
    exact; otherwise the difference rounds to half an ulp of d.  Three more
    ulps of r cover d^2, rsqrt and r.  With |dr| bounded, the change of each
    weight is bounded by its values at w -/+ dr/r_c (the weights are
    monotone), so a pair moves the force by at most
    sigma |xi| dw_R / sqrt(dt) + gamma |v_ij| dw_D + alpha dr / r_c, with the
    pair's own noise draw xi.  With `which`, only the sampled particles get
    a bound (from their own pairs; the others 0)."""
    if which is None:
        p, _ = o.pairs(pos.astype(np.float32), 0, k=k)
    else:
        p = _pairs_of_sample(cfg, pos, which)
    xi_ = pos[p[:, 0]].astype(np.float64)
    xj = pos[p[:, 1]].astype(np.float64)
    d = xj - xi_
    L = np.asarray(cfg.box)
    shear = float(getattr(cfg, "shear_rate", 0.0))
    le = np.zeros(len(p), bool)
    if shear != 0.0:
        # pairs across the sheared y boundary: the lower particle is lifted
        # by +L_y and by delta + m L_x in x (two roundings of values < 2 L_x)
        a = float(np.float32(shear)) * float(np.float32(L[1]))
        delta = float(np.float32(np.fmod(a * (k * float(np.float32(cfg.dt))), float(np.float32(L[0])))))
        le = np.abs(d[:, 1]) > 0.5 * L[1]
        sgn = -np.sign(d[le, 1])
        d[le, 1] += sgn * L[1]
        d[le, 0] += sgn * delta
        # the lower particle's lifted coordinates, before the x wrap
        low = np.where((sgn < 0)[:, None], xi_[le], xj[le])
        X1 = low[:, 0] + delta
        Yl = low[:, 1] + L[1]
    shift = -L * np.round(d / L)
    d += shift
    r = np.linalg.norm(d, axis=1)
    # across the boundary the coordinate nearer 0 is lifted by +L in FP32,
    # rounding to half an ulp of the lifted value (>= L); the difference of
    # the lifted coordinate and the other is then exact (Sterbenz), else the
    # plain difference rounds to half an ulp of d
    lifted = np.minimum(xi_, xj) + L
    dd = np.where(shift != 0.0, 0.5 * _ulp32(lifted), 0.5 * _ulp32(d))
    if le.any():
        # y: fl(y + L_y); x: fl(x + delta), then fl(X1 + m L_x) when m != 0;
        # the differences round to half an ulp of d
        m_ne0 = shift[le, 0] != 0.0
        dd[le, 0] = (0.5 * _ulp32(X1) + np.where(m_ne0, 0.5 * _ulp32(2.0 * L[0]), 0.0)
                     + 0.5 * _ulp32(d[le, 0]))
        dd[le, 1] = 0.5 * _ulp32(Yl) + 0.5 * _ulp32(d[le, 1])
    dr = (np.abs(d) / r[:, None] * dd).sum(axis=1) + 3.0 * _ulp32(r)
    w = np.clip(1.0 - r / cfg.rc, 0.0, 1.0)
    dw = dr / cfg.rc
    # (the same as w -/+ dw clipped to [0, 1] inside r_c; a sampled pair
    # beyond r_c moves only if its rounding can bring it inside)
    wlo = np.clip(1.0 - (r + dr) / cfg.rc, 0.0, 1.0)
    whi = np.clip(1.0 - (r - dr) / cfg.rc, 0.0, 1.0)
    s = cfg.s_exp

    def spread(e):
        return np.maximum(w ** e - wlo ** e, whi ** e - w ** e)

    xi = np.abs(pair_normals_batch(cfg, k, p[:, 0], p[:, 1], 0)[:, 0])
    vv = vel[p[:, 0]].astype(np.float64) - vel[p[:, 1]]
    if shear != 0.0:
        vv[le, 0] -= sgn * a  # the lifted particle's image moves with +u
    vij = np.linalg.norm(vv, axis=1)
    sig = float(np.max(cfg.sigma))
    gam = float(np.max(cfg.gamma))
    alp = float(np.max(cfg.alpha))
    sens = (sig * xi * spread(0.5 * s) / np.sqrt(cfg.dt) + gam * vij * spread(s) + alp * dw)
    tot = np.zeros(pos.shape[0])
    np.add.at(tot, p[:, 0], sens)
    if which is None:  # unordered pairs: the bound is the partner's too
        np.add.at(tot, p[:, 1], sens)
    mobile = (cfg.flags & tdpd.FLAG_FROZEN) == 0  # frozen particles have F = 0 exactly
    return np.where(mobile, tot, 0.0)


def near_cutoff(o, cfg, pos, vel, ref, k, tol=TOL, which=None):
    """(mask, sens): particles whose force cannot be resolved to the parity
    bound in FP32 -- the rounding of their pair distances alone
    (near_cutoff_sensitivity, sens) may move the force by more than half of
    force_bound.  compare_forces checks them against force_bound + sens."""
    sens = near_cutoff_sensitivity(o, cfg, pos, vel, k, which=which)
    return sens > 0.5 * force_bound(ref, tol), sens


def force_bound(ref, tol=TOL, tol_mem=TOL_MEM):
    """Per-particle force bound: tol times the pair terms' magnitude sum plus
    tol_mem times the membrane terms' (+ a floor of FP32 resolution of the
    result itself)."""
    fm = ref.get("Fmabs", np.zeros_like(ref["Fabs"]))
    return (tol * (ref["Fabs"] - fm) + tol_mem * fm
            + 4e-7 * np.linalg.norm(ref["F"], axis=1) + 1e-6)


def compare_forces(F, Q, ref, exclude=None, tol=TOL, which=None, label="", tol_mem=TOL_MEM,
                   sens=None, sens_q=None):
    """Per-particle check |F - F_ref| <= force_bound(ref); |Q - Q_ref| <=
    tol * sum_j |Q_ij| (+ a floor).  Excluded particles (near_cutoff_mask)
    are checked against force_bound + sens when sens is given (badF_excl).
    Returns a report dict (with the median and largest bound of membrane
    vertices)."""
    n = F.shape[0]
    sel = np.ones(n, bool) if which is None else which.astype(bool)
    if exclude is not None:
        sel &= ~exclude
    eF = np.linalg.norm(F.astype(np.float64) - ref["F"], axis=1)
    bF = force_bound(ref, tol, tol_mem)
    eQ = np.abs(Q.astype(np.float64) - ref["Q"])
    bQ = tol * ref["Qabs"] + 4e-7 * np.abs(ref["Q"]) + 1e-7
    if sens_q is not None:  # flux_sensitivity: the weight's rounding near r_cc
        bQ = bQ + sens_q
    badF = sel & (eF > bF)
    badQ = sel[:, None] & (eQ > bQ)
    rF = (eF / np.maximum(ref["Fabs"], 1e-30))[sel]
    rQ = (eQ / np.maximum(ref["Qabs"], 1e-30))[sel]
    rep = dict(label=label, n=int(sel.sum()), excluded=int(n - sel.sum()),
               max_relF=float(rF.max()) if rF.size else 0.0,
               p999_relF=float(np.quantile(rF, 0.999)) if rF.size else 0.0,
               max_relQ=float(rQ.max()) if rQ.size else 0.0,
               badF=int(badF.sum()), badQ=int(badQ.sum()))
    if exclude is not None and sens is not None:
        # excluded particles: within the bound widened by their own
        # distance-rounding sensitivity (counted into badF)
        ex = exclude & (np.ones(n, bool) if which is None else which.astype(bool))
        rep["badF_excl"] = int((ex & (eF > bF + sens)).sum())
        rep["badF"] += rep["badF_excl"]
        rep["excl_err_over_bound_max"] = float((eF / (bF + sens))[ex].max()) if ex.any() else 0.0
    vert = ref.get("Fmabs", np.zeros(n)) > 0
    if vert.any():
        rep["vertex_bound_median"] = float(np.median(bF[vert]))
        rep["vertex_bound_max"] = float(bF[vert].max())
        rep["vertex_err_over_bound_max"] = float((eF / bF)[vert & sel].max()) if (vert & sel).any() else 0.0
    worst = np.argsort(-np.where(sel, eF / bF, 0))[:3]
    rep["worst"] = [(int(i), float(eF[i] / max(ref["Fabs"][i], 1e-30))) for i in worst]
    print("parity", rep, flush=True)
    return rep
