"""Shared helpers of the GPU parity tests."""
import os

import numpy as np

from oracle import Oracle
from paper_1611_06163_amd import tdpd

TOL = 1e-5          # per-particle force / flux tolerance, relative to sum_j |term_ij|
CUT_DELTA = 2e-4    # pairs this close to r_c have FP32-limited random-force weights


def gpu_system(cfg, kernel=None, terms=tdpd.TERMS_ALL):
    old = os.environ.get("TDPD_PAIR_KERNEL")
    if kernel is not None:
        os.environ["TDPD_PAIR_KERNEL"] = str(kernel)
    try:
        return tdpd.System(cfg, terms=terms)
    finally:
        if kernel is not None:
            if old is None:
                os.environ.pop("TDPD_PAIR_KERNEL", None)
            else:
                os.environ["TDPD_PAIR_KERNEL"] = old


def near_cutoff_mask(o, cfg, pos, delta=CUT_DELTA):
    """Particles with a force pair whose distance is within delta of r_c."""
    p, _ = o.pairs(pos.astype(np.float32), 0)
    d = pos[p[:, 1]].astype(np.float64) - pos[p[:, 0]]
    L = np.asarray(cfg.box)
    d -= L * np.round(d / L)
    r = np.linalg.norm(d, axis=1)
    near = np.abs(r - cfg.rc) < delta
    m = np.zeros(pos.shape[0], bool)
    m[p[near, 0]] = True
    m[p[near, 1]] = True
    return m


def compare_forces(F, Q, ref, exclude=None, tol=TOL, which=None, label=""):
    """Per-particle check |F - F_ref| <= tol * sum_j |F_ij| (+ a floor of FP32
    resolution of the result itself); same for Q.  Returns a report dict."""
    n = F.shape[0]
    sel = np.ones(n, bool) if which is None else which.astype(bool)
    if exclude is not None:
        sel &= ~exclude
    eF = np.linalg.norm(F.astype(np.float64) - ref["F"], axis=1)
    bF = tol * ref["Fabs"] + 4e-7 * np.linalg.norm(ref["F"], axis=1) + 1e-6
    eQ = np.abs(Q.astype(np.float64) - ref["Q"])
    bQ = tol * ref["Qabs"] + 4e-7 * np.abs(ref["Q"]) + 1e-7
    badF = sel & (eF > bF)
    badQ = sel[:, None] & (eQ > bQ)
    rF = (eF / np.maximum(ref["Fabs"], 1e-30))[sel]
    rQ = (eQ / np.maximum(ref["Qabs"], 1e-30))[sel]
    rep = dict(label=label, n=int(sel.sum()), excluded=int(n - sel.sum()),
               max_relF=float(rF.max()) if rF.size else 0.0,
               p999_relF=float(np.quantile(rF, 0.999)) if rF.size else 0.0,
               max_relQ=float(rQ.max()) if rQ.size else 0.0,
               badF=int(badF.sum()), badQ=int(badQ.sum()))
    print("parity", rep, flush=True)
    return rep
