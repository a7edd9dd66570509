"""Throughput benchmark of the tDPD + RBC time step on one MI355X.

Default workload: a single 500-vertex red cell in a 20^3 periodic box of
density-3 solvent (24,000 solvent + 500 membrane particles, two species),
the single-RBC configuration.  Prints one JSON line: particle-steps/s of the
whole step (pair forces and fluxes, membrane terms, binning, velocity
Verlet) with inputs resident in HBM, the pair kernel's ALU roofline figure
from HIP events on the library's stream, and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue slots per unit of pair-kernel work (non-packed FP32; quarter-rate
# transcendentals and 32-bit multiplies count 4).  A candidate test is 3 sub,
# 1 mul, 2 fma, 1 compare; a flux pair and species is rsqrt (4), r, weight
# fma, max, square, C difference, two multiplies and the accumulate; a force
# pair is rsqrt, e, weights incl. exp2/log2, e.v, three terms, the
# accumulate, Philox-4x32-10 (10 rounds of two 32x32->64 products, xors
# and key adds = 140) and Box-Muller (about 21).
OPS_CANDIDATE = 7
OPS_FLUX_PER_SPECIES = 12
OPS_FORCE = 200
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
METRIC = "tDPD particle-steps/s on 1 MI355X; batched & surrogate vs plain at tol"

# HBM bytes per launch of the pair kernel from two rocprofv3 counter runs
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0, the factors a 256 MiB copy gives;
# profiles/pair_tiled_single_rbc_20cube_hbm.md).  Valid only for the kernel
# sources they were taken with: reported when the hash still matches.
PAIR_SOURCES = ("kernels_pair_tiled.hip", "pair_terms.h", "tdpd_device.h", "launch.h")
PAIR_TRAFFIC = {
    "c2": {"sha256": "c578969bedbfc4bfe393e6c9e0a92551604d111b9efcac0c738c4f254c1c8db5", "read_bytes": 2.648e6, "write_bytes": 0.490e6},
}


def pair_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_06163_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pair_traffic(name):
    t = PAIR_TRAFFIC.get(name)
    if t is None or t["sha256"] != pair_source_hash():
        return None
    return t["read_bytes"] + t["write_bytes"]


def workload(name):
    from paper_1611_06163_amd import inputs as I
    if name == "c2":
        return I.c2(), "single RBC (500 vertices) in 20^3 periodic tDPD solvent, rho=3, 2 species"
    if name == "c1":
        return I.c1(), "plain tDPD fluid 10^3, rho=4, 4000 particles, 1 species"
    if name == "c3":
        return I.c3(), "100 RBCs in 64x32x32 wall-bounded channel, rho=3, body force 0.02, 2 species"
    raise SystemExit(f"unknown workload {name}")


def pair_work(sysg, cfg):
    """Ordered candidate tests, flux pairs and force pairs at the current state."""
    import numpy as np
    pos, _, _ = sysg.get_state()
    rmax = max(cfg.rc, cfg.rcc)
    nc = [int(np.floor(L / (rmax * (1 + 1e-4)))) for L in cfg.box]
    idx = [np.minimum((pos[:, a] * np.float32(nc[a] / cfg.box[a])).astype(np.int64), nc[a] - 1)
           for a in range(3)]
    occ = np.zeros(nc[::-1], np.int64)
    np.add.at(occ, (idx[2], idx[1], idx[0]), 1)
    nb = np.zeros_like(occ)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb += np.roll(occ, (dz, dy, dx), axis=(0, 1, 2))
    frozen = (cfg.flags & (1 << 8)) != 0
    home_mobile = np.zeros_like(occ)
    np.add.at(home_mobile, (idx[2][~frozen], idx[1][~frozen], idx[0][~frozen]), 1)
    n_cand = int((home_mobile * nb).sum())
    pf = sysg.pairs(0)
    body = np.full(cfg.n, -1)
    for r, g0 in enumerate(cfg.rbc_first_gid):
        body[g0:g0 + cfg.mesh_xyz.shape[0]] = r
    same = (body[pf[:, 0]] >= 0) & (body[pf[:, 0]] == body[pf[:, 1]])
    pf = pf[~same]
    n_force = int((~frozen[pf[:, 0]]).sum() + (~frozen[pf[:, 1]]).sum())
    pq = sysg.pairs(1)
    n_flux = int((~frozen[pq[:, 0]]).sum() + (~frozen[pq[:, 1]]).sum())
    return n_cand, n_flux, n_force


def cpu_baseline(cfg, target_s=15.0):
    import numpy as np
    from oracle import Oracle
    o = Oracle(cfg)
    st = o.init_state()
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    k = 0
    while True:
        k += 1
        o.step(st, k)
        el = time.perf_counter() - t0
        if el > target_s or k >= 400:
            break
    return dict(value=cfg.n * k / el, unit="particle-steps/s", cores=cores, kind="oracle",
                sample=f"{k} velocity-Verlet steps of the same workload from its initial "
                       f"state, FP64 oracle, {cores} OpenMP threads, {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", type=int, default=None, help="pair kernel: 0 simple, 1 tiled")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shape of the pair kernel")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device-to-device with torch (a plain "
                         "copy of known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_1611_06163_amd import tdpd
    if args.kernel is not None:
        os.environ["TDPD_PAIR_KERNEL"] = str(args.kernel)
    torch.cuda.set_device(0)
    cfg, desc = workload(args.workload)
    sysg = tdpd.System(cfg)
    sysg.compute_forces(0)
    if not args.no_autotune:
        sysg.autotune(reps=5)  # before the warm-up: untimed
    n_cand, n_flux, n_force = pair_work(sysg, cfg)
    sysg.step(args.warmup)
    sysg.sync()
    sysg.set_timing(tdpd.PHASE["pair"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysg.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sysg.sync()
    pair_ms, pair_n = sysg.get_timing(tdpd.PHASE["pair"])
    sysg.set_timing(0)
    el = t1 - t0
    value = cfg.n * args.steps / el
    ops = OPS_CANDIDATE * n_cand + OPS_FLUX_PER_SPECIES * cfg.n_species * n_flux + OPS_FORCE * n_force
    pair_avg_s = pair_ms / max(pair_n, 1) / 1e3
    achieved = ops / pair_avg_s / 1e12
    d = sysg.diagnostics()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "particles": cfg.n, "box": list(cfg.box),
                   "n_species": cfg.n_species, "rbcs": len(cfg.rbc_first_gid),
                   "dt": cfg.dt, "pair_kernel": os.environ.get("TDPD_PAIR_KERNEL", "1"),
                   "tile": list(sysg.tile)},
        "roofline": {"bound": "alu", "kernel": "pair (forces + fluxes)",
                     "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": pair_traffic(args.workload),
                     "traffic_unit": "bytes per launch",
                     "avg_launch_us": pair_avg_s * 1e6, "launches": pair_n,
                     "ops_per_launch": ops,
                     "units_per_launch": {"candidate_tests": n_cand, "flux_pairs": n_flux,
                                          "force_pairs": n_force}},
        "diagnostics": {"kT": d["kT"], "P": [float(x) for x in d["P"]]},
    }
    sysg.close()
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
