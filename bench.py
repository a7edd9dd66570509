"""Throughput benchmark of the tDPD + RBC time step on one MI355X.

Default workload: the large suspension, 1000 red cells of 500 vertices in a
96x96x72 periodic box of density-3 solvent (1,990,656 solvent + 500,000
membrane particles, two species), the largest single-GPU configuration.
Prints one JSON line: particle-steps/s of the whole step (pair forces and
fluxes, membrane terms, binning, velocity Verlet) with inputs resident in
HBM -- the median of several timed windows of exactly --steps steps -- the
pair kernel's ALU roofline figure from HIP events on the library's stream,
and the CPU oracle timed on a bounded sample of the same workload.  Further
objects: the single-cell box, the batched ensemble, ten species, Verlet
lists, the random flux and the membrane surrogate, each against the plain
path on the same GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU lane-operations per unit of pair-kernel work (non-packed
# FP32; quarter-rate transcendentals and 32-bit integer multiplies count 4):
# a candidate test (displacement, squared distance, cutoff compare), a force
# pair (weights, three force terms, Philox-4x32-10 and Box-Muller) and a flux
# pair per species (weight, Fickian term, accumulate).  Candidate tests are
# those of the 27-cell stencil of every mobile home particle.
OPS_CANDIDATE = 10
OPS_FLUX_PER_SPECIES = 16
OPS_FORCE = 250
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
METRIC = "tDPD particle-steps/s on 1 MI355X; batched & surrogate vs plain at tol"

# HBM bytes per launch of the pair kernel from two rocprofv3 counter runs
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0, the factors a 256 MiB copy gives;
# profiles/hbm_traffic_suspension_1000rbc.md).  Valid only for the kernel
# sources and tile shape they were taken with: reported when both match.
PAIR_SOURCES = ("pair_tiled.h", "kernels_pair_tiled.hip", "pair_terms.h", "tdpd_device.h",
                "launch.h", "membrane_cell.h")
PAIR_TRAFFIC = {
    "c5": {"sha256": "7d2cdba79f3b3886c9886947a8f9ed73812679e5c833e02a77a90426f9ea9f93",
           "tiles": {"2,3,1,1": [1.3824e+08, 5.0040e+07]}},
}


def pair_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_06163_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pair_traffic(name, tile):
    """Read + write bytes per launch for a measured (sources, shape), else None."""
    t = PAIR_TRAFFIC.get(name)
    if t is None or t["sha256"] != pair_source_hash():
        return None
    rw = t["tiles"].get(",".join(str(v) for v in tile))
    return None if rw is None else rw[0] + rw[1]


def workload(name):
    from paper_1611_06163_amd import inputs as I
    if name == "c5":
        return I.c5(), ("1000 RBCs (500 vertices each) in 96x96x72 periodic tDPD solvent, rho=3, "
                        "2 species")
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
    """The FP64 oracle stepping the same workload from its initial state (the
    set-up force evaluation untimed) until target_s seconds have passed."""
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
        if el > target_s or k >= 5000:
            break
    return dict(value=cfg.n * k / el, unit="particle-steps/s", cores=cores, kind="oracle",
                sample=f"{k} velocity-Verlet steps of the same workload ({cfg.n} particles) from "
                       f"its initial state, FP64 oracle, {cores} OpenMP threads, {el:.1f} s")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _timed_steps(torch, sysg, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysg.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sysg.sync()
    return el


def batched_leg(torch, tdpd, steps, warmup, n_boxes=256):
    """The batched ensemble (256 uneven sheared periodic boxes, 2k-60k
    particles, 0-4 cells each, own seed and shear rate) as one system against
    the same boxes as separate systems stepped one after another."""
    from paper_1611_06163_amd import inputs as I
    boxes = I.ensemble(n_boxes=n_boxes)
    n_tot = sum(b.n for b in boxes)
    _log(f"batched: {n_boxes} boxes, {n_tot} particles")
    sb = tdpd.System(boxes)
    sb.compute_forces(0)
    sb.autotune(reps=3)
    sb.step(warmup)
    sb.sync()
    el_b = _timed_steps(torch, sb, steps)
    tile = list(sb.tile)
    sb.close()
    solo = []
    for b in boxes:
        s = tdpd.System(b)
        s.compute_forces(0)
        s.autotune(reps=3)
        s.step(warmup)
        solo.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solo:
        s.step(steps)
    torch.cuda.synchronize()
    el_s = time.perf_counter() - t0
    for s in solo:
        s.sync()
        s.close()
    vb, vs = n_tot * steps / el_b, n_tot * steps / el_s
    return dict(workload=f"{n_boxes} Lees-Edwards boxes, N log-uniform in [2000, 60000], rho=3, "
                         "0-4 cells each, shear rate U[0, 0.5], 1 species",
                particles=n_tot, steps=steps, tile=tile, value=vb, unit="particle-steps/s",
                plain_value=vs, plain="the same boxes as separate systems, stepped in turn",
                speedup=vb / vs, tol="bitwise: a box in the batch follows its solo trajectory "
                                     "at the same tile shape (tests/test_gpu_batch.py)")


def species_leg(torch, tdpd, steps, warmup, n_species=10):
    """The single-RBC workload with ten species instead of two (the paper's
    many-species regime), on the same default path."""
    from paper_1611_06163_amd import inputs as I
    cfg = I.c2_species(n_species)
    sysg = tdpd.System(cfg)
    sysg.compute_forces(0)
    sysg.autotune(reps=3)
    sysg.step(warmup)
    sysg.sync()
    import numpy as np
    el = float(np.median([_timed_steps(torch, sysg, steps) for _ in range(5)]))
    sysg.set_timing(tdpd.PHASE["pair"])
    sysg.step(steps)
    pair_ms, pair_n = sysg.get_timing(tdpd.PHASE["pair"])
    sysg.set_timing(0)
    tile = list(sysg.tile)
    sysg.close()
    return dict(workload=f"single RBC (500 vertices) in 20^3 periodic tDPD solvent, rho=3, "
                         f"{n_species} species", n_species=n_species, particles=cfg.n,
                value=cfg.n * steps / el, unit="particle-steps/s", ms_per_step=el * 1e3 / steps,
                pair_us=pair_ms * 1e3 / max(pair_n, 1), tile=tile)


def verlet_leg(torch, tdpd, steps, warmup, wl, skin, every):
    """The same workload on Verlet neighbour lists (radius max(rc, rcc) +
    skin, rebuilt with the binning every `every` steps) instead of per-step
    cell scans; the pair kernel is timed as in the main run."""
    cfg, desc = workload(wl)
    sysg = tdpd.System(cfg)
    sysg.set_verlet(skin, every)
    sysg.compute_forces(0)
    sysg.step(warmup)
    sysg.sync()
    el = _timed_steps(torch, sysg, steps)
    sysg.set_timing(tdpd.PHASE["pair"] | tdpd.PHASE["bin"])
    sysg.step(steps)
    pair_ms, pair_n = sysg.get_timing(tdpd.PHASE["pair"])
    bin_ms, bin_n = sysg.get_timing(tdpd.PHASE["bin"])
    sysg.set_timing(0)
    cap = sysg.verlet[2]
    sysg.close()
    return dict(workload=desc, skin=skin, every=every, capacity=cap, particles=cfg.n,
                value=cfg.n * steps / el, unit="particle-steps/s", ms_per_step=el * 1e3 / steps,
                pair_us=pair_ms * 1e3 / max(pair_n, 1),
                kick_bin_list_us_per_step=bin_ms * 1e3 / max(bin_n, 1))


def surrogate_leg(torch, tdpd, steps, warmup, cfg, desc):
    """Train the membrane surrogate on samples of plain channel runs, then run
    the evaluation workload plain and with the network (fallback tolerance
    1e-2 of the cell's RMS plain force, checked every 10 steps)."""
    from paper_1611_06163_amd import inputs as I
    from paper_1611_06163_amd import surrogate as SU
    t0 = time.perf_counter()
    X, T = SU.collect(I.c3(seed=11, scale=0.25, n_cells=25), steps=450, every=5, skip=50)
    t1 = time.perf_counter()
    net, s_F, rep = SU.train(X, T, seed=0, batch=4096, steps=3000, lr=1e-3)
    t2 = time.perf_counter()
    _log(f"surrogate: {X.shape[0]} samples in {t1 - t0:.1f} s, trained in {t2 - t1:.1f} s: {rep}")
    runs = []
    for tol in (None, 1e-2, 0.1, 0.5):
        sysg = tdpd.System(cfg)
        sysg.compute_forces(0)
        sysg.autotune(reps=3)
        if tol is not None:
            sysg.surrogate_enable(net, s_F, tol=tol, check_every=10)
        sysg.step(warmup)
        sysg.sync()
        el = _timed_steps(torch, sysg, steps)
        r = dict(tol=tol, value=cfg.n * steps / el, ms_per_step=el * 1e3 / steps)
        if tol is not None:
            st = sysg.surrogate_stats()
            r.update(on_network=st["on_network"], eligible=st["eligible"],
                     check_max_err=st["max_err"], check_mean_err=st["mean_err"])
        runs.append(r)
        sysg.close()
        _log(f"surrogate run {r}")
    # the network's forward pass alone on as many rows as the workload has
    # vertices (host buffers in and out; the kernel's own time is in the
    # kernel trace)
    import numpy as np
    nv = 0 if cfg.mesh_xyz is None else len(cfg.mesh_xyz) * len(cfg.rbc_first_gid)
    nrow = min(nv, X.shape[0]) or X.shape[0]
    Xr = np.ascontiguousarray(X[:nrow])
    net.forward(Xr)
    t3 = time.perf_counter()
    for _ in range(5):
        net.forward(Xr)
    fwd_ms = (time.perf_counter() - t3) * 1e3 / 5
    plain, at = runs[0], runs[1]
    return dict(workload=desc, particles=cfg.n, value=at["value"], unit="particle-steps/s", tol=1e-2,
                plain_value=plain["value"], on_network=at["on_network"],
                by_tol=runs[1:],
                network_forward=dict(rows=nrow, ms_host_buffers=fwd_ms,
                                     flop_per_row=2 * (20 * 128 + 2 * 128 * 128 + 128 * 3)),
                error="per-vertex |F_net - F_plain| / RMS_cell |F_plain| of bending + "
                      "local-area force at the last check; vertices above tol use F_plain",
                training=dict(rep, collect_s=t1 - t0, train_s=t2 - t1,
                              data="channel 16x32x32, 25 cells, samples every 5 steps"))


def plain_leg(torch, tdpd, cfg, desc, steps, warmup, windows=1):
    """Median whole-step time of `windows` windows of `steps` steps on the
    default path, after autotuning and warm-up."""
    import numpy as np
    sysg = tdpd.System(cfg)
    sysg.compute_forces(0)
    sysg.autotune(reps=3)
    sysg.step(warmup)
    sysg.sync()
    els = [_timed_steps(torch, sysg, steps) for _ in range(windows)]
    el = float(np.median(els))
    tile = list(sysg.tile)
    sysg.close()
    return dict(workload=desc, particles=cfg.n, value=cfg.n * steps / el,
                unit="particle-steps/s", ms_per_step=el * 1e3 / steps, tile=tile)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--windows", type=int, default=7,
                    help="timed windows of --steps steps each; the median is reported")
    ap.add_argument("--workload", default="c5", choices=["c5", "c3", "c2", "c1"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", type=int, default=None, help="pair kernel: 0 simple, 1 tiled")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile shape of the pair kernel")
    ap.add_argument("--no-census", action="store_true",
                    help="skip the pair census (units of the roofline figure)")
    ap.add_argument("--no-legs", action="store_true", help="skip every leg below")
    ap.add_argument("--no-single", action="store_true", help="skip the single-cell leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate leg")
    ap.add_argument("--no-species", action="store_true", help="skip the ten-species leg")
    ap.add_argument("--no-randflux", action="store_true", help="skip the random-flux leg")
    ap.add_argument("--no-tube", action="store_true",
                    help="skip the Dirichlet-tube leg (source term and cylindrical wall)")
    ap.add_argument("--no-verlet", action="store_true", help="skip the neighbour-list leg")
    ap.add_argument("--verlet", default="0.6,5", metavar="SKIN,EVERY",
                    help="skin and rebuild interval of the neighbour-list leg")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device-to-device with torch (a plain "
                         "copy of known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the library has no "
                                   "multi-GPU path, so --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.no_legs:
        args.no_single = args.no_batched = args.no_surrogate = args.no_species = True
        args.no_randflux = args.no_verlet = args.no_tube = True
    import numpy as np
    import torch
    from paper_1611_06163_amd import tdpd
    if args.kernel is not None:
        os.environ["TDPD_PAIR_KERNEL"] = str(args.kernel)
    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    cfg, desc = workload(args.workload)
    _log(f"{args.workload}: {cfg.n} particles, {len(cfg.rbc_first_gid)} cells, generated in "
         f"{time.perf_counter() - t_gen:.1f} s")
    sysg = tdpd.System(cfg)
    sysg.compute_forces(0)
    if not args.no_autotune:
        sysg.autotune(reps=5)  # before the warm-up: untimed
    n_cand = n_flux = n_force = None
    if not args.no_census:
        n_cand, n_flux, n_force = pair_work(sysg, cfg)
    sysg.step(args.warmup)
    sysg.sync()
    # the timed windows run on the library's default path (captured
    # multi-step graphs), each exactly --steps steps between two device
    # synchronisations; per-phase HIP events need the uncaptured path, so
    # the pair kernel's launches are timed by events over one more window of
    # as many steps right after
    els = [_timed_steps(torch, sysg, args.steps) for _ in range(args.windows)]
    el = float(np.median(els))
    sysg.set_timing(tdpd.PHASE["pair"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sysg.step(args.steps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    sysg.sync()
    pair_ms, pair_n = sysg.get_timing(tdpd.PHASE["pair"])
    sysg.set_timing(0)
    value = cfg.n * args.steps / el
    pair_avg_s = pair_ms / max(pair_n, 1) / 1e3
    roof = {"bound": "alu", "kernel": "pair (forces + fluxes)", "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s", "traffic": pair_traffic(args.workload, sysg.tile),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
            "avg_launch_us": pair_avg_s * 1e6, "launches": pair_n,
            "timing": "HIP events around each pair launch on the library's stream, over one "
                      "more window of the same number of steps (uncaptured path, "
                      f"{(t3 - t2) * 1e3 / args.steps:.4f} ms per step)",
            "ops_per_unit": {"candidate_test": OPS_CANDIDATE, "force_pair": OPS_FORCE,
                             "flux_pair_per_species": OPS_FLUX_PER_SPECIES}}
    if n_cand is not None:
        ops = (OPS_CANDIDATE * n_cand + OPS_FLUX_PER_SPECIES * cfg.n_species * n_flux
               + OPS_FORCE * n_force)
        achieved = ops / pair_avg_s / 1e12
        roof.update(achieved=achieved, frac=achieved / VALU_PEAK_TOPS, ops_per_launch=ops,
                    units_per_launch={"candidate_tests": n_cand, "flux_pairs": n_flux,
                                      "force_pairs": n_force})
    else:
        roof.update(achieved=None, frac=None)
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
        "windows": {"count": args.windows, "steps_each": args.steps,
                    "ms_per_step": [e * 1e3 / args.steps for e in els], "reported": "median"},
        "roofline": roof,
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
    single = None
    if not args.no_single or not args.no_species or not args.no_randflux:
        c2, c2desc = workload("c2")
        single = plain_leg(torch, tdpd, c2, c2desc, steps=200, warmup=20, windows=5)
        out["single_rbc"] = single
    if not args.no_batched:
        out["batched"] = batched_leg(torch, tdpd, steps=20, warmup=5)
    if not args.no_verlet:
        skin, every = args.verlet.split(",")
        try:
            vl = verlet_leg(torch, tdpd, steps=200, warmup=20, wl="c2", skin=float(skin),
                            every=int(every))
            vl["vs_cells"] = vl["value"] / single["value"] if single else None
        except tdpd.TdpdError as e:  # e.g. the skin was too small for the interval
            vl = {"skin": float(skin), "every": int(every), "error": str(e)}
        out["verlet"] = vl
    if not args.no_species:
        sp = species_leg(torch, tdpd, steps=200, warmup=20)
        sp["vs_two_species"] = sp["value"] / single["value"]
        out["species"] = sp
    if not args.no_randflux:
        from paper_1611_06163_amd import inputs as I
        cr = I.c2()
        cr.m_s = 0.05
        rf = plain_leg(torch, tdpd, cr, "single RBC box with the random flux of Eqs. (9)-(10) "
                                        "(m_s = 0.05)", steps=200, warmup=20, windows=5)
        rf["vs_without"] = rf["value"] / single["value"]
        out["random_flux"] = rf
    if not args.no_tube:
        from paper_1611_06163_amd import inputs as I
        ct = I.cylinder(radius=20.0, length=80.0, rho=4.0, seed=23, moving=True)
        ct.source = np.zeros((1, ct.n_types))
        ct.decay = np.zeros((1, ct.n_types))
        ct.decay[0, I.T_SOLVENT] = 0.05  # a first-order reaction in the fluid (Q^S)
        tl = plain_leg(torch, tdpd, ct, "tube of radius 20, length 80, density 4 with a "
                                        "Dirichlet wall of held particles and a first-order "
                                        "reaction (Eqs. 7, 20)", steps=100, warmup=10, windows=3)
        out["tube"] = tl
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(torch, tdpd, steps=100, warmup=10, cfg=cfg, desc=desc)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
