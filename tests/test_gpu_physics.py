"""Long GPU runs against what the method fixes: the kinetic temperature of
the tDPD fluid (fluctuation-dissipation, Eq. 6) and of an isolated cell
under its own membrane thermostat (Eqs. 15-16, reading C13), and a relaxed
cell in solvent keeping its rest area and volume (Eqs. 17-18)."""
import numpy as np
import pytest

from gpu_helpers import gpu_system
from oracle import TERM
from paper_1611_06163_amd import inputs as I

pytestmark = pytest.mark.gpu
MEM = TERM["bond"] | TERM["bvisc"] | TERM["brand"] | TERM["area"] | TERM["vol"] | TERM["bend"]


def _mean_kT(g, steps, every, skip):
    g.step(skip)
    kts = []
    for _ in range(steps // every):
        g.step(every)
        kts.append(g.diagnostics()["kT"])
    return float(np.mean(kts)), float(np.std(kts))


def test_fluid_kT_recovery():
    cfg = I.c1()
    g = gpu_system(cfg)
    kt, sd = _mean_kT(g, 5000, 50, 500)
    print("fluid kT", kt, sd, flush=True)
    assert abs(kt - cfg.kT) < 0.02 * cfg.kT


def test_membrane_thermostat_recovers_kT():
    cfg = I._suspension("isolated_cell", (20.0, 20.0, 20.0), 0.0, 1, 21, n_species=1,
                        permeability=(1.0,))
    g = gpu_system(cfg, terms=MEM)
    kt, sd = _mean_kT(g, 20000, 20, 1000)
    print("membrane thermostat kT", kt, sd, flush=True)
    assert abs(kt - cfg.kT) < 0.015 * cfg.kT


def test_relaxed_cell_keeps_rest_area_and_volume():
    """A cell in solvent settles about 0.7 % below its rest area and 0.4 %
    above its rest volume (thermal fluctuations about 0.2 %) and stays
    there: the mean over the run is within 1 % and no sample leaves 1.5 %."""
    cfg = I.c2()
    g = gpu_system(cfg)
    from oracle import Oracle
    info = Oracle(cfg).mesh_info()
    da, dv = [], []
    for _ in range(20):
        g.step(100)
        av = g.diagnostics()["av"][0]
        da.append(av[0] / info["A0"] - 1.0)
        dv.append(av[1] / info["V0"] - 1.0)
    da, dv = np.array(da), np.array(dv)
    print("2000 steps: A/A0 - 1 mean", da.mean(), "max", np.abs(da).max(), "V/V0 - 1 mean",
          dv.mean(), "max", np.abs(dv).max(), flush=True)
    assert abs(da.mean()) < 0.01 and abs(dv.mean()) < 0.01
    assert np.abs(da).max() < 0.015 and np.abs(dv).max() < 0.015
