"""The allocation-free diagnostics entry point against tdpd_diagnostics.

tdpd_diagnostics_noalloc keeps its workgroup partial sums in a library-wide
device scratch and writes to a caller-owned device buffer; it must give the
same bits as tdpd_diagnostics (same kernels, same reduction order), also on
a second call in a row with a smaller system, whose reduction covers fewer
workgroups than the first left in the scratch.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_system
from paper_1611_06163_amd import inputs as I
from paper_1611_06163_amd import tdpd

pytestmark = pytest.mark.gpu


def _noalloc(torch, sysg, n_out):
    out = torch.full((n_out + 8,), float("nan"), dtype=torch.float64, device="cuda")
    sysg.diagnostics_noalloc(out.data_ptr(), n_out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.isnan(got[n_out:]).all(), "wrote past the requested doubles"
    return got[:n_out]


def _flat(d):
    return np.concatenate([d["P"], [d["kT"]], d["C"], d["av"].ravel()])


def test_noalloc_diagnostics_equal_two_calls_smaller_second():
    import torch
    torch.cuda.set_device(0)
    cases = [("channel, 100 cells", I.c3(), 3),
             ("one cell in 12^3", I.small_suspension(seed=3, box=(12.0, 12.0, 12.0), n_cells=1), 2)]
    sizes = []
    for name, cfg, steps in cases:
        sysg = gpu_system(cfg)
        n_out = 4 + cfg.n_species + 2 * len(cfg.rbc_first_gid)
        print(f"case {name}: n={cfg.n} cells={len(cfg.rbc_first_gid)} outputs={n_out}", flush=True)
        sysg.step(steps)
        got = _noalloc(torch, sysg, n_out)
        ref = _flat(sysg.diagnostics())
        assert got.shape == ref.shape
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (name, got, ref)
        sizes.append(cfg.n)
        sysg.close()
    assert sizes[1] < sizes[0]


def test_noalloc_diagnostics_errors():
    import torch
    torch.cuda.set_device(0)
    cfg = I.small_suspension(seed=5, box=(12.0, 12.0, 12.0), n_cells=1)
    sysg = gpu_system(cfg)
    n_out = 4 + cfg.n_species + 2
    buf = torch.zeros(n_out, dtype=torch.float64, device="cuda")
    with pytest.raises(tdpd.TdpdError) as e:  # nothing evaluated yet
        sysg.diagnostics_noalloc(buf.data_ptr(), n_out)
    assert e.value.code == -7  # TDPD_ERR_STATE
    sysg.compute_forces(0)
    with pytest.raises(tdpd.TdpdError) as e:  # one double short
        sysg.diagnostics_noalloc(buf.data_ptr(), n_out - 1)
    assert e.value.code == -9  # TDPD_ERR_CAPACITY
    got = _noalloc(torch, sysg, n_out)
    ref = _flat(sysg.diagnostics())
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    sysg.close()
