"""The allocation-free energy readout against wdg_energy, through the C ABI (GPU).

Two calls in a row on one GPU, the second on a smaller mesh (fewer blocks than the first left in the shared
scratch array): each must equal wdg_energy of the same fields bit for bit (same kernels, same summation order).
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2006_02551_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sim(wdg, name, precision, **over):
    cfg = inputs.config(name, **over)
    vx, ev = inputs.mesh_for(cfg)
    sim = wdg.Simulation(vx, ev, cfg["N"], inputs.load_rule(cfg["cub_degree"]), cfg["pml"], cfg["alpha"], precision)
    q = np.random.default_rng(7).standard_normal((sim.dims.K, 12, sim.dims.Np))
    sim.set_fields(q)
    return sim


@pytest.mark.parametrize("precision", [0, 1])
def test_energy_noalloc_matches_energy(precision):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2006_02551_amd import wdg
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for name, over in (("c2", {"mesh.n": 8}), ("c1", {"mesh.n": 3})):  # the second has fewer blocks
        sim = _sim(wdg, name, precision, **over)
        _say(f"energy_noalloc: {name} {over}, precision {precision}, {sim.dims.nblk} blocks")
        want = sim.energy()
        rc = wdg.wdg_energy_noalloc(sim.h, C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream))
        assert rc == wdg.WDG_OK, wdg.wdg_last_error(sim.h)
        torch.cuda.synchronize()
        got = out[0].item()
        assert got == want, (got, want)
        assert np.isnan(out[1].item())  # only the first double is written
        sim.step(1e-3, 2)  # the fields change; the readout follows
        want = sim.energy()
        assert wdg.wdg_energy_noalloc(sim.h, C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream)) == wdg.WDG_OK
        torch.cuda.synchronize()
        assert out[0].item() == want
        del sim


def test_energy_noalloc_errors():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2006_02551_amd import wdg
    sim = _sim(wdg, "c1", 0, **{"mesh.n": 2})
    assert wdg.wdg_energy_noalloc(sim.h, None, None) == wdg.WDG_EINVAL
    assert wdg.wdg_energy_noalloc(None, None, None) == wdg.WDG_EINVAL
