"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Tolerances: FP64 results agree with the oracle to 1e-12 relative (max norm of
a right-hand side relative to its largest entry; L2 norm of states after many
steps); FP32 stepping agrees with the FP64 oracle to 1e-5 relative L2.
"""
import sys

import numpy as np
import pytest

from paper_2006_02551_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wdg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2006_02551_amd import wdg as w
    return w


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


KERNELS = [0, 1]  # WDG_KERNEL_AUTO (matrix cores where available), WDG_KERNEL_SCALAR


def _pair(wdg, cfg, precision=0, init="gaussian", seed=0, kernel=0):
    from oracle.run import Simulation as OSim
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], precision)
    sim.set_kernel(kernel)
    osim = OSim(cfg, vx, ev, *rule)
    if init == "gaussian":
        q0 = inputs.gaussian_fields(cfg, osim.mesh.x)
    else:
        q0 = np.random.default_rng(seed).standard_normal((osim.mesh.K, 12, osim.ref.Np))
    q0[~osim.op.is_pml, 6:] = 0.0
    if cfg.get("source"):
        sim.set_dipole(cfg["source"])
    sim.set_fields(q0)
    osim.set_state(q0)
    return sim, osim


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


RHS_CASES = [
    ("c1", {}),
    ("c1", {"N": 1, "cub_degree": 2, "mesh.n": 3}),
    ("c1", {"N": 3, "cub_degree": 6, "mesh.n": 3, "mesh.perturb": 0.1}),
    ("c1", {"N": 4, "cub_degree": 8, "mesh.n": 2}),
    ("c1", {"pml.kappa_max": 2.0, "mesh.perturb": 0.1}),          # non-trivial a^{-1} sandwich
    ("c1", {"N": 1, "cub_degree": 2, "mesh.n": 3, "pml.kappa_max": 2.0}),
    ("c1", {"N": 3, "cub_degree": 6, "mesh.n": 3, "mesh.perturb": 0.1, "pml.kappa_max": 2.0}),
    ("c1", {"N": 4, "cub_degree": 8, "mesh.n": 2, "mesh.perturb": 0.1, "pml.kappa_max": 2.0}),
    ("c1", {"alpha": 0.0, "mesh.n": 3}),                             # central flux
    ("c1", {"pml": None}),                                           # no PML at all
    ("c1", {"pml.lo": [0.0] * 3, "pml.hi": [0.0] * 3, "pml.L": [1.0] * 3}),  # all elements PML
    ("c2", {"mesh.n": 5}),                                           # dipole source, cubic profile
]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name,over", RHS_CASES, ids=[str(i) for i in range(len(RHS_CASES))])
def test_rhs_parity_fp64(wdg, name, over, kernel):
    cfg = inputs.config(name, **over)
    _say(f"rhs parity {name} {over} kernel {kernel}")
    sim, osim = _pair(wdg, cfg, init="random", seed=3, kernel=kernel)
    if kernel == 0:  # matrix cores at every order (FP64 at N = 4 with one tile per workgroup)
        assert sim.dims.kernel == wdg.WDG_KERNEL_MFMA
    t = 0.61
    sim.rhs(t)
    got = sim.get_residual()
    ref = osim.op.rhs(osim.q, t)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale, np.max(np.abs(got - ref)) / scale
    # fields untouched
    assert np.array_equal(sim.get_fields(), osim.q)


KAPPA_CASES = [i for i, (_, over) in enumerate(RHS_CASES) if over.get("pml.kappa_max", 1.0) != 1.0]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("case", KAPPA_CASES + [0, 8, 11])
def test_rhs_parity_fp32(wdg, case, kernel):
    # FP32 stage arithmetic against the FP64 oracle: max-norm error <= 1e-5 of the largest entry
    name, over = RHS_CASES[case]
    cfg = inputs.config(name, **over)
    _say(f"rhs parity fp32 {name} {over} kernel {kernel}")
    sim, osim = _pair(wdg, cfg, precision=1, init="random", seed=3, kernel=kernel)
    t = 0.61
    sim.rhs(t)
    got = sim.get_residual()
    ref = osim.op.rhs(osim.q, t)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / scale
    _say(f"  fp32 rhs max error {err:.3e} of the largest entry")
    assert err <= 1e-5


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_graded_kappa_100_steps(wdg, kernel, precision, tol):
    # kappa_max = 2 (Sec. III's graded stretching): the a^-1 sandwich of eq. (21) is not the identity
    cfg = inputs.config("c1", **{"pml.kappa_max": 2.0, "mesh.perturb": 0.1})
    _say(f"kappa_max 2, 100 steps, precision {precision} kernel {kernel}")
    sim, osim = _pair(wdg, cfg, precision=precision, kernel=kernel)
    sim.step(osim.dt, 100)
    osim.run(100)
    q = sim.get_fields()
    assert np.max(np.abs(osim.q[:, 6:])) > 1e-3 * np.max(np.abs(osim.q[:, :6]))  # the layer is active
    assert _rel_l2(q[:, :6], osim.q[:, :6]) <= tol
    assert _rel_l2(q[:, 6:], osim.q[:, 6:]) <= tol


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("precision", [0, 1])
def test_waa_shortcut_is_opt_in(wdg, kernel, precision):
    # the weight-adjusted inverse runs by default; skipping it where it is the identity changes only rounding
    cfg = inputs.config("c2", **{"mesh.n": 5})
    _say(f"weight-adjusted inverse shortcut, precision {precision} kernel {kernel}")
    sim, osim = _pair(wdg, cfg, precision=precision, init="random", seed=4, kernel=kernel)
    sim.rhs(0.4)
    full = sim.get_residual()
    sim.set_waa_shortcut(True)
    sim.rhs(0.4)
    short = sim.get_residual()
    sim.set_waa_shortcut(False)
    sim.rhs(0.4)
    assert np.array_equal(sim.get_residual(), full)
    tol = 1e-13 if precision == 0 else 1e-5
    assert np.max(np.abs(full - short)) <= tol * np.max(np.abs(full))
    assert not np.array_equal(full, short)  # the default really applies the products
    kap = inputs.config("c1", **{"pml.kappa_max": 2.0, "mesh.n": 2})
    ksim, _ = _pair(wdg, kap, precision=precision, kernel=kernel)
    with pytest.raises(wdg.WdgError) as e:
        ksim.set_waa_shortcut(True)
    assert e.value.code == wdg.WDG_EINVAL


@pytest.mark.parametrize("kernel", KERNELS)
def test_c1_100_steps_fp64(wdg, kernel):
    cfg = inputs.config("c1")
    _say(f"c1 100 steps fp64 kernel {kernel}")
    sim, osim = _pair(wdg, cfg, kernel=kernel)
    e0 = sim.energy()
    assert abs(e0 - osim.energy()) <= 1e-13 * e0
    sim.step(osim.dt, 100)
    osim.run(100)
    q = sim.get_fields()
    assert _rel_l2(q[:, :6], osim.q[:, :6]) <= 1e-12
    assert _rel_l2(q[:, 6:], osim.q[:, 6:]) <= 1e-12
    e = sim.energy()
    assert abs(e - osim.energy()) <= 1e-12 * e
    assert e < e0
    d = sim.get_dims()
    assert d.steps == 100 and abs(d.time - 100 * osim.dt) < 1e-12


def test_c2_small_probes_fp64(wdg):
    cfg = inputs.config("c2", **{"mesh.n": 6})
    _say("c2 small probes fp64")
    sim, osim = _pair(wdg, cfg)
    sim.set_probes(np.asarray(cfg["probes"]), 64)
    steps = 40
    sim.step(osim.dt, steps)
    rows = osim.run(steps, record_probes=True)
    got = sim.probe_read(64)
    assert got.shape == rows.shape == (steps, 8, 6)
    assert np.max(np.abs(got - rows)) <= 1e-12 * np.max(np.abs(rows))
    q = sim.get_fields()
    assert _rel_l2(q[:, :6], osim.q[:, :6]) <= 1e-12
    assert np.max(np.abs(osim.q[:, :6])) > 0  # the source has radiated


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name,over,steps", [("c1", {}, 100), ("c2", {"mesh.n": 6}, 40),
                                             ("c1", {"N": 4, "cub_degree": 8, "mesh.n": 2}, 30)])
def test_fp32_against_fp64_oracle(wdg, name, over, steps, kernel):
    cfg = inputs.config(name, **over)
    _say(f"fp32 {name} {over} kernel {kernel}")
    sim, osim = _pair(wdg, cfg, precision=1, kernel=kernel)
    sim.step(osim.dt, steps)
    osim.run(steps)
    q = sim.get_fields()
    err = _rel_l2(q[:, :6], osim.q[:, :6])
    _say(f"  fp32 relative L2 error {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_c2_full_size_rhs_sampled(wdg, precision, tol):
    # The 48,000-tet N=3 mesh in the launch configuration the benchmark times;
    # the oracle evaluates the right-hand side of a sample of elements only.
    cfg = inputs.config("c2")
    _say(f"c2 full size sampled rhs precision {precision}")
    sim, osim = _pair(wdg, cfg, init="random", seed=11, precision=precision)
    t = 0.9
    sim.rhs(t)
    got = sim.get_residual()
    rng = np.random.default_rng(5)
    el = np.unique(np.concatenate([rng.choice(osim.mesh.K, 400, replace=False), osim.op.pml_elems[:50],
                                   np.nonzero(~osim.op.is_pml)[0][:50], [0, osim.mesh.K - 1]]))
    ref = osim.op.rhs(osim.q, t, el=el)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got[el] - ref)) <= tol * scale


def test_kernels_agree(wdg):
    # the two stage-kernel variants compute the same stage (to FP64 rounding)
    cfg = inputs.config("c2", **{"mesh.n": 5})
    _say("kernel variants agree")
    sim, osim = _pair(wdg, cfg, init="random", seed=2, kernel=1)
    sim.rhs(0.7)
    a = sim.get_residual()
    sim.set_kernel(2)
    sim.rhs(0.7)
    b = sim.get_residual()
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_determinism_and_restart(wdg):
    cfg = inputs.config("c2", **{"mesh.n": 4})
    _say("determinism and restart")
    for precision in (0, 1):
        sim, osim = _pair(wdg, cfg, precision=precision)
        dt = osim.dt
        q0 = osim.q.copy()
        sim.step(dt, 10)
        mid = sim.get_fields()
        mid_t = sim.get_dims().time
        sim.step(dt, 10)
        a = sim.get_fields()
        # same run again from scratch
        sim.set_fields(q0)
        sim.set_time(0.0)
        sim.step(dt, 20)
        b = sim.get_fields()
        assert np.array_equal(a, b)
        # restart from the checkpoint taken after 10 steps
        sim.set_fields(mid)  # FP32 states round-trip through FP64 exactly
        sim.set_time(mid_t)
        sim.step(dt, 10)
        assert np.array_equal(a, sim.get_fields())


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kernel", KERNELS)
def test_schedule_permutation_is_bitwise_neutral(wdg, precision, kernel):
    """Workgroups taking the tiles in natural, reversed or alternating order (the default) give bitwise-identical
    states (no cross-element read-after-write hazard: each stage reads q_in and writes its own rows of q_out and
    the residual)."""
    cfg = inputs.config("c2", **{"mesh.n": 6})
    _say(f"schedule permutation: precision {precision} kernel {kernel}")
    modes = (wdg.WDG_SCHEDULE_FORWARD, wdg.WDG_SCHEDULE_REVERSED, wdg.WDG_SCHEDULE_ALTERNATING)
    out = []
    for mode in modes:
        sim, osim = _pair(wdg, cfg, precision=precision, kernel=kernel)
        sim.set_schedule(mode)
        sim.step(osim.dt, 12)
        out.append(sim.get_fields())
    assert all(np.array_equal(out[0], o) for o in out[1:])
    if kernel == 0:  # the direct scheme's second launch too
        out = []
        for mode in modes:
            sim, osim = _pair(wdg, cfg, precision=precision, kernel=kernel)
            sim.set_pml_scheme(wdg.WDG_PML_DIRECT, inputs.product_rule(5))
            sim.set_schedule(mode)
            sim.step(osim.dt, 4)
            out.append(sim.get_fields())
        assert all(np.array_equal(out[0], o) for o in out[1:])
    with pytest.raises(wdg.WdgError):
        sim.set_schedule(3)


def test_edge_cases(wdg):
    cfg = inputs.config("c1", **{"mesh.n": 1})  # 6 elements: one partial block per class
    _say("edge cases")
    sim, osim = _pair(wdg, cfg, init="random")
    q = sim.get_fields()
    sim.step(osim.dt, 0)
    assert np.array_equal(sim.get_fields(), q)
    sim.step(osim.dt, 3)
    osim.run(3)
    assert _rel_l2(sim.get_fields(), osim.q) <= 1e-12
    # probe buffer overflow is refused before anything is enqueued
    sim.set_probes(np.zeros((1, 3)), 2)
    with pytest.raises(wdg.WdgError) as e:
        sim.step(osim.dt, 3)
    assert e.value.code == wdg.WDG_EPROBE
    with pytest.raises(wdg.WdgError) as e:
        sim.set_probes(np.array([[5.0, 5.0, 5.0]]), 2)
    assert e.value.code == wdg.WDG_EPROBE
    # non-finite fields are reported by the energy readout
    bad = q.copy()
    bad[0, 0, 0] = np.nan
    sim.set_fields(bad)
    with pytest.raises(wdg.WdgError) as e:
        sim.energy()
    assert e.value.code == wdg.WDG_ENONFINITE
    # state buffers must be 16-byte aligned; a refused bind keeps the buffers already bound
    import ctypes
    import torch
    spare = torch.empty(sim.dims.state_bytes + 64, dtype=torch.uint8, device="cuda")
    p = ctypes.c_void_p(spare.data_ptr() + 8)
    assert wdg.wdg_bind_state(sim.h, p, p, p, sim.dims.state_bytes) == wdg.WDG_EINVAL
    assert "aligned" in wdg.wdg_last_error(sim.h).decode()
    assert np.array_equal(sim.get_fields(), bad, equal_nan=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_watchdog_after_a_time_step_beyond_the_stability_bound(wdg, precision):
    """The vacuum cavity of the oracle's stability pin: at the dt rule the library follows the oracle and the
    energy stays below its start; at fifty times that step the fields overflow and the energy readout returns
    WDG_ENONFINITE (every kernel runs to its end: the condition is only in the data)."""
    cfg = inputs.config("c1", **{"mesh.n": 2, "mesh.perturb": 0.1, "pml.lo": [-1.0] * 3, "pml.hi": [1.0] * 3})
    _say(f"watchdog beyond the stability bound, precision {precision}")
    sim, osim = _pair(wdg, cfg, precision=precision, init="random", seed=7)
    e0 = sim.energy()
    sim.step(osim.dt, 30)
    osim.run(30)
    assert _rel_l2(sim.get_fields(), osim.q) <= (1e-12 if precision == 0 else 1e-5)
    assert sim.energy() <= e0
    code = None
    for _ in range(40):
        sim.step(50 * osim.dt, 5)
        try:
            sim.energy()
        except wdg.WdgError as e:
            code = e.code
            break
    assert code == wdg.WDG_ENONFINITE


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kernel", KERNELS)
def test_stale_residual_is_not_read(wdg, precision, kernel):
    """The first LSERK stage (A_1 = 0) and the right-hand side must not read the residual
    buffer: NaN left there changes nothing, bitwise (the kernels may load it, but not use it)."""
    import torch
    cfg = inputs.config("c1", **{"mesh.n": 2})
    _say(f"stale residual: precision {precision} kernel {kernel}")
    clean, osim = _pair(wdg, cfg, precision=precision, init="random", kernel=kernel)
    dirty, _ = _pair(wdg, cfg, precision=precision, init="random", kernel=kernel)
    dt = osim.dt
    for sim in (clean, dirty):
        sim.rhs(0.0)
    torch.cuda.synchronize()
    dirty.bufs[2].fill_(255)  # all-ones bytes: NaN in either precision
    dirty.rhs(0.0)
    torch.cuda.synchronize()
    assert np.array_equal(dirty.get_residual(), clean.get_residual())
    for sim in (clean, dirty):
        sim.set_fields(osim.q)
    dirty.bufs[2].fill_(255)
    clean.step(dt, 1)
    dirty.step(dt, 1)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(dirty.get_fields()))
    assert np.array_equal(dirty.get_fields(), clean.get_fields())
