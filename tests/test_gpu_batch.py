"""The batching form on the GPU: independent simulations in one context (one
launch per stage), captured stepping and the stage-kernel autotuner.

Every simulation of a batch must reproduce its standalone run bit for bit
(disjoint meshes, per-simulation profile and time step, and element-local
arithmetic in every kernel).
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


def _standalone(wdg, b, i, precision, q0, nsteps):
    vx, ev = b.meshes[i]
    sim = wdg.Simulation(vx, ev, b.cfg["N"], b.rule, b.standalone_pml(i), b.cfg["alpha"], precision)
    sim.set_fields(q0)
    sim.step(float(b.dt[i]), nsteps)
    return sim.get_fields()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_standalone_runs(wdg, precision):
    from paper_2006_02551_amd.batch import Batch
    cfg = inputs.config("c4", batch={"nsim": 4, "n_range": [3, 5], "sigma_range": [10.0, 50.0], "orders": [2, 3, 4],
                                     "seed": 1})
    _say(f"batch of 4, precision {precision}")
    b = Batch(cfg, precision)
    q0 = b.initial_fields()
    nsteps = 12
    for graph in (False, True):
        b.set_fields(q0)
        b.step(nsteps, graph=graph)
        q = b.sim.get_fields()
        for i in range(4):
            ref = _standalone(wdg, b, i, precision, b.fields(i, q0), nsteps)
            assert np.array_equal(b.fields(i, q), ref), (graph, i)
    assert len(set(np.round(b.dt, 12))) > 1  # the simulations really run at different steps


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_batch_members_match_oracle(wdg, precision, tol):
    """Each simulation of a stepped batch against the oracle run with its own mesh, profile and time step."""
    from oracle.run import Simulation as OSim
    from paper_2006_02551_amd.batch import Batch
    cfg = inputs.config("c4", batch={"nsim": 4, "n_range": [3, 5], "sigma_range": [10.0, 50.0], "orders": [2, 3, 4],
                                     "seed": 1})
    _say(f"batch of 4 against the oracle, precision {precision}")
    b = Batch(cfg, precision)
    nsteps = 30
    q0 = b.initial_fields()
    b.set_fields(q0)
    b.step(nsteps, graph=True)
    q = b.sim.get_fields()
    for i in range(4):
        vx, ev = b.meshes[i]
        ocfg = dict(cfg, pml=b.standalone_pml(i))
        osim = OSim(ocfg, vx, ev, *b.rule)
        assert abs(osim.dt - b.dt[i]) <= 1e-14 * osim.dt
        osim.set_state(inputs.gaussian_fields(ocfg, osim.mesh.x))
        osim.run(nsteps)
        got = b.fields(i, q)
        for sl in (slice(0, 6), slice(6, 12)):
            err = np.linalg.norm(got[:, sl] - osim.q[:, sl]) / np.linalg.norm(osim.q[:, sl])
            _say(f"  simulation {i} (K = {osim.mesh.K}, sigma_max {b.recipe[i]['sigma_max']:.1f}, order "
                 f"{b.recipe[i]['order']}), components {sl.start}..{sl.stop - 1}: relative L2 error {err:.2e}")
            assert err <= tol


def test_autotune_cache_and_environment_overrides(wdg, tmp_path, monkeypatch):
    cfg = inputs.config("c2", **{"mesh.n": 5})
    _say("autotune cache and WDG_* overrides")
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("WDG_AUTOTUNE_CACHE", str(cache))

    def make():
        sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], wdg.WDG_FP32)
        sim.set_fields(np.zeros((sim.dims.K, 12, sim.dims.Np)))
        return sim
    a = make()
    first = a.autotune_cached(reps=3)
    b = make()
    assert b.autotune_cached(reps=3)  # same architecture, order, rule, precision, scheme and size class
    assert (b.dims.kernel, b.dims.tiles) == (a.dims.kernel, a.dims.tiles)
    if not first:
        lines = cache.read_text().split("\n")
        assert any(line.startswith("gfx") and "/N3/q24/f32/" in line for line in lines), lines
    monkeypatch.setenv("WDG_KERNEL", "scalar")
    assert make().dims.kernel == wdg.WDG_KERNEL_SCALAR
    monkeypatch.setenv("WDG_KERNEL", "mfma")
    monkeypatch.setenv("WDG_TILES", "1")
    s = make()
    assert s.dims.kernel == wdg.WDG_KERNEL_MFMA and s.dims.tiles == 1
    monkeypatch.setenv("WDG_TILES", "3")
    with pytest.raises(wdg.WdgError):
        make()
    monkeypatch.delenv("WDG_TILES")
    monkeypatch.setenv("WDG_KERNEL", "fastest")
    with pytest.raises(wdg.WdgError):
        make()


@pytest.mark.parametrize("precision", [0, 1])
def test_grouped_capture_is_bitwise_equal(wdg, precision):
    """Step groups (aligned components, both steps of a pair group after group) change no bit of any field."""
    from paper_2006_02551_amd.batch import Batch
    cfg = inputs.config("c4", batch={"nsim": 6, "n_range": [3, 6], "sigma_range": [10.0, 50.0], "orders": [2, 3, 4],
                                     "seed": 2})
    _say(f"grouped capture, precision {precision}")
    plain = Batch(cfg, precision)
    grouped = Batch(cfg, precision, group_mb=1.0)
    assert grouped.step_groups is not None and grouped.step_groups.max() >= 2  # several groups
    q0 = plain.initial_fields()
    assert np.array_equal(q0, grouped.initial_fields())
    for b in (plain, grouped):
        b.set_fields(q0)
    plain.step(10, graph=False)   # eager, one launch per stage over every block
    grouped.step(10, graph=True)  # captured, group after group
    assert np.array_equal(grouped.sim.get_fields(), plain.sim.get_fields())
    grouped.step(3, graph=True)   # an odd last step runs eagerly
    plain.step(3, graph=True)
    assert np.array_equal(grouped.sim.get_fields(), plain.sim.get_fields())
    d = grouped.sim.get_dims()
    assert d.steps == 13
    # groups must not split a simulation, and need an aligned context
    bad = grouped.step_groups[grouped.group].copy()
    bad[0] = bad[-1]
    with pytest.raises(wdg.WdgError):
        grouped.sim.set_step_groups(bad)
    with pytest.raises(wdg.WdgError) as e:
        plain.sim.set_step_groups(np.zeros(plain.K, np.int32))
    assert e.value.code == wdg.WDG_ESTATE


def test_graph_replay_matches_eager(wdg):
    import torch
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1})
    _say("graph replay")
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    dt = cfg["cfl"]
    sims = [wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], 0) for _ in range(2)]
    q0 = inputs.gaussian_fields(cfg, sims[0].node_coords())
    dt = cfg["cfl"] * sims[0].dims.dt_unit
    for s in sims:
        s.set_fields(q0)
    stream = torch.cuda.Stream()
    # replays interleaved with eager work on the same context and host synchronisations
    plan = [4, 1, 6, 3, 2]
    for n in plan:
        torch.cuda.synchronize()
        sims[0].step(dt, n)
        with torch.cuda.stream(stream):
            sims[1].step_graph(dt, n, stream)
        torch.cuda.synchronize()
        assert np.array_equal(sims[1].get_fields(), sims[0].get_fields()), n
        sims[1].step(dt, 1)          # eager work on the graph's context between replays
        sims[0].step(dt, 1)
        e1, e0 = sims[1].energy(), sims[0].energy()
        assert e1 == e0
    d0, d1 = sims[0].get_dims(), sims[1].get_dims()
    assert d0.steps == d1.steps and d0.time == d1.time
    # a new dt is captured again
    with torch.cuda.stream(stream):
        sims[1].step_graph(0.5 * dt, 4, stream)
    sims[0].step(0.5 * dt, 4)
    torch.cuda.synchronize()
    assert np.array_equal(sims[1].get_fields(), sims[0].get_fields())
    # refused with a source or on the null stream
    with pytest.raises(wdg.WdgError):
        sims[1].step_graph(dt, 2, torch.cuda.default_stream())
    sims[1].set_dipole(inputs.config("c2")["source"])
    with pytest.raises(wdg.WdgError):
        sims[1].step_graph(dt, 2, stream)


def test_autotune_and_tile_counts(wdg):
    from oracle.run import Simulation as OSim
    cfg = inputs.config("c2", **{"mesh.n": 5})
    _say("autotune")
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    osim = OSim(cfg, vx, ev, *rule)
    q = np.random.default_rng(7).standard_normal((osim.mesh.K, 12, osim.ref.Np))
    q[~osim.op.is_pml, 6:] = 0.0
    ref = osim.op.rhs(q, 0.4)
    for precision in (0, 1):
        sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], precision)
        sim.set_dipole(cfg["source"])
        sim.set_fields(q)
        res = {}
        for tiles in (1, 2):
            sim.set_tiles(tiles)
            assert sim.dims.tiles == tiles
            sim.rhs(0.4)
            res[tiles] = sim.get_residual()
        tol = 1e-12 if precision == 0 else 2e-5
        # element-local arithmetic in the same order: the tile counts agree to rounding (the two are
        # separately compiled, so contractions into fused multiply-adds may differ)
        assert np.max(np.abs(res[1] - res[2])) <= (1e-15 if precision == 0 else 1e-6) * np.max(np.abs(ref))
        assert np.max(np.abs(res[1] - ref)) <= tol * np.max(np.abs(ref))
        before = sim.get_fields()
        times = sim.autotune(reps=3)
        _say(f"  precision {precision}: {times}, chose kernel {sim.dims.kernel} tiles {sim.dims.tiles}")
        assert all(t is not None and t > 0 for t in times.values())
        assert np.array_equal(sim.get_fields(), before)  # autotuning leaves the fields alone
        sim.rhs(0.4)
        assert np.max(np.abs(sim.get_residual() - ref)) <= tol * np.max(np.abs(ref))


def test_c4_full_batch_matches_standalone(wdg):
    # the 32-simulation batch (8^3 x 6 .. 24^3 x 6, 1.28M tets) in FP32 with captured steps;
    # the smallest and the largest simulation are checked against standalone runs
    from paper_2006_02551_amd.batch import Batch
    cfg = inputs.config("c4")
    _say("c4 batch setup")
    b = Batch(cfg, 1)
    q0 = b.initial_fields()
    b.set_fields(q0)
    nsteps = 20
    b.step(nsteps, graph=True)
    q = b.sim.get_fields()
    ns = [r["n"] for r in b.recipe]
    for i in (int(np.argmin(ns)), int(np.argmax(ns))):
        _say(f"  simulation {i} (n = {ns[i]}) against its standalone run")
        ref = _standalone(wdg, b, i, 1, b.fields(i, q0), nsteps)
        assert np.array_equal(b.fields(i, q), ref)
