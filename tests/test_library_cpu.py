"""CPU checks of the HIP library: it loads, exports the C ABI, and its host-side
setup (reference operators, geometry, connectivity, PML classification) agrees
with the independent oracle.  No kernels are launched."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2006_02551_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wdg.h")

wdg = pytest.importorskip("paper_2006_02551_amd.wdg", reason="libwdg.so not built")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(wdg_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", wdg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (wdg_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(wdg._lib, n)
    assert wdg.wdg_version() >= 10000


def _ctx(cfg, **kw):
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    return wdg.Context(vx, ev, cfg["N"], rule, cfg["pml"], host_only=True, **kw), vx, ev, rule


@pytest.mark.parametrize("over", [{}, {"N": 3, "cub_degree": 6, "mesh.perturb": 0.1},
                                  {"N": 1, "cub_degree": 2, "mesh.n": 3},
                                  {"N": 4, "cub_degree": 8, "mesh.n": 2, "pml.kappa_max": 2.0}])
def test_host_setup_matches_oracle(over):
    from oracle.run import Simulation as OSim
    cfg = inputs.config("c1", **over)
    if not os.path.exists(os.path.join(inputs.configs.RULE_DIR, f"tet_deg{cfg['cub_degree']}.txt")):
        pytest.skip("cubature rule not generated")
    ctx, vx, ev, rule = _ctx(cfg)
    osim = OSim(cfg, vx, ev, *rule)
    ref, m = osim.ref, osim.mesh
    pairs = [(wdg.WDG_OP_DR, ref.Dr), (wdg.WDG_OP_DS, ref.Ds), (wdg.WDG_OP_DT, ref.Dt), (wdg.WDG_OP_LIFT, ref.LIFT),
             (wdg.WDG_OP_VQ, ref.Vq), (wdg.WDG_OP_PQ, ref.Pq), (wdg.WDG_OP_M, ref.M)]
    for which, expect in pairs:
        got = ctx.reference_op(which)
        assert np.max(np.abs(got - expect)) <= 1e-12 * max(1.0, np.max(np.abs(expect))), which
    info = ctx.element_info()
    assert np.allclose(info["J"], m.J, rtol=1e-14, atol=0)
    assert np.allclose(info["Fscale"], m.Fscale, rtol=1e-13, atol=0)
    assert np.allclose(info["normals"], m.nrm, atol=1e-14)
    assert np.array_equal(info["etoe"], m.EToE) and np.array_equal(info["etof"], m.EToF)
    assert np.array_equal(info["is_pml"], osim.op.is_pml)
    assert np.allclose(ctx.node_coords(), m.x, atol=1e-14)
    assert abs(ctx.dims.dt_unit * cfg["cfl"] - osim.dt) < 1e-15
    d = ctx.dims
    assert d.K == m.K and d.K_pml == int(osim.op.is_pml.sum())
    assert d.nblk_pml == -(-d.K_pml // d.block)


def test_memory_report_matches_paper_model():
    cfg = inputs.config("c1")
    ctx, *_ = _ctx(cfg)
    d = ctx.dims
    mem = ctx.memory_report()
    # Sec. II-B: direct storage 15 N_p^2 per PML element, WAA 15 N_q per PML element + 2 N_p N_q
    assert mem["paper_direct"] == 15 * d.Np ** 2 * d.K_pml * 8
    assert mem["paper_waa"] == (15 * d.Nq * d.K_pml + 2 * d.Np * d.Nq) * 8
    assert mem["coefficients"] == d.nblk_pml * d.block * 3 * d.Nq * 8


def test_error_paths():
    cfg = inputs.config("c1")
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(6)
    with pytest.raises(wdg.WdgError) as e:
        wdg.Context(vx, ev[:0], 2, rule, cfg["pml"], host_only=True)
    assert e.value.code == wdg.WDG_EMESH
    with pytest.raises(wdg.WdgError) as e:
        wdg.Context(vx, ev, 7, rule, cfg["pml"], host_only=True)
    assert e.value.code == wdg.WDG_EINVAL
    # a rule of degree 2 is not exact to 2N for N = 2 (P_q V_q != I)
    with pytest.raises(wdg.WdgError) as e:
        wdg.Context(vx, ev, 2, inputs.load_rule(2), cfg["pml"], host_only=True)
    assert e.value.code == wdg.WDG_EINVAL
    # degenerate tetrahedron
    bad = ev.copy()
    bad[0, 3] = bad[0, 2]
    with pytest.raises(wdg.WdgError) as e:
        wdg.Context(vx, bad, 2, rule, cfg["pml"], host_only=True)
    assert e.value.code == wdg.WDG_EMESH
    # a face shared by three tetrahedra
    extra = np.vstack([ev, ev[:1, [0, 1, 2, 3]]])
    with pytest.raises(wdg.WdgError) as e:
        wdg.Context(vx, extra, 2, rule, cfg["pml"], host_only=True)
    assert e.value.code == wdg.WDG_EMESH
    # host-only contexts cannot step
    ctx = wdg.Context(vx, ev, 2, rule, cfg["pml"], host_only=True)
    assert wdg.wdg_step(ctx.h, 0.01, 1, None) == wdg.WDG_ESTATE
    assert wdg.wdg_bind_state(ctx.h, None, None, None, 0) == wdg.WDG_ESTATE
    # schedule modes: forward, reversed, alternating (the default); nothing else
    for mode in (wdg.WDG_SCHEDULE_FORWARD, wdg.WDG_SCHEDULE_REVERSED, wdg.WDG_SCHEDULE_ALTERNATING):
        assert wdg.wdg_set_schedule(ctx.h, mode) == 0
    assert wdg.wdg_set_schedule(ctx.h, 3) == wdg.WDG_EINVAL
    assert wdg.wdg_set_schedule(ctx.h, -1) == wdg.WDG_EINVAL


def test_negative_orientation_is_swapped_like_the_oracle():
    from oracle.run import Simulation as OSim
    cfg = inputs.config("c1")
    vx, ev = inputs.mesh_for(cfg)
    ev2 = ev.copy()
    ev2[::3, 2], ev2[::3, 3] = ev[::3, 3], ev[::3, 2]
    rule = inputs.load_rule(6)
    ctx = wdg.Context(vx, ev2, 2, rule, cfg["pml"], host_only=True)
    osim = OSim(cfg, vx, ev2, *rule)
    assert np.allclose(ctx.node_coords(), osim.mesh.x, atol=1e-14)
    assert np.allclose(ctx.element_info()["J"], osim.mesh.J)


def test_sigma_readout_override_and_cubature_points():
    from oracle.run import Simulation as OSim
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1})
    ctx, vx, ev, rule = _ctx(cfg)
    osim = OSim(cfg, vx, ev, *rule)
    assert np.allclose(ctx.cubature_points(), osim.op.xq, atol=1e-14)
    sig = ctx.get_sigma_q()
    assert np.max(np.abs(sig - osim.op.sigma)) <= 1e-13 * np.max(sig)
    # a valid override round-trips; non-zero sigma outside the PML is refused
    new = sig * 1.5
    ctx.set_sigma_q(new)
    assert np.array_equal(ctx.get_sigma_q(), new)
    bad = new.copy()
    k_int = int(np.nonzero(~osim.op.is_pml)[0][0])
    bad[k_int, 0, 0] = 1.0
    with pytest.raises(wdg.WdgError) as e:
        ctx.set_sigma_q(bad)
    assert e.value.code == wdg.WDG_EINVAL
    bad = new.copy()
    bad[int(osim.op.pml_elems[0]), 0, 1] = np.nan
    with pytest.raises(wdg.WdgError):
        ctx.set_sigma_q(bad)
    assert np.array_equal(ctx.get_sigma_q(), new)


def test_pml_profile_resampling_matches_oracle():
    """wdg_set_pml_profile re-samples sigma with new (sigma_max, L, order), the outer wall fixed: the oracle's
    profile with the interface moved by the change of L gives the same samples."""
    from oracle.pml import sigma_kappa
    from oracle.run import Simulation as OSim
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1})
    ctx, vx, ev, rule = _ctx(cfg)
    osim = OSim(cfg, vx, ev, *rule)
    pml = cfg["pml"]
    smax, L, order = [22.0, 18.0, 25.0], [0.45, 0.48, 0.42], 2.5
    ctx.set_pml_profile(smax, L, order)
    wall_lo = np.asarray(pml["lo"]) - np.asarray(pml["L"])
    wall_hi = np.asarray(pml["hi"]) + np.asarray(pml["L"])
    moved = dict(pml, lo=list(wall_lo + L), hi=list(wall_hi - np.asarray(L)), L=L, sigma_max=smax, order=order)
    want, _ = sigma_kappa(osim.op.xq, moved)
    got = ctx.get_sigma_q()
    assert np.max(np.abs(got - want)) <= 1e-13 * max(smax)
    assert np.max(got[~osim.op.is_pml]) == 0.0
    # the original profile restored exactly
    ctx.set_pml_profile(pml["sigma_max"], pml["L"], pml["order"])
    assert np.max(np.abs(ctx.get_sigma_q() - osim.op.sigma)) <= 1e-13 * max(pml["sigma_max"])
    for bad in (([1.0] * 3, [0.0] * 3, 2.0), ([-1.0] * 3, [0.5] * 3, 2.0), ([1.0] * 3, [0.5] * 3, -1.0),
                ([1.0] * 3, [0.6] * 3, 2.0)):  # the last reaches elements created outside the layer
        with pytest.raises(wdg.WdgError) as e:
            ctx.set_pml_profile(*bad)
        assert e.value.code == wdg.WDG_EINVAL
    assert np.max(np.abs(ctx.get_sigma_q() - osim.op.sigma)) <= 1e-13 * max(pml["sigma_max"])


def test_aligned_components_layout():
    """WDG_ALIGN_COMPONENTS: every simulation of a concatenated batch starts at a block boundary of each class, no
    block holds elements of two simulations, and the per-element setup is unchanged."""
    cfg = inputs.config("c4", batch={"nsim": 5, "n_range": [2, 4], "sigma_range": [10.0, 50.0], "orders": [2, 3],
                                     "seed": 3})
    recipe = inputs.batch_recipe(cfg["batch"])
    meshes = inputs.batch_meshes(cfg, recipe)
    vx, ev, group, offsets = inputs.concat_meshes(meshes)
    rule = inputs.load_rule(cfg["cub_degree"])
    plain = wdg.Context(vx, ev, cfg["N"], rule, cfg["pml"], host_only=True)
    al = wdg.Context(vx, ev, cfg["N"], rule, cfg["pml"], host_only=True, flags=wdg.WDG_ALIGN_COMPONENTS)
    d, B = al.dims, al.dims.block
    slots = al.element_slots()
    assert len(np.unique(slots)) == d.K and slots.min() >= 0 and slots.max() < d.nblk * B
    blk = slots // B
    owner = {}
    for k in range(d.K):
        assert owner.setdefault(int(blk[k]), int(group[k])) == int(group[k])  # one simulation per block
    pml = blk < d.nblk_pml
    for i in range(len(meshes)):
        for cls in (pml, ~pml):
            sel = np.nonzero((group == i) & cls)[0]
            if len(sel):
                assert slots[sel].min() % B == 0  # starts at a block boundary
                assert blk[sel].max() - blk[sel].min() + 1 == (len(sel) + B - 1) // B  # contiguous, dense
    assert d.nblk >= plain.dims.nblk and d.K_pml == plain.dims.K_pml
    assert np.array_equal(al.node_coords(), plain.node_coords())
    assert np.array_equal(al.get_sigma_q(), plain.get_sigma_q())


def test_loss_gradient_needs_device_state():
    cfg = inputs.config("c1")
    ctx, *_ = _ctx(cfg)
    sh = wdg.make_shell({"outer_lo": [-0.5] * 3, "outer_hi": [0.5] * 3, "inner_lo": [-0.4] * 3, "inner_hi": [0.4] * 3})
    import ctypes as C
    loss = C.c_double(0.0)
    assert wdg.wdg_loss_gradient(ctx.h, 0.01, 5, C.byref(sh), 0, C.byref(loss), None, None, None) == wdg.WDG_ESTATE
    assert wdg.wdg_loss_gradient(ctx.h, 0.01, -1, C.byref(sh), 0, C.byref(loss), None, None, None) == wdg.WDG_EINVAL
    assert wdg.wdg_shell_energy(ctx.h, C.byref(sh), C.byref(loss), None) == wdg.WDG_ESTATE


def test_batch_recipe_and_group_profiles():
    cfg = inputs.config("c4", batch={"nsim": 3, "n_range": [2, 3], "sigma_range": [10.0, 50.0], "orders": [2, 3, 4],
                                     "seed": 4})
    rec = inputs.batch_recipe(cfg["batch"])
    assert rec == inputs.batch_recipe(cfg["batch"])  # seeded
    meshes = inputs.batch_meshes(cfg, rec)
    vx, ev, group, offs = inputs.concat_meshes(meshes)
    # disjoint vertex sets per simulation
    for g in range(3):
        used = np.unique(ev[offs[g]:offs[g + 1]])
        assert used.min() >= sum(len(m[0]) for m in meshes[:g]) and used.max() < sum(len(m[0]) for m in meshes[:g + 1])
    rule = inputs.load_rule(cfg["cub_degree"])
    pml = dict(cfg["pml"], sigma_max=[1.0] * 3, order=2.0)
    ctx = wdg.Context(vx, ev, cfg["N"], rule, pml, host_only=True)
    ctx.set_sigma_profile(group, [[r["sigma_max"]] * 3 for r in rec], [r["order"] for r in rec])
    sig = ctx.get_sigma_q()
    for g, r in enumerate(rec):
        alone = wdg.Context(*meshes[g], cfg["N"], rule, dict(cfg["pml"], sigma_max=[r["sigma_max"]] * 3, order=r["order"]),
                            host_only=True)
        assert np.array_equal(sig[offs[g]:offs[g + 1]], alone.get_sigma_q())
        assert np.array_equal(ctx.element_info()["is_pml"][offs[g]:offs[g + 1]], alone.element_info()["is_pml"])
    with pytest.raises(wdg.WdgError):
        ctx.set_sigma_profile(group, [[1.0] * 3], [2.0])  # group index out of range


def test_pml_scheme_errors_on_host_only_context(rules):
    cfg = inputs.config("c1")
    vx, ev = inputs.mesh_for(cfg)
    ctx = wdg.Context(vx, ev, cfg["N"], rules(cfg["cub_degree"]), cfg["pml"], host_only=True)
    # the scheme call lives on Simulation (it needs a device); call the ABI directly
    with pytest.raises(wdg.WdgError) as e:
        wdg._check(wdg.wdg_set_pml_scheme(ctx.h, 9, 0, None, None), ctx.h)
    assert e.value.code == wdg.WDG_EINVAL
    with pytest.raises(wdg.WdgError) as e:
        wdg._check(wdg.wdg_set_pml_scheme(ctx.h, wdg.WDG_PML_CONSTANT, 0, None, None), ctx.h)
    assert e.value.code == wdg.WDG_ESTATE


def test_periodic_connectivity_matches_oracle(rules):
    from oracle.mesh import Mesh
    from oracle.refel import RefElement
    vx, ev, vid = inputs.kuhn_grid((3, 3, 6), [0.0] * 3, [0.3, 0.3, 0.6], 0.15, seed=4, periodic=(True, True, False))
    pml = {"lo": [-1e9, -1e9, 0.1], "hi": [1e9, 1e9, 0.5], "L": [1.0, 1.0, 0.1], "sigma_max": [0.0, 0.0, 5.0],
           "order": 2.0, "kappa_max": 1.0}
    ctx = wdg.Context(vx, ev, 2, rules(4), pml, host_only=True, vertex_id=vid)
    m = Mesh(vx, ev, RefElement(2, *rules(4)), vertex_id=vid)
    info = ctx.element_info()
    assert np.array_equal(info["etoe"], m.EToE) and np.array_equal(info["etof"], m.EToF)
    assert int((info["etoe"] == np.arange(m.K)[:, None]).sum()) == 36  # walls only at the two z ends
    # without the identification the side faces are walls
    plain = wdg.Context(vx, ev, 2, rules(4), pml, host_only=True)
    assert int((plain.element_info()["etoe"] == np.arange(m.K)[:, None]).sum()) > 36
    bad = vid.copy()
    bad[bad == bad[ev[0, 1]]] = bad[ev[0, 0]]
    with pytest.raises(wdg.WdgError):
        wdg.Context(vx, ev, 2, rules(4), pml, host_only=True, vertex_id=bad)
    with pytest.raises(wdg.WdgError):
        wdg.Context(vx, ev, 2, rules(4), pml, host_only=True, vertex_id=np.full(len(vx), len(vx), np.int32))
