"""The direct (stored-matrix) and element-constant PML schemes on the GPU against the FP64 oracle.

Direct scheme: the library and the oracle (`oracle.brute`) integrate the weighted mass matrices with
the same input rule, `inputs.product_rule(n)` (two rules of equal polynomial degree give different
values for the interface-cut elements, whose weights have a kink), and both solve with the resulting
matrices, so they agree to rounding (1e-11 relative in FP64).
Element-constant scheme: `oracle.ec` (pointwise closed form).
Both schemes run on either stage kernel (matrix-core by default, scalar-operand on request); the
right-hand-side parity cases check both.
"""
import sys

import numpy as np
import pytest

from paper_2006_02551_amd import inputs

pytestmark = pytest.mark.gpu

RULE_N = 8  # product rule n^3 points on both sides


@pytest.fixture(scope="module")
def wdg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2006_02551_amd import wdg as w
    return w


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ctx(wdg, cfg, precision, scheme):
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], precision)
    sim.set_pml_scheme(scheme, inputs.product_rule(RULE_N) if scheme == wdg.WDG_PML_DIRECT else None)
    if cfg.get("source"):
        sim.set_dipole(cfg["source"])
    return sim, vx, ev, rule


def _oracle(cfg, vx, ev, rule, scheme, elements=None):
    from oracle.brute import BruteOperator
    from oracle.ec import ECOperator
    from oracle.mesh import Mesh
    from oracle.refel import RefElement
    ref = RefElement(cfg["N"], *rule)
    mesh = Mesh(vx, ev, ref)
    if scheme == "direct":
        return BruteOperator(mesh, ref, cfg["pml"], cfg["alpha"], cfg.get("source"), elements=elements,
                             rule=inputs.product_rule(RULE_N))
    return ECOperator(mesh, ref, cfg["pml"], cfg["alpha"], cfg.get("source"))


CASES = [
    ("c1", {"mesh.perturb": 0.1}),
    ("c1", {"N": 1, "cub_degree": 2, "mesh.n": 3, "mesh.perturb": 0.1}),
    ("c1", {"N": 3, "cub_degree": 6, "mesh.n": 3, "mesh.perturb": 0.1}),
    ("c1", {"N": 4, "cub_degree": 8, "mesh.n": 2, "mesh.perturb": 0.1}),
    ("c1", {"pml.kappa_max": 2.0, "mesh.perturb": 0.1}),     # (M^a)^-1 is not the plain inverse mass
    ("c2", {"mesh.n": 5}),                                    # dipole source, cubic profile, N = 3
]


@pytest.mark.parametrize("scheme", ["direct", "ec"])
@pytest.mark.parametrize("name,over", CASES, ids=[str(i) for i in range(len(CASES))])
def test_rhs_parity(wdg, name, over, scheme):
    cfg = inputs.config(name, **over)
    code = wdg.WDG_PML_DIRECT if scheme == "direct" else wdg.WDG_PML_CONSTANT
    _say(f"{scheme} rhs parity {name} {over}")
    op = None
    for precision, tol in ((0, 1e-11), (1, 2e-5)):
        sim, vx, ev, rule = _ctx(wdg, cfg, precision, code)
        assert sim.dims.pml_scheme == code and sim.dims.kernel == wdg.WDG_KERNEL_MFMA
        if op is None:
            op = _oracle(cfg, vx, ev, rule, scheme)
            q = np.random.default_rng(11).standard_normal((sim.dims.K, 12, sim.dims.Np))
            q[~op.is_pml, 6:] = 0.0
            ref = op.rhs(q, 0.57)
            scale = np.max(np.abs(ref))
        sim.set_fields(q)
        for kernel in (wdg.WDG_KERNEL_MFMA, wdg.WDG_KERNEL_SCALAR):
            sim.set_kernel(kernel)
            sim.rhs(0.57)
            err = np.max(np.abs(sim.get_residual() - ref)) / scale
            _say(f"  precision {precision}, kernel {kernel}: {err:.2e}")
            assert err <= tol
        # the two schemes really differ from the weight-adjusted one on this case
        if precision == 0 and cfg["pml"] is not None:
            sim.set_pml_scheme(wdg.WDG_PML_WAA)
            sim.rhs(0.57)
            assert np.max(np.abs(sim.get_residual() - ref)) / scale > 1e-9


@pytest.mark.parametrize("scheme", ["direct", "ec"])
def test_stepping_parity(wdg, scheme):
    from oracle import lserk
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1, "pml.kappa_max": 1.5})
    code = wdg.WDG_PML_DIRECT if scheme == "direct" else wdg.WDG_PML_CONSTANT
    _say(f"{scheme} stepping parity")
    sim, vx, ev, rule = _ctx(wdg, cfg, 0, code)
    op = _oracle(cfg, vx, ev, rule, scheme)
    q = inputs.gaussian_fields(cfg, sim.node_coords())
    sim.set_fields(q)
    dt = cfg["cfl"] * sim.dims.dt_unit
    t = 0.0
    for _ in range(20):
        q = lserk.step(op.rhs, q, t, dt)
        t += dt
    sim.step(dt, 20)
    got = sim.get_fields()
    err = np.linalg.norm(got - q) / np.linalg.norm(q)
    _say(f"  20 steps: relative L2 {err:.2e}")
    assert err <= 1e-12


def test_scheme_data_switching_and_errors(wdg):
    import torch
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1})
    sim, vx, ev, rule = _ctx(wdg, cfg, 0, wdg.WDG_PML_DIRECT)
    d = sim.dims
    mem = sim.memory_report()
    # stored products plus the work buffer of the vacuum right-hand side (6 N_p words per PML slot)
    assert mem["scheme_data"] == d.nblk_pml * d.block * (15 * d.Np * d.Np + 6 * d.Np) * 8
    assert mem["paper_direct"] == 15 * d.Np * d.Np * d.K_pml * 8
    # captured stepping follows the scheme
    q = inputs.gaussian_fields(cfg, sim.node_coords())
    twin, _, _, _ = _ctx(wdg, cfg, 0, wdg.WDG_PML_DIRECT)
    for s in (sim, twin):
        s.set_fields(q)
    dt = cfg["cfl"] * d.dt_unit
    stream = torch.cuda.Stream()
    sim.step_graph(dt, 6, stream)
    twin.step(dt, 6)
    torch.cuda.synchronize()
    assert np.array_equal(sim.get_fields(), twin.get_fields())
    # switching scheme drops the captured graph; element-constant, then back to weight-adjusted
    for code in (wdg.WDG_PML_CONSTANT, wdg.WDG_PML_WAA):
        sim.set_pml_scheme(code)
        twin.set_pml_scheme(code)
        assert sim.memory_report()["scheme_data"] == (d.nblk_pml * d.block * 6 * 8 if code else 0)
        sim.step_graph(dt, 4, stream)
        twin.step(dt, 4)
        torch.cuda.synchronize()
        assert np.array_equal(sim.get_fields(), twin.get_fields()), code
    # every scheme runs on the matrix-core kernel by default
    assert sim.dims.kernel == wdg.WDG_KERNEL_MFMA
    # the autotuner times both kernels for every scheme and leaves the fields alone
    for code in (wdg.WDG_PML_DIRECT, wdg.WDG_PML_CONSTANT, wdg.WDG_PML_WAA):
        sim.set_pml_scheme(code, inputs.product_rule(RULE_N) if code == wdg.WDG_PML_DIRECT else None)
        before = sim.get_fields()
        times = sim.autotune(reps=2)
        assert all(times[k] is not None and times[k] > 0 for k in ("scalar", "mfma_1tile", "mfma_2tiles")), (code, times)
        assert np.array_equal(sim.get_fields(), before)
        sim.set_kernel(wdg.WDG_KERNEL_MFMA)
    sim.set_tiles(2)  # as a fresh context (the tile counts are separately compiled kernels)
    fresh = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], 0)
    fresh.set_fields(q)
    sim.set_fields(q)
    fresh.rhs(0.3)
    sim.rhs(0.3)
    assert np.array_equal(fresh.get_residual(), sim.get_residual())
    # errors
    with pytest.raises(wdg.WdgError):
        sim.set_pml_scheme(7)
    with pytest.raises(wdg.WdgError):
        sim.set_pml_scheme(wdg.WDG_PML_DIRECT, (np.zeros((0, 3)), np.zeros(0)))
    with pytest.raises(wdg.WdgError):
        sim.set_pml_scheme(wdg.WDG_PML_DIRECT, (np.full((4, 3), np.nan), np.ones(4)))
    sim.set_pml_scheme(wdg.WDG_PML_CONSTANT)
    with pytest.raises(wdg.WdgError):
        sim.set_sigma_q(sim.get_sigma_q())          # sigma samples belong to the weight-adjusted scheme
    with pytest.raises(wdg.WdgError):
        sim.loss_gradient(dt, 2, inputs.config("c5")["shell"])
    sim.set_pml_scheme(wdg.WDG_PML_WAA)
    sim.set_sigma_q(sim.get_sigma_q())
    with pytest.raises(wdg.WdgError):
        sim.set_pml_scheme(wdg.WDG_PML_CONSTANT)    # the samples no longer follow the method's profile


def test_c2_full_size_direct_sampled(wdg):
    # the 48,000-tet N=3 workload (37,632 PML elements, 1.8 GB of stored matrices in FP64):
    # the right-hand side of sampled PML and interior elements against the oracle
    cfg = inputs.config("c2")
    _say("c2 direct scheme setup")
    sim, vx, ev, rule = _ctx(wdg, cfg, 0, wdg.WDG_PML_DIRECT)
    info = sim.element_info()
    rng = np.random.default_rng(2)
    pml = np.nonzero(info["is_pml"])[0]
    el = np.unique(np.concatenate([rng.choice(pml, 150, replace=False), rng.choice(sim.dims.K, 50, replace=False),
                                   pml[:5], pml[-5:]]))
    op = _oracle(cfg, vx, ev, rule, "direct", elements=el)
    q = rng.standard_normal((sim.dims.K, 12, sim.dims.Np))
    q[~op.is_pml, 6:] = 0.0
    ref = op.rhs(q, 0.9, el=el)
    sim.set_fields(q)
    sim.rhs(0.9)
    err = np.max(np.abs(sim.get_residual()[el] - ref)) / np.max(np.abs(ref))
    _say(f"  {len(el)} sampled elements: {err:.2e}")
    assert err <= 1e-11
