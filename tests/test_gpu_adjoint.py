"""GPU parity of the loss-gradient path (through the C ABI) against the FP64
oracle's discrete adjoint (oracle.adjoint), plus finite-difference checks at
the full 48,000-tetrahedron size where the oracle is too slow.

Tolerances: FP64 loss 1e-12 relative, gradients 1e-10 relative to their
largest entry (the per-tile sums over the six components are accumulated with
LDS atomics, so their order, and the last bits, vary between runs); FP32
1e-5 (loss) and 2e-4 (gradient) against the FP64 oracle.
"""
import sys

import numpy as np
import pytest

from paper_2006_02551_amd import inputs

pytestmark = pytest.mark.gpu

SHELL_C1 = {"outer_lo": [-0.5] * 3, "outer_hi": [0.5] * 3, "inner_lo": [-0.3] * 3, "inner_hi": [0.3] * 3}
# the shell 0.1 inside the PML interface of the 48,000-tetrahedron workload
SHELL_C5 = {"outer_lo": [-1.0] * 3, "outer_hi": [1.0] * 3, "inner_lo": [-0.9] * 3, "inner_hi": [0.9] * 3}


@pytest.fixture(scope="module")
def wdg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2006_02551_amd import wdg as w
    return w


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(wdg, cfg, precision=0, seed=0):
    from oracle.run import Simulation as OSim
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], precision)
    osim = OSim(cfg, vx, ev, *rule)
    rng = np.random.default_rng(seed)
    q0 = inputs.gaussian_fields(cfg, osim.mesh.x)
    q0[:, 0:6] += 0.05 * rng.standard_normal(q0[:, 0:6].shape)
    q0[osim.op.is_pml, 6:] = 0.05 * rng.standard_normal((int(osim.op.is_pml.sum()), 6, osim.ref.Np))
    if cfg.get("source"):
        sim.set_dipole(cfg["source"])
    sim.set_fields(q0)
    osim.set_state(q0)
    return sim, osim, q0


def _oracle_grad(osim, q0, nsteps, shell):
    from oracle import adjoint as A
    J, g, _ = A.loss_and_gradient(osim.op, q0, 0.0, osim.dt, nsteps, shell)
    full = np.zeros((osim.mesh.K, osim.ref.Nq, 3))
    full[osim.op.pml_elems] = g
    return J, full, A.profile_gradient(osim.op, _pml(osim.cfg), g)


def _pml(cfg):
    p = dict(cfg["pml"])
    p["order"] = float(p["order"])
    return p


def test_shell_energy_matches_oracle(wdg):
    from oracle import adjoint as A
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1, "init.width": 0.35})
    _say("shell energy")
    for precision, tol in ((0, 1e-13), (1, 1e-6)):
        sim, osim, q0 = _pair(wdg, cfg, precision)
        chi = A.shell_weights(osim.op, SHELL_C1)
        ref = A.shell_energy(osim.op, chi, q0)
        got = sim.shell_energy(SHELL_C1)
        assert ref > 0 and abs(got - ref) <= tol * ref, (precision, got, ref)


def test_shell_energy_with_a_large_rule(wdg):
    """A 125-point rule at N = 3: in FP64 the block's shell indicator does not fit in the shell kernel's LDS beside
    V_q and is read from global memory inside the cubature loop; in FP32 it is staged."""
    from oracle import adjoint as A
    from oracle.run import Simulation as OSim
    cfg = inputs.config("c1", **{"N": 3, "mesh.n": 3, "mesh.perturb": 0.1, "init.width": 0.35})
    rule = inputs.product_rule(5)
    assert len(rule[1]) == 125
    vx, ev = inputs.mesh_for(cfg)
    osim = OSim(cfg, vx, ev, *rule)
    q0 = inputs.gaussian_fields(cfg, osim.mesh.x)
    q0[:, 0:6] += 0.05 * np.random.default_rng(3).standard_normal(q0[:, 0:6].shape)
    osim.set_state(q0)
    chi = A.shell_weights(osim.op, SHELL_C1)
    ref = A.shell_energy(osim.op, chi, osim.q)
    _say("shell energy, 125-point rule")
    for precision, tol in ((0, 1e-13), (1, 1e-6)):
        sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], precision)
        sim.set_fields(q0)
        got = sim.shell_energy(SHELL_C1)
        assert ref > 0 and abs(got - ref) <= tol * ref, (precision, got, ref)


@pytest.mark.parametrize("name,over,nsteps", [
    ("c1", {"mesh.perturb": 0.1, "init.width": 0.35}, 12),            # N = 2, quadratic profile
    ("c2", {"mesh.n": 5, "init": {"component": 2, "center": [0.0] * 3, "width": 0.5}}, 8),  # N = 3, cubic, dipole
], ids=["c1", "c2n5"])
def test_loss_and_gradient_match_oracle_fp64(wdg, name, over, nsteps):
    cfg = inputs.config(name, **over)
    shell = SHELL_C1 if name == "c1" else SHELL_C5
    _say(f"loss gradient fp64 {name} {over} {nsteps} steps")
    sim, osim, q0 = _pair(wdg, cfg, 0)
    J, g, gp = sim.loss_gradient(osim.dt, nsteps, shell)
    Jr, gr, gpr = _oracle_grad(osim, q0, nsteps, shell)
    assert Jr > 0 and abs(J - Jr) <= 1e-12 * Jr, (J, Jr)
    scale = np.max(np.abs(gr))
    assert scale > 0
    assert np.max(np.abs(g - gr)) <= 1e-10 * scale, np.max(np.abs(g - gr)) / scale
    assert np.max(np.abs(gp - gpr)) <= 1e-10 * np.max(np.abs(gpr)), (gp, gpr)
    # the state advanced exactly as plain stepping does
    sim2, _, _ = _pair(wdg, cfg, 0)
    sim2.step(osim.dt, nsteps)
    assert np.array_equal(sim.get_fields(), sim2.get_fields())


@pytest.mark.parametrize("name,over,nsteps", [
    ("c1", {"mesh.perturb": 0.1, "init.width": 0.35}, 12),
    ("c2", {"mesh.n": 5, "init": {"component": 2, "center": [0.0] * 3, "width": 0.5}}, 8),
], ids=["c1", "c2n5"])
def test_loss_and_gradient_fp32_against_fp64_oracle(wdg, name, over, nsteps):
    cfg = inputs.config(name, **over)
    shell = SHELL_C1 if name == "c1" else SHELL_C5
    _say(f"loss gradient fp32 {name} {over} {nsteps} steps")
    sim, osim, q0 = _pair(wdg, cfg, 1)
    J, g, gp = sim.loss_gradient(osim.dt, nsteps, shell)
    Jr, gr, gpr = _oracle_grad(osim, q0, nsteps, shell)
    err_j, err_g = abs(J - Jr) / Jr, np.max(np.abs(g - gr)) / np.max(np.abs(gr))
    _say(f"  fp32 loss error {err_j:.2e}, gradient error {err_g:.2e}")
    assert err_j <= 1e-5 and err_g <= 2e-4


@pytest.mark.parametrize("precision", [0, 1])
def test_adjoint_schedule_permutation(wdg, precision):
    # natural, reversed and alternating tile order: the loss and the final state bitwise equal; the sigma
    # gradient (LDS atomic sums in no fixed order) to rounding
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1, "init.width": 0.35})
    _say(f"adjoint schedule permutation, precision {precision}")
    res = []
    for mode in (wdg.WDG_SCHEDULE_FORWARD, wdg.WDG_SCHEDULE_REVERSED, wdg.WDG_SCHEDULE_ALTERNATING):
        sim, osim, q0 = _pair(wdg, cfg, precision)
        sim.set_schedule(mode)
        J, g, gp = sim.loss_gradient(osim.dt, 10, SHELL_C1)
        res.append((J, g, sim.get_fields()))
    tol = 1e-12 if precision == 0 else 1e-5
    for r in res[1:]:
        assert r[0] == res[0][0]
        assert np.array_equal(r[2], res[0][2])
        assert np.max(np.abs(r[1] - res[0][1])) <= tol * np.max(np.abs(res[0][1]))


def test_checkpoint_interval_and_empty_shell(wdg):
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1, "init.width": 0.35})
    _say("checkpoint intervals")
    res = []
    plain, osim, q0 = _pair(wdg, cfg, 0)
    plain.step(osim.dt, 10)
    want = plain.get_fields()
    for interval in (1, 3, 0, 7, 20):  # 20: one segment, nothing recomputed
        sim, osim, q0 = _pair(wdg, cfg, 0)
        res.append(sim.loss_gradient(osim.dt, 10, SHELL_C1, interval))
        # the state advances exactly as plain stepping (bitwise), whichever segment kept its stage inputs
        assert np.array_equal(sim.get_fields(), want), interval
        assert sim.get_dims().steps == 10
    for J, g, gp in res[1:]:
        assert J == res[0][0]  # the forward sweep is deterministic
        assert np.max(np.abs(g - res[0][1])) <= 1e-13 * np.max(np.abs(res[0][1]))
    sim, osim, q0 = _pair(wdg, cfg, 0)
    empty = {"outer_lo": [5.0] * 3, "outer_hi": [6.0] * 3, "inner_lo": [5.5] * 3, "inner_hi": [5.6] * 3}
    J, g, gp = sim.loss_gradient(osim.dt, 4, empty)
    assert J == 0.0 and not np.any(g) and not np.any(gp)
    assert sim.shell_energy(empty) == 0.0


def test_c5_full_size_gradient_matches_finite_differences(wdg):
    # The differentiation workload: the 48,000-tet N = 3 mesh, 500 steps, a
    # pulse that reaches the layer, the loss in the shell 0.1 inside the PML
    # interface.  The oracle would take hours, so the adjoint gradient is
    # checked against central differences (relative step 1e-6) of the GPU loss.
    cfg = inputs.config("c5")
    shell = cfg["shell"]
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    nsteps = cfg["steps"]
    _say("c5 full size: adjoint vs central differences")
    sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], 0)
    q0 = inputs.gaussian_fields(cfg, sim.node_coords())
    dt = cfg["cfl"] * sim.dims.dt_unit
    sig0 = sim.get_sigma_q()
    sim.set_fields(q0)
    sim.set_time(0.0)
    J, g, gp = sim.loss_gradient(dt, nsteps, shell)
    _say(f"  J = {J:.6e}, dJ/dsigma_max = {gp[:3]}, dJ/dL = {gp[3:6]}, dJ/dp = {gp[6]:.4e}")
    assert J > 0 and np.all(np.isfinite(g)) and np.max(np.abs(gp[:3])) > 0

    def loss_with(sig):
        sim.set_sigma_q(sig)
        sim.set_fields(q0)
        sim.set_time(0.0)
        return sim.loss_gradient(dt, nsteps, shell, profile=False)[0]

    rounding = 100 * np.finfo(float).eps * J
    smax = np.asarray(cfg["pml"]["sigma_max"], float)
    for a in range(3):
        h = 1e-6 * smax[a]
        sp, sm = sig0.copy(), sig0.copy()
        sp[..., a] *= 1.0 + h / smax[a]   # sigma_a is proportional to sigma_max_a
        sm[..., a] *= 1.0 - h / smax[a]
        fd = (loss_with(sp) - loss_with(sm)) / (2 * h)
        _say(f"  axis {a}: adjoint {gp[a]:.10e}  central difference {fd:.10e}  rounding bound {rounding / h:.1e}")
        assert abs(fd - gp[a]) <= 1e-5 * abs(fd) + rounding / h
    # all three sigma_max scaled together: d/de J((1 + e) sigma) = sum_a sigma_max_a dJ/dsigma_max_a,
    # large enough for the rounding bound to be a small fraction of it
    eps = 1e-6
    fd = (loss_with(sig0 * (1 + eps)) - loss_with(sig0 * (1 - eps))) / (2 * eps)
    adj = float(np.dot(smax, gp[:3]))
    _say(f"  uniform scaling: adjoint {adj:.10e}  central difference {fd:.10e}  rounding bound {rounding / eps:.1e}")
    assert rounding / eps < 0.1 * abs(fd)  # the check is not vacuous
    assert abs(fd - adj) <= 1e-5 * abs(fd) + rounding / eps
    # the profile order, sigma recomputed at the cubature points (interface and wall unchanged)
    from oracle.pml import sigma_kappa
    xq = sim.cubature_points()
    p0 = float(cfg["pml"]["order"])
    h = 1e-6 * p0
    vals = []
    for sgn in (1.0, -1.0):
        pml = dict(cfg["pml"], order=p0 + sgn * h)
        sig = sigma_kappa(xq, pml)[0]
        assert not np.any((sig != 0) != (sig0 != 0))
        vals.append(loss_with(sig))
    fd = (vals[0] - vals[1]) / (2 * h)
    _say(f"  order: adjoint {gp[6]:.10e}  central difference {fd:.10e}  rounding bound {rounding / h:.1e}")
    assert rounding / h < 0.1 * abs(fd)
    assert abs(fd - gp[6]) <= 1e-5 * abs(fd) + rounding / h
    # a few single cubature nodes with the largest sensitivity
    idx = np.argsort(np.abs(g).ravel())[::-1][:2]
    for i in idx:
        k, q, a = np.unravel_index(i, g.shape)
        h = 1e-6 * max(1.0, abs(sig0[k, q, a]))
        sp, sm = sig0.copy(), sig0.copy()
        sp[k, q, a] += h
        sm[k, q, a] -= h
        fd = (loss_with(sp) - loss_with(sm)) / (2 * h)
        _say(f"  node {(k, q, a)}: adjoint {g[k, q, a]:.10e}  central difference {fd:.10e}")
        assert abs(fd - g[k, q, a]) <= 1e-5 * abs(fd) + rounding / h
    sim.set_sigma_q(sig0)


def _torch_profile(xq, sigma_max, L, order, wall_lo, wall_hi):
    """sigma_max (d / L)^order per axis (Sec. III), d the distance into the layer [wall - L, wall] of a fixed
    outer wall; differentiable in sigma_max [3], L [3] and order (the test's own statement of the profile)."""
    import torch
    lo = torch.as_tensor(wall_lo, dtype=xq.dtype) + L
    hi = torch.as_tensor(wall_hi, dtype=xq.dtype) - L
    d = torch.clamp(torch.maximum(xq - hi, lo - xq), min=0.0)
    inside = d > 0
    r = torch.where(inside, d / L, torch.ones_like(d))
    return sigma_max * torch.where(inside, r ** order, torch.zeros_like(d))


def test_autograd_function_chain_rule(wdg):
    """The library's profile chain rule (ProfileLoss) against torch's, through the per-node gradient (ShellLoss),
    at the creation profile and at re-sampled profiles with a moved interface."""
    import torch
    cfg = inputs.config("c1", **{"mesh.perturb": 0.1, "init.width": 0.35})
    _say("torch.autograd.Function")
    sim, osim, q0 = _pair(wdg, cfg, 0)
    pml = cfg["pml"]
    xq = torch.from_numpy(sim.cubature_points())
    wall_lo = np.asarray(pml["lo"], float) - np.asarray(pml["L"], float)
    wall_hi = np.asarray(pml["hi"], float) + np.asarray(pml["L"], float)
    for smax0, L0, order0 in ((pml["sigma_max"], pml["L"], pml["order"]),
                              ([22.0, 18.0, 25.0], [0.45, 0.48, 0.42], 2.5)):
        smax = torch.tensor(smax0, dtype=torch.float64, requires_grad=True)
        L = torch.tensor(L0, dtype=torch.float64, requires_grad=True)
        order = torch.tensor(float(order0), dtype=torch.float64, requires_grad=True)
        sig = _torch_profile(xq, smax, L, order, wall_lo, wall_hi)
        loss = wdg.ShellLoss.apply(sig, sim, q0, 0.0, osim.dt, 10, SHELL_C1, 0)
        loss.backward()
        want = np.concatenate([smax.grad.numpy(), L.grad.numpy(), [order.grad.item()]])
        theta = torch.tensor(list(smax0) + list(L0) + [float(order0)], dtype=torch.float64, requires_grad=True)
        loss2 = wdg.ProfileLoss.apply(theta, sim, q0, 0.0, osim.dt, 10, SHELL_C1, 0)
        # the library re-sampled the same profile
        assert np.max(np.abs(sig.detach().numpy() - sim.get_sigma_q())) <= 1e-12 * max(smax0)
        assert abs(loss2.item() - loss.item()) <= 1e-12 * abs(loss.item())
        loss2.backward()
        got = theta.grad.numpy()
        assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want)), (got, want)
    # a layer reaching elements created outside it is refused; a point-wise sigma has no profile gradient
    with pytest.raises(wdg.WdgError) as e:
        sim.set_pml_profile(pml["sigma_max"], [0.55] * 3, pml["order"])
    assert e.value.code == wdg.WDG_EINVAL
    sim.set_sigma_q(sim.get_sigma_q())
    sim.set_fields(q0)
    with pytest.raises(wdg.WdgError) as e:
        sim.loss_gradient(osim.dt, 2, SHELL_C1)
    assert e.value.code == wdg.WDG_ESTATE
    sim.set_pml_profile(pml["sigma_max"], pml["L"], pml["order"])
    sim.set_fields(q0)
    sim.loss_gradient(osim.dt, 2, SHELL_C1)
