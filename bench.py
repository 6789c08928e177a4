"""Benchmark: element-DOF updates per second of the WAA SC-PML DGTD step on one GPU.

Workload (the 48,000-tetrahedron configuration): cube [-1.5, 1.5]^3 cut into
20^3 x 6 tetrahedra with interior vertices perturbed by up to 10% of h (seed 0),
order N = 3 (N_p = 20), cubature of degree 6, PML of thickness 0.5 with a
cubic sigma profile (sigma_max = 30), Gaussian-modulated dipole source,
8 probes recorded every step, upwind flux, PEC outer wall, LSERK4.

A step is one full LSERK4 step: five launches of the fused stage kernel
(right-hand side of eqs. (26)-(29) with the upwind curl, the weight-adjusted
inverse mass P_q a^-1 V_q of eq. (21) applied on every PML element, and the
Runge-Kutta update) plus the probe readout.  Fields live in HBM before the
timed region starts.  The metric is K * N_p * steps / seconds, reported for
FP64 (`value`) and FP32 (`fp32`).  The same stepping with the inverse skipped
where it is the identity (kappa = 1) is reported separately (`waa_shortcut`).

Roofline: algorithmic bytes and flops per stage launch (see
`algorithmic_traffic`) over the average launch time of the timed region
(HIP events on the launch stream; the per-step probe launch is included, so
the figure is slightly conservative), against the vendor peaks and against
peaks measured on the same GPU (`measured_peaks`: a 1 GiB device copy and
chains of the MFMA instructions the kernel issues); the bound is whichever of
bytes / bandwidth and flops / peak is larger. `traffic` is the counted
memory-side bytes per launch (`MEASURED_TRAFFIC`).

Also reported: the adjoint/forward wall-time ratio of the loss gradient (`adjoint_forward_ratio`), the
batching form's throughput (`batch`: 32 independent simulations in one context), the Table I contrast
(`table_i`: memory and time per step of the weight-adjusted, direct stored-matrix and element-constant
PML schemes, N = 1..4) and the precision form at full size (`precision_form`: 384,000 tets, N = 4, FP64 and
FP32).

Usage: python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--no-cpu-baseline] [--stepping-only]
                       [--table-i-only | --adjoint-only | --precision-form-only [--pf-steps K] | --batch-only]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
# Memory-side bytes per stage launch from rocprofv3's TCC_EA0 request-size counters (reads: 32 B x RDREQ_32B +
# 64 B x RDREQ_64B + 128 B x RDREQ_128B; writes: 64 B x WRREQ_64B + 32 B x the other WRREQ), one pass for
# the reads and one for the writes. The same counters read 1.000 x 1 GiB each way for the library's 1 GiB
# device copy, so no scale factor is applied. Per kernel: (first stage of a step, which reads no residual;
# each of the other four stages), reads and writes in bytes; a launch's figure is the five-stage average.
# Taken on the kernel sources with this sha256 (kernels_mfma.hip + device.hpp); reported only while they are
# unchanged.
MEASURED_TRAFFIC = {
    "source_sha256": "ddf702916dadfc80c9b5ef40f1c14375df0cccc1f44252a87918d26e3b1cc2c0",
    "stage_mfma_kernel<double,N=3,Nq=24>": {"read": (178197248, 264747651), "write": (164413440, 164413440)},
    "stage_mfma_kernel<float,N=3,Nq=24>": {"read": (87352160, 130684352), "write": (89520294, 91302426)},
    "stage_mfma_kernel<double,N=4,Nq=51>": {"read": (2583748462, 3789409410), "write": (2226524160, 2226524160)},
    "stage_mfma_kernel<float,N=4,Nq=51>": {"read": (1287543653, 1920225666), "write": (1175017728, 1253561611)},
}
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 (packed vector / matrix)


def algorithmic_traffic(d, word: int, waa_inverse: bool = True):
    """Algorithmic HBM bytes and flops per stage launch, averaged over the five stages.

    Per PML element and stage: read q_in (12 N_p words), read the residual
    (12 N_p, stages 2-5 only: the first LSERK coefficient is zero), write the
    residual and q_out (12 N_p each), sigma at the cubature points (3 N_q),
    geometry (25 words) and the face-node neighbour map (4 N_fp int32).
    Interior elements move the 6 E,H components only and no sigma.
    Neighbour traces are re-reads of q_in (cache traffic, not counted).
    Flops per PML element (one FMA = 2 flops), the products the kernel executes
    (without the 16-row padding of the matrix-core tiles):
      volume 3*2*6 N_p^2 + lift 2*6*4 N_fp N_p + flux ~ 40*4 N_fp
      + PML terms 4*2*6 N_q N_p (V_q f, V_q P, P_q t_2, P_q t_1 per component)
      + weight-adjusted inverse 2*2*6 N_q N_p (V_q R, P_q Z per component;
        skipped with the kappa = 1 shortcut);
    interior elements have no PML term.
    """
    Np, Nq, Nfp = d.Np, d.Nq, d.Nfp
    K, Kp = d.K, d.K_pml
    Ki = K - Kp
    fixed_pml = (12 * Np * 3 + 3 * Nq + 25) * word + 4 * Nfp * 4
    fixed_int = (6 * Np * 3 + 25) * word + 4 * Nfp * 4
    res_pml = 12 * Np * word
    res_int = 6 * Np * word
    bytes_per_launch = Kp * (fixed_pml + 0.8 * res_pml) + Ki * (fixed_int + 0.8 * res_int)
    fl_common = 36 * Np * Np + 48 * Nfp * Np + 160 * Nfp
    flops_per_launch = Kp * (fl_common + (72 if waa_inverse else 48) * Nq * Np) + Ki * fl_common
    return bytes_per_launch, flops_per_launch


def roofline(bytes_per_launch, flops_per_launch, launch_us, word, peaks=None, traffic=None):
    """Roofline block of one kernel: bound = max(bytes / HBM peak, flops / compute peak of its dtype)."""
    t = launch_us * 1e-6
    fpk = FP64_PEAK_TFLOPS if word == 8 else FP32_PEAK_TFLOPS
    t_hbm, t_flop = bytes_per_launch / (HBM_PEAK_GBS * 1e9), flops_per_launch / (fpk * 1e12)
    gbs, tfl = bytes_per_launch / t / 1e9, flops_per_launch / t / 1e12
    if t_hbm >= t_flop:
        out = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    else:
        out = {"bound": "mfma", "achieved": tfl, "peak": fpk, "unit": "TFLOP/s", "frac": tfl / fpk}
    out.update({"traffic": traffic, "bytes_per_launch": bytes_per_launch, "flops_per_launch": flops_per_launch,
                "launch_us": launch_us, "roofline_us": max(t_hbm, t_flop) * 1e6,
                "achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS, "achieved_tflops": tfl, "flop_frac": tfl / fpk})
    if peaks:
        bw_m = peaks["copy_gbs"]
        fp_m = peaks["mfma_f64_tflops" if word == 8 else "mfma_f32_tflops"]
        out["measured_peaks"] = {"hbm_gbs": bw_m, "tflops": fp_m,
                                 "frac": max(bytes_per_launch / (bw_m * 1e9), flops_per_launch / (fp_m * 1e12)) / t}
    return out


def measured_peaks():
    """Peaks measured on this GPU: a 1 GiB device-to-device copy (bytes read + written over the time) and the
    sustained MFMA rate in FP64 (four-block 4x4x4, as the stage kernel issues it) and FP32 (16x16x4), from the
    library's microbenchmarks."""
    import torch

    from paper_2006_02551_amd import wdg

    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    reps = 10
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    torch_gbs = 2 * 4 * n * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    lib_gbs = wdg.measure_copy_bandwidth(1 << 30)
    return {"copy_gbs": max(torch_gbs, lib_gbs), "copy_torch_gbs": torch_gbs, "copy_library_gbs": lib_gbs,
            "mfma_f64_tflops": wdg.measure_mfma_peak(wdg.WDG_FP64, 4000),
            "mfma_f32_tflops": wdg.measure_mfma_peak(wdg.WDG_FP32, 4000),
            "how": "copy: the faster of a 1 GiB FP32 torch tensor copy (10 reps) and the library's 16-byte "
                   "copy kernel over 1 GiB (best of 5), bytes read + written; MFMA: chains of 16x16x4 steps "
                   "(FP64 as four 4x4x4 four-block instructions, as the stage kernel issues them), 8 per "
                   "wavefront, 32 wavefronts per compute unit"}


def measured_traffic(kernel):
    """Counted bytes per launch of `kernel` (five-stage average), or None once its sources have changed."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels_mfma.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2006_02551_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != MEASURED_TRAFFIC["source_sha256"] or kernel not in MEASURED_TRAFFIC:
        return None
    m = MEASURED_TRAFFIC[kernel]
    return sum((first + 4 * rest) / 5 for first, rest in (m["read"], m["write"]))


def run_gpu(cfg, precision, steps, warmup, shortcut=False, peaks=None):
    import torch

    from paper_2006_02551_amd import inputs, wdg

    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], precision)
    sim.set_waa_shortcut(shortcut)
    d = sim.dims
    q0 = inputs.gaussian_fields(cfg, sim.node_coords())
    sim.set_fields(q0)
    sim.set_dipole(cfg["source"])
    sim.set_probes(cfg["probes"], steps + warmup + 1)
    dt = cfg["cfl"] * d.dt_unit
    stream = torch.cuda.current_stream()
    sim.step(dt, warmup, stream)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    sim.step(dt, steps, stream)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    rows = sim.probe_read(steps + warmup + 1)
    e = sim.energy()
    kernel = {wdg.WDG_KERNEL_MFMA: "stage_mfma_kernel", wdg.WDG_KERNEL_SCALAR: "stage_kernel"}[sim.get_dims().kernel]
    word = 8 if precision == wdg.WDG_FP64 else 4
    b, f = algorithmic_traffic(d, word, waa_inverse=not shortcut)
    launch_ms = ms / (5 * steps)
    kname = f"{kernel}<{'double' if word == 8 else 'float'},N={d.N},Nq={d.Nq}>"
    out = {
        "value": d.K * d.Np * steps / (ms / 1e3),
        "ms_per_step": ms / steps,
        "stage_launch_us": launch_ms * 1e3,
        "roofline": roofline(b, f, launch_ms * 1e3, word, peaks, None if shortcut else measured_traffic(kname)),
        "energy": e,
        "probe_rows": int(rows.shape[0]),
        "kernel": kname,
        "dims": {"K": d.K, "K_pml": d.K_pml, "Np": d.Np, "Nq": d.Nq, "nblk": d.nblk, "N": d.N},
    }
    del sim
    return out


def run_adjoint(precision):
    """Wall time of the loss and its adjoint gradient (sqrt(T) checkpoints) against plain stepping, on the
    differentiation workload (48,000 tets, N=3, 500 steps, shell loss)."""
    import torch

    from paper_2006_02551_amd import inputs, wdg

    cfg = inputs.config("c5")
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    torch.cuda.empty_cache()  # the two-segment run allocates ~100 GB of state buffers in the library
    sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], precision)
    q0 = inputs.gaussian_fields(cfg, sim.node_coords())
    dt = cfg["cfl"] * sim.dims.dt_unit
    steps = cfg["steps"]
    sim.set_fields(q0)
    sim.loss_gradient(dt, 4, cfg["shell"])  # warm-up (kernel loading)
    sim.set_fields(q0)
    sim.set_time(0.0)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    sim.step(dt, steps, stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms_fwd = a.elapsed_time(b)
    sim.set_fields(q0)
    sim.set_time(0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, _, gp = sim.loss_gradient(dt, steps, cfg["shell"])
    ms_adj = (time.perf_counter() - t0) * 1e3
    # the same with two checkpoint segments (half the steps recomputed; 2 + 5 ceil(T/2) + 5 state buffers, about
    # 103 GB in FP64: the memory of one MI355X buys back half of the recomputation)
    half = (steps + 1) // 2
    sim.set_fields(q0)
    sim.set_time(0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J2, _, _ = sim.loss_gradient(dt, steps, cfg["shell"], half)
    ms_half = (time.perf_counter() - t0) * 1e3
    assert J2 == J
    del sim
    return {"ratio": ms_adj / ms_fwd, "ms_forward": ms_fwd, "ms_loss_gradient": ms_adj, "loss": J,
            "checkpoint_interval": int(math.ceil(math.sqrt(steps))),
            "ratio_two_segments": ms_half / ms_fwd, "ms_loss_gradient_two_segments": ms_half,
            "two_segments_state_buffers": 2 + 5 * half + 5,
            "dJ_dsigma_max": list(gp[:3]), "dJ_dL": list(gp[3:6]), "dJ_dorder": gp[6]}


def run_batch(steps, warmup, seq_steps=50, group_mb=256.0):
    """The batching form: 32 independent simulations (8^3 x 6 .. 24^3 x 6 tets, 1,282,008 in all, N=3, each
    with its own sigma profile and time step) stepped in one context in FP32 with captured two-step graphs,
    against the same simulations stepped one after another, each in a context of its own."""
    import torch

    from paper_2006_02551_amd import inputs, wdg
    from paper_2006_02551_amd.batch import Batch

    cfg = inputs.config("c4")
    b = Batch(cfg, wdg.WDG_FP32)
    d = b.sim.dims
    tune = b.sim.autotune(reps=5, stream=b.stream)
    chosen = {"kernel": "mfma" if b.sim.dims.kernel == wdg.WDG_KERNEL_MFMA else "scalar", "tiles": b.sim.dims.tiles}
    b.set_fields(b.initial_fields())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    b.step(warmup, graph=True)
    torch.cuda.synchronize()
    ev[0].record(b.stream)
    b.step(steps, graph=True)
    ev[1].record(b.stream)
    b.step(steps, graph=False)
    ev[2].record(b.stream)
    torch.cuda.synchronize()
    ms_graph, ms_eager = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    q = b.sim.get_fields()
    assert all(bool(abs(x) < 1e30) for x in (q.max(), q.min()))
    dofs = d.K * d.Np
    del b.sim
    # the same batch with cache-sized step groups (aligned components, both steps of a captured pair group
    # after group); groups of about 256 MB of fields and setup data were the fastest of 32-384 MB
    # (3.52e9 DOF/s against 3.39e9 at 128 MB and 3.02e9 ungrouped)
    gb = Batch(cfg, wdg.WDG_FP32, group_mb=group_mb)
    gb.sim.set_kernel(wdg.WDG_KERNEL_MFMA if chosen["kernel"] == "mfma" else wdg.WDG_KERNEL_SCALAR)
    if chosen["kernel"] == "mfma":
        gb.sim.set_tiles(chosen["tiles"])
    gb.set_fields(gb.initial_fields())
    gb.step(warmup, graph=True)
    torch.cuda.synchronize()
    ev[0].record(gb.stream)
    gb.step(steps, graph=True)
    ev[1].record(gb.stream)
    torch.cuda.synchronize()
    ms_grouped = ev[0].elapsed_time(ev[1])
    ngroups = int(gb.step_groups.max()) + 1
    dofs_g = gb.sim.dims.K * gb.sim.dims.Np
    del gb.sim
    # the same simulations one after another
    ms_seq = 0.0
    stream = torch.cuda.current_stream()
    for i, (vx, ev_i) in enumerate(b.meshes):
        sim = wdg.Simulation(vx, ev_i, cfg["N"], b.rule, b.standalone_pml(i), cfg["alpha"], wdg.WDG_FP32)
        sim.set_fields(inputs.gaussian_fields(cfg, sim.node_coords()))
        sim.step(float(b.dt[i]), 2, stream)
        torch.cuda.synchronize()
        ev[0].record(stream)
        sim.step(float(b.dt[i]), seq_steps, stream)
        ev[3].record(stream)
        torch.cuda.synchronize()
        ms_seq += ev[0].elapsed_time(ev[3]) / seq_steps
        del sim
    best_ms = min(ms_graph, ms_grouped)
    return {"value": dofs * steps / (best_ms / 1e3), "ms_per_step": best_ms / steps, "dtype": "f32",
            "form": "grouped" if ms_grouped < ms_graph else "ungrouped",
            "ungrouped_value": dofs * steps / (ms_graph / 1e3), "ungrouped_ms_per_step": ms_graph / steps,
            "grouped_value": dofs_g * steps / (ms_grouped / 1e3), "grouped_ms_per_step": ms_grouped / steps,
            "grouped_groups": ngroups, "group_mb": group_mb,
            "eager_value": dofs * steps / (ms_eager / 1e3),
            "sequential_value": dofs / (ms_seq / 1e3), "sequential_ms_per_step": ms_seq,
            "speedup_vs_sequential": ms_seq / (best_ms / steps),
            "ungrouped_speedup_vs_sequential": ms_seq / (ms_graph / steps),
            "autotune_us_per_stage": tune, "chosen": chosen, "K": d.K, "K_pml": d.K_pml, "nsim": len(b.meshes),
            "steps": steps,
            "workload": "c4: 32 simulations, meshes 8^3x6 .. 24^3x6 perturbed tets (1,282,008 in all), N=3, "
                        "sigma_max in [10, 50] and order in {2, 3, 4} per simulation, per-simulation dt, "
                        "Gaussian Ez pulse, FP32, one launch per stage for the whole batch, two-step HIP graphs; "
                        "sequential = each simulation in its own context, eager steps, one after another"}


def run_precision_form(steps=100, warmup=5, peaks=None):
    """The precision form at full size: 40^3 x 6 = 384,000 perturbed tets, N = 4 (51-point rule), dipole; element-DOF
    updates/s in FP64 and FP32 from zero fields, and the FP32 state against the FP64 state after the timed steps."""
    import numpy as np
    import torch

    from paper_2006_02551_amd import inputs, wdg

    cfg = inputs.config("c3")
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    out, states = {}, {}
    stream = torch.cuda.current_stream()
    for prec, name in ((wdg.WDG_FP64, "fp64"), (wdg.WDG_FP32, "fp32")):
        sim = wdg.Simulation(vx, ev, cfg["N"], rule, cfg["pml"], cfg["alpha"], prec)
        d = sim.dims
        sim.set_dipole(cfg["source"])
        sim.set_fields(np.zeros((d.K, 12, d.Np)))
        dt = cfg["cfl"] * d.dt_unit
        sim.step(dt, warmup, stream)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(dt, steps, stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        kernel = "mfma" if sim.dims.kernel == wdg.WDG_KERNEL_MFMA else "scalar"
        word = 8 if prec == wdg.WDG_FP64 else 4
        kname = (f"{'stage_mfma_kernel' if kernel == 'mfma' else 'stage_kernel'}<{'double' if word == 8 else 'float'},"
                 f"N={d.N},Nq={d.Nq}>")
        nb, nf = algorithmic_traffic(d, word)
        out[name] = {"value": d.K * d.Np / (ms / 1e3), "ms_per_step": ms, "kernel": kernel, "tiles": sim.dims.tiles,
                     "roofline": roofline(nb, nf, ms * 1e3 / 5, word, peaks, measured_traffic(kname))}
        states[name] = sim.get_fields()[:, 0:6]
        del sim
    out["fp32_rel_l2_vs_fp64"] = float(np.linalg.norm(states["fp32"] - states["fp64"]) / np.linalg.norm(states["fp64"]))
    out["steps"] = warmup + steps
    out["workload"] = ("c3: 40^3x6 = 384,000 perturbed tets, N=4 (Np=35), 51-point degree-8 rule, quadratic PML "
                       "sigma_max=40, dipole, fields from zero")
    return out


def run_table_i(steps=40, warmup=3):
    """The Table I contrast on the GPU: memory and time per step of the weight-adjusted scheme against the
    direct scheme with stored per-element matrices (and element-constant coefficients), N = 1..4, FP64, on
    the 73,002-tet stand-in of Table I's mesh."""
    import torch

    from paper_2006_02551_amd import inputs, wdg

    rows = []
    stream = torch.cuda.current_stream()
    for N in (1, 2, 3, 4):
        cfg = inputs.config("t1", N=N, cub_degree=2 * N)
        vx, ev = inputs.mesh_for(cfg)
        sim = wdg.Simulation(vx, ev, N, inputs.load_rule(2 * N), cfg["pml"], cfg["alpha"], wdg.WDG_FP64)
        d = sim.dims
        q0 = inputs.gaussian_fields(cfg, sim.node_coords())
        dt = cfg["cfl"] * d.dt_unit

        def timed():
            sim.set_fields(q0)
            sim.step(dt, warmup, stream)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            sim.step(dt, steps, stream)
            b.record(stream)
            torch.cuda.synchronize()
            assert abs(sim.energy()) < 1e30
            return a.elapsed_time(b) / steps

        mem = sim.memory_report()
        common = mem["state"] + mem["geometry"] + mem["connectivity"] + mem["operators"]
        row = {"N": N, "Np": d.Np, "Nq": d.Nq, "K": d.K, "K_pml": d.K_pml}
        default_kernel = sim.dims.kernel
        # every scheme on the default (matrix-core) kernel, and on the scalar-operand kernel for reference
        t = {"waa": timed(), "waa_kernel": "mfma" if default_kernel == wdg.WDG_KERNEL_MFMA else "scalar"}
        sim.set_kernel(wdg.WDG_KERNEL_SCALAR)
        t["waa_scalar"] = timed()
        sim.set_kernel(default_kernel)
        t0 = time.perf_counter()
        sim.set_pml_scheme(wdg.WDG_PML_DIRECT, inputs.product_rule(N + 4))
        row["direct_setup_s"] = time.perf_counter() - t0
        direct_bytes = sim.memory_report()["scheme_data"]
        t["direct"] = timed()
        sim.set_kernel(wdg.WDG_KERNEL_SCALAR)
        t["direct_scalar"] = timed()
        sim.set_kernel(default_kernel)
        sim.set_pml_scheme(wdg.WDG_PML_CONSTANT)
        t["element_constant"] = timed()
        sim.set_kernel(wdg.WDG_KERNEL_SCALAR)
        t["element_constant_scalar"] = timed()
        row["ms_per_step"] = t
        row["memory_MB"] = {"waa_total": (common + mem["coefficients"]) / 1e6,
                            "direct_total": (common + direct_bytes) / 1e6,
                            "waa_pml_data": mem["coefficients"] / 1e6, "direct_pml_data": direct_bytes / 1e6,
                            "paper_model_waa": mem["paper_waa"] / 1e6, "paper_model_direct": mem["paper_direct"] / 1e6}
        row["direct_over_waa"] = {"memory": row["memory_MB"]["direct_total"] / row["memory_MB"]["waa_total"],
                                  "time": t["direct"] / t["waa"]}
        print(f"bench: table I N={N} ({t['waa_kernel']} kernel; scalar-operand in brackets): WAA {t['waa']:.3f} "
              f"({t['waa_scalar']:.3f}) ms/step, direct {t['direct']:.3f} ({t['direct_scalar']:.3f}), element-constant "
              f"{t['element_constant']:.3f} ({t['element_constant_scalar']:.3f}); memory {row['memory_MB']['waa_total']:.0f} "
              f"vs {row['memory_MB']['direct_total']:.0f} MB", file=sys.stderr, flush=True)
        rows.append(row)
        del sim
    return {"workload": "t1: 23^3x6 = 73,002 perturbed tets, 52,752 in the PML (Table I: 72,762 / 52,657), cubic "
                        "profile sigma_max = 30, cubature of degree 2N, FP64, Gaussian Ez pulse; direct matrices "
                        "integrated with the conical product rule of (N+4)^3 points",
            "steps": steps, "rows": rows}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, steps=2, par_steps=8, workers=None):
    """The FP64 oracle on the host cores for a bounded sample: `steps` LSERK4 steps in one process (single-threaded
    NumPy einsum), then `par_steps` steps with the oracle's right-hand side split over element chunks in
    `workers` forked processes (the host's CPU share: at most 16)."""
    import numpy as np

    from oracle.pool import ChunkedRHS
    from oracle.run import Simulation as OSim
    from paper_2006_02551_amd import inputs

    workers = workers or min(16, os.cpu_count() or 1)
    vx, ev = inputs.mesh_for(cfg)
    rule = inputs.load_rule(cfg["cub_degree"])
    osim = OSim(cfg, vx, ev, *rule)
    osim.set_state(inputs.gaussian_fields(cfg, osim.mesh.x))
    K, Np = osim.mesh.K, osim.ref.Np
    t0 = time.perf_counter()
    osim.run(steps)
    sec1 = time.perf_counter() - t0
    with ChunkedRHS(osim.op, osim.q.shape, workers) as pool:
        osim.rhs = pool
        osim.run(1)  # workers started and warm
        t0 = time.perf_counter()
        osim.run(par_steps)
        secp = time.perf_counter() - t0
    assert np.all(np.isfinite(osim.q))
    one = K * Np * steps / sec1
    return {"value": K * Np * par_steps / secp, "unit": "element-DOF updates/s", "cores": workers, "kind": "oracle",
            "single_thread_value": one, "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
            "sample": f"the 48,000-tet N=3 workload in the NumPy FP64 oracle: {par_steps} LSERK4 steps with the "
                      f"right-hand side over {workers} forked processes ({secp:.1f} s), and {steps} steps in one "
                      f"process, single-threaded ({sec1:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stepping-only", action="store_true",
                    help="run the c2 stepping legs only (no adjoint or batch legs), e.g. under a profiler")
    ap.add_argument("--table-i-only", action="store_true",
                    help="run the Table I contrast only and print its JSON (e.g. under a profiler)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run the loss-gradient leg only and print its JSON (e.g. under a profiler)")
    ap.add_argument("--precision-form-only", action="store_true",
                    help="run the 384,000-tet N=4 precision-form leg only and print its JSON (e.g. under a profiler)")
    ap.add_argument("--pf-steps", type=int, default=100,
                    help="timed steps of the precision-form leg (e.g. fewer under a counter profiler)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run the 32-simulation batching leg only and print its JSON (e.g. under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the element-partitioned "
              f"multi-GPU path is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2006_02551_amd import inputs, wdg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.table_i_only:
        print(json.dumps({"table_i": run_table_i()}))
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint_fp64": run_adjoint(wdg.WDG_FP64), "adjoint_fp32": run_adjoint(wdg.WDG_FP32)}))
        return
    if args.batch_only:
        print(json.dumps({"batch": run_batch(max(args.steps // 5, 20), 4)}))
        return
    peaks = measured_peaks()
    print(f"bench: measured peaks: copy {peaks['copy_gbs']:.0f} GB/s, MFMA FP64 {peaks['mfma_f64_tflops']:.1f} "
          f"TFLOP/s, FP32 {peaks['mfma_f32_tflops']:.1f} TFLOP/s", file=sys.stderr, flush=True)
    if args.precision_form_only:
        print(json.dumps({"precision_form": run_precision_form(steps=args.pf_steps, peaks=peaks), "measured_peaks": peaks}))
        return
    cfg = inputs.config("c2")
    print(f"bench: c2 workload, {args.warmup} warmup + {args.steps} timed steps, FP64", file=sys.stderr, flush=True)
    r64 = run_gpu(cfg, wdg.WDG_FP64, args.steps, args.warmup, peaks=peaks)
    print(f"bench: FP64 {r64['value']:.3e} DOF/s, {r64['ms_per_step']:.3f} ms/step; FP32 next",
          file=sys.stderr, flush=True)
    r32 = run_gpu(cfg, wdg.WDG_FP32, args.steps, args.warmup, peaks=peaks)
    print(f"bench: FP32 {r32['value']:.3e} DOF/s, {r32['ms_per_step']:.3f} ms/step; kappa = 1 shortcut next",
          file=sys.stderr, flush=True)
    s64 = run_gpu(cfg, wdg.WDG_FP64, args.steps, args.warmup, shortcut=True, peaks=peaks)
    s32 = run_gpu(cfg, wdg.WDG_FP32, args.steps, args.warmup, shortcut=True, peaks=peaks)
    adj64 = adj32 = batch = table_i = c3 = None
    if not args.stepping_only:
        print("bench: adjoint (loss gradient) against plain stepping, 500 steps, FP64 and FP32", file=sys.stderr,
              flush=True)
        adj64 = run_adjoint(wdg.WDG_FP64)
        adj32 = run_adjoint(wdg.WDG_FP32)
        print(f"bench: adjoint/forward {adj64['ratio']:.2f} (FP64), {adj32['ratio']:.2f} (FP32); batch next",
              file=sys.stderr, flush=True)
        batch = run_batch(max(args.steps // 5, 20), 4)
        print(f"bench: batch {batch['value']:.3e} DOF/s ({batch['speedup_vs_sequential']:.2f}x sequential); "
              f"Table I contrast next", file=sys.stderr, flush=True)
        table_i = run_table_i()
        print("bench: precision form (c3, 384,000 tets, N=4) FP64 and FP32", file=sys.stderr, flush=True)
        c3 = run_precision_form(steps=args.pf_steps, peaks=peaks)
        print(f"bench: c3 FP64 {c3['fp64']['value']:.3e} DOF/s, FP32 {c3['fp32']['value']:.3e} DOF/s, "
              f"FP32 vs FP64 {c3['fp32_rel_l2_vs_fp64']:.1e}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle (one process, then all host cores)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg)
    d = r64["dims"]
    line = {
        "metric": "element-DOF updates/s (WADG-PML RHS+LSERK) FP64 vs FP32; adjoint/forward ratio",
        "value": r64["value"],
        "unit": "element-DOF updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2: 20^3x6=48000 perturbed tets, N=3, Nq=24, cubic PML sigma_max=30, dipole, "
                               "8 probes, LSERK4; weight-adjusted inverse applied on every PML element",
                   "K": d["K"], "K_pml": d["K_pml"], "N": 3, "Np": d["Np"],
                   "Nq": d["Nq"], "parallelism": "single GPU"},
        "roofline": dict(r64["roofline"], kernel=r64["kernel"]),
        "fp32": {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "dtype": "f32", "kernel": r32["kernel"],
                 "speedup_vs_fp64": r32["value"] / r64["value"], "roofline": r32["roofline"]},
        "waa_shortcut": {"what": "the same stepping with P_q a^-1 V_q skipped where it is the identity (kappa = 1)",
                         "fp64": {"value": s64["value"], "ms_per_step": s64["ms_per_step"],
                                  "roofline": s64["roofline"]},
                         "fp32": {"value": s32["value"], "ms_per_step": s32["ms_per_step"],
                                  "roofline": s32["roofline"]}},
        "measured_peaks": peaks,
        "adjoint_forward_ratio": None if adj64 is None else {
            "value": adj64["ratio"], "fp32": adj32["ratio"],
            "workload": "c5: the 48,000-tet N=3 mesh, Gaussian Ez pulse, 500 LSERK4 steps, loss = time-integrated "
                        "energy in the shell 0.1 inside the PML interface, gradient by the discrete adjoint with "
                        "sqrt(T) checkpoints (wall time of wdg_loss_gradient / 500 plain steps)",
            "fp64": {k: v for k, v in adj64.items() if k != "ratio"},
            "fp32_detail": {k: v for k, v in adj32.items() if k != "ratio"}},
        "batch": batch,
        "table_i": table_i,
        "precision_form": c3,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
