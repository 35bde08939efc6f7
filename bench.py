"""Throughput of the coupled ALE lattice Boltzmann FSI step on one MI355X.

One step = the whole coupled update of one instance: collision + ALE
semi-Lagrangian streaming of both population sets at every node, far-field
and Grad wall boundaries, the traction reduction and the body update.

Default workload: cylinder in compressible flow (Ma 0.5, Re 1000) on a
2048 (radial) x 4096 (azimuthal) O-grid, 8,388,608 nodes, with blending
mesh motion from a prescribed heave of amplitude 0.2 D, FP32 populations.
Metric: MLUPS, one lattice update = both f and g (18 populations) at one node.

Prints ONE JSON line.  Inputs are synthetic and resident in HBM before the
timed region starts.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "MLUPS (f+g, D2Q9) and % HBM roofline; batched/FP16 vs plain FP32"
HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 2.4 GHz x one 64-lane wave instruction per cycle per CU
VALU_PEAK_G = 256 * 2.4
# the source of the collision-streaming kernel (the counter records are tied to
# it): the shared device header and its section of the kernel file
CSRC = os.path.join(ROOT, "paper_2107_01370_amd", "csrc")
K1_SECTION = ("// Fused collision + ALE interpolating streaming.", "// Boundary kernels")


def algorithmic_bytes_per_node(storage: int, unstructured: bool = False) -> int:
    """Populations read once and written once (18 values each way) plus the
    FP64 node coordinates (16 B) needed to recompute the departure points.
    Unstructured 9-node meshes (static): the populations plus the static
    connectivity and geometry, 0.25 elements per node of 9 node indices and 9
    FP32 offsets (108 B) and the node-to-element table (3.25 ints): 40 B."""
    per_pop = 2 if storage == 1 else 4
    if unstructured:
        return 2 * 18 * per_pop + 40
    return 2 * 18 * per_pop + 16


def kernel_source_hash() -> str:
    """Hash of what a counter summary of the collision-streaming kernel depends
    on: its source, the shared device and layout headers, and the host routine
    that orders its tiles (the order decides which halo reads hit in L2)."""
    h = hashlib.sha256()
    for name in ("fsilbm_device.h", "fsilbm_internal.h"):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(CSRC, "fsilbm_host.hip"), encoding="utf-8") as fh:
        text = fh.read()
    a = text.index("void append_tiles(")
    h.update(text[a:text.index("\n}\n", a)].encode())
    with open(os.path.join(CSRC, "fsilbm_kernels.hip"), encoding="utf-8") as fh:
        text = fh.read()
    a = text.index(K1_SECTION[0])
    h.update(text[a:text.index(K1_SECTION[1], a)].encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: int, n_nodes: int):
    """HBM bytes per launch of the collision-streaming kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_collide_stream_{workload}_"
                                          f"{'fp16' if storage else 'fp32'}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def measured_valu(workload: str, storage: int, n_nodes: int, k1_ms: float):
    """VALU issue of the collision-streaming kernel from the committed counter
    summary (SQ_INSTS_VALU, wave instructions per dispatch), if it was taken on
    the current kernel source: against one wave instruction per cycle per CU
    (four 16-lane SIMDs, 4 cycles per 64-lane instruction; packed FP32 off)."""
    path = os.path.join(ROOT, "profiles", f"valu_collide_stream_{workload}_"
                                          f"{'fp16' if storage else 'fp32'}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    wi = float(rec["valu_wave_instructions_per_dispatch"])
    achieved = wi / (k1_ms * 1e-3) / 1e9
    return {"wave_instructions_per_launch": round(wi),
            "per_node": round(wi * 64 / n_nodes, 1),
            "achieved": round(achieved, 1), "peak": VALU_PEAK_G, "unit": "G wave-instr/s",
            "frac": round(achieved / VALU_PEAK_G, 4)}


WORKLOADS = {
    "cylinder_heave_2048x4096": "O-grid cylinder, Ma 0.5, Re 1000, blended mesh with prescribed "
                                "heave 0.2 D",
    "cylinder_viv_256x512": "O-grid cylinder, 1DOF VIV, Ma 0.2, Re 100, m* 10, U* 5",
    "airfoil_flutter_768x256": "C-grid NACA0012, 2DOF pitch-plunge, Ma 0.85, Re 1e5, T 0.2, "
                               "m* 60, alpha0 1 deg",
    "batched_sweep_64": "64 independent 1DOF cylinder instances, n_r ~ U[128,384], "
                        "n_theta = 2 n_r, seed 0, one launch per kernel per step",
    "tandem_independent_2304x320": "twin O-grid, two cylinders in tandem (L/D 5, D 200) each "
                                   "on its own spring (1+1DOF), Ma 0.1, Re 1000, m* 4, U* 6",
    "tandem_linked_2304x320": "twin O-grid, two rigidly linked cylinders in tandem (L/D 5, "
                              "D 200) on one spring (1DOF), Ma 0.1, Re 1000, m* 4, U* 6",
    "unstructured_q9_1572864": "unstructured periodic mesh of 393,216 nine-node quadrilateral "
                               "elements (1,572,864 nodes, triangles split into quadrilaterals), "
                               "diagonal stream Ma 0.1 with a density pulse",
    "unstructured_cylinder_q9_2103296": "unstructured mesh of 525,312 nine-node quadrilateral "
                                        "elements (2,103,296 nodes) round a fixed cylinder (D 640, "
                                        "far field 8 D), Ma 0.2, Re 1000, Grad wall, free-stream "
                                        "far field",
    "unstructured_cylinder_heave_q9_2103296": "the same unstructured mesh round a cylinder in "
                                              "prescribed heave (0.1 D, St 0.2) in the same "
                                              "stream, blended mesh motion (rigid to R + D/4, "
                                              "blended to R + 2 D), departure points located "
                                              "every step",
}


def workload_case(name: str, storage: int):
    if name == "cylinder_heave_2048x4096":
        return synth.large_heave_case(storage=storage)
    if name == "cylinder_viv_256x512":
        c = synth.cylinder_viv_case()
        c.fluid.storage = storage
        return c
    if name == "airfoil_flutter_768x256":
        return synth.airfoil_flutter_case(storage=storage)
    if name == "tandem_independent_2304x320":
        return synth.tandem_cylinders_case(linked=False, h0_frac=0.01, storage=storage)
    if name == "tandem_linked_2304x320":
        return synth.tandem_cylinders_case(linked=True, h0_frac=0.01, storage=storage)
    if name == "unstructured_q9_1572864":
        return unstructured_case(256, storage)
    if name == "unstructured_cylinder_q9_2103296":
        return unstructured_cylinder_case(512, 640.0, storage)
    if name == "unstructured_cylinder_heave_q9_2103296":
        return unstructured_cylinder_case(512, 640.0, storage, heave_D=0.1)
    raise SystemExit(f"unknown workload {name}")


def unstructured_case(m: int, storage: int):
    from synth.configs import Case
    from synth.unstructured import unstructured_pulse_case
    mesh, fluid, (rho, ux, uy, T) = unstructured_pulse_case(m, storage=storage)
    return Case(f"unstructured_q9_{mesh.n_nodes}", mesh, fluid, [], rho[None], ux[None], uy[None],
                T[None])


def unstructured_cylinder_case(n_theta: int, D: float, storage: int, heave_D: float = 0.0):
    from synth.configs import Case
    from synth.unstructured import q9_cylinder_case
    mesh, fluid, body, (rho, ux, uy, T) = q9_cylinder_case(n_theta, D, 8.0, seed=1, Ma=0.2,
                                                          Re=1000.0, storage=storage,
                                                          heave_D=heave_D)
    kind = "cylinder_heave" if heave_D > 0.0 else "cylinder"
    return Case(f"unstructured_{kind}_q9_{mesh.n_nodes}", mesh, fluid, [body], rho[None],
                ux[None], uy[None], T[None])


def copy_ceiling_gbs(reps: int = 5) -> dict:
    """A measured bandwidth ceiling beside the vendor peak: a plain 1 GiB
    device-to-device copy (torch), bytes read plus bytes written per second."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"GBs": round(2 * (1 << 30) / (ms * 1e-3) / 1e9, 1),
            "how": "1 GiB device-to-device copy (torch copy_), read + write bytes per second"}


def time_gpu(case, steps: int, warmup: int, kernel_reps: int = 20, subiterations: int = 1,
             relaxation: float = 1.0):
    import torch

    from paper_2107_01370_amd.fsilbm import Simulation

    sim = Simulation(case.mesh, case.fluid, case.bodies, device="cuda:0")
    sim.init_equilibrium(case.rho, case.ux, case.uy, case.T)
    if subiterations > 1:
        sim.set_coupling(subiterations, relaxation)
    sim.step(warmup)
    # both captured graphs (16 steps and one step) exist before the timed
    # region, whatever the warm-up count: no capture is timed
    sim.step(16)
    sim.step(1)
    sim.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(sim.stream)
    sim.step(steps)
    stop.record(sim.stream)
    stop.synchronize()
    sim.synchronize()                 # also checks the device error word
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    # per-kernel mean launch durations, HIP events on the simulation stream
    kms = sim.time_kernels(kernel_reps)
    rho, ux, uy, T = sim.macro()
    finite = bool(np.all(np.isfinite(rho)) and np.all(np.isfinite(T)))
    sim.close()
    return total_ms, kms, finite


def time_batch(cases, steps: int, warmup: int, kernel_reps: int = 10):
    """All instances in one Batch: one launch per kernel per step, schedule
    picked by the library's autotuner."""
    import torch

    from paper_2107_01370_amd.fsilbm import Batch

    b = Batch(cases, device="cuda:0")
    for k, c in enumerate(cases):
        b.init_equilibrium(k, c.rho, c.ux, c.uy, c.T)
    b.step(warmup)
    b.synchronize()
    grid, order, shape, _ = b.autotune(reps=5)
    b.step(16)                                 # capture the tuned graphs (16 steps, one step)
    b.step(1)
    b.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    b.step(steps)
    stop.record(b.stream)
    stop.synchronize()
    b.synchronize()
    total_ms = start.elapsed_time(stop)
    kms = b.time_kernels(kernel_reps)
    finite = all(bool(np.all(np.isfinite(b.macro(k)[0]))) for k in range(len(cases)))
    b.close()
    return total_ms, kms, (grid, order, shape), finite


def time_sequential(cases, steps: int, warmup: int):
    """The same instances each in its own Simulation, run one after another
    (per-instance launches, one HIP graph per step each)."""
    import torch

    from paper_2107_01370_amd.fsilbm import Simulation

    sims = []
    for c in cases:
        s = Simulation(c.mesh, c.fluid, c.bodies, device="cuda:0")
        s.init_equilibrium(c.rho, c.ux, c.uy, c.T)
        s.step(warmup)
        s.step(16)                             # both graphs captured before timing
        s.step(1)
        sims.append(s)
    for s in sims:
        s.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps)
    for s in sims:
        s.synchronize()
    total_ms = (time.perf_counter() - t0) * 1e3
    for s in sims:
        s.close()
    return total_ms


def cpu_baseline_unstructured(target_s: float = 20.0, m: int = 48):
    """Oracle (plain FP64 NumPy) timed on a smaller mesh of the same
    construction and physics (m = 48: 55,296 nodes), started from the
    populations the GPU path initialises; returns the timing and the accuracy
    of the GPU path against it on the same steps."""
    from oracle.unstructured import UnstructuredSolver
    from paper_2107_01370_amd.fsilbm import Simulation
    from synth.unstructured import unstructured_pulse_case

    mesh, fluid, (rho, ux, uy, T) = unstructured_pulse_case(m)
    sim = Simulation(mesh, fluid, [], device="cuda:0")
    sim.init_equilibrium(rho[None], ux[None], uy[None], T[None])
    f0, g0 = sim.populations()
    ora = UnstructuredSolver(mesh, fluid, rho, ux, uy, T)
    ora.f = f0[:, 0, :].astype(np.float64)
    ora.g = g0[:, 0, :].astype(np.float64)
    ora.step()
    t0 = time.perf_counter()
    n = 0
    while True:
        ora.step()
        n += 1
        el = time.perf_counter() - t0
        if el >= target_s or n >= 200:
            break
    sim.step(n + 1)
    r, _, _, Tg = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    sim.close()
    sample = (f"{n} steps of the same construction at m = {m} ({mesh.n_nodes} nodes, "
              f"{mesh.n_elems} elements) with the same physics, {el:.1f} s, single-threaded "
              f"NumPy (BLAS/OpenMP pools limited to one thread), os.cpu_count()={os.cpu_count()}")
    accuracy = {
        "against": "FP64 oracle, same sample as cpu_baseline, from the same initial populations",
        "steps": n + 1,
        "rho_max_rel": float(np.max(np.abs(r[0] - r_o) / r_o)),
        "p_max_rel": float(np.max(np.abs(r[0] * Tg[0] - r_o * T_o) / (r_o * T_o))),
    }
    return {"value": mesh.n_nodes * n / el / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": sample}, accuracy


def cpu_baseline_unstructured_cylinder(target_s: float = 20.0, n_theta: int = 64,
                                       heave_D: float = 0.0):
    """Oracle (plain FP64 NumPy) timed on a smaller mesh of the same
    construction round the same body shape and physics (n_theta = 64,
    D = 80), started from the populations the GPU path initialises; returns
    the timing and the accuracy of the GPU path against it on the same steps."""
    from oracle.unstructured import UnstructuredWallSolver
    from paper_2107_01370_amd.fsilbm import Simulation

    case = unstructured_cylinder_case(n_theta, 80.0, 0, heave_D=heave_D)
    mesh, fluid, body = case.mesh, case.fluid, case.bodies[0]
    rho, ux, uy, T = case.rho[0], case.ux[0], case.uy[0], case.T[0]
    sim = Simulation(mesh, fluid, [body], device="cuda:0")
    sim.init_equilibrium(case.rho, case.ux, case.uy, case.T)
    f0, g0 = sim.populations()
    ora = UnstructuredWallSolver(mesh, fluid, body, rho, ux, uy, T)
    ora.f = f0[:, 0, :].astype(np.float64)
    ora.g = g0[:, 0, :].astype(np.float64)
    ora.step()
    t0 = time.perf_counter()
    n = 0
    while True:
        ora.step()
        n += 1
        el = time.perf_counter() - t0
        if el >= target_s or n >= 200:
            break
    nsteps = n + 1
    sim.step(nsteps)
    r, _, _, Tg = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    hist = sim.forces(0, nsteps)
    ho = np.array(ora.history)[:nsteps]
    fscale = float(np.max(np.hypot(ho[:, 1], ho[:, 2])))
    sim.close()
    accuracy = {
        "against": "FP64 oracle, same sample as cpu_baseline, from the same initial populations",
        "steps": nsteps,
        "rho_max_rel": float(np.max(np.abs(r[0] - r_o) / r_o)),
        "p_max_rel": float(np.max(np.abs(r[0] * Tg[0] - r_o * T_o) / (r_o * T_o))),
        "body0": {"drag_max_rel": float(np.max(np.abs(hist[:, 1] - ho[:, 1])) / fscale),
                  "lift_max_rel": float(np.max(np.abs(hist[:, 2] - ho[:, 2])) / fscale)},
    }
    return {"value": mesh.n_nodes * n / el / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps of the same construction at n_theta = {n_theta}, D = 80 "
                      f"({mesh.n_nodes} nodes, {mesh.n_elems} elements) with the same physics, "
                      f"{el:.1f} s, single-threaded NumPy (BLAS/OpenMP pools limited to one thread), "
                      f"os.cpu_count()={os.cpu_count()}"}, accuracy


def cpu_baseline(case, target_s: float = 20.0, rows: int = 64):
    """Oracle (plain FP64 NumPy) timed on a strip of the same workload: the
    first `rows` radial rows of the O-grid (wall included) with the same
    physics, stepped until about `target_s` seconds of CPU work, from the
    populations the GPU path initialises on that strip; returns the timing and
    the accuracy of the GPU path against it on the same steps (density,
    pressure, wall forces, heave)."""
    from dataclasses import replace

    from oracle.solver import OracleSolver
    from paper_2107_01370_amd.fsilbm import Simulation

    m = case.mesh
    strip = replace(m, nj=rows, X=m.X[:rows].copy(), Y=m.Y[:rows].copy())
    macro = (case.rho[:rows], case.ux[:rows], case.uy[:rows], case.T[:rows])
    sim = Simulation(strip, case.fluid, case.bodies, device="cuda:0")
    sim.init_equilibrium(*macro)
    f0, g0 = sim.populations()
    ora = OracleSolver(strip, case.fluid, case.bodies, *macro)
    ora.f = f0.astype(np.float64)
    ora.g = g0.astype(np.float64)
    ora.step()                         # warm-up (first-call overheads)
    t0 = time.perf_counter()
    n = 0
    while True:
        ora.step()
        n += 1
        el = time.perf_counter() - t0
        if el >= target_s or n >= 50:
            break
    nsteps = n + 1
    sim.step(nsteps)
    r, _, _, Tg = sim.macro()
    r_o, _, _, _, T_o = ora.macroscopic()
    accuracy = {
        "against": "FP64 oracle, same sample as cpu_baseline, from the same initial populations",
        "steps": nsteps,
        "rho_max_rel": float(np.max(np.abs(r - r_o) / r_o)),
        "p_max_rel": float(np.max(np.abs(r * Tg - r_o * T_o) / (r_o * T_o))),
    }
    for k in range(len(case.bodies)):
        # the records of levels 0 .. nsteps-1 (the oracle records a level when
        # it steps from it)
        hist = sim.forces(0, nsteps, body=k)
        ho = np.array(ora.histories[k])[:nsteps]
        fscale = float(np.max(np.hypot(ho[:, 1], ho[:, 2])))
        # drag and lift against the peak force magnitude (they share the
        # dynamic-pressure scale), heave against the body diameter scale of
        # its own motion
        accuracy[f"body{k}"] = {
            "drag_max_rel": float(np.max(np.abs(hist[:, 1] - ho[:, 1])) / fscale),
            "lift_max_rel": float(np.max(np.abs(hist[:, 2] - ho[:, 2])) / fscale),
            "heave_max_abs": float(np.max(np.abs(hist[:, 4] - ho[:, 4]))),
        }
    sim.close()
    nodes = strip.ni * strip.nj
    return {
        "value": nodes * n / el / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n} steps of a {strip.ni}x{rows} strip (rows 0..{rows - 1}, wall included) "
                  f"of the same mesh and physics, {el:.1f} s, single-threaded NumPy "
                  f"(BLAS/OpenMP pools limited to one thread), host "
                  f"{platform.processor() or platform.machine()}, "
                  f"os.cpu_count()={os.cpu_count()}",
    }, accuracy


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cylinder_heave_2048x4096")
    ap.add_argument("--storage", choices=("fp32", "fp16"), default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--subiterations", type=int, default=1,
                    help="strong coupling: fluid passes per step (1 = staggered scheme); "
                         "MLUPS then count accepted steps")
    ap.add_argument("--relaxation", type=float, default=1.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device-to-device copy, the reference "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is described as a design and not implemented.", file=sys.stderr)
        sys.exit(2)
    storage = 1 if args.storage == "fp16" else 0
    if args.workload not in WORKLOADS:
        raise SystemExit(f"unknown workload {args.workload}; one of {sorted(WORKLOADS)}")
    if args.calibrate_copy:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "batched_sweep_64":
        return main_batched(args, storage)
    case = workload_case(args.workload, storage)
    N = case.mesh.n_nodes
    total_ms, kms, finite = time_gpu(case, args.steps, args.warmup,
                                     subiterations=args.subiterations,
                                     relaxation=args.relaxation)
    ms_per_step = total_ms / args.steps
    mlups = N * args.steps / (total_ms * 1e-3) / 1e6
    bpn = algorithmic_bytes_per_node(storage, args.workload.startswith("unstructured"))
    k1_ms = float(kms[0])
    achieved = bpn * N / (k1_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, storage, N)
    copy_ceiling = copy_ceiling_gbs()
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {WORKLOADS[args.workload]}, {args.storage} "
                        f"population storage",
            "nodes": N,
            "storage": args.storage,
            "coupling": {"subiterations": args.subiterations, "relaxation": args.relaxation},
            "kernel_ms": {"collide_stream": round(k1_ms, 5),
                          "wall_targets_farfield": round(float(kms[1]), 5),
                          "wall_grad_traction": round(float(kms[2]), 5),
                          "body": round(float(kms[3]), 5)},
            "finite_state": finite,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("2 k_u_egrad + k_u_nodeD + k_u_collide_stream_blk"
                       if args.workload.startswith("unstructured") else "k_collide_stream"),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_node": bpn,
            "valu_issue": (None if args.workload.startswith("unstructured")
                           else measured_valu(args.workload, storage, N, k1_ms)),
            "copy_ceiling": copy_ceiling,
            "frac_of_copy": round(achieved / copy_ceiling["GBs"], 4),
        },
    }
    if not args.no_variants and args.workload == "cylinder_heave_2048x4096" and storage == 0:
        case16 = workload_case(args.workload, 1)
        t16, k16, fin16 = time_gpu(case16, args.steps, args.warmup)
        out["variants"] = [{
            "storage": "fp16_shifted",
            "value": round(N * args.steps / (t16 * 1e-3) / 1e6, 1),
            "unit": "MLUPS",
            "ms_per_step": round(t16 / args.steps, 5),
            "collide_stream_ms": round(float(k16[0]), 5),
            "achieved_GBs": round(algorithmic_bytes_per_node(1) * N / (float(k16[0]) * 1e-3) / 1e9, 1),
            "finite_state": fin16,
        }]
    if not args.no_variants and args.workload == "cylinder_heave_2048x4096" and storage == 0:
        cases = synth.batched_sweep_cases(64)
        nb = sum(c.mesh.n_nodes for c in cases)
        bsteps = max(1, args.steps // 2)
        tb, kb, sched, finb = time_batch(cases, bsteps, args.warmup)
        ts = time_sequential(cases, bsteps, args.warmup)
        out["variants"].append({
            "workload": "batched_sweep_64: 64 independent 1DOF cylinder instances, "
                        "n_r ~ U[128,384], n_theta = 2 n_r, seed 0, FP32 storage",
            "nodes": nb,
            "steps": bsteps,
            "batched_MLUPS": round(nb * bsteps / (tb * 1e-3) / 1e6, 1),
            "batched_ms_per_step": round(tb / bsteps, 5),
            "schedule": {"grid": sched[0], "order": sched[1], "tile_shape": sched[2]},
            "collide_stream_ms": round(float(kb[0]), 5),
            "achieved_GBs": round(bpn * nb / (float(kb[0]) * 1e-3) / 1e9, 1),
            "one_at_a_time_MLUPS": round(nb * bsteps / (ts * 1e-3) / 1e6, 1),
            "finite_state": finb,
        })
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            out["cpu_baseline"], out["accuracy"] = (
                cpu_baseline_unstructured_cylinder(
                    heave_D=0.1 if "heave" in args.workload else 0.0)
                if args.workload.startswith("unstructured_cyl")
                else cpu_baseline_unstructured() if args.workload.startswith("unstructured")
                else cpu_baseline(case))
    print(json.dumps(out), flush=True)


def main_batched(args, storage: int):
    """The parameter sweep as the measured workload (its own JSON line)."""
    cases = synth.batched_sweep_cases(64)
    for c in cases:
        c.fluid.storage = storage
    N = sum(c.mesh.n_nodes for c in cases)
    total_ms, kms, sched, finite = time_batch(cases, args.steps, args.warmup)
    bpn = algorithmic_bytes_per_node(storage)
    k1_ms = float(kms[0])
    achieved = bpn * N / (k1_ms * 1e-3) / 1e9
    copy_ceiling = copy_ceiling_gbs()
    out = {
        "metric": METRIC,
        "value": round(N * args.steps / (total_ms * 1e-3) / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batched_sweep_64: {WORKLOADS['batched_sweep_64']}, {args.storage} "
                        f"population storage",
            "nodes": N,
            "storage": args.storage,
            "schedule": {"grid": sched[0], "order": sched[1], "tile_shape": sched[2]},
            "kernel_ms": {"collide_stream": round(k1_ms, 5),
                          "wall_targets_farfield": round(float(kms[1]), 5),
                          "wall_grad_traction": round(float(kms[2]), 5),
                          "body": round(float(kms[3]), 5)},
            "finite_state": finite,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_collide_stream",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "algorithmic_bytes_per_node": bpn,
            "copy_ceiling": copy_ceiling,
            "frac_of_copy": round(achieved / copy_ceiling["GBs"], 4),
        },
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
