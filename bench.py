"""Benchmark: D3Q19 MRT lattice Boltzmann step with the single-node boundary
scheme on a 256^3 random sphere packing (120 spheres, r ~ U[10, 20], seed 3,
pressure-driven x, tau = 0.7), on one MI355X.

Timed, each with inputs resident in HBM:
  * FP32 forward step (deviation storage): `value` = MLUPS over all N nodes,
    `ms_per_step` (median of windows of K steps), and the roofline of the
    step kernel from HIP events on the library's stream (algorithmic bytes
    2*Q*s*N_fluid + 48*N_links + N_nodes / median launch time);
  * FP64 forward step: MLUPS and the FP32/FP64 speedup;
  * the velocity difference between FP32 and FP64 after the workload's
    configured 500 steps;
  * FP32 and FP64 forward + adjoint: a checkpointed run of A steps followed
    by the reverse sweep (segment replay + adjoint steps + gradient sums), as
    MLUPS of differentiated time steps and the reverse/forward cost ratio;
  * the forward step of the other workloads (per_config);
  * the CPU oracle (numpy, float64) on a bounded slab of the same workload,
    on one thread and with all BLAS threads, with the CPU model.
Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per k_step<D3Q19, float> launch on this workload from rocprofv3
# FETCH_SIZE/WRITE_SIZE (scaled by a copy of known size), valid for the
# kernel sources with this hash (profiles/k_step_d3q19_fp32_spheres256.md).
MEASURED_TRAFFIC = {"sources_sha256_16": "1672476243682091", "bytes": 2600527467}
KERNEL_SOURCES = ["paper_1712_08288_amd/csrc/forward.hip",
                  "paper_1712_08288_amd/csrc/kernels.hpp",
                  "paper_1712_08288_amd/csrc/lattice.hpp"]


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(Q, s, n_nodes, n_fluid, n_links):
    """Algorithmic bytes of one forward step: each fluid node reads and
    writes Q values (2 Q s), each cut link moves 48 bytes of link data, and
    each node one byte of its type."""
    return 2 * Q * s * n_fluid + 48 * n_links + n_nodes


def kernel_bytes(Q, s, n_nodes, n_fluid, n_links):
    """The same with what this step kernel actually has to move: a 4-byte
    node word per node, and per cut link its direction byte, four
    coefficients in the populations' precision, one link-slot read and one
    link-slot write (25 bytes in FP32, 49 in FP64)."""
    return 2 * Q * s * n_fluid + 4 * n_nodes + n_links * (1 + 4 * s + 2 * s)


def timed_windows(sv, steps, windows):
    """`windows` timed windows of exactly `steps` steps, each between
    synchronisations: wall ms per step and the step kernel's HIP-event ms
    per step (library stream) of every window."""
    import torch
    walls, kers = [], []
    for _ in range(windows):
        sv.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv.step(steps)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3 / steps)
        kers.append(sv.last_step_ms())
        sv.set_timing(False)
    return walls, kers


def time_forward(binding, geom, w, precision, steps, warmup, windows=5):
    """W untimed steps, then `windows` windows of K steps; medians."""
    sv = binding.solver_for(geom, w.s, g=w.g, precision=precision, dp=w.dp, l_rule=w.l_rule)
    sv.init()
    sv.step(warmup)
    walls, kers = timed_windows(sv, steps, windows)
    return sv, float(np.median(walls)), float(np.median(kers)), walls, kers


def copy_ceiling(binding, torch, nbytes=1 << 31, reps=20, all_modes=False):
    """Best streaming-copy rate (read + write of nbytes) of the library's
    probe kernels, and of the HIP runtime copy used by torch."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    out = {"bytes": nbytes}
    best = 0.0
    for mode in (0, 1, 2):
        ms = binding.stream_copy(b, a, nbytes, mode=mode, reps=reps)
        gbs = 2 * nbytes / (ms * 1e-3) / 1e9
        out["mode%d_GBps" % mode] = round(gbs, 1)
        best = max(best, gbs)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    out["hip_memcpy_GBps"] = round(2 * nbytes / ((time.perf_counter() - t0) / reps) / 1e9, 1)
    out["best_GBps"] = round(best, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def pattern_ceiling(binding, torch, shape=(256, 256, 256), reps=20):
    """Rate of the step's own access pattern without its arithmetic (every
    plane read at the pull source, written at the node; D3Q19 FP32), raw
    bytes moved per second."""
    n = int(np.prod(shape))
    a = torch.empty(binding.population_elements("D3Q19", shape), dtype=torch.float32,
                    device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    ms = binding.pull_pattern_copy("D3Q19", "fp32", b, a, shape, reps=reps)
    del a, b
    torch.cuda.empty_cache()
    return 2 * 19 * n * 4 / (ms * 1e-3) / 1e9


def adjoint_pattern_ceiling(binding, torch, shape=(256, 256, 256), reps=20):
    """Rate of the adjoint step's access pattern without its arithmetic (the
    forward state pulled, the adjoint gathered from x + e_i, the result
    written; D3Q19 FP32), raw bytes moved per second."""
    n = int(np.prod(shape))
    a = torch.empty(binding.population_elements("D3Q19", shape), dtype=torch.float32,
                    device="cuda").fill_(1.0)
    b = torch.empty_like(a).fill_(2.0)
    c = torch.empty_like(a)
    ms = binding.adjoint_pattern_copy("D3Q19", "fp32", c, a, b, shape, reps=reps)
    del a, b, c
    torch.cuda.empty_cache()
    return 3 * 19 * n * 4 / (ms * 1e-3) / 1e9


def pattern_study(binding, torch, shape=(256, 256, 256), reps=20):
    """Raw GB/s of D3Q19 access patterns without arithmetic, FP32 and FP64:
    the step's pull in the engine's layout (blocks of 2048 nodes holding
    their Q direction runs), the same pull with blocks of B nodes (B = N:
    one plane per direction), the in-place two-pass (AA) pattern on planes,
    the adjoint's pattern, and a flat copy of the same bytes."""
    n = int(np.prod(shape))
    out = {"shape": list(shape)}
    for prec, dt, s in (("fp32", torch.float32, 4), ("fp64", torch.float64, 8)):
        a = torch.ones(binding.population_elements("D3Q19", shape), dtype=dt, device="cuda")
        b = torch.empty_like(a)
        raw = 2 * 19 * n * s
        r = {}
        ms = min(binding.stream_copy(b, a, 19 * n * s, mode=m, reps=reps) for m in (0, 1, 2))
        r["copy"] = round(raw / (ms * 1e-3) / 1e9, 1)
        r["pull"] = round(raw / (binding.pull_pattern_copy("D3Q19", prec, b, a, shape, reps=reps) * 1e-3) / 1e9, 1)
        for B in (256, 1024, 4096, 16384, n):
            ms = binding.blocked_pull_pattern_copy("D3Q19", prec, B, b, a, shape, reps=reps)
            r["pull_planes" if B == n else "pull_blocks_%d" % B] = round(raw / (ms * 1e-3) / 1e9, 1)
        e_ms, o_ms = binding.aa_pattern_copy("D3Q19", prec, a, shape, reps=reps)
        r["aa_even"] = round(raw / (e_ms * 1e-3) / 1e9, 1)
        r["aa_odd"] = round(raw / (o_ms * 1e-3) / 1e9, 1)
        r["aa_two_pass"] = round(2 * raw / ((e_ms + o_ms) * 1e-3) / 1e9, 1)
        c = torch.empty_like(a)
        ms = binding.adjoint_pattern_copy("D3Q19", prec, c, a, b, shape, reps=reps)
        r["adjoint_pattern"] = round(3 * 19 * n * s / (ms * 1e-3) / 1e9, 1)
        del a, b, c
        torch.cuda.empty_cache()
        out[prec] = r
    return out


def cpu_baseline(geom, w, slab=48, steps=20, threads=None):
    """Oracle on the z-slab 0 <= z < slab of the same workload (window mode:
    reads across the slab faces see NaN and are not used; slab=None runs the
    whole domain).  threads limits the BLAS threads (None: all).  The
    oracle's elementwise numpy work runs on one thread whatever the limit;
    only its dense moment products use the BLAS threads."""
    from oracle.lbm import Oracle
    import contextlib
    try:
        import threadpoolctl
        ctl = threadpoolctl.threadpool_limits(threads) if threads else contextlib.nullcontext()
    except Exception:
        threadpoolctl, ctl = None, contextlib.nullcontext()
    with ctl:
        used = (max(i["num_threads"] for i in threadpoolctl.threadpool_info())
                if threadpoolctl else 1)
        nx, ny, nz = geom.shape
        plane = nx * ny if nz > 1 else nx          # slab: z-planes (3D) or rows (2D)
        depth = nz if nz > 1 else ny
        zs = depth if slab is None else min(slab, depth)
        nodes = None if zs == depth else np.arange(plane * zs, dtype=np.int64)
        n = plane * zs
        o = Oracle(geom, w.s, g=w.g, dp=w.dp, l_rule=w.l_rule, nodes=nodes)
        f = o.init_equilibrium()
        t0 = time.perf_counter()
        o.run(f, steps)
        dt = time.perf_counter() - t0
    fluid = int((geom.solid.reshape(-1)[:n] == 0).sum())
    return {"value": round(n * steps / dt / 1e6, 4), "unit": "MLUPS",
            "fluid_mlups": round(fluid * steps / dt / 1e6, 4),
            "cores": int(used), "kind": "oracle",
            "sample": "%d steps on %s (%d nodes) of the same geometry, numpy float64 "
                      "(BLAS threads %d), %.1f s"
                      % (steps, "the whole %dx%dx%d domain" % (nx, ny, nz) if nodes is None
                         else ("the %dx%dx%d z-slab" % (nx, ny, zs) if nz > 1
                               else "the %dx%d row slab" % (nx, zs)), n, used, dt)}


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "cores_available": len(os.sched_getaffinity(0))}


def _timed_steps(sv, n):
    import torch
    torch.cuda.synchronize()
    sv.set_timing(True)
    t0 = time.perf_counter()
    sv.step(n)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / max(n, 1)
    ms = sv.last_step_ms()
    sv.set_timing(False)
    return ms, wall


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _progress(what):
    print("[bench] " + what, file=sys.stderr, flush=True)


def pattern_rate(binding, torch, lattice, shape, prec, Q):
    """Raw bytes per second of the step's pull pattern without arithmetic on
    this grid and precision (the kernel's own ceiling)."""
    n = int(np.prod(shape))
    dt = torch.float32 if prec == "fp32" else torch.float64
    a = torch.ones(binding.population_elements(lattice, shape), dtype=dt, device="cuda")
    b = torch.empty_like(a)
    ms = binding.pull_pattern_copy(lattice, prec, b, a, shape, reps=10)
    del a, b
    torch.cuda.empty_cache()
    return 2 * Q * n * (4 if prec == "fp32" else 8) / (ms * 1e-3) / 1e9


def fwd_rev(sv, steps, every, torch):
    """Forward + adjoint of `steps` steps (checkpoint every `every`; the
    mean-u_x objective over them, gradients in g and every q, rate gradients
    off so the reverse sweep reads step records).  One untimed cycle
    allocates the checkpoints, the replay pool and the adjoint arrays (kept);
    the second is timed.  The per-link gradients end in device tensors, as
    the autograd path returns them.  Returns J, the gradients and the
    forward and reverse ms per step; the state is restored."""
    sv.set_rate_gradient(False)
    state0 = torch.empty(sv.state_bytes(), dtype=torch.uint8, device="cuda")
    sv.get_state(state0)
    t_start = sv.time
    nl = sv.counts()[1]
    dq_dev = torch.empty(nl, dtype=torch.float64, device="cuda")
    du_dev = torch.empty((nl, 3), dtype=torch.float64, device="cuda")
    for _ in range(2):
        sv.set_state(state0, t_start)
        sv.set_objective("mean_ux", 0, t_start, t_start + steps)
        torch.cuda.synchronize()
        a = time.perf_counter()
        sv.run_checkpointed(steps, every)
        torch.cuda.synchronize()
        b = time.perf_counter()
        sv.adjoint()
        gr = sv.grad_device(dq_dev, du_dev)
        torch.cuda.synchronize()
        c = time.perf_counter()
    sv.set_state(state0, t_start)
    return sv.objective(), gr, (b - a) * 1e3 / steps, (c - b) * 1e3 / steps


def per_config_forward(binding, torch, windows=3):
    """The forward step of every workload in its benchmark precisions, from
    rest: MLUPS over all nodes, the HBM fraction by the algorithmic bytes
    2*Q*s*N_fluid + 48*N_links + N_nodes, and the fraction of the step's own access pattern on
    the same grid (periodic, no arithmetic).  Medians over `windows` timed
    windows.  The 256^3 sphere packing is the headline line itself; one
    GPU's z-slab share of it (256x256x32) is measured here at its real
    shape."""
    from workloads import configs
    plan = [("c1_couette_64", configs.c1_couette(64), ("fp64",), 640),
            ("c2_cylinders_2048", configs.c2_cylinders(), ("fp64", "fp32"), 200),
            ("c4_cylinder_1024x512", configs.c4_cylinder(), ("fp64", "fp32"), 200),
            ("c5_porous_384x256x256", configs.c5_porous(), ("fp32",), 100),
            ("c3_shard_256x256x32", configs.c3_shard(), ("fp32", "fp64"), 200)]
    out = {}
    for name, w, precs, steps in plan:
        geom = w.geometry()
        Q = 9 if geom.lattice == "D2Q9" else 19
        res = {"n_nodes": geom.n_nodes, "n_fluid": geom.n_fluid, "n_links": geom.n_links}
        for prec in precs:
            s = 4 if prec == "fp32" else 8
            sv = binding.solver_for(geom, w.s, g=w.g, precision=prec, dp=w.dp, l_rule=w.l_rule)
            sv.init()
            sv.step(20)
            walls, kers = timed_windows(sv, steps, windows)
            rev = None
            if name.startswith("c3_shard") and prec == "fp32":
                # the reverse sweep at the shard's shape too: 64 steps, every
                # step recorded
                _, _, ms_f, ms_r = fwd_rev(sv, 64, 1, torch)
                rev = {"ms_per_step_forward_recording": round(ms_f, 5),
                       "ms_per_step_reverse": round(ms_r, 5)}
            sv.close()
            ms, kms = float(np.median(walls)), float(np.median(kers))
            by = algorithmic_bytes(Q, s, geom.n_nodes, geom.n_fluid, geom.n_links)
            pat = pattern_rate(binding, torch, geom.lattice, geom.shape, prec, Q)
            res[prec] = {"ms_per_step": round(ms, 5), "kernel_ms": round(kms, 5),
                         "mlups": round(geom.n_nodes / (ms * 1e-3) / 1e6, 1),
                         "fluid_mlups": round(geom.n_fluid / (ms * 1e-3) / 1e6, 1),
                         "algorithmic_GBps": round(by / (kms * 1e-3) / 1e9, 1),
                         "hbm_frac": round(by / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "pattern_ceiling_GBps": round(pat, 1),
                         "frac_of_pattern": round(by / (kms * 1e-3) / 1e9 / pat, 4)}
            if rev:
                res[prec]["adjoint_every_step_recorded"] = rev
        if name.startswith("c1"):
            res["note"] = "0.6 MB working set, graph replay: launch-bound, not an HBM measurement"
        if name.startswith("c4"):
            res["note"] = "19-38 MB working set: runs partly from the 256 MB last-level cache"
        if name.startswith("c3_shard"):
            res["note"] = ("one of eight z-slabs of the 256^3 packing at its real shape "
                           "(independent packing of the same density, periodic in z)")
        out[name] = res
        del geom
    return out


def next_rows_forward(binding, torch, geom, w, steps=100, windows=3):
    """The forward step of the follow-on variants on the benchmark workload
    (256^3, same spheres and seam): the two-node scheme Eq. (211), the b
    family Eq. (213) at b = 0.7, TRT through the MRT rates, and the D3Q15
    lattice on the same spheres; FP32 (and FP64 for D3Q15).  Kernel time
    from HIP events, medians over `windows` windows; the HBM fraction by the
    same algorithmic bytes for the variant's Q."""
    from workloads import configs
    from workloads import geometry as G
    out = {}

    def one(g, s, prec, Q, collision=None, **kw):
        sv = binding.solver_for(g, s, g=w.g, precision=prec, dp=w.dp, l_rule=w.l_rule, **kw)
        if collision:
            sv.set_collision(*collision)
        sv.init()
        sv.step(20)
        walls, kers = timed_windows(sv, steps, windows)
        sv.close()
        ms, kms = float(np.median(walls)), float(np.median(kers))
        by = algorithmic_bytes(Q, 4 if prec == "fp32" else 8, g.n_nodes, g.n_fluid, g.n_links)
        return {"ms_per_step": round(ms, 5), "kernel_ms": round(kms, 5),
                "mlups": round(g.n_nodes / (ms * 1e-3) / 1e6, 1),
                "hbm_frac": round(by / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out["two_node_eq211_fp32"] = one(geom, w.s, "fp32", 19, two_node=True)
    out["b_0.7_eq213_fp32"] = one(geom, w.s, "fp32", 19, b=0.7)
    out["trt_fp32"] = one(geom, w.s, "fp32", 19, collision=("trt", 1.0 / 0.7))
    n = geom.shape[0]
    g15 = G.random_spheres(n, n, n, 120, 10.0, 20.0, 3, x_bc="pressure", lattice="D3Q15")
    s15 = configs.d3q15_paper_rates(1.0 / 0.7)
    res = {"n_fluid": g15.n_fluid, "n_links": g15.n_links}
    for prec in ("fp32", "fp64"):
        res[prec] = one(g15, s15, prec, 15)
        res[prec]["pattern_ceiling_GBps"] = round(
            pattern_rate(binding, torch, "D3Q15", g15.shape, prec, 15), 1)
    out["d3q15_256"] = res
    del g15
    return out


def all_configs(binding, torch):
    """Every benchmark workload: MLUPS and HBM fraction per precision,
    accuracy figures, and the checkpointed adjoints of C4 and C5."""
    from workloads import analytic, configs
    out = {}

    def fwd(w, geom, prec, steps, warm=10, **kw):
        sv = binding.solver_for(geom, w.s, g=w.g, precision=prec, dp=w.dp,
                                l_rule=w.l_rule, **kw)
        sv.init()
        sv.step(warm)
        ms, wall = _timed_steps(sv, steps)
        Q = 9 if geom.lattice == "D2Q9" else 19
        by = algorithmic_bytes(Q, 4 if prec == "fp32" else 8, geom.n_nodes,
                               geom.n_fluid, geom.n_links)
        pat = pattern_rate(binding, torch, geom.lattice, geom.shape, prec, Q)
        return sv, {"ms_per_step": round(ms, 5), "wall_ms_per_step": round(wall, 5),
                    "mlups": round(geom.n_nodes / (ms * 1e-3) / 1e6, 1),
                    "hbm_frac": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "pattern_ceiling_GBps": round(pat, 1),
                    "algorithmic_frac_of_pattern": round(by / (ms * 1e-3) / 1e9 / pat, 4)}

    _progress("C1")
    # C1: circular Couette, FP64, refinement under diffusive scaling
    errs, sizes = [], [32, 64, 128]
    for n in sizes:
        w = configs.c1_couette(n)
        geom = w.geometry()
        sv = binding.solver_for(geom, w.s, precision="fp64", l_rule=w.l_rule)
        sv.init()
        ms, wall = _timed_steps(sv, w.steps)
        _, u = sv.moments()
        sv.close()
        e = analytic.relative_l2(u, analytic.couette_velocity(geom), geom.solid == 0)
        errs.append(e)
        if n == 64:
            by = algorithmic_bytes(9, 8, geom.n_nodes, geom.n_fluid, geom.n_links)
            out["c1_couette_64"] = {"steps": w.steps, "ms_per_step": round(ms, 5),
                                    "mlups": round(geom.n_nodes / (ms * 1e-3) / 1e6, 1),
                                    "hbm_frac": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                    "note": "0.6 MB working set: launch-bound, not an HBM measurement",
                                    "u_rel_l2_vs_analytic": e}
    out["c1_refinement"] = {"sizes": sizes, "u_rel_l2": errs,
                            "fitted_order": float(-np.polyfit(np.log(sizes), np.log(errs), 1)[0])}

    _progress("C2")
    # C2: 2048^2 cylinders, FP64 and FP32, 1000 steps
    w = configs.c2_cylinders()
    geom = w.geometry()
    res = {"n_fluid": geom.n_fluid, "n_links": geom.n_links}
    us = {}
    for prec in ("fp64", "fp32"):
        sv, r = fwd(w, geom, prec, w.steps - 10)
        _, us[prec] = sv.moments()
        sv.close()
        res[prec] = r
    fl = geom.solid == 0
    res["u_rel_l2_fp32_vs_fp64"] = _rel(us["fp32"][fl], us["fp64"][fl])
    out["c2_cylinders_2048"] = res

    _progress("C3")
    # C3: 256^3 spheres, 500 steps in both precisions
    w = configs.c3_spheres()
    geom = w.geometry()
    res = {}
    for prec in ("fp32", "fp64"):
        sv, r = fwd(w, geom, prec, w.steps - 10)
        _, us[prec] = sv.moments()
        sv.close()
        res[prec] = r
    fl = geom.solid == 0
    res["u_rel_l2_fp32_vs_fp64"] = _rel(us["fp32"][fl], us["fp64"][fl])
    res["speedup_fp32_over_fp64"] = round(res["fp64"]["ms_per_step"] / res["fp32"]["ms_per_step"], 3)
    out["c3_spheres_256"] = res
    del geom

    _progress("C4")
    # C4: channel + cylinder, drag over the last 1000 of 3000 steps, sqrt(N)
    # checkpointing, gradients in q, u_in and tau; FD checks in FP64
    w = configs.c4_cylinder()
    geom = w.geometry()
    t0, t1 = w.extra["obj_window"]
    every = int(round(np.sqrt(w.steps)))
    res = {"n_links": geom.n_links, "checkpoint_every": every}
    for prec in ("fp64", "fp32"):
        sv, r = fwd(w, geom, prec, 500)
        sv.close()
        res["forward_" + prec] = r
    for prec in ("fp64", "fp32"):
        sv = binding.solver_for(geom, w.s, precision=prec, l_rule=w.l_rule)
        sv.init()
        sv.set_objective("force_x", 1, t0, t1)
        torch.cuda.synchronize()
        a = time.perf_counter()
        sv.run_checkpointed(w.steps, every)
        torch.cuda.synchronize()
        b = time.perf_counter()
        sv.adjoint()
        gr = sv.grad()
        torch.cuda.synchronize()
        c = time.perf_counter()
        J = sv.objective()
        inlet = geom.tag == 2
        tau = 1.0 / w.s[7]
        r = {"J_drag": J, "dJ_du_in": float(gr["wall_u"][inlet, 0].sum()),
             "dJ_dtau": float(-(gr["s"][7] + gr["s"][8]) * w.s[7] ** 2),
             "forward_s": round(b - a, 4), "reverse_s": round(c - b, 4),
             "reverse_over_forward": round((c - b) / (b - a), 3)}
        if prec == "fp64":
            h = 1e-6

            def J_at(q=geom.q, wu=geom.wall_u, s=w.s):
                sv.update_links(q, wu)
                sv.set_parameters(s, (0.0, 0.0))
                sv.init()
                sv.set_objective("force_x", 1, t0, t1)
                sv.step(w.steps)
                return sv.objective()
            up, um = geom.wall_u.copy(), geom.wall_u.copy()
            up[inlet, 0] += h
            um[inlet, 0] -= h
            fd_u = (J_at(wu=up) - J_at(wu=um)) / (2 * h)
            sp, sm = w.s.copy(), w.s.copy()
            sp[7:9] = 1.0 / (tau + h)
            sm[7:9] = 1.0 / (tau - h)
            fd_tau = (J_at(s=sp) - J_at(s=sm)) / (2 * h)
            # a single link moves J by ~1e-9: a larger step keeps the
            # difference above round-off, away from the l-rule kink at 1/2
            hq = 1e-4
            cyl = np.nonzero((geom.tag == 1) & (np.abs(geom.q - 0.5) > 10 * hq))[0]
            k = cyl[np.argsort(-np.abs(gr["q"][cyl]))[:3]]
            fd_q = []
            for kk in k:
                qp, qm = geom.q.copy(), geom.q.copy()
                qp[kk] += hq
                qm[kk] -= hq
                fd_q.append((J_at(q=qp) - J_at(q=qm)) / (2 * hq))
            r["fd_rel_err"] = {"u_in": abs(fd_u - r["dJ_du_in"]) / abs(fd_u),
                               "tau": abs(fd_tau - r["dJ_dtau"]) / abs(fd_tau),
                               "q_top3": [abs(f - gr["q"][kk]) / abs(f) for f, kk in zip(fd_q, k)]}
            g64 = gr
        else:
            ref = res["fp64"]["dJ_du_in"]
            r["grad_rel_err_vs_fp64"] = {"q": _rel(gr["q"], g64["q"]),
                                         "u_in": abs(r["dJ_du_in"] - ref) / abs(ref)}
        sv.close()
        res[prec] = r
    out["c4_cylinder_1024x512"] = res

    _progress("C5")
    # C5: 384x256x256 porous medium, FP32, 2000 steps + adjoint, every 64
    w = configs.c5_porous()
    geom = w.geometry()
    sv, c5_fwd = fwd(w, geom, "fp32", 200)
    sv.close()
    sv = binding.solver_for(geom, w.s, g=w.g, precision="fp32", l_rule=w.l_rule)
    sv.set_rate_gradient(False)
    sv.init()
    sv.set_objective("mean_ux", 0, w.steps - 500, w.steps)
    torch.cuda.synchronize()
    a = time.perf_counter()
    sv.run_checkpointed(w.steps, 64)
    torch.cuda.synchronize()
    b = time.perf_counter()
    sv.adjoint()
    gr = sv.grad()
    torch.cuda.synchronize()
    c = time.perf_counter()
    J = sv.objective()
    sv.close()
    out["c5_porous_384x256x256"] = {
        "n_fluid": geom.n_fluid, "n_links": geom.n_links, "J_mean_ux": J,
        "dJ_dgx": float(gr["g"][0]), "J_over_gx": J / w.g[0],
        "forward": c5_fwd,
        "forward_ms_per_step": round((b - a) * 1e3 / w.steps, 4),
        "reverse_ms_per_step": round((c - b) * 1e3 / w.steps, 4)}
    del geom
    # crop-sized medium: FP32 gradient against the FP64 GPU gradient
    w = configs.c5_crop(steps=400)
    geom = w.geometry()
    gsets = {}
    for prec in ("fp64", "fp32"):
        sv = binding.solver_for(geom, w.s, g=w.g, precision=prec, l_rule=w.l_rule)
        sv.init()
        sv.set_objective("mean_ux", 0, w.steps - 100, w.steps)
        sv.run_checkpointed(w.steps, 20)
        sv.adjoint()
        gsets[prec] = (sv.objective(), sv.grad())
        sv.close()
    out["c5_crop_96x64x64"] = {
        "steps": w.steps,
        "J_rel_err_fp32": abs(gsets["fp32"][0] - gsets["fp64"][0]) / abs(gsets["fp64"][0]),
        "dJ_dg_rel_err_fp32": _rel(gsets["fp32"][1]["g"], gsets["fp64"][1]["g"]),
        "dJ_dq_rel_l2_fp32": _rel(gsets["fp32"][1]["q"], gsets["fp64"][1]["q"])}

    # the FP64 oracle on the host's cores at every workload (bounded samples;
    # a baseline, not the target): all available cores and one core
    _progress("CPU oracle per workload")
    cpu = {"host": host_info()}
    samples = [("c1_couette_64", configs.c1_couette(64), None, 500),
               ("c2_cylinders_2048", configs.c2_cylinders(), 256, 10),
               ("c3_spheres_256", configs.c3_spheres(), 48, 10),
               ("c4_cylinder_1024x512", configs.c4_cylinder(), None, 10),
               ("c5_porous_384x256x256", configs.c5_porous(), 24, 5),
               ("c5_crop_96x64x64", configs.c5_crop(), None, 20)]
    for name, w, slab, steps in samples:
        geom = w.geometry()
        cpu[name] = {"all_cores": cpu_baseline(geom, w, slab=slab, steps=steps),
                     "one_core": cpu_baseline(geom, w, slab=slab, steps=max(2, steps // 2),
                                              threads=1)}
        del geom
    out["cpu_oracle"] = cpu
    return out


def run_study(name):
    """One of the paper's Section 3 sweeps on the GPU; one JSON line per
    (rule, gamma, s_nu, ...) group with the errors and the fitted order."""
    from paper_1712_08288_amd import studies
    log = _progress
    t0 = time.time()
    if name == "poiseuille":
        out = studies.poiseuille_study(log=log, max_size_by_snu={1.99: 41})
    elif name == "taylor_green":
        out = studies.taylor_green_study(log=log)
    elif name == "hagen_poiseuille":
        out = studies.hagen_poiseuille_study(lattice="D3Q15", log=log, max_size_by_snu={1.99: 40})
    elif name == "hagen_poiseuille_d3q19":
        out = studies.hagen_poiseuille_study(lattice="D3Q19", log=log, max_size_by_snu={1.99: 40})
    elif name == "b":
        out = studies.b_study(log=log)
    elif name == "b_bgk":   # does b < 1 stabilise BGK / TRT where they fail at b = 1?
        out = []
        for col in ("bgk", "trt"):
            out += studies.b_study(bs=(1.0, 0.9, 0.7, 0.5, 0.3), s_nus=(1.99,), rules=("gamma",),
                                   sizes=(11, 21, 41), gamma=0.25, collision=col, log=log)
    else:   # collisions: BGK, TRT and MRT (and Eq. (211)) on the same sweep
        out = []
        for kw in (dict(collision="bgk"), dict(collision="trt"), dict(two_node=True)):
            out += studies.poiseuille_study(rules=["gamma", "gamma2"], gammas=(0.25, 0.75),
                                            s_nus=(0.5, 1.0, 1.5, 1.99), sizes=(11, 21, 41, 61),
                                            max_size_by_snu={1.99: 41}, log=log, **kw)
    for r in out:
        print(json.dumps({"study": name, **r}), flush=True)
    _progress("study %s: %d groups in %.0f s" % (name, len(out), time.time() - t0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--adjoint-steps", type=int, default=64)
    ap.add_argument("--every", type=int, default=8)
    ap.add_argument("--n", type=int, default=256, help="lattice edge (256 = the benchmark)")
    ap.add_argument("--windows", type=int, default=5,
                    help="timed windows of --steps steps (the median is reported)")
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the forward step of the other workloads")
    ap.add_argument("--study", choices=["poiseuille", "taylor_green", "hagen_poiseuille",
                                        "hagen_poiseuille_d3q19", "b", "b_bgk", "collisions"],
                    help="run one of the paper's Section 3 sweeps on the GPU instead")
    ap.add_argument("--all", action="store_true",
                    help="also measure every workload (C1-C5) in detail into 'all_configs'")
    ap.add_argument("--only", choices=["fwd32", "fwd64", "adjoint32", "copy", "pattern"],
                    help="profiling runs: time only this part and print its line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path is a single-GPU kernel "
              "(multi-GPU slab decomposition is a design, not built); got --gpus %d"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_1712_08288_amd import binding
    from workloads import configs

    if args.study:
        run_study(args.study)
        return

    if args.only == "copy":
        # reference copies of known size: HBM ceiling and counter scaling
        print(json.dumps(copy_ceiling(binding, torch, reps=args.steps, all_modes=True)))
        return
    if args.only == "pattern":
        # the step's and the adjoint's access patterns without arithmetic,
        # and the alternatives to the step's layout and addressing
        print(json.dumps(pattern_study(binding, torch, reps=args.steps)))
        return

    w = configs.c3_spheres(args.n)
    geom = w.geometry()
    N, NF, NL = geom.n_nodes, geom.n_fluid, geom.n_links
    if args.only in ("fwd32", "fwd64"):
        prec = args.only.replace("fwd", "fp")
        sv, ms, kms, _, _ = time_forward(binding, geom, w, prec, args.steps, args.warmup, windows=1)
        s = 4 if prec == "fp32" else 8
        by = algorithmic_bytes(19, s, N, NF, NL)
        print(json.dumps({"only": args.only, "ms_per_step": ms, "kernel_ms": kms,
                          "algorithmic_bytes": by, "GBps": by / (kms * 1e-3) / 1e9}))
        sv.close()
        return
    if args.only == "adjoint32":
        sv = binding.solver_for(geom, w.s, precision="fp32", dp=w.dp, l_rule=w.l_rule)
        sv.init()
        sv.step(args.warmup)
        sv.set_rate_gradient(False)
        sv.set_objective("mean_ux", 0, sv.time, sv.time + args.adjoint_steps)
        sv.run_checkpointed(args.adjoint_steps, args.every)
        sv.adjoint()
        g = sv.grad()
        torch.cuda.synchronize()
        print(json.dumps({"only": "adjoint32", "dJ_dg": [float(v) for v in g["g"]]}))
        sv.close()
        return

    W, K, R = args.warmup, args.steps, args.windows
    _progress("FP32 and FP64 forward: %d warm-up steps, %d windows of %d steps" % (W, R, K))
    # FP32 forward (headline): median over R windows of exactly K steps
    sv32, ms32, kms32, walls32, kers32 = time_forward(binding, geom, w, "fp32", K, W, R)
    # FP64 forward
    sv64, ms64, kms64, walls64, kers64 = time_forward(binding, geom, w, "fp64", K, W, R)
    # FP32 against FP64 after the workload's configured steps (both from rest)
    t_cmp = max(w.steps, sv32.time)
    sv32.step(t_cmp - sv32.time)
    sv64.step(t_cmp - sv64.time)
    _, u32 = sv32.moments()
    _, u64 = sv64.moments()
    fl = geom.solid == 0
    du = float(np.sqrt(((u32 - u64)[fl] ** 2).sum() / (u64[fl] ** 2).sum()))
    del u32, u64

    # forward + adjoint (checkpointed run, then the reverse sweep), both
    # precisions; mean u_x over the window, gradients in g and every q
    A = args.adjoint_steps

    _progress("FP64 forward + adjoint")
    J64, g64, ms64_fwd_ckpt, ms64_adj = fwd_rev(sv64, A, args.every, torch)
    sv64.close()
    _progress("FP32 forward + adjoint")
    J32, g32, ms_fwd_ckpt, ms_adj = fwd_rev(sv32, A, args.every, torch)
    # every step recorded (no snapshot, no replay): A step records of 3
    # values per node and 3 per link, 14 GB at 256^3 FP32 with A = 64
    _, _, ms_fwd_all, ms_adj_all = fwd_rev(sv32, A, 1, torch)
    sv32.close()
    torch.cuda.empty_cache()

    _progress("ceilings")
    ceiling = copy_ceiling(binding, torch)
    pattern = pattern_ceiling(binding, torch)
    adj_pattern = adjoint_pattern_ceiling(binding, torch)
    traffic = (MEASURED_TRAFFIC["bytes"]
               if kernel_sources_hash() == MEASURED_TRAFFIC["sources_sha256_16"] else None)
    bytes32 = algorithmic_bytes(19, 4, N, NF, NL)
    bytes64 = algorithmic_bytes(19, 8, N, NF, NL)
    kbytes32 = kernel_bytes(19, 4, N, NF, NL)
    achieved = bytes32 / (kms32 * 1e-3) / 1e9
    frac = achieved / HBM_PEAK_GBS
    mlups32 = N / (ms32 * 1e-3) / 1e6
    mlups64 = N / (ms64 * 1e-3) / 1e6
    out = {
        "metric": "MLUPS & % HBM roofline, D3Q19 MRT 256^3 fwd+adjoint, FP32 vs FP64",
        "value": round(mlups32, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "timing": "median over %d windows of exactly %d steps, each between device "
                  "synchronisations, after %d untimed steps" % (R, K, W),
        "config": {
            "workload": "D3Q19 MRT %d^3, 120 random spheres r~U[10,20] seed 3, "
                        "pressure-driven x drho=1e-3, tau=0.7, l=max(0,2q-1), "
                        "FP32 deviation storage, forward step" % args.n,
            "n_nodes": N, "n_fluid": NF, "n_links": NL,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(frac, 4),
            "traffic": traffic,
            "traffic_source": ("rocprofv3 FETCH_SIZE + WRITE_SIZE per launch of this kernel "
                               "source (hash %s), scaled by a copy of known size; "
                               "profiles/k_step_d3q19_fp32_spheres256.md; null when the "
                               "kernel source changed since" % MEASURED_TRAFFIC["sources_sha256_16"]),
            "kernel": "k_step<D3Q19,float,pressure>",
            "kernel_ms": round(kms32, 4),
            "windows_kernel_ms": [round(v, 4) for v in kers32],
            "algorithmic_bytes": int(bytes32),
            "algorithmic_bytes_rule": "2*Q*s*N_fluid + 48*N_links + N_nodes",
            "kernel_count_bytes": int(kbytes32),
            "kernel_count_frac": round(kbytes32 / (kms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "target_frac": 0.70,
            "target_met": bool(frac >= 0.70),
            "copy_ceiling_GBps": ceiling["best_GBps"],
            "frac_of_copy_ceiling": round(achieved / ceiling["best_GBps"], 4),
            # the same access pattern without the arithmetic, measured here;
            # compared with the kernel's measured HBM bytes per second
            "pattern_ceiling_GBps": round(pattern, 1),
            "traffic_GBps": (round(traffic / (kms32 * 1e-3) / 1e9, 1) if traffic else None),
            "frac_of_pattern_ceiling": round((traffic or kbytes32) / (kms32 * 1e-3) / 1e9 / pattern, 4),
        },
        "windows_ms_per_step": [round(v, 4) for v in walls32],
        "fluid_mlups": round(NF / (ms32 * 1e-3) / 1e6, 1),
        "fp64": {
            "mlups": round(mlups64, 1), "ms_per_step": round(ms64, 4),
            "fluid_mlups": round(NF / (ms64 * 1e-3) / 1e6, 1),
            "kernel_ms": round(kms64, 4),
            "hbm_frac": round(bytes64 / (kms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "fp32_over_fp64_speedup": round(ms64 / ms32, 3),
        },
        "fp32_vs_fp64": {"steps": int(t_cmp), "u_rel_l2": du},
        "adjoint": {
            "steps": A, "checkpoint_every": args.every,
            "objective": "mean u_x over the window; gradients in g and every gamma",
            "fp32": {
                "J": J32, "dJ_dg": [float(v) for v in g32["g"]],
                "ms_per_step_checkpointed_forward": round(ms_fwd_ckpt, 4),
                "ms_per_step_reverse": round(ms_adj, 4),
                "fwd_adjoint_mlups": round(N / ((ms_fwd_ckpt + ms_adj) * 1e-3) / 1e6, 1),
                "reverse_over_forward": round(ms_adj / ms32, 3),
                "forward_plus_reverse_over_forward": round((ms_fwd_ckpt + ms_adj) / ms32, 3),
                "every_step_recorded": {
                    "ms_per_step_forward": round(ms_fwd_all, 4),
                    "ms_per_step_reverse": round(ms_adj_all, 4),
                    "fwd_adjoint_mlups": round(N / ((ms_fwd_all + ms_adj_all) * 1e-3) / 1e6, 1),
                    "reverse_over_forward": round(ms_adj_all / ms32, 3)},
            },
            "fp64": {
                "J": J64, "dJ_dg": [float(v) for v in g64["g"]],
                "ms_per_step_checkpointed_forward": round(ms64_fwd_ckpt, 4),
                "ms_per_step_reverse": round(ms64_adj, 4),
                "fwd_adjoint_mlups": round(N / ((ms64_fwd_ckpt + ms64_adj) * 1e-3) / 1e6, 1),
                "reverse_over_forward": round(ms64_adj / ms64, 3),
                "forward_plus_reverse_over_forward": round((ms64_fwd_ckpt + ms64_adj) / ms64, 3),
            },
            "fp32_vs_fp64": {"J_rel": abs(J32 - J64) / abs(J64),
                             "dJ_dg_rel": _rel(g32["g"], g64["g"])},
            # the adjoint's access pattern without arithmetic, raw bytes
            # per second (the adjoint kernels' own ceiling)
            "pattern_ceiling_GBps": round(adj_pattern, 1),
        },
    }
    if not args.no_configs:
        _progress("follow-on variants of the step")
        out["next_rows"] = next_rows_forward(binding, torch, geom, w)
        del geom
        _progress("forward step of every workload")
        out["per_config"] = per_config_forward(binding, torch)
    if not args.no_cpu:
        _progress("CPU oracle")
        geom = w.geometry()
        one = cpu_baseline(geom, w, steps=args.cpu_steps, threads=1)
        many = cpu_baseline(geom, w, steps=args.cpu_steps)
        out["cpu_baseline"] = dict(one, all_cores=many, **host_info())
    if args.all:
        out["all_configs"] = all_configs(binding, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
