"""Benchmark: D3Q19 MRT lattice Boltzmann step with the single-node boundary
scheme on a 256^3 random sphere packing (120 spheres, r ~ U[10, 20], seed 3,
pressure-driven x, tau = 0.7), on one MI355X.

Timed, each with inputs resident in HBM:
  * FP32 forward step (deviation storage): `value` = MLUPS over all N nodes,
    `ms_per_step`, and the roofline of the step kernel from HIP events on the
    library's stream (algorithmic bytes / average launch time);
  * FP64 forward step: MLUPS and the FP32/FP64 speedup;
  * FP32 forward + adjoint: a checkpointed run of A steps followed by the
    reverse sweep (segment replay + adjoint steps + gradient sums), as MLUPS
    of differentiated time steps and the adjoint/forward cost ratio;
  * the velocity difference between the FP32 and FP64 runs (same steps);
  * the CPU oracle (numpy, float64) on a bounded slab of the same workload.
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
MEASURED_TRAFFIC = {"sources_sha256_16": "f15b3f57086f4019", "bytes": 2609470182}
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
    """Bytes one forward step must move: each fluid node reads and writes Q
    values, every node's 4-byte node word is read, and each cut link reads
    its direction byte, four double coefficients and one link slot and
    writes one link slot."""
    return 2 * Q * s * n_fluid + 4 * n_nodes + n_links * (1 + 32 + 2 * s)


def time_forward(binding, geom, w, precision, steps, warmup):
    import torch
    sv = binding.solver_for(geom, w.s, precision=precision, dp=w.dp, l_rule=w.l_rule)
    sv.init()
    sv.step(warmup)
    torch.cuda.synchronize()
    sv.set_timing(True)
    t0 = time.perf_counter()
    sv.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = sv.last_step_ms()
    sv.set_timing(False)
    return sv, (t1 - t0) * 1e3 / steps, kernel_ms


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


def cpu_baseline(geom, w, slab=48, steps=20):
    """Oracle on the z-slab 0 <= z < slab of the same workload (window mode:
    reads across the slab faces see NaN and are not used)."""
    from oracle.lbm import Oracle
    try:
        import threadpoolctl
        threads = max(i["num_threads"] for i in threadpoolctl.threadpool_info())
    except Exception:
        threads = 1
    nx, ny, nz = geom.shape
    nodes = np.arange(nx * ny * min(slab, nz), dtype=np.int64)
    o = Oracle(geom, w.s, dp=w.dp, l_rule=w.l_rule, nodes=nodes)
    f = o.init_equilibrium()
    t0 = time.perf_counter()
    o.run(f, steps)
    dt = time.perf_counter() - t0
    return {"value": round(len(nodes) * steps / dt / 1e6, 4), "unit": "MLUPS",
            "cores": int(threads), "kind": "oracle",
            "sample": "%d steps on the %dx%dx%d z-slab (%d nodes) of the same "
                      "geometry, numpy float64 (BLAS threads %d), %.1f s"
                      % (steps, nx, ny, min(slab, nz), len(nodes), threads, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--adjoint-steps", type=int, default=64)
    ap.add_argument("--every", type=int, default=8)
    ap.add_argument("--n", type=int, default=256, help="lattice edge (256 = the benchmark)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["fwd32", "fwd64", "adjoint32", "copy"],
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

    if args.only == "copy":
        # reference copies of known size: HBM ceiling and counter scaling
        print(json.dumps(copy_ceiling(binding, torch, reps=args.steps, all_modes=True)))
        return

    w = configs.c3_spheres(args.n)
    geom = w.geometry()
    N, NF, NL = geom.n_nodes, geom.n_fluid, geom.n_links
    if args.only in ("fwd32", "fwd64"):
        prec = args.only.replace("fwd", "fp")
        sv, ms, kms = time_forward(binding, geom, w, prec, args.steps, args.warmup)
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

    # FP32 forward (headline)
    sv32, ms32, kms32 = time_forward(binding, geom, w, "fp32", args.steps, args.warmup)
    # FP64 forward
    sv64, ms64, kms64 = time_forward(binding, geom, w, "fp64", args.steps, args.warmup)
    # same number of steps on both: velocity difference FP32 vs FP64
    _, u32 = sv32.moments()
    _, u64 = sv64.moments()
    fl = geom.solid == 0
    du = float(np.sqrt(((u32 - u64)[fl] ** 2).sum() / (u64[fl] ** 2).sum()))
    sv64.close()

    # FP32 forward + adjoint (checkpointed run, then the reverse sweep)
    A = args.adjoint_steps
    sv32.set_rate_gradient(False)      # the benchmark objective needs dJ/dg and dJ/dq
    sv32.set_objective("mean_ux", 0, sv32.time, sv32.time + A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv32.run_checkpointed(A, args.every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sv32.adjoint()
    g = sv32.grad()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    J = sv32.objective()
    ms_fwd_ckpt = (t1 - t0) * 1e3 / A
    ms_adj = (t2 - t1) * 1e3 / A
    sv32.close()

    ceiling = copy_ceiling(binding, torch)
    bytes32 = algorithmic_bytes(19, 4, N, NF, NL)
    bytes64 = algorithmic_bytes(19, 8, N, NF, NL)
    achieved = bytes32 / (kms32 * 1e-3) / 1e9
    mlups32 = N / (ms32 * 1e-3) / 1e6
    mlups64 = N / (ms64 * 1e-3) / 1e6
    out = {
        "metric": "MLUPS & % HBM roofline, D3Q19 MRT 256^3 fwd+adjoint, FP32 vs FP64",
        "value": round(mlups32, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
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
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (MEASURED_TRAFFIC["bytes"]
                        if kernel_sources_hash() == MEASURED_TRAFFIC["sources_sha256_16"]
                        else None),
            "kernel": "k_step<D3Q19,float,pressure>",
            "copy_ceiling_GBps": ceiling["best_GBps"],
            "frac_of_copy_ceiling": round(achieved / ceiling["best_GBps"], 4),
            "kernel_ms": round(kms32, 4),
            "algorithmic_bytes": int(bytes32),
        },
        "fp64": {
            "mlups": round(mlups64, 1), "ms_per_step": round(ms64, 4),
            "kernel_ms": round(kms64, 4),
            "hbm_frac": round(bytes64 / (kms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "fp32_over_fp64_speedup": round(ms64 / ms32, 3),
            "u_rel_l2_fp32_vs_fp64": du,
        },
        "adjoint": {
            "steps": A, "checkpoint_every": args.every,
            "objective": "mean u_x over the window", "J": J,
            "dJ_dg": [float(v) for v in g["g"]],
            "ms_per_step_checkpointed_forward": round(ms_fwd_ckpt, 4),
            "ms_per_step_reverse": round(ms_adj, 4),
            "fwd_adjoint_mlups": round(N / ((ms_fwd_ckpt + ms_adj) * 1e-3) / 1e6, 1),
            "adjoint_over_forward_cost": round((ms_fwd_ckpt + ms_adj) / ms32, 3),
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(geom, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
