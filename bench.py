#!/usr/bin/env python3
"""Benchmark of the LNV energy + gradient step on one MI355X.

One step = the whole hot path on resident inputs: the three forward truncated
products (X = LS, M = LSL, P = LSLSL on H's range), K assembly, E = 2 Tr(KH)
and the five adjoint products giving dE/dL, all in the library's kernels.
Default workload: diamond Si 16x16x16 cells (32,768 atoms), S/H/L ranges
8/12/16 bohr, 4 functions per atom, seeded synthetic S, H, L.

Prints one JSON line (rank 0, N = 1).  The value is useful GFLOP/s of the
primary precision (useful = 2 nfn_i nfn_k nfn_j per block triple of the
truncated products).  Extra modes are reported with their energy error per
atom against the FP64 result.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # MI355X dense matrix peaks
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(lnv, sysm, rS, dev):
    import torch
    import workloads
    out = {}
    for w in "LSH":
        i, j, img = lnv.patterns[w].keys()
        out[w] = torch.from_numpy(workloads.block_values(sysm, w, i, j, img, seed=0, rS=rS)).to(dev)
    return out


def time_mode(lnv, inp, prec, steps, warmup):
    import torch
    E = torch.empty(1, dtype=torch.float64, device="cuda:0")
    G = torch.empty(lnv.patterns["L"].n_values, dtype=torch.float64, device="cuda:0")
    for _ in range(warmup):
        lnv.energy_grad(inp["L"], inp["S"], inp["H"], prec=prec, E=E, G=G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lnv.energy_grad(inp["L"], inp["S"], inp["H"], prec=prec, E=E, G=G)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, E.item(), G


def profile_mode(lnv, inp, prec, steps):
    """Per-product kernel times from HIP events recorded around each launch."""
    import torch
    E = torch.empty(1, dtype=torch.float64, device="cuda:0")
    G = torch.empty(lnv.patterns["L"].n_values, dtype=torch.float64, device="cuda:0")
    lnv.profile(True)
    for _ in range(steps):
        lnv.energy_grad(inp["L"], inp["S"], inp["H"], prec=prec, E=E, G=G)
    rec = lnv.profile_read()
    lnv.profile(False)
    return rec


def cpu_baseline(cfg, flops_per_atom):
    """The oracle (FP64 C++/OpenMP, untuned) on a bounded sample of the same
    workload: the 2x2x2-cell periodic crystal with the same ranges, whose
    per-atom work equals the large cell's (translation invariance)."""
    import oracle
    import workloads
    s = workloads.diamond(2)
    rS, rH, rL = cfg["rS"], cfg["rH"], cfg["rL"]
    inp = oracle.make_inputs(s, rS, rH, rL)
    t0 = time.perf_counter()
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(flops_per_atom * s.n / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle E + dE/dL of the 64-atom 2x2x2 periodic cell at the same ranges "
                      f"({dt:.2f} s; same per-atom work as the full cell), equivalent useful GFLOP/s",
            "seconds": round(dt, 3), "energy_per_atom": r["E"] / s.n}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32"])
    ap.add_argument("--modes", default="fp64,fp32", help="modes to time; fp64 is the error reference")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X and has no multi-GPU mode "
              "(sharding by spatial row ownership is a design note only).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_0911_3584_amd as lsdm
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    cfg = workloads.config(args.config)
    sysm = cfg["system"]
    t0 = time.perf_counter()
    gs = lsdm.System.from_workload(sysm)
    lnv = lsdm.LNV(gs, cfg["rS"], cfg["rH"], cfg["rL"])
    t_sym = time.perf_counter() - t0
    n_triples, flops = lnv.info(True)
    log(f"[bench] config {args.config} {cfg['name']}: {sysm.n} atoms, symbolic {t_sym:.1f} s, "
        f"{n_triples / sysm.n:.0f} triples/atom, {flops:.3e} flop/step")
    t0 = time.perf_counter()
    inp = make_inputs(lnv, sysm, cfg["rS"], "cuda:0")
    log(f"[bench] inputs {time.perf_counter() - t0:.1f} s")

    modes = [m for m in args.modes.split(",") if m]
    if args.prec not in modes:
        modes.append(args.prec)
    res = {}
    for m in modes:
        ms, E, G = time_mode(lnv, inp, m, args.steps, args.warmup)
        res[m] = {"ms_per_step": ms, "E": E, "gflops": flops / (ms * 1e-3) / 1e9}
        log(f"[bench] {m}: {ms:.3f} ms/step  {res[m]['gflops']:.1f} GFLOP/s  E = {E:.12f}")
    if "fp64" in res:
        for m in res:
            res[m]["err_uHa_per_atom"] = 1e6 * abs(res[m]["E"] - res["fp64"]["E"]) / sysm.n

    prim = res[args.prec]
    rec = profile_mode(lnv, inp, args.prec, args.profile_steps)
    tot_ms = sum(v[0] for v in rec.values())
    tot_fl = sum(v[1] * v[2] for v in rec.values())
    launches = sum(v[1] for v in rec.values())
    achieved = tot_fl / (tot_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.prec]
    per_product = {k: {"avg_ms": round(v[0] / max(v[1], 1), 4), "tflops": round(v[1] * v[2] / max(v[0], 1e-12) / 1e9, 2)}
                   for k, v in rec.items()}
    log(f"[bench] product kernels: {launches} launches, {tot_ms / args.profile_steps:.3f} ms/step, "
        f"{achieved:.2f} TFLOP/s useful; {per_product}")

    out = {
        "metric": "LNV energy+gradient step: useful block-sparse GFLOP/s (s/step in ms_per_step)",
        "value": round(prim["gflops"], 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(prim["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic (seeded diamond-Si geometry and S/H/L value laws)",
        "config": {"workload": cfg["name"], "atoms": sysm.n, "ranges_bohr": [cfg["rS"], cfg["rH"], cfg["rL"]],
                   "fns_per_atom": "4" if args.config != 5 else "13/5", "flop_per_step": flops,
                   "triples_per_step": n_triples, "symbolic_s": round(t_sym, 2), "parallelism": "single GPU"},
        "modes": {m: {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()} for m, r in res.items()},
        "roofline": {"kernel": f"k_prod_{args.prec} (all 8 product launches of a step)", "bound": "mfma",
                     "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": None, "per_product": per_product},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, flops / sysm.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
