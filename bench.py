#!/usr/bin/env python3
"""Benchmark of the LNV energy + gradient step on one MI355X.

One step = the whole hot path on resident inputs: the three forward truncated
products (X = LS, M = LSL, P = LSLSL on H's range), K assembly, E = 2 Tr(KH)
and the five adjoint products giving dE/dL, all in the library's kernels.
Default workload: diamond Si 16x16x16 cells (32,768 atoms), S/H/L ranges
8/12/16 bohr, 4 functions per atom, seeded synthetic S, H, L.

By default the chain runs in symmetric mode (L, S and H are symmetric, so
M, P and dE/dL are computed on one half and mirrored); --full times the chain
without that, and the JSON line also carries the FP32 step time of the full
chain for comparison.

Prints one JSON line (rank 0, N = 1).  The value is useful GFLOP/s of the
primary precision (useful = 2 nfn_i nfn_k nfn_j per block triple that the
step's products compute).  Extra modes are reported with their energy error
per atom against the FP64 result.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp32_rc": 157.3}   # MI355X dense matrix peaks
HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "si32768_rl16"    # diamond Si 16x16x16 cells, ranges 8/12/16 bohr


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


def algorithmic_bytes(lnv, symmetric, op_bytes, out_bytes):
    """Compulsory bytes of one step's products: every operand read once
    (op_bytes per value) and every output written once (out_bytes per value;
    read too where the product accumulates), on the block layout's values; a
    half-output product writes half of its output.  In symmetric mode the
    6 HX term is a projection of Y = HX, not a product, and is not counted."""
    n = {w: lnv.patterns[w].n_values for w in "SHLXM"}
    #        A    B    C    output share  accumulates
    prods = [("L", "S", "X", 1.0, False), ("X", "L", "M", 0.5 if symmetric else 1.0, False),
             ("X", "M", "H", 0.5 if symmetric else 1.0, False), ("X", "H", "M", 1.0, False),
             ("H", "M", "X", 1.0, False)]
    if symmetric:
        prods += [("X", "M", "L", 0.5, False), ("X", "S", "L", 1.0, True)]
    else:
        prods += [("M", "L", "X", 1.0, True), ("X", "M", "L", 1.0, False), ("X", "S", "L", 1.0, True)]
    tot = 0.0
    for a, b, c, share, acc in prods:
        tot += (n[a] + n[b]) * op_bytes + n[c] * share * out_bytes * (2 if acc else 1)
    return tot


def cpu_baseline(cfg, flops_per_atom):
    """The oracle (FP64 C++/OpenMP, untuned) on a bounded sample of the same
    workload: the 12x12x12-cell (13824-atom) periodic crystal with the same
    ranges, whose per-atom work equals the 32768-atom cell's (translation
    invariance); about 10-30 s of host time."""
    import oracle
    import workloads
    s = workloads.diamond(12)
    rS, rH, rL = cfg["rS"], cfg["rH"], cfg["rL"]
    inp = oracle.make_inputs(s, rS, rH, rL)
    t0 = time.perf_counter()
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(flops_per_atom * s.n / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle E + dE/dL of the 13824-atom 12x12x12 periodic cell at the same ranges "
                      f"({dt:.2f} s; same per-atom work as the full cell), equivalent useful GFLOP/s",
            "seconds": round(dt, 3), "energy_per_atom": r["E"] / s.n, "cpu_model": model}


# sources that decide what the product kernels read and write: the kernels,
# the symbolic pass (atom order, tiles, steps) and the chain's choice of plans
KERNEL_SRC = [os.path.join(ROOT, "paper_0911_3584_amd", "csrc", f)
              for f in ("kernels.hip", "symbolic.cpp", "plan_common.h", "lsdm_internal.h", "api.cpp")]
PRODUCT_KERNEL = {"fp64": "k_gprod<double>", "fp32": "k_gprod<float>", "bf16": "k_gprod_bf16",
                  "fp32_rc": "k_gprod<float> (R_A R_B; FP64 corrections in k_rc_apply not counted)"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_si32768.json")


def workloads_default_name():
    import workloads
    return DEFAULT_WORKLOAD


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_per_step(prec, workload):
    """HBM bytes (fetch + write) of one step's product launches, from the
    committed counter summary when it was taken on the current kernel source,
    the same precision and the 32768-atom workload; None otherwise."""
    if workload != workloads_default_name():
        return None
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("prec") != prec or not t.get("dispatches"):
        return None
    per_step = t.get("steps", 1)
    return round(sum(d["fetch_bytes"] + d["write_bytes"] for d in t["dispatches"]) / per_step, 0)


def summarize_pmc(fetch_dir, write_dir, prec, out, steps=1):
    """Per-dispatch HBM bytes of the product kernels from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE in KiB), scaled by what the same counters read
    for the calibration copy (a torch copy of known size in the same run)."""
    import csv
    import glob

    def rows(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit(f"no counter_collection.csv under {d}")
        return list(csv.DictReader(open(f[0])))

    res = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = {}
        for r in rows(d):
            if r.get("Counter_Name") != name:
                continue
            per.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
        res[name] = per
    # the calibration copy: the copy dispatch that writes the most (its write
    # count is the copy size; the fetch counter may read a fraction of it)
    copies = [(v, did) for did, (kn, v) in res["WRITE_SIZE"].items() if "copy" in kn.lower()]
    if not copies or max(copies)[0] < 512 * 1024:
        raise SystemExit("calibration copy dispatch not found (run bench.py with --calib-copy-mib 1024)")
    calib = max(copies)[1]
    exp_kib = 1024 * 1024
    f_fac = exp_kib / res["FETCH_SIZE"][calib][1]
    w_fac = exp_kib / res["WRITE_SIZE"][calib][1]
    prods = {}
    for did, (kn, v) in res["FETCH_SIZE"].items():
        if "prod" not in kn:
            continue
        w = res["WRITE_SIZE"].get(did, [kn, 0.0])[1]
        prods[did] = (kn, v * f_fac * 1024, w * w_fac * 1024)
    summ = {"kernel_hash": kernel_hash(), "prec": prec, "steps": steps, "fetch_scale": f_fac, "write_scale": w_fac,
            "dispatches": [{"id": d, "kernel": k.split("(")[0], "fetch_bytes": f, "write_bytes": w}
                           for d, (k, f, w) in sorted(prods.items())]}
    with open(out, "w") as fh:
        json.dump(summ, fh, indent=1)
    print(f"wrote {out}: {len(prods)} product dispatches, fetch scale {f_fac:.3f}, write scale {w_fac:.3f}")


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-pmc":
        # --summarize-pmc FETCH_DIR WRITE_DIR PREC [OUT [STEPS]]: the counter runs
        # of STEPS chain steps (default 1)
        summarize_pmc(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5] if len(sys.argv) > 5 else TRAFFIC_FILE,
                      int(sys.argv[6]) if len(sys.argv) > 6 else 1)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, help="workload name (workloads.WORKLOADS)")
    ap.add_argument("--prec", default="fp32", choices=["fp64", "fp32", "bf16", "fp32_rc"])
    ap.add_argument("--modes", default="fp64,fp32,bf16",
                    help="modes to time (fp64, fp32, bf16, fp32_rc); fp64 is the error reference.  FP32_RC is not "
                         "timed by default: native FP64 MFMA is the route to FP64-level results on this GPU")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--full", action="store_true", help="no symmetric mode (every product computes all its strips)")
    ap.add_argument("--no-full-compare", action="store_true", help="skip the FP32 timing of the full chain")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (reference dispatch for HBM counters)")
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

    cfg = workloads.workload(args.workload)
    sysm = cfg["system"]
    t0 = time.perf_counter()
    gs = lsdm.System.from_workload(sysm)
    symmetric = not args.full
    lnv = lsdm.LNV(gs, cfg["rS"], cfg["rH"], cfg["rL"], symmetric=symmetric)
    t_sym = time.perf_counter() - t0
    n_triples, flops = lnv.info(True)
    log(f"[bench] {cfg['name']}: {sysm.n} atoms, symbolic {t_sym:.1f} s, "
        f"{n_triples / sysm.n:.0f} triples/atom, {flops:.3e} flop/step")
    t0 = time.perf_counter()
    inp = make_inputs(lnv, sysm, cfg["rS"], "cuda:0")
    log(f"[bench] inputs {time.perf_counter() - t0:.1f} s")

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del a, b

    modes = [m for m in args.modes.split(",") if m]
    if args.prec not in modes:
        modes.append(args.prec)
    res = {}
    for m in modes:
        ms, E, G = time_mode(lnv, inp, m, args.steps, args.warmup)
        # useful flops of the products this mode launches (symmetric FP64
        # forms E without P, so it runs one product fewer)
        fl_m = sum(v[1] * v[2] for v in profile_mode(lnv, inp, m, 1).values()) if args.profile_steps > 0 else flops
        res[m] = {"ms_per_step": ms, "E": E, "gflops": fl_m / (ms * 1e-3) / 1e9, "flop_per_step": fl_m}
        log(f"[bench] {m}: {ms:.3f} ms/step  {res[m]['gflops']:.1f} GFLOP/s  E = {E:.12f}")
    if "fp64" in res:
        for m in res:
            res[m]["err_uHa_per_atom"] = 1e6 * abs(res[m]["E"] - res["fp64"]["E"]) / sysm.n

    full_cmp = None
    if symmetric and not args.no_full_compare and args.profile_steps > 0:
        full = lsdm.LNV(gs, cfg["rS"], cfg["rH"], cfg["rL"])
        ms_full, E_full, _ = time_mode(full, inp, "fp32", args.steps, args.warmup)
        full_cmp = {"ms_per_step": round(ms_full, 4), "flop_per_step": full.info(True)[1],
                    "E": E_full}
        log(f"[bench] full chain fp32: {ms_full:.3f} ms/step")
        del full
        torch.cuda.empty_cache()

    prim = res[args.prec]
    if args.profile_steps <= 0:
        log("[bench] no profile steps: roofline not computed")
        return
    rec = profile_mode(lnv, inp, args.prec, args.profile_steps)
    tot_ms = sum(v[0] for v in rec.values())
    tot_fl = sum(v[1] * v[2] for v in rec.values())
    launches = sum(v[1] for v in rec.values())
    per_product = {k: {"avg_ms": round(v[0] / max(v[1], 1), 4), "tflops": round(v[1] * v[2] / max(v[0], 1e-12) / 1e9, 2)}
                   for k, v in rec.items() if v[1] > 0}
    log(f"[bench] product kernels: {launches} launches, {tot_ms / args.profile_steps:.3f} ms/step, "
        f"{tot_fl / (tot_ms * 1e-3) / 1e12:.2f} TFLOP/s useful; {per_product}")
    step_s = prim["ms_per_step"] * 1e-3
    if args.prec == "bf16":
        # bf16 operands against an FP32 MFMA-accumulated output: far below the
        # MFMA ridge, so the bound is HBM on the products' algorithmic bytes
        alg = algorithmic_bytes(lnv, symmetric, 2, 4) * args.profile_steps
        achieved = alg / (tot_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "frac_step": round(alg / args.profile_steps / step_s / 1e9 / HBM_PEAK_GBS, 4),
                "algorithmic_bytes_per_step": alg / args.profile_steps}
    else:
        peak = PEAK_TFLOPS[args.prec]
        achieved = tot_fl / (tot_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "frac_step": round(prim["flop_per_step"] / step_s / 1e12 / peak, 4)}

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
        "data": f"synthetic (seeded {sysm.name} geometry and S/H/L value laws)",
        "config": {"workload": cfg["name"], "atoms": sysm.n, "ranges_bohr": [cfg["rS"], cfg["rH"], cfg["rL"]],
                   "fns_per_atom": "/".join(str(int(k)) for k in sorted(set(sysm.nfn.tolist()), reverse=True)), "flop_per_step": flops,
                   "triples_per_step": n_triples, "symbolic_s": round(t_sym, 2), "symmetric": symmetric,
                   "parallelism": "single GPU"},
        "modes": {m: {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()} for m, r in res.items()},
        "roofline": dict({"kernel": f"{PRODUCT_KERNEL[args.prec]} (all product launches of a step, HIP-event "
                                    f"time; frac_step: the same work over the whole step; traffic in HBM bytes "
                                    f"per step)"}, **roof,
                         traffic=traffic_per_step(args.prec, cfg["name"]), per_product=per_product),
    }
    if full_cmp is not None:
        out["full_chain_fp32"] = full_cmp
    if not args.no_cpu_baseline and args.workload == DEFAULT_WORKLOAD:
        out["cpu_baseline"] = cpu_baseline(cfg, flops / sysm.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
