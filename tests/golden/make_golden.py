"""Writes the stored oracle results in this folder (regression fixtures).

Uses only the oracle and the seeded input generator: E = 2 Tr(KH) with K of
eq. 3 (section 2), dE/dL, and N_e = 2 Tr(KS), for two small workloads.  Rerun
it only when a change to the oracle's arithmetic is justified by the paper;
the commit that does so names the passage.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle      # noqa: E402
import workloads   # noqa: E402


def cases():
    w = workloads.workload("si64_rl12")
    yield "si64_rl12", w["system"], w["rS"], w["rH"], w["rL"]
    yield "mixed_cluster_40", workloads.random_cluster(40, 12.0, nfn=np.arange(40) % 5 + 1, seed=21), 4.0, 5.0, 5.5


def record(name, s, rS, rH, rL):
    inp = oracle.make_inputs(s, rS, rH, rL)
    r = oracle.lnv_energy(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    G = oracle.lnv_gradient(inp["L"], inp["S"], inp["H"], rS, rH, rL)
    N = oracle.electron_number(inp["L"], inp["S"], rS, rH, rL)
    pick = np.linspace(0, G.val.size - 1, 12).astype(int)
    kpick = np.linspace(0, r["K"].val.size - 1, 12).astype(int)
    return {"workload": name, "atoms": int(s.n), "ranges_bohr": [rS, rH, rL],
            "source": "Bowler & Miyazaki, section 2, eq. 3 and N_e = 2 Tr(KS); seeded synthetic S, H, L",
            "E": r["E"], "N_e": N, "grad_norm": float(np.linalg.norm(G.val)),
            "grad_samples": {str(int(i)): float(G.val[i]) for i in pick},
            "K_samples": {str(int(i)): float(r["K"].val[i]) for i in kpick}}


if __name__ == "__main__":
    for c in cases():
        out = record(*c)
        with open(os.path.join(HERE, f"oracle_{c[0]}.json"), "w") as fh:
            json.dump(out, fh, indent=1)
        print("wrote", c[0], out["E"])
