"""Writes the oracle's whole-run results that the GPU whole-run tests compare
against (the oracle is slow at these sizes, so its results are stored).

Calls only the oracle (oracle/) and the seeded input generators
(rcp_inputs/).  Each run: random sequential addition with the run's seed,
then the default rung table for the packing's size ratio to the stop
criterion, then shrink to contact (App. A).

    python tests/golden/make_oracle_phi.py c2        # -> c2_phi_oracle.json
    python tests/golden/make_oracle_phi.py census8   # -> census8_phi_oracle.json
    python tests/golden/make_oracle_phi.py cascade   # -> cascade_phi_oracle.json

The cascade case runs the oracle's sequential multimodal cascade (Sec. 4,
oracle.cascade): 20 coarse spheres, diameter ratio 7, two classes.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle            # noqa: E402
import rcp_inputs as ri  # noqa: E402


def one_run(w, seed, skin=0.5):
    x = oracle.rsa(w.d0, w.L, 1.0, seed)
    st = oracle.RunState(x, w.d0, w.L, 1.0)
    S = float(w.d0.max() / w.d0.min())
    t0 = time.time()
    status, res, _ = oracle.run(st, oracle.default_params(w.d0, s=skin),
                                oracle.default_schedule(w.n, S=S))
    return {"seed": int(seed), "n": int(w.n), "phi": res.phi, "status": int(status),
            "iterations": int(res.iterations), "max_overlap": res.max_overlap,
            "seconds": time.time() - t0}


def c2():
    runs = []
    for seed in range(8):
        w = ri.c2_powerlaw(seed=seed)
        runs.append(one_run(w, w.seed))
        print(runs[-1], flush=True)
    return {"workload": "powerlaw p=-3 S=20 N=1e5, RSA at phi0=0.05, seeds 0-7, default schedule",
            "runs": runs}


def census8():
    wl = sorted(ri.census_draw(64), key=lambda w: w.n)[:8]
    runs = []
    for w in wl:
        for seed in range(8):
            r = one_run(w, 1000 + seed)
            r["name"] = w.name
            runs.append(r)
            print(r, flush=True)
    return {"workload": "the 8 smallest packings of the 64-packing census draw (seed 2026), "
                        "placement seeds 1000-1007 each, default schedule",
            "runs": runs}


def cascade():
    n1, rho, classes = 20, 7.0, 2
    runs = []
    for seed in range(8):
        t0 = time.time()
        phis, counts = oracle.cascade(n1, rho, classes, seed=seed)
        runs.append({"seed": seed, "phi": phis, "counts": counts, "seconds": time.time() - t0})
        print(runs[-1], flush=True)
    return {"workload": "sequential multimodal cascade, 20 coarse spheres, diameter ratio 7, "
                        "two classes (counts of the ideal cascade), seeds 0-7",
            "n1": n1, "rho": rho, "classes": classes, "runs": runs}


if __name__ == "__main__":
    which = sys.argv[1]
    out = {"c2": c2, "census8": census8, "cascade": cascade}[which]()
    out["threads"] = oracle.num_threads()
    path = os.path.join(HERE, "%s_phi_oracle.json" % which)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)
