"""Discount choice per configuration and variant (reading C12 of the design notes).

The paper tests ten evenly spaced discounts in [0, 1] for Momentum-BP and
EWAInit-BP and keeps the one that decodes best (section IV-A, applied again in
section IV-B, with one value for every code length).  This script does that on
the FP64 oracle only and writes ``alpha_choice.json`` beside it:

* grid alpha in {0.1, 0.2, ..., 1.0};
* score = logical failures summed over the configuration's codes and error
  rates (detected + undetected, section IV); smallest score wins, ties go to
  the larger alpha;
* shots are drawn by the oracle's sampler on stream 1 of each configuration's
  key, so they are independent of the stream-0 shots that the tests and the
  benchmark decode;
* planar d=3 (configuration 1) is scored by its exact logical error rate
  (every syndrome decoded, every coset summed; ``make_d3_exact.exact_ler``)
  instead of samples.

Sizes: configuration 2 (toric L=8, p = 0.02..0.16, iter_max 100) and 3 (the
eleven mixed-batch codes at p = 0.08, iter_max 100) use 10^4 shots per code and
error rate; configuration 5 (planar d=31 and toric L=32 at p = 0.10, iter_max
200) uses 2^10 shots per code, because the oracle spends about 40 ms of one
host core per shot there (140-200 iterations of 7,320-8,192 edges).

Run: python -m tests.golden.choose_alpha [--threads N]
"""
import argparse
import json
import os
import time

import numpy as np

import qecgen
from oracle import oracle as O

GRID = [round(0.1 * k, 1) for k in range(1, 11)]
CONFIG2_P = [0.02, 0.04, 0.06, 0.08, 0.10, 0.12, 0.14, 0.16]
CONFIG3 = [("planar", 5), ("planar", 7), ("planar", 9), ("planar", 11), ("planar", 13),
           ("toric", 6), ("toric", 10), ("toric", 14), ("xzzx", 5), ("xzzx", 9), ("xzzx", 13)]
CONFIG5 = [("planar", 31), ("toric", 32)]
STREAM = 1


def failures(code, variant, alpha, p, shots, seed, max_iter, nthreads):
    thr = qecgen.thresholds(p / 3, p / 3, p / 3)
    err, syn = O.sample(code.hx, code.hz, shots, thr, seed=seed, stream=STREAM, nthreads=nthreads)
    pi = O.prior_llr(qecgen.depolarizing_probs(code.n, p))
    r = O.decode(code.hx, code.hz, O.Params(variant=variant, alpha=alpha, max_iter=max_iter), pi, syn,
                 nthreads=nthreads)
    _, counts = O.bookkeep(code.hx, code.hz, code.lx, code.lz, err, r["est"])
    return int(counts[1] + counts[2]), float(r["iters"].mean())


def pick(scores):
    """Smallest score; ties to the larger alpha."""
    best = min(scores.values())
    return max(a for a, s in scores.items() if s == best)


def choose(cases, variant, max_iter, shots, nthreads, label):
    """cases: list of (code, p, seed).  Returns the grid's scores and the choice."""
    scores, iters = {}, {}
    for a in GRID:
        t0 = time.time()
        tot, its = 0, []
        for code, p, seed in cases:
            f, it = failures(code, variant, a, p, shots, seed, max_iter, nthreads)
            tot += f
            its.append(it)
        scores[a] = tot
        iters[a] = float(np.mean(its))
        print(f"{label} {variant} alpha={a}: failures {tot} mean iters {iters[a]:.2f} ({time.time() - t0:.0f} s)",
              flush=True)
    return {"failures": {str(a): s for a, s in scores.items()}, "mean_iters": {str(a): v for a, v in iters.items()},
            "alpha": pick(scores), "shots_per_case": shots, "cases": len(cases)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", default="")
    args = ap.parse_args()
    O.build()
    path = os.path.join(os.path.dirname(__file__), "alpha_choice.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    out["_cite"] = ("discount grid of ten values in [0, 1], best one kept (section IV-A, IV-B); score = logical "
                    "failures of the FP64 oracle summed over each configuration's codes and error rates, ties to "
                    "the larger alpha; written by tests/golden/choose_alpha.py")
    out["grid"] = GRID
    todo = args.only.split(",") if args.only else ["config1", "config2", "config3", "config5"]

    if "config1" in todo:
        from tests.golden.make_d3_exact import exact_ler
        exact = {a: exact_ler("ewainit", a, 0.05, 50)[0] for a in GRID}
        rounded = {a: round(v, 12) for a, v in exact.items()}
        out["config1"] = {"ewainit": {"exact_ler": {str(a): v for a, v in exact.items()}, "alpha": pick(rounded),
                                      "note": "planar d=3, p=0.05, iter_max 50, exact over all 2^12 syndromes"}}
        print("config1", out["config1"], flush=True)

    if "config2" in todo:
        code = qecgen.toric(8)
        cases = [(code, p, qecgen.config_seed(2, 0, i)) for i, p in enumerate(CONFIG2_P)]
        out["config2"] = {v: choose(cases, v, 100, 10000, args.threads, "config2") for v in ("momentum", "ewainit")}
        out["config2"]["note"] = "toric L=8, p = 0.02..0.16 (8 points), iter_max 100, 10^4 shots per point"
        with open(path, "w") as f:
            json.dump(out, f, indent=1)

    if "config3" in todo:
        cases = [(qecgen.make(fam, L), 0.08, qecgen.config_seed(3, i, 0)) for i, (fam, L) in enumerate(CONFIG3)]
        out["config3"] = {"ewainit": choose(cases, "ewainit", 100, 10000, args.threads, "config3")}
        out["config3"]["note"] = "the eleven mixed-batch codes at p = 0.08, iter_max 100, 10^4 shots per code"
        with open(path, "w") as f:
            json.dump(out, f, indent=1)

    if "config5" in todo:
        cases = [(qecgen.make(fam, L), 0.10, qecgen.config_seed(5, i, 0)) for i, (fam, L) in enumerate(CONFIG5)]
        out["config5"] = {"ewainit": choose(cases, "ewainit", 200, 1024, args.threads, "config5")}
        out["config5"]["note"] = "planar d=31 and toric L=32 at p = 0.10, iter_max 200, 2^10 shots per code"

    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: (v if k in ("_cite", "grid") else {vv: (x["alpha"] if isinstance(x, dict) else x)
                                                             for vv, x in v.items()}) for k, v in out.items()},
                     indent=1))


if __name__ == "__main__":
    main()
