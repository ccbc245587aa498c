"""Write oracle_bura_coefficients.json: the oracle's (k,k) BURA of t^(1-alpha).

Calls only ``oracle.remez`` (Algorithm 3.1 in multiprecision).  The stored
strings carry 30 significant digits; tests and the benchmark's CPU-baseline
leg read them instead of re-running the multiprecision Remez.

Usage:  python tests/golden/make_oracle_coefficients.py [--serving] [-j N]
"""

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "oracle_bura_coefficients.json")

# (alpha, k) pairs used by the parity tests and the benchmark workloads
CORE = [(0.5, 5), (0.25, 5), (0.75, 5), (0.5, 7), (0.25, 7), (0.75, 7), (0.25, 8), (0.5, 8),
        (0.25, 9), (0.5, 9), (0.75, 9), (0.6, 7)]
SERVING = [(a / 10, k) for a in range(1, 10) for k in range(5, 13)]


def one(pair):
    import mpmath as mp
    from oracle.remez import RemezError, remez
    alpha, k = pair
    t0 = time.time()
    try:
        b = remez(alpha, k)
    except RemezError as exc:
        return pair, {"error": str(exc)}
    with mp.workdps(b.dps):
        return pair, {
            "E": mp.nstr(b.E, 30),
            "c": [mp.nstr(x, 30) for x in b.c],
            "d": [mp.nstr(x, 30) for x in b.d],
            "eta": [mp.nstr(x, 20) for x in b.eta],
            "dps": b.dps,
            "iterations": b.iterations,
            "seconds": round(time.time() - t0, 2),
        }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--serving", action="store_true")
    ap.add_argument("-j", type=int, default=4)
    args = ap.parse_args()
    pairs = list(CORE)
    if args.serving:
        pairs += [p for p in SERVING if p not in pairs]
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    todo = [p for p in pairs if f"{p[0]:.2f},{p[1]}" not in data]
    with ProcessPoolExecutor(args.j) as ex:
        for (alpha, k), rec in ex.map(one, todo):
            data[f"{alpha:.2f},{k}"] = rec
            print(alpha, k, rec.get("E", rec.get("error")), flush=True)
            doc = {"_source": "written by tests/golden/make_oracle_coefficients.py from oracle.remez "
                              "(Algorithm 3.1, Section 3.2; partial fractions eq. (15))"}
            doc.update(dict(sorted((k_, v) for k_, v in data.items() if not k_.startswith("_"))))
            with open(OUT + ".tmp", "w") as fh:
                json.dump(doc, fh, indent=1)
            os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
