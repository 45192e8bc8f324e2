"""Write the FP64 oracle's drainage results that the GPU drainage tests
compare against (tests/golden/drain_oracle.json).

Calls only the oracle and the seeded input generators: every stored value is
the oracle's.  The drains follow the pressure-controlled ramp of Sec. 2.2.2
(each imposed capillary pressure held until the wetting saturation changes by
less than tol over check_every steps, then bisection of the first invaded
interval down to bisect_rel); the inputs are rebuilt from the same seeds by
the tests.  Run from the repository root:

    python tests/golden/make_drain_golden.py [--only NAME]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from tests.golden import drain_cases  # noqa: E402

OUT = os.path.join(HERE, "drain_oracle.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None, help="comma-separated case names")
    args = ap.parse_args()
    only = set(args.only.split(",")) if args.only else None
    old = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            old = json.load(f)
    res = dict(old.get("cases", {}))
    for name in drain_cases.NAMES:
        if only and name not in only:
            continue
        prob, pcs = drain_cases.case(name)
        t0 = time.time()
        d = oracle.Oracle(prob).drain(pcs, **drain_cases.CONV)
        dt = time.time() - t0
        res[name] = dict(pc=[float(v) for v in pcs], S=[float(v) for v in d["S"]],
                         steps=[int(v) for v in d["steps"]],
                         status=[int(v) for v in d["status"]],
                         invaded_at=int(d["invaded_at"]),
                         pce_lo=float(d["pce_lo"]), pce=float(d["pce"]),
                         pce_hi=float(d["pce_hi"]), oracle_seconds=round(dt, 1))
        print(name, res[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(dict(conv=drain_cases.CONV, cases=res), f, indent=1)


if __name__ == "__main__":
    main()
