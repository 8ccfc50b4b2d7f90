"""Write tests/golden/feast_<workload>.json: the oracle's FEAST result.

Calls only the oracle (and the seeded input recipes).  Stored: the in-interval
eigenvalues, the count M, the loop count, the trace per loop, the largest
residual, and the run time of the oracle on this machine.

Usage:  python tests/golden/make_feast_golden.py tb6400 [tb128k ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import feast_oracle as O  # noqa: E402
from paper_0901_2665_amd import workloads as W  # noqa: E402


def main(names):
    for name in names:
        p, emin, emax, m0, ne, Y0 = W.make_workload(name)
        t0 = time.time()
        r = O.feast(p, emin, emax, m0, ne, Y0,
                    log=lambda k, M, T, tr: print(f"  loop {k} M {M} trace {T!r} rel {tr:.3e}",
                                                  flush=True))
        dt = time.time() - t0
        out = dict(workload=name, emin=emin, emax=emax, M0=m0, Ne=ne, M=int(r.M),
                   loops=int(r.loops), status=int(r.status),
                   lam=[float(v) for v in r.lam[:r.M]],
                   traces=[float(t) for t in r.traces], counts=[int(c) for c in r.counts],
                   max_res=float(r.max_res), trace_rel=float(r.trace_rel),
                   oracle_seconds=dt)
        with open(os.path.join(HERE, f"feast_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "M", r.M, "loops", r.loops, "max_res", r.max_res, "s", dt, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
