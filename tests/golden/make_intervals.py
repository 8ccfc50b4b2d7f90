"""Write tests/golden/intervals.json: the search interval of every named workload.

Calls only the oracle.  For workload ``w`` with parameters k0 and n_eig, the
interval is [mid-gap below eigenvalue k0, mid-gap above eigenvalue
k0 + n_eig - 1] (0-based, ascending), so that it holds exactly n_eig
eigenvalues and both ends sit half-way between neighbouring eigenvalues
(the filter is exactly 1/2 at the ends, so an eigenvalue there would be only
half captured).  Small pencils use the dense solver; large ones bisect on the
Sylvester inertia count.

Usage:  python tests/golden/make_intervals.py [name ...]
        python tests/golden/make_intervals.py --batch COUNT   (intervals_batch.json)
        python tests/golden/make_intervals.py --batch256 COUNT [PROCS]
                                                  (intervals_batch256.json)
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import feast_oracle as O  # noqa: E402
from paper_0901_2665_amd import workloads as W  # noqa: E402


def kth_eigenvalue(p, j, lo, hi, rtol=1e-13, count=O.inertia_count):
    """Bisection for eigenvalue j (0-based): count(lo) <= j < count(hi)."""
    while hi - lo > rtol * max(1.0, abs(lo), abs(hi)):
        mid = 0.5 * (lo + hi)
        if count(p, mid) <= j:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _hermitian_eig(args):
    name, j, lo, hi = args
    return kth_eigenvalue(W.make_pencil(name), j, lo, hi, rtol=1e-14,
                          count=O.inertia_count_hermitian)


def interval_for(name):
    w = W.WORKLOADS[name]
    p = W.make_pencil(name)
    k0, m = w["k0"], w["n_eig"]
    herm = w["kind"] == "hchain"
    count = O.inertia_count_hermitian if herm else O.inertia_count
    if p.n <= 2000:
        lam = (O.bruteforce_hermitian(p) if herm else O.bruteforce(p))[0]
        e = [lam[k0 - 1], lam[k0], lam[k0 + m - 1], lam[k0 + m]]
        method = "dense"
    else:
        lo, hi = -100.0, 100.0
        assert count(p, lo) == 0 and count(p, hi) == p.n
        e = [kth_eigenvalue(p, j, lo, hi, count=count) for j in (k0 - 1, k0, k0 + m - 1, k0 + m)]
        method = "inertia-bisection"
    emin = 0.5 * (e[0] + e[1])
    emax = 0.5 * (e[2] + e[3])
    cnt = count(p, emax) - count(p, emin)
    assert cnt == m, (name, cnt, m)
    out = dict(emin=emin, emax=emax, n_eig=m, k0=k0, method=method,
               gap_lo=e[1] - e[0], gap_hi=e[3] - e[2])
    if herm:  # the eigenvalues inside, by bisection on the inertia count
        import multiprocessing
        with multiprocessing.Pool(8) as pool:
            out["eigenvalues"] = pool.map(_hermitian_eig,
                                          [(name, j, emin, emax) for j in range(k0, k0 + m)])
    return out


def batch_interval(p):
    """Interval of batch problem p (workloads.batch_shape): round(0.6 M0)
    eigenvalues from index n // 4, ends half-way between neighbours."""
    sh = W.batch_shape(p)
    pen = W.batch_pencil(p)
    k0, m = sh["k0"], sh["n_eig"]
    lo, hi = -100.0, 100.0
    assert O.inertia_count(pen, lo) == 0 and O.inertia_count(pen, hi) == pen.n
    e = [kth_eigenvalue(pen, j, lo, hi) for j in (k0 - 1, k0, k0 + m - 1, k0 + m)]
    emin, emax = 0.5 * (e[0] + e[1]), 0.5 * (e[2] + e[3])
    cnt = O.inertia_count(pen, emax) - O.inertia_count(pen, emin)
    assert cnt == m, (p, cnt, m)
    return dict(emin=emin, emax=emax, n_eig=m, k0=k0, nc=sh["nc"], b=sh["b"], M0=sh["M0"],
                gap_lo=e[1] - e[0], gap_hi=e[3] - e[2])


def batch256_interval(p):
    """Interval of problem p of the full-shape batched workload
    (workloads.batch256_shape), as batch_interval."""
    sh = W.batch256_shape(p)
    pen = W.batch256_pencil(p)
    k0, m = sh["k0"], sh["n_eig"]
    lo, hi = -100.0, 100.0
    assert O.inertia_count(pen, lo) == 0 and O.inertia_count(pen, hi) == pen.n
    e = [kth_eigenvalue(pen, j, lo, hi) for j in (k0 - 1, k0, k0 + m - 1, k0 + m)]
    emin, emax = 0.5 * (e[0] + e[1]), 0.5 * (e[2] + e[3])
    cnt = O.inertia_count(pen, emax) - O.inertia_count(pen, emin)
    assert cnt == m, (p, cnt, m)
    return dict(emin=emin, emax=emax, n_eig=m, k0=k0, nc=sh["nc"], b=sh["b"], M0=sh["M0"],
                gap_lo=e[1] - e[0], gap_hi=e[3] - e[2])


def main_batch256(count, procs):
    import multiprocessing
    path = os.path.join(HERE, "intervals_batch256.json")
    with multiprocessing.Pool(procs) as pool:
        res = pool.map(batch256_interval, range(count), chunksize=1)
    data = {str(p): r for p, r in enumerate(res)}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print("wrote", path, len(data), flush=True)


def main_batch(count):
    path = os.path.join(HERE, "intervals_batch.json")
    data = {}
    for p in range(count):
        data[str(p)] = batch_interval(p)
        print(p, data[str(p)], flush=True)
        with open(path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


def main(names):
    path = os.path.join(HERE, "intervals.json")
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    for name in names or list(W.WORKLOADS):
        data[name] = interval_for(name)
        print(name, data[name], flush=True)
        with open(path, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    if sys.argv[1:2] == ["--batch"]:
        main_batch(int(sys.argv[2]))
    elif sys.argv[1:2] == ["--batch256"]:
        main_batch256(int(sys.argv[2]), int(sys.argv[3]) if len(sys.argv) > 3 else 8)
    else:
        main(sys.argv[1:])
