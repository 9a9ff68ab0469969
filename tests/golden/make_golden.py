"""Write stored oracle values for the GPU parity tests.

Calls only ``oracle/`` (exact arithmetic) and ``inputs/`` (seeded generators).
Each output line is

    name n sha256(input bytes) log2_den re_num im_num

meaning Per = (re_num + i im_num) / 2^log2_den exactly, for the complex128
input whose C-contiguous bytes hash to sha256.  Lines are appended as they
finish, so an interrupted run keeps its progress; rerunning skips names
already present.

usage: python tests/golden/make_golden.py {haar|batch|minors|boson} [workers]
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import inputs as I  # noqa: E402
import oracle as O  # noqa: E402


def _encode(v):
    re, im = v
    den = max(re.denominator, im.denominator)
    e = den.bit_length() - 1
    assert den == 1 << e, "dyadic denominator expected"
    return e, re.numerator * (den // re.denominator), im.numerator * (den // im.denominator)


def _done(path):
    if not os.path.exists(path):
        return set()
    with open(path) as f:
        return {l.split()[0] for l in f if l.strip() and not l.startswith("#")}


def _emit(path, name, a, v):
    e, re, im = _encode(v)
    with open(path, "a") as f:
        f.write(f"{name} {a.shape[0]} {I.sha256_of(a)} {e} {re} {im}\n")
        f.flush()


def _run(path, jobs, workers):
    done = _done(path)
    for name, a in jobs:
        if name in done:
            continue
        t = time.time()
        v = O.perm_exact_parallel(a, workers) if a.shape[0] > 14 else O.perm_exact(a)
        _emit(path, name, a, v)
        print(f"{name} n={a.shape[0]} {time.time() - t:.1f}s", flush=True)


def haar_jobs():
    yield "haar400_block20", I.haar400_block20()
    for n in (22, 24, 26, 28, 30):
        yield f"haar1600_block_n{n}", I.haar1600_block(n)


def batch_jobs():
    ns, mats = I.mixed_batch_16_26()
    picks = set(int(x) for x in np.random.default_rng(23).choice(len(ns), 32, replace=False))
    picks |= {b for b, n in enumerate(ns) if n <= 17}
    for b in sorted(picks, key=lambda b: (ns[b], b)):
        yield f"mixed_batch_b{b}", mats[b]


def minors_jobs():
    a = I.grad_batch_20()[0]
    for i in range(a.shape[0]):
        for j in range(a.shape[1]):
            yield f"grad_batch_m0_{i}_{j}", O.minor(a, i, j)


def boson_jobs():
    """U_{S,T} of three patterns of the 900-mode, 30-photon, 256-pattern
    workload (main text, Eq. (1)): patterns 11 and 234 (each 3888
    multiplicity-grouped sweeps of 14 single-photon columns in the library,
    the most any pattern takes) and 5 (3 grouped sweeps of 28 columns).  Per
    is stored; the probability is |Per|^2 / prod t_j!."""
    u, ins, pats = I.boson_workload()
    for p in (11, 234, 5):
        yield f"boson_workload_p{p}", O.gather_u_st(u, ins, pats[p])


def main():
    which = sys.argv[1]
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else O.host_cores()
    path = os.path.join(HERE, f"{which}_perms.txt")
    jobs = {"haar": haar_jobs, "batch": batch_jobs, "minors": minors_jobs, "boson": boson_jobs}[which]()
    _run(path, jobs, workers)


if __name__ == "__main__":
    main()
