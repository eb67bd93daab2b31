"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI and
the FP64 oracle on the same seeded inputs."""
import sys

import numpy as np

from oracle import spand_oracle as O
from paper_1901_02971_amd import Solver


def note(msg):
    sys.stderr.write(f"[gpu-case] {msg}\n")
    sys.stderr.flush()


def to_dev(a):
    """numpy (n, nrhs) -> torch float64 (nrhs, n) on cuda:0 (= n x nrhs column-major)."""
    import torch
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda:0")


def from_dev(t):
    return t.cpu().numpy().T.copy()


def gpu_factor(p, levels, tol, skip=0, prec=0, geometry=True, variant="OrthS"):
    import torch
    s = Solver.from_problem(p, levels, geometry)
    s.set_variant(variant)
    vals = torch.from_numpy(p.values).to("cuda:0")
    s.factor(vals, tol, skip, prec)
    return s


def gpu_solve(s, b, rtol=1e-12, maxit=500, check=True):
    import torch
    bt = to_dev(b)
    xt = torch.empty_like(bt)
    it, rr, st = s.solve(bt, xt, rtol, maxit, check=check)
    return from_dev(xt), it, rr, st


def gpu_apply(s, r):
    import torch
    rt = to_dev(r)
    zt = torch.empty_like(rt)
    s.apply(rt, zt)
    return from_dev(zt)


def oracle_run(p, levels, tol, skip=0, geometry=True):
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords if geometry else None, levels, skip)
    fac = O.factor(an, p.values, tol)
    return an, fac


def rank_mismatches(s, an, fac):
    """Number of clusters whose kept size differs between the library and the oracle."""
    bad = 0
    for t, (st, sf) in enumerate(zip(an.steps, fac.steps), start=1):
        sizes, ranks = s.step_ranks(t)
        if not np.array_equal(sizes, np.array(sf.sizes, dtype=np.int32)):
            bad += int(np.sum(sizes != np.array(sf.sizes)))
        for p, r in sf.ranks.items():
            if ranks[p] != r:
                bad += 1
    return bad
