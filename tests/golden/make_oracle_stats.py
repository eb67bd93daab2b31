"""Write the FP64 oracle's results on a named workload to tests/golden/oracle_<name>.json.

Calls only the oracle and the seeded input generators (no library code), so the
stored values are the oracle's.  The workloads are the grid problems of
gridgen.config_problem; the 64^3 and 128^3 cases take minutes to an hour of CPU.

Stored per elimination step t: the sum of the cluster sizes before elimination,
the sum of the kept sizes, and SHA-256 digests of the two int32 arrays

    sizes[c] = active dofs of cluster c before the step's elimination
    kept[c]  = -1 if c is eliminated at step t, else its size after the step's
               sparsification (its size when the step does not sparsify it)

in cluster order; plus s_top, m_F, and the PCG iteration count and true relative
residual of every right-hand side.  With the interpolative variants (Sec. 2.6.2) a
factorization that loses positive definiteness stores the site instead (step,
cluster, phase).

Usage:  python tests/golden/make_oracle_stats.py c3 [tol [variant [rtol]]]
        (variant OrthS, In or InS; files of In and InS end in _In / _InS)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gridgen  # noqa: E402
from oracle import spand_oracle as O  # noqa: E402


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def step_arrays(an, fac):
    out = []
    for st, sf in zip(an.steps, fac.steps):
        sizes = np.asarray(sf.sizes, dtype=np.int64)
        kept = sizes.copy()
        kept[:st.n_elim] = -1
        for p, r in sf.ranks.items():
            kept[p] = r
        out.append((sizes, kept))
    return out


def main():
    name = sys.argv[1]
    tol = float(sys.argv[2]) if len(sys.argv) > 2 else 1e-2
    variant = sys.argv[3] if len(sys.argv) > 3 else "OrthS"
    rtol = float(sys.argv[4]) if len(sys.argv) > 4 else 1e-12
    p, b, levels = gridgen.config_problem(name)
    tag = f"{tol:.0e}".replace("e-0", "e-")
    suffix = "" if variant == "OrthS" else "_" + variant
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}_tol{tag}{suffix}.json")
    t0 = time.perf_counter()
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, levels)
    t1 = time.perf_counter()
    try:
        fac = O.factor(an, p.values, tol, variant=variant)
    except O.NotSPD as e:
        rec = {"workload": name, "n": int(p.n), "levels": int(levels), "tol": tol, "skip": 0, "variant": variant,
               "not_spd": {"step": int(e.step), "cluster": int(e.cluster), "phase": e.phase}}
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(f"{name} {variant}: not SPD at step {e.step}, cluster {e.cluster} ({e.phase}); wrote {path}", flush=True)
        return
    t2 = time.perf_counter()
    print(f"{name}: analyze {t1 - t0:.1f}s factor {t2 - t1:.1f}s", flush=True)
    _, it, rr = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r), rtol)
    t3 = time.perf_counter()
    print(f"{name}: pcg {t3 - t2:.1f}s iters {it.tolist()} relres {rr.max():.2e}", flush=True)
    steps = []
    for t, (sizes, kept) in enumerate(step_arrays(an, fac), start=1):
        steps.append({"step": t, "clusters": int(len(sizes)), "size_sum": int(sizes.sum()),
                      "kept_sum": int(kept[kept >= 0].sum()), "sizes_sha256": digest(sizes),
                      "kept_sha256": digest(kept)})
    rec = {"workload": name, "n": int(p.n), "levels": int(levels), "tol": tol, "skip": 0, "rtol": rtol,
           "maxit": 500, "s_top": int(fac.stats["s_top"]), "m_F": int(fac.stats["m_F"]),
           "pcg_iters": [int(v) for v in it], "relres": [float(v) for v in rr], "steps": steps,
           "oracle_seconds": {"analyze": round(t1 - t0, 1), "factor": round(t2 - t1, 1), "pcg": round(t3 - t2, 1)}}
    if variant != "OrthS":
        rec["variant"] = variant
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
