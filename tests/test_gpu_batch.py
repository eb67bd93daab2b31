"""GPU: the batched factor and solve (spand_factor_batch / spand_solve_batch).

Problems shaped like the batched workload (variable coefficients 10^U(-2,2) on
grids of uneven edge lengths, depth from the grid size, 16 right-hand sides), at
sizes the oracle finishes in seconds.  Bars: every problem's result equals that of
the same handle driven alone (bit for bit: the batch shares launches between the
problems, but no problem's arithmetic depends on another's); kept ranks equal the
oracle's; PCG iterations within +-1 of the oracle's and true relative residual
<= 1e-12.
"""
import numpy as np
import pytest

import gridgen
from oracle import spand_oracle as O
from paper_1901_02971_amd import Solver, factor_batch, solve_batch
from tests.gpu_util import from_dev, note, oracle_run, rank_mismatches, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    note(request.node.nodeid)


def small_batch(count=6, nrhs=16, seed=7):
    edges = np.random.default_rng(seed).integers(9, 17, (count, 3))
    out = []
    for j in range(count):
        rng = np.random.default_rng(seed * 1000 + j)
        p = gridgen.variable_coefficient(tuple(int(e) for e in edges[j]), rng, -2.0, 2.0)
        out.append((p, gridgen.rhs(rng, p.n, nrhs), gridgen.levels_for(p.n)))
    return out


def test_batch_equals_single_handles_and_oracle():
    probs = small_batch()
    tol = 1e-2
    solvers = [Solver.from_problem(p, L) for p, _, L in probs]
    vals = [torch.from_numpy(p.values).to("cuda:0") for p, _, _ in probs]
    factor_batch(solvers, vals, tol)
    bt = [to_dev(b) for _, b, _ in probs]
    xt = [torch.empty_like(t) for t in bt]
    it, rr, st = solve_batch(solvers, bt, xt)
    assert st == 0
    for q, (p, b, L) in enumerate(probs):
        # the same problem on a handle of its own
        s1 = Solver.from_problem(p, L)
        s1.factor(vals[q], tol)
        x1 = torch.empty_like(bt[q])
        it1, rr1, _ = s1.solve(bt[q], x1)
        assert np.array_equal(it[q], it1)
        assert torch.equal(xt[q], x1), f"problem {q}: batched x differs from the single-handle x"
        assert solvers[q].stats()["m_F"] == s1.stats()["m_F"]
        # against the oracle
        an, fac = oracle_run(p, L, tol)
        assert rank_mismatches(solvers[q], an, fac) == 0
        _, it_ref, _ = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
        assert np.all(np.abs(it[q] - it_ref) <= 1), (q, it[q].tolist(), it_ref.tolist())
        assert np.all(rr[q] <= 1e-12), rr[q]
        x = from_dev(xt[q])
        res = np.linalg.norm(b - p.scipy() @ x, axis=0) / np.linalg.norm(b, axis=0)
        assert np.all(res <= 1e-12)


def test_batch_reports_failing_problem():
    probs = small_batch(count=3, nrhs=1, seed=9)
    solvers = [Solver.from_problem(p, L) for p, _, L in probs]
    vals = [torch.from_numpy(p.values).to("cuda:0") for p, _, _ in probs]
    bad = probs[1][0].values.copy()
    bad[probs[1][0].rowptr[5]:probs[1][0].rowptr[6]] *= -1.0  # row 5 of problem 1: negative diagonal
    vals[1] = torch.from_numpy(bad).to("cuda:0")
    with pytest.raises(Exception) as ei:
        factor_batch(solvers, vals, 1e-2)
    assert "batch problem 1" in str(ei.value)
    # the other problems were factored and solve normally
    bt = to_dev(probs[0][1])
    x = torch.empty_like(bt)
    it, rr, st = solvers[0].solve(bt, x)
    assert st == 0 and rr.max() <= 1e-12
