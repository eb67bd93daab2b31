"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a hand-stepped
run of Algorithm 2, an exact dense solve (the method is exact when nothing is
truncated), LAPACK's geqp3 through SciPy (the routine the paper used), the
Schur-complement identity of the stability theorem (Sec. 3.2), a brute-force
symbolic elimination, closed-form special cases and invariants.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import gridgen
from oracle import spand_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _code(s):
    if s == "-":
        return 0
    l, k = s.split(".")
    return int(O.pack(int(l), int(k)))


@pytest.mark.parametrize("fname,shape,levels", [("nd_7x7_L3.txt", (7, 7), 3), ("nd_6x4_L2.txt", (6, 4), 2)])
def test_alg2_hand_stepped(fname, shape, levels):
    """Algorithm 2 (Sec. 2.3) on small grids against hand-stepped runs."""
    rows = [ln.split(":")[1].split() for ln in open(os.path.join(GOLDEN, fname))
            if ln.startswith("y")]
    p = gridgen.laplacian(shape)
    S, L, R = O.nd_order(p.n, p.rowptr, p.colind, p.coords, levels)
    assert len(rows) == shape[1]
    for y, row in enumerate(rows):
        assert len(row) == shape[0]
        for x, ent in enumerate(row):
            s, l, r = ent.split("/")
            v = x + shape[0] * y
            assert (S[v], L[v], R[v]) == (_code(s), _code(l), _code(r)), (x, y)


@pytest.mark.parametrize("fname,shape,levels", [("nd_4x4x4_L3.txt", (4, 4, 4), 3),
                                                ("nd_3x3x5_L3.txt", (3, 3, 5), 3)])
def test_alg2_hand_stepped_3d(fname, shape, levels):
    """Algorithm 2 (Sec. 2.3) on small 3D grids against hand-stepped runs: the axis
    tie-break (x, y and z tied, then y and z), a cut along z, and boundary vertices
    of the middle set keeping their pointers."""
    nx, ny, nz = shape
    rows = {}
    for ln in open(os.path.join(GOLDEN, fname)):
        if ln.startswith("z"):
            head, body = ln.split(":")
            z, y = (int(w[1:]) for w in head.split())
            rows[(z, y)] = body.split()
    assert len(rows) == ny * nz
    p = gridgen.laplacian(shape)
    S, L, R = O.nd_order(p.n, p.rowptr, p.colind, p.coords, levels)
    for (z, y), row in rows.items():
        assert len(row) == nx
        for x, ent in enumerate(row):
            s, l, r = ent.split("/")
            v = x + nx * (y + ny * z)
            assert (S[v], L[v], R[v]) == (_code(s), _code(l), _code(r)), (x, y, z)


def test_alg2_graph_separator_hand_stepped():
    """Algorithm 2 with the breadth-first level-structure separator (no coordinates)
    on the 4x4 grid at 3 levels against a hand-stepped run."""
    rows = [ln.split(":")[1].split() for ln in open(os.path.join(GOLDEN, "nd_graph_4x4_L3.txt"))
            if ln.startswith("y")]
    p = gridgen.laplacian((4, 4))
    S, L, R = O.nd_order(p.n, p.rowptr, p.colind, None, 3)
    for y, row in enumerate(rows):
        for x, ent in enumerate(row):
            s, l, r = ent.split("/")
            v = x + 4 * y
            assert (S[v], L[v], R[v]) == (_code(s), _code(l), _code(r)), (x, y)


def _graph_cases():
    two = gridgen.laplacian((5, 4))
    # two disconnected copies of a small grid (block diagonal)
    import scipy.sparse as sp
    A = sp.block_diag([two.scipy(), 2.0 * two.scipy()]).tocsr()
    A.sort_indices()
    disc = gridgen.GridProblem(n=A.shape[0], rowptr=A.indptr.astype(np.int64), colind=A.indices.astype(np.int32),
                               values=A.data, coords=np.zeros((A.shape[0], 2)), dim=2, shape=(A.shape[0],))
    return [("grid2d", gridgen.laplacian((16, 16)), 5),
            ("grid3d", gridgen.laplacian((9, 7, 6)), 4),
            ("permuted3d", gridgen.permuted(gridgen.laplacian((8, 9, 10)), np.random.default_rng(3)), 5),
            ("knn", gridgen.knn_graph_laplacian(600, 6, np.random.default_rng(4)), 5),
            ("disconnected", disc, 4)]


@pytest.mark.parametrize("name,p,levels", _graph_cases(), ids=[c[0] for c in _graph_cases()])
def test_graph_separator_invariants(name, p, levels):
    """Without coordinates: every edge joins equal S or an ancestor/descendant pair
    (the middle set separates), each separator is one cluster at its step, and the
    factorization stays exact at eps = 0."""
    S, L, R = O.nd_order(p.n, p.rowptr, p.colind, None, levels)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    a, b = S[rows], S[p.colind]
    la, lb = O.lev_of(a), O.lev_of(b)
    deep = np.where(la >= lb, a, b)
    shallow = np.where(la >= lb, b, a)
    assert np.all(O.truncate(deep, np.minimum(la, lb)) == shallow)
    an = O.Analysis(p.n, p.rowptr, p.colind, None, levels)
    for st in an.steps:
        ids = st.keys[: st.n_elim, 0]
        assert len(np.unique(ids)) == st.n_elim
    if p.n <= 700:
        A = p.scipy().toarray()
        bb = np.random.default_rng(1).standard_normal((p.n, 2))
        fac = O.factor(an, p.values, 0.0)
        z = O.apply(fac, bb)
        x_ref = sla.cho_solve(sla.cho_factor(A), bb)
        assert np.abs(z - x_ref).max() <= 1e-10 * np.abs(x_ref).max()


@pytest.mark.parametrize("shape,levels", [((7, 7), 3), ((16, 16), 5), ((9, 7, 6), 4), ((8, 8, 8), 5)])
def test_alg2_invariants(shape, levels):
    """ND invariants: an edge never joins two different separators unless one is an
    ancestor of the other in the ND tree; leaves number 2^(L-1); pointers of a
    separator vertex point below its own level."""
    p = gridgen.laplacian(shape)
    S, L, R = O.nd_order(p.n, p.rowptr, p.colind, p.coords, levels)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    a, b = S[rows], S[p.colind]
    la, lb = O.lev_of(a), O.lev_of(b)
    # ancestor test: truncating the deeper id to the shallower level gives the shallower id
    deep = np.where(la >= lb, a, b)
    shallow = np.where(la >= lb, b, a)
    anc = O.truncate(deep, np.minimum(la, lb)) == shallow
    assert np.all(anc)
    leaves = np.unique(S[O.lev_of(S) == levels])
    assert len(leaves) == 2 ** (levels - 1)
    sep = O.lev_of(S) < levels
    assert np.all(O.lev_of(L[sep]) > O.lev_of(S[sep]))
    assert np.all(O.lev_of(R[sep]) > O.lev_of(S[sep]))
    assert np.all(L[~sep] == 0) and np.all(R[~sep] == 0)


@pytest.mark.parametrize("shape,levels", [((7, 7), 3), ((12, 10), 4), ((6, 5, 7), 4), ((8, 8, 8), 4)])
def test_each_separator_is_one_cluster(shape, levels):
    """At the step that eliminates level l, every separator (l, k) is exactly one cluster."""
    p = gridgen.laplacian(shape)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, levels)
    for st in an.steps:
        ids = st.keys[: st.n_elim, 0]
        assert len(np.unique(ids)) == st.n_elim
        assert np.all(O.lev_of(ids) == st.level)


@pytest.mark.parametrize("shape,levels", [((16, 16), 5), ((9, 7, 6), 4), ((12, 12, 12), 6)])
def test_colouring_proper_and_greedy(shape, levels):
    """The sparsification colouring lets a GPU run one colour class at once with the
    result of the sequential order: no two interfaces joined by a block may share a
    colour.  It is also the greedy one in ascending cluster id: every colour below
    p's is taken by a lower-numbered neighbour of p, and p's is not."""
    p = gridgen.laplacian(shape)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, levels)
    checked = 0
    for st in an.steps:
        if not st.sparsify:
            assert np.all(st.colour == -1)
            continue
        assert np.all(st.colour[: st.n_elim] == -1)
        for (i, j) in st.after:
            if i != j:
                assert st.colour[i] != st.colour[j], (st.level, i, j)
                checked += 1
        for q in range(st.n_elim, len(st.keys)):
            lower = {int(st.colour[u]) for u in st.nbrs[q] if u < q}
            c = int(st.colour[q])
            assert c >= 0 and c not in lower and all(k in lower for k in range(c))
    assert checked > 0


def _brute_force_pattern(p, an):
    """Vertex-level symbolic elimination: eliminating a vertex joins all its
    remaining neighbours.  Returns, per step, the set of cluster pairs joined by a
    (filled) edge among the clusters present before that step's elimination."""
    n = p.n
    adj = [set() for _ in range(n)]
    for v in range(n):
        for u in p.colind[p.rowptr[v]:p.rowptr[v + 1]]:
            if u != v:
                adj[v].add(int(u))
    # vertex -> cluster id per step
    owner = []
    step_of_vertex = np.empty(n, dtype=np.int64)
    cl = np.empty(n, dtype=np.int64)
    for c, ch in enumerate(an.steps[0].children):
        cl[ch] = c
    for t, st in enumerate(an.steps):
        if t > 0:
            prev = an.steps[t - 1]
            cl = np.where(cl >= 0, prev.parent[np.maximum(cl, 0)], -1)
            cl[(cl < 0)] = -1
        owner.append(cl.copy())
        step_of_vertex[(cl >= 0) & (cl < st.n_elim)] = t
    alive = np.ones(n, dtype=bool)
    pats = []
    for t, st in enumerate(an.steps):
        cl = owner[t]
        pat = set()
        for v in np.nonzero(alive)[0]:
            pat.add((cl[v], cl[v]))
            for u in adj[v]:
                a, b = cl[v], cl[u]
                pat.add((max(a, b), min(a, b)))
        pats.append(pat)
        for v in np.nonzero(alive & (step_of_vertex == t))[0]:
            nb = [u for u in adj[v] if alive[u] and u != v]
            for u in nb:
                adj[u].discard(int(v))
                for w in nb:
                    if w != u:
                        adj[u].add(int(w))
            alive[v] = False
    return pats


@pytest.mark.parametrize("shape,levels", [((7, 7), 3), ((16, 16), 4), ((6, 5, 7), 4), ((8, 8, 8), 4)])
def test_fill_pattern_brute_force(shape, levels):
    """Block pattern of every step against a vertex-level symbolic elimination
    (ND creates fill only among neighbours of an eliminated cluster, Sec. 2.1/2.4)."""
    p = gridgen.laplacian(shape)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, levels)
    pats = _brute_force_pattern(p, an)
    for st, pat in zip(an.steps, pats):
        assert set(map(tuple, st.blocks)) == pat


@pytest.mark.parametrize("shape,levels", [((7, 7), 3), ((16, 16), 5), ((6, 5, 7), 4), ((8, 8, 8), 5)])
@pytest.mark.parametrize("tol,skip", [(0.0, 0), (0.3, 99)])
def test_exact_when_nothing_truncated(shape, levels, tol, skip):
    """With eps = 0 (full rank kept) or sparsification skipped ("Direct", Sec. 4),
    M M^T = A^-1: the preconditioned solve equals a dense Cholesky solve."""
    p = gridgen.laplacian(shape)
    A = p.scipy().toarray()
    b = np.random.default_rng(7).standard_normal((p.n, 3))
    x_ref = sla.cho_solve(sla.cho_factor(A), b)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, levels, skip)
    fac = O.factor(an, p.values, tol)
    z = O.apply(fac, b)
    assert np.abs(z - x_ref).max() <= 1e-12 * np.abs(x_ref).max()
    _, it, rr = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
    assert np.all(it == 1) and np.all(rr < 1e-13)


def test_exact_variable_coefficients():
    """Exactness also holds for the high-contrast variable-coefficient operator."""
    p = gridgen.variable_coefficient((6, 7, 5), np.random.default_rng(3), -3, 3)
    A = p.scipy().toarray()
    b = np.random.default_rng(1).standard_normal((p.n, 2))
    x_ref = sla.cho_solve(sla.cho_factor(A), b)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 4)
    fac = O.factor(an, p.values, 0.0)
    z = O.apply(fac, b)
    assert np.abs(z - x_ref).max() <= 1e-10 * np.abs(x_ref).max()


def test_full_preconditioner_dense_identity():
    """F A F^T = I exactly at eps = 0, where z = F^T F r is the apply (Sec. 2.8)."""
    p = gridgen.laplacian((9, 8))
    A = p.scipy().toarray()
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 4)
    fac = O.factor(an, p.values, 0.0)
    Minv = O.apply(fac, np.eye(p.n))          # = F^T F
    assert np.abs(Minv @ A - np.eye(p.n)).max() < 1e-12


@pytest.mark.parametrize("eps", [1e-12, 1e-2, 0.5, 0.9, 1.0, 2.0])
def test_never_breaks_down(eps):
    """OrthS never breaks down for any eps >= 0 (Corollary, Sec. 3.2), including on
    a high-contrast operator; M M^T stays SPD."""
    p = gridgen.variable_coefficient((9, 8, 7), np.random.default_rng(11), -3, 3)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 5)
    fac = O.factor(an, p.values, eps)
    P = O.apply(fac, np.eye(p.n))
    assert np.allclose(P, P.T, atol=1e-10 * np.abs(P).max())
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0


def test_accuracy_improves_as_eps_decreases():
    """||I - F A F^T|| shrinks with eps (qualitative claim of Sec. 4)."""
    p = gridgen.laplacian((8, 8, 8))
    A = p.scipy().toarray()
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 5)
    errs = []
    for eps in [0.5, 1e-1, 1e-2, 1e-4, 1e-8]:
        fac = O.factor(an, p.values, eps)
        P = O.apply(fac, np.eye(p.n))
        w = np.linalg.eigvals(P @ A).real
        errs.append(w.max() / w.min())
    assert all(a >= b * 0.999 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1 + 1e-6


def test_cg_iterations_fall_with_eps():
    p = gridgen.laplacian((12, 12, 12))
    b = gridgen.rhs(np.random.default_rng(5), p.n, 1)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 6)
    its = []
    for eps in [1e-1, 1e-2, 1e-4]:
        fac = O.factor(an, p.values, eps)
        _, it, rr = O.pcg(p.scipy(), b, lambda r: O.apply(fac, r))
        assert rr[0] <= 1e-12
        its.append(int(it[0]))
    assert its[0] > its[1] > its[2], its


# ---------------------------------------------------------------- CPQR pins
@pytest.mark.parametrize("m,n,seed", [(20, 35, 0), (35, 20, 1), (49, 120, 2), (7, 7, 3)])
def test_cpqr_matches_geqp3(m, n, seed):
    """Pivots and |R_ii| agree with LAPACK geqp3 (the routine of Sec. 4 intro) on
    random matrices, whose column norms have no ties."""
    A = np.random.default_rng(seed).standard_normal((m, n))
    r, V, tau, W, perm = O.cpqr(A, 0.0)
    Q, R, P = sla.qr(A, pivoting=True, mode="economic")
    k = min(m, n)
    assert r == k
    assert np.array_equal(perm[:k], P[:k])
    Rd = np.abs(np.diag(W[:, perm]))
    assert np.allclose(Rd, np.abs(np.diag(R)), rtol=1e-12)
    # W = Q^T A restricted to the kept rows; Q orthogonal
    Qf = O.apply_q(V, tau, np.eye(m))
    assert np.abs(Qf.T @ Qf - np.eye(m)).max() < 1e-13
    assert np.abs((Qf.T @ A)[:r] - W).max() < 1e-12 * np.abs(A).max()
    if m > k:
        assert np.abs((Qf.T @ A)[r:]).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("eps", [1e-8, 1e-6, 1e-3])
def test_cpqr_rank_of_noisy_low_rank(eps):
    rng = np.random.default_rng(4)
    k = 9
    A = rng.standard_normal((40, k)) @ rng.standard_normal((k, 90)) + 1e-10 * rng.standard_normal((40, 90))
    r, *_ = O.cpqr(A, eps)
    assert r == k


def test_cpqr_special_cases():
    assert O.cpqr(np.zeros((5, 8)), 1e-2)[0] == 0          # R_00 = 0
    A = np.random.default_rng(0).standard_normal((6, 9))
    assert O.cpqr(A, 0.0)[0] == 6                           # eps = 0 keeps min(m, n)
    assert O.cpqr(A, 1.5)[0] == 0                           # eps > 1 keeps nothing
    assert O.cpqr(A, 1.0)[0] >= 1                           # |R_00| >= 1 * |R_00|


def test_cpqr_tie_goes_to_smallest_original_column():
    A = np.eye(4) * 2.0
    r, V, tau, W, perm = O.cpqr(A, 0.0)
    assert list(perm) == [0, 1, 2, 3]
    # column 3 wins step 0; afterwards columns 0, 1, 2 tie and go in index order
    # (a swap-order rule would take column 3's old position's occupant, 0, last)
    B = np.diag([1.0, 1.0, 1.0, 2.0])
    r, V, tau, W, perm = O.cpqr(B, 0.0)
    assert list(perm) == [3, 0, 1, 2]


def test_cpqr_position_rule_matches_geqp3_on_exact_ties():
    """The tie="position" rule is LAPACK's: with exact ties after a swap, geqp3 takes
    the first column at its current position."""
    B = np.diag([1.0, 1.0, 1.0, 2.0])
    _, _, P = sla.qr(B, pivoting=True)
    r, V, tau, W, perm = O.cpqr(B, 0.0, tie="position")
    assert list(perm) == list(P) == [3, 1, 2, 0]
    # the two rules agree whenever no tie is met
    A = np.random.default_rng(8).standard_normal((15, 40))
    assert np.array_equal(O.cpqr(A, 1e-3, tie="position")[4], O.cpqr(A, 1e-3)[4])
    with pytest.raises(ValueError):
        O.cpqr(B, 0.0, tie="other")


def _dense_trailing(blocks, sizes, ids):
    """Dense matrix of the clusters `ids` (in that order) from the block dict."""
    off = np.concatenate([[0], np.cumsum([sizes[c] for c in ids])]).astype(int)
    T = np.zeros((off[-1], off[-1]))
    for a, i in enumerate(ids):
        for b, j in enumerate(ids):
            key = (max(i, j), min(i, j))
            if key in blocks:
                blk = blocks[key] if i >= j else blocks[key].T
                T[off[a]:off[a + 1], off[b]:off[b + 1]] = blk
    return T, off


def _explicit_q(V, tau, m):
    """Q = H_0 H_1 ... H_{r-1} as a dense matrix, from its reflectors."""
    Q = np.eye(m)
    for j in range(V.shape[1]):
        v = V[:, j]
        Q = Q @ (np.eye(m) - tau[j] * np.outer(v, v))
    return Q


@pytest.mark.parametrize("tol", [0.3, 1e-2])
def test_sparsification_in_context(tol):
    """Orthogonal sparsification inside Algorithm 3 at eps > 0, on the live trailing
    matrix of a small 3D grid (Sec. 2.6.1 and the stability theorem of Sec. 3.2):
    the scaled A_pp is I; with A_pn = Q [W_cn; W_fn], the Schur complement onto the
    rest after dropping f is S_B = S_A + W_fn^T W_fn, i.e. the error is
    E_nn = W_fn^T W_fn >= 0; the new trailing matrix stays SPD; and what the step
    writes back is W_cn in row block p with A_cc = I_r."""
    p = gridgen.variable_coefficient((7, 6, 8), np.random.default_rng(21), -2, 2)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 4)
    seen = {"n": 0, "dropped": 0, "writeback": 0}
    prev = {}

    def hook(t, q, nb, sizes, blocks, Apn, res):
        # the previous interface of this step wrote back its kept rows
        if prev.get("t") == t:
            pq, W, pnb, psz = prev["p"], prev["W"], prev["nb"], prev["sizes"]
            r = W.shape[0]
            assert np.array_equal(blocks[(pq, pq)], np.eye(r))
            col = 0
            for u in pnb:
                wu = W[:, col:col + psz[u]]
                col += psz[u]
                got = blocks[(pq, u)] if pq >= u else blocks[(u, pq)].T
                assert np.array_equal(got, wu)
            seen["writeback"] += 1
        r, V, tau, W, perm = res
        alive = sorted({i for key in blocks for i in key})
        rest = [c for c in alive if c != q]
        T, off = _dense_trailing(blocks, sizes, [q] + rest)
        k = sizes[q]
        assert np.abs(T[:k, :k] - np.eye(k)).max() < 1e-13      # scaled: A_pp = I
        Apn_dense = T[:k, k:]
        # the gathered row block is A_pn on the neighbour columns, zero elsewhere
        noff = dict(zip(rest, off[1:-1] - k))
        cols = np.concatenate([np.arange(noff[u], noff[u] + sizes[u]) for u in nb]).astype(int)
        assert np.array_equal(Apn_dense[:, cols], Apn)
        mask = np.ones(Apn_dense.shape[1], bool)
        mask[cols] = False
        assert not np.any(Apn_dense[:, mask])
        Q = _explicit_q(V, tau, k)
        assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-13
        full = Q.T @ Apn
        Wc, Wf = full[:r], full[r:]
        assert np.abs(Wc - W).max() <= 1e-12 * max(1.0, np.abs(Apn).max())
        Ann = T[k:, k:]
        Wc_d = np.zeros((r, Ann.shape[0]))
        Wc_d[:, cols] = W
        Wf_d = np.zeros((k - r, Ann.shape[0]))
        Wf_d[:, cols] = Wf
        S_A = Ann - Apn_dense.T @ Apn_dense
        S_B = Ann - Wc_d.T @ Wc_d
        E = S_B - S_A
        assert np.abs(E - Wf_d.T @ Wf_d).max() <= 1e-12 * max(1.0, np.abs(Ann).max())
        assert np.linalg.eigvalsh(E).min() >= -1e-12 * max(1.0, np.abs(E).max())
        newT = np.block([[np.eye(r), Wc_d], [Wc_d.T, Ann]])
        assert np.linalg.eigvalsh(newT).min() > 0
        seen["n"] += 1
        seen["dropped"] += int(r < k)
        prev.update(t=t, p=q, W=W.copy(), nb=list(nb), sizes=list(sizes))

    O.factor(an, p.values, tol, on_sparsify=hook)
    assert seen["n"] > 20 and seen["dropped"] > 5 and seen["writeback"] > 10, seen


def test_sparsification_schur_identity():
    """Theorem of Sec. 3.2: with A_pp = I and A_pn = Q [W_cn; W_fn], the n-n Schur
    complement after dropping f is S_B = S_A + W_fn^T W_fn, and B_p is SPD."""
    rng = np.random.default_rng(2)
    np_, nn = 12, 30
    X = rng.standard_normal((np_ + nn, np_ + nn))
    A = X @ X.T + (np_ + nn) * np.eye(np_ + nn)
    Lp = np.linalg.cholesky(A[:np_, :np_])
    Apn = sla.solve_triangular(Lp, A[:np_, np_:], lower=True)   # scaled so A_pp = I
    Ann = A[np_:, np_:]
    for eps in [0.5, 0.1, 1e-2]:
        r, V, tau, W, perm = O.cpqr(Apn, eps)
        Qf = O.apply_q(V, tau, np.eye(np_))
        full = Qf.T @ Apn
        Wc, Wf = full[:r], full[r:]
        assert np.abs(Wc - W).max() < 1e-12
        S_A = Ann - Apn.T @ Apn
        S_B = Ann - Wc.T @ Wc
        assert np.abs(S_B - (S_A + Wf.T @ Wf)).max() < 1e-10
        B = np.block([[np.eye(r), Wc], [Wc.T, Ann]])
        assert np.linalg.eigvalsh(B).min() > 0
        # dropped part bounded by the truncation rule
        if r < np_:
            assert np.linalg.norm(Wf, 2) <= np.sqrt(nn) * eps * np.linalg.norm(Apn[:, perm[0]])


# ---------------------------------------------------------------- misc pins
def test_scale_invariance():
    """A -> 7.3 A leaves ranks and iteration counts unchanged (ratio rule + Cholesky scaling)."""
    p = gridgen.laplacian((10, 9, 8))
    b = gridgen.rhs(np.random.default_rng(9), p.n, 1)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 5)
    f1 = O.factor(an, p.values, 1e-2)
    f2 = O.factor(an, 7.3 * p.values, 1e-2)
    assert f1.stats["ranks"] == f2.stats["ranks"]
    A = p.scipy()
    _, i1, _ = O.pcg(A, b, lambda r: O.apply(f1, r))
    _, i2, _ = O.pcg(7.3 * A, b, lambda r: O.apply(f2, r))
    assert np.array_equal(i1, i2)


def test_not_spd_detected():
    p = gridgen.laplacian((8, 8))
    vals = p.values.copy()
    d = np.nonzero(p.colind == 0)[0][0]     # row 0 diagonal
    vals[d] = -4.0
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 3)
    with pytest.raises(O.NotSPD) as e:
        O.factor(an, vals, 1e-2)
    assert e.value.step == 1


def test_pcg_zero_rhs_and_solution():
    p, b, L = gridgen.config_problem("c1")
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, L)
    fac = O.factor(an, p.values, 1e-2)
    A = p.scipy()
    x, it, rr = O.pcg(A, np.zeros((p.n, 1)), lambda r: O.apply(fac, r))
    assert it[0] == 0 and np.all(x == 0)
    x, it, rr = O.pcg(A, b, lambda r: O.apply(fac, r))
    xs = spla.spsolve(A.tocsc(), b[:, 0])
    assert rr[0] <= 1e-12
    assert np.abs(x[:, 0] - xs).max() <= 1e-10 * np.abs(xs).max()


def test_pcg_checks_the_true_residual():
    """The stop rule is on the true residual: a target below what FP64 can reach
    runs to maxit instead of stopping on a recursive residual that keeps falling."""
    p = gridgen.laplacian((20, 20))
    b = gridgen.rhs(np.random.default_rng(3), p.n, 1)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 4)
    fac = O.factor(an, p.values, 0.3)
    A = p.scipy()
    _, it, rr = O.pcg(A, b, lambda r: O.apply(fac, r), rtol=1e-19, maxit=40)
    assert it[0] == 40 and rr[0] > 1e-19
    _, it, rr = O.pcg(A, b, lambda r: O.apply(fac, r), rtol=1e-12, maxit=40)
    assert it[0] < 40 and rr[0] <= 1e-12


def test_pcg_breakdown_is_reported():
    p = gridgen.laplacian((6, 6))
    b = gridgen.rhs(np.random.default_rng(3), p.n, 2)
    with pytest.raises(O.Breakdown) as e:
        O.pcg(p.scipy(), b, lambda r: np.full_like(r, np.nan))
    assert e.value.column == 0 and e.value.iteration == 1


def test_generator_operator():
    """The generator builds the stated stencil: SPD, symmetric, row sums 0 inside."""
    p = gridgen.laplacian((5, 4, 3))
    A = p.scipy().toarray()
    assert np.array_equal(A, A.T)
    v = 1 + 5 * (1 + 4 * 1)   # interior vertex (1,1,1)
    assert A[v, v] == 6 and A[v].sum() == 0
    q = gridgen.variable_coefficient((4, 3, 5), np.random.default_rng(0), -3, 3)
    B = q.scipy().toarray()
    assert np.allclose(B, B.T) and np.linalg.eigvalsh(B).min() > 0


# ---------------------------------------------------------------------------
# Interpolative variants In / InS (Sec. 2.6.2, Sec. 3.1, Sec. 4.1.1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("variant", ["In", "InS"])
def test_interpolative_congruence_in_context(variant):
    """The interpolative step on the live trailing matrix of a small 2D grid, against
    an explicit dense congruence: with T_p = [I_f 0; -T_cf I_c] (written out as a
    matrix over p's dofs), T_p^T B T_p has f-f block C_ff and c-f block C_cf as the
    step computes them, leaves the c-c and c-n blocks of B unchanged, and its f-n
    block A_nf - A_nc T_cf = Q_2 R_22 has every column below eps times the largest
    column of A_np (the CPQR stop rule).  With scaling (InS) A_pp = I, so
    C_ff = I + T_cf^T T_cf and C_cf = -T_cf (Sec. 3.1)."""
    tol = 1e-2
    p = gridgen.variable_coefficient((24, 20), np.random.default_rng(3), -1, 1)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 5)
    seen = {"n": 0}

    def hook(t, q, nb, sizes, blocks, Anp, res, interp=None):
        if interp is None:
            return
        r, _, _, _, perm = res
        c, f, T = interp["c"], interp["f"], interp["T"]
        assert np.array_equal(np.sort(np.concatenate([c, f])), np.arange(sizes[q]))
        ids = [q] + list(nb)
        B, off = _dense_trailing(blocks, sizes, ids)
        k = sizes[q]
        assert np.array_equal(B[k:, :k], Anp)
        Tp = np.eye(B.shape[0])
        Tp[np.ix_(c, f)] = -T
        C = Tp.T @ B @ Tp
        scale = max(1.0, np.abs(B).max())
        assert np.abs(C[np.ix_(f, f)] - interp["Cff"]).max() <= 1e-12 * scale * (1 + np.abs(T).max()) ** 2
        assert np.abs(C[np.ix_(c, f)] - interp["Ccf"]).max() <= 1e-12 * scale * (1 + np.abs(T).max())
        assert np.array_equal(C[np.ix_(c, c)], B[np.ix_(c, c)])
        assert np.array_equal(C[c, k:], B[c, k:])
        Ynf = C[k:, f]
        cmax = np.sqrt((Anp ** 2).sum(axis=0)).max()
        assert np.sqrt((Ynf ** 2).sum(axis=0)).max() < tol * cmax * (1 + 1e-9)
        if variant == "InS":
            assert np.abs(B[:k, :k] - np.eye(k)).max() < 1e-13
            assert np.abs(interp["Cff"] - (np.eye(len(f)) + T.T @ T)).max() <= 1e-13 * (1 + np.abs(T).max()) ** 2
            assert np.abs(interp["Ccf"] + T).max() <= 1e-13 * (1 + np.abs(T).max())
        seen["n"] += 1

    O.factor(an, p.values, tol, on_sparsify=hook, variant=variant)
    assert seen["n"] >= 5


@pytest.mark.parametrize("variant", ["In", "InS"])
def test_interpolative_error_follows_eps(variant):
    """z = M M^T b against an exact dense solve: the interpolative preconditioner is
    exact up to the dropped f-n coupling, so the error falls with eps (Sec. 3.1:
    ||E_nn|| = O(eps^2) ||C_ff^-1||), down to rounding once nothing is dropped."""
    p = gridgen.variable_coefficient((24, 20), np.random.default_rng(3), -1, 1)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 5)
    A = p.scipy().toarray()
    b = np.random.default_rng(1).standard_normal((p.n, 2))
    x = np.linalg.solve(A, b)
    for tol in (1e-4, 1e-6, 1e-8):
        fac = O.factor(an, p.values, tol, variant=variant)
        assert sum(len(sf.I) for sf in fac.steps) >= 1          # something was dropped
        assert not any(sf.Q for sf in fac.steps)
        assert bool(any(sf.S for sf in fac.steps)) == (variant == "InS")
        err = np.abs(O.apply(fac, b) - x).max() / np.abs(x).max()
        assert err <= 100 * tol
    fac = O.factor(an, p.values, 1e-12, variant=variant)
    assert not any(sf.I for sf in fac.steps)
    assert np.abs(O.apply(fac, b) - x).max() / np.abs(x).max() < 1e-12


def test_interpolative_stored_factors_and_slots():
    """The stored pieces of an interpolative step are consistent: L_f is the lower
    Cholesky factor of C_ff, G_cf L_f^T = C_cf, perm is a permutation of p whose first
    r entries name the kept (coarse) dofs and the rest the fine ones, in the order
    the step handed them out; the apply is symmetric (M M^T)."""
    p = gridgen.variable_coefficient((24, 20), np.random.default_rng(3), -1, 1)
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 5)
    got = {}

    def hook(t, q, nb, sizes, blocks, Anp, res, interp=None):
        if interp is not None:
            got.setdefault(t, []).append(interp)   # in the order the step stores them

    fac = O.factor(an, p.values, 1e-2, on_sparsify=hook, variant="In")
    assert got
    for t, sf in enumerate(fac.steps, start=1):
        assert len(sf.I) == len(got.get(t, []))
        for (sp, perm, k, T, Lf, G), it in zip(sf.I, got.get(t, [])):
            assert np.array_equal(np.sort(perm), np.arange(len(sp)))
            assert np.array_equal(perm[:k], it["c"]) and np.array_equal(perm[k:], it["f"])
            assert np.allclose(Lf @ Lf.T, it["Cff"], rtol=0, atol=1e-12 * np.abs(it["Cff"]).max())
            assert np.all(np.triu(Lf, 1) == 0)
            assert np.allclose(G @ Lf.T, it["Ccf"], rtol=0, atol=1e-12 * max(1, np.abs(it["Ccf"]).max()))
    Z = O.apply(fac, np.eye(p.n)[:, :40])
    ZT = O.apply(fac, np.eye(p.n))[:40, :].T
    assert np.abs(Z - ZT).max() <= 1e-12 * np.abs(Z).max()


def test_interpolative_breaks_down_where_orths_does_not():
    """Sec. 3.2 / Sec. 4.1.1: on a 2D high-contrast field (rho = 100, 64 x 64, five
    levels) the interpolative factorization loses positive definiteness, without
    scaling at eps = 1e-2 and with scaling at eps = 1e-1, while OrthS factors and
    PCG converges at both."""
    prob = gridgen.high_contrast((64, 64), np.random.default_rng(1064), 100.0)
    an = O.Analysis(prob.n, prob.rowptr, prob.colind, prob.coords, 5)
    A = prob.scipy()
    b = gridgen.rhs(np.random.default_rng(7), prob.n, 1)
    with pytest.raises(O.NotSPD):
        O.factor(an, prob.values, 1e-2, variant="In")
    with pytest.raises(O.NotSPD):
        O.factor(an, prob.values, 1e-1, variant="InS")
    for tol in (1e-1, 1e-2):
        fac = O.factor(an, prob.values, tol)
        _, it, rr = O.pcg(A, b, lambda r: O.apply(fac, r), 1e-10, 100)
        assert rr[0] <= 1e-10 and it[0] < 100


def test_variant_argument_checked():
    p = gridgen.laplacian((6, 6))
    an = O.Analysis(p.n, p.rowptr, p.colind, p.coords, 2)
    with pytest.raises(ValueError):
        O.factor(an, p.values, 1e-2, variant="Orth")
