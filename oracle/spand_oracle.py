"""Plain FP64 CPU oracle for sparsified nested dissection (spaND: OrthS, In, InS).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or runs
this module; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It is written for readability against the paper (Cambier et al.,
"An algebraic sparsified nested dissection algorithm using low-rank
approximations"), not for speed: every dense step is a numpy/scipy primitive
(Cholesky, triangular solve, matrix product) or a short explicit loop, with no
blocking, fusion or reordering beyond what the paper's algorithms state.

Contents, each following the cited passage:
  * ``nd_order``      Algorithm 2 (modified ND ordering and clustering, Sec. 2.3)
                      with the geometric vertex separator of Sec. 2.3 / 4.1.1, or a
                      breadth-first level-structure separator for graphs without
                      coordinates.
  * ``symbolic``      the cluster hierarchy of each separator (Sec. 2.3, 2.7) and the
                      block pattern of the trailing matrix with the fill of Sec. 2.4.
  * ``factor``        Algorithm 3 (OrthS): elimination (Sec. 2.4), block scaling
                      (Sec. 2.5), orthogonal sparsification (Sec. 2.6.1) with the
                      truncation rule of Sec. 4 (intro), merge (Sec. 2.7); and the
                      interpolative variants In (no scaling) and InS (scaling) of
                      Sec. 2.6.2 / Sec. 3.1.
  * ``apply``         z = M M^T r with M from Sec. 2.8 (operator order of the
                      caption of the spaND illustration figure).
  * ``pcg``           CG preconditioned by M M^T, stopped at ||b-Ax||/||b|| <= rtol (Sec. 4).
  * ``cpqr``          column-pivoted Householder QR (Businger-Golub pivoting).

Readings of points the paper leaves open are listed where they are used and are
the same ones the GPU library implements (separator tie-breaks, cluster order,
sparsification order, CPQR tie-break and stop rule, skip semantics).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

# Relative window inside which CPQR column norms count as tied.  Among tied
# columns the pivot is the one with the smallest original column index
# (tie="original", the default), or the one at the smallest current position
# after the swaps of the earlier steps (tie="position", the rule of LAPACK's
# geqp3, whose idamax takes the first maximum).
TIE_RTOL = 1e-10
TIE_RULES = ("original", "position")

# Sparsification variants compared in Sec. 3.1 / Sec. 4.1: orthogonal with block
# scaling (the method), interpolative without and with block scaling.
VARIANTS = ("OrthS", "In", "InS")


class NotSPD(Exception):
    """A pivot or interface block failed Cholesky: (step, cluster, phase)."""

    def __init__(self, step, cluster, phase):
        super().__init__(f"not SPD at step {step}, cluster {cluster}, phase {phase}")
        self.step, self.cluster, self.phase = step, cluster, phase


# ---------------------------------------------------------------------------
# Separator ids.  A separator (level l, index k), 1 <= k <= 2^(l-1), is packed
# as l * 2^32 + k so that integer order equals (level, index) order; "none" is 0.
# ---------------------------------------------------------------------------
def pack(level, index):
    return (np.int64(level) << 32) | np.int64(index)


def lev_of(code):
    return np.asarray(code, dtype=np.int64) >> 32


def idx_of(code):
    return np.asarray(code, dtype=np.int64) & 0xFFFFFFFF


def truncate(code, level):
    """Ancestor at ``level`` of a separator id deeper than ``level`` (Sec. 2.7: one
    merge per level moves a cluster one level up the cluster tree); ids at or
    above ``level`` and "none" are returned unchanged."""
    code = np.asarray(code, dtype=np.int64)
    lv = lev_of(code)
    ix = idx_of(code)
    deeper = lv > level
    shift = np.where(deeper, lv - level, 0)
    new_ix = np.where(deeper, ((ix - 1) >> shift) + 1, ix)
    new_lv = np.where(deeper, level, lv)
    return np.where(code == 0, 0, (new_lv << 32) | new_ix)


# ---------------------------------------------------------------------------
# Algorithm 2 with recursive coordinate bisection as the vertex separator.
# ---------------------------------------------------------------------------
def rcb_separator(U, coords, rowptr, colind, n):
    """Geometric vertex separator of the vertex set U (Sec. 2.3, last paragraph).

    Reading of the paper's description: the axis is the one with the largest
    coordinate span (ties to the lowest axis); the two "equal parts" are a
    threshold split at the lower median m of that coordinate, first part =
    {coord <= m} (or {coord < m} if that would leave the second part empty), so
    that grid planes stay whole; the separator is the set of first-part vertices
    with an edge (inside U) to the second part.  Returns (left, middle, right).
    """
    X = coords[U]
    span = X.max(axis=0) - X.min(axis=0)
    d = int(np.argmax(span))
    c = X[:, d]
    h = (len(U) - 1) // 2
    m = np.sort(c, kind="stable")[h]
    first = c <= m
    if first.all():
        first = c < m
    in_second = np.zeros(n, dtype=bool)
    in_second[U[~first]] = True
    F = U[first]
    start = rowptr[F]
    deg = rowptr[F + 1] - start
    owner = np.repeat(np.arange(len(F)), deg)
    within = np.arange(int(deg.sum())) - np.repeat(np.cumsum(deg) - deg, deg)
    nbr = colind[np.repeat(start, deg) + within]
    touches = np.zeros(len(F), dtype=bool)
    hit = in_second[nbr]
    touches[owner[hit]] = True
    return F[~touches], F[touches], U[~first]


def _bfs_levels(root, inU, rowptr, colind):
    """Breadth-first distances from root inside the vertex set inU (a boolean mask):
    dict vertex -> level."""
    lev = {int(root): 0}
    frontier = [int(root)]
    d = 0
    while frontier:
        d += 1
        nxt = []
        for v in frontier:
            for u in colind[rowptr[v]:rowptr[v + 1]]:
                u = int(u)
                if inU[u] and u not in lev:
                    lev[u] = d
                    nxt.append(u)
        frontier = nxt
    return lev


def graph_separator(U, rowptr, colind, n):
    """Vertex separator of U from the graph alone, for inputs without coordinates
    (the paper's Algorithm 2 takes any separator; Sec. 2.3 names a graph partitioner
    as the alternative to the geometric one).  A level structure replaces the
    coordinate of the geometric separator:

    * the components of the graph restricted to U are taken in the order of their
      smallest vertex id; in each, a pseudo-peripheral root is found by the
      George-Liu iteration (start at the smallest id; move to the vertex of the
      last breadth-first level with the smallest degree inside U, ties to the
      smallest id, while that increases the eccentricity), and its breadth-first
      levels, shifted past the levels of the earlier components, are the
      vertices' keys;
    * the split is the threshold split of the geometric separator on these keys:
      m = the key at sorted position floor((|U|-1)/2), first part {key <= m} (or
      {key < m} if that is all of U), separator = first-part vertices with an edge
      inside U to the second part.  Returns (left, middle, right).
    """
    U = np.asarray(U, dtype=np.int64)
    inU = np.zeros(n, dtype=bool)
    inU[U] = True
    deg = {}
    for v in U.tolist():
        nb = colind[rowptr[v]:rowptr[v + 1]]
        deg[v] = int(np.sum(inU[nb] & (nb != v)))
    key = {}
    offset = 0
    for start in sorted(U.tolist()):
        if start in key:
            continue
        root = start
        lev = _bfs_levels(root, inU, rowptr, colind)
        ecc = max(lev.values())
        while True:
            last = [v for v, d in lev.items() if d == ecc]
            x = min(last, key=lambda v: (deg[v], v))
            lx = _bfs_levels(x, inU, rowptr, colind)
            ex = max(lx.values())
            if ex > ecc:
                root, lev, ecc = x, lx, ex
            else:
                break
        for v, d in lev.items():
            key[v] = offset + d
        offset += ecc + 1
    c = np.array([key[v] for v in U.tolist()], dtype=np.int64)
    h = (len(U) - 1) // 2
    m = np.sort(c, kind="stable")[h]
    first = c <= m
    if first.all():
        first = c < m
    in_second = np.zeros(n, dtype=bool)
    in_second[U[~first]] = True
    F = U[first]
    touches = np.array([bool(np.any(in_second[colind[rowptr[v]:rowptr[v + 1]]])) for v in F.tolist()], dtype=bool)
    return F[~touches], F[touches], U[~first]


def nd_order(n, rowptr, colind, coords, levels):
    """Algorithm 2: per-vertex (S, L, R) separator ids for an ND tree of depth ``levels``.

    The root is level 1 and leaves are level ``levels``; levels-1 dissections are
    made.  Boxes of one level are processed in increasing k (their updates never
    touch the same field of a vertex, so the order does not change the result).
    Vertices of the middle set that lie on the boundary keep their pointers.  With
    coords None the separator is the graph one (``graph_separator``), else the
    geometric one (``rcb_separator``).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    S = np.full(n, pack(1, 1), dtype=np.int64)
    Lp = np.zeros(n, dtype=np.int64)
    Rp = np.zeros(n, dtype=np.int64)
    for l in range(1, levels):
        for k in range(1, 2 ** (l - 1) + 1):
            me = pack(l, k)
            I = np.nonzero(S == me)[0]
            B = np.nonzero((Lp == me) | (Rp == me))[0]
            U = np.union1d(I, B)
            if len(U) == 0:
                continue
            if coords is None:
                left, mid, right = graph_separator(U, rowptr, colind, n)
            else:
                left, mid, right = rcb_separator(U, coords, rowptr, colind, n)
            inI = np.zeros(n, dtype=bool)
            inI[I] = True
            a, b = pack(l + 1, 2 * k - 1), pack(l + 1, 2 * k)
            # separator vertices keep S=(l,k); interiors go to the two children
            S[left[inI[left]]] = a
            S[right[inI[right]]] = b
            m_int = mid[inI[mid]]
            Lp[m_int] = a
            Rp[m_int] = b
            for part, child in ((left, a), (right, b)):
                bnd = part[~inI[part]]
                on_left = Lp[bnd] == me
                Lp[bnd[on_left]] = child
                Rp[bnd[~on_left]] = child
    return S, Lp, Rp


# ---------------------------------------------------------------------------
# Cluster hierarchy and symbolic block pattern.
# ---------------------------------------------------------------------------
@dataclass
class Step:
    level: int                       # ND level eliminated at this step
    keys: np.ndarray                 # (nc, 3) int64: S, L, R of each cluster (truncated)
    children: list                   # per cluster: ids of step t-1 clusters (step 1: vertex ids)
    n_elim: int                      # clusters 0..n_elim-1 are eliminated
    blocks: list                     # sorted (i, j), i >= j, pattern before elimination
    elim_nbrs: list                  # per eliminated cluster: sorted neighbour ids
    after: list                      # sorted (i, j), i >= j, among remaining clusters after fill
    nbrs: list                       # per cluster (remaining): sorted neighbour ids after fill
    sparsify: bool
    colour: np.ndarray               # per cluster colour (-1 for eliminated)
    parent: np.ndarray               # per cluster its id at the next step (-1 if eliminated)


def cluster_order(keys):
    """Canonical cluster order: separator level descending, then separator index,
    then left pointer, then right pointer (pointers as (level, index))."""
    return np.lexsort((keys[:, 2], keys[:, 1], idx_of(keys[:, 0]), -lev_of(keys[:, 0])))


def symbolic(n, rowptr, colind, S, Lp, Rp, levels, skip=0):
    """Cluster tree and block pattern for every elimination step (Sec. 2.3, 2.4, 2.7).

    Step t = 1..levels eliminates ND level l = levels - t + 1.  A cluster at step t
    is a set of not-yet-eliminated vertices with equal (S, trunc_l(L), trunc_l(R));
    every separator is then one cluster when eliminated and clusters of one
    separator merge one level of their tree per step.  The pattern is structural:
    a block exists once created.  Elimination of s adds a block for every pair of
    its neighbours; scaling and sparsification create none (Sec. 2.6.1).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    steps = []
    prev_keys = None
    prev_members = None
    cl_of_vertex = None
    prev_after = None
    prev_parent = None
    for t in range(1, levels + 1):
        l = levels - t + 1
        if t == 1:
            raw = np.stack([S, truncate(Lp, l), truncate(Rp, l)], axis=1)
            uniq, inv = np.unique(raw, axis=0, return_inverse=True)
            order = cluster_order(uniq)
            rank = np.empty(len(order), dtype=np.int64)
            rank[order] = np.arange(len(order))
            keys = uniq[order]
            cl_of_vertex = rank[inv.ravel()]
            by_cluster = np.argsort(cl_of_vertex, kind="stable")
            bounds = np.cumsum(np.bincount(cl_of_vertex, minlength=len(keys)))[:-1]
            children = [list(x) for x in np.split(by_cluster, bounds)]
            # block pattern from the graph of A
            rows = np.repeat(np.arange(n), rowptr[1:] - rowptr[:-1])
            ci, cj = cl_of_vertex[rows], cl_of_vertex[colind]
            pairs = set(zip(np.maximum(ci, cj).tolist(), np.minimum(ci, cj).tolist()))
        else:
            alive = np.nonzero(prev_parent >= 0)[0]
            keys = steps[-1].next_keys
            children = [[] for _ in range(len(keys))]
            for c in alive:
                children[prev_parent[c]].append(int(c))
            pairs = set()
            for (i, j) in prev_after:
                a, b = prev_parent[i], prev_parent[j]
                pairs.add((max(a, b), min(a, b)))
        nc = len(keys)
        n_elim = int(np.sum(lev_of(keys[:, 0]) == l))
        blocks = sorted(pairs)
        adj = [set() for _ in range(nc)]
        for (i, j) in blocks:
            if i != j:
                adj[i].add(j)
                adj[j].add(i)
        elim_nbrs = []
        fill = set(p for p in pairs if p[0] >= n_elim and p[1] >= n_elim)
        for s in range(n_elim):
            nb = sorted(adj[s])
            assert all(x >= n_elim for x in nb), "same-level separators must not touch"
            elim_nbrs.append(nb)
            for a in range(len(nb)):
                for b in range(a + 1):
                    fill.add((nb[a], nb[b]))
        after = sorted(fill)
        nbrs = [[] for _ in range(nc)]
        for (i, j) in after:
            if i != j:
                nbrs[i].append(j)
                nbrs[j].append(i)
        nbrs = [sorted(x) for x in nbrs]
        sparsify = (t > skip) and (l > 1)
        colour = np.full(nc, -1, dtype=np.int64)
        if sparsify:
            # greedy colouring in ascending cluster id: smallest colour not used
            # by an already coloured neighbour
            for p in range(n_elim, nc):
                used = {colour[q] for q in nbrs[p] if colour[q] >= 0}
                c = 0
                while c in used:
                    c += 1
                colour[p] = c
        # parents at the next step
        parent = np.full(nc, -1, dtype=np.int64)
        next_keys = None
        if l > 1:
            rem = np.arange(n_elim, nc)
            nk = np.stack([keys[rem, 0], truncate(keys[rem, 1], l - 1), truncate(keys[rem, 2], l - 1)], axis=1)
            uniq, inv = np.unique(nk, axis=0, return_inverse=True)
            order = cluster_order(uniq)
            rank = np.empty(len(order), dtype=np.int64)
            rank[order] = np.arange(len(order))
            parent[rem] = rank[inv.ravel()]
            next_keys = uniq[order]
        st = Step(level=l, keys=keys, children=children, n_elim=n_elim, blocks=blocks,
                  elim_nbrs=elim_nbrs, after=after, nbrs=nbrs, sparsify=sparsify,
                  colour=colour, parent=parent)
        st.next_keys = next_keys
        steps.append(st)
        prev_after, prev_parent = after, parent
    return steps


# ---------------------------------------------------------------------------
# Column-pivoted QR, truncated by the ratio rule.
# ---------------------------------------------------------------------------
def householder(x):
    """Reflector H = I - tau v v^T with v[0] = 1 and H x = beta e_1 (LAPACK dlarfg
    convention: beta = -sign(x_0) ||x||; tau = 0 when x[1:] is zero)."""
    alpha = x[0]
    xn = np.linalg.norm(x[1:])
    v = np.zeros_like(x)
    v[0] = 1.0
    if xn == 0.0:
        return v, 0.0, alpha
    beta = -np.copysign(np.hypot(alpha, xn), alpha)
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def cpqr(A, eps, tie="original"):
    """Truncated column-pivoted Householder QR of A (m x n) (Sec. 2.6.1, Sec. 4 intro).

    At step j the norms of the trailing columns A[j:, j:] are recomputed; the pivot
    is, among the columns whose norm is within TIE_RTOL of the largest, the one
    with the smallest original column index (tie="original") or the one at the
    smallest current position (tie="position").  Ties are a reading: the paper's
    routine, geqp3, does not define them as part of the method.  The rank r
    is the number of leading steps with |R_jj| >= eps |R_00| (r = 0 when R_00 = 0,
    r = min(m, n) when no step fails).  Returns (r, V, tau, W, perm) where V (m x r)
    holds the reflectors (unit first entry, zero above), and W = (Q^T A)[:r, :],
    i.e. R[:r, :] with the column permutation undone.
    """
    if tie not in TIE_RULES:
        raise ValueError(f"tie must be one of {TIE_RULES}")
    A = np.array(A, dtype=np.float64, copy=True)
    m, n = A.shape
    perm = np.arange(n)
    k = min(m, n)
    V = np.zeros((m, k))
    taus = np.zeros(k)
    r = k
    r00 = 0.0
    for j in range(k):
        norms = np.sqrt(np.sum(A[j:, j:] ** 2, axis=0))
        cmax = norms.max()
        cand = np.nonzero(norms >= cmax * (1.0 - TIE_RTOL))[0]
        if tie == "original":
            piv = j + int(cand[np.argmin(perm[j + cand])])
        else:
            piv = j + int(cand[0])
        if j == 0:
            r00 = norms[piv - j]
            if r00 == 0.0:
                r = 0
                break
        if norms[piv - j] < eps * r00:
            r = j
            break
        if piv != j:
            A[:, [j, piv]] = A[:, [piv, j]]
            perm[[j, piv]] = perm[[piv, j]]
        v, tau, beta = householder(A[j:, j].copy())
        A[j:, j + 1:] -= tau * np.outer(v, v @ A[j:, j + 1:])
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        V[j:, j] = v
        taus[j] = tau
    W = np.zeros((r, n))
    W[:, perm] = np.triu(A[:r, :])
    return r, V[:, :r].copy(), taus[:r].copy(), W, perm


def apply_qt(V, tau, x):
    """x <- Q^T x with Q = H_0 H_1 ... H_{r-1}: reflectors applied in increasing order."""
    for j in range(V.shape[1]):
        v = V[:, j]
        x -= tau[j] * np.outer(v, v @ x)
    return x


def apply_q(V, tau, x):
    """x <- Q x: reflectors applied in decreasing order."""
    for j in reversed(range(V.shape[1])):
        v = V[:, j]
        x -= tau[j] * np.outer(v, v @ x)
    return x


# ---------------------------------------------------------------------------
# Algorithm 3 (OrthS).
# ---------------------------------------------------------------------------
@dataclass
class StepFactor:
    E: list = field(default_factory=list)   # (slots_s, L_s, [(slots_n, G_ns)])
    S: list = field(default_factory=list)   # (slots_p, L_p)
    Q: list = field(default_factory=list)   # (slots_p, V, tau)
    I: list = field(default_factory=list)   # (slots_p, perm, r, T_cf, L_f, G_cf): interpolative
    ranks: dict = field(default_factory=dict)   # cluster id -> kept size after sparsification
    sizes: list = field(default_factory=list)   # cluster sizes before elimination


@dataclass
class Factor:
    n: int
    steps: list
    stats: dict


class Analysis:
    """Ordering, clusters and symbolic pattern of one matrix pattern (``spand_analyze``)."""

    def __init__(self, n, rowptr, colind, coords, levels, skip=0):
        self.n = n
        self.rowptr = np.asarray(rowptr, dtype=np.int64)
        self.colind = np.asarray(colind, dtype=np.int64)
        self.coords = None if coords is None else np.asarray(coords, dtype=np.float64).reshape(n, -1)
        self.levels = levels
        self.skip = skip
        self.S, self.L, self.R = nd_order(n, self.rowptr, self.colind, self.coords, levels)
        self.steps = symbolic(n, self.rowptr, self.colind, self.S, self.L, self.R, levels, skip)


def nd_permutation(an: Analysis):
    """The elimination order of the vertices under Algorithm 2 + the cluster tree: a
    vertex goes at the step that eliminates its separator's level, inside the
    cluster its step-1 cluster has merged into by then; ties by vertex id."""
    cl = np.empty(an.n, dtype=np.int64)
    for c, ch in enumerate(an.steps[0].children):
        cl[ch] = c
    up = [np.arange(len(an.steps[0].keys))]
    for st in an.steps[:-1]:
        prev = up[-1]
        up.append(np.where(prev >= 0, st.parent[np.maximum(prev, 0)], -1))
    t = an.levels - lev_of(an.S)   # 0-based step of each vertex
    c = np.array([up[t[v]][cl[v]] for v in range(an.n)], dtype=np.int64)
    return np.lexsort((np.arange(an.n), c, t))


def _get(blocks, i, j):
    if i >= j:
        return blocks[(i, j)]
    return blocks[(j, i)].T


def factor(an: Analysis, values, tol, tie="original", on_sparsify=None, variant="OrthS"):
    """Algorithm 3: returns a Factor, or raises NotSPD(step, cluster, phase).

    ``tie`` selects the CPQR tie rule (see ``cpqr``).  ``on_sparsify``, when given,
    is called as on_sparsify(t, p, nbrs, sizes, blocks, Apn, result) right before the
    sparsification of interface p at step t writes its result back: ``blocks`` is the
    live trailing matrix (scaled, so A_pp = I), ``Apn`` the gathered row block and
    ``result`` the tuple returned by ``cpqr``.  It lets tests inspect the step in
    context; it must not modify anything.

    ``variant`` is one of VARIANTS.  "In" skips the block scaling and sparsifies by
    the interpolative transformation of Sec. 2.6.2; "InS" scales first, then does
    the same.  For those the hook receives A_np (not A_pn), the ``cpqr`` result of
    A_np, and a keyword ``interp`` = dict(c, f, T, Cff, Ccf) of the congruence.
    The phase of a failed Cholesky of C_ff is "sparsify".
    """
    if variant not in VARIANTS:
        raise ValueError(f"variant must be one of {VARIANTS}")
    n = an.n
    steps = an.steps
    values = np.asarray(values, dtype=np.float64)
    out = []
    stats = {"s_top": 0, "m_F": 0, "ranks": []}
    # step-1 clusters: vertices in ascending id; slots are vertex ids
    slots = [np.array(ch, dtype=np.int64) for ch in steps[0].children]
    sizes = [len(x) for x in slots]
    pos = np.empty(n, dtype=np.int64)
    cl = np.empty(n, dtype=np.int64)
    for c, sl in enumerate(slots):
        pos[sl] = np.arange(len(sl))
        cl[sl] = c
    blocks = {(i, j): np.zeros((sizes[i], sizes[j])) for (i, j) in steps[0].blocks}
    rows = np.repeat(np.arange(n), an.rowptr[1:] - an.rowptr[:-1])
    ci, cj = cl[rows], cl[an.colind]
    keep = np.nonzero(ci >= cj)[0]
    order = keep[np.lexsort((cj[keep], ci[keep]))]
    bi, bj = ci[order], cj[order]
    cut = np.nonzero((np.diff(bi) != 0) | (np.diff(bj) != 0))[0] + 1
    for grp in np.split(order, cut):
        if len(grp):
            blocks[(ci[grp[0]], cj[grp[0]])][pos[rows[grp]], pos[an.colind[grp]]] = values[grp]
    m_F = 0
    for t, st in enumerate(steps, start=1):
        sf = StepFactor(sizes=list(sizes))
        if st.level == 1:
            stats["s_top"] = int(sum(sizes[s] for s in range(st.n_elim)))
        # -- elimination of every level-l cluster (Sec. 2.4) --
        for s in range(st.n_elim):
            try:
                Ls = np.linalg.cholesky(blocks[(s, s)])
            except np.linalg.LinAlgError:
                raise NotSPD(t, s, "elim")
            nb = st.elim_nbrs[s]
            G = [solve_triangular(Ls, blocks[(q, s)].T, lower=True).T for q in nb]   # A_ns L_s^-T
            for a in range(len(nb)):
                for b in range(a + 1):
                    key = (nb[a], nb[b])
                    upd = G[a] @ G[b].T
                    if key in blocks:
                        blocks[key] = blocks[key] - upd
                    else:
                        blocks[key] = -upd
            sf.E.append((slots[s].copy(), Ls, [(slots[q].copy(), g) for q, g in zip(nb, G)]))
            m_F += sizes[s] * (sizes[s] + 1) // 2 + sizes[s] * sum(sizes[q] for q in nb)
            for q in nb:
                del blocks[(q, s)]
            del blocks[(s, s)]
        nc = len(st.keys)
        rem = range(st.n_elim, nc)
        if st.sparsify and variant != "OrthS":
            if variant == "InS":
                _scale(t, rem, st, blocks, sizes, slots, sf)
            m_F += sum(sizes[p] * (sizes[p] + 1) // 2 for p in rem) if variant == "InS" else 0
            for p in sorted(rem, key=lambda p: (st.colour[p], p)):
                m_F += _interpolative(t, p, st, blocks, sizes, slots, sf, tol, tie, on_sparsify)
        elif st.sparsify:
            # -- block scaling of every interface (Sec. 2.5) --
            Lp = {}
            for p in rem:
                try:
                    Lp[p] = np.linalg.cholesky(blocks[(p, p)])
                except np.linalg.LinAlgError:
                    raise NotSPD(t, p, "scale")
                sf.S.append((slots[p].copy(), Lp[p]))
                m_F += sizes[p] * (sizes[p] + 1) // 2
            for (i, j) in st.after:
                if i != j:
                    X = solve_triangular(Lp[i], blocks[(i, j)], lower=True)          # L_i^-1 A_ij
                    blocks[(i, j)] = solve_triangular(Lp[j], X.T, lower=True).T      # ... L_j^-T
            for p in rem:
                blocks[(p, p)] = np.eye(sizes[p])
            # -- orthogonal sparsification, in (colour, id) order (Sec. 2.6.1) --
            order = sorted(rem, key=lambda p: (st.colour[p], p))
            for p in order:
                nb = st.nbrs[p]
                # no coupled dofs (no neighbour, or all neighbours reduced to
                # zero size): p is left as it is, with A_pp = I after scaling
                if sizes[p] == 0 or sum(sizes[q] for q in nb) == 0:
                    sf.ranks[p] = sizes[p]
                    continue
                Apn = np.hstack([_get(blocks, p, q) for q in nb])
                res = cpqr(Apn, tol, tie)
                if on_sparsify is not None:
                    on_sparsify(t, p, nb, list(sizes), blocks, Apn, res)
                r, V, tau, W, _ = res
                col = 0
                for q in nb:
                    wq = W[:, col:col + sizes[q]]
                    col += sizes[q]
                    if p >= q:
                        blocks[(p, q)] = wq
                    else:
                        blocks[(q, p)] = wq.T
                blocks[(p, p)] = np.eye(r)
                sf.Q.append((slots[p].copy(), V, tau))
                m_F += int(sum(sizes[p] - j for j in range(r))) + r
                sizes[p] = r
                slots[p] = slots[p][:r].copy()
                sf.ranks[p] = r
        out.append(sf)
        # -- merge one level up the cluster trees (Sec. 2.7) --
        if st.level > 1:
            nxt = steps[t]
            new_slots = []
            new_sizes = []
            for ch in nxt.children:
                sl = np.concatenate([slots[c] for c in ch]) if ch else np.zeros(0, np.int64)
                new_slots.append(sl)
                new_sizes.append(len(sl))
            new_blocks = {}
            for (I, J) in nxt.blocks:
                Bm = np.zeros((new_sizes[I], new_sizes[J]))
                ro = 0
                for i in nxt.children[I]:
                    co = 0
                    for j in nxt.children[J]:
                        a, b = max(i, j), min(i, j)
                        if (a, b) in blocks:
                            Bm[ro:ro + sizes[i], co:co + sizes[j]] = _get(blocks, i, j)
                        co += sizes[j]
                    ro += sizes[i]
                new_blocks[(I, J)] = Bm
            blocks, slots, sizes = new_blocks, new_slots, new_sizes
    stats["m_F"] = int(m_F)
    stats["ranks"] = [sf.ranks for sf in out]
    return Factor(n=n, steps=out, stats=stats)


def _scale(t, rem, st, blocks, sizes, slots, sf):
    """Block scaling of the interfaces ``rem`` (Sec. 2.5): A_pp = L_p L_p^T,
    A_pq <- L_p^-1 A_pq L_q^-T, A_pp <- I."""
    Lp = {}
    for p in rem:
        try:
            Lp[p] = np.linalg.cholesky(blocks[(p, p)])
        except np.linalg.LinAlgError:
            raise NotSPD(t, p, "scale")
        sf.S.append((slots[p].copy(), Lp[p]))
    for (i, j) in st.after:
        if i != j:
            X = solve_triangular(Lp[i], blocks[(i, j)], lower=True)
            blocks[(i, j)] = solve_triangular(Lp[j], X.T, lower=True).T
    for p in rem:
        blocks[(p, p)] = np.eye(sizes[p])


def _interpolative(t, p, st, blocks, sizes, slots, sf, tol, tie, on_sparsify):
    """Interpolative sparsification of interface p (Sec. 2.6.2); returns the entries
    it stores.

    The truncated CPQR of A_np (pivoting over the dofs of p) splits p into the
    coarse dofs c (the r pivot columns, in pivot order) and the fine dofs f (the
    rest), and gives T_cf = R_11^-1 R_12, so that A_nf ~ A_nc T_cf.  The congruence
    with T_p = [I_f 0; -T_cf I_c] leaves

        C_ff = A_ff - A_fc T_cf - T_cf^T A_cf + T_cf^T A_cc T_cf,
        C_cf = A_cf - A_cc T_cf,

    and an f-n coupling A_nf - A_nc T_cf that is dropped.  f, now coupled to c
    only, is eliminated (Sec. 2.4 on the pair f, c): C_ff = L_f L_f^T,
    G_cf = C_cf L_f^-T, A_cc <- A_cc - G_cf G_cf^T.  p keeps the dofs c, whose rows
    of A_pn are A_cn unchanged.  Nothing is done when p has no coupled dofs or no
    fine dof (r = |p|).
    """
    nb = st.nbrs[p]
    if sizes[p] == 0 or sum(sizes[q] for q in nb) == 0:
        sf.ranks[p] = sizes[p]
        return 0
    Anp = np.vstack([_get(blocks, q, p) for q in nb])
    res = cpqr(Anp, tol, tie)
    r, _, _, W, perm = res
    if r == sizes[p]:
        if on_sparsify is not None:
            on_sparsify(t, p, nb, list(sizes), blocks, Anp, res, interp=None)
        sf.ranks[p] = r
        return 0
    c, f = perm[:r], perm[r:]
    R = W[:, perm]                                         # R_11 | R_12, pivot order
    T = solve_triangular(R[:, :r], R[:, r:], lower=False)  # T_cf
    App = blocks[(p, p)]
    Acc, Acf, Aff = App[np.ix_(c, c)], App[np.ix_(c, f)], App[np.ix_(f, f)]
    Cff = Aff - Acf.T @ T - T.T @ Acf + T.T @ Acc @ T
    Ccf = Acf - Acc @ T
    if on_sparsify is not None:
        on_sparsify(t, p, nb, list(sizes), blocks, Anp, res,
                    interp=dict(c=c.copy(), f=f.copy(), T=T, Cff=Cff, Ccf=Ccf))
    try:
        Lf = np.linalg.cholesky(Cff)
    except np.linalg.LinAlgError:
        raise NotSPD(t, p, "sparsify")
    G = solve_triangular(Lf, Ccf.T, lower=True).T          # C_cf L_f^-T
    blocks[(p, p)] = Acc - G @ G.T
    for q in nb:
        if p >= q:
            blocks[(p, q)] = blocks[(p, q)][c, :]
        else:
            blocks[(q, p)] = blocks[(q, p)][:, c]
    sf.I.append((slots[p].copy(), perm.copy(), r, T, Lf, G))
    nf = sizes[p] - r
    sizes[p] = r
    slots[p] = slots[p][c].copy()
    sf.ranks[p] = r
    return r * nf + nf * (nf + 1) // 2 + r * nf


def apply(fac: Factor, r):
    """z = M M^T r = F^T F r with F = M^T (Sec. 2.8): forward sweep over the steps
    applying E_s, S_p, Q_p^T; the trailing diagonal is the identity; backward sweep
    applying Q_p, S_p^T, E_s^T in reverse order."""
    x = np.array(r, dtype=np.float64, copy=True)
    if x.ndim == 1:
        x = x[:, None]
    for sf in fac.steps:
        for (ss, Ls, nbl) in sf.E:
            xs = solve_triangular(Ls, x[ss], lower=True)
            x[ss] = xs
            for (sn, G) in nbl:
                x[sn] -= G @ xs
        for (sp, Lp) in sf.S:
            x[sp] = solve_triangular(Lp, x[sp], lower=True)
        for (sp, V, tau) in sf.Q:
            x[sp] = apply_qt(V, tau, x[sp])
        for (sp, perm, k, T, Lf, G) in sf.I:
            # T_p^T, then the elimination of f: y_f = L_f^-1 (x_f - T^T x_c),
            # y_c = x_c - G y_f
            sc, sfn = sp[perm[:k]], sp[perm[k:]]
            yf = solve_triangular(Lf, x[sfn] - T.T @ x[sc], lower=True)
            x[sc] = x[sc] - G @ yf
            x[sfn] = yf
    for sf in reversed(fac.steps):
        for (sp, perm, k, T, Lf, G) in sf.I:
            # the elimination of f backward, then T_p: y_f = L_f^-T (y_f - G^T y_c),
            # x_c = y_c - T y_f
            sc, sfn = sp[perm[:k]], sp[perm[k:]]
            yf = solve_triangular(Lf.T, x[sfn] - G.T @ x[sc], lower=False)
            x[sc] = x[sc] - T @ yf
            x[sfn] = yf
        for (sp, V, tau) in sf.Q:
            x[sp] = apply_q(V, tau, x[sp])
        for (sp, Lp) in sf.S:
            x[sp] = solve_triangular(Lp.T, x[sp], lower=False)
        for (ss, Ls, nbl) in sf.E:
            y = x[ss].copy()
            for (sn, G) in nbl:
                y -= G.T @ x[sn]
            x[ss] = solve_triangular(Ls.T, y, lower=False)
    return x


class Breakdown(Exception):
    """PCG produced a non-finite residual norm (column, iteration)."""

    def __init__(self, column, iteration):
        super().__init__(f"PCG breakdown in column {column} at iteration {iteration}")
        self.column, self.iteration = column, iteration


def pcg(A, b, precond, rtol=1e-12, maxit=500):
    """Preconditioned CG (Hestenes-Stiefel), x0 = 0, one right-hand side per column.

    The target is the true residual, ||b - A x|| <= rtol ||b|| (Sec. 4).  The
    recursive residual r is the cheap test: when it passes, the true residual is
    formed; if that also passes the column stops, otherwise r is replaced by the
    true residual and the iteration goes on (residual replacement).  The iteration
    count is the number of updates of x.  A non-finite residual norm raises
    Breakdown.  Returns (x, iters, true relres).
    """
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[:, None]
    n, k = b.shape
    X = np.zeros((n, k))
    iters = np.zeros(k, dtype=np.int64)
    relres = np.zeros(k)
    for c in range(k):
        bc = b[:, c]
        nb = np.linalg.norm(bc)
        x = np.zeros(n)
        if nb == 0.0:
            continue
        r = bc.copy()
        z = precond(r[:, None])[:, 0]
        p = z.copy()
        rz = r @ z
        it = 0
        while it < maxit:
            q = A @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            it += 1
            rn = np.linalg.norm(r)
            if not np.isfinite(rn):
                raise Breakdown(c, it)
            if rn <= rtol * nb:
                rt = bc - A @ x
                if np.linalg.norm(rt) <= rtol * nb:
                    break
                r = rt
            z = precond(r[:, None])[:, 0]
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        X[:, c] = x
        iters[c] = it
        relres[c] = np.linalg.norm(bc - A @ x) / nb
    return X, iters, relres


def solve(problem, b, levels, tol, skip=0, rtol=1e-12, maxit=500, variant="OrthS"):
    """Convenience: analyze + factor + PCG on a gridgen problem."""
    an = Analysis(problem.n, problem.rowptr, problem.colind, problem.coords, levels, skip)
    fac = factor(an, problem.values, tol, variant=variant)
    A = problem.scipy()
    x, it, rr = pcg(A, b, lambda r: apply(fac, r), rtol, maxit)
    return an, fac, x, it, rr
