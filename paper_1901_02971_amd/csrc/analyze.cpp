// Host-side analysis: Algorithm 2 (modified nested dissection ordering and
// clustering, Sec. 2.3) with a recursive-coordinate-bisection vertex separator (or,
// without coordinates, a breadth-first level-structure separator),
// the cluster hierarchy of every separator (Sec. 2.3, 2.7) and the structural
// block pattern of the trailing matrix with the fill of block elimination
// (Sec. 2.4).  Integer work only; never touches the GPU.
#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>

#include "spand_internal.h"

namespace spand {
namespace {

// Geometric vertex separator of U (Sec. 2.3, last paragraph; Sec. 4.1.1): widest
// coordinate axis (lowest axis on ties); threshold at the lower median m of that
// coordinate, first part {c <= m} (or {c < m} when that is all of U); the middle
// set is the first-part vertices adjacent (inside U) to the second part.
// side[v] receives 0 (left), 1 (middle) or 2 (right) for v in U.
void rcb_split(const Analysis& an, const std::vector<int32_t>& U, std::vector<int32_t>& mark,
               int32_t stamp, std::vector<uint8_t>& side) {
  const int d = an.dim;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t v : U)
    for (int a = 0; a < d; ++a) {
      double c = an.coords[size_t(v) * d + a];
      lo[a] = std::min(lo[a], c);
      hi[a] = std::max(hi[a], c);
    }
  int axis = 0;
  double best = hi[0] - lo[0];
  for (int a = 1; a < d; ++a)
    if (hi[a] - lo[a] > best) {
      best = hi[a] - lo[a];
      axis = a;
    }
  std::vector<double> c(U.size());
  for (size_t q = 0; q < U.size(); ++q) c[q] = an.coords[size_t(U[q]) * d + axis];
  std::vector<double> tmp(c);
  size_t h = (U.size() - 1) / 2;
  std::nth_element(tmp.begin(), tmp.begin() + h, tmp.end());
  const double m = tmp[h];
  bool all_first = true;
  for (double x : c)
    if (!(x <= m)) {
      all_first = false;
      break;
    }
  // second part gets the stamp in `mark`
  for (size_t q = 0; q < U.size(); ++q) {
    bool first = all_first ? (c[q] < m) : (c[q] <= m);
    side[q] = first ? 0 : 2;
    if (!first) mark[U[q]] = stamp;
  }
  for (size_t q = 0; q < U.size(); ++q) {
    if (side[q] != 0) continue;
    int32_t v = U[q];
    for (int64_t e = an.rowptr[v]; e < an.rowptr[v + 1]; ++e)
      if (mark[an.colind[e]] == stamp) {
        side[q] = 1;
        break;
      }
  }
}

// Per-vertex scratch of the graph separator, stamped so that nothing is cleared
// between calls.
struct GraphScratch {
  std::vector<int32_t> in_u;   // == u_stamp: v is in the current U
  std::vector<int32_t> seen;   // == seen_stamp: v reached by the current breadth-first search
  std::vector<int32_t> dist;   // its level in that search
  std::vector<int64_t> key;    // final level key of v in U
  std::vector<int32_t> deg;    // degree of v inside U
  int32_t u_stamp = 0, seen_stamp = 0;
  explicit GraphScratch(int64_t n) : in_u(n, -1), seen(n, -1), dist(n, 0), key(n, -1), deg(n, 0) {}
};

// Breadth-first search from root inside U; `order` receives the vertices reached in
// search order (so by level), dist their levels.  Returns the eccentricity.
int32_t bfs_in_u(const Analysis& an, GraphScratch& g, int32_t root, std::vector<int32_t>& order) {
  ++g.seen_stamp;
  order.clear();
  order.push_back(root);
  g.seen[root] = g.seen_stamp;
  g.dist[root] = 0;
  int32_t ecc = 0;
  for (size_t h = 0; h < order.size(); ++h) {
    const int32_t v = order[h];
    for (int64_t e = an.rowptr[v]; e < an.rowptr[v + 1]; ++e) {
      const int32_t u = an.colind[e];
      if (g.in_u[u] != g.u_stamp || g.seen[u] == g.seen_stamp) continue;
      g.seen[u] = g.seen_stamp;
      g.dist[u] = g.dist[v] + 1;
      ecc = std::max(ecc, g.dist[u]);
      order.push_back(u);
    }
  }
  return ecc;
}

// Vertex separator of U from the graph alone, for inputs without coordinates: a
// breadth-first level structure gives every vertex a key, and the threshold split of
// the geometric separator is taken on the keys.  The components of the graph inside
// U are taken in the order of their smallest vertex id; each gets a pseudo-peripheral
// root by the George-Liu iteration (start at the smallest id; go to the last-level
// vertex of smallest degree inside U, ties to the smallest id, while that raises the
// eccentricity), and its levels from that root, shifted past the keys of the earlier
// components.  Then m = the key at sorted position floor((|U|-1)/2), first part
// {key <= m} (or {key < m} when that is all of U), middle = first-part vertices
// adjacent (inside U) to the second part.  side[q] as in rcb_split.
void graph_split(const Analysis& an, const std::vector<int32_t>& U, std::vector<int32_t>& mark, int32_t stamp,
                 std::vector<uint8_t>& side, GraphScratch& g) {
  ++g.u_stamp;
  for (int32_t v : U) g.in_u[v] = g.u_stamp;
  for (int32_t v : U) {
    int32_t d = 0;
    for (int64_t e = an.rowptr[v]; e < an.rowptr[v + 1]; ++e) {
      const int32_t u = an.colind[e];
      if (u != v && g.in_u[u] == g.u_stamp) ++d;
    }
    g.deg[v] = d;
    g.key[v] = -1;
  }
  std::vector<int32_t> byid(U);
  std::sort(byid.begin(), byid.end());
  std::vector<int32_t> order, trial;
  int64_t offset = 0;
  for (int32_t start : byid) {
    if (g.key[start] >= 0) continue;
    int32_t ecc = bfs_in_u(an, g, start, order);
    for (;;) {
      int32_t x = -1;
      for (size_t h = order.size(); h-- > 0;) {  // the last level is at the end of the search order
        const int32_t v = order[h];
        if (g.dist[v] != ecc) break;
        if (x < 0 || g.deg[v] < g.deg[x] || (g.deg[v] == g.deg[x] && v < x)) x = v;
      }
      const int32_t ex = bfs_in_u(an, g, x, trial);
      if (ex > ecc) {
        ecc = ex;
        order.swap(trial);
      } else {
        // the accepted search is `order`, whose levels were overwritten by the trial:
        // search again from its root (order[0]) to restore them
        const int32_t root = order[0];
        ecc = bfs_in_u(an, g, root, order);
        break;
      }
    }
    for (int32_t v : order) g.key[v] = offset + g.dist[v];
    offset += int64_t(ecc) + 1;
  }
  std::vector<int64_t> c(U.size());
  for (size_t q = 0; q < U.size(); ++q) c[q] = g.key[U[q]];
  std::vector<int64_t> tmp(c);
  const size_t h = (U.size() - 1) / 2;
  std::nth_element(tmp.begin(), tmp.begin() + h, tmp.end());
  const int64_t m = tmp[h];
  bool all_first = true;
  for (int64_t x : c)
    if (!(x <= m)) {
      all_first = false;
      break;
    }
  for (size_t q = 0; q < U.size(); ++q) {
    const bool first = all_first ? (c[q] < m) : (c[q] <= m);
    side[q] = first ? 0 : 2;
    if (!first) mark[U[q]] = stamp;
  }
  for (size_t q = 0; q < U.size(); ++q) {
    if (side[q] != 0) continue;
    const int32_t v = U[q];
    for (int64_t e = an.rowptr[v]; e < an.rowptr[v + 1]; ++e)
      if (mark[an.colind[e]] == stamp) {
        side[q] = 1;
        break;
      }
  }
}

// Algorithm 2: fills S, L, R.
void order_and_cluster(Analysis& an) {
  const int64_t n = an.n;
  an.S.assign(n, sep_pack(1, 1));
  an.L.assign(n, 0);
  an.R.assign(n, 0);
  std::vector<int32_t> mark(n, -1);
  int32_t stamp = 0;
  std::unique_ptr<GraphScratch> gs;
  if (an.dim == 0) gs.reset(new GraphScratch(n));
  for (int32_t l = 1; l < an.levels; ++l) {
    const int64_t nbox = int64_t(1) << (l - 1);
    // Bucket interiors (S at level l) and boundaries (L or R at level l) by box.
    // Updates made while processing one box never change another box's bucket
    // membership at the same level, so pre-bucketing equals the literal loop.
    std::vector<int64_t> iptr(nbox + 2, 0), bptr(nbox + 2, 0);
    for (int64_t v = 0; v < n; ++v) {
      if (sep_level(an.S[v]) == l) iptr[sep_index(an.S[v]) + 1]++;
      if (sep_level(an.L[v]) == l) bptr[sep_index(an.L[v]) + 1]++;
      if (sep_level(an.R[v]) == l) bptr[sep_index(an.R[v]) + 1]++;
    }
    for (int64_t k = 1; k <= nbox + 1; ++k) {
      iptr[k] += iptr[k - 1];
      bptr[k] += bptr[k - 1];
    }
    std::vector<int32_t> ilist(iptr[nbox + 1]), blist(bptr[nbox + 1]);
    {
      std::vector<int64_t> ic(iptr.begin(), iptr.end()), bc(bptr.begin(), bptr.end());
      for (int64_t v = 0; v < n; ++v) {
        if (sep_level(an.S[v]) == l) ilist[ic[sep_index(an.S[v])]++] = int32_t(v);
        if (sep_level(an.L[v]) == l) blist[bc[sep_index(an.L[v])]++] = int32_t(v);
        if (sep_level(an.R[v]) == l) blist[bc[sep_index(an.R[v])]++] = int32_t(v);
      }
    }
    std::vector<int32_t> U;
    std::vector<uint8_t> side;
    for (int64_t k = 1; k <= nbox; ++k) {
      const int64_t me = sep_pack(l, k);
      // box k (1-based) owns entries [ptr[k], ptr[k+1])
      const int64_t ni = iptr[k + 1] - iptr[k], nb = bptr[k + 1] - bptr[k];
      if (ni + nb == 0) continue;
      U.assign(ilist.begin() + iptr[k], ilist.begin() + iptr[k + 1]);
      U.insert(U.end(), blist.begin() + bptr[k], blist.begin() + bptr[k + 1]);
      side.assign(U.size(), 0);
      if (gs)
        graph_split(an, U, mark, stamp++, side, *gs);
      else
        rcb_split(an, U, mark, stamp++, side);
      const int64_t a = sep_pack(l + 1, 2 * k - 1), b = sep_pack(l + 1, 2 * k);
      for (size_t q = 0; q < U.size(); ++q) {
        const int32_t v = U[q];
        const bool interior = int64_t(q) < ni;
        if (interior) {
          if (side[q] == 0) an.S[v] = a;
          else if (side[q] == 2) an.S[v] = b;
          else {  // separator vertex: keeps S = (l,k), points to both children
            an.L[v] = a;
            an.R[v] = b;
          }
        } else if (side[q] != 1) {  // boundary vertex left/right of the cut
          const int64_t child = side[q] == 0 ? a : b;
          if (an.L[v] == me) an.L[v] = child;
          else an.R[v] = child;
        }
      }
    }
  }
}

// Canonical cluster order on (S, L, R) keys.
bool key_less(const int64_t* x, const int64_t* y) {
  if (sep_level(x[0]) != sep_level(y[0])) return sep_level(x[0]) > sep_level(y[0]);
  if (sep_index(x[0]) != sep_index(y[0])) return sep_index(x[0]) < sep_index(y[0]);
  if (x[1] != y[1]) return x[1] < y[1];
  return x[2] < y[2];
}
bool key_eq(const int64_t* x, const int64_t* y) { return x[0] == y[0] && x[1] == y[1] && x[2] == y[2]; }

// Sorts the m keys (3 each) of `raw`, returning the distinct keys in canonical
// order and, for every input, its rank among them.
void rank_keys(const std::vector<int64_t>& raw, std::vector<int64_t>& uniq, std::vector<int32_t>& rank) {
  const size_t m = raw.size() / 3;
  std::vector<int64_t> ord(m);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    const int64_t* x = &raw[3 * a];
    const int64_t* y = &raw[3 * b];
    if (key_less(x, y)) return true;
    if (key_less(y, x)) return false;
    return a < b;
  });
  uniq.clear();
  rank.assign(m, -1);
  for (size_t q = 0; q < m; ++q) {
    const int64_t* x = &raw[3 * ord[q]];
    if (uniq.empty() || !key_eq(&uniq[uniq.size() - 3], x)) uniq.insert(uniq.end(), x, x + 3);
    rank[ord[q]] = int32_t(uniq.size() / 3 - 1);
  }
}

void sort_unique(std::vector<uint64_t>& v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

// Symbolic factorization over all steps.
std::string symbolic(Analysis& an) {
  const int64_t n = an.n;
  const int32_t Lv = an.levels;
  an.steps.clear();
  an.steps.resize(Lv);
  std::vector<int32_t> cl_of_vertex(n);
  for (int32_t t = 1; t <= Lv; ++t) {
    SymStep& st = an.steps[t - 1];
    const int32_t l = Lv - t + 1;
    st.level = l;
    if (t == 1) {
      std::vector<int64_t> raw(3 * n);
      for (int64_t v = 0; v < n; ++v) {
        raw[3 * v] = an.S[v];
        raw[3 * v + 1] = sep_truncate(an.L[v], l);
        raw[3 * v + 2] = sep_truncate(an.R[v], l);
      }
      rank_keys(raw, st.key, cl_of_vertex);
      st.nc = int32_t(st.key.size() / 3);
      st.child_ptr.assign(st.nc + 1, 0);
      for (int64_t v = 0; v < n; ++v) st.child_ptr[cl_of_vertex[v] + 1]++;
      for (int32_t c = 0; c < st.nc; ++c) st.child_ptr[c + 1] += st.child_ptr[c];
      st.child.resize(n);
      std::vector<int64_t> fillp(st.child_ptr.begin(), st.child_ptr.end() - 1);
      for (int64_t v = 0; v < n; ++v) st.child[fillp[cl_of_vertex[v]]++] = int32_t(v);
      st.before.reserve(an.colind.size());
      for (int64_t v = 0; v < n; ++v)
        for (int64_t e = an.rowptr[v]; e < an.rowptr[v + 1]; ++e) {
          int32_t a = cl_of_vertex[v], b = cl_of_vertex[an.colind[e]];
          st.before.push_back(pair_pack(std::max(a, b), std::min(a, b)));
        }
      sort_unique(st.before);
    } else {
      const SymStep& pv = an.steps[t - 2];
      // keys of this step were produced by the previous step's merge
      st.nc = int32_t(st.key.size() / 3);
      st.child_ptr.assign(st.nc + 1, 0);
      for (int32_t c = 0; c < pv.nc; ++c)
        if (pv.parent[c] >= 0) st.child_ptr[pv.parent[c] + 1]++;
      for (int32_t c = 0; c < st.nc; ++c) st.child_ptr[c + 1] += st.child_ptr[c];
      st.child.resize(st.child_ptr[st.nc]);
      std::vector<int64_t> fillp(st.child_ptr.begin(), st.child_ptr.end() - 1);
      for (int32_t c = 0; c < pv.nc; ++c)
        if (pv.parent[c] >= 0) st.child[fillp[pv.parent[c]]++] = c;
      st.before.reserve(pv.after.size());
      for (uint64_t p : pv.after) {
        int32_t a = pv.parent[pair_i(p)], b = pv.parent[pair_j(p)];
        st.before.push_back(pair_pack(std::max(a, b), std::min(a, b)));
      }
      sort_unique(st.before);
    }
    const int32_t nc = st.nc;
    int32_t ne = 0;
    while (ne < nc && sep_level(st.key[3 * ne]) == l) ++ne;
    st.ne = ne;
    // neighbours of eliminated clusters; fill among them
    st.enb_ptr.assign(ne + 1, 0);
    for (uint64_t p : st.before) {
      int32_t i = pair_i(p), j = pair_j(p);
      if (i != j && j < ne) {
        if (i < ne) return "two clusters of the same nested-dissection level are adjacent";
        st.enb_ptr[j + 1]++;
      }
    }
    for (int32_t s = 0; s < ne; ++s) st.enb_ptr[s + 1] += st.enb_ptr[s];
    st.enb.resize(st.enb_ptr[ne]);
    {
      std::vector<int64_t> fp(st.enb_ptr.begin(), st.enb_ptr.end() - 1);
      for (uint64_t p : st.before) {  // sorted by (i, j): neighbours come out ascending
        int32_t i = pair_i(p), j = pair_j(p);
        if (i != j && j < ne) st.enb[fp[j]++] = i;
      }
    }
    for (int32_t s = 0; s < ne; ++s) std::sort(st.enb.begin() + st.enb_ptr[s], st.enb.begin() + st.enb_ptr[s + 1]);
    st.after.clear();
    for (uint64_t p : st.before)
      if (pair_j(p) >= ne) st.after.push_back(p);
    for (int32_t s = 0; s < ne; ++s)
      for (int64_t a = st.enb_ptr[s]; a < st.enb_ptr[s + 1]; ++a)
        for (int64_t b = st.enb_ptr[s]; b <= a; ++b) st.after.push_back(pair_pack(st.enb[a], st.enb[b]));
    sort_unique(st.after);
    // neighbours of remaining clusters after fill
    st.nb_ptr.assign(nc + 1, 0);
    for (uint64_t p : st.after)
      if (pair_i(p) != pair_j(p)) {
        st.nb_ptr[pair_i(p) + 1]++;
        st.nb_ptr[pair_j(p) + 1]++;
      }
    for (int32_t c = 0; c < nc; ++c) st.nb_ptr[c + 1] += st.nb_ptr[c];
    st.nb.resize(st.nb_ptr[nc]);
    {
      std::vector<int64_t> fp(st.nb_ptr.begin(), st.nb_ptr.end() - 1);
      for (uint64_t p : st.after)
        if (pair_i(p) != pair_j(p)) {
          st.nb[fp[pair_i(p)]++] = pair_j(p);
          st.nb[fp[pair_j(p)]++] = pair_i(p);
        }
    }
    for (int32_t c = 0; c < nc; ++c) std::sort(st.nb.begin() + st.nb_ptr[c], st.nb.begin() + st.nb_ptr[c + 1]);
    // greedy colouring of the remaining clusters in ascending id
    st.colour.assign(nc, -1);
    if (l > 1) {
      std::vector<int32_t> used;
      for (int32_t p = ne; p < nc; ++p) {
        used.clear();
        for (int64_t e = st.nb_ptr[p]; e < st.nb_ptr[p + 1]; ++e)
          if (st.colour[st.nb[e]] >= 0) used.push_back(st.colour[st.nb[e]]);
        std::sort(used.begin(), used.end());
        int32_t c = 0;
        for (int32_t u : used) {
          if (u == c) ++c;
          else if (u > c) break;
        }
        st.colour[p] = c;
      }
    }
    // merge: clusters of the next step
    st.parent.assign(nc, -1);
    if (l > 1) {
      std::vector<int64_t> raw(3 * size_t(nc - ne));
      for (int32_t c = ne; c < nc; ++c) {
        raw[3 * (c - ne)] = st.key[3 * c];
        raw[3 * (c - ne) + 1] = sep_truncate(st.key[3 * c + 1], l - 1);
        raw[3 * (c - ne) + 2] = sep_truncate(st.key[3 * c + 2], l - 1);
      }
      std::vector<int32_t> rk;
      rank_keys(raw, an.steps[t].key, rk);
      for (int32_t c = ne; c < nc; ++c) st.parent[c] = rk[c - ne];
    }
  }
  return "";
}

}  // namespace

std::string analyze_pattern(Analysis& an) {
  order_and_cluster(an);
  return symbolic(an);
}

}  // namespace spand
