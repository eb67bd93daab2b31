// Numerical factorization driver: Algorithm 3 (OrthS) level by level on the GPU.
//
// Storage.  The trailing matrix of step t is a set of column panels: the panel of
// cluster j stacks the dense blocks (i, j), i >= j, of the block pattern (diagonal
// block first, then ascending i), column-major with the panel height as leading
// dimension.  Eliminated clusters come first in the canonical order, so the panel
// of an eliminated s is exactly [A_ss; A_{N_s s}]; those panels live in persistent
// factor storage (they become [L_s; G_s]), the panels of the remaining clusters in
// a per-step arena that the next step's merge consumes.
//
// Per step (t = 1..L, level l = L - t + 1):
//   1. assemble: scatter the CSR values (t = 1) or merge the previous arena
//      (Sec. 2.7: parent blocks are the concatenation of child blocks);
//   2. eliminate every level-l cluster s (Sec. 2.4): blocked Cholesky of the panel
//      [A_ss; A_{N_s s}] -> [L_s; G = A_{N_s s} L_s^{-T}]; C_s = G G^T; every target
//      block subtracts its contributions in ascending s (deterministic);
//   3. if t > skip and l > 1: scale every remaining cluster (Sec. 2.5): blocked
//      Cholesky of its panel gives L_p and the right-scaled blocks below it, a
//      blocked left triangular solve applies L_i^{-1} to every block (i, p), A_pp <- I;
//   4. then sparsify every remaining cluster, one colour class per launch
//      (Sec. 2.6.1), and read the kept ranks back to the host;
//   5. plan the next step's layout from the ranks.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>

#include "context.h"

namespace spand {

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) return set_err(h, SPAND_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

spand_status dalloc(spand_ctx* h, DevBuf& b, size_t bytes) {
  b.release();
  if (bytes == 0) return SPAND_OK;
  void* p = nullptr;
  size_t cap = 0;
  hipError_t e = h->pool.get(bytes, &p, &cap);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(h, SPAND_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.p = p;
  b.bytes = bytes;
  b.cap = cap;
  b.pool = &h->pool;
  return SPAND_OK;
}

// Host-to-device copy through the call's pinned staging (asynchronous on the
// handle's stream).
spand_status stage_copy(spand_ctx* h, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return SPAND_OK;
  char* hp = h->stage.get(bytes);
  if (!hp) return set_err(h, SPAND_E_NOMEM, "pinned staging of " + std::to_string(bytes) + " bytes failed");
  std::memcpy(hp, src, bytes);
  HIPCHK(hipMemcpyAsync(dst, hp, bytes, hipMemcpyHostToDevice, h->stream));
  return SPAND_OK;
}

template <typename T>
spand_status upload(spand_ctx* h, DevBuf& b, const std::vector<T>& v) {
  spand_status st = dalloc(h, b, v.size() * sizeof(T));
  if (st != SPAND_OK) return st;
  return stage_copy(h, b.p, v.data(), v.size() * sizeof(T));
}

// Column-panel layout of one step.  Panels of eliminated clusters (j < ne) are
// placed in the persistent elimination buffer, the others in the step arena.
struct Layout {
  int32_t ne = 0;
  std::vector<int64_t> pan_ptr;  // nc+1
  std::vector<int32_t> prow;     // row cluster of each panel entry (diagonal first)
  std::vector<int64_t> proff;    // row offset of each entry inside its panel
  std::vector<int64_t> H;        // panel heights
  std::vector<int64_t> base;     // panel start (elements) inside its buffer
  int64_t total_elim = 0, total_arena = 0;
  int64_t find(int32_t i, int32_t j) const {
    auto b = prow.begin() + pan_ptr[j], e = prow.begin() + pan_ptr[j + 1];
    auto it = std::lower_bound(b, e, i);
    if (it == e || *it != i) return -1;
    return proff[it - prow.begin()];
  }
  double* panel(int32_t j, double* E, double* A) const { return (j < ne ? E : A) + base[j]; }
};

void build_layout(const SymStep& st, const std::vector<int32_t>& size, Layout& L) {
  const int32_t nc = st.nc, ne = st.ne;
  L.ne = ne;
  L.pan_ptr.assign(nc + 1, 0);
  auto each = [&](auto&& f) {
    for (uint64_t p : st.before)
      if (pair_j(p) < ne) f(p);
    for (uint64_t p : st.after) f(p);
  };
  each([&](uint64_t p) { L.pan_ptr[pair_j(p) + 1]++; });
  for (int32_t c = 0; c < nc; ++c) L.pan_ptr[c + 1] += L.pan_ptr[c];
  L.prow.resize(L.pan_ptr[nc]);
  L.proff.resize(L.pan_ptr[nc]);
  std::vector<int64_t> fill(L.pan_ptr.begin(), L.pan_ptr.end() - 1);
  // `before` (j < ne) and `after` (j >= ne) touch disjoint panels, each in ascending i
  each([&](uint64_t p) { L.prow[fill[pair_j(p)]++] = pair_i(p); });
  L.H.assign(nc, 0);
  L.base.assign(nc, 0);
  int64_t te = 0, ta = 0;
  for (int32_t j = 0; j < nc; ++j) {
    int64_t h = 0;
    for (int64_t e = L.pan_ptr[j]; e < L.pan_ptr[j + 1]; ++e) {
      L.proff[e] = h;
      h += size[L.prow[e]];
    }
    L.H[j] = h;
    int64_t& tot = (j < ne) ? te : ta;
    L.base[j] = tot;
    tot += h * size[j];
  }
  L.total_elim = te;
  L.total_arena = ta;
}

// A sequence of batched-GEMM launches.  The host uploads the products only; a
// device kernel expands them into the tile -> product map the launches read.
// part: 0 every tile, 1 tiles on or below the diagonal, 2 tiles on or above it.
struct GemmSeq {
  std::vector<GemmDesc> d;
  std::vector<int64_t> cut;  // tile range end of every launch
  std::vector<int> prec;
  int64_t ntiles = 0;
  DevBuf dd, dmap;
  void add(GemmDesc g, int part) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return;
    g.part = part;
    g.t0 = ntiles;
    ntiles += gemm_tiles(g.M, g.N, part);
    d.push_back(g);
  }
  void end_launch(int p) {
    cut.push_back(ntiles);
    prec.push_back(p);
  }
  spand_status upload_all(spand_ctx* h) {
    spand_status st = upload(h, dd, d);
    if (st != SPAND_OK) return st;
    if ((st = dalloc(h, dmap, size_t(ntiles) * sizeof(int32_t))) != SPAND_OK) return st;
    launch_expand_tiles(dd.as<GemmDesc>(), int32_t(d.size()), dmap.as<int32_t>(), h->stream);
    return SPAND_OK;
  }
  void launch(spand_ctx* h, size_t q) const {
    const int64_t b = q ? cut[q - 1] : 0;
    if (cut[q] > b) launch_gemm(dd.as<GemmDesc>(), dmap.as<int32_t>(), b, cut[q] - b, prec[q], h->stream);
  }
};

// One panel factorized by the blocked Cholesky: diagonal n x n on top, m rows in all.
struct Front {
  double* P;
  double* dinv;  // ceil(n / CHOL_NB) blocks of CHOL_NB^2 doubles
  int32_t ld, n, m, id;
};

// I_n into the n x n block D (ld ld), in column ranges of at most COPY_CHUNK entries
void add_identity(std::vector<IdentDesc>& v, double* D, int32_t n, int32_t ld) {
  const int32_t step = std::max(1, COPY_CHUNK / std::max(n, 1));
  for (int32_t c0 = 0; c0 < n; c0 += step) v.push_back(IdentDesc{D, n, ld, c0, std::min(n, c0 + step)});
}

int64_t dinv_size(int32_t n) { return int64_t((n + CHOL_NB - 1) / CHOL_NB) * CHOL_NB * CHOL_NB; }

// Right-looking blocked Cholesky of every front in lockstep over its diagonal
// blocks.  Updates inside the n x n pivot block are FP64; `prec_below` selects the
// arithmetic of the rows below it (the TRSM and Schur-side updates).
// The trailing updates go in groups of h->tune.chol_group block columns.
spand_status blocked_cholesky(spand_ctx* h, const std::vector<Front>& F, int32_t* d_fail, int prec_below) {
  const int32_t CHOL_GROUP = std::max(1, h->tune.chol_group);
  int32_t nmax = 0;
  for (const Front& f : F) nmax = std::max(nmax, f.n);
  std::vector<PotrfDesc> pd;
  std::vector<PanelDesc> td;
  std::vector<int64_t> pcut, tcut;
  GemmSeq g;
  for (int32_t kb = 0; kb < nmax; kb += CHOL_NB) {
    for (const Front& f : F) {
      if (f.n <= kb) continue;
      const int32_t w = std::min(CHOL_NB, f.n - kb);
      double* Dk = f.dinv + int64_t(kb / CHOL_NB) * CHOL_NB * CHOL_NB;
      pd.push_back(PotrfDesc{f.P + kb + int64_t(kb) * f.ld, Dk, f.ld, w, f.id, 0});
      for (int32_t r0 = kb + w; r0 < f.m; r0 += 256)
        td.push_back(PanelDesc{f.P + int64_t(kb) * f.ld, Dk, f.ld, w, r0, std::min(f.m, r0 + 256)});
    }
    pcut.push_back(int64_t(pd.size()));
    tcut.push_back(int64_t(td.size()));
    // Trailing updates in groups of CHOL_GROUP block columns: inside a group only the
    // next block column is updated (it is factored next), with every block of the
    // group so far; at the group's last block, the group goes into every column beyond
    // in one product of depth CHOL_GROUP NB, so the far trailing matrix is read and
    // written once per group.
    const int32_t kblk = kb / CHOL_NB;
    const bool pair = (kblk % CHOL_GROUP) == CHOL_GROUP - 1;
    const int32_t kg = (kblk / CHOL_GROUP) * CHOL_GROUP * CHOL_NB;  // first column of the group
    for (const Front& f : F) {  // trailing update inside the pivot block (FP64)
      if (f.n <= kb) continue;
      const int32_t w = std::min(CHOL_NB, f.n - kb);
      const int32_t ks = kg, c0 = kb + w;
      const int32_t c1 = pair ? f.n : std::min(f.n, c0 + CHOL_NB);
      if (c1 <= c0) continue;
      GemmDesc q{};
      q.A = f.P + c0 + int64_t(ks) * f.ld; q.lda = f.ld;
      q.B = q.A; q.ldb = f.ld;
      q.C = f.P + c0 + int64_t(c0) * f.ld; q.ldc = f.ld;
      q.M = f.n - c0; q.N = c1 - c0; q.K = kb + w - ks;
      q.flags = G_TB; q.alpha = -1.0; q.beta = 1.0;
      if (pair) {  // square: the lower tiles only
        q.flags |= G_LOWERC;
        g.add(q, 1);
      } else {     // one block column: every tile is on or below the diagonal
        g.add(q, 0);
      }
    }
    g.end_launch(0);
    for (const Front& f : F) {  // rows below the pivot block
      if (f.n <= kb) continue;
      const int32_t w = std::min(CHOL_NB, f.n - kb);
      const int32_t ks = kg, c0 = kb + w;
      const int32_t c1 = pair ? f.n : std::min(f.n, c0 + CHOL_NB);
      if (c1 <= c0 || f.m <= f.n) continue;
      GemmDesc q{};
      q.A = f.P + f.n + int64_t(ks) * f.ld; q.lda = f.ld;
      q.B = f.P + c0 + int64_t(ks) * f.ld; q.ldb = f.ld;
      q.C = f.P + f.n + int64_t(c0) * f.ld; q.ldc = f.ld;
      q.M = f.m - f.n; q.N = c1 - c0; q.K = kb + w - ks;
      q.flags = G_TB; q.alpha = -1.0; q.beta = 1.0;
      g.add(q, 0);
    }
    g.end_launch(prec_below);
  }
  DevBuf dp, dt;
  spand_status st;
  if ((st = upload(h, dp, pd)) != SPAND_OK) return st;
  if ((st = upload(h, dt, td)) != SPAND_OK) return st;
  if ((st = g.upload_all(h)) != SPAND_OK) return st;
  for (size_t q = 0; q < pcut.size(); ++q) {
    const int64_t pb = q ? pcut[q - 1] : 0, tb = q ? tcut[q - 1] : 0;
    launch_potrf_diag(dp.as<PotrfDesc>() + pb, int32_t(pcut[q] - pb), d_fail, h->stream);
    launch_panel_trsm(dt.as<PanelDesc>() + tb, int32_t(tcut[q] - tb), h->stream);
    g.launch(h, 2 * q);
    g.launch(h, 2 * q + 1);
  }
  HIPCHK(hipGetLastError());
  // the descriptor blocks go back to the handle's pool; a later allocation that
  // reuses them is ordered after these launches on the stream
  return SPAND_OK;
}

// X (nrows x ncols, ld ldx) <- L^{-1} X for lower-triangular L (ld ldl) whose diagonal
// blocks have the inverses `dinv`.
struct LeftBlock {
  double* X;
  const double* L;
  const double* dinv;
  int32_t ldx, ldl, nrows, ncols;
};

spand_status left_trsm(spand_ctx* h, const std::vector<LeftBlock>& B) {
  const int32_t CHOL_GROUP = std::max(1, h->tune.chol_group);
  int32_t nmax = 0;
  for (const LeftBlock& b : B) nmax = std::max(nmax, b.nrows);
  std::vector<LeftDesc> ld;
  std::vector<int64_t> lcut;
  GemmSeq g;
  for (int32_t kb = 0; kb < nmax; kb += CHOL_NB) {
    // grouped as in blocked_cholesky: inside a group only the next block row is
    // updated, at the group's end every row below, at depth CHOL_GROUP NB
    const int32_t kblk = kb / CHOL_NB;
    const bool pair = (kblk % CHOL_GROUP) == CHOL_GROUP - 1;
    const int32_t kg = (kblk / CHOL_GROUP) * CHOL_GROUP * CHOL_NB;
    for (const LeftBlock& b : B) {
      if (b.nrows <= kb) continue;
      const int32_t w = std::min(CHOL_NB, b.nrows - kb);
      const double* Dk = b.dinv + int64_t(kb / CHOL_NB) * CHOL_NB * CHOL_NB;
      for (int32_t c0 = 0; c0 < b.ncols; c0 += 256)
        ld.push_back(LeftDesc{b.X + kb, Dk, b.ldx, w, c0, std::min(b.ncols, c0 + 256)});
      const int32_t ks = kg, r0 = kb + w;
      const int32_t r1 = pair ? b.nrows : std::min(b.nrows, r0 + CHOL_NB);
      GemmDesc q{};
      q.A = b.L + r0 + int64_t(ks) * b.ldl; q.lda = b.ldl;
      q.B = b.X + ks; q.ldb = b.ldx;
      q.C = b.X + r0; q.ldc = b.ldx;
      q.M = r1 - r0; q.N = b.ncols; q.K = kb + w - ks;
      q.flags = 0; q.alpha = -1.0; q.beta = 1.0;
      g.add(q, 0);
    }
    lcut.push_back(int64_t(ld.size()));
    g.end_launch(0);
  }
  DevBuf dl;
  spand_status st;
  if ((st = upload(h, dl, ld)) != SPAND_OK) return st;
  if ((st = g.upload_all(h)) != SPAND_OK) return st;
  for (size_t q = 0; q < lcut.size(); ++q) {
    const int64_t b = q ? lcut[q - 1] : 0;
    launch_left_trsm_diag(dl.as<LeftDesc>() + b, int32_t(lcut[q] - b), h->stream);
    g.launch(h, q);
  }
  HIPCHK(hipGetLastError());
  return SPAND_OK;
}

}  // namespace

// Apply descriptors of step t (its eliminations, target updates, scalings and
// Householder products), built from the step's stored sizes, slots and factor
// offsets.  The factorization calls this while the next step's kernels run.
struct ApplyPlan {
  int32_t t = 0;
  std::vector<int64_t> ed_off, sc_off, v_off, t_off;
  std::vector<int32_t> nN, nref;
};

spand_status build_apply(spand_ctx* h, const SymStep& sy, StepNum& sn, const Layout& lay, const ApplyPlan& pl) {
  const int32_t nc = sy.nc, ne = sy.ne;
  const double* E = sn.elim.as<double>();
  const std::vector<int64_t>& ed_off = pl.ed_off;
  const std::vector<int64_t>& sc_off = pl.sc_off;
  const std::vector<int64_t>& v_off = pl.v_off;
  const std::vector<int64_t>& t_off = pl.t_off;
  const std::vector<int32_t>& nN = pl.nN;
  const std::vector<int32_t>& nref = pl.nref;
  spand_status st;
  std::vector<int32_t> nslot;
  int64_t tmp = 0;
  sn.h_elim.clear();
  for (int32_t s = 0; s < ne; ++s) {
    ElimAp e{};
    e.L = E + lay.base[s];
    e.G = E + lay.base[s] + sn.size[s];
    e.Dinv = sn.edinv.as<double>() + ed_off[s];
    e.ld = int32_t(lay.H[s]);
    e.ns = sn.size[s];
    e.nN = nN[s];
    e.slot_s = sn.slot_ptr[s];
    e.slot_N = int64_t(nslot.size());
    for (int64_t q = sy.enb_ptr[s]; q < sy.enb_ptr[s + 1]; ++q) {
      const int32_t nb = sy.enb[q];
      nslot.insert(nslot.end(), sn.slot.begin() + sn.slot_ptr[nb], sn.slot.begin() + sn.slot_ptr[nb + 1]);
    }
    e.nchunk = std::max(1, (e.nN + ELIM_RC - 1) / ELIM_RC);
    e.tmp = tmp;
    tmp += int64_t(std::max(e.ns, 1)) * (e.nchunk > 1 ? 1 + e.nchunk : 1);
    sn.h_elim.push_back(e);
  }
  sn.tmp_elim = tmp;
  sn.h_etile.clear();
  for (int32_t s = 0; s < ne; ++s)
    for (int32_t c = 0; c < sn.h_elim[s].nchunk; ++c)
      for (int32_t k0 = 0; k0 < sn.h_elim[s].ns; k0 += 64) sn.h_etile.push_back(ElimTile{s, k0, c, 0});
  // forward target updates, grouped by receiving cluster in ascending s
  struct TI { int32_t n, s; int64_t row; };
  std::vector<TI> tis;
  for (int32_t s = 0; s < ne; ++s) {
    int64_t row = 0;
    for (int64_t q = sy.enb_ptr[s]; q < sy.enb_ptr[s + 1]; ++q) {
      const int32_t nb = sy.enb[q];
      if (sn.size[nb] > 0 && sn.size[s] > 0) tis.push_back(TI{nb, s, row});
      row += sn.size[nb];
    }
  }
  std::stable_sort(tis.begin(), tis.end(), [](const TI& x, const TI& y) { return x.n < y.n; });
  sn.h_target.clear();
  sn.h_contrib.clear();
  for (size_t q = 0; q < tis.size();) {
    size_t r = q;
    TargetAp ta{};
    ta.nn = sn.size[tis[q].n];
    ta.slot_n = sn.slot_ptr[tis[q].n];
    ta.cbeg = int32_t(sn.h_contrib.size());
    while (r < tis.size() && tis[r].n == tis[q].n) {
      const int32_t s = tis[r].s;
      sn.h_contrib.push_back(TargetContrib{sn.h_elim[s].G + tis[r].row, sn.h_elim[s].ld, sn.size[s], sn.h_elim[s].tmp});
      ++r;
    }
    ta.cend = int32_t(sn.h_contrib.size());
    for (int32_t r0 = 0; r0 < ta.nn; r0 += 64) {  // one workgroup per 64-row tile
      ta.r0 = r0;
      sn.h_target.push_back(ta);
    }
    q = r;
  }
  sn.h_scale.clear();
  sn.h_stile.clear();
  sn.h_sgather.clear();
  sn.h_house.clear();
  sn.h_hr.clear();
  sn.h_hv.clear();
  int64_t tmp2 = 0, tmp3 = 0;
  // interfaces of at most 64 dofs, and of at most 128 when a step has enough of
  // them to fill the GPU: scaling and Householder product in one wave (np <= 64
  // first, then np <= 128); the others by the tiled kernels
  std::vector<IfaceAp> if1, if2;
  int32_t n128 = 0;
  for (int32_t p = ne; p < nc; ++p)
    if (sc_off[p] >= 0 && sn.size[p] > 64 && sn.size[p] <= 128) ++n128;
  const int32_t fuse_max = (h->tune.fuse128_min >= 0 && n128 >= h->tune.fuse128_min) ? 128 : 64;
  for (int32_t p = ne; p < nc; ++p) {
    if (sc_off[p] >= 0 && sn.size[p] <= fuse_max) {
      IfaceAp f{};
      f.Linv = sn.scale.as<double>() + sc_off[p];
      f.np = sn.size[p];
      f.slot_p = sn.slot_ptr[p];
      if (v_off[p] >= 0 && nref[p] > 0) {
        f.V = sn.house.as<double>() + v_off[p];
        f.T = sn.house.as<double>() + t_off[p];
        f.r = nref[p];
      }
      (f.np <= 64 ? if1 : if2).push_back(f);
      continue;
    }
    if (sc_off[p] >= 0) {
      ScaleAp a{};
      a.Linv = sn.scale.as<double>() + sc_off[p];
      a.np = sn.size[p];
      a.slot_p = sn.slot_ptr[p];
      a.tmp = tmp2;
      tmp2 += sn.size[p];
      const int32_t sid = int32_t(sn.h_scale.size());
      for (int32_t r0 = 0; r0 < a.np; r0 += 64) sn.h_stile.push_back(ScaleTile{sid, r0});
      sn.h_sgather.insert(sn.h_sgather.end(), sn.slot.begin() + sn.slot_ptr[p],
                          sn.slot.begin() + sn.slot_ptr[p] + sn.size[p]);
      sn.h_scale.push_back(a);
    }
    if (v_off[p] >= 0 && nref[p] > 0) {
      HouseAp hp{};
      hp.V = sn.house.as<double>() + v_off[p];
      hp.T = sn.house.as<double>() + t_off[p];
      hp.np = sn.size[p];
      hp.r = nref[p];
      hp.slot_p = sn.slot_ptr[p];
      hp.tmp = tmp3;
      tmp3 += 2 * int64_t(nref[p]);
      const int32_t hid = int32_t(sn.h_house.size());
      for (int32_t j0 = 0; j0 < hp.r; j0 += 64) sn.h_hr.push_back(HouseTile{hid, j0});
      for (int32_t r0 = 0; r0 < hp.np; r0 += 64) sn.h_hv.push_back(HouseTile{hid, r0});
      sn.h_house.push_back(hp);
    }
  }
  sn.n_iface1 = int32_t(if1.size());
  sn.n_iface2 = int32_t(if2.size());
  sn.h_iface = std::move(if1);
  sn.h_iface.insert(sn.h_iface.end(), if2.begin(), if2.end());
  sn.tmp_scale = std::max(tmp2, tmp3);
  sn.nslot_len = int64_t(nslot.size());
  h->max_tmp = std::max(h->max_tmp, std::max(sn.tmp_elim, sn.tmp_scale));
  h->max_gather = std::max(h->max_gather, sn.nslot_len);
  sn.n_elim_ap = int32_t(sn.h_elim.size());
  sn.n_target = int32_t(sn.h_target.size());
  sn.n_scale = int32_t(sn.h_scale.size());
  sn.n_house = int32_t(sn.h_house.size());
  sn.n_etile = int32_t(sn.h_etile.size());
  sn.n_stile = int32_t(sn.h_stile.size());
  sn.sgather_len = int64_t(sn.h_sgather.size());
  sn.n_hr = int32_t(sn.h_hr.size());
  sn.n_hv = int32_t(sn.h_hv.size());
  if ((st = upload(h, sn.d_slot, sn.slot)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_nslot, nslot)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_elim, sn.h_elim)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_target, sn.h_target)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_contrib, sn.h_contrib)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_scale, sn.h_scale)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_house, sn.h_house)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_etile, sn.h_etile)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_stile, sn.h_stile)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_sgather, sn.h_sgather)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_hr, sn.h_hr)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_hv, sn.h_hv)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_iface, sn.h_iface)) != SPAND_OK) return st;
  return SPAND_OK;
}

spand_status factor_numeric(spand_ctx* h, const double* values, double tol, int32_t skip, spand_prec prec) {
  Analysis& an = h->an;
  const int32_t Lv = an.levels;
  const int gemm_prec = (prec == SPAND_FP64) ? 0 : (prec == SPAND_FP32 ? 1 : 2);
  h->stage.reset();
  h->num.clear();
  h->num.resize(Lv);
  h->max_tmp = 0;
  h->max_gather = 0;
  spand_status st;

  DevBuf dflag;  // [0] elimination failure id, [1] scaling failure id, [2] non-finite input
  if ((st = dalloc(h, dflag, 4 * sizeof(int32_t))) != SPAND_OK) return st;
  const int32_t flag_init[4] = {0x7fffffff, 0x7fffffff, 0, 0};
  if ((st = stage_copy(h, dflag.p, flag_init, sizeof(flag_init))) != SPAND_OK) return st;
  int32_t* d_fail_elim = dflag.as<int32_t>();
  int32_t* d_fail_scale = dflag.as<int32_t>() + 1;
  int32_t* d_nonfinite = dflag.as<int32_t>() + 2;

  // phase boundaries of every step (5 events per step), read after the last sync
  EventPool phev;
  std::vector<char> elim_ran(size_t(Lv) + 1, 0);
  // The device flags are read at one sync per step: the rank read-back of a
  // sparsified step, or the end of any other step.  Kernels that run after a
  // failure in the same step only see bad values, never bad indices.
  auto check_flags = [&](int32_t t) -> spand_status {
    int32_t flags[4];
    HIPCHK(hipMemcpyAsync(flags, dflag.p, sizeof(flags), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (flags[2]) return set_err(h, SPAND_E_INVALID, "matrix values contain NaN or Inf");
    if (flags[0] != 0x7fffffff) {
      h->stats.fail_step = t;
      h->stats.fail_cluster = flags[0];
      h->stats.fail_phase = 0;
      return set_err(h, SPAND_E_NOT_SPD, "pivot block not SPD at step " + std::to_string(t) + ", cluster " +
                                             std::to_string(flags[0]) + " (elimination)");
    }
    if (flags[1] != 0x7fffffff) {
      h->stats.fail_step = t;
      h->stats.fail_cluster = flags[1];
      h->stats.fail_phase = 1;
      return set_err(h, SPAND_E_NOT_SPD, "interface block not SPD at step " + std::to_string(t) + ", cluster " +
                                             std::to_string(flags[1]) + " (scaling)");
    }
    return SPAND_OK;
  };
  std::memset(h->stats.step_phase_seconds, 0, sizeof(h->stats.step_phase_seconds));
  std::memset(h->stats.step_m_F, 0, sizeof(h->stats.step_m_F));

  EventPool evpool;  // per-launch timing of the CPQR
  int64_t m_F = 0;
  double elim_flops = 0.0, elim_ms = 0.0;
  double cpqr_flops = 0.0, cpqr_ms = 0.0;
  int64_t cpqr_launches = 0;
  int64_t cpqr_ifaces[4] = {0, 0, 0, 0};  // single, wide, multi (32 x 2), multi (20 x 3)
  int32_t s_top = 0;

  DevBuf arena_prev;
  Layout lay_prev;
  // apply descriptors of the previous step, built while the current step runs
  // (lay_prev is that step's layout until the end of the current one)
  ApplyPlan pending;
  // Compact-WY factors T_p of the interfaces sparsified in the last step: launched
  // after the next step's sparsification (or at the end) so that their planning is
  // off the path between a rank read-back and the next step's first kernels.
  std::vector<TDesc> t_pending;
  auto flush_t = [&]() -> spand_status {
    if (t_pending.empty()) return SPAND_OK;
    const std::vector<TDesc> tds = std::move(t_pending);
    t_pending.clear();
    spand_status st = SPAND_OK;
    // S = V^T V into the T blocks (MFMA, upper tiles), then the T recurrence
    GemmSeq vtv;
    for (const TDesc& td : tds) {
      GemmDesc q{};
      q.A = td.V; q.lda = td.m;
      q.B = td.V; q.ldb = td.m;
      q.C = td.T; q.ldc = td.r;
      q.M = td.r; q.N = td.r; q.K = td.m;
      q.flags = G_TA;
      q.alpha = 1.0; q.beta = 0.0;
      vtv.add(q, 2);
    }
    vtv.end_launch(0);
    if ((st = vtv.upload_all(h)) != SPAND_OK) return st;
    vtv.launch(h, 0);
    HIPCHK(hipGetLastError());
    // T by 64-wide block columns: the diagonal blocks, then for J = 1, 2, ...
    // X = S[:J0, J] T_JJ and T[:J0, J] = -T[:J0, :J0] X (GEMMs across interfaces)
    std::vector<TBlock> tbs;
    int32_t rmax = 0;
    int64_t x_total = 0;
    std::vector<int64_t> x_off(tds.size(), -1);
    for (size_t q = 0; q < tds.size(); ++q) {
      const TDesc& td = tds[q];
      for (int32_t j0 = 0; j0 < td.r; j0 += 64) tbs.push_back(TBlock{td.T, td.tau, td.r, j0});
      rmax = std::max(rmax, td.r);
      if (td.r > 64) {
        x_off[q] = x_total;
        x_total += int64_t(td.r) * 64;
      }
    }
    DevBuf dtb, xb;
    if ((st = upload(h, dtb, tbs)) != SPAND_OK) return st;
    launch_build_t_diag(dtb.as<TBlock>(), int32_t(tbs.size()), h->stream);
    HIPCHK(hipGetLastError());
    if (rmax > 64) {
      if ((st = dalloc(h, xb, size_t(x_total) * sizeof(double))) != SPAND_OK) return st;
      GemmSeq tg2;
      for (int32_t j0 = 64; j0 < rmax; j0 += 64) {
        for (size_t q = 0; q < tds.size(); ++q) {
          const TDesc& td = tds[q];
          if (td.r <= j0) continue;
          const int32_t w = std::min(64, td.r - j0);
          GemmDesc g{};  // X = S[:j0, J] T_JJ
          g.A = td.T + int64_t(j0) * td.r; g.lda = td.r;
          g.B = td.T + j0 + int64_t(j0) * td.r; g.ldb = td.r;
          g.C = xb.as<double>() + x_off[q]; g.ldc = td.r;
          g.M = j0; g.N = w; g.K = w;
          g.alpha = 1.0; g.beta = 0.0;
          tg2.add(g, 0);
        }
        tg2.end_launch(0);
        for (size_t q = 0; q < tds.size(); ++q) {
          const TDesc& td = tds[q];
          if (td.r <= j0) continue;
          const int32_t w = std::min(64, td.r - j0);
          GemmDesc g{};  // T[:j0, J] = -T[:j0, :j0] X
          g.A = td.T; g.lda = td.r;
          g.B = xb.as<double>() + x_off[q]; g.ldb = td.r;
          g.C = td.T + int64_t(j0) * td.r; g.ldc = td.r;
          g.M = j0; g.N = w; g.K = j0;
          g.alpha = -1.0; g.beta = 0.0;
          tg2.add(g, 0);
        }
        tg2.end_launch(0);
      }
      if ((st = tg2.upload_all(h)) != SPAND_OK) return st;
      for (size_t q = 0; q < tg2.cut.size(); ++q) tg2.launch(h, q);
      HIPCHK(hipGetLastError());
    }
    return SPAND_OK;
  };

  auto flush_apply = [&]() -> spand_status {
    if (pending.t == 0) return SPAND_OK;
    const int32_t pt = pending.t;
    pending.t = 0;
    return build_apply(h, an.steps[pt - 1], h->num[pt - 1], lay_prev, pending);
  };

  for (int32_t t = 1; t <= Lv; ++t) {
    const SymStep& sy = an.steps[t - 1];
    StepNum& sn = h->num[t - 1];
    const int32_t nc = sy.nc, ne = sy.ne;
    const bool sparsify = (t > skip) && (sy.level > 1);
    bool flags_read = false;  // this step's flags were checked at its rank read-back
    hipEvent_t ph[5];
    for (int q = 0; q < 5; ++q) HIPCHK(phev.get(5 * size_t(t - 1) + q, &ph[q]));

    // ---- sizes and slots of this step's clusters
    sn.size.assign(nc, 0);
    sn.slot_ptr.assign(nc + 1, 0);
    if (t == 1) {
      for (int32_t c = 0; c < nc; ++c) sn.size[c] = int32_t(sy.child_ptr[c + 1] - sy.child_ptr[c]);
      sn.slot.assign(sy.child.begin(), sy.child.end());
      for (int32_t c = 0; c < nc; ++c) sn.slot_ptr[c + 1] = sy.child_ptr[c + 1];
    } else {
      const StepNum& pv = h->num[t - 2];
      for (int32_t c = 0; c < nc; ++c) {
        int32_t s = 0;
        for (int64_t e = sy.child_ptr[c]; e < sy.child_ptr[c + 1]; ++e) s += pv.rank[sy.child[e]];
        sn.size[c] = s;
        sn.slot_ptr[c + 1] = sn.slot_ptr[c] + s;
      }
      sn.slot.resize(sn.slot_ptr[nc]);
      for (int32_t c = 0; c < nc; ++c) {
        int64_t o = sn.slot_ptr[c];
        for (int64_t e = sy.child_ptr[c]; e < sy.child_ptr[c + 1]; ++e) {
          const int32_t ch = sy.child[e];
          const int32_t r = pv.rank[ch];
          std::copy(pv.slot.begin() + pv.slot_ptr[ch], pv.slot.begin() + pv.slot_ptr[ch] + r, sn.slot.begin() + o);
          o += r;
        }
      }
    }
    if (sy.level == 1)
      for (int32_t s = 0; s < ne; ++s) s_top += sn.size[s];

    // ---- layout and assembly
    HIPCHK(hipEventRecord(ph[0], h->stream));
    Layout lay;
    build_layout(sy, sn.size, lay);
    DevBuf arena;
    if ((st = dalloc(h, sn.elim, size_t(lay.total_elim) * sizeof(double))) != SPAND_OK) return st;
    if ((st = dalloc(h, arena, size_t(lay.total_arena) * sizeof(double))) != SPAND_OK) return st;
    double* E = sn.elim.as<double>();
    double* A = arena.as<double>();
    if (lay.total_elim) HIPCHK(hipMemsetAsync(E, 0, size_t(lay.total_elim) * sizeof(double), h->stream));
    if (lay.total_arena) HIPCHK(hipMemsetAsync(A, 0, size_t(lay.total_arena) * sizeof(double), h->stream));
    DevBuf d_copy;
    std::vector<CopyDesc> copies;
    if (t == 1 && h->d_dst1.p) {
      // the step-1 layout depends on the pattern only: reuse the map of an earlier factor
      launch_scatter_values(values, h->d_dst1.as<int64_t>(), int64_t(an.colind.size()), A, E, d_nonfinite, h->stream);
      HIPCHK(hipGetLastError());
    } else if (t == 1) {
      // destination of every CSR entry inside the step-1 panels: >= 0 arena offset,
      // <= -2 elimination-buffer offset -(d+2), -1 skipped (upper triangle)
      std::vector<int32_t> cl(an.n), pos(an.n);
      for (int32_t c = 0; c < nc; ++c)
        for (int64_t e = sy.child_ptr[c]; e < sy.child_ptr[c + 1]; ++e) {
          cl[sy.child[e]] = c;
          pos[sy.child[e]] = int32_t(e - sy.child_ptr[c]);
        }
      std::vector<int64_t> dst(an.colind.size(), -1);
      for (int64_t v = 0; v < an.n; ++v)
        for (int64_t e = an.rowptr[v]; e < an.rowptr[v + 1]; ++e) {
          const int32_t u = an.colind[e];
          const int32_t i = cl[v], j = cl[u];
          if (i < j) continue;
          const int64_t off = lay.base[j] + lay.find(i, j) + pos[v] + int64_t(pos[u]) * lay.H[j];
          dst[e] = (j < ne) ? -(off + 2) : off;
        }
      if ((st = upload(h, h->d_dst1, dst)) != SPAND_OK) return st;
      launch_scatter_values(values, h->d_dst1.as<int64_t>(), int64_t(dst.size()), A, E, d_nonfinite, h->stream);
      HIPCHK(hipGetLastError());
    } else {
      const StepNum& pv = h->num[t - 2];
      // the copies of the pairs [q0, q1) of `before`, in order
      auto plan_copies = [&](size_t q0, size_t q1, std::vector<CopyDesc>& out) {
        for (size_t q = q0; q < q1; ++q) {
          const uint64_t pr = sy.before[q];
          const int32_t I = pair_i(pr), J = pair_j(pr);
          double* dbase = lay.panel(J, E, A) + lay.find(I, J);
          int64_t ro = 0;
          for (int64_t a = sy.child_ptr[I]; a < sy.child_ptr[I + 1]; ++a) {
            const int32_t i = sy.child[a];
            const int32_t ri = pv.rank[i];
            int64_t co = 0;
            for (int64_t b = sy.child_ptr[J]; b < sy.child_ptr[J + 1]; ++b) {
              const int32_t j = sy.child[b];
              const int32_t rj = pv.rank[j];
              if (ri > 0 && rj > 0) {
                const int32_t hi = std::max(i, j), lo = std::min(i, j);
                const int64_t so = lay_prev.find(hi, lo);
                if (so >= 0) {
                  CopyDesc cd;
                  cd.src = arena_prev.as<double>() + lay_prev.base[lo] + so;
                  cd.lds = int32_t(lay_prev.H[lo]);
                  cd.trans = (i < j) ? 1 : 0;
                  cd.rows = ri;
                  cd.dst = dbase + ro + co * lay.H[J];
                  cd.ldd = int32_t(lay.H[J]);
                  const int32_t step = std::max(1, COPY_CHUNK / ri);  // column ranges of at most COPY_CHUNK entries
                  for (int32_t c0 = 0; c0 < rj; c0 += step) {
                    cd.c0 = c0;
                    cd.c1 = std::min(rj, c0 + step);
                    out.push_back(cd);
                  }
                }
              }
              co += rj;
            }
            ro += ri;
          }
        }
      };
      // large steps are planned by several host threads over contiguous ranges of
      // pairs (they only read); each thread then writes its part into the pinned
      // staging buffer at its offset, so the list is the same as one thread's
      const size_t npair = sy.before.size();
      const size_t nth = std::min<size_t>(8, std::max<size_t>(1, npair / 4096));
      if (nth == 1) {
        plan_copies(0, npair, copies);
        if ((st = upload(h, d_copy, copies)) != SPAND_OK) return st;
        launch_copy(d_copy.as<CopyDesc>(), int64_t(copies.size()), h->stream);
      } else {
        std::vector<std::vector<CopyDesc>> part(nth);
        {
          std::vector<std::thread> pool;
          for (size_t k = 1; k < nth; ++k)
            pool.emplace_back(plan_copies, npair * k / nth, npair * (k + 1) / nth, std::ref(part[k]));
          plan_copies(0, npair / nth, part[0]);
          for (std::thread& th : pool) th.join();
        }
        std::vector<size_t> off(nth + 1, 0);
        for (size_t k = 0; k < nth; ++k) off[k + 1] = off[k] + part[k].size();
        const size_t bytes = off[nth] * sizeof(CopyDesc);
        if ((st = dalloc(h, d_copy, bytes)) != SPAND_OK) return st;
        char* hp = h->stage.get(bytes);
        if (bytes > 0 && !hp) return set_err(h, SPAND_E_NOMEM, "pinned staging of " + std::to_string(bytes) + " bytes failed");
        {
          auto put = [&](size_t k) {
            if (!part[k].empty()) std::memcpy(hp + off[k] * sizeof(CopyDesc), part[k].data(), part[k].size() * sizeof(CopyDesc));
          };
          std::vector<std::thread> pool;
          for (size_t k = 1; k < nth; ++k) pool.emplace_back(put, k);
          put(0);
          for (std::thread& th : pool) th.join();
        }
        if (bytes > 0) {
          HIPCHK(hipMemcpyAsync(d_copy.p, hp, bytes, hipMemcpyHostToDevice, h->stream));
          launch_copy(d_copy.as<CopyDesc>(), int64_t(off[nth]), h->stream);
        }
      }
      HIPCHK(hipGetLastError());
    }

    // ---- elimination (Sec. 2.4)
    HIPCHK(hipEventRecord(ph[1], h->stream));
    HIPCHK(hipEventRecord(ph[2], h->stream));  // recorded again after the reduction
    std::vector<int64_t> c_off(ne), ed_off(ne);
    std::vector<int32_t> nN(ne);
    int64_t cbuf_total = 0, ed_total = 0;
    for (int32_t s = 0; s < ne; ++s) {
      nN[s] = int32_t(lay.H[s] - sn.size[s]);
      c_off[s] = cbuf_total;
      cbuf_total += int64_t(nN[s]) * nN[s];
      ed_off[s] = ed_total;
      ed_total += dinv_size(sn.size[s]);
      const double ns = sn.size[s], nn = nN[s];
      elim_flops += nn * ns * ns + nn * (nn + 1.0) * ns;
      m_F += int64_t(sn.size[s]) * (sn.size[s] + 1) / 2 + int64_t(sn.size[s]) * nN[s];
    }
    if ((st = dalloc(h, sn.edinv, size_t(ed_total) * sizeof(double))) != SPAND_OK) return st;
    DevBuf cbuf;
    if ((st = dalloc(h, cbuf, size_t(cbuf_total) * sizeof(double))) != SPAND_OK) return st;
    {
      std::vector<Front> fr;
      for (int32_t s = 0; s < ne; ++s)
        if (sn.size[s] > 0)
          fr.push_back(Front{E + lay.base[s], sn.edinv.as<double>() + ed_off[s], int32_t(lay.H[s]), sn.size[s],
                             int32_t(lay.H[s]), s});
      if ((st = blocked_cholesky(h, fr, d_fail_elim, gemm_prec)) != SPAND_OK) return st;
      GemmSeq syrk;
      for (int32_t s = 0; s < ne; ++s) {
        const int32_t ns = sn.size[s], nn = nN[s];
        GemmDesc y{};
        y.A = E + lay.base[s] + ns; y.lda = int32_t(lay.H[s]);
        y.B = y.A; y.ldb = y.lda;
        y.C = cbuf.as<double>() + c_off[s]; y.ldc = nn;
        y.M = nn; y.N = nn; y.K = ns;
        y.flags = G_TB | G_LOWERC;
        y.alpha = 1.0; y.beta = 0.0;
        syrk.add(y, 1);
      }
      syrk.end_launch(gemm_prec);
      if ((st = syrk.upload_all(h)) != SPAND_OK) return st;
      syrk.launch(h, 0);
      HIPCHK(hipGetLastError());
      // deterministic reduction of C_s into the targets
      struct Item { uint64_t tgt; int32_t s; int64_t coff; };
      std::vector<Item> items;
      for (int32_t s = 0; s < ne; ++s) {
        const int64_t b = sy.enb_ptr[s], e = sy.enb_ptr[s + 1];
        int64_t oa = 0;
        for (int64_t a = b; a < e; ++a) {
          const int32_t na = sy.enb[a];
          int64_t ob = 0;
          for (int64_t q = b; q <= a; ++q) {
            const int32_t nb = sy.enb[q];
            if (sn.size[na] > 0 && sn.size[nb] > 0 && sn.size[s] > 0)
              items.push_back(Item{pair_pack(na, nb), s, c_off[s] + oa + ob * nN[s]});
            ob += sn.size[nb];
          }
          oa += sn.size[na];
        }
      }
      std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.tgt < y.tgt; });
      std::vector<ReduceDesc> rds;
      std::vector<ContribDesc> cds2;
      for (size_t q = 0; q < items.size();) {
        size_t r = q;
        const int32_t ia = pair_i(items[q].tgt), ib = pair_j(items[q].tgt);
        ReduceDesc rd{};
        rd.T = A + lay.base[ib] + lay.find(ia, ib);
        rd.ldT = int32_t(lay.H[ib]);
        rd.rows = sn.size[ia];
        rd.cols = sn.size[ib];
        rd.diag = (ia == ib);
        rd.c_begin = int32_t(cds2.size());
        while (r < items.size() && items[r].tgt == items[q].tgt) {
          cds2.push_back(ContribDesc{cbuf.as<double>() + items[r].coff, nN[items[r].s], 0});
          ++r;
        }
        rd.c_end = int32_t(cds2.size());
        // large blocks are split into ranges of entries, one workgroup each
        const int64_t cnt = int64_t(rd.rows) * rd.cols;
        for (int64_t e0 = 0; e0 < cnt; e0 += REDUCE_CHUNK) {
          rd.e0 = int32_t(e0);
          rd.e1 = int32_t(std::min<int64_t>(cnt, e0 + REDUCE_CHUNK));
          rds.push_back(rd);
        }
        q = r;
      }
      DevBuf drd, dcd;
      if ((st = upload(h, drd, rds)) != SPAND_OK) return st;
      if ((st = upload(h, dcd, cds2)) != SPAND_OK) return st;
      launch_reduce(drd.as<ReduceDesc>(), int32_t(rds.size()), dcd.as<ContribDesc>(), h->stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(ph[2], h->stream));
      elim_ran[t] = 1;
    }
    cbuf.release();

    // ---- scaling (Sec. 2.5) and sparsification (Sec. 2.6.1)
    sn.rank.assign(nc, -1);
    for (int32_t c = ne; c < nc; ++c) sn.rank[c] = sn.size[c];
    std::vector<int64_t> sc_off(nc, -1), sd_off(nc, -1), v_off(nc, -1), tau_off(nc, -1), t_off(nc, -1);
    std::vector<int32_t> nref(nc, 0);
    HIPCHK(hipEventRecord(ph[3], h->stream));
    HIPCHK(hipEventRecord(ph[4], h->stream));
    if (sparsify && nc > ne) {
      int64_t sc_total = 0, sd_total = 0;
      for (int32_t p = ne; p < nc; ++p) {
        if (sn.size[p] == 0) continue;
        sc_off[p] = sc_total;
        sc_total += int64_t(sn.size[p]) * sn.size[p];
        sd_off[p] = sd_total;
        sd_total += dinv_size(sn.size[p]);
        m_F += int64_t(sn.size[p]) * (sn.size[p] + 1) / 2;
      }
      if ((st = dalloc(h, sn.scale, size_t(sc_total) * sizeof(double))) != SPAND_OK) return st;
      if ((st = dalloc(h, sn.sdinv, size_t(sd_total) * sizeof(double))) != SPAND_OK) return st;
      double* SC = sn.scale.as<double>();
      double* SD = sn.sdinv.as<double>();
      std::vector<Front> fr;
      for (int32_t p = ne; p < nc; ++p)
        if (sn.size[p] > 0)
          fr.push_back(Front{A + lay.base[p], SD + sd_off[p], int32_t(lay.H[p]), sn.size[p], int32_t(lay.H[p]), p});
      if ((st = blocked_cholesky(h, fr, d_fail_scale, 0)) != SPAND_OK) return st;
      // L_p^{-1} for the apply (the identity solved against L_p), and L_i^{-1} from the
      // left on every block (i, p), in one blocked left solve
      std::vector<LeftBlock> lb;
      std::vector<IdentDesc> ids;
      for (int32_t p = ne; p < nc; ++p) {
        if (sn.size[p] == 0) continue;
        add_identity(ids, SC + sc_off[p], sn.size[p], sn.size[p]);
        lb.push_back(LeftBlock{SC + sc_off[p], A + lay.base[p], SD + sd_off[p], sn.size[p], int32_t(lay.H[p]),
                               sn.size[p], sn.size[p]});
        for (int64_t e = lay.pan_ptr[p] + 1; e < lay.pan_ptr[p + 1]; ++e) {
          const int32_t i = lay.prow[e];
          if (sn.size[i] == 0) continue;
          lb.push_back(LeftBlock{A + lay.base[p] + lay.proff[e], A + lay.base[i], SD + sd_off[i], int32_t(lay.H[p]),
                                 int32_t(lay.H[i]), sn.size[i], sn.size[p]});
        }
      }
      {
        DevBuf d1;
        if ((st = upload(h, d1, ids)) != SPAND_OK) return st;
        launch_set_identity(d1.as<IdentDesc>(), int32_t(ids.size()), h->stream);
        HIPCHK(hipGetLastError());
        if ((st = left_trsm(h, lb)) != SPAND_OK) return st;
      }
      std::vector<IdentDesc> did;
      for (int32_t p = ne; p < nc; ++p)
        if (sn.size[p] > 0) add_identity(did, A + lay.base[p], sn.size[p], int32_t(lay.H[p]));
      DevBuf d1;
      if ((st = upload(h, d1, did)) != SPAND_OK) return st;
      launch_set_identity(d1.as<IdentDesc>(), int32_t(did.size()), h->stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(ph[3], h->stream));

      // sparsification, colour by colour.  A_pn of interface p lives in the registers
      // of slabS[p] workgroups with tg[p] lanes per column.  Interfaces of one slab go
      // in one plain launch per team size; interfaces of several slabs go in one
      // cooperative launch per colour, as rounds of at most the co-resident number of
      // workgroups.
      std::vector<int64_t> ncols(nc, 0);
      int32_t ncolour = 0;
      int64_t house_total = 0, xch_total = 0;
      std::vector<int64_t> xch_off(nc, -1);
      std::vector<int32_t> slabS(nc, 0), tg(nc, 0), nseg(nc, 0);
      std::vector<char> wide(nc, 0);  // single slab of the wide layout (teams of 2)
      std::vector<int32_t> rlay(nc, 0);  // register layout of a multi-slab interface
      for (int32_t p = ne; p < nc; ++p) {
        for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e)
          if (sn.size[sy.nb[e]] > 0) {
            ncols[p] += sn.size[sy.nb[e]];
            nseg[p]++;
          }
        if (sn.size[p] == 0 || ncols[p] == 0) continue;
        ncolour = std::max(ncolour, sy.colour[p] + 1);
        const int64_t m = sn.size[p];
        const int32_t G = cpqr_team(sn.size[p]);
        if (G < 0)
          return set_err(h, SPAND_E_INVALID, "interface of " + std::to_string(m) +
                                                 " dofs exceeds the largest CPQR team (2048 rows)");
        tg[p] = G;
        const int64_t cap = cpqr_capacity(G);
        slabS[p] = int32_t((ncols[p] + cap - 1) / cap);
        if (slabS[p] > 1 && G == 2 && m <= cpqr_wide_rows() && ncols[p] <= cpqr_wide_capacity()) {
          wide[p] = 1;  // fits one workgroup of the wide layout: no exchange between slabs
          slabS[p] = 1;
        }
        if (slabS[p] > 1) {  // layout 1 when it needs fewer slabs (and still more than one)
          const int32_t G1 = cpqr_team(sn.size[p], 1);
          if (G1 > 0) {
            const int64_t cap1 = cpqr_capacity(G1, 1);
            const int32_t S1 = int32_t((ncols[p] + cap1 - 1) / cap1);
            if (S1 > 1 && S1 < slabS[p]) {
              rlay[p] = 1;
              tg[p] = G1;
              slabS[p] = S1;
            }
          }
          xch_off[p] = xch_total;
          xch_total += 3 * int64_t(slabS[p]) * cpqr_record(tg[p], rlay[p]);  // three exchange buffers
        }
        const int64_t kmax = std::min<int64_t>(sn.size[p], ncols[p]);
        v_off[p] = house_total;
        house_total += int64_t(sn.size[p]) * kmax;
        tau_off[p] = house_total;
        house_total += kmax;
        t_off[p] = house_total;  // compact WY factor T (r x r, r <= kmax)
        house_total += kmax * kmax;
      }
      if ((st = dalloc(h, sn.house, size_t(house_total) * sizeof(double))) != SPAND_OK) return st;
      DevBuf xchb, curb, nrefb, errb;
      if ((st = dalloc(h, xchb, size_t(xch_total) * sizeof(double))) != SPAND_OK) return st;
      // the exchange headers start with tag 0; the first exchange of a buffer uses tag 1
      if (xch_total > 0) HIPCHK(hipMemsetAsync(xchb.p, 0, size_t(xch_total) * sizeof(double), h->stream));
      if ((st = dalloc(h, errb, sizeof(int32_t))) != SPAND_OK) return st;
      HIPCHK(hipMemsetAsync(errb.p, 0, sizeof(int32_t), h->stream));
      // current sizes: interfaces shrink to their rank as their colour class finishes
      if ((st = upload(h, curb, sn.size)) != SPAND_OK) return st;
      if ((st = upload(h, nrefb, std::vector<int32_t>(nc, 0))) != SPAND_OK) return st;
      for (int32_t p = ne; p < nc; ++p)
        if (v_off[p] >= 0) ++cpqr_ifaces[slabS[p] > 1 ? 2 + rlay[p] : (wide[p] ? 1 : 0)];
      std::vector<std::vector<int32_t>> by_colour(ncolour);
      for (int32_t p = ne; p < nc; ++p)
        if (v_off[p] >= 0) by_colour[sy.colour[p]].push_back(p);
      struct CpqrLaunch {
        bool multi;
        int32_t G, nslab, nround;
        size_t lds, d0, s0;
      };
      std::vector<CpqrLaunch> launches;
      std::vector<SparsDesc> all_sds;
      std::vector<SegDesc> all_segs;
      std::vector<SlabRef> all_slabs;
      size_t nlaunch = 0;
      // launch groups of one colour: single-slab interfaces per team size G
      // (group G), the wide single-slab ones (group 128), then every multi-slab
      // interface of the colour together (group 256)
      for (int32_t c = 0; c < ncolour; ++c) {
        if (by_colour[c].empty()) continue;
        for (int32_t grp = 1; grp <= 256; grp <<= 1) {
          const bool multi = grp == 256, wgrp = grp == 128;
          std::vector<int32_t> plist;
          for (int32_t p : by_colour[c])
            if (multi ? slabS[p] > 1 : wgrp ? wide[p] != 0 : (slabS[p] == 1 && !wide[p] && tg[p] == grp))
              plist.push_back(p);
          if (plist.empty()) continue;
          // largest first: interfaces of similar step counts share a launch
          std::stable_sort(plist.begin(), plist.end(), [&](int32_t x, int32_t y) {
            if (multi) return sn.size[x] > sn.size[y];
            return int64_t(sn.size[x]) * ncols[x] > int64_t(sn.size[y]) * ncols[y];
          });
          size_t lds = 0;
          for (int32_t p : plist)
            lds = std::max(lds, wgrp ? cpqr_wide_lds_bytes(nseg[p]) : cpqr_lds_bytes(tg[p], rlay[p], nseg[p]));
          int cap = INT_MAX;
          if (multi) {
            cap = cpqr_max_coresident(lds);
            if (cap <= 0) return set_err(h, SPAND_E_HIP, "occupancy query for the CPQR kernel failed");
          }
          // The chunks of at most cap co-resident slabs: one plain launch each for the
          // single-slab interfaces; for the multi-slab ones, the rounds of one launch.
          CpqrLaunch L{};
          L.multi = multi;
          L.G = multi ? 0 : grp;  // 128: the wide layout
          L.lds = lds;
          L.d0 = all_sds.size();
          std::vector<std::vector<SlabRef>> rounds;
          size_t pos = 0;
          while (pos < plist.size()) {
            std::vector<SlabRef> rd;
            while (pos < plist.size()) {
              const int32_t p = plist[pos];
              if (multi && slabS[p] > cap)
                return set_err(h, SPAND_E_INVALID, "interface needs more co-resident workgroups than the GPU holds");
              if (multi && !rd.empty() && int64_t(rd.size()) + slabS[p] > cap) break;
              SparsDesc d{};
              d.V = sn.house.as<double>() + v_off[p];
              d.tau = sn.house.as<double>() + tau_off[p];
              d.diag = A + lay.base[p];
              d.ldd = int32_t(lay.H[p]);
              d.m = sn.size[p];
              d.id = p;
              d.S = slabS[p];
              d.G = tg[p];
              d.lay = rlay[p];
              if (multi) d.xch = xchb.as<double>() + xch_off[p];
              d.seg_begin = int32_t(all_segs.size());
              for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e) {
                const int32_t q = sy.nb[e];
                if (sn.size[q] == 0) continue;
                SegDesc g{};
                if (q < p) {  // block (p, q) in panel q
                  g.blk = A + lay.base[q] + lay.find(p, q);
                  g.ld = int32_t(lay.H[q]);
                  g.trans = 0;
                } else {      // block (q, p) in panel p holds A_pq^T
                  g.blk = A + lay.base[p] + lay.find(q, p);
                  g.ld = int32_t(lay.H[p]);
                  g.trans = 1;
                }
                g.q = q;
                all_segs.push_back(g);
              }
              d.seg_end = int32_t(all_segs.size());
              for (int32_t w = 0; w < slabS[p]; ++w) rd.push_back(SlabRef{int32_t(all_sds.size() - L.d0), w});
              all_sds.push_back(d);
              ++pos;
            }
            rounds.push_back(std::move(rd));
          }
          if (!multi) {
            for (const auto& rd : rounds) {
              CpqrLaunch P = L;
              P.s0 = all_slabs.size();
              P.nslab = int32_t(rd.size());
              P.nround = 1;
              all_slabs.insert(all_slabs.end(), rd.begin(), rd.end());
              launches.push_back(P);
            }
          } else {
            // List scheduling over the co-resident workgroups: each interface, in
            // plist order, takes the slabS workgroups that free up first, by an
            // estimate of the steps (min(m, ncols) bounds the rank).  A workgroup runs
            // its slabs in that same order, so the earliest unfinished interface has
            // all its slabs at the heads of their lists: no cycle of waits.
            std::vector<std::pair<const SlabRef*, int32_t>> ifs;  // first slab, count
            for (const auto& rd : rounds)
              for (size_t k = 0; k < rd.size();) {
                size_t e = k;
                while (e < rd.size() && rd[e].desc == rd[k].desc) ++e;
                ifs.emplace_back(&rd[k], int32_t(e - k));
                k = e;
              }
            if (ifs.size() != plist.size()) return set_err(h, SPAND_E_INVALID, "sparsification schedule: interfaces and slabs disagree");
            size_t total = 0;
            for (const auto& f : ifs) total += size_t(f.second);
            const size_t grid = std::min(total, size_t(cap));
            std::vector<std::vector<SlabRef>> lists(grid);
            // min-heap of (time the workgroup frees up, workgroup)
            using Slot = std::pair<int64_t, int32_t>;
            std::vector<Slot> heap(grid);
            for (size_t b = 0; b < grid; ++b) heap[b] = Slot{0, int32_t(b)};
            std::make_heap(heap.begin(), heap.end(), std::greater<Slot>());
            std::vector<int32_t> wg;
            for (size_t q = 0; q < ifs.size(); ++q) {
              const int32_t p = plist[q];
              const int32_t S = ifs[q].second;
              wg.clear();
              int64_t t = 0;
              for (int32_t k = 0; k < S; ++k) {
                std::pop_heap(heap.begin(), heap.end(), std::greater<Slot>());
                t = std::max(t, heap.back().first);
                wg.push_back(heap.back().second);
                heap.pop_back();
              }
              t += std::min<int64_t>(sn.size[p], ncols[p]);
              for (int32_t k = 0; k < S; ++k) {
                lists[wg[k]].push_back(ifs[q].first[k]);
                heap.push_back(Slot{t, wg[k]});
                std::push_heap(heap.begin(), heap.end(), std::greater<Slot>());
              }
            }
            size_t nround = 0;
            for (const auto& l : lists) nround = std::max(nround, l.size());
            L.s0 = all_slabs.size();
            L.nslab = int32_t(grid);
            L.nround = int32_t(nround);
            for (size_t k = 0; k < nround; ++k)
              for (size_t b = 0; b < grid; ++b) all_slabs.push_back(k < lists[b].size() ? lists[b][k] : SlabRef{-1, 0});
            launches.push_back(L);
          }
        }
      }
      // every launch of the step is planned: one upload, then the launches back to back
      DevBuf a, b, sl;
      if ((st = upload(h, a, all_sds)) != SPAND_OK) return st;
      if ((st = upload(h, b, all_segs)) != SPAND_OK) return st;
      if ((st = upload(h, sl, all_slabs)) != SPAND_OK) return st;
      for (const CpqrLaunch& L : launches) {
        hipEvent_t e0, e1;
        HIPCHK(evpool.get(2 * nlaunch, &e0));
        HIPCHK(evpool.get(2 * nlaunch + 1, &e1));
        HIPCHK(hipEventRecord(e0, h->stream));
        const SparsDesc* dd = a.as<SparsDesc>() + L.d0;
        const SlabRef* ss = sl.as<SlabRef>() + L.s0;
        hipError_t le = L.multi ? launch_cpqr_multi(dd, ss, L.nslab, L.nround, b.as<SegDesc>(), tol,
                                                    curb.as<int32_t>(), nrefb.as<int32_t>(), errb.as<int32_t>(),
                                                    L.lds, h->stream)
                    : L.G == 128 ? launch_cpqr_one_wide(dd, ss, L.nslab, b.as<SegDesc>(), tol, curb.as<int32_t>(),
                                                        nrefb.as<int32_t>(), errb.as<int32_t>(), L.lds, h->stream)
                                 : launch_cpqr_one(L.G, dd, ss, L.nslab, b.as<SegDesc>(), tol, curb.as<int32_t>(),
                                                   nrefb.as<int32_t>(), errb.as<int32_t>(), L.lds, h->stream);
        if (le != hipSuccess)
          return set_err(h, SPAND_E_HIP, std::string("sparsification launch: ") + hipGetErrorString(le));
        HIPCHK(hipEventRecord(e1, h->stream));
        ++nlaunch;
      }
      std::vector<int32_t> rk(nc, -1);
      HIPCHK(hipEventRecord(ph[4], h->stream));
      if ((st = flush_t()) != SPAND_OK) return st;      // the previous step's, while this one runs
      if ((st = flush_apply()) != SPAND_OK) return st;
      if ((st = check_flags(t)) != SPAND_OK) return st;
      flags_read = true;
      HIPCHK(hipMemcpyAsync(rk.data(), curb.p, size_t(nc) * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipMemcpyAsync(nref.data(), nrefb.p, size_t(nc) * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      int32_t serr = 0;
      HIPCHK(hipMemcpyAsync(&serr, errb.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      if (serr) return set_err(h, SPAND_E_HIP, "sparsification slab exchange timed out");
      for (size_t q = 0; q < nlaunch; ++q) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, evpool.ev[2 * q], evpool.ev[2 * q + 1]));
        cpqr_ms += ms;
      }
      cpqr_launches += int64_t(nlaunch);
      std::vector<TDesc> tds;
      for (int32_t p = ne; p < nc; ++p)
        if (v_off[p] >= 0) {
          sn.rank[p] = rk[p];
          const int64_t r = nref[p];
          {
            // sum over steps j < r of 2 (m-j)(n-j) + 4 (m-j)(n-j-1) + 3 (m-j)
            // = 6 (m-j)(n-j) - (m-j), in closed form (exact in 64-bit integers)
            const int64_t m = sn.size[p], nq = ncols[p];
            const int64_t s1 = r * (r - 1) / 2, s2 = (r - 1) * r * (2 * r - 1) / 6;
            const int64_t f = 6 * (r * m * nq - (m + nq) * s1 + s2) - (r * m - s1);
            cpqr_flops += double(f);
            if (r < std::min<int64_t>(m, nq)) cpqr_flops += 2.0 * double(m - r) * double(nq - r);
          }
          m_F += (2 * int64_t(sn.size[p]) - r + 1) * r / 2 + r;
          if (r > 0)
            tds.push_back(TDesc{sn.house.as<double>() + v_off[p], sn.house.as<double>() + tau_off[p],
                                sn.house.as<double>() + t_off[p], sn.size[p], int32_t(r)});
        }
      // the compact-WY factors are only read by the apply: they are built while the
      // next step runs (flush_t)
      t_pending = std::move(tds);
    }
    if (t <= 32) h->stats.step_m_F[t - 1] = m_F;

    if (!flags_read) {
      if ((st = flush_t()) != SPAND_OK) return st;
      if ((st = flush_apply()) != SPAND_OK) return st;
      if ((st = check_flags(t)) != SPAND_OK) return st;
    }
    pending = ApplyPlan{t, std::move(ed_off), std::move(sc_off), std::move(v_off), std::move(t_off), std::move(nN),
                        std::move(nref)};

    arena_prev = std::move(arena);
    lay_prev = std::move(lay);
  }
  if ((st = flush_t()) != SPAND_OK) return st;
  if ((st = flush_apply()) != SPAND_OK) return st;
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int32_t t = 1; t <= Lv; ++t) {  // phase times from the events of every step
    hipEvent_t ph[5];
    for (int q = 0; q < 5; ++q) ph[q] = phev.ev[5 * size_t(t - 1) + q];
    float ms[4] = {0.f, 0.f, 0.f, 0.f};
    HIPCHK(hipEventElapsedTime(&ms[0], ph[0], ph[1]));
    HIPCHK(hipEventElapsedTime(&ms[1], ph[1], ph[2]));
    HIPCHK(hipEventElapsedTime(&ms[2], ph[2], ph[3]));
    HIPCHK(hipEventElapsedTime(&ms[3], ph[3], ph[4]));
    if (t <= 32)
      for (int q = 0; q < 4; ++q) h->stats.step_phase_seconds[t - 1][q] = 1e-3 * ms[q];
    if (elim_ran[t]) elim_ms += ms[1];
  }
  arena_prev.release();
  h->stats.m_F = m_F;
  h->stats.s_top = s_top;
  h->stats.schur_flops = elim_flops;
  h->stats.schur_seconds = elim_ms * 1e-3;
  h->stats.cpqr_flops = cpqr_flops;
  h->stats.cpqr_seconds = cpqr_ms * 1e-3;
  h->stats.cpqr_launches = cpqr_launches;
  for (int q = 0; q < 4; ++q) h->stats.cpqr_interfaces[q] = cpqr_ifaces[q];
  for (int q = 0; q < 3; ++q) h->stats.apply_interfaces[q] = 0;
  for (const StepNum& sn : h->num) {
    h->stats.apply_interfaces[0] += sn.n_iface1;
    h->stats.apply_interfaces[1] += sn.n_iface2;
    h->stats.apply_interfaces[2] += sn.n_scale;
  }
  return SPAND_OK;
}

}  // namespace spand
