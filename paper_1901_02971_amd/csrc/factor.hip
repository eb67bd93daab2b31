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

// Host-to-device copy of a descriptor list through pinned staging, with the pinned
// copy done by several threads when the list is large.
template <typename T>
spand_status upload_big(spand_ctx* h, DevBuf& b, const std::vector<T>& v) {
  const size_t bytes = v.size() * sizeof(T);
  spand_status st = dalloc(h, b, bytes);
  if (st != SPAND_OK || bytes == 0) return st;
  char* hp = h->stage.get(bytes);
  if (!hp) return set_err(h, SPAND_E_NOMEM, "pinned staging of " + std::to_string(bytes) + " bytes failed");
  const size_t nth = std::min<size_t>(8, std::max<size_t>(1, bytes >> 22));
  if (nth == 1) {
    std::memcpy(hp, v.data(), bytes);
  } else {
    std::vector<std::thread> pool;
    auto put = [&](size_t k) {
      const size_t a = v.size() * k / nth, e = v.size() * (k + 1) / nth;
      std::memcpy(hp + a * sizeof(T), v.data() + a, (e - a) * sizeof(T));
    };
    for (size_t k = 1; k < nth; ++k) pool.emplace_back(put, k);
    put(0);
    for (std::thread& th : pool) th.join();
  }
  HIPCHK(hipMemcpyAsync(b.p, hp, bytes, hipMemcpyHostToDevice, h->stream));
  return SPAND_OK;
}

// Column-panel layout of one step.  Panels of eliminated clusters (j < ne) are
// placed in the persistent elimination buffer, the others in the step arena.
struct Layout {
  int32_t ne = 0;
  std::vector<int64_t> pan_ptr;  // nc+1
  std::vector<int32_t> prow;     // row cluster of each panel entry (diagonal first)
  std::vector<int64_t> proff;    // row offset of each entry inside its panel
  std::vector<int64_t> H;        // leading dimension of each panel: its height rounded up to 16
                                 // entries, so every column starts on a 128-byte line
  std::vector<int64_t> Hr;       // panel heights (rows in use)
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
  L.Hr.assign(nc, 0);
  L.base.assign(nc, 0);
  int64_t te = 0, ta = 0;
  for (int32_t j = 0; j < nc; ++j) {
    int64_t h = 0;
    for (int64_t e = L.pan_ptr[j]; e < L.pan_ptr[j + 1]; ++e) {
      L.proff[e] = h;
      h += size[L.prow[e]];
    }
    L.Hr[j] = h;
    L.H[j] = (h + 15) / 16 * 16;
    h = L.H[j];
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
// The products of a launch are numbered at end_launch, once its arithmetic (and so
// its output tile: the sequence's variant, or 64 for BF16x3) is known.
struct GemmSeq {
  explicit GemmSeq(int variant_ = 0) : variant(variant_), ts0(gemm_variant_tile(variant_)) {}
  int variant, ts0;
  std::vector<GemmDesc> d;
  std::vector<int64_t> cut;  // tile range end of every launch
  std::vector<int> prec;
  int64_t ntiles = 0;
  size_t open = 0;  // first product of the launch being filled
  DevBuf dd, dmap;
  // Products go straight into the list with their first tile number for the tuned
  // tile; a launch of BF16x3 products (64-wide tiles only) renumbers its own.
  void add(GemmDesc g, int part) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return;
    g.part = part;
    g.ts = ts0;
    g.t0 = ntiles;
    ntiles += gemm_tiles(g.M, g.N, part, ts0);
    d.push_back(g);
  }
  void end_launch(int p) {
    if (p == 2 && ts0 != 64) {
      ntiles = cut.empty() ? 0 : cut.back();
      for (size_t k = open; k < d.size(); ++k) {
        d[k].ts = 64;
        d[k].t0 = ntiles;
        ntiles += gemm_tiles(d[k].M, d[k].N, d[k].part, 64);
      }
    }
    open = d.size();
    cut.push_back(ntiles);
    prec.push_back(p);
  }
  spand_status upload_all(spand_ctx* h) {
    spand_status st = upload_big(h, dd, d);
    if (st != SPAND_OK) return st;
    if ((st = dalloc(h, dmap, size_t(ntiles) * sizeof(int32_t))) != SPAND_OK) return st;
    launch_expand_tiles(dd.as<GemmDesc>(), int32_t(d.size()), dmap.as<int32_t>(), h->stream);
    return SPAND_OK;
  }
  void launch(spand_ctx* h, size_t q) const {
    const int64_t b = q ? cut[q - 1] : 0;
    if (cut[q] > b) launch_gemm(dd.as<GemmDesc>(), dmap.as<int32_t>(), b, cut[q] - b, prec[q], variant, h->stream);
  }
};

// One panel factorized by the blocked Cholesky: diagonal n x n on top, m rows in all.
struct Front {
  double* P;
  double* dinv;  // ceil(n / CHOL_NB) blocks of CHOL_NB^2 doubles
  int32_t ld, n, m, id;
  int32_t* fail;  // the problem's failure flag word (atomicMin of the cluster id)
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
spand_status blocked_cholesky(spand_ctx* h, const std::vector<Front>& F, int prec_below) {
  const int32_t CHOL_GROUP = std::max(1, h->tune.chol_group);
  int32_t nmax = 0;
  for (const Front& f : F) nmax = std::max(nmax, f.n);
  std::vector<PotrfDesc> pd;
  std::vector<PanelDesc> td;
  std::vector<int64_t> pcut, tcut;
  GemmSeq g(h->tune.gemm_chol);
  for (int32_t kb = 0; kb < nmax; kb += CHOL_NB) {
    for (const Front& f : F) {
      if (f.n <= kb) continue;
      const int32_t w = std::min(CHOL_NB, f.n - kb);
      double* Dk = f.dinv + int64_t(kb / CHOL_NB) * CHOL_NB * CHOL_NB;
      pd.push_back(PotrfDesc{f.P + kb + int64_t(kb) * f.ld, Dk, f.fail, f.ld, w, f.id, 0});
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
    launch_potrf_diag(dp.as<PotrfDesc>() + pb, int32_t(pcut[q] - pb), h->stream);
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
  // X[kb:kb+w, :] <- L_kk^{-1} X[kb:kb+w, :] is a product with the lower-triangular
  // inverse, done in place by the batched GEMM: with w <= 64 rows one 64 x 64 output
  // tile holds every row of its columns, so the workgroup that writes them has read
  // them all (the 64-wide tile, whatever the tuned tile of the updates).  The
  // products of an entry are added in k order, as the substitution adds them.
  GemmSeq gd(0), g(h->tune.gemm_scale);
  size_t nprod = 0;
  for (const LeftBlock& b : B) nprod += size_t((b.nrows + CHOL_NB - 1) / CHOL_NB);
  gd.d.reserve(nprod);
  g.d.reserve(nprod);
  for (int32_t kb = 0; kb < nmax; kb += CHOL_NB) {
    // grouped as in blocked_cholesky: inside a group only the next block row is
    // updated, at the group's end every row below, at depth CHOL_GROUP NB
    const int32_t kblk = kb / CHOL_NB;
    const bool pair = (kblk % CHOL_GROUP) == CHOL_GROUP - 1;
    const int32_t kg = (kblk / CHOL_GROUP) * CHOL_GROUP * CHOL_NB;
    for (const LeftBlock& b : B) {
      if (b.nrows <= kb) continue;
      const int32_t w = std::min(CHOL_NB, b.nrows - kb);
      GemmDesc s{};
      s.A = b.dinv + int64_t(kb / CHOL_NB) * CHOL_NB * CHOL_NB; s.lda = w;
      s.B = b.X + kb; s.ldb = b.ldx;
      s.C = b.X + kb; s.ldc = b.ldx;
      s.M = w; s.N = b.ncols; s.K = w;
      s.flags = G_TRIA; s.alpha = 1.0; s.beta = 0.0;
      gd.add(s, 0);
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
    gd.end_launch(0);
    g.end_launch(0);
  }
  spand_status st;
  if ((st = gd.upload_all(h)) != SPAND_OK) return st;
  if ((st = g.upload_all(h)) != SPAND_OK) return st;
  for (size_t q = 0; q < g.cut.size(); ++q) {
    gd.launch(h, q);
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
  std::vector<int64_t> iso_off;  // offset of L_s^{-1} in the step's iso buffer, -1 if none
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
  const std::vector<int64_t>& iso_off = pl.iso_off;
  auto isolated = [&](int32_t s) { return s < int32_t(iso_off.size()) && iso_off[s] >= 0; };
  for (int32_t s = 0; s < ne; ++s) {
    ElimAp e{};
    e.L = E + lay.base[s];
    e.G = E + lay.base[s] + sn.size[s];
    e.Dinv = sn.edinv.as<double>() + ed_off[s];
    e.ld = int32_t(lay.H[s]);
    // a cluster with no neighbours and an explicit inverse goes through the scaling
    // kernels below (x_s <- L_s^{-1} x_s, and its transpose backward), not through
    // the blocked substitution
    e.ns = isolated(s) ? 0 : sn.size[s];
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
    e.ytmp = tmp;
    tmp += e.nN;
    sn.h_elim.push_back(e);
  }
  sn.tmp_elim = tmp;
  // forward products y_s = G_s (L_s^{-1} x_s): 64-row tiles at multiples of 64 panel
  // rows covering the rows of G (ns .. ns + nN)
  sn.h_ftile.clear();
  for (int32_t s = 0; s < ne; ++s) {
    const ElimAp& e = sn.h_elim[s];
    if (e.ns == 0 || e.nN == 0) continue;
    for (int32_t r0 = e.ns / 64 * 64; r0 < e.ns + e.nN; r0 += 64) sn.h_ftile.push_back(FwdTile{s, r0});
  }
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
      sn.h_contrib.push_back(TargetContrib{sn.h_elim[s].ytmp + tis[r].row});
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
      f.ldl = pad16(f.np);
      f.ldv = pad16(f.np);
      f.slot_p = sn.slot_ptr[p];
      if (v_off[p] >= 0 && nref[p] > 0) {
        f.V = sn.house.as<double>() + v_off[p];
        f.T = sn.house.as<double>() + t_off[p];
        f.r = nref[p];
        f.ldt = pad16(f.r);
      }
      (f.np <= 64 ? if1 : if2).push_back(f);
      continue;
    }
    if (sc_off[p] >= 0) {
      ScaleAp a{};
      a.Linv = sn.scale.as<double>() + sc_off[p];
      a.np = sn.size[p];
      a.ldl = pad16(a.np);
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
      hp.ldv = pad16(hp.np);
      hp.ldt = pad16(hp.r);
      hp.slot_p = sn.slot_ptr[p];
      hp.tmp = tmp3;
      tmp3 += 2 * int64_t(nref[p]);
      const int32_t hid = int32_t(sn.h_house.size());
      for (int32_t j0 = 0; j0 < hp.r; j0 += 64) sn.h_hr.push_back(HouseTile{hid, j0});
      for (int32_t r0 = 0; r0 < hp.np; r0 += 64) sn.h_hv.push_back(HouseTile{hid, r0});
      sn.h_house.push_back(hp);
    }
  }
  sn.n_iso = 0;
  for (int32_t s = 0; s < ne; ++s) {
    if (!isolated(s) || sn.size[s] == 0) continue;
    ++sn.n_iso;
    ScaleAp a{};
    a.Linv = sn.iso.as<double>() + iso_off[s];
    a.np = sn.size[s];
    a.ldl = pad16(a.np);
    a.slot_p = sn.slot_ptr[s];
    a.tmp = tmp2;
    tmp2 += sn.size[s];
    const int32_t sid = int32_t(sn.h_scale.size());
    for (int32_t r0 = 0; r0 < a.np; r0 += 64) sn.h_stile.push_back(ScaleTile{sid, r0});
    sn.h_sgather.insert(sn.h_sgather.end(), sn.slot.begin() + sn.slot_ptr[s],
                        sn.slot.begin() + sn.slot_ptr[s] + sn.size[s]);
    sn.h_scale.push_back(a);
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
  sn.n_ftile = int32_t(sn.h_ftile.size());
  sn.n_stile = int32_t(sn.h_stile.size());
  sn.sgather_len = int64_t(sn.h_sgather.size());
  sn.n_hr = int32_t(sn.h_hr.size());
  sn.n_hv = int32_t(sn.h_hv.size());
  if ((st = upload(h, sn.d_slot, sn.slot)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_nslot, nslot)) != SPAND_OK) return st;
  sn.h_nslot = std::move(nslot);
  if ((st = upload(h, sn.d_elim, sn.h_elim)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_target, sn.h_target)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_contrib, sn.h_contrib)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_scale, sn.h_scale)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_house, sn.h_house)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_etile, sn.h_etile)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_ftile, sn.h_ftile)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_stile, sn.h_stile)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_sgather, sn.h_sgather)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_hr, sn.h_hr)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_hv, sn.h_hv)) != SPAND_OK) return st;
  if ((st = upload(h, sn.d_iface, sn.h_iface)) != SPAND_OK) return st;
  sn.n_interp = int32_t(sn.h_interp.size());
  if ((st = upload(h, sn.d_interp, sn.h_interp)) != SPAND_OK) return st;
  return SPAND_OK;
}

namespace {

// One problem of a factorization run: its handle and what the run keeps for it
// across the steps.  A run factors one problem, or several in lockstep (step t of
// every problem together), with the work of all of them in shared launches.
struct Prob {
  spand_ctx* h = nullptr;
  const double* values = nullptr;
  int32_t L = 0;
  bool live = true;             // false once it failed (its handle holds the error)
  int32_t* flags = nullptr;     // [0] elimination failure id, [1] scaling failure id, [2] non-finite input,
                                // [3] interpolative sparsification failure id
  DevBuf arena, arena_prev;     // trailing panels of the remaining clusters, this and the last step
  Layout lay, lay_prev;
  ApplyPlan pending;            // apply descriptors of the last step, built while this one runs
  std::vector<TDesc> t_pending; // compact-WY factors of the last step's interfaces
  int64_t m_F = 0;
  double elim_flops = 0.0, cpqr_flops = 0.0;
  int64_t cpqr_ifaces[4] = {0, 0, 0, 0};  // single, wide, multi (32 x 2), multi (20 x 3)
  int32_t s_top = 0;
  std::vector<int32_t> frozen;  // vertices in the order the steps freeze them (freeze_order)
  size_t frozen_up = 0;         // entries of frozen already copied to the device (d_inv)
  // this step
  bool on = false, sparsify = false;
  int64_t cbase = 0;            // first entry of this problem's clusters in the run's size and rank arrays
  std::vector<int64_t> c_off, ed_off, sc_off, sd_off, v_off, tau_off, t_off, xch_off, ncols, iso_off;
  std::vector<int32_t> nN, nref, slabS, tg, nseg, rlay, kslots;
  std::vector<char> wide, big;
  int64_t cpqr_big = 0;         // interfaces of the global-memory CPQR kernel
  int32_t cpqr_one_launch = 0;  // steps whose CPQRs ran in one launch
  int32_t cpqr_slot = 0;        // interfaces whose CPQR teams used the LDS column slot
  DevBuf cbuf;
};

// Compact-WY factors T_p (Q = I - V T V^T) of interfaces of any problems of the run:
// S = V^T V (MFMA, upper tiles), the 64-wide diagonal blocks of T in LDS, then
// T[:J0, J] = -T[:J0, :J0] (S[:J0, J] T_JJ) by block columns.
spand_status build_t_factors(spand_ctx* h, const std::vector<TDesc>& tds) {
  if (tds.empty()) return SPAND_OK;
  spand_status st = SPAND_OK;
  GemmSeq vtv(h->tune.gemm_scale);
  for (const TDesc& td : tds) {
    GemmDesc q{};
    q.A = td.V; q.lda = td.ldv;
    q.B = td.V; q.ldb = td.ldv;
    q.C = td.T; q.ldc = td.ldt;
    q.M = td.r; q.N = td.r; q.K = td.m;
    q.flags = G_TA;
    q.alpha = 1.0; q.beta = 0.0;
    vtv.add(q, 2);
  }
  vtv.end_launch(0);
  if ((st = vtv.upload_all(h)) != SPAND_OK) return st;
  vtv.launch(h, 0);
  HIPCHK(hipGetLastError());
  std::vector<TBlock> tbs;
  int32_t rmax = 0;
  int64_t x_total = 0;
  std::vector<int64_t> x_off(tds.size(), -1);
  for (size_t q = 0; q < tds.size(); ++q) {
    const TDesc& td = tds[q];
    for (int32_t j0 = 0; j0 < td.r; j0 += 64) tbs.push_back(TBlock{td.T, td.tau, td.r, j0, td.ldt, 0});
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
    GemmSeq tg2(h->tune.gemm_scale);
    for (int32_t j0 = 64; j0 < rmax; j0 += 64) {
      for (size_t q = 0; q < tds.size(); ++q) {
        const TDesc& td = tds[q];
        if (td.r <= j0) continue;
        const int32_t w = std::min(64, td.r - j0);
        GemmDesc g{};  // X = S[:j0, J] T_JJ
        g.A = td.T + int64_t(j0) * td.ldt; g.lda = td.ldt;
        g.B = td.T + j0 + int64_t(j0) * td.ldt; g.ldb = td.ldt;
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
        g.A = td.T; g.lda = td.ldt;
        g.B = xb.as<double>() + x_off[q]; g.ldb = td.r;
        g.C = td.T + int64_t(j0) * td.ldt; g.ldc = td.ldt;
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
}

// Sizes and slots of step t of one problem, from the ranks kept at step t-1.
void step_sizes(const SymStep& sy, int32_t t, std::vector<StepNum>& num) {
  StepNum& sn = num[t - 1];
  const int32_t nc = sy.nc;
  sn.size.assign(nc, 0);
  sn.slot_ptr.assign(nc + 1, 0);
  if (t == 1) {
    for (int32_t c = 0; c < nc; ++c) sn.size[c] = int32_t(sy.child_ptr[c + 1] - sy.child_ptr[c]);
    sn.slot.assign(sy.child.begin(), sy.child.end());
    for (int32_t c = 0; c < nc; ++c) sn.slot_ptr[c + 1] = sy.child_ptr[c + 1];
    return;
  }
  const StepNum& pv = num[t - 2];
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

// Merge copies of step t (> 1) of one problem: parent blocks are the concatenation
// of the children's kept blocks (Sec. 2.7).  Large steps are planned by several host
// threads over contiguous ranges of block pairs; the list is the same as one thread's.
// The merge of one problem into step t: copy descriptors of the blocks of the previous
// step's kept dofs into the new panels, by cluster pairs of the new step.
struct MergeJob {
  const SymStep* sy;
  const StepNum* pv;
  const Layout* lay;
  const Layout* lay_prev;
  double *E, *A;
  const double* arena_prev;
  // the descriptors of pairs [q0, q1) (count only when dst is null); returns how many
  size_t plan(size_t q0, size_t q1, CopyDesc* dst) const {
    size_t n = 0;
    for (size_t q = q0; q < q1; ++q) {
      const uint64_t pr = sy->before[q];
      const int32_t I = pair_i(pr), J = pair_j(pr);
      double* dbase = dst ? lay->panel(J, E, A) + lay->find(I, J) : nullptr;
      int64_t ro = 0;
      for (int64_t a = sy->child_ptr[I]; a < sy->child_ptr[I + 1]; ++a) {
        const int32_t i = sy->child[a];
        const int32_t ri = pv->rank[i];
        int64_t co = 0;
        for (int64_t b = sy->child_ptr[J]; b < sy->child_ptr[J + 1]; ++b) {
          const int32_t j = sy->child[b];
          const int32_t rj = pv->rank[j];
          if (ri > 0 && rj > 0) {
            const int32_t hi = std::max(i, j), lo = std::min(i, j);
            const int64_t so = lay_prev->find(hi, lo);
            if (so >= 0) {
              const int32_t step = std::max(1, COPY_CHUNK / ri);  // column ranges of at most COPY_CHUNK entries
              if (!dst) {
                n += size_t((rj + step - 1) / step);
              } else {
                CopyDesc cd;
                cd.src = arena_prev + lay_prev->base[lo] + so;
                cd.lds = int32_t(lay_prev->H[lo]);
                cd.trans = (i < j) ? 1 : 0;
                cd.rows = ri;
                cd.dst = dbase + ro + co * lay->H[J];
                cd.ldd = int32_t(lay->H[J]);
                for (int32_t c0 = 0; c0 < rj; c0 += step) {
                  cd.c0 = c0;
                  cd.c1 = std::min(rj, c0 + step);
                  dst[n++] = cd;
                }
              }
            }
          }
          co += rj;
        }
        ro += ri;
      }
    }
    return n;
  }
};

// The copy descriptors of every merge job, counted and then written straight into
// the pinned staging (in job and pair order, the same list one thread would build) by
// up to 8 threads over ranges of cluster pairs; one upload.  Returns the count.
spand_status plan_merges(spand_ctx* h, const std::vector<MergeJob>& jobs, DevBuf& out, int64_t& count) {
  struct Range {
    size_t job, q0, q1, off, n;
  };
  std::vector<Range> rs;
  for (size_t k = 0; k < jobs.size(); ++k) {
    const size_t npair = jobs[k].sy->before.size();
    const size_t nr = std::min<size_t>(32, std::max<size_t>(1, npair / 2048));
    for (size_t c = 0; c < nr; ++c) rs.push_back(Range{k, npair * c / nr, npair * (c + 1) / nr, 0, 0});
  }
  const size_t nth = std::min<size_t>(8, rs.size());
  auto run = [&](auto&& fn) {
    if (nth <= 1) {
      for (size_t r = 0; r < rs.size(); ++r) fn(r);
      return;
    }
    std::vector<std::thread> pool;
    auto worker = [&](size_t w) {
      for (size_t r = w; r < rs.size(); r += nth) fn(r);
    };
    for (size_t w = 1; w < nth; ++w) pool.emplace_back(worker, w);
    worker(0);
    for (std::thread& th : pool) th.join();
  };
  run([&](size_t r) { rs[r].n = jobs[rs[r].job].plan(rs[r].q0, rs[r].q1, nullptr); });
  size_t total = 0;
  for (Range& r : rs) {
    r.off = total;
    total += r.n;
  }
  count = int64_t(total);
  if (total == 0) return SPAND_OK;
  const size_t bytes = total * sizeof(CopyDesc);
  spand_status st = dalloc(h, out, bytes);
  if (st != SPAND_OK) return st;
  CopyDesc* hp = reinterpret_cast<CopyDesc*>(h->stage.get(bytes));
  if (!hp) return set_err(h, SPAND_E_NOMEM, "pinned staging of " + std::to_string(bytes) + " bytes failed");
  run([&](size_t r) { (void)jobs[rs[r].job].plan(rs[r].q0, rs[r].q1, hp + rs[r].off); });
  HIPCHK(hipMemcpyAsync(out.p, hp, bytes, hipMemcpyHostToDevice, h->stream));
  return SPAND_OK;
}


// Interpolative sparsification (Sec. 2.6.2) of the interfaces of step t of one
// problem (after the scaling for InS), one colour class at a time: an interface's
// A_np takes the final sizes of the neighbours sparsified before it, and the launches
// after its CPQR need its rank on the host.  Per class: A_np of every interface
// gathered twice (the CPQR's work copy and a copy kept for the new rows), the
// truncated CPQR of every A_np with its pivots, one sync for the ranks, then for the
// interfaces that drop dofs, in shared launches: perm, T_cf, X = A_pp in (f, c)
// order, the congruence C_cf = A_cf - A_cc T, C_ff = A_ff - A_fc T - T^T C_cf, the
// blocked Cholesky of [C_ff; C_cf] (L_f and G_cf = C_cf L_f^{-T} in place), A_cc -=
// G G^T, and the write-back of A_cc and of the rows c of every A_pq, c first in
// pivot order (the apply moves the values of the interface the same way).
spand_status sparsify_interp(Prob& pb, int32_t t, double tol, double& cpqr_ms, int64_t& cpqr_launches) {
  spand_ctx* h = pb.h;
  const SymStep& sy = h->an.steps[t - 1];
  StepNum& sn = h->num[t - 1];
  const Layout& lay = pb.lay;
  double* A = pb.arena.as<double>();
  const int32_t nc = sy.nc, ne = sy.ne;
  std::vector<int32_t> cur(sn.size.begin(), sn.size.end());
  int32_t ncolour = 0;
  for (int32_t p = ne; p < nc; ++p) ncolour = std::max(ncolour, sy.colour[p] + 1);
  EventPool ev;
  spand_status st;
  for (int32_t colr = 0; colr < ncolour; ++colr) {
    struct It {
      int32_t p, m, np, G, r;
      bool big;
      int64_t ow, ov, otau, ox, opiv, ot;
    };
    std::vector<It> its;
    int64_t tw = 0, tv = 0, ttau = 0, tx = 0, tpiv = 0, bigmax = 0, bign = 0;
    for (int32_t p = ne; p < nc; ++p) {
      if (sy.colour[p] != colr || cur[p] == 0) continue;
      int64_t m = 0;
      for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e) m += cur[sy.nb[e]];
      if (m == 0) continue;  // no coupled dofs: p is left as it is
      const int32_t np = cur[p];
      if (np > INTERP_MAX_NP)
        return set_err(h, SPAND_E_INVALID, "interface of " + std::to_string(np) +
                                               " dofs exceeds the interpolative limit (" +
                                               std::to_string(INTERP_MAX_NP) + ")");
      if (m > cpqr_big_max_rows())
        return set_err(h, SPAND_E_INVALID, "A_np of " + std::to_string(m) + " rows exceeds the CPQR limit (" +
                                               std::to_string(cpqr_big_max_rows()) + " rows)");
      It it{};
      it.p = p;
      it.m = int32_t(m);
      it.np = np;
      it.G = cpqr_team(it.m);
      it.big = it.G < 0 || np > cpqr_capacity(it.G) || (h->tune.cpqr_big_min > 0 && m >= h->tune.cpqr_big_min);
      const int64_t k = std::min<int64_t>(m, np);
      it.ow = tw;
      tw += m * np;
      it.ov = tv;
      tv += m * k;
      it.otau = ttau;
      ttau += k;
      it.ox = tx;
      tx += int64_t(np) * np;
      it.opiv = tpiv;
      tpiv += 2 * int64_t(np);  // the pivots, then perm
      if (it.big) {
        bigmax = std::max(bigmax, m * np);
        bign = std::max<int64_t>(bign, np);
      }
      its.push_back(it);
    }
    if (its.empty()) continue;
    const int32_t K = int32_t(its.size());
    DevBuf work, keep, vbuf, taub, xbuf, pbuf, curb, nrefb, errb;
    if ((st = dalloc(h, work, size_t(tw) * sizeof(double))) != SPAND_OK) return st;
    if ((st = dalloc(h, keep, size_t(tw) * sizeof(double))) != SPAND_OK) return st;
    if ((st = dalloc(h, vbuf, size_t(tv) * sizeof(double))) != SPAND_OK) return st;
    if ((st = dalloc(h, taub, size_t(ttau) * sizeof(double))) != SPAND_OK) return st;
    if ((st = dalloc(h, xbuf, size_t(tx) * sizeof(double))) != SPAND_OK) return st;
    if ((st = dalloc(h, pbuf, size_t(tpiv) * sizeof(int32_t))) != SPAND_OK) return st;
    if ((st = dalloc(h, errb, sizeof(int32_t))) != SPAND_OK) return st;
    // pivots and perm start at 0: every index they hand out stays inside the interface
    HIPCHK(hipMemsetAsync(pbuf.p, 0, size_t(tpiv) * sizeof(int32_t), h->stream));
    HIPCHK(hipMemsetAsync(errb.p, 0, sizeof(int32_t), h->stream));
    // sizes the CPQR kernels read and write: [2k] the width of A_np (np), [2k + 1] the rank
    std::vector<int32_t> c2(size_t(2) * K);
    for (int32_t k = 0; k < K; ++k) c2[2 * k] = c2[2 * k + 1] = its[k].np;
    if ((st = upload(h, curb, c2)) != SPAND_OK) return st;
    if ((st = upload(h, nrefb, std::vector<int32_t>(size_t(2) * K, 0))) != SPAND_OK) return st;
    // A_np = [A_qp] over the neighbours q (m x np, ld m), into both copies
    std::vector<CopyDesc> cps;
    for (const It& it : its) {
      const int32_t p = it.p;
      int64_t off = 0;
      for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e) {
        const int32_t q = sy.nb[e], nq = cur[q];
        if (nq == 0) continue;
        const double* src;
        int32_t lds, trans;
        if (q > p) {  // block (q, p) in panel p: A_qp itself
          src = A + lay.base[p] + lay.find(q, p);
          lds = int32_t(lay.H[p]);
          trans = 0;
        } else {      // block (p, q) in panel q: A_pq, transposed
          src = A + lay.base[q] + lay.find(p, q);
          lds = int32_t(lay.H[q]);
          trans = 1;
        }
        const int32_t step = std::max(1, COPY_CHUNK / nq);
        for (double* dst : {work.as<double>() + it.ow + off, keep.as<double>() + it.ow + off})
          for (int32_t c0 = 0; c0 < it.np; c0 += step)
            cps.push_back(CopyDesc{src, dst, lds, it.m, nq, c0, std::min(it.np, c0 + step), trans});
        off += nq;
      }
    }
    DevBuf dcp;
    if ((st = upload_big(h, dcp, cps)) != SPAND_OK) return st;
    launch_copy(dcp.as<CopyDesc>(), int64_t(cps.size()), h->stream);
    HIPCHK(hipGetLastError());
    // the truncated CPQR of every A_np, with its pivots
    std::vector<SparsDesc> sds(K);
    std::vector<SegDesc> segs(K);
    for (int32_t k = 0; k < K; ++k) {
      const It& it = its[k];
      SparsDesc d{};
      d.V = vbuf.as<double>() + it.ov;
      d.ldv = it.m;
      d.tau = taub.as<double>() + it.otau;
      d.diag = xbuf.as<double>() + it.ox;  // I_r lands in X, which is rewritten later
      d.ldd = it.np;
      d.m = it.m;
      d.seg_begin = k;
      d.seg_end = k + 1;
      d.id = 2 * k + 1;
      d.S = 1;
      d.G = it.big ? 0 : it.G;
      d.kslots = it.big ? 0 : cpqr_kslots(it.G, 0, true);  // the capacity that admitted it
      d.piv = pbuf.as<int32_t>() + it.opiv;
      sds[k] = d;
      SegDesc g{};
      g.blk = work.as<double>() + it.ow;
      g.ld = it.m;
      g.trans = 0;
      g.q = 2 * k;
      segs[k] = g;
    }
    std::vector<SlabRef> slabs;
    std::vector<std::pair<int32_t, size_t>> one;  // (team size, first slab) of each plain launch
    for (int32_t G = 1; G <= 64; G <<= 1) {
      const size_t s0 = slabs.size();
      for (int32_t k = 0; k < K; ++k)
        if (!its[k].big && its[k].G == G) slabs.push_back(SlabRef{k, 0});
      if (slabs.size() > s0) one.emplace_back(G, s0);
    }
    DevBuf dsd, dsg, dsl;
    if ((st = upload(h, dsd, sds)) != SPAND_OK) return st;
    if ((st = upload(h, dsg, segs)) != SPAND_OK) return st;
    if ((st = upload(h, dsl, slabs)) != SPAND_OK) return st;
    DevBuf bwk, bnrm, bpst, brb, bpost, bpcd, bbar;
    if (bigmax > 0) {
      if ((st = dalloc(h, bwk, size_t(bigmax) * sizeof(double))) != SPAND_OK) return st;
      if ((st = dalloc(h, bnrm, size_t(bign) * sizeof(double))) != SPAND_OK) return st;
      if ((st = dalloc(h, bpst, size_t(bign) * sizeof(int32_t))) != SPAND_OK) return st;
      if ((st = dalloc(h, brb, size_t(bign) * sizeof(double))) != SPAND_OK) return st;
      if ((st = dalloc(h, bpost, 1024 * sizeof(double))) != SPAND_OK) return st;
      if ((st = dalloc(h, bpcd, 1024 * sizeof(int32_t))) != SPAND_OK) return st;
      if ((st = dalloc(h, bbar, 256)) != SPAND_OK) return st;
    }
    hipEvent_t e0, e1;
    HIPCHK(ev.get(0, &e0));
    HIPCHK(ev.get(1, &e1));
    HIPCHK(hipEventRecord(e0, h->stream));
    int64_t nl = 0;
    for (size_t q = 0; q < one.size(); ++q) {
      const size_t s1 = q + 1 < one.size() ? one[q + 1].second : slabs.size();
      const int32_t G = one[q].first;
      hipError_t le = launch_cpqr_one(G, dsd.as<SparsDesc>(), dsl.as<SlabRef>() + one[q].second,
                                      int32_t(s1 - one[q].second), dsg.as<SegDesc>(), tol, curb.as<int32_t>(),
                                      nrefb.as<int32_t>(), errb.as<int32_t>(), cpqr_lds_bytes(G, 0, 1), h->stream);
      if (le != hipSuccess) return set_err(h, SPAND_E_HIP, std::string("sparsification launch: ") + hipGetErrorString(le));
      ++nl;
      pb.cpqr_ifaces[0] += int64_t(s1 - one[q].second);
    }
    for (int32_t k = 0; k < K; ++k) {
      if (!its[k].big) continue;
      const int capb = cpqr_big_max_coresident(1);
      if (capb <= 0) return set_err(h, SPAND_E_HIP, "occupancy query for the large-interface CPQR failed");
      const int32_t nb = int32_t(std::max<int64_t>(1, std::min<int64_t>(std::min(capb, 1024), (its[k].np + 15) / 16)));
      HIPCHK(hipMemsetAsync(bbar.p, 0, 256, h->stream));
      hipError_t le = launch_cpqr_big(sds[k], 1, dsg.as<SegDesc>(), tol, curb.as<int32_t>(), nrefb.as<int32_t>(),
                                      errb.as<int32_t>(), nb, bwk.as<double>(), bnrm.as<double>(), bpst.as<int32_t>(),
                                      brb.as<double>(), bpost.as<double>(), bpcd.as<int32_t>(), bbar.as<uint32_t>(),
                                      h->stream);
      if (le != hipSuccess)
        return set_err(h, SPAND_E_HIP, std::string("large-interface sparsification launch: ") + hipGetErrorString(le));
      ++nl;
      ++pb.cpqr_big;
    }
    HIPCHK(hipEventRecord(e1, h->stream));
    int32_t serr = 0;
    HIPCHK(hipMemcpyAsync(c2.data(), curb.p, c2.size() * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(&serr, errb.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (serr) return set_err(h, SPAND_E_HIP, "sparsification barrier timed out");
    {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      cpqr_ms += ms;
      cpqr_launches += nl;
    }
    // the interfaces that drop dofs
    std::vector<InterpPermDesc> pds;
    std::vector<InterpTDesc> tds;
    std::vector<InterpCol> tcols;
    std::vector<InterpXDesc> xds;
    std::vector<InterpRowDesc> rws;
    std::vector<CopyDesc> back;
    std::vector<Front> fr;
    GemmSeq cong(h->tune.gemm_chol), syrk(h->tune.gemm_syrk);
    int64_t ttot = 0, dtot = 0;
    int32_t rmax = 0;
    for (It& it : its) {
      it.r = std::min(std::max(c2[2 * (&it - its.data()) + 1], 0), it.np);
      const int64_t r = it.r, m = it.m, np = it.np;
      {
        // CPQR flops as in the orthogonal path: 6 (m-j)(np-j) - (m-j) per step
        const int64_t s1 = r * (r - 1) / 2, s2 = (r - 1) * r * (2 * r - 1) / 6;
        pb.cpqr_flops += double(6 * (r * m * np - (m + np) * s1 + s2) - (r * m - s1));
      }
      if (it.r == it.np) continue;
      it.ot = ttot;
      ttot += r * (np - r);
      dtot += dinv_size(int32_t(np - r));
      rmax = std::max(rmax, it.r);
    }
    DevBuf tbuf, dinvb;
    if ((st = dalloc(h, tbuf, size_t(std::max<int64_t>(ttot, 1)) * sizeof(double))) != SPAND_OK) return st;
    if ((st = dalloc(h, dinvb, size_t(std::max<int64_t>(dtot, 1)) * sizeof(double))) != SPAND_OK) return st;
    int64_t doff = 0;
    for (const It& it : its) {
      if (it.r == it.np) continue;
      const int32_t p = it.p, np = it.np, r = it.r, nf = np - r;
      int32_t* piv = pbuf.as<int32_t>() + it.opiv;
      int32_t* perm = piv + np;
      double* X = xbuf.as<double>() + it.ox;
      double* T = tbuf.as<double>() + it.ot;
      pds.push_back(InterpPermDesc{piv, perm, np, r});
      if (r > 0) {
        const int32_t td = int32_t(tds.size());
        tds.push_back(InterpTDesc{work.as<double>() + it.ow, perm, T, it.m, r});
        for (int32_t j = 0; j < nf; ++j) tcols.push_back(InterpCol{td, j});
      }
      const int64_t ne2 = int64_t(np) * np;
      for (int64_t e0 = 0; e0 < ne2; e0 += INTERP_CHUNK)
        xds.push_back(InterpXDesc{A + lay.base[p], perm, X, int32_t(lay.H[p]), np, r, 0, e0,
                                  std::min<int64_t>(ne2, e0 + INTERP_CHUNK)});
      // X = [X_ff X_fc; X_cf X_cc] (ld np): rows and columns 0..nf are f, nf..np are c
      GemmDesc g{};
      g.A = X + nf + int64_t(nf) * np; g.lda = np;  // X_cc
      g.B = T; g.ldb = r;
      g.C = X + nf; g.ldc = np;                     // X_cf <- C_cf = A_cf - A_cc T
      g.M = r; g.N = nf; g.K = r;
      g.flags = 0; g.alpha = -1.0; g.beta = 1.0;
      cong.add(g, 0);
      GemmDesc f1{};
      f1.A = X + int64_t(nf) * np; f1.lda = np;     // X_fc = A_fc
      f1.B = T; f1.ldb = r;
      f1.C = X; f1.ldc = np;                        // X_ff -= A_fc T
      f1.M = nf; f1.N = nf; f1.K = r;
      f1.flags = G_LOWERC; f1.alpha = -1.0; f1.beta = 1.0;
      cong.add(f1, 1);
      fr.push_back(Front{X, dinvb.as<double>() + doff, np, nf, np, p, pb.flags + 3});
      doff += dinv_size(nf);
      GemmDesc s{};
      s.A = X + nf; s.lda = np;                     // G_cf
      s.B = X + nf; s.ldb = np;
      s.C = X + nf + int64_t(nf) * np; s.ldc = np;  // X_cc -= G G^T
      s.M = r; s.N = r; s.K = nf;
      s.flags = G_TB | G_LOWERC; s.alpha = -1.0; s.beta = 1.0;
      syrk.add(s, 1);
      // A_cc back into the diagonal block of p; the rows c of every A_pq
      if (r > 0) {
        const int32_t step = std::max(1, COPY_CHUNK / r);
        for (int32_t c0 = 0; c0 < r; c0 += step)
          back.push_back(CopyDesc{X + nf + int64_t(nf) * np, A + lay.base[p], np, int32_t(lay.H[p]), r, c0,
                                  std::min(r, c0 + step), 0});
        int32_t row0 = 0;
        for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e) {
          const int32_t q = sy.nb[e], nq = cur[q];
          if (nq == 0) continue;
          InterpRowDesc rd{};
          rd.keep = keep.as<double>() + it.ow;
          rd.perm = perm;
          rd.ldk = it.m;
          rd.row0 = row0;
          rd.nq = nq;
          rd.r = r;
          if (q < p) {  // block (p, q) in panel q, rows over p
            rd.blk = A + lay.base[q] + lay.find(p, q);
            rd.ld = int32_t(lay.H[q]);
            rd.trans = 0;
          } else {      // block (q, p) in panel p, columns over p
            rd.blk = A + lay.base[p] + lay.find(q, p);
            rd.ld = int32_t(lay.H[p]);
            rd.trans = 1;
          }
          const int64_t cnt = int64_t(r) * nq;
          for (int64_t e0 = 0; e0 < cnt; e0 += INTERP_CHUNK) {
            rd.e0 = e0;
            rd.e1 = std::min<int64_t>(cnt, e0 + INTERP_CHUNK);
            rws.push_back(rd);
          }
          row0 += nq;
        }
      }
      sn.h_interp.push_back(InterpAp{perm, T, X, np, r, sn.slot_ptr[p]});
      pb.m_F += 2 * int64_t(r) * nf + int64_t(nf) * (nf + 1) / 2;
    }
    if (!pds.empty()) {
      cong.end_launch(0);
      GemmDesc g2{};
      for (const It& it : its) {  // X_ff -= T^T C_cf, once C_cf is formed
        if (it.r == it.np || it.r == 0) continue;
        const int32_t np = it.np, r = it.r, nf = np - r;
        double* X = xbuf.as<double>() + it.ox;
        g2.A = tbuf.as<double>() + it.ot; g2.lda = r;
        g2.B = X + nf; g2.ldb = np;
        g2.C = X; g2.ldc = np;
        g2.M = nf; g2.N = nf; g2.K = r;
        g2.flags = G_TA | G_LOWERC; g2.alpha = -1.0; g2.beta = 1.0;
        cong.add(g2, 1);
      }
      cong.end_launch(0);
      syrk.end_launch(0);
      DevBuf dpd, dtd, dtc, dxd, drw, dbk;
      if ((st = upload(h, dpd, pds)) != SPAND_OK) return st;
      if ((st = upload(h, dtd, tds)) != SPAND_OK) return st;
      if ((st = upload_big(h, dtc, tcols)) != SPAND_OK) return st;
      if ((st = upload_big(h, dxd, xds)) != SPAND_OK) return st;
      if ((st = upload_big(h, drw, rws)) != SPAND_OK) return st;
      if ((st = upload_big(h, dbk, back)) != SPAND_OK) return st;
      if ((st = cong.upload_all(h)) != SPAND_OK) return st;
      if ((st = syrk.upload_all(h)) != SPAND_OK) return st;
      launch_interp_perm(dpd.as<InterpPermDesc>(), int32_t(pds.size()), h->stream);
      launch_interp_t(dtd.as<InterpTDesc>(), dtc.as<InterpCol>(), int64_t(tcols.size()), rmax, h->stream);
      launch_interp_x(dxd.as<InterpXDesc>(), int64_t(xds.size()), h->stream);
      HIPCHK(hipGetLastError());
      cong.launch(h, 0);
      cong.launch(h, 1);
      HIPCHK(hipGetLastError());
      if ((st = blocked_cholesky(h, fr, 0)) != SPAND_OK) return st;
      syrk.launch(h, 0);
      launch_copy(dbk.as<CopyDesc>(), int64_t(back.size()), h->stream);
      launch_interp_rows(drw.as<InterpRowDesc>(), int64_t(rws.size()), h->stream);
      HIPCHK(hipGetLastError());
      sn.interp_store.push_back(std::move(xbuf));
      sn.interp_store.push_back(std::move(pbuf));
      sn.interp_store.push_back(std::move(tbuf));
      // the descriptor and scratch buffers of this class go back to the pool; later
      // allocations that reuse them are ordered after these launches on the stream
    }
    for (const It& it : its) {
      cur[it.p] = it.r;
      sn.rank[it.p] = it.r;
    }
  }
  return SPAND_OK;
}

// The order in which the factorization freezes the dofs: step by step, the slots of
// every eliminated cluster, then those an interface drops at its sparsification (the
// slots from its rank on), each in slot-list order.  In this order every cluster's
// slot list at every step is a few contiguous runs (its dropped part, and the kept
// parts of its children inside the parents they are frozen with), so the apply's
// gathers and scatters through the slots read whole lines.  The order grows step by
// step on the host (frozen_at); at the end the device slot arrays of every step are
// rewritten with positions in this order by one kernel.  The host keeps the vertex
// ids (the batched solve works in vertex order).
void frozen_at(const SymStep& sy, const StepNum& sn, std::vector<int32_t>& inv) {
  for (int32_t c = 0; c < sy.nc; ++c) {
    const int64_t b = sn.slot_ptr[c];
    const int32_t size = sn.size[c];
    const int32_t from = c < sy.ne ? 0 : std::max(0, std::min(size, sn.rank[c]));
    inv.insert(inv.end(), sn.slot.begin() + b + from, sn.slot.begin() + b + size);
  }
}

spand_status freeze_order(spand_ctx* h, const std::vector<int32_t>& inv, size_t uploaded, DevBuf& bad) {
  const int64_t n = h->an.n;
  if (int64_t(inv.size()) != n) return set_err(h, SPAND_E_INVALID, "freeze order does not cover every dof");
  if (h->d_inv.bytes < size_t(n) * sizeof(int32_t) || uploaded > inv.size())
    return set_err(h, SPAND_E_INVALID, "freeze order buffer missing");
  spand_status st;
  // entries [0, uploaded) went to the device during the steps; the rest goes now
  if ((st = stage_copy(h, h->d_inv.as<int32_t>() + uploaded, inv.data() + uploaded,
                       (inv.size() - uploaded) * sizeof(int32_t))) != SPAND_OK)
    return st;
  // the inverse is formed on the device; bad is read at the end of the factorization
  if ((st = dalloc(h, h->d_pos, size_t(n) * sizeof(int32_t))) != SPAND_OK) return st;
  if ((st = dalloc(h, bad, sizeof(int32_t))) != SPAND_OK) return st;
  HIPCHK(hipMemsetAsync(h->d_pos.p, 0xFF, size_t(n) * sizeof(int32_t), h->stream));
  HIPCHK(hipMemsetAsync(bad.p, 0, sizeof(int32_t), h->stream));
  launch_invert_perm(h->d_inv.as<int32_t>(), n, h->d_pos.as<int32_t>(), bad.as<int32_t>(), h->stream);
  std::vector<RemapSeg> segs;
  auto add = [&](DevBuf& b, int64_t len) {
    for (int64_t o = 0; o < len; o += REMAP_CHUNK)
      segs.push_back(RemapSeg{b.as<int32_t>() + o, std::min<int64_t>(REMAP_CHUNK, len - o)});
  };
  for (StepNum& sn : h->num) {
    add(sn.d_slot, int64_t(sn.slot.size()));
    add(sn.d_nslot, int64_t(sn.h_nslot.size()));
    add(sn.d_sgather, int64_t(sn.h_sgather.size()));
  }
  DevBuf dsg;
  if ((st = upload_big(h, dsg, segs)) != SPAND_OK) return st;
  launch_remap(dsg.as<RemapSeg>(), int64_t(segs.size()), h->d_pos.as<int32_t>(), h->stream);
  HIPCHK(hipGetLastError());
  return SPAND_OK;
}

// Problem index and cluster of a failure id of a run (ids carry the problem in
// their high bits so that one flag word may serve several problems).
constexpr int32_t FAIL_NONE = 0x7fffffff;

spand_status factor_run(std::vector<Prob>& P, double tol, int32_t skip, spand_prec prec) {
  spand_ctx* h = P[0].h;  // the run's stream, staging and scratch; errors of shared work
  const int gemm_prec = (prec == SPAND_FP64) ? 0 : (prec == SPAND_FP32 ? 1 : 2);
  const int32_t NP = int32_t(P.size());
  int32_t Lmax = 0;
  spand_status st;
  for (Prob& pb : P) {
    pb.L = pb.h->an.levels;
    Lmax = std::max(Lmax, pb.L);
    pb.h->stage.reset();
    pb.h->num.clear();
    pb.h->num.resize(pb.L);
    pb.h->max_tmp = 0;
    pb.h->max_gather = 0;
    pb.h->d_pos.release();
    pb.h->d_inv.release();
    pb.frozen.clear();
    pb.frozen_up = 0;
    if (P.size() == 1) {
      pb.frozen.reserve(size_t(pb.h->an.n));
      // the freeze order is copied to the device step by step, while later steps run
      if ((st = dalloc(pb.h, pb.h->d_inv, size_t(pb.h->an.n) * sizeof(int32_t))) != SPAND_OK) return st;
    }
    std::memset(pb.h->stats.step_phase_seconds, 0, sizeof(pb.h->stats.step_phase_seconds));
    std::memset(pb.h->stats.step_m_F, 0, sizeof(pb.h->stats.step_m_F));
  }
  // failure and input flags of every problem, read back at one sync per step
  DevBuf dflag;
  {
    std::vector<int32_t> init(size_t(4) * NP);
    for (int32_t q = 0; q < NP; ++q) {
      init[4 * q] = init[4 * q + 1] = init[4 * q + 3] = FAIL_NONE;
      init[4 * q + 2] = 0;
    }
    if ((st = upload(h, dflag, init)) != SPAND_OK) return st;
    for (int32_t q = 0; q < NP; ++q) P[q].flags = dflag.as<int32_t>() + 4 * q;
  }
  std::vector<int32_t> hflags(size_t(4) * NP);
  auto fail_problem = [&](Prob& pb, spand_status s2, const std::string& msg) {
    set_err(pb.h, s2, msg);
    pb.live = false;
  };

  EventPool phev;   // 5 phase boundaries per step, read after the last sync
  EventPool evpool; // every CPQR launch
  EventPool joinev; // the joins of the two streams of the sparsification
  size_t njoin = 0;
  struct ColourSpan {
    size_t ev, l0, l1;  // start event in joinev, CPQR launches [l0, l1) of evpool
  };
  std::vector<ColourSpan> colour_span;  // colour classes of the current step
  EventPool rbev;   // the rank read-back of every step
  std::vector<char> elim_ran(size_t(Lmax) + 1, 0);
  double cpqr_ms = 0.0;
  int64_t cpqr_launches = 0;

  for (int32_t t = 1; t <= Lmax; ++t) {
    std::vector<Prob*> act;
    for (Prob& pb : P) {
      pb.on = pb.live && t <= pb.L;
      if (pb.on) act.push_back(&pb);
    }
    if (act.empty()) break;
    hipEvent_t ph[5];
    for (int q = 0; q < 5; ++q) HIPCHK(phev.get(5 * size_t(t - 1) + q, &ph[q]));

    // ---- sizes, slots, layout and assembly of every problem
    HIPCHK(hipEventRecord(ph[0], h->stream));
    std::vector<MergeJob> merges;
    std::vector<ZeroDesc> zeros;  // the new step buffers of every problem, zeroed in one launch
    std::vector<Prob*> scatters;  // step 1: the CSR values go in after the fill
    auto add_zero = [&](double* p0, int64_t len) {
      for (int64_t o = 0; o < len; o += ZERO_CHUNK) zeros.push_back(ZeroDesc{p0 + o, std::min<int64_t>(ZERO_CHUNK, len - o)});
    };
    for (Prob* pp : act) {
      Prob& pb = *pp;
      spand_ctx* hq = pb.h;
      const SymStep& sy = hq->an.steps[t - 1];
      step_sizes(sy, t, hq->num);
      StepNum& sn = hq->num[t - 1];
      const int32_t nc = sy.nc, ne = sy.ne;
      pb.sparsify = (t > skip) && (sy.level > 1);
      if (sy.level == 1)
        for (int32_t s = 0; s < ne; ++s) pb.s_top += sn.size[s];
      pb.lay = Layout();
      build_layout(sy, sn.size, pb.lay);
      const Layout& lay = pb.lay;
      if ((st = dalloc(hq, sn.elim, size_t(lay.total_elim) * sizeof(double))) != SPAND_OK) return st;
      if ((st = dalloc(hq, pb.arena, size_t(lay.total_arena) * sizeof(double))) != SPAND_OK) return st;
      double* E = sn.elim.as<double>();
      double* A = pb.arena.as<double>();
      add_zero(E, lay.total_elim);
      add_zero(A, lay.total_arena);
      if (t == 1) {
        if (!hq->d_dst1.p) {
          // destination of every CSR entry inside the step-1 panels (it depends on the
          // pattern only, so later factors reuse it): >= 0 arena offset, <= -2
          // elimination-buffer offset -(d+2), -1 skipped (upper triangle)
          const Analysis& an = hq->an;
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
          if ((st = upload(hq, hq->d_dst1, dst)) != SPAND_OK) return st;
        }
        scatters.push_back(pp);
      } else {
        merges.push_back(MergeJob{&sy, &hq->num[t - 2], &pb.lay, &pb.lay_prev, E, A, pb.arena_prev.as<double>()});
      }
    }
    if (!zeros.empty()) {
      DevBuf dz;
      if ((st = upload_big(h, dz, zeros)) != SPAND_OK) return st;
      launch_zero(dz.as<ZeroDesc>(), int64_t(zeros.size()), h->stream);
      HIPCHK(hipGetLastError());
    }
    for (Prob* pp : scatters) {
      spand_ctx* hq = pp->h;
      launch_scatter_values(pp->values, hq->d_dst1.as<int64_t>(), int64_t(hq->an.colind.size()), pp->arena.as<double>(),
                            hq->num[0].elim.as<double>(), pp->flags + 2, h->stream);
      HIPCHK(hipGetLastError());
    }
    if (!merges.empty()) {
      DevBuf d_copy;
      int64_t ncopy = 0;
      if ((st = plan_merges(h, merges, d_copy, ncopy)) != SPAND_OK) return st;
      launch_copy(d_copy.as<CopyDesc>(), ncopy, h->stream);
      HIPCHK(hipGetLastError());
    }

    // ---- elimination (Sec. 2.4) of every problem's level-l clusters, in shared launches
    HIPCHK(hipEventRecord(ph[1], h->stream));
    HIPCHK(hipEventRecord(ph[2], h->stream));  // recorded again after the reduction
    {
      std::vector<Front> fr;
      GemmSeq syrk(h->tune.gemm_syrk);
      struct Item { int32_t prob; uint64_t tgt; int32_t s; int64_t coff; };
      std::vector<ReduceDesc> rds;
      std::vector<ContribDesc> cds2;
      for (Prob* pp : act) {
        Prob& pb = *pp;
        spand_ctx* hq = pb.h;
        const SymStep& sy = hq->an.steps[t - 1];
        StepNum& sn = hq->num[t - 1];
        const Layout& lay = pb.lay;
        const int32_t ne = sy.ne;
        double* E = sn.elim.as<double>();
        double* A = pb.arena.as<double>();
        pb.c_off.assign(ne, 0);
        pb.ed_off.assign(ne, 0);
        pb.nN.assign(ne, 0);
        int64_t cbuf_total = 0, ed_total = 0;
        for (int32_t s = 0; s < ne; ++s) {
          pb.nN[s] = int32_t(lay.Hr[s] - sn.size[s]);
          pb.c_off[s] = cbuf_total;
          cbuf_total += int64_t(pb.nN[s]) * pb.nN[s];
          pb.ed_off[s] = ed_total;
          ed_total += dinv_size(sn.size[s]);
          const double ns = sn.size[s], nn = pb.nN[s];
          pb.elim_flops += nn * ns * ns + nn * (nn + 1.0) * ns;
          pb.m_F += int64_t(sn.size[s]) * (sn.size[s] + 1) / 2 + int64_t(sn.size[s]) * pb.nN[s];
        }
        if ((st = dalloc(hq, sn.edinv, size_t(ed_total) * sizeof(double))) != SPAND_OK) return st;
        if ((st = dalloc(hq, pb.cbuf, size_t(cbuf_total) * sizeof(double))) != SPAND_OK) return st;
        const int32_t qid = int32_t(pp - P.data());
        for (int32_t s = 0; s < ne; ++s)
          if (sn.size[s] > 0)
            fr.push_back(Front{E + lay.base[s], sn.edinv.as<double>() + pb.ed_off[s], int32_t(lay.H[s]), sn.size[s],
                               int32_t(lay.Hr[s]), s, P[qid].flags + 0});
        for (int32_t s = 0; s < ne; ++s) {
          const int32_t ns = sn.size[s], nn = pb.nN[s];
          GemmDesc y{};
          y.A = E + lay.base[s] + ns; y.lda = int32_t(lay.H[s]);
          y.B = y.A; y.ldb = y.lda;
          y.C = pb.cbuf.as<double>() + pb.c_off[s]; y.ldc = nn;
          y.M = nn; y.N = nn; y.K = ns;
          y.flags = G_TB | G_LOWERC;
          y.alpha = 1.0; y.beta = 0.0;
          syrk.add(y, 1);
        }
      }
      // the Cholesky and the SYRK go first; the reduction plan is built while they run
      if ((st = blocked_cholesky(h, fr, gemm_prec)) != SPAND_OK) return st;
      syrk.end_launch(gemm_prec);
      if ((st = syrk.upload_all(h)) != SPAND_OK) return st;
      syrk.launch(h, 0);
      HIPCHK(hipGetLastError());
      {
        // Clusters without neighbours (the top separator): L_s^{-1} itself (the
        // identity solved against L_s), so that the apply multiplies by it over
        // 64-row tiles in parallel instead of a substitution chained over its
        // 64-row blocks in one workgroup.
        std::vector<LeftBlock> lb;
        std::vector<IdentDesc> ids;
        for (Prob* pp : act) {
          Prob& pb = *pp;
          spand_ctx* hq = pb.h;
          const SymStep& sy = hq->an.steps[t - 1];
          StepNum& sn = hq->num[t - 1];
          const Layout& lay = pb.lay;
          const int32_t ne = sy.ne;
          pb.iso_off.assign(ne, -1);
          int64_t iso_total = 0;
          for (int32_t s = 0; s < ne; ++s)
            if (sn.size[s] > 0 && pb.nN[s] == 0) {
              pb.iso_off[s] = iso_total;
              iso_total += int64_t(pad16(sn.size[s])) * sn.size[s];
            }
          if (iso_total == 0) {
            sn.iso.release();
            continue;
          }
          if ((st = dalloc(hq, sn.iso, size_t(iso_total) * sizeof(double))) != SPAND_OK) return st;
          double* E = sn.elim.as<double>();
          double* ISO = sn.iso.as<double>();
          for (int32_t s = 0; s < ne; ++s) {
            if (pb.iso_off[s] < 0) continue;
            add_identity(ids, ISO + pb.iso_off[s], sn.size[s], pad16(sn.size[s]));
            lb.push_back(LeftBlock{ISO + pb.iso_off[s], E + lay.base[s], sn.edinv.as<double>() + pb.ed_off[s],
                                   pad16(sn.size[s]), int32_t(lay.H[s]), sn.size[s], sn.size[s]});
          }
        }
        if (!lb.empty()) {
          DevBuf di;
          if ((st = upload(h, di, ids)) != SPAND_OK) return st;
          launch_set_identity(di.as<IdentDesc>(), int32_t(ids.size()), h->stream);
          HIPCHK(hipGetLastError());
          if ((st = left_trsm(h, lb)) != SPAND_OK) return st;
        }
      }
      for (Prob* pp : act) {
        Prob& pb = *pp;
        spand_ctx* hq = pb.h;
        const SymStep& sy = hq->an.steps[t - 1];
        StepNum& sn = hq->num[t - 1];
        const Layout& lay = pb.lay;
        const int32_t ne = sy.ne;
        double* A = pb.arena.as<double>();
        const int32_t qid = int32_t(pp - P.data());
        // deterministic reduction of C_s into the targets: contributions to one target
        // block in ascending s
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
                items.push_back(Item{qid, pair_pack(na, nb), s, pb.c_off[s] + oa + ob * pb.nN[s]});
              ob += sn.size[nb];
            }
            oa += sn.size[na];
          }
        }
        std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.tgt < y.tgt; });
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
            cds2.push_back(ContribDesc{pb.cbuf.as<double>() + items[r].coff, pb.nN[items[r].s], 0});
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
      }
      DevBuf drd, dcd;
      if ((st = upload_big(h, drd, rds)) != SPAND_OK) return st;
      if ((st = upload_big(h, dcd, cds2)) != SPAND_OK) return st;
      launch_reduce(drd.as<ReduceDesc>(), int32_t(rds.size()), dcd.as<ContribDesc>(), h->stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(ph[2], h->stream));
      elim_ran[t] = 1;
      for (Prob* pp : act) pp->cbuf.release();
    }

    // ---- scaling (Sec. 2.5) of every sparsified problem's interfaces
    HIPCHK(hipEventRecord(ph[3], h->stream));
    HIPCHK(hipEventRecord(ph[4], h->stream));
    bool any_sparsify = false;
    {
      std::vector<Front> fr;
      std::vector<LeftBlock> lb;
      std::vector<IdentDesc> ids, did;
      for (Prob* pp : act) {
        Prob& pb = *pp;
        spand_ctx* hq = pb.h;
        const SymStep& sy = hq->an.steps[t - 1];
        StepNum& sn = hq->num[t - 1];
        const int32_t nc = sy.nc, ne = sy.ne;
        sn.rank.assign(nc, -1);
        for (int32_t c = ne; c < nc; ++c) sn.rank[c] = sn.size[c];
        pb.sc_off.assign(nc, -1);
        pb.sd_off.assign(nc, -1);
        pb.v_off.assign(nc, -1);
        pb.tau_off.assign(nc, -1);
        pb.t_off.assign(nc, -1);
        pb.nref.assign(nc, 0);
        if (!(pb.sparsify && nc > ne) || hq->variant == SPAND_IN) continue;
        any_sparsify = true;
        const Layout& lay = pb.lay;
        double* A = pb.arena.as<double>();
        int64_t sc_total = 0, sd_total = 0;
        for (int32_t p = ne; p < nc; ++p) {
          if (sn.size[p] == 0) continue;
          pb.sc_off[p] = sc_total;
          sc_total += int64_t(pad16(sn.size[p])) * sn.size[p];
          pb.sd_off[p] = sd_total;
          sd_total += dinv_size(sn.size[p]);
          pb.m_F += int64_t(sn.size[p]) * (sn.size[p] + 1) / 2;
        }
        if ((st = dalloc(hq, sn.scale, size_t(sc_total) * sizeof(double))) != SPAND_OK) return st;
        if ((st = dalloc(hq, sn.sdinv, size_t(sd_total) * sizeof(double))) != SPAND_OK) return st;
        double* SC = sn.scale.as<double>();
        double* SD = sn.sdinv.as<double>();
        for (int32_t p = ne; p < nc; ++p)
          if (sn.size[p] > 0)
            fr.push_back(Front{A + lay.base[p], SD + pb.sd_off[p], int32_t(lay.H[p]), sn.size[p], int32_t(lay.Hr[p]), p,
                               pb.flags + 1});
        // L_p^{-1} for the apply (the identity solved against L_p), and L_i^{-1} from the
        // left on every block (i, p), in one blocked left solve
        for (int32_t p = ne; p < nc; ++p) {
          if (sn.size[p] == 0) continue;
          add_identity(ids, SC + pb.sc_off[p], sn.size[p], pad16(sn.size[p]));
          lb.push_back(LeftBlock{SC + pb.sc_off[p], A + lay.base[p], SD + pb.sd_off[p], pad16(sn.size[p]), int32_t(lay.H[p]),
                                 sn.size[p], sn.size[p]});
          for (int64_t e = lay.pan_ptr[p] + 1; e < lay.pan_ptr[p + 1]; ++e) {
            const int32_t i = lay.prow[e];
            if (sn.size[i] == 0) continue;
            lb.push_back(LeftBlock{A + lay.base[p] + lay.proff[e], A + lay.base[i], SD + pb.sd_off[i],
                                   int32_t(lay.H[p]), int32_t(lay.H[i]), sn.size[i], sn.size[p]});
          }
        }
        for (int32_t p = ne; p < nc; ++p)
          if (sn.size[p] > 0) add_identity(did, A + lay.base[p], sn.size[p], int32_t(lay.H[p]));
      }
      if (any_sparsify) {
        if ((st = blocked_cholesky(h, fr, 0)) != SPAND_OK) return st;
        DevBuf d1, d2;
        if ((st = upload(h, d1, ids)) != SPAND_OK) return st;
        launch_set_identity(d1.as<IdentDesc>(), int32_t(ids.size()), h->stream);
        HIPCHK(hipGetLastError());
        if ((st = left_trsm(h, lb)) != SPAND_OK) return st;
        if ((st = upload(h, d2, did)) != SPAND_OK) return st;
        launch_set_identity(d2.as<IdentDesc>(), int32_t(did.size()), h->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(ph[3], h->stream));
      }
    }

    // ---- sparsification (Sec. 2.6.1), one colour class of every problem at a time.
    // A_pn of interface p lives in the registers of slabS[p] workgroups with tg[p]
    // lanes per column.  Interfaces of one slab go in one plain launch per team size;
    // interfaces of several slabs go in one cooperative launch per colour.
    size_t nlaunch = 0;
    DevBuf curb, nrefb, errb, xchb, doneb;
    int64_t ncl = 0;  // clusters of the sparsified problems in the run's size and rank arrays
    auto orth = [&](const Prob& pb) {
      const SymStep& sy = pb.h->an.steps[t - 1];
      return pb.sparsify && sy.nc > sy.ne && pb.h->variant == SPAND_ORTHS;
    };
    bool any_orth = false;
    for (Prob* pp : act) any_orth = any_orth || orth(*pp);
    if (any_orth) {
      int32_t ncolour = 0;
      int64_t xch_total = 0;
      std::vector<int32_t> cur_h;
      // The LDS slot of the register layouts (a third, or fourth, column per team)
      // serves a single-slab interface that it spares an exchange, and the multi-slab
      // interfaces of a step with many of them (fewer slab steps in all); at a step of
      // few multi-slab interfaces, whose time is the chain of its longest ones, those
      // keep to the register slots (more slabs, less work per step).
      bool slot_multi = false;
      {
        int64_t nmulti = 0;
        for (Prob* pp : act) {
          if (!orth(*pp)) continue;
          const SymStep& sy = pp->h->an.steps[t - 1];
          const StepNum& sn = pp->h->num[t - 1];
          for (int32_t p = sy.ne; p < sy.nc; ++p) {
            const int32_t G = cpqr_team(sn.size[p]);
            if (sn.size[p] == 0 || G < 0) continue;
            int64_t ncols = 0;
            for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e) ncols += sn.size[sy.nb[e]];
            if (ncols > cpqr_capacity(G, 0, true)) ++nmulti;
          }
        }
        slot_multi = nmulti >= 100;
      }
      for (Prob* pp : act) {
        Prob& pb = *pp;
        spand_ctx* hq = pb.h;
        const SymStep& sy = hq->an.steps[t - 1];
        StepNum& sn = hq->num[t - 1];
        const int32_t nc = sy.nc, ne = sy.ne;
        if (!orth(pb)) continue;
        pb.cbase = ncl;
        ncl += nc;
        cur_h.insert(cur_h.end(), sn.size.begin(), sn.size.end());
        pb.ncols.assign(nc, 0);
        pb.xch_off.assign(nc, -1);
        pb.slabS.assign(nc, 0);
        pb.tg.assign(nc, 0);
        pb.nseg.assign(nc, 0);
        pb.wide.assign(nc, 0);
        pb.rlay.assign(nc, 0);
        pb.big.assign(nc, 0);
        pb.kslots.assign(nc, 0);
        int64_t house_total = 0;
        for (int32_t p = ne; p < nc; ++p) {
          for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e)
            if (sn.size[sy.nb[e]] > 0) {
              pb.ncols[p] += sn.size[sy.nb[e]];
              pb.nseg[p]++;
            }
          if (sn.size[p] == 0 || pb.ncols[p] == 0) continue;
          ncolour = std::max(ncolour, sy.colour[p] + 1);
          const int64_t m = sn.size[p];
          const int32_t G = cpqr_team(sn.size[p]);
          // beyond the register layouts (or asked for by the tuning): the global-memory
          // kernel, one cooperative launch per interface
          bool big = G < 0 || (h->tune.cpqr_big_min > 0 && m >= h->tune.cpqr_big_min);
          if (!big) {
            const int64_t cap = cpqr_capacity(G, 0, slot_multi);
            const int64_t S0 = (pb.ncols[p] + cap - 1) / cap;
            if (S0 > 1 && S0 > cpqr_max_coresident(cpqr_lds_bytes(G, 0, pb.nseg[p]))) {
              const int32_t G1 = cpqr_team(sn.size[p], 1);
              const int64_t cap1 = G1 > 0 ? cpqr_capacity(G1, 1, slot_multi) : cap;
              const int64_t S1 = G1 > 0 ? (pb.ncols[p] + cap1 - 1) / cap1 : S0;
              if (S1 > cpqr_max_coresident(cpqr_lds_bytes(G1 > 0 ? G1 : G, G1 > 0 ? 1 : 0, pb.nseg[p]))) big = true;
            }
          }
          if (big) {
            if (m > cpqr_big_max_rows())
              return set_err(h, SPAND_E_INVALID, "interface of " + std::to_string(m) + " dofs exceeds the CPQR limit (" +
                                                     std::to_string(cpqr_big_max_rows()) + " rows)");
            pb.big[p] = 1;
          } else {
          pb.tg[p] = G;
          const int64_t cap_r = cpqr_capacity(G, 0, false), cap_s = cpqr_capacity(G, 0, true);
          if (pb.ncols[p] <= cap_s) {  // one slab; the LDS slot only when the registers are short
            pb.slabS[p] = 1;
            pb.kslots[p] = cpqr_kslots(G, 0, pb.ncols[p] > cap_r);
            if (pb.ncols[p] > cap_r && G == 2 && m <= cpqr_wide_rows() && pb.ncols[p] <= cpqr_wide_capacity())
              pb.wide[p] = 1;  // the wide layout holds it in registers alone
          } else {
            const int64_t cap = cpqr_capacity(G, 0, slot_multi);
            pb.slabS[p] = int32_t((pb.ncols[p] + cap - 1) / cap);
            pb.kslots[p] = cpqr_kslots(G, 0, slot_multi);
          }
          if (pb.slabS[p] > 1) {  // layout 1 when it needs fewer slabs (and still more than one)
            const int32_t G1 = cpqr_team(sn.size[p], 1);
            if (G1 > 0) {
              const int64_t cap1 = cpqr_capacity(G1, 1, slot_multi);
              const int32_t S1 = int32_t((pb.ncols[p] + cap1 - 1) / cap1);
              if (S1 > 1 && S1 < pb.slabS[p]) {
                pb.rlay[p] = 1;
                pb.tg[p] = G1;
                pb.slabS[p] = S1;
                pb.kslots[p] = cpqr_kslots(G1, 1, slot_multi);
              }
            }
            pb.xch_off[p] = xch_total;
            xch_total += 3 * int64_t(pb.slabS[p]) * cpqr_record(pb.tg[p], pb.rlay[p]);  // three exchange buffers
          }
          }
          const int64_t kmax = std::min<int64_t>(sn.size[p], pb.ncols[p]);
          pb.v_off[p] = house_total;
          house_total += int64_t(pad16(sn.size[p])) * kmax;
          pb.tau_off[p] = house_total;
          house_total += (kmax + 15) / 16 * 16;
          pb.t_off[p] = house_total;  // compact WY factor T (r x r, r <= kmax, ld pad16(r))
          house_total += (kmax + 15) / 16 * 16 * kmax;
        }
        if ((st = dalloc(hq, sn.house, size_t(house_total) * sizeof(double))) != SPAND_OK) return st;
        for (int32_t p = ne; p < nc; ++p)
          if (pb.v_off[p] >= 0 && !pb.big[p]) {
            ++pb.cpqr_ifaces[pb.slabS[p] > 1 ? 2 + pb.rlay[p] : (pb.wide[p] ? 1 : 0)];
            if (!pb.wide[p] && pb.kslots[p] > cpqr_kslots(pb.tg[p], pb.rlay[p], false)) ++pb.cpqr_slot;
          }
          else if (pb.v_off[p] >= 0)
            ++pb.cpqr_big;
      }
      // Householder steps of an interface, for the schedules: min(m, ncols) bounds the
      // rank; a refactorization at the same tolerance takes the rank that the interface
      // kept the last time, plus the step that stops
      auto est_steps = [&](const Prob& pb, int32_t p) -> int64_t {
        const spand_ctx* hq = pb.h;
        const int64_t ub = std::min<int64_t>(hq->num[t - 1].size[p], pb.ncols[p]);
        if (hq->last_rank_tol == tol && int64_t(hq->last_rank.size()) >= t) {
          const std::vector<int32_t>& lr = hq->last_rank[t - 1];
          if (p < int32_t(lr.size()) && lr[p] >= 0) return std::min<int64_t>(ub, int64_t(lr[p]) + 1);
        }
        return ub;
      };
      // A step whose work lies mostly in multi-slab interfaces runs all its colour
      // classes in one cooperative launch, where an interface waits on the device for
      // its neighbours of earlier classes only, not for the whole previous class.  Its
      // single-slab interfaces then run in that launch as teams of one slab (an
      // exchange with itself at every step).  A step with an interface beyond the
      // register layouts keeps the launches per class.
      bool unified = false;
      {
        int64_t w1 = 0, wm = 0;
        bool anybig = false;
        for (Prob* pp : act) {
          if (!orth(*pp)) continue;
          const SymStep& sy = pp->h->an.steps[t - 1];
          for (int32_t p = sy.ne; p < sy.nc; ++p) {
            if (pp->v_off[p] < 0) continue;
            if (pp->big[p]) {
              anybig = true;
              continue;
            }
            const int64_t e = est_steps(*pp, p);
            if (pp->slabS[p] > 1)
              wm += e * pp->slabS[p];
            else
              w1 += e;
          }
        }
        unified = !anybig && wm > 0 && 10 * w1 <= wm;
      }
      if (unified)
        for (Prob* pp : act) {
          if (!orth(*pp)) continue;
          Prob& pb = *pp;
          ++pb.cpqr_one_launch;
          const SymStep& sy = pb.h->an.steps[t - 1];
          for (int32_t p = sy.ne; p < sy.nc; ++p) {
            if (pb.v_off[p] < 0 || pb.slabS[p] > 1) continue;
            if (pb.wide[p]) {  // the standard layout of teams of 2 instead
              --pb.cpqr_ifaces[1];
              pb.wide[p] = 0;
              pb.slabS[p] = int32_t((pb.ncols[p] + cpqr_capacity(2, 0, true) - 1) / cpqr_capacity(2, 0, true));
              pb.kslots[p] = cpqr_kslots(2, 0, true);
              ++pb.cpqr_ifaces[pb.slabS[p] > 1 ? 2 : 0];
            }
            pb.xch_off[p] = xch_total;
            xch_total += 3 * int64_t(pb.slabS[p]) * cpqr_record(pb.tg[p], pb.rlay[p]);
          }
        }
      if ((st = dalloc(h, xchb, size_t(xch_total) * sizeof(double))) != SPAND_OK) return st;
      // the exchange headers start with tag 0; the first exchange of a buffer uses tag 1
      if (xch_total > 0) HIPCHK(hipMemsetAsync(xchb.p, 0, size_t(xch_total) * sizeof(double), h->stream));
      if ((st = dalloc(h, errb, sizeof(int32_t))) != SPAND_OK) return st;
      HIPCHK(hipMemsetAsync(errb.p, 0, sizeof(int32_t), h->stream));
      // finished slabs of every interface (the multi-slab kernel counts them)
      if ((st = dalloc(h, doneb, size_t(std::max<int64_t>(ncl, 1)) * sizeof(int32_t))) != SPAND_OK) return st;
      HIPCHK(hipMemsetAsync(doneb.p, 0, size_t(std::max<int64_t>(ncl, 1)) * sizeof(int32_t), h->stream));
      // current sizes: interfaces shrink to their rank as their colour class finishes
      if ((st = upload(h, curb, cur_h)) != SPAND_OK) return st;
      if ((st = upload(h, nrefb, std::vector<int32_t>(size_t(ncl), 0))) != SPAND_OK) return st;
      struct Ref { Prob* pb; int32_t p; };
      std::vector<std::vector<Ref>> by_colour(ncolour);
      for (Prob* pp : act) {
        if (!orth(*pp)) continue;
        const SymStep& sy = pp->h->an.steps[t - 1];
        for (int32_t p = sy.ne; p < sy.nc; ++p)
          if (pp->v_off[p] >= 0) by_colour[sy.colour[p]].push_back(Ref{pp, p});
      }
      struct CpqrLaunch {
        bool multi;
        int32_t G, nslab, nround;
        size_t lds, d0, s0;
        int32_t big_nseg = -1;  // >= 0: one global-memory launch of descriptor d0 with nslab workgroups
      };
      // scratch of the large-interface launches (they run one after another on the stream)
      int64_t big_m = 0, big_mn = 0, big_nc = 0;
      for (const auto& cl : by_colour)
        for (const Ref& f : cl)
          if (f.pb->big[f.p]) {
            const int64_t m = f.pb->h->num[t - 1].size[f.p], n = f.pb->ncols[f.p];
            big_m = std::max(big_m, m);
            big_mn = std::max(big_mn, m * n);
            big_nc = std::max(big_nc, n);
          }
      DevBuf bwk, bnrm, bpst, brb, bpost, bpcd, bbar;
      if (big_m > 0) {
        if ((st = dalloc(h, bwk, size_t(big_mn) * sizeof(double))) != SPAND_OK) return st;
        if ((st = dalloc(h, bnrm, size_t(big_nc) * sizeof(double))) != SPAND_OK) return st;
        if ((st = dalloc(h, bpst, size_t(big_nc) * sizeof(int32_t))) != SPAND_OK) return st;
        if ((st = dalloc(h, brb, size_t(std::min(big_m, big_nc)) * sizeof(double))) != SPAND_OK) return st;
        if ((st = dalloc(h, bpost, 1024 * sizeof(double))) != SPAND_OK) return st;
        if ((st = dalloc(h, bpcd, 1024 * sizeof(int32_t))) != SPAND_OK) return st;
        if ((st = dalloc(h, bbar, 256)) != SPAND_OK) return st;
      }
      // Each colour class is planned, uploaded and launched before the next one is
      // planned, so the GPU runs a colour while the host plans the next.  The
      // descriptor buffers of the colours stay allocated until the step ends.
      std::vector<DevBuf> colour_bufs;
      hipEvent_t b_done = nullptr;  // the last multi-slab launch on the second stream
      bool b_pending = false;       // ... not yet waited for on the handle's stream
      // launch groups of one colour: single-slab interfaces per team size G
      // (group G), the wide single-slab ones (group 128), then every multi-slab
      // interface of the colour together (group 256)
      if (unified) {
        // Every interface by its estimated path to the end of the step: its own steps
        // plus the longest such path among the neighbours of later classes that wait for
        // it.  A neighbour an interface waits for has a longer path, so this order
        // (that of the workgroups' lists) puts it first; the longest chains start first.
        std::vector<int64_t> bl(size_t(ncl), 0);
        for (int32_t c = ncolour - 1; c >= 0; --c)
          for (const Ref& f : by_colour[c]) {
            const Prob& pb = *f.pb;
            const SymStep& sy = pb.h->an.steps[t - 1];
            int64_t below = 0;
            for (int64_t e = sy.nb_ptr[f.p]; e < sy.nb_ptr[f.p + 1]; ++e) {
              const int32_t q = sy.nb[e];
              if (pb.v_off[q] >= 0 && sy.colour[q] > c) below = std::max(below, bl[size_t(pb.cbase + q)]);
            }
            bl[size_t(pb.cbase + f.p)] = est_steps(pb, f.p) + below;
          }
        std::vector<Ref> plist;
        for (int32_t c = 0; c < ncolour; ++c) plist.insert(plist.end(), by_colour[c].begin(), by_colour[c].end());
        auto colour_of = [&](const Ref& f) { return f.pb->h->an.steps[t - 1].colour[f.p]; };
        std::stable_sort(plist.begin(), plist.end(), [&](const Ref& x, const Ref& y) {
          const int64_t bx = bl[size_t(x.pb->cbase + x.p)], by = bl[size_t(y.pb->cbase + y.p)];
          if (bx != by) return bx > by;
          if (colour_of(x) != colour_of(y)) return colour_of(x) < colour_of(y);
          return x.pb->h->num[t - 1].size[x.p] > y.pb->h->num[t - 1].size[y.p];
        });
        size_t lds = 0, total = 0;
        for (const Ref& f : plist) {
          lds = std::max(lds, cpqr_lds_bytes(f.pb->tg[f.p], f.pb->rlay[f.p], f.pb->nseg[f.p]));
          total += size_t(f.pb->slabS[f.p]);
        }
        const int cap = cpqr_max_coresident(lds);
        if (cap <= 0) return set_err(h, SPAND_E_HIP, "occupancy query for the CPQR kernel failed");
        std::vector<SparsDesc> sds;
        std::vector<SegDesc> segs;
        std::vector<int2> deps;
        size_t nsegs = 0;
        for (const Ref& f : plist) nsegs += size_t(f.pb->nseg[f.p]);
        sds.reserve(plist.size());
        segs.reserve(nsegs);
        deps.reserve(nsegs);
        // List scheduling over the co-resident workgroups as for one class, with an
        // interface's start no earlier than the estimated end of the neighbours it
        // waits for
        const size_t grid = std::min(total, size_t(cap));
        std::vector<std::vector<SlabRef>> lists(grid);
        using Slot = std::pair<int64_t, int32_t>;  // (time the workgroup frees up, workgroup)
        std::vector<Slot> heap(grid);
        for (size_t b = 0; b < grid; ++b) heap[b] = Slot{0, int32_t(b)};
        std::make_heap(heap.begin(), heap.end(), std::greater<Slot>());
        std::vector<int64_t> fin(size_t(ncl), 0);  // estimated end of every interface
        std::vector<int32_t> wg;
        for (const Ref& f : plist) {
          Prob& pb = *f.pb;
          const int32_t p = f.p;
          const StepNum& sn = pb.h->num[t - 1];
          const SymStep& sy = pb.h->an.steps[t - 1];
          const Layout& lay = pb.lay;
          double* A = pb.arena.as<double>();
          const int32_t S = pb.slabS[p];
          if (S > cap) return set_err(h, SPAND_E_INVALID, "interface needs more co-resident workgroups than the GPU holds");
          SparsDesc d{};
          d.V = sn.house.as<double>() + pb.v_off[p];
          d.ldv = pad16(sn.size[p]);
          d.tau = sn.house.as<double>() + pb.tau_off[p];
          d.diag = A + lay.base[p];
          d.ldd = int32_t(lay.H[p]);
          d.m = sn.size[p];
          d.id = int32_t(pb.cbase + p);
          d.S = S;
          d.G = pb.tg[p];
          d.lay = pb.rlay[p];
          d.kslots = pb.kslots[p];
          d.xch = xchb.as<double>() + pb.xch_off[p];
          d.seg_begin = int32_t(segs.size());
          d.dep_begin = int32_t(deps.size());
          int64_t ready = 0;
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
            g.q = int32_t(pb.cbase + q);
            segs.push_back(g);
            if (pb.v_off[q] >= 0 && sy.colour[q] < sy.colour[p]) {
              deps.push_back(make_int2(int32_t(pb.cbase + q), pb.slabS[q]));
              ready = std::max(ready, fin[size_t(pb.cbase + q)]);
            }
          }
          d.seg_end = int32_t(segs.size());
          d.dep_end = int32_t(deps.size());
          wg.clear();
          int64_t tt = ready;
          for (int32_t k = 0; k < S; ++k) {
            std::pop_heap(heap.begin(), heap.end(), std::greater<Slot>());
            tt = std::max(tt, heap.back().first);
            wg.push_back(heap.back().second);
            heap.pop_back();
          }
          tt += est_steps(pb, p);
          fin[size_t(pb.cbase + p)] = tt;
          for (int32_t k = 0; k < S; ++k) {
            lists[size_t(wg[k])].push_back(SlabRef{int32_t(sds.size()), k});
            heap.push_back(Slot{tt, wg[k]});
            std::push_heap(heap.begin(), heap.end(), std::greater<Slot>());
          }
          sds.push_back(d);
        }
        size_t nround = 0;
        for (const auto& l : lists) nround = std::max(nround, l.size());
        std::vector<SlabRef> slabs;
        slabs.reserve(nround * grid);
        for (size_t k = 0; k < nround; ++k)
          for (size_t b = 0; b < grid; ++b) slabs.push_back(k < lists[b].size() ? lists[b][k] : SlabRef{-1, 0});
        DevBuf a, b, sl, dp;
        if ((st = upload_big(h, a, sds)) != SPAND_OK) return st;
        if ((st = upload_big(h, b, segs)) != SPAND_OK) return st;
        if ((st = upload_big(h, sl, slabs)) != SPAND_OK) return st;
        if (deps.empty()) deps.push_back(make_int2(0, 0));
        if ((st = upload_big(h, dp, deps)) != SPAND_OK) return st;
        hipEvent_t cstart, e1;
        HIPCHK(joinev.get(njoin, &cstart));
        HIPCHK(hipEventRecord(cstart, h->stream));
        colour_span.push_back(ColourSpan{njoin++, nlaunch, nlaunch + 1});
        HIPCHK(evpool.get(2 * nlaunch, &e1));  // the start event of the launch is not read
        HIPCHK(evpool.get(2 * nlaunch + 1, &e1));
        const hipError_t le =
            launch_cpqr_multi(a.as<SparsDesc>(), sl.as<SlabRef>(), int32_t(grid), int32_t(nround), b.as<SegDesc>(),
                              tol, curb.as<int32_t>(), nrefb.as<int32_t>(), errb.as<int32_t>(), dp.as<int2>(),
                              doneb.as<int32_t>(), lds, h->stream);
        if (le != hipSuccess) return set_err(h, SPAND_E_HIP, std::string("sparsification launch: ") + hipGetErrorString(le));
        HIPCHK(hipEventRecord(e1, h->stream));
        ++nlaunch;
        colour_bufs.push_back(std::move(a));
        colour_bufs.push_back(std::move(b));
        colour_bufs.push_back(std::move(sl));
        colour_bufs.push_back(std::move(dp));
      }
      for (int32_t c = 0; c < ncolour && !unified; ++c) {
        if (by_colour[c].empty()) continue;
        std::vector<CpqrLaunch> launches;
        std::vector<SparsDesc> all_sds;
        std::vector<SegDesc> all_segs;
        std::vector<SlabRef> all_slabs;
        for (int32_t grp = 1; grp <= 256; grp <<= 1) {
          const bool multi = grp == 256, wgrp = grp == 128;
          std::vector<Ref> plist;
          for (const Ref& f : by_colour[c]) {
            const Prob& pb = *f.pb;
            const int32_t p = f.p;
            if (pb.big[p]) continue;
            if (multi ? pb.slabS[p] > 1
                      : wgrp ? pb.wide[p] != 0 : (pb.slabS[p] == 1 && !pb.wide[p] && pb.tg[p] == grp))
              plist.push_back(f);
          }
          if (plist.empty()) continue;
          auto msize = [&](const Ref& f) { return f.pb->h->num[t - 1].size[f.p]; };
          auto steps_est = [&](const Ref& f) { return est_steps(*f.pb, f.p); };
          // longest first: interfaces of similar step counts share a launch
          std::stable_sort(plist.begin(), plist.end(), [&](const Ref& x, const Ref& y) {
            if (multi) {
              const int64_t ex = steps_est(x), ey = steps_est(y);
              return ex != ey ? ex > ey : msize(x) > msize(y);
            }
            return int64_t(msize(x)) * x.pb->ncols[x.p] > int64_t(msize(y)) * y.pb->ncols[y.p];
          });
          size_t lds = 0;
          for (const Ref& f : plist)
            lds = std::max(lds, wgrp ? cpqr_wide_lds_bytes(f.pb->nseg[f.p])
                                     : cpqr_lds_bytes(f.pb->tg[f.p], f.pb->rlay[f.p], f.pb->nseg[f.p]));
          int cap = INT_MAX;
          if (multi) {
            cap = cpqr_max_coresident(lds);
            if (cap <= 0) return set_err(h, SPAND_E_HIP, "occupancy query for the CPQR kernel failed");
          }
          // The chunks of at most cap co-resident slabs: one plain launch each for the
          // single-slab interfaces; for the multi-slab ones, the rounds of one launch.
          CpqrLaunch Lc{};
          Lc.multi = multi;
          Lc.G = multi ? 0 : grp;  // 128: the wide layout
          Lc.lds = lds;
          Lc.d0 = all_sds.size();
          std::vector<std::vector<SlabRef>> rounds;
          size_t pos = 0;
          while (pos < plist.size()) {
            std::vector<SlabRef> rd;
            while (pos < plist.size()) {
              const Prob& pb = *plist[pos].pb;
              const int32_t p = plist[pos].p;
              const StepNum& sn = pb.h->num[t - 1];
              const SymStep& sy = pb.h->an.steps[t - 1];
              const Layout& lay = pb.lay;
              double* A = pb.arena.as<double>();
              if (multi && pb.slabS[p] > cap)
                return set_err(h, SPAND_E_INVALID, "interface needs more co-resident workgroups than the GPU holds");
              if (multi && !rd.empty() && int64_t(rd.size()) + pb.slabS[p] > cap) break;
              SparsDesc d{};
              d.V = sn.house.as<double>() + pb.v_off[p];
              d.ldv = pad16(sn.size[p]);
              d.tau = sn.house.as<double>() + pb.tau_off[p];
              d.diag = A + lay.base[p];
              d.ldd = int32_t(lay.H[p]);
              d.m = sn.size[p];
              d.id = int32_t(pb.cbase + p);
              d.S = pb.slabS[p];
              d.G = pb.tg[p];
              d.lay = pb.rlay[p];
              d.kslots = pb.kslots[p];
              if (multi) d.xch = xchb.as<double>() + pb.xch_off[p];
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
                g.q = int32_t(pb.cbase + q);
                all_segs.push_back(g);
              }
              d.seg_end = int32_t(all_segs.size());
              for (int32_t w = 0; w < pb.slabS[p]; ++w) rd.push_back(SlabRef{int32_t(all_sds.size() - Lc.d0), w});
              all_sds.push_back(d);
              ++pos;
            }
            rounds.push_back(std::move(rd));
          }
          if (!multi) {
            for (const auto& rd : rounds) {
              CpqrLaunch Pl = Lc;
              Pl.s0 = all_slabs.size();
              Pl.nslab = int32_t(rd.size());
              Pl.nround = 1;
              all_slabs.insert(all_slabs.end(), rd.begin(), rd.end());
              launches.push_back(Pl);
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
            if (ifs.size() != plist.size())
              return set_err(h, SPAND_E_INVALID, "sparsification schedule: interfaces and slabs disagree");
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
              const Ref& f = plist[q];
              const int32_t S = ifs[q].second;
              wg.clear();
              int64_t tt = 0;
              for (int32_t k = 0; k < S; ++k) {
                std::pop_heap(heap.begin(), heap.end(), std::greater<Slot>());
                tt = std::max(tt, heap.back().first);
                wg.push_back(heap.back().second);
                heap.pop_back();
              }
              tt += steps_est(f);
              for (int32_t k = 0; k < S; ++k) {
                lists[wg[k]].push_back(ifs[q].first[k]);
                heap.push_back(Slot{tt, wg[k]});
                std::push_heap(heap.begin(), heap.end(), std::greater<Slot>());
              }
            }
            size_t nround = 0;
            for (const auto& l : lists) nround = std::max(nround, l.size());
            Lc.s0 = all_slabs.size();
            Lc.nslab = int32_t(grid);
            Lc.nround = int32_t(nround);
            for (size_t k = 0; k < nround; ++k)
              for (size_t b = 0; b < grid; ++b) all_slabs.push_back(k < lists[b].size() ? lists[b][k] : SlabRef{-1, 0});
            launches.push_back(Lc);
          }
        }
        // the interfaces of this colour beyond the register layouts, one launch each
        for (const Ref& f : by_colour[c]) {
          const Prob& pb = *f.pb;
          const int32_t p = f.p;
          if (!pb.big[p]) continue;
          const StepNum& sn = pb.h->num[t - 1];
          const SymStep& sy = pb.h->an.steps[t - 1];
          const Layout& lay = pb.lay;
          double* A = pb.arena.as<double>();
          SparsDesc d{};
          d.V = sn.house.as<double>() + pb.v_off[p];
          d.ldv = pad16(sn.size[p]);
          d.tau = sn.house.as<double>() + pb.tau_off[p];
          d.diag = A + lay.base[p];
          d.ldd = int32_t(lay.H[p]);
          d.m = sn.size[p];
          d.id = int32_t(pb.cbase + p);
          d.S = 1;
          d.seg_begin = int32_t(all_segs.size());
          for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e) {
            const int32_t q = sy.nb[e];
            if (sn.size[q] == 0) continue;
            SegDesc g{};
            if (q < p) {
              g.blk = A + lay.base[q] + lay.find(p, q);
              g.ld = int32_t(lay.H[q]);
              g.trans = 0;
            } else {
              g.blk = A + lay.base[p] + lay.find(q, p);
              g.ld = int32_t(lay.H[p]);
              g.trans = 1;
            }
            g.q = int32_t(pb.cbase + q);
            all_segs.push_back(g);
          }
          d.seg_end = int32_t(all_segs.size());
          const int capb = cpqr_big_max_coresident(pb.nseg[p]);
          if (capb <= 0) return set_err(h, SPAND_E_HIP, "occupancy query for the large-interface CPQR failed");
          CpqrLaunch Lb{};
          Lb.multi = false;
          Lb.big_nseg = pb.nseg[p];
          Lb.d0 = all_sds.size();
          // at most 1024 workgroups: the size of the launch's post arrays
          Lb.nslab = int32_t(std::max<int64_t>(1, std::min<int64_t>(std::min(capb, 1024), (pb.ncols[p] + 15) / 16)));
          all_sds.push_back(d);
          launches.push_back(Lb);
        }
        // this colour's launches: one upload of each descriptor list, then the launches.
        // The multi-slab launch runs on the second stream beside the single-slab ones
        // (independent interfaces of one colour; the single-slab workgroups never
        // wait, so the multi-slab ones always get their CUs); the large-interface
        // launches, which hold grid barriers, run after it.
        DevBuf a, b, sl;
        if ((st = upload_big(h, a, all_sds)) != SPAND_OK) return st;
        if ((st = upload_big(h, b, all_segs)) != SPAND_OK) return st;
        if ((st = upload_big(h, sl, all_slabs)) != SPAND_OK) return st;
        if (b_pending) {  // the previous colour's multi-slab launch
          HIPCHK(hipStreamWaitEvent(h->stream, b_done, 0));
          b_pending = false;
        }
        // start of the colour on the handle's stream: after everything before it,
        // this colour's uploads included; the CPQR time of the colour runs from here
        // to the last end of its launches on either stream
        hipEvent_t cstart;
        HIPCHK(joinev.get(njoin, &cstart));
        HIPCHK(hipEventRecord(cstart, h->stream));
        colour_span.push_back(ColourSpan{njoin++, nlaunch, 0});
        auto issue = [&](const CpqrLaunch& Lc, hipStream_t sq) -> spand_status {
          hipEvent_t e0, e1;
          HIPCHK(evpool.get(2 * nlaunch, &e0));
          HIPCHK(evpool.get(2 * nlaunch + 1, &e1));
          HIPCHK(hipEventRecord(e0, sq));
          const SparsDesc* dd = a.as<SparsDesc>() + Lc.d0;
          const SlabRef* ss = sl.as<SlabRef>() + Lc.s0;
          hipError_t le;
          if (Lc.big_nseg >= 0) {
            HIPCHK(hipMemsetAsync(bbar.p, 0, 256, sq));
            le = launch_cpqr_big(all_sds[Lc.d0], Lc.big_nseg, b.as<SegDesc>(), tol, curb.as<int32_t>(),
                                 nrefb.as<int32_t>(), errb.as<int32_t>(), Lc.nslab, bwk.as<double>(), bnrm.as<double>(),
                                 bpst.as<int32_t>(), brb.as<double>(), bpost.as<double>(), bpcd.as<int32_t>(),
                                 bbar.as<uint32_t>(), sq);
          } else if (Lc.multi) {
            le = launch_cpqr_multi(dd, ss, Lc.nslab, Lc.nround, b.as<SegDesc>(), tol, curb.as<int32_t>(),
                                   nrefb.as<int32_t>(), errb.as<int32_t>(), nullptr, doneb.as<int32_t>(), Lc.lds,
                                   sq);
          } else if (Lc.G == 128) {
            le = launch_cpqr_one_wide(dd, ss, Lc.nslab, b.as<SegDesc>(), tol, curb.as<int32_t>(), nrefb.as<int32_t>(),
                                      errb.as<int32_t>(), Lc.lds, sq);
          } else {
            le = launch_cpqr_one(Lc.G, dd, ss, Lc.nslab, b.as<SegDesc>(), tol, curb.as<int32_t>(), nrefb.as<int32_t>(),
                                 errb.as<int32_t>(), Lc.lds, sq);
          }
          if (le != hipSuccess)
            return set_err(h, SPAND_E_HIP, std::string("sparsification launch: ") + hipGetErrorString(le));
          HIPCHK(hipEventRecord(e1, sq));
          ++nlaunch;
          return SPAND_OK;
        };
        for (const CpqrLaunch& Lc : launches) {
          if (!Lc.multi) continue;
          if (!h->stream2) HIPCHK(hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking));
          HIPCHK(hipStreamWaitEvent(h->stream2, cstart, 0));
          if ((st = issue(Lc, h->stream2)) != SPAND_OK) return st;
          HIPCHK(joinev.get(njoin++, &b_done));
          HIPCHK(hipEventRecord(b_done, h->stream2));
          b_pending = true;
        }
        // the single-slab launches (independent interfaces) alternate between the
        // handle's stream and a third one, so that one launch's last workgroups run
        // beside the next one's first
        {
          int nsingle = 0;
          for (const CpqrLaunch& Lc : launches) nsingle += (!Lc.multi && Lc.big_nseg < 0) ? 1 : 0;
          if (nsingle > 1 && !h->stream3) HIPCHK(hipStreamCreateWithFlags(&h->stream3, hipStreamNonBlocking));
          if (nsingle > 1) HIPCHK(hipStreamWaitEvent(h->stream3, cstart, 0));
          int k = 0;
          for (const CpqrLaunch& Lc : launches)
            if (!Lc.multi && Lc.big_nseg < 0 && (st = issue(Lc, (k++ & 1) ? h->stream3 : h->stream)) != SPAND_OK)
              return st;
          if (nsingle > 1) {
            hipEvent_t s3;
            HIPCHK(joinev.get(njoin++, &s3));
            HIPCHK(hipEventRecord(s3, h->stream3));
            HIPCHK(hipStreamWaitEvent(h->stream, s3, 0));
          }
        }
        for (const CpqrLaunch& Lc : launches) {
          if (Lc.big_nseg < 0) continue;
          if (b_pending) {
            HIPCHK(hipStreamWaitEvent(h->stream, b_done, 0));
            b_pending = false;
          }
          if ((st = issue(Lc, h->stream)) != SPAND_OK) return st;
        }
        colour_span.back().l1 = nlaunch;
        colour_bufs.push_back(std::move(a));
        colour_bufs.push_back(std::move(b));
        colour_bufs.push_back(std::move(sl));
      }
      if (b_pending) HIPCHK(hipStreamWaitEvent(h->stream, b_done, 0));
      HIPCHK(hipEventRecord(ph[4], h->stream));
    }
    // ---- interpolative sparsification (Sec. 2.6.2) of the problems that ask for it
    for (Prob* pp : act) {
      const SymStep& sy = pp->h->an.steps[t - 1];
      if (!(pp->sparsify && sy.nc > sy.ne && pp->h->variant != SPAND_ORTHS)) continue;
      if ((st = sparsify_interp(*pp, t, tol, cpqr_ms, cpqr_launches)) != SPAND_OK) return st;
      HIPCHK(hipEventRecord(ph[4], h->stream));
    }

    // ---- the flags of every problem and the ranks go to pinned host memory right
    // behind the step's kernels; the previous step's T factors and apply descriptors
    // are enqueued after those copies, and the host waits for the copies only, so the
    // GPU builds those factors while the host plans the next step
    int32_t* pin = reinterpret_cast<int32_t*>(h->stage.get((hflags.size() + 2 * size_t(ncl) + 1) * sizeof(int32_t)));
    if (!pin) return set_err(h, SPAND_E_NOMEM, "pinned staging for the rank read-back failed");
    int32_t* pin_rk = pin + hflags.size();
    int32_t* pin_nref = pin_rk + ncl;
    int32_t* pin_err = pin_nref + ncl;
    *pin_err = 0;
    HIPCHK(hipMemcpyAsync(pin, dflag.p, hflags.size() * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    if (any_orth) {
      HIPCHK(hipMemcpyAsync(pin_rk, curb.p, size_t(ncl) * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipMemcpyAsync(pin_nref, nrefb.p, size_t(ncl) * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipMemcpyAsync(pin_err, errb.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    }
    hipEvent_t readback;
    HIPCHK(rbev.get(size_t(t - 1), &readback));
    HIPCHK(hipEventRecord(readback, h->stream));
    {
      std::vector<TDesc> tds;
      for (Prob& pb : P) {
        tds.insert(tds.end(), pb.t_pending.begin(), pb.t_pending.end());
        pb.t_pending.clear();
      }
      if ((st = build_t_factors(h, tds)) != SPAND_OK) return st;
    }
    for (Prob& pb : P) {
      if (pb.pending.t == 0) continue;
      const int32_t pt = pb.pending.t;
      pb.pending.t = 0;
      if (!pb.live) continue;
      if ((st = build_apply(pb.h, pb.h->an.steps[pt - 1], pb.h->num[pt - 1], pb.lay_prev, pb.pending)) != SPAND_OK)
        return st;
      if (NP == 1 && pb.frozen.size() > pb.frozen_up) {  // the dofs frozen so far
        if ((st = stage_copy(pb.h, pb.h->d_inv.as<int32_t>() + pb.frozen_up, pb.frozen.data() + pb.frozen_up,
                             (pb.frozen.size() - pb.frozen_up) * sizeof(int32_t))) != SPAND_OK)
          return st;
        pb.frozen_up = pb.frozen.size();
      }
    }
    HIPCHK(hipEventSynchronize(readback));
    std::copy(pin, pin + hflags.size(), hflags.begin());
    std::vector<int32_t> rk(pin_rk, pin_rk + ncl), nrefh(pin_nref, pin_nref + ncl);
    const int32_t serr = *pin_err;
    if (serr) return set_err(h, SPAND_E_HIP, "sparsification slab exchange timed out");
    for (const ColourSpan& cs : colour_span) {  // the launches of a colour overlap
      float span = 0.f;
      for (size_t q = cs.l0; q < cs.l1; ++q) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, joinev.ev[cs.ev], evpool.ev[2 * q + 1]));
        span = std::max(span, ms);
      }
      cpqr_ms += span;
    }
    colour_span.clear();
    cpqr_launches += int64_t(nlaunch);
    // Kernels that ran after a failure in the same step only saw bad values, never bad
    // indices; the failed problem stops here, the others go on.
    for (Prob* pp : act) {
      Prob& pb = *pp;
      const int32_t q = int32_t(pp - P.data());
      const int32_t* fl = hflags.data() + 4 * q;
      spand_ctx* hq = pb.h;
      if (fl[2]) {
        fail_problem(pb, SPAND_E_INVALID, "matrix values contain NaN or Inf");
      } else if (fl[0] != FAIL_NONE) {
        hq->stats.fail_step = t;
        hq->stats.fail_cluster = fl[0];
        hq->stats.fail_phase = 0;
        fail_problem(pb, SPAND_E_NOT_SPD, "pivot block not SPD at step " + std::to_string(t) + ", cluster " +
                                              std::to_string(fl[0]) + " (elimination)");
      } else if (fl[1] != FAIL_NONE) {
        hq->stats.fail_step = t;
        hq->stats.fail_cluster = fl[1];
        hq->stats.fail_phase = 1;
        fail_problem(pb, SPAND_E_NOT_SPD, "interface block not SPD at step " + std::to_string(t) + ", cluster " +
                                              std::to_string(fl[1]) + " (scaling)");
      } else if (fl[3] != FAIL_NONE) {
        hq->stats.fail_step = t;
        hq->stats.fail_cluster = fl[3];
        hq->stats.fail_phase = 2;
        fail_problem(pb, SPAND_E_NOT_SPD, "C_ff not SPD at step " + std::to_string(t) + ", cluster " +
                                              std::to_string(fl[3]) + " (interpolative sparsification)");
      }
      if (!pb.live) {
        pb.t_pending.clear();
        pb.arena.release();
        pb.arena_prev.release();
        hq->num.clear();
        continue;
      }
      const SymStep& sy = hq->an.steps[t - 1];
      StepNum& sn = hq->num[t - 1];
      const int32_t nc = sy.nc, ne = sy.ne;
      if (orth(pb)) {
        std::vector<TDesc> tds;
        for (int32_t p = ne; p < nc; ++p)
          if (pb.v_off[p] >= 0) {
            sn.rank[p] = rk[pb.cbase + p];
            const int64_t r = nrefh[pb.cbase + p];
            pb.nref[p] = int32_t(r);
            {
              // sum over steps j < r of 2 (m-j)(n-j) + 4 (m-j)(n-j-1) + 3 (m-j)
              // = 6 (m-j)(n-j) - (m-j), in closed form (exact in 64-bit integers)
              const int64_t m = sn.size[p], nq = pb.ncols[p];
              const int64_t s1 = r * (r - 1) / 2, s2 = (r - 1) * r * (2 * r - 1) / 6;
              const int64_t f = 6 * (r * m * nq - (m + nq) * s1 + s2) - (r * m - s1);
              pb.cpqr_flops += double(f);
              if (r < std::min<int64_t>(m, nq)) pb.cpqr_flops += 2.0 * double(m - r) * double(nq - r);
            }
            pb.m_F += (2 * int64_t(sn.size[p]) - r + 1) * r / 2 + r;
            if (r > 0)
              tds.push_back(TDesc{sn.house.as<double>() + pb.v_off[p], sn.house.as<double>() + pb.tau_off[p],
                                  sn.house.as<double>() + pb.t_off[p], sn.size[p], int32_t(r), pad16(sn.size[p]),
                                  pad16(int32_t(r))});
          }
        // the compact-WY factors are only read by the apply: they are built while the
        // next step runs
        pb.t_pending = std::move(tds);
      }
      if (NP == 1) frozen_at(sy, sn, pb.frozen);
      if (t <= 32) hq->stats.step_m_F[t - 1] = pb.m_F;
      pb.pending = ApplyPlan{t, std::move(pb.ed_off), std::move(pb.sc_off), std::move(pb.v_off), std::move(pb.t_off),
                             std::move(pb.nN), std::move(pb.nref), std::move(pb.iso_off)};
      pb.arena_prev = std::move(pb.arena);
      pb.lay_prev = std::move(pb.lay);
    }
  }
  {
    std::vector<TDesc> tds;
    for (Prob& pb : P) {
      tds.insert(tds.end(), pb.t_pending.begin(), pb.t_pending.end());
      pb.t_pending.clear();
    }
    if ((st = build_t_factors(h, tds)) != SPAND_OK) return st;
  }
  for (Prob& pb : P) {
    if (pb.pending.t == 0 || !pb.live) continue;
    const int32_t pt = pb.pending.t;
    pb.pending.t = 0;
    if ((st = build_apply(pb.h, pb.h->an.steps[pt - 1], pb.h->num[pt - 1], pb.lay_prev, pb.pending)) != SPAND_OK)
      return st;
  }
  // (a batch solves in vertex order, through the host's slot lists: no freeze order)
  DevBuf badperm;
  int32_t* pin_bad = nullptr;
  if (NP == 1 && P[0].live) {
    if ((st = freeze_order(P[0].h, P[0].frozen, P[0].frozen_up, badperm)) != SPAND_OK) return st;
    pin_bad = reinterpret_cast<int32_t*>(h->stage.get(sizeof(int32_t)));
    if (!pin_bad) return set_err(h, SPAND_E_NOMEM, "pinned staging for the freeze-order check failed");
    HIPCHK(hipMemcpyAsync(pin_bad, badperm.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  if (pin_bad && *pin_bad) {
    P[0].h->d_pos.release();
    P[0].h->d_inv.release();
    return set_err(h, SPAND_E_INVALID, "freeze order is not a permutation");
  }
  double elim_ms = 0.0;
  double phase_s[32][4] = {};
  for (int32_t t = 1; t <= Lmax && 5 * size_t(t) <= phev.ev.size(); ++t) {  // phase times from the events of every step
    hipEvent_t ph[5];
    for (int q = 0; q < 5; ++q) ph[q] = phev.ev[5 * size_t(t - 1) + q];
    float ms[4] = {0.f, 0.f, 0.f, 0.f};
    HIPCHK(hipEventElapsedTime(&ms[0], ph[0], ph[1]));
    HIPCHK(hipEventElapsedTime(&ms[1], ph[1], ph[2]));
    HIPCHK(hipEventElapsedTime(&ms[2], ph[2], ph[3]));
    HIPCHK(hipEventElapsedTime(&ms[3], ph[3], ph[4]));
    if (t <= 32)
      for (int q = 0; q < 4; ++q) phase_s[t - 1][q] = 1e-3 * ms[q];
    if (elim_ran[t]) elim_ms += ms[1];
  }
  for (Prob& pb : P) {
    pb.arena_prev.release();
    if (!pb.live) continue;
    pb.h->last_rank.resize(pb.h->num.size());
    for (size_t q = 0; q < pb.h->num.size(); ++q) pb.h->last_rank[q] = pb.h->num[q].rank;
    pb.h->last_rank_tol = tol;
    spand_stats& s = pb.h->stats;
    std::memcpy(s.step_phase_seconds, phase_s, sizeof(phase_s));
    s.m_F = pb.m_F;
    s.s_top = pb.s_top;
    s.schur_flops = pb.elim_flops;
    s.schur_seconds = elim_ms * 1e-3;
    s.cpqr_flops = pb.cpqr_flops;
    s.cpqr_seconds = cpqr_ms * 1e-3;
    s.cpqr_launches = cpqr_launches;
    for (int q = 0; q < 4; ++q) s.cpqr_interfaces[q] = pb.cpqr_ifaces[q];
    s.cpqr_big_interfaces = pb.cpqr_big;
    s.cpqr_one_launch_steps = pb.cpqr_one_launch;
    s.cpqr_lds_slot_interfaces = pb.cpqr_slot;
    s.apply_scratch_per_rhs = std::max<int64_t>(pb.h->max_tmp, 1) + std::max<int64_t>(pb.h->max_gather, 1) +
                              (pb.h->d_inv.p ? pb.h->an.n : 0);
    for (int q = 0; q < 3; ++q) s.apply_interfaces[q] = 0;
    for (const StepNum& sn : pb.h->num) {
      s.apply_interfaces[0] += sn.n_iface1;
      s.apply_interfaces[1] += sn.n_iface2;
      s.apply_interfaces[2] += sn.n_scale - sn.n_iso;
    }
  }
  return SPAND_OK;
}

}  // namespace

spand_status factor_numeric(spand_ctx* h, const double* values, double tol, int32_t skip, spand_prec prec) {
  std::vector<Prob> P(1);
  P[0].h = h;
  P[0].values = values;
  spand_status st = factor_run(P, tol, skip, prec);
  if (st == SPAND_OK && !P[0].live) {
    // the problem's own failure: its status is in the error text's class
    st = h->stats.fail_step >= 0 ? SPAND_E_NOT_SPD : SPAND_E_INVALID;
  }
  return st;
}

spand_status factor_numeric_batch(spand_ctx* const* hs, const double* const* values, int32_t np, double tol,
                                  int32_t skip, spand_prec prec, spand_status* per) {
  std::vector<Prob> P(np);
  for (int32_t q = 0; q < np; ++q) {
    P[q].h = hs[q];
    P[q].values = values[q];
  }
  spand_status st = factor_run(P, tol, skip, prec);
  for (int32_t q = 0; q < np; ++q) {
    if (st != SPAND_OK) {
      per[q] = st;
      if (q > 0) set_err(hs[q], st, "batched factor: " + hs[0]->err);
    } else if (!P[q].live) {
      per[q] = hs[q]->stats.fail_step >= 0 ? SPAND_E_NOT_SPD : SPAND_E_INVALID;
    } else {
      per[q] = SPAND_OK;
    }
  }
  return st;
}

}  // namespace spand
