// Numerical factorization driver: Algorithm 3 (OrthS) level by level on the GPU.
//
// Storage.  At step t the trailing matrix lives in one device arena as column
// panels: the panel of cluster j stacks the dense blocks (i, j), i >= j, of the
// block pattern (diagonal block first, then the others in ascending i), column-
// major with the panel height as leading dimension.  Eliminated clusters come
// first in the canonical order, so the panel of an eliminated s is exactly
// [A_ss; A_{N_s s}].
//
// Per step (t = 1..L, level l = L - t + 1):
//   1. assemble: scatter the CSR values (t = 1) or merge the previous arena
//      (Sec. 2.7: parent blocks are the concatenation of child blocks);
//   2. eliminate every level-l cluster s (Sec. 2.4): L_s = chol(A_ss) and
//      L_s^{-1}; G = A_{N_s s} L_s^{-T}; C_s = G G^T; every target block
//      subtracts its contributions in ascending s (deterministic);
//   3. if t > skip and l > 1: scale every remaining cluster (Sec. 2.5):
//      L_p = chol(A_pp); A_ij <- L_i^{-1} A_ij L_j^{-T}; A_pp <- I;
//   4. then sparsify every remaining cluster, one colour class per launch
//      (Sec. 2.6.1), and read the kept ranks back to the host;
//   5. plan the next step's layout from the ranks.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>

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
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return set_err(h, SPAND_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return SPAND_OK;
}

template <typename T>
spand_status upload(spand_ctx* h, DevBuf& b, const std::vector<T>& v) {
  spand_status st = dalloc(h, b, v.size() * sizeof(T));
  if (st != SPAND_OK) return st;
  if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
  return SPAND_OK;
}

// Column-panel layout of one step's arena.
struct Layout {
  std::vector<int64_t> pan_ptr;  // nc+1
  std::vector<int32_t> prow;     // row cluster of each panel entry (diagonal first)
  std::vector<int64_t> proff;    // row offset of each entry inside its panel
  std::vector<int64_t> H;        // panel heights
  std::vector<int64_t> base;     // panel start (elements)
  int64_t total = 0;
  int64_t find(int32_t i, int32_t j) const {
    auto b = prow.begin() + pan_ptr[j], e = prow.begin() + pan_ptr[j + 1];
    auto it = std::lower_bound(b, e, i);
    if (it == e || *it != i) return -1;
    return proff[it - prow.begin()];
  }
};

void build_layout(const SymStep& st, const std::vector<int32_t>& size, Layout& L) {
  const int32_t nc = st.nc, ne = st.ne;
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
  int64_t tot = 0;
  for (int32_t j = 0; j < nc; ++j) {
    int64_t h = 0;
    for (int64_t e = L.pan_ptr[j]; e < L.pan_ptr[j + 1]; ++e) {
      L.proff[e] = h;
      h += size[L.prow[e]];
    }
    L.H[j] = h;
    L.base[j] = tot;
    tot += h * size[j];
  }
  L.total = tot;
}

void add_tiles(std::vector<TileRef>& tiles, int32_t desc, int32_t M, int32_t N, bool lower) {
  const int32_t tm = (M + GEMM_TILE - 1) / GEMM_TILE, tn = (N + GEMM_TILE - 1) / GEMM_TILE;
  for (int32_t a = 0; a < tm; ++a)
    for (int32_t b = 0; b < tn; ++b) {
      if (lower && b > a) continue;
      tiles.push_back(TileRef{desc, a, b, 0});
    }
}

struct GemmBatch {
  std::vector<GemmDesc> d;
  std::vector<TileRef> t;
  DevBuf dd, dt;
  void add(const GemmDesc& g, bool lower) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return;
    d.push_back(g);
    add_tiles(t, int32_t(d.size() - 1), g.M, g.N, lower);
  }
  spand_status run(spand_ctx* h, int prec) {
    if (t.empty()) return SPAND_OK;
    spand_status st = upload(h, dd, d);
    if (st != SPAND_OK) return st;
    st = upload(h, dt, t);
    if (st != SPAND_OK) return st;
    launch_gemm(dd.as<GemmDesc>(), dt.as<TileRef>(), int64_t(t.size()), prec, h->stream);
    HIPCHK(hipGetLastError());
    return SPAND_OK;
  }
};

}  // namespace

spand_status factor_numeric(spand_ctx* h, const double* values, double tol, int32_t skip, spand_prec prec) {
  Analysis& an = h->an;
  const int32_t Lv = an.levels;
  const int gemm_prec = (prec == SPAND_FP64) ? 0 : 1;
  h->num.clear();
  h->num.resize(Lv);
  h->max_tmp = 0;
  h->max_gather = 0;
  spand_status st;

  DevBuf dflag;  // [0] elimination failure id, [1] scaling failure id, [2] non-finite input
  if ((st = dalloc(h, dflag, 4 * sizeof(int32_t))) != SPAND_OK) return st;
  const int32_t flag_init[4] = {0x7fffffff, 0x7fffffff, 0, 0};
  HIPCHK(hipMemcpyAsync(dflag.p, flag_init, sizeof(flag_init), hipMemcpyHostToDevice, h->stream));
  int32_t* d_fail_elim = dflag.as<int32_t>();
  int32_t* d_fail_scale = dflag.as<int32_t>() + 1;
  int32_t* d_nonfinite = dflag.as<int32_t>() + 2;

  // ev[0..1]: Schur GEMMs; ph[0..4]: phase boundaries of a step
  hipEvent_t ev[2], ph[5];
  struct EvGuard {
    hipEvent_t* e;
    int n = 0;
    ~EvGuard() {
      for (int q = 0; q < n; ++q) (void)hipEventDestroy(e[q]);
    }
  } g1{ev}, g2{ph};
  for (int q = 0; q < 2; ++q, ++g1.n) HIPCHK(hipEventCreate(&ev[q]));
  for (int q = 0; q < 5; ++q, ++g2.n) HIPCHK(hipEventCreate(&ph[q]));
  hipEvent_t ev0 = ev[0], ev1 = ev[1];
  std::memset(h->stats.step_phase_seconds, 0, sizeof(h->stats.step_phase_seconds));
  std::memset(h->stats.step_m_F, 0, sizeof(h->stats.step_m_F));

  int64_t m_F = 0;
  double schur_flops = 0.0, schur_ms = 0.0;
  int32_t s_top = 0;

  DevBuf arena_prev;
  Layout lay_prev;
  std::vector<int32_t> rank_prev;

  for (int32_t t = 1; t <= Lv; ++t) {
    const SymStep& sy = an.steps[t - 1];
    StepNum& sn = h->num[t - 1];
    const int32_t nc = sy.nc, ne = sy.ne;
    const bool sparsify = (t > skip) && (sy.level > 1);

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

    // ---- arena layout and assembly
    HIPCHK(hipEventRecord(ph[0], h->stream));
    Layout lay;
    build_layout(sy, sn.size, lay);
    DevBuf arena;
    if ((st = dalloc(h, arena, size_t(lay.total) * sizeof(double))) != SPAND_OK) return st;
    double* A = arena.as<double>();
    if (lay.total) HIPCHK(hipMemsetAsync(A, 0, size_t(lay.total) * sizeof(double), h->stream));
    DevBuf d_dst, d_copy;
    std::vector<CopyDesc> copies;
    if (t == 1) {
      // destination of every CSR entry inside the step-1 panels
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
          const int64_t ro = lay.find(i, j);
          dst[e] = lay.base[j] + ro + pos[v] + int64_t(pos[u]) * lay.H[j];
        }
      if ((st = upload(h, d_dst, dst)) != SPAND_OK) return st;
      launch_scatter_values(values, d_dst.as<int64_t>(), int64_t(dst.size()), A, d_nonfinite, h->stream);
      HIPCHK(hipGetLastError());
    } else {
      const SymStep& ps = an.steps[t - 2];
      const StepNum& pv = h->num[t - 2];
      for (uint64_t pr : sy.before) {
        const int32_t I = pair_i(pr), J = pair_j(pr);
        const int64_t dro = lay.find(I, J);
        double* dbase = A + lay.base[J] + dro;
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
                cd.cols = rj;
                cd.dst = dbase + ro + co * lay.H[J];
                cd.ldd = int32_t(lay.H[J]);
                cd.pad = 0;
                copies.push_back(cd);
              }
            }
            co += rj;
          }
          ro += ri;
        }
      }
      (void)ps;
      if ((st = upload(h, d_copy, copies)) != SPAND_OK) return st;
      launch_copy(d_copy.as<CopyDesc>(), int64_t(copies.size()), h->stream);
      HIPCHK(hipGetLastError());
    }

    // ---- elimination (Sec. 2.4)
    HIPCHK(hipEventRecord(ph[1], h->stream));
    std::vector<int64_t> linv_off(ne), g_off(ne), c_off(ne);
    std::vector<int32_t> nN(ne);
    int64_t elim_total = 0, cbuf_total = 0;
    for (int32_t s = 0; s < ne; ++s) {
      nN[s] = int32_t(lay.H[s] - sn.size[s]);
      linv_off[s] = elim_total;
      elim_total += int64_t(sn.size[s]) * sn.size[s];
      g_off[s] = elim_total;
      elim_total += int64_t(nN[s]) * sn.size[s];
      c_off[s] = cbuf_total;
      cbuf_total += int64_t(nN[s]) * nN[s];
      const double ns = sn.size[s], nn = nN[s];
      schur_flops += nn * ns * ns + nn * (nn + 1.0) * ns;
      m_F += int64_t(sn.size[s]) * (sn.size[s] + 1) / 2 + int64_t(sn.size[s]) * nN[s];
    }
    if ((st = dalloc(h, sn.elim, size_t(elim_total) * sizeof(double))) != SPAND_OK) return st;
    DevBuf cbuf;
    if ((st = dalloc(h, cbuf, size_t(cbuf_total) * sizeof(double))) != SPAND_OK) return st;
    double* E = sn.elim.as<double>();
    {
      std::vector<CholDesc> cds;
      for (int32_t s = 0; s < ne; ++s) {
        if (sn.size[s] == 0) continue;
        cds.push_back(CholDesc{A + lay.base[s], E + linv_off[s], sn.size[s], int32_t(lay.H[s]), s, 0});
      }
      DevBuf dc;
      if ((st = upload(h, dc, cds)) != SPAND_OK) return st;
      launch_chol_inv(dc.as<CholDesc>(), int32_t(cds.size()), d_fail_elim, h->stream);
      HIPCHK(hipGetLastError());
      GemmBatch trsm, syrk;
      for (int32_t s = 0; s < ne; ++s) {
        const int32_t ns = sn.size[s], nn = nN[s];
        GemmDesc g{};
        g.A = A + lay.base[s] + ns;  // A_{N_s s}
        g.lda = int32_t(lay.H[s]);
        g.B = E + linv_off[s];       // op(B)(k, n) = Linv[n][k]
        g.ldb = ns;
        g.C = E + g_off[s];
        g.ldc = nn;
        g.M = nn; g.N = ns; g.K = ns;
        g.flags = G_TB | G_TRIB;
        g.alpha = 1.0; g.beta = 0.0;
        trsm.add(g, false);
        GemmDesc y{};
        y.A = E + g_off[s]; y.lda = nn;
        y.B = E + g_off[s]; y.ldb = nn;
        y.C = cbuf.as<double>() + c_off[s]; y.ldc = nn;
        y.M = nn; y.N = nn; y.K = ns;
        y.flags = G_TB | G_LOWERC;
        y.alpha = 1.0; y.beta = 0.0;
        syrk.add(y, true);
      }
      HIPCHK(hipEventRecord(ev0, h->stream));
      if ((st = trsm.run(h, gemm_prec)) != SPAND_OK) return st;
      if ((st = syrk.run(h, gemm_prec)) != SPAND_OK) return st;
      HIPCHK(hipEventRecord(ev1, h->stream));
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
            if (sn.size[na] > 0 && sn.size[nb] > 0)
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
        rds.push_back(rd);
        q = r;
      }
      DevBuf drd, dcd;
      if ((st = upload(h, drd, rds)) != SPAND_OK) return st;
      if ((st = upload(h, dcd, cds2)) != SPAND_OK) return st;
      launch_reduce(drd.as<ReduceDesc>(), int32_t(rds.size()), dcd.as<ContribDesc>(), h->stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(ph[2], h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
      schur_ms += ms;
    }
    int32_t flags[4];
    HIPCHK(hipMemcpy(flags, dflag.p, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[2]) return set_err(h, SPAND_E_INVALID, "matrix values contain NaN or Inf");
    if (flags[0] != 0x7fffffff) {
      h->stats.fail_step = t;
      h->stats.fail_cluster = flags[0];
      h->stats.fail_phase = 0;
      return set_err(h, SPAND_E_NOT_SPD, "pivot block not SPD at step " + std::to_string(t) + ", cluster " +
                                             std::to_string(flags[0]) + " (elimination)");
    }
    cbuf.release();

    // ---- scaling (Sec. 2.5) and sparsification (Sec. 2.6.1)
    sn.rank.assign(nc, -1);
    for (int32_t c = ne; c < nc; ++c) sn.rank[c] = sn.size[c];
    std::vector<int64_t> sc_off(nc, -1), v_off(nc, -1), tau_off(nc, -1);
    std::vector<int32_t> nref(nc, 0);
    HIPCHK(hipEventRecord(ph[3], h->stream));
    HIPCHK(hipEventRecord(ph[4], h->stream));
    if (sparsify && nc > ne) {
      int64_t sc_total = 0;
      for (int32_t p = ne; p < nc; ++p) {
        if (sn.size[p] == 0) continue;
        sc_off[p] = sc_total;
        sc_total += int64_t(sn.size[p]) * sn.size[p];
        m_F += int64_t(sn.size[p]) * (sn.size[p] + 1) / 2;
      }
      if ((st = dalloc(h, sn.scale, size_t(sc_total) * sizeof(double))) != SPAND_OK) return st;
      double* SC = sn.scale.as<double>();
      std::vector<CholDesc> cds;
      for (int32_t p = ne; p < nc; ++p)
        if (sn.size[p] > 0) cds.push_back(CholDesc{A + lay.base[p], SC + sc_off[p], sn.size[p], int32_t(lay.H[p]), p, 0});
      DevBuf dc;
      if ((st = upload(h, dc, cds)) != SPAND_OK) return st;
      launch_chol_inv(dc.as<CholDesc>(), int32_t(cds.size()), d_fail_scale, h->stream);
      HIPCHK(hipGetLastError());
      // X <- L_i^{-1} X L_j^{-T}: T_j = (panel j below its diagonal) L_j^{-T}, then per block L_i^{-1} T
      std::vector<int64_t> toff(nc, 0);
      int64_t ttot = 0;
      for (int32_t p = ne; p < nc; ++p) {
        toff[p] = ttot;
        ttot += (lay.H[p] - sn.size[p]) * sn.size[p];
      }
      DevBuf tbuf;
      if ((st = dalloc(h, tbuf, size_t(ttot) * sizeof(double))) != SPAND_OK) return st;
      GemmBatch right, left;
      for (int32_t p = ne; p < nc; ++p) {
        const int32_t np_ = sn.size[p];
        const int32_t Mp = int32_t(lay.H[p] - np_);
        if (np_ == 0 || Mp == 0) continue;
        GemmDesc g{};
        g.A = A + lay.base[p] + np_; g.lda = int32_t(lay.H[p]);
        g.B = SC + sc_off[p]; g.ldb = np_;
        g.C = tbuf.as<double>() + toff[p]; g.ldc = Mp;
        g.M = Mp; g.N = np_; g.K = np_;
        g.flags = G_TB | G_TRIB; g.alpha = 1.0; g.beta = 0.0;
        right.add(g, false);
        for (int64_t e = lay.pan_ptr[p] + 1; e < lay.pan_ptr[p + 1]; ++e) {
          const int32_t i = lay.prow[e];
          const int32_t ni = sn.size[i];
          if (ni == 0) continue;
          GemmDesc q{};
          q.A = SC + sc_off[i]; q.lda = ni;
          q.B = tbuf.as<double>() + toff[p] + (lay.proff[e] - np_); q.ldb = Mp;
          q.C = A + lay.base[p] + lay.proff[e]; q.ldc = int32_t(lay.H[p]);
          q.M = ni; q.N = np_; q.K = ni;
          q.flags = G_TRIA; q.alpha = 1.0; q.beta = 0.0;
          left.add(q, false);
        }
      }
      if ((st = right.run(h, 0)) != SPAND_OK) return st;
      if ((st = left.run(h, 0)) != SPAND_OK) return st;
      std::vector<double*> dptr;
      std::vector<int32_t> dn, dld;
      for (int32_t p = ne; p < nc; ++p)
        if (sn.size[p] > 0) {
          dptr.push_back(A + lay.base[p]);
          dn.push_back(sn.size[p]);
          dld.push_back(int32_t(lay.H[p]));
        }
      DevBuf d1, d2, d3;
      if ((st = upload(h, d1, dptr)) != SPAND_OK) return st;
      if ((st = upload(h, d2, dn)) != SPAND_OK) return st;
      if ((st = upload(h, d3, dld)) != SPAND_OK) return st;
      launch_set_identity(d1.as<double*>(), d2.as<int32_t>(), d3.as<int32_t>(), int32_t(dptr.size()), h->stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(ph[3], h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      HIPCHK(hipMemcpy(flags, dflag.p, sizeof(flags), hipMemcpyDeviceToHost));
      if (flags[1] != 0x7fffffff) {
        h->stats.fail_step = t;
        h->stats.fail_cluster = flags[1];
        h->stats.fail_phase = 1;
        return set_err(h, SPAND_E_NOT_SPD, "interface block not SPD at step " + std::to_string(t) + ", cluster " +
                                               std::to_string(flags[1]) + " (scaling)");
      }
      tbuf.release();

      // sparsification, colour by colour; A_pn of each interface is cut into
      // LDS-resident column slabs (one workgroup each)
      std::vector<int64_t> ncols(nc, 0);
      int32_t ncolour = 0;
      int64_t house_total = 0, gn_total = 0, pc_total = 0;
      std::vector<int64_t> gn_off(nc, -1), pc_off(nc, -1);
      std::vector<int32_t> slabS(nc, 0), slabC(nc, 0), nseg(nc, 0);
      int32_t nmulti = 0;
      for (int32_t p = ne; p < nc; ++p) {
        for (int64_t e = sy.nb_ptr[p]; e < sy.nb_ptr[p + 1]; ++e)
          if (sn.size[sy.nb[e]] > 0) {
            ncols[p] += sn.size[sy.nb[e]];
            nseg[p]++;
          }
        if (sn.size[p] == 0 || ncols[p] == 0) continue;
        ncolour = std::max(ncolour, sy.colour[p] + 1);
        const int64_t m = sn.size[p];
        const int64_t budget = int64_t(sparsify_lds_limit()) - 64 - 4 * (nseg[p] + 1) - 8 * m;
        const int64_t cfit = budget / (8 * (m + 1) + 4);
        if (cfit < 1)
          return set_err(h, SPAND_E_INVALID, "interface of " + std::to_string(m) + " dofs exceeds the LDS of one CU");
        if (ncols[p] <= std::min<int64_t>(cfit, 1024)) {
          slabS[p] = 1;
          slabC[p] = int32_t(ncols[p]);
        } else {
          slabC[p] = int32_t(std::min<int64_t>(cfit, 256));
          slabS[p] = int32_t((ncols[p] + slabC[p] - 1) / slabC[p]);
          gn_off[p] = gn_total;
          gn_total += ncols[p];
          pc_off[p] = pc_total;
          pc_total += m;
          ++nmulti;
        }
        const int64_t kmax = std::min<int64_t>(sn.size[p], ncols[p]);
        v_off[p] = house_total;
        house_total += int64_t(sn.size[p]) * kmax;
        tau_off[p] = house_total;
        house_total += kmax;
      }
      if ((st = dalloc(h, sn.house, size_t(house_total) * sizeof(double))) != SPAND_OK) return st;
      DevBuf gnb, pcb, cntb, curb, nrefb, errb;
      if ((st = dalloc(h, gnb, size_t(gn_total) * sizeof(double))) != SPAND_OK) return st;
      if ((st = dalloc(h, pcb, size_t(pc_total) * sizeof(double))) != SPAND_OK) return st;
      if ((st = dalloc(h, cntb, size_t(std::max(nmulti, 1)) * sizeof(int32_t))) != SPAND_OK) return st;
      HIPCHK(hipMemsetAsync(cntb.p, 0, size_t(std::max(nmulti, 1)) * sizeof(int32_t), h->stream));
      if ((st = dalloc(h, errb, sizeof(int32_t))) != SPAND_OK) return st;
      HIPCHK(hipMemsetAsync(errb.p, 0, sizeof(int32_t), h->stream));
      // current sizes: interfaces shrink to their rank as their colour class finishes
      if ((st = upload(h, curb, sn.size)) != SPAND_OK) return st;
      if ((st = upload(h, nrefb, std::vector<int32_t>(nc, 0))) != SPAND_OK) return st;
      std::vector<std::vector<int32_t>> by_colour(ncolour);
      for (int32_t p = ne; p < nc; ++p)
        if (v_off[p] >= 0) by_colour[sy.colour[p]].push_back(p);
      std::vector<DevBuf> keep;
      int32_t multi_idx = 0;
      for (int32_t c = 0; c < ncolour; ++c) {
        if (by_colour[c].empty()) continue;
        for (int pass = 0; pass < 2; ++pass) {  // pass 0: single-slab interfaces; pass 1: multi-slab
          std::vector<int32_t> plist;
          for (int32_t p : by_colour[c])
            if ((slabS[p] > 1) == (pass == 1)) plist.push_back(p);
          size_t pos = 0;
          while (pos < plist.size()) {
            std::vector<SparsDesc> sds;
            std::vector<SegDesc> segs;
            std::vector<SlabRef> slabs;
            size_t lds = 0;
            int cap = 0;
            if (pass == 1) {
              size_t lmax = 0;
              for (int32_t p : plist) lmax = std::max(lmax, sparsify_lds_bytes(sn.size[p], slabC[p], nseg[p]));
              cap = sparsify_max_coresident(lmax);
              lds = lmax;
              if (cap <= 0) return set_err(h, SPAND_E_HIP, "occupancy query for the sparsification kernel failed");
            }
            while (pos < plist.size()) {
              const int32_t p = plist[pos];
              if (pass == 1 && !slabs.empty() && int(slabs.size()) + slabS[p] > cap) break;
              if (pass == 1 && slabS[p] > cap)
                return set_err(h, SPAND_E_INVALID, "interface needs more co-resident workgroups than the GPU holds");
              SparsDesc d{};
              d.V = sn.house.as<double>() + v_off[p];
              d.tau = sn.house.as<double>() + tau_off[p];
              d.diag = A + lay.base[p];
              d.ldd = int32_t(lay.H[p]);
              d.m = sn.size[p];
              d.id = p;
              d.S = slabS[p];
              d.C = slabC[p];
              if (slabS[p] > 1) {
                d.gnrm = gnb.as<double>() + gn_off[p];
                d.pivcol = pcb.as<double>() + pc_off[p];
                d.cnt = cntb.as<int32_t>() + multi_idx++;
              }
              d.seg_begin = int32_t(segs.size());
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
                segs.push_back(g);
              }
              d.seg_end = int32_t(segs.size());
              for (int32_t w = 0; w < slabS[p]; ++w) slabs.push_back(SlabRef{int32_t(sds.size()), w});
              lds = std::max(lds, sparsify_lds_bytes(d.m, d.C, d.seg_end - d.seg_begin));
              sds.push_back(d);
              ++pos;
            }
            DevBuf a, b, sl;
            if ((st = upload(h, a, sds)) != SPAND_OK) return st;
            if ((st = upload(h, b, segs)) != SPAND_OK) return st;
            if ((st = upload(h, sl, slabs)) != SPAND_OK) return st;
            hipError_t le = launch_sparsify(a.as<SparsDesc>(), sl.as<SlabRef>(), int32_t(slabs.size()),
                                            b.as<SegDesc>(), tol, curb.as<int32_t>(), nrefb.as<int32_t>(),
                                            errb.as<int32_t>(), lds, pass == 1, h->stream);
            if (le != hipSuccess)
              return set_err(h, SPAND_E_HIP, std::string("sparsification launch: ") + hipGetErrorString(le));
            keep.push_back(std::move(a));
            keep.push_back(std::move(b));
            keep.push_back(std::move(sl));
          }
        }
      }
      std::vector<int32_t> rk(nc, -1);
      HIPCHK(hipEventRecord(ph[4], h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      HIPCHK(hipMemcpy(rk.data(), curb.p, size_t(nc) * sizeof(int32_t), hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(nref.data(), nrefb.p, size_t(nc) * sizeof(int32_t), hipMemcpyDeviceToHost));
      int32_t serr = 0;
      HIPCHK(hipMemcpy(&serr, errb.p, sizeof(int32_t), hipMemcpyDeviceToHost));
      if (serr) return set_err(h, SPAND_E_HIP, "sparsification slab barrier timed out");
      for (int32_t p = ne; p < nc; ++p)
        if (v_off[p] >= 0) {
          sn.rank[p] = rk[p];
          const int64_t r = nref[p];
          m_F += (2 * int64_t(sn.size[p]) - r + 1) * r / 2 + r;
        }
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    if (t <= 32) {
      float ms[4] = {0.f, 0.f, 0.f, 0.f};
      HIPCHK(hipEventElapsedTime(&ms[0], ph[0], ph[1]));
      HIPCHK(hipEventElapsedTime(&ms[1], ph[1], ph[2]));
      HIPCHK(hipEventElapsedTime(&ms[2], ph[2], ph[3]));
      HIPCHK(hipEventElapsedTime(&ms[3], ph[3], ph[4]));
      for (int q = 0; q < 4; ++q) h->stats.step_phase_seconds[t - 1][q] = 1e-3 * ms[q];
      h->stats.step_m_F[t - 1] = m_F;
    }

    // ---- apply descriptors of this step
    {
      std::vector<int32_t> nslot;
      int64_t tmp = 0;
      sn.h_elim.clear();
      for (int32_t s = 0; s < ne; ++s) {
        ElimAp e{};
        e.Linv = E + linv_off[s];
        e.G = E + g_off[s];
        e.ns = sn.size[s];
        e.nN = nN[s];
        e.slot_s = sn.slot_ptr[s];
        e.slot_N = int64_t(nslot.size());
        for (int64_t q = sy.enb_ptr[s]; q < sy.enb_ptr[s + 1]; ++q) {
          const int32_t nb = sy.enb[q];
          nslot.insert(nslot.end(), sn.slot.begin() + sn.slot_ptr[nb], sn.slot.begin() + sn.slot_ptr[nb + 1]);
        }
        e.tmp = tmp;
        tmp += std::max(e.ns, 1);
        sn.h_elim.push_back(e);
      }
      sn.tmp_elim = tmp;
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
          sn.h_contrib.push_back(TargetContrib{E + g_off[s] + tis[r].row, nN[s], sn.size[s], sn.h_elim[s].tmp});
          ++r;
        }
        ta.cend = int32_t(sn.h_contrib.size());
        sn.h_target.push_back(ta);
        q = r;
      }
      sn.h_scale.clear();
      sn.h_house.clear();
      int64_t tmp2 = 0;
      for (int32_t p = ne; p < nc; ++p) {
        if (sc_off[p] >= 0) {
          ScaleAp a{};
          a.Linv = sn.scale.as<double>() + sc_off[p];
          a.np = sn.size[p];
          a.slot_p = sn.slot_ptr[p];
          a.tmp = tmp2;
          tmp2 += sn.size[p];
          sn.h_scale.push_back(a);
        }
        if (v_off[p] >= 0 && nref[p] > 0) {
          HouseAp hp{};
          hp.V = sn.house.as<double>() + v_off[p];
          hp.tau = sn.house.as<double>() + tau_off[p];
          hp.np = sn.size[p];
          hp.r = nref[p];
          hp.slot_p = sn.slot_ptr[p];
          sn.h_house.push_back(hp);
        }
      }
      sn.tmp_scale = tmp2;
      sn.nslot_len = int64_t(nslot.size());
      h->max_tmp = std::max(h->max_tmp, std::max(sn.tmp_elim, sn.tmp_scale));
      h->max_gather = std::max(h->max_gather, sn.nslot_len);
      sn.n_elim_ap = int32_t(sn.h_elim.size());
      sn.n_target = int32_t(sn.h_target.size());
      sn.n_scale = int32_t(sn.h_scale.size());
      sn.n_house = int32_t(sn.h_house.size());
      if ((st = upload(h, sn.d_slot, sn.slot)) != SPAND_OK) return st;
      if ((st = upload(h, sn.d_nslot, nslot)) != SPAND_OK) return st;
      if ((st = upload(h, sn.d_elim, sn.h_elim)) != SPAND_OK) return st;
      if ((st = upload(h, sn.d_target, sn.h_target)) != SPAND_OK) return st;
      if ((st = upload(h, sn.d_contrib, sn.h_contrib)) != SPAND_OK) return st;
      if ((st = upload(h, sn.d_scale, sn.h_scale)) != SPAND_OK) return st;
      if ((st = upload(h, sn.d_house, sn.h_house)) != SPAND_OK) return st;
      HIPCHK(hipStreamSynchronize(h->stream));
    }

    arena_prev = std::move(arena);
    lay_prev = std::move(lay);
  }
  arena_prev.release();
  h->stats.m_F = m_F;
  h->stats.s_top = s_top;
  h->stats.schur_flops = schur_flops;
  h->stats.schur_seconds = schur_ms * 1e-3;
  return SPAND_OK;
}

}  // namespace spand
