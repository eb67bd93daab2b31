// Preconditioner apply and FP64 PCG driver (Sec. 2.8 and Sec. 4).
//
// PCG (Hestenes-Stiefel), x0 = 0, independent per right-hand side:
//   r = b, z = M M^T r, p = z, rz = r.z
//   repeat: q = A p; alpha = rz / p.q; x += alpha p; r -= alpha q;
//           if ||r|| <= rtol ||b||: form the true residual b - A x; stop the column
//           if it passes too, else replace r by it (residual replacement);
//           z = M M^T r; beta = r.z / rz; p = z + beta p.
// The target is the true residual (Sec. 4); the recursive one is the cheap test.
// A non-finite residual norm is a breakdown.  Scalars stay on the device; the
// host reads the residual norms once per iteration to retire converged columns.
#include <algorithm>
#include <cmath>
#include <vector>

#include "context.h"

namespace spand {

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) return set_err(h, SPAND_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

StepDev step_dev(const StepNum& s) {
  StepDev d{};
  d.elim = s.d_elim.as<ElimAp>();
  d.target = s.d_target.as<TargetAp>();
  d.contrib = s.d_contrib.as<TargetContrib>();
  d.scale = s.d_scale.as<ScaleAp>();
  d.house = s.d_house.as<HouseAp>();
  d.etile = s.d_etile.as<ElimTile>();
  d.n_etile = s.n_etile;
  d.ftile = s.d_ftile.as<FwdTile>();
  d.n_ftile = s.n_ftile;
  d.stile = s.d_stile.as<ScaleTile>();
  d.n_stile = s.n_stile;
  d.sgather = s.d_sgather.as<int32_t>();
  d.sgather_len = s.sgather_len;
  d.hr = s.d_hr.as<HouseTile>();
  d.hv = s.d_hv.as<HouseTile>();
  d.n_hr = s.n_hr;
  d.n_hv = s.n_hv;
  d.iface = s.d_iface.as<IfaceAp>();
  d.n_iface1 = s.n_iface1;
  d.n_iface2 = s.n_iface2;
  d.interp = s.d_interp.as<InterpAp>();
  d.n_interp = s.n_interp;
  d.slot = s.d_slot.as<int32_t>();
  d.nslot = s.d_nslot.as<int32_t>();
  d.nslot_len = s.nslot_len;
  d.n_elim = s.n_elim_ap;
  d.n_target = s.n_target;
  d.n_scale = s.n_scale;
  d.n_house = s.n_house;
  return d;
}

spand_status ensure_work(spand_ctx* h, size_t bytes) {
  if (h->work.bytes >= bytes) return SPAND_OK;
  h->work.release();
  hipError_t e = hipMalloc(&h->work.p, bytes);
  if (e != hipSuccess) {
    h->work.p = nullptr;
    (void)hipGetLastError();
    return set_err(h, SPAND_E_NOMEM, "device allocation of solve workspace failed");
  }
  h->work.bytes = bytes;
  return SPAND_OK;
}

}  // namespace

// z = M M^T r on stream st; scratch holds apply_scratch_doubles(h, nrhs) doubles.
// Only kernels are launched (no memset or memcpy nodes), so the sequence can be
// captured into a graph.  The sweeps run on a copy of r in the factorization's
// freeze order (h->d_inv), which comes back to the vertex order at the end.
spand_status apply_precond(spand_ctx* h, int32_t nrhs, const double* r, double* z, double* scratch, hipStream_t st) {
  const int64_t n = h->an.n;
  ApplyArgs a{};
  a.nrhs = nrhs;
  a.tmp = scratch;
  a.ldt = std::max<int64_t>(h->max_tmp, 1);
  a.gbuf = scratch + a.ldt * nrhs;
  a.ldg = std::max<int64_t>(h->max_gather, 1);
  a.ldx = n;
  if (h->d_inv.p) {
    a.x = a.gbuf + a.ldg * nrhs;
    launch_permute(r, a.x, h->d_inv.as<int32_t>(), n, nrhs, n, st);
  } else {
    a.x = z;
    if (z != r) launch_copy_vec(r, z, n * nrhs, st);
  }
  for (size_t t = 0; t < h->num.size(); ++t) {
    const StepDev d = step_dev(h->num[t]);
    a.slot = d.slot;
    apply_step_forward(d, a, st);
  }
  for (size_t t = h->num.size(); t-- > 0;) {
    const StepDev d = step_dev(h->num[t]);
    a.slot = d.slot;
    apply_step_backward(d, a, st);
  }
  if (h->d_inv.p) launch_permute(a.x, z, h->d_pos.as<int32_t>(), n, nrhs, n, st);
  HIPCHK(hipGetLastError());
  return SPAND_OK;
}

namespace {

// Capture the apply for (nrhs, r, z, scratch) on a private stream into h->graph_exec.
// Returns false (and leaves no graph) if the runtime refuses the capture.
bool capture_apply(spand_ctx* h, int32_t nrhs, const double* r, double* z, double* scratch) {
  if (h->graph_exec) {
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  hipStream_t cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return false;
  hipGraph_t graph = nullptr;
  bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) == hipSuccess;
  if (ok) {
    const spand_status st = apply_precond(h, nrhs, r, z, scratch, cap);
    ok = (hipStreamEndCapture(cap, &graph) == hipSuccess) && st == SPAND_OK && graph;
  }
  if (ok) ok = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (!ok) h->graph_exec = nullptr;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  (void)hipGetLastError();
  return ok;
}

}  // namespace

size_t apply_scratch_doubles(const spand_ctx* h, int32_t nrhs) {
  const int64_t perm = h->d_inv.p ? h->an.n : 0;
  return size_t(std::max<int64_t>(h->max_tmp, 1) + std::max<int64_t>(h->max_gather, 1) + perm) * size_t(nrhs);
}

spand_status apply_public(spand_ctx* h, int32_t nrhs, const double* r, double* z) {
  spand_status st = ensure_work(h, apply_scratch_doubles(h, nrhs) * sizeof(double));
  if (st != SPAND_OK) return st;
  st = apply_precond(h, nrhs, r, z, h->work.as<double>(), h->stream);
  if (st != SPAND_OK) return st;
  HIPCHK(hipStreamSynchronize(h->stream));
  return SPAND_OK;
}

spand_status pcg_solve(spand_ctx* h, int32_t nrhs, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t* iters, double* relres) {
  const int64_t n = h->an.n;
  const size_t vec = size_t(n) * nrhs;
  const int nblk = int(std::min<int64_t>((n + 255) / 256, 1024));
  // workspace: r, z, p, q, partials, 8 scalar rows, apply scratch
  const size_t scal = size_t(nrhs);
  const size_t doubles = 4 * vec + size_t(nblk) * nrhs + 8 * scal + apply_scratch_doubles(h, nrhs) + 16;
  spand_status st = ensure_work(h, doubles * sizeof(double) + 64 * sizeof(int32_t) + nrhs * sizeof(int32_t));
  if (st != SPAND_OK) return st;
  double* w = h->work.as<double>();
  double* r = w;
  double* z = r + vec;
  double* p = z + vec;
  double* q = p + vec;
  double* partial = q + vec;
  double* bb = partial + size_t(nblk) * nrhs;
  double* rz = bb + scal;
  double* rz_new = rz + scal;
  double* pq = rz_new + scal;
  double* rr = pq + scal;
  double* scratch = rr + 4 * scal;
  int32_t* active_d = reinterpret_cast<int32_t*>(scratch + apply_scratch_doubles(h, nrhs) + 16);
  const hipStream_t s = h->stream;

  std::vector<double> hb(nrhs), hr(nrhs), ht(nrhs);
  std::vector<int32_t> act(nrhs, 0);
  bool broke = false;
  int broke_col = -1;
  int64_t replaced = 0;
  // the apply of this solve: one captured graph (same vectors every iteration),
  // replayed on the handle's stream from the second apply on; the first one is
  // launched kernel by kernel and the graph is captured while the GPU runs it.
  // Device time of every apply from a pair of events around it.
  bool use_graph = false;
  EventPool evpool;
  size_t napply = 0;
  auto timed_apply = [&]() -> spand_status {
    hipEvent_t e0, e1;
    HIPCHK(evpool.get(2 * napply, &e0));
    HIPCHK(evpool.get(2 * napply + 1, &e1));
    HIPCHK(hipEventRecord(e0, s));
    if (use_graph) {
      HIPCHK(hipGraphLaunch(h->graph_exec, s));
    } else {
      spand_status sa = apply_precond(h, nrhs, r, z, scratch, s);
      if (sa != SPAND_OK) return sa;
    }
    HIPCHK(hipEventRecord(e1, s));
    ++napply;
    return SPAND_OK;
  };
  launch_dot(b, b, n, nrhs, partial, nblk, bb, s);
  HIPCHK(hipMemcpyAsync(hb.data(), bb, scal * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int c = 0; c < nrhs; ++c) {
    if (!std::isfinite(hb[c])) return set_err(h, SPAND_E_INVALID, "right-hand side contains NaN or Inf");
    hb[c] = std::sqrt(hb[c]);
    act[c] = hb[c] > 0.0 ? 1 : 0;
    iters[c] = 0;
  }
  HIPCHK(hipMemsetAsync(x, 0, vec * sizeof(double), s));
  HIPCHK(hipMemcpyAsync(r, b, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(active_d, act.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
  bool any = std::any_of(act.begin(), act.end(), [](int a) { return a != 0; });
  if (any) {
    if ((st = timed_apply()) != SPAND_OK) return st;
    HIPCHK(hipMemcpyAsync(p, z, vec * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_dot(r, z, n, nrhs, partial, nblk, rz, s);
  }
  use_graph = any && h->apply_graph && capture_apply(h, nrhs, r, z, scratch);
  int32_t it = 0;
  while (any && it < maxit) {
    launch_spmv(h->d_rowptr.as<int64_t>(), h->d_colind.as<int32_t>(), h->d_values.as<double>(), n, nrhs, p, q, s);
    launch_dot(p, q, n, nrhs, partial, nblk, pq, s);
    launch_update_xr(n, nrhs, rz, pq, active_d, p, q, x, r, s);
    launch_dot(r, r, n, nrhs, partial, nblk, rr, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hr.data(), rr, scal * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ++it;
    bool check_true = false;
    for (int c = 0; c < nrhs; ++c) {
      if (!act[c]) continue;
      iters[c] = it;
      if (!std::isfinite(hr[c])) {
        act[c] = 0;
        broke = true;
        if (broke_col < 0) broke_col = c;
      } else if (std::sqrt(hr[c]) <= rtol * hb[c]) {
        check_true = true;
      }
    }
    if (check_true) {  // true residuals of the columns whose recursive residual passed
      launch_spmv(h->d_rowptr.as<int64_t>(), h->d_colind.as<int32_t>(), h->d_values.as<double>(), n, nrhs, x, q, s);
      launch_residual(int64_t(vec), b, q, s);
      launch_dot(q, q, n, nrhs, partial, nblk, rr, s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(ht.data(), rr, scal * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int c = 0; c < nrhs; ++c) {
        if (!act[c] || !std::isfinite(hr[c]) || std::sqrt(hr[c]) > rtol * hb[c]) continue;
        if (std::sqrt(ht[c]) <= rtol * hb[c]) {
          act[c] = 0;
        } else {  // the recursive residual drifted: continue from the true one
          HIPCHK(hipMemcpyAsync(r + size_t(c) * n, q + size_t(c) * n, size_t(n) * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
          ++replaced;
        }
      }
    }
    any = std::any_of(act.begin(), act.end(), [](int a) { return a != 0; });
    if (!any || it >= maxit) break;
    HIPCHK(hipMemcpyAsync(active_d, act.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if ((st = timed_apply()) != SPAND_OK) return st;
    launch_dot(r, z, n, nrhs, partial, nblk, rz_new, s);
    launch_update_p(n, nrhs, rz_new, rz, active_d, z, p, s);
    HIPCHK(hipMemcpyAsync(rz, rz_new, scal * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipGetLastError());
  }
  // true residual
  launch_spmv(h->d_rowptr.as<int64_t>(), h->d_colind.as<int32_t>(), h->d_values.as<double>(), n, nrhs, x, q, s);
  launch_residual(int64_t(vec), b, q, s);
  launch_dot(q, q, n, nrhs, partial, nblk, rr, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hr.data(), rr, scal * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  bool noconv = false;
  for (int c = 0; c < nrhs; ++c) {
    relres[c] = hb[c] > 0.0 ? std::sqrt(hr[c]) / hb[c] : 0.0;
    if (act[c]) noconv = true;
  }
  double apply_ms = 0.0;
  for (size_t q = 0; q < napply; ++q) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, evpool.ev[2 * q], evpool.ev[2 * q + 1]));
    apply_ms += ms;
  }
  h->stats.apply_seconds = apply_ms * 1e-3;
  h->stats.apply_calls = int64_t(napply);
  h->stats.apply_graph = use_graph ? 1 : 0;
  h->stats.apply_bytes = 16.0 * double(h->stats.m_F) + 4.0 * 8.0 * double(n) * nrhs;
  h->stats.last_iters = 0;
  for (int c = 0; c < nrhs; ++c) h->stats.last_iters = std::max(h->stats.last_iters, iters[c]);
  h->stats.pcg_replacements = replaced;
  if (broke)
    return set_err(h, SPAND_E_BREAKDOWN, "PCG breakdown: non-finite residual in right-hand side " +
                                             std::to_string(broke_col));
  if (noconv) return set_err(h, SPAND_E_NOCONV, "PCG reached maxit = " + std::to_string(maxit));
  return SPAND_OK;
}

}  // namespace spand

namespace spand {

namespace {

// Capture fn(stream) on a private stream into an executable graph; false if the
// runtime refuses.
template <class F>
bool capture(F&& fn, hipGraphExec_t* out) {
  *out = nullptr;
  hipStream_t cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return false;
  hipGraph_t graph = nullptr;
  bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) == hipSuccess;
  if (ok) {
    const bool fok = fn(cap);
    ok = (hipStreamEndCapture(cap, &graph) == hipSuccess) && fok && graph;
  }
  if (ok) ok = hipGraphInstantiate(out, graph, nullptr, nullptr, 0) == hipSuccess;
  if (!ok) *out = nullptr;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  (void)hipGetLastError();
  return ok;
}

struct GraphExec {
  hipGraphExec_t g = nullptr;
  ~GraphExec() {
    if (g) (void)hipGraphExecDestroy(g);
  }
};

// Device memory of one batched solve, from the first handle's pool.
spand_status pool_alloc(spand_ctx* h, DevBuf& b, size_t bytes) {
  b.release();
  if (bytes == 0) return SPAND_OK;
  void* p = nullptr;
  size_t cap = 0;
  if (h->pool.get(bytes, &p, &cap) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(h, SPAND_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes for the batched solve failed");
  }
  b.p = p;
  b.bytes = bytes;
  b.cap = cap;
  b.pool = &h->pool;
  return SPAND_OK;
}

template <typename T>
spand_status pool_upload(spand_ctx* h, DevBuf& b, const std::vector<T>& v) {
  spand_status st = pool_alloc(h, b, v.size() * sizeof(T));
  if (st != SPAND_OK || v.empty()) return st;
  HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
  return SPAND_OK;
}

// The apply of all problems of a batch as one: their vectors stacked (problem q in
// rows off[q] ..), and the descriptors of step t of every problem concatenated, with
// slot and neighbour-slot values shifted by the problem's row offset, offsets into
// the slot arrays, the scratch and the descriptor arrays shifted by the sizes of the
// earlier problems' parts.  Every descriptor still computes what it computes alone.
struct MergedStep {
  StepDev d{};
  DevBuf slot, nslot, elim, target, contrib, scale, house, etile, ftile, stile, sgather, hr, hv, iface;
};

spand_status build_merged(spand_ctx* const* hs, int32_t P, const std::vector<int64_t>& off,
                          std::vector<MergedStep>& out, int64_t& ldt, int64_t& ldg) {
  spand_ctx* h = hs[0];
  int32_t Lmax = 0;
  for (int32_t q = 0; q < P; ++q) Lmax = std::max<int32_t>(Lmax, int32_t(hs[q]->num.size()));
  out.clear();
  out.resize(Lmax);
  ldt = 1;
  ldg = 1;
  spand_status st = SPAND_OK;
  for (int32_t t = 0; t < Lmax; ++t) {
    std::vector<int32_t> slot, nslot, sgather;
    std::vector<ElimAp> elim;
    std::vector<TargetAp> target;
    std::vector<TargetContrib> contrib;
    std::vector<ScaleAp> scale;
    std::vector<HouseAp> house;
    std::vector<ElimTile> etile;
    std::vector<FwdTile> ftile;
    std::vector<ScaleTile> stile;
    std::vector<HouseTile> hr, hv;
    std::vector<IfaceAp> if1, if2;
    int64_t te = 0, ts = 0;  // scratch rows of the elimination and of the scaling phase so far
    for (int32_t q = 0; q < P; ++q) {
      if (t >= int32_t(hs[q]->num.size())) continue;
      const StepNum& sn = hs[q]->num[t];
      const int64_t so = int64_t(slot.size()), no = int64_t(nslot.size());
      const int32_t eo = int32_t(elim.size()), co = int32_t(contrib.size());
      const int32_t sco = int32_t(scale.size()), ho = int32_t(house.size());
      const int32_t v0 = int32_t(off[q]);
      for (int32_t v : sn.slot) slot.push_back(v + v0);
      for (ElimAp e : sn.h_elim) {
        e.slot_s += so;
        e.slot_N += no;
        e.tmp += te;
        e.ytmp += te;
        elim.push_back(e);
      }
      for (TargetAp a : sn.h_target) {
        a.cbeg += co;
        a.cend += co;
        a.slot_n += so;
        target.push_back(a);
      }
      for (TargetContrib c : sn.h_contrib) {
        c.y += te;
        contrib.push_back(c);
      }
      for (ScaleAp a : sn.h_scale) {
        a.slot_p += so;
        a.tmp += ts;
        scale.push_back(a);
      }
      for (HouseAp a : sn.h_house) {
        a.slot_p += so;
        a.tmp += ts;
        house.push_back(a);
      }
      for (ElimTile e : sn.h_etile) {
        e.s += eo;
        etile.push_back(e);
      }
      for (FwdTile f : sn.h_ftile) {
        f.s += eo;
        ftile.push_back(f);
      }
      for (ScaleTile s2 : sn.h_stile) {
        s2.p += sco;
        stile.push_back(s2);
      }
      for (HouseTile s2 : sn.h_hr) {
        s2.p += ho;
        hr.push_back(s2);
      }
      for (HouseTile s2 : sn.h_hv) {
        s2.p += ho;
        hv.push_back(s2);
      }
      for (int32_t k = 0; k < int32_t(sn.h_iface.size()); ++k) {
        IfaceAp a = sn.h_iface[k];
        a.slot_p += so;
        (k < sn.n_iface1 ? if1 : if2).push_back(a);
      }
      // scratch rows of the scaled interfaces (gathered by row): this problem's rows at
      // ts.., padded with row 0 of the stacked vector up to its scaling-phase scratch
      sgather.resize(size_t(ts), v0);
      for (int32_t v : sn.h_sgather) sgather.push_back(v + v0);
      sgather.resize(size_t(ts + sn.tmp_scale), v0);
      te += sn.tmp_elim;
      ts += sn.tmp_scale;
      // the neighbour slots of the step's eliminated clusters (gathered rows of gbuf)
      nslot.insert(nslot.end(), sn.h_nslot.begin(), sn.h_nslot.end());
      for (int64_t k = no; k < int64_t(nslot.size()); ++k) nslot[k] += v0;
    }
    ldt = std::max(ldt, std::max(te, ts));
    ldg = std::max<int64_t>(ldg, int64_t(nslot.size()));
    MergedStep& m = out[t];
    if ((st = pool_upload(h, m.slot, slot)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.nslot, nslot)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.elim, elim)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.target, target)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.contrib, contrib)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.scale, scale)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.house, house)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.etile, etile)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.ftile, ftile)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.stile, stile)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.sgather, sgather)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.hr, hr)) != SPAND_OK) return st;
    if ((st = pool_upload(h, m.hv, hv)) != SPAND_OK) return st;
    std::vector<IfaceAp> ifs(if1);
    ifs.insert(ifs.end(), if2.begin(), if2.end());
    if ((st = pool_upload(h, m.iface, ifs)) != SPAND_OK) return st;
    StepDev& d = m.d;
    d.elim = m.elim.as<ElimAp>();
    d.target = m.target.as<TargetAp>();
    d.contrib = m.contrib.as<TargetContrib>();
    d.scale = m.scale.as<ScaleAp>();
    d.house = m.house.as<HouseAp>();
    d.etile = m.etile.as<ElimTile>();
    d.n_etile = int32_t(etile.size());
    d.ftile = m.ftile.as<FwdTile>();
    d.n_ftile = int32_t(ftile.size());
    d.stile = m.stile.as<ScaleTile>();
    d.n_stile = int32_t(stile.size());
    d.sgather = m.sgather.as<int32_t>();
    d.sgather_len = int64_t(sgather.size());
    d.hr = m.hr.as<HouseTile>();
    d.hv = m.hv.as<HouseTile>();
    d.n_hr = int32_t(hr.size());
    d.n_hv = int32_t(hv.size());
    d.iface = m.iface.as<IfaceAp>();
    d.n_iface1 = int32_t(if1.size());
    d.n_iface2 = int32_t(if2.size());
    d.slot = m.slot.as<int32_t>();
    d.nslot = m.nslot.as<int32_t>();
    d.nslot_len = int64_t(nslot.size());
    d.n_elim = int32_t(elim.size());
    d.n_target = int32_t(target.size());
    d.n_scale = int32_t(scale.size());
    d.n_house = int32_t(house.size());
  }
  return SPAND_OK;
}

}  // namespace

// PCG on P problems as one block-diagonal system on the stream of hs[0] (every
// handle's stream is that one): the vectors of all problems stacked, and every
// vector, SpMV and apply kernel one launch for the batch (scalars per problem and
// column).  Each half of an iteration is one captured graph
// replayed every iteration; one copy per iteration brings every residual norm to the
// host, which retires converged columns through device-side flags.  The arithmetic
// of every problem (dot-product order included) is that of its own solve.
spand_status pcg_solve_batch(spand_ctx* const* hs, int32_t P, int32_t nrhs, const double* const* b,
                             double* const* x, double rtol, int32_t maxit, int32_t* iters, double* relres,
                             spand_status* per) {
  spand_ctx* h = hs[0];
  const hipStream_t s = h->stream;
  const size_t scal = size_t(nrhs);
  const size_t ps = size_t(P) * scal;
  spand_status st = SPAND_OK;
  std::vector<int64_t> off(P + 1, 0), n(P);
  for (int32_t q = 0; q < P; ++q) {
    n[q] = hs[q]->an.n;
    off[q + 1] = off[q] + n[q];
    per[q] = SPAND_OK;
  }
  const int64_t ntot = off[P];
  if (ntot > INT32_MAX) return set_err(h, SPAND_E_INVALID, "the batch has more than 2^31 unknowns in all");
  const size_t vec = size_t(ntot) * scal;
  // segmented dot products: problem q keeps its own block count
  std::vector<SegBlk> blks;
  std::vector<int64_t> pbase(P);
  std::vector<int32_t> nblk(P), pid(ntot);
  // the batched SpMV and the stacking copies: 256-row blocks of every problem
  std::vector<SpmvProb> sprobs(P);
  std::vector<StackProb> bprobs(P), xprobs(P);
  std::vector<int2> rblk;
  for (int32_t q = 0; q < P; ++q) {
    sprobs[q] = SpmvProb{hs[q]->d_rowptr.as<int64_t>(), hs[q]->d_colind.as<int32_t>(), hs[q]->d_values.as<double>(),
                         n[q], off[q]};
    bprobs[q] = StackProb{b[q], nullptr, n[q], off[q]};
    xprobs[q] = StackProb{nullptr, x[q], n[q], off[q]};
    for (int64_t k = 0; k * 256 < n[q]; ++k) rblk.push_back(make_int2(q, int(k)));
  }
  for (int32_t q = 0; q < P; ++q) {
    nblk[q] = int32_t(std::min<int64_t>((n[q] + 255) / 256, 1024));
    pbase[q] = int64_t(blks.size());
    for (int32_t k = 0; k < nblk[q]; ++k) blks.push_back(SegBlk{off[q], n[q], k, nblk[q]});
    std::fill(pid.begin() + off[q], pid.begin() + off[q + 1], q);
  }
  const int64_t nb_tot = int64_t(blks.size());
  std::vector<MergedStep> steps;
  int64_t ldt = 1, ldg = 1;
  if ((st = build_merged(hs, P, off, steps, ldt, ldg)) != SPAND_OK) return st;
  DevBuf vecs, scalars, dblks, dpbase, dnblk, dpid, dact, dsp, dbp, dxp, drb;
  if ((st = pool_upload(h, dsp, sprobs)) != SPAND_OK) return st;
  if ((st = pool_upload(h, dbp, bprobs)) != SPAND_OK) return st;
  if ((st = pool_upload(h, dxp, xprobs)) != SPAND_OK) return st;
  if ((st = pool_upload(h, drb, rblk)) != SPAND_OK) return st;
  const int64_t nrb = int64_t(rblk.size());
  const size_t nvec = 6;  // r, z, p, q, x, b
  if ((st = pool_alloc(h, vecs, (nvec * vec + size_t(ldt + ldg) * scal) * sizeof(double))) != SPAND_OK) return st;
  if ((st = pool_alloc(h, scalars, (size_t(nb_tot) * scal + 7 * ps) * sizeof(double))) != SPAND_OK) return st;
  if ((st = pool_upload(h, dblks, blks)) != SPAND_OK) return st;
  if ((st = pool_upload(h, dpbase, pbase)) != SPAND_OK) return st;
  if ((st = pool_upload(h, dnblk, nblk)) != SPAND_OK) return st;
  if ((st = pool_upload(h, dpid, pid)) != SPAND_OK) return st;
  if ((st = pool_alloc(h, dact, ps * sizeof(int32_t))) != SPAND_OK) return st;
  double* R = vecs.as<double>();
  double* Z = R + vec;
  double* Pv = Z + vec;
  double* Q = Pv + vec;
  double* X = Q + vec;
  double* B = X + vec;
  double* TMP = B + vec;
  double* GB = TMP + size_t(ldt) * scal;
  double* partial = scalars.as<double>();
  double* bb = partial + size_t(nb_tot) * scal;
  double* rz = bb + ps;
  double* rz_new = rz + ps;
  double* pq = rz_new + ps;
  double* rr = pq + ps;
  double* tt = rr + ps;
  int32_t* act_d = dact.as<int32_t>();
  const SegBlk* SB = dblks.as<SegBlk>();
  const int64_t* PB = dpbase.as<int64_t>();
  const int32_t* NB = dnblk.as<int32_t>();
  const int32_t* PID = dpid.as<int32_t>();
  launch_stack(dbp.as<StackProb>(), drb.as<int2>(), nrb, nrhs, ntot, B, true, s);
  auto dot = [&](const double* u, const double* v, double* outp, hipStream_t cs) {
    launch_seg_dot(u, v, ntot, nrhs, SB, nb_tot, PB, NB, P, partial, outp, cs);
  };
  auto spmv_all = [&](const double* xin, double* yout, hipStream_t cs) {
    launch_spmv_batch(dsp.as<SpmvProb>(), drb.as<int2>(), nrb, nrhs, ntot, xin, yout, cs);
  };
  // z = M M^T r for the stacked vector: the merged steps forward, then backward
  auto apply_all = [&](hipStream_t cs) {
    launch_copy_vec(R, Z, int64_t(vec), cs);
    ApplyArgs a{};
    a.x = Z;
    a.ldx = ntot;
    a.nrhs = nrhs;
    a.tmp = TMP;
    a.ldt = ldt;
    a.gbuf = GB;
    a.ldg = ldg;
    for (size_t t = 0; t < steps.size(); ++t) {
      a.slot = steps[t].d.slot;
      apply_step_forward(steps[t].d, a, cs);
    }
    for (size_t t = steps.size(); t-- > 0;) {
      a.slot = steps[t].d.slot;
      apply_step_backward(steps[t].d, a, cs);
    }
  };
  std::vector<double> hr(ps), ht(ps), hb(ps);
  std::vector<int32_t> act(ps, 0);
  std::vector<char> broke(P, 0), live(P, 1);
  std::vector<int64_t> replaced(P, 0);
  dot(B, B, bb, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hb.data(), bb, ps * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int32_t q = 0; q < P; ++q) {
    for (int c = 0; c < nrhs; ++c) {
      const size_t o = size_t(q) * scal + c;
      iters[o] = 0;
      if (!std::isfinite(hb[o]) && live[q]) {
        per[q] = set_err(hs[q], SPAND_E_INVALID, "right-hand side contains NaN or Inf");
        live[q] = 0;
      }
      hb[o] = std::sqrt(hb[o]);
    }
    for (int c = 0; c < nrhs; ++c) {
      const size_t o = size_t(q) * scal + c;
      act[o] = (live[q] && hb[o] > 0.0) ? 1 : 0;
    }
  }
  HIPCHK(hipMemsetAsync(X, 0, vec * sizeof(double), s));
  launch_copy_vec(B, R, int64_t(vec), s);
  HIPCHK(hipMemcpyAsync(act_d, act.data(), ps * sizeof(int32_t), hipMemcpyHostToDevice, s));
  auto half1 = [&](hipStream_t cs) {
    spmv_all(Pv, Q, cs);
    dot(Pv, Q, pq, cs);
    launch_seg_update_xr(ntot, nrhs, PID, rz, pq, act_d, Pv, Q, X, R, cs);
    dot(R, R, rr, cs);
    return hipGetLastError() == hipSuccess;
  };
  auto half2 = [&](hipStream_t cs) {
    apply_all(cs);
    dot(R, Z, rz_new, cs);
    launch_seg_update_p(ntot, nrhs, PID, rz_new, rz, act_d, Z, Pv, cs);
    launch_copy_vec(rz_new, rz, int64_t(ps), cs);
    return hipGetLastError() == hipSuccess;
  };
  GraphExec g1, g2;
  const bool graphs = h->apply_graph && capture(half1, &g1.g) && capture(half2, &g2.g);
  EventPool evpool;
  size_t napply = 0;
  auto run_apply = [&](bool with_rest) -> spand_status {
    hipEvent_t e0, e1;
    HIPCHK(evpool.get(2 * napply, &e0));
    HIPCHK(evpool.get(2 * napply + 1, &e1));
    HIPCHK(hipEventRecord(e0, s));
    if (with_rest) {
      if (graphs) {
        HIPCHK(hipGraphLaunch(g2.g, s));
      } else if (!half2(s)) {
        return set_err(h, SPAND_E_HIP, "batched PCG: launch failed");
      }
    } else {
      apply_all(s);
    }
    HIPCHK(hipEventRecord(e1, s));
    ++napply;
    return SPAND_OK;
  };
  bool any = std::any_of(act.begin(), act.end(), [](int32_t a) { return a != 0; });
  if (any) {  // z = M M^T r, p = z, rz = r.z
    if ((st = run_apply(false)) != SPAND_OK) return st;
    launch_copy_vec(Z, Pv, int64_t(vec), s);
    dot(R, Z, rz, s);
    HIPCHK(hipGetLastError());
  }
  int32_t it = 0;
  while (any && it < maxit) {
    if (graphs) {
      HIPCHK(hipGraphLaunch(g1.g, s));
    } else if (!half1(s)) {
      return set_err(h, SPAND_E_HIP, "batched PCG: launch failed");
    }
    HIPCHK(hipMemcpyAsync(hr.data(), rr, ps * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ++it;
    bool check = false;
    for (int32_t q = 0; q < P; ++q)
      for (int c = 0; c < nrhs; ++c) {
        const size_t o = size_t(q) * scal + c;
        if (!act[o]) continue;
        iters[o] = it;
        if (!std::isfinite(hr[o])) {
          act[o] = 0;
          broke[q] = 1;
        } else if (std::sqrt(hr[o]) <= rtol * hb[o]) {
          check = true;
        }
      }
    if (check) {  // true residuals (every problem: one SpMV launch per problem is cheap here)
      spmv_all(X, Q, s);
      launch_residual(int64_t(vec), B, Q, s);
      dot(Q, Q, tt, s);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(ht.data(), tt, ps * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int32_t q = 0; q < P; ++q)
        for (int c = 0; c < nrhs; ++c) {
          const size_t o = size_t(q) * scal + c;
          if (!act[o] || !std::isfinite(hr[o]) || std::sqrt(hr[o]) > rtol * hb[o]) continue;
          if (std::sqrt(ht[o]) <= rtol * hb[o]) {
            act[o] = 0;
          } else {  // the recursive residual drifted: continue from the true one
            HIPCHK(hipMemcpyAsync(R + off[q] + size_t(c) * ntot, Q + off[q] + size_t(c) * ntot,
                                  size_t(n[q]) * sizeof(double), hipMemcpyDeviceToDevice, s));
            ++replaced[q];
          }
        }
    }
    any = std::any_of(act.begin(), act.end(), [](int32_t a) { return a != 0; });
    if (!any || it >= maxit) break;
    HIPCHK(hipMemcpyAsync(act_d, act.data(), ps * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if ((st = run_apply(true)) != SPAND_OK) return st;
  }
  // true residuals and the solutions back to the callers' arrays
  spmv_all(X, Q, s);
  launch_residual(int64_t(vec), B, Q, s);
  dot(Q, Q, tt, s);
  HIPCHK(hipGetLastError());
  launch_stack(dxp.as<StackProb>(), drb.as<int2>(), nrb, nrhs, ntot, X, false, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(ht.data(), tt, ps * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double apply_ms = 0.0;
  for (size_t q = 0; q < napply; ++q) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, evpool.ev[2 * q], evpool.ev[2 * q + 1]));
    apply_ms += ms;
  }
  for (int32_t q = 0; q < P; ++q) {
    spand_ctx* hq = hs[q];
    bool noconv = false;
    hq->stats.last_iters = 0;
    for (int c = 0; c < nrhs; ++c) {
      const size_t o = size_t(q) * scal + c;
      relres[o] = (live[q] && hb[o] > 0.0) ? std::sqrt(ht[o]) / hb[o] : 0.0;
      if (act[o]) noconv = true;
      hq->stats.last_iters = std::max(hq->stats.last_iters, iters[o]);
    }
    hq->stats.apply_seconds = apply_ms * 1e-3;  // the shared applies (with the second half of each iteration)
    hq->stats.apply_calls = int64_t(napply);
    hq->stats.apply_graph = graphs ? 1 : 0;
    hq->stats.apply_bytes = 16.0 * double(hq->stats.m_F) + 4.0 * 8.0 * double(hq->an.n) * nrhs;
    hq->stats.pcg_replacements = replaced[q];
    if (per[q] != SPAND_OK) continue;
    if (broke[q])
      per[q] = set_err(hq, SPAND_E_BREAKDOWN, "PCG breakdown: non-finite residual");
    else if (noconv)
      per[q] = set_err(hq, SPAND_E_NOCONV, "PCG reached maxit = " + std::to_string(maxit));
  }
  return SPAND_OK;
}

}  // namespace spand
