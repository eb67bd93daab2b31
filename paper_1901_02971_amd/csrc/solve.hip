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

// z = M M^T r on stream st; scratch holds (max_tmp + max_gather) * nrhs doubles.
// Only kernels are launched (no memset or memcpy nodes), so the sequence can be
// captured into a graph.
spand_status apply_precond(spand_ctx* h, int32_t nrhs, const double* r, double* z, double* scratch, hipStream_t st) {
  const int64_t n = h->an.n;
  if (z != r) launch_copy_vec(r, z, n * nrhs, st);
  ApplyArgs a{};
  a.x = z;
  a.ldx = n;
  a.nrhs = nrhs;
  a.tmp = scratch;
  a.ldt = std::max<int64_t>(h->max_tmp, 1);
  a.gbuf = scratch + a.ldt * nrhs;
  a.ldg = std::max<int64_t>(h->max_gather, 1);
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
  return size_t(std::max<int64_t>(h->max_tmp, 1) + std::max<int64_t>(h->max_gather, 1)) * size_t(nrhs);
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
  // replayed on the handle's stream; device time of every apply from a pair of
  // events around it
  const bool use_graph = h->apply_graph && capture_apply(h, nrhs, r, z, scratch);
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

// Vectors and scalars of one problem of a batched solve, inside its handle's
// workspace; the residual norms, true-residual norms, |b| and the active flags of
// every problem live in shared arrays so that one copy moves them all.
struct PcgVecs {
  spand_ctx* h = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  int64_t n = 0;
  size_t vec = 0;
  int nblk = 0;
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *partial = nullptr;
  double *rz = nullptr, *rz_new = nullptr, *pq = nullptr, *scratch = nullptr;
  double *rr = nullptr, *tt = nullptr, *bb = nullptr;  // in the shared arrays
  int32_t* act = nullptr;                              // in the shared array
  bool live = true;
};

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

}  // namespace

// PCG on P problems in lockstep on the stream of hs[0] (every handle's stream is
// that one): each half of an iteration, for every problem, is one captured graph
// (the first: SpMV, p.q, x and r updates, r.r; the second: the preconditioner apply,
// r.z, p update), replayed each iteration; the host reads every residual norm with
// one copy per iteration and retires converged columns through device-side flags.
spand_status pcg_solve_batch(spand_ctx* const* hs, int32_t P, int32_t nrhs, const double* const* b,
                             double* const* x, double rtol, int32_t maxit, int32_t* iters, double* relres,
                             spand_status* per) {
  spand_ctx* h = hs[0];
  const hipStream_t s = h->stream;
  const size_t scal = size_t(nrhs);
  spand_status st = SPAND_OK;
  // shared arrays: rr, tt, bb (doubles) and act (ints), P * nrhs each
  DevBuf shared;
  {
    void* p = nullptr;
    size_t cap = 0;
    const size_t bytes = 3 * size_t(P) * scal * sizeof(double) + size_t(P) * scal * sizeof(int32_t);
    if (h->pool.get(bytes, &p, &cap) != hipSuccess) {
      (void)hipGetLastError();
      return set_err(h, SPAND_E_NOMEM, "device allocation of the batched solve's shared scalars failed");
    }
    shared.p = p;
    shared.bytes = bytes;
    shared.cap = cap;
    shared.pool = &h->pool;
  }
  double* rr_all = shared.as<double>();
  double* tt_all = rr_all + size_t(P) * scal;
  double* bb_all = tt_all + size_t(P) * scal;
  int32_t* act_all = reinterpret_cast<int32_t*>(bb_all + size_t(P) * scal);
  std::vector<PcgVecs> V(P);
  for (int32_t k = 0; k < P; ++k) {
    PcgVecs& v = V[k];
    spand_ctx* hq = hs[k];
    v.h = hq;
    v.b = b[k];
    v.x = x[k];
    v.n = hq->an.n;
    v.vec = size_t(v.n) * scal;
    v.nblk = int(std::min<int64_t>((v.n + 255) / 256, 1024));
    const size_t doubles = 4 * v.vec + size_t(v.nblk) * scal + 4 * scal + apply_scratch_doubles(hq, nrhs) + 16;
    if ((st = ensure_work(hq, doubles * sizeof(double))) != SPAND_OK) {
      per[k] = st;
      return st;
    }
    double* w = hq->work.as<double>();
    v.r = w;
    v.z = v.r + v.vec;
    v.p = v.z + v.vec;
    v.q = v.p + v.vec;
    v.partial = v.q + v.vec;
    v.rz = v.partial + size_t(v.nblk) * scal;
    v.rz_new = v.rz + scal;
    v.pq = v.rz_new + scal;
    v.scratch = v.pq + 2 * scal;
    v.rr = rr_all + size_t(k) * scal;
    v.tt = tt_all + size_t(k) * scal;
    v.bb = bb_all + size_t(k) * scal;
    v.act = act_all + size_t(k) * scal;
  }
  std::vector<double> hr(size_t(P) * scal), ht(size_t(P) * scal), hb(size_t(P) * scal);
  std::vector<int32_t> act(size_t(P) * scal, 0);
  std::vector<char> broke(P, 0);
  std::vector<int64_t> replaced(P, 0);
  for (int32_t k = 0; k < P; ++k) {
    const PcgVecs& v = V[k];
    launch_dot(v.b, v.b, v.n, nrhs, v.partial, v.nblk, v.bb, s);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hb.data(), bb_all, hb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int32_t k = 0; k < P; ++k) {
    per[k] = SPAND_OK;
    for (int c = 0; c < nrhs; ++c) {
      const size_t o = size_t(k) * scal + c;
      iters[o] = 0;
      if (!std::isfinite(hb[o])) {
        per[k] = set_err(hs[k], SPAND_E_INVALID, "right-hand side contains NaN or Inf");
        V[k].live = false;
      }
      hb[o] = std::sqrt(hb[o]);
    }
    for (int c = 0; c < nrhs; ++c) {
      const size_t o = size_t(k) * scal + c;
      act[o] = (V[k].live && hb[o] > 0.0) ? 1 : 0;
    }
  }
  for (int32_t k = 0; k < P; ++k) {
    const PcgVecs& v = V[k];
    HIPCHK(hipMemsetAsync(v.x, 0, v.vec * sizeof(double), s));
    launch_copy_vec(v.b, v.r, int64_t(v.vec), s);
  }
  HIPCHK(hipMemcpyAsync(act_all, act.data(), act.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(hipGetLastError());
  // the two halves of an iteration, for every live problem
  auto half1 = [&](hipStream_t cs) {
    for (const PcgVecs& v : V) {
      if (!v.live) continue;
      launch_spmv(v.h->d_rowptr.as<int64_t>(), v.h->d_colind.as<int32_t>(), v.h->d_values.as<double>(), v.n, nrhs,
                  v.p, v.q, cs);
      launch_dot(v.p, v.q, v.n, nrhs, v.partial, v.nblk, v.pq, cs);
      launch_update_xr(v.n, nrhs, v.rz, v.pq, v.act, v.p, v.q, v.x, v.r, cs);
      launch_dot(v.r, v.r, v.n, nrhs, v.partial, v.nblk, v.rr, cs);
    }
    return hipGetLastError() == hipSuccess;
  };
  auto applies = [&](hipStream_t cs) {
    for (const PcgVecs& v : V)
      if (v.live && apply_precond(v.h, nrhs, v.r, v.z, v.scratch, cs) != SPAND_OK) return false;
    return true;
  };
  auto half2 = [&](hipStream_t cs) {
    if (!applies(cs)) return false;
    for (const PcgVecs& v : V) {
      if (!v.live) continue;
      launch_dot(v.r, v.z, v.n, nrhs, v.partial, v.nblk, v.rz_new, cs);
      launch_update_p(v.n, nrhs, v.rz_new, v.rz, v.act, v.z, v.p, cs);
      launch_copy_vec(v.rz_new, v.rz, int64_t(nrhs), cs);
    }
    return hipGetLastError() == hipSuccess;
  };
  GraphExec g1, g2;
  const bool graphs = h->apply_graph && capture(half1, &g1.g) && capture(half2, &g2.g);
  EventPool evpool;
  size_t nhalf2 = 0;
  auto run_half2 = [&]() -> spand_status {
    hipEvent_t e0, e1;
    HIPCHK(evpool.get(2 * nhalf2, &e0));
    HIPCHK(evpool.get(2 * nhalf2 + 1, &e1));
    HIPCHK(hipEventRecord(e0, s));
    if (graphs) {
      HIPCHK(hipGraphLaunch(g2.g, s));
    } else if (!half2(s)) {
      return set_err(h, SPAND_E_HIP, "batched PCG: apply launch failed");
    }
    HIPCHK(hipEventRecord(e1, s));
    ++nhalf2;
    return SPAND_OK;
  };
  bool any = std::any_of(act.begin(), act.end(), [](int32_t a) { return a != 0; });
  if (any) {
    // z = M M^T r, p = z, rz = r.z
    hipEvent_t e0, e1;
    HIPCHK(evpool.get(2 * nhalf2, &e0));
    HIPCHK(evpool.get(2 * nhalf2 + 1, &e1));
    HIPCHK(hipEventRecord(e0, s));
    if (!applies(s)) return set_err(h, SPAND_E_HIP, "batched PCG: apply launch failed");
    HIPCHK(hipEventRecord(e1, s));
    ++nhalf2;
    for (const PcgVecs& v : V) {
      if (!v.live) continue;
      launch_copy_vec(v.z, v.p, int64_t(v.vec), s);
      launch_dot(v.r, v.z, v.n, nrhs, v.partial, v.nblk, v.rz, s);
    }
    HIPCHK(hipGetLastError());
  }
  int32_t it = 0;
  while (any && it < maxit) {
    if (graphs) {
      HIPCHK(hipGraphLaunch(g1.g, s));
    } else if (!half1(s)) {
      return set_err(h, SPAND_E_HIP, "batched PCG: launch failed");
    }
    HIPCHK(hipMemcpyAsync(hr.data(), rr_all, hr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    ++it;
    std::vector<int32_t> check;
    for (int32_t k = 0; k < P; ++k) {
      bool need = false;
      for (int c = 0; c < nrhs; ++c) {
        const size_t o = size_t(k) * scal + c;
        if (!act[o]) continue;
        iters[o] = it;
        if (!std::isfinite(hr[o])) {
          act[o] = 0;
          broke[k] = 1;
        } else if (std::sqrt(hr[o]) <= rtol * hb[o]) {
          need = true;
        }
      }
      if (need) check.push_back(k);
    }
    if (!check.empty()) {  // true residuals of the problems with a column whose recursive residual passed
      for (int32_t k : check) {
        const PcgVecs& v = V[k];
        launch_spmv(v.h->d_rowptr.as<int64_t>(), v.h->d_colind.as<int32_t>(), v.h->d_values.as<double>(), v.n, nrhs,
                    v.x, v.q, s);
        launch_residual(int64_t(v.vec), v.b, v.q, s);
        launch_dot(v.q, v.q, v.n, nrhs, v.partial, v.nblk, v.tt, s);
      }
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(ht.data(), tt_all, ht.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (int32_t k : check) {
        const PcgVecs& v = V[k];
        for (int c = 0; c < nrhs; ++c) {
          const size_t o = size_t(k) * scal + c;
          if (!act[o] || !std::isfinite(hr[o]) || std::sqrt(hr[o]) > rtol * hb[o]) continue;
          if (std::sqrt(ht[o]) <= rtol * hb[o]) {
            act[o] = 0;
          } else {  // the recursive residual drifted: continue from the true one
            HIPCHK(hipMemcpyAsync(v.r + size_t(c) * v.n, v.q + size_t(c) * v.n, size_t(v.n) * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
            ++replaced[k];
          }
        }
      }
    }
    any = std::any_of(act.begin(), act.end(), [](int32_t a) { return a != 0; });
    if (!any || it >= maxit) break;
    HIPCHK(hipMemcpyAsync(act_all, act.data(), act.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if ((st = run_half2()) != SPAND_OK) return st;
  }
  // true residuals
  for (const PcgVecs& v : V) {
    if (!v.live) continue;
    launch_spmv(v.h->d_rowptr.as<int64_t>(), v.h->d_colind.as<int32_t>(), v.h->d_values.as<double>(), v.n, nrhs,
                v.x, v.q, s);
    launch_residual(int64_t(v.vec), v.b, v.q, s);
    launch_dot(v.q, v.q, v.n, nrhs, v.partial, v.nblk, v.tt, s);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(ht.data(), tt_all, ht.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double apply_ms = 0.0;
  for (size_t q = 0; q < nhalf2; ++q) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, evpool.ev[2 * q], evpool.ev[2 * q + 1]));
    apply_ms += ms;
  }
  for (int32_t k = 0; k < P; ++k) {
    spand_ctx* hq = hs[k];
    bool noconv = false;
    hq->stats.last_iters = 0;
    for (int c = 0; c < nrhs; ++c) {
      const size_t o = size_t(k) * scal + c;
      relres[o] = (V[k].live && hb[o] > 0.0) ? std::sqrt(ht[o]) / hb[o] : 0.0;
      if (act[o]) noconv = true;
      hq->stats.last_iters = std::max(hq->stats.last_iters, iters[o]);
    }
    hq->stats.apply_seconds = apply_ms * 1e-3;  // the shared second halves (applies of every problem)
    hq->stats.apply_calls = int64_t(nhalf2);
    hq->stats.apply_graph = graphs ? 1 : 0;
    hq->stats.apply_bytes = 16.0 * double(hq->stats.m_F) + 4.0 * 8.0 * double(hq->an.n) * nrhs;
    hq->stats.pcg_replacements = replaced[k];
    if (per[k] != SPAND_OK) continue;
    if (broke[k])
      per[k] = set_err(hq, SPAND_E_BREAKDOWN, "PCG breakdown: non-finite residual");
    else if (noconv)
      per[k] = set_err(hq, SPAND_E_NOCONV, "PCG reached maxit = " + std::to_string(maxit));
  }
  return SPAND_OK;
}

}  // namespace spand
