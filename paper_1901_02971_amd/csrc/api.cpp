// C ABI of libspand (declared in include/spand.h): argument checking, handle
// lifecycle, timing and error reporting around the analysis, factorization and
// solve drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "context.h"

namespace spand {

spand_status set_err(spand_ctx* h, spand_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

spand_status apply_public(spand_ctx* h, int32_t nrhs, const double* r, double* z);

}  // namespace spand

namespace {

using spand::set_err;

thread_local std::string g_last_error;

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

spand_status fail_null(spand_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

std::string check_pattern(int64_t n, const int64_t* rowptr, const int32_t* colind) {
  if (rowptr[0] != 0) return "rowptr[0] must be 0";
  for (int64_t v = 0; v < n; ++v) {
    if (rowptr[v + 1] < rowptr[v]) return "rowptr must be non-decreasing";
    bool diag = false;
    for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      const int32_t u = colind[e];
      if (u < 0 || u >= n) return "column index out of range in row " + std::to_string(v);
      if (e > rowptr[v] && colind[e - 1] >= u) return "column indices must be strictly increasing in row " + std::to_string(v);
      if (u == v) diag = true;
    }
    if (!diag) return "missing diagonal entry in row " + std::to_string(v);
  }
  // symmetry of the pattern: every (v, u) has a matching (u, v)
  for (int64_t v = 0; v < n; ++v)
    for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      const int32_t u = colind[e];
      const int32_t* b = colind + rowptr[u];
      const int32_t* en = colind + rowptr[u + 1];
      const int32_t* it = std::lower_bound(b, en, int32_t(v));
      if (it == en || *it != v) return "pattern is not symmetric at (" + std::to_string(v) + ", " + std::to_string(u) + ")";
    }
  return "";
}

std::string check_factor_args(double tol, int32_t skip, spand_prec prec) {
  if (!(tol >= 0.0) || !std::isfinite(tol)) return "tol must be finite and >= 0";
  if (skip < 0) return "skip must be >= 0";
  if (prec != SPAND_FP64 && prec != SPAND_FP32 && prec != SPAND_BF16X3) return "unknown precision";
  return "";
}

// Device copies of the matrix pattern (on the first factor) and of the values (on
// every factor) of h, on its stream.
spand_status load_values(spand_ctx* h, const double* values) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_err(h, SPAND_E_HIP, "no HIP device");
  h->device = dev;
  const int64_t nnz = h->an.rowptr[h->an.n];
  if (!h->d_rowptr.p) {
    if (hipMalloc(&h->d_rowptr.p, size_t(h->an.n + 1) * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&h->d_colind.p, size_t(nnz) * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&h->d_values.p, size_t(nnz) * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return set_err(h, SPAND_E_NOMEM, "device allocation of the matrix failed");
    }
    h->d_rowptr.bytes = size_t(h->an.n + 1) * sizeof(int64_t);
    h->d_colind.bytes = size_t(nnz) * sizeof(int32_t);
    h->d_values.bytes = size_t(nnz) * sizeof(double);
    if (hipMemcpyAsync(h->d_rowptr.p, h->an.rowptr.data(), h->d_rowptr.bytes, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(h->d_colind.p, h->an.colind.data(), h->d_colind.bytes, hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return set_err(h, SPAND_E_HIP, "copy of the matrix pattern failed");
  }
  if (hipMemcpyAsync(h->d_values.p, values, h->d_values.bytes, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
    return set_err(h, SPAND_E_HIP, "copy of the matrix values failed");
  return SPAND_OK;
}

// The handles of a batched call, distinct and non-NULL, all run on one stream for
// the duration of the call: the first handle's, or a non-blocking stream created for
// the call.  The destructor restores every handle's own stream.
struct BatchStream {
  int32_t P = 0;
  spand_t* hs = nullptr;
  std::vector<hipStream_t> saved;
  hipStream_t own = nullptr, s = nullptr;
  std::string err;
  BatchStream(int32_t P_, spand_t* hs_) : P(P_), hs(hs_) {
    if (P < 1 || !hs) {
      err = "batch needs P >= 1 handles";
      return;
    }
    for (int32_t q = 0; q < P; ++q) {
      if (!hs[q]) {
        err = "NULL handle in batch at " + std::to_string(q);
        return;
      }
    }
    std::vector<spand_t> sorted(hs, hs + P);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) {
      err = "a handle appears twice in the batch";
      return;
    }
    s = hs[0]->stream;
    if (!s) {
      if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) {
        err = "stream creation failed";
        return;
      }
      s = own;
    }
    saved.resize(P);
    for (int32_t q = 0; q < P; ++q) {
      saved[q] = hs[q]->stream;
      hs[q]->stream = s;
    }
  }
  bool ok() const { return err.empty(); }
  ~BatchStream() {
    if (s) (void)hipStreamSynchronize(s);
    for (size_t q = 0; q < saved.size(); ++q) hs[q]->stream = saved[q];
    if (own) (void)hipStreamDestroy(own);
  }
};

}  // namespace

using spand::set_err;

extern "C" {

spand_status spand_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind, int32_t dim, const double* coords,
                           int32_t levels, spand_t* out) {
  if (!out) return fail_null(SPAND_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > INT32_MAX - 1) return fail_null(SPAND_E_INVALID, "n must be in [1, 2^31-2]");
  if (!rowptr || !colind) return fail_null(SPAND_E_INVALID, "NULL input array");
  if (dim == 0 && coords) return fail_null(SPAND_E_INVALID, "dim = 0 (graph separator) takes no coordinates");
  if (dim != 0 && dim != 2 && dim != 3) return fail_null(SPAND_E_INVALID, "dim must be 0, 2 or 3");
  if (dim != 0 && !coords) return fail_null(SPAND_E_INVALID, "coords is NULL");
  if (levels < 1 || levels > 30) return fail_null(SPAND_E_INVALID, "levels must be in [1, 30]");
  const double t0 = now();
  std::string msg = check_pattern(n, rowptr, colind);
  if (!msg.empty()) return fail_null(SPAND_E_INVALID, msg);
  for (int64_t q = 0; q < n * dim; ++q)
    if (!std::isfinite(coords[q])) return fail_null(SPAND_E_INVALID, "coordinates must be finite");
  spand_ctx* h = new (std::nothrow) spand_ctx();
  if (!h) return fail_null(SPAND_E_NOMEM, "host allocation failed");
  try {
    h->an.n = n;
    h->an.levels = levels;
    h->an.dim = dim;
    h->an.rowptr.assign(rowptr, rowptr + n + 1);
    h->an.colind.assign(colind, colind + rowptr[n]);
    if (dim) h->an.coords.assign(coords, coords + n * dim);
    msg = spand::analyze_pattern(h->an);
  } catch (const std::bad_alloc&) {
    delete h;
    return fail_null(SPAND_E_NOMEM, "host allocation failed during analysis");
  }
  if (!msg.empty()) {
    delete h;
    return fail_null(SPAND_E_INVALID, msg);
  }
  h->stats.n = n;
  h->stats.levels = levels;
  h->stats.n_steps = levels;
  h->stats.t_analyze = now() - t0;
  *out = h;
  return SPAND_OK;
}

spand_status spand_factor(spand_t h, const double* values, double tol, int32_t skip, spand_prec prec) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  if (!values) return set_err(h, SPAND_E_INVALID, "values is NULL");
  std::string msg = check_factor_args(tol, skip, prec);
  if (!msg.empty()) return set_err(h, SPAND_E_INVALID, msg);
  h->factored = false;
  h->stats.fail_step = h->stats.fail_cluster = h->stats.fail_phase = -1;
  const double t0 = now();
  try {
    spand_status st = load_values(h, values);
    if (st != SPAND_OK) return st;
    st = spand::factor_numeric(h, h->d_values.as<double>(), tol, skip, prec);
    if (hipStreamSynchronize(h->stream) != hipSuccess && st == SPAND_OK)
      st = set_err(h, SPAND_E_HIP, "stream synchronisation failed after factor");
    if (st != SPAND_OK) {
      h->num.clear();
      return st;
    }
  } catch (const std::bad_alloc&) {
    h->num.clear();
    return set_err(h, SPAND_E_NOMEM, "host allocation failed during factor");
  }
  h->stats.t_factor = now() - t0;
  h->factored = true;
  return SPAND_OK;
}

spand_status spand_solve(spand_t h, int32_t nrhs, const double* b, double* x, double rtol, int32_t maxit,
                         int32_t* iters, double* relres) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  if (!h->factored) return set_err(h, SPAND_E_STATE, "solve called before a successful factor");
  if (nrhs < 1 || !b || !x || !iters || !relres) return set_err(h, SPAND_E_INVALID, "bad solve arguments");
  if (!(rtol >= 0.0) || maxit < 1) return set_err(h, SPAND_E_INVALID, "rtol must be >= 0 and maxit >= 1");
  if (b == x) return set_err(h, SPAND_E_INVALID, "b and x must not alias");
  const double t0 = now();
  spand_status st;
  try {
    st = spand::pcg_solve(h, nrhs, b, x, rtol, maxit, iters, relres);
  } catch (const std::bad_alloc&) {
    return set_err(h, SPAND_E_NOMEM, "host allocation failed during solve");
  }
  h->stats.t_solve = now() - t0;
  return st;
}

spand_status spand_apply(spand_t h, int32_t nrhs, const double* r, double* z) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  if (!h->factored) return set_err(h, SPAND_E_STATE, "apply called before a successful factor");
  if (nrhs < 1 || !r || !z || r == z) return set_err(h, SPAND_E_INVALID, "bad apply arguments");
  return spand::apply_public(h, nrhs, r, z);
}

spand_status spand_set_stream(spand_t h, void* hip_stream) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  h->stream = static_cast<hipStream_t>(hip_stream);
  return SPAND_OK;
}

spand_status spand_set_apply_graph(spand_t h, int32_t enable) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  h->apply_graph = enable != 0;
  return SPAND_OK;
}

spand_status spand_set_tuning(spand_t h, const spand_tuning* t) {
  if (!h || !t) return fail_null(SPAND_E_INVALID, "NULL argument");
  if (t->chol_group < 1 || t->chol_group > 4) return set_err(h, SPAND_E_INVALID, "chol_group must be in [1, 4]");
  if (t->fuse128_min < -1) return set_err(h, SPAND_E_INVALID, "fuse128_min must be >= -1");
  if (t->cpqr_big_min < 0) return set_err(h, SPAND_E_INVALID, "cpqr_big_min must be >= 0");
  for (int32_t v : {t->gemm_syrk, t->gemm_chol, t->gemm_scale})
    if (v < 0 || v >= spand::gemm_variant_count()) return set_err(h, SPAND_E_INVALID, "unknown GEMM variant");
  h->tune = *t;
  return SPAND_OK;
}

spand_status spand_get_tuning(spand_t h, spand_tuning* t) {
  if (!h || !t) return fail_null(SPAND_E_INVALID, "NULL argument");
  *t = h->tune;
  return SPAND_OK;
}

spand_status spand_set_variant(spand_t h, spand_variant v) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  if (v != SPAND_ORTHS && v != SPAND_IN && v != SPAND_INS)
    return set_err(h, SPAND_E_INVALID, "unknown sparsification variant");
  h->variant = v;
  return SPAND_OK;
}

spand_status spand_get_variant(spand_t h, spand_variant* v) {
  if (!h || !v) return fail_null(SPAND_E_INVALID, "NULL argument");
  *v = h->variant;
  return SPAND_OK;
}

spand_status spand_get_stats(spand_t h, spand_stats* s) {
  if (!h || !s) return fail_null(SPAND_E_INVALID, "NULL argument");
  *s = h->stats;
  return SPAND_OK;
}

spand_status spand_get_ordering(spand_t h, int64_t* S, int64_t* L, int64_t* R) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  const size_t n = size_t(h->an.n);
  if (S) std::memcpy(S, h->an.S.data(), n * sizeof(int64_t));
  if (L) std::memcpy(L, h->an.L.data(), n * sizeof(int64_t));
  if (R) std::memcpy(R, h->an.R.data(), n * sizeof(int64_t));
  return SPAND_OK;
}

spand_status spand_get_permutation(spand_t h, int64_t* perm) {
  if (!h || !perm) return fail_null(SPAND_E_INVALID, "NULL argument");
  // vertex v is eliminated at the step of its separator, t = L - level(S) + 1, inside
  // the cluster its step-1 cluster has merged into by then
  const spand::Analysis& an = h->an;
  const int64_t n = an.n;
  std::vector<int32_t> cl(n), ptr(n);
  const spand::SymStep& s1 = an.steps[0];
  for (int32_t c = 0; c < s1.nc; ++c)
    for (int64_t e = s1.child_ptr[c]; e < s1.child_ptr[c + 1]; ++e) cl[s1.child[e]] = c;
  struct Key { int32_t t, c; int64_t v; };
  std::vector<Key> keys(n);
  std::vector<std::vector<int32_t>> up(an.levels);  // cluster of step t holding each step-1 cluster
  up[0].resize(s1.nc);
  for (int32_t c = 0; c < s1.nc; ++c) up[0][c] = c;
  for (int32_t t = 1; t < an.levels; ++t) {
    up[t].resize(s1.nc);
    const spand::SymStep& pv = an.steps[t - 1];
    for (int32_t c = 0; c < s1.nc; ++c) up[t][c] = up[t - 1][c] >= 0 ? pv.parent[up[t - 1][c]] : -1;
  }
  for (int64_t v = 0; v < n; ++v) {
    const int32_t t = an.levels - int32_t(spand::sep_level(an.S[v]));  // 0-based step
    keys[v] = Key{t, up[t][cl[v]], v};
  }
  std::sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
    if (a.t != b.t) return a.t < b.t;
    if (a.c != b.c) return a.c < b.c;
    return a.v < b.v;
  });
  for (int64_t q = 0; q < n; ++q) perm[q] = keys[q].v;
  return SPAND_OK;
}

spand_status spand_step_counts(spand_t h, int32_t step, int64_t* counts) {
  if (!h || !counts) return fail_null(SPAND_E_INVALID, "NULL argument");
  if (step < 1 || step > h->an.levels) return set_err(h, SPAND_E_INVALID, "step out of range");
  const spand::SymStep& st = h->an.steps[step - 1];
  counts[0] = st.nc;
  counts[1] = st.ne;
  counts[2] = int64_t(st.before.size());
  counts[3] = int64_t(st.after.size());
  counts[4] = st.level;
  counts[5] = int64_t(st.enb.size());
  return SPAND_OK;
}

spand_status spand_step_structure(spand_t h, int32_t step, int64_t* keys, int32_t* parent, int32_t* colour,
                                  int32_t* before, int32_t* after) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  if (step < 1 || step > h->an.levels) return set_err(h, SPAND_E_INVALID, "step out of range");
  const spand::SymStep& st = h->an.steps[step - 1];
  if (keys) std::memcpy(keys, st.key.data(), st.key.size() * sizeof(int64_t));
  if (parent) std::memcpy(parent, st.parent.data(), st.parent.size() * sizeof(int32_t));
  if (colour) std::memcpy(colour, st.colour.data(), st.colour.size() * sizeof(int32_t));
  if (before)
    for (size_t q = 0; q < st.before.size(); ++q) {
      before[2 * q] = spand::pair_i(st.before[q]);
      before[2 * q + 1] = spand::pair_j(st.before[q]);
    }
  if (after)
    for (size_t q = 0; q < st.after.size(); ++q) {
      after[2 * q] = spand::pair_i(st.after[q]);
      after[2 * q + 1] = spand::pair_j(st.after[q]);
    }
  return SPAND_OK;
}

spand_status spand_step_ranks(spand_t h, int32_t step, int32_t* sizes, int32_t* ranks) {
  if (!h) return fail_null(SPAND_E_INVALID, "handle is NULL");
  if (!h->factored) return set_err(h, SPAND_E_STATE, "no factorization");
  if (step < 1 || step > h->an.levels) return set_err(h, SPAND_E_INVALID, "step out of range");
  const spand::StepNum& sn = h->num[step - 1];
  if (sizes) std::memcpy(sizes, sn.size.data(), sn.size.size() * sizeof(int32_t));
  if (ranks) std::memcpy(ranks, sn.rank.data(), sn.rank.size() * sizeof(int32_t));
  return SPAND_OK;
}

const char* spand_error_string(spand_t h) {
  if (!h) return g_last_error.c_str();
  return h->err.c_str();
}

spand_status spand_factor_batch(int32_t P, spand_t* hs, const double* const* values, double tol, int32_t skip,
                                spand_prec prec) {
  if (!values) return fail_null(SPAND_E_INVALID, "values is NULL");
  BatchStream bs(P, hs);
  if (!bs.ok()) return fail_null(SPAND_E_INVALID, bs.err);
  const std::string msg = check_factor_args(tol, skip, prec);
  if (!msg.empty()) return fail_null(SPAND_E_INVALID, msg);
  for (int32_t q = 0; q < P; ++q) {
    if (!values[q]) return fail_null(SPAND_E_INVALID, "values[" + std::to_string(q) + "] is NULL");
    if (hs[q]->variant != SPAND_ORTHS)
      return fail_null(SPAND_E_INVALID, "the batched factor supports the OrthS variant only (handle " +
                                            std::to_string(q) + ")");
  }
  const double t0 = now();
  std::vector<spand_status> per(P, SPAND_OK);
  std::vector<const double*> dv(P);
  spand_status st = SPAND_OK;
  try {
    for (int32_t q = 0; q < P && st == SPAND_OK; ++q) {
      hs[q]->factored = false;
      hs[q]->stats.fail_step = hs[q]->stats.fail_cluster = hs[q]->stats.fail_phase = -1;
      st = load_values(hs[q], values[q]);
      if (st != SPAND_OK) per[q] = st;
      dv[q] = hs[q]->d_values.as<double>();
    }
    if (st == SPAND_OK) st = spand::factor_numeric_batch(hs, dv.data(), P, tol, skip, prec, per.data());
    if (hipStreamSynchronize(bs.s) != hipSuccess && st == SPAND_OK) {
      st = set_err(hs[0], SPAND_E_HIP, "stream synchronisation failed after the batched factor");
      for (int32_t q = 0; q < P; ++q) per[q] = st;
    }
  } catch (const std::bad_alloc&) {
    st = set_err(hs[0], SPAND_E_NOMEM, "host allocation failed during the batched factor");
    for (int32_t q = 0; q < P; ++q) per[q] = st;
  }
  const double t1 = now();
  for (int32_t q = 0; q < P; ++q) {
    if (per[q] == SPAND_OK) {
      hs[q]->factored = true;
      hs[q]->stats.t_factor = t1 - t0;
    } else {
      hs[q]->num.clear();
    }
  }
  for (int32_t q = 0; q < P; ++q)
    if (per[q] != SPAND_OK) {
      g_last_error = "batch problem " + std::to_string(q) + ": " + hs[q]->err;
      return per[q];
    }
  return SPAND_OK;
}

spand_status spand_solve_batch(int32_t P, spand_t* hs, int32_t nrhs, const double* const* b, double* const* x,
                               double rtol, int32_t maxit, int32_t* iters, double* relres) {
  if (!b || !x || !iters || !relres) return fail_null(SPAND_E_INVALID, "NULL batch argument");
  BatchStream bs(P, hs);
  if (!bs.ok()) return fail_null(SPAND_E_INVALID, bs.err);
  if (nrhs < 1) return fail_null(SPAND_E_INVALID, "nrhs must be >= 1");
  if (!(rtol >= 0.0) || maxit < 1) return fail_null(SPAND_E_INVALID, "rtol must be >= 0 and maxit >= 1");
  for (int32_t q = 0; q < P; ++q) {
    if (!hs[q]->factored) {
      set_err(hs[q], SPAND_E_STATE, "solve called before a successful factor");
      g_last_error = "batch problem " + std::to_string(q) + ": " + hs[q]->err;
      return SPAND_E_STATE;
    }
    if (!b[q] || !x[q] || b[q] == x[q]) return fail_null(SPAND_E_INVALID, "bad b/x of batch problem " + std::to_string(q));
    for (const spand::StepNum& sn : hs[q]->num)
      if (sn.n_interp > 0)
        return fail_null(SPAND_E_INVALID, "the batched solve supports OrthS factorizations only (problem " +
                                              std::to_string(q) + ")");
  }
  const double t0 = now();
  std::vector<spand_status> per(P, SPAND_OK);
  spand_status st;
  try {
    st = spand::pcg_solve_batch(hs, P, nrhs, b, x, rtol, maxit, iters, relres, per.data());
  } catch (const std::bad_alloc&) {
    st = set_err(hs[0], SPAND_E_NOMEM, "host allocation failed during the batched solve");
  }
  const double t1 = now();
  if (st != SPAND_OK) {
    g_last_error = "batched solve: " + hs[0]->err;
    return st;
  }
  for (int32_t q = 0; q < P; ++q) hs[q]->stats.t_solve = t1 - t0;
  for (int32_t q = 0; q < P; ++q)
    if (per[q] != SPAND_OK) {
      g_last_error = "batch problem " + std::to_string(q) + ": " + hs[q]->err;
      return per[q];
    }
  return SPAND_OK;
}

void spand_destroy(spand_t h) { delete h; }

}  // extern "C"
