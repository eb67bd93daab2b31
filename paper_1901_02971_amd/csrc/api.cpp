// C ABI of libspand (declared in include/spand.h): argument checking, handle
// lifecycle, timing and error reporting around the analysis, factorization and
// solve drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
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

// Runs fn(q) for q = 0..P-1 on up to 16 host threads.  Every problem of the batch
// works on its own handle and HIP stream: a handle without a stream gets a
// non-blocking one for the call.  The factor and the solve synchronise their
// stream several times per call (rank read-back, convergence checks), so the
// threads keep many problems in flight on the GPU.
template <class F>
spand_status run_batch(int32_t P, spand_t* hs, F&& fn) {
  if (P < 1 || !hs) return fail_null(SPAND_E_INVALID, "batch needs P >= 1 handles");
  for (int32_t q = 0; q < P; ++q) {
    if (!hs[q]) return fail_null(SPAND_E_INVALID, "NULL handle in batch at " + std::to_string(q));
    for (int32_t o = 0; o < q; ++o)
      if (hs[o] == hs[q]) return fail_null(SPAND_E_INVALID, "a handle appears twice in the batch");
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail_null(SPAND_E_HIP, "no HIP device");
  std::vector<hipStream_t> own(P, nullptr);
  for (int32_t q = 0; q < P; ++q)
    if (!hs[q]->stream) {
      if (hipStreamCreateWithFlags(&own[q], hipStreamNonBlocking) != hipSuccess) {
        for (int32_t o = 0; o < q; ++o)
          if (own[o]) {
            (void)hipStreamDestroy(own[o]);
            hs[o]->stream = nullptr;
          }
        return fail_null(SPAND_E_HIP, "stream creation failed");
      }
      hs[q]->stream = own[q];
    }
  std::vector<spand_status> st(P, SPAND_OK);
  std::atomic<int32_t> next{0};
  auto work = [&]() {
    if (hipSetDevice(dev) != hipSuccess) return;
    for (;;) {
      const int32_t q = next.fetch_add(1);
      if (q >= P) break;
      try {
        st[q] = fn(q);
      } catch (...) {
        st[q] = spand::set_err(hs[q], SPAND_E_NOMEM, "host exception during batched call");
      }
    }
  };
  const int32_t nt = std::min<int32_t>(P, 16);
  std::vector<std::thread> pool;
  try {
    for (int32_t k = 1; k < nt; ++k) pool.emplace_back(work);
  } catch (...) {
    // fewer threads: the calling thread and those started share the work
  }
  work();
  for (std::thread& t : pool) t.join();
  if (next.load() < P) {  // no worker could select the device
    for (int32_t q = 0; q < P; ++q)
      if (own[q]) hs[q]->stream = nullptr;
    return fail_null(SPAND_E_HIP, "hipSetDevice failed in the batch workers");
  }
  for (int32_t q = 0; q < P; ++q)
    if (own[q]) {
      (void)hipStreamSynchronize(own[q]);
      (void)hipStreamDestroy(own[q]);
      hs[q]->stream = nullptr;
    }
  for (int32_t q = 0; q < P; ++q)
    if (st[q] != SPAND_OK) {
      g_last_error = "batch problem " + std::to_string(q) + ": " + hs[q]->err;
      return st[q];
    }
  return SPAND_OK;
}

}  // namespace

using spand::set_err;

extern "C" {

spand_status spand_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind, int32_t dim, const double* coords,
                           int32_t levels, spand_t* out) {
  if (!out) return fail_null(SPAND_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1 || n > INT32_MAX - 1) return fail_null(SPAND_E_INVALID, "n must be in [1, 2^31-2]");
  if (!rowptr || !colind || !coords) return fail_null(SPAND_E_INVALID, "NULL input array");
  if (dim != 2 && dim != 3) return fail_null(SPAND_E_INVALID, "dim must be 2 or 3");
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
    h->an.coords.assign(coords, coords + n * dim);
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
  if (!(tol >= 0.0) || !std::isfinite(tol)) return set_err(h, SPAND_E_INVALID, "tol must be finite and >= 0");
  if (skip < 0) return set_err(h, SPAND_E_INVALID, "skip must be >= 0");
  if (prec != SPAND_FP64 && prec != SPAND_FP32 && prec != SPAND_BF16X3)
    return set_err(h, SPAND_E_INVALID, "unknown precision");
  h->factored = false;
  h->stats.fail_step = h->stats.fail_cluster = h->stats.fail_phase = -1;
  const double t0 = now();
  try {
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
      if (hipMemcpyAsync(h->d_rowptr.p, h->an.rowptr.data(), h->d_rowptr.bytes, hipMemcpyHostToDevice,
                         h->stream) != hipSuccess ||
          hipMemcpyAsync(h->d_colind.p, h->an.colind.data(), h->d_colind.bytes, hipMemcpyHostToDevice,
                         h->stream) != hipSuccess ||
          hipStreamSynchronize(h->stream) != hipSuccess)
        return set_err(h, SPAND_E_HIP, "copy of the matrix pattern failed");
    }
    if (hipMemcpyAsync(h->d_values.p, values, h->d_values.bytes, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
      return set_err(h, SPAND_E_HIP, "copy of the matrix values failed");
    spand_status st = spand::factor_numeric(h, h->d_values.as<double>(), tol, skip, prec);
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
  if (t->gemm_variant < 0 || t->gemm_variant >= spand::gemm_variant_count())
    return set_err(h, SPAND_E_INVALID, "unknown gemm_variant");
  h->tune = *t;
  return SPAND_OK;
}

spand_status spand_get_tuning(spand_t h, spand_tuning* t) {
  if (!h || !t) return fail_null(SPAND_E_INVALID, "NULL argument");
  *t = h->tune;
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
  return run_batch(P, hs, [&](int32_t q) { return spand_factor(hs[q], values[q], tol, skip, prec); });
}

spand_status spand_solve_batch(int32_t P, spand_t* hs, int32_t nrhs, const double* const* b, double* const* x,
                               double rtol, int32_t maxit, int32_t* iters, double* relres) {
  if (!b || !x || !iters || !relres) return fail_null(SPAND_E_INVALID, "NULL batch argument");
  return run_batch(P, hs, [&](int32_t q) {
    return spand_solve(hs[q], nrhs, b[q], x[q], rtol, maxit, iters + int64_t(q) * nrhs, relres + int64_t(q) * nrhs);
  });
}

void spand_destroy(spand_t h) { delete h; }

}  // extern "C"
