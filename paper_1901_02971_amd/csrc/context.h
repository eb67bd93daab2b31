// Handle state of libspand: symbolic analysis, device factor storage and the
// per-step descriptors of the preconditioner apply.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "apply.h"
#include "kernels.h"
#include "spand_internal.h"

namespace spand {

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// HIP events for per-launch device timing, owned by one factor or solve call and
// destroyed before it returns, while the stream they were recorded on still exists.
struct EventPool {
  std::vector<hipEvent_t> ev;
  EventPool() = default;
  EventPool(const EventPool&) = delete;
  EventPool& operator=(const EventPool&) = delete;
  ~EventPool() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  hipError_t get(size_t i, hipEvent_t* out) {
    while (ev.size() <= i) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ev.push_back(e);
    }
    *out = ev[i];
    return hipSuccess;
  }
};

struct StepNum {
  std::vector<int32_t> size;    // cluster sizes before elimination
  std::vector<int32_t> rank;    // kept size after sparsification (-1: eliminated)
  std::vector<int64_t> slot_ptr;
  std::vector<int32_t> slot;    // current dofs of every cluster (vertex ids)
  DevBuf elim, scale, house;    // factor pieces: [L_s; G_s] panels, L_p, reflectors
  DevBuf edinv, sdinv;          // inverses of the CHOL_NB-wide diagonal blocks of L_s, L_p
                                // (scale holds L_p^{-1} itself)
  DevBuf d_slot, d_nslot;       // slot arrays on the device
  // apply descriptors
  DevBuf d_elim, d_target, d_contrib, d_scale, d_house, d_etile, d_hr, d_hv, d_stile, d_sgather;
  int32_t n_elim_ap = 0, n_target = 0, n_scale = 0, n_house = 0, n_etile = 0, n_hr = 0, n_hv = 0, n_stile = 0;
  int64_t sgather_len = 0;
  int64_t nslot_len = 0;
  int64_t tmp_elim = 0, tmp_scale = 0;  // doubles per RHS of temp needed
  std::vector<ElimAp> h_elim;
  std::vector<TargetAp> h_target;
  std::vector<TargetContrib> h_contrib;
  std::vector<ScaleAp> h_scale;
  std::vector<HouseAp> h_house;
  std::vector<ElimTile> h_etile;
  std::vector<HouseTile> h_hr, h_hv;
  std::vector<ScaleTile> h_stile;
  std::vector<int32_t> h_sgather;
};

}  // namespace spand

struct spand_ctx {
  spand::Analysis an;
  std::string err;
  hipStream_t stream = nullptr;
  spand_stats stats{};
  bool factored = false;
  int device = -1;
  std::vector<spand::StepNum> num;
  spand::DevBuf d_rowptr, d_colind, d_values;  // CSR of A for the SpMV
  spand::DevBuf d_dst1;                         // step-1 destination of every CSR entry (pattern-only)
  int64_t max_tmp = 0;                          // doubles per RHS for apply scratch
  int64_t max_gather = 0;                       // doubles per RHS for gathered neighbours
  // PCG / apply scratch, grown on demand
  spand::DevBuf work;
  size_t work_bytes = 0;
  // The apply inside PCG, captured once per solve as a HIP graph and replayed on
  // the handle's stream (apply_graph = false launches it kernel by kernel).
  bool apply_graph = true;
  hipGraphExec_t graph_exec = nullptr;
  ~spand_ctx() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  }
};

namespace spand {
spand_status factor_numeric(spand_ctx* h, const double* values, double tol, int32_t skip, spand_prec prec);
spand_status apply_precond(spand_ctx* h, int32_t nrhs, const double* r, double* z, double* tmp, hipStream_t st);
spand_status pcg_solve(spand_ctx* h, int32_t nrhs, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t* iters, double* relres);
spand_status set_err(spand_ctx* h, spand_status st, const std::string& msg);
}  // namespace spand
