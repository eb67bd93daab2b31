// Handle state of libspand: symbolic analysis, device factor storage and the
// per-step descriptors of the preconditioner apply.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "apply.h"
#include "kernels.h"
#include "spand_internal.h"

namespace spand {

// Device blocks of one handle, recycled instead of returned to the driver (whose
// free synchronizes the device).  A released block goes back to the free list; a
// later request takes the smallest free block that holds it if that block is at
// most twice its size, else a new block is allocated.  All work of a handle runs on
// its stream and every call synchronizes that stream before it returns, so a block
// reused inside a call is ordered after its last use on the stream, and one reused
// in a later call is idle.
struct DevPool {
  std::multimap<size_t, void*> free_blocks;  // capacity -> block
  std::vector<void*> owned;
  DevPool() = default;
  DevPool(const DevPool&) = delete;
  DevPool& operator=(const DevPool&) = delete;
  ~DevPool() {
    for (void* p : owned) (void)hipFree(p);
  }
  static size_t round(size_t bytes) {
    const size_t q = bytes >= (size_t(1) << 24) ? (size_t(1) << 21) : 4096;
    return (bytes + q - 1) / q * q;
  }
  hipError_t get(size_t bytes, void** p, size_t* cap) {
    auto it = free_blocks.lower_bound(bytes);
    if (it != free_blocks.end() && it->first <= 2 * bytes + 65536) {
      *p = it->second;
      *cap = it->first;
      free_blocks.erase(it);
      return hipSuccess;
    }
    const size_t c = round(bytes);
    hipError_t e = hipMalloc(p, c);
    if (e != hipSuccess && !free_blocks.empty()) {  // give the cached blocks back and retry
      (void)hipGetLastError();
      (void)hipDeviceSynchronize();
      for (auto& fb : free_blocks) {
        (void)hipFree(fb.second);
        for (auto& o : owned)
          if (o == fb.second) o = nullptr;
      }
      free_blocks.clear();
      std::vector<void*> keep;
      for (void* o : owned)
        if (o) keep.push_back(o);
      owned.swap(keep);
      e = hipMalloc(p, c);
    }
    if (e != hipSuccess) return e;
    owned.push_back(*p);
    *cap = c;
    return hipSuccess;
  }
  void put(void* p, size_t cap) { free_blocks.emplace(cap, p); }
};

// Pinned host staging for the descriptor uploads of one call: bump allocation,
// reset at the start of the next call (the previous call's copies have completed
// by then).  A call that outgrows the current chunk adds one; the next reset
// replaces the chunks by one of their total size.
struct HostStage {
  std::vector<std::pair<char*, size_t>> chunks;
  size_t cur = 0, used = 0;
  HostStage() = default;
  HostStage(const HostStage&) = delete;
  HostStage& operator=(const HostStage&) = delete;
  ~HostStage() {
    for (auto& c : chunks) (void)hipHostFree(c.first);
  }
  void reset() {
    if (chunks.size() > 1) {
      size_t total = 0;
      for (auto& c : chunks) {
        total += c.second;
        (void)hipHostFree(c.first);
      }
      chunks.clear();
      void* p = nullptr;
      if (hipHostMalloc(&p, total, hipHostMallocDefault) == hipSuccess) chunks.emplace_back(static_cast<char*>(p), total);
    }
    cur = 0;
    used = 0;
  }
  char* get(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    while (cur < chunks.size() && used + bytes > chunks[cur].second) {
      ++cur;
      used = 0;
    }
    if (cur == chunks.size()) {
      size_t sz = std::max<size_t>(bytes, size_t(4) << 20);
      if (!chunks.empty()) sz = std::max(sz, 2 * chunks.back().second);
      void* p = nullptr;
      if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) return nullptr;
      chunks.emplace_back(static_cast<char*>(p), sz);
      used = 0;
    }
    char* r = chunks[cur].first + used;
    used += bytes;
    return r;
  }
};

// Owning device allocation (from a handle's DevPool, or from the driver when pool
// is null).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  size_t cap = 0;
  DevPool* pool = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), cap(o.cap), pool(o.pool) {
    o.p = nullptr;
    o.bytes = o.cap = 0;
    o.pool = nullptr;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      cap = o.cap;
      pool = o.pool;
      o.p = nullptr;
      o.bytes = o.cap = 0;
      o.pool = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (pool)
        pool->put(p, cap);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    bytes = cap = 0;
    pool = nullptr;
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
  DevBuf iso;                   // L_s^{-1} of eliminated clusters without neighbours (the top separator)
  DevBuf edinv, sdinv;          // inverses of the CHOL_NB-wide diagonal blocks of L_s, L_p
                                // (scale holds L_p^{-1} itself)
  DevBuf d_slot, d_nslot;       // slot arrays on the device
  // apply descriptors
  DevBuf d_elim, d_target, d_contrib, d_scale, d_house, d_etile, d_ftile, d_hr, d_hv, d_stile, d_sgather, d_iface;
  int32_t n_iface1 = 0, n_iface2 = 0;  // small interfaces with np <= 64, then np <= 128
  int32_t n_elim_ap = 0, n_target = 0, n_scale = 0, n_house = 0, n_etile = 0, n_hr = 0, n_hv = 0, n_stile = 0;
  int32_t n_ftile = 0;
  int32_t n_iso = 0;  // entries of h_scale that are eliminated clusters (their L_s^{-1})
  int64_t sgather_len = 0;
  int64_t nslot_len = 0;
  int64_t tmp_elim = 0, tmp_scale = 0;  // doubles per RHS of temp needed
  std::vector<ElimAp> h_elim;
  std::vector<TargetAp> h_target;
  std::vector<TargetContrib> h_contrib;
  std::vector<ScaleAp> h_scale;
  std::vector<HouseAp> h_house;
  std::vector<ElimTile> h_etile;
  std::vector<FwdTile> h_ftile;
  std::vector<HouseTile> h_hr, h_hv;
  std::vector<ScaleTile> h_stile;
  std::vector<int32_t> h_sgather;
  std::vector<int32_t> h_nslot;  // neighbour slots of the eliminated clusters (vertex ids)
  std::vector<IfaceAp> h_iface;
  // interpolative interfaces (Sec. 2.6.2): their apply descriptors and the buffers
  // holding perm, T_cf and [L_f; G_cf]
  std::vector<InterpAp> h_interp;
  DevBuf d_interp;
  int32_t n_interp = 0;
  std::vector<DevBuf> interp_store;
};

}  // namespace spand

struct spand_ctx {
  spand::Analysis an;
  spand_tuning tune = spand::default_tuning();
  spand_variant variant = SPAND_ORTHS;  // sparsification variant of the next factor
  // Kept ranks of the last completed factorization (per step and cluster) and its
  // tolerance.  A refactorization at the same tolerance takes them as the step
  // counts of its CPQR list schedule; the schedule never changes what is computed.
  std::vector<std::vector<int32_t>> last_rank;
  double last_rank_tol = -1.0;
  std::string err;
  hipStream_t stream = nullptr;
  // second stream of the factorization: the multi-slab CPQR launch of a colour class
  // runs on it beside that class's single-slab launches (created on first use)
  hipStream_t stream2 = nullptr;
  hipStream_t stream3 = nullptr;  // every other single-slab CPQR launch of a colour class
  spand_stats stats{};
  bool factored = false;
  int device = -1;
  // declared before every DevBuf of the handle, so destroyed after them
  spand::DevPool pool;
  spand::HostStage stage;
  std::vector<spand::StepNum> num;
  spand::DevBuf d_rowptr, d_colind, d_values;  // CSR of A for the SpMV
  spand::DevBuf d_dst1;                         // step-1 destination of every CSR entry (pattern-only)
  int64_t max_tmp = 0;                          // doubles per RHS for apply scratch
  int64_t max_gather = 0;                       // doubles per RHS for gathered neighbours
  // The apply works on its vector in the order in which the factorization freezes the
  // dofs (every cluster's slots are then a few contiguous runs); the device slot arrays
  // hold positions in that order.  d_pos[v] = position of vertex v, d_inv its inverse.
  spand::DevBuf d_pos, d_inv;
  // PCG / apply scratch, grown on demand
  spand::DevBuf work;
  size_t work_bytes = 0;
  // The apply inside PCG, captured once per solve as a HIP graph and replayed on
  // the handle's stream (apply_graph = false launches it kernel by kernel).
  bool apply_graph = true;
  hipGraphExec_t graph_exec = nullptr;
  ~spand_ctx() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (stream2) (void)hipStreamDestroy(stream2);
    if (stream3) (void)hipStreamDestroy(stream3);
  }
};

namespace spand {
spand_status factor_numeric(spand_ctx* h, const double* values, double tol, int32_t skip, spand_prec prec);
// Several problems in lockstep with shared launches on the stream of hs[0] (every
// handle's stream must be that one); per[q] receives each problem's status.  The
// return value is SPAND_OK unless the run as a whole failed (then every problem has it).
spand_status factor_numeric_batch(spand_ctx* const* hs, const double* const* values, int32_t np, double tol,
                                  int32_t skip, spand_prec prec, spand_status* per);
spand_status apply_precond(spand_ctx* h, int32_t nrhs, const double* r, double* z, double* tmp, hipStream_t st);
spand_status pcg_solve(spand_ctx* h, int32_t nrhs, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t* iters, double* relres);
spand_status set_err(spand_ctx* h, spand_status st, const std::string& msg);
// PCG on several factored problems in lockstep on the stream of hs[0] (every handle's
// stream must be that one); per[q] receives each problem's status.
spand_status pcg_solve_batch(spand_ctx* const* hs, int32_t P, int32_t nrhs, const double* const* b,
                             double* const* x, double rtol, int32_t maxit, int32_t* iters, double* relres,
                             spand_status* per);
}  // namespace spand
