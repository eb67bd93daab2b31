// Truncated column-pivoted QR of the interfaces (Sec. 2.6.1; ratio rule of Sec. 4
// intro) with the block A_pn held in registers.
//
// Interface p couples its m dofs to nc neighbour dofs through A_pn (m x nc).  A
// workgroup of NT = 512 threads (two waves per SIMD, so the whole register file of
// a CU) holds a slab of CAP = K * NT / G columns: a team of G consecutive lanes (G a
// power of two, G * CQ_MR >= m) owns K column slots, and lane g of the team keeps
// rows i = q * G + g (q < CQ_MR) of each of them: CQ_CPL slots in registers, and,
// where the LDS holds it and the host asks for it, one more slot in LDS (K =
// CQ_CPL + 1).  Column c of A_pn lives in slab c / CAP, team (c % CAP) % (NT / G),
// slot (c % CAP) / (NT / G).  Interface p uses S = ceil(nc / CAP) slabs.
//
// Step j of Householder QR with column pivoting:
//   1. every column knows the exact norm of its rows j..m-1 (recomputed from the
//      updated entries at the end of the previous step, never downdated);
//   2. pivot = among the remaining columns whose norm is within a relative 1e-10 of
//      the largest, the smallest column index.  A workgroup finds its largest norm,
//      then its smallest index inside that window (two exact reductions); for
//      S > 1 the slabs exchange (largest norm, candidate, its norm) and combine
//      them like the lanes, and when a slab's largest norm lies inside the window
//      of a larger one without its candidate, a second exchange finds the exact
//      index.  Stop when |R_jj| < eps |R_00|;
//   3. the team owning the pivot column publishes its rows (LDS for S = 1, the
//      slab's exchange record for S > 1, one exchange per step) and every thread
//      forms its rows of the reflector (LAPACK dlarfg convention) with identical
//      arithmetic;
//   4. every remaining column is updated in registers, a <- a - tau v (v^T a), and
//      its new trailing norm formed (team sums by lane shuffles).
// Columns are never moved: a column pivoted at step j keeps R_0j..R_j-1,j in its
// rows 0..j-1 and R_jj is set at the end.  At the end every slab writes
// W_cn = R[:r, :] P^T straight into the blocks of p, and slab 0 stores the
// reflectors, sets A_cc = I and publishes the rank.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.h"

namespace spand {

#define CQ_NT 512
#define CQ_MR 32
#define CQ_CPL 2
#define CQ_MR_W 28  // the wide single-slab layout for teams of 2 (k_cpqr_one_w2)
#define CQ_CPL_W 3
#define CQ_MR_1 20  // layout 1 of the multi-slab kernel: fewer rows, more columns per lane
#define CQ_CPL_1 3
#define CQ_XH 16  // doubles of an exchange record's header: a 128-byte line of its own
// Column slots a team keeps in LDS next to its CQ_CPL (or CQ_CPL_1) register slots:
// one when the LDS of a workgroup holds it (MR rows of every thread) beside the
// reflector, pivot-column and R_jj buffers (3 G MR doubles), with 16 KB left for the
// segment offsets and the static LDS; none otherwise (teams of 32 and 64 with 32 rows).
// A thread keeps its MR rows of the slot together (MR + 1 doubles apart from the next
// thread's, so the lanes of a wave spread over the banks): one address and immediate
// offsets reach them all.
__host__ __device__ constexpr int cq_lds_slots(int G, int MR) {
  return (3 * G * MR + (MR + 1) * CQ_NT) * 8 + 16 * 1024 <= 160 * 1024 ? 1 : 0;
}
#define CW 256  // threads of k_build_t
#define TIE_RTOL 1e-10
#define SPIN_LIMIT (1L << 22)

namespace {

// Pivot candidate of a set of columns: the largest norm mx, the smallest column
// index cd among the columns with norm >= mx (1 - TIE_RTOL), its norm cn, and amb
// set when the exact smallest index at a larger threshold is not known.
struct Cand {
  double mx, cn, x2;  // x2: squared norm below row j of candidate cd
  int cd, amb;
};

__device__ inline Cand cand_combine(const Cand& a, const Cand& b) {
  Cand o;
  o.mx = fmax(a.mx, b.mx);
  const double thr = o.mx * (1.0 - TIE_RTOL);
  const bool oka = a.cd != INT_MAX && a.cn >= thr;
  const bool okb = b.cd != INT_MAX && b.cn >= thr;
  o.amb = a.amb | b.amb | ((!oka && a.mx >= thr) ? 1 : 0) | ((!okb && b.mx >= thr) ? 1 : 0);
  o.cd = INT_MAX;
  o.cn = -1.0;
  o.x2 = 0.0;
  if (oka) {
    o.cd = a.cd;
    o.cn = a.cn;
    o.x2 = a.x2;
  }
  if (okb && b.cd < o.cd) {
    o.cd = b.cd;
    o.cn = b.cn;
    o.x2 = b.x2;
  }
  return o;
}

// Cross-lane moves inside rows of 16 lanes (DPP): quad_perm [1,0,3,2] and
// [2,3,0,1] exchange with lane^1 and lane^2, row_half_mirror pairs lane i with
// 7 - i of its 8-lane half, row_mirror pairs i with 15 - i.  Applied in this order
// a combine of the two operands reaches every lane of a group of 2, 4, 8, 16 lanes.
constexpr int DPP_X1 = 0xB1, DPP_X2 = 0x4E, DPP_HMIR = 0x141, DPP_MIR = 0x140;

template <int CTRL>
__device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
// lane ^ 16 inside each half of the wave (ds_swizzle, bit-mask mode)
__device__ inline double swz_x16(double v) {
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
  return __hiloint2double(hi, lo);
}
__device__ inline double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the G lanes of a team (G consecutive lanes, G a power of two <= 64).
// Every step adds two partial sums in either order, so all lanes of the team end
// with the same bits.
template <int G>
__device__ inline double team_sum(double v) {
  if constexpr (G >= 2) v += dpp_d<DPP_X1>(v);
  if constexpr (G >= 4) v += dpp_d<DPP_X2>(v);
  if constexpr (G >= 8) v += dpp_d<DPP_HMIR>(v);
  if constexpr (G >= 16) v += dpp_d<DPP_MIR>(v);
  if constexpr (G >= 32) v += swz_x16(v);
  if constexpr (G >= 64) v = read_lane(v, 0) + read_lane(v, 32);
  return v;
}

// Largest value / smallest int of the wave, returned wave-uniform.
__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_d<DPP_X1>(v));
  v = fmax(v, dpp_d<DPP_X2>(v));
  v = fmax(v, dpp_d<DPP_HMIR>(v));
  v = fmax(v, dpp_d<DPP_MIR>(v));
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}
__device__ inline int wave_min(int v) {
  v = min(v, dpp_i<DPP_X1>(v));
  v = min(v, dpp_i<DPP_X2>(v));
  v = min(v, dpp_i<DPP_HMIR>(v));
  v = min(v, dpp_i<DPP_MIR>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ inline double first_lane(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

// Exchange among the S workgroups of one interface.  Every exchanged value is
// written and read with agent-scope atomic accesses, which are coherent across the
// L2 caches of the XCDs.  A slab stores the rows of its record first; once each of
// its waves has seen its own stores complete, one thread stores the header words.
// Every header word carries the exchange's tag in its sign bit (the values are
// >= 0), so a reader that finds the current tag in all words of a header holds that
// slab's header and may read its rows.  A record buffer is reused every other
// exchange and the tag alternates between its uses; the buffers start zeroed and
// the first tag is 1.  Polls are bounded: on time-out the error flag is raised and
// the workgroup goes on with what it read, so every wave terminates.
__device__ inline double tag_word(double v, int tag) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull;
  return __longlong_as_double((long long)(b | ((unsigned long long)tag << 63)));
}
__device__ inline int word_tag(double x) { return (int)((unsigned long long)__double_as_longlong(x) >> 63); }
__device__ inline double word_val(double x) {
  return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(x) & 0x7FFFFFFFFFFFFFFFull));
}

// Global-space accesses: flat ones would also hold up every wait for LDS.
typedef __attribute__((address_space(1))) double gdouble;
__device__ double g_cq_zero;  // read by the loads of an empty column slot
__device__ inline double shared_load(const double* p) {
  return __hip_atomic_load((const gdouble*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void shared_store(double* p, double v) {
  __hip_atomic_store((gdouble*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the error flag of the launch, read by a poll so that it stops after a time-out
__device__ inline bool timed_out(int32_t* err) {
  return (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4) != 0;
}

// Address of column c of A_pn: entry i at base[i * stride].
__device__ inline void column_ptr(const SegDesc* sg, const int* segoff, int c, double*& base, int64_t& stride) {
  int s = 0;
  while (segoff[s + 1] <= c) ++s;
  const SegDesc g = sg[s];
  const int cs = c - segoff[s];
  if (g.trans) {
    base = g.blk + cs;
    stride = g.ld;
  } else {
    base = g.blk + (int64_t)cs * g.ld;
    stride = 1;
  }
}

}  // namespace

// Row group gi of the update loops: register rows 4 gi .. 4 gi + 3 of every
// column, i.e. rows [4 gi G, 4 gi G + 4 G) of A_pn across the team.
template <int G>
__device__ __forceinline__ void cpqr_load_group(const double* vl, int gi, double (&v)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = vl[(4 * gi + u) * G];
}
template <int MR, int CPL>
__device__ __forceinline__ void cpqr_dot_group(const double (&a)[CPL][MR], int gi, const double (&v)[4],
                                               double (&dot)[CPL]) {
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int k = 0; k < CPL; ++k) dot[k] = fma(v[u], a[k][4 * gi + u], dot[k]);
}
// a <- a - w v and the squared norm of the rows below j (jg = j - g); only the
// group holding row j (mixed) has rows on both sides of it.
template <int G, int MR, int CPL>
__device__ __forceinline__ void cpqr_update_group(double (&a)[CPL][MR], int gi, const double (&v)[4],
                                                  const double (&wv)[CPL], double (&sq)[CPL], bool mixed,
                                                  int jg) {
  if (mixed) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const double x = fma(-wv[k], v[u], a[k][4 * gi + u]);
        a[k][4 * gi + u] = x;
        sq[k] = ((4 * gi + u) * G > jg) ? fma(x, x, sq[k]) : sq[k];
      }
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const double x = fma(-wv[k], v[u], a[k][4 * gi + u]);
        a[k][4 * gi + u] = x;
        sq[k] = fma(x, x, sq[k]);
      }
  }
}

// Slab w of interface d (w = 0, S = 1 when MULTI is false); a lane keeps MR rows
// of CPL columns.
template <int G, bool MULTI, int MR = CQ_MR, int CPL = CQ_CPL, int CPL2 = 0>
__device__ __forceinline__ void cpqr_slab(const SparsDesc& d, int wslab, const SegDesc* __restrict__ segs, double eps,
                                          int32_t* cursize, int32_t* nref, int32_t* err, int32_t* done = nullptr) {
  constexpr int NT = CQ_NT;
  constexpr int NTEAM = NT / G;
  constexpr int KS = CPL + CPL2;  // column slots of a team: CPL in registers, CPL2 (0 or 1) in LDS
  // slots in use for this interface (the host leaves the LDS slot empty where more
  // slabs with less work per step serve better), and the columns of a slab
  const int KU = (CPL2 > 0 && d.kslots > CPL) ? KS : CPL;
  const int CAP = KU * NTEAM;
  constexpr int NW = NT / 64;
  constexpr int ROWS = G * MR;    // rows a team can hold (>= m)
  constexpr int NGRP = MR / 4;    // row groups: group u is rows [4uG, 4uG + 4G), registers 4u..4u+3
  constexpr int RPT = (ROWS + NT - 1) / NT;  // reflector rows formed per thread
  extern __shared__ double lds[];
  __shared__ double pmx[2][NW];
  __shared__ int pcd[2][NW];
  __shared__ double sh_pn, sh_x2;
  __shared__ double xg_mx, xg_pn, xg_x2;  // result of the header reduction of the current exchange
  __shared__ int xg_cd, xg_amb;
  const int m = d.m, S = MULTI ? d.S : 1, w = MULTI ? wslab : 0;
  int tid = threadIdx.x;
  // the round loop of the multi-slab kernel would otherwise hoist the row indices
  // of every slab out of the loop and keep them live, in scratch, for its duration
  if constexpr (MULTI) asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane & (G - 1), team = tid / G;
  const int nseg = d.seg_end - d.seg_begin;
  const SegDesc* sg = segs + d.seg_begin;
  // vv: the reflector of the current step (v_i = 0 above row j and from row m on,
  // v_j = 1); cv: the pivot column as its team publishes it (single slab); rb:
  // R_jj of every step, written into the pivot columns at the end
  double* vv = lds;
  double* cv = lds + ROWS;
  double* rb = lds + 2 * ROWS;
  // the LDS column slot of this thread: its rows q * G + g at lcs[q]
  double* lcs = lds + 3 * ROWS + tid * (MR + 1);
  int* segoff = reinterpret_cast<int*>(lds + 3 * ROWS + CPL2 * (MR + 1) * NT);  // nseg + 1
  // exchange record of slab q in buffer b: header [max, cand norm, cand xn2, cand index + 1,
  // unused up to CQ_XH], then ROWS column rows
  auto xrec = [&](int b, int q) { return d.xch + ((size_t)b * S + q) * (size_t)(ROWS + CQ_XH); };

  // column layout of A_pn from the neighbours' current sizes
  if (tid == 0) {
    int off = 0;
    for (int s = 0; s < nseg; ++s) {
      segoff[s] = off;
      // a neighbour sparsified earlier in the same launch published its rank with a
      // device-scope store
      off += MULTI ? __hip_atomic_load(cursize + sg[s].q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   : cursize[sg[s].q];
    }
    segoff[nseg] = off;
  }
  __syncthreads();
  const int nc = segoff[nseg];
  if (nc == 0) {  // no coupled dofs left: p keeps its size, no reflectors
    if (w == 0 && tid == 0) nref[d.id] = 0;
    if (MULTI && tid == 0 && done) __hip_atomic_fetch_add(done + d.id, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }

  double a[CPL][MR];
  double nrm[KS];  // squared norm of rows j..m-1 (identical in the lanes of a team)
  int col[KS];     // column index in A_pn, -1 if the slot is empty
  int pst[KS];     // -1 remaining, >= 0 step at which the column was the pivot, -2 empty
  // row q * G + g of slot k of this team: registers for k < CPL, LDS for k = CPL
  auto val = [&](int k, int q) -> double { return k < CPL ? a[k < CPL ? k : 0][q] : lcs[q]; };
  if constexpr (CPL2 > 0) {  // the LDS slot (k = CPL), four rows at a time
    const int c = KU > CPL ? w * CAP + CPL * NTEAM + team : nc;
    col[CPL] = c < nc ? c : -1;
    pst[CPL] = c < nc ? -1 : -2;
    const gdouble* base = (const gdouble*)&g_cq_zero;
    int64_t stride = 0;
    if (c < nc) {
      double* b;
      column_ptr(sg, segoff, c, b, stride);
      base = (const gdouble*)b;
    }
    const int rows = (c < nc) ? m : 0;
    double sq = 0.0;
#pragma unroll
    for (int q0 = 0; q0 < MR; q0 += 4) {
      double t4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = (q0 + u) * G + g;
        const gdouble* e = base + (i < rows ? i : 0) * (int)stride;
        t4[u] = MULTI ? __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *e;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double v = ((q0 + u) * G + g < rows) ? t4[u] : 0.0;
        lcs[q0 + u] = v;
        sq = fma(v, v, sq);
      }
      __builtin_amdgcn_sched_barrier(0);  // four rows in registers at a time
    }
    nrm[CPL] = team_sum<G>(sq);
  }
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    const int c = w * CAP + k * NTEAM + team;
    col[k] = c < nc ? c : -1;
    pst[k] = c < nc ? -1 : -2;
    // every load is issued (a row outside the column reads row 0, an empty slot
    // reads g_cq_zero), so the loads of a column are in flight together
    const gdouble* base = (const gdouble*)&g_cq_zero;
    int64_t stride = 0;
    if (c < nc) {
      double* b;
      column_ptr(sg, segoff, c, b, stride);
      base = (const gdouble*)b;
    }
    const int rows = (c < nc) ? m : 0;
#pragma unroll
    for (int q = 0; q < MR; ++q) {
      const int i = q * G + g;
      // device-scope loads in the multi-slab kernel: a neighbour sparsified earlier
      // in the same launch wrote these blocks (from another XCD, perhaps)
      const gdouble* e = base + (i < rows ? i : 0) * (int)stride;
      a[k][q] = MULTI ? __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *e;
    }
    // keep the loads ahead of their uses: scheduled among them the loads would
    // be issued one at a time
    __builtin_amdgcn_sched_barrier(0);
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < MR; ++q) {
      const double v = (q * G + g < rows) ? a[k][q] : 0.0;
      a[k][q] = v;
      sq = fma(v, v, sq);
    }
    nrm[k] = team_sum<G>(sq);
  }

  const int kmax = min(m, nc);
  const int uend = (m + 4 * G - 1) / (4 * G);  // groups holding rows below m
  int r = kmax;
  double r00 = 0.0;
  int namb = 0;  // second exchange rounds so far (identical in all slabs)
  for (int j = 0; j < kmax; ++j) {
    const int jg = j - g;  // row q * G + g of this lane lies below row j iff q * G > jg
    // ---- pivot of this slab: the largest remaining norm M, then the smallest column
    // index whose norm is >= M (1 - TIE_RTOL); two exact reductions
    double nv[KS];
    double lmx = -1.0;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      nv[k] = (pst[k] == -1) ? sqrt(nrm[k]) : -1.0;
      lmx = fmax(lmx, nv[k]);
    }
    lmx = wave_max(lmx);
    if (lane == 0) pmx[j & 1][wave] = lmx;
    __syncthreads();
    double smx = pmx[j & 1][0];
#pragma unroll
    for (int q = 1; q < NW; ++q) smx = fmax(smx, pmx[j & 1][q]);
    int scd;
    {
      const double thr = smx * (1.0 - TIE_RTOL);
      int c = INT_MAX;
#pragma unroll
      for (int k = 0; k < KS; ++k)
        if (pst[k] == -1 && nv[k] >= thr) c = min(c, col[k]);
      c = wave_min(c);
      if (lane == 0) pcd[j & 1][wave] = c;
      __syncthreads();
      scd = pcd[j & 1][0];
#pragma unroll
      for (int q = 1; q < NW; ++q) scd = min(scd, pcd[j & 1][q]);
    }
    if (!MULTI && scd == INT_MAX) {  // only non-finite norms left
      r = j;
      break;
    }
    // team and register slot of this slab's candidate
    const int lc = scd - w * CAP;
    const bool own = scd != INT_MAX && team == lc % NTEAM;
    const int pk = own ? lc / NTEAM : 0;
    const int ujp = j / (4 * G);  // row group holding row j
    int piv;
    double pn, x2, alpha;
    const double* rc = nullptr;
    if constexpr (!MULTI) {
      // the owner team publishes its column and the squared norm of its rows below j
      if (own) {
#pragma unroll
        for (int k = 0; k < KS; ++k)
          if (k == pk) {
            double s2 = 0.0;
#pragma unroll
            for (int gi = 0; gi < NGRP; ++gi) {
              if (gi >= ujp && gi < uend) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                  const int q = 4 * gi + u;
                  const double x = val(k, q);
                  cv[q * G + g] = x;
                  s2 = (gi > ujp || q * G > jg) ? fma(x, x, s2) : s2;
                }
              }
            }
            s2 = team_sum<G>(s2);
            if (g == 0) {
              sh_pn = nv[k];
              sh_x2 = s2;
            }
          }
      }
      __syncthreads();
      piv = scd;
      pn = sh_pn;
      x2 = sh_x2;
    } else {
      // publish (slab max, slab candidate + 1, its norm, its rows and its squared
      // norm below j).  The rows of a record are stored lane-major: row q * G + g
      // at g * MR + q.
      const int tg = ((j >> 1) & 1) ^ 1;
      {
        double* rw = xrec(j & 1, w);
        if (own) {
#pragma unroll
          for (int k = 0; k < KS; ++k)
            if (k == pk) {
              double* rl = rw + CQ_XH + g * MR;
              double s2 = 0.0;
#pragma unroll
              for (int gi = 0; gi < NGRP; ++gi) {
                if (gi >= ujp && gi < uend) {
#pragma unroll
                  for (int u = 0; u < 4; ++u) {
                    const int q = 4 * gi + u;
                    const double x = val(k, q);
                    shared_store(rl + q, x);
                    s2 = (gi > ujp || q * G > jg) ? fma(x, x, s2) : s2;
                  }
                }
              }
              s2 = team_sum<G>(s2);
              if (g == 0) {
                // the team lies in one wave: once this wave's stores have completed
                // the rows are visible, and the header may follow
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                __builtin_amdgcn_s_waitcnt(0);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                shared_store(rw, tag_word(smx, tg));
                shared_store(rw + 1, tag_word(nv[k], tg));
                shared_store(rw + 2, tag_word(s2, tg));
                shared_store(rw + 3, tag_word((double)scd + 1.0, tg));
              }
            }
        }
        if (scd == INT_MAX && tid == 0) {  // no candidate left in this slab
          shared_store(rw, tag_word(0.0, tg));
          shared_store(rw + 1, tag_word(0.0, tg));
          shared_store(rw + 2, tag_word(0.0, tg));
          shared_store(rw + 3, tag_word(0.0, tg));
        }
      }
      int xb = j & 1;
      // wave 0 polls the S headers (one memory round trip per poll) and reduces them
      // like the lanes: lanes 0..P-1 end with the same result, which carries the
      // winner's norm and squared norm below j.  The owning slab of column c is c / CAP.
      if (wave == 0) {
        int P = 1;
        while (P < S && P < 64) P <<= 1;
        Cand u;
        for (long spins = 0;; ++spins) {
          u.mx = -1.0;
          u.cn = -1.0;
          u.x2 = 0.0;
          u.cd = INT_MAX;
          u.amb = 0;
          int ok = 1;
          for (int q = lane; q < S; q += 64) {  // S may exceed the wave size
            const double* rq = xrec(xb, q);
            const double w0 = shared_load(rq), w1 = shared_load(rq + 1), w2 = shared_load(rq + 2),
                         w3 = shared_load(rq + 3);
            ok &= (word_tag(w0) == tg) & (word_tag(w1) == tg) & (word_tag(w2) == tg) & (word_tag(w3) == tg);
            const double cq = word_val(w3);
            Cand v;
            v.mx = (cq > 0.0) ? word_val(w0) : -1.0;
            v.cn = (cq > 0.0) ? word_val(w1) : -1.0;
            v.x2 = word_val(w2);
            v.cd = (cq > 0.0) ? (int)cq - 1 : INT_MAX;
            v.amb = 0;
            u = cand_combine(u, v);
          }
          if (__all(ok)) break;
          if (spins > SPIN_LIMIT) {
            if (lane == 0) atomicOr(err, 4);
            break;
          }
          if ((spins & 1023) == 1023 && timed_out(err)) break;  // after a time-out the polls give up at once
          __builtin_amdgcn_s_sleep(1);
        }
        for (int o = 1; o < P; o <<= 1) {
          Cand v;
          v.mx = __shfl_xor(u.mx, o, 64);
          v.cn = __shfl_xor(u.cn, o, 64);
          v.x2 = __shfl_xor(u.x2, o, 64);
          v.cd = __shfl_xor(u.cd, o, 64);
          v.amb = __shfl_xor(u.amb, o, 64);
          u = cand_combine(u, v);
        }
        if (lane == 0) {
          xg_mx = u.mx;
          xg_cd = u.cd;
          xg_amb = u.amb;
          xg_pn = u.cn;
          xg_x2 = u.x2;
        }
      }
      __syncthreads();
      piv = xg_cd;
      if (xg_amb) {  // second round with the exact global threshold (near-ties across slabs)
        xb = 2;
        const int tg2 = (namb & 1) ^ 1;
        ++namb;
        const double thr = xg_mx * (1.0 - TIE_RTOL);
        int c2 = INT_MAX;
#pragma unroll
        for (int k = 0; k < KS; ++k)
          if (pst[k] == -1 && nv[k] >= thr) c2 = min(c2, col[k]);
        c2 = wave_min(c2);
        if (lane == 0) pcd[j & 1][wave] = c2;  // free: every wave has read pcd[j & 1]
        __syncthreads();
        int best = pcd[j & 1][0];
#pragma unroll
        for (int q = 1; q < NW; ++q) best = min(best, pcd[j & 1][q]);
        const int lc2 = best - w * CAP;
        double* rw = xrec(2, w);
        if (best != INT_MAX && team == lc2 % NTEAM) {
          const int pk2 = lc2 / NTEAM;
#pragma unroll
          for (int k = 0; k < KS; ++k)
            if (k == pk2) {
              double* rl = rw + CQ_XH + g * MR;
              double s2 = 0.0;
#pragma unroll
              for (int q = 0; q < MR; ++q) {
                const double x = val(k, q);
                shared_store(rl + q, x);
                s2 = (q * G > jg) ? fma(x, x, s2) : s2;
              }
              s2 = team_sum<G>(s2);
              if (g == 0) {
                shared_store(rw + 2, s2);
                sh_pn = nv[k];
              }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
          const bool none = best == INT_MAX;
          shared_store(rw + 1, tag_word(none ? 0.0 : sh_pn, tg2));
          shared_store(rw + 3, tag_word(none ? 0.0 : (double)best + 1.0, tg2));
        }
        if (wave == 0) {
          int b2;
          for (long spins = 0;; ++spins) {
            b2 = INT_MAX;
            int ok = 1;
            for (int q = lane; q < S; q += 64) {
              const double* rq = xrec(2, q);
              const double w1 = shared_load(rq + 1), w3 = shared_load(rq + 3);
              ok &= (word_tag(w1) == tg2) & (word_tag(w3) == tg2);
              const double cq = word_val(w3);
              if (cq > 0.0) b2 = min(b2, (int)cq - 1);
            }
            if (__all(ok)) break;
            if (spins > SPIN_LIMIT) {
              if (lane == 0) atomicOr(err, 4);
              break;
            }
            if ((spins & 1023) == 1023 && timed_out(err)) break;
            __builtin_amdgcn_s_sleep(1);
          }
          b2 = wave_min(b2);
          if (lane == 0) xg_cd = b2;
        }
        __syncthreads();
        piv = xg_cd;
      }
      if (piv == INT_MAX) {  // only non-finite norms left
        r = j;
        break;
      }
      rc = xrec(xb, piv / CAP);
      if (xb == 2) {  // second round: its header is read here
        pn = word_val(shared_load(rc + 1));
        x2 = shared_load(rc + 2);
      } else {
        pn = xg_pn;
        x2 = xg_x2;
      }
    }
    if (j == 0) {
      r00 = pn;
      if (r00 == 0.0) {
        r = 0;
        break;
      }
    }
    if (pn < eps * r00) {
      r = j;
      break;
    }
    // every thread forms the reflector (LAPACK dlarfg convention) with identical
    // arithmetic, then its share of the rows of v; alpha (row j of the pivot column)
    // and the rows are read together
    double tau = 0.0, scale = 0.0, beta;
    {
      double xs[RPT];
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int i = tid + u * NT;
        if constexpr (MULTI) {
          // every thread loads (row j when its row is not below j): the loads of
          // all rows are in flight together
          const bool use = i > j && i < m;
          const int ir = use ? i : j;
          const double x = shared_load(rc + CQ_XH + (ir % G) * MR + ir / G);
          xs[u] = use ? x : 0.0;
        } else
          xs[u] = (i < ROWS) ? cv[i] : 0.0;
      }
      if constexpr (MULTI)
        alpha = shared_load(rc + CQ_XH + (j % G) * MR + j / G);
      else
        alpha = cv[j];
      beta = alpha;
      if (x2 != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + x2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int i = tid + u * NT;
        if (i < ROWS) {
          const double v = (i > j) ? xs[u] * scale : ((i == j) ? 1.0 : 0.0);
          vv[i] = v;
          if (w == 0 && i < m) d.V[(int64_t)j * d.ldv + i] = v;
        }
      }
    }
    if (tid == 0) {
      rb[j] = beta;
      if (w == 0) d.tau[j] = tau;
    }
    {  // the pivot column becomes column j of R (its rows are set at the write-back)
      const int plc = piv - w * CAP;
      if (plc >= 0 && plc < CAP && team == plc % NTEAM) {
#pragma unroll
        for (int k = 0; k < KS; ++k)
          if (k == plc / NTEAM) pst[k] = j;
      }
    }
    __syncthreads();
    // ---- apply H_j to the remaining columns and form their new trailing norms.
    // Only the row groups uj..uend-1 take part: rows above j have v = 0 and leave
    // the norms, rows from m on are zero.  Group uj holds row j and is the only one
    // with rows on both sides of it.
    const int uj = j / (4 * G);
    const double* vl = vv + g;
    // v of a group is read one group ahead into two register sets used by even
    // and odd groups in turn, so the reads overlap the previous group's FMAs
    double va[4], vb[4];
    double dot[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) dot[k] = 0.0;

    if (uj & 1) {
#pragma unroll
      for (int u = 0; u < 4; ++u) vb[u] = vl[(4 * uj + u) * G];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) va[u] = vl[(4 * uj + u) * G];
    }
#pragma unroll
    for (int gp = 0; gp < NGRP; gp += 2) {
      if (gp >= uj && gp < uend) {
        cpqr_load_group<G>(vl, gp + 1, vb);  // unconditional: a fixed count of LDS reads in flight
        cpqr_dot_group<MR, CPL>(a, gp, va, dot);
      }
      if (gp + 1 >= uj && gp + 1 < uend) {
        if (gp + 2 < NGRP) cpqr_load_group<G>(vl, gp + 2, va);
        cpqr_dot_group<MR, CPL>(a, gp + 1, vb, dot);
      }
    }
    double wv[CPL], sq[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      dot[k] = team_sum<G>(dot[k]);
      wv[k] = (pst[k] == -1) ? tau * dot[k] : 0.0;
      sq[k] = 0.0;
    }

    if (uj & 1) {
#pragma unroll
      for (int u = 0; u < 4; ++u) vb[u] = vl[(4 * uj + u) * G];
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) va[u] = vl[(4 * uj + u) * G];
    }
#pragma unroll
    for (int gp = 0; gp < NGRP; gp += 2) {
      if (gp >= uj && gp < uend) {
        cpqr_load_group<G>(vl, gp + 1, vb);  // unconditional: a fixed count of LDS reads in flight
        cpqr_update_group<G, MR, CPL>(a, gp, va, wv, sq, gp == uj, jg);
      }
      if (gp + 1 >= uj && gp + 1 < uend) {
        if (gp + 2 < NGRP) cpqr_load_group<G>(vl, gp + 2, va);
        cpqr_update_group<G, MR, CPL>(a, gp + 1, vb, wv, sq, gp + 1 == uj, jg);
      }
    }
#pragma unroll
    for (int k = 0; k < CPL; ++k) nrm[k] = team_sum<G>(sq[k]);
    if (CPL2 > 0 && pst[CPL] == -1) {
      // the LDS slot, after the register slots (fewer values live at once): the same
      // two passes, a <- a - tau (v . a) v and its squared norm below j (a team whose
      // slot is empty or holds a pivot column skips them)
      double dot2 = 0.0;
#pragma unroll
      for (int gi = 0; gi < NGRP; ++gi)
        if (gi >= uj && gi < uend) {
#pragma unroll
          for (int u = 0; u < 4; ++u) dot2 = fma(vl[(4 * gi + u) * G], lcs[4 * gi + u], dot2);
        }
      dot2 = team_sum<G>(dot2);
      const double wv2 = tau * dot2;
      double sq2 = 0.0;
#pragma unroll
      for (int gi = 0; gi < NGRP; ++gi)
        if (gi >= uj && gi < uend) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = 4 * gi + u;
            const double x = fma(-wv2, vl[q * G], lcs[q]);
            lcs[q] = x;
            sq2 = (gi > uj || q * G > jg) ? fma(x, x, sq2) : sq2;
          }
        }
      nrm[CPL] = team_sum<G>(sq2);
    }
  }
  __syncthreads();  // rb complete
  // ---- W_cn = R[:r, :] (column order of A_pn) into the blocks of p.  A pivot
  // column of step s holds R_ij for i < s; its row s is R_ss and the rows below are 0.
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    if (col[k] < 0 || r == 0) continue;
    double* base;
    int64_t stride;
    column_ptr(sg, segoff, col[k], base, stride);
    const int ps = pst[k];
    const double rss = (ps >= 0) ? rb[ps] : 0.0;
    if (d.piv && ps >= 0 && g == 0) d.piv[ps] = col[k];
#pragma unroll
    for (int q = 0; q < MR; ++q) {
      const int i = q * G + g;
      if (i < r) {
        const double v = (ps >= 0 && i >= ps) ? ((i == ps) ? rss : 0.0) : val(k, q);
        if constexpr (MULTI)
          shared_store(base + (int64_t)i * stride, v);  // read by later neighbours of the launch
        else
          base[(int64_t)i * stride] = v;
      }
    }
  }
  if (w == 0) {
    for (int64_t e = tid; e < (int64_t)r * r; e += NT) {
      const int x = (int)(e % r), y = (int)(e / r);
      d.diag[x + (int64_t)y * d.ldd] = (x == y) ? 1.0 : 0.0;
    }
    if (tid == 0) {
      if constexpr (MULTI)
        __hip_atomic_store(cursize + d.id, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        cursize[d.id] = r;
      nref[d.id] = r;
    }
  }
  if constexpr (MULTI) {
    // this slab is done once its stores have completed: the neighbours that wait for
    // p count the slabs of p (k_cpqr_multi)
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0 && done) __hip_atomic_fetch_add(done + d.id, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Single-slab interfaces: one launch per team size.
template <int G>
__global__ void __launch_bounds__(CQ_NT) k_cpqr_one(const SparsDesc* __restrict__ descs,
                                                    const SlabRef* __restrict__ slabs,
                                                    const SegDesc* __restrict__ segs, double eps, int32_t* cursize,
                                                    int32_t* nref, int32_t* err) {
  const SlabRef sr = slabs[blockIdx.x];
  cpqr_slab<G, false, CQ_MR, CQ_CPL, cq_lds_slots(G, CQ_MR)>(descs[sr.desc], 0, segs, eps, cursize, nref, err);
}

// Single-slab interfaces of at most 2 * CQ_MR_W rows whose width needs more than
// one slab of the standard layout: teams of 2 lanes with CQ_MR_W rows and
// CQ_CPL_W columns per lane, so one workgroup holds CQ_CPL_W * CQ_NT / 2 columns.
__global__ void __launch_bounds__(CQ_NT) k_cpqr_one_w2(const SparsDesc* __restrict__ descs,
                                                       const SlabRef* __restrict__ slabs,
                                                       const SegDesc* __restrict__ segs, double eps, int32_t* cursize,
                                                       int32_t* nref, int32_t* err) {
  const SlabRef sr = slabs[blockIdx.x];
  cpqr_slab<2, false, CQ_MR_W, CQ_CPL_W>(descs[sr.desc], 0, segs, eps, cursize, nref, err);
}

// Multi-slab interfaces of every team size in one cooperative launch: each
// workgroup takes the code path of its interface's G.  Workgroup b runs the slabs
// slabs[k * gridDim.x + b], k = 0 .. nround - 1, in turn (a negative descriptor
// index is an unused place).  The host numbers the interfaces and every workgroup's
// slabs come in that order.  An interface may depend on neighbours numbered before
// it (a launch that holds several colour classes): deps[dep_begin, dep_end) lists
// (neighbour id, its slab count), and its slabs wait until done[neighbour] has
// counted every slab of the neighbour; the neighbour's blocks, rank and current
// size are then read with device-scope loads.  The lowest-numbered unfinished
// interface therefore has every neighbour it waits for finished and each of its
// slabs at the head of its workgroup's remaining list (all workgroups are
// resident): it completes, and by induction every later one.  The waits are
// bounded like the exchange polls.
__global__ void __launch_bounds__(CQ_NT) k_cpqr_multi(const SparsDesc* __restrict__ descs,
                                                      const SlabRef* __restrict__ slabs, int32_t nround,
                                                      const SegDesc* __restrict__ segs, double eps,
                                                      int32_t* cursize, int32_t* nref, int32_t* err,
                                                      const int2* __restrict__ deps, int32_t* done) {
  for (int32_t rd = 0; rd < nround; ++rd) {
    const SlabRef sr = slabs[(size_t)rd * gridDim.x + blockIdx.x];
    if (sr.desc < 0) continue;
    const SparsDesc d = descs[sr.desc];
    if (d.dep_end > d.dep_begin) {
      if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        for (long spins = 0;; ++spins) {
          int ok = 1;
          for (int e = d.dep_begin + lane; e < d.dep_end; e += 64) {
            const int2 q = deps[e];
            ok &= __hip_atomic_load(done + q.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= q.y;
          }
          if (__all(ok)) break;
          if (spins > SPIN_LIMIT) {
            if (lane == 0) atomicOr(err, 4);
            break;
          }
          if ((spins & 1023) == 1023 && timed_out(err)) break;
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __syncthreads();
    }
#define CQ_CASE(GG)                                                                   \
  case GG: cpqr_slab<GG, true, CQ_MR, CQ_CPL, cq_lds_slots(GG, CQ_MR)>(d, sr.w, segs, eps, cursize, nref, err, done); \
    break;                                                                                                          \
  case GG | 256:                                                                                                    \
    cpqr_slab<GG, true, CQ_MR_1, CQ_CPL_1, cq_lds_slots(GG, CQ_MR_1)>(d, sr.w, segs, eps, cursize, nref, err, done); \
    break;
    switch (d.G | (d.lay << 8)) {
      CQ_CASE(1)
      CQ_CASE(2)
      CQ_CASE(4)
      CQ_CASE(8)
      CQ_CASE(16)
      CQ_CASE(32)
      CQ_CASE(64)
      default: break;  // the host only builds the team sizes and layouts above
    }
#undef CQ_CASE
    __syncthreads();  // the LDS of this slab is reused by the next round's
  }
}


// Compact WY factor of Q = H_0 ... H_{r-1} = I - V T V^T (T upper triangular):
// T_jj = tau_j, T[:j, j] = -tau_j T[:j, :j] (V[:, :j]^T v_j).  On entry the upper
// triangle of T holds S = V^T V (a batched GEMM).  T is built by 64-wide block
// columns: every diagonal block T_JJ follows from S_JJ and the taus of its columns
// alone (k_build_t_diag, all blocks of all interfaces in one launch, recurrence in
// LDS); the blocks above it follow from splitting Q = Q_1 Q_2 at column J0,
//   T[:J0, J] = -T[:J0, :J0] (S[:J0, J] T_JJ),
// two batched GEMMs per block column J = 1, 2, ... issued by the host.  The strict
// lower triangle is set to zero (the tiled products of the apply read it).
__global__ void __launch_bounds__(CW) k_build_t_diag(const TBlock* __restrict__ blocks) {
  const TBlock b = blocks[blockIdx.x];
  const int r = b.r, j0 = b.j0, w = min(64, r - j0);
  const int64_t ld = b.ld;
  __shared__ double tl[64 * 65];
  const int below = r - j0;
  for (int q = threadIdx.x; q < below * w; q += CW) {  // zeros under the diagonal of this block column
    const int i = j0 + q % below, j = j0 + q / below;
    if (i > j) b.T[i + j * ld] = 0.0;
  }
  for (int q = threadIdx.x; q < w * w; q += CW) {
    const int i = q % w, j = q / w;
    tl[i + j * 65] = (i < j) ? b.T[(j0 + i) + (j0 + j) * ld] : 0.0;
  }
  __syncthreads();
  const int i = threadIdx.x;
  for (int j = 0; j < w; ++j) {
    double acc = 0.0;
    if (i < j)
      for (int l = i; l < j; ++l) acc += tl[i + l * 65] * tl[l + j * 65];
    __syncthreads();
    if (i < j) tl[i + j * 65] = -b.tau[j0 + j] * acc;
    if (i == j) tl[j + j * 65] = b.tau[j0 + j];
    __syncthreads();
  }
  for (int q = threadIdx.x; q < w * w; q += CW) {
    const int ii = q % w, jj = q / w;
    if (ii <= jj) b.T[(j0 + ii) + (j0 + jj) * ld] = tl[ii + jj * 65];
  }
}

void launch_build_t_diag(const TBlock* blocks, int32_t count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_build_t_diag, dim3(count), dim3(CW), 0, s, blocks);
}

static int32_t layout_rows(int32_t lay) { return lay == 1 ? CQ_MR_1 : CQ_MR; }
int32_t cpqr_team(int32_t m, int32_t lay) {
  int32_t G = 1;
  while (G * layout_rows(lay) < m) G <<= 1;
  return G <= 64 ? G : -1;
}

int32_t cpqr_kslots(int32_t G, int32_t lay, bool lds_slot) {
  return (lay == 1 ? CQ_CPL_1 : CQ_CPL) + (lds_slot ? cq_lds_slots(G, layout_rows(lay)) : 0);
}
int32_t cpqr_capacity(int32_t G, int32_t lay, bool lds_slot) { return cpqr_kslots(G, lay, lds_slot) * CQ_NT / G; }

size_t cpqr_lds_bytes(int32_t G, int32_t lay, int32_t nseg) {
  const size_t mr = size_t(layout_rows(lay));
  return (3 * size_t(G) * mr + size_t(cq_lds_slots(G, int(mr))) * (mr + 1) * CQ_NT) * sizeof(double) +
         (size_t(nseg) + 1) * sizeof(int32_t) + 16;
}

int32_t cpqr_record(int32_t G, int32_t lay) { return G * layout_rows(lay) + CQ_XH; }

int32_t cpqr_wide_rows() { return 2 * CQ_MR_W; }
int32_t cpqr_wide_capacity() { return CQ_CPL_W * CQ_NT / 2; }
size_t cpqr_wide_lds_bytes(int32_t nseg) {
  return 3 * size_t(2) * CQ_MR_W * sizeof(double) + (size_t(nseg) + 1) * sizeof(int32_t) + 16;
}
hipError_t launch_cpqr_one_wide(const SparsDesc* d, const SlabRef* slabs, int32_t nslab, const SegDesc* seg,
                                double eps, int32_t* cursize, int32_t* nref, int32_t* err, size_t lds,
                                hipStream_t s) {
  if (nslab == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpqr_one_w2, dim3(nslab), dim3(CQ_NT), lds, s, d, slabs, seg, eps, cursize, nref, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interfaces beyond the register layouts (more than 2048 rows, or more columns than
// the co-resident slabs hold): one cooperative launch per interface.  The NB
// workgroups of the launch own the columns c = b, b + NB, ... of A_pn, kept in a
// global work copy Wk (m x nc, ld m); the same Householder QR with column pivoting
// as the slab kernels (exact trailing norms recomputed every step, the pivot is the
// smallest column index whose norm is within TIE_RTOL of the largest, the dlarfg
// reflector convention, the ratio stop rule), with two grid-wide barriers per step:
//   after the update, each workgroup posts the largest norm of its remaining
//   columns; barrier; every workgroup combines them and posts its smallest column
//   index inside the window; barrier; every workgroup combines those, reads the
//   pivot column, forms the reflector in LDS with identical arithmetic, and
//   updates its own columns.
// Wk, the posts and the barrier counter are written and read with agent-scope
// atomic accesses (coherent across the XCD caches); a workgroup waits for its stores
// to complete before it arrives at a barrier.  Waits are bounded: on time-out bit 2
// of err is set and every workgroup leaves.
#define CB_NT 256
#define CB_MAXM 7680  // rows of the reflector kept in LDS
struct BigScratch {
  double* wk;      // m x nc, ld m
  double* nrm;     // nc: squared norm of rows j..m-1 of each column
  int32_t* pst;    // nc: step at which the column was the pivot, -1 remaining
  double* rb;      // R_jj of every step
  double* post_mx; // NB
  int32_t* post_cd;// NB
  uint32_t* bar;   // barrier counter, zero at launch
};

__device__ inline double big_wave_sum(double v) {
  v += dpp_d<DPP_X1>(v);
  v += dpp_d<DPP_X2>(v);
  v += dpp_d<DPP_HMIR>(v);
  v += dpp_d<DPP_MIR>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

__device__ inline int big_pst(const BigScratch& bs, int c) {
  return __hip_atomic_load(bs.pst + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier number k (1, 2, ...) of the launch; false on time-out.
__device__ inline bool big_barrier(uint32_t* bar, uint32_t k, int32_t* err) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t target = k * gridDim.x;
    for (long spins = 0;; ++spins) {
      if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (spins > SPIN_LIMIT || ((spins & 1023) == 1023 && timed_out(err))) {
        atomicOr(err, 4);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  return ok != 0;
}

__global__ void __launch_bounds__(CB_NT) k_cpqr_big(SparsDesc d, const SegDesc* __restrict__ segs, double eps,
                                                   int32_t* cursize, int32_t* nref, int32_t* err, BigScratch bs) {
  __shared__ double vv[CB_MAXM];
  __shared__ double red[CB_NT / 64];
  __shared__ int redi[CB_NT / 64];
  __shared__ int segoff_s[65];
  extern __shared__ int segoff_dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NWV = CB_NT / 64;
  const int NB = gridDim.x, b = blockIdx.x;
  const int nseg = d.seg_end - d.seg_begin;
  const SegDesc* sg = segs + d.seg_begin;
  int* segoff = nseg < 64 ? segoff_s : segoff_dyn;
  if (tid == 0) {
    int off = 0;
    for (int s = 0; s < nseg; ++s) {
      segoff[s] = off;
      off += cursize[sg[s].q];
    }
    segoff[nseg] = off;
  }
  __syncthreads();
  const int m = d.m, nc = segoff[nseg];
  if (nc == 0) {
    if (b == 0 && tid == 0) nref[d.id] = 0;
    return;
  }
  double* wk = bs.wk;
  auto W = [&](int i, int c) -> double* { return wk + (int64_t)c * m + i; };
  // load the owned columns and their norms
  for (int c = b + NB * wave; c < nc; c += NB * NWV) {
    double* base;
    int64_t stride;
    column_ptr(sg, segoff, c, base, stride);
    double s2 = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double v = base[(int64_t)i * stride];
      shared_store(W(i, c), v);
      s2 = fma(v, v, s2);
    }
    s2 = big_wave_sum(s2);
    if (lane == 0) {
      shared_store(bs.nrm + c, s2);
      __hip_atomic_store(bs.pst + c, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  uint32_t nbar = 0;
  const int kmax = min(m, nc);
  int r = kmax;
  double r00 = 0.0;
  bool alive = true;
  for (int j = 0; j < kmax && alive; ++j) {
    // largest remaining norm of this workgroup
    __syncthreads();  // the owner-written norms of this workgroup are visible to its threads
    double lmx = -1.0;
    for (int c = b + NB * tid; c < nc; c += NB * CB_NT)
      if (big_pst(bs, c) == -1) lmx = fmax(lmx, sqrt(shared_load(bs.nrm + c)));
    lmx = wave_max(lmx);
    if (lane == 0) red[wave] = lmx;
    __syncthreads();
    if (tid == 0) {
      double x = red[0];
      for (int q = 1; q < NWV; ++q) x = fmax(x, red[q]);
      shared_store(bs.post_mx + b, x);
    }
    if (!big_barrier(bs.bar, ++nbar, err)) { alive = false; break; }
    double gmx = -1.0;
    for (int q = 0; q < NB; ++q) gmx = fmax(gmx, shared_load(bs.post_mx + q));
    const double thr = gmx * (1.0 - TIE_RTOL);
    int lcd = INT_MAX;
    for (int c = b + NB * tid; c < nc; c += NB * CB_NT)
      if (big_pst(bs, c) == -1 && sqrt(shared_load(bs.nrm + c)) >= thr) lcd = min(lcd, c);
    lcd = wave_min(lcd);
    if (lane == 0) redi[wave] = lcd;
    __syncthreads();
    if (tid == 0) {
      int x = redi[0];
      for (int q = 1; q < NWV; ++q) x = min(x, redi[q]);
      __hip_atomic_store(bs.post_cd + b, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!big_barrier(bs.bar, ++nbar, err)) { alive = false; break; }
    int piv = INT_MAX;
    for (int q = 0; q < NB; ++q)
      piv = min(piv, __hip_atomic_load(bs.post_cd + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (piv == INT_MAX) {  // only non-finite norms left
      r = j;
      break;
    }
    // the pivot column: its norm (rows j..), alpha and the squared norm below j, by
    // every workgroup with the same arithmetic
    double s_all = 0.0, s_low = 0.0;
    for (int i = j + tid; i < m; i += CB_NT) {
      const double x = shared_load(W(i, piv));
      vv[i] = x;
      s_all = fma(x, x, s_all);
      if (i > j) s_low = fma(x, x, s_low);
    }
    s_all = big_wave_sum(s_all);
    s_low = big_wave_sum(s_low);
    __shared__ double red2[2][CB_NT / 64];
    if (lane == 0) {
      red2[0][wave] = s_all;
      red2[1][wave] = s_low;
    }
    __syncthreads();
    double pn2 = 0.0, x2 = 0.0;
    for (int q = 0; q < NWV; ++q) {
      pn2 += red2[0][q];
      x2 += red2[1][q];
    }
    const double pn = sqrt(pn2);
    if (j == 0) {
      r00 = pn;
      if (r00 == 0.0) {
        r = 0;
        break;
      }
    }
    if (pn < eps * r00) {
      r = j;
      break;
    }
    const double alpha = vv[j];
    double tau = 0.0, scale = 0.0, beta = alpha;
    if (x2 != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + x2), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();  // every thread has read alpha
    for (int i = j + tid; i < m; i += CB_NT) vv[i] = (i == j) ? 1.0 : vv[i] * scale;
    __syncthreads();
    if (b == 0) {
      for (int i = tid; i < m; i += CB_NT) d.V[(int64_t)j * d.ldv + i] = (i >= j) ? vv[i] : 0.0;
      if (tid == 0) {
        d.tau[j] = tau;
        shared_store(bs.rb + j, beta);
      }
    }
    if (piv % NB == b && tid == 0) __hip_atomic_store(bs.pst + piv, j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // apply H_j to the owned remaining columns and form their new trailing norms
    for (int c = b + NB * wave; c < nc; c += NB * NWV) {
      if (big_pst(bs, c) != -1) continue;
      double dt = 0.0;
      for (int i = j + lane; i < m; i += 64) dt = fma(vv[i], shared_load(W(i, c)), dt);
      dt = big_wave_sum(dt);
      const double wv = tau * dt;
      double s2 = 0.0;
      for (int i = j + lane; i < m; i += 64) {
        const double x = fma(-wv, vv[i], shared_load(W(i, c)));
        shared_store(W(i, c), x);
        if (i > j) s2 = fma(x, x, s2);
      }
      s2 = big_wave_sum(s2);
      if (lane == 0) shared_store(bs.nrm + c, s2);
    }
  }
  // every R_jj (posted by workgroup 0) is visible past one more barrier
  if (alive && !big_barrier(bs.bar, ++nbar, err)) alive = false;
  if (!alive) return;
  // W_cn = R[:r, :] into the blocks of p; a pivot column of step s holds R_is for
  // i < s, R_ss = rb[s] and zeros below
  for (int c = b + NB * wave; c < nc; c += NB * NWV) {
    if (r == 0) break;
    double* base;
    int64_t stride;
    column_ptr(sg, segoff, c, base, stride);
    const int ps = big_pst(bs, c);
    if (d.piv && ps >= 0 && lane == 0) d.piv[ps] = c;
    for (int i = lane; i < r; i += 64) {
      double v;
      if (ps >= 0 && i >= ps)
        v = (i == ps) ? shared_load(bs.rb + ps) : 0.0;
      else
        v = shared_load(W(i, c));
      base[(int64_t)i * stride] = v;
    }
  }
  if (b == 0) {
    for (int64_t e = tid; e < (int64_t)r * r; e += CB_NT) {
      const int x = (int)(e % r), y = (int)(e / r);
      d.diag[x + (int64_t)y * d.ldd] = (x == y) ? 1.0 : 0.0;
    }
    if (tid == 0) {
      cursize[d.id] = r;
      nref[d.id] = r;
    }
  }
}

int32_t cpqr_big_max_rows() { return CB_MAXM; }

namespace {

// Co-resident workgroups of a cooperative CPQR kernel on the current device for a
// dynamic LDS size: the runtime's occupancy answer, remembered per (device, kernel,
// LDS bytes), since the host asks once per interface while it plans a step.
int coresident(const void* kernel, int nt, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, size_t>, int> known;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = std::make_tuple(dev, kernel, lds);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = known.find(key);
    if (it != known.end()) return it->second;
  }
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, lds) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> g(mu);
  known[key] = per_cu * cus;
  return per_cu * cus;
}

}  // namespace

int cpqr_big_max_coresident(int32_t nseg) {
  const size_t lds = nseg < 64 ? 0 : (size_t(nseg) + 1) * sizeof(int);
  return coresident(reinterpret_cast<const void*>(&k_cpqr_big), CB_NT, lds);
}

hipError_t launch_cpqr_big(const SparsDesc& d, int32_t nseg, const SegDesc* seg, double eps, int32_t* cursize,
                           int32_t* nref, int32_t* err, int32_t nb, double* wk, double* nrm, int32_t* pst, double* rb,
                           double* post_mx, int32_t* post_cd, uint32_t* bar, hipStream_t s) {
  BigScratch bs{wk, nrm, pst, rb, post_mx, post_cd, bar};
  SparsDesc dd = d;
  const size_t lds = nseg < 64 ? 0 : (size_t(nseg) + 1) * sizeof(int);
  void* args[] = {(void*)&dd, (void*)&seg, (void*)&eps, (void*)&cursize, (void*)&nref, (void*)&err, (void*)&bs};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_cpqr_big), dim3(nb), dim3(CB_NT), args,
                                    (unsigned int)lds, s);
}

int cpqr_max_coresident(size_t lds) {
  return coresident(reinterpret_cast<const void*>(&k_cpqr_multi), CQ_NT, lds);
}

hipError_t launch_cpqr_one(int32_t G, const SparsDesc* d, const SlabRef* slabs, int32_t nslab, const SegDesc* seg,
                           double eps, int32_t* cursize, int32_t* nref, int32_t* err, size_t lds, hipStream_t s) {
  if (nslab == 0) return hipSuccess;
  switch (G) {
#define ONE(GG) \
  case GG: hipLaunchKernelGGL(k_cpqr_one<GG>, dim3(nslab), dim3(CQ_NT), lds, s, d, slabs, seg, eps, cursize, nref, err); break;
    ONE(1) ONE(2) ONE(4) ONE(8) ONE(16) ONE(32) ONE(64)
#undef ONE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cpqr_multi(const SparsDesc* d, const SlabRef* slabs, int32_t nslab, int32_t nround,
                             const SegDesc* seg, double eps, int32_t* cursize, int32_t* nref, int32_t* err,
                             const int2* deps, int32_t* done, size_t lds, hipStream_t s) {
  if (nslab == 0 || nround == 0) return hipSuccess;
  void* args[] = {(void*)&d,   (void*)&slabs,   (void*)&nround, (void*)&seg,  (void*)&eps,
                  (void*)&cursize, (void*)&nref, (void*)&err,   (void*)&deps, (void*)&done};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_cpqr_multi), dim3(nslab), dim3(CQ_NT), args,
                                    (unsigned int)lds, s);
}

}  // namespace spand
