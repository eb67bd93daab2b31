// Truncated column-pivoted QR of the interfaces (Sec. 2.6.1; ratio rule of Sec. 4
// intro) with the block A_pn held in registers.
//
// Interface p couples its m dofs to nc neighbour dofs through A_pn (m x nc).  A
// workgroup of NT = 512 threads (two waves per SIMD, so the whole register file of
// a CU) holds a slab of CAP = CQ_CPL * NT / G columns: a team of G consecutive
// lanes (G a power of two, G * CQ_MR >= m) owns CQ_CPL columns, and lane g of the
// team keeps rows i = q * G + g (q < CQ_MR) of each of them in registers.  Column c
// of A_pn lives in slab c / CAP, team (c % CAP) % (NT / G), register slot
// (c % CAP) / (NT / G).  Interface p uses S = ceil(nc / CAP) slabs.
//
// Step j of Householder QR with column pivoting:
//   1. every column knows the exact norm of its rows j..m-1 (recomputed from the
//      updated entries at the end of the previous step, never downdated);
//   2. pivot = among the remaining columns whose norm is within a relative 1e-10 of
//      the largest, the smallest column index.  One fused reduction carries
//      (largest norm, smallest index within the window of that partial maximum,
//      its norm) through the lanes, the waves and, for S > 1, the slabs; when a
//      partial maximum grows past a side's own window the exact index is found in
//      a second round.  Stop when |R_jj| < eps |R_00|;
//   3. the team owning the pivot column publishes its rows j..m-1 (LDS for S = 1,
//      the slab exchange buffer for S > 1, one slab barrier per step) and every
//      lane forms the reflector (LAPACK dlarfg convention) from it with identical
//      arithmetic;
//   4. every remaining column is updated in registers, a <- a - tau v (v^T a), and
//      its new trailing norm formed (team sums by lane shuffles).
// Columns are never moved: a column pivoted at step j keeps R_0j..R_jj in its rows
// 0..j.  At the end every slab writes W_cn = R[:r, :] P^T straight into the blocks of
// p, and slab 0 stores the reflectors, sets A_cc = I and publishes the rank.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "kernels.h"

namespace spand {

#define CQ_NT 512
#define CQ_MR 32
#define CQ_CPL 2
#define CW 256  // threads of k_build_t
#define TIE_RTOL 1e-10
#define SPIN_LIMIT (1L << 22)

namespace {

// Pivot candidate of a set of columns: the largest norm mx, the smallest column
// index cd among the columns with norm >= mx (1 - TIE_RTOL), its norm cn, and amb
// set when the exact smallest index at a larger threshold is not known.
struct Cand {
  double mx, cn;
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
  if (oka) {
    o.cd = a.cd;
    o.cn = a.cn;
  }
  if (okb && b.cd < o.cd) {
    o.cd = b.cd;
    o.cn = b.cn;
  }
  return o;
}

template <int G>
__device__ inline double team_sum(double v) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline int wave_min(int v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// Barrier among the S workgroups of one interface: a monotone counter; barrier
// number b completes when the counter reaches b*S.  Everything the slabs exchange
// is written and read with agent-scope atomic accesses, which are coherent across
// the L2 caches of the XCDs; each wave waits for its own stores to complete before
// the counter is raised, so no L2 writeback or invalidation is needed.  Bounded
// spin: on time-out the error flag is raised and the workgroup continues, so every
// wave terminates.
__device__ inline void slab_barrier(int32_t* cnt, int32_t target, int32_t* err) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's exchange stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SPIN_LIMIT) {
        atomicOr(err, 4);
        break;
      }
      // after any time-out every later barrier falls through at once
      if ((spins & 1023) == 0 && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4)) break;
    }
  }
  __syncthreads();
}

__device__ inline double shared_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void shared_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Slab w of interface d (w = 0, S = 1 when MULTI is false).
template <int G, bool MULTI>
__device__ __forceinline__ void cpqr_slab(const SparsDesc& d, int wslab, const SegDesc* __restrict__ segs, double eps,
                                          int32_t* cursize, int32_t* nref, int32_t* err) {
  constexpr int NT = CQ_NT;
  constexpr int NTEAM = NT / G;
  constexpr int CAP = CQ_CPL * NTEAM;
  constexpr int NW = NT / 64;
  constexpr int ROWS = G * CQ_MR;  // rows a team can hold (>= m)
  extern __shared__ double lds[];
  __shared__ Cand red[2][NW], redx[2][NW];
  __shared__ int red2[NW];
  __shared__ double sh_pn, sh_tau;
  const int m = d.m, S = MULTI ? d.S : 1, w = MULTI ? wslab : 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane & (G - 1), team = tid / G;
  const int nseg = d.seg_end - d.seg_begin;
  const SegDesc* sg = segs + d.seg_begin;
  // vm[i] = (v_i, [i > j]): the reflector of the current step, v_i = 0 above row j,
  // v_j = 1, zero below row m; the flag selects the rows of the trailing norms
  double2* vm = reinterpret_cast<double2*>(lds);
  int* segoff = reinterpret_cast<int*>(lds + 2 * ROWS);  // nseg + 1
  // exchange record of slab q in buffer b: [max, cand norm, cand xn2, cand index, ROWS column rows]
  auto xrec = [&](int b, int q) { return d.xch + ((size_t)b * S + q) * (size_t)(ROWS + 4); };

  // column layout of A_pn from the neighbours' current sizes
  if (tid == 0) {
    int off = 0;
    for (int s = 0; s < nseg; ++s) {
      segoff[s] = off;
      off += cursize[sg[s].q];
    }
    segoff[nseg] = off;
  }
  __syncthreads();
  const int nc = segoff[nseg];
  if (nc == 0) {  // no coupled dofs left: p keeps its size, no reflectors
    if (w == 0 && tid == 0) nref[d.id] = 0;
    return;
  }

  double a[CQ_CPL][CQ_MR];
  double nrm[CQ_CPL];  // squared norm of rows j..m-1 (identical in the lanes of a team)
  int col[CQ_CPL];     // column index in A_pn, -1 if the slot is empty
  int pst[CQ_CPL];     // -1 remaining, >= 0 step at which the column was the pivot, -2 empty
#pragma unroll
  for (int k = 0; k < CQ_CPL; ++k) {
    const int c = w * CAP + k * NTEAM + team;
    col[k] = c < nc ? c : -1;
    pst[k] = c < nc ? -1 : -2;
    double* base = nullptr;
    int64_t stride = 0;
    if (c < nc) column_ptr(sg, segoff, c, base, stride);
    const int rows = (c < nc) ? m : 0;
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < CQ_MR; ++q) {
      const int i = q * G + g;
      const double v = (i < rows) ? base[(int64_t)i * stride] : 0.0;
      a[k][q] = v;
      sq = fma(v, v, sq);
    }
    nrm[k] = team_sum<G>(sq);
  }

  const int kmax = min(m, nc);
  int r = kmax;
  double r00 = 0.0;
  int bar = 0;
  for (int j = 0; j < kmax; ++j) {
    // ---- pivot candidate of this lane, then of the wave and the workgroup
    double nv[CQ_CPL];
    Cand t;
    t.mx = -1.0;
#pragma unroll
    for (int k = 0; k < CQ_CPL; ++k) {
      nv[k] = (pst[k] == -1) ? sqrt(nrm[k]) : -1.0;
      t.mx = fmax(t.mx, nv[k]);
    }
    t.cd = INT_MAX;
    t.cn = -1.0;
    t.amb = 0;
    {
      const double thr = t.mx * (1.0 - TIE_RTOL);
#pragma unroll
      for (int k = 0; k < CQ_CPL; ++k)
        if (pst[k] == -1 && nv[k] >= thr && col[k] < t.cd) {
          t.cd = col[k];
          t.cn = nv[k];
        }
    }
#pragma unroll
    for (int o = G; o < 64; o <<= 1) {
      Cand u;
      u.mx = __shfl_xor(t.mx, o, 64);
      u.cn = __shfl_xor(t.cn, o, 64);
      u.cd = __shfl_xor(t.cd, o, 64);
      u.amb = __shfl_xor(t.amb, o, 64);
      t = cand_combine(t, u);
    }
    if (lane == 0) red[j & 1][wave] = t;
    __syncthreads();
    Cand wg = red[j & 1][0];
#pragma unroll
    for (int q = 1; q < NW; ++q) wg = cand_combine(wg, red[j & 1][q]);
    if (wg.amb) {  // exact smallest index at the workgroup's threshold
      const double thr = wg.mx * (1.0 - TIE_RTOL);
      int c2 = INT_MAX;
#pragma unroll
      for (int k = 0; k < CQ_CPL; ++k)
        if (pst[k] == -1 && nv[k] >= thr) c2 = min(c2, col[k]);
      c2 = wave_min(c2);
      if (lane == 0) red2[wave] = c2;
      __syncthreads();
      int best = red2[0];
#pragma unroll
      for (int q = 1; q < NW; ++q) best = min(best, red2[q]);
      __syncthreads();  // red2 is rewritten by its next use
      wg.cd = best;
    }
    if (!MULTI && wg.cd == INT_MAX) {  // only non-finite norms left
      r = j;
      break;
    }
    // team and register slot of this slab's candidate
    const int lc = wg.cd - w * CAP;
    const bool own = wg.cd != INT_MAX && team == lc % NTEAM;
    const int pk = own ? lc / NTEAM : 0;
    int piv;
    if constexpr (!MULTI) {
      // the owner team forms the reflector from its column and publishes it
      if (own) {
#pragma unroll
        for (int k = 0; k < CQ_CPL; ++k)
          if (k == pk) {
            double x2 = 0.0, al = 0.0;
#pragma unroll
            for (int q = 0; q < CQ_MR; ++q) {
              const int jq = j - q * G;
              x2 = (g > jq) ? fma(a[k][q], a[k][q], x2) : x2;
              al = (g == jq) ? a[k][q] : al;
            }
            x2 = team_sum<G>(x2);
            const double alpha = team_sum<G>(al);  // one lane holds row j, the others add 0
            const double pn = nv[k];
            const double r0 = (j == 0) ? pn : r00;
            const bool stop = (r0 == 0.0) || (pn < eps * r0);
            double tau = 0.0, scale = 0.0, beta = alpha;
            if (x2 != 0.0) {
              beta = -copysign(sqrt(alpha * alpha + x2), alpha);
              tau = (beta - alpha) / beta;
              scale = 1.0 / (alpha - beta);
            }
            if (!stop) {
#pragma unroll
              for (int q = 0; q < CQ_MR; ++q) {
                const int jq = j - q * G;
                const double x = a[k][q];
                vm[q * G + g] = make_double2((g > jq) ? x * scale : ((g == jq) ? 1.0 : 0.0), (g > jq) ? 1.0 : 0.0);
                a[k][q] = (g == jq) ? beta : ((g > jq) ? 0.0 : x);  // column j of R
              }
              pst[k] = j;
            }
            if (g == 0) {
              sh_pn = pn;
              sh_tau = tau;
            }
          }
      }
      __syncthreads();
      piv = wg.cd;
    } else {
      // publish (slab max, slab candidate, its norm, its rows); one barrier
      {
        double* rc = xrec(j & 1, w);
        if (own) {
#pragma unroll
          for (int k = 0; k < CQ_CPL; ++k)
            if (k == pk) {
              double x2 = 0.0;
#pragma unroll
              for (int q = 0; q < CQ_MR; ++q) {
                shared_store(rc + 4 + q * G + g, a[k][q]);
                x2 = (g > j - q * G) ? fma(a[k][q], a[k][q], x2) : x2;
              }
              x2 = team_sum<G>(x2);
              if (g == 0) {
                shared_store(rc + 1, nv[k]);
                shared_store(rc + 2, x2);
              }
            }
        }
        if (tid == 0) {
          shared_store(rc, wg.mx);
          shared_store(rc + 3, (wg.cd == INT_MAX) ? -1.0 : (double)wg.cd);
          if (wg.cd == INT_MAX) shared_store(rc + 1, -1.0);
        }
      }
      int xb = j & 1;
      slab_barrier(d.cnt, ++bar * S, err);
      // the S records are read in parallel (one memory round trip) and reduced like
      // the lanes; the owning slab of column c is c / CAP
      Cand u;
      u.mx = -1.0;
      u.cn = -1.0;
      u.cd = INT_MAX;
      u.amb = 0;
      for (int q = tid; q < S; q += NT) {  // S may exceed the workgroup size
        const double* rc = xrec(xb, q);
        const double mx = shared_load(rc), cn = shared_load(rc + 1), cq = shared_load(rc + 3);
        Cand v;
        v.mx = mx;
        v.cn = (cq >= 0.0) ? cn : -1.0;
        v.cd = (cq >= 0.0) ? (int)cq : INT_MAX;
        v.amb = 0;
        u = cand_combine(u, v);
      }
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        Cand v;
        v.mx = __shfl_xor(u.mx, o, 64);
        v.cn = __shfl_xor(u.cn, o, 64);
        v.cd = __shfl_xor(u.cd, o, 64);
        v.amb = __shfl_xor(u.amb, o, 64);
        u = cand_combine(u, v);
      }
      if (lane == 0) redx[j & 1][wave] = u;
      __syncthreads();
      Cand gc = redx[j & 1][0];
#pragma unroll
      for (int q = 1; q < NW; ++q) gc = cand_combine(gc, redx[j & 1][q]);
      piv = gc.cd;
      if (gc.amb) {  // second round with the exact global threshold (near-ties across slabs)
        xb = 2;
        const double thr = gc.mx * (1.0 - TIE_RTOL);
        int c2 = INT_MAX;
#pragma unroll
        for (int k = 0; k < CQ_CPL; ++k)
          if (pst[k] == -1 && nv[k] >= thr) c2 = min(c2, col[k]);
        c2 = wave_min(c2);
        if (lane == 0) red2[wave] = c2;
        __syncthreads();
        int best = red2[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) best = min(best, red2[q]);
        const int lc2 = best - w * CAP;
        double* rc = xrec(2, w);
        if (best != INT_MAX && team == lc2 % NTEAM) {
          const int pk2 = lc2 / NTEAM;
#pragma unroll
          for (int k = 0; k < CQ_CPL; ++k)
            if (k == pk2) {
              double x2 = 0.0;
#pragma unroll
              for (int q = 0; q < CQ_MR; ++q) {
                shared_store(rc + 4 + q * G + g, a[k][q]);
                x2 = (g > j - q * G) ? fma(a[k][q], a[k][q], x2) : x2;
              }
              x2 = team_sum<G>(x2);
              if (g == 0) {
                shared_store(rc + 1, nv[k]);
                shared_store(rc + 2, x2);
              }
            }
        }
        if (tid == 0) shared_store(rc + 3, (best == INT_MAX) ? -1.0 : (double)best);
        slab_barrier(d.cnt, ++bar * S, err);
        int b2 = INT_MAX;
        for (int q = tid; q < S; q += NT) {
          const double cq = shared_load(xrec(2, q) + 3);
          if (cq >= 0.0) b2 = min(b2, (int)cq);
        }
        b2 = wave_min(b2);
        if (lane == 0) red2[wave] = b2;
        __syncthreads();
        piv = red2[0];
#pragma unroll
        for (int q = 1; q < NW; ++q) piv = min(piv, red2[q]);
        __syncthreads();  // red2 is rewritten by its next use
      }
      if (piv == INT_MAX) {  // only non-finite norms left
        r = j;
        break;
      }
      // every thread forms the reflector from the winning record (identical arithmetic)
      const double* rc = xrec(xb, piv / CAP);
      const double pn = shared_load(rc + 1);
      const double x2 = shared_load(rc + 2);
      const double alpha = shared_load(rc + 4 + j);
      const double r0 = (j == 0) ? pn : r00;
      const bool stop = (r0 == 0.0) || (pn < eps * r0);
      double tau = 0.0, scale = 0.0, beta = alpha;
      if (x2 != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + x2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      if (!stop) {
        for (int i = tid; i < ROWS; i += NT) {
          const double x = (i > j) ? shared_load(rc + 4 + i) : 0.0;
          vm[i] = make_double2((i > j) ? x * scale : ((i == j) ? 1.0 : 0.0), (i > j) ? 1.0 : 0.0);
        }
        const int plc = piv - w * CAP;
        if (plc >= 0 && plc < CAP && team == plc % NTEAM) {
          const int ppk = plc / NTEAM;
#pragma unroll
          for (int k = 0; k < CQ_CPL; ++k)
            if (k == ppk) {
#pragma unroll
              for (int q = 0; q < CQ_MR; ++q) {
                const int jq = j - q * G;
                a[k][q] = (g == jq) ? beta : ((g > jq) ? 0.0 : a[k][q]);  // column j of R
              }
              pst[k] = j;
            }
        }
      }
      if (tid == 0) {
        sh_pn = pn;
        sh_tau = tau;
      }
      __syncthreads();
    }
    const double pn = sh_pn;
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
    const double tau = sh_tau;
    if (w == 0) {
      double* V = d.V + (int64_t)j * m;
      for (int i = tid; i < m; i += NT) V[i] = vm[i].x;
      if (tid == 0) d.tau[j] = tau;
    }
    // ---- apply H_j to the remaining columns; new trailing norms (rows j+1..).  The
    // (v_i, [i > j]) pairs are read four rows ahead of their use (two passes).
    const double2* vl = vm + g;
    double dot[CQ_CPL];
#pragma unroll
    for (int k = 0; k < CQ_CPL; ++k) dot[k] = 0.0;
    {
      double2 cur[4], nxt[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cur[u] = vl[u * G];
#pragma unroll
      for (int q0 = 0; q0 < CQ_MR; q0 += 4) {
        if (q0 + 4 < CQ_MR) {
#pragma unroll
          for (int u = 0; u < 4; ++u) nxt[u] = vl[(q0 + 4 + u) * G];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < CQ_CPL; ++k) dot[k] = fma(cur[u].x, a[k][q0 + u], dot[k]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) cur[u] = nxt[u];
      }
    }
    double wv[CQ_CPL], sq[CQ_CPL];
#pragma unroll
    for (int k = 0; k < CQ_CPL; ++k) {
      dot[k] = team_sum<G>(dot[k]);
      wv[k] = (pst[k] == -1) ? tau * dot[k] : 0.0;
      sq[k] = 0.0;
    }
    {
      double2 cur[4], nxt[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cur[u] = vl[u * G];
#pragma unroll
      for (int q0 = 0; q0 < CQ_MR; q0 += 4) {
        if (q0 + 4 < CQ_MR) {
#pragma unroll
          for (int u = 0; u < 4; ++u) nxt[u] = vl[(q0 + 4 + u) * G];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < CQ_CPL; ++k) {
            const double x = fma(-wv[k], cur[u].x, a[k][q0 + u]);
            a[k][q0 + u] = x;
            sq[k] = fma(x * cur[u].y, x, sq[k]);
          }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) cur[u] = nxt[u];
      }
    }
#pragma unroll
    for (int k = 0; k < CQ_CPL; ++k) nrm[k] = team_sum<G>(sq[k]);
  }
  // ---- W_cn = R[:r, :] (column order of A_pn) into the blocks of p
#pragma unroll
  for (int k = 0; k < CQ_CPL; ++k) {
    if (col[k] < 0 || r == 0) continue;
    double* base;
    int64_t stride;
    column_ptr(sg, segoff, col[k], base, stride);
#pragma unroll
    for (int q = 0; q < CQ_MR; ++q) {
      const int i = q * G + g;
      if (i < r) base[(int64_t)i * stride] = a[k][q];
    }
  }
  if (w == 0) {
    for (int64_t e = tid; e < (int64_t)r * r; e += NT) {
      const int x = (int)(e % r), y = (int)(e / r);
      d.diag[x + (int64_t)y * d.ldd] = (x == y) ? 1.0 : 0.0;
    }
    if (tid == 0) {
      cursize[d.id] = r;
      nref[d.id] = r;
    }
  }
}

// Single-slab interfaces: one launch per team size.
template <int G>
__global__ void __launch_bounds__(CQ_NT) k_cpqr_one(const SparsDesc* __restrict__ descs,
                                                    const SlabRef* __restrict__ slabs,
                                                    const SegDesc* __restrict__ segs, double eps, int32_t* cursize,
                                                    int32_t* nref, int32_t* err) {
  const SlabRef sr = slabs[blockIdx.x];
  cpqr_slab<G, false>(descs[sr.desc], 0, segs, eps, cursize, nref, err);
}

// Multi-slab interfaces of every team size in one cooperative launch: each
// workgroup takes the code path of its interface's G.
__global__ void __launch_bounds__(CQ_NT) k_cpqr_multi(const SparsDesc* __restrict__ descs,
                                                      const SlabRef* __restrict__ slabs,
                                                      const SegDesc* __restrict__ segs, double eps,
                                                      int32_t* cursize, int32_t* nref, int32_t* err) {
  const SlabRef sr = slabs[blockIdx.x];
  const SparsDesc d = descs[sr.desc];
  switch (d.G) {
    case 1: cpqr_slab<1, true>(d, sr.w, segs, eps, cursize, nref, err); break;
    case 2: cpqr_slab<2, true>(d, sr.w, segs, eps, cursize, nref, err); break;
    case 4: cpqr_slab<4, true>(d, sr.w, segs, eps, cursize, nref, err); break;
    case 8: cpqr_slab<8, true>(d, sr.w, segs, eps, cursize, nref, err); break;
    case 16: cpqr_slab<16, true>(d, sr.w, segs, eps, cursize, nref, err); break;
    case 32: cpqr_slab<32, true>(d, sr.w, segs, eps, cursize, nref, err); break;
    case 64: cpqr_slab<64, true>(d, sr.w, segs, eps, cursize, nref, err); break;
    default: break;  // the host only builds the team sizes above
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
  __shared__ double tl[64 * 65];
  const int below = r - j0;
  for (int q = threadIdx.x; q < below * w; q += CW) {  // zeros under the diagonal of this block column
    const int i = j0 + q % below, j = j0 + q / below;
    if (i > j) b.T[i + (int64_t)j * r] = 0.0;
  }
  for (int q = threadIdx.x; q < w * w; q += CW) {
    const int i = q % w, j = q / w;
    tl[i + j * 65] = (i < j) ? b.T[(j0 + i) + (int64_t)(j0 + j) * r] : 0.0;
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
    if (ii <= jj) b.T[(j0 + ii) + (int64_t)(j0 + jj) * r] = tl[ii + jj * 65];
  }
}

void launch_build_t_diag(const TBlock* blocks, int32_t count, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_build_t_diag, dim3(count), dim3(CW), 0, s, blocks);
}

int32_t cpqr_team(int32_t m) {
  int32_t G = 1;
  while (G * CQ_MR < m) G <<= 1;
  return G <= 64 ? G : -1;
}

int32_t cpqr_capacity(int32_t G) { return CQ_CPL * CQ_NT / G; }

size_t cpqr_lds_bytes(int32_t G, int32_t nseg) {
  return 2 * size_t(G) * CQ_MR * sizeof(double) + (size_t(nseg) + 1) * sizeof(int32_t) + 16;
}

int32_t cpqr_record(int32_t G) { return G * CQ_MR + 4; }

int cpqr_max_coresident(size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cpqr_multi, CQ_NT, lds) != hipSuccess) return 0;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
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

hipError_t launch_cpqr_multi(const SparsDesc* d, const SlabRef* slabs, int32_t nslab, const SegDesc* seg, double eps,
                             int32_t* cursize, int32_t* nref, int32_t* err, size_t lds, hipStream_t s) {
  if (nslab == 0) return hipSuccess;
  void* args[] = {(void*)&d, (void*)&slabs, (void*)&seg, (void*)&eps, (void*)&cursize, (void*)&nref, (void*)&err};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_cpqr_multi), dim3(nslab), dim3(CQ_NT), args,
                                    (unsigned int)lds, s);
}

}  // namespace spand
