// Truncated column-pivoted QR of the interfaces (Sec. 2.6.1; ratio rule of Sec. 4
// intro), distributed over LDS-resident column slabs.
//
// Interface p couples its m dofs to ncols neighbour dofs through A_pn (m x ncols).
// Its columns are cut into S slabs of C columns; workgroup w holds slab w in LDS
// (row-major, m x C).  Step j of Householder QR with column pivoting:
//   1. every slab finds the largest exact norm of its remaining columns (rows
//      j..m-1, recomputed from the updated entries, never downdated) and, after a
//      barrier, the global largest;
//   2. each slab stages its first column within a relative 1e-10 of that maximum;
//      after a second barrier every workgroup takes the smallest such column index
//      as the pivot; stop when |R_jj| < eps |R_00|;
//   3. every workgroup forms the reflector from the staged pivot column (LAPACK
//      dlarfg convention, identical arithmetic everywhere) and applies it to its
//      own remaining columns.
// Interfaces too large for one LDS but moderate in size use one workgroup with the
// slab in a global workspace (no barriers).
// Columns are not swapped: a column pivoted at step j keeps R_0j..R_jj in rows
// 0..j of its slab.  With S > 1 the slabs exchange only their largest norm, their
// first candidate column and its entries.  At the end every slab writes W_cn = R[:r, :] P^T straight
// into the blocks of p, and workgroup 0 stores the reflectors, sets A_cc = I and
// publishes the rank.  With S = 1 the barriers reduce to __syncthreads.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace spand {

#define CW 256
#define TIE_RTOL 1e-10
#define SPIN_LIMIT (1L << 22)
#define T_MAX_R 4096

namespace {

__device__ inline double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wmax(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wmini(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// Barrier among the S workgroups of one interface: a monotone counter; barrier
// number b completes when the counter reaches b*S.  Bounded spin: on time-out the
// error flag is raised and the workgroup continues, so every wave terminates.
__device__ inline void slab_barrier(int32_t* cnt, int32_t target, int32_t* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(cnt, 1);
    long spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > SPIN_LIMIT) {
        atomicOr(err, 4);
        break;
      }
      // after any time-out every later barrier falls through at once
      if ((spins & 1023) == 0 && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4)) break;
    }
    __threadfence();
  }
  __syncthreads();
}

__device__ inline double shared_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

// Block reductions with four rotating LDS slots: one __syncthreads each.  A slot
// is reused only four reductions later, after at least three intervening barriers.
struct RedSlots {
  double d[4][CW / 64];
  int i[4][CW / 64];
};
__device__ inline double rmax(double v, RedSlots& rs, int& k) {
  v = wmax(v);
  double* r = rs.d[k & 3];
  ++k;
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = r[0];
  for (int q = 1; q < CW / 64; ++q) s = fmax(s, r[q]);
  return s;
}
__device__ inline double rsum(double v, RedSlots& rs, int& k) {
  v = wsum(v);
  double* r = rs.d[k & 3];
  ++k;
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < CW / 64; ++q) s += r[q];
  return s;
}
__device__ inline int rmini(int v, RedSlots& rs, int& k) {
  v = wmini(v);
  int* r = rs.i[k & 3];
  ++k;
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
  __syncthreads();
  int s = r[0];
  for (int q = 1; q < CW / 64; ++q) s = min(s, r[q]);
  return s;
}

template <bool GLOBAL>
__global__ void __launch_bounds__(CW) k_sparsify(const SparsDesc* __restrict__ descs, const SlabRef* __restrict__ slabs,
                                                 const SegDesc* __restrict__ segs, double eps, int32_t* cursize,
                                                 int32_t* nref, int32_t* err) {
  extern __shared__ double lds[];
  __shared__ RedSlots rs;
  __shared__ double redc[2][CW / 64][64];
  __shared__ double sh_pn;
  __shared__ int sh_piv, sh_owner;
  const SlabRef sr = slabs[blockIdx.x];
  const SparsDesc d = descs[sr.desc];
  const int m = d.m, S = d.S, C = d.C, w = sr.w;
  const int nseg = d.seg_end - d.seg_begin;
  const SegDesc* sg = segs + d.seg_begin;
  double* slab;  // m x C, row-major
  double* nrm;   // C: squared norms of the remaining columns (rows j..m-1)
  int* colstep;  // C: step at which a column was pivoted (-1 remaining, -2 absent)
  double* vbuf;  // m
  int* segoff;   // nseg + 1
  if (GLOBAL) {
    slab = d.ws;
    nrm = d.ws + (size_t)m * C;
    colstep = reinterpret_cast<int*>(nrm + C);
    vbuf = lds;
    segoff = reinterpret_cast<int*>(vbuf + m);
  } else {
    slab = lds;
    nrm = slab + (size_t)m * C;
    vbuf = nrm + C;
    colstep = reinterpret_cast<int*>(vbuf + m);
    segoff = colstep + C;
  }
  const int tid = threadIdx.x;
  int rk = 0;  // reduction slot counter
  // Slab exchange: three buffers of [S maxima | S candidate norms | S*m staged
  // columns] and S candidate indices.  Buffer (j & 1) serves step j (a slab can be
  // one step ahead of another, never two) and buffer 2 the near-tie second round.
  auto xbuf = [&](int b) { return d.xch + (size_t)b * S * (m + 2); };

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
  const int c0 = w * C;
  const int c1 = min(c0 + C, nc);
  const int nloc = max(0, c1 - c0);

  // gather this slab of A_pn
  for (int s = 0; s < nseg; ++s) {
    const int a = max(segoff[s], c0), b = min(segoff[s + 1], c1);
    if (a >= b) continue;
    const SegDesc g = sg[s];
    const int wdt = b - a;
    const int64_t cntE = (int64_t)m * wdt;
    for (int64_t e = tid; e < cntE; e += CW) {
      int r, cc;
      if (g.trans) { cc = (int)(e % wdt); r = (int)(e / wdt); } else { r = (int)(e % m); cc = (int)(e / m); }
      const int lcs = a + cc - segoff[s];
      const double v = g.trans ? g.blk[lcs + (int64_t)r * g.ld] : g.blk[r + (int64_t)lcs * g.ld];
      slab[(size_t)r * C + (a + cc - c0)] = v;
    }
  }
  if (GLOBAL) __threadfence_block();
  __syncthreads();
  for (int lc = tid; lc < C; lc += CW) {
    double s = -1.0;
    if (lc < nloc) {
      s = 0.0;
      for (int i = 0; i < m; ++i) {
        const double v = slab[(size_t)i * C + lc];
        s += v * v;
      }
    }
    nrm[lc] = s;
    colstep[lc] = (lc < nloc) ? -1 : -2;
  }
  if (GLOBAL) __threadfence_block();
  __syncthreads();
  const int kmax = min(m, nc);
  int r = kmax;
  double r00 = 0.0;
  int bar = 0;
  for (int j = 0; j < kmax; ++j) {
    // ---- pivot.  Rule: among all remaining columns whose norm is within TIE_RTOL of
    // the largest, the smallest column index.
    double lmax = 0.0;
    for (int lc = tid; lc < nloc; lc += CW)
      if (colstep[lc] == -1) lmax = fmax(lmax, sqrt(nrm[lc]));
    lmax = rmax(lmax, rs, rk);
    int lidx = 0x7fffffff;
    {
      const double lthr = lmax * (1.0 - TIE_RTOL);
      for (int lc = tid; lc < nloc; lc += CW)
        if (colstep[lc] == -1 && sqrt(nrm[lc]) >= lthr) { lidx = c0 + lc; break; }
    }
    int cand = rmini(lidx, rs, rk);
    int xb = 0;  // exchange buffer holding the pivot column
    if (S > 1) {
      // publish (slab max, first column within the window of the slab max, its
      // norm and entries); one barrier
      xb = j & 1;
      double* xmax = xbuf(xb);
      double* xnrm = xmax + S;
      double* xcol = xmax + 2 * S;
      int* xcand = d.xcand + (size_t)xb * S;
      if (cand < nc)
        for (int i = j + tid; i < m; i += CW) xcol[(size_t)w * m + i] = slab[(size_t)i * C + (cand - c0)];
      if (tid == 0) {
        xmax[w] = lmax;
        xcand[w] = cand;
        xnrm[w] = (cand < nc) ? sqrt(nrm[cand - c0]) : 0.0;
      }
      slab_barrier(d.cnt, ++bar * S, err);
      if (tid == 0) {
        double gmax = 0.0;
        for (int q = 0; q < S; ++q) gmax = fmax(gmax, shared_load(xmax + q));
        const double thr = gmax * (1.0 - TIE_RTOL);
        int best = 0x7fffffff, own = -1;
        bool ambiguous = false;
        for (int q = 0; q < S; ++q) {
          const int c = __hip_atomic_load(xcand + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (c >= nc) continue;
          if (shared_load(xnrm + q) >= thr) {
            if (c < best) { best = c; own = q; }
          } else if (shared_load(xmax + q) >= thr) {
            ambiguous = true;  // the slab's first column at the global threshold lies further on
          }
        }
        sh_piv = ambiguous ? -1 : best;
        sh_owner = own;
        sh_pn = ambiguous ? gmax : ((own >= 0) ? shared_load(xnrm + own) : 0.0);
      }
      __syncthreads();
      if (sh_piv == -1) {  // second round with the exact global threshold (near-ties across slabs)
        const double thr = sh_pn * (1.0 - TIE_RTOL);
        xb = 2;
        double* xnrm2 = xbuf(2) + S;
        double* xcol2 = xbuf(2) + 2 * S;
        int* xcand2 = d.xcand + 2 * (size_t)S;
        int l2 = 0x7fffffff;
        for (int lc = tid; lc < nloc; lc += CW)
          if (colstep[lc] == -1 && sqrt(nrm[lc]) >= thr) { l2 = c0 + lc; break; }
        const int c2 = rmini(l2, rs, rk);
        if (c2 < nc)
          for (int i = j + tid; i < m; i += CW) xcol2[(size_t)w * m + i] = slab[(size_t)i * C + (c2 - c0)];
        if (tid == 0) {
          xcand2[w] = c2;
          xnrm2[w] = (c2 < nc) ? sqrt(nrm[c2 - c0]) : 0.0;
        }
        slab_barrier(d.cnt, ++bar * S, err);
        if (tid == 0) {
          int best = 0x7fffffff, own = -1;
          for (int q = 0; q < S; ++q) {
            const int c = __hip_atomic_load(xcand2 + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (c < best) { best = c; own = q; }
          }
          sh_piv = best;
          sh_owner = own;
          sh_pn = (own >= 0 && best < nc) ? shared_load(xnrm2 + own) : 0.0;
        }
        __syncthreads();
      }
    } else {
      if (tid == 0) {
        sh_piv = cand;
        sh_owner = 0;
        sh_pn = (cand < nc) ? sqrt(nrm[cand - c0]) : 0.0;
      }
      __syncthreads();
    }
    const int piv = sh_piv, owner = sh_owner;
    if (piv >= nc) { r = j; break; }  // only non-finite norms left
    const double pn = sh_pn;
    if (j == 0) {
      r00 = pn;
      if (r00 == 0.0) { r = 0; break; }
    }
    if (pn < eps * r00) { r = j; break; }
    // ---- pivot column rows j..m-1 into vbuf; reflector (dlarfg convention)
    if (S > 1) {
      const double* xcol = xbuf(xb) + 2 * S;
      for (int i = j + tid; i < m; i += CW) vbuf[i] = shared_load(xcol + (size_t)owner * m + i);
    } else {
      for (int i = j + tid; i < m; i += CW) vbuf[i] = slab[(size_t)i * C + (piv - c0)];
    }
    __syncthreads();
    const double alpha = vbuf[j];
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += CW) part += vbuf[i] * vbuf[i];
    const double xn2 = rsum(part, rs, rk);
    double tau, scale, beta;
    if (xn2 == 0.0) {
      tau = 0.0; beta = alpha; scale = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();  // everyone has read vbuf[j] and the pivot column
    for (int i = j + 1 + tid; i < m; i += CW) vbuf[i] *= scale;
    if (tid == 0) vbuf[j] = 1.0;
    if (owner == w) {
      const int lc = piv - c0;
      for (int i = j + tid; i < m; i += CW) slab[(size_t)i * C + lc] = (i == j) ? beta : 0.0;
      if (tid == 0) {
        colstep[lc] = j;
        nrm[lc] = -1.0;
      }
    }
    if (GLOBAL) __threadfence_block();
    __syncthreads();
    if (w == 0) {
      double* V = d.V + (int64_t)j * m;
      for (int i = tid; i < m; i += CW) V[i] = (i < j) ? 0.0 : vbuf[i];
      if (tid == 0) d.tau[j] = tau;
    }
    // ---- apply H_j to the remaining columns of this slab; recompute their norms
    if (m <= 64) {  // short columns: one thread per column
      for (int lc = tid; lc < nloc; lc += CW) {
        if (colstep[lc] != -1) continue;
        double dot = slab[(size_t)j * C + lc];
        for (int i = j + 1; i < m; ++i) dot += vbuf[i] * slab[(size_t)i * C + lc];
        const double wv = tau * dot;
        slab[(size_t)j * C + lc] -= wv;
        double s = 0.0;
        for (int i = j + 1; i < m; ++i) {
          const double x = slab[(size_t)i * C + lc] - wv * vbuf[i];
          slab[(size_t)i * C + lc] = x;
          s += x * x;
        }
        nrm[lc] = s;
      }
    } else {  // tall columns: 64 columns per pass, the 4 waves split the rows
      const int lane = tid & 63, wv4 = tid >> 6;
      for (int t0 = 0; t0 < nloc; t0 += 64) {
        const int lc = t0 + lane;
        const bool act = lc < nloc && colstep[lc] == -1;
        double d0 = 0.0, d1 = 0.0;
        if (act) {
          int i = j + wv4;
          for (; i + 4 < m; i += 8) {
            d0 += vbuf[i] * slab[(size_t)i * C + lc];
            d1 += vbuf[i + 4] * slab[(size_t)(i + 4) * C + lc];
          }
          if (i < m) d0 += vbuf[i] * slab[(size_t)i * C + lc];
        }
        redc[0][wv4][lane] = d0 + d1;
        __syncthreads();
        const double wvv = tau * (redc[0][0][lane] + redc[0][1][lane] + redc[0][2][lane] + redc[0][3][lane]);
        double s0 = 0.0, s1 = 0.0;
        if (act) {
          int i = j + wv4;
          for (; i + 4 < m; i += 8) {
            const double x0 = slab[(size_t)i * C + lc] - wvv * vbuf[i];
            const double x1 = slab[(size_t)(i + 4) * C + lc] - wvv * vbuf[i + 4];
            slab[(size_t)i * C + lc] = x0;
            slab[(size_t)(i + 4) * C + lc] = x1;
            if (i > j) s0 += x0 * x0;
            s1 += x1 * x1;
          }
          if (i < m) {
            const double x0 = slab[(size_t)i * C + lc] - wvv * vbuf[i];
            slab[(size_t)i * C + lc] = x0;
            if (i > j) s0 += x0 * x0;
          }
        }
        redc[1][wv4][lane] = s0 + s1;
        __syncthreads();
        if (act && wv4 == 0) nrm[lc] = redc[1][0][lane] + redc[1][1][lane] + redc[1][2][lane] + redc[1][3][lane];
      }
    }
    if (GLOBAL) __threadfence_block();
    __syncthreads();
  }
  __syncthreads();
  // ---- W_cn = R[:r, :] (column order of A_pn) into the blocks of p
  for (int s = 0; s < nseg; ++s) {
    const int a = max(segoff[s], c0), b = min(segoff[s + 1], c1);
    if (a >= b || r == 0) continue;
    const SegDesc g = sg[s];
    const int wdt = b - a;
    const int64_t cntE = (int64_t)r * wdt;
    for (int64_t e = tid; e < cntE; e += CW) {
      int i, cc;
      if (g.trans) { cc = (int)(e % wdt); i = (int)(e / wdt); } else { i = (int)(e % r); cc = (int)(e / r); }
      const int lc = a + cc - c0;
      const int lcs = a + cc - segoff[s];
      const int cs = colstep[lc];
      const double v = (cs >= 0 && i > cs) ? 0.0 : slab[(size_t)i * C + lc];
      if (g.trans) g.blk[lcs + (int64_t)i * g.ld] = v;
      else g.blk[i + (int64_t)lcs * g.ld] = v;
    }
  }
  if (w == 0) {
    for (int64_t e = tid; e < (int64_t)r * r; e += CW) {
      const int a = (int)(e % r), b = (int)(e / r);
      d.diag[a + (int64_t)b * d.ldd] = (a == b) ? 1.0 : 0.0;
    }
    if (tid == 0) {
      cursize[d.id] = r;
      nref[d.id] = r;
    }
  }
}

// Compact WY factor of Q = H_0 ... H_{r-1} = I - V T V^T (T upper triangular):
// T_jj = tau_j, T[:j, j] = -tau_j T[:j, :j] (V[:, :j]^T v_j).  One workgroup per
// interface; the strict upper part of T first holds V^T V.
__global__ void __launch_bounds__(CW) k_build_t(const TDesc* __restrict__ descs) {
  const TDesc d = descs[blockIdx.x];
  const int m = d.m, r = d.r;
  __shared__ double y[T_MAX_R];
  const int64_t npair = (int64_t)r * (r - 1) / 2;
  for (int64_t q = threadIdx.x; q < npair; q += CW) {  // pair (i, j), i < j, packed by columns
    int j = (int)((1.0 + sqrt(1.0 + 8.0 * (double)q)) * 0.5);
    while ((int64_t)j * (j - 1) / 2 > q) --j;
    while ((int64_t)(j + 1) * j / 2 <= q) ++j;
    const int i = (int)(q - (int64_t)j * (j - 1) / 2);
    const double* vi = d.V + (int64_t)i * m;
    const double* vj = d.V + (int64_t)j * m;
    double s = vi[j];  // v_j[j] = 1
    for (int k = j + 1; k < m; ++k) s += vi[k] * vj[k];
    d.T[i + (int64_t)j * r] = s;
  }
  __threadfence_block();
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    const double tj = d.tau[j];
    // T[i][j] = -tau_j sum_{l=i}^{j-1} T[i][l] Y[l][j]; Y[:j, j] is staged in LDS
    // before column j is overwritten (r <= T_MAX_R, checked by the host)
    if (j > 0) {
      for (int i = threadIdx.x; i < j; i += CW) y[i] = d.T[i + (int64_t)j * r];
      __syncthreads();
      for (int i = threadIdx.x; i < j; i += CW) {
        double s = 0.0;
        for (int l = i; l < j; ++l) s += d.T[i + (int64_t)l * r] * y[l];
        d.T[i + (int64_t)j * r] = -tj * s;
      }
    }
    if (threadIdx.x == 0) d.T[j + (int64_t)j * r] = tj;
    __threadfence_block();
    __syncthreads();
  }
}

void launch_build_t(const TDesc* d, int32_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_build_t, dim3(count), dim3(CW), 0, s, d);
}

size_t sparsify_lds_bytes(int32_t m, int32_t C, int32_t nseg, bool global_slab) {
  if (global_slab) return size_t(m) * sizeof(double) + (size_t(nseg) + 1) * sizeof(int32_t) + 64;
  return (size_t(m) * C + C + m) * sizeof(double) + (size_t(C) + nseg + 1) * sizeof(int32_t) + 64;
}

size_t sparsify_lds_limit() { return 150 * 1024; }

namespace {
void set_lds_attr() {
  static bool done = false;
  if (done) return;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sparsify<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(sparsify_lds_limit()));
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sparsify<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(sparsify_lds_limit()));
  done = true;
}
}  // namespace

int sparsify_max_coresident(size_t lds_bytes) {
  set_lds_attr();
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sparsify<false>, CW, lds_bytes) != hipSuccess) return 0;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
}

hipError_t launch_sparsify(const SparsDesc* d, const SlabRef* slabs, int32_t nslab, const SegDesc* seg, double eps,
                           int32_t* cursize, int32_t* nref, int32_t* err, size_t lds_bytes, bool cooperative,
                           bool global_slab, hipStream_t s) {
  if (nslab == 0) return hipSuccess;
  set_lds_attr();
  if (global_slab) {
    hipLaunchKernelGGL(k_sparsify<true>, dim3(nslab), dim3(CW), lds_bytes, s, d, slabs, seg, eps, cursize, nref,
                       err);
    return hipGetLastError();
  }
  if (!cooperative) {
    hipLaunchKernelGGL(k_sparsify<false>, dim3(nslab), dim3(CW), lds_bytes, s, d, slabs, seg, eps, cursize, nref,
                       err);
    return hipGetLastError();
  }
  void* args[] = {(void*)&d, (void*)&slabs, (void*)&seg, (void*)&eps, (void*)&cursize, (void*)&nref, (void*)&err};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_sparsify<false>), dim3(nslab), dim3(CW), args,
                                    (unsigned int)lds_bytes, s);
}

}  // namespace spand
