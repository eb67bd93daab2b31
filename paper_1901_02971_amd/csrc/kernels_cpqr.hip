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
__device__ inline double bsum(double v, double* red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < CW / 64; ++q) s += red[q];
  return s;
}
__device__ inline double bmax(double v, double* red) {
  v = wmax(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
  for (int q = 1; q < CW / 64; ++q) s = fmax(s, red[q]);
  return s;
}
__device__ inline int bmini(int v, int* red) {
  v = wmini(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int s = red[0];
  for (int q = 1; q < CW / 64; ++q) s = min(s, red[q]);
  return s;
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

template <bool GLOBAL>
__global__ void __launch_bounds__(CW) k_sparsify(const SparsDesc* __restrict__ descs, const SlabRef* __restrict__ slabs,
                                                 const SegDesc* __restrict__ segs, double eps, int32_t* cursize,
                                                 int32_t* nref, int32_t* err) {
  extern __shared__ double lds[];
  __shared__ double red[CW / 64];
  __shared__ int redi[CW / 64];
  __shared__ double sh_beta, sh_tau, sh_scale, sh_pn;
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
  double* xmax = d.xch;           // S
  double* xnrm = d.xch + S;       // S
  double* xcol = d.xch + 2 * S;   // S * m

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
  const int kmax = min(m, nc);
  int r = kmax;
  double r00 = 0.0;
  int bar = 0;
  for (int j = 0; j < kmax; ++j) {
    __syncthreads();
    // ---- pivot: largest norm over all slabs, then the smallest column index within
    //      TIE_RTOL of it
    double lmax = 0.0;
    for (int lc = tid; lc < nloc; lc += CW)
      if (colstep[lc] == -1) lmax = fmax(lmax, sqrt(nrm[lc]));
    double gmax = bmax(lmax, red);
    if (S > 1) {
      if (tid == 0) xmax[w] = gmax;
      slab_barrier(d.cnt, ++bar * S, err);
      double g = 0.0;
      for (int q = tid; q < S; q += CW) g = fmax(g, shared_load(xmax + q));
      gmax = bmax(g, red);
    }
    const double thr = gmax * (1.0 - TIE_RTOL);
    int lidx = 0x7fffffff;
    for (int lc = tid; lc < nloc; lc += CW)
      if (colstep[lc] == -1 && sqrt(nrm[lc]) >= thr) { lidx = c0 + lc; break; }
    const int cand = bmini(lidx, redi);
    if (S > 1) {
      if (cand < nc) {  // stage this slab's candidate column
        for (int i = j + tid; i < m; i += CW) xcol[(size_t)w * m + i] = slab[(size_t)i * C + (cand - c0)];
        if (tid == 0) xnrm[w] = nrm[cand - c0];
      }
      if (tid == 0) d.xcand[w] = cand;
      slab_barrier(d.cnt, ++bar * S, err);
      if (tid == 0) {
        int best = 0x7fffffff, own = -1;
        for (int q = 0; q < S; ++q) {
          const int c = __hip_atomic_load(d.xcand + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (c < best) { best = c; own = q; }
        }
        sh_piv = best;
        sh_owner = own;
        sh_pn = (own >= 0 && best < nc) ? sqrt(shared_load(xnrm + own)) : 0.0;
      }
      __syncthreads();
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
    // ---- pivot column rows j..m-1 into vbuf
    if (S > 1) {
      for (int i = j + tid; i < m; i += CW) vbuf[i] = shared_load(xcol + (size_t)owner * m + i);
    } else {
      for (int i = j + tid; i < m; i += CW) vbuf[i] = slab[(size_t)i * C + (piv - c0)];
    }
    __syncthreads();
    // ---- reflector (dlarfg convention)
    const double alpha = vbuf[j];
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += CW) part += vbuf[i] * vbuf[i];
    const double xn2 = bsum(part, red);
    if (tid == 0) {
      if (xn2 == 0.0) {
        sh_tau = 0.0; sh_beta = alpha; sh_scale = 0.0;
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        sh_tau = (beta - alpha) / beta;
        sh_beta = beta;
        sh_scale = 1.0 / (alpha - beta);
      }
    }
    __syncthreads();
    const double tau = sh_tau, scale = sh_scale;
    for (int i = j + 1 + tid; i < m; i += CW) vbuf[i] *= scale;
    if (tid == 0) vbuf[j] = 1.0;
    __syncthreads();
    if (w == 0) {
      double* V = d.V + (int64_t)j * m;
      for (int i = tid; i < m; i += CW) V[i] = (i < j) ? 0.0 : vbuf[i];
      if (tid == 0) d.tau[j] = tau;
    }
    if (owner == w) {
      const int lc = piv - c0;
      for (int i = j + tid; i < m; i += CW) slab[(size_t)i * C + lc] = (i == j) ? sh_beta : 0.0;
      if (tid == 0) {
        colstep[lc] = j;
        nrm[lc] = -1.0;
      }
    }
    if (GLOBAL) __threadfence_block();
    __syncthreads();
    // ---- apply H_j to the remaining columns of this slab; recompute their norms
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
    if (GLOBAL) __threadfence_block();
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
