// Preconditioner apply z = F^T F r (F = M^T, Sec. 2.8) and the FP64 PCG vector
// kernels.  Vectors are n x nrhs column-major (FP64); the dofs of a cluster are
// addressed through its slot list (vertex ids of the dofs it currently carries).
//
// Forward sweep of one step (levels L -> 1):
//   k_elim_fwd    x_s <- L_s^{-1} x_s            (one workgroup per eliminated s;
//                                                  blocked substitution with the
//                                                  inverses of the diagonal blocks)
//   k_target_fwd  x_n <- x_n - sum_s G_ns x_s     (one workgroup per receiving n,
//                                                  contributions in ascending s)
//   k_scale_fwd   x_p <- L_p^{-1} x_p
//   k_house_fwd   x_p <- Q_p^T x_p                (reflectors in increasing order)
// Backward sweep (levels 1 -> L), the transposes in reverse order:
//   k_house_bwd   x_p <- Q_p x_p
//   k_scale_bwd   x_p <- L_p^{-T} x_p
//   k_gather      neighbour dofs of every s into a contiguous buffer
//   k_elim_bwd    x_s <- L_s^{-T} (x_s - G_{N_s s}^T x_{N_s})
#include <hip/hip_runtime.h>

#include "apply.h"
#include "kernels.h"

namespace spand {

#define AW 256
#define RB 8  // right-hand sides per register pass

__device__ inline double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Blocked triangular solves on a vector segment v (n rows, nr <= RB columns, ld ldv)
// held in the apply scratch.  L is lower triangular (ld), its CHOL_NB-wide diagonal
// blocks have the inverses Dinv (block k at k*CHOL_NB^2, ld = block width).
struct TrsvShared {
  double part[AW / 64][CHOL_NB][RB];
  double tb[CHOL_NB][RB];
};

// L y = v, in place: y_k = D_k^{-1} (v_k - sum_{l<k} L_kl y_l)
__device__ void trsv_fwd(const double* __restrict__ L, int ld, const double* __restrict__ Dinv, int n, double* v,
                         int64_t ldv, int nr, TrsvShared& sh) {
  const int rr = threadIdx.x & 63, g = threadIdx.x >> 6;
  for (int kb = 0; kb < n; kb += CHOL_NB) {
    const int w = min(CHOL_NB, n - kb);
    double acc[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) acc[c] = 0.0;
    if (rr < w) {
      const double* Lr = L + kb + rr;
      for (int k = g; k < kb; k += AW / 64) {
        const double l = Lr[(int64_t)k * ld];
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (c < nr) acc[c] += l * v[k + (int64_t)c * ldv];
      }
    }
#pragma unroll
    for (int c = 0; c < RB; ++c) sh.part[g][rr][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < w) {
      const int i = threadIdx.x;
#pragma unroll
      for (int c = 0; c < RB; ++c)
        if (c < nr)
          sh.tb[i][c] = v[kb + i + (int64_t)c * ldv] - (sh.part[0][i][c] + sh.part[1][i][c] + sh.part[2][i][c] +
                                                       sh.part[3][i][c]);
    }
    __syncthreads();
    if (threadIdx.x < w) {
      const int i = threadIdx.x;
      const double* Dk = Dinv + (int64_t)(kb / CHOL_NB) * CHOL_NB * CHOL_NB;
      double y[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) y[c] = 0.0;
      for (int k = 0; k <= i; ++k) {
        const double dv = Dk[i + k * w];
#pragma unroll
        for (int c = 0; c < RB; ++c) y[c] += dv * sh.tb[k][c];
      }
#pragma unroll
      for (int c = 0; c < RB; ++c)
        if (c < nr) v[kb + i + (int64_t)c * ldv] = y[c];
    }
    __threadfence_block();
    __syncthreads();
  }
}

// L^T x = v, in place: x_k = D_k^{-T} (v_k - sum_{l>k} L_lk^T x_l)
__device__ void trsv_bwd(const double* __restrict__ L, int ld, const double* __restrict__ Dinv, int n, double* v,
                         int64_t ldv, int nr, TrsvShared& sh) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nblk = (n + CHOL_NB - 1) / CHOL_NB;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int kb = bi * CHOL_NB;
    const int w = min(CHOL_NB, n - kb);
    for (int cc = wave; cc < w; cc += AW / 64) {
      double acc[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) acc[c] = 0.0;
      const double* Lc = L + (int64_t)(kb + cc) * ld;
      for (int r = kb + w + lane; r < n; r += 64) {
        const double l = Lc[r];
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (c < nr) acc[c] += l * v[r + (int64_t)c * ldv];
      }
#pragma unroll
      for (int c = 0; c < RB; ++c) {
        const double sum = wsum(acc[c]);
        if (lane == 0 && c < nr) sh.tb[cc][c] = v[kb + cc + (int64_t)c * ldv] - sum;
      }
    }
    __syncthreads();
    if (threadIdx.x < w) {
      const int i = threadIdx.x;
      const double* Dk = Dinv + (int64_t)bi * CHOL_NB * CHOL_NB;
      double x[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) x[c] = 0.0;
      for (int q = i; q < w; ++q) {
        const double dv = Dk[q + i * w];
#pragma unroll
        for (int c = 0; c < RB; ++c) x[c] += dv * sh.tb[q][c];
      }
#pragma unroll
      for (int c = 0; c < RB; ++c)
        if (c < nr) v[kb + i + (int64_t)c * ldv] = x[c];
    }
    __threadfence_block();
    __syncthreads();
  }
}

__device__ inline void gather_seg(const int32_t* sl, int n, const ApplyArgs& a, int64_t off) {
  for (int c = 0; c < a.nrhs; ++c)
    for (int r = threadIdx.x; r < n; r += AW) a.tmp[off + r + (int64_t)c * a.ldt] = a.x[sl[r] + (int64_t)c * a.ldx];
  __threadfence_block();
  __syncthreads();
}
__device__ inline void scatter_seg(const int32_t* sl, int n, const ApplyArgs& a, int64_t off) {
  for (int c = 0; c < a.nrhs; ++c)
    for (int r = threadIdx.x; r < n; r += AW) a.x[sl[r] + (int64_t)c * a.ldx] = a.tmp[off + r + (int64_t)c * a.ldt];
}

// y_s = L_s^{-1} x_s; y_s stays in the scratch for the target updates and replaces x_s.
__global__ void __launch_bounds__(AW) k_elim_fwd(const ElimAp* __restrict__ ds, ApplyArgs a) {
  __shared__ TrsvShared sh;
  const ElimAp e = ds[blockIdx.x];
  const int32_t* sl = a.slot + e.slot_s;
  gather_seg(sl, e.ns, a, e.tmp);
  for (int c0 = 0; c0 < a.nrhs; c0 += RB)
    trsv_fwd(e.L, e.ld, e.Dinv, e.ns, a.tmp + e.tmp + (int64_t)c0 * a.ldt, a.ldt, min(RB, a.nrhs - c0), sh);
  scatter_seg(sl, e.ns, a, e.tmp);
}

__global__ void __launch_bounds__(AW) k_target_fwd(const TargetAp* __restrict__ ts, const TargetContrib* __restrict__ cs,
                                                   ApplyArgs a) {
  const TargetAp t = ts[blockIdx.x];
  const int32_t* sl = a.slot + t.slot_n;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    for (int r = threadIdx.x; r < t.nn; r += AW) {
      double acc[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) acc[c] = 0.0;
      for (int q = t.cbeg; q < t.cend; ++q) {
        const TargetContrib tc = cs[q];
        const double* y = a.tmp + tc.tmp_s + (int64_t)c0 * a.ldt;
        for (int k = 0; k < tc.ns; ++k) {
          const double g = tc.G[r + (int64_t)k * tc.ldG];
#pragma unroll
          for (int c = 0; c < RB; ++c)
            if (c < nr) acc[c] += g * y[k + (int64_t)c * a.ldt];
        }
      }
      double* xp = a.x + sl[r] + (int64_t)c0 * a.ldx;
#pragma unroll
      for (int c = 0; c < RB; ++c)
        if (c < nr) xp[(int64_t)c * a.ldx] -= acc[c];
    }
  }
}

__global__ void __launch_bounds__(AW) k_scale_fwd(const ScaleAp* __restrict__ ds, ApplyArgs a) {
  __shared__ TrsvShared sh;
  const ScaleAp e = ds[blockIdx.x];
  const int32_t* sl = a.slot + e.slot_p;
  gather_seg(sl, e.np, a, e.tmp);
  for (int c0 = 0; c0 < a.nrhs; c0 += RB)
    trsv_fwd(e.L, e.np, e.Dinv, e.np, a.tmp + e.tmp + (int64_t)c0 * a.ldt, a.ldt, min(RB, a.nrhs - c0), sh);
  scatter_seg(sl, e.np, a, e.tmp);
}

__global__ void __launch_bounds__(AW) k_scale_bwd(const ScaleAp* __restrict__ ds, ApplyArgs a) {
  __shared__ TrsvShared sh;
  const ScaleAp e = ds[blockIdx.x];
  const int32_t* sl = a.slot + e.slot_p;
  gather_seg(sl, e.np, a, e.tmp);
  for (int c0 = 0; c0 < a.nrhs; c0 += RB)
    trsv_bwd(e.L, e.np, e.Dinv, e.np, a.tmp + e.tmp + (int64_t)c0 * a.ldt, a.ldt, min(RB, a.nrhs - c0), sh);
  scatter_seg(sl, e.np, a, e.tmp);
}

// Householder sweep over the r reflectors of Q_p (V column-major, ld np, unit
// diagonal and zeros above); dir = +1 applies Q^T (increasing), -1 applies Q.
template <int DIR>
__global__ void __launch_bounds__(AW) k_house(const HouseAp* __restrict__ ds, ApplyArgs a) {
  const HouseAp e = ds[blockIdx.x];
  const int np = e.np;
  const int32_t* sl = a.slot + e.slot_p;
  __shared__ double red[AW / 64][RB];
  __shared__ double w[RB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    for (int jj = 0; jj < e.r; ++jj) {
      const int j = DIR > 0 ? jj : e.r - 1 - jj;
      const double* v = e.V + (int64_t)j * np;
      double acc[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) acc[c] = 0.0;
      for (int i = j + threadIdx.x; i < np; i += AW) {
        const double vi = v[i];
        const double* xp = a.x + sl[i] + (int64_t)c0 * a.ldx;
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (c < nr) acc[c] += vi * xp[(int64_t)c * a.ldx];
      }
#pragma unroll
      for (int c = 0; c < RB; ++c) {
        const double s = wsum(acc[c]);
        if (lane == 0) red[wave][c] = s;
      }
      __syncthreads();
      if (threadIdx.x < RB) {
        double s = 0.0;
        for (int q = 0; q < AW / 64; ++q) s += red[q][threadIdx.x];
        w[threadIdx.x] = e.tau[j] * s;
      }
      __syncthreads();
      for (int i = j + threadIdx.x; i < np; i += AW) {
        const double vi = v[i];
        double* xp = a.x + sl[i] + (int64_t)c0 * a.ldx;
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (c < nr) xp[(int64_t)c * a.ldx] -= w[c] * vi;
      }
      __threadfence_block();
      __syncthreads();
    }
  }
}

__global__ void k_gather(const int32_t* __restrict__ nslot, int64_t len, ApplyArgs a) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= len) return;
  const int32_t s = nslot[q];
  for (int c = 0; c < a.nrhs; ++c) a.gbuf[q + (int64_t)c * a.ldg] = a.x[s + (int64_t)c * a.ldx];
}

// t_k = x_s[k] - sum_r G[r][k] xN[r] (wave per k), then x_s = L_s^{-T} t.
__global__ void __launch_bounds__(AW) k_elim_bwd(const ElimAp* __restrict__ ds, ApplyArgs a) {
  __shared__ TrsvShared sh;
  const ElimAp e = ds[blockIdx.x];
  const int ns = e.ns, nN = e.nN;
  const int32_t* sl = a.slot + e.slot_s;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c0 = 0; c0 < a.nrhs; c0 += RB) {
    const int nr = min(RB, a.nrhs - c0);
    for (int k = wave; k < ns; k += AW / 64) {
      double acc[RB];
#pragma unroll
      for (int c = 0; c < RB; ++c) acc[c] = 0.0;
      const double* Gk = e.G + (int64_t)k * e.ld;
      for (int r = lane; r < nN; r += 64) {
        const double g = Gk[r];
        const double* xp = a.gbuf + e.slot_N + r + (int64_t)c0 * a.ldg;
#pragma unroll
        for (int c = 0; c < RB; ++c)
          if (c < nr) acc[c] += g * xp[(int64_t)c * a.ldg];
      }
#pragma unroll
      for (int c = 0; c < RB; ++c) {
        const double v = wsum(acc[c]);
        if (lane == 0 && c < nr)
          a.tmp[e.tmp + k + (int64_t)(c0 + c) * a.ldt] = a.x[sl[k] + (int64_t)(c0 + c) * a.ldx] - v;
      }
    }
  }
  __threadfence_block();
  __syncthreads();
  for (int c0 = 0; c0 < a.nrhs; c0 += RB)
    trsv_bwd(e.L, e.ld, e.Dinv, ns, a.tmp + e.tmp + (int64_t)c0 * a.ldt, a.ldt, min(RB, a.nrhs - c0), sh);
  scatter_seg(sl, ns, a, e.tmp);
}

void apply_step_forward(const StepDev& s, const ApplyArgs& a, hipStream_t st) {
  if (s.n_elim) hipLaunchKernelGGL(k_elim_fwd, dim3(s.n_elim), dim3(AW), 0, st, s.elim, a);
  if (s.n_target) hipLaunchKernelGGL(k_target_fwd, dim3(s.n_target), dim3(AW), 0, st, s.target, s.contrib, a);
  if (s.n_scale) hipLaunchKernelGGL(k_scale_fwd, dim3(s.n_scale), dim3(AW), 0, st, s.scale, a);
  if (s.n_house) hipLaunchKernelGGL(k_house<1>, dim3(s.n_house), dim3(AW), 0, st, s.house, a);
}

void apply_step_backward(const StepDev& s, const ApplyArgs& a, hipStream_t st) {
  if (s.n_house) hipLaunchKernelGGL(k_house<-1>, dim3(s.n_house), dim3(AW), 0, st, s.house, a);
  if (s.n_scale) hipLaunchKernelGGL(k_scale_bwd, dim3(s.n_scale), dim3(AW), 0, st, s.scale, a);
  if (s.n_elim) {
    if (s.nslot_len)
      hipLaunchKernelGGL(k_gather, dim3((s.nslot_len + 255) / 256), dim3(256), 0, st, s.nslot, s.nslot_len, a);
    hipLaunchKernelGGL(k_elim_bwd, dim3(s.n_elim), dim3(AW), 0, st, s.elim, a);
  }
}

// ---------------------------------------------------------------- PCG vector kernels
__global__ void k_spmv(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                       const double* __restrict__ val, int64_t n, int nrhs, const double* __restrict__ x,
                       double* __restrict__ y) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t b = rowptr[v], e = rowptr[v + 1];
  for (int c = 0; c < nrhs; ++c) {
    const double* xc = x + (int64_t)c * n;
    double s = 0.0;
    for (int64_t q = b; q < e; ++q) s += val[q] * xc[colind[q]];
    y[v + (int64_t)c * n] = s;
  }
}

// partial[blk + c*nblk] = sum over this block's rows of a[:,c] * b[:,c]
__global__ void __launch_bounds__(256) k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t n, double* __restrict__ partial) {
  const int c = blockIdx.y;
  const int64_t nblk = gridDim.x;
  const double* ac = a + (int64_t)c * n;
  const double* bc = b + (int64_t)c * n;
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += nblk * 256) s += ac[i] * bc[i];
  __shared__ double red[4];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x + (int64_t)c * nblk] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_dot_final(const double* __restrict__ partial, int nblk,
                                                   double* __restrict__ out) {
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += partial[i + (int64_t)c * nblk];
  __shared__ double red[4];
  s = wsum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = red[0] + red[1] + red[2] + red[3];
}

// alpha_c = active ? rz/pq : 0; x += alpha p; r -= alpha q
__global__ void k_update_xr(int64_t n, int nrhs, const double* __restrict__ rz, const double* __restrict__ pq,
                            const int32_t* __restrict__ active, const double* __restrict__ p,
                            const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nrhs; ++c) {
    if (!active[c]) continue;
    const double alpha = rz[c] / pq[c];
    const int64_t o = i + (int64_t)c * n;
    x[o] += alpha * p[o];
    r[o] -= alpha * q[o];
  }
}

// p = z + beta p with beta = rz_new/rz (active columns only)
__global__ void k_update_p(int64_t n, int nrhs, const double* __restrict__ rz_new, const double* __restrict__ rz,
                           const int32_t* __restrict__ active, const double* __restrict__ z, double* __restrict__ p) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nrhs; ++c) {
    if (!active[c]) continue;
    const double beta = rz_new[c] / rz[c];
    const int64_t o = i + (int64_t)c * n;
    p[o] = z[o] + beta * p[o];
  }
}

// y = b - y (true residual)
__global__ void k_residual(int64_t len, const double* __restrict__ b, double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < len) y[i] = b[i] - y[i];
}

void launch_spmv(const int64_t* rowptr, const int32_t* colind, const double* val, int64_t n, int nrhs,
                 const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3((n + 255) / 256), dim3(256), 0, s, rowptr, colind, val, n, nrhs, x, y);
}
void launch_dot(const double* a, const double* b, int64_t n, int nrhs, double* partial, int nblk, double* out,
                hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(nblk, nrhs), dim3(256), 0, s, a, b, n, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(nrhs), dim3(256), 0, s, partial, nblk, out);
}
void launch_update_xr(int64_t n, int nrhs, const double* rz, const double* pq, const int32_t* active,
                      const double* p, const double* q, double* x, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_update_xr, dim3((n + 255) / 256), dim3(256), 0, s, n, nrhs, rz, pq, active, p, q, x, r);
}
void launch_update_p(int64_t n, int nrhs, const double* rz_new, const double* rz, const int32_t* active,
                     const double* z, double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p, dim3((n + 255) / 256), dim3(256), 0, s, n, nrhs, rz_new, rz, active, z, p);
}
void launch_residual(int64_t len, const double* b, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3((len + 255) / 256), dim3(256), 0, s, len, b, y);
}

}  // namespace spand
