// Descriptors and launchers of the preconditioner apply and PCG vector kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spand {

struct ElimAp {
  const double* L;     // ns x ns lower-triangular factor L_s (top of the panel), ld ld
  const double* G;     // nN x ns, A_{N_s s} L_s^{-T} (below L_s in the panel), ld ld
  const double* Dinv;  // inverses of the diagonal blocks of L_s (CHOL_NB^2 doubles each)
  int32_t ld, ns, nN;
  int32_t nchunk;      // row chunks of G in the backward product (their partial sums follow t in the scratch)
  int64_t slot_s;      // offset of s's slots in the step slot array
  int64_t slot_N;      // offset of s's neighbour slots in the step neighbour-slot array
  int64_t tmp;         // offset of s's rows in the apply scratch: t, then nchunk > 1 partial sums
  int64_t ytmp;        // offset of the nN rows of y = G L_s^{-1} x_s (forward sweep) in the scratch
};
struct FwdTile {      // panel rows [r0, r0 + 64) of eliminated cluster s (r0 a multiple of 64), those of G
  int32_t s, r0;
};
struct ElimTile {     // columns [k0, min(k0 + 64, ns)) of eliminated cluster s, rows of G in chunk c
  int32_t s, k0, c, pad;
};
#define ELIM_RC 512  // rows of G per chunk of the backward product
struct TargetAp {     // rows [r0, min(r0 + 64, nn)) of receiving cluster n
  int32_t nn, cbeg, cend, r0;
  int64_t slot_n;
};
struct TargetContrib {
  int64_t y;        // where the rows of n of y_s = G_s L_s^{-1} x_s live in the apply scratch
};
struct ScaleAp {
  const double* Linv;  // np x np lower-triangular L_p^{-1}, ld ldl (np rounded up to 16)
  int32_t np, ldl;
  int64_t slot_p;
  int64_t tmp;         // np rows of scratch: x_p gathered
};
struct ScaleTile {    // rows [r0, r0 + 64) of the product with L_p^{-1} (or its transpose)
  int32_t p, r0;
};
struct HouseAp {
  const double* V;    // np x r reflectors, ld ldv (unit diagonal, zeros above)
  const double* T;    // r x r upper-triangular factor of Q = I - V T V^T, ld ldt
  int32_t np, r, ldv, ldt;
  int64_t slot_p;
  int64_t tmp;        // 2*r rows of scratch: V^T x, then the T-product
};
// A small interface p (np <= 128) whose scaling and Householder product are
// applied together by one wave (k_iface).
struct IfaceAp {
  const double* Linv;  // np x np lower-triangular L_p^{-1}, ld ldl
  const double* V;     // np x r reflectors, ld ldv (unused when r == 0)
  const double* T;     // r x r upper-triangular T, ld ldt
  int32_t np, r, ldl, ldv, ldt, pad;
  int64_t slot_p;
};
struct HouseTile {    // 64 reflectors [j0, j0 + 64) or 64 rows [j0, j0 + 64) of interface p
  int32_t p, j0;
};
// An interface sparsified by the interpolative transformation (Sec. 2.6.2): its
// coarse dofs c = perm[0..r) and fine dofs f = perm[r..np) (indices into its slots
// at the step), T_cf, and X = [L_f; G_cf] (np x nf, ld np: L_f the nf x nf lower
// Cholesky factor of C_ff on top, G_cf = C_cf L_f^{-T} below).  The forward sweep
// leaves y_c in the first r slots and y_f in the others.
struct InterpAp {
  const int32_t* perm;
  const double* T;    // r x nf, ld r
  const double* X;    // ld np
  int32_t np, r;
  int64_t slot_p;
};

// Device-side view of one step for the apply.
struct StepDev {
  const ElimAp* elim;
  const TargetAp* target;
  const TargetContrib* contrib;
  const ScaleAp* scale;
  const HouseAp* house;
  const ElimTile* etile;
  const FwdTile* ftile;    // 64-row tiles of every G_s for the forward products
  int32_t n_ftile, pad_ftile;
  const ScaleTile* stile;  // row tiles of every L_p^{-1}
  const int32_t* sgather;  // slot of every scratch row of the scaled interfaces
  int64_t sgather_len;
  const HouseTile* hr;   // reflector tiles of every Q_p
  const HouseTile* hv;   // row tiles of every Q_p
  const IfaceAp* iface;  // small interfaces: np <= 64 first (n_iface1), then np <= 128 (n_iface2)
  int32_t n_iface1, n_iface2;
  const InterpAp* interp;  // interpolative interfaces (after the scaling of the step)
  int32_t n_interp, pad_interp;
  const int32_t* slot;
  const int32_t* nslot;
  int64_t nslot_len;
  int32_t n_elim, n_target, n_scale, n_house, n_etile, n_hr, n_hv, n_stile;
};

struct ApplyArgs {
  double* x;        // n x nrhs vector being transformed, ld ldx
  int64_t ldx;
  int32_t nrhs, pad;
  double* tmp;      // scratch, ld ldt
  int64_t ldt;
  double* gbuf;     // gathered neighbour values, ld ldg
  int64_t ldg;
  const int32_t* slot;   // step slot array
};

// Interpolative interfaces of a step (kernels_interp.hip): dir > 0 forward, < 0 backward.
void launch_interp_apply(const InterpAp* d, int32_t count, const ApplyArgs& a, int dir, hipStream_t s);
void apply_step_forward(const StepDev& s, const ApplyArgs& a, hipStream_t st);
void apply_step_backward(const StepDev& s, const ApplyArgs& a, hipStream_t st);

// y = A x; x and y have leading dimension ld (n when ld <= 0).
void launch_spmv(const int64_t* rowptr, const int32_t* colind, const double* val, int64_t n, int nrhs,
                 const double* x, double* y, hipStream_t s, int64_t ld = 0);

// Batched PCG over problems stacked in one vector (leading dimension ld): the blocks
// of the segmented dot products (problem q: nblk[q] blocks of its n_q rows at off).
struct SegBlk {
  int64_t off, n;
  int32_t local, nblk;
};
// One problem of a stacked system: its CSR (local indices) and its first row.
struct SpmvProb {
  const int64_t* rowptr;
  const int32_t* colind;
  const double* val;
  int64_t n, off;
};
// One problem's own vector block (leading dimension n) and its first stacked row.
struct StackProb {
  const double* own_in;
  double* own_out;
  int64_t n, off;
};
// blk[k] = (problem, 256-row block) of workgroup k.
void launch_spmv_batch(const SpmvProb* probs, const int2* blk, int64_t nblk, int nrhs, int64_t ld, const double* x,
                       double* y, hipStream_t s);
void launch_stack(const StackProb* probs, const int2* blk, int64_t nblk, int nrhs, int64_t ld, double* stacked,
                  bool to_stack, hipStream_t s);
void launch_seg_dot(const double* a, const double* b, int64_t ld, int nrhs, const SegBlk* blks, int64_t nb_tot,
                    const int64_t* pbase, const int32_t* nblk, int32_t P, double* partial, double* out, hipStream_t s);
void launch_seg_update_xr(int64_t ntot, int nrhs, const int32_t* pid, const double* rz, const double* pq,
                          const int32_t* active, const double* p, const double* q, double* x, double* r, hipStream_t s);
void launch_seg_update_p(int64_t ntot, int nrhs, const int32_t* pid, const double* rz_new, const double* rz,
                         const int32_t* active, const double* z, double* p, hipStream_t s);
void launch_dot(const double* a, const double* b, int64_t n, int nrhs, double* partial, int nblk, double* out,
                hipStream_t s);
void launch_update_xr(int64_t n, int nrhs, const double* rz, const double* pq, const int32_t* active,
                      const double* p, const double* q, double* x, double* r, hipStream_t s);
void launch_update_p(int64_t n, int nrhs, const double* rz_new, const double* rz, const int32_t* active,
                     const double* z, double* p, hipStream_t s);
void launch_residual(int64_t len, const double* b, double* y, hipStream_t s);
void launch_copy_vec(const double* r, double* z, int64_t len, hipStream_t s);
// dst[i + c ld] = src[idx[i] + c ld] for i < n and the nrhs columns
void launch_permute(const double* src, double* dst, const int32_t* idx, int64_t n, int nrhs, int64_t ld,
                    hipStream_t s);

}  // namespace spand
