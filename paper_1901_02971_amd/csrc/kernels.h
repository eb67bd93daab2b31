// Device-side descriptor types and kernel launchers of libspand (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spand {

// Blocked Cholesky (kernels_chol.hip).  Diagonal blocks are CHOL_NB wide.
constexpr int CHOL_NB = 64;
// Leading dimension of the factor matrices of the interfaces (L_p^{-1}, V, T): the
// row count rounded up to 16 entries, so that every column starts on a 128-byte line.
__host__ __device__ inline int32_t pad16(int32_t n) { return (n + 15) / 16 * 16; }
struct PotrfDesc {
  double* P;     // diagonal block start (column-major, ld)
  double* Dinv;  // w x w output: inverse of the diagonal block's factor, ld w
  int32_t* fail; // on a non-positive pivot: atomicMin(fail, id) (the problem's flag word)
  int32_t ld, w, id, pad;
};
struct PanelDesc {
  double* P;           // panel column kb (row 0 of the panel), ld
  const double* Dinv;  // w x w
  int32_t ld, w, r0, r1;  // rows [r0, r1) are solved
};
void launch_potrf_diag(const PotrfDesc* d, int32_t count, hipStream_t s);
void launch_panel_trsm(const PanelDesc* d, int32_t count, hipStream_t s);

// One product C = alpha * op(A) op(B) + beta * C on column-major operands.
enum : int32_t {
  G_TA = 1,      // op(A) = A^T
  G_TB = 2,      // op(B) = B^T
  G_TRIA = 4,    // op(A)(m,k) = 0 for k > m (lower-triangular op(A))
  G_TRIB = 8,    // op(B)(k,n) = 0 for k > n
  G_LOWERC = 16  // only tiles with tile row >= tile column are produced (host side)
};
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int32_t M, N, K;
  int32_t lda, ldb, ldc;
  int32_t flags;
  int32_t part;  // 64x64 output tiles produced: 0 all, 1 on or below the diagonal, 2 on or above (M == N)
  double alpha, beta;
  int64_t t0;    // first tile of this product in the numbering of its launch sequence
  int32_t ts;    // output tile edge of the launch (64, 128 or 32)
  int32_t pad;
};
// Output tiles of edge ts of one product (part != 0 requires M == N).
__host__ __device__ inline int64_t gemm_tiles(int32_t M, int32_t N, int32_t part, int32_t ts = 64) {
  const int64_t tm = (M + ts - 1) / ts, tn = (N + ts - 1) / ts;
  return part == 0 ? tm * tn : tm * (tm + 1) / 2;
}

// Target block of the Schur complement reduction.
struct ReduceDesc {
  double* T;          // target block, ld ldT
  int32_t ldT, rows, cols, diag;  // diag: target is a diagonal (square) block
  int32_t c_begin, c_end;         // contributions [c_begin, c_end) in ascending s
  int32_t e0, e1;                 // entries [e0, e1) of the block (column-major index) for this workgroup
};
#define REDUCE_CHUNK 16384  // block entries per workgroup of the Schur reduction
struct ContribDesc {
  const double* C;  // contribution block start inside C_s, ld ldC
  int32_t ldC, pad;
};

// Strided copy (optionally transposed) used by merge and assembly.
struct CopyDesc {      // columns [c0, c1) of a rows-row block (or of its transpose when trans)
  const double* src;
  double* dst;
  int32_t lds, ldd, rows, c0, c1, trans;
};
// I_n into columns [c0, c1) of the n x n block D (ld ld)
struct IdentDesc {
  double* D;
  int32_t n, ld, c0, c1;
};
#define COPY_CHUNK 16384  // entries per workgroup of the copies and identity fills
struct ZeroDesc {  // len (<= ZERO_CHUNK) doubles at p set to zero
  double* p;
  int64_t len;
};
#define ZERO_CHUNK 65536
void launch_zero(const ZeroDesc* d, int64_t count, hipStream_t s);
struct RemapSeg {  // p[k] <- pos[p[k]] for k < len (<= REMAP_CHUNK)
  int32_t* p;
  int64_t len;
};
#define REMAP_CHUNK 65536
void launch_remap(const RemapSeg* d, int64_t count, const int32_t* pos, hipStream_t s);
void launch_invert_perm(const int32_t* inv, int64_t n, int32_t* pos, int32_t* bad, hipStream_t s);

// Sparsification of one interface p (Sec. 2.6.1).  A_pn is held in the registers of
// S workgroups (slabs) of CAP = cpqr_capacity(G) columns each.  The width of A_pn is
// known only on the device: a neighbour q sparsified in an earlier colour class has
// shrunk to its rank, read from cursize[q].
struct SparsDesc {
  double* V;       // m x min(m, ncols_max) reflectors, column-major, ld m
  double* tau;     // min(m, ncols_max)
  double* diag;    // diagonal block of p (ld ldd), set to I_r on exit
  double* xch;     // slab exchange (S > 1): 3 buffers x S records of cpqr_record(G) doubles, zeroed
                   // before the launch
  int32_t* piv;    // when not null: piv[j] = column (index in A_pn) chosen at step j < r
  int32_t m, ldd, seg_begin, seg_end, id, S, G, lay;  // G: lanes per column (team size);
                                                      // lay: register layout (multi-slab kernel)
  int32_t ldv;                                        // leading dimension of V (>= m)
  int32_t dep_begin, dep_end;                         // multi-slab launch: neighbours to wait for
  int32_t kslots;  // column slots per team in use: the register slots, plus the LDS slot when
                   // cpqr_capacity(G, lay, true) sized the slabs
};
struct SegDesc {
  double* blk;  // block holding A_pq: trans=0 -> A_pq[r][c] = blk[r + c*ld]; trans=1 -> blk[c + r*ld]
  int32_t ld, trans, q, pad;
};
struct SlabRef {
  int32_t desc, w;  // desc < 0: an unused place of a multi-slab round
};

// dst >= 0: arena[dst]; dst <= -2: elim[-dst - 2]; dst == -1: skipped.
void launch_scatter_values(const double* vals, const int64_t* dst, int64_t nnz, double* arena, double* elim,
                           int32_t* flag, hipStream_t s);
// Batched GEMM over 64x64 output tiles on the matrix cores (kernels_mfma.hip);
// prec: 0 FP64, 1 FP32, 2 BF16x3.  Carries the trailing updates of the blocked
// Cholesky, the SYRK of the Schur update (Sec. 2.4) and the left scaling (Sec. 2.5).
// tile_desc[t] = product of tile t, for the tiles of nd products numbered by their t0.
void launch_expand_tiles(const GemmDesc* d, int32_t nd, int32_t* tile_desc, hipStream_t s);
// Tiles [tile0, tile0 + ntiles) of a sequence, one workgroup each.
// variant: output tile 64 (0), 128 (1) or 32 (2) of the FP64 / FP32 kernels (BF16x3: 64);
// every variant adds an entry's products in the same order, so results agree bit for bit.
void launch_gemm(const GemmDesc* d, const int32_t* tile_desc, int64_t tile0, int64_t ntiles, int prec, int variant,
                 hipStream_t s);
// Number of output-tile variants of the batched GEMM, and the tile edge of each.
int gemm_variant_count();
int gemm_variant_tile(int variant);
void launch_reduce(const ReduceDesc* d, int32_t count, const ContribDesc* c, hipStream_t s);
void launch_copy(const CopyDesc* d, int64_t count, hipStream_t s);
void launch_set_identity(const IdentDesc* d, int32_t count, hipStream_t s);
// cursize: current size of every cluster of the step; the kernel sets
// cursize[p] = kept rank when it finishes p and nref[p] = number of reflectors
// stored (0 when no coupled dofs were left and p was not sparsified).  err
// receives bit 2 if a slab barrier timed out.  Launches with more than one slab
// per interface are cooperative (all workgroups resident).
// Register layouts of a slab: lay 0 keeps 32 rows of 2 columns per lane (every
// kernel), lay 1 20 rows of 3 columns (multi-slab kernel only).
// Team size G (lanes per column, a power of two) for m rows; -1 if m is too large.
int32_t cpqr_team(int32_t m, int32_t lay = 0);
// Columns of one slab: the register slots only, or with the LDS slot where the layout
// has one (SparsDesc::kslots tells the kernel which).
int32_t cpqr_capacity(int32_t G, int32_t lay = 0, bool lds_slot = true);
int32_t cpqr_kslots(int32_t G, int32_t lay, bool lds_slot);
// Doubles of one slab's exchange record (S > 1): the header + the rows of a team.
int32_t cpqr_record(int32_t G, int32_t lay = 0);
size_t cpqr_lds_bytes(int32_t G, int32_t lay, int32_t nseg);
// The wide single-slab layout (teams of 2 lanes, more columns per lane): the rows
// and columns one workgroup holds, and its dynamic LDS size.
int32_t cpqr_wide_rows();
int32_t cpqr_wide_capacity();
size_t cpqr_wide_lds_bytes(int32_t nseg);
hipError_t launch_cpqr_one_wide(const SparsDesc* d, const SlabRef* slabs, int32_t nslab, const SegDesc* seg,
                                double eps, int32_t* cursize, int32_t* nref, int32_t* err, size_t lds_bytes,
                                hipStream_t s);
// Co-resident workgroups of the multi-slab kernel at this dynamic LDS size.
int cpqr_max_coresident(size_t lds_bytes);
// Single-slab interfaces of team size G (plain launch), and multi-slab interfaces of
// any team size (cooperative launch: all nslab workgroups resident).
hipError_t launch_cpqr_one(int32_t G, const SparsDesc* d, const SlabRef* slabs, int32_t nslab, const SegDesc* seg,
                           double eps, int32_t* cursize, int32_t* nref, int32_t* err, size_t lds_bytes, hipStream_t s);
// The multi-slab launch gives workgroup b the places slabs[k * nslab + b], k < nround,
// in turn; the interfaces must appear in one order in every workgroup's places.
// Interface d waits until done[deps[e].x] >= deps[e].y for e in [dep_begin, dep_end)
// (neighbours earlier in that order); every slab adds 1 to done[id] when it ends.
// done starts at zero.
hipError_t launch_cpqr_multi(const SparsDesc* d, const SlabRef* slabs, int32_t nslab, int32_t nround,
                             const SegDesc* seg, double eps, int32_t* cursize, int32_t* nref, int32_t* err,
                             const int2* deps, int32_t* done, size_t lds_bytes, hipStream_t s);
// Interfaces beyond the register layouts (kernels_cpqr.hip k_cpqr_big): one
// cooperative launch of nb workgroups per interface, A_pn in a global work copy.
// Rows at most cpqr_big_max_rows(); the scratch holds wk (m * ncols doubles), nrm
// (ncols), pst (ncols ints), rb (min(m, ncols)), post_mx (nb), post_cd (nb ints) and
// the barrier counter bar, which must be zero at launch.
int32_t cpqr_big_max_rows();
int cpqr_big_max_coresident(int32_t nseg);
hipError_t launch_cpqr_big(const SparsDesc& d, int32_t nseg, const SegDesc* seg, double eps, int32_t* cursize,
                           int32_t* nref, int32_t* err, int32_t nb, double* wk, double* nrm, int32_t* pst, double* rb,
                           double* post_mx, int32_t* post_cd, uint32_t* bar, hipStream_t s);
struct TDesc {
  const double* V;    // m x r, ld ldv
  const double* tau;  // r
  double* T;          // r x r output, ld ldt
  int32_t m, r, ldv, ldt;
};
// Diagonal 64-wide block j0 of the compact-WY factor T (r x r, ld r) of one
// interface; on entry the upper triangle of T holds V^T V.
struct TBlock {
  double* T;          // ld ld
  const double* tau;
  int32_t r, j0, ld, pad;
};
void launch_build_t_diag(const TBlock* blocks, int32_t count, hipStream_t s);

constexpr int GEMM_TILE = 64;

// Interpolative sparsification (Sec. 2.6.2, kernels_interp.hip).  For one interface
// p of np dofs, the truncated CPQR of A_np (m x np, ld m, in W) has chosen r pivot
// columns piv[0..r); nf = np - r.
struct InterpPermDesc {  // perm = the pivots in pivot order, then the other columns ascending
  const int32_t* piv;
  int32_t* perm;
  int32_t np, r;
};
struct InterpTDesc {     // T_cf = R_11^-1 R_12 (r x nf, ld r); R = W[0..r, perm]
  const double* W;
  const int32_t* perm;
  double* T;
  int32_t ldw, r;
};
struct InterpCol {       // column j of T of interface desc
  int32_t desc, j;
};
struct InterpXDesc {     // entries [e0, e1) of X = A_pp[s, s], s = (perm[r..np), perm[0..r)), ld np;
  const double* App;     // A_pp read from its lower triangle (ld lda)
  const int32_t* perm;
  double* X;
  int32_t lda, np, r, pad;
  int64_t e0, e1;
};
struct InterpRowDesc {   // entries [e0, e1) of the r x nq block A_cq (c = perm[0..r)) from a copy of A_np
  const double* keep;    // A_np, ld ldk; neighbour q occupies rows [row0, row0 + nq)
  const int32_t* perm;
  double* blk;           // trans = 0: A_cq[i][k] at blk[i + k ld]; 1: at blk[k + i ld]
  int32_t ldk, row0, nq, r, ld, trans;
  int64_t e0, e1;
};
#define INTERP_CHUNK 16384   // entries per workgroup of the gathers
#define INTERP_MAX_NP 4096   // interface dofs an interpolative step handles
void launch_interp_perm(const InterpPermDesc* d, int32_t count, hipStream_t s);
void launch_interp_t(const InterpTDesc* d, const InterpCol* cols, int64_t ncols, int32_t rmax, hipStream_t s);
void launch_interp_x(const InterpXDesc* d, int64_t count, hipStream_t s);
void launch_interp_rows(const InterpRowDesc* d, int64_t count, hipStream_t s);

}  // namespace spand
