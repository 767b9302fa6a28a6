// Host-side launchers of the HIP kernels (one launch = one tree level or one
// per-node step over a task list).
#pragma once
#include <hip/hip_runtime.h>

#include "hss_internal.hpp"

namespace hss {

enum class MMStep { LeafUp, Up, Couple, Down, LeafOut };

template <typename T>
void launch_mm_level(MMStep step, const KArgs<T, CallMM<T>>& a, int nblocks, int ytiles,
                     int max_rows, hipStream_t s);

// Y = A X in three launches (kernels_mmf.hip): Up over the nodes at level
// max(p - mmf_up_height(), 0) (their subtrees, then the upward pass and core
// blocks carried on by the last arrival at each node), Down over the nodes at
// level max(p - mmf_down_height(), 0), Leaf over the leaves.  nrhs: the largest right-hand-side count of the launch; max_ku: the
// largest leaf rank ku; max_k: the largest rank of any node.
// Leaf: Y = D X + U y^ in one pass; LeafDX: Y = D X; LeafUY: Y += U y^;
// UpDX: the up pass with the leaves' Y = D X in the same launch (one rhs,
// ranks <= 32, single instance)
enum class MMFStep { Up, Down, Leaf, LeafDX, LeafUY, UpDX };
template <typename T>
void launch_mmf(MMFStep step, const KArgs<T, CallMM<T>>& a, int nblocks, int nrhs, int max_ku,
                int max_k, hipStream_t s);
int mmf_down_height();
int mmf_up_height();

// Y = A X for blocks of right-hand sides, one launch per level
// (kernels_mmw.hip): LeafUp over the leaves, Up over levels p-1 .. 0, Down
// over levels 1 .. p-1, LeafOut over the leaves.  Single instance, op N,
// leaves <= 128 rows and ranks <= 32 (mmw_fits).
enum class MMWStep { LeafUp, Up, Down, LeafOut };
bool mmw_fits(int max_leaf, int max_k);
template <typename T>
void launch_mmw(MMWStep step, const KArgs<T, CallMM<T>>& a, int nblocks, int nrhs,
                hipStream_t s, int max_m = kMaxBlock);   // max_m: the largest leaf (LeafUp, LeafOut)
enum class UlvStep { Merge, Factor, RootLU, Fwd, Root, Bwd, FwdOp };

// Step 1 (QL / LQ) on one level of blocks, register-resident (kernels_factor.hip).
template <typename T>
void launch_factor_reg(const KArgs<T, CallSV<T>>& a, int nblocks, int max_mp, hipStream_t s);

// Step 1 blocked (kernels_factor_blk.hip): panels of 32 Householder vectors
// applied in compact WY form on the matrix cores, for blocks of 65..128 rows
// with every rank <= 32.
template <typename T>
bool factor_blk_fits(int max_mp, int max_k);
template <typename T>
void launch_factor_blk(const KArgs<T, CallSV<T>>& a, int nblocks, hipStream_t s);

// Solve sweeps, one wavefront per (node, right-hand-side column) (kernels_solve.hip).
// stage_elems > 0: one wavefront per work-group with that many elements of T
// of dynamic LDS for the node's factor copies.
template <typename T>
void launch_solve_w(UlvStep step, const KArgs<T, CallSV<T>>& a, int nitems, int ncols,
                    int64_t stage_elems, hipStream_t s);

// max_k: the largest rank of the nodes involved; max_mp: the largest block.
template <typename T>
void launch_ulv(UlvStep step, const KArgs<T, CallSV<T>>& a, int nblocks, int max_k,
                int max_mp, hipStream_t s);

// Hadamard product C = A o B of two matrices on one tree (kernels_hadamard.hip):
// the packed D arrays elementwise (nD entries), then two work-groups per node
// (row and column side) for the bases, translation operators and core blocks.  g*[0..6] are the
// FP64 generator arrays D, U, V, R, W, B12, B21; n* the device node tables.
void launch_hadamard(const NodeInfo* nA, const NodeInfo* nB, const NodeInfo* nC,
                     const double* const gA[7], const double* const gB[7], double* const gC[7],
                     int64_t nD, int32_t nnodes, int32_t p, hipStream_t s);

// HSS recompression (kernels_compress.hip).  Work copies of the generators in
// the input's packed layout; TU / TV hold kMaxRank x kMaxRank per node (the
// phase-1 QR factors, then the phase-2 left singular factors), su / sv
// kMaxRank singular values per node, rku / rkv the ranks after phase 1,
// nku / nkv after phase 2.  node0, count: the nodes of the launch.
enum class CompressStep { LeafQR, UpQR, Core, Svd, ApplyParent, ApplyChild };
struct CompressBufs {
  const NodeInfo* nodes;
  double *U, *V, *R, *W, *B12, *B21;
  double *TU, *TV, *su, *sv;
  int32_t *rku, *rkv, *nku, *nkv;
};
void launch_compress(CompressStep step, const CompressBufs& b, int node0, int count, double tau,
                     hipStream_t s);
// Pack the work blocks (work[0..5] = U, V, R, W, B12, B21 in the layout of
// `in`) at the ranks of `out` into dst[0..5].
void launch_compress_gather(const NodeInfo* in, const NodeInfo* out, const double* const work[6],
                            double* const dst[6], int nnodes, hipStream_t s);

// Dense-to-HSS construction (kernels_construct.hip).
constexpr int kCnMaxRows = 128;   // rows of a block row one truncation takes (slot ld)
// One block row H: rows row0 .. row0 + r - 1 (r <= kCnMaxRows) of the
// column-major X (leading dimension ld), every column 0 .. ncols - 1 except
// ex0 .. ex1 - 1.  Out: U (r x r, ld kCnMaxRows) its left singular vectors by
// decreasing singular value, sig the singular values, *rank the count kept
// (sigma > eps * sigma_1, at least one).
struct CnTask {
  const double* X;
  int64_t ld, row0;
  int32_t r, pad;
  int64_t ncols, ex0, ex1;
  double* U;
  double* sig;
  int32_t* rank;
};
// Y(:, ycol0 .. ycol0 + k - 1) = X(:, xcol0 .. xcol0 + s - 1) B for rows
// 0 .. rows - 1; B is s x k (ld ldb), s <= 128, k <= 64.
struct CnRmul {
  const double* X;
  int64_t ldx, rows, xcol0;
  int32_t s, k;
  const double* B;
  int64_t ldb;
  double* Y;
  int64_t ldy, ycol0;
};
// dst (rows x cols, ld rows) = the block of src at leading dimension lds.
struct CnCopy {
  const double* src;
  int64_t lds;
  double* dst;
  int32_t rows, cols;
};
// leaves: the launch of the leaf level (named apart in the per-kernel timing)
void launch_cn_trunc(const CnTask* tasks, int count, double eps, bool leaves, hipStream_t s);
void launch_cn_rmul(const CnRmul* tasks, int count, int64_t rows, hipStream_t s);
void launch_cn_trans(const double* X, int64_t ldx, int64_t rows, int64_t cols, double* Y,
                     int64_t ldy, hipStream_t s);
void launch_cn_copy(const CnCopy* tasks, int count, hipStream_t s);

// Elementwise / reduction helpers (kernels_util.hip).
void launch_cast_f64_f32(const double* src, float* dst, int64_t n, hipStream_t s);
// dst[i + j*ldd] = (float)(src[i + j*lds] * scale[j])   (scale may be null -> 1)
// gate (all launchers that take one): NULL, or a device flag; the launch does
// nothing when it reads 0.
void launch_scale_cast(const double* src, int64_t lds, float* dst, int64_t ldd, int64_t n,
                       int64_t nrhs, const double* scale, hipStream_t s,
                       const int32_t* gate = nullptr);
// x[i + j*ldx] += scale[j] * d[i + j*ldd]
void launch_axpy_cast(const float* d, int64_t ldd, double* x, int64_t ldx, int64_t n,
                      int64_t nrhs, const double* scale, hipStream_t s,
                      const int32_t* gate = nullptr);
// sums[j] (+)= sum_i a[i+j*lda]^2 ; maxabs[j] = max |a| (optional)
void launch_colstats(const double* a, int64_t lda, int64_t n, int64_t nrhs, double* sumsq,
                     double* maxabs, hipStream_t s);
void launch_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                   int64_t nrhs, hipStream_t s, const int32_t* gate = nullptr);
void launch_fill(double* p, double v, int64_t n, hipStream_t s);
// Fused refinement check (residual, norms, eta, max |r|, the refinement gate
// and step count in the status block st) and per-column max |a|; part holds
// check_partials(nrhs) doubles, cnt one counter that starts at 0 (each
// launch leaves it at 0).  out = [eta_max, 0, eta_0 .. eta_{nrhs-1}].
int check_partials(int64_t nrhs);
void launch_check(const double* b, int64_t ldb, double* r, int64_t ldr, const double* x,
                  int64_t ldx, int64_t n, int64_t nrhs, double normA, double* part,
                  unsigned* cnt, int32_t* st, double* rmax, double* out, const int32_t* gate,
                  double tol, int step, int max_refine, hipStream_t s);
// Writes the solve report (include/hss.h, hss_solve_info + nrhs etas) at info.
void launch_solve_info(void* info, int64_t nrhs, const double* out, const int32_t* st,
                       double normA, double tol, bool have_eta, hipStream_t s);
void launch_colmax(const double* a, int64_t lda, int64_t n, int64_t nrhs, double* part,
                   unsigned* cnt, double* amax, hipStream_t s);
// dst = scale[j] * (double)src
void launch_cast_back(const float* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                      int64_t nrhs, const double* scale, hipStream_t s);
// dst += src (FP64)
void launch_axpy64(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                   int64_t nrhs, hipStream_t s, const int32_t* gate = nullptr);
void launch_normalize(const double* src, double* dst, int64_t n, const double* sumsq,
                      hipStream_t s);
void launch_hash_fill(double* d, int64_t n, uint64_t seed, hipStream_t s);
// Iterative refinement over many instances (one launch per operation).
struct IRSeg {
  double* B;        // solution being refined (caller's memory), leading dimension ldb
  int64_t ldb;
  double *b0, *res, *d64;   // n x nrhs, leading dimension n
  float* r32;
  int64_t n;
  int32_t nrhs;
  int32_t pad;
  double* stats;    // rr | xx | bb | rmax | bmax | eta | out (nrhs each)
  double norm2;
  double tol;
  int32_t* st;      // the instance's status block (gate, steps, status bits)
  void* info;       // solve report (include/hss.h) or NULL
};
enum IROp {
  IR_ZERO = 0,      // clear rr, xx, rmax
  IR_SAVE_B0,       // b0 = B
  IR_STATS_B0,      // bb += ||b0_j||^2
  IR_STATS_BMAX,    // bmax = max |B_j|
  IR_SCALE_B,       // r32 = B / bmax
  IR_CAST_BACK,     // B = bmax * r32
  IR_RESID,         // res = b0 - res; rr, rmax
  IR_STATS_X,       // xx += ||B_j||^2
  IR_ETA,           // eta_j, out = max_j eta_j; the gate and step count in st
  IR_SCALE_RES,     // r32 = res / rmax
  IR_AXPY_CAST,     // B += rmax * r32
  IR_COPY_RES,      // d64 = res
  IR_AXPY64,        // B += d64
  IR_ZERO_ALL,      // clear all stats
  IR_INFO           // write the solve report (have_eta = step != 0)
};
// gated: instances whose gate (st[kStGate]) is 0 are skipped.  step and
// max_refine: the refinement step a check (IR_ETA) belongs to.
// max_cols: the largest nrhs of the instances (per-column passes take one
// grid slice per column).
void launch_ir_batch(int op, const IRSeg* segs, int count, int64_t max_n, int max_cols,
                     bool gated, int step, int max_refine, hipStream_t s);

}  // namespace hss
