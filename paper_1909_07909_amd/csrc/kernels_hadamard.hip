// Hadamard product C = A o B of two HSS matrices on one cluster tree
// (Sec. 4.4, eq. "hadamard" and the figure of its pseudo-codes, right):
//   leaves:   D_C = D_A o D_B,  U_C = U_A .T U_B,  V_C = V_A .T V_B
//   internal: R_C = R_A kron R_B per child block of the stacked R (likewise
//             W), B12_C = B12_A kron B12_B, B21_C = B21_A kron B21_B,
// where row i of X .T Y is kron(x_i, y_i), so column a kB + b of U_C is
// U_A(:, a) o U_B(:, b).  Every output entry is one FP64 product of one
// entry of A and one of B.
//
// Two launches.  The diagonal blocks are a flat elementwise product over the
// packed D arrays, which have the same layout in A, B and C (same tree): a
// stream of 16-byte loads and stores, one vector per thread, bound by HBM.  The bases,
// translation operators and core blocks (ranks multiply, so these are the
// only arrays whose shape changes) take two work-groups per node, one per
// basis side; their sources are small and read through the caches.
#include <hip/hip_runtime.h>

#include "hss_internal.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {
namespace {

constexpr int kHB = 256;   // threads per work-group
static_assert(kMaxBlock <= kHB, "a leaf's rows fit one row group of a work-group");

// c[i] = a[i] * b[i], i < n: one 16-byte vector per thread when vec (all
// three arrays then start on 16-byte boundaries) over a grid that covers the
// array (measured at the plain-copy rate; grid-stride loops with several
// vectors in flight per thread were slower), scalars otherwise.
__global__ __launch_bounds__(kHB) void k_hadamard_diag(const double* __restrict__ a,
                                                       const double* __restrict__ b,
                                                       double* __restrict__ c, int64_t n, int vec) {
  const int64_t nth = (int64_t)gridDim.x * kHB;
  const int64_t tid = (int64_t)blockIdx.x * kHB + threadIdx.x;
  if (vec) {
    const int64_t nv = n / 2;
    const double2* a2 = reinterpret_cast<const double2*>(a);
    const double2* b2 = reinterpret_cast<const double2*>(b);
    double2* c2 = reinterpret_cast<double2*>(c);
    for (int64_t i = tid; i < nv; i += nth) {
      const double2 x = a2[i], y = b2[i];
      c2[i] = make_double2(x.x * y.x, x.y * y.y);
    }
    if (tid == 0 && (n & 1)) c[n - 1] = a[n - 1] * b[n - 1];
  } else {
    for (int64_t i = tid; i < n; i += nth) c[i] = a[i] * b[i];
  }
}

// out (m x qa qb) with out(i, a qb + b) = X(i, a) Y(i, b): the transpose
// Khatri-Rao product of X (m x qa) and Y (m x qb), column-major, ld = m for
// all three (m <= 128).  Lane i of a row group holds row i; the G = 256 / m
// row groups split the columns b of Y, so each thread loads X(i, a) once per
// a and the stores of a group are contiguous.
__device__ __forceinline__ void khatri_rao(const double* X, const double* Y, double* out, int m,
                                           int qa, int qb) {
  const int G = kHB / m;
  const int i = threadIdx.x % m, gi = threadIdx.x / m;
  if (gi >= G) return;
  for (int a = 0; a < qa; ++a) {
    const double xa = X[i + a * m];
    double* o = out + (int64_t)a * qb * m + i;
    for (int bb = gi; bb < qb; bb += G) o[bb * m] = xa * Y[i + bb * m];
  }
}

// out = X kron Y written into a block of ld rows at row offset r0:
// X is xr x xc (ld ldx), Y is yr x yc (ld ldy), out(a yr + b, c yc + d) =
// X(a, c) Y(b, d).
__device__ __forceinline__ void kron_block(const double* X, int ldx, int xr, int xc,
                                           const double* Y, int ldy, int yr, int yc, double* out,
                                           int ld, int r0) {
  const int rows = xr * yr, total = rows * xc * yc;
  for (int e = threadIdx.x; e < total; e += kHB) {
    const int col = e / rows, row = e - col * rows;
    const int a = row / yr, b = row - a * yr;
    const int c = col / yc, d = col - c * yc;
    out[r0 + row + (int64_t)col * ld] = X[a + c * ldx] * Y[b + d * ldy];
  }
}

struct HadArgs {
  const NodeInfo *nA, *nB, *nC;
  const double *AU, *AV, *AR, *AW, *AB12, *AB21;
  const double *BU, *BV, *BR, *BW, *BB12, *BB21;
  double *CU, *CV, *CR, *CW, *CB12, *CB21;
  int p;
};

// two work-groups per node (heap id = blockIdx.x): blockIdx.y = 0 forms the
// row-basis side (U, R, B12), 1 the column-basis side (V, W, B21)
__global__ __launch_bounds__(kHB) void k_hadamard_gen(HadArgs h) {
  const int t = blockIdx.x;
  const bool col = blockIdx.y != 0;
  const NodeInfo A = h.nA[t], B = h.nB[t], C = h.nC[t];
  if (A.is_leaf) {
    if (h.p == 0) return;
    if (!col) khatri_rao(h.AU + A.oU, h.BU + B.oU, h.CU + C.oU, C.m, A.ku, B.ku);
    else khatri_rao(h.AV + A.oV, h.BV + B.oV, h.CV + C.oV, C.m, A.kv, B.kv);
    return;
  }
  const int c1 = 2 * t + 1, c2 = 2 * t + 2;
  const NodeInfo A1 = h.nA[c1], A2 = h.nA[c2], B1 = h.nB[c1], B2 = h.nB[c2];
  if (!col) {
    if (t != 0) {
      // stacked [R_c1; R_c2]: one Kronecker product per child block
      const int lra = A1.ku + A2.ku, lrb = B1.ku + B2.ku, lrc = A1.ku * B1.ku + A2.ku * B2.ku;
      kron_block(h.AR + A.oR, lra, A1.ku, A.ku, h.BR + B.oR, lrb, B1.ku, B.ku, h.CR + C.oR, lrc,
                 0);
      kron_block(h.AR + A.oR + A1.ku, lra, A2.ku, A.ku, h.BR + B.oR + B1.ku, lrb, B2.ku, B.ku,
                 h.CR + C.oR, lrc, A1.ku * B1.ku);
    }
    // B12: ku_c1 x kv_c2
    kron_block(h.AB12 + A.oB12, A1.ku, A1.ku, A2.kv, h.BB12 + B.oB12, B1.ku, B1.ku, B2.kv,
               h.CB12 + C.oB12, A1.ku * B1.ku, 0);
  } else {
    if (t != 0) {
      const int lwa = A1.kv + A2.kv, lwb = B1.kv + B2.kv, lwc = A1.kv * B1.kv + A2.kv * B2.kv;
      kron_block(h.AW + A.oW, lwa, A1.kv, A.kv, h.BW + B.oW, lwb, B1.kv, B.kv, h.CW + C.oW, lwc,
                 0);
      kron_block(h.AW + A.oW + A1.kv, lwa, A2.kv, A.kv, h.BW + B.oW + B1.kv, lwb, B2.kv, B.kv,
                 h.CW + C.oW, lwc, A1.kv * B1.kv);
    }
    // B21: ku_c2 x kv_c1
    kron_block(h.AB21 + A.oB21, A2.ku, A2.ku, A1.kv, h.BB21 + B.oB21, B2.ku, B2.ku, B1.kv,
               h.CB21 + C.oB21, A2.ku * B2.ku, 0);
  }
}

}  // namespace

void launch_hadamard(const NodeInfo* nA, const NodeInfo* nB, const NodeInfo* nC,
                     const double* const gA[7], const double* const gB[7], double* const gC[7],
                     int64_t nD, int32_t nnodes, int32_t p, hipStream_t s) {
  if (nD > 0) {
    TimedLaunch tl("hadamard_diag", s);
    const bool vec = ((reinterpret_cast<uintptr_t>(gA[0]) | reinterpret_cast<uintptr_t>(gB[0]) |
                       reinterpret_cast<uintptr_t>(gC[0])) & 15) == 0;
    const int64_t items = vec ? nD / 2 : nD;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((items + kHB - 1) / kHB, 1 << 30));
    hipLaunchKernelGGL(k_hadamard_diag, dim3(grid), dim3(kHB), 0, s, gA[0], gB[0], gC[0], nD,
                       vec ? 1 : 0);
  }
  if (nnodes > 1) {
    TimedLaunch tl("hadamard_gen", s);
    HadArgs h{nA, nB, nC, gA[1], gA[2], gA[3], gA[4], gA[5], gA[6], gB[1], gB[2], gB[3],
              gB[4], gB[5], gB[6], gC[1], gC[2], gC[3], gC[4], gC[5], gC[6], p};
    hipLaunchKernelGGL(k_hadamard_gen, dim3(nnodes, 2), dim3(kHB), 0, s, h);
  }
}

}  // namespace hss
