// HSS recompression (Sec. 4.5 and App. A): proper form by bottom-up QR, then
// top-down truncated SVDs of the block rows and columns.
//
// Every launch covers one tree level (or all leaves, or all internal nodes)
// with one work-group per node and side; the node's matrices (at most
// 128 x 64 in FP64) are staged in LDS.  The work copies of the generators
// keep the input's packed layout: a block whose rank drops keeps its slot
// and leading dimension (for a stacked R, the second child's rows stay at
// their original row offset); the final gather packs the blocks at the new
// ranks.
//
//   Phase 1 (proper form), bottom-up:
//     leaves:    U = Q T (Householder QR), U <- Q, T kept per node and side
//     level l:   [T_c1 R_t,1; T_c2 R_t,2] = Q T_t, R_t <- Q  (likewise W)
//     all internal nodes at the end: B12 <- T^U_c1 B12 (T^V_c2)^T,
//                                    B21 <- T^U_c2 B21 (T^V_c1)^T
//   Phase 2, levels l = 1..p, children c of the nodes i of level l - 1:
//     row side:    SVD of [S_h | R_{i,h} diag(s_i)] (S_1 = B12_i, S_2 = B21_i)
//     column side: SVD of [S'_h | W_{i,h} diag(s'_i)] (S'_1 = B21_i^T, S'_2 = B12_i^T)
//     keep the singular values > tau (at least one), then
//     parents:  B12_i <- U1^T B12_i V2', B21_i <- U2^T B21_i V1',
//               R_{i,h} <- Uh^T R_{i,h}, W_{i,h} <- Vh'^T W_{i,h}
//     children: U_c <- U_c Uh or R_c <- R_c Uh (and V, W with Vh').
//   The SVD is one-sided Jacobi (Hestenes) on the columns of M^T: the
//   accumulated rotations are the left singular vectors of M, the column
//   norms its singular values, with high relative accuracy.
#include <hip/hip_runtime.h>

#include "hss_internal.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {
namespace {

constexpr int kCT = 256;           // threads per work-group
constexpr int kK = kMaxRank;       // slot size of a T / left-factor block (ld)
constexpr int kLR = kMaxBlock;     // largest row count of a staged block
constexpr int kLX = kLR + 1;       // LDS leading dimension of a staged block
static_assert(kK <= 64 && kLR <= 128, "staged blocks fit the LDS arrays");

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Householder QR of X (r x c, column-major, ld kLX, in LDS), r <= 128,
// c <= 64: R in the upper triangle, the reflectors below the diagonal
// (unit leading entry implicit), their scalars in tau[0 .. min(r, c)).
// H = I - tau v v^T with beta = -sign(alpha) ||x|| (no reflection when the
// part below the diagonal is zero).
__device__ void lds_qr(double* X, int r, int c, double* tau) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int kq = min(r, c);
  for (int j = 0; j < kq; ++j) {
    if (w == 0) {
      double s = 0.0;
      for (int i = j + 1 + lane; i < r; i += 64) {
        const double x = X[i + j * kLX];
        s += x * x;
      }
      s = wave_sum(s);
      const double alpha = X[j + j * kLX];
      double t = 0.0, beta = alpha, scale = 0.0;
      if (s > 0.0) {
        const double nrm = sqrt(alpha * alpha + s);
        beta = alpha >= 0.0 ? -nrm : nrm;
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int i = j + 1 + lane; i < r; i += 64) X[i + j * kLX] *= scale;
      if (lane == 0) {
        X[j + j * kLX] = beta;
        tau[j] = t;
      }
    }
    __syncthreads();
    const double t = tau[j];
    if (t != 0.0) {
      for (int l = j + 1 + w; l < c; l += 4) {
        double d = 0.0;
        for (int i = j + 1 + lane; i < r; i += 64) d += X[i + j * kLX] * X[i + l * kLX];
        d = (wave_sum(d) + X[j + l * kLX]) * t;
        for (int i = j + 1 + lane; i < r; i += 64) X[i + l * kLX] -= d * X[i + j * kLX];
        if (lane == 0) X[j + l * kLX] -= d;
      }
    }
    __syncthreads();
  }
}

// The first kq columns of Q = H_0 ... H_{kq-1} in place of the reflectors
// (the R part must have been saved).
__device__ void lds_form_q(double* X, int r, int kq, const double* tau) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = kq - 1; j >= 0; --j) {
    const double t = tau[j];
    for (int l = j + 1 + w; l < kq; l += 4) {
      double d = 0.0;
      for (int i = j + 1 + lane; i < r; i += 64) d += X[i + j * kLX] * X[i + l * kLX];
      d = (wave_sum(d) + X[j + l * kLX]) * t;
      for (int i = j + 1 + lane; i < r; i += 64) X[i + l * kLX] -= d * X[i + j * kLX];
      if (lane == 0) X[j + l * kLX] -= d;
    }
    __syncthreads();
    for (int i = tid; i < r; i += kCT) {
      const double v = X[i + j * kLX];
      X[i + j * kLX] = i < j ? 0.0 : (i == j ? 1.0 - t : -t * v);
    }
    __syncthreads();
  }
}

// QR of the staged X (r x c): T (min(r, c) x c, upper trapezoidal) to the
// slot Tout (ld kK), Q (r x min(r, c)) left in X.
__device__ void qr_to_slot(double* X, int r, int c, double* tau, double* Tout) {
  lds_qr(X, r, c, tau);
  const int kq = min(r, c);
  for (int e = threadIdx.x; e < kq * c; e += kCT) {
    const int b = e / kq, a = e - b * kq;
    Tout[a + b * kK] = a <= b ? X[a + b * kLX] : 0.0;
  }
  __syncthreads();
  lds_form_q(X, r, kq, tau);
}

// One-sided Jacobi on the k columns of G (nr x k, ld kLX, LDS), J (k x k,
// ld kK + 1, LDS) accumulating the rotations; 32 groups of 8 lanes take
// the disjoint column pairs of a round (round-robin order, k <= 64).
__device__ void lds_jacobi(double* G, int nr, int k, double* J, int* flag) {
  constexpr int LJ = kK + 1;
  const int tid = threadIdx.x, grp = tid >> 3, sl = tid & 7;
  for (int e = tid; e < k * k; e += kCT) {
    const int b = e / k, a = e - b * k;
    J[a + b * LJ] = a == b ? 1.0 : 0.0;
  }
  const int kh = k + (k & 1);
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int rd = 0; rd + 1 < kh; ++rd) {
      if (grp < kh / 2) {
        // circle method: position 0 fixed, positions 1 .. kh-1 rotate
        const int g2 = kh - 1 - grp;
        int p = grp == 0 ? 0 : 1 + (grp - 1 + rd) % (kh - 1);
        int q = 1 + (g2 - 1 + rd) % (kh - 1);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        if (q < k) {
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int i = sl; i < nr; i += 8) {
            const double x = G[i + p * kLX], y = G[i + q * kLX];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
#pragma unroll
          for (int o = 1; o < 8; o <<= 1) {
            al += __shfl_xor(al, o);
            be += __shfl_xor(be, o);
            ga += __shfl_xor(ga, o);
          }
          if (ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
            for (int i = sl; i < nr; i += 8) {
              const double x = G[i + p * kLX], y = G[i + q * kLX];
              G[i + p * kLX] = cs * x - sn * y;
              G[i + q * kLX] = sn * x + cs * y;
            }
            for (int i = sl; i < k; i += 8) {
              const double x = J[i + p * LJ], y = J[i + q * LJ];
              J[i + p * LJ] = cs * x - sn * y;
              J[i + q * LJ] = sn * x + cs * y;
            }
            if (sl == 0) *flag = 1;
          }
        }
      }
      __syncthreads();
    }
    const int more = *flag;
    __syncthreads();
    if (!more) break;
  }
}

struct CpArgs {
  const NodeInfo* nodes;   // the input's plan: original ranks, offsets, sizes
  double *U, *V, *R, *W, *B12, *B21;   // work copies, input layout
  double *TU, *TV;         // per node kK x kK: phase-1 T, then the phase-2 left factors
  double *su, *sv;         // per node kK kept singular values
  int32_t *rku, *rkv;      // ranks after phase 1
  int32_t *nku, *nkv;      // ranks after phase 2
  double tau;
  int node0;               // first heap id of the launch
};

__device__ __forceinline__ int ldR(const NodeInfo* nd, int t) {
  return nd[2 * t + 1].ku + nd[2 * t + 2].ku;
}
__device__ __forceinline__ int ldW(const NodeInfo* nd, int t) {
  return nd[2 * t + 1].kv + nd[2 * t + 2].kv;
}

// ---- phase 1 ---------------------------------------------------------------
// leaves (blockIdx.x = leaf, blockIdx.y = side)
__global__ __launch_bounds__(kCT) void k_cp_leaf_qr(CpArgs a) {
  __shared__ double X[kLX * kK];
  __shared__ double tau[kK];
  const int t = a.node0 + blockIdx.x;
  const bool col = blockIdx.y != 0;
  const NodeInfo nd = a.nodes[t];
  const int m = nd.m, k = col ? nd.kv : nd.ku;
  double* B = col ? a.V + nd.oV : a.U + nd.oU;
  for (int e = threadIdx.x; e < m * k; e += kCT) {
    const int b = e / m, i = e - b * m;
    X[i + b * kLX] = B[e];
  }
  __syncthreads();
  qr_to_slot(X, m, k, tau, (col ? a.TV : a.TU) + (int64_t)t * kK * kK);
  const int kq = min(m, k);
  for (int e = threadIdx.x; e < m * kq; e += kCT) {
    const int b = e / m, i = e - b * m;
    B[e] = X[i + b * kLX];
  }
  if (threadIdx.x == 0) (col ? a.rkv : a.rku)[t] = kq;
}

// one internal level, not the root (blockIdx.x = node - node0, blockIdx.y = side)
__global__ __launch_bounds__(kCT) void k_cp_up_qr(CpArgs a) {
  __shared__ double X[kLX * kK];
  __shared__ double tau[kK];
  const int t = a.node0 + blockIdx.x;
  const bool col = blockIdx.y != 0;
  const NodeInfo nd = a.nodes[t];
  const int c1 = 2 * t + 1, c2 = 2 * t + 2;
  const NodeInfo n1 = a.nodes[c1], n2 = a.nodes[c2];
  const int k1o = col ? n1.kv : n1.ku, k2o = col ? n2.kv : n2.ku, kt = col ? nd.kv : nd.ku;
  const int ld = k1o + k2o;
  const int32_t* rk = col ? a.rkv : a.rku;
  const int r1 = rk[c1], r2 = rk[c2], rows = r1 + r2;
  double* Rt = col ? a.W + nd.oW : a.R + nd.oR;
  const double* T1 = (col ? a.TV : a.TU) + (int64_t)c1 * kK * kK;
  const double* T2 = (col ? a.TV : a.TU) + (int64_t)c2 * kK * kK;
  // M = [T_c1 R_t,1; T_c2 R_t,2]
  for (int e = threadIdx.x; e < rows * kt; e += kCT) {
    const int j = e / rows, i = e - j * rows;
    double s = 0.0;
    if (i < r1) {
      for (int b = 0; b < k1o; ++b) s += T1[i + b * kK] * Rt[b + j * ld];
    } else {
      for (int b = 0; b < k2o; ++b) s += T2[(i - r1) + b * kK] * Rt[k1o + b + j * ld];
    }
    X[i + j * kLX] = s;
  }
  __syncthreads();
  qr_to_slot(X, rows, kt, tau, (col ? a.TV : a.TU) + (int64_t)t * kK * kK);
  const int kq = min(rows, kt);
  // Q back to the slot: the second child's rows at their original offset
  for (int e = threadIdx.x; e < rows * kq; e += kCT) {
    const int j = e / rows, i = e - j * rows;
    Rt[(i < r1 ? i : k1o + i - r1) + j * ld] = X[i + j * kLX];
  }
  if (threadIdx.x == 0) (col ? a.rkv : a.rku)[t] = kq;
}

constexpr int kLS = kK + 1;        // LDS leading dimension of a staged rank x rank block

// out (rows x cols, ld ldo) = L (rows x inner) * Bm (inner x mid) * Rm (mid x cols),
// all dimensions <= kK, with element accessors; Bm staged in Xs, the
// partial product in Ys.
template <typename FL, typename FB, typename FR>
__device__ void sandwich(double* Xs, double* Ys, int rows, int inner, int mid, int cols, FL L, FB Bm,
                         FR Rm, double* out, int ldo) {
  for (int e = threadIdx.x; e < inner * mid; e += kCT) {
    const int j = e / inner, i = e - j * inner;
    Xs[i + j * kLS] = Bm(i, j);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * mid; e += kCT) {
    const int j = e / rows, i = e - j * rows;
    double s = 0.0;
    for (int x = 0; x < inner; ++x) s += L(i, x) * Xs[x + j * kLS];
    Ys[i + j * kLS] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * cols; e += kCT) {
    const int j = e / rows, i = e - j * rows;
    double s = 0.0;
    for (int x = 0; x < mid; ++x) s += Ys[i + x * kLS] * Rm(x, j);
    out[i + (int64_t)j * ldo] = s;
  }
  __syncthreads();
}

// all internal nodes: the core blocks in the orthonormal bases
__global__ __launch_bounds__(kCT) void k_cp_core(CpArgs a) {
  __shared__ double Xs[kLS * kK];
  __shared__ double Ys[kLS * kK];
  const int t = a.node0 + blockIdx.x;
  const NodeInfo nd = a.nodes[t];
  const int c1 = 2 * t + 1, c2 = 2 * t + 2;
  const NodeInfo n1 = a.nodes[c1], n2 = a.nodes[c2];
  for (int which = 0; which < 2; ++which) {
    // B12: rows c1 (U side), columns c2 (V side); B21: rows c2, columns c1
    const int cr = which ? c2 : c1, cc = which ? c1 : c2;
    const NodeInfo& nr = which ? n2 : n1;
    const NodeInfo& nc = which ? n1 : n2;
    double* Bp = which ? a.B21 + nd.oB21 : a.B12 + nd.oB12;
    const int ld = nr.ku;
    const double* TL = a.TU + (int64_t)cr * kK * kK;
    const double* TR = a.TV + (int64_t)cc * kK * kK;
    sandwich(
        Xs, Ys, a.rku[cr], nr.ku, nc.kv, a.rkv[cc], [&](int i, int x) { return TL[i + x * kK]; },
        [&](int i, int j) { return Bp[i + j * ld]; },
        [&](int x, int j) { return TR[j + x * kK]; }, Bp, ld);
  }
}

// ---- phase 2 ---------------------------------------------------------------
// one level of children (blockIdx.x = child - node0, blockIdx.y = side): the
// truncated SVD of the child's block row (side 0) or block column (side 1)
__global__ __launch_bounds__(kCT) void k_cp_svd(CpArgs a) {
  __shared__ double G[kLX * kK];
  __shared__ double J[(kK + 1) * kK];
  __shared__ double sig[kK];
  __shared__ int flag, keep_s;
  const int c = a.node0 + blockIdx.x;
  const bool col = blockIdx.y != 0;
  const int i = (c - 1) / 2;
  const int h = c == 2 * i + 1 ? 0 : 1;
  const int c1 = 2 * i + 1, c2 = 2 * i + 2;
  const NodeInfo ni = a.nodes[i], n1 = a.nodes[c1], n2 = a.nodes[c2];
  const int k = col ? a.rkv[c] : a.rku[c];
  int ns, nkp = 0;
  if (!col) {
    // G = M^T, M = [S_h | R_{i,h} diag(s_i)]; S_0 = B12_i, S_1 = B21_i
    const double* S = h == 0 ? a.B12 + ni.oB12 : a.B21 + ni.oB21;
    const int lds = h == 0 ? n1.ku : n2.ku;
    ns = h == 0 ? a.rkv[c2] : a.rkv[c1];
    for (int e = threadIdx.x; e < k * ns; e += kCT) {
      const int r = e / k, x = e - r * k;
      G[r + x * kLX] = S[x + r * lds];
    }
    if (i != 0) {
      nkp = a.nku[i];
      const int ld = ldR(a.nodes, i), off = h == 0 ? 0 : n1.ku;
      const double* Rb = a.R + ni.oR + off;
      const double* s = a.su + (int64_t)i * kK;
      for (int e = threadIdx.x; e < k * nkp; e += kCT) {
        const int j = e / k, x = e - j * k;
        G[ns + j + x * kLX] = Rb[x + j * ld] * s[j];
      }
    }
  } else {
    // G = M'^T, M' = [S'_h | W_{i,h} diag(s'_i)]; S'_0 = B21_i^T, S'_1 = B12_i^T
    const double* S = h == 0 ? a.B21 + ni.oB21 : a.B12 + ni.oB12;
    const int lds = h == 0 ? n2.ku : n1.ku;
    ns = h == 0 ? a.rku[c2] : a.rku[c1];
    for (int e = threadIdx.x; e < k * ns; e += kCT) {
      const int x = e / ns, r = e - x * ns;
      G[r + x * kLX] = S[r + x * lds];
    }
    if (i != 0) {
      nkp = a.nkv[i];
      const int ld = ldW(a.nodes, i), off = h == 0 ? 0 : n1.kv;
      const double* Wb = a.W + ni.oW + off;
      const double* s = a.sv + (int64_t)i * kK;
      for (int e = threadIdx.x; e < k * nkp; e += kCT) {
        const int j = e / k, x = e - j * k;
        G[ns + j + x * kLX] = Wb[x + j * ld] * s[j];
      }
    }
  }
  const int nr = ns + nkp;
  __syncthreads();
  lds_jacobi(G, nr, k, J, &flag);
  // singular values = column norms of G
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int x = w; x < k; x += 4) {
    double s = 0.0;
    for (int r = lane; r < nr; r += 64) s += G[r + x * kLX] * G[r + x * kLX];
    s = wave_sum(s);
    if (lane == 0) sig[x] = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int keep = 0;
    for (int x = 0; x < k; ++x) keep += sig[x] > a.tau ? 1 : 0;
    if (k > 0 && keep == 0) keep = 1;
    keep_s = keep;
    (col ? a.nkv : a.nku)[c] = keep;
  }
  __syncthreads();
  const int keep = keep_s;
  // order by decreasing singular value (ties by index); the kept columns of
  // the rotations are the new left factor
  double* F = (col ? a.TV : a.TU) + (int64_t)c * kK * kK;
  double* sout = (col ? a.sv : a.su) + (int64_t)c * kK;
  for (int x = threadIdx.x; x < k; x += kCT) {
    const double sx = sig[x];
    int pos = 0;
    for (int y = 0; y < k; ++y) pos += (sig[y] > sx || (sig[y] == sx && y < x)) ? 1 : 0;
    if (pos < keep) {
      sout[pos] = sx;
      for (int r = 0; r < k; ++r) F[r + pos * kK] = J[r + x * (kK + 1)];
    }
  }
}

// the parents of one level (blockIdx.x = parent - node0): core blocks and
// translation-operator rows in the truncated bases of their children
__global__ __launch_bounds__(kCT) void k_cp_apply_parent(CpArgs a) {
  __shared__ double Xs[kLS * kK];
  __shared__ double Ys[kLS * kK];
  const int i = a.node0 + blockIdx.x;
  const NodeInfo ni = a.nodes[i];
  const int c1 = 2 * i + 1, c2 = 2 * i + 2;
  const NodeInfo n1 = a.nodes[c1], n2 = a.nodes[c2];
  for (int which = 0; which < 2; ++which) {
    const int cr = which ? c2 : c1, cc = which ? c1 : c2;
    const NodeInfo& nr = which ? n2 : n1;
    double* Bp = which ? a.B21 + ni.oB21 : a.B12 + ni.oB12;
    const int ld = nr.ku;
    const double* FU = a.TU + (int64_t)cr * kK * kK;
    const double* FV = a.TV + (int64_t)cc * kK * kK;
    sandwich(
        Xs, Ys, a.nku[cr], a.rku[cr], a.rkv[cc], a.nkv[cc],
        [&](int r, int x) { return FU[x + r * kK]; }, [&](int r, int j) { return Bp[r + j * ld]; },
        [&](int x, int j) { return FV[x + j * kK]; }, Bp, ld);
  }
  if (i == 0) return;
  for (int side = 0; side < 2; ++side) {
    const bool col = side != 0;
    double* Rt = col ? a.W + ni.oW : a.R + ni.oR;
    const int ld = col ? ldW(a.nodes, i) : ldR(a.nodes, i);
    const int ncol = col ? a.nkv[i] : a.nku[i];
    for (int h = 0; h < 2; ++h) {
      const int c = h ? c2 : c1;
      const int off = h ? (col ? n1.kv : n1.ku) : 0;
      const int kin = col ? a.rkv[c] : a.rku[c], kout = col ? a.nkv[c] : a.nku[c];
      const double* F = (col ? a.TV : a.TU) + (int64_t)c * kK * kK;
      double* blk = Rt + off;
      for (int e = threadIdx.x; e < kin * ncol; e += kCT) {
        const int j = e / kin, x = e - j * kin;
        Xs[x + j * kLS] = blk[x + j * ld];
      }
      __syncthreads();
      for (int e = threadIdx.x; e < kout * ncol; e += kCT) {
        const int j = e / kout, r = e - j * kout;
        double s = 0.0;
        for (int x = 0; x < kin; ++x) s += F[x + r * kK] * Xs[x + j * kLS];
        blk[r + j * ld] = s;
      }
      __syncthreads();
    }
  }
}

// the children of one level (blockIdx.x = child - node0, blockIdx.y = side):
// U <- U Uh at a leaf, R <- R Uh at an internal node (likewise V, W)
__global__ __launch_bounds__(kCT) void k_cp_apply_child(CpArgs a) {
  __shared__ double Xs[kLX * kK];
  const int c = a.node0 + blockIdx.x;
  const bool col = blockIdx.y != 0;
  const NodeInfo nc = a.nodes[c];
  double* X;
  int rows;
  if (nc.is_leaf) {
    X = col ? a.V + nc.oV : a.U + nc.oU;
    rows = nc.m;
  } else {
    X = col ? a.W + nc.oW : a.R + nc.oR;
    rows = col ? ldW(a.nodes, c) : ldR(a.nodes, c);
  }
  const int kin = col ? a.rkv[c] : a.rku[c], kout = col ? a.nkv[c] : a.nku[c];
  const double* F = (col ? a.TV : a.TU) + (int64_t)c * kK * kK;
  for (int e = threadIdx.x; e < rows * kin; e += kCT) {
    const int j = e / rows, r = e - j * rows;
    Xs[r + j * kLX] = X[e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * kout; e += kCT) {
    const int j = e / rows, r = e - j * rows;
    double s = 0.0;
    for (int x = 0; x < kin; ++x) s += Xs[r + x * kLX] * F[x + j * kK];
    X[e] = s;
  }
}

// ---- gather ----------------------------------------------------------------
struct GatherArgs {
  const NodeInfo* in;    // input plan (work layout)
  const NodeInfo* out;   // output plan
  const double *U, *V, *R, *W, *B12, *B21;
  double *oU, *oV, *oR, *oW, *oB12, *oB21;
};

__device__ void copy_block(const double* src, int ld_src, double* dst, int ld_dst, int rows,
                           int cols, int r_src, int r_dst) {
  for (int e = threadIdx.x; e < rows * cols; e += kCT) {
    const int j = e / rows, i = e - j * rows;
    dst[r_dst + i + (int64_t)j * ld_dst] = src[r_src + i + (int64_t)j * ld_src];
  }
}

// one work-group per node
__global__ __launch_bounds__(kCT) void k_cp_gather(GatherArgs g) {
  const int t = blockIdx.x;
  const NodeInfo a = g.in[t], b = g.out[t];
  if (a.is_leaf) {
    if (a.oU < 0) return;
    copy_block(g.U + a.oU, a.m, g.oU + b.oU, b.m, b.m, b.ku, 0, 0);
    copy_block(g.V + a.oV, a.m, g.oV + b.oV, b.m, b.m, b.kv, 0, 0);
    return;
  }
  const NodeInfo a1 = g.in[2 * t + 1], a2 = g.in[2 * t + 2];
  const NodeInfo b1 = g.out[2 * t + 1], b2 = g.out[2 * t + 2];
  if (t != 0) {
    const int lai = a1.ku + a2.ku, lbo = b1.ku + b2.ku;
    copy_block(g.R + a.oR, lai, g.oR + b.oR, lbo, b1.ku, b.ku, 0, 0);
    copy_block(g.R + a.oR, lai, g.oR + b.oR, lbo, b2.ku, b.ku, a1.ku, b1.ku);
    const int lwi = a1.kv + a2.kv, lwo = b1.kv + b2.kv;
    copy_block(g.W + a.oW, lwi, g.oW + b.oW, lwo, b1.kv, b.kv, 0, 0);
    copy_block(g.W + a.oW, lwi, g.oW + b.oW, lwo, b2.kv, b.kv, a1.kv, b1.kv);
  }
  copy_block(g.B12 + a.oB12, a1.ku, g.oB12 + b.oB12, b1.ku, b1.ku, b2.kv, 0, 0);
  copy_block(g.B21 + a.oB21, a2.ku, g.oB21 + b.oB21, b2.ku, b2.ku, b1.kv, 0, 0);
}

}  // namespace

void launch_compress(CompressStep step, const CompressBufs& b, int node0, int count, double tau,
                     hipStream_t s) {
  if (count <= 0) return;
  CpArgs a{b.nodes, b.U,   b.V,   b.R,   b.W,   b.B12, b.B21, b.TU, b.TV,
           b.su,    b.sv,  b.rku, b.rkv, b.nku, b.nkv, tau,   node0};
  switch (step) {
    case CompressStep::LeafQR: {
      TimedLaunch tl("compress_leaf_qr", s);
      hipLaunchKernelGGL(k_cp_leaf_qr, dim3(count, 2), dim3(kCT), 0, s, a);
      break;
    }
    case CompressStep::UpQR: {
      TimedLaunch tl("compress_up_qr", s);
      hipLaunchKernelGGL(k_cp_up_qr, dim3(count, 2), dim3(kCT), 0, s, a);
      break;
    }
    case CompressStep::Core: {
      TimedLaunch tl("compress_core", s);
      hipLaunchKernelGGL(k_cp_core, dim3(count), dim3(kCT), 0, s, a);
      break;
    }
    case CompressStep::Svd: {
      TimedLaunch tl("compress_svd", s);
      hipLaunchKernelGGL(k_cp_svd, dim3(count, 2), dim3(kCT), 0, s, a);
      break;
    }
    case CompressStep::ApplyParent: {
      TimedLaunch tl("compress_apply", s);
      hipLaunchKernelGGL(k_cp_apply_parent, dim3(count), dim3(kCT), 0, s, a);
      break;
    }
    case CompressStep::ApplyChild: {
      TimedLaunch tl("compress_apply", s);
      hipLaunchKernelGGL(k_cp_apply_child, dim3(count, 2), dim3(kCT), 0, s, a);
      break;
    }
  }
}

void launch_compress_gather(const NodeInfo* in, const NodeInfo* out, const double* const work[6],
                            double* const dst[6], int nnodes, hipStream_t s) {
  TimedLaunch tl("compress_gather", s);
  GatherArgs g{in,      out,     work[0], work[1], work[2], work[3], work[4], work[5],
               dst[0],  dst[1],  dst[2],  dst[3],  dst[4],  dst[5]};
  hipLaunchKernelGGL(k_cp_gather, dim3(nnodes), dim3(kCT), 0, s, g);
}

}  // namespace hss
