// Dense-to-HSS construction (Sec. 3.2, the dense constructor): truncated
// SVDs of the HSS block rows and columns from the leaves to the root.
//
// The host drives the levels; these kernels are its steps:
//   k_cn_trunc   one work-group per block row H (r <= 128 rows of a
//                column-major matrix X, every column of X outside one
//                excluded range): the left singular vectors and values of H.
//                H^T is reduced to its triangular factor by a streaming
//                Householder QR (128 columns of H at a time below the
//                128 x 128 triangle, which stays in LDS), then one-sided
//                Jacobi (Hestenes) orthogonalizes the rows of that factor:
//                H = T^T Q^T, so H's left singular pairs are those of T^T,
//                whose rotated columns, normalized, are the left singular
//                vectors (high relative accuracy; no Q, no V is formed).
//                Keeps sigma > eps * sigma_1, at least one.
//   k_cn_rmul    Y(:, block j) = X(:, block j) B_j for a list of blocks (the
//                products with blkdiag(V_j) or blkdiag(W_t))
//   k_cn_trans   Y = X^T (tiles through LDS)
//   k_cn_copy    a list of small column-major block copies (the packed
//                generators at the end)
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "hss_internal.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {
namespace {

constexpr int kQT = 1024;          // threads of k_cn_trunc
constexpr int kQR = kCnMaxRows;    // largest block row (rows)
constexpr int kRP = kQR + 1;       // LDS row stride of the triangle (bank spread)
constexpr int kCH = 128;           // columns of H per streaming step
constexpr int kTR = 8;             // threads per row of H
constexpr int kHC = kCH / kTR;     // columns of H per thread and step
static_assert(kQR == 128 && kQT == kTR * kQR, "eight threads per row of the block");

// sum over the 8 lanes of an aligned group: quad permutes, then the other
// quad of the group by a row shift of 4 (left in the low quad, right in the
// high one)
__device__ __forceinline__ double oct_sum(double x, int lane) {
  x += dpp<kDppQuadXor1>(x);
  x += dpp<kDppQuadXor2>(x);
  const double lo = dpp<0x104>(x);   // row_shl:4
  const double hi = dpp<0x114>(x);   // row_shr:4
  return x + ((lane & 4) ? hi : lo);
}

__device__ __forceinline__ int64_t cn_col(int64_t q, int64_t ex0, int64_t ex1) {
  return q < ex0 ? q : q + (ex1 - ex0);
}

// Round-robin pair of slot i in round s over an even number e of indices:
// every pair meets once in e - 1 rounds.
__device__ __forceinline__ void rr_pair(int i, int s, int e, int& a, int& b) {
  const int m = e - 1;
  a = i == 0 ? 0 : (i - 1 + s) % m + 1;
  b = (e - 2 - i + s) % m + 1;
}

__global__ __launch_bounds__(kQT) void k_cn_trunc(const CnTask* tasks, double eps) {
  __shared__ double R[kQR * kRP];
  // reflector entries: chunk row h * kHC + i at (i / 2) * 2 kTR + 2 h + i % 2 (a
  // thread's pairs adjacent for 16-byte accesses, the eight threads of a row
  // on distinct banks)
  __shared__ __align__(16) double vb[2][kCH];
  __shared__ double tb[2];
  __shared__ double sig[kQR];
  __shared__ int flag;
  const CnTask tk = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int c = tid >> 3, h = tid & 7;   // row c of H (column c of H^T), eighth h of a chunk
  const int lane = tid & 63;
  const int r = tk.r;
  for (int i = tid; i < kQR * kRP; i += kQT) R[i] = 0.0;
  __syncthreads();
  // ---- streaming QR of H^T: [T; next 128 columns of H, transposed] = Q T'
  const int64_t nc = tk.ncols - (tk.ex1 - tk.ex0);
  const double* xr = tk.X + tk.row0 + c;
  double v[kHC];
  for (int64_t q0 = 0; q0 < nc; q0 += kCH) {
#pragma unroll
    for (int i = 0; i < kHC; ++i) {
      const int64_t q = q0 + h * kHC + i;
      v[i] = (c < r && q < nc) ? xr[cn_col(q, tk.ex0, tk.ex1) * tk.ld] : 0.0;
    }
    for (int j = 0; j < r; ++j) {
      const int b = j & 1;
      if (c == j) {
        // four independent partial sums: the chains, not the issue rate, bound a step
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < kHC; ++i) s4[i & 3] += v[i] * v[i];
        const double ss = oct_sum((s4[0] + s4[1]) + (s4[2] + s4[3]), lane);
        const double alpha = R[j * kRP + j];
        double tau = 0.0, inv = 0.0;
        if (ss > 0.0) {
          const double nrm = sqrt(alpha * alpha + ss);
          const double beta = alpha >= 0.0 ? -nrm : nrm;
          inv = 1.0 / (alpha - beta);
          tau = (beta - alpha) / beta;
          if (h == 0) R[j * kRP + j] = beta;
        }
#pragma unroll
        for (int i = 0; i < kHC; ++i) vb[b][(i >> 1) * (2 * kTR) + 2 * h + (i & 1)] = v[i] * inv;
        if (h == 0) tb[b] = tau;
      }
      __syncthreads();
      const double tau = tb[b];
      if (c > j && c < r && tau != 0.0) {
        double w4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < kHC; ++i) w4[i & 3] += vb[b][(i >> 1) * (2 * kTR) + 2 * h + (i & 1)] * v[i];
        double w = oct_sum((w4[0] + w4[1]) + (w4[2] + w4[3]), lane);
        w = tau * (w + R[j * kRP + c]);
        if (h == 0) R[j * kRP + c] -= w;
#pragma unroll
        for (int i = 0; i < kHC; ++i) v[i] -= w * vb[b][(i >> 1) * (2 * kTR) + 2 * h + (i & 1)];
      }
    }
    __syncthreads();
  }
  // ---- one-sided Jacobi on the rows of the triangle (columns of T^T)
  const int e = (r + 1) & ~1;   // an odd count gets a zero row as partner
  const int pr = tid >> 4, sub = tid & 15;   // 64 pairs x 16 lanes
  const double tol = 2.5e-15;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int s = 0; s < e - 1; ++s) {
      if (pr < e / 2) {
        int a, b;
        rr_pair(pr, s, e, a, b);
        double* ra = R + a * kRP;
        double* rb = R + b * kRP;
        double aa = 0.0, bb = 0.0, ab = 0.0;
        for (int x = sub; x < r; x += 16) {
          const double p = ra[x], q = rb[x];
          aa += p * p;
          bb += q * q;
          ab += p * q;
        }
        aa = oct_sum(aa, lane);
        bb = oct_sum(bb, lane);
        ab = oct_sum(ab, lane);
        aa += dpp<kDppRowRor8>(aa);   // the other half of the row of 16
        bb += dpp<kDppRowRor8>(bb);
        ab += dpp<kDppRowRor8>(ab);
        if (ab != 0.0 && fabs(ab) > tol * sqrt(aa) * sqrt(bb)) {
          const double zeta = (bb - aa) / (2.0 * ab);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int x = sub; x < r; x += 16) {
            const double p = ra[x], q = rb[x];
            ra[x] = cs * p - sn * q;
            rb[x] = sn * p + cs * q;
          }
          if (sub == 0) flag = 1;
        }
      }
      __syncthreads();
    }
    if (flag == 0) break;
    __syncthreads();
  }
  // ---- singular values (row norms), order, kept count, normalized vectors
  if (tid < r) {
    double s2 = 0.0;
    for (int x = 0; x < r; ++x) s2 += R[tid * kRP + x] * R[tid * kRP + x];
    sig[tid] = sqrt(s2);
  }
  __syncthreads();
  double smax = 0.0;
  for (int x = 0; x < r; ++x) smax = fmax(smax, sig[x]);
  int keep = 0;
  for (int x = 0; x < r; ++x) keep += sig[x] > eps * smax ? 1 : 0;
  if (keep == 0) keep = 1;
  if (tid == 0) *tk.rank = keep;
  if (tid < r) {
    const double sx = sig[tid];
    int pos = 0;
    for (int y = 0; y < r; ++y) pos += (sig[y] > sx || (sig[y] == sx && y < tid)) ? 1 : 0;
    tk.sig[pos] = sx;
    double* u = tk.U + (int64_t)pos * kQR;
    if (smax == 0.0) {
      for (int x = 0; x < r; ++x) u[x] = (x == pos) ? 1.0 : 0.0;
    } else {
      const double inv = sx > 0.0 ? 1.0 / sx : 0.0;
      for (int x = 0; x < r; ++x) u[x] = R[tid * kRP + x] * inv;
    }
  }
}

// Y(:, ycol0 + 0..k) = X(:, xcol0 + 0..s) B: 64 rows x up to 64 columns per
// work-group, 4 x 4 outputs per thread, the inner dimension in steps of 32
// through LDS.
constexpr int kMT = 64, kMK = 32;
__global__ __launch_bounds__(256) void k_cn_rmul(const CnRmul* tasks) {
  __shared__ double Xs[kMK][kMT + 1];
  __shared__ double Bs[kMK][kMT + 1];
  const CnRmul tk = tasks[blockIdx.y];
  const int64_t row0 = (int64_t)blockIdx.x * kMT;
  if (row0 >= tk.rows) return;
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  double acc[4][4] = {};
  for (int s0 = 0; s0 < tk.s; s0 += kMK) {
    const int sl = min(kMK, tk.s - s0);
    for (int e = tid; e < kMK * kMT; e += 256) {
      const int i = e & (kMT - 1), q = e >> 6;
      const int64_t row = row0 + i;
      Xs[q][i] = (q < sl && row < tk.rows) ? tk.X[row + (tk.xcol0 + s0 + q) * tk.ldx] : 0.0;
      const int j = e & (kMT - 1);
      Bs[q][j] = (q < sl && j < tk.k) ? tk.B[(s0 + q) + (int64_t)j * tk.ldb] : 0.0;
    }
    __syncthreads();
    for (int q = 0; q < sl; ++q) {
      double xa[4], ba[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xa[u] = Xs[q][tr + 16 * u];
        ba[u] = Bs[q][tc + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[u][w] += xa[u] * ba[w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int j = tc + 16 * w;
    if (j >= tk.k) continue;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = row0 + tr + 16 * u;
      if (row < tk.rows) tk.Y[row + (tk.ycol0 + j) * tk.ldy] = acc[u][w];
    }
  }
}

constexpr int kTT = 32;
__global__ __launch_bounds__(256) void k_cn_trans(const double* X, int64_t ldx, int64_t rows,
                                                  int64_t cols, double* Y, int64_t ldy) {
  __shared__ double t[kTT][kTT + 1];
  const int64_t r0 = (int64_t)blockIdx.x * kTT, c0 = (int64_t)blockIdx.y * kTT;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < kTT; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    t[j][tx] = (r < rows && c < cols) ? X[r + c * ldx] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < kTT; j += 8) {
    const int64_t c = c0 + tx, r = r0 + j;
    if (r < rows && c < cols) Y[c + r * ldy] = t[tx][j];
  }
}

__global__ __launch_bounds__(256) void k_cn_copy(const CnCopy* tasks) {
  const CnCopy tk = tasks[blockIdx.x];
  const int64_t n = (int64_t)tk.rows * tk.cols;
  for (int64_t e = threadIdx.x; e < n; e += 256) {
    const int64_t j = e / tk.rows, i = e - j * tk.rows;
    tk.dst[e] = tk.src[i + j * tk.lds];
  }
}

}  // namespace

void launch_cn_trunc(const CnTask* tasks, int count, double eps, bool leaves, hipStream_t s) {
  if (count <= 0) return;
  TimedLaunch tl(leaves ? "construct_trunc_leaf" : "construct_trunc", s);
  hipLaunchKernelGGL(k_cn_trunc, dim3(count), dim3(kQT), 0, s, tasks, eps);
}

void launch_cn_rmul(const CnRmul* tasks, int count, int64_t rows, hipStream_t s) {
  if (count <= 0 || rows <= 0) return;
  TimedLaunch tl("construct_rmul", s);
  hipLaunchKernelGGL(k_cn_rmul, dim3((unsigned)((rows + kMT - 1) / kMT), count), dim3(256), 0, s,
                     tasks);
}

void launch_cn_trans(const double* X, int64_t ldx, int64_t rows, int64_t cols, double* Y,
                     int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  TimedLaunch tl("construct_transpose", s);
  hipLaunchKernelGGL(k_cn_trans, dim3((unsigned)((rows + kTT - 1) / kTT), (unsigned)((cols + kTT - 1) / kTT)),
                     dim3(256), 0, s, X, ldx, rows, cols, Y, ldy);
}

void launch_cn_copy(const CnCopy* tasks, int count, hipStream_t s) {
  if (count <= 0) return;
  TimedLaunch tl("construct_gather", s);
  hipLaunchKernelGGL(k_cn_copy, dim3(count), dim3(256), 0, s, tasks);
}

}  // namespace hss
