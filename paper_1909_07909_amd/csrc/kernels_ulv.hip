// Implicit ULV factorization and solve (Sec. 4.3), telescoped into one
// sibling correction per node.
//
// Factor, per node t (leaves first, then each merged level):
//   merge (internal t): D' = [[D~22_c1, U~_c1 B12_t V^b_c2^T],
//                             [U~_c2 B21_t V^b_c1^T, D~22_c2]],
//                       U' = blkdiag(U~_c1, U~_c2) R_t,
//                       V' = blkdiag(V^b_c1, V^b_c2) W_t          (Step 3)
//   factor: QL of U' (Householder, pivots at the bottom): Q^T U' = [0; U~];
//           M = Q^T D'; LQ of the leading e rows: M Z = [[L, 0], [D~21, D~22]];
//           V^ = Z^T V' (Step 1 on the merged leaf)
//   root:   LU with partial pivoting of D'_root, always FP64.
// Solve (telescoped Steps 2 and 4):
//   forward, leaves then levels: rhs_t = b_i (leaf) or
//       [c_c1 - U~_c1 B12_t z_c2; c_c2 - U~_c2 B21_t z_c1] (internal);
//       b~ = Q^T rhs; y = L^{-1} b~_top; c_t = b~_bot - D~21 y;
//       z_t = V^_top^T y (+ W_t^T [z_c1; z_c2] at internal nodes)
//   root: x'_root = LU \ rhs_root, split into x^_c1, x^_c2
//   backward, levels then leaves: x'_t = Z_t [y_t; x^_t], split to children
//       (leaves: written to B).
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {


// U~ of node n as a kept x ku matrix: trailing kept rows of FU; when rows were
// eliminated the entries above the diagonal of U~ hold reflector data and
// read as zero.
template <typename T>
__device__ __forceinline__ T utilde(const T* FU, const NodeInfo& n, int a, int x) {
  if (n.e > 0 && a < x) return T(0);
  return FU[n.e + a + (int64_t)x * n.mp];
}

// ---------------------------------------------------------------------------
// Merge two factored children into the block of their parent (Step 3).
// Every product is a small GEMM on operands staged in LDS (ld kMaxRank + 1).
// ---------------------------------------------------------------------------
template <typename T, typename F>
__device__ __forceinline__ void stage(int M, int N, F f, T* dst) {
  constexpr int ld = kMaxRank + 1;
  if (M <= 0 || N <= 0) return;
  wg_stage<8, T>(M, N, f, [&](int i, int j, T v) { dst[i + j * ld] = v; });
}

// out(i, j) = sum_l A(i, l) B(l, j) (TB: B(l, j) = Bs[j + l*ld]), A, B in LDS
template <typename T, bool TB, typename FC>
__device__ __forceinline__ void lds_gemm(int M, int N, int K, const T* As, const T* Bs, FC fc) {
  constexpr int ld = kMaxRank + 1;
  for (int o = threadIdx.x; o < M * N; o += blockDim.x) {
    const int i = o % M, j = o / M;
    T acc = 0;
    for (int l = 0; l < K; ++l) acc += As[i + l * ld] * (TB ? Bs[j + l * ld] : Bs[l + j * ld]);
    fc(i, j, acc);
  }
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_ulv_merge(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  constexpr int ld = kMaxRank + 1;
  const NodeInfo nd = I.nodes[node];
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int k1 = n1.kept, k2 = n2.kept, mp = nd.mp;
  const T* FD1 = I.FD + n1.oFD; const T* FD2 = I.FD + n2.oFD;
  const T* FU1 = I.FU + n1.oFU; const T* FU2 = I.FU + n2.oFU;
  const T* FV1 = I.FV + n1.oFV; const T* FV2 = I.FV + n2.oFV;
  T* FD = I.FD + nd.oFD;
  T* As = smem;
  T* Bs = As + kMaxRank * ld;
  T* Cs = Bs + kMaxRank * ld;
  // diagonal blocks D~22 of the children
  if (k1 > 0)
    wg_stage<8, T>(k1, k1, [&](int i, int j) { return FD1[n1.e + i + (int64_t)(n1.e + j) * n1.mp]; },
                   [&](int i, int j, T v) { FD[i + (int64_t)j * mp] = v; });
  if (k2 > 0)
    wg_stage<8, T>(k2, k2, [&](int i, int j) { return FD2[n2.e + i + (int64_t)(n2.e + j) * n2.mp]; },
                   [&](int i, int j, T v) { FD[k1 + i + (int64_t)(k1 + j) * mp] = v; });
  const T* B12 = I.B12 + nd.oB12;
  const T* B21 = I.B21 + nd.oB21;
  auto ut1 = [&](int i, int x) {
    const T v = FU1[n1.e + i + (int64_t)x * n1.mp];
    return ((n1.e > 0) & (i < x)) ? T(0) : v;
  };
  auto ut2 = [&](int i, int x) {
    const T v = FU2[n2.e + i + (int64_t)x * n2.mp];
    return ((n2.e > 0) & (i < x)) ? T(0) : v;
  };
  auto vb1 = [&](int i, int x) { return FV1[n1.e + i + (int64_t)x * n1.mp]; };
  auto vb2 = [&](int i, int x) { return FV2[n2.e + i + (int64_t)x * n2.mp]; };
  // D'(c1, c2) = U~_c1 (B12 V^b_c2^T)
  stage<T>(n1.ku, n2.kv, [&](int i, int j) { return B12[i + (int64_t)j * n1.ku]; }, As);
  stage<T>(k2, n2.kv, vb2, Bs);
  __syncthreads();
  lds_gemm<T, true>(n1.ku, k2, n2.kv, As, Bs, [&](int i, int j, T v) { Cs[i + j * ld] = v; });
  __syncthreads();
  stage<T>(k1, n1.ku, ut1, As);
  __syncthreads();
  lds_gemm<T, false>(k1, k2, n1.ku, As, Cs,
                     [&](int i, int j, T v) { FD[i + (int64_t)(k1 + j) * mp] = v; });
  __syncthreads();
  // D'(c2, c1) = U~_c2 (B21 V^b_c1^T)
  stage<T>(n2.ku, n1.kv, [&](int i, int j) { return B21[i + (int64_t)j * n2.ku]; }, As);
  stage<T>(k1, n1.kv, vb1, Bs);
  __syncthreads();
  lds_gemm<T, true>(n2.ku, k1, n1.kv, As, Bs, [&](int i, int j, T v) { Cs[i + j * ld] = v; });
  __syncthreads();
  stage<T>(k2, n2.ku, ut2, As);
  __syncthreads();
  lds_gemm<T, false>(k2, k1, n2.ku, As, Cs,
                     [&](int i, int j, T v) { FD[k1 + i + (int64_t)j * mp] = v; });
  if (node == 0) return;
  __syncthreads();
  // U' = blkdiag(U~_c1, U~_c2) R_t, V' = blkdiag(V^b_c1, V^b_c2) W_t
  const T* R = I.R + nd.oR;
  const T* W = I.W + nd.oW;
  const int kr = n1.ku + n2.ku, kw = n1.kv + n2.kv;
  T* FU = I.FU + nd.oFU;
  T* FV = I.FV + nd.oFV;
  stage<T>(k1, n1.ku, ut1, As);
  stage<T>(n1.ku, nd.ku, [&](int i, int j) { return R[i + (int64_t)j * kr]; }, Bs);
  stage<T>(k2, n2.ku, ut2, Cs);
  __syncthreads();
  lds_gemm<T, false>(k1, nd.ku, n1.ku, As, Bs,
                     [&](int i, int j, T v) { FU[i + (int64_t)j * mp] = v; });
  __syncthreads();
  stage<T>(n2.ku, nd.ku, [&](int i, int j) { return R[n1.ku + i + (int64_t)j * kr]; }, Bs);
  __syncthreads();
  lds_gemm<T, false>(k2, nd.ku, n2.ku, Cs, Bs,
                     [&](int i, int j, T v) { FU[k1 + i + (int64_t)j * mp] = v; });
  __syncthreads();
  stage<T>(k1, n1.kv, vb1, As);
  stage<T>(n1.kv, nd.kv, [&](int i, int j) { return W[i + (int64_t)j * kw]; }, Bs);
  stage<T>(k2, n2.kv, vb2, Cs);
  __syncthreads();
  lds_gemm<T, false>(k1, nd.kv, n1.kv, As, Bs,
                     [&](int i, int j, T v) { FV[i + (int64_t)j * mp] = v; });
  __syncthreads();
  stage<T>(n2.kv, nd.kv, [&](int i, int j) { return W[n1.kv + i + (int64_t)j * kw]; }, Bs);
  __syncthreads();
  lds_gemm<T, false>(k2, nd.kv, n2.kv, Cs, Bs,
                     [&](int i, int j, T v) { FV[k1 + i + (int64_t)j * mp] = v; });
}

// The merge with every input staged in LDS in one pass (all loads in flight
// together), then two product phases.  For blocks of at most kMB elements.
constexpr int kMB = 2048;
constexpr int kMU = kMB / kNT;   // elements per thread and block

// Element o = threadIdx.x + u kNT of an M-row column-major block is (i, c)
// with o = i + c M; (i, c) advance by the constant (kNT mod M, kNT / M) per u,
// so only the first index of a block costs a division.
struct BlkIdx {
  int i, c, qi, ri, M;
  __device__ __forceinline__ explicit BlkIdx(int m) : M(max(m, 1)) {
    i = (int)threadIdx.x % M;
    c = (int)threadIdx.x / M;
    qi = kNT / M;
    ri = kNT - qi * M;
  }
  __device__ __forceinline__ void next() {
    i += ri;
    c += qi;
    const bool wrap = i >= M;
    i = wrap ? i - M : i;
    c = wrap ? c + 1 : c;
  }
};

template <typename T, typename F>
__device__ __forceinline__ void blk_load(T (&v)[kMU], int M, int N, F f) {
  BlkIdx x(M);
  const int ni = max(M - 1, 0), nc = max(N - 1, 0);
#pragma unroll
  for (int u = 0; u < kMU; ++u) {
    // past the end: the last element (a valid address), never stored
    const bool past = x.c >= N;
    v[u] = M * N > 0 ? f(past ? ni : x.i, past ? nc : x.c) : T(0);
    x.next();
  }
}
template <typename T>
__device__ __forceinline__ void blk_store(const T (&v)[kMU], int M, int N, T* dst) {
  BlkIdx x(M);
#pragma unroll
  for (int u = 0; u < kMU; ++u) {
    if (x.c < N) dst[x.i + x.c * (M + 1)] = v[u];
    x.next();
  }
}
// C(i, j) = sum_l A(i, l) B(l, j) (TB: B(l, j) = B[j + l*ldb]) over LDS blocks.
template <typename T, bool TB>
__device__ __forceinline__ T lds_dot(const T* A, int lda, const T* B, int ldb, int i, int j,
                                     int K) {
  T s = T(0);
  for (int l = 0; l < K; ++l) s += A[i + l * lda] * (TB ? B[j + l * ldb] : B[l + j * ldb]);
  return s;
}

// 2 x 2 tile of C = A B at (i0, j0), A(i, l) = A[i + l*lda], B(l, j) = B[l + j*ldb]
// (TB: B[j + l*ldb]); out(i, j, value) for the in-range entries.
template <typename T, bool TB, typename Out>
__device__ __forceinline__ void tile22(const T* A, int lda, const T* B, int ldb, int M, int N,
                                       int K, int i0, int j0, Out out) {
  const int i1 = min(i0 + 1, M - 1), j1 = min(j0 + 1, N - 1);
  T c00 = T(0), c01 = T(0), c10 = T(0), c11 = T(0);
#pragma unroll 4
  for (int l = 0; l < K; ++l) {
    const T a0 = A[i0 + l * lda], a1 = A[i1 + l * lda];
    const T b0 = TB ? B[j0 + l * ldb] : B[l + j0 * ldb];
    const T b1 = TB ? B[j1 + l * ldb] : B[l + j1 * ldb];
    c00 += a0 * b0; c01 += a0 * b1; c10 += a1 * b0; c11 += a1 * b1;
  }
  out(i0, j0, c00);
  if (j0 + 1 < N) out(i0, j0 + 1, c01);
  if (i0 + 1 < M) out(i0 + 1, j0, c10);
  if (i0 + 1 < M && j0 + 1 < N) out(i0 + 1, j0 + 1, c11);
}
// number of 2 x 2 tiles of an M x N product
__device__ __forceinline__ int ntiles(int M, int N) { return ((M + 1) >> 1) * ((N + 1) >> 1); }

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_ulv_merge1(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* sm = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int k1 = n1.kept, k2 = n2.kept, mp = nd.mp;
  const int ku1 = n1.ku, ku2 = n2.ku, kv1 = n1.kv, kv2 = n2.kv;
  const int kr = ku1 + ku2, kw = kv1 + kv2;
  const bool top = node != 0;   // U', V' below the root
  const int ku = top ? nd.ku : 0, kv = top ? nd.kv : 0;
  const T* FD1 = I.FD + n1.oFD; const T* FD2 = I.FD + n2.oFD;
  const T* FU1 = I.FU + n1.oFU; const T* FU2 = I.FU + n2.oFU;
  const T* FV1 = I.FV + n1.oFV; const T* FV2 = I.FV + n2.oFV;
  const T* B12 = I.B12 + nd.oB12;
  const T* B21 = I.B21 + nd.oB21;
  const T* R = I.R + (top ? nd.oR : 0);
  const T* W = I.W + (top ? nd.oW : 0);
  T* FD = I.FD + nd.oFD;
  // LDS blocks (leading dimension rows + 1)
  T* sB12 = sm;                         T* sB21 = sB12 + (ku1 + 1) * kv2;
  T* sV1 = sB21 + (ku2 + 1) * kv1;      T* sV2 = sV1 + (k1 + 1) * kv1;
  T* sU1 = sV2 + (k2 + 1) * kv2;        T* sU2 = sU1 + (k1 + 1) * ku1;
  T* sR = sU2 + (k2 + 1) * ku2;         T* sW = sR + (kr + 1) * ku;
  T* sC12 = sW + (kw + 1) * kv;         T* sC21 = sC12 + (ku1 + 1) * k2;
  {
    T v0[kMU], v1[kMU], v2[kMU], v3[kMU], v4[kMU], v5[kMU], v6[kMU], v7[kMU], v8[kMU], v9[kMU];
    blk_load(v0, ku1, kv2, [&](int i, int j) { return B12[i + (int64_t)j * ku1]; });
    blk_load(v1, ku2, kv1, [&](int i, int j) { return B21[i + (int64_t)j * ku2]; });
    blk_load(v2, k1, kv1, [&](int i, int j) { return FV1[n1.e + i + (int64_t)j * n1.mp]; });
    blk_load(v3, k2, kv2, [&](int i, int j) { return FV2[n2.e + i + (int64_t)j * n2.mp]; });
    blk_load(v4, k1, ku1, [&](int i, int j) {
      const T x = FU1[n1.e + i + (int64_t)j * n1.mp];
      return ((n1.e > 0) & (i < j)) ? T(0) : x;
    });
    blk_load(v5, k2, ku2, [&](int i, int j) {
      const T x = FU2[n2.e + i + (int64_t)j * n2.mp];
      return ((n2.e > 0) & (i < j)) ? T(0) : x;
    });
    blk_load(v6, kr, ku, [&](int i, int j) { return R[i + (int64_t)j * kr]; });
    blk_load(v7, kw, kv, [&](int i, int j) { return W[i + (int64_t)j * kw]; });
    // diagonal blocks D~22 of the children, copied through registers
    blk_load(v8, k1, k1, [&](int i, int j) { return FD1[n1.e + i + (int64_t)(n1.e + j) * n1.mp]; });
    blk_load(v9, k2, k2, [&](int i, int j) { return FD2[n2.e + i + (int64_t)(n2.e + j) * n2.mp]; });
    blk_store(v0, ku1, kv2, sB12);
    blk_store(v1, ku2, kv1, sB21);
    blk_store(v2, k1, kv1, sV1);
    blk_store(v3, k2, kv2, sV2);
    blk_store(v4, k1, ku1, sU1);
    blk_store(v5, k2, ku2, sU2);
    blk_store(v6, kr, ku, sR);
    blk_store(v7, kw, kv, sW);
    {
      BlkIdx x1(k1), x2(k2);
#pragma unroll
      for (int u = 0; u < kMU; ++u) {
        if (x1.c < k1) FD[x1.i + (int64_t)x1.c * mp] = v8[u];
        if (x2.c < k2) FD[k1 + x2.i + (int64_t)(k1 + x2.c) * mp] = v9[u];
        x1.next();
        x2.next();
      }
    }
  }
  __syncthreads();
  // phase 1 (2 x 2 tiles): C12 = B12 V^b_c2^T, C21 = B21 V^b_c1^T,
  //   U' = blkdiag(U~_c1, U~_c2) R_t, V' = blkdiag(V^b_c1, V^b_c2) W_t
  {
    T* FU = I.FU + nd.oFU;
    T* FV = I.FV + nd.oFV;
    const int t0 = ntiles(ku1, k2), t1 = t0 + ntiles(ku2, k1);
    const int t2 = t1 + ntiles(k1, ku), t3 = t2 + ntiles(k2, ku);
    const int t4 = t3 + ntiles(k1, kv), t5 = t4 + ntiles(k2, kv);
    for (int o = threadIdx.x; o < t5; o += kNT) {
      if (o < t0) {
        const int nr = (ku1 + 1) >> 1;
        tile22<T, true>(sB12, ku1 + 1, sV2, k2 + 1, ku1, k2, kv2, 2 * (o % nr), 2 * (o / nr),
                        [&](int i, int j, T v) { sC12[i + j * (ku1 + 1)] = v; });
      } else if (o < t1) {
        const int q = o - t0, nr = (ku2 + 1) >> 1;
        tile22<T, true>(sB21, ku2 + 1, sV1, k1 + 1, ku2, k1, kv1, 2 * (q % nr), 2 * (q / nr),
                        [&](int i, int j, T v) { sC21[i + j * (ku2 + 1)] = v; });
      } else if (o < t2) {
        const int q = o - t1, nr = (k1 + 1) >> 1;
        tile22<T, false>(sU1, k1 + 1, sR, kr + 1, k1, ku, ku1, 2 * (q % nr), 2 * (q / nr),
                         [&](int i, int j, T v) { FU[i + (int64_t)j * mp] = v; });
      } else if (o < t3) {
        const int q = o - t2, nr = (k2 + 1) >> 1;
        tile22<T, false>(sU2, k2 + 1, sR + ku1, kr + 1, k2, ku, ku2, 2 * (q % nr), 2 * (q / nr),
                         [&](int i, int j, T v) { FU[k1 + i + (int64_t)j * mp] = v; });
      } else if (o < t4) {
        const int q = o - t3, nr = (k1 + 1) >> 1;
        tile22<T, false>(sV1, k1 + 1, sW, kw + 1, k1, kv, kv1, 2 * (q % nr), 2 * (q / nr),
                         [&](int i, int j, T v) { FV[i + (int64_t)j * mp] = v; });
      } else {
        const int q = o - t4, nr = (k2 + 1) >> 1;
        tile22<T, false>(sV2, k2 + 1, sW + kv1, kw + 1, k2, kv, kv2, 2 * (q % nr), 2 * (q / nr),
                         [&](int i, int j, T v) { FV[k1 + i + (int64_t)j * mp] = v; });
      }
    }
  }
  __syncthreads();
  // phase 2: D'(c1, c2) = U~_c1 C12, D'(c2, c1) = U~_c2 C21
  {
    const int t0 = ntiles(k1, k2), t1 = t0 + ntiles(k2, k1);
    for (int o = threadIdx.x; o < t1; o += kNT) {
      if (o < t0) {
        const int nr = (k1 + 1) >> 1;
        tile22<T, false>(sU1, k1 + 1, sC12, ku1 + 1, k1, k2, ku1, 2 * (o % nr), 2 * (o / nr),
                         [&](int i, int j, T v) { FD[i + (int64_t)(k1 + j) * mp] = v; });
      } else {
        const int q = o - t0, nr = (k2 + 1) >> 1;
        tile22<T, false>(sU2, k2 + 1, sC21, ku2 + 1, k2, k1, ku2, 2 * (q % nr), 2 * (q / nr),
                         [&](int i, int j, T v) { FD[k1 + i + (int64_t)j * mp] = v; });
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The merge on the matrix cores, for nodes whose children's kept sizes and
// all ranks involved are at most 32: every operand is staged in LDS as a
// zero-padded 32 x 32 block (buffer loads past a block's end read zero), and
// each product is one 32 x 32 x 32 product of 16 x 16 x 4 MFMAs (2 x 2 output
// tiles, 8 k-steps) by one wavefront.
//   phase 1: C12 = B12 V^b_c2^T, C21 = B21 V^b_c1^T (to LDS),
//            U' = [U~_c1 R_top; U~_c2 R_bot], V' = [V^b_c1 W_top; V^b_c2 W_bot];
//   phase 2: D'(c1, c2) = U~_c1 C12, D'(c2, c1) = U~_c2 C21;
// the diagonal blocks D~22 of the children are copied through registers.
// ---------------------------------------------------------------------------
constexpr int kMP = 33;          // LDS pitch of a staged 32 x 32 operand
constexpr int kMBlk = 32 * kMP;  // elements of one staged operand

// acc = A B for staged 32 x 32 operands; TA: A(i, k) = A[k + i kMP] (A stored
// transposed), TB: B(k, j) = B[j + k kMP].
template <typename T, bool TA, bool TB>
__device__ __forceinline__ void mma_gemm32(const T* A, const T* B, mma4_t<T> (&acc)[2][2], int g,
                                           int c) {
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) acc[it][jt] = mma_zero<T>();
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    const int k = 4 * kk + g;
    T a[2], b[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int i = 16 * it + c;
      a[it] = TA ? A[k + i * kMP] : A[i + k * kMP];
    }
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int j = 16 * jt + c;
      b[jt] = TB ? B[j + k * kMP] : B[k + j * kMP];
    }
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) acc[it][jt] = mma16(a[it], b[jt], acc[it][jt]);
  }
}

// Entries (i, j), i < M, j < N, of a 32 x 32 product to dst[i + j ld] (global,
// through a buffer descriptor of `bytes` bytes) or, LDS, to dst[i + j kMP].
template <typename T>
__device__ __forceinline__ void mma_store_global(const mma4_t<T> (&acc)[2][2], T* dst, int ld,
                                                 int M, int N, uint32_t bytes, int g, int c) {
  const auto R = buf_rsrc(dst, bytes);
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * it + mma_row<T>(g, r), j = 16 * jt + c;
        const bool in = (i < M) & (j < N);
        buf_store<T>(acc[it][jt][r], R, in ? (uint32_t)(i + j * ld) * (uint32_t)sizeof(T) : kBufOOB,
                     0);
      }
}
template <typename T>
__device__ __forceinline__ void mma_store_lds(const mma4_t<T> (&acc)[2][2], T* dst, int g, int c) {
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int jt = 0; jt < 2; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        dst[16 * it + mma_row<T>(g, r) + (16 * jt + c) * kMP] = acc[it][jt][r];
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_ulv_merge_mma(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* sm = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int k1 = n1.kept, k2 = n2.kept, mp = nd.mp;
  const int ku1 = n1.ku, ku2 = n2.ku, kv1 = n1.kv, kv2 = n2.kv;
  const int kr = ku1 + ku2, kw = kv1 + kv2;
  const bool top = node != 0;   // U', V' below the root
  const int ku = top ? nd.ku : 0, kv = top ? nd.kv : 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  constexpr uint32_t sz = sizeof(T);
  // staged operands: 0 B12, 1 B21, 2 V^b_c1, 3 V^b_c2, 4 U~_c1, 5 U~_c2,
  // 6 R_top, 7 R_bot, 8 W_top, 9 W_bot; then C12 (10), C21 (11)
  {
    struct Src {
      const T* p;
      uint32_t bytes;
      int off, ld, M, N;
      bool tri;   // U~ with rows eliminated: zeros above the diagonal
    };
    const T* R = I.R + (top ? nd.oR : 0);
    const T* W = I.W + (top ? nd.oW : 0);
    const Src src[10] = {
        {I.B12 + nd.oB12, (uint32_t)(ku1 * kv2) * sz, 0, ku1, ku1, kv2, false},
        {I.B21 + nd.oB21, (uint32_t)(ku2 * kv1) * sz, 0, ku2, ku2, kv1, false},
        {I.FV + n1.oFV, (uint32_t)(n1.mp * kv1) * sz, n1.e, n1.mp, k1, kv1, false},
        {I.FV + n2.oFV, (uint32_t)(n2.mp * kv2) * sz, n2.e, n2.mp, k2, kv2, false},
        {I.FU + n1.oFU, (uint32_t)(n1.mp * ku1) * sz, n1.e, n1.mp, k1, ku1, n1.e > 0},
        {I.FU + n2.oFU, (uint32_t)(n2.mp * ku2) * sz, n2.e, n2.mp, k2, ku2, n2.e > 0},
        {R, (uint32_t)(kr * ku) * sz, 0, kr, ku1, ku, false},
        {R, (uint32_t)(kr * ku) * sz, ku1, kr, ku2, ku, false},
        {W, (uint32_t)(kw * kv) * sz, 0, kw, kv1, kv, false},
        {W, (uint32_t)(kw * kv) * sz, kv1, kw, kv2, kv, false}};
    // D~22 of the children (copied to the parent's diagonal blocks)
    const T* FD1 = I.FD + n1.oFD;
    const T* FD2 = I.FD + n2.oFD;
    const auto RD1 = buf_rsrc(FD1, (uint32_t)(n1.mp * n1.mp) * sz);
    const auto RD2 = buf_rsrc(FD2, (uint32_t)(n2.mp * n2.mp) * sz);
    T v[10][4], d1[4], d2[4];
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const auto Rq = buf_rsrc(src[q].p, src[q].bytes);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = tid + u * kNT, i = o & 31, j = o >> 5;
        const bool in = (i < src[q].M) & (j < src[q].N) & !(src[q].tri & (i < j));
        v[q][u] = buf_load<T>(Rq, in ? (uint32_t)(src[q].off + i + j * src[q].ld) * sz : kBufOOB, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = tid + u * kNT, i = o & 31, j = o >> 5;
      d1[u] = buf_load<T>(RD1, (i < k1) & (j < k1) ? (uint32_t)(n1.e + i + (n1.e + j) * n1.mp) * sz
                                                   : kBufOOB, 0);
      d2[u] = buf_load<T>(RD2, (i < k2) & (j < k2) ? (uint32_t)(n2.e + i + (n2.e + j) * n2.mp) * sz
                                                   : kBufOOB, 0);
    }
#pragma unroll
    for (int q = 0; q < 10; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int o = tid + u * kNT, i = o & 31, j = o >> 5;
        sm[q * kMBlk + i + j * kMP] = v[q][u];
      }
    const auto RD = buf_rsrc(I.FD + nd.oFD, (uint32_t)(mp * mp) * sz);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = tid + u * kNT, i = o & 31, j = o >> 5;
      buf_store<T>(d1[u], RD, (i < k1) & (j < k1) ? (uint32_t)(i + j * mp) * sz : kBufOOB, 0);
      buf_store<T>(d2[u], RD, (i < k2) & (j < k2) ? (uint32_t)(k1 + i + (k1 + j) * mp) * sz
                                                 : kBufOOB, 0);
    }
  }
  __syncthreads();
  const T* sB12 = sm;
  const T* sB21 = sm + kMBlk;
  const T* sV1 = sm + 2 * kMBlk;
  const T* sV2 = sm + 3 * kMBlk;
  const T* sU1 = sm + 4 * kMBlk;
  const T* sU2 = sm + 5 * kMBlk;
  const T* sRt = sm + 6 * kMBlk;
  const T* sRb = sm + 7 * kMBlk;
  const T* sWt = sm + 8 * kMBlk;
  const T* sWb = sm + 9 * kMBlk;
  T* sC12 = sm + 10 * kMBlk;
  T* sC21 = sm + 11 * kMBlk;
  T* FU = I.FU + nd.oFU;
  T* FV = I.FV + nd.oFV;
  T* FD = I.FD + nd.oFD;
  mma4_t<T> acc[2][2];
  if (w == 0) {
    mma_gemm32<T, false, true>(sB12, sV2, acc, g, c);   // C12 = B12 V^b_c2^T
    mma_store_lds<T>(acc, sC12, g, c);
    if (kv > 0) {
      mma_gemm32<T, false, false>(sV1, sWt, acc, g, c);   // V'_top
      mma_store_global<T>(acc, FV, mp, k1, kv, (uint32_t)(mp * kv) * sz, g, c);
    }
  } else if (w == 1) {
    mma_gemm32<T, false, true>(sB21, sV1, acc, g, c);   // C21 = B21 V^b_c1^T
    mma_store_lds<T>(acc, sC21, g, c);
    if (kv > 0) {
      mma_gemm32<T, false, false>(sV2, sWb, acc, g, c);   // V'_bot
      mma_store_global<T>(acc, FV + k1, mp, k2, kv, (uint32_t)(mp * kv - k1) * sz, g, c);
    }
  } else if (w == 2) {
    if (ku > 0) {
      mma_gemm32<T, false, false>(sU1, sRt, acc, g, c);   // U'_top
      mma_store_global<T>(acc, FU, mp, k1, ku, (uint32_t)(mp * ku) * sz, g, c);
    }
  } else {
    if (ku > 0) {
      mma_gemm32<T, false, false>(sU2, sRb, acc, g, c);   // U'_bot
      mma_store_global<T>(acc, FU + k1, mp, k2, ku, (uint32_t)(mp * ku - k1) * sz, g, c);
    }
  }
  __syncthreads();
  if (w == 0) {
    mma_gemm32<T, false, false>(sU1, sC12, acc, g, c);   // D'(c1, c2) = U~_c1 C12
    mma_store_global<T>(acc, FD + (int64_t)k1 * mp, mp, k1, k2, (uint32_t)(mp * (mp - k1)) * sz,
                        g, c);
  } else if (w == 1) {
    mma_gemm32<T, false, false>(sU2, sC21, acc, g, c);   // D'(c2, c1) = U~_c2 C21
    mma_store_global<T>(acc, FD + k1, mp, k2, k1, (uint32_t)(mp * mp - k1) * sz, g, c);
  }
}

// ---------------------------------------------------------------------------
// Forward-operator records of a factored level (nodes with fwd_op_ok; record
// layout kRec* in hss_internal.hpp).  The forward step of the solve,
// rhs = [c_c1 - U~_c1 B12 z_c2; c_c2 - U~_c2 B21 z_c1], b~ = Q^T rhs,
// y = L^-1 b~_top, c = b~_bot - D~21 y, z = V^_top^T y + W^T [z_c1; z_c2],
// becomes four products instead of ku + e sequential steps:
//   Q^T = H_0 ... H_{ku-1} = I - Y T Y^T (compact WY: Y the QL reflectors
//   with their unit pivots, T upper triangular with
//   T(i, j) = tau_i (delta_ij - sum_{m > i} (Y^T Y)(i, m) T(m, j)), rows from
//   the bottom up), so b~ = rhs - (Y T) (Y^T rhs);
//   [y; D~21 y; V^_top^T y] = [L^-1; D~21 L^-1; V^_top^T L^-1] b~_top.
// Y^T Y, U~ B and the products of the last phase on the matrix cores
// (zero-padded 32 x 32 blocks in LDS), T and L^-1 by one wavefront each
// (lane j: column j).  The record is cleared first, then written.
// ---------------------------------------------------------------------------
// acc (+)= A B for staged 32 x 32 operands (see mma_gemm32), without zeroing.
template <typename T, bool TA, bool TB>
__device__ __forceinline__ void mma_gemm32_acc(const T* A, const T* B, mma4_t<T> (&acc)[2][2],
                                               int g, int c) {
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    const int k = 4 * kk + g;
    T a[2], b[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int i = 16 * it + c;
      a[it] = TA ? A[k + i * kMP] : A[i + k * kMP];
    }
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
      const int j = 16 * jt + c;
      b[jt] = TB ? B[j + k * kMP] : B[k + j * kMP];
    }
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) acc[it][jt] = mma16(a[it], b[jt], acc[it][jt]);
  }
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_ulv_fwdop(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* sm = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  if (nd.oOP < 0) return;
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int mp = nd.mp, ku = nd.ku, kv = nd.kv, e = nd.e, kept = nd.kept;
  const int k1 = n1.kept, k2 = n2.kept, ku1 = n1.ku, ku2 = n2.ku, kv1 = n1.kv, kv2 = n2.kv;
  const int kw = kv1 + kv2;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  constexpr uint32_t sz = sizeof(T);
  // staged: 0 Y rows 0-31, 1 Y rows 32-63, 2 L^T (L(i, k) at k + i kMP, k <= i),
  // 3 D~21, 4 V^_top, 5 U~_c1, 6 U~_c2, 7 B12, 8 B21, then G = Y^T Y (9),
  // T (10), L^-1 (11); taus after them
  T* sY0 = sm;
  T* sY1 = sm + kMBlk;
  T* sLt = sm + 2 * kMBlk;
  T* sD = sm + 3 * kMBlk;
  T* sV = sm + 4 * kMBlk;
  T* sU1 = sm + 5 * kMBlk;
  T* sU2 = sm + 6 * kMBlk;
  T* sB12 = sm + 7 * kMBlk;
  T* sB21 = sm + 8 * kMBlk;
  T* sG = sm + 9 * kMBlk;
  T* sT = sm + 10 * kMBlk;
  T* sLi = sm + 11 * kMBlk;
  T* staus = sm + 12 * kMBlk;
  T* rec = I.FOP + nd.oOP;
  {
    const auto RU = buf_rsrc(I.FU + nd.oFU, (uint32_t)(mp * ku) * sz);
    const auto RD = buf_rsrc(I.FD + nd.oFD, (uint32_t)(mp * mp) * sz);
    const auto RV = buf_rsrc(I.FV + nd.oFV, (uint32_t)(mp * kv) * sz);
    const auto RU1 = buf_rsrc(I.FU + n1.oFU, (uint32_t)(n1.mp * ku1) * sz);
    const auto RU2 = buf_rsrc(I.FU + n2.oFU, (uint32_t)(n2.mp * ku2) * sz);
    const auto R12 = buf_rsrc(I.B12 + nd.oB12, (uint32_t)(ku1 * kv2) * sz);
    const auto R21 = buf_rsrc(I.B21 + nd.oB21, (uint32_t)(ku2 * kv1) * sz);
    T v[9][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = tid + u * kNT, i = o & 31, j = o >> 5;
      // Y: reflector j above its pivot row e + j (the pivot itself is a unit)
      const int r0 = i, r1 = 32 + i;
      v[0][u] = buf_load<T>(RU, (j < ku) & (r0 < e + j) ? (uint32_t)(r0 + j * mp) * sz : kBufOOB, 0);
      v[1][u] = buf_load<T>(RU, (j < ku) & (r1 < e + j) & (r1 < mp) ? (uint32_t)(r1 + j * mp) * sz
                                                                     : kBufOOB, 0);
      // L(i, j) for j <= i < e (rows of FD above e hold L left of the diagonal)
      v[2][u] = buf_load<T>(RD, (i < e) & (j <= i) ? (uint32_t)(i + j * mp) * sz : kBufOOB, 0);
      v[3][u] = buf_load<T>(RD, (i < kept) & (j < e) ? (uint32_t)(e + i + j * mp) * sz : kBufOOB, 0);
      v[4][u] = buf_load<T>(RV, (i < e) & (j < kv) ? (uint32_t)(i + j * mp) * sz : kBufOOB, 0);
      // U~ of the children: trailing kept rows of FU, zero above the diagonal
      // when rows were eliminated
      v[5][u] = buf_load<T>(RU1, (i < k1) & (j < ku1) & !((n1.e > 0) & (i < j))
                                     ? (uint32_t)(n1.e + i + j * n1.mp) * sz : kBufOOB, 0);
      v[6][u] = buf_load<T>(RU2, (i < k2) & (j < ku2) & !((n2.e > 0) & (i < j))
                                     ? (uint32_t)(n2.e + i + j * n2.mp) * sz : kBufOOB, 0);
      v[7][u] = buf_load<T>(R12, (i < ku1) & (j < kv2) ? (uint32_t)(i + j * ku1) * sz : kBufOOB, 0);
      v[8][u] = buf_load<T>(R21, (i < ku2) & (j < kv1) ? (uint32_t)(i + j * ku2) * sz : kBufOOB, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = tid + u * kNT, i = o & 31, j = o >> 5;
      const bool p0 = (j < ku) & (i == e + j), p1 = (j < ku) & (32 + i == e + j);
      sY0[i + j * kMP] = p0 ? T(1) : v[0][u];
      sY1[i + j * kMP] = p1 ? T(1) : v[1][u];
      sLt[j + i * kMP] = v[2][u];
      sD[i + j * kMP] = v[3][u];
      sV[i + j * kMP] = v[4][u];
      sU1[i + j * kMP] = v[5][u];
      sU2[i + j * kMP] = v[6][u];
      sB12[i + j * kMP] = v[7][u];
      sB21[i + j * kMP] = v[8][u];
    }
    if (tid < 32) staus[tid] = tid < ku ? I.tq[nd.otq + tid] : T(0);
    // the record starts cleared (its unused rows and columns stay zero),
    // 16 bytes per store
    int4* r4 = reinterpret_cast<int4*>(rec);
    constexpr int n4 = kRecSize * (int)sizeof(T) / 16;
    for (int o = tid; o < n4; o += kNT) r4[o] = make_int4(0, 0, 0, 0);
  }
  __syncthreads();
  mma4_t<T> acc[2][2];
  constexpr uint32_t rb = (uint32_t)kRecSize * sz;
  if (w == 0) {
    // G = Y^T Y over both row halves
#pragma unroll
    for (int it = 0; it < 2; ++it)
#pragma unroll
      for (int jt = 0; jt < 2; ++jt) acc[it][jt] = mma_zero<T>();
    mma_gemm32_acc<T, true, false>(sY0, sY0, acc, g, c);
    mma_gemm32_acc<T, true, false>(sY1, sY1, acc, g, c);
    mma_store_lds<T>(acc, sG, g, c);
  } else if (w == 1) {
    // W (kw x kv, pitch 65) and Y (with its unit pivots, pitch 65) into the record
    const T* W = I.W + nd.oW;
    for (int o = lane; o < kw * kv; o += 64) {
      const int i = o % kw, j = o / kw;
      rec[kRecW + i + j * 65] = W[o];
    }
    for (int o = lane; o < mp * ku; o += 64) {
      const int i = o % mp, j = o / mp;
      rec[kRecY + i + j * 65] = i < 32 ? sY0[i + j * kMP] : sY1[i - 32 + j * kMP];
    }
  } else if (w == 2) {
    // rows 0 .. k1-1, columns kv1 .. of G: U~_c1 B12
    mma_gemm32<T, false, false>(sU1, sB12, acc, g, c);
    mma_store_global<T>(acc, rec + kRecG + (int64_t)kv1 * 64, 64, k1, kv2,
                        rb - (uint32_t)(kRecG + kv1 * 64) * sz, g, c);
  } else {
    // rows k1 .. mp-1, columns 0 .. kv1-1 of G: U~_c2 B21
    mma_gemm32<T, false, false>(sU2, sB21, acc, g, c);
    mma_store_global<T>(acc, rec + kRecG + k1, 64, k2, kv1, rb - (uint32_t)(kRecG + k1) * sz, g,
                        c);
  }
  __syncthreads();
  // T and L^-1, one column per lane; every sum over four partial sums (the
  // dependence chain of a column is what these steps wait on)
  if (w == 0 && lane < 32) {
    // column j = lane of T, rows from the bottom up
    const int j = lane;
    T t[32];
#pragma unroll
    for (int i = 31; i >= 0; --i) {
      T q[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int m = i + 1; m < 32; ++m) q[(m - i - 1) & 3] += sG[i + m * kMP] * t[m];
      const T s = ((i == j) ? T(1) : T(0)) - ((q[0] + q[1]) + (q[2] + q[3]));
      t[i] = (i < ku) & (j < ku) ? staus[i] * s : T(0);
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) sT[i + j * kMP] = t[i];
  } else if (w == 1 && lane < 32) {
    // column j = lane of L^-1 by forward substitution (rows i < j stay zero)
    const int j = lane;
    T x[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      T q[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int k = 0; k < i; ++k) q[k & 3] += sLt[k + i * kMP] * x[k];
      const T s = ((i == j) ? T(1) : T(0)) - ((q[0] + q[1]) + (q[2] + q[3]));
      const T d = sLt[i + i * kMP];
      x[i] = (i < e) & (j < e) ? s / d : T(0);
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) sLi[i + j * kMP] = x[i];
  }
  __syncthreads();
  if (w == 0) {
    mma_gemm32<T, false, false>(sY0, sT, acc, g, c);   // (Y T), rows 0..31
    mma_store_global<T>(acc, rec + kRecYT, 64, min(mp, 32), ku, rb - (uint32_t)kRecYT * sz, g, c);
  } else if (w == 1) {
    if (mp > 32) {
      mma_gemm32<T, false, false>(sY1, sT, acc, g, c);   // (Y T), rows 32..
      mma_store_global<T>(acc, rec + kRecYT + 32, 64, mp - 32, ku,
                          rb - (uint32_t)(kRecYT + 32) * sz, g, c);
    }
    // L^-1 into F, rows 0 .. e-1
    for (int o = lane; o < e * e; o += 64) {
      const int i = o % e, j = o / e;
      rec[kRecF + i + j * 96] = sLi[i + j * kMP];
    }
  } else if (w == 2) {
    mma_gemm32<T, false, false>(sD, sLi, acc, g, c);   // D~21 L^-1
    mma_store_global<T>(acc, rec + kRecF + e, 96, kept, e, rb - (uint32_t)(kRecF + e) * sz, g, c);
  } else {
    mma_gemm32<T, true, false>(sV, sLi, acc, g, c);    // V^_top^T L^-1
    mma_store_global<T>(acc, rec + kRecF + e + kept, 96, kv, e,
                        rb - (uint32_t)(kRecF + e + kept) * sz, g, c);
  }
}

// ---------------------------------------------------------------------------
// Root: LU with partial pivoting (FP64) of D'_root (or of D when p = 0).
// ---------------------------------------------------------------------------
// After the interchanges piv[0 .. mp) of a factored root block: the
// permutation they make (position i holds original row perm[i]) to
// piv[mp + i], so that the solve permutes its right-hand side in one gather.
// Called by the whole work-group; mp <= 256 (the block fits LDS).
__device__ void store_perm(int32_t* piv, int mp) {
  __shared__ int ps[256], pv[256];
  __syncthreads();   // the interchanges written by thread 0 are visible
  for (int o = threadIdx.x; o < mp; o += blockDim.x) {
    ps[o] = o;
    pv[o] = piv[o];
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < mp; ++j) {
      const int q = pv[j], t = ps[j];
      ps[j] = ps[q];
      ps[q] = t;
    }
  __syncthreads();
  for (int o = threadIdx.x; o < mp; o += blockDim.x) piv[mp + o] = ps[o];
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_ulv_root_lu(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  double* Ls = reinterpret_cast<double*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int mp = nd.mp, ld = mp + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ int pivs;
  const T* src = I.p == 0 ? I.D + nd.oD : I.FD + nd.oFD;
  wg_stage<16, T>(mp, mp, [&](int i, int j) { return src[i + (int64_t)j * mp]; },
                  [&](int i, int j, T v) { Ls[i + j * ld] = (double)v; });
  __syncthreads();
  for (int j = 0; j < mp; ++j) {
    if (tid < 64) {
      double best = -1.0;
      int bi = j;
      for (int r = j + tid; r < mp; r += 64) {
        const double v = fabs(Ls[r + j * ld]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        pivs = bi;
        I.piv[j] = bi;
        if (best == 0.0) {
          atomicOr(I.status, 1 << kCodeSingular);
          atomicMax(I.status + kStSingularNode, node + 1);
        }
      }
    }
    __syncthreads();
    const int pr = pivs;
    if (pr != j)
      for (int c = tid; c < mp; c += nt) {
        const double t = Ls[j + c * ld];
        Ls[j + c * ld] = Ls[pr + c * ld];
        Ls[pr + c * ld] = t;
      }
    __syncthreads();
    const double d = Ls[j + j * ld];
    if (d != 0.0)
      for (int r = j + 1 + tid; r < mp; r += nt) Ls[r + j * ld] /= d;
    __syncthreads();
    const int rem = mp - j - 1;
    for (int o = tid; o < rem * rem; o += nt) {
      const int r = j + 1 + o % rem, c = j + 1 + o / rem;
      Ls[r + c * ld] -= Ls[r + j * ld] * Ls[j + c * ld];
    }
    __syncthreads();
  }
  for (int o = tid; o < mp * mp; o += nt) I.rootLU[o] = Ls[o % mp + (o / mp) * ld];
  store_perm(I.piv, mp);
}

// The same factorization for mp <= 128, organised for short steps: the pivot
// search by wavefront 0 (wavefront max, then the smallest row index among
// equals), one reciprocal per column, and a rank-1 update in which thread t
// owns column j+1 + t % 64 and every fourth row below the pivot; three
// barriers per column.
template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_ulv_root_lu2(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  double* Ls = reinterpret_cast<double*>(smem_raw);
  __shared__ int s_piv;
  __shared__ int s_sing;
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int mp = nd.mp, ld = mp + 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const T* src = I.p == 0 ? I.D + nd.oD : I.FD + nd.oFD;
  wg_stage<16, T>(mp, mp, [&](int i, int j) { return src[i + (int64_t)j * mp]; },
                  [&](int i, int j, T v) { Ls[i + j * ld] = (double)v; });
  if (tid == 0) s_sing = 0;
  __syncthreads();
  for (int j = 0; j < mp; ++j) {
    if (w == 0) {
      const int r0 = j + lane, r1 = j + 64 + lane;
      const double v0 = r0 < mp ? fabs(Ls[r0 + j * ld]) : -1.0;
      const double v1 = r1 < mp ? fabs(Ls[r1 + j * ld]) : -1.0;
      const double mx = wave_max(max(v0, v1));
      const double cand = v0 == mx ? (double)r0 : (v1 == mx ? (double)r1 : 1e9);
      int p = (int)wave_min(cand);
      if (!(mx > 0.0)) p = j;
      if (lane == 0) {
        s_piv = p;
        I.piv[j] = p;
        if (!(mx > 0.0)) s_sing = 1;
      }
    }
    __syncthreads();
    const int p = s_piv;
    // swap rows j and p (columns tid), then scale the column below the pivot
    if (p != j)
      for (int c = tid; c < mp; c += kNT) {
        const double t = Ls[j + c * ld];
        Ls[j + c * ld] = Ls[p + c * ld];
        Ls[p + c * ld] = t;
      }
    __syncthreads();
    const double d = Ls[j + j * ld];
    const double dinv = d != 0.0 ? 1.0 / d : 0.0;
    for (int r = j + 1 + tid; r < mp; r += kNT) Ls[r + j * ld] *= dinv;
    __syncthreads();
    // rank-1 update of the trailing block
    const int c = j + 1 + lane;
    if (c < mp) {
      const double u = Ls[j + c * ld];
      for (int r = j + 1 + w; r < mp; r += kNT / 64) Ls[r + c * ld] -= Ls[r + j * ld] * u;
    }
    if (mp - j - 1 > 64) {   // columns beyond the first 64 of the trailing block
      const int c2 = j + 65 + lane;
      if (c2 < mp) {
        const double u = Ls[j + c2 * ld];
        for (int r = j + 1 + w; r < mp; r += kNT / 64) Ls[r + c2 * ld] -= Ls[r + j * ld] * u;
      }
    }
    __syncthreads();
  }
  if (tid == 0 && s_sing) {
    atomicOr(I.status, 1 << kCodeSingular);
    atomicMax(I.status + kStSingularNode, node + 1);
  }
  for (int o = tid; o < mp * mp; o += kNT) I.rootLU[o] = Ls[o % mp + (o / mp) * ld];
  store_perm(I.piv, mp);
}

// FP64 LU with partial pivoting of a root block of at most 64 rows, the block
// in registers: lane i of every wavefront holds row i, wavefront w columns
// 16 w .. 16 w + 15.  Rows are not moved: step j picks the largest |A(i, j)|
// among the rows not yet chosen (the first lane on ties) in the wavefront
// that holds column j, which publishes the pivot row and the multipliers in
// LDS (double-buffered by step parity, one barrier per step); every
// wavefront then subtracts multiplier times pivot row from its columns past
// j (the pivot row's entries read from the pivot lane's registers).  Row i,
// closed at step s_i, holds its multipliers left of column s_i and its U row
// from there on, so writing it to row s_i of the output gives the in-place
// L U of the permuted block; the sequence of row interchanges (LAPACK's
// convention, as the solve reads it) is reconstructed at the end from the
// order in which rows were chosen.
template <typename T, bool BATCH>
__global__ __launch_bounds__(256) void k_ulv_root_lu_w(KArgs<T, CallSV<T>> a) {
  __shared__ double ls[2][64];
  __shared__ int sp[2];
  __shared__ int order[64];
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int mp = nd.mp;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const T* src = I.p == 0 ? I.D + nd.oD : I.FD + nd.oFD;
  const bool row_ok = lane < mp;
  double A[16];
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) {
    const int c = 16 * w + cc;
    const bool ok = row_ok & (c < mp);
    A[cc] = ok ? (double)src[(ok ? lane : 0) + (int64_t)(ok ? c : 0) * mp] : 0.0;
  }
  bool open = row_ok;
  int rank = lane;
  bool sing = false;
  // a rolled loop over the steps (compact code: the kernel runs once per
  // factorization, so its instructions are fetched cold); column j of the
  // owner's registers is picked and replaced by selects
  for (int j = 0; j < mp; ++j) {
    const int par = j & 1;
    if (w == (j >> 4)) {
      const int jc = j & 15;
      double aj = 0.0;
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) aj = cc == jc ? A[cc] : aj;
      const double v = open ? fabs(aj) : -1.0;
      const double mx = wave_max(v);
      const uint64_t hit = __ballot(open && v == mx);
      const uint64_t avail = __ballot(open);
      const int p = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(hit ? hit : avail));
      if (!(mx > 0.0)) sing = true;
      const double pv = lane_read(aj, p);
      const double dinv = mx > 0.0 ? 1.0 / pv : 0.0;
      const bool elim = open && lane != p;
      const double l = elim ? aj * dinv : 0.0;
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) A[cc] = (cc == jc) & elim ? l : A[cc];
      ls[par][lane] = l;
      if (lane == 0) {
        sp[par] = p;
        order[j] = p;
      }
    }
    __syncthreads();
    const int p = sp[par];
    const double l = ls[par][lane];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc)
      if (16 * w + cc > j) A[cc] -= l * lane_read(A[cc], p);   // (uniform test)
    if (lane == p) {
      open = false;
      rank = j;
    }
  }
  double* LU = I.rootLU;
  if (row_ok) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int c = 16 * w + cc;
      if (c < mp) LU[rank + (int64_t)c * mp] = A[cc];
    }
  }
  if (w == 0) {
    // interchanges: position j takes the row chosen at step j from wherever
    // the earlier interchanges left it (cur: row at each position, at:
    // position of each row, one entry per lane)
    int cur = lane, at = lane;
    for (int j = 0; j < mp; ++j) {
      const int r = order[j];
      const int q = __builtin_amdgcn_readlane(at, r);
      const int rj = __builtin_amdgcn_readlane(cur, j);
      if (lane == j) I.piv[j] = q;
      if (lane == j) I.piv[mp + j] = r;   // the permutation: position j holds row r
      if (lane == j) cur = r;
      if (lane == q) cur = rj;
      if (lane == r) at = j;
      if (lane == rj) at = q;
    }
  }
  const uint64_t sg = __ballot(sing);
  if (threadIdx.x % 64 == 0 && sg && w == 0) {
    atomicOr(I.status, 1 << kCodeSingular);
    atomicMax(I.status + kStSingularNode, node + 1);
  }
}

// ---------------------------------------------------------------------------
template <typename T>
void launch_ulv(UlvStep step, const KArgs<T, CallSV<T>>& a, int nblocks, int max_k, int max_mp,
                hipStream_t s) {
  if (nblocks <= 0) return;
  const bool batch = a.tasks != nullptr;
  dim3 block(kNT);
  size_t sm = 0;
  dim3 grid(nblocks, 1);
  const size_t TB = sizeof(T);
  switch (step) {
    case UlvStep::Merge:
      // one-pass merge while every block has at most kMB elements (ranks <= 32)
      sm = (max_mp <= 64 && max_k <= 32) ? (size_t)(8 * 33 * 32 + 2 * 65 * 32) * TB
                                         : (size_t)3 * kMaxRank * (kMaxRank + 1) * TB;
      break;
    case UlvStep::Factor: break;
    case UlvStep::RootLU: sm = (size_t)max_mp * (max_mp + 1) * sizeof(double); break;
    default: break;
  }
  // leaf launches (nblocks == number of leaves at the bottom level) get their own names
  static const char* names64[] = {"ulv_merge_f64", "ulv_factor_f64", "ulv_root_lu_f64",
                                  "sv_fwd_f64", "sv_root_f64", "sv_bwd_f64", "ulv_fwdop_f64"};
  static const char* names32[] = {"ulv_merge_f32", "ulv_factor_f32", "ulv_root_lu_f32",
                                  "sv_fwd_f32", "sv_root_f32", "sv_bwd_f32", "ulv_fwdop_f32"};
  static const char* leaf64[] = {"", "ulv_factor_leaf_f64", "", "sv_fwd_leaf_f64", "",
                                 "sv_bwd_leaf_f64", ""};
  static const char* leaf32[] = {"", "ulv_factor_leaf_f32", "", "sv_fwd_leaf_f32", "",
                                 "sv_bwd_leaf_f32", ""};
  const bool leafy = a.node0 > 0 && a.node0 == a.inst.nnodes / 2 && !batch;
  const char* nm = leafy ? (sizeof(T) == 8 ? leaf64 : leaf32)[(int)step]
                         : (sizeof(T) == 8 ? names64 : names32)[(int)step];
  TimedLaunch tl(nm, s);
#define HSS_LAUNCH(K)                                                         \
  if (batch) hipLaunchKernelGGL((K<T, true>), grid, block, sm, s, a);         \
  else hipLaunchKernelGGL((K<T, false>), grid, block, sm, s, a);
#define HSS_LAUNCH_SM(K, SM)                                                  \
  if (batch) hipLaunchKernelGGL((K<T, true>), grid, block, SM, s, a);         \
  else hipLaunchKernelGGL((K<T, false>), grid, block, SM, s, a);
  switch (step) {
    case UlvStep::Merge:
      if (max_mp <= 64 && max_k <= 32) {
        sm = (size_t)12 * kMBlk * TB;
        HSS_LAUNCH(k_ulv_merge_mma);
      }
      else { HSS_LAUNCH(k_ulv_merge); }
      break;
    case UlvStep::FwdOp:
      HSS_LAUNCH_SM(k_ulv_fwdop, (size_t)(12 * kMBlk + 32) * TB);
      break;
    case UlvStep::Factor:
      if (factor_blk_fits<T>(max_mp, max_k)) launch_factor_blk<T>(a, nblocks, s);
      else launch_factor_reg<T>(a, nblocks, max_mp, s);
      break;
    case UlvStep::RootLU:
      if (max_mp <= 64) {
        block = dim3(256);
        sm = 0;
        HSS_LAUNCH(k_ulv_root_lu_w);
      } else if (max_mp <= 128) { HSS_LAUNCH(k_ulv_root_lu2); }
      else { HSS_LAUNCH(k_ulv_root_lu); }
      break;
    default: break;
  }
#undef HSS_LAUNCH
#undef HSS_LAUNCH_SM
}

template void launch_ulv<double>(UlvStep, const KArgs<double, CallSV<double>>&, int, int, int,
                                 hipStream_t);
template void launch_ulv<float>(UlvStep, const KArgs<float, CallSV<float>>&, int, int, int,
                                hipStream_t);

}  // namespace hss
