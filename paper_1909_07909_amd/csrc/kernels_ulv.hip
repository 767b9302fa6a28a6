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

namespace hss {

constexpr int32_t kStatusSingular = 4;

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
// ---------------------------------------------------------------------------
template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_ulv_merge(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int k1 = n1.kept, k2 = n2.kept, mp = nd.mp;
  const T* FD1 = I.FD + n1.oFD; const T* FD2 = I.FD + n2.oFD;
  const T* FU1 = I.FU + n1.oFU; const T* FU2 = I.FU + n2.oFU;
  const T* FV1 = I.FV + n1.oFV; const T* FV2 = I.FV + n2.oFV;
  T* FD = I.FD + nd.oFD;
  T* T1 = smem;                              // ku1 x k2 : B12 V^b_c2^T
  T* T2 = T1 + n1.ku * k2;                   // ku2 x k1 : B21 V^b_c1^T
  T* red = T2 + n2.ku * k1;
  // diagonal blocks D~22 of the children
  for (int o = threadIdx.x; o < k1 * k1; o += blockDim.x) {
    const int i = o % k1, j = o / k1;
    FD[i + (int64_t)j * mp] = FD1[n1.e + i + (int64_t)(n1.e + j) * n1.mp];
  }
  for (int o = threadIdx.x; o < k2 * k2; o += blockDim.x) {
    const int i = o % k2, j = o / k2;
    FD[k1 + i + (int64_t)(k1 + j) * mp] = FD2[n2.e + i + (int64_t)(n2.e + j) * n2.mp];
  }
  const T* B12 = I.B12 + nd.oB12;
  const T* B21 = I.B21 + nd.oB21;
  // T1 = B12 (ku1 x kv2) * V^b_c2^T (kv2 x k2)
  wg_gemm_f<T>(n1.ku, k2, n2.kv,
               [&](int i, int l) { return B12[i + (int64_t)l * n1.ku]; },
               [&](int l, int j) { return FV2[n2.e + j + (int64_t)l * n2.mp]; },
               [&](int i, int j, T v) { T1[i + j * n1.ku] = v; }, red);
  wg_gemm_f<T>(n2.ku, k1, n1.kv,
               [&](int i, int l) { return B21[i + (int64_t)l * n2.ku]; },
               [&](int l, int j) { return FV1[n1.e + j + (int64_t)l * n1.mp]; },
               [&](int i, int j, T v) { T2[i + j * n2.ku] = v; }, red);
  __syncthreads();
  // off-diagonal blocks U~_c1 T1 and U~_c2 T2
  wg_gemm_f<T>(k1, k2, n1.ku,
               [&](int i, int l) { return utilde(FU1, n1, i, l); },
               [&](int l, int j) { return T1[l + j * n1.ku]; },
               [&](int i, int j, T v) { FD[i + (int64_t)(k1 + j) * mp] = v; }, red);
  wg_gemm_f<T>(k2, k1, n2.ku,
               [&](int i, int l) { return utilde(FU2, n2, i, l); },
               [&](int l, int j) { return T2[l + j * n2.ku]; },
               [&](int i, int j, T v) { FD[k1 + i + (int64_t)j * mp] = v; }, red);
  if (node == 0) return;
  // U' = blkdiag(U~_c1, U~_c2) R_t, V' = blkdiag(V^b_c1, V^b_c2) W_t
  const T* R = I.R + nd.oR;
  const T* W = I.W + nd.oW;
  const int kr = n1.ku + n2.ku, kw = n1.kv + n2.kv;
  T* FU = I.FU + nd.oFU;
  T* FV = I.FV + nd.oFV;
  wg_gemm_f<T>(k1, nd.ku, n1.ku,
               [&](int i, int l) { return utilde(FU1, n1, i, l); },
               [&](int l, int j) { return R[l + (int64_t)j * kr]; },
               [&](int i, int j, T v) { FU[i + (int64_t)j * mp] = v; }, red);
  wg_gemm_f<T>(k2, nd.ku, n2.ku,
               [&](int i, int l) { return utilde(FU2, n2, i, l); },
               [&](int l, int j) { return R[n1.ku + l + (int64_t)j * kr]; },
               [&](int i, int j, T v) { FU[k1 + i + (int64_t)j * mp] = v; }, red);
  wg_gemm_f<T>(k1, nd.kv, n1.kv,
               [&](int i, int l) { return FV1[n1.e + i + (int64_t)l * n1.mp]; },
               [&](int l, int j) { return W[l + (int64_t)j * kw]; },
               [&](int i, int j, T v) { FV[i + (int64_t)j * mp] = v; }, red);
  wg_gemm_f<T>(k2, nd.kv, n2.kv,
               [&](int i, int l) { return FV2[n2.e + i + (int64_t)l * n2.mp]; },
               [&](int l, int j) { return W[n1.kv + l + (int64_t)j * kw]; },
               [&](int i, int j, T v) { FV[k1 + i + (int64_t)j * mp] = v; }, red);
}

// Householder vector of [x; alpha] (pivot alpha at the end, QL) or
// [alpha; x] (LQ): H = I - tau u u^T, u = (pivot 1, x * scale), H [.] = beta e.
template <typename T>
__device__ __forceinline__ void householder(T alpha, T sigma, T& beta, T& tau, T& scale) {
  if (sigma == T(0)) {
    beta = alpha;
    tau = T(0);
    scale = T(0);
  } else {
    const T nrm = sqrt(alpha * alpha + sigma);
    beta = alpha >= T(0) ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scale = T(1) / (alpha - beta);
  }
}

// ---------------------------------------------------------------------------
// Step 1 on one (leaf or merged) block: QL of U', Q^T D', LQ, Z^T V'.
// D' lives in LDS; U' and V' are updated in the node's factor arrays.
// ---------------------------------------------------------------------------
template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_ulv_factor(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int mp = nd.mp, ku = nd.ku, kv = nd.kv, e = nd.e;
  const int ld = mp + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  T* Ds = smem;                  // mp x mp, ld = mp + 1
  T* vb = Ds + mp * ld;          // reflector, kMaxBlock
  T* sc = vb + kMaxBlock;        // tau broadcast
  T* FU = I.FU + nd.oFU;
  T* FV = I.FV + nd.oFV;
  T* FD = I.FD + nd.oFD;
  if (nd.is_leaf) {
    const T* D = I.D + nd.oD;
    const T* U = I.U + nd.oU;
    const T* V = I.V + nd.oV;
    wg_load(mp, mp, D, mp, Ds, ld);
    for (int o = tid; o < mp * ku; o += nt) FU[o] = U[o];
    for (int o = tid; o < mp * kv; o += nt) FV[o] = V[o];
  } else {
    wg_load(mp, mp, FD, mp, Ds, ld);
  }
  __syncthreads();
  // QL of U': columns j = ku-1 .. 0, pivot row e + j.
  if (e > 0) {
    for (int j = ku - 1; j >= 0; --j) {
      const int pr = e + j;
      T* Uj = FU + (int64_t)j * mp;
      if (tid < 64) {
        T s = 0;
        for (int r = tid; r < pr; r += 64) { const T x = Uj[r]; s += x * x; }
        s = wave_sum(s);
        const T alpha = Uj[pr];
        T beta, tau, scale;
        householder(alpha, s, beta, tau, scale);
        for (int r = tid; r < pr; r += 64) { const T v = Uj[r] * scale; vb[r] = v; Uj[r] = v; }
        if (tid == 0) {
          vb[pr] = T(1);
          sc[0] = tau;
          Uj[pr] = beta;
          I.tq[nd.otq + j] = tau;
        }
      }
      __syncthreads();
      const T tau = sc[0];
      if (tau != T(0)) {
        for (int c = tid; c < mp + j; c += nt) {
          T* col = c < mp ? Ds + c * ld : FU + (int64_t)(c - mp) * mp;
          T w = 0;
          for (int r = 0; r <= pr; ++r) w += vb[r] * col[r];
          w *= tau;
          for (int r = 0; r <= pr; ++r) col[r] -= w * vb[r];
        }
      }
      __syncthreads();
    }
  }
  // LQ of rows 0..e-1 of M = Q^T D'; V' <- Z^T V'.
  for (int i = 0; i < e; ++i) {
    if (tid < 64) {
      T s = 0;
      for (int c = i + 1 + tid; c < mp; c += 64) { const T x = Ds[i + c * ld]; s += x * x; }
      s = wave_sum(s);
      const T alpha = Ds[i + i * ld];
      T beta, tau, scale;
      householder(alpha, s, beta, tau, scale);
      for (int c = i + 1 + tid; c < mp; c += 64) {
        const T v = Ds[i + c * ld] * scale;
        vb[c] = v;
        Ds[i + c * ld] = v;
      }
      if (tid == 0) {
        vb[i] = T(1);
        sc[0] = tau;
        Ds[i + i * ld] = beta;
        I.tz[nd.otz + i] = tau;
        if (beta == T(0)) atomicOr(I.status, 1 << kStatusSingular);
      }
    }
    __syncthreads();
    const T tau = sc[0];
    if (tau != T(0)) {
      const int nr = mp - i - 1;
      for (int q = tid; q < nr + kv; q += nt) {
        if (q < nr) {
          const int r = i + 1 + q;
          T w = 0;
          for (int c = i; c < mp; ++c) w += Ds[r + c * ld] * vb[c];
          w *= tau;
          for (int c = i; c < mp; ++c) Ds[r + c * ld] -= w * vb[c];
        } else {
          T* col = FV + (int64_t)(q - nr) * mp;
          T w = 0;
          for (int c = i; c < mp; ++c) w += vb[c] * col[c];
          w *= tau;
          for (int c = i; c < mp; ++c) col[c] -= w * vb[c];
        }
      }
    }
    __syncthreads();
  }
  wg_store(mp, mp, Ds, ld, FD, mp);
}

// ---------------------------------------------------------------------------
// Root: LU with partial pivoting (FP64) of D'_root (or of D when p = 0).
// ---------------------------------------------------------------------------
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
  for (int o = tid; o < mp * mp; o += nt) Ls[o % mp + (o / mp) * ld] = (double)src[o];
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
        if (best == 0.0) atomicOr(I.status, 1 << kStatusSingular);
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
}

// ---------------------------------------------------------------------------
// Solve: right-hand side of node t in LDS (mp x nc).
// ---------------------------------------------------------------------------
template <typename T>
__device__ void sv_gather_rhs(const Inst<T>& I, const CallSV<T>& C, const NodeInfo& nd, int node,
                              int c0, int nc, T* bs, T* tmp, T* red) {
  const int mp = nd.mp;
  if (nd.is_leaf) {
    wg_load(mp, nc, C.B + nd.row0 + (int64_t)c0 * C.ldb, C.ldb, bs, mp);
    __syncthreads();
    return;
  }
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int k1 = n1.kept, k2 = n2.kept;
  const int64_t co = (int64_t)c0 * I.lds;
  const T* B12 = I.B12 + nd.oB12;
  const T* B21 = I.B21 + nd.oB21;
  const T* z1 = I.wz + n1.oz + co;
  const T* z2 = I.wz + n2.oz + co;
  const T* FU1 = I.FU + n1.oFU;
  const T* FU2 = I.FU + n2.oFU;
  // tmp1 = B12 z_c2 (ku1 x nc), tmp2 = B21 z_c1 (ku2 x nc)
  T* t1 = tmp;
  T* t2 = tmp + n1.ku * nc;
  const int64_t lds = I.lds;
  wg_gemm_f<T>(n1.ku, nc, n2.kv, [&](int i, int l) { return B12[i + (int64_t)l * n1.ku]; },
               [&](int l, int j) { return z2[l + j * lds]; },
               [&](int i, int j, T v) { t1[i + j * n1.ku] = v; }, red);
  wg_gemm_f<T>(n2.ku, nc, n1.kv, [&](int i, int l) { return B21[i + (int64_t)l * n2.ku]; },
               [&](int l, int j) { return z1[l + j * lds]; },
               [&](int i, int j, T v) { t2[i + j * n2.ku] = v; }, red);
  __syncthreads();
  const T* cc1 = I.wc + n1.oc + co;
  const T* cc2 = I.wc + n2.oc + co;
  wg_gemm_f<T>(k1, nc, n1.ku, [&](int i, int l) { return utilde(FU1, n1, i, l); },
               [&](int l, int j) { return t1[l + j * n1.ku]; },
               [&](int i, int j, T v) { bs[i + j * mp] = cc1[i + j * lds] - v; }, red);
  wg_gemm_f<T>(k2, nc, n2.ku, [&](int i, int l) { return utilde(FU2, n2, i, l); },
               [&](int l, int j) { return t2[l + j * n2.ku]; },
               [&](int i, int j, T v) { bs[k1 + i + j * mp] = cc2[i + j * lds] - v; }, red);
  __syncthreads();
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_sv_fwd(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int c0 = blockIdx.y * kRT;
  if (c0 >= C.nrhs) return;
  const int nc = min(kRT, C.nrhs - c0);
  const int mp = nd.mp, e = nd.e, ku = nd.ku, kv = nd.kv;
  const int tid = threadIdx.x, nt = blockDim.x;
  T* bs = smem;                     // mp x nc
  T* wv = bs + kMaxBlock * kRT;     // nc
  T* tmp = wv + kRT;                // 2 * kMaxRank * nc
  T* red = tmp + 2 * kMaxRank * kRT;
  sv_gather_rhs(I, C, nd, node, c0, nc, bs, tmp, red);
  const T* FU = I.FU + nd.oFU;
  const T* FD = I.FD + nd.oFD;
  const T* FV = I.FV + nd.oFV;
  const int64_t lds = I.lds, co = (int64_t)c0 * lds;
  // b~ = Q^T rhs: reflectors j = ku-1 .. 0
  if (e > 0) {
    for (int j = ku - 1; j >= 0; --j) {
      const int pr = e + j;
      const T tau = I.tq[nd.otq + j];
      if (tau == T(0)) continue;
      const T* Uj = FU + (int64_t)j * mp;
      wg_gemm_f<T>(1, nc, pr + 1,
                   [&](int, int l) { return l == pr ? T(1) : Uj[l]; },
                   [&](int l, int jj) { return bs[l + jj * mp]; },
                   [&](int, int jj, T v) { wv[jj] = v * tau; }, red);
      __syncthreads();
      for (int o = tid; o < (pr + 1) * nc; o += nt) {
        const int r = o % (pr + 1), jj = o / (pr + 1);
        bs[r + jj * mp] -= wv[jj] * (r == pr ? T(1) : Uj[r]);
      }
      __syncthreads();
    }
  }
  // y = L^{-1} b~_top (column-oriented forward substitution)
  for (int i = 0; i < e; ++i) {
    const T d = FD[i + (int64_t)i * mp];
    for (int jj = tid; jj < nc; jj += nt) bs[i + jj * mp] /= d;
    __syncthreads();
    const int rem = e - i - 1;
    for (int o = tid; o < rem * nc; o += nt) {
      const int r = i + 1 + o % rem, jj = o / rem;
      bs[r + jj * mp] -= FD[r + (int64_t)i * mp] * bs[i + jj * mp];
    }
    __syncthreads();
  }
  // c = b~_bot - D~21 y
  T* cout = I.wc + nd.oc + co;
  wg_gemm_f<T>(nd.kept, nc, e, [&](int i, int l) { return FD[e + i + (int64_t)l * mp]; },
               [&](int l, int j) { return bs[l + j * mp]; },
               [&](int i, int j, T v) { cout[i + j * lds] = bs[e + i + j * mp] - v; }, red);
  // y -> work
  T* yout = I.wy + nd.oy + co;
  for (int o = tid; o < e * nc; o += nt) {
    const int r = o % e, jj = o / e;
    yout[r + jj * lds] = bs[r + jj * mp];
  }
  // z = V^_top^T y (+ W^T [z_c1; z_c2])
  T* zout = I.wz + nd.oz + co;
  if (nd.is_leaf) {
    wg_gemm_f<T>(kv, nc, e, [&](int i, int l) { return FV[l + (int64_t)i * mp]; },
                 [&](int l, int j) { return bs[l + j * mp]; },
                 [&](int i, int j, T v) { zout[i + j * lds] = v; }, red);
  } else {
    const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
    const T* W = I.W + nd.oW;
    const int kw = n1.kv + n2.kv;
    const T* z1 = I.wz + n1.oz + co;
    const T* z2 = I.wz + n2.oz + co;
    wg_gemm_f<T>(kv, nc, e + kw,
                 [&](int i, int l) {
                   return l < e ? FV[l + (int64_t)i * mp] : W[(l - e) + (int64_t)i * kw];
                 },
                 [&](int l, int j) {
                   return l < e ? bs[l + j * mp]
                                : (l - e < n1.kv ? z1[(l - e) + j * lds]
                                                 : z2[(l - e - n1.kv) + j * lds]);
                 },
                 [&](int i, int j, T v) { zout[i + j * lds] = v; }, red);
  }
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_sv_root(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int c0 = blockIdx.y * kRT;
  if (c0 >= C.nrhs) return;
  const int nc = min(kRT, C.nrhs - c0);
  const int mp = nd.mp;
  const int tid = threadIdx.x, nt = blockDim.x;
  T* bs = smem;
  T* tmp = bs + kMaxBlock * kRT;
  T* red = tmp + 2 * kMaxRank * kRT;
  double* xs = reinterpret_cast<double*>(red + kNT);   // mp x nc in FP64
  sv_gather_rhs(I, C, nd, node, c0, nc, bs, tmp, red);
  for (int o = tid; o < mp * nc; o += nt) xs[o] = (double)bs[o];
  __syncthreads();
  const double* LU = I.rootLU;
  // row interchanges, then L (unit) and U
  if (tid < nc)
    for (int j = 0; j < mp; ++j) {
      const int pr = I.piv[j];
      if (pr != j) {
        const double t = xs[j + tid * mp];
        xs[j + tid * mp] = xs[pr + tid * mp];
        xs[pr + tid * mp] = t;
      }
    }
  __syncthreads();
  for (int i = 0; i < mp; ++i) {
    const int rem = mp - i - 1;
    for (int o = tid; o < rem * nc; o += nt) {
      const int r = i + 1 + o % rem, jj = o / rem;
      xs[r + jj * mp] -= LU[r + (int64_t)i * mp] * xs[i + jj * mp];
    }
    __syncthreads();
  }
  for (int i = mp - 1; i >= 0; --i) {
    for (int jj = tid; jj < nc; jj += nt) xs[i + jj * mp] /= LU[i + (int64_t)i * mp];
    __syncthreads();
    for (int o = tid; o < i * nc; o += nt) {
      const int r = o % i, jj = o / i;
      xs[r + jj * mp] -= LU[r + (int64_t)i * mp] * xs[i + jj * mp];
    }
    __syncthreads();
  }
  if (I.p == 0) {
    T* out = C.B + nd.row0 + (int64_t)c0 * C.ldb;
    for (int o = tid; o < mp * nc; o += nt) out[o % mp + (o / mp) * C.ldb] = (T)xs[o];
    return;
  }
  const NodeInfo n1 = I.nodes[1], n2 = I.nodes[2];
  const int64_t lds = I.lds, co = (int64_t)c0 * lds;
  T* x1 = I.wx + n1.ox + co;
  T* x2 = I.wx + n2.ox + co;
  for (int o = tid; o < mp * nc; o += nt) {
    const int r = o % mp, jj = o / mp;
    if (r < n1.kept) x1[r + jj * lds] = (T)xs[o];
    else x2[r - n1.kept + jj * lds] = (T)xs[o];
  }
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_sv_bwd(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int c0 = blockIdx.y * kRT;
  if (c0 >= C.nrhs) return;
  const int nc = min(kRT, C.nrhs - c0);
  const int mp = nd.mp, e = nd.e;
  const int tid = threadIdx.x, nt = blockDim.x;
  T* bs = smem;
  T* wv = bs + kMaxBlock * kRT;
  T* red = wv + kRT;
  const int64_t lds = I.lds, co = (int64_t)c0 * lds;
  const T* yin = I.wy + nd.oy + co;
  const T* xin = I.wx + nd.ox + co;
  for (int o = tid; o < mp * nc; o += nt) {
    const int r = o % mp, jj = o / mp;
    bs[o] = r < e ? yin[r + jj * lds] : xin[r - e + jj * lds];
  }
  __syncthreads();
  const T* FD = I.FD + nd.oFD;
  for (int i = e - 1; i >= 0; --i) {
    const T tau = I.tz[nd.otz + i];
    if (tau == T(0)) continue;
    wg_gemm_f<T>(1, nc, mp - i,
                 [&](int, int l) { return l == 0 ? T(1) : FD[i + (int64_t)(i + l) * mp]; },
                 [&](int l, int jj) { return bs[i + l + jj * mp]; },
                 [&](int, int jj, T v) { wv[jj] = v * tau; }, red);
    __syncthreads();
    for (int o = tid; o < (mp - i) * nc; o += nt) {
      const int l = o % (mp - i), jj = o / (mp - i);
      const T v = l == 0 ? T(1) : FD[i + (int64_t)(i + l) * mp];
      bs[i + l + jj * mp] -= wv[jj] * v;
    }
    __syncthreads();
  }
  if (nd.is_leaf) {
    T* out = C.B + nd.row0 + (int64_t)c0 * C.ldb;
    for (int o = tid; o < mp * nc; o += nt) out[o % mp + (o / mp) * C.ldb] = bs[o];
    return;
  }
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  T* x1 = I.wx + n1.ox + co;
  T* x2 = I.wx + n2.ox + co;
  for (int o = tid; o < mp * nc; o += nt) {
    const int r = o % mp, jj = o / mp;
    if (r < n1.kept) x1[r + jj * lds] = bs[o];
    else x2[r - n1.kept + jj * lds] = bs[o];
  }
}

// ---------------------------------------------------------------------------
template <typename T>
void launch_ulv(UlvStep step, const KArgs<T, CallSV<T>>& a, int nblocks, int ytiles, int max_mp,
                hipStream_t s) {
  if (nblocks <= 0) return;
  const bool batch = a.tasks != nullptr;
  dim3 block(kNT);
  size_t sm = 0;
  dim3 grid(nblocks, 1);
  const size_t TB = sizeof(T);
  switch (step) {
    case UlvStep::Merge: sm = (2 * kMaxRank * kMaxRank + kNT) * TB; break;
    case UlvStep::Factor: sm = ((size_t)max_mp * (max_mp + 1) + kMaxBlock + 8) * TB; break;
    case UlvStep::RootLU: sm = (size_t)max_mp * (max_mp + 1) * sizeof(double); break;
    case UlvStep::Fwd:
    case UlvStep::Root:
    case UlvStep::Bwd:
      grid.y = ytiles;
      sm = ((size_t)kMaxBlock * kRT + kRT + 2 * kMaxRank * kRT + kNT) * TB +
           (step == UlvStep::Root ? (size_t)kMaxBlock * kRT * sizeof(double) : 0);
      break;
  }
#define HSS_LAUNCH(K)                                                         \
  if (batch) hipLaunchKernelGGL((K<T, true>), grid, block, sm, s, a);         \
  else hipLaunchKernelGGL((K<T, false>), grid, block, sm, s, a);
  switch (step) {
    case UlvStep::Merge: HSS_LAUNCH(k_ulv_merge); break;
    case UlvStep::Factor: HSS_LAUNCH(k_ulv_factor); break;
    case UlvStep::RootLU: HSS_LAUNCH(k_ulv_root_lu); break;
    case UlvStep::Fwd: HSS_LAUNCH(k_sv_fwd); break;
    case UlvStep::Root: HSS_LAUNCH(k_sv_root); break;
    case UlvStep::Bwd: HSS_LAUNCH(k_sv_bwd); break;
  }
#undef HSS_LAUNCH
}

template void launch_ulv<double>(UlvStep, const KArgs<double, CallSV<double>>&, int, int, int,
                                 hipStream_t);
template void launch_ulv<float>(UlvStep, const KArgs<float, CallSV<float>>&, int, int, int,
                                hipStream_t);

}  // namespace hss
