// HSS matrix x block product Y = A X (Sec. 4.1) for blocks of several
// right-hand sides, one launch per tree level:
//   leaf up   x^_i = V_i^T X_i                                  (leaves)
//   up        x^_t = W_t^T [x^_c1; x^_c2] (below the root) and the core
//             blocks y^_c1 = B12_t x^_c2, y^_c2 = B21_t x^_c1    (levels p-1 .. 0)
//   down      [y^_c1; y^_c2] += R_t y^_t                         (levels 1 .. p-1)
//   leaf out  Y_i = D_i X_i + U_i y^_i                           (leaves)
// Every work-group stages the operands of its node (and column tile) in LDS
// with all global reads in flight together, then forms its outputs as dot
// products out of LDS.  The leaf-out kernel streams D_i and U_i once per
// 32-column tile: thread (row r, half h) keeps row r of 16 output columns in
// registers, reads D_i and U_i coalesced down their columns and takes the
// X / y^ entries as LDS broadcasts.  Ranks <= 32 and leaves <= 128 rows.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {

namespace {

constexpr int kWT = 256;   // threads of every kernel here
constexpr int kWR = 32;    // largest rank
constexpr int kWC = 16;    // right-hand-side columns per tile of the level kernels
constexpr int kWL = 32;    // right-hand-side columns per tile of the leaf-out kernel

// Node t of the launch: a level is a contiguous heap range from node0.
// Stage a rows x cols block (element (i, j) at src[i + j*ld]) into LDS at
// dst[i*lr + j] (TR) or dst[i + j*lr]: NPT elements per thread, every load
// issued (from a clamped, valid address) before the first store.
template <typename T, int NPT, bool TR>
struct Stage {
  T v[NPT];
  __device__ __forceinline__ void load(const T* src, int64_t ld, int rows, int cols) {
    const int total = rows * cols;
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const int o = min((int)threadIdx.x + u * kWT, max(total - 1, 0));
      const int i = o % max(rows, 1), j = o / max(rows, 1);
      v[u] = total > 0 ? src[i + j * ld] : T(0);
    }
  }
  __device__ __forceinline__ void store(T* dst, int lr, int rows, int cols) const {
    const int total = rows * cols;
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const int o = (int)threadIdx.x + u * kWT;
      if (o < total) {
        const int i = o % rows, j = o / rows;
        dst[TR ? i * lr + j : i + j * lr] = v[u];
      }
    }
  }
};

// LDS row of a kWC-column tile: 16-byte aligned halves of eight columns.
constexpr int kXR = kWC + 2;

// s[c] += coef * x[c] for the eight columns of one half-tile row (two 16-byte
// LDS reads, the same address for every lane of the wavefront).
template <typename T>
__device__ __forceinline__ void axpy8(T (&s)[8], T coef, const T* x) {
#pragma unroll
  for (int c = 0; c < 8; ++c) s[c] += coef * x[c];
}

// x^_i = V_i^T X_i for leaf i and columns c0 .. c0 + kWC - 1: wavefront w sums
// a quarter of the rows of V and X (rows w kb .. w kb + kb - 1, kb = m / 4
// rounded up); lane (a = lane % 32, half h = lane / 32) keeps
// x^[a, 8h .. 8h + 7]; the four partial sums meet in LDS.  MR: the largest
// leaf the launch takes (64 or 128), which sizes the LDS tiles.
template <typename T, bool BATCH, int MR>
__global__ __launch_bounds__(kWT) void k_mmw_leaf_up(KArgs<T, CallMM<T>> a) {
  __shared__ T Vs[MR * (kWR + 1)];              // Vs[k][a] (row k of V)
  __shared__ __align__(16) T Xs[MR * kXR];       // Xs[k][c]
  T* Ps = Vs;   // the four partial sums, once V has been read
  static_assert(4 * kWR * kWC <= MR * (kWR + 1), "partial sums fit in Vs");
  Inst<T> I; CallMM<T> C; int t;
  resolve<BATCH>(a, I, C, t);
  if (gated_off(C.gate)) return;
  const int c0 = blockIdx.y * kWC;
  const NodeInfo nd = I.nodes[t];
  const int m = nd.m, kv = nd.kv, nc = min(kWC, C.nrhs - c0);
  {
    Stage<T, MR * kWR / kWT, true> sv;
    Stage<T, MR * kWC / kWT, true> sx;
    sv.load(I.V + nd.oV, m, m, kv);
    sx.load(C.X + nd.row0 + (int64_t)c0 * C.ldx, C.ldx, m, nc);
    sv.store(Vs, kWR + 1, m, kv);
    sx.store(Xs, kXR, m, nc);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  T s[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) s[c] = T(0);
  const int kb = (m + 3) >> 2, k1 = min(kb * w + kb, m);
  for (int k = kb * w; k < k1; ++k) axpy8(s, Vs[k * (kWR + 1) + r], Xs + k * kXR + 8 * h);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 8; ++c) Ps[(w * kWR + r) * kWC + 8 * h + c] = s[c];
  __syncthreads();
  T* xo = I.xh + nd.oxh + (int64_t)c0 * I.ldm;
  for (int o = threadIdx.x; o < kWR * kWC; o += kWT) {
    const int ra = o % kWR, c = o / kWR;
    const T v = (Ps[ra * kWC + c] + Ps[(kWR + ra) * kWC + c]) +
                (Ps[(2 * kWR + ra) * kWC + c] + Ps[(3 * kWR + ra) * kWC + c]);
    if (ra < kv && c < nc) xo[ra + (int64_t)c * I.ldm] = v;
  }
}

// Node t at one level: x^_t = W_t^T [x^_c1; x^_c2] below the root, and the
// core blocks y^_c1 = B12_t x^_c2, y^_c2 = B21_t x^_c1.  Thread (row i, half
// h) forms one output row for eight columns as a dot product of a
// coefficient row (column i of W_t, or a row of B12 / B21) with rows of the
// stacked children's x^.
template <typename T, bool BATCH>
__global__ __launch_bounds__(kWT) void k_mmw_up(KArgs<T, CallMM<T>> a) {
  __shared__ __align__(16) T Xs[2 * kWR * kXR];      // [x^_c1; x^_c2]
  __shared__ T Ws[2 * kWR * (kWR + 1)];              // Ws[j][b] = W_t(j, b)
  __shared__ T Bs[2 * kWR * (kWR + 1)];              // B12 rows 0..ku1-1, then B21
  Inst<T> I; CallMM<T> C; int t;
  resolve<BATCH>(a, I, C, t);
  if (gated_off(C.gate)) return;
  const int c0 = blockIdx.y * kWC;
  const NodeInfo nd = I.nodes[t], n1 = I.nodes[2 * t + 1], n2 = I.nodes[2 * t + 2];
  const int kv1 = n1.kv, kv2 = n2.kv, ku1 = n1.ku, ku2 = n2.ku, kw = kv1 + kv2;
  const int kv = t > 0 ? nd.kv : 0;
  const int nc = min(kWC, C.nrhs - c0);
  {
    constexpr int NX = kWR * kWC / kWT, NW = 2 * kWR * kWR / kWT, NB = kWR * kWR / kWT;
    Stage<T, NX, true> x1, x2;
    Stage<T, NW, true> sw;
    Stage<T, NB, true> b12, b21;
    x1.load(I.xh + n1.oxh + (int64_t)c0 * I.ldm, I.ldm, kv1, nc);
    x2.load(I.xh + n2.oxh + (int64_t)c0 * I.ldm, I.ldm, kv2, nc);
    sw.load(I.W + (kv > 0 ? nd.oW : 0), kw, kw, kv);
    b12.load(I.B12 + nd.oB12, ku1, ku1, kv2);
    b21.load(I.B21 + nd.oB21, ku2, ku2, kv1);
    x1.store(Xs, kXR, kv1, nc);
    x2.store(Xs + kv1 * kXR, kXR, kv2, nc);
    sw.store(Ws, kWR + 1, kw, kv);
    b12.store(Bs, kWR + 1, ku1, kv2);
    b21.store(Bs + ku1 * (kWR + 1), kWR + 1, ku2, kv1);
  }
  __syncthreads();
  // rows 0..kv-1: x^_t; then ku1 rows of y^_c1; then ku2 rows of y^_c2 (<= 96)
  const int i = threadIdx.x & 127, h = threadIdx.x >> 7;
  const int rows = kv + ku1 + ku2;
  if (i >= rows) return;
  const T* cf;     // coefficient j at cf[j * cs]
  int cs, len;
  const T* xr;     // row j of the x^ operand at xr + j * kXR
  T* out;
  if (i < kv) {
    cf = Ws + i; cs = kWR + 1; len = kw; xr = Xs; out = I.xh + nd.oxh + i;
  } else if (i < kv + ku1) {
    const int b = i - kv;
    cf = Bs + b * (kWR + 1); cs = 1; len = kv2; xr = Xs + kv1 * kXR; out = I.yh + n1.oyh + b;
  } else {
    const int b = i - kv - ku1;
    cf = Bs + (ku1 + b) * (kWR + 1); cs = 1; len = kv1; xr = Xs; out = I.yh + n2.oyh + b;
  }
  T s[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) s[c] = T(0);
  for (int j = 0; j < len; ++j) axpy8(s, cf[j * cs], xr + j * kXR + 8 * h);
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (8 * h + c < nc) out[(int64_t)(c0 + 8 * h + c) * I.ldm] = s[c];
}

// Node t below the root: [y^_c1; y^_c2] += R_t y^_t.  Thread (row i, quarter
// q) updates row i of four columns.
template <typename T, bool BATCH>
__global__ __launch_bounds__(kWT) void k_mmw_down(KArgs<T, CallMM<T>> a) {
  __shared__ __align__(16) T Ys[kWR * kXR];          // y^_t
  __shared__ T Rs[2 * kWR * (kWR + 1)];              // Rs[i][j] = R_t(i, j)
  Inst<T> I; CallMM<T> C; int t;
  resolve<BATCH>(a, I, C, t);
  if (gated_off(C.gate)) return;
  const int c0 = blockIdx.y * kWC;
  const NodeInfo nd = I.nodes[t], n1 = I.nodes[2 * t + 1], n2 = I.nodes[2 * t + 2];
  const int ku = nd.ku, ku1 = n1.ku, ku2 = n2.ku, kr = ku1 + ku2;
  const int nc = min(kWC, C.nrhs - c0);
  {
    Stage<T, kWR * kWC / kWT, true> sy;
    Stage<T, 2 * kWR * kWR / kWT, true> sr;
    sy.load(I.yh + nd.oyh + (int64_t)c0 * I.ldm, I.ldm, ku, nc);
    sr.load(I.R + nd.oR, kr, kr, ku);
    sy.store(Ys, kXR, ku, nc);
    sr.store(Rs, kWR + 1, kr, ku);
  }
  __syncthreads();
  const int i = threadIdx.x & 63, q = threadIdx.x >> 6;
  if (i >= kr) return;
  T s[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) s[c] = T(0);
  for (int j = 0; j < ku; ++j) {
    const T rij = Rs[i * (kWR + 1) + j];
    const T* yj = Ys + j * kXR + 4 * q;
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] += rij * yj[c];
  }
  T* yc = i < ku1 ? I.yh + n1.oyh + i : I.yh + n2.oyh + (i - ku1);
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (4 * q + c < nc) yc[(int64_t)(c0 + 4 * q + c) * I.ldm] += s[c];
}

// Y_i = D_i X_i + U_i y^_i for leaf i and columns c0 .. c0 + kWL - 1: thread
// (r = tid % 128, h = tid / 128) forms row r of columns 16h .. 16h + 15.
template <typename T, bool BATCH>
__global__ __launch_bounds__(kWT) void k_mmw_leaf_out(KArgs<T, CallMM<T>> a) {
  constexpr int XL = kWL + 2;                // LDS row: 16-byte aligned halves
  __shared__ __align__(16) T Xs[kMaxBlock * XL];
  __shared__ __align__(16) T Ys[kWR * XL];
  Inst<T> I; CallMM<T> C; int t;
  resolve<BATCH>(a, I, C, t);
  if (gated_off(C.gate)) return;
  const int c0 = blockIdx.y * kWL;
  const NodeInfo nd = I.nodes[t];
  const int m = nd.m, ku = I.p > 0 ? nd.ku : 0, nc = min(kWL, C.nrhs - c0);
  {
    Stage<T, kMaxBlock * kWL / kWT, true> sx;
    Stage<T, kWR * kWL / kWT, true> sy;
    sx.load(C.X + nd.row0 + (int64_t)c0 * C.ldx, C.ldx, m, nc);
    sy.load(I.yh + nd.oyh + (int64_t)c0 * I.ldm, I.ldm, ku, nc);
    // columns past nc read as zero
    for (int o = threadIdx.x; o < kMaxBlock * XL; o += kWT) Xs[o] = T(0);
    for (int o = threadIdx.x; o < kWR * XL; o += kWT) Ys[o] = T(0);
    __syncthreads();
    sx.store(Xs, XL, m, nc);
    sy.store(Ys, XL, ku, nc);
  }
  __syncthreads();
  const int r = threadIdx.x & (kMaxBlock - 1), h = threadIdx.x / kMaxBlock;
  const int rc = min(r, m - 1);
  T acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = T(0);
  const T* Dr = I.D + nd.oD + rc;
  constexpr int KB = 16;   // columns of D in flight
  T dv[KB];
#pragma unroll
  for (int u = 0; u < KB; ++u) dv[u] = Dr[(int64_t)min(u, m - 1) * m];
  for (int k0 = 0; k0 < m; k0 += KB) {
    T dn[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) dn[u] = Dr[(int64_t)min(k0 + KB + u, m - 1) * m];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int k = k0 + u;
      const T d = k < m ? dv[u] : T(0);
      const T* xk = Xs + min(k, kMaxBlock - 1) * XL + 16 * h;
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[c] += d * xk[c];
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) dv[u] = dn[u];
  }
  if (ku > 0) {
    const T* Ur = I.U + nd.oU + rc;
    T uv[kWR];
#pragma unroll
    for (int j = 0; j < kWR; ++j) uv[j] = Ur[(int64_t)min(j, ku - 1) * m];
#pragma unroll
    for (int j = 0; j < kWR; ++j) {
      const T u = j < ku ? uv[j] : T(0);
      const T* yk = Ys + j * XL + 16 * h;
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[c] += u * yk[c];
    }
  }
  if (r < m) {
    T* Yr = C.Y + nd.row0 + r;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (16 * h + c < nc) Yr[(int64_t)(c0 + 16 * h + c) * C.ldy] = acc[c];
  }
}

// Y = D X + U y^ for a tile of at most 16 columns: row r of the leaf on lane
// r of one of G = 256 / RW row groups (RW = 64 for leaves of at most 64 rows,
// else 128), the inner dimension (columns of D, then of U) split over the
// groups, the G partial sums reduced through LDS: every entry of D and U is
// read once, by a coalesced column read.
template <typename T, bool BATCH, int RW>
__global__ __launch_bounds__(kWT) void k_mmw_leaf_out_n(KArgs<T, CallMM<T>> a) {
  constexpr int G = kWT / RW;
  constexpr int NC = 16;
  constexpr int PP = NC + 1;   // pitch of the partial sums
  // the X and y^ tiles, then (after a barrier) the partial sums in the same
  // space: the smaller footprint keeps more work-groups per compute unit
  constexpr int kTiles = (kMaxBlock + kWR) * NC, kParts = kWT * PP;
  __shared__ __align__(16) T lds[kTiles > kParts ? kTiles : kParts];
  T* Xs = lds;
  T* Ys = lds + kMaxBlock * NC;
  T* Ps = lds;
  Inst<T> I; CallMM<T> C; int t;
  resolve<BATCH>(a, I, C, t);
  if (gated_off(C.gate)) return;
  const int c0 = blockIdx.y * NC;
  const NodeInfo nd = I.nodes[t];
  const int m = nd.m, ku = I.p > 0 ? nd.ku : 0, nc = min(NC, C.nrhs - c0);
  const int tid = threadIdx.x;
  // X and y^ tiles, columns past nc zero
  for (int o = tid; o < m * NC; o += kWT) {
    const int c = o / m, k = o - c * m;
    Xs[k * NC + c] = c < nc ? C.X[nd.row0 + k + (int64_t)(c0 + c) * C.ldx] : T(0);
  }
  for (int o = tid; o < ku * NC; o += kWT) {
    const int c = o / ku, j = o - c * ku;
    Ys[j * NC + c] = c < nc ? I.yh[nd.oyh + j + (int64_t)(c0 + c) * I.ldm] : T(0);
  }
  __syncthreads();
  const int r = tid % RW, h = tid / RW;
  const int rc = min(r, m - 1);
  T acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = T(0);
  {
    const int kb = (m + G - 1) / G, k0 = h * kb, k1 = min(m, k0 + kb);
    const T* Dr = I.D + nd.oD + rc;
    constexpr int KB = 8;   // columns of D in flight
    for (int kk = k0; kk < k1; kk += KB) {
      T dv[KB];
#pragma unroll
      for (int u = 0; u < KB; ++u) dv[u] = Dr[(int64_t)min(kk + u, k1 - 1) * m];
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const T d = kk + u < k1 ? dv[u] : T(0);
        const T* xk = Xs + min(kk + u, m - 1) * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += d * xk[c];
      }
    }
  }
  if (ku > 0) {
    const int jb = (ku + G - 1) / G, j0 = h * jb, j1 = min(ku, j0 + jb);
    const T* Ur = I.U + nd.oU + rc;
    for (int j = j0; j < j1; ++j) {
      const T u = Ur[(int64_t)j * m];
      const T* yk = Ys + j * NC;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += u * yk[c];
    }
  }
  __syncthreads();   // every read of the tiles done
#pragma unroll
  for (int c = 0; c < NC; ++c) Ps[tid * PP + c] = acc[c];
  __syncthreads();
  for (int o = tid; o < RW * NC; o += kWT) {
    const int c = o / RW, rr = o - c * RW;
    T sum = T(0);
#pragma unroll
    for (int g = 0; g < G; ++g) sum += Ps[(g * RW + rr) * PP + c];
    if (rr < m && c < nc) C.Y[nd.row0 + rr + (int64_t)(c0 + c) * C.ldy] = sum;
  }
}

}  // namespace

bool mmw_fits(int max_leaf, int max_k) { return max_leaf <= kMaxBlock && max_k <= kWR; }

template <typename T>
void launch_mmw(MMWStep step, const KArgs<T, CallMM<T>>& a, int nblocks, int nrhs,
                hipStream_t s, int max_m) {
  if (nblocks <= 0 || nrhs <= 0) return;
  static const char* n64[] = {"mmw_leaf_up_f64", "mmw_up_f64", "mmw_down_f64", "mmw_leaf_out_f64"};
  static const char* n32[] = {"mmw_leaf_up_f32", "mmw_up_f32", "mmw_down_f32", "mmw_leaf_out_f32"};
  TimedLaunch tl((sizeof(T) == 8 ? n64 : n32)[(int)step], s);
  const dim3 b(kWT);
  const dim3 g(nblocks, (nrhs + kWC - 1) / kWC), gl(nblocks, (nrhs + kWL - 1) / kWL);
  const bool batch = a.tasks != nullptr;
#define HSS_MMW(K, G)                                                  \
  if (batch) hipLaunchKernelGGL((K<T, true>), G, b, 0, s, a);          \
  else hipLaunchKernelGGL((K<T, false>), G, b, 0, s, a);
  switch (step) {
    case MMWStep::LeafUp:
      if (max_m <= 64) {
        if (batch) hipLaunchKernelGGL((k_mmw_leaf_up<T, true, 64>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_mmw_leaf_up<T, false, 64>), g, b, 0, s, a);
      } else {
        if (batch) hipLaunchKernelGGL((k_mmw_leaf_up<T, true, kMaxBlock>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_mmw_leaf_up<T, false, kMaxBlock>), g, b, 0, s, a);
      }
      break;
    case MMWStep::Up: HSS_MMW(k_mmw_up, g); break;
    case MMWStep::Down: HSS_MMW(k_mmw_down, g); break;
    case MMWStep::LeafOut:
      if (nrhs <= 16) {
        // narrow tiles: every row lane and every read of D and U useful
        const dim3 gn(nblocks, 1);
        if (max_m <= 64) {
          if (batch) hipLaunchKernelGGL((k_mmw_leaf_out_n<T, true, 64>), gn, b, 0, s, a);
          else hipLaunchKernelGGL((k_mmw_leaf_out_n<T, false, 64>), gn, b, 0, s, a);
        } else {
          if (batch) hipLaunchKernelGGL((k_mmw_leaf_out_n<T, true, 128>), gn, b, 0, s, a);
          else hipLaunchKernelGGL((k_mmw_leaf_out_n<T, false, 128>), gn, b, 0, s, a);
        }
      } else {
        HSS_MMW(k_mmw_leaf_out, gl);
      }
      break;
  }
#undef HSS_MMW
}

template void launch_mmw<double>(MMWStep, const KArgs<double, CallMM<double>>&, int, int,
                                 hipStream_t, int);
template void launch_mmw<float>(MMWStep, const KArgs<float, CallMM<float>>&, int, int,
                                hipStream_t, int);

}  // namespace hss
