// Telescoped ULV solve (Sec. 4.3, Steps 2 and 4 applied to a block of
// right-hand sides with the stored factors).  One wavefront per (node,
// right-hand-side column): lane l holds rows l and l + 64 of the node's
// vector in registers, factor columns are read coalesced, reductions are
// wavefront reductions and broadcasts are lane reads.
//   forward:  rhs_t = b_i (leaf) or [c_c1 - U~_c1 B12_t z_c2; c_c2 - U~_c2 B21_t z_c1];
//             b~ = Q^T rhs; y = L^{-1} b~_top; c = b~_bot - D~21 y;
//             z_t = V^_top^T y (+ W_t^T [z_c1; z_c2] at internal nodes)
//   root:     x' = (P L U)^{-1} rhs_root in FP64, split into x^_c1, x^_c2
//   backward: x'_t = Z_t [y; x^_t], split to the children (leaves: into B).
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {

constexpr int kSW = 4;   // wavefronts per work-group (direct sweeps)
constexpr int kSWS = 8;  // wavefronts per work-group of the staged forward sweep on
                         // short levels and of the root: one factor block each, so
                         // the staging is one round trip
constexpr int kSWSMaxItems = 1024;   // longest level given kSWS wavefronts

template <typename T>
__device__ __forceinline__ T bcast(T v, int src) {
  return lane_read(v, src);
}
template <typename T>
__device__ __forceinline__ T row_of(T x0, T x1, int row) {
  return bcast(row < 64 ? x0 : x1, row & 63);
}

// v[0..63] per lane; lane l returns the sum over all lanes of v[l]
// (butterfly: at width w a lane keeps the half selected by bit w of its id and
// receives the partner's copy of that half).
template <typename T, int W>
__device__ __forceinline__ void tsum_step(T (&v)[64], bool b) {
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const T send = b ? v[k] : v[W + k];
    const T keep = b ? v[W + k] : v[k];
    v[k] = keep + __shfl_xor(send, W, 64);
  }
}

// tsum_step on a 32-entry array (widths 16 .. 1).
template <typename T, int W>
__device__ __forceinline__ void tsum_half(T (&v)[32], bool b) {
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const T send = b ? v[k] : v[W + k];
    const T keep = b ? v[W + k] : v[k];
    v[k] = keep + __shfl_xor(send, W, 64);
  }
}

template <typename T>
__device__ __forceinline__ T wave_transpose_sum64(T (&v)[64]) {
  const int lane = threadIdx.x & 63;
  tsum_step<T, 32>(v, (lane & 32) != 0);
  tsum_step<T, 16>(v, (lane & 16) != 0);
  tsum_step<T, 8>(v, (lane & 8) != 0);
  tsum_step<T, 4>(v, (lane & 4) != 0);
  tsum_step<T, 2>(v, (lane & 2) != 0);
  tsum_step<T, 1>(v, (lane & 1) != 0);
  return v[0];
}

// v[0..31] per lane; lanes l and l + 32 return the sum over all lanes of
// v[l & 31].
template <typename T>
__device__ __forceinline__ T wave_transpose_sum32(T (&v)[32]) {
  const int lane = threadIdx.x & 63;
  // the 16-wide and narrower butterflies of the 64-value version, then the
  // two 32-lane halves added
  T x[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) x[k] = v[k];
  tsum_half<T, 16>(x, (lane & 16) != 0);
  tsum_half<T, 8>(x, (lane & 8) != 0);
  tsum_half<T, 4>(x, (lane & 4) != 0);
  tsum_half<T, 2>(x, (lane & 2) != 0);
  tsum_half<T, 1>(x, (lane & 1) != 0);
  return x[0] + __shfl_xor(x[0], 32, 64);
}

// Where the sweeps read a node's factors: the factor arrays themselves, or
// copies staged in LDS (one bulk load before the sequential steps).
template <typename T>
struct NodeSrc {
  const T* U; int ldu;     // Q reflectors (FU), mp x ku
  const T* L; int ldl;     // FD columns 0..e-1: L above, D~21 below
  const T* V; int ldv;     // FV rows 0..e-1 (V^_top)
  const T* W; int ldw;     // W_t
  const T* U1; int ldu1; bool m1;   // U~ of the children; m: read zeros above the diagonal
  const T* U2; int ldu2; bool m2;
  const T* B12; int ld12;
  const T* B21; int ld21;
  const T* Z; int ldz;     // FZ (backward)
};

template <typename T>
__device__ __forceinline__ T ut(const T* U, int ld, bool m, int a, int x) {
  const T v = U[a + x * ld];
  return (m & (a < x)) ? T(0) : v;
}

// Row r of [a; b] (ka + kb rows), zero past the end; both reads are issued
// from clamped (valid) addresses whatever r is.
template <typename T>
__device__ __forceinline__ T stacked(const T* a, int ka, const T* b, int kb, int r) {
  // (ka and kb are uniform: an empty part is not read at all)
  const T va = ka > 0 ? a[min(r, ka - 1)] : T(0);
  const T vb = kb > 0 ? b[min(max(r - ka, 0), kb - 1)] : T(0);
  return r < ka ? va : (r < ka + kb ? vb : T(0));
}

template <typename T>
__device__ __forceinline__ NodeSrc<T> src_global(const Inst<T>& I, const NodeInfo& nd,
                                                 const NodeInfo& n1, const NodeInfo& n2) {
  NodeSrc<T> S{};
  S.U = I.FU + nd.oFU; S.ldu = nd.mp;
  S.L = I.FD + nd.oFD; S.ldl = nd.mp;
  S.V = I.FV + nd.oFV; S.ldv = nd.mp;
  S.Z = I.FZ + nd.oFZ; S.ldz = nd.mp;
  if (!nd.is_leaf) {
    S.W = I.W + nd.oW; S.ldw = n1.kv + n2.kv;
    S.U1 = I.FU + n1.oFU + n1.e; S.ldu1 = n1.mp; S.m1 = n1.e > 0;
    S.U2 = I.FU + n2.oFU + n2.e; S.ldu2 = n2.mp; S.m2 = n2.e > 0;
    S.B12 = I.B12 + nd.oB12; S.ld12 = n1.ku;
    S.B21 = I.B21 + nd.oB21; S.ld21 = n2.ku;
  }
  return S;
}

// Copy a rows x cols block (rows <= 128) into LDS with every thread of the
// work-group: thread t covers rows t%64 and t%64 + 64 of the columns
// congruent to t/64; 8 columns are loaded before any is stored so that 16
// loads per thread are in flight.
template <typename T, typename F>
__device__ __forceinline__ T* stage_block(T* dst, int rows, int cols, F f) {
  const int lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6, w = threadIdx.x >> 6;
  if (rows <= 0 || cols <= 0) return dst;
  const int ra = min(lane, rows - 1), rb = min(lane + 64, rows - 1);
  for (int j0 = w; j0 < cols; j0 += 8 * nw) {
    T v[16];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int jc = min(j0 + u * nw, cols - 1);
      v[2 * u] = f(ra, jc);        // unconditional reads from clamped indices
      v[2 * u + 1] = f(rb, jc);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * nw;
      if (j < cols && lane < rows) dst[lane + j * rows] = v[2 * u];
      if (j < cols && lane + 64 < rows) dst[lane + 64 + j * rows] = v[2 * u + 1];
    }
  }
  return dst + rows * cols;
}

// A block copied to LDS: element (i, j) of a rows x cols block is src[i + j*ld]
// (zero above the diagonal when upper_zero) and lands at dst[i + j*rows].
template <typename T>
struct SBlk {
  const T* src;
  int ld, rows, cols;
  bool upper_zero;
  T* dst;
};

// Copy NB blocks to LDS: the block table goes through LDS, wavefront w copies
// blocks w, w + nw, ... with 32 reads in flight per lane (compact code: the
// sweeps of the upper levels are short, and their instructions are fetched
// afresh by every launch).  Element o = lane + 64 u of a block is (i, c) with
// o = i + c rows; (i, c) advance by the constant (64 mod rows, 64 / rows) per
// u, so no division is done per element.
template <typename T, int NB>
__device__ __forceinline__ void stage_blocks(const SBlk<T> (&b)[NB], SBlk<T>* tab) {
  constexpr int U = 32;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NB; ++q) tab[q] = b[q];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll 1
  for (int q = w; q < NB; q += nw) {
    const SBlk<T> B = tab[q];
    const int total = B.rows * B.cols;
    if (total <= 0) continue;
    const int qr = 64 / B.rows, rr = 64 - qr * B.rows;   // 64 = qr rows + rr
#pragma unroll 1
    for (int o0 = 0; o0 < total; o0 += U * 64) {
      const int oa = min(o0 + lane, total - 1);
      int i = oa % B.rows, c = oa / B.rows;
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const T x = B.src[i + (int64_t)c * B.ld];
        v[u] = (B.upper_zero & (i < c)) ? T(0) : x;
        // next element (clamped to the last one past the end)
        i += rr;
        c += qr;
        const bool wrap = i >= B.rows;
        i = wrap ? i - B.rows : i;
        c = wrap ? c + 1 : c;
        const bool past = c >= B.cols;
        i = past ? B.rows - 1 : i;
        c = past ? B.cols - 1 : c;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int o = o0 + lane + 64 * u;
        if (o < total) B.dst[o] = v[u];
      }
    }
  }
}

// Copies of everything the forward sweep of an internal node reads, in LDS,
// staged in one pass (all reads in flight together).
template <typename T>
__device__ NodeSrc<T> src_stage_fwd(const Inst<T>& I, const NodeInfo& nd, const NodeInfo& n1,
                                    const NodeInfo& n2, T* sm) {
  const NodeSrc<T> G = src_global(I, nd, n1, n2);
  const int mp = nd.mp, e = nd.e, ku = nd.ku, kv = nd.kv, kw = n1.kv + n2.kv;
  NodeSrc<T> S = G;
  T* p = sm;
  SBlk<T> b[8];
  const int kq = e > 0 ? ku : 0;
  S.U = p; S.ldu = mp;         b[0] = {G.U, mp, mp, kq, false, p}; p += mp * kq;
  S.L = p; S.ldl = mp;         b[1] = {G.L, mp, mp, e, false, p}; p += mp * e;
  S.V = p; S.ldv = e;          b[2] = {G.V, mp, e, kv, false, p}; p += e * kv;
  S.W = p; S.ldw = kw;         b[3] = {G.W, kw, kw, kv, false, p}; p += kw * kv;
  S.U1 = p; S.ldu1 = n1.kept; S.m1 = false;
  b[4] = {G.U1, G.ldu1, n1.kept, n1.ku, G.m1, p}; p += n1.kept * n1.ku;
  S.U2 = p; S.ldu2 = n2.kept; S.m2 = false;
  b[5] = {G.U2, G.ldu2, n2.kept, n2.ku, G.m2, p}; p += n2.kept * n2.ku;
  S.B12 = p; S.ld12 = n1.ku;   b[6] = {G.B12, n1.ku, n1.ku, n2.kv, false, p}; p += n1.ku * n2.kv;
  S.B21 = p; S.ld21 = n2.ku;   b[7] = {G.B21, n2.ku, n2.ku, n1.kv, false, p};
  __shared__ SBlk<T> tab[8];
  stage_blocks<T, 8>(b, tab);
  return S;   // the caller synchronizes the work-group
}

// The children's c and z an internal node's rhs is built from (rows lane,
// lane + 64 of [c_c1; c_c2]; entries lane of z_c1, z_c2), for CPW columns
// col0 .. (columns >= nrhs read as zero).  Independent of the node's own
// factors, so they can be read before those are staged.
template <typename T, int CPW>
struct Gathered {
  T x0[CPW], x1[CPW], z1[CPW], z2[CPW];
};

template <typename T, int CPW>
__device__ __forceinline__ void gather_load(const Inst<T>& I, const NodeInfo& nd, const NodeInfo& n1,
                                            const NodeInfo& n2, int col0, int nrhs, int lane,
                                            Gathered<T, CPW>& G) {
  const int k1 = n1.kept, mp = nd.mp;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const bool cv = col0 + c < nrhs;
    const int64_t co = (int64_t)(cv ? col0 + c : 0) * I.lds;
    const T* z1 = I.wz + n1.oz + co;
    const T* z2 = I.wz + n2.oz + co;
    const T* c1 = I.wc + n1.oc + co;
    const T* c2 = I.wc + n2.oc + co;
    G.z1[c] = n1.kv > 0 ? ld_early_or0(z1 + min(lane, n1.kv - 1), cv & (lane < n1.kv)) : T(0);
    G.z2[c] = n2.kv > 0 ? ld_early_or0(z2 + min(lane, n2.kv - 1), cv & (lane < n2.kv)) : T(0);
    // rows r of [c_c1; c_c2] (both parts read from clamped, valid addresses)
    const int k2 = mp - k1;
    const T c1a = k1 > 0 ? ld_early_or0(c1 + min(lane, k1 - 1), true) : T(0);
    const T c1b = k1 > 0 ? ld_early_or0(c1 + min(lane + 64, k1 - 1), true) : T(0);
    const T c2a = k2 > 0 ? ld_early_or0(c2 + min(max(lane - k1, 0), k2 - 1), true) : T(0);
    const T c2b = k2 > 0 ? ld_early_or0(c2 + min(max(lane + 64 - k1, 0), k2 - 1), true) : T(0);
    const T a0 = lane < k1 ? c1a : (lane < mp ? c2a : T(0));
    const T a1 = lane + 64 < k1 ? c1b : (lane + 64 < mp ? c2b : T(0));
    G.x0[c] = cv ? a0 : T(0);
    G.x1[c] = cv ? a1 : T(0);
  }
}

// rhs of an internal node (rows lane, lane + 64) from the children's c and z
// (already read into G): [c_c1 - U~_c1 B12 z_c2; c_c2 - U~_c2 B21 z_c1].
template <typename T, int CPW>
__device__ void gather_apply(const NodeInfo& nd, const NodeInfo& n1, const NodeInfo& n2, int lane,
                             const NodeSrc<T>& S, const Gathered<T, CPW>& G, T (&x0)[CPW],
                             T (&x1)[CPW]) {
  const int k1 = n1.kept, mp = nd.mp;
  const int r0 = lane, r1 = lane + 64;
  T t1[CPW], t2[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    x0[c] = G.x0[c];
    x1[c] = G.x1[c];
    t1[c] = T(0);
    t2[c] = T(0);
  }
  // t1 = B12 z_c2, t2 = B21 z_c1 (lane = row), then x -= [U~_c1 t1; U~_c2 t2]:
  // chunks of 8 terms, the reads of a chunk issued together, masked terms
  // instead of branches
  const int ny1 = n1.ku > 0 ? n2.kv : 0, ny2 = n2.ku > 0 ? n1.kv : 0;
  const int lb1 = max(min(lane, n1.ku - 1), 0), lb2 = max(min(lane, n2.ku - 1), 0);
  for (int y0 = 0; y0 < ny1; y0 += 8) {
    T bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) bv[u] = S.B12[lb1 + min(y0 + u, ny1 - 1) * S.ld12];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const T b = ((lane < n1.ku) & (y0 + u < ny1)) ? bv[u] : T(0);
#pragma unroll
      for (int c = 0; c < CPW; ++c) t1[c] += b * bcast(G.z2[c], min(y0 + u, 63));
    }
  }
  for (int y0 = 0; y0 < ny2; y0 += 8) {
    T bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) bv[u] = S.B21[lb2 + min(y0 + u, ny2 - 1) * S.ld21];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const T b = ((lane < n2.ku) & (y0 + u < ny2)) ? bv[u] : T(0);
#pragma unroll
      for (int c = 0; c < CPW; ++c) t2[c] += b * bcast(G.z1[c], min(y0 + u, 63));
    }
  }
  const int k2 = mp - k1;
  const int a10 = min(r0, k1 - 1), a11 = min(r1, k1 - 1);
  const int a20 = min(max(r0 - k1, 0), k2 - 1), a21 = min(max(r1 - k1, 0), k2 - 1);
  const bool in10 = r0 < k1, in11 = r1 < k1;
  const bool in20 = (r0 >= k1) & (r0 < mp), in21 = (r1 >= k1) & (r1 < mp);
  for (int x0c = 0; x0c < n1.ku; x0c += 8) {
    T ua[8], ub[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int x = min(x0c + u, n1.ku - 1);
      ua[u] = ut(S.U1, S.ldu1, S.m1, a10, x);
      ub[u] = ut(S.U1, S.ldu1, S.m1, a11, x);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool ok = x0c + u < n1.ku;
      const T u0 = (in10 & ok) ? ua[u] : T(0), u1 = (in11 & ok) ? ub[u] : T(0);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const T tx = bcast(t1[c], min(x0c + u, 63));
        x0[c] -= u0 * tx;
        x1[c] -= u1 * tx;
      }
    }
  }
  for (int x0c = 0; x0c < n2.ku; x0c += 8) {
    T ua[8], ub[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int x = min(x0c + u, n2.ku - 1);
      ua[u] = ut(S.U2, S.ldu2, S.m2, a20, x);
      ub[u] = ut(S.U2, S.ldu2, S.m2, a21, x);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool ok = x0c + u < n2.ku;
      const T u0 = (in20 & ok) ? ua[u] : T(0), u1 = (in21 & ok) ? ub[u] : T(0);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const T tx = bcast(t2[c], min(x0c + u, 63));
        x0[c] -= u0 * tx;
        x1[c] -= u1 * tx;
      }
    }
  }
}

template <typename T, int CPW>
__device__ void gather_internal(const Inst<T>& I, const NodeInfo& nd, const NodeInfo& n1,
                                const NodeInfo& n2, int col0, int nrhs, int lane,
                                const NodeSrc<T>& S, T (&x0)[CPW], T (&x1)[CPW]) {
  Gathered<T, CPW> G;
  gather_load<T, CPW>(I, nd, n1, n2, col0, nrhs, lane, G);
  gather_apply<T, CPW>(nd, n1, n2, lane, S, G, x0, x1);
}

// Work item of this wavefront.  Direct kernels: kSW wavefronts per
// work-group, one node each, CPW columns per wavefront.  Staged kernels: one
// node per work-group, its wavefronts (kSWS or kSW) take consecutive groups of
// CPW columns.
template <bool BATCH, bool STAGED, int CPW, typename T>
__device__ __forceinline__ bool sv_resolve(const KArgs<T, CallSV<T>>& a, Inst<T>& I,
                                           CallSV<T>& C, int& node, int& col0) {
  const int w = threadIdx.x >> 6;
  const int item = STAGED ? blockIdx.x : blockIdx.x * kSW + w;
  col0 = (STAGED ? blockIdx.y * (blockDim.x >> 6) + w : blockIdx.y) * CPW;
  if (item >= a.ntasks) return false;
  if constexpr (BATCH) {
    const int2 tk = a.tasks[item];
    I = a.insts[tk.x];
    C = a.calls[tk.x];
    node = tk.y;
  } else {
    I = a.inst;
    C = a.call;
    node = a.node0 + item;
  }
  return !gated_off(C.gate);
}

// A node's record and its children's, all three reads issued together (the
// children's from clamped indices, so that they do not wait for is_leaf);
// a leaf's children come back empty.
__device__ __forceinline__ void node_and_children(const NodeInfo* nodes, int nnodes, int node,
                                                  NodeInfo& nd, NodeInfo& n1, NodeInfo& n2) {
  const int c1 = min(2 * node + 1, nnodes - 1), c2 = min(2 * node + 2, nnodes - 1);
  nd = nodes[node];
  const NodeInfo a1 = nodes[c1], a2 = nodes[c2];
  n1 = nd.is_leaf ? NodeInfo{} : a1;
  n2 = nd.is_leaf ? NodeInfo{} : a2;
}

// Forward sweep at one node.  (Single-matrix leaf launches keep a node's
// reflectors and L columns in registers, 32 at a time, all requested ahead of
// use; batched launches, whose long levels need more wavefronts per CU than
// those registers allow, read them one step ahead.)  STAGED: the node's factors are copied to LDS by
// the whole work-group first (internal nodes); otherwise kSW wavefronts per
// work-group read the factor arrays (leaves).  Each wavefront carries CPW
// right-hand-side columns through the same factor reads.
template <typename T, bool BATCH, bool STAGED, int CPW>
__global__ __launch_bounds__((STAGED && !BATCH ? kSWS : kSW) * 64) void k_sv_fwd_w(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  Inst<T> I; CallSV<T> C; int node, col0;
  if (!sv_resolve<BATCH, STAGED, CPW>(a, I, C, node, col0)) return;   // uniform when STAGED
  const int lane = threadIdx.x & 63;
  // the node's and children's records, read once (reads after a barrier are
  // not merged with those before it)
  NodeInfo nd, n1, n2;
  node_and_children(I.nodes, I.nnodes, node, nd, n1, n2);
  const int mp = nd.mp, e = nd.e, ku = nd.ku, kv = nd.kv;
  const int r0 = lane, r1 = lane + 64;
  NodeSrc<T> S;
  Gathered<T, CPW> G;
  if (!nd.is_leaf) gather_load<T, CPW>(I, nd, n1, n2, col0, C.nrhs, lane, G);   // before the staging
  const T taul = ku > 0 ? ld_early_or0(I.tq + nd.otq + min(lane, ku - 1), lane < ku) : T(0);
  if (STAGED) {
    S = src_stage_fwd(I, nd, n1, n2, reinterpret_cast<T*>(smem_raw));
    __syncthreads();
  } else {
    S = src_global(I, nd, n1, n2);
  }
  if (col0 >= C.nrhs) return;
  T x0[CPW], x1[CPW];
  if (nd.is_leaf) {
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const bool cv = col0 + c < C.nrhs;
      const T* b = C.B + nd.row0 + (int64_t)(cv ? col0 + c : 0) * C.ldb;
      x0[c] = ld_or0(b + min(r0, mp - 1), cv & (r0 < mp));
      x1[c] = ld_or0(b + min(r1, mp - 1), cv & (r1 < mp));
    }
  } else {
    gather_apply<T, CPW>(nd, n1, n2, lane, S, G, x0, x1);
  }
  if (e > 0) {
    // b~ = Q^T rhs = H_0 ... H_{ku-1} rhs, H_{ku-1} applied first (lane j holds tau_j);
    // the next reflector is read while this one is applied; a leaf (factors
    // in global memory, one wavefront per node) has all of them in flight at
    // once instead
    bool u_done = false;
    if constexpr (!STAGED && !BATCH) {
      if (ku > 0 && ku <= 32) {
        T ua[32], ub[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) {
          const T* vj = S.U + min(j, ku - 1) * S.ldu;
          ua[j] = vj[min(r0, mp - 1)];
          ub[j] = vj[min(r1, mp - 1)];
        }
#pragma unroll
        for (int j = 31; j >= 0; --j) {
          if (j < ku) {
            const T tau = bcast(taul, j);
            const int pr = e + j;
            const T v0 = r0 < pr ? ua[j] : (r0 == pr ? T(1) : T(0));
            const T v1 = r1 < pr ? ub[j] : (r1 == pr ? T(1) : T(0));
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
              const T w = wave_sum(v0 * x0[c] + v1 * x1[c]) * tau;
              x0[c] -= w * v0;
              x1[c] -= w * v1;
            }
          }
        }
        u_done = true;
      }
    }
    T n0 = T(0), n1 = T(0);
    if (ku > 0 && !u_done) {
      n0 = S.U[(ku - 1) * S.ldu + min(r0, mp - 1)];
      n1 = S.U[(ku - 1) * S.ldu + min(r1, mp - 1)];
    }
#pragma unroll(STAGED ? 1 : 8)
    for (int j = u_done ? -1 : ku - 1; j >= 0; --j) {
      const T tau = bcast(taul, j);
      const int pr = e + j;
      const T a0 = n0, a1 = n1;
      const T* vn = S.U + max(j - 1, 0) * S.ldu;
      n0 = vn[min(r0, mp - 1)];
      n1 = vn[min(r1, mp - 1)];
      const T v0 = r0 < pr ? a0 : (r0 == pr ? T(1) : T(0));
      const T v1 = r1 < pr ? a1 : (r1 == pr ? T(1) : T(0));
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const T w = wave_sum(v0 * x0[c] + v1 * x1[c]) * tau;
        x0[c] -= w * v0;
        x1[c] -= w * v1;
      }
    }
    // y = L^{-1} b~_top; the same column sweep leaves b~_bot - D~21 y below
    // (the reciprocals of L's diagonal are formed up front, one per lane)
    const int ec = max(e - 1, 0);
    const T dg0 = S.L[min(r0, ec) * (S.ldl + 1)], dg1 = S.L[min(r1, ec) * (S.ldl + 1)];
    const T dinv0 = T(1) / dg0, dinv1 = T(1) / dg1;
    bool l_done = false;
    if constexpr (!STAGED && !BATCH) {
      // 32 columns of L in registers, the next 32 requested before these are used
      T la0[32], la1[32];
#pragma unroll
      for (int ii = 0; ii < 32; ++ii) {
        const T* Ln = S.L + min(ii, ec) * S.ldl;
        la0[ii] = Ln[min(r0, mp - 1)];
        la1[ii] = Ln[min(r1, mp - 1)];
      }
      for (int i0 = 0; i0 < e; i0 += 32) {
        T lb0[32], lb1[32];
#pragma unroll
        for (int ii = 0; ii < 32; ++ii) {
          const T* Ln = S.L + min(i0 + 32 + ii, ec) * S.ldl;
          lb0[ii] = Ln[min(r0, mp - 1)];
          lb1[ii] = Ln[min(r1, mp - 1)];
        }
#pragma unroll
        for (int ii = 0; ii < 32; ++ii) {
          const int i = i0 + ii;
          if (i < e) {
            const T l0 = ((r0 > i) & (r0 < mp)) ? la0[ii] : T(0);
            const T l1 = ((r1 > i) & (r1 < mp)) ? la1[ii] : T(0);
            const T dinv = row_of(dinv0, dinv1, i);
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
              const T yi = row_of(x0[c], x1[c], i) * dinv;
              if (r0 == i) x0[c] = yi;
              if (r1 == i) x1[c] = yi;
              x0[c] -= l0 * yi;
              x1[c] -= l1 * yi;
            }
          }
        }
#pragma unroll
        for (int ii = 0; ii < 32; ++ii) {
          la0[ii] = lb0[ii];
          la1[ii] = lb1[ii];
        }
      }
      l_done = true;
    }
    T m0 = S.L[min(r0, mp - 1)], m1 = S.L[min(r1, mp - 1)];
#pragma unroll(STAGED ? 1 : 16)
    for (int i = l_done ? e : 0; i < e; ++i) {
      const T a0 = m0, a1 = m1;
      const T* Ln = S.L + min(i + 1, ec) * S.ldl;
      m0 = Ln[min(r0, mp - 1)];
      m1 = Ln[min(r1, mp - 1)];
      const T l0 = ((r0 > i) & (r0 < mp)) ? a0 : T(0);
      const T l1 = ((r1 > i) & (r1 < mp)) ? a1 : T(0);
      const T dinv = row_of(dinv0, dinv1, i);
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const T yi = row_of(x0[c], x1[c], i) * dinv;
        if (r0 == i) x0[c] = yi;
        if (r1 == i) x1[c] = yi;
        x0[c] -= l0 * yi;
        x1[c] -= l1 * yi;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    if (col0 + c >= C.nrhs) break;
    const int64_t co = (int64_t)(col0 + c) * I.lds;
    T* yo = I.wy + nd.oy + co;
    T* cout = I.wc + nd.oc + co;
    if (r0 < e) yo[r0] = x0[c]; else if (r0 < mp) cout[r0 - e] = x0[c];
    if (r1 < e) yo[r1] = x1[c]; else if (r1 < mp) cout[r1 - e] = x1[c];
  }
  if (node == 0) return;
  // z = V^_top^T y (+ W^T [z_c1; z_c2])
  T zc0[CPW], zc1[CPW];
  int kw = 0;
  int kv1 = 0;
  if (!nd.is_leaf) {
    kv1 = n1.kv;
    kw = n1.kv + n2.kv;
  }
  // rows r0, r1 of [z_c1; z_c2], from the children's z read at the start
  // (lane l holds entry l of each): a lane shift for the z_c2 part
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    zc0[c] = zc1[c] = T(0);
    if (kw) {
      const T s0 = __shfl(G.z2[c], min(max(r0 - kv1, 0), 63), 64);
      const T s1 = __shfl(G.z2[c], min(max(r1 - kv1, 0), 63), 64);
      zc0[c] = r0 < kv1 ? G.z1[c] : (r0 < kw ? s0 : T(0));
      zc1[c] = r1 < kv1 ? G.z1[c] : (r1 < kw ? s1 : T(0));
    }
  }
  if (CPW == 1 && kv <= 32) {
    // every lane forms its terms of all kv entries, one transposed sum over
    // the wavefront leaves entry aa in lanes aa and aa + 32
    T v[32];
    const int ec = max(e - 1, 0);
    const T* V0 = S.V + min(r0, ec);
    const T* V1 = S.V + min(r1, ec);
    const T x0e = r0 < e ? x0[0] : T(0), x1e = r1 < e ? x1[0] : T(0);
#pragma unroll
    for (int aa = 0; aa < 32; ++aa) {
      const int ac = min(aa, max(kv - 1, 0));
      v[aa] = V0[ac * S.ldv] * x0e + V1[ac * S.ldv] * x1e;
    }
    if (kw) {
      const T* W0 = S.W + min(r0, kw - 1);
      const T* W1 = S.W + min(r1, kw - 1);
      const T z0e = r0 < kw ? zc0[0] : T(0), z1e = r1 < kw ? zc1[0] : T(0);
#pragma unroll
      for (int aa = 0; aa < 32; ++aa) {
        const int ac = min(aa, max(kv - 1, 0));
        v[aa] += W0[ac * S.ldw] * z0e + W1[ac * S.ldw] * z1e;
      }
    }
#pragma unroll
    for (int aa = 0; aa < 32; ++aa) v[aa] = aa < kv ? v[aa] : T(0);
    const T zs = wave_transpose_sum32(v);
    if (col0 < C.nrhs && lane < kv) I.wz[nd.oz + (int64_t)col0 * I.lds + lane] = zs;
  } else {
    // one wavefront reduction per (entry, column); results kept by lane aa
    T zr[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) zr[c] = T(0);
#pragma unroll(STAGED ? 4 : 8)
    for (int aa = 0; aa < kv; ++aa) {
      const T* Va = S.V + aa * S.ldv;
      const int ec = max(e - 1, 0);
      const T a0 = Va[min(r0, ec)], a1 = Va[min(r1, ec)];
      const T va0 = r0 < e ? a0 : T(0), va1 = r1 < e ? a1 : T(0);
      T wa0 = T(0), wa1 = T(0);
      if (kw) {
        const T w0 = S.W[min(r0, kw - 1) + aa * S.ldw], w1 = S.W[min(r1, kw - 1) + aa * S.ldw];
        wa0 = r0 < kw ? w0 : T(0);
        wa1 = r1 < kw ? w1 : T(0);
      }
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const T sz = wave_sum(va0 * x0[c] + va1 * x1[c] + wa0 * zc0[c] + wa1 * zc1[c]);
        if (lane == aa) zr[c] = sz;
      }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c)
      if (col0 + c < C.nrhs && lane < kv) I.wz[nd.oz + (int64_t)(col0 + c) * I.lds + lane] = zr[c];
  }
}

// Forward step of an internal node from its forward-operator record (layout
// kRec* in hss_internal.hpp):
//   rhs = [c_c1; c_c2] - G [z_c1; z_c2];  zw = W^T [z_c1; z_c2];
//   w = Y^T rhs;  b~ = rhs - YT w;
//   [y; d; v] = F b~(0:e);  c = b~(e:) - d;  z = v + zw.
// One node per work-group: the record is copied to LDS with 16-byte loads
// (all issued before any is stored); then wavefront w carries columns
// col0 = CPW (4 blockIdx.y + w) ...; lane r holds entry r of every length-64
// vector and each product is a dot product over LDS with fixed trip counts
// (unused rows and columns of the record are zero).
constexpr int kOpW = 4;                        // wavefronts per work-group
constexpr int kOpScrW = 4 * 64;                // per wavefront and column: x, z, w, b

int fwd_op_lds_elems(int cpw) { return kRecSize + kOpW * kOpScrW * cpw; }

template <typename T, bool BATCH, int CPW>
__global__ __launch_bounds__(kOpW * 64) void k_sv_fwd_op(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* sm = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node, col0;
  if (!sv_resolve<BATCH, true, CPW>(a, I, C, node, col0)) return;   // uniform
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  NodeInfo nd, n1, n2;
  node_and_children(I.nodes, I.nnodes, node, nd, n1, n2);
  const int mp = nd.mp, e = nd.e, kv = nd.kv, kept = nd.kept;
  const int kw = n1.kv + n2.kv, kv1 = n1.kv;
  const int ldf = e + kept + kv;
  Gathered<T, CPW> G;
  gather_load<T, CPW>(I, nd, n1, n2, col0, C.nrhs, lane, G);   // before the copy
  {
    // the record: kRecSize elements = kRecSize * sizeof(T) / 16 chunks
    constexpr int nch = kRecSize * (int)sizeof(T) / 16;
    constexpr int per = (nch + kOpW * 64 - 1) / (kOpW * 64);
    const int4* src = reinterpret_cast<const int4*>(I.FOP + nd.oOP);
    int4* dst = reinterpret_cast<int4*>(sm);
    int4 v[per];
#pragma unroll
    for (int u = 0; u < per; ++u) v[u] = src[min((int)threadIdx.x + u * kOpW * 64, nch - 1)];
#pragma unroll
    for (int u = 0; u < per; ++u) {
      const int q = (int)threadIdx.x + u * kOpW * 64;
      if (q < nch) dst[q] = v[u];
    }
  }
  __syncthreads();
  if (col0 >= C.nrhs) return;
  const T* sG = sm + kRecG;
  const T* sW = sm + kRecW;
  const T* sY = sm + kRecY;
  const T* sYT = sm + kRecYT;
  const T* sF = sm + kRecF;
  T* scr = sm + kRecSize + w * kOpScrW * CPW;
  T* zs = scr;                 // 64 per column: [z_c1; z_c2]
  T* xs = scr + 64 * CPW;      // 64 per column: rhs
  T* ws = xs + 64 * CPW;       // 32 per column: Y^T rhs
  T* bs = ws + 32 * CPW;       // 64 per column: b~
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    // entry lane of [z_c1; z_c2]: z_c1 in lanes < kv1, then z_c2
    const T z2s = __shfl(G.z2[c], min(max(lane - kv1, 0), 63), 64);
    zs[lane + 64 * c] = lane < kv1 ? G.z1[c] : (lane < kw ? z2s : T(0));
  }
  wave_lds_sync();
  // rhs = c - G zc (lane r); zw = W^T zc (lane a)
  T x[CPW], zw[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    x[c] = G.x0[c];
    zw[c] = T(0);
  }
  {
    const int aw = min(lane, 31);
#pragma unroll 16
    for (int q = 0; q < 64; ++q) {
      const T gq = sG[lane + q * 64];
      const T wq = sW[q + aw * 65];
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const T zq = zs[q + 64 * c];
        x[c] -= gq * zq;
        zw[c] += wq * zq;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) xs[lane + 64 * c] = lane < mp ? x[c] : T(0);
  wave_lds_sync();
  // w = Y^T rhs (lane i < 32)
  {
    const int i = min(lane, 31);
    T wv[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) wv[c] = T(0);
#pragma unroll 16
    for (int r = 0; r < 64; ++r) {
      const T y = sY[r + i * 65];
#pragma unroll
      for (int c = 0; c < CPW; ++c) wv[c] += y * xs[r + 64 * c];
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c)
      if (lane < 32) ws[lane + 32 * c] = wv[c];
  }
  wave_lds_sync();
  // b~ = rhs - (Y T) w (lane r)
#pragma unroll 16
  for (int i = 0; i < 32; ++i) {
    const T yt = sYT[lane + i * 64];
#pragma unroll
    for (int c = 0; c < CPW; ++c) x[c] -= yt * ws[i + 32 * c];
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) bs[lane + 64 * c] = lane < mp ? x[c] : T(0);
  wave_lds_sync();
  // [y; d; v] = F b~(0:e): outputs o = lane and o = lane + 64 (ldf <= 96)
  T o0[CPW], o1[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) { o0[c] = T(0); o1[c] = T(0); }
  {
    const int ob = min(lane + 64, 95);
#pragma unroll 16
    for (int i = 0; i < 32; ++i) {
      const T fa = sF[lane + i * 96], fb = sF[ob + i * 96];
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const T bi = bs[i + 64 * c];
        o0[c] += fa * bi;
        o1[c] += fb * bi;
      }
    }
  }
  // outputs: o < e -> y; e <= o < e + kept -> c = b~[o] - d; else z = v + zw
  // (z entry a is output row e + kept + a; its W^T zc part is zw of lane a,
  // fetched by every lane before the stores)
  const int64_t lds = I.lds;
  const int ea = e + kept;
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const T zwa0 = __shfl(zw[c], min(max(lane - ea, 0), 63), 64);
    const T zwa1 = __shfl(zw[c], min(max(lane + 64 - ea, 0), 63), 64);
    if (col0 + c >= C.nrhs) continue;
    const int64_t co = (int64_t)(col0 + c) * lds;
    T* yo = I.wy + nd.oy + co;
    T* cout = I.wc + nd.oc + co;
    T* zo = I.wz + nd.oz + co;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int o = lane + 64 * h;
      const T val = h ? o1[c] : o0[c];
      if (o < e) yo[o] = val;
      else if (o < ea) cout[o - e] = bs[min(o, 63) + 64 * c] - val;
      else if (o < ldf) zo[o - ea] = val + (h ? zwa1 : zwa0);
    }
  }
}

// Root: rhs from the children, then the FP64 LU of the merged root block
// (staged in LDS with its pivots), split into the children's x^.
template <typename T, bool BATCH, int CPW>
__global__ __launch_bounds__(kSWS * 64) void k_sv_root_w(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  Inst<T> I; CallSV<T> C; int node, col0;
  if (!sv_resolve<BATCH, true, CPW>(a, I, C, node, col0)) return;
  const int lane = threadIdx.x & 63;
  NodeInfo nd, n1, n2;
  node_and_children(I.nodes, I.nnodes, node, nd, n1, n2);
  const int mp = nd.mp;
  const int r0 = lane, r1 = lane + 64;
  double* LU = reinterpret_cast<double*>(smem_raw);
  int* piv = reinterpret_cast<int*>(LU + mp * mp);
  T* rest = reinterpret_cast<T*>(piv + ((mp + 3) & ~3));
  stage_block(LU, mp, mp, [&](int i, int j) { return I.rootLU[i + j * mp]; });
  // the row permutation of the root LU (position i holds original row piv[i])
  for (int o = threadIdx.x; o < mp; o += blockDim.x) piv[o] = I.piv[mp + o];   // (mp <= 128 < blockDim)
  NodeSrc<T> S = (nd.is_leaf || !(a.flags & 1)) ? src_global(I, nd, n1, n2)
                                                 : src_stage_fwd(I, nd, n1, n2, rest);
  __syncthreads();
  if (col0 >= C.nrhs) return;
  T t0[CPW], t1[CPW];
  if (nd.is_leaf) {
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const bool cv = col0 + c < C.nrhs;
      const T* b = C.B + nd.row0 + (int64_t)(cv ? col0 + c : 0) * C.ldb;
      t0[c] = ld_or0(b + min(r0, mp - 1), cv & (r0 < mp));
      t1[c] = ld_or0(b + min(r1, mp - 1), cv & (r1 < mp));
    }
  } else {
    gather_internal<T, CPW>(I, nd, n1, n2, col0, C.nrhs, lane, S, t0, t1);
  }
  double x0[CPW], x1[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    x0[c] = (double)t0[c];
    x1[c] = (double)t1[c];
  }
  {
    // x <- P x in one gather: row r takes original row piv[r]
    const int s0 = r0 < mp ? piv[r0] : r0, s1 = r1 < mp ? piv[r1] : r1;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double a0 = __shfl(x0[c], s0 & 63, 64), b0 = __shfl(x1[c], s0 & 63, 64);
      const double a1 = __shfl(x0[c], s1 & 63, 64), b1 = __shfl(x1[c], s1 & 63, 64);
      x0[c] = s0 < 64 ? a0 : b0;
      x1[c] = s1 < 64 ? a1 : b1;
    }
  }
  // (unrolled so that the LDS reads of the next columns are in flight)
#pragma unroll 8
  for (int i = 0; i < mp; ++i) {
    const double* Li = LU + i * mp;
    const double l0 = r0 > i && r0 < mp ? Li[r0] : 0.0;
    const double l1 = r1 > i && r1 < mp ? Li[r1] : 0.0;
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double xi = row_of(x0[c], x1[c], i);
      x0[c] -= l0 * xi;
      x1[c] -= l1 * xi;
    }
  }
#pragma unroll 8
  for (int i = mp - 1; i >= 0; --i) {
    const double* Ui = LU + i * mp;
    const double u0 = r0 < i ? Ui[r0] : 0.0, u1 = r1 < i ? Ui[r1] : 0.0;
    const double dinv = 1.0 / Ui[i];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const double xi = row_of(x0[c], x1[c], i) * dinv;
      if (r0 == i) x0[c] = xi;
      if (r1 == i) x1[c] = xi;
      x0[c] -= u0 * xi;
      x1[c] -= u1 * xi;
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    if (col0 + c >= C.nrhs) break;
    if (nd.is_leaf) {
      T* out = C.B + nd.row0 + (int64_t)(col0 + c) * C.ldb;
      if (r0 < mp) out[r0] = (T)x0[c];
      if (r1 < mp) out[r1] = (T)x1[c];
      continue;
    }
    const NodeInfo n1 = I.nodes[1], n2 = I.nodes[2];
    const int64_t co = (int64_t)(col0 + c) * I.lds;
    T* xa = I.wx + n1.ox + co;
    T* xb = I.wx + n2.ox + co;
    const int k1 = n1.kept;
    if (r0 < k1) xa[r0] = (T)x0[c]; else if (r0 < mp) xb[r0 - k1] = (T)x0[c];
    if (r1 < k1) xa[r1] = (T)x1[c]; else if (r1 < mp) xb[r1 - k1] = (T)x1[c];
  }
}

template <typename T, bool BATCH, bool STAGED, int CPW>
__global__ __launch_bounds__(kSW * 64) void k_sv_bwd_w(KArgs<T, CallSV<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  Inst<T> I; CallSV<T> C; int node, col0;
  if (!sv_resolve<BATCH, STAGED, CPW>(a, I, C, node, col0)) return;
  const int lane = threadIdx.x & 63;
  const NodeInfo nd = I.nodes[node];
  const int mp = nd.mp, e = nd.e;
  const int r0 = lane, r1 = lane + 64;
  const T* Z = I.FZ + nd.oFZ;
  const int ldz = mp;
  if (STAGED) {
    T* sz = reinterpret_cast<T*>(smem_raw);
    stage_block(sz, mp, e, [&](int i, int j) { return Z[i + j * mp]; });
    __syncthreads();
    Z = sz;
  }
  if (col0 >= C.nrhs) return;
  T x0[CPW], x1[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const bool cv = col0 + c < C.nrhs;
    const int64_t co = (int64_t)(cv ? col0 + c : 0) * I.lds;
    const T* yi = I.wy + nd.oy + co;
    const T* xi = I.wx + nd.ox + co;
    const T a0 = stacked(yi, e, xi, mp - e, r0), a1 = stacked(yi, e, xi, mp - e, r1);
    x0[c] = cv ? a0 : T(0);
    x1[c] = cv ? a1 : T(0);
  }
  // Z [y; x^] = H_0 ... H_{e-1} [y; x^], H_{e-1} applied first
  const int ec = max(e - 1, 0);
  const T taul0 = e > 0 ? ld_or0(I.tz + nd.otz + min(r0, ec), r0 < e) : T(0);
  const T taul1 = e > 0 ? ld_or0(I.tz + nd.otz + min(r1, ec), r1 < e) : T(0);
  bool z_done = false;
  if constexpr (!STAGED && !BATCH) {
    // factors in global memory, one wavefront per node: 32 reflectors in
    // registers, the next 32 requested before these are applied
    if (e > 0) {
      T za0[32], za1[32];
#pragma unroll
      for (int qq = 0; qq < 32; ++qq) {
        const T* v = Z + max(e - 1 - qq, 0) * ldz;
        za0[qq] = v[min(r0, mp - 1)];
        za1[qq] = v[min(r1, mp - 1)];
      }
      for (int q0 = 0; q0 < e; q0 += 32) {
        T zb0[32], zb1[32];
#pragma unroll
        for (int qq = 0; qq < 32; ++qq) {
          const T* v = Z + max(e - 1 - q0 - 32 - qq, 0) * ldz;
          zb0[qq] = v[min(r0, mp - 1)];
          zb1[qq] = v[min(r1, mp - 1)];
        }
#pragma unroll
        for (int qq = 0; qq < 32; ++qq) {
          const int i = e - 1 - q0 - qq;
          if (i >= 0) {
            const T tau = row_of(taul0, taul1, i);
            const T v0 = r0 < mp ? za0[qq] : T(0);
            const T v1 = r1 < mp ? za1[qq] : T(0);
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
              const T w = wave_sum(v0 * x0[c] + v1 * x1[c]) * tau;
              x0[c] -= w * v0;
              x1[c] -= w * v1;
            }
          }
        }
#pragma unroll
        for (int qq = 0; qq < 32; ++qq) {
          za0[qq] = zb0[qq];
          za1[qq] = zb1[qq];
        }
      }
    }
    z_done = true;
  }
#pragma unroll 4
  for (int i = z_done ? -1 : e - 1; i >= 0; --i) {
    const T tau = row_of(taul0, taul1, i);
    const T* v = Z + i * ldz;
    const T a0 = v[min(r0, mp - 1)], a1 = v[min(r1, mp - 1)];
    const T v0 = r0 < mp ? a0 : T(0);
    const T v1 = r1 < mp ? a1 : T(0);
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const T w = wave_sum(v0 * x0[c] + v1 * x1[c]) * tau;
      x0[c] -= w * v0;
      x1[c] -= w * v1;
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    if (col0 + c >= C.nrhs) break;
    if (nd.is_leaf) {
      T* out = C.B + nd.row0 + (int64_t)(col0 + c) * C.ldb;
      if (r0 < mp) out[r0] = x0[c];
      if (r1 < mp) out[r1] = x1[c];
      continue;
    }
    const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
    const int64_t co = (int64_t)(col0 + c) * I.lds;
    T* xa = I.wx + n1.ox + co;
    T* xb = I.wx + n2.ox + co;
    const int k1 = n1.kept;
    if (r0 < k1) xa[r0] = x0[c]; else if (r0 < mp) xb[r0 - k1] = x0[c];
    if (r1 < k1) xa[r1] = x1[c]; else if (r1 < mp) xb[r1 - k1] = x1[c];
  }
}

template <typename T>
void launch_solve_w(UlvStep step, const KArgs<T, CallSV<T>>& a, int nitems, int ncols,
                    int64_t stage_elems, hipStream_t s) {
  if (nitems <= 0 || ncols <= 0) return;
  KArgs<T, CallSV<T>> b = a;
  b.ntasks = nitems;
  const bool batch = a.tasks != nullptr;
  const bool staged = stage_elems > 0;
  const size_t sm = staged ? (size_t)stage_elems * sizeof(T) : 0;
  const bool leafy = !batch && a.node0 > 0 && a.node0 == a.inst.nnodes / 2;
  static const char* nm64[] = {"sv_fwd_f64", "sv_fwd_leaf_f64", "sv_bwd_f64", "sv_bwd_leaf_f64",
                               "sv_root_f64"};
  static const char* nm32[] = {"sv_fwd_f32", "sv_fwd_leaf_f32", "sv_bwd_f32", "sv_bwd_leaf_f32",
                               "sv_root_f32"};
  const int ni = step == UlvStep::Root
                     ? 4
                     : (step == UlvStep::Fwd || step == UlvStep::FwdOp ? 0 : 2) + (leafy ? 1 : 0);
  TimedLaunch tl((sizeof(T) == 8 ? nm64 : nm32)[ni], s);
  // columns per wavefront: 4 when there are enough columns to share the factor
  // reads (8 in batched calls of 8 or more columns, where there are nodes
  // enough to fill the chip with half the wavefronts), unless the caller
  // chose (a tuned choice)
  const int cpw = a.cpw == 1 || a.cpw == 4 || a.cpw == 8 ? a.cpw
                : (ncols >= 8 && batch ? 8 : (ncols >= 4 ? 4 : 1));
  const int cgroups = (ncols + cpw - 1) / cpw;
  dim3 gridw((nitems + kSW - 1) / kSW, cgroups), blockw(kSW * 64);
  // eight wavefronts (one staging round trip) for the root and for the
  // forward sweep of a short single-matrix level; four (more nodes per CU)
  // for long or batched levels and for the backward sweep (one block)
  const int sw = step == UlvStep::Root ? kSWS
               : (step == UlvStep::Fwd && !batch && nitems <= kSWSMaxItems ? kSWS : kSW);
  dim3 grid1(nitems, (cgroups + sw - 1) / sw), block1(sw * 64);
#define HSS_SL(K, ST, CP, G, B)                                                   \
  if (batch) hipLaunchKernelGGL((K<T, true, ST, CP>), G, B, sm, s, b);            \
  else hipLaunchKernelGGL((K<T, false, ST, CP>), G, B, sm, s, b);
#define HSS_SL2(K, ST, G, B)                 \
  if (cpw == 8) { HSS_SL(K, ST, 8, G, B) }   \
  else if (cpw == 4) { HSS_SL(K, ST, 4, G, B) }   \
  else { HSS_SL(K, ST, 1, G, B) }
  switch (step) {
    case UlvStep::FwdOp: {
      // at most four columns per wavefront here (eight spill the record products)
      const int cpo = cpw == 8 ? 4 : cpw;
      const int g4 = ((ncols + cpo - 1) / cpo + kOpW - 1) / kOpW;
      const dim3 go(nitems, g4), bo(kOpW * 64);
      const size_t smo = (size_t)fwd_op_lds_elems(cpo) * sizeof(T);
      if (cpo == 4) {
        if (batch) hipLaunchKernelGGL((k_sv_fwd_op<T, true, 4>), go, bo, smo, s, b);
        else hipLaunchKernelGGL((k_sv_fwd_op<T, false, 4>), go, bo, smo, s, b);
      } else {
        if (batch) hipLaunchKernelGGL((k_sv_fwd_op<T, true, 1>), go, bo, smo, s, b);
        else hipLaunchKernelGGL((k_sv_fwd_op<T, false, 1>), go, bo, smo, s, b);
      }
      break;
    }
    case UlvStep::Fwd:
      if (staged) { HSS_SL2(k_sv_fwd_w, true, grid1, block1) }
      else { HSS_SL2(k_sv_fwd_w, false, gridw, blockw) }
      break;
    case UlvStep::Bwd:
      if (staged) { HSS_SL2(k_sv_bwd_w, true, grid1, block1) }
      else { HSS_SL2(k_sv_bwd_w, false, gridw, blockw) }
      break;
    case UlvStep::Root:
      if (cpw == 8) {
        if (batch) hipLaunchKernelGGL((k_sv_root_w<T, true, 8>), grid1, block1, sm, s, b);
        else hipLaunchKernelGGL((k_sv_root_w<T, false, 8>), grid1, block1, sm, s, b);
      } else if (cpw == 4) {
        if (batch) hipLaunchKernelGGL((k_sv_root_w<T, true, 4>), grid1, block1, sm, s, b);
        else hipLaunchKernelGGL((k_sv_root_w<T, false, 4>), grid1, block1, sm, s, b);
      } else {
        if (batch) hipLaunchKernelGGL((k_sv_root_w<T, true, 1>), grid1, block1, sm, s, b);
        else hipLaunchKernelGGL((k_sv_root_w<T, false, 1>), grid1, block1, sm, s, b);
      }
      break;
    default: break;
  }
#undef HSS_SL2
#undef HSS_SL
}

template void launch_solve_w<double>(UlvStep, const KArgs<double, CallSV<double>>&, int, int,
                                     int64_t, hipStream_t);
template void launch_solve_w<float>(UlvStep, const KArgs<float, CallSV<float>>&, int, int,
                                    int64_t, hipStream_t);

}  // namespace hss
