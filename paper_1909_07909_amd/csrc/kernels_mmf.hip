// HSS matrix x block product Y = A X (Sec. 4.1) in three launches:
//
//   up    one work-group per leaf: x^_i = V_i^T X_i; the work-group that
//         completes the second child of a node goes on to that node
//         (arrival counted by an atomic per node): core blocks
//         y^_c1 = B12_t x^_c2, y^_c2 = B21_t x^_c1, and, below the root,
//         x^_t = W_t^T [x^_c1; x^_c2]; so the whole upward pass and all
//         core blocks are one launch;
//   down  one work-group per node s at level max(p-3, 0): walks the path
//         from the root to s and then the levels of its subtree,
//         y^_c = y^_c(core) + R_t[c rows] y^_t, and stores y^ of its leaves;
//   leaf  one work-group per (leaf, chunk of right-hand sides):
//         Y_i = D_i X_i + U_i y^_i, D_i and U_i streamed once into registers.
//
// The per-level launches of kernels_mm.hip remain for A^T X.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {

constexpr int kDC = 8;       // right-hand-side columns per down work-group
constexpr int kUT = 256;     // threads of the up kernel
constexpr int kDT = 512;     // threads of the down kernel
constexpr int kLT = 512;     // threads of the leaf kernel
constexpr int kDnH = 3;      // subtree height of a down work-group
constexpr int kUpH = 2;      // subtree height of an up work-group
constexpr int kXP = kMaxBlock + 8;   // padded LDS column of an X chunk

// LDS row of element i of an X chunk: a gap of two after every 32 rows so that
// the four quarter-wavefronts of the leaf kernel read different banks.
__device__ __forceinline__ int xrow(int i) { return i + ((i >> 5) << 1); }

// x^ values cross work-groups inside the up kernel: agent-scope atomic
// accesses, which are coherent across the XCDs' L2 caches without cache-wide
// write-back or invalidation.
template <typename T>
__device__ __forceinline__ void xh_put(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T xh_get(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// dst[i + c*ldd] = src[i + c*lds] for i < rows (zero for rows <= i < ldd),
// c < nc <= MC, by all threads of the work-group: every load is issued (from
// a clamped, valid address) before the first LDS store.
template <int MC, typename T>
__device__ __forceinline__ void stage_cols(T* dst, int ldd, int rows, int nc, const T* src,
                                           int64_t lds) {
  const int total = ldd * nc;
  constexpr int U = (kMaxBlock * MC + 255) / 256;
  const int nt = blockDim.x;
  T v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int o = threadIdx.x + u * nt;
    const int i = o % ldd, c = min(o / ldd, nc - 1);
    const T x = src[min(i, rows - 1) + (int64_t)c * lds];
    v[u] = (i < rows) ? x : T(0);
    if (u * nt >= total) break;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int o = threadIdx.x + u * nt;
    if (o < total) dst[o] = v[u];
  }
}

// out(i, c, sum_l A(i, l) * in[l + c*ldi]) for i < M, c < nc, by all threads of
// the work-group; A(i, l) = A[i + l*lda] (or A[l + i*lda] when TA).  One thread
// per output; its coefficient loads are issued 64 at a time from clamped
// (always valid) addresses and masked afterwards, so they are all in flight
// together instead of one round trip each.
template <typename T, bool TA, typename Out>
__device__ __forceinline__ void wg_small_gemm(int M, int K, int nc, const T* __restrict__ A,
                                              int lda, const T* in, int ldi, Out out) {
  constexpr int KB = 32;
  const uint32_t span = TA ? (uint32_t)((M - 1) * lda + K) : (uint32_t)((K - 1) * lda + M);
  const auto Ar = buf_rsrc(A, span * (uint32_t)sizeof(T));
  const uint32_t ls = (uint32_t)(TA ? 1 : lda) * (uint32_t)sizeof(T);   // stride of l
  for (int o = threadIdx.x; o < M * nc; o += blockDim.x) {
    const int i = o % M, c = o / M;
    const uint32_t vo = (uint32_t)(TA ? i * lda : i) * (uint32_t)sizeof(T);
    T s = T(0);
    for (int l0 = 0; l0 < K; l0 += KB) {
      T av[KB];
#pragma unroll
      for (int l = 0; l < KB; ++l) av[l] = buf_load<T>(Ar, vo, (uint32_t)(l0 + l) * ls);
#pragma unroll
      for (int l = 0; l < KB; ++l) {
        const int lc = min(l0 + l, K - 1);
        const T t = av[l] * in[lc + c * ldi];
        s += (l0 + l < K) ? t : T(0);
      }
    }
    out(i, c, s);
  }
}

// Products of one node t with its children's x^ staged in xs (rows
// [x^_c1; x^_c2], column c at xs + c*kMaxBlock), one per wavefront:
//   wavefront 0: y^_c1 = B12 x^_c2 (global, read by the down kernel)
//   wavefront 1: y^_c2 = B21 x^_c1
//   wavefronts 2, 3 (below the root): x^_t = W^T [x^_c1; x^_c2], half of the
//   outputs each, into xo (kMaxRank x nc in LDS)
// The coefficients are loaded into registers first (cf_load) so that their
// loads overlap with the staging of xs; cf_apply runs after a barrier.
template <typename T, int KQ>
struct NodeStep {
  int t, kv1, kk, ni, i0;
  bool bw;
  T cf[KQ];

  __device__ __forceinline__ void load(const Inst<T>& I, int node, int w, int lane) {
    t = node;
    const NodeInfo nt = I.nodes[t];
    const NodeInfo n1 = I.nodes[2 * t + 1], n2 = I.nodes[2 * t + 2];
    kv1 = n1.kv;
    kk = n1.kv + n2.kv;
    bw = w < 2;
    const int kvt = (t > 0 && kk > 0) ? nt.kv : 0;
    const int half = (kvt + 1) >> 1;
    i0 = (w - 2) * half;
    ni = bw ? 0 : min(half, kvt - i0);
    const int bM = w == 0 ? n1.ku : n2.ku, bK = w == 0 ? n2.kv : n1.kv;
    // (clamped addresses, loads unconditional, masks applied to the values)
    if (bw && bM > 0 && bK > 0) {
      const T* Bm = w == 0 ? I.B12 + nt.oB12 : I.B21 + nt.oB21;
      const int rr = min(lane, bM - 1);
      const bool lr = lane < bM;
#pragma unroll
      for (int k = 0; k < KQ; ++k)
        cf[k] = ld_or0(Bm + rr + (int64_t)min(k, bK - 1) * bM, lr & (k < bK));
    } else if (!bw && ni > 0) {
      // lane l: W[l + i*kk] (cf[q]) and W[l + 64 + i*kk] (cf[KQ/2 + q]) for
      // the ni <= KQ/2 outputs i0 .. i0+ni-1; the root has no W block
      const T* Wt = I.W + nt.oW;
      const int la = min(lane, kk - 1), lb = min(lane + 64, kk - 1);
      const bool ka = lane < kk, kb = lane + 64 < kk;
#pragma unroll
      for (int q = 0; q < KQ / 2; ++q) {
        const T* wi = Wt + (int64_t)(i0 + min(q, ni - 1)) * kk;
        cf[q] = ld_or0(wi + la, ka & (q < ni));
        cf[KQ / 2 + q] = ld_or0(wi + lb, kb & (q < ni));
      }
    } else {
#pragma unroll
      for (int q = 0; q < KQ; ++q) cf[q] = T(0);
    }
  }

  __device__ __forceinline__ void apply(const Inst<T>& I, int w, int lane, int c0, int nc,
                                        const T* xs, T* xo) const {
    if (bw) {
      const NodeInfo nc1 = I.nodes[2 * t + 1 + w];
      const int bM = nc1.ku, bK = w == 0 ? kk - kv1 : kv1, bx = w == 0 ? kv1 : 0;
      T* bout = I.yh + nc1.oyh;
      for (int c = 0; c < nc; ++c) {
        const T* x = xs + bx + c * kMaxBlock;
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < KQ; ++k) acc += cf[k] * x[min(k, max(bK - 1, 0))];
        if (lane < bM) bout[lane + (int64_t)(c0 + c) * I.ldm] = acc;
      }
    } else if (ni > 0) {
      for (int c = 0; c < nc; ++c) {
        const T xa = xs[min(lane, kk - 1) + c * kMaxBlock];
        const T xb = xs[min(lane + 64, kk - 1) + c * kMaxBlock];
#pragma unroll
        for (int q = 0; q < KQ / 2; ++q) {
          if (q < ni) {
            const T sum = wave_sum(cf[q] * xa + cf[KQ / 2 + q] * xb);
            if (lane == 0) xo[i0 + q + c * kMaxRank] = sum;
          }
        }
      }
    }
  }
};

template <typename T>
__device__ __forceinline__ T tsum8_dpp(T (&v)[8]);

// One work-group per subtree of 2^h leaves (h = min(kUpH, p)), rooted at node
// g of level p - h.  Each wavefront projects its leaves (x^_i = V_i^T X_i),
// the subtree's internal nodes are then taken bottom-up inside the
// work-group (x^ kept in LDS), and from g the work-group climbs while it is
// the second arrival at the next node (arrival counted by an atomic per node).
// MC: right-hand-side chunk; KQ: coefficients per lane of a product (>= every
// rank; a W^T wavefront takes at most KQ/2 outputs, children's ranks <= 128).
template <typename T, bool BATCH, int MC, int KQ>
__global__ __launch_bounds__(kUT) void k_mmf_up(KArgs<T, CallMM<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  __shared__ unsigned s_arrive;
  Inst<T> I; CallMM<T> C; int g;
  resolve<BATCH>(a, I, C, g);
  if (gated_off(C.gate)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nrhs = C.nrhs;
  const int ncw = min(MC, nrhs);
  const int64_t ldm = I.ldm;
  const int h = I.p - I.nodes[g].level;          // subtree height (<= kUpH)
  const int nl = 1 << h;                          // leaves of the subtree
  T* xs = reinterpret_cast<T*>(smem_raw);         // kMaxBlock x ncw: children's x^
  T* xl = xs + kMaxBlock * ncw;                   // 2 x nl x kMaxRank x ncw: x^ of a level
  const int64_t slot = (int64_t)kMaxRank * ncw;
  for (int c0 = 0; c0 < nrhs; c0 += MC) {
    const int nc = min(MC, nrhs - c0);
    // ---- leaves: wavefront w takes leaves w, w+4, ...; lane rows l, l+64
    for (int j = w; j < nl; j += kUT / 64) {
      const int leaf = ((g + 1) << h) - 1 + j;
      const NodeInfo nd = I.nodes[leaf];
      const int m = nd.m, kv = nd.kv;
      const int r0 = min(lane, m - 1), r1 = min(lane + 64, m - 1);
      T x0[MC], x1[MC];
      const T* Xb = C.X + nd.row0 + (int64_t)c0 * C.ldx;
#pragma unroll
      for (int c = 0; c < MC; ++c) {
        const int cc = min(c, nc - 1);
        x0[c] = ld_or0(Xb + r0 + (int64_t)cc * C.ldx, (lane < m) & (c < nc));
        x1[c] = ld_or0(Xb + r1 + (int64_t)cc * C.ldx, (lane + 64 < m) & (c < nc));
      }
      const auto Vr = buf_rsrc(I.V + nd.oV, (uint32_t)(m * kv * (int)sizeof(T)));
      const uint32_t cs = (uint32_t)(m * (int)sizeof(T));
      const uint32_t o0 = (uint32_t)(r0 * (int)sizeof(T)), o1 = (uint32_t)(r1 * (int)sizeof(T));
      T* out = xl + (int64_t)j * slot;
      for (int b = 0; b < kv; b += 16) {       // 16 columns of V in flight
        T va[16], vb[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          va[u] = buf_load<T>(Vr, o0, (uint32_t)(b + u) * cs);   // columns >= kv read zero
          vb[u] = buf_load<T>(Vr, o1, (uint32_t)(b + u) * cs);
        }
        // eight columns of V per transposed sum: lane j < 8 ends with the
        // total for column b + 8 hf + j
#pragma unroll
        for (int c = 0; c < MC; ++c) {
          if (c < nc) {
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
              if (b + 8 * hf < kv) {
                T pv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) pv[u] = va[8 * hf + u] * x0[c] + vb[8 * hf + u] * x1[c];
                const T sv = tsum8_dpp(pv);
                if (lane < 8 && b + 8 * hf + lane < kv) out[b + 8 * hf + lane + c * kMaxRank] = sv;
              }
            }
          }
        }
      }
    }
    __syncthreads();
    // ---- internal nodes of the subtree, level by level (x^ of level d in
    // half (d & 1) of xl, node j of the level in slot j)
    for (int d = h - 1; d >= 0; --d) {
      T* src = xl + (int64_t)((h - 1 - d) & 1) * nl * slot;   // children level
      T* dst = xl + (int64_t)((h - d) & 1) * nl * slot;
      if (d == h - 1) src = xl;                                // the leaves' x^
      for (int j = 0; j < (1 << d); ++j) {
        const int t = ((g + 1) << d) - 1 + j;
        NodeStep<T, KQ> st;
        st.load(I, t, w, lane);
        // children's x^ -> xs
        const int kv1 = st.kv1, kk = st.kk;
        for (int o = tid; o < kk * nc; o += kUT) {
          const int i = o % kk, c = o / kk;
          xs[i + c * kMaxBlock] = i < kv1 ? src[(int64_t)(2 * j) * slot + i + c * kMaxRank]
                                          : src[(int64_t)(2 * j + 1) * slot + i - kv1 + c * kMaxRank];
        }
        __syncthreads();
        st.apply(I, w, lane, c0, nc, xs, dst + (int64_t)j * slot);
        __syncthreads();
      }
    }
    // x^ of g (below the root) for the climb
    if (g > 0) {
      const T* xg = h == 0 ? xl : xl + (int64_t)(h & 1) * nl * slot;
      const int kvg = I.nodes[g].kv;
      if (w == 0)
        for (int o = lane; o < kvg * nc; o += 64)
          xh_put(I.xh + I.nodes[g].oxh + o % kvg + (int64_t)(c0 + o / kvg) * ldm,
                 xg[o % kvg + (o / kvg) * kMaxRank]);
    }
    __syncthreads();
  }
  // Climb: the second arrival at a node carries on with it.  Every x^ that
  // crosses work-groups is written with agent-coherent stores and read with
  // agent-coherent loads; the writers wait for their stores to complete
  // before the barrier that precedes the arrival count, and the reads of the
  // children's x^ are issued only after the count has been seen.
  T* os = xl;   // x^ being formed
  int t = g;
  while (t > 0) {
    const int par = (t - 1) >> 1;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) s_arrive = atomicAdd(I.cnt + par, 1u);
    __syncthreads();
    const bool second = (s_arrive & 1u) != 0;
    __syncthreads();
    if (!second) return;
    t = par;
    NodeStep<T, KQ> st;
    st.load(I, t, w, lane);
    const NodeInfo n1 = I.nodes[2 * t + 1], n2 = I.nodes[2 * t + 2];
    const int kv1 = st.kv1, kk = st.kk;
    for (int c0 = 0; c0 < nrhs; c0 += MC) {
      const int nc = min(MC, nrhs - c0);
      if (kk > 0) {
        constexpr int UX = (2 * kMaxRank * MC + kUT - 1) / kUT;
        T xv[UX];
#pragma unroll
        for (int u = 0; u < UX; ++u) {
          const int o = min(tid + u * kUT, kk * nc - 1);
          const int i = o % kk, c = o / kk;
          const int64_t co = (int64_t)(c0 + c) * ldm;
          xv[u] = xh_get(I.xh + (i < kv1 ? n1.oxh + i : n2.oxh + i - kv1) + co);
        }
#pragma unroll
        for (int u = 0; u < UX; ++u) {
          const int o = tid + u * kUT;
          if (o < kk * nc) xs[o % kk + (o / kk) * kMaxBlock] = xv[u];
        }
      }
      __syncthreads();
      st.apply(I, w, lane, c0, nc, xs, os);
      __syncthreads();
      if (t > 0 && w == 0) {
        const NodeInfo nt = I.nodes[t];
        for (int o = lane; o < nt.kv * nc; o += 64)
          xh_put(I.xh + nt.oxh + o % nt.kv + (int64_t)(c0 + o / nt.kv) * ldm,
                 os[o % nt.kv + (o / nt.kv) * kMaxRank]);
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Up kernel for one right-hand side with every rank <= 32: the work split of
// k_mmf_up (a subtree of 2^h leaves per work-group, then the climb), with
// each internal node taken by ONE wavefront whose coefficients it loaded
// ahead of need, every load coalesced:
//   lane i < 32      row i of B12_t        -> (B12_t x^_c2)[i]
//   lane 32 + i      row i of B21_t        -> (B21_t x^_c1)[i]
//   lane l           row l of W_t          -> W_t[l, :] [x^_c1; x^_c2][l],
//                    summed over the lanes by one transposed reduction
// The wavefronts take the subtree's nodes first and then climb steps s in
// rotation (step s by wavefront (c + s) mod 4, c = number of subtree nodes);
// each loads its next node's coefficients as soon as it is free, so every
// node's loads are in flight while the levels below it are formed.  The
// loads go straight into the coefficient registers (clamped, valid
// addresses; the masks act on the results), so nothing waits for them before
// their use.  x^ vectors live in LDS slots of 32 entries, zero past the rank.
template <typename T>
struct UpCoef {
  T b[32], w[32];
  int kv1, kk, kvt;     // children's ranks (kv1, kv1 + kv2) and the node's
  int bM, bK;           // core block of this lane's half: rows, columns
  int64_t oy;           // y^ of the child this lane's half writes
  const T* bp;          // this lane's row of the core block (b[k] = bp[min(k, bk) * bs])
  int bs, bk;
};

// What a node's coefficient loads need from the node table: read a climb
// step ahead of the loads themselves, so that no wavefront waits for the
// table in front of a barrier.
struct UpMeta {
  int64_t oB12, oB21, oW, oy1, oy2;
  int ku1, ku2, kv1, kv2, kvt;
};

template <typename T>
__device__ __forceinline__ T ld_early(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename T>
__device__ __forceinline__ void up_meta_load(const Inst<T>& I, int t, UpMeta& m) {
  const NodeInfo* nt = I.nodes + t;
  const NodeInfo* n1 = I.nodes + 2 * t + 1;
  const NodeInfo* n2 = I.nodes + 2 * t + 2;
  m.oB12 = ld_early(&nt->oB12);
  m.oB21 = ld_early(&nt->oB21);
  m.oW = ld_early(&nt->oW);
  m.kvt = t > 0 ? ld_early(&nt->kv) : 0;
  m.oy1 = ld_early(&n1->oyh);
  m.oy2 = ld_early(&n2->oyh);
  m.ku1 = ld_early(&n1->ku);
  m.ku2 = ld_early(&n2->ku);
  m.kv1 = ld_early(&n1->kv);
  m.kv2 = ld_early(&n2->kv);
}

// LOADB: load the core-block row now (else up_core_load brings it in later)
template <typename T, bool LOADB = true>
__device__ __forceinline__ void up_coef_issue(const Inst<T>& I, const UpMeta& m, int lane,
                                              UpCoef<T>& c) {
  const int i = lane & 31;
  const bool h = lane >= 32;
  c.kv1 = m.kv1;
  c.kk = m.kv1 + m.kv2;
  c.kvt = m.kvt;
  c.bM = h ? m.ku2 : m.ku1;
  c.bK = h ? m.kv1 : m.kv2;
  c.oy = h ? m.oy2 : m.oy1;
  // an empty block reads the node table instead (a valid address; its
  // result is masked)
  const T* dummy = reinterpret_cast<const T*>(I.nodes);
  const bool bv = c.bM > 0 && c.bK > 0;
  const T* br = bv ? (h ? I.B21 + m.oB21 : I.B12 + m.oB12) + min(i, c.bM - 1) : dummy;
  const int bs = bv ? c.bM : 0, bk = bv ? c.bK - 1 : 0;
  c.bp = br;
  c.bs = bs;
  c.bk = bk;
  if (LOADB) {
#pragma unroll
    for (int k = 0; k < 32; ++k) c.b[k] = ld_early(br + (int64_t)min(k, bk) * bs);
  }
  const bool wv = c.kvt > 0 && c.kk > 0;
  const T* wr = wv ? I.W + m.oW + min(lane, c.kk - 1) : dummy;
  const int ws = wv ? c.kk : 0, wk = wv ? c.kvt - 1 : 0;
#pragma unroll
  for (int q = 0; q < 32; ++q) c.w[q] = ld_early(wr + (int64_t)min(q, wk) * ws);
}

template <typename T, bool LOADB = true>
__device__ __forceinline__ void up_coef_load(const Inst<T>& I, int t, int lane, UpCoef<T>& c) {
  UpMeta m;
  up_meta_load(I, t, m);
  up_coef_issue<T, LOADB>(I, m, lane, c);
}
template <typename T>
__device__ __forceinline__ void up_core_load(UpCoef<T>& c) {
#pragma unroll
  for (int k = 0; k < 32; ++k) c.b[k] = c.bp[(int64_t)min(k, c.bk) * c.bs];
}

// update_dpp with an old value and a bank mask (banks: lanes 4b..4b+3 of a row)
template <int CTRL, int BANKS>
__device__ __forceinline__ double dpp_old(double old, double v) {
  const long long o = __double_as_longlong(old), b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), CTRL,
                                             0xF, BANKS, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xF, BANKS, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int BANKS>
__device__ __forceinline__ float dpp_old(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                    0xF, BANKS, false));
}
// (x, y) -> the permlane swap pair; .first + .second is the butterfly sum
template <bool P32>
__device__ __forceinline__ void plswap(float& x, float& y) {
  const auto r = P32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false)
                     : __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  x = __uint_as_float(r[0]);
  y = __uint_as_float(r[1]);
}
template <bool P32>
__device__ __forceinline__ void plswap(double& x, double& y) {
  const uint64_t a = __double_as_longlong(x), b = __double_as_longlong(y);
  const auto l = P32 ? __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false)
                     : __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
  const auto u = P32 ? __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false)
                     : __builtin_amdgcn_permlane16_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
  x = __longlong_as_double(((uint64_t)u[0] << 32) | l[0]);
  y = __longlong_as_double(((uint64_t)u[1] << 32) | l[1]);
}

// Transposed wavefront sum: v[0..31] per lane; lanes i and i + 32 return the
// sum over all 64 lanes of v[i].  Five halving butterflies over lane bits
// 4..0 (value k stays with the lanes whose bit is clear, k + W with the
// others), then the two 32-lane halves are added; every exchange is a
// permlane swap or a DPP move, no LDS.
template <typename T>
__device__ __forceinline__ T tsum32_dpp(T (&v)[32]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 16; ++k) {          // bit 4: permlane16 swap
    T x = v[k], y = v[16 + k];
    plswap<false>(x, y);
    v[k] = x + y;
  }
  {
    const bool b = (lane & 8) != 0;       // bit 3: rotate rows by 8
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T send = b ? v[k] : v[8 + k], keep = b ? v[8 + k] : v[k];
      v[k] = keep + dpp<kDppRowRor8>(send);
    }
  }
  {
    const bool b = (lane & 4) != 0;       // bit 2: shift left 4 into banks 0, 2, right 4 into 1, 3
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T send = b ? v[k] : v[4 + k], keep = b ? v[4 + k] : v[k];
      const T r = dpp_old<0x114, 0xA>(dpp_old<0x104, 0x5>(T(0), send), send);
      v[k] = keep + r;
    }
  }
  {
    const bool b = (lane & 2) != 0;       // bit 1
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T send = b ? v[k] : v[2 + k], keep = b ? v[2 + k] : v[k];
      v[k] = keep + dpp<kDppQuadXor2>(send);
    }
  }
  {
    const bool b = (lane & 1) != 0;       // bit 0
    const T send = b ? v[0] : v[1], keep = b ? v[1] : v[0];
    v[0] = keep + dpp<kDppQuadXor1>(send);
  }
  T x = v[0], y = v[0];
  plswap<true>(x, y);
  return x + y;
}

// tsum32_dpp for v[0..15]: lanes i, i + 16, i + 32, i + 48 return the sum over
// all 64 lanes of v[i].
template <typename T>
__device__ __forceinline__ T tsum16_dpp(T (&v)[16]) {
  const int lane = threadIdx.x & 63;
  {
    const bool b = (lane & 8) != 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T send = b ? v[k] : v[8 + k], keep = b ? v[8 + k] : v[k];
      v[k] = keep + dpp<kDppRowRor8>(send);
    }
  }
  {
    const bool b = (lane & 4) != 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T send = b ? v[k] : v[4 + k], keep = b ? v[4 + k] : v[k];
      const T r = dpp_old<0x114, 0xA>(dpp_old<0x104, 0x5>(T(0), send), send);
      v[k] = keep + r;
    }
  }
  {
    const bool b = (lane & 2) != 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T send = b ? v[k] : v[2 + k], keep = b ? v[2 + k] : v[k];
      v[k] = keep + dpp<kDppQuadXor2>(send);
    }
  }
  {
    const bool b = (lane & 1) != 0;
    const T send = b ? v[0] : v[1], keep = b ? v[1] : v[0];
    v[0] = keep + dpp<kDppQuadXor1>(send);
  }
  T x = v[0], y = v[0];
  plswap<false>(x, y);
  T x2 = x + y, y2 = x + y;
  plswap<true>(x2, y2);
  return x2 + y2;
}

// tsum32_dpp for v[0..7]: lane l returns the sum over all 64 lanes of v[l & 7].
template <typename T>
__device__ __forceinline__ T tsum8_dpp(T (&v)[8]) {
  const int lane = threadIdx.x & 63;
  {
    const bool b = (lane & 4) != 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T send = b ? v[k] : v[4 + k], keep = b ? v[4 + k] : v[k];
      const T r = dpp_old<0x114, 0xA>(dpp_old<0x104, 0x5>(T(0), send), send);
      v[k] = keep + r;
    }
  }
  {
    const bool b = (lane & 2) != 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T send = b ? v[k] : v[2 + k], keep = b ? v[2 + k] : v[k];
      v[k] = keep + dpp<kDppQuadXor2>(send);
    }
  }
  {
    const bool b = (lane & 1) != 0;
    const T send = b ? v[0] : v[1], keep = b ? v[1] : v[0];
    v[0] = keep + dpp<kDppQuadXor1>(send);
  }
  T x = v[0] + dpp<kDppRowRor8>(v[0]);
  T y = x;
  plswap<false>(x, y);
  T x2 = x + y, y2 = x + y;
  plswap<true>(x2, y2);
  return x2 + y2;
}

// Core products of node t from its children's x^ in LDS (xa: c1, xb: c2,
// 32 entries each): y^_c1 = B12_t x^_c2 (lanes < 32), y^_c2 = B21_t x^_c1.
template <typename T>
__device__ __forceinline__ void up_core(const Inst<T>& I, int lane, const UpCoef<T>& c,
                                        const T* xa, const T* xb, int nc = 1) {
  const int i = lane & 31;
  for (int col = 0; col < nc; ++col) {
    const T* xo = (lane >= 32 ? xa : xb) + 32 * col;
    T b0 = T(0), b1 = T(0);
#pragma unroll
    for (int k = 0; k < 32; k += 2) {
      b0 += c.b[k] * xo[k];
      b1 += c.b[k + 1] * xo[k + 1];
    }
    if (i < c.bM) I.yh[c.oy + i + (int64_t)col * I.ldm] = c.bK > 0 ? b0 + b1 : T(0);
  }
}
// x^_t[lane & 31] = (W_t^T [x^_c1; x^_c2]) (zero when W_t is empty; unused at
// the root).  Consumes the W coefficients.
// Column col of x^_t for several right-hand sides (keeps the coefficients).
template <typename T>
__device__ __forceinline__ T up_w_col(int lane, const UpCoef<T>& c, const T* xa, const T* xb,
                                      int col) {
  const T x1 = xa[32 * col + min(lane, 31)], x2 = xb[32 * col + min(max(lane - c.kv1, 0), 31)];
  const T xl = lane < c.kv1 ? x1 : (lane < c.kk ? x2 : T(0));
  // outputs 0..15, then 16..31 (lane i < 32 keeps output i)
  T p[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) p[q] = c.w[q] * xl;
  const T lo = tsum16_dpp(p);
#pragma unroll
  for (int q = 0; q < 16; ++q) p[q] = c.w[16 + q] * xl;
  const T hi = tsum16_dpp(p);
  const T x = (lane & 16) ? hi : lo;
  return c.kk > 0 ? x : T(0);
}
template <typename T>
__device__ __forceinline__ T up_w(int lane, UpCoef<T>& c, const T* xa, const T* xb) {
  const T x1 = xa[min(lane, 31)], x2 = xb[min(max(lane - c.kv1, 0), 31)];
  const T xl = lane < c.kv1 ? x1 : (lane < c.kk ? x2 : T(0));
#pragma unroll
  for (int q = 0; q < 32; ++q) c.w[q] *= xl;
  const T x = tsum32_dpp(c.w);
  return c.kk > 0 ? x : T(0);
}

static_assert(kUpH <= 2, "k_mmf_up1 keeps at most three subtree nodes in LDS slots 4-6");

// Mailbox entries: written once per product by the first arrival at a node,
// read and emptied again by the second.
__device__ __forceinline__ bool mb_empty(double v) {
  return (uint64_t)__double_as_longlong(v) == kMbEmpty64;
}
__device__ __forceinline__ bool mb_empty(float v) { return __float_as_uint(v) == kMbEmpty32; }
template <typename T>
__device__ __forceinline__ T mb_empty_value();
template <>
__device__ __forceinline__ double mb_empty_value<double>() {
  return __longlong_as_double((long long)kMbEmpty64);
}
template <>
__device__ __forceinline__ float mb_empty_value<float>() {
  return __uint_as_float(kMbEmpty32);
}
constexpr int kMbPolls = 1 << 20;   // bound of a mailbox wait (~0.1 s); never reached in practice

// Y_i = D_i X_i for one leaf (one right-hand side) by a work-group of kUT
// threads: wavefront w takes the row blocks of waves w and w + 4 of the leaf
// kernel's layout (rows 16v .. 16v+15, lane quarter q: columns 32q .. 32q+31)
// with the same sums in the same order, so Y matches k_mmf_leaf bit for bit.
template <typename T>
__device__ __forceinline__ void up_leaf_dx(const Inst<T>& I, const CallMM<T>& C, int leaf,
                                           T* xs) {
  const NodeInfo nd = I.nodes[leaf];
  const int m = nd.m;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4;
  const auto Dr = buf_rsrc(I.D + nd.oD, (uint32_t)(m * m * (int)sizeof(T)));
  const uint32_t cs = (uint32_t)(m * (int)sizeof(T));
  T dv[2][32];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int row = 16 * (w + 4 * v) + (lane & 15);
    const uint32_t rb = (uint32_t)(min(row, m - 1) * (int)sizeof(T));
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) {
      const T x = buf_load<T>(Dr, rb + (uint32_t)(32 * q) * cs, (uint32_t)jj * cs);
      dv[v][jj] = row < m ? x : T(0);
    }
  }
  if (threadIdx.x < kMaxBlock) {
    const int i = threadIdx.x;
    const T x = C.X[nd.row0 + min(i, m - 1)];
    xs[xrow(i)] = i < m ? x : T(0);
  }
  __syncthreads();
  const T* xc = xs + xrow(32 * q);
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int row = 16 * (w + 4 * v) + (lane & 15);
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int jj = 0; jj < 32; jj += 2) {
      s0 += dv[v][jj] * xc[jj];
      s1 += dv[v][jj + 1] * xc[jj + 1];
    }
    T sd = s0 + s1;
    sd += __shfl_xor(sd, 16, 64);
    sd += __shfl_xor(sd, 32, 64);
    if (q == 0 && row < m) C.Y[nd.row0 + row] = sd;
  }
}

// DX: blocks a.ntasks .. a.ntasks + 2^p - 1 (dispatched after the subtree
// blocks, so they start as those finish their leaves) form Y_i = D_i X_i.
// NC > 1: up to NC right-hand sides (columns c of a slot at 32 c), the
// products column by column with the coefficients kept, the leaves' x^ by
// 16-column transposed sums.
template <typename T, bool BATCH, bool DX, int NC>
__global__ __launch_bounds__(kUT) __attribute__((amdgpu_waves_per_eu(2))) void k_mmf_up1(
    KArgs<T, CallMM<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  __shared__ unsigned s_arrive;
  if constexpr (DX) {
    if ((int)blockIdx.x >= a.ntasks) {
      if (gated_off(a.call.gate)) return;
      up_leaf_dx(a.inst, a.call, (1 << a.inst.p) - 1 + (int)blockIdx.x - a.ntasks,
                 reinterpret_cast<T*>(smem_raw));
      return;
    }
  }
  Inst<T> I; CallMM<T> C; int g;
  resolve<BATCH>(a, I, C, g);
  if (gated_off(C.gate)) return;
  if constexpr (!BATCH && NC > 1) {
    // column chunk blockIdx.y (the grid has no empty chunk): its columns, and
    // arrival counters and mailboxes of its own, so that the chunks climb
    // side by side
    const int y = blockIdx.y;
    C.X += (int64_t)y * NC * C.ldx;
    C.nrhs -= y * NC;
    I.yh += (int64_t)y * NC * I.ldm;
    I.cnt += (int64_t)y * ((I.nnodes + 2) & ~1);
    I.mb += (int64_t)y * I.nnodes * kMbSlot * kMbCols;
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int SL = 32 * NC;                // LDS slot
  constexpr int MB = kMbSlot * NC;           // mailbox entries per node
  const int nc = min(NC, C.nrhs);
  // LDS slots of SL entries: leaves 0-3, subtree nodes 4-6, then per climb
  // step s: the node's x^ in 7 + (s & 3), its sibling child's x^ in 11 + (s & 3)
  T* xs = reinterpret_cast<T*>(smem_raw);
  const int h = I.p - I.nodes[g].level;     // subtree height (<= kUpH)
  const int nl = 1 << h, cnt = nl - 1;       // leaves and internal nodes of the subtree
  // internal node q of the subtree, bottom-up: level d = h-1 first
  auto sub_node = [&](int q) {
    const int d = q < nl - 2 ? h - 1 : 0;    // (h <= 2: at most two levels)
    const int j = d == h - 1 ? q : q - (nl - 2);
    return ((g + 1) << d) - 1 + j;
  };
  // node of climb step s (the ancestor of g s + 1 levels up; -1 past the root)
  // and its wavefront
  auto step_node = [&](int s) { return s < 31 ? ((g + 1) >> (s + 1)) - 1 : -1; };
  auto holder = [&](int s) { return (cnt + s) & 3; };
  UpCoef<T> cf;
  UpMeta mt;   // node table entries of this wavefront's next climb node
  {
    const int t0 = w < cnt ? sub_node(w) : (w == holder(0) ? step_node(0) : -1);
    if (t0 >= 0) up_coef_load<T, NC == 1>(I, t0, lane, cf);
    const int tm = w == holder(1) ? step_node(1) : (w == holder(2) ? step_node(2) : -1);
    if (tm >= 0) up_meta_load(I, tm, mt);
  }
  // ---- leaves: wavefront w takes leaf w; lane rows l, l + 64
  if (NC > 1 && w < nl) {
    const int leaf = ((g + 1) << h) - 1 + w;
    const NodeInfo nd = I.nodes[leaf];
    const int m = nd.m, kv = nd.kv;
    const int r0 = min(lane, m - 1), r1 = min(lane + 64, m - 1);
    T x0[NC], x1[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T* Xc = C.X + nd.row0 + (int64_t)min(c, nc - 1) * C.ldx;
      x0[c] = ld_or0(Xc + r0, (lane < m) & (c < nc));
      x1[c] = ld_or0(Xc + r1, (lane + 64 < m) & (c < nc));
    }
    const auto Vr = buf_rsrc(I.V + nd.oV, (uint32_t)(m * kv * (int)sizeof(T)));
    const uint32_t cs = (uint32_t)(m * (int)sizeof(T));
    const uint32_t o0 = (uint32_t)(r0 * (int)sizeof(T)), o1 = (uint32_t)(r1 * (int)sizeof(T));
    T* out = xs + SL * w;
    for (int b = 0; b < kv; b += 8) {        // 8 columns of V at a time
      T va[8], vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        va[u] = buf_load<T>(Vr, o0, (uint32_t)(b + u) * cs);   // columns >= kv read zero
        vb[u] = buf_load<T>(Vr, o1, (uint32_t)(b + u) * cs);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (c < nc) {
          T pv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) pv[u] = va[u] * x0[c] + vb[u] * x1[c];
          const T sv = tsum8_dpp(pv);
          if (lane < 8) out[32 * c + b + lane] = b + lane < kv ? sv : T(0);
        }
      }
    }
    if (lane < 32)
      for (int c = 0; c < nc; ++c)
        if (lane >= kv) out[32 * c + lane] = T(0);
  }
  if (NC == 1 && w < nl) {
    const int leaf = ((g + 1) << h) - 1 + w;
    const NodeInfo nd = I.nodes[leaf];
    const int m = nd.m, kv = nd.kv;
    const int r0 = min(lane, m - 1), r1 = min(lane + 64, m - 1);
    const T* Xb = C.X + nd.row0;
    const T x0 = ld_or0(Xb + r0, lane < m), x1 = ld_or0(Xb + r1, lane + 64 < m);
    const auto Vr = buf_rsrc(I.V + nd.oV, (uint32_t)(m * kv * (int)sizeof(T)));
    const uint32_t cs = (uint32_t)(m * (int)sizeof(T));
    const uint32_t o0 = (uint32_t)(r0 * (int)sizeof(T)), o1 = (uint32_t)(r1 * (int)sizeof(T));
    T* out = xs + SL * w;
    for (int b = 0; b < kv; b += 16) {       // 16 columns of V in flight
      T va[16], vb[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        va[u] = buf_load<T>(Vr, o0, (uint32_t)(b + u) * cs);   // columns >= kv read zero
        vb[u] = buf_load<T>(Vr, o1, (uint32_t)(b + u) * cs);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (b + u < kv) {
          const T sv = wave_sum(va[u] * x0 + vb[u] * x1);
          if (lane == 0) out[b + u] = sv;
        }
      }
    }
    if (lane >= kv && lane < 32) out[lane] = T(0);
  }
  __syncthreads();
  // ---- internal nodes of the subtree, one wavefront each (core products and W)
  T xmine[NC];   // lanes < 32 of the wavefront that formed the latest x^: its entries
#pragma unroll
  for (int c = 0; c < NC; ++c) xmine[c] = T(0);
  for (int d = h - 1; d >= 0; --d) {
    const int qb = (1 << h) - (1 << (d + 1));         // nodes below level d
    const int q = w - qb;
    if (q >= 0 && q < (1 << d)) {
      const int t = ((g + 1) << d) - 1 + q;
      const int cs0 = d == h - 1 ? 2 * q : 4 + (qb - (1 << (d + 1))) + 2 * q;
      const T* xa = xs + SL * cs0;
      const T* xb = xs + SL * (cs0 + 1);
      if constexpr (NC == 1) {
        const T x = up_w(lane, cf, xa, xb);
        xmine[0] = lane < cf.kvt ? x : T(0);
        if (lane < 32) xs[SL * (4 + w) + lane] = xmine[0];
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c < nc) {
            const T x = up_w_col(lane, cf, xa, xb, c);
            xmine[c] = lane < cf.kvt ? x : T(0);
            if (lane < 32) xs[SL * (4 + w) + 32 * c + lane] = xmine[c];
          }
        }
      }
      if (NC > 1) up_core_load(cf);
      up_core(I, lane, cf, xa, xb, nc);
    }
    __syncthreads();
  }
  const int gslot = h > 0 ? 4 + cnt - 1 : 0;   // x^_g
  int prod = h > 0 ? cnt - 1 : 0;              // wavefront holding x^ of the climb's node in xmine
  // ---- climb: the second arrival at a node carries on with it.  The first
  // arrival hands its x^ over through the node's mailbox after counting (so
  // it waits for nothing); the second polls the sibling's mailbox until every
  // entry is written (the writer is running: it has already counted), takes
  // the values and empties the mailbox for the next product.  Mailbox
  // accesses are agent-coherent (across the XCDs' L2 caches).
  // Step s: wavefront holder(s) forms x^ of node s (W part), wavefront
  // holder(s-1) forms the core products of node s-1 (off the critical path)
  // and reads the node table for node s+3, wavefront holder(s+2) loads the
  // coefficients of node s+2.
  auto own_slot = [&](int s) { return s == 0 ? gslot : 7 + ((s - 1) & 3); };
  auto core_of = [&](int s) {   // core products of climb step s, by holder(s)
    const int ch = s == 0 ? g : step_node(s - 1);
    const bool first = (ch & 1) != 0;
    const T* xo = xs + SL * own_slot(s);
    const T* xn = xs + SL * (11 + (s & 3));
    if (NC > 1) up_core_load(cf);
    up_core(I, lane, cf, first ? xo : xn, first ? xn : xo, nc);
  };
  int t = g, s = 0;
  while (t > 0) {
    const int par = (t - 1) >> 1;
    __syncthreads();
    if (tid == 0) s_arrive = atomicAdd(I.cnt + par, 1u);
    __syncthreads();
    const bool go = (s_arrive & 1u) != 0;
    // first arrival: x^_t (zero past its rank) into t's mailbox
    if (!go && w == prod && lane < kMbSlot) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c < nc) xh_put(I.mb + (int64_t)t * MB + 32 * c + lane, xmine[c]);
    }
    if (s > 0 && w == holder(s - 1)) core_of(s - 1);
    if (!go) return;
    if (s == 0 && w == holder(1)) {
      if (step_node(1) >= 0) up_coef_issue<T, NC == 1>(I, mt, lane, cf);
    } else if (w == holder(s + 2)) {
      if (step_node(s + 2) >= 0) up_coef_issue<T, NC == 1>(I, mt, lane, cf);
    } else if (w == holder(s + 3)) {
      if (step_node(s + 3) >= 0) up_meta_load(I, step_node(s + 3), mt);
    }
    if (w == holder(s)) {
      const bool first = (t & 1) != 0;   // t is c1 of par; the sibling is the other child
      const int sib = first ? t + 1 : t - 1;
      T* xn = xs + SL * (11 + (s & 3));
      T* box = I.mb + (int64_t)sib * MB + min(lane, kMbSlot - 1);
      T v[NC];
      auto poll = [&]() {
        bool empty = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          v[c] = c < nc ? xh_get(box + 32 * c) : T(0);
          empty |= c < nc && mb_empty(v[c]);
        }
        return empty;
      };
      for (int it = 0; __any(poll()); ++it) {
        if (it == kMbPolls) {   // the writer never came: report, go on
          if (lane == 0) atomicOr(I.status, 1 << kStatusWaitCode);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (lane < kMbSlot) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c < nc) {
            xn[32 * c + lane] = v[c];
            xh_put(box + 32 * c, mb_empty_value<T>());
          }
        }
      }
      wave_lds_sync();
      const T* xo = xs + SL * own_slot(s);
      if constexpr (NC == 1) {
        const T x = up_w(lane, cf, first ? xo : xn, first ? xn : xo);
        xmine[0] = lane < cf.kvt ? x : T(0);
        if (lane < 32) xs[SL * (7 + (s & 3)) + lane] = xmine[0];
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (c < nc) {
            const T x = up_w_col(lane, cf, first ? xo : xn, first ? xn : xo, c);
            xmine[c] = lane < cf.kvt ? x : T(0);
            if (lane < 32) xs[SL * (7 + (s & 3)) + 32 * c + lane] = xmine[c];
          }
        }
      }
    }
    prod = holder(s);
    t = par;
    ++s;
  }
  // the root's core products (by the wavefront that formed nothing else
  // since: its own LDS writes precede these reads in program order)
  if (s > 0 && w == holder(s - 1)) core_of(s - 1);
}

// Down work-group for subtree root s at level ls: levels 1 .. p of the path
// from the root to s and then of the subtree of s.  Level 1 starts from the
// core values alone; at a deeper level every (node c, row i) slot computes
//   y^_c[i, :] = y^_c(core)[i, :] + R_t[row of c's block + i, :] y^_t
// with t the parent.  Slots are numbered level by level (KR slots per node)
// and dealt to the threads round-robin; the R rows and core values of the
// first NR rounds are loaded before any level is computed, so that the walk
// costs one memory round trip plus one barrier per level.
struct DownMap {
  int ls, p, s;
  // node of slot-level d (d >= 1) and position j (0 .. cnt(d)-1)
  __device__ int cnt(int d) const { return d <= ls ? 1 : 1 << (d - ls); }
  __device__ int node(int d, int j) const {
    return d <= ls ? ((s + 1) >> (ls - d)) - 1 : ((s + 1) << (d - ls)) - 1 + j;
  }
};

// KR <= 32: the row of R is prefetched into registers; above that (64 FP64
// coefficients would take half the register file) it is read from the cache
// when the slot is applied.
template <typename T, int KR, int DC>
struct DownSlot {
  static constexpr bool kRegR = KR <= 32;
  int d = 0, j = 0, i = 0, ku = 0;   // level (0: none), position, row, rank of the node
  T r[kRegR ? KR : 1];
  const T* rp = nullptr;   // the row of R (stride rs, rn coefficients) when not in registers
  int rs = 0, rn = 0;
  T yc[DC];
};

// level of slot g (0: past the last slot)
template <int KR>
__device__ __forceinline__ int down_slot_level(const DownMap& mp, int g) {
  int base = 0;
  for (int d = 2; d <= mp.p; ++d) {
    base += mp.cnt(d) * KR;
    if (g < base) return d;
  }
  return 0;
}

template <typename T, int KR, int DC>
__device__ __forceinline__ void down_slot_load(const Inst<T>& I, const DownMap& mp, int g,
                                               int c0, int nc, DownSlot<T, KR, DC>& sl) {
  sl.d = 0;
  int d = 2, base = 0;
  for (; d <= mp.p; ++d) {
    const int n = mp.cnt(d) * KR;
    if (g < base + n) break;
    base += n;
  }
  const bool have = d <= mp.p;
  const int dd = have ? d : mp.p;
  const int j = have ? (g - base) / KR : 0, i = have ? (g - base) % KR : 0;
  const int cn = mp.node(dd, j), t = (cn - 1) >> 1;
  const NodeInfo nt = I.nodes[t], nn = I.nodes[cn];
  const NodeInfo n1 = I.nodes[2 * t + 1], n2 = I.nodes[2 * t + 2];
  const int kk = n1.ku + n2.ku;
  const int ro = cn == 2 * t + 1 ? 0 : n1.ku;
  const bool live = have & (i < nn.ku) & (nt.ku > 0);   // rows ku .. KR-1 are written as zero
  const int ic = max(min(i, nn.ku - 1), 0);
  const T* Rr = I.R + nt.oR + ro + ic;
  if constexpr (!DownSlot<T, KR, DC>::kRegR) {
    sl.rp = Rr;
    sl.rs = kk;
    sl.rn = (live && nn.ku > 0) ? min(nt.ku, KR) : 0;
  }
  if (nn.ku > 0 && nt.ku > 0) {
    if constexpr (DownSlot<T, KR, DC>::kRegR) {
#pragma unroll
      for (int l = 0; l < KR; ++l) {
        const T v = Rr[(int64_t)min(l, nt.ku - 1) * kk];
        sl.r[l] = (l < nt.ku) ? v : T(0);
      }
    }
    const T* yc = I.yh + nn.oyh + ic + (int64_t)c0 * I.ldm;
#pragma unroll
    for (int c = 0; c < DC; ++c) sl.yc[c] = yc[(int64_t)min(c, nc - 1) * I.ldm];
  } else {
    if constexpr (DownSlot<T, KR, DC>::kRegR) {
#pragma unroll
      for (int l = 0; l < KR; ++l) sl.r[l] = T(0);
    }
#pragma unroll
    for (int c = 0; c < DC; ++c) sl.yc[c] = T(0);
  }
  if (!live) {
    if constexpr (DownSlot<T, KR, DC>::kRegR) {
#pragma unroll
      for (int l = 0; l < KR; ++l) sl.r[l] = T(0);
    }
#pragma unroll
    for (int c = 0; c < DC; ++c) sl.yc[c] = T(0);
  }
  sl.d = have ? dd : 0;
  sl.j = j;
  sl.i = i;
  sl.ku = nn.ku;
}

template <typename T, int KR, int DC>
__device__ __forceinline__ void down_slot_apply(const DownSlot<T, KR, DC>& sl, int nc,
                                                const T* src, T* dst, int64_t blk) {
  const T* ps = src + (int64_t)(sl.j >> 1) * blk;
  T* o = dst + (int64_t)sl.j * blk + sl.i;
  if constexpr (DownSlot<T, KR, DC>::kRegR) {
#pragma unroll
    for (int c = 0; c < DC; ++c) {
      if (c >= nc) break;
      T acc = sl.yc[c];
#pragma unroll
      for (int l = 0; l < KR; ++l) acc += sl.r[l] * ps[l + c * kMaxRank];
      o[c * kMaxRank] = sl.i < sl.ku ? acc : T(0);
    }
  } else {
    T acc[DC];
#pragma unroll
    for (int c = 0; c < DC; ++c) acc[c] = sl.yc[c];
    for (int l = 0; l < sl.rn; ++l) {
      const T rv = sl.rp[(int64_t)l * sl.rs];
#pragma unroll
      for (int c = 0; c < DC; ++c) acc[c] += rv * ps[l + c * kMaxRank];
    }
#pragma unroll
    for (int c = 0; c < DC; ++c)
      if (c < nc) o[c * kMaxRank] = sl.i < sl.ku ? acc[c] : T(0);
  }
}

template <typename T, bool BATCH, int KR, int NR, int DC>
__global__ __launch_bounds__(kDT) void k_mmf_down(KArgs<T, CallMM<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  Inst<T> I; CallMM<T> C; int s;
  resolve<BATCH>(a, I, C, s);
  if (gated_off(C.gate)) return;
  const int c0 = blockIdx.y * DC;
  if (c0 >= C.nrhs) return;
  const int nc = min(DC, C.nrhs - c0);
  const int ncw = min(DC, C.nrhs);
  const int64_t blk = (int64_t)kMaxRank * ncw;
  T* cur = reinterpret_cast<T*>(smem_raw);   // two levels x 2^kDnH nodes x blk
  T* nxt = cur + (int64_t)(1 << kDnH) * blk;
  DownMap mp;
  mp.s = s;
  mp.p = I.p;
  mp.ls = I.nodes[s].level;
  // every slot's level: total count and the prefetched rounds
  int total = 0;
  for (int d = 2; d <= mp.p; ++d) total += mp.cnt(d) * KR;
  DownSlot<T, KR, DC> sl[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) down_slot_load(I, mp, threadIdx.x + r * kDT, c0, nc, sl[r]);
  // level 1: core values of its node(s)
  {
    const int n1c = mp.cnt(1);
    for (int o = threadIdx.x; o < n1c * kMaxRank * nc; o += kDT) {
      const int j = o / (kMaxRank * nc), rem = o % (kMaxRank * nc);
      const int i = rem % kMaxRank, c = rem / kMaxRank;
      const NodeInfo nn = I.nodes[mp.node(1, j)];
      cur[j * blk + i + c * kMaxRank] =
          i < nn.ku ? I.yh[nn.oyh + i + (int64_t)(c0 + c) * I.ldm] : T(0);
    }
  }
  __syncthreads();
  const int rounds = (total + kDT - 1) / kDT;
  for (int d = 2; d <= mp.p; ++d) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (sl[r].d == d) down_slot_apply(sl[r], nc, cur, nxt, blk);
    for (int r = NR; r < rounds; ++r) {   // slots beyond the prefetched rounds
      const int g = threadIdx.x + r * kDT;
      if (down_slot_level<KR>(mp, g) != d) continue;
      DownSlot<T, KR, DC> x;
      down_slot_load(I, mp, g, c0, nc, x);
      down_slot_apply(x, nc, cur, nxt, blk);
    }
    __syncthreads();
    T* q = cur; cur = nxt; nxt = q;
  }
  // y^ of the leaves of the subtree
  const int dl = mp.p > mp.ls ? mp.p : mp.ls;
  const int nl = mp.cnt(dl);
  for (int o = threadIdx.x; o < nl * kMaxRank * nc; o += kDT) {
    const int j = o / (kMaxRank * nc), rem = o % (kMaxRank * nc);
    const int i = rem % kMaxRank, c = rem / kMaxRank;
    const NodeInfo nn = I.nodes[mp.node(dl, j)];
    if (i < nn.ku) I.yh[nn.oyh + i + (int64_t)(c0 + c) * I.ldm] = cur[j * blk + i + c * kMaxRank];
  }
}

// Y_i = D_i X_i + U_i y^_i.  Wavefront w owns rows 16w .. 16w+15; lane l holds
// row 16w + (l & 15) of the columns 32q .. 32q+31 of D_i (q = l >> 4) and of
// the columns q, q+4, ... of U_i; the four quarters are combined by two lane
// exchanges.  MODE 1 computes only Y_i = D_i X_i (it needs nothing from the
// up and down kernels, so it can run beside them); MODE 2 then adds U_i y^_i
// to Y_i.
template <typename T, bool BATCH, int NU, int MC, int MODE>
__global__ __launch_bounds__(kLT) void k_mmf_leaf(KArgs<T, CallMM<T>> a) {
  constexpr bool WD = MODE != 2, WU = MODE != 1;
  HIP_DYNAMIC_SHARED(char, smem_raw)
  Inst<T> I; CallMM<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  if (gated_off(C.gate)) return;
  const int c0 = blockIdx.y * MC;
  if (c0 >= C.nrhs) return;
  const int nc = min(MC, C.nrhs - c0);
  const int ncw = min(MC, C.nrhs);
  T* xs = reinterpret_cast<T*>(smem_raw);   // kXP x ncw
  T* ys = xs + kXP * ncw;                   // kMaxRank x ncw
  const NodeInfo nd = I.nodes[node];
  const int m = nd.m, ku = I.p > 0 ? nd.ku : 0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int row = 16 * w + (lane & 15), q = lane >> 4;
  const bool rv = row < m;
  // every global load of the work-group is issued before the first use: D and
  // U into registers, X and y^ into registers and then LDS.  Out-of-range
  // rows and columns read a valid element and are zeroed afterwards.
  // buffer loads: the block base in a resource descriptor, one lane offset
  // register for all columns (the column offset is uniform), and reads past
  // the block (columns >= m, or >= ku) return zero
  const uint32_t rb = (uint32_t)(min(row, m - 1) * (int)sizeof(T));
  const auto Dr = buf_rsrc(I.D + nd.oD, (uint32_t)(m * m * (int)sizeof(T)));
  const auto Ur = buf_rsrc(ku > 0 ? I.U + nd.oU : I.D + nd.oD,
                           (uint32_t)(m * ku * (int)sizeof(T)));
  const uint32_t cs = (uint32_t)(m * (int)sizeof(T));   // column stride in bytes
  T dv[32];
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) {
    const T v = WD ? buf_load<T>(Dr, rb + (uint32_t)(32 * q) * cs, (uint32_t)jj * cs) : T(0);
    dv[jj] = rv ? v : T(0);
  }
  T uv[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    const T v = WU ? buf_load<T>(Ur, rb + (uint32_t)q * cs, (uint32_t)(4 * i) * cs) : T(0);
    uv[i] = rv ? v : T(0);
  }
  T yo[MC];   // MODE 2: the D X part already in Y
#pragma unroll
  for (int c = 0; c < MC; ++c) {
    const int cc = min(c, nc - 1);
    yo[c] = MODE == 2 ? C.Y[nd.row0 + min(row, m - 1) + (int64_t)(c0 + cc) * C.ldy] : T(0);
  }
  constexpr int UX = (kMaxBlock * MC + kLT - 1) / kLT, UY = (kMaxRank * MC + kLT - 1) / kLT;
  T xv[UX], yv[UY];
  const T* Xb = C.X + nd.row0 + (int64_t)c0 * C.ldx;
#pragma unroll
  for (int u = 0; u < UX; ++u) {
    const int o = tid + u * kLT, i = o % kMaxBlock, c = min(o / kMaxBlock, nc - 1);
    const T v = WD ? Xb[min(i, m - 1) + (int64_t)c * C.ldx] : T(0);
    xv[u] = (i < m) ? v : T(0);
  }
  const T* Yh = I.yh + nd.oyh + (int64_t)c0 * I.ldm;
#pragma unroll
  for (int u = 0; u < UY; ++u) {
    const int o = tid + u * kLT, i = o % kMaxRank, c = min(o / kMaxRank, nc - 1);
    const T v = (WU && ku > 0) ? Yh[min(i, ku - 1) + (int64_t)c * I.ldm] : T(0);
    yv[u] = (i < ku) ? v : T(0);
  }
#pragma unroll
  for (int u = 0; u < UX; ++u) {
    const int o = tid + u * kLT;
    if (WD && o < kMaxBlock * nc) xs[xrow(o % kMaxBlock) + (o / kMaxBlock) * kXP] = xv[u];
  }
#pragma unroll
  for (int u = 0; u < UY; ++u) {
    const int o = tid + u * kLT;
    if (WU && o < kMaxRank * nc) ys[o % kMaxRank + (o / kMaxRank) * kMaxRank] = yv[u];
  }
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    const T* xc = xs + c * kXP + xrow(32 * q);
    const T* yc = ys + c * kMaxRank + q;
    // the D X and U y^ parts are reduced separately and added last, in every
    // mode, so that the split and the one-pass forms round identically
    T sd = T(0), su = T(0);
    if (WD) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int jj = 0; jj < 32; jj += 2) {
        s0 += dv[jj] * xc[jj];
        s1 += dv[jj + 1] * xc[jj + 1];
      }
      sd = s0 + s1;
      sd += __shfl_xor(sd, 16, 64);
      sd += __shfl_xor(sd, 32, 64);
    }
    if (WU) {
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int i = 0; i < NU; i += 2) {
        s0 += uv[i] * yc[4 * i];
        s1 += uv[i + 1] * yc[4 * i + 4];
      }
      su = s0 + s1;
      su += __shfl_xor(su, 16, 64);
      su += __shfl_xor(su, 32, 64);
    }
    if (MODE == 2) {
      T yc0 = yo[0];
#pragma unroll
      for (int cc = 1; cc < MC; ++cc) yc0 = cc == c ? yo[cc] : yc0;
      sd = yc0;
    }
    if (q == 0 && rv) C.Y[nd.row0 + row + (int64_t)(c0 + c) * C.ldy] = MODE == 1 ? sd : sd + su;
  }
}

template <typename T>
void launch_mmf(MMFStep step, const KArgs<T, CallMM<T>>& a, int nblocks, int nrhs, int max_ku,
                int max_k, hipStream_t s) {
  if (nblocks <= 0 || nrhs <= 0) return;
  const bool batch = a.tasks != nullptr;
  // right-hand-side chunk of the leaf kernel: 1, 8 or 32 columns; of the up
  // kernel: 1 or 8
  const int mc = nrhs == 1 ? 1 : (nrhs <= 8 ? 8 : 32);
  const int ytiles = (nrhs + mc - 1) / mc;
  const int ncw = nrhs < mc ? nrhs : mc;
  const int mcu = nrhs == 1 ? 1 : 8;
  const int ncu = nrhs < mcu ? nrhs : mcu;
  const bool wide = max_k > 32;
  static const char* n64[] = {"mmf_up_f64", "mmf_down_f64", "mmf_leaf_f64", "mmf_leaf_dx_f64",
                              "mmf_leaf_uy_f64", "mmf_up_dx_f64"};
  static const char* n32[] = {"mmf_up_f32", "mmf_down_f32", "mmf_leaf_f32", "mmf_leaf_dx_f32",
                              "mmf_leaf_uy_f32", "mmf_up_dx_f32"};
  TimedLaunch tl((sizeof(T) == 8 ? n64 : n32)[(int)step], s);
#define HSS_MMF_UP(MC, KQ)                                                                   \
  if (batch) hipLaunchKernelGGL((k_mmf_up<T, true, MC, KQ>), dim3(nblocks), dim3(kUT), sm, s, a); \
  else hipLaunchKernelGGL((k_mmf_up<T, false, MC, KQ>), dim3(nblocks), dim3(kUT), sm, s, a);
#define HSS_MMF_LEAF(NU, MC)                                                                   \
  if (batch) hipLaunchKernelGGL((k_mmf_leaf<T, true, NU, MC, 0>), g, b, sm, s, a);               \
  else if (step == MMFStep::LeafDX) hipLaunchKernelGGL((k_mmf_leaf<T, false, NU, MC, 1>), g, b, sm, s, a); \
  else if (step == MMFStep::LeafUY) hipLaunchKernelGGL((k_mmf_leaf<T, false, NU, MC, 2>), g, b, sm, s, a); \
  else hipLaunchKernelGGL((k_mmf_leaf<T, false, NU, MC, 0>), g, b, sm, s, a);
  switch (step) {
    case MMFStep::Up: {
      const size_t sm = (size_t)(kMaxBlock + 2 * (1 << kUpH) * kMaxRank) * ncu * sizeof(T);
      if (mcu == 1 && !wide) {
        const size_t sm1 = (size_t)15 * 32 * sizeof(T);
        if (batch) hipLaunchKernelGGL((k_mmf_up1<T, true, false, 1>), dim3(nblocks), dim3(kUT), sm1, s, a);
        else hipLaunchKernelGGL((k_mmf_up1<T, false, false, 1>), dim3(nblocks), dim3(kUT), sm1, s, a);
      } else if (mcu == 1) {
        HSS_MMF_UP(1, 64)
      } else if (!wide && (!batch || nrhs <= kMbCols)) {
        // up to kMbChunks chunks of kMbCols columns per launch (grid.y), a
        // wider block in successive launches; batched: one chunk
        const size_t sm8 = (size_t)15 * 32 * kMbCols * sizeof(T);
        const int span = kMbCols * kMbChunks;
        for (int c0 = 0; c0 < nrhs; c0 += batch ? nrhs : span) {
          KArgs<T, CallMM<T>> b = a;
          int ny = 1;
          if (!batch) {
            b.call.X += (int64_t)c0 * a.call.ldx;
            b.call.nrhs = std::min(span, nrhs - c0);
            b.inst.yh += (int64_t)c0 * a.inst.ldm;
            ny = (b.call.nrhs + kMbCols - 1) / kMbCols;
          }
          if (batch) hipLaunchKernelGGL((k_mmf_up1<T, true, false, kMbCols>), dim3(nblocks), dim3(kUT), sm8, s, b);
          else hipLaunchKernelGGL((k_mmf_up1<T, false, false, kMbCols>), dim3(nblocks, ny), dim3(kUT), sm8, s, b);
        }
      }
      else { if (wide) { HSS_MMF_UP(8, 64) } else { HSS_MMF_UP(8, 32) } }
      break;
    }
    case MMFStep::Down: {
      // one right-hand side: every slot of a work-group prefetched (two rounds)
      const int dc = nrhs == 1 ? 1 : kDC;
      const size_t sm = (size_t)2 * (1 << kDnH) * kMaxRank * (nrhs < dc ? nrhs : dc) * sizeof(T);
      const dim3 g(nblocks, (nrhs + dc - 1) / dc), b(kDT);
      if (nrhs == 1 && !wide) {
        if (batch) hipLaunchKernelGGL((k_mmf_down<T, true, 32, 2, 1>), g, b, sm, s, a);
        else hipLaunchKernelGGL((k_mmf_down<T, false, 32, 2, 1>), g, b, sm, s, a);
      } else if (!wide) {
        if (batch) hipLaunchKernelGGL((k_mmf_down<T, true, 32, 1, kDC>), g, b, sm, s, a);
        else hipLaunchKernelGGL((k_mmf_down<T, false, 32, 1, kDC>), g, b, sm, s, a);
      } else {
        if (batch) hipLaunchKernelGGL((k_mmf_down<T, true, 64, 1, kDC>), g, b, sm, s, a);
        else hipLaunchKernelGGL((k_mmf_down<T, false, 64, 1, kDC>), g, b, sm, s, a);
      }
      break;
    }
    case MMFStep::UpDX: {
      // (single instance, one right-hand side, ranks <= 32 only): nblocks
      // subtree blocks, then one block per leaf
      if (batch || nrhs != 1 || wide) break;
      KArgs<T, CallMM<T>> b = a;
      b.ntasks = nblocks;
      const int nleaf = 1 << a.inst.p;
      const size_t sm1 = (size_t)std::max(15 * 32, kXP) * sizeof(T);
      hipLaunchKernelGGL((k_mmf_up1<T, false, true, 1>), dim3(nblocks + nleaf), dim3(kUT), sm1, s, b);
      break;
    }
    case MMFStep::Leaf:
    case MMFStep::LeafDX:
    case MMFStep::LeafUY: {
      const size_t sm = (size_t)(kXP + kMaxRank) * ncw * sizeof(T);
      const dim3 g(nblocks, ytiles), b(kLT);
      const bool wu = max_ku > 32;
      if (mc == 1) { if (wu) { HSS_MMF_LEAF(16, 1) } else { HSS_MMF_LEAF(8, 1) } }
      else if (mc == 8) { if (wu) { HSS_MMF_LEAF(16, 8) } else { HSS_MMF_LEAF(8, 8) } }
      else { if (wu) { HSS_MMF_LEAF(16, 32) } else { HSS_MMF_LEAF(8, 32) } }
      break;
    }
  }
#undef HSS_MMF_UP
#undef HSS_MMF_LEAF
#undef HSS_MMF
#undef HSS_MMF
}

int mmf_down_height() { return kDnH; }
int mmf_up_height() { return kUpH; }

template void launch_mmf<double>(MMFStep, const KArgs<double, CallMM<double>>&, int, int, int,
                                 int, hipStream_t);
template void launch_mmf<float>(MMFStep, const KArgs<float, CallMM<float>>&, int, int, int, int,
                                hipStream_t);

}  // namespace hss
