// Step 1 of the ULV factorization (Sec. 4.3) for blocks of up to 128 rows with
// ranks up to 32, blocked: the Householder vectors are formed 32 at a time
// (a panel) by one wavefront, and each panel is applied to the rest of the
// block at once in compact WY form on the matrix cores:
//   H_0 H_1 ... H_{b-1} = I - Y T Y^T,  T upper triangular with
//   T^{-1} = diag(1 / tau) + strictly-upper(Y^T Y)
// (the inverse of the usual column recurrence for T; T is obtained from it by
// back substitution, so a zero tau gives a zero row and column of T; the
// entries of Y^T Y come out of the panel steps themselves).
//   QL of U' (one panel: the ku columns), Q^T = H_0 ... H_{ku-1} applied as
//   M = Q^T D' = D' - Y (T (Y^T D'));
//   LQ of the leading e rows of M, panels of 32 rows; the rows below a panel
//   and V'^T are multiplied from the right by H_i0 ... H_i1-1, i.e. in
//   transposed form A^T <- A^T - Y (T^T (Y^T A^T)).
// The stored factors are exactly those of the register kernel
// (kernels_factor.hip): FU, tq, FD, FZ, tz, FV in the same formats.
//
// Work-group: four wavefronts, each holding a 128 x 32 slab of the working
// matrix as 16 accumulator tiles of the 16x16x4 MFMA: tile (rt, ct), lane
// l = 16 g + c, component r holds element (16 rt + rho(g, r), 16 ct + c) with
// rho = 4 g + r for the FP32 instruction and g + 4 r for the FP64 one.
//   QL phase: wavefront w holds columns 32 w .. 32 w + 31 of D', its rows
//   shifted down by 128 - mp, so that the pivot rows of U' are always the
//   last ku <= 32 rows (tiles 6 and 7).
//   LQ phase: wavefront q holds rows 32 q .. 32 q + 31 of M transposed
//   (element (column, row - 32 q)), so that panel q is wavefront q's slab and
//   the rows of a panel's pivots are tiles 2q and 2q + 1; after its panel,
//   wavefront 0 holds V' (element (row, column)) in the same way.
// A panel is factored by the one wavefront whose slab it is (U' is loaded as
// wavefront 0's slab first), with no work-group barrier between its steps;
// the other wavefronts load their slabs or apply the previous panel
// meanwhile.
// The QL-phase slabs reach the LQ layout through the node's FD block (written,
// one barrier, read back transposed), which the kernel overwrites with the
// final factor afterwards.
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {
namespace {

constexpr int kBP = 128;        // padded block size
constexpr int kBW = 32;         // panel width; the largest ku and kv taken
constexpr int kLY = kBP + 8;    // row pitch of the reflector store Yt (vector-major)
constexpr int kLT = kBW + 8;    // row pitch of G / T

template <typename T> struct V4T;
template <> struct V4T<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct V4T<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <typename T> using v4 = typename V4T<T>::type;

// D = A B + C for one 16x16x4 block: lane 16 g + c supplies A(c, g) and
// B(g, c); D(4 g + r, c) is component r of lane 16 g + c.
__device__ __forceinline__ v4<float> mfma4(float a, float b, v4<float> c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4<double> mfma4(double a, double b, v4<double> c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The four rows 16 t + rho(g, 0 .. 3) of a position-indexed LDS vector (base
// at position 16 t): contiguous for FP32, a stride of four for FP64.
template <typename T>
__device__ __forceinline__ v4<T> lds_rows4(const T* base, int g) {
  if constexpr (sizeof(T) == 4) {
    return *reinterpret_cast<const v4<T>*>(base + 4 * g);
  } else {
    v4<T> v;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = base[g + 4 * r];
    return v;
  }
}
template <typename T>
__device__ __forceinline__ void lds_put_rows4(T* base, int g, v4<T> v) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<v4<T>*>(base + 4 * g) = v;
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) base[g + 4 * r] = v[r];
  }
}

template <typename T>
__device__ __forceinline__ v4<T> v4zero() {
  v4<T> z;
  z[0] = z[1] = z[2] = z[3] = T(0);
  return z;
}

// A wavefront-uniform integer, kept in a scalar register: element masks are
// written as (lane quantity) < (uniform threshold) so that no per-element
// position register is needed.
__device__ __forceinline__ int su(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum over the four lanes l, l ^ 16, l ^ 32, l ^ 48 (the four g of one c),
// returned in all of them.  The row swaps exchange 16- and 32-lane halves in
// the VALU: swapping v with itself leaves the two halves' values in the two
// results, whose sum is the pairwise sum in every lane.
__device__ __forceinline__ float xsum_rows(float v) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ __forceinline__ double xsum_rows(double v) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  const auto al = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto ah = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  v = __longlong_as_double(((uint64_t)ah[0] << 32) | al[0]) +
      __longlong_as_double(((uint64_t)ah[1] << 32) | al[1]);
  const uint64_t w = __double_as_longlong(v);
  const uint32_t lo2 = (uint32_t)w, hi2 = (uint32_t)(w >> 32);
  const auto bl = __builtin_amdgcn_permlane32_swap(lo2, lo2, false, false);
  const auto bh = __builtin_amdgcn_permlane32_swap(hi2, hi2, false, false);
  return __longlong_as_double(((uint64_t)bh[0] << 32) | bl[0]) +
         __longlong_as_double(((uint64_t)bh[1] << 32) | bl[1]);
}

// Offsets of buffer accesses stay non-negative in the offset register: the
// hardware checks that register (with the immediate) against the size, so an
// offset that is negative there and positive only after the immediate is
// added would read zero.  Shifted accesses (s > 0) therefore clamp the row
// per element instead of folding the shift into the register.

// Slab element (R, C) = A[(R - s) + (c0 + C) * ld] for 0 <= R - s < rows and
// c0 + C < cols, else 0 (A holds ld * cols elements, ld >= rows).  Buffer
// reads: with no shift, one offset register per tile column plus immediate
// offsets; reads past the array return zero.
template <typename T>
__device__ __forceinline__ void slab_load_cols(v4<T> (&X)[8][2], const T* A, int ld, int rows,
                                               int cols, int s, int c0, int g, int c) {
  constexpr uint32_t sz = sizeof(T);
  const auto R = buf_rsrc(A, (uint32_t)(ld * cols) * sz);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int col = c0 + 16 * ct + c;
    const bool cok = col < cols;
    if (s == 0) {
      const uint32_t vo = cok ? (uint32_t)(mma_row<T>(g, 0) + col * ld) * sz : kBufOOB;
#pragma unroll
      for (int rt = 0; rt < 8; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          X[rt][ct][r] = buf_load<T>(R, vo + (16 * rt + mma_row<T>(0, r)) * sz, 0);
    } else {
#pragma unroll
      for (int rt = 0; rt < 8; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * rt + mma_row<T>(g, r) - s;
          const uint32_t o = cok & (row >= 0) ? (uint32_t)(row + col * ld) * sz : kBufOOB;
          X[rt][ct][r] = buf_load<T>(R, o, 0);
        }
    }
  }
}

// Transposed slab: element (R, C) = A[(r0 + C) + R * ld] for r0 + C < rows and
// R < cols, else 0 (A holds ld * cols elements).
template <typename T>
__device__ __forceinline__ void slab_load_rows(v4<T> (&X)[8][2], const T* A, int ld, int rows,
                                               int cols, int r0, int g, int c) {
  constexpr uint32_t sz = sizeof(T);
  const auto R = buf_rsrc(A, (uint32_t)(ld * cols) * sz);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int row = r0 + 16 * ct + c;
    const uint32_t vo = row < rows ? (uint32_t)(row + mma_row<T>(g, 0) * ld) * sz : kBufOOB;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t vr = vo + (uint32_t)(mma_row<T>(0, r) * ld) * sz;
#pragma unroll
      for (int rt = 0; rt < 8; ++rt)
        X[rt][ct][r] = buf_load<T>(R, vr, (uint32_t)(16 * rt * ld) * sz);
    }
  }
}

// Column slab back to A (same element map as slab_load_cols): elements with
// 0 <= R - s < rows and c0 + C < cols are written, the others dropped.
template <typename T>
__device__ __forceinline__ void slab_store_cols(const v4<T> (&X)[8][2], T* A, int ld, int rows,
                                                int cols, int s, int c0, int g, int c) {
  constexpr uint32_t sz = sizeof(T);
  const auto R = buf_rsrc(A, (uint32_t)(ld * cols) * sz);
  // (a full block needs no per-element mask: the offsets stay immediates)
  const bool full = (s == 0) & (rows >= kBP);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int col = c0 + 16 * ct + c;
    const bool cok = col < cols;
    if (full) {
      const uint32_t vo = cok ? (uint32_t)(mma_row<T>(g, 0) + col * ld) * sz : kBufOOB;
#pragma unroll
      for (int rt = 0; rt < 8; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          buf_store<T>(X[rt][ct][r], R, vo + (16 * rt + mma_row<T>(0, r)) * sz, 0);
    } else {
#pragma unroll
      for (int rt = 0; rt < 8; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * rt + mma_row<T>(g, r) - s;
          const bool in = cok & (row >= 0) & (row < rows);
          buf_store<T>(X[rt][ct][r], R, in ? (uint32_t)(row + col * ld) * sz : kBufOOB, 0);
        }
    }
  }
}

// A panel is one wavefront's slab: vector 16 ct + c of the panel is column
// 16 ct + c of the slab, its position R the slab row.  The position of lane
// (g, c), tile rt, component r is 16 rt + rho(g, r) = tile_pos(rt, r) +
// lane_pos(g).
template <typename T>
__device__ __forceinline__ int lane_pos(int g) {
  return sizeof(T) == 4 ? 4 * g : g;
}
template <typename T>
__device__ __forceinline__ constexpr int tile_pos(int rt, int r) {
  return 16 * rt + (sizeof(T) == 4 ? r : 4 * r);
}

__device__ __forceinline__ float lane_fetch(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_fetch(int addr, double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Per-panel scalars in LDS: the scale of every reflector's off-pivot part,
// beta and tau, indexed by vector.
template <typename T>
struct PanelScal {
  T* scale;
  T* bet;
  T* taus;
};

// One Householder step of a panel held by one wavefront (no work-group
// barrier).
//   QL: vector jv is column jv of U', pivot position pp, support positions
//       below pp; the vectors still to update are those before jv.
//   LQ: vector jv is row i0 + jv of M, pivot position pp = i0 + jv, support
//       positions above pp; the vectors still to update are those after jv.
// x, the pivot vector on its support (zero elsewhere), reaches every lane
// from the lane of the same g that holds vector jv (CT = jv / 16).  With
// v = scale x + e_pp the reflector, v . y = scale (x . y) + y(pp) for every
// vector y, so every lane forms x . y and y(pp) for its two vectors at its
// positions, the four lanes of a column (g = 0..3) add them up, and ||x||^2
// and alpha = x(pp) are the pivot vector's own sums.  The update is
// y <- y - tau (v . y) v; the pivot vector keeps x (unscaled) and alpha, and
// its scale, beta and tau go to the LDS scalars, from which the caller
// composes the finished vector.  RTB = pp / 16 is the tile of the pivot:
// tiles wholly outside the support are skipped, those wholly inside need no
// mask (both known at compile time).
template <typename T, bool QL, int CT, int RTB>
__device__ __forceinline__ void wave_step(v4<T> (&X)[8][2], int jv, int pp,
                                          const PanelScal<T>& S, T* Gs, T (&msc)[2], int g,
                                          int c, int lane, int* sing) {
  const int cj = su(jv & 15);
  const int src = (16 * g + cj) * 4;
  const int lp = lane_pos<T>(g);
  T xm[8][4];
  T d0[2] = {T(0), T(0)}, d1[2] = {T(0), T(0)};
  T y0 = T(0), y1 = T(0);
#pragma unroll
  for (int rt = 0; rt < 8; ++rt) {
    if (QL ? rt < RTB : rt > RTB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T x = lane_fetch(src, X[rt][CT][r]);
        xm[rt][r] = x;
        d0[r & 1] += x * X[rt][0][r];
        d1[r & 1] += x * X[rt][1][r];
      }
    } else if (rt == RTB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int th = su(pp - tile_pos<T>(rt, r));   // position - pp = lp - th
        const T xr = lane_fetch(src, X[rt][CT][r]);
        const bool in = QL ? lp < th : lp > th;
        const bool at = lp == th;
        const T x = in ? xr : T(0);
        xm[rt][r] = x;
        d0[r & 1] += x * X[rt][0][r];
        d1[r & 1] += x * X[rt][1][r];
        y0 += at ? X[rt][0][r] : T(0);
        y1 += at ? X[rt][1][r] : T(0);
      }
    }
  }
  const T dot0 = xsum_rows(d0[0] + d0[1]);
  const T dot1 = xsum_rows(d1[0] + d1[1]);
  y0 = xsum_rows(y0);
  y1 = xsum_rows(y1);
  const T sigma = lane_read(CT ? dot1 : dot0, cj);
  const T alpha = lane_read(CT ? y1 : y0, cj);
  T beta, tau, scale;
  householder_fast(alpha, sigma, beta, tau, scale);
  // h = v . y for both vectors: the update of the vectors still to come, and
  // for the finished ones (which keep their unscaled x) the Gram entry
  // Y_k^T Y_jv = scale_k h_k of the compact-WY factor
  const T h0 = scale * dot0 + y0, h1 = scale * dot1 + y1;
  const T w0 = (QL ? c < jv : c > jv) ? tau * h0 : T(0);
  const T w1 = (QL ? 16 + c < jv : 16 + c > jv) ? tau * h1 : T(0);
  const T s0 = w0 * scale, s1 = w1 * scale;
  if (g == 0) {
    const T gv0 = (QL ? c > jv : c < jv) ? msc[0] * h0 : T(0);
    const T gv1 = (QL ? 16 + c > jv : 16 + c < jv) ? msc[1] * h1 : T(0);
    if (QL) {
      Gs[jv * kLT + c] = gv0;
      Gs[jv * kLT + 16 + c] = gv1;
    } else {
      Gs[c * kLT + jv] = gv0;
      Gs[(16 + c) * kLT + jv] = gv1;
    }
  }
  if (c == cj) msc[CT] = scale;
#pragma unroll
  for (int rt = 0; rt < 8; ++rt) {
    if (QL ? rt < RTB : rt > RTB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        X[rt][0][r] -= s0 * xm[rt][r];
        X[rt][1][r] -= s1 * xm[rt][r];
      }
    } else if (rt == RTB) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int th = su(pp - tile_pos<T>(rt, r));
        const bool at = lp == th;
        X[rt][0][r] -= at ? w0 : s0 * xm[rt][r];
        X[rt][1][r] -= at ? w1 : s1 * xm[rt][r];
      }
    }
  }
  if (lane == 0) {
    S.scale[jv] = scale;
    S.bet[jv] = beta;
    S.taus[jv] = tau;
    if (!QL && beta == T(0)) *sing = 1;
  }
}

// Zero the scalars and the Gram block before a panel: the compact-WY T reads
// tau and G of all kBW vectors, and those past the panel's reflectors must be
// zero.
template <typename T>
__device__ __forceinline__ void panel_clear(const PanelScal<T>& S, T* Gs, T (&msc)[2], int lane) {
  if (lane < kBW) {
    S.scale[lane] = T(0);
    S.bet[lane] = T(0);
    S.taus[lane] = T(0);
  }
  for (int o = lane; o < kBW * kLT; o += 64) Gs[o] = T(0);
  msc[0] = msc[1] = T(0);
  wave_lds_sync();
}

// The QL panel (columns of U' shifted so that the pivots are the last ku
// positions, ku <= 32), columns jq = ku - 1 down to 0: the pivot of column jq
// lies in tile 7 when jq >= ku - 16, else in tile 6.
template <typename T>
__device__ __forceinline__ void ql_panel(v4<T> (&X)[8][2], int ku, const PanelScal<T>& S, T* Gs,
                                         T (&msc)[2], int g, int c, int lane, int* sing) {
  const int a = max(16, ku - 16), b = max(ku - 16, 0);
  for (int jq = ku - 1; jq >= a; --jq)
    wave_step<T, true, 1, 7>(X, jq, kBP - ku + jq, S, Gs, msc, g, c, lane, sing);
  for (int jq = min(ku, 16) - 1; jq >= b; --jq)
    wave_step<T, true, 0, 7>(X, jq, kBP - ku + jq, S, Gs, msc, g, c, lane, sing);
  for (int jq = min(b, 16) - 1; jq >= 0; --jq)
    wave_step<T, true, 0, 6>(X, jq, kBP - ku + jq, S, Gs, msc, g, c, lane, sing);
}

// LQ panel P (rows 32 P + j of M, pivot position 32 P + j): the pivot lies in
// tile 2 P + j / 16.
template <typename T, int P>
__device__ __forceinline__ void lq_panel(v4<T> (&X)[8][2], int cnt, const PanelScal<T>& S, T* Gs,
                                         T (&msc)[2], int g, int c, int lane, int* sing) {
  const int c0 = min(cnt, 16);
  for (int j = 0; j < c0; ++j)
    wave_step<T, false, 0, 2 * P>(X, j, 32 * P + j, S, Gs, msc, g, c, lane, sing);
  for (int j = 16; j < cnt; ++j)
    wave_step<T, false, 1, 2 * P + 1>(X, j, 32 * P + j, S, Gs, msc, g, c, lane, sing);
}

// After the panel: this lane's vector v (tile column ct) with pivot position
// pp_v (refl: v holds a reflector).  Per element, dpos = position - pp_v.
// Y (for the compact-WY update): scale x on the support, 1 at the pivot,
// 0 elsewhere, vector-major in Yt.
template <typename T, bool QL>
__device__ __forceinline__ void panel_to_yt(const v4<T> (&X)[8][2], const PanelScal<T>& S, T* Yt,
                                            int pp0, int nref, int g, int c) {
  const int lp = lane_pos<T>(g);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int v = 16 * ct + c;
    const bool refl = v < nref;
    const T sc = S.scale[v];
    const int d0 = lp - (pp0 + v);   // position - pp_v = tile_pos + d0
#pragma unroll
    for (int rt = 0; rt < 8; ++rt) {
      v4<T> y;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int d = d0 + tile_pos<T>(rt, r);
        const bool in = QL ? d < 0 : d > 0;
        y[r] = !refl ? T(0) : (in ? X[rt][ct][r] * sc : (d == 0 ? T(1) : T(0)));
      }
      lds_put_rows4(Yt + v * kLY + 16 * rt, g, y);
    }
  }
}

// T of the panel into Ts (TRANS: T^T) from its Gram block Gs (G(i, m) =
// Y_i^T Y_m for i < m, gathered during the steps) and taus, by one wavefront,
// lane j < 32 computing column j: T(i, j) = tau_i (delta_ij - sum_{m > i}
// G(i, m) T(m, j)), i from the bottom up.
template <typename T, bool TRANS>
__device__ __forceinline__ void make_t(const T* Gs, T* Ts, const T* taus, int lane) {
  // right-looking: once T(m, j) is known its multiples leave every row above
  // (a dependency chain of kBW steps rather than of kBW^2 / 2 products)
  const int j = lane & 31;
  T t[kBW];
#pragma unroll
  for (int i = 0; i < kBW; ++i) t[i] = i == j ? T(1) : T(0);
#pragma unroll
  for (int m = kBW - 1; m >= 0; --m) {
    t[m] *= taus[m];
#pragma unroll
    for (int i = 0; i < m; ++i) t[i] -= Gs[i * kLT + m] * t[m];
  }
  if (lane < kBW) {
#pragma unroll
    for (int i = 0; i < kBW; ++i) {
      if (TRANS) Ts[j * kLT + i] = t[i];
      else Ts[i * kLT + j] = t[i];
    }
  }
}

// X <- X - Y (Tm (Y^T X)) on this wavefront's slab (Y in Yt, Tm in Ts);
// positions below 16 RLO are zero in Y and skipped.
template <typename T, int RLO>
__device__ __forceinline__ void block_update(v4<T> (&X)[8][2], const T* Yt, const T* Ts, int g, int c) {
  v4<T> P[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) P[a][b] = v4zero<T>();
#pragma unroll
  for (int rt = RLO; rt < 8; ++rt) {
    const v4<T> y0 = lds_rows4(Yt + c * kLY + 16 * rt, g);
    const v4<T> y1 = lds_rows4(Yt + (16 + c) * kLY + 16 * rt, g);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        P[0][ct] = mfma4(y0[r], X[rt][ct][r], P[0][ct]);
        P[1][ct] = mfma4(y1[r], X[rt][ct][r], P[1][ct]);
      }
    }
  }
  v4<T> Q[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) Q[a][b] = v4zero<T>();
#pragma unroll
  for (int pt = 0; pt < 2; ++pt) {
    const v4<T> t0 = lds_rows4(Ts + c * kLT + 16 * pt, g);
    const v4<T> t1 = lds_rows4(Ts + (16 + c) * kLT + 16 * pt, g);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        Q[0][ct] = mfma4(t0[r], P[pt][ct][r], Q[0][ct]);
        Q[1][ct] = mfma4(t1[r], P[pt][ct][r], Q[1][ct]);
      }
    }
  }
#pragma unroll
  for (int qt = 0; qt < 2; ++qt) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const T* yk = Yt + (16 * qt + mma_row<T>(g, r)) * kLY + c;
#pragma unroll
      for (int rt = RLO; rt < 8; ++rt) {
        const T a = -yk[16 * rt];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) X[rt][ct] = mfma4(a, Q[qt][ct][r], X[rt][ct]);
      }
    }
  }
}

// Rows [lo, hi) of the transposed slab (rows 32 q + C of the block) to FD:
// FD[row + col * mp] = X(col, row - 32 q) for col < mp.
template <typename T>
__device__ __forceinline__ void store_rows(const v4<T> (&X)[8][2], T* FD, int mp, int q, int lo,
                                           int hi, int g, int c) {
  constexpr uint32_t sz = sizeof(T);
  const auto R = buf_rsrc(FD, (uint32_t)(mp * mp) * sz);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int row = 32 * q + 16 * ct + c;
    const uint32_t vo =
        (row >= lo) & (row < hi) ? (uint32_t)(row + mma_row<T>(g, 0) * mp) * sz : kBufOOB;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t vr = vo + (uint32_t)(mma_row<T>(0, r) * mp) * sz;
#pragma unroll
      for (int rt = 0; rt < 8; ++rt)
        buf_store<T>(X[rt][ct][r], R, vr, (uint32_t)(16 * rt * mp) * sz);
    }
  }
}

// QL-phase slabs to LQ-phase slabs through LDS (blocks of exactly 128 rows):
// wavefront Q holds columns 32 Q .. 32 Q + 31 of M (rows in position order)
// and needs rows 32 Q .. 32 Q + 31 (columns in position order).  Four rounds
// over the 32 x 32 blocks, one barrier pair each: in round r wavefront Q
// writes its block of rows 32 (Q ^ r) to its own LDS region (pitch 33) and
// reads back, transposed, the block wavefront Q ^ r wrote for it, into the
// tiles it has just written out.
constexpr int kTP = 33, kTBlk = 32 * 33;

template <typename T, int Q, int R>
__device__ __forceinline__ void tr_round(v4<T> (&X)[8][2], T* buf, int g, int c) {
  constexpr int S = Q ^ R;
  T* dst = buf + Q * kTBlk;
#pragma unroll
  for (int rl = 0; rl < 2; ++rl)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        dst[(16 * ct + c) * kTP + 16 * rl + mma_row<T>(g, r)] = X[2 * S + rl][ct][r];
  __syncthreads();
  const T* src = buf + S * kTBlk;
#pragma unroll
  for (int rl = 0; rl < 2; ++rl)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        X[2 * S + rl][ct][r] = src[(16 * rl + mma_row<T>(g, r)) * kTP + 16 * ct + c];
  __syncthreads();
}

template <typename T, int Q>
__device__ __forceinline__ void transpose_slabs(v4<T> (&X)[8][2], T* buf, int g, int c) {
  tr_round<T, Q, 0>(X, buf, g, c);
  tr_round<T, Q, 1>(X, buf, g, c);
  tr_round<T, Q, 2>(X, buf, g, c);
  tr_round<T, Q, 3>(X, buf, g, c);
}

// U~ and the QL reflectors from the panel wavefront's slab (vector v = column
// v of U', position = row + s): the reflector above the pivot, beta on it,
// U~ below, to FU.
template <typename T>
__device__ __forceinline__ void ql_panel_out(const v4<T> (&X)[8][2], const PanelScal<T>& S, T* FU,
                                             int mp, int ku, int s, int g, int c) {
  constexpr uint32_t sz = sizeof(T);
  const auto RU = buf_rsrc(FU, (uint32_t)(mp * ku) * sz);
  const int lp = lane_pos<T>(g);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int v = 16 * ct + c;
    const bool refl = v < ku;
    const T sc = S.scale[v], b = S.bet[v];
    const int d0 = lp - (kBP - ku + v);   // position - pp_v = tile_pos + d0
#pragma unroll
    for (int rt = 0; rt < 8; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tp = tile_pos<T>(rt, r);
        const int d = d0 + tp;
        const T x = X[rt][ct][r];
        const T val = d < 0 ? x * sc : (d == 0 ? b : x);
        const int row = tp + lp - s;
        const bool in = refl & (row >= 0);
        buf_store<T>(val, RU, in ? (uint32_t)(row + v * mp) * sz : kBufOOB, 0);
      }
  }
}

// Outputs of LQ panel P from wavefront P's slab (positions = columns of M,
// vector v = row 32 P + v; scv / bv: scale and beta of this lane's vectors
// c and 16 + c): rows 32 P + v, v < cnt, of FD (L left of the
// diagonal, beta on it, the reflector to the right) and columns 32 P + v of
// FZ (the reflector with its unit and zeros above); when the panel holds rows
// >= e (the last panel), those rows of FD as they are.
template <typename T>
__device__ __forceinline__ void lq_panel_out(const v4<T> (&X)[8][2], const T (&scv)[2],
                                             const T (&bv)[2], T* FD, T* FZ, int mp, int e, int P,
                                             int cnt, bool last, int g, int c) {
  constexpr uint32_t sz = sizeof(T);
  const auto RD = buf_rsrc(FD, (uint32_t)(mp * mp) * sz);
  const auto RZ = buf_rsrc(FZ, (uint32_t)(mp * e) * sz);
  const int lp = lane_pos<T>(g);
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int v = 16 * ct + c, row = 32 * P + v;
    const bool refl = v < cnt;
    const bool wr = (row < mp) & (refl | last);
    const T sc = scv[ct], b = bv[ct];
    const int d0 = lp - row;   // position - pp_v = tile_pos + d0
    const uint32_t vd = wr ? (uint32_t)(row + lp * mp) * sz : kBufOOB;
    const uint32_t vz = refl ? (uint32_t)(lp + row * mp) * sz : kBufOOB;
#pragma unroll
    for (int rt = 0; rt < 8; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tp = tile_pos<T>(rt, r);
        const int d = d0 + tp;
        const T x = X[rt][ct][r];
        const T dv = refl ? (d < 0 ? x : (d == 0 ? b : x * sc)) : x;
        const T zv = d > 0 ? x * sc : (d == 0 ? T(1) : T(0));
        buf_store<T>(dv, RD, vd, (uint32_t)(tp * mp) * sz);
        const bool pin = lp < mp - tp;
        buf_store<T>(zv, RZ, pin ? vz : kBufOOB, (uint32_t)tp * sz);
      }
  }
}

// FP32: four waves per SIMD (128 registers); FP64: two (its accumulator
// tiles take twice the space).
template <typename T, bool BATCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) void k_ulv_factor_blk(
    KArgs<T, CallSV<T>> a) {
  __shared__ __attribute__((aligned(16))) T Yt[kBW * kLY];
  __shared__ __attribute__((aligned(16))) T Ts[kBW * kLT];
  __shared__ __attribute__((aligned(16))) T Gs[kBW * kLT];
  __shared__ T scal[3 * kBW];
  __shared__ int sing;
  static_assert(kBW * kLY >= 4 * kTBlk, "the transposition blocks fit in Yt");
  const PanelScal<T> S{scal, scal + kBW, scal + 2 * kBW};
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int mp = nd.mp, ku = nd.ku, kv = nd.kv, e = nd.e;
  const int tid = threadIdx.x, lane = tid & 63;
  // the roles of the four wavefronts rotate with the work-group, so that the
  // panel wavefronts of the work-groups sharing a compute unit are spread
  // over its SIMDs
  const int w = __builtin_amdgcn_readfirstlane(((tid >> 6) + (int)blockIdx.x) & 3);
  const int g = lane >> 4, c = lane & 15;
  const int s = kBP - mp;
  T* FU = I.FU + nd.oFU;
  T* FV = I.FV + nd.oFV;
  T* FD = I.FD + nd.oFD;
  T* FZ = I.FZ + nd.oFZ;
  const T* Dsrc = nd.is_leaf ? I.D + nd.oD : FD;
  const T* Usrc = nd.is_leaf ? I.U + nd.oU : FU;
  const T* Vsrc = nd.is_leaf ? I.V + nd.oV : FV;
  if (e == 0) {
    // nothing to eliminate: Q = Z = I, the generators pass through
    if (nd.is_leaf) {
      for (int o = tid; o < mp * ku; o += 256) FU[o] = Usrc[o];
      for (int o = tid; o < mp * kv; o += 256) FV[o] = Vsrc[o];
      for (int o = tid; o < mp * mp; o += 256) FD[o] = Dsrc[o];
    }
    return;
  }
  v4<T> X[8][2];
  // ---- QL of U' (one panel, wavefront 0) and M = Q^T D'
  if (ku > 0) {
    if (w == 0) {
      slab_load_cols(X, Usrc, mp, mp, ku, s, 0, g, c);
      T msc[2];
      panel_clear(S, Gs, msc, lane);
      ql_panel(X, ku, S, Gs, msc, g, c, lane, &sing);
      wave_lds_sync();
      panel_to_yt<T, true>(X, S, Yt, kBP - ku, ku, g, c);
      ql_panel_out(X, S, FU, mp, ku, s, g, c);
      if (lane < ku) I.tq[nd.otq + lane] = S.taus[lane];
      slab_load_cols(X, Dsrc, mp, mp, mp, s, 0, g, c);
      make_t<T, false>(Gs, Ts, S.taus, lane);
    } else {
      slab_load_cols(X, Dsrc, mp, mp, mp, s, 32 * w, g, c);
    }
    __syncthreads();
    block_update<T, 0>(X, Yt, Ts, g, c);
    if (sizeof(T) == 4 && s == 0) {
      // FP32 blocks of 128 rows: M from column slabs to row slabs through
      // LDS (Yt is free again once every slab's update has read it)
      __syncthreads();
      switch (w) {
        case 0: transpose_slabs<T, 0>(X, Yt, g, c); break;
        case 1: transpose_slabs<T, 1>(X, Yt, g, c); break;
        case 2: transpose_slabs<T, 2>(X, Yt, g, c); break;
        default: transpose_slabs<T, 3>(X, Yt, g, c); break;
      }
    } else {
      // shifted positions: M to FD (column slabs), then back as row slabs
      slab_store_cols(X, FD, mp, mp, mp, s, 32 * w, g, c);
      __syncthreads();
      slab_load_rows(X, FD, mp, mp, mp, 32 * w, g, c);
    }
  } else {
    slab_load_rows(X, Dsrc, mp, mp, mp, 32 * w, g, c);
  }
  // ---- LQ of rows 0 .. e-1 of M, panels of 32 rows: panel P is wavefront
  // P's slab, factored by that wavefront and applied to the slabs below it
  // and to V' (wavefront 0 after panel 0).  Wavefront P + 1 starts its panel
  // as soon as its own slab has the update with panel P, while the others
  // are still applying it.
  const int plast = (e - 1) >> 5;
#define HSS_LQ_PANEL(P)                                                                     \
  if (P <= plast) {                                                                         \
    const int cnt = min(kBW, e - 32 * P);                                                   \
    if (w == P) {                                                                           \
      T msc[2];                                                                             \
      if (P == 0 && lane == 0) sing = 0;                                                    \
      panel_clear(S, Gs, msc, lane);                                                        \
      lq_panel<T, P>(X, cnt, S, Gs, msc, g, c, lane, &sing);                                \
    }                                                                                       \
    __syncthreads();   /* the updates with the previous panel have read Yt and Ts */        \
    /* the scalars the outputs need, read before the next panel may reuse them */          \
    T scv[2], bv[2], tzv = T(0);                                                            \
    if (w == ((P + 3) & 3)) make_t<T, true>(Gs, Ts, S.taus, lane);                          \
    if (w == P) {                                                                           \
      panel_to_yt<T, false>(X, S, Yt, 32 * P, cnt, g, c);                                   \
      scv[0] = S.scale[c];                                                                  \
      scv[1] = S.scale[16 + c];                                                             \
      bv[0] = S.bet[c];                                                                     \
      bv[1] = S.bet[16 + c];                                                                \
      tzv = S.taus[lane & 31];                                                              \
    }                                                                                       \
    __syncthreads();                                                                        \
    if (w == P) {   /* outputs while the others apply the panel */                          \
      lq_panel_out(X, scv, bv, FD, FZ, mp, e, P, cnt, P == plast, g, c);                    \
      if (lane < cnt) I.tz[nd.otz + 32 * P + lane] = tzv;                                   \
      if (P == 0 && kv > 0) slab_load_cols(X, Vsrc, mp, mp, kv, 0, 0, g, c);                \
    }                                                                                       \
    if (w > P || (w == 0 && kv > 0)) block_update<T, 2 * P>(X, Yt, Ts, g, c);               \
  }
  HSS_LQ_PANEL(0)
  HSS_LQ_PANEL(1)
  HSS_LQ_PANEL(2)
  HSS_LQ_PANEL(3)
#undef HSS_LQ_PANEL
  if (w > plast) store_rows(X, FD, mp, w, e, mp, g, c);
  if (w == 0 && kv > 0) slab_store_cols(X, FV, mp, mp, kv, 0, 0, g, c);
  if (tid == 0 && sing) {
    atomicOr(I.status, 1 << kCodeSingular);
    atomicMax(I.status + kStSingularNode, node + 1);
  }
}

}  // namespace

template <typename T>
bool factor_blk_fits(int max_mp, int max_k) {
  return max_mp > 64 && max_mp <= kBP && max_k <= kBW;
}

template <typename T>
void launch_factor_blk(const KArgs<T, CallSV<T>>& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return;
  if (a.tasks != nullptr)
    hipLaunchKernelGGL((k_ulv_factor_blk<T, true>), dim3(nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_ulv_factor_blk<T, false>), dim3(nblocks), dim3(256), 0, s, a);
}

template bool factor_blk_fits<float>(int, int);
template bool factor_blk_fits<double>(int, int);
template void launch_factor_blk<float>(const KArgs<float, CallSV<float>>&, int, hipStream_t);
template void launch_factor_blk<double>(const KArgs<double, CallSV<double>>&, int, hipStream_t);

}  // namespace hss
