// Step 1 of the ULV factorization (Sec. 4.3) for blocks of up to 128 rows with
// ranks up to 32, blocked: the Householder vectors are formed 32 at a time
// (a panel) by one wavefront, and each panel is applied to the rest of the
// block at once in compact WY form on the matrix cores:
//   H_0 H_1 ... H_{b-1} = I - Y T Y^T,  T upper triangular with
//   T^{-1} = diag(1 / tau) + strictly-upper(Y^T Y)
// (the inverse of the usual column recurrence for T; T is obtained from it by
// back substitution, so a zero tau gives a zero row and column of T).
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

// A panel of 32 vectors spread over the four wavefronts by position:
// wavefront w holds positions 32 w .. 32 w + 31 of every vector as tiles
// (rl, ct); lane (g, c), component r holds vector 16 ct + c at position
// 32 w + 16 rl + 4 g + r.
template <typename T>
struct Panel {
  v4<T> t[2][2];
};

// LDS of the panel steps.
template <typename T>
struct PanelLds {
  T* red;     // partial squared norms: [parity][wavefront] (2 x 4)
  T* dred;    // partial sums of vector v: [parity][v][wavefront][raw dot, value at pp] (2 x kBW x 8)
  T* Yt;      // reflectors, vector-major (kBW x kLY)
  T* bet;
  T* taus;
};

// Panel element (vector C, position R) = A[(R - s) + C * ld] for C < cols and
// R >= s, else 0.
template <typename T>
__device__ __forceinline__ void panel_load_cols(Panel<T>& Pn, const T* A, int ld, int cols, int s,
                                                int w, int g, int c) {
  constexpr uint32_t sz = sizeof(T);
  const auto R = buf_rsrc(A, (uint32_t)(ld * cols) * sz);
  const int base = 32 * w;
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int vec = 16 * ct + c;
    const bool vok = vec < cols;
#pragma unroll
    for (int rl = 0; rl < 2; ++rl)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = base + 16 * rl + 4 * g + r - s;
        const uint32_t o = vok & (row >= 0) ? (uint32_t)(row + vec * ld) * sz : kBufOOB;
        Pn.t[rl][ct][r] = buf_load<T>(R, o, 0);
      }
  }
}

// This wavefront's positions of a panel stored vector-major in LDS (pitch kLY).
template <typename T>
__device__ __forceinline__ void panel_load_lds(Panel<T>& Pn, const T* Pb, int w, int g, int c) {
#pragma unroll
  for (int ct = 0; ct < 2; ++ct)
#pragma unroll
    for (int rl = 0; rl < 2; ++rl)
      Pn.t[rl][ct] =
          *reinterpret_cast<const v4<T>*>(Pb + (16 * ct + c) * kLY + 32 * w + 16 * rl + 4 * g);
}

// Zero this wavefront's positions of every reflector (and, wavefront 0, the
// scalars) before a panel.
template <typename T>
__device__ __forceinline__ void panel_clear(const PanelLds<T>& L, int w, int lane) {
  const int q = lane & 7, row0 = lane >> 3;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    *reinterpret_cast<v4<T>*>(L.Yt + (row0 + 8 * u) * kLY + 32 * w + 4 * q) = v4zero<T>();
  if (w == 0 && lane < kBW) {
    L.bet[lane] = T(0);
    L.taus[lane] = T(0);
  }
  wave_lds_sync();
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

// One Householder step of a panel (all four wavefronts, one barrier).
//   QL: vector jv is column jv of U', pivot position pp, support positions
//       <= pp; the vectors still to update are those before jv.
//   LQ: vector jv is row i0 + jv of M, pivot position pp = i0 + jv, support
//       positions >= pp; the vectors still to update are those after jv.
// With x the pivot vector off the pivot position (zero outside the support)
// and v = scale x + e_pp the reflector, v . y = scale (x . y) + y(pp) for
// every vector y, so each wavefront reduces ||x||^2 and, per vector, x . y
// and y(pp) over its positions before the scale is known: one exchange
// (double-buffered by step parity) per step.  The reflector goes to row jv
// of Yt, beta and tau to bet / taus; the pivot vector itself is left as it
// was (the caller composes its final form).
// MODE: 0 this wavefront's positions are all outside the support, 1 all
// inside it, 2 the pivot or an end of the support may lie among them.
template <typename T, bool QL, int MODE>
__device__ __forceinline__ void step_sums(const Panel<T>& Pn, const v4<T> (&xp)[2], int pp, int base,
                                          int g, T (&acc)[5]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) acc[q] = T(0);
  if (MODE == 0) return;
#pragma unroll
  for (int rl = 0; rl < 2; ++rl)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      T y = xp[rl][r];
      if (MODE == 2) {
        const int th = su(pp - base - 16 * rl - r);   // position - pp = 4 g - th
        const bool in = QL ? 4 * g < th : 4 * g > th;
        const bool at = 4 * g == th;
        y = in ? y : T(0);
        acc[3] += at ? Pn.t[rl][0][r] : T(0);
        acc[4] += at ? Pn.t[rl][1][r] : T(0);
      }
      acc[0] += y * y;
      acc[1] += y * Pn.t[rl][0][r];
      acc[2] += y * Pn.t[rl][1][r];
    }
}

template <typename T, bool QL>
__device__ __forceinline__ void panel_step(Panel<T>& Pn, int jv, int pp, const PanelLds<T>& L,
                                           int w, int lane, int g, int c) {
  const int ctj = jv >> 4, cj = jv & 15;
  const int base = 32 * w;
  const int par = jv & 1;
  // the pivot vector at this lane's positions, from lane (g, cj)
  const int src = (16 * g + cj) * 4;
  v4<T> xp[2];
  if (ctj) {
#pragma unroll
    for (int rl = 0; rl < 2; ++rl)
#pragma unroll
      for (int r = 0; r < 4; ++r) xp[rl][r] = lane_fetch(src, Pn.t[rl][1][r]);
  } else {
#pragma unroll
    for (int rl = 0; rl < 2; ++rl)
#pragma unroll
      for (int r = 0; r < 4; ++r) xp[rl][r] = lane_fetch(src, Pn.t[rl][0][r]);
  }
  // where this wavefront's positions lie relative to the support
  const bool inside = QL ? base + 31 < pp : base > pp;
  const bool outside = QL ? base > pp : base + 31 < pp;
  T acc[5];
  if (inside) step_sums<T, QL, 1>(Pn, xp, pp, base, g, acc);
  else if (outside) step_sums<T, QL, 0>(Pn, xp, pp, base, g, acc);
  else step_sums<T, QL, 2>(Pn, xp, pp, base, g, acc);
#pragma unroll
  for (int q = 0; q < 5; ++q) acc[q] = xsum_rows(acc[q]);
  T* red = L.red + 4 * par;
  T* dred = L.dred + 8 * kBW * par;
  if (lane == 0) red[w] = acc[0];
  if (g == 0) {
    dred[8 * c + 2 * w] = acc[1];
    dred[8 * c + 2 * w + 1] = acc[3];
    dred[8 * (16 + c) + 2 * w] = acc[2];
    dred[8 * (16 + c) + 2 * w + 1] = acc[4];
  }
  __syncthreads();
  const v4<T> rd = *reinterpret_cast<const v4<T>*>(red);
  const T sigma = (rd[0] + rd[1]) + (rd[2] + rd[3]);
  const T* pj = dred + 8 * jv;
  const T alpha = (pj[1] + pj[3]) + (pj[5] + pj[7]);
  T beta, tau, scale;
  householder_fast(alpha, sigma, beta, tau, scale);
  const v4<T> e0a = *reinterpret_cast<const v4<T>*>(dred + 8 * c);
  const v4<T> e0b = *reinterpret_cast<const v4<T>*>(dred + 8 * c + 4);
  const v4<T> e1a = *reinterpret_cast<const v4<T>*>(dred + 8 * (16 + c));
  const v4<T> e1b = *reinterpret_cast<const v4<T>*>(dred + 8 * (16 + c) + 4);
  const T x0 = (e0a[0] + e0a[2]) + (e0b[0] + e0b[2]), y0 = (e0a[1] + e0a[3]) + (e0b[1] + e0b[3]);
  const T x1 = (e1a[0] + e1a[2]) + (e1b[0] + e1b[2]), y1 = (e1a[1] + e1a[3]) + (e1b[1] + e1b[3]);
  const int v0 = c, v1 = 16 + c;
  const T w0 = (QL ? v0 < jv : v0 > jv) ? tau * (scale * x0 + y0) : T(0);
  const T w1 = (QL ? v1 < jv : v1 > jv) ? tau * (scale * x1 + y1) : T(0);
  // the reflector at this lane's positions, and the update
  if (inside) {
#pragma unroll
    for (int rl = 0; rl < 2; ++rl)
#pragma unroll
      for (int r = 0; r < 4; ++r) xp[rl][r] *= scale;
  } else if (outside) {
#pragma unroll
    for (int rl = 0; rl < 2; ++rl) xp[rl] = v4zero<T>();
  } else {
#pragma unroll
    for (int rl = 0; rl < 2; ++rl)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int th = su(pp - base - 16 * rl - r);
        const bool in = QL ? 4 * g < th : 4 * g > th;
        const T y = xp[rl][r] * scale;
        xp[rl][r] = in ? y : (4 * g == th ? T(1) : T(0));
      }
  }
#pragma unroll
  for (int rl = 0; rl < 2; ++rl)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Pn.t[rl][0][r] -= w0 * xp[rl][r];
      Pn.t[rl][1][r] -= w1 * xp[rl][r];
    }
  if (c == 0) {
#pragma unroll
    for (int rl = 0; rl < 2; ++rl)
      *reinterpret_cast<v4<T>*>(L.Yt + jv * kLY + base + 16 * rl + 4 * g) = xp[rl];
  }
  if (w == 0 && lane == 0) {
    L.bet[jv] = beta;
    L.taus[jv] = tau;
  }
}

// T of the panel in Yt / taus into Ts (TRANS: T^T), by the whole work-group.
// G = Y^T Y (its three upper 16x16 tiles) by the wavefronts other than pw,
// then the back substitution by wavefront (pw + 1) & 3, lane j < 32 computing
// column j: T(i, j) = tau_i (delta_ij - sum_{m > i} G(i, m) T(m, j)), i from
// the bottom up.
// G and T share Ts (the back substitution reads all of G before it writes).
template <typename T, int RLO, bool TRANS>
__device__ __forceinline__ void make_t(const T* Yt, T* Ts, const T* taus, int w, int pw, int lane,
                                       int g, int c) {
  __syncthreads();
  const int gw = (w - pw + 4) & 3;
  if (gw >= 1) {
    const int it = gw == 3 ? 1 : 0, jt = gw == 1 ? 0 : 1;
    v4<T> acc = v4zero<T>();
#pragma unroll
    for (int rt = RLO; rt < 8; ++rt) {
      const v4<T> va = *reinterpret_cast<const v4<T>*>(Yt + (16 * it + c) * kLY + 16 * rt + 4 * g);
      const v4<T> vb = *reinterpret_cast<const v4<T>*>(Yt + (16 * jt + c) * kLY + 16 * rt + 4 * g);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma4(va[r], vb[r], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Ts[(16 * it + mma_row<T>(g, r)) * kLT + 16 * jt + c] = acc[r];
  }
  __syncthreads();
  if (gw == 1) {
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
      for (int i = 0; i < m; ++i) t[i] -= Ts[i * kLT + m] * t[m];
    }
    if (lane < kBW) {
#pragma unroll
      for (int i = 0; i < kBW; ++i) {
        if (TRANS) Ts[j * kLT + i] = t[i];
        else Ts[i * kLT + j] = t[i];
      }
    }
  }
  __syncthreads();
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

// Outputs of LQ panel P from the panel registers (every wavefront its
// positions): rows i = 32 P + jv, jv < cnt, of FD (L left of the diagonal,
// beta on it, the reflector to the right) and columns i of FZ (the reflector
// with its unit and zeros above); when the panel holds rows >= e (the last
// panel), those rows of FD as they are.
template <typename T>
__device__ __forceinline__ void store_lq_panel(const Panel<T>& Pn, const PanelLds<T>& L, T* FD,
                                               T* FZ, int mp, int e, int P, int cnt, bool last,
                                               int w, int g, int c) {
  constexpr uint32_t sz = sizeof(T);
  const int base = 32 * w;
  const auto RD = buf_rsrc(FD, (uint32_t)(mp * mp) * sz);
  const auto RZ = buf_rsrc(FZ, (uint32_t)(mp * e) * sz);
  const int dgc = 4 * g - c;   // column - row = dgc - th
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int jv = 16 * ct + c, row = 32 * P + jv;
    const bool refl = jv < cnt;
    const bool wr = (row < mp) & (refl | last);
    const T b = L.bet[jv];
    const T* y = L.Yt + jv * kLY + base + 4 * g;
    const uint32_t vd = wr ? (uint32_t)(row + (base + 4 * g) * mp) * sz : kBufOOB;
    const uint32_t vz = refl ? (uint32_t)(base + 4 * g + row * mp) * sz : kBufOOB;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t vdr = vd + (uint32_t)(r * mp) * sz;
#pragma unroll
      for (int rl = 0; rl < 2; ++rl) {
        const int th = su(32 * P + 16 * ct - base - 16 * rl - r);
        const T yv = y[16 * rl + r];
        const T x = Pn.t[rl][ct][r];
        const T dv = refl ? (dgc < th ? x : (dgc == th ? b : yv)) : x;
        const T zv = dgc > th ? yv : (dgc == th ? T(1) : T(0));
        buf_store<T>(dv, RD, vdr, (uint32_t)(16 * rl * mp) * sz);
        const bool cin = (mp >= kBP) | (4 * g < su(mp - base - 16 * rl - r));
        buf_store<T>(zv, RZ, cin ? vz + (16 * rl + r) * sz : kBufOOB, 0);
      }
    }
  }
}

// FP32: four waves per SIMD (128 registers); FP64: two (its accumulator
// tiles and panel registers take twice the space).
template <typename T, bool BATCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2))) void k_ulv_factor_blk(
    KArgs<T, CallSV<T>> a) {
  __shared__ __attribute__((aligned(16))) T Yt[kBW * kLY];
  __shared__ __attribute__((aligned(16))) T Ts[kBW * kLT];
  __shared__ __attribute__((aligned(16))) T red[2 * 4];
  __shared__ __attribute__((aligned(16))) T dred[2 * 8 * kBW];
  __shared__ T bet[kBW], taus[kBW];
  __shared__ int sing;
  const PanelLds<T> L{red, dred, Yt, bet, taus};
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int mp = nd.mp, ku = nd.ku, kv = nd.kv, e = nd.e;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  const int s = kBP - mp;
  T* FU = I.FU + nd.oFU;
  T* FV = I.FV + nd.oFV;
  T* FD = I.FD + nd.oFD;
  T* FZ = I.FZ + nd.oFZ;
  const T* Dsrc = nd.is_leaf ? I.D + nd.oD : FD;
  const T* Usrc = nd.is_leaf ? I.U + nd.oU : FU;
  const T* Vsrc = nd.is_leaf ? I.V + nd.oV : FV;
  if (tid == 0) sing = 0;
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
  Panel<T> Pn;
  // ---- QL of U' (one panel over the four wavefronts) and M = Q^T D'
  if (ku > 0) {
    panel_load_cols(Pn, Usrc, mp, ku, s, w, g, c);
    panel_clear(L, w, lane);
    for (int jq = ku - 1; jq >= 0; --jq) panel_step<T, true>(Pn, jq, kBP - ku + jq, L, w, lane, g, c);
    __syncthreads();
    {
      // finished columns: reflector above the pivot, beta, U~ below
      constexpr uint32_t sz = sizeof(T);
      const int base = 32 * w, dgc = 4 * g - c;   // position - pp = dgc - th
      const auto RU = buf_rsrc(FU, (uint32_t)(mp * ku) * sz);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const int jv = 16 * ct + c;
        const T b = bet[jv];
        const T* y = Yt + jv * kLY + base + 4 * g;
#pragma unroll
        for (int rl = 0; rl < 2; ++rl)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int th = su(kBP - ku + 16 * ct - base - 16 * rl - r);
            const T yv = y[16 * rl + r];
            const T v = dgc < th ? yv : (dgc == th ? b : Pn.t[rl][ct][r]);
            const int row = base + 16 * rl + 4 * g + r - s;
            const bool in = (jv < ku) & (row >= 0);
            buf_store<T>(v, RU, in ? (uint32_t)(row + jv * mp) * sz : kBufOOB, 0);
          }
      }
      if (tid < ku) I.tq[nd.otq + tid] = taus[tid];
    }
    slab_load_cols(X, Dsrc, mp, mp, mp, s, 32 * w, g, c);
    make_t<T, 0, false>(Yt, Ts, taus, w, 0, lane, g, c);
    block_update<T, 0>(X, Yt, Ts, g, c);
    // M to FD (column slabs), then back as transposed row slabs
    slab_store_cols(X, FD, mp, mp, mp, s, 32 * w, g, c);
    __syncthreads();
    slab_load_rows(X, FD, mp, mp, mp, 32 * w, g, c);
  } else {
    slab_load_rows(X, Dsrc, mp, mp, mp, 32 * w, g, c);
  }
  // ---- LQ of rows 0 .. e-1 of M, panels of 32 rows: wavefront P's slab is
  // spread over the four wavefronts by position (through Yt), factored, and
  // applied to the slabs below it and to V' (wavefront 0 after panel 0).
  const int plast = (e - 1) >> 5;
#define HSS_LQ_PANEL(P)                                                                     \
  if (P <= plast) {                                                                         \
    const int cnt = min(kBW, e - 32 * P);                                                   \
    if (w == P) {                                                                           \
      _Pragma("unroll") for (int ct = 0; ct < 2; ++ct)                                      \
        _Pragma("unroll") for (int rt = 0; rt < 8; ++rt)                                    \
          lds_put_rows4(Yt + (16 * ct + c) * kLY + 16 * rt, g, X[rt][ct]);                 \
    }                                                                                       \
    __syncthreads();                                                                        \
    panel_load_lds(Pn, Yt, w, g, c);                                                        \
    panel_clear(L, w, lane);                                                                \
    for (int j = 0; j < cnt; ++j) panel_step<T, false>(Pn, j, 32 * P + j, L, w, lane, g, c); \
    __syncthreads();                                                                        \
    store_lq_panel(Pn, L, FD, FZ, mp, e, P, cnt, P == plast, w, g, c);                      \
    if (tid < cnt) I.tz[nd.otz + 32 * P + tid] = taus[tid];                                 \
    if (tid == 0) {                                                                         \
      for (int j = 0; j < cnt; ++j)                                                         \
        if (bet[j] == T(0)) sing = 1;                                                       \
    }                                                                                       \
    if (P == 0 && w == 0 && kv > 0) slab_load_cols(X, Vsrc, mp, mp, kv, 0, 0, g, c);        \
    make_t<T, 2 * P, true>(Yt, Ts, taus, w, 0, lane, g, c);                                 \
    if (w > P || (w == 0 && kv > 0)) block_update<T, 2 * P>(X, Yt, Ts, g, c);               \
    __syncthreads();                                                                        \
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
