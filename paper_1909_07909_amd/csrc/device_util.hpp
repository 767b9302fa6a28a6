// Device helpers for the gfx950 kernels: work-group small GEMM, wavefront
// reductions, task resolution.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hss_internal.hpp"

namespace hss {

// Cross-lane moves through DPP (executed in the VALU, no LDS crossbar).
// Control codes of the GFX9 DPP encoding.
constexpr int kDppQuadXor1 = 0xB1;    // quad_perm(1,0,3,2)
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm(2,3,0,1)
constexpr int kDppRowRor4 = 0x124;
constexpr int kDppRowRor8 = 0x128;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;

template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF,
                                                    false));
}
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float lane_read(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_read(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// value of lane ^ 1 (the partner of a lane pair)
template <typename T>
__device__ __forceinline__ T xor1(T v) {
  return dpp<kDppQuadXor1>(v);
}

// Sum over the 64 lanes of a wavefront, returned in every lane: pairs and
// quads by quad permutes, rows of 16 by two row rotations, then the four
// rows by the row broadcasts (the total lands in row 3) and a lane read.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp<kDppQuadXor1>(v);
  v += dpp<kDppQuadXor2>(v);
  v += dpp<kDppRowRor4>(v);
  v += dpp<kDppRowRor8>(v);
  v += dpp<kDppRowBcast15, 0xA>(v);
  v += dpp<kDppRowBcast31, 0x8>(v);
  return lane_read(v, 63);
}

// *p if ok, else 0.  p must be a valid address either way (callers clamp the
// index): the load is issued unconditionally and the mask applied to its
// result, so that a sequence of such loads is in flight together instead of
// being turned into one branch and one memory round trip per element.
template <typename T>
__device__ __forceinline__ T ld_or0(const T* p, bool ok) {
  const T v = *p;
  return ok ? v : T(0);
}

// ld_or0 for a read issued where it is written: a relaxed atomic load may not
// be moved past a work-group barrier that follows, so it stays in flight
// across it (a plain load would be sunk to its first use).
template <typename T>
__device__ __forceinline__ T ld_early_or0(const T* p, bool ok) {
  const T v = __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return ok ? v : T(0);
}

// store(i, j, f(i, j)) for i < M, j < N by all threads of the work-group.  f
// must be a plain read that is valid for every (i, j) in range: each thread
// issues the reads of U elements before it stores any, so that they are in
// flight together.
template <int U, typename T, typename F, typename S>
__device__ __forceinline__ void wg_stage(int M, int N, F f, S store) {
  const int total = M * N, nt = blockDim.x;
  for (int base = 0; base < total; base += U * nt) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int o = min(base + (int)threadIdx.x + u * nt, total - 1);
      v[u] = f(o % M, o / M);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int o = base + (int)threadIdx.x + u * nt;
      if (o < total) store(o % M, o / M, v[u]);
    }
  }
}

// Maximum / minimum over the 64 lanes (same DPP pattern as wave_sum).
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  v = max(v, dpp<kDppQuadXor1>(v));
  v = max(v, dpp<kDppQuadXor2>(v));
  v = max(v, dpp<kDppRowRor4>(v));
  v = max(v, dpp<kDppRowRor8>(v));
  v = max(v, dpp<kDppRowBcast15, 0xA>(v));
  v = max(v, dpp<kDppRowBcast31, 0x8>(v));
  return lane_read(v, 63);
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
  return -wave_max(-v);
}

// Resolve (instance, call, node) of this work-group.
template <bool BATCH, typename T, typename Call>
__device__ __forceinline__ void resolve(const KArgs<T, Call>& a, Inst<T>& I, Call& C, int& node) {
  if constexpr (BATCH) {
    const int2 tk = a.tasks[blockIdx.x];
    I = a.insts[tk.x];
    C = a.calls[tk.x];
    node = tk.y;
  } else {
    I = a.inst;
    C = a.call;
    node = a.node0 + blockIdx.x;
  }
}

template <typename T, bool TA>
__device__ __forceinline__ T ldA(const T* __restrict__ A, int64_t lda, int i, int l) {
  return TA ? A[l + (int64_t)i * lda] : A[i + (int64_t)l * lda];
}

// C (=|+=) op(A) * B, op(A) = A (M x K, ld lda) or A^T (A is K x M).  B is
// K x N (ld ldb), C is M x N (ld ldc).  All pointers generic (LDS or global).
// Each output is produced by one thread; K is split over up to 16 thread
// slices when the output is small.  red: LDS scratch of blockDim.x entries.
// Must be called by all threads of the work-group.
template <typename T, bool TA>
__device__ void wg_gemm(int M, int N, int K, const T* __restrict__ A, int64_t lda,
                        const T* B, int64_t ldb, T* C, int64_t ldc, bool accumulate, T* red) {
  const int nt = blockDim.x, tid = threadIdx.x;
  const int MN = M * N;
  if (MN <= 0) return;
  int S = 1;
  if (K > 16 && MN < nt) {
    S = nt / MN;
    if (S > 16) S = 16;
    S = 1 << (31 - __clz(S));
  }
  if (S == 1) {
    for (int o = tid; o < MN; o += nt) {
      const int i = o % M, j = o / M;
      T s = 0;
      for (int l = 0; l < K; ++l) s += ldA<T, TA>(A, lda, i, l) * B[l + (int64_t)j * ldb];
      T* c = C + i + (int64_t)j * ldc;
      *c = accumulate ? *c + s : s;
    }
  } else {
    const int o = tid % MN, s = tid / MN;
    T part = 0;
    if (tid < MN * S) {
      const int i = o % M, j = o / M;
      for (int l = s; l < K; l += S) part += ldA<T, TA>(A, lda, i, l) * B[l + (int64_t)j * ldb];
    }
    red[tid] = part;
    __syncthreads();
    if (tid < MN) {
      T sum = 0;
      for (int q = 0; q < S; ++q) sum += red[tid + q * MN];
      const int i = tid % M, j = tid / M;
      T* c = C + i + (int64_t)j * ldc;
      *c = accumulate ? *c + sum : sum;
    }
    __syncthreads();
  }
}

// Accessor form: C(i, j) <- fa(i, l) fb(l, j) summed over l < K; fc(i, j, v)
// stores the result.  Same thread mapping as wg_gemm.
template <typename T, typename FA, typename FB, typename FC>
__device__ void wg_gemm_f(int M, int N, int K, FA fa, FB fb, FC fc, T* red) {
  const int nt = blockDim.x, tid = threadIdx.x;
  const int MN = M * N;
  if (MN <= 0) return;
  int S = 1;
  if (K > 16 && MN < nt) {
    S = nt / MN;
    if (S > 16) S = 16;
    S = 1 << (31 - __clz(S));
  }
  if (S == 1) {
    for (int o = tid; o < MN; o += nt) {
      const int i = o % M, j = o / M;
      T s = 0;
      for (int l = 0; l < K; ++l) s += fa(i, l) * fb(l, j);
      fc(i, j, s);
    }
  } else {
    const int o = tid % MN, s = tid / MN;
    T part = 0;
    if (tid < MN * S) {
      const int i = o % M, j = o / M;
      for (int l = s; l < K; l += S) part += fa(i, l) * fb(l, j);
    }
    red[tid] = part;
    __syncthreads();
    if (tid < MN) {
      T sum = 0;
      for (int q = 0; q < S; ++q) sum += red[tid + q * MN];
      fc(tid % M, tid / M, sum);
    }
    __syncthreads();
  }
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

// LDS written by some lanes and then read by other lanes of the same
// wavefront: the hardware executes a wavefront's LDS operations in order, so
// only the compiler has to be kept from reordering or forwarding across this
// point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// householder() for the FP32 factors with the hardware square root and
// reciprocal (about one ulp each): FP32 factors only precondition the FP64
// refinement, which restores the accuracy.  FP64 keeps the exact operations.
__device__ __forceinline__ void householder_fast(float alpha, float sigma, float& beta, float& tau,
                                                 float& scale) {
  if (sigma == 0.f) {
    beta = alpha;
    tau = 0.f;
    scale = 0.f;
  } else {
    const float nrm = __builtin_amdgcn_sqrtf(alpha * alpha + sigma);
    beta = alpha >= 0.f ? -nrm : nrm;
    tau = (beta - alpha) * __builtin_amdgcn_rcpf(beta);
    scale = __builtin_amdgcn_rcpf(alpha - beta);
  }
}
__device__ __forceinline__ void householder_fast(double alpha, double sigma, double& beta,
                                                 double& tau, double& scale) {
  householder(alpha, sigma, beta, tau, scale);
}

// Copy an M x N block (generic pointers) into LDS with leading dimension lds.
template <typename T, typename S>
__device__ __forceinline__ void wg_load(int M, int N, const S* __restrict__ src, int64_t ld,
                                        T* dst, int lds) {
  for (int o = threadIdx.x; o < M * N; o += blockDim.x) {
    const int i = o % M, j = o / M;
    dst[i + j * lds] = (T)src[i + (int64_t)j * ld];
  }
}

template <typename T>
__device__ __forceinline__ void wg_store(int M, int N, const T* src, int lds, T* dst, int64_t ld) {
  for (int o = threadIdx.x; o < M * N; o += blockDim.x) {
    const int i = o % M, j = o / M;
    dst[i + (int64_t)j * ld] = src[i + j * lds];
  }
}

// Raw buffer access: base and size in a resource descriptor (SGPRs), a
// per-lane byte offset and a uniform byte offset; reads at or beyond the size
// return zero.
// Every caller passes wavefront-uniform bases, sizes and uniform offsets; they
// are moved to scalar registers explicitly so that the compiler does not fall
// back to a per-lane loop over descriptors.
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  const uint64_t b = reinterpret_cast<uint64_t>(base);
  const uint64_t ub = ((uint64_t)uni((uint32_t)(b >> 32)) << 32) | uni((uint32_t)b);
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(ub), 0, (int)uni(bytes),
                                           0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                   uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, uni(soff), 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                 uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, uni(soff), 0));
}

template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff);
template <>
__device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r,
                                                  uint32_t voff, uint32_t soff) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, uni(soff), 0);
}
template <>
__device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                 uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, uni(soff), 0);
}
// A byte offset that every buffer access treats as out of range (stores are
// dropped, loads return zero).
constexpr uint32_t kBufOOB = 0x80000000u;

// ---------------------------------------------------------------------------
// 16 x 16 x 4 matrix-core products (one wavefront): lane 16 g + c supplies
// A(c, g) and B(g, c) and holds four entries of the 16 x 16 accumulator D:
// component r is D(mma_row<T>(g, r), c), where the FP32 instruction keeps rows
// 4 g .. 4 g + 3 in a lane and the FP64 one rows g, g + 4, g + 8, g + 12.
template <typename T> struct MmaV4;
template <> struct MmaV4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct MmaV4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <typename T> using mma4_t = typename MmaV4<T>::type;

__device__ __forceinline__ mma4_t<float> mma16(float a, float b, mma4_t<float> c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mma4_t<double> mma16(double a, double b, mma4_t<double> c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T>
__device__ __forceinline__ constexpr int mma_row(int g, int r) {
  return sizeof(T) == 8 ? g + 4 * r : 4 * g + r;
}
template <typename T>
__device__ __forceinline__ mma4_t<T> mma_zero() {
  mma4_t<T> z;
  z[0] = z[1] = z[2] = z[3] = T(0);
  return z;
}

}  // namespace hss
