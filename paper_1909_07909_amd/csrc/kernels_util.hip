// Elementwise and column-reduction kernels around the HSS path: the resident
// FP32 generator copy, the FP64 residual of iterative refinement, per-column
// norms and the backward error of Sec. 5.1.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace hss {

namespace {
constexpr int kB = 256;

inline int grid_for(int64_t n, int cap = 8192) {
  int64_t g = (n + kB - 1) / kB;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

__global__ void k_cast(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    d[i] = (float)s[i];
}

__global__ void k_scale_cast(const double* __restrict__ s, int64_t lds, float* __restrict__ d,
                             int64_t ldd, int64_t n, const double* __restrict__ scale,
                             const int32_t* gate) {
  if (gated_off(gate)) return;
  const int64_t j = blockIdx.y;
  // a zero column stays zero (its scale is 0)
  const double f = scale ? (scale[j] > 0.0 ? 1.0 / scale[j] : 0.0) : 1.0;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    d[i + j * ldd] = (float)(s[i + j * lds] * f);
}

__global__ void k_axpy_cast(const float* __restrict__ dd, int64_t ldd, double* __restrict__ x,
                            int64_t ldx, int64_t n, const double* __restrict__ scale,
                            const int32_t* gate) {
  if (gated_off(gate)) return;   // converged: the correction is not applied
  const int64_t j = blockIdx.y;
  const double f = scale ? scale[j] : 1.0;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    x[i + j * ldx] += f * (double)dd[i + j * ldd];
}

__global__ void k_cast_back(const float* __restrict__ s, int64_t lds, double* __restrict__ d,
                            int64_t ldd, int64_t n, const double* __restrict__ scale) {
  const int64_t j = blockIdx.y;
  const double f = scale ? scale[j] : 1.0;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    d[i + j * ldd] = f * (double)s[i + j * lds];
}

__global__ void k_axpy64(const double* __restrict__ s, int64_t lds, double* __restrict__ d,
                         int64_t ldd, int64_t n, const int32_t* gate) {
  if (gated_off(gate)) return;
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    d[i + j * ldd] += s[i + j * lds];
}

// dst = src / sqrt(sumsq[0]) (power-method normalization, no host round trip)
__global__ void k_normalize(const double* __restrict__ s, double* __restrict__ d, int64_t n,
                            const double* __restrict__ sumsq) {
  const double nr = sqrt(sumsq[0]);
  const double f = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    d[i] = s[i] * f;
}

// deterministic start vector in [-1, 1) (splitmix64 of the index)
__global__ void k_hash_fill(double* d, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    uint64_t z = (uint64_t)i + seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    d[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

__global__ void k_copy2d(const double* __restrict__ s, int64_t lds, double* __restrict__ d,
                         int64_t ldd, int64_t n, const int32_t* gate) {
  if (gated_off(gate)) return;
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    d[i + j * ldd] = s[i + j * lds];
}

__global__ void k_fill(double* p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    p[i] = v;
}

// Per-column sum of squares and max |.|; sumsq / maxabs must start at 0.
__global__ void k_colstats(const double* __restrict__ a, int64_t lda, int64_t n,
                           double* __restrict__ sumsq, double* __restrict__ maxabs) {
  const int64_t j = blockIdx.y;
  double s = 0.0, mx = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    const double v = a[i + j * lda];
    s += v * v;
    mx = fmax(mx, fabs(v));
  }
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    mx = fmax(mx, __shfl_xor(mx, off, 64));
  }
  __shared__ double ss[kB / 64], sm[kB / 64];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) { ss[w] = s; sm[w] = mx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, m = 0.0;
    for (int q = 0; q < kB / 64; ++q) { t += ss[q]; m = fmax(m, sm[q]); }
    atomicAdd(&sumsq[j], t);
    if (maxabs) {
      // non-negative doubles order like their bit patterns
      atomicMax(reinterpret_cast<unsigned long long*>(&maxabs[j]),
                (unsigned long long)__double_as_longlong(m));
    }
  }
}

// ---------------------------------------------------------------------------
// Fused single-instance refinement bookkeeping.  Each block reduces its rows
// into per-block partials; the last block to finish (arrival counter, which it
// resets) reduces the partials, so neither kernel needs zeroed accumulators.
constexpr int kChkBlocks = 128;   // blocks per column of the fused kernels

__device__ __forceinline__ void block_reduce2(double& s, double& m) {
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    m = fmax(m, __shfl_xor(m, off, 64));
  }
  __shared__ double bs[kB / 64], bm[kB / 64];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) { bs[w] = s; bm[w] = m; }
  __syncthreads();
  s = 0.0; m = 0.0;
  for (int q = 0; q < kB / 64; ++q) { s += bs[q]; m = fmax(m, bm[q]); }
  __syncthreads();
}

// true in the last block to arrive (after a device-scope release of the
// block's partials; the last block acquires everyone's)
__device__ __forceinline__ bool last_block(unsigned* cnt, unsigned total) {
  __shared__ unsigned s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(cnt, 1u) == total - 1 ? 1u : 0u;
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last != 0;
}

// One backward-error check: r = b - r (r holds A x on entry); per column
// ||r||^2, max |r|, ||x||^2, ||b||^2; then, in the last block,
// eta_j = ||r_j|| / (||A|| ||x_j|| + ||b_j||), out = [max_j eta_j, 0,
// eta_0 .. eta_{nrhs-1}], rmax_j = max |r_j| (the scale of the next
// correction), and the refinement state st (an instance's status block):
// st[kStIters] = step, st[kStGate] = 1 if another correction is to run
// (eta above tol and step < max_refine).  gate: skip the check when 0.
__global__ void k_check(const double* __restrict__ b, int64_t ldb, double* __restrict__ r,
                        int64_t ldr, const double* __restrict__ x, int64_t ldx, int64_t n,
                        int nrhs, double normA, double* part, unsigned* cnt,
                        int32_t* st, double* rmax, double* out, const int32_t* gate,
                        double tol, int step, int max_refine) {
  if (gated_off(gate)) return;
  const int64_t j = blockIdx.y;
  double sr = 0.0, mr = 0.0, sx = 0.0, sb = 0.0, dummy = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    const double bv = b[i + j * ldb];
    const double rv = bv - r[i + j * ldr];
    const double xv = x[i + j * ldx];
    r[i + j * ldr] = rv;
    sr += rv * rv;
    mr = fmax(mr, fabs(rv));
    sx += xv * xv;
    sb += bv * bv;
  }
  block_reduce2(sr, mr);
  block_reduce2(sx, dummy);
  block_reduce2(sb, dummy);
  const int nb = gridDim.x;
  double* pj = part + (int64_t)4 * nb * j;
  if (threadIdx.x == 0) {
    pj[blockIdx.x] = sr;
    pj[nb + blockIdx.x] = mr;
    pj[2 * nb + blockIdx.x] = sx;
    pj[3 * nb + blockIdx.x] = sb;
  }
  if (!last_block(cnt, (unsigned)(nb * nrhs))) return;
  double emax = 0.0;
  for (int c = 0; c < nrhs; ++c) {
    const double* pc = part + (int64_t)4 * nb * c;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int q = threadIdx.x; q < nb; q += kB) {
      a0 += pc[q];
      a1 = fmax(a1, pc[nb + q]);
      a2 += pc[2 * nb + q];
      a3 += pc[3 * nb + q];
    }
    block_reduce2(a0, a1);
    block_reduce2(a2, dummy);
    block_reduce2(a3, dummy);
    const double den = normA * sqrt(a2) + sqrt(a3);
    const double e = den > 0.0 ? sqrt(a0) / den : (a0 > 0.0 ? INFINITY : 0.0);
    if (threadIdx.x == 0) {
      out[2 + c] = e;
      rmax[c] = a1;
    }
    emax = fmax(emax, e);
  }
  if (threadIdx.x == 0) {
    out[0] = emax;
    out[1] = 0.0;
    st[kStIters] = step;
    st[kStGate] = (tol > 0.0 && emax > tol && step < max_refine) ? 1 : 0;
    *cnt = 0u;
  }
}

// The solve report (hss_solve_info followed by nrhs doubles): backward
// errors from out (when computed), refinement steps and the status from the
// instance's status block st.
__global__ void k_solve_info(char* info, int nrhs, const double* out, const int32_t* st,
                             double normA, double tol, int have_eta) {
  double* hd = reinterpret_cast<double*>(info);
  int32_t* hi = reinterpret_cast<int32_t*>(info + 16);
  double* eta = reinterpret_cast<double*>(info + 32);
  for (int c = threadIdx.x; c < nrhs; c += blockDim.x) eta[c] = have_eta ? out[2 + c] : 0.0;
  if (threadIdx.x == 0) {
    const double em = have_eta ? out[0] : 0.0;
    const int32_t bits = st[0];
    int32_t status = 0;
    if (bits & (1 << kStatusWaitCode)) status = kStatusWaitCode;
    else if (bits & (1 << kCodeSingular)) status = kCodeSingular;
    else if (have_eta && tol > 0.0 && !(em <= tol)) status = kCodeNoConv;
    hd[0] = em;
    hd[1] = normA;
    hi[0] = have_eta ? st[kStIters] : 0;
    hi[1] = status;
    hi[2] = st[kStSingularNode] - 1;
    hi[3] = nrhs;
  }
}

// Per-column max |a| (the scale of an FP32 correction), by the same scheme.
__global__ void k_colmax(const double* __restrict__ a, int64_t lda, int64_t n, int nrhs,
                         double* part, unsigned* cnt, double* amax) {
  const int64_t j = blockIdx.y;
  double m = 0.0, dummy = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    m = fmax(m, fabs(a[i + j * lda]));
  block_reduce2(dummy, m);
  const int nb = gridDim.x;
  if (threadIdx.x == 0) part[(int64_t)nb * j + blockIdx.x] = m;
  if (!last_block(cnt, (unsigned)(nb * nrhs))) return;
  for (int c = 0; c < nrhs; ++c) {
    double mm = 0.0, d2 = 0.0;
    for (int q = threadIdx.x; q < nb; q += kB) mm = fmax(mm, part[(int64_t)nb * c + q]);
    block_reduce2(d2, mm);
    if (threadIdx.x == 0) amax[c] = mm;
  }
  if (threadIdx.x == 0) *cnt = 0u;
}

// ---------------------------------------------------------------------------
// Refinement bookkeeping over many instances in one launch: blockIdx.y picks
// the instance, the x dimension strides over the rows of every column.
__device__ __forceinline__ void atomic_max_nonneg(double* p, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
}

__global__ void k_ir_batch(int op, const IRSeg* __restrict__ segs, int count, int gated,
                           int step, int max_refine) {
  const IRSeg S = segs[blockIdx.y];
  if (gated && S.st[kStGate] == 0) return;
  const int64_t n = S.n;
  const int nr = S.nrhs;
  double* rr = S.stats;
  double* xx = rr + nr;
  double* bb = xx + nr;
  double* rmax = bb + nr;
  double* bmax = rmax + nr;
  double* eta = bmax + nr;
  double* outv = eta + nr;
  const int64_t i0 = blockIdx.x * (int64_t)kB + threadIdx.x, st = (int64_t)gridDim.x * kB;
  if (op == IR_ZERO_ALL || op == IR_ZERO) {
    if (blockIdx.x == 0 && blockIdx.z == 0)
      for (int j = threadIdx.x; j < 7 * nr; j += kB) {
        const int blk = j / nr;   // 0 rr, 1 xx, 2 bb, 3 rmax, 4 bmax, 5 eta, 6 out
        if (op == IR_ZERO_ALL || blk == 0 || blk == 1 || blk == 3) S.stats[j] = 0.0;
      }
    return;
  }
  if (op == IR_ETA) {
    if (blockIdx.x == 0 && blockIdx.z == 0 && threadIdx.x == 0) {
      double mx = 0.0;
      for (int j = 0; j < nr; ++j) {
        const double den = S.norm2 * sqrt(xx[j]) + sqrt(bb[j]);
        const double v = den > 0.0 ? sqrt(rr[j]) / den : (rr[j] > 0.0 ? INFINITY : 0.0);
        eta[j] = v;
        mx = fmax(mx, v);
      }
      outv[0] = mx;
      S.st[kStIters] = step;
      S.st[kStGate] = (S.tol > 0.0 && mx > S.tol && step < max_refine) ? 1 : 0;
    }
    return;
  }
  if (op == IR_INFO) {
    if (blockIdx.x != 0 || blockIdx.z != 0 || !S.info) return;
    char* info = static_cast<char*>(S.info);
    double* hd = reinterpret_cast<double*>(info);
    int32_t* hi = reinterpret_cast<int32_t*>(info + 16);
    double* eo = reinterpret_cast<double*>(info + 32);
    const bool have_eta = step != 0;
    for (int c = threadIdx.x; c < nr; c += kB) eo[c] = have_eta ? eta[c] : 0.0;
    if (threadIdx.x == 0) {
      const double em = have_eta ? outv[0] : 0.0;
      const int32_t bits = S.st[0];
      int32_t status = 0;
      if (bits & (1 << kStatusWaitCode)) status = kStatusWaitCode;
      else if (bits & (1 << kCodeSingular)) status = kCodeSingular;
      else if (have_eta && S.tol > 0.0 && !(em <= S.tol)) status = kCodeNoConv;
      hd[0] = em;
      hd[1] = S.norm2;
      hi[0] = have_eta ? S.st[kStIters] : 0;
      hi[1] = status;
      hi[2] = S.st[kStSingularNode] - 1;
      hi[3] = nr;
    }
    return;
  }
  {
    // one column per grid slice: blockIdx.z
    const int j = blockIdx.z;
    if (j >= nr) return;
    double* Bj = S.B + j * S.ldb;
    double* b0 = S.b0 + j * n;
    double* rs = S.res + j * n;
    double* d64 = S.d64 + j * n;
    float* r32 = S.r32 + j * n;
    double acc = 0.0, mx = 0.0;
    for (int64_t i = i0; i < n; i += st) {
      switch (op) {
        case IR_SAVE_B0: b0[i] = Bj[i]; break;
        case IR_STATS_B0: acc += b0[i] * b0[i]; break;
        case IR_STATS_BMAX: mx = fmax(mx, fabs(Bj[i])); break;
        case IR_SCALE_B: r32[i] = bmax[j] > 0.0 ? (float)(Bj[i] / bmax[j]) : 0.f; break;
        case IR_CAST_BACK: Bj[i] = bmax[j] * (double)r32[i]; break;
        case IR_RESID: {
          const double r = b0[i] - rs[i];
          rs[i] = r;
          acc += r * r;
          mx = fmax(mx, fabs(r));
          break;
        }
        case IR_STATS_X: acc += Bj[i] * Bj[i]; break;
        case IR_SCALE_RES: r32[i] = rmax[j] > 0.0 ? (float)(rs[i] / rmax[j]) : 0.f; break;
        case IR_AXPY_CAST: Bj[i] += rmax[j] * (double)r32[i]; break;
        case IR_COPY_RES: d64[i] = rs[i]; break;
        case IR_AXPY64: Bj[i] += d64[i]; break;
        default: break;
      }
    }
    if (op == IR_STATS_B0 || op == IR_RESID || op == IR_STATS_X || op == IR_STATS_BMAX) {
      for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, 64);
        mx = fmax(mx, __shfl_xor(mx, off, 64));
      }
      if ((threadIdx.x & 63) == 0) {
        if (op == IR_STATS_B0) atomicAdd(&bb[j], acc);
        if (op == IR_STATS_X) atomicAdd(&xx[j], acc);
        if (op == IR_RESID) {
          atomicAdd(&rr[j], acc);
          atomic_max_nonneg(&rmax[j], mx);
        }
        if (op == IR_STATS_BMAX) atomic_max_nonneg(&bmax[j], mx);
      }
    }
  }
}
}  // namespace

void launch_ir_batch(int op, const IRSeg* segs, int count, int64_t max_n, int max_cols,
                     bool gated, int step, int max_refine, hipStream_t s) {
  if (count <= 0) return;
  // the per-column passes take one grid slice per column (z); the zeroing,
  // check and report passes one slice
  const bool per_col = !(op == IR_ZERO_ALL || op == IR_ZERO || op == IR_ETA || op == IR_INFO);
  const int gz = per_col ? std::max(max_cols, 1) : 1;
  hipLaunchKernelGGL(k_ir_batch, dim3(grid_for(max_n, 64), count, gz), dim3(kB), 0, s, op, segs,
                     count, gated ? 1 : 0, step, max_refine);
}

void launch_cast_f64_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cast, dim3(grid_for(n)), dim3(kB), 0, s, src, dst, n);
}

void launch_scale_cast(const double* src, int64_t lds, float* dst, int64_t ldd, int64_t n,
                       int64_t nrhs, const double* scale, hipStream_t s, const int32_t* gate) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_scale_cast, dim3(grid_for(n, 1024), nrhs), dim3(kB), 0, s, src, lds, dst,
                     ldd, n, scale, gate);
}

void launch_axpy_cast(const float* d, int64_t ldd, double* x, int64_t ldx, int64_t n,
                      int64_t nrhs, const double* scale, hipStream_t s, const int32_t* gate) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_axpy_cast, dim3(grid_for(n, 1024), nrhs), dim3(kB), 0, s, d, ldd, x, ldx,
                     n, scale, gate);
}

void launch_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                   int64_t nrhs, hipStream_t s, const int32_t* gate) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_copy2d, dim3(grid_for(n, 1024), nrhs), dim3(kB), 0, s, src, lds, dst, ldd,
                     n, gate);
}

void launch_cast_back(const float* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                      int64_t nrhs, const double* scale, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_cast_back, dim3(grid_for(n, 1024), nrhs), dim3(kB), 0, s, src, lds, dst,
                     ldd, n, scale);
}

void launch_axpy64(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                   int64_t nrhs, hipStream_t s, const int32_t* gate) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_axpy64, dim3(grid_for(n, 1024), nrhs), dim3(kB), 0, s, src, lds, dst, ldd,
                     n, gate);
}

void launch_normalize(const double* src, double* dst, int64_t n, const double* sumsq,
                      hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_normalize, dim3(grid_for(n)), dim3(kB), 0, s, src, dst, n, sumsq);
}

void launch_hash_fill(double* d, int64_t n, uint64_t seed, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_hash_fill, dim3(grid_for(n)), dim3(kB), 0, s, d, n, seed);
}

void launch_fill(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kB), 0, s, p, v, n);
}

void launch_colstats(const double* a, int64_t lda, int64_t n, int64_t nrhs, double* sumsq,
                     double* maxabs, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_colstats, dim3(grid_for(n, 256), nrhs), dim3(kB), 0, s, a, lda, n, sumsq,
                     maxabs);
}

int check_partials(int64_t nrhs) { return 4 * kChkBlocks * (int)std::max<int64_t>(nrhs, 1); }

void launch_check(const double* b, int64_t ldb, double* r, int64_t ldr, const double* x,
                  int64_t ldx, int64_t n, int64_t nrhs, double normA, double* part,
                  unsigned* cnt, int32_t* st, double* rmax, double* out, const int32_t* gate,
                  double tol, int step, int max_refine, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  const int nb = (int)std::min<int64_t>(kChkBlocks, (n + kB - 1) / kB);
  hipLaunchKernelGGL(k_check, dim3(nb, nrhs), dim3(kB), 0, s, b, ldb, r, ldr, x, ldx, n,
                     (int)nrhs, normA, part, cnt, st, rmax, out, gate, tol, step, max_refine);
}

void launch_solve_info(void* info, int64_t nrhs, const double* out, const int32_t* st,
                       double normA, double tol, bool have_eta, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_info, dim3(1), dim3(kB), 0, s, static_cast<char*>(info), (int)nrhs,
                     out, st, normA, tol, have_eta ? 1 : 0);
}

void launch_colmax(const double* a, int64_t lda, int64_t n, int64_t nrhs, double* part,
                   unsigned* cnt, double* amax, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  const int nb = (int)std::min<int64_t>(kChkBlocks, (n + kB - 1) / kB);
  hipLaunchKernelGGL(k_colmax, dim3(nb, nrhs), dim3(kB), 0, s, a, lda, n, (int)nrhs, part, cnt,
                     amax);
}

}  // namespace hss
