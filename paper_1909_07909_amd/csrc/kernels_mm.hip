// HSS matrix x block product (Sec. 4.1, the four steps of the HSS product):
//   K1 leaf projections   x^_i = V_i^T X_i                    (op T: U_i^T)
//   K2 upward pass        x^_t = W_t^T [x^_c1; x^_c2]          (op T: R_t^T)
//   K3 core blocks        y^_c1 = B12_t x^_c2, y^_c2 = B21_t x^_c1 for all
//                         internal t in one launch       (op T: B21^T, B12^T)
//   K4 downward pass      [y^_c1; y^_c2] += R_t y^_t            (op T: W_t)
//   K5 leaf outputs       Y_i = D_i X_i + U_i y^_i       (op T: D_i^T, V_i)
// One work-group per node (and per tile of kRT right-hand-side columns).
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_mm_leaf_up(KArgs<T, CallMM<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallMM<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int c0 = blockIdx.y * kRT;
  if (c0 >= C.nrhs) return;
  const int nc = min(kRT, C.nrhs - c0);
  const bool tr = C.op != 0;
  const int k = tr ? nd.ku : nd.kv;
  const T* basis = tr ? I.U + nd.oU : I.V + nd.oV;
  T* xs = smem;                         // m x nc
  T* red = smem + nd.m * nc;
  wg_load(nd.m, nc, C.X + nd.row0 + (int64_t)c0 * C.ldx, C.ldx, xs, nd.m);
  __syncthreads();
  wg_gemm<T, true>(k, nc, nd.m, basis, nd.m, xs, nd.m, I.xh + nd.oxh + (int64_t)c0 * I.ldm,
                   I.ldm, false, red);
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_mm_up(KArgs<T, CallMM<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallMM<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int c0 = blockIdx.y * kRT;
  if (c0 >= C.nrhs) return;
  const int nc = min(kRT, C.nrhs - c0);
  const bool tr = C.op != 0;
  const int k1 = tr ? n1.ku : n1.kv, k2 = tr ? n2.ku : n2.kv, k = tr ? nd.ku : nd.kv;
  const T* Tr = tr ? I.R + nd.oR : I.W + nd.oW;
  const int kk = k1 + k2;
  T* xs = smem;
  T* red = smem + kk * nc;
  wg_load(k1, nc, I.xh + n1.oxh + (int64_t)c0 * I.ldm, I.ldm, xs, kk);
  wg_load(k2, nc, I.xh + n2.oxh + (int64_t)c0 * I.ldm, I.ldm, xs + k1, kk);
  __syncthreads();
  wg_gemm<T, true>(k, nc, kk, Tr, kk, xs, kk, I.xh + nd.oxh + (int64_t)c0 * I.ldm, I.ldm,
                   false, red);
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_mm_couple(KArgs<T, CallMM<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallMM<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int c0 = blockIdx.y * kRT;
  if (c0 >= C.nrhs) return;
  const int nc = min(kRT, C.nrhs - c0);
  T* red = smem;
  const int64_t co = (int64_t)c0 * I.ldm;
  if (C.op == 0) {
    // y^_c1 = B12 x^_c2 (ku1 x kv2), y^_c2 = B21 x^_c1 (ku2 x kv1)
    wg_gemm<T, false>(n1.ku, nc, n2.kv, I.B12 + nd.oB12, n1.ku, I.xh + n2.oxh + co, I.ldm,
                      I.yh + n1.oyh + co, I.ldm, false, red);
    wg_gemm<T, false>(n2.ku, nc, n1.kv, I.B21 + nd.oB21, n2.ku, I.xh + n1.oxh + co, I.ldm,
                      I.yh + n2.oyh + co, I.ldm, false, red);
  } else {
    // A^T: y^_c1 = B21^T x^_c2 (kv1 x ku2), y^_c2 = B12^T x^_c1 (kv2 x ku1)
    wg_gemm<T, true>(n1.kv, nc, n2.ku, I.B21 + nd.oB21, n2.ku, I.xh + n2.oxh + co, I.ldm,
                     I.yh + n1.oyh + co, I.ldm, false, red);
    wg_gemm<T, true>(n2.kv, nc, n1.ku, I.B12 + nd.oB12, n1.ku, I.xh + n1.oxh + co, I.ldm,
                     I.yh + n2.oyh + co, I.ldm, false, red);
  }
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_mm_down(KArgs<T, CallMM<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallMM<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const NodeInfo n1 = I.nodes[2 * node + 1], n2 = I.nodes[2 * node + 2];
  const int c0 = blockIdx.y * kRT;
  if (c0 >= C.nrhs) return;
  const int nc = min(kRT, C.nrhs - c0);
  const bool tr = C.op != 0;
  const int k1 = tr ? n1.kv : n1.ku, k2 = tr ? n2.kv : n2.ku, k = tr ? nd.kv : nd.ku;
  const T* Tr = tr ? I.W + nd.oW : I.R + nd.oR;
  const int kk = k1 + k2;
  T* ys = smem;
  T* red = smem + k * nc;
  const int64_t co = (int64_t)c0 * I.ldm;
  wg_load(k, nc, I.yh + nd.oyh + co, I.ldm, ys, k);
  __syncthreads();
  // rows 0..k1-1 of Tr go to c1, rows k1..kk-1 to c2
  wg_gemm<T, false>(k1, nc, k, Tr, kk, ys, k, I.yh + n1.oyh + co, I.ldm, true, red);
  wg_gemm<T, false>(k2, nc, k, Tr + k1, kk, ys, k, I.yh + n2.oyh + co, I.ldm, true, red);
}

template <typename T, bool BATCH>
__global__ __launch_bounds__(kNT) void k_mm_leaf_out(KArgs<T, CallMM<T>> a) {
  HIP_DYNAMIC_SHARED(char, smem_raw)
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallMM<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int c0 = blockIdx.y * kRT;
  if (c0 >= C.nrhs) return;
  const int nc = min(kRT, C.nrhs - c0);
  const bool tr = C.op != 0;
  const int m = nd.m;
  T* xs = smem;
  T* red = smem + m * nc;
  wg_load(m, nc, C.X + nd.row0 + (int64_t)c0 * C.ldx, C.ldx, xs, m);
  __syncthreads();
  T* Y = C.Y + nd.row0 + (int64_t)c0 * C.ldy;
  if (tr)
    wg_gemm<T, true>(m, nc, m, I.D + nd.oD, m, xs, m, Y, C.ldy, false, red);
  else
    wg_gemm<T, false>(m, nc, m, I.D + nd.oD, m, xs, m, Y, C.ldy, false, red);
  if (I.p > 0) {
    const int k = tr ? nd.kv : nd.ku;
    const T* basis = tr ? I.V + nd.oV : I.U + nd.oU;
    wg_gemm<T, false>(m, nc, k, basis, m, I.yh + nd.oyh + (int64_t)c0 * I.ldm, I.ldm, Y,
                      C.ldy, true, red);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline size_t mm_smem(int rows, int bytes) {
  return (size_t)(rows * kRT + kNT) * bytes;
}

template <typename T>
void launch_mm_level(MMStep step, const KArgs<T, CallMM<T>>& a, int nblocks, int ytiles,
                     int max_rows, hipStream_t s) {
  if (nblocks <= 0 || ytiles <= 0) return;
  dim3 grid(nblocks, ytiles), block(kNT);
  const size_t sm = mm_smem(max_rows, sizeof(T));
  const bool batch = a.tasks != nullptr;
  static const char* names64[] = {"mm_leaf_up_f64", "mm_up_f64", "mm_couple_f64", "mm_down_f64",
                                  "mm_leaf_out_f64"};
  static const char* names32[] = {"mm_leaf_up_f32", "mm_up_f32", "mm_couple_f32", "mm_down_f32",
                                  "mm_leaf_out_f32"};
  TimedLaunch tl((sizeof(T) == 8 ? names64 : names32)[(int)step], s);
#define HSS_LAUNCH(K)                                                         \
  if (batch) hipLaunchKernelGGL((K<T, true>), grid, block, sm, s, a);         \
  else hipLaunchKernelGGL((K<T, false>), grid, block, sm, s, a);
  switch (step) {
    case MMStep::LeafUp: HSS_LAUNCH(k_mm_leaf_up); break;
    case MMStep::Up: HSS_LAUNCH(k_mm_up); break;
    case MMStep::Couple: HSS_LAUNCH(k_mm_couple); break;
    case MMStep::Down: HSS_LAUNCH(k_mm_down); break;
    case MMStep::LeafOut: HSS_LAUNCH(k_mm_leaf_out); break;
  }
#undef HSS_LAUNCH
}

template void launch_mm_level<double>(MMStep, const KArgs<double, CallMM<double>>&, int, int,
                                      int, hipStream_t);
template void launch_mm_level<float>(MMStep, const KArgs<float, CallMM<float>>&, int, int, int,
                                     hipStream_t);

}  // namespace hss
