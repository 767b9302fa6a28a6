// Step 1 of the ULV factorization (Sec. 4.3) on one level of blocks, with the
// working matrices resident in registers:
//   QL of U' (Householder, pivot rows at the bottom): Q^T U' = [0; U~], and
//   M = Q^T D'  -- column-owned: every (column, half) pair of lanes holds half
//                  a column of [D' | U'] in registers;
//   LQ of the leading e rows of M: M Z = [[L, 0], [D~21, D~22]], and
//   V^T <- V'^T Z (i.e. V^ = Z^T V')  -- row-owned: every (row, half) pair of
//                  lanes holds half a row of [M; V'^T] in registers.
// One Householder step: the owner pair publishes its column / row in LDS, the
// owner's wavefront forms the reflector with two elements per lane and parks
// the finished column / row in LDS, one barrier, then every other pair applies
// the reflector with a dot product over its registers and one lane exchange.
// The two layouts are swapped once through LDS.
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace hss {

// threads of a work-group: 2 MAXC owner slots (columns of [D' U'], rows of
// [M; V'^T]) x 2 halves
template <int MAXC>
constexpr int fnt() { return 4 * MAXC; }

// reg <- reg - tau (v . reg_pair) v on the half vector this lane holds; the
// dot product of the lane pair is combined with one lane exchange and runs on
// four independent partial sums (a single chain of dependent FMAs would leave
// the VALU waiting on its own latency).
template <typename T, int COLS>
__device__ __forceinline__ void apply_reflector(const T* v, T (&reg)[COLS], T tau) {
  T p[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int j = 0; j < COLS; ++j) p[j & 3] += v[j] * reg[j];
  T w = (p[0] + p[1]) + (p[2] + p[3]);
  w += xor1(w);
  w *= tau;
#pragma unroll
  for (int j = 0; j < COLS; ++j) reg[j] -= w * v[j];
}

template <typename T, int MAXC, bool BATCH>
__global__ __launch_bounds__(fnt<MAXC>()) void k_ulv_factor_reg(KArgs<T, CallSV<T>> a) {
  constexpr int kFNT = fnt<MAXC>();
  constexpr int COLS = MAXC / 2;
  constexpr int VB = MAXC + 8;
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];   // 16-byte aligned: vector LDS reads
  T* smem = reinterpret_cast<T*>(smem_raw);
  Inst<T> I; CallSV<T> C; int node;
  resolve<BATCH>(a, I, C, node);
  const NodeInfo nd = I.nodes[node];
  const int mp = nd.mp, ku = nd.ku, kv = nd.kv, e = nd.e;
  const int tid = threadIdx.x;
  const int idx = tid >> 1, s = tid & 1;
  const int lane = tid & 63, wave = tid >> 6;
  const int base = s * COLS;
  const int ldm = mp + 1;
  T* Ms = smem;                           // MAXC x (MAXC+1): U~ park, swap buffer, finished rows
  T* vbuf = Ms + MAXC * (MAXC + 1);       // 2 reflector buffers (v, then tau at [MAXC])
  T* pub = vbuf + 2 * VB;                 // the owner's published column / row (MAXC)
  T* taus = pub + MAXC;                   // tau_Q (kMaxRank) then tau_Z (MAXC)
  __shared__ int sing;
  if (tid == 0) sing = 0;
  T* FU = I.FU + nd.oFU;
  T* FV = I.FV + nd.oFV;
  T* FD = I.FD + nd.oFD;
  T* FZ = I.FZ + nd.oFZ;
  const T* Dsrc = nd.is_leaf ? I.D + nd.oD : FD;
  const T* Usrc = nd.is_leaf ? I.U + nd.oU : FU;
  const T* Vsrc = nd.is_leaf ? I.V + nd.oV : FV;
  T reg[COLS];
  const int r0 = lane, r1 = lane + 64;   // the two elements of a lane in owner-wave work

  // ---- column-owned: slot c < mp is column c of D', mp <= c < mp+ku column c-mp of U'
  const int c = idx;
  const bool isD = c < mp;
  const bool isU = c >= mp && c < mp + ku;
  {
    // clamped addresses, unconditional loads (all in flight together), masks after
    const T* src = isD ? Dsrc + (int64_t)c * mp : (isU ? Usrc + (int64_t)(c - mp) * mp : Dsrc);
    const bool any = isD | isU;
    if (base + COLS <= mp) {   // whole half in range: constant offsets from one address
#pragma unroll
      for (int j = 0; j < COLS; ++j) reg[j] = ld_or0(src + base + j, any);
    } else {
#pragma unroll
      for (int j = 0; j < COLS; ++j) {
        const int r = base + j;
        reg[j] = ld_or0(src + min(r, mp - 1), any & (r < mp));
      }
    }
  }
  if (e > 0) {
    for (int jq = ku - 1; jq >= 0; --jq) {
      const int pr = e + jq;
      const int owner = mp + jq;
      T* vb = vbuf + (jq & 1) * VB;
      if (c == owner) {
#pragma unroll
        for (int j = 0; j < COLS; ++j) pub[base + j] = reg[j];
      }
      wave_lds_sync();
      if (wave == (2 * owner) >> 6) {
        const T x0 = pub[r0];
        const T x1 = MAXC > 64 ? pub[r1] : T(0);
        const T sig = wave_sum((r0 < pr ? x0 * x0 : T(0)) + (r1 < pr ? x1 * x1 : T(0)));
        const T al = pub[pr];
        T beta, tau, scale;
        householder_fast(al, sig, beta, tau, scale);
        const T v0 = r0 < pr ? x0 * scale : (r0 == pr ? T(1) : T(0));
        const T v1 = r1 < pr ? x1 * scale : (r1 == pr ? T(1) : T(0));
        vb[r0] = v0;
        if (MAXC > 64) vb[r1] = v1;
        // finished column jq of U': reflector above the pivot, beta, U~ below
        if (r0 < mp) Ms[r0 + jq * mp] = r0 < pr ? v0 : (r0 == pr ? beta : x0);
        if (MAXC > 64 && r1 < mp) Ms[r1 + jq * mp] = r1 < pr ? v1 : (r1 == pr ? beta : x1);
        if (lane == 0) {
          vb[MAXC] = tau;
          taus[jq] = tau;
        }
      }
      __syncthreads();
      const T tau = vb[MAXC];
      if (tau != T(0) && (isD || (c >= mp && c < owner))) apply_reflector<T, COLS>(vb + base, reg, tau);
    }
    __syncthreads();
    for (int o = tid; o < mp * ku; o += kFNT) FU[o] = Ms[o];
    if (tid < ku) I.tq[nd.otq + tid] = taus[tid];
  } else if (isU) {
    T* dst = FU + (int64_t)(c - mp) * mp;
#pragma unroll
    for (int j = 0; j < COLS; ++j)
      if (base + j < mp) dst[base + j] = reg[j];
  }
  __syncthreads();
  // ---- swap layouts: M = Q^T D' through LDS
  if (isD) {
#pragma unroll
    for (int j = 0; j < COLS; ++j)
      if (base + j < mp) Ms[base + j + c * ldm] = reg[j];
  }
  __syncthreads();
  // ---- row-owned: slot r < mp is row r of M, mp <= r < mp+kv row r-mp of V'^T
  const int r = idx;
  const bool isM = r < mp;
  const bool isV = r >= mp && r < mp + kv;
  if (isM) {
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
      const int cc = base + j;
      const T v = Ms[r + min(cc, mp - 1) * ldm];
      reg[j] = cc < mp ? v : T(0);
    }
  } else {
    const T* src = Vsrc + (int64_t)(isV ? r - mp : 0) * mp;
    if (base + COLS <= mp) {
#pragma unroll
      for (int j = 0; j < COLS; ++j) reg[j] = ld_or0(src + base + j, isV);
    } else {
#pragma unroll
      for (int j = 0; j < COLS; ++j) {
        const int cc = base + j;
        reg[j] = ld_or0(src + min(cc, mp - 1), isV & (cc < mp));
      }
    }
  }
  __syncthreads();   // Ms now parks the finished rows 0..e-1
  for (int i = 0; i < e; ++i) {
    T* vb = vbuf + (i & 1) * VB;
    if (r == i) {
#pragma unroll
      for (int j = 0; j < COLS; ++j) pub[base + j] = reg[j];
    }
    wave_lds_sync();
    if (wave == (2 * i) >> 6) {
      const T x0 = pub[r0];
      const T x1 = MAXC > 64 ? pub[r1] : T(0);
      const T sig = wave_sum((r0 > i && r0 < mp ? x0 * x0 : T(0)) +
                             (r1 > i && r1 < mp ? x1 * x1 : T(0)));
      const T al = pub[i];
      T beta, tau, scale;
      householder_fast(al, sig, beta, tau, scale);
      const T v0 = r0 > i ? x0 * scale : (r0 == i ? T(1) : T(0));
      const T v1 = r1 > i ? x1 * scale : (r1 == i ? T(1) : T(0));
      vb[r0] = v0;
      if (MAXC > 64) vb[r1] = v1;
      // finished row i: L part, beta on the diagonal, the reflector to the right
      if (r0 < mp) Ms[i + r0 * ldm] = r0 < i ? x0 : (r0 == i ? beta : v0);
      if (MAXC > 64 && r1 < mp) Ms[i + r1 * ldm] = r1 < i ? x1 : (r1 == i ? beta : v1);
      if (lane == 0) {
        vb[MAXC] = tau;
        taus[kMaxRank + i] = tau;
        if (beta == T(0)) sing = 1;
      }
    }
    __syncthreads();
    const T tau = vb[MAXC];
    if (tau != T(0) && r > i && (isM || isV)) apply_reflector<T, COLS>(vb + base, reg, tau);
  }
  __syncthreads();
  if (tid < e) I.tz[nd.otz + tid] = taus[kMaxRank + tid];
  if (tid == 0 && sing) {
    atomicOr(I.status, 1 << kCodeSingular);
    atomicMax(I.status + kStSingularNode, node + 1);
  }
  // rows 0..e-1 (parked) -> FD and, as columns, FZ
  for (int o = tid; o < e * mp; o += kFNT) {
    const int i = o % e, cc = o / e;
    FD[i + (int64_t)cc * mp] = Ms[i + cc * ldm];
  }
  for (int o = tid; o < e * mp; o += kFNT) {
    const int cc = o % mp, i = o / mp;
    FZ[o] = cc > i ? Ms[i + cc * ldm] : (cc == i ? T(1) : T(0));
  }
  if (isM && r >= e) {
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
      const int cc = base + j;
      if (cc < mp) FD[r + (int64_t)cc * mp] = reg[j];
    }
  } else if (isV) {
    T* dst = FV + (int64_t)(r - mp) * mp;
#pragma unroll
    for (int j = 0; j < COLS; ++j)
      if (base + j < mp) dst[base + j] = reg[j];
  }
}

template <typename T>
void launch_factor_reg(const KArgs<T, CallSV<T>>& a, int nblocks, int max_mp, hipStream_t s) {
  if (nblocks <= 0) return;
  const bool batch = a.tasks != nullptr;
  dim3 grid(nblocks);
#define HSS_FLAUNCH(MC)                                                                      \
  {                                                                                          \
    const size_t sm = ((size_t)MC * (MC + 1) + 2 * (MC + 8) + MC + kMaxRank + MC) * sizeof(T); \
    const dim3 block(fnt<MC>());                                                             \
    if (batch) hipLaunchKernelGGL((k_ulv_factor_reg<T, MC, true>), grid, block, sm, s, a);    \
    else hipLaunchKernelGGL((k_ulv_factor_reg<T, MC, false>), grid, block, sm, s, a);        \
  }
  if (max_mp <= 64) HSS_FLAUNCH(64) else HSS_FLAUNCH(128)
#undef HSS_FLAUNCH
}

template void launch_factor_reg<double>(const KArgs<double, CallSV<double>>&, int, int,
                                        hipStream_t);
template void launch_factor_reg<float>(const KArgs<float, CallSV<float>>&, int, int, hipStream_t);

}  // namespace hss
