// Internal structures shared by the HIP kernels and the host engine.
//
// Device data of one matrix ("instance"):
//   * generators in the canonical packed layout of include/hss.h, FP64 and a
//     resident FP32 copy (same offsets);
//   * a node table (NodeInfo, heap order) with every size and offset the
//     kernels need, so a kernel reads one small record per node;
//   * per-precision factor arrays (Sec. 4.3 Step 1 and the merged levels):
//       FD  mp x mp per node: rows 0..e-1 hold L (lower, diagonal included)
//           and the Householder vectors of the LQ step (right of the
//           diagonal); rows e..mp-1 hold [D~21 | D~22];
//       FU  mp x ku per node: Householder vectors of the QL step above the
//           pivot rows, U~ = the trailing kept rows (lower triangular when e>0);
//       FV  mp x kv per node: Z^T V' (leading e rows V^_top, trailing V^_bot);
//       FZ  mp x e per node: the LQ reflectors again, reflector i as column i
//           (zeros above row i, 1 at row i) for the backward sweep;
//       tq, tz  the Householder scalars; the root block is LU-factored in
//           FP64 (rootLU, piv);
//       FOP (internal nodes with a forward operator, fwd_op_ok) the forward
//           step of the solve as products, one record of kRecSize elements
//           per node laid out as the solve stages it in LDS (see kRec*);
//   * work vectors for the product (x^ up values, y^ down values) and the
//     solve (c, z, y, x^), node blocks stacked with one leading dimension.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hss {

constexpr int kMaxBlock = 128;   // largest leaf / merged block the kernels take
constexpr int kMaxRank = 64;     // largest ku / kv
constexpr int kNT = 256;         // threads per work-group of the per-node kernels
constexpr int kRT = 32;          // right-hand-side columns per work-group tile

struct NodeInfo {
  int64_t row0;    // first row of I_t
  int32_t m;       // |I_t|
  int32_t ku, kv;  // basis ranks (0 at the root)
  int32_t mp;      // size of the block factored at t: leaf m, internal kept_c1 + kept_c2
  int32_t e;       // eliminated rows/cols: max(mp - ku, 0); 0 at the root
  int32_t kept;    // mp - e
  int32_t level;
  int32_t is_leaf;
  // generator offsets (elements); -1 where absent
  int64_t oD, oU, oV, oR, oW, oB12, oB21;
  // product work offsets (rows; capacity max(ku, kv))
  int64_t oxh, oyh;
  // factor offsets (elements)
  int64_t oFD, oFU, oFV, otq, otz, oFZ;
  // forward-operator record offset (elements), -1 where the node has none
  int64_t oOP;
  // solve work offsets (rows): c and x^ have kept rows, z has kv rows, y e rows
  int64_t oc, oz, oy, ox;
};

// Empty-mailbox marker of the one-rhs product: signalling NaNs, which no
// arithmetic produces, so a mailbox entry is either this or a written value.
constexpr uint64_t kMbEmpty64 = 0x7FF4A5A5A5A5A5A5ull;
constexpr uint32_t kMbEmpty32 = 0x7FA5A5A5u;
constexpr int kMbSlot = 32;   // mailbox entries per node and right-hand side
constexpr int kMbCols = 8;    // right-hand sides per work-group of the mailbox product
constexpr int kMbChunks = 4;  // column chunks of kMbCols one product launch takes side by
                              // side, each with its own arrival counters and mailboxes
// Status bit (1 << code) set by a kernel whose bounded wait for another
// work-group ran out; the code is HSS_EHIP.
constexpr int kStatusWaitCode = 2;
// Device status block of an instance (int32 entries): [0] status bits
// (1 << HSS_ESINGULAR, 1 << kStatusWaitCode), [1] 1 + the largest heap id of a
// node with an exact zero pivot (0 if none), [2] refinement gate (1 while
// the next correction is to run), [3] refinement steps taken.
constexpr int kStatusWords = 4;
constexpr int kCodeSingular = 4;   // HSS_ESINGULAR
constexpr int kCodeNoConv = 5;     // HSS_ENOCONV
constexpr int kStSingularNode = 1;
constexpr int kStGate = 2;
constexpr int kStIters = 3;

template <typename T>
struct Inst {
  const NodeInfo* nodes;
  const T *D, *U, *V, *R, *W, *B12, *B21;
  T *FD, *FU, *FV, *tq, *tz, *FZ;
  T* FOP;           // forward-operator records (internal nodes that have them)
  double* rootLU;
  int32_t* piv;     // root LU: mp interchanges, then the permutation they make (mp)
  T *xh, *yh;       // product work, leading dimension ldm
  int64_t ldm;
  T *wc, *wz, *wy, *wx;   // solve work, leading dimension lds
  int64_t lds;
  int32_t* status;  // device status word (HSS_ESINGULAR ...)
  uint32_t* cnt;    // per-node arrival counters of the fused product (even between calls)
  T* mb;            // per-node x^ mailboxes of the one-rhs product (32 entries, empty = kMbEmpty)
  int32_t p;
  int32_t nnodes;
};

// Whether an internal node's forward step is precomputed as products (FY,
// FF): every operand fits a 32 x 32 block of the matrix-core kernels (the
// node's ranks and eliminated count, and its children's ranks, at most 32;
// child_k is the largest of ku_c1, kv_c1, ku_c2, kv_c2).
__host__ __device__ inline bool fwd_op_ok(int is_leaf, int node, int mp, int e, int ku, int kv,
                                          int child_k) {
  return !is_leaf && node != 0 && e > 0 && e <= 32 && mp <= 64 && ku <= 32 && kv <= 32 &&
         child_k <= 32;
}

// Forward-operator record of an internal node (elements; every block at a
// 16-byte boundary, unused rows and columns zero):
//   G  = [[0, U~_c1 B12], [U~_c2 B21, 0]]  mp x (kv_c1 + kv_c2), pitch 64:
//        rhs = [c_c1; c_c2] - G [z_c1; z_c2];
//   W  = W_t                               (kv_c1 + kv_c2) x kv, pitch 65;
//   Y  = the QL reflectors with their unit pivots, mp x ku, pitch 65, and
//   YT = Y T (compact WY: Q^T = I - Y T Y^T), mp x ku, pitch 64:
//        b~ = rhs - YT (Y^T rhs);
//   F  = [L^-1; D~21 L^-1; V^_top^T L^-1]  (e + kept + kv) x e, pitch 96:
//        [y; d; v] = F b~(0:e), c = b~(e:) - d, z = v + W^T [z_c1; z_c2].
constexpr int kRecG = 0;
constexpr int kRecW = kRecG + 64 * 64;
constexpr int kRecY = kRecW + 65 * 32;
constexpr int kRecYT = kRecY + 65 * 32;
constexpr int kRecF = kRecYT + 64 * 32;
constexpr int kRecSize = kRecF + 96 * 32;
static_assert(kRecW % 4 == 0 && kRecY % 4 == 0 && kRecYT % 4 == 0 && kRecF % 4 == 0 &&
                  kRecSize % 4 == 0, "record blocks at 16-byte boundaries");

// gate: NULL, or a device flag read when a work-group starts; 0 makes the
// call's work-groups return at once (refinement steps enqueued after the
// backward error has met its tolerance).
template <typename T>
struct CallMM {
  const T* X;
  T* Y;
  int64_t ldx, ldy;
  int32_t nrhs;
  int32_t op;
  const int32_t* gate;
};

template <typename T>
struct CallSV {
  T* B;           // right-hand sides / solution in precision T
  int64_t ldb;
  int32_t nrhs;
  int32_t pad;
  const int32_t* gate;
};

__device__ __forceinline__ bool gated_off(const int32_t* gate) {
  return gate != nullptr && *gate == 0;
}

// Kernel argument bundle: single-instance launches pass the instance and the
// call by value and address nodes node0 + blockIdx.x; batched launches pass
// device arrays and a task list of (instance, node) pairs.
template <typename T, typename Call>
struct KArgs {
  Inst<T> inst;
  Call call;
  const Inst<T>* insts;
  const Call* calls;
  const int2* tasks;
  int32_t node0;
  int32_t ntasks;
  int32_t flags;   // kernel-specific options (root solve: bit 0 = children staged in LDS)
  int32_t cpw;     // solve sweeps: right-hand-side columns per wavefront (0: by the count)
};

}  // namespace hss
