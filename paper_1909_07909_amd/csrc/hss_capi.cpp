// C ABI of the HSS library (include/hss.h): handle management, launch
// schedules over the tree levels, iterative refinement and the power-method
// norm estimate.  All arithmetic runs in the HIP kernels; this file only
// plans, allocates and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <string>
#include <vector>

#include "../../include/hss.h"
#include "hss_internal.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace hss;

namespace {

template <typename T>
struct FactorSet {
  T *FD = nullptr, *FU = nullptr, *FV = nullptr, *tq = nullptr, *tz = nullptr, *FZ = nullptr;
  T* FOP = nullptr;
  double* rootLU = nullptr;
  int32_t* piv = nullptr;
  bool valid = false;
};

template <typename T>
struct Work {
  T *xh = nullptr, *yh = nullptr;     // product
  T* mb = nullptr;                    // one-rhs product mailboxes (kMbSlot per node)
  int64_t cap_mm = 0;
  T *wc = nullptr, *wz = nullptr, *wy = nullptr, *wx = nullptr;   // solve
  int64_t cap_sv = 0;
};

}  // namespace

static_assert(kStatusWaitCode == HSS_EHIP, "status bit of a run-out wait");

struct hss_handle {
  Plan plan;
  hss_alloc alloc{};
  bool custom_alloc = false;
  std::vector<std::pair<void*, size_t>> blocks;   // everything we allocated
  int64_t resident = 0;
  NodeInfo* d_nodes = nullptr;
  double* g64[7] = {};
  float* g32[7] = {};
  FactorSet<double> f64;
  FactorSet<float> f32;
  Work<double> w64;
  Work<float> w32;
  int32_t* d_status = nullptr;
  uint32_t* d_cnt = nullptr;   // arrival counters of the fused product, one per node and column chunk
  // refinement / norm work
  double *b0 = nullptr, *res = nullptr, *d64 = nullptr;
  float* r32 = nullptr;
  int64_t cap_ir = 0;
  double* stats = nullptr;   // 8 * cap_stats doubles
  int64_t cap_stats = 0;
  double* part = nullptr;    // partials of the fused check kernels (check_partials(cap_stats))
  uint32_t* chk_cnt = nullptr;   // their arrival counter (0 between launches)
  double norm2 = -1.0;
  // second stream of the product: the leaves' D X runs on it beside the
  // up and down kernels (forked from and joined back to the caller's stream)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace {

hss_status hip_status(hipError_t e) { return e == hipSuccess ? HSS_OK : HSS_EHIP; }

void* dev_alloc(hss_handle* h, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (h->custom_alloc) {
    p = h->alloc.alloc(bytes, h->alloc.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) {
    h->blocks.emplace_back(p, bytes);
    h->resident += (int64_t)bytes;
  }
  return p;
}

void dev_free(hss_handle* h, void* p) {
  if (!p) return;
  for (size_t i = 0; i < h->blocks.size(); ++i)
    if (h->blocks[i].first == p) {
      h->resident -= (int64_t)h->blocks[i].second;
      h->blocks.erase(h->blocks.begin() + i);
      break;
    }
  if (h->custom_alloc) h->alloc.free(p, h->alloc.ctx);
  else (void)hipFree(p);
}

template <typename T>
T* dalloc(hss_handle* h, int64_t n) {
  return static_cast<T*>(dev_alloc(h, sizeof(T) * (size_t)std::max<int64_t>(n, 1)));
}

template <typename T>
FactorSet<T>& factors(hss_handle* h);
template <>
FactorSet<double>& factors<double>(hss_handle* h) { return h->f64; }
template <>
FactorSet<float>& factors<float>(hss_handle* h) { return h->f32; }
template <typename T>
Work<T>& work(hss_handle* h);
template <>
Work<double>& work<double>(hss_handle* h) { return h->w64; }
template <>
Work<float>& work<float>(hss_handle* h) { return h->w32; }
template <typename T>
const T* gen(hss_handle* h, int i);
template <>
const double* gen<double>(hss_handle* h, int i) { return h->g64[i]; }
template <>
const float* gen<float>(hss_handle* h, int i) { return h->g32[i]; }

template <typename T>
hss_status ensure_factors(hss_handle* h) {
  FactorSet<T>& F = factors<T>(h);
  if (F.FD) return HSS_OK;
  const Plan& P = h->plan;
  F.FD = dalloc<T>(h, P.nFD);
  F.FU = dalloc<T>(h, P.nFU);
  F.FV = dalloc<T>(h, P.nFV);
  F.tq = dalloc<T>(h, P.ntq);
  F.tz = dalloc<T>(h, P.ntz);
  F.FZ = dalloc<T>(h, P.nFZ);
  F.FOP = dalloc<T>(h, sizeof(T) == 4 ? P.nOP : 0);
  F.rootLU = dalloc<double>(h, (int64_t)P.nodes[0].mp * P.nodes[0].mp);
  F.piv = dalloc<int32_t>(h, 2 * (int64_t)P.nodes[0].mp);   // interchanges, then the permutation
  if (!F.FD || !F.FU || !F.FV || !F.tq || !F.tz || !F.FZ || !F.FOP || !F.rootLU || !F.piv)
    return HSS_ENOMEM;
  return HSS_OK;
}

// Work buffers grow to the widest call so far.  The buffers they replace are
// not freed before hss_destroy: a HIP graph captured from an earlier call
// still holds their addresses.  Growth is geometric (at least doubling, in
// multiples of 8 columns), so the retired buffers never add up to more than
// the live ones.
int64_t grown_cap(int64_t old_cap, int64_t nrhs, int64_t min_cap) {
  const int64_t want = std::max<int64_t>((nrhs + 7) / 8 * 8, min_cap);
  return old_cap > 0 ? std::max<int64_t>(want, 2 * old_cap) : want;
}

template <typename T>
hss_status ensure_work_mm(hss_handle* h, int64_t nrhs) {
  Work<T>& w = work<T>(h);
  if (w.cap_mm >= nrhs && w.xh) return HSS_OK;
  const int64_t cap = grown_cap(w.xh ? w.cap_mm : 0, nrhs, kRT);
  w.xh = dalloc<T>(h, h->plan.ldm * cap);
  w.yh = dalloc<T>(h, h->plan.ldm * cap);
  w.cap_mm = (w.xh && w.yh) ? cap : 0;
  return w.cap_mm ? HSS_OK : HSS_ENOMEM;
}

template <typename T>
hss_status ensure_work_sv(hss_handle* h, int64_t nrhs) {
  Work<T>& w = work<T>(h);
  if (w.cap_sv >= nrhs && w.wc) return HSS_OK;
  const int64_t cap = grown_cap(w.wc ? w.cap_sv : 0, nrhs, kRT);
  const int64_t sz = h->plan.lds * cap;
  w.wc = dalloc<T>(h, sz);
  w.wz = dalloc<T>(h, sz);
  w.wy = dalloc<T>(h, sz);
  w.wx = dalloc<T>(h, sz);
  w.cap_sv = (w.wc && w.wz && w.wy && w.wx) ? cap : 0;
  return w.cap_sv ? HSS_OK : HSS_ENOMEM;
}

hss_status ensure_ir(hss_handle* h, int64_t nrhs) {
  nrhs = std::max<int64_t>(nrhs, 1);
  if (h->cap_ir < nrhs || !h->b0) {
    const int64_t cap = grown_cap(h->b0 ? h->cap_ir : 0, nrhs, 1);
    const int64_t n = h->plan.n;
    h->b0 = dalloc<double>(h, n * cap);
    h->res = dalloc<double>(h, n * cap);
    h->d64 = dalloc<double>(h, n * cap);
    h->r32 = dalloc<float>(h, n * cap);
    h->cap_ir = (h->b0 && h->res && h->d64 && h->r32) ? cap : 0;
    if (!h->cap_ir) return HSS_ENOMEM;
  }
  if (h->cap_stats < nrhs || !h->stats) {
    const int64_t cap = grown_cap(h->stats ? h->cap_stats : 0, nrhs, 1);
    h->stats = dalloc<double>(h, 8 * cap + 8);
    h->part = dalloc<double>(h, check_partials(cap));
    h->cap_stats = (h->stats && h->part) ? cap : 0;
    if (!h->cap_stats) return HSS_ENOMEM;
  }
  return HSS_OK;
}

// Work sets an instance record carries: the product's (x^, y^, mailboxes)
// and the solve's (c, z, y, x).  A batched call's device table holds only the
// set its kernels read, so it does not change when another call grows the
// other set (a table equal to an earlier one is reused, also under capture).
constexpr int kUseMM = 1, kUseSV = 2;

template <typename T>
Inst<T> make_inst(hss_handle* h, int uses = kUseMM | kUseSV) {
  Inst<T> I{};
  I.nodes = h->d_nodes;
  I.D = gen<T>(h, 0); I.U = gen<T>(h, 1); I.V = gen<T>(h, 2); I.R = gen<T>(h, 3);
  I.W = gen<T>(h, 4); I.B12 = gen<T>(h, 5); I.B21 = gen<T>(h, 6);
  FactorSet<T>& F = factors<T>(h);
  I.FD = F.FD; I.FU = F.FU; I.FV = F.FV; I.tq = F.tq; I.tz = F.tz; I.FZ = F.FZ;
  I.FOP = F.FOP;
  I.rootLU = F.rootLU; I.piv = F.piv;
  Work<T>& w = work<T>(h);
  if (uses & kUseMM) {
    I.xh = w.xh; I.yh = w.yh; I.ldm = h->plan.ldm;
    I.mb = w.mb;
  }
  if (uses & kUseSV) {
    I.wc = w.wc; I.wz = w.wz; I.wy = w.wy; I.wx = w.wx; I.lds = h->plan.lds;
  }
  I.status = h->d_status;
  I.cnt = h->d_cnt;
  I.p = h->plan.p;
  I.nnodes = h->plan.nnodes;
  return I;
}

inline int level_first(int l) { return (1 << l) - 1; }

// Forward-operator records (FOP) are built by the FP32 factorization, whose
// solves run at least twice per refined solve; an FP64 factorization is
// usually solved once, and its solves keep the sequential forward steps.
template <typename T>
bool use_fwd_op(const Plan& P) {
  return sizeof(T) == 4 && P.nOP > 0;
}

// ---------------------------------------------------------------------------
// Single-instance schedules
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Tuned launch choices (hss_autotune): per shape class of a matrix (leaf
// block size, largest rank, depth), precision and right-hand-side bucket,
// the product's kernel family and the solve sweeps' columns per wavefront
// that measured fastest.  Process-wide; calls without an entry use the
// default rules.  While the tuner times a variant it forces it through the
// thread-local overrides.
struct TuneKey {
  int leaf_mp, max_k, p, prec, bucket;
  bool operator<(const TuneKey& o) const {
    return std::tie(leaf_mp, max_k, p, prec, bucket) <
           std::tie(o.leaf_mp, o.max_k, o.p, o.prec, o.bucket);
  }
};
struct TuneVal {
  int mm = -1;    // product: 1 per-level wide kernels, 0 mailbox kernels, -1 default
  int cpw = 0;    // solve sweeps: columns per wavefront (1 or 4), 0 default
  double t_mm[2] = {0, 0}, t_sv[2] = {0, 0};   // measured us (mailbox, wide; cpw 1, 4)
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
thread_local int g_force_mm = -1;
thread_local int g_force_cpw = 0;

int rhs_bucket(int64_t n) { return n <= 1 ? 0 : n < 4 ? 1 : n < 8 ? 2 : n < 16 ? 3 : n < 32 ? 4 : 5; }
TuneKey tune_key(const Plan& P, int prec, int64_t nrhs) {
  return TuneKey{P.level_max_mp[P.p], P.max_k, P.p, prec, rhs_bucket(nrhs)};
}
bool tune_lookup(const Plan& P, int prec, int64_t nrhs, TuneVal* v) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(tune_key(P, prec, nrhs));
  if (it == g_tune.end()) return false;
  *v = it->second;
  return true;
}

// Which products run the per-level wide kernels (leaves <= 128, ranks <= 32)
// rather than the mailbox kernels: a single matrix from kMmwFromCols columns
// on (below that the mailbox climb is faster: 297 against 349 us at 8
// columns on the n = 2^18 matrix), a batch from kMmwBatchFromCols (many small
// trees: the per-level launches are 1.5x faster at 8 columns).
constexpr int kMmwFromCols = kMbCols + 1;
constexpr int kMmwBatchFromCols = 2;
inline bool use_mmw(int p, int64_t nrhs, int leaf_mp, int max_k, int from = kMmwFromCols) {
  return p > 0 && nrhs >= from && mmw_fits(leaf_mp, max_k);
}

template <typename T>
void run_matmul(hss_handle* h, int op, int64_t nrhs, const T* X, int64_t ldx, T* Y, int64_t ldy,
                hipStream_t s, const int32_t* gate = nullptr, T* xh = nullptr, T* yh = nullptr) {
  KArgs<T, CallMM<T>> a{};
  a.inst = make_inst<T>(h);
  if (xh) {
    // caller-provided x^ / y^ work vectors (leading dimension ldm)
    a.inst.xh = xh;
    a.inst.yh = yh;
  }
  a.call = CallMM<T>{X, Y, ldx, ldy, (int32_t)nrhs, op, gate};
  const int p = h->plan.p;
  if (op == HSS_OP_N) {
    // fused: leaves (with the climb), subtree walks, leaf outputs
    const int mku = h->plan.leaf_max_ku, mk = h->plan.max_k;
    if (p > 0 && nrhs == 1 && mk <= 32) {
      // one launch for the up pass and the leaves' D X (their blocks start as
      // the subtree blocks finish their leaves), then the down pass, then U y^
      const int lu = std::max(p - mmf_up_height(), 0);
      a.node0 = level_first(lu);
      launch_mmf<T>(MMFStep::UpDX, a, 1 << lu, (int)nrhs, mku, mk, s);
      const int ls = std::max(p - mmf_down_height(), 0);
      a.node0 = level_first(ls);
      launch_mmf<T>(MMFStep::Down, a, 1 << ls, (int)nrhs, mku, mk, s);
      a.node0 = level_first(p);
      launch_mmf<T>(MMFStep::LeafUY, a, 1 << p, (int)nrhs, mku, mk, s);
      return;
    }
    bool wide = use_mmw(p, nrhs, h->plan.level_max_mp[p], mk);
    if (p > 0 && nrhs >= 2 && mmw_fits(h->plan.level_max_mp[p], mk)) {
      TuneVal tv;
      if (g_force_mm >= 0) wide = g_force_mm == 1;
      else if (tune_lookup(h->plan, sizeof(T) == 8 ? HSS_F64 : HSS_F32, nrhs, &tv) && tv.mm >= 0)
        wide = tv.mm == 1;
    }
    if (wide) {
      // wide blocks: one launch per level
      a.node0 = level_first(p);
      launch_mmw<T>(MMWStep::LeafUp, a, 1 << p, (int)nrhs, s, h->plan.level_max_mp[p]);
      for (int l = p - 1; l >= 0; --l) {
        a.node0 = level_first(l);
        launch_mmw<T>(MMWStep::Up, a, 1 << l, (int)nrhs, s);
      }
      for (int l = 1; l <= p - 1; ++l) {
        a.node0 = level_first(l);
        launch_mmw<T>(MMWStep::Down, a, 1 << l, (int)nrhs, s);
      }
      a.node0 = level_first(p);
      launch_mmw<T>(MMWStep::LeafOut, a, 1 << p, (int)nrhs, s, h->plan.level_max_mp[p]);
      return;
    }
    if (p > 0) {
      // D X on the side stream, beside the up and down passes; U y^ after both
      const bool fork = h->side != nullptr &&
                        hipEventRecord(h->ev_fork, s) == hipSuccess &&
                        hipStreamWaitEvent(h->side, h->ev_fork, 0) == hipSuccess;
      const int lu = std::max(p - mmf_up_height(), 0);
      a.node0 = level_first(lu);
      launch_mmf<T>(MMFStep::Up, a, 1 << lu, (int)nrhs, mku, mk, s);
      if (fork) {
        a.node0 = level_first(p);
        launch_mmf<T>(MMFStep::LeafDX, a, 1 << p, (int)nrhs, mku, mk, h->side);
        (void)hipEventRecord(h->ev_join, h->side);
      }
      const int ls = std::max(p - mmf_down_height(), 0);
      a.node0 = level_first(ls);
      launch_mmf<T>(MMFStep::Down, a, 1 << ls, (int)nrhs, mku, mk, s);
      if (fork) {
        (void)hipStreamWaitEvent(s, h->ev_join, 0);
        a.node0 = level_first(p);
        launch_mmf<T>(MMFStep::LeafUY, a, 1 << p, (int)nrhs, mku, mk, s);
        return;
      }
    }
    a.node0 = level_first(p);
    launch_mmf<T>(MMFStep::Leaf, a, 1 << p, (int)nrhs, mku, mk, s);
    return;
  }
  const int yt = (int)((nrhs + kRT - 1) / kRT);
  const int rows = kMaxBlock;
  if (p == 0) {
    a.node0 = 0;
    launch_mm_level<T>(MMStep::LeafOut, a, 1, yt, rows, s);
    return;
  }
  a.node0 = level_first(p);
  launch_mm_level<T>(MMStep::LeafUp, a, 1 << p, yt, rows, s);
  for (int l = p - 1; l >= 1; --l) {
    a.node0 = level_first(l);
    launch_mm_level<T>(MMStep::Up, a, 1 << l, yt, rows, s);
  }
  a.node0 = 0;
  launch_mm_level<T>(MMStep::Couple, a, (1 << p) - 1, yt, rows, s);
  for (int l = 1; l <= p - 1; ++l) {
    a.node0 = level_first(l);
    launch_mm_level<T>(MMStep::Down, a, 1 << l, yt, rows, s);
  }
  a.node0 = level_first(p);
  launch_mm_level<T>(MMStep::LeafOut, a, 1 << p, yt, rows, s);
}

// on_level(l): called once the factors of level l (leaves: l = p) are
// enqueued on s, before the next level's launches.
template <typename T, typename F>
void run_factor(hss_handle* h, hipStream_t s, F&& on_level) {
  KArgs<T, CallSV<T>> a{};
  a.inst = make_inst<T>(h);
  const Plan& P = h->plan;
  const int p = P.p;
  if (p == 0) {
    a.node0 = 0;
    launch_ulv<T>(UlvStep::RootLU, a, 1, P.max_k, P.max_mp, s);
    return;
  }
  a.node0 = level_first(p);
  launch_ulv<T>(UlvStep::Factor, a, 1 << p, P.max_k, P.level_max_mp[p], s);
  on_level(p);
  for (int l = p - 1; l >= 1; --l) {
    a.node0 = level_first(l);
    launch_ulv<T>(UlvStep::Merge, a, 1 << l, P.max_k, P.level_max_mp[l], s);
    launch_ulv<T>(UlvStep::Factor, a, 1 << l, P.max_k, P.level_max_mp[l], s);
    if (use_fwd_op<T>(P)) launch_ulv<T>(UlvStep::FwdOp, a, 1 << l, P.max_k, P.level_max_mp[l], s);
    on_level(l);
  }
  a.node0 = 0;
  launch_ulv<T>(UlvStep::Merge, a, 1, P.max_k, P.nodes[0].mp, s);
  launch_ulv<T>(UlvStep::RootLU, a, 1, P.max_k, P.nodes[0].mp, s);
}

template <typename T>
void run_factor(hss_handle* h, hipStream_t s) {
  run_factor<T>(h, s, [](int) {});
}

// LDS bytes a work-group may use for staged copies of one node's factors.
constexpr int64_t kStageBudget = 120 * 1024;

// One solve's launch schedule: its kernel arguments and LDS budgets.
template <typename T>
struct SolveSched {
  KArgs<T, CallSV<T>> a{};
  int nc = 0;
  int64_t root_elems = 0;
};

template <typename T>
SolveSched<T> solve_sched(hss_handle* h, int64_t nrhs, T* B, int64_t ldb, const int32_t* gate) {
  SolveSched<T> S;
  S.a.inst = make_inst<T>(h);
  S.a.call = CallSV<T>{B, ldb, (int32_t)nrhs, 0, gate};
  S.nc = (int)nrhs;
  const Plan& P = h->plan;
  const int p = P.p;
  // columns per wavefront: tuned (or forced by the tuner), else the default
  {
    TuneVal tv;
    if (g_force_cpw > 0) S.a.cpw = g_force_cpw;
    else if (nrhs >= 4 && tune_lookup(P, sizeof(T) == 8 ? HSS_F64 : HSS_F32, nrhs, &tv))
      S.a.cpw = tv.cpw;
  }
  // root: FP64 LU + pivots (+ the children's blocks when everything fits in LDS)
  const int64_t mpr = P.nodes[0].mp;
  int64_t root_bytes = mpr * mpr * 8 + 4 * ((mpr + 3) & ~int64_t(3));
  const int64_t child_bytes = p > 0 ? P.level_fwd_stage[0] * (int64_t)sizeof(T) : 0;
  S.a.flags = 0;
  if (p > 0 && root_bytes + child_bytes <= 160 * 1024) {
    root_bytes += child_bytes;
    S.a.flags = 1;
  }
  S.root_elems = (root_bytes + sizeof(T) - 1) / sizeof(T);
  return S;
}

// forward sweep of level l (leaves: l = p), p > 0
template <typename T>
void solve_fwd_level(hss_handle* h, SolveSched<T>& S, int l, hipStream_t s) {
  const Plan& P = h->plan;
  S.a.node0 = level_first(l);
  if (l == P.p) {
    launch_solve_w<T>(UlvStep::Fwd, S.a, 1 << l, S.nc, 0, s);
    return;
  }
  const int64_t e = P.level_fwd_stage[l];
  const int64_t st = e > 0 && e * (int64_t)sizeof(T) <= kStageBudget ? e : 0;
  if (use_fwd_op<T>(P) && P.level_fwd_op[l]) launch_solve_w<T>(UlvStep::FwdOp, S.a, 1 << l, S.nc, 0, s);
  else launch_solve_w<T>(UlvStep::Fwd, S.a, 1 << l, S.nc, st, s);
}

// the root solve and the backward sweep
template <typename T>
void solve_root_bwd(hss_handle* h, SolveSched<T>& S, hipStream_t s) {
  const Plan& P = h->plan;
  const int p = P.p;
  S.a.node0 = 0;
  launch_solve_w<T>(UlvStep::Root, S.a, 1, S.nc, S.root_elems, s);
  if (p == 0) return;
  for (int l = 1; l <= p - 1; ++l) {
    S.a.node0 = level_first(l);
    const int64_t e = P.level_bwd_stage[l];
    const int64_t st = e > 0 && e * (int64_t)sizeof(T) <= kStageBudget ? e : 0;
    launch_solve_w<T>(UlvStep::Bwd, S.a, 1 << l, S.nc, st, s);
  }
  S.a.node0 = level_first(p);
  launch_solve_w<T>(UlvStep::Bwd, S.a, 1 << p, S.nc, 0, s);
}

template <typename T>
void run_solve(hss_handle* h, int64_t nrhs, T* B, int64_t ldb, hipStream_t s,
               const int32_t* gate = nullptr) {
  SolveSched<T> S = solve_sched<T>(h, nrhs, B, ldb, gate);
  for (int l = h->plan.p; l >= 1; --l) solve_fwd_level<T>(h, S, l, s);
  solve_root_bwd<T>(h, S, s);
}

// Factorization, then the forward sweep of a solve, overlapped (FP64): the
// sweep of level l runs on the handle's second stream as soon as level l is
// factored, beside the factorization of the levels above (they read and
// write different nodes); the root solve and the backward sweep follow on s.
template <typename T>
void run_factor_solve(hss_handle* h, int64_t nrhs, T* B, int64_t ldb, hipStream_t s) {
  SolveSched<T> S = solve_sched<T>(h, nrhs, B, ldb, nullptr);
  if (h->plan.p == 0) {
    run_factor<T>(h, s);
    solve_root_bwd<T>(h, S, s);
    return;
  }
  // FP64: every level's sweep on the second stream.  FP32: none (lov = 0),
  // the sweeps run on s between the factor levels: a level's FP32 sweep
  // (forward-operator records, ~15 us) is shorter than the event round trip
  // that hands it to the second stream and back (measured: the overlapped
  // FP32 step 2.34-2.36 ms against 2.25 ms in order; FP64 2.55 against 2.79)
  const int lov = sizeof(T) == 8 ? h->plan.p : 0;
  run_factor<T>(h, s, [&](int l) {
    if (l > lov) {
      solve_fwd_level<T>(h, S, l, s);
      return;
    }
    (void)hipEventRecord(h->ev_fork, s);
    (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
    solve_fwd_level<T>(h, S, l, h->side);
  });
  (void)hipEventRecord(h->ev_join, h->side);
  (void)hipStreamWaitEvent(s, h->ev_join, 0);
  solve_root_bwd<T>(h, S, s);
}

hss_status last_launch_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HSS_OK : HSS_EHIP;
}

// ||A||_2 by the power method on A^T A (Sec. 4.5), 16 steps from a fixed
// hash-filled start vector; run once, by hss_create.
hss_status compute_norm2(hss_handle* h, hipStream_t s) {
  hss_status st = ensure_ir(h, 1);
  if (st) return st;
  if ((st = ensure_work_mm<double>(h, 1))) return st;
  const int64_t n = h->plan.n;
  double* v = h->d64;
  double* w = h->res;
  double* u = h->b0;
  double* ss = h->stats;   // [0] ||w||^2, [1] ||u||^2
  launch_hash_fill(v, n, 0x5eedull, s);
  launch_fill(ss, 0.0, 2, s);
  launch_colstats(v, n, n, 1, ss + 1, nullptr, s);
  launch_normalize(v, v, n, ss + 1, s);
  const int iters = 16;
  for (int it = 0; it < iters; ++it) {
    launch_fill(ss, 0.0, 2, s);
    run_matmul<double>(h, HSS_OP_N, 1, v, n, w, n, s);
    launch_colstats(w, n, n, 1, ss, nullptr, s);           // ||A v||^2, ||v|| = 1
    run_matmul<double>(h, HSS_OP_T, 1, w, n, u, n, s);
    launch_colstats(u, n, n, 1, ss + 1, nullptr, s);
    launch_normalize(u, v, n, ss + 1, s);
  }
  if ((st = last_launch_status())) return st;
  double lam = 0.0;
  if (hipMemcpyAsync(&lam, ss, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return HSS_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return HSS_EHIP;
  h->norm2 = std::sqrt(std::max(lam, 0.0));
  return HSS_OK;
}

}  // namespace

// ===========================================================================
// Batched execution over many handles: one launch per tree level for all
// instances.  Upward passes are aligned at the leaves (step s = level p_j - s),
// downward passes at the root (step s = level s).  Task lists of (instance,
// node) pairs and the per-instance pointer tables are uploaded to a device
// scratch buffer owned by the library (one per process; batched calls on
// different streams must not overlap).
// ===========================================================================
namespace {

// Device copies of the task / pointer tables of batched calls, one cache per
// stream: batched calls on different streams run concurrently, calls on one
// stream are serialized by the cache's lock (and by the stream itself).  A
// table is looked up by its bytes: a call whose tables equal an earlier
// call's reuses that device copy without an upload, which is what lets a
// batched call run under HIP graph capture (after an eager call with the same
// handles and blocks) -- tables used while capturing are kept for good, since
// a captured graph holds their addresses.  Other tables are replaced least
// recently used first; the upload that replaces one is ordered on the stream
// after every earlier launch that read it.
struct TableEntry {
  std::vector<char> bytes;
  void* dev = nullptr;
  size_t cap = 0;
  uint64_t last_use = 0;
  bool pinned = false;
};
constexpr size_t kTableCacheEntries = 64;
struct BatchScratch {
  std::vector<TableEntry> tables;
  uint64_t clock = 0;
  std::mutex mu;
};
std::mutex g_scratch_mu;
std::map<hipStream_t, BatchScratch*> g_scratch;

BatchScratch& scratch_for(hipStream_t s) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  BatchScratch*& p = g_scratch[s];
  if (!p) p = new BatchScratch();
  return *p;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs == hipStreamCaptureStatusActive;
}

// Device copy of the table `host` (see BatchScratch).  Under capture a table
// that no eager call has uploaded is refused (HSS_ESTATE): its upload would
// be recorded from host memory that is gone when the graph is replayed.
hss_status scratch_upload(BatchScratch& B, const std::vector<char>& host, hipStream_t s,
                          void** dptr) {
  const bool capturing = stream_capturing(s);
  ++B.clock;
  for (TableEntry& e : B.tables)
    if (e.bytes.size() == host.size() &&
        (host.empty() || std::memcmp(e.bytes.data(), host.data(), host.size()) == 0)) {
      e.last_use = B.clock;
      e.pinned = e.pinned || capturing;
      *dptr = e.dev;
      return HSS_OK;
    }
  if (capturing) return HSS_ESTATE;
  TableEntry* e = nullptr;
  if (B.tables.size() < kTableCacheEntries) {
    B.tables.emplace_back();
    e = &B.tables.back();
  } else {
    for (TableEntry& t : B.tables)
      if (!t.pinned && (!e || t.last_use < e->last_use)) e = &t;
    if (!e) {
      B.tables.emplace_back();
      e = &B.tables.back();
    }
  }
  if (e->cap < host.size() || !e->dev) {
    // the buffer being replaced may still be read by launches in flight:
    // kept (never freed), as are the buffers of pinned tables
    void* d = nullptr;
    const size_t c = std::max<size_t>(host.size() * 2, 1 << 16);
    if (hipMalloc(&d, c) != hipSuccess) {
      (void)hipGetLastError();
      return HSS_ENOMEM;
    }
    e->dev = d;
    e->cap = c;
  }
  e->bytes = host;
  e->last_use = B.clock;
  e->pinned = false;
  // pageable source: the runtime stages it before the call returns
  if (!host.empty() &&
      hipMemcpyAsync(e->dev, host.data(), host.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return HSS_EHIP;
  *dptr = e->dev;
  return HSS_OK;
}

// Packs several arrays into one upload with 256-byte alignment.
struct Packer {
  std::vector<char> buf;
  template <typename X>
  size_t add(const std::vector<X>& v) {
    size_t off = (buf.size() + 255) & ~size_t(255);
    buf.resize(off + v.size() * sizeof(X));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(X));
    return off;
  }
};

struct StepList {
  std::vector<int2> tasks;
  struct Range {
    size_t off;
    int cnt;
    int max_mp;
    int64_t stage;   // max staging elements over the tasks
    bool all_op;     // every task's node has a forward operator
  };
  std::vector<Range> ranges;
  // One step: for every instance, the nodes of tree levels lev(P) = {lo, hi}
  // (a contiguous heap range; hi < lo: none), in instance then heap order.
  template <typename Lev, typename Stage>
  void add_step(hss_handle* const* hs, int count, Lev lev, Stage stage) {
    Range r{tasks.size(), 0, 0, 0, true};
    for (int j = 0; j < count; ++j) {
      const Plan& P = hs[j]->plan;
      const std::pair<int, int> lh = lev(P);
      if (lh.second < lh.first) continue;
      const int t1 = (2 << lh.second) - 1;
      for (int t = (1 << lh.first) - 1; t < t1; ++t) {
        tasks.push_back(make_int2(j, t));
        r.max_mp = std::max(r.max_mp, P.nodes[t].mp);
        r.stage = std::max<int64_t>(r.stage, stage(P, t));
        r.all_op = r.all_op && P.nodes[t].oOP >= 0;
        ++r.cnt;
      }
    }
    ranges.push_back(r);
  }
};

// Level ranges of the batched steps.
inline std::pair<int, int> lv_one(int l) { return {l, l}; }
inline std::pair<int, int> lv_none() { return {1, 0}; }

int max_depth(hss_handle* const* hs, int count) {
  int mp = 0;
  for (int j = 0; j < count; ++j) mp = std::max(mp, hs[j]->plan.p);
  return mp;
}

// The instance records and per-level task lists of a batched product (op N)
// or solve sweep, uploaded once; runs differ only in their calls (right-hand
// sides, gating), a small table of their own.
template <typename T>
struct BatchPlan {
  StepList L;
  const Inst<T>* insts = nullptr;   // device
  const int2* tasks = nullptr;      // device
  int pmax = 0, mku = 0, mk = 0;
  bool wide = false;   // product: per-level wide kernels
  int64_t root_bytes = 0, child_bytes = 0;
};

template <typename C>
hss_status upload_calls(BatchScratch& BS, const std::vector<C>& calls, hipStream_t s,
                        const C** out) {
  std::vector<char> bytes(sizeof(C) * calls.size());
  if (!calls.empty()) std::memcpy(bytes.data(), calls.data(), bytes.size());
  void* d = nullptr;
  hss_status st = scratch_upload(BS, bytes, s, &d);
  *out = reinterpret_cast<const C*>(d);
  return st;
}

template <typename T>
hss_status plan_upload(BatchScratch& BS, const std::vector<Inst<T>>& insts, BatchPlan<T>& bp,
                       hipStream_t s) {
  Packer pk;
  const size_t oi = pk.add(insts), ot = pk.add(bp.L.tasks);
  void* d = nullptr;
  hss_status st = scratch_upload(BS, pk.buf, s, &d);
  if (st) return st;
  bp.insts = reinterpret_cast<const Inst<T>*>((char*)d + oi);
  bp.tasks = reinterpret_cast<const int2*>((char*)d + ot);
  return HSS_OK;
}

// op N product: up (subtree roots), down (subtree roots), leaf outputs.
template <typename T>
hss_status plan_mm_n(BatchScratch& BS, hss_handle* const* hs, int count, const int64_t* nrhs,
                     hipStream_t s, BatchPlan<T>& bp) {
  std::vector<Inst<T>> insts(count);
  for (int j = 0; j < count; ++j) {
    hss_status st = ensure_work_mm<T>(hs[j], std::max<int64_t>(nrhs[j], 1));
    if (st) return st;
    insts[j] = make_inst<T>(hs[j], kUseMM);
    bp.mku = std::max(bp.mku, hs[j]->plan.leaf_max_ku);
    bp.mk = std::max(bp.mk, hs[j]->plan.max_k);
  }
  bp.pmax = max_depth(hs, count);
  auto none = [](const Plan&, int) -> int64_t { return 0; };
  int64_t maxr = 0;
  bp.wide = true;
  for (int j = 0; j < count; ++j) {
    const Plan& P = hs[j]->plan;
    maxr = std::max(maxr, nrhs[j]);
    bp.wide = bp.wide && use_mmw(P.p, kMmwBatchFromCols, P.level_max_mp[P.p], P.max_k,
                                 kMmwBatchFromCols);
  }
  bp.wide = bp.wide && maxr >= kMmwBatchFromCols;
  if (bp.wide) {
    // leaf projections; upward levels aligned at the leaves (down to each
    // root, whose core blocks the up step applies); downward levels aligned
    // at the roots; leaf outputs
    const int pmax = bp.pmax;
    bp.L.add_step(hs, count, [&](const Plan& P) { return lv_one(P.p); }, none);
    for (int st = 1; st <= pmax; ++st)
      bp.L.add_step(hs, count, [&](const Plan& P) {
        return P.p - st >= 0 ? lv_one(P.p - st) : lv_none(); }, none);
    for (int st = 1; st <= pmax - 1; ++st)
      bp.L.add_step(hs, count, [&](const Plan& P) {
        return st <= P.p - 1 ? lv_one(st) : lv_none(); }, none);
    bp.L.add_step(hs, count, [&](const Plan& P) { return lv_one(P.p); }, none);
    return plan_upload(BS, insts, bp, s);
  }
  const int dh = mmf_down_height(), uh = mmf_up_height();
  bp.L.add_step(hs, count, [&](const Plan& P) {
    return P.p > 0 ? lv_one(std::max(P.p - uh, 0)) : lv_none(); }, none);   // up: subtree roots
  bp.L.add_step(hs, count, [&](const Plan& P) {
    return P.p > 0 ? lv_one(std::max(P.p - dh, 0)) : lv_none(); }, none);   // down: subtree roots
  bp.L.add_step(hs, count, [&](const Plan& P) { return lv_one(P.p); }, none);  // leaf outputs
  return plan_upload(BS, insts, bp, s);
}

template <typename T>
hss_status run_mm_n(BatchScratch& BS, const BatchPlan<T>& bp, hss_handle* const* hs, int count,
                    const int64_t* nrhs, const void* const* X, const int64_t* ldx,
                    void* const* Y, const int64_t* ldy, hipStream_t s, bool gated) {
  std::vector<CallMM<T>> calls(count);
  int64_t maxr = 0;
  for (int j = 0; j < count; ++j) {
    calls[j] = CallMM<T>{(const T*)X[j], (T*)Y[j], ldx[j], ldy[j], (int32_t)nrhs[j], HSS_OP_N,
                         gated ? hs[j]->d_status + kStGate : nullptr};
    maxr = std::max(maxr, nrhs[j]);
  }
  if (maxr == 0) return HSS_OK;
  KArgs<T, CallMM<T>> a{};
  hss_status st = upload_calls(BS, calls, s, &a.calls);
  if (st) return st;
  a.insts = bp.insts;
  if (bp.wide) {
    size_t k = 0;
    auto go = [&](MMWStep stp) {
      const auto& r = bp.L.ranges[k++];
      a.tasks = bp.tasks + r.off;
      a.ntasks = r.cnt;
      launch_mmw<T>(stp, a, r.cnt, (int)maxr, s, r.max_mp);
    };
    go(MMWStep::LeafUp);
    for (int q = 1; q <= bp.pmax; ++q) go(MMWStep::Up);
    for (int q = 1; q <= bp.pmax - 1; ++q) go(MMWStep::Down);
    go(MMWStep::LeafOut);
    return last_launch_status();
  }
  const MMFStep steps[3] = {MMFStep::Up, MMFStep::Down, MMFStep::Leaf};
  for (int q = 0; q < 3; ++q) {
    const auto& r = bp.L.ranges[q];
    a.tasks = bp.tasks + r.off;
    a.ntasks = r.cnt;
    launch_mmf<T>(steps[q], a, r.cnt, (int)maxr, bp.mku, bp.mk, s);
  }
  return last_launch_status();
}

// A batched op-N product split by rank class: instances whose ranks are all
// <= 32 (per-level wide kernels or the one-wavefront climb) and those with a
// larger rank (the general kernels), one plan per class, run back to back.
// One instance of rank 64 would otherwise send every instance of the batch
// down the general kernels.
template <typename T>
struct MMSplit {
  BatchPlan<T> bp[2];
  std::vector<int> idx[2];
};

template <typename T>
hss_status plan_mm_split(BatchScratch& BS, hss_handle* const* hs, int count, const int64_t* nrhs,
                         hipStream_t s, MMSplit<T>& ms) {
  for (int j = 0; j < count; ++j) ms.idx[hs[j]->plan.max_k > 32 ? 1 : 0].push_back(j);
  for (int g = 0; g < 2; ++g) {
    if (ms.idx[g].empty()) continue;
    std::vector<hss_handle*> h;
    std::vector<int64_t> r;
    for (int j : ms.idx[g]) {
      h.push_back(hs[j]);
      r.push_back(nrhs[j]);
    }
    const hss_status st = plan_mm_n<T>(BS, h.data(), (int)h.size(), r.data(), s, ms.bp[g]);
    if (st) return st;
  }
  return HSS_OK;
}

template <typename T>
hss_status run_mm_split(BatchScratch& BS, const MMSplit<T>& ms, hss_handle* const* hs,
                        const int64_t* nrhs, const void* const* X, const int64_t* ldx,
                        void* const* Y, const int64_t* ldy, hipStream_t s, bool gated) {
  for (int g = 0; g < 2; ++g) {
    if (ms.idx[g].empty()) continue;
    std::vector<hss_handle*> h;
    std::vector<int64_t> r, lx, ly;
    std::vector<const void*> x;
    std::vector<void*> y;
    for (int j : ms.idx[g]) {
      h.push_back(hs[j]);
      r.push_back(nrhs[j]);
      x.push_back(X[j]);
      lx.push_back(ldx[j]);
      y.push_back(Y[j]);
      ly.push_back(ldy[j]);
    }
    const hss_status st = run_mm_n<T>(BS, ms.bp[g], h.data(), (int)h.size(), r.data(), x.data(),
                                      lx.data(), y.data(), ly.data(), s, gated);
    if (st) return st;
  }
  return HSS_OK;
}

template <typename T>
hss_status batch_matmul_impl(BatchScratch& BS, hss_handle* const* hs, int count, int op,
                             const int64_t* nrhs,
                             const void* const* X, const int64_t* ldx, void* const* Y,
                             const int64_t* ldy, hipStream_t s) {
  int64_t maxr = 0;
  for (int j = 0; j < count; ++j) maxr = std::max(maxr, nrhs[j]);
  if (maxr == 0) return HSS_OK;
  if (op == HSS_OP_N) {
    MMSplit<T> ms;
    hss_status st = plan_mm_split<T>(BS, hs, count, nrhs, s, ms);
    if (st) return st;
    return run_mm_split<T>(BS, ms, hs, nrhs, X, ldx, Y, ldy, s, false);
  }
  std::vector<Inst<T>> insts(count);
  std::vector<CallMM<T>> calls(count);
  for (int j = 0; j < count; ++j) {
    hss_status st = ensure_work_mm<T>(hs[j], std::max<int64_t>(nrhs[j], 1));
    if (st) return st;
    insts[j] = make_inst<T>(hs[j], kUseMM);
    calls[j] = CallMM<T>{(const T*)X[j], (T*)Y[j], ldx[j], ldy[j], (int32_t)nrhs[j], op, nullptr};
  }
  const int pmax = max_depth(hs, count);
  StepList L;
  auto none = [](const Plan&, int) -> int64_t { return 0; };
  L.add_step(hs, count, [&](const Plan& P) { return P.p > 0 ? lv_one(P.p) : lv_none(); },
             none);                                                      // 0: leaf up
  for (int st = 1; st <= pmax - 1; ++st)                                 // 1..: up
    L.add_step(hs, count, [&](const Plan& P) {
      return P.p - st >= 1 ? lv_one(P.p - st) : lv_none(); }, none);
  L.add_step(hs, count, [&](const Plan& P) { return std::make_pair(0, P.p - 1); }, none);
  for (int st = 1; st <= pmax - 1; ++st)
    L.add_step(hs, count, [&](const Plan& P) {
      return st <= P.p - 1 ? lv_one(st) : lv_none(); }, none);
  L.add_step(hs, count, [&](const Plan& P) { return lv_one(P.p); }, none);
  Packer pk;
  const size_t oi = pk.add(insts), oc = pk.add(calls), ot = pk.add(L.tasks);
  void* d = nullptr;
  hss_status st = scratch_upload(BS, pk.buf, s, &d);
  if (st) return st;
  KArgs<T, CallMM<T>> a{};
  a.insts = reinterpret_cast<const Inst<T>*>((char*)d + oi);
  a.calls = reinterpret_cast<const CallMM<T>*>((char*)d + oc);
  const int yt = (int)((maxr + kRT - 1) / kRT);
  size_t k = 0;
  auto run = [&](MMStep stp) {
    const auto& r = L.ranges[k++];
    a.tasks = reinterpret_cast<const int2*>((char*)d + ot) + r.off;
    a.ntasks = r.cnt;
    launch_mm_level<T>(stp, a, r.cnt, yt, kMaxBlock, s);
  };
  run(MMStep::LeafUp);
  for (int q = 1; q <= pmax - 1; ++q) run(MMStep::Up);
  run(MMStep::Couple);
  for (int q = 1; q <= pmax - 1; ++q) run(MMStep::Down);
  run(MMStep::LeafOut);
  return last_launch_status();
}

template <typename T>
hss_status batch_matmul(hss_handle* const* hs, int count, int op, const int64_t* nrhs,
                        const void* const* X, const int64_t* ldx, void* const* Y,
                        const int64_t* ldy, hipStream_t s) {
  BatchScratch& B = scratch_for(s);
  std::lock_guard<std::mutex> g(B.mu);
  return batch_matmul_impl<T>(B, hs, count, op, nrhs, X, ldx, Y, ldy, s);
}

template <typename T>
hss_status batch_factor(hss_handle* const* hs, int count, hipStream_t s) {
  BatchScratch& BS = scratch_for(s);
  std::lock_guard<std::mutex> g(BS.mu);
  std::vector<Inst<T>> insts(count);
  for (int j = 0; j < count; ++j) {
    hss_status st = ensure_factors<T>(hs[j]);
    if (st) return st;
    insts[j] = make_inst<T>(hs[j], 0);
  }
  const int pmax = max_depth(hs, count);
  StepList L;
  auto none = [](const Plan&, int) -> int64_t { return 0; };
  L.add_step(hs, count, [&](const Plan& P) { return P.p > 0 ? lv_one(P.p) : lv_none(); },
             none);
  for (int st = 1; st <= pmax - 1; ++st)
    L.add_step(hs, count, [&](const Plan& P) {
      return P.p - st >= 1 ? lv_one(P.p - st) : lv_none(); }, none);
  L.add_step(hs, count, [&](const Plan& P) { return P.p > 0 ? lv_one(0) : lv_none(); }, none);
  L.add_step(hs, count, [&](const Plan&) { return lv_one(0); }, none);
  Packer pk;
  const size_t oi = pk.add(insts), ot = pk.add(L.tasks);
  void* d = nullptr;
  hss_status st = scratch_upload(BS, pk.buf, s, &d);
  if (st) return st;
  for (int j = 0; j < count; ++j) launch_fill(reinterpret_cast<double*>(hs[j]->d_status), 0.0, 2, s);
  int mk = 0;
  for (int j = 0; j < count; ++j) mk = std::max(mk, hs[j]->plan.max_k);
  KArgs<T, CallSV<T>> a{};
  a.insts = reinterpret_cast<const Inst<T>*>((char*)d + oi);
  size_t k = 0;
  auto rng = [&]() -> const StepList::Range& {
    const auto& r = L.ranges[k++];
    a.tasks = reinterpret_cast<const int2*>((char*)d + ot) + r.off;
    a.ntasks = r.cnt;
    return r;
  };
  {
    const auto& r = rng();
    launch_ulv<T>(UlvStep::Factor, a, r.cnt, mk, r.max_mp, s);
  }
  bool any_op = false;
  for (int j = 0; j < count; ++j) any_op |= use_fwd_op<T>(hs[j]->plan);
  for (int q = 1; q <= pmax - 1; ++q) {
    const auto& r = rng();
    launch_ulv<T>(UlvStep::Merge, a, r.cnt, mk, r.max_mp, s);
    launch_ulv<T>(UlvStep::Factor, a, r.cnt, mk, r.max_mp, s);
    if (any_op) launch_ulv<T>(UlvStep::FwdOp, a, r.cnt, mk, r.max_mp, s);
  }
  {
    const auto& r = rng();
    launch_ulv<T>(UlvStep::Merge, a, r.cnt, mk, r.max_mp, s);
  }
  {
    const auto& r = rng();
    launch_ulv<T>(UlvStep::RootLU, a, r.cnt, mk, r.max_mp, s);
  }
  for (int j = 0; j < count; ++j) (sizeof(T) == 8 ? hs[j]->f64.valid : hs[j]->f32.valid) = true;
  return last_launch_status();
}

// Batched solve sweep (forward, root, backward): plan once, run on
// per-instance right-hand sides rhs[j] (precision T, leading dimension ld[j]).
template <typename T>
hss_status plan_sweep(BatchScratch& BS, hss_handle* const* hs, int count, const int64_t* nrhs,
                      hipStream_t s, BatchPlan<T>& bp) {
  std::vector<Inst<T>> insts(count);
  for (int j = 0; j < count; ++j) {
    hss_status st = ensure_work_sv<T>(hs[j], std::max<int64_t>(nrhs[j], 1));
    if (st) return st;
    insts[j] = make_inst<T>(hs[j], kUseSV);
  }
  const int pmax = bp.pmax = max_depth(hs, count);
  StepList& L = bp.L;
  auto fst = [](const Plan& P, int t) { return P.level_fwd_stage[P.nodes[t].level]; };
  auto bst = [](const Plan& P, int t) { return P.level_bwd_stage[P.nodes[t].level]; };
  auto none = [](const Plan&, int) -> int64_t { return 0; };
  L.add_step(hs, count, [&](const Plan& P) { return P.p > 0 ? lv_one(P.p) : lv_none(); },
             none);
  for (int st = 1; st <= pmax - 1; ++st)
    L.add_step(hs, count, [&](const Plan& P) {
      return P.p - st >= 1 ? lv_one(P.p - st) : lv_none(); }, fst);
  L.add_step(hs, count, [&](const Plan&) { return lv_one(0); }, fst);
  for (int st = 1; st <= pmax - 1; ++st)
    L.add_step(hs, count, [&](const Plan& P) {
      return st <= P.p - 1 ? lv_one(st) : lv_none(); }, bst);
  L.add_step(hs, count, [&](const Plan& P) { return P.p > 0 ? lv_one(P.p) : lv_none(); },
             none);
  // root staging: FP64 LU + pivots (+ children when everything fits)
  for (int j = 0; j < count; ++j) {
    const Plan& P = hs[j]->plan;
    const int64_t mpr = P.nodes[0].mp;
    bp.root_bytes = std::max(bp.root_bytes, mpr * mpr * 8 + 4 * ((mpr + 3) & ~int64_t(3)));
    if (P.p > 0)
      bp.child_bytes = std::max(bp.child_bytes, P.level_fwd_stage[0] * (int64_t)sizeof(T));
  }
  return plan_upload(BS, insts, bp, s);
}

template <typename T>
hss_status run_sweep(BatchScratch& BS, const BatchPlan<T>& bp, hss_handle* const* hs, int count,
                     const int64_t* nrhs, T* const* rhs, const int64_t* ld, hipStream_t s,
                     bool gated) {
  std::vector<CallSV<T>> calls(count);
  int64_t maxr = 0;
  for (int j = 0; j < count; ++j) {
    calls[j] = CallSV<T>{rhs[j], ld[j], (int32_t)nrhs[j], 0,
                         gated ? hs[j]->d_status + kStGate : nullptr};
    maxr = std::max(maxr, nrhs[j]);
  }
  if (maxr == 0) return HSS_OK;
  KArgs<T, CallSV<T>> a{};
  hss_status st = upload_calls(BS, calls, s, &a.calls);
  if (st) return st;
  a.insts = bp.insts;
  const StepList& L = bp.L;
  const int pmax = bp.pmax;
  const int nc = (int)maxr;
  size_t k = 0;
  auto staged = [&](int64_t e) -> int64_t {
    return e > 0 && e * (int64_t)sizeof(T) <= kStageBudget ? e : 0;
  };
  auto go = [&](UlvStep stp, bool use_stage) {
    const auto& r = L.ranges[k++];
    a.tasks = bp.tasks + r.off;
    a.ntasks = r.cnt;
    launch_solve_w<T>(stp, a, r.cnt, nc, use_stage ? staged(r.stage) : 0, s);
  };
  go(UlvStep::Fwd, false);
  for (int q = 1; q <= pmax - 1; ++q) {
    const bool op = L.ranges[k].all_op && sizeof(T) == 4;
    go(op ? UlvStep::FwdOp : UlvStep::Fwd, !op);
  }
  {
    const auto& r = L.ranges[k++];
    a.tasks = bp.tasks + r.off;
    a.ntasks = r.cnt;
    int64_t rb = bp.root_bytes;
    a.flags = 0;
    if (bp.root_bytes + bp.child_bytes <= 160 * 1024) {
      rb += bp.child_bytes;
      a.flags = 1;
    }
    launch_solve_w<T>(UlvStep::Root, a, r.cnt, nc, (rb + sizeof(T) - 1) / sizeof(T), s);
    a.flags = 0;
  }
  for (int q = 1; q <= pmax - 1; ++q) go(UlvStep::Bwd, true);
  go(UlvStep::Bwd, false);
  return last_launch_status();
}

hss_status batch_solve(hss_handle* const* hs, int count, const int64_t* nrhs, double* const* B,
                       const int64_t* ldb, const hss_solve_opts& opt, hss_solve_info* const* info,
                       hipStream_t s) {
  BatchScratch& BS = scratch_for(s);
  std::lock_guard<std::mutex> g(BS.mu);
  const bool is64 = opt.prec == HSS_F64;
  const bool need_eta = opt.want_eta || opt.tol > 0.0;
  hss_status st;
  int64_t maxn = 0;
  for (int j = 0; j < count; ++j) {
    if ((st = ensure_ir(hs[j], std::max<int64_t>(nrhs[j], 1)))) return st;
    if (need_eta && (st = ensure_work_mm<double>(hs[j], std::max<int64_t>(nrhs[j], 1)))) return st;
    maxn = std::max(maxn, hs[j]->plan.n);
  }
  std::vector<IRSeg> segs(count);
  std::vector<int64_t> n_ld(count);
  std::vector<float*> r32(count);
  std::vector<double*> d64(count), res(count), Bv(B, B + count);
  for (int j = 0; j < count; ++j) {
    hss_handle* h = hs[j];
    segs[j] = IRSeg{B[j], ldb[j], h->b0, h->res, h->d64, h->r32, h->plan.n, (int32_t)nrhs[j], 0,
                    h->stats, h->norm2, opt.tol, h->d_status, info ? (void*)info[j] : nullptr};
    n_ld[j] = h->plan.n;
    r32[j] = h->r32;
    d64[j] = h->d64;
    res[j] = h->res;
  }
  // every table before any launch: the sweep's and the residual product's
  // records and task lists (built once, whatever the number of steps), then
  // the refinement descriptors
  BatchPlan<double> sv64;
  MMSplit<double> mm;
  BatchPlan<float> sv32;
  if (is64) {
    if ((st = plan_sweep<double>(BS, hs, count, nrhs, s, sv64))) return st;
  } else {
    if ((st = plan_sweep<float>(BS, hs, count, nrhs, s, sv32))) return st;
  }
  if (need_eta && (st = plan_mm_split<double>(BS, hs, count, nrhs, s, mm))) return st;
  std::vector<char> segbytes(sizeof(IRSeg) * count);
  std::memcpy(segbytes.data(), segs.data(), segbytes.size());
  void* dsegp = nullptr;
  if ((st = scratch_upload(BS, segbytes, s, &dsegp))) return st;
  IRSeg* dsegs = reinterpret_cast<IRSeg*>(dsegp);
  int maxc = 0;
  for (int j = 0; j < count; ++j) maxc = std::max(maxc, (int)nrhs[j]);
  auto ir = [&](int op, bool gated = false, int step = 0) {
    launch_ir_batch(op, dsegs, count, maxn, maxc, gated, step, opt.max_refine, s);
  };
  ir(IR_ZERO_ALL);
  if (need_eta) ir(IR_SAVE_B0);
  // first: B <- A^-1 B; later (gated per instance): B += A^-1 r
  auto correction = [&](bool first) -> hss_status {
    hss_status e;
    if (is64) {
      if (first) return run_sweep<double>(BS, sv64, hs, count, nrhs, Bv.data(), ldb, s, false);
      ir(IR_COPY_RES, true);
      if ((e = run_sweep<double>(BS, sv64, hs, count, nrhs, d64.data(), n_ld.data(), s, true)))
        return e;
      ir(IR_AXPY64, true);
      return HSS_OK;
    }
    if (first) {
      ir(IR_STATS_BMAX);
      ir(IR_SCALE_B);
    } else {
      ir(IR_SCALE_RES, true);
    }
    if ((e = run_sweep<float>(BS, sv32, hs, count, nrhs, r32.data(), n_ld.data(), s, !first)))
      return e;
    ir(first ? IR_CAST_BACK : IR_AXPY_CAST, !first);
    return HSS_OK;
  };
  auto check = [&](int k) -> hss_status {
    const bool gated = k > 0;
    hss_status e;
    std::vector<const void*> xv(Bv.begin(), Bv.end());
    std::vector<void*> yv(res.begin(), res.end());
    if ((e = run_mm_split<double>(BS, mm, hs, nrhs, xv.data(), ldb, yv.data(), n_ld.data(), s,
                                  gated)))
      return e;
    ir(IR_ZERO, gated);
    ir(IR_RESID, gated);
    ir(IR_STATS_X, gated);
    ir(IR_ETA, gated, k);
    return HSS_OK;
  };
  if ((st = correction(true))) return st;
  if (need_eta) {
    ir(IR_STATS_B0);
    if ((st = check(0))) return st;
    const int steps = opt.tol > 0.0 ? opt.max_refine : 0;
    for (int k = 1; k <= steps; ++k) {
      if ((st = correction(false))) return st;
      if ((st = check(k))) return st;
    }
  }
  if (info) ir(IR_INFO, false, need_eta ? 1 : 0);
  return last_launch_status();
}

// ---------------------------------------------------------------------------
// Fixed device scratch of hss_matmul_noalloc: the product's x^ and y^ work
// vectors for callers that cannot allocate.  Each GPU the library runs on
// holds its own copy from load until the process ends.  Its device address is
// looked up once per device (hipGetSymbolAddress with that device current);
// host code uses only that address, never the array's name.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr int kNoAllocMinCols = 8;   // columns reserved per work vector (a product chunk)
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kMaxDevices] = {};

hss_status noalloc_scratch(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HSS_EHIP;
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return HSS_EHIP;
    }
    g_noalloc_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return HSS_OK;
}

// Bytes of scratch the product of nrhs columns takes: x^ and y^, each ldm
// rows by max(nrhs, kNoAllocMinCols) columns.
int64_t noalloc_bytes(const Plan& P, int64_t nrhs, size_t es) {
  return 2 * P.ldm * std::max<int64_t>(nrhs, kNoAllocMinCols) * (int64_t)es;
}

}  // namespace

// ===========================================================================
// ---------------------------------------------------------------------------
// Autotuning: median of five timed calls (after one untimed) per variant.
template <typename F>
double time_calls(hipStream_t s, F fn) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  fn();
  double t[5];
  for (int i = 0; i < 5; ++i) {
    (void)hipEventRecord(e0, s);
    fn();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    t[i] = 1e3 * ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::sort(t, t + 5);
  return t[2];
}

template <typename T>
hss_status autotune(hss_handle* h, int64_t nrhs, hipStream_t s, TuneVal& tv, bool& did_mm,
                    bool& did_sv) {
  const Plan& P = h->plan;
  const int64_t n = P.n;
  did_mm = did_sv = false;
  hss_status st = HSS_OK;
  if (P.p > 0 && nrhs >= 2 && mmw_fits(P.level_max_mp[P.p], P.max_k)) {
    T* X = dalloc<T>(h, n * nrhs);
    T* Y = dalloc<T>(h, n * nrhs);
    if (!X || !Y) st = HSS_ENOMEM;
    else if ((st = ensure_work_mm<T>(h, nrhs)) == HSS_OK &&
             hipMemsetAsync(X, 0, sizeof(T) * n * nrhs, s) == hipSuccess) {
      for (int v = 0; v < 2; ++v) {
        g_force_mm = v;
        tv.t_mm[v] = time_calls(s, [&] { run_matmul<T>(h, HSS_OP_N, nrhs, X, n, Y, n, s); });
      }
      g_force_mm = -1;
      tv.mm = tv.t_mm[1] < tv.t_mm[0] ? 1 : 0;
      did_mm = true;
    }
    (void)hipStreamSynchronize(s);
    dev_free(h, X);
    dev_free(h, Y);
    if (st) return st;
    if ((st = last_launch_status())) return st;
  }
  const bool factored = sizeof(T) == 8 ? h->f64.valid : h->f32.valid;
  if (factored && nrhs >= 4) {
    T* B = dalloc<T>(h, n * nrhs);
    if (!B) return HSS_ENOMEM;
    if ((st = ensure_work_sv<T>(h, nrhs)) == HSS_OK &&
        hipMemsetAsync(B, 0, sizeof(T) * n * nrhs, s) == hipSuccess) {
      const int cand[2] = {1, 4};
      for (int v = 0; v < 2; ++v) {
        g_force_cpw = cand[v];
        tv.t_sv[v] = time_calls(s, [&] { run_solve<T>(h, nrhs, B, n, s); });
      }
      g_force_cpw = 0;
      tv.cpw = tv.t_sv[1] < tv.t_sv[0] ? 4 : 1;
      did_sv = true;
    }
    (void)hipStreamSynchronize(s);
    dev_free(h, B);
    if (st) return st;
    if ((st = last_launch_status())) return st;
  }
  return HSS_OK;
}

std::string tune_line(const TuneKey& k, const TuneVal& v) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "%d %d %d %d %d %d %d %.2f %.2f %.2f %.2f\n", k.leaf_mp, k.max_k,
                k.p, k.prec, k.bucket, v.mm, v.cpw, v.t_mm[0], v.t_mm[1], v.t_sv[0], v.t_sv[1]);
  return buf;
}

hss_status copy_out(const std::string& txt, char* buf, int64_t cap) {
  if (!buf || cap <= 0) return HSS_OK;
  const size_t nb = std::min<size_t>(txt.size(), (size_t)cap - 1);
  std::memcpy(buf, txt.data(), nb);
  buf[nb] = 0;
  return txt.size() < (size_t)cap ? HSS_OK : HSS_ESCRATCH;
}

namespace {

// A handle for the plan P with every device array allocated and initialized
// except the contents of the FP64 generators (g64), which the caller fills
// on stream s before finish_handle.
hss_status new_handle(Plan&& P, const hss_alloc* alloc, hipStream_t s, hss_handle** out) {
  hss_handle* h = new hss_handle();
  h->plan = std::move(P);
  const Plan& Q = h->plan;
  if (alloc) {
    h->alloc = *alloc;
    h->custom_alloc = true;
  }
  auto fail = [&](hss_status e) {
    hss_destroy(h);
    return e;
  };
  if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess)
    return fail(HSS_EHIP);
  h->d_nodes = dalloc<NodeInfo>(h, Q.nnodes);
  h->d_status = dalloc<int32_t>(h, 4);
  h->d_cnt = dalloc<uint32_t>(h, (int64_t)((Q.nnodes + 2) & ~1) * kMbChunks);
  h->chk_cnt = dalloc<uint32_t>(h, 2);
  if (!h->d_nodes || !h->d_status || !h->d_cnt || !h->chk_cnt) return fail(HSS_ENOMEM);
  if (hipMemcpyAsync(h->d_nodes, Q.nodes.data(), sizeof(NodeInfo) * Q.nnodes,
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(HSS_EHIP);
  const int64_t sizes[7] = {Q.nD, Q.nU, Q.nV, Q.nR, Q.nW, Q.nB12, Q.nB21};
  for (int i = 0; i < 7; ++i) {
    h->g64[i] = dalloc<double>(h, sizes[i]);
    h->g32[i] = dalloc<float>(h, sizes[i]);
    if (!h->g64[i] || !h->g32[i]) return fail(HSS_ENOMEM);
  }
  launch_fill(reinterpret_cast<double*>(h->d_status), 0.0, 2, s);
  launch_fill(reinterpret_cast<double*>(h->d_cnt), 0.0, (int64_t)((Q.nnodes + 2) / 2) * kMbChunks, s);
  launch_fill(reinterpret_cast<double*>(h->chk_cnt), 0.0, 1, s);
  {
    // product mailboxes (one set per column chunk), all empty
    const int64_t nmb = (int64_t)Q.nnodes * kMbSlot * kMbCols * kMbChunks;
    h->w64.mb = dalloc<double>(h, nmb);
    h->w32.mb = dalloc<float>(h, nmb + 1);
    if (!h->w64.mb || !h->w32.mb) return fail(HSS_ENOMEM);
    const uint64_t e32 = ((uint64_t)kMbEmpty32 << 32) | kMbEmpty32;
    double v64, v32;
    std::memcpy(&v64, &kMbEmpty64, sizeof v64);
    std::memcpy(&v32, &e32, sizeof v32);
    launch_fill(h->w64.mb, v64, nmb, s);
    launch_fill(reinterpret_cast<double*>(h->w32.mb), v32, (nmb + 1) / 2, s);
  }
  hss_status st = last_launch_status();
  if (st) return fail(st);
  *out = h;
  return HSS_OK;
}

// Device scratch of one call from the caller's allocator hooks (or
// hipMalloc), released when it goes out of scope: every path that leaves
// its scope must have synchronized the stream first.
struct TempDev {
  const hss_alloc* al;
  std::vector<void*> ptrs;
  explicit TempDev(const hss_alloc* a) : al(a) {}
  TempDev(const TempDev&) = delete;
  TempDev& operator=(const TempDev&) = delete;
  void* get(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void* q = nullptr;
    if (al) {
      q = al->alloc(bytes, al->ctx);
    } else if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      q = nullptr;
    }
    if (q) ptrs.push_back(q);
    return q;
  }
  ~TempDev() {
    for (void* q : ptrs) {
      if (al) al->free(q, al->ctx);
      else (void)hipFree(q);
    }
  }
};

// The resident FP32 copy of the generators and ||A||_2, then a stream
// synchronization (the handle is complete when this returns HSS_OK).
hss_status finish_handle(hss_handle* h, hipStream_t s) {
  const Plan& P = h->plan;
  const int64_t sizes[7] = {P.nD, P.nU, P.nV, P.nR, P.nW, P.nB12, P.nB21};
  for (int i = 0; i < 7; ++i)
    if (sizes[i] > 0) launch_cast_f64_f32(h->g64[i], h->g32[i], sizes[i], s);
  hss_status st = last_launch_status();
  if (st) return st;
  if ((st = compute_norm2(h, s))) return st;
  return hipStreamSynchronize(s) == hipSuccess ? HSS_OK : HSS_EHIP;
}

}  // namespace

extern "C" {

const char* hss_status_str(hss_status s) {
  switch (s) {
    case HSS_OK: return "ok";
    case HSS_ENOMEM: return "device allocation failed";
    case HSS_EHIP: return "HIP runtime error";
    case HSS_ESTATE: return "call out of order (e.g. solve before factor)";
    case HSS_ESINGULAR: return "exactly singular pivot";
    case HSS_ENOCONV: return "refinement did not reach the tolerance";
    case HSS_EUNSUP: return "sizes beyond what the kernels support";
    case HSS_ESCRATCH:
      return "the product needs more than the fixed scratch of the allocation-free entry point";
    default: return s < 0 ? "invalid argument" : "unknown status";
  }
}

int32_t hss_plan_depth(int64_t n, int64_t nmin) { return default_depth(n, nmin); }

hss_status hss_plan_leaf_offsets(int64_t n, int64_t nmin, int64_t* leaf_off, int64_t cap) {
  if (n <= 0) return -1;
  if (nmin <= 0) return -2;
  if (!leaf_off) return -3;
  const int32_t p = default_depth(n, nmin);
  const int64_t nleaf = int64_t(1) << p;
  if (cap < nleaf + 1) return -4;
  // ceil-halving, level by level (Sec. 3.1): store boundaries of the current level
  std::vector<int64_t> b = {0, n};
  for (int32_t l = 0; l < p; ++l) {
    std::vector<int64_t> nb;
    nb.reserve(2 * b.size() - 1);
    for (size_t i = 0; i + 1 < b.size(); ++i) {
      const int64_t s = b[i + 1] - b[i];
      nb.push_back(b[i]);
      nb.push_back(b[i] + (s + 1) / 2);
    }
    nb.push_back(n);
    b.swap(nb);
  }
  std::copy(b.begin(), b.end(), leaf_off);
  return HSS_OK;
}

hss_status hss_plan_node_ranges(const hss_tree_desc* tree, int64_t* start, int64_t* size) {
  if (!start) return -2;
  if (!size) return -3;
  Plan P;
  const hss_status st = build_plan(tree, P, nullptr);
  if (st) return st;
  for (int32_t t = 0; t < P.nnodes; ++t) {
    start[t] = P.nodes[t].row0;
    int64_t m = 0;
    // node size as the sum of its leaves (exact int64)
    int64_t lo = t, hi = t;
    while (lo < (int64_t(1) << P.p) - 1) { lo = 2 * lo + 1; hi = 2 * hi + 2; }
    const int64_t f = (int64_t(1) << P.p) - 1;
    m = P.leaf_off[hi - f + 1] - P.leaf_off[lo - f];
    size[t] = m;
  }
  return HSS_OK;
}

hss_status hss_create(const hss_tree_desc* tree, const hss_gen_host* g, const hss_alloc* alloc,
                      void* stream, hss_handle** out) {
  if (!out) return -5;
  *out = nullptr;
  if (!g) return -2;
  if (alloc && (!alloc->alloc || !alloc->free)) return -3;
  Plan P;
  hss_status st = build_plan(tree, P, nullptr);
  if (st) return st;
  const int64_t sizes[7] = {P.nD, P.nU, P.nV, P.nR, P.nW, P.nB12, P.nB21};
  const double* src[7] = {g->D, g->U, g->V, g->R, g->W, g->B12, g->B21};
  for (int i = 0; i < 7; ++i)
    if (sizes[i] > 0 && !src[i]) return -2;
  hipStream_t s = (hipStream_t)stream;
  hss_handle* h = nullptr;
  if ((st = new_handle(std::move(P), alloc, s, &h))) return st;
  for (int i = 0; i < 7; ++i)
    if (sizes[i] > 0 && hipMemcpyAsync(h->g64[i], src[i], sizeof(double) * sizes[i],
                                       hipMemcpyHostToDevice, s) != hipSuccess) {
      hss_destroy(h);
      return HSS_EHIP;
    }
  if ((st = finish_handle(h, s))) {
    hss_destroy(h);
    return st;
  }
  *out = h;
  return HSS_OK;
}

hss_status hss_hadamard(const hss_handle* A, const hss_handle* B, const hss_alloc* alloc,
                        void* stream, hss_handle** out) {
  if (!out) return -5;
  *out = nullptr;
  if (!A) return -1;
  if (!B) return -2;
  if (alloc && (!alloc->alloc || !alloc->free)) return -3;
  const Plan& PA = A->plan;
  const Plan& PB = B->plan;
  if (PA.n != PB.n || PA.p != PB.p || PA.leaf_off != PB.leaf_off) return -2;
  // the tree of A o B: A's partition, ranks multiplied node by node
  std::vector<int32_t> ku(PA.nnodes), kv(PA.nnodes);
  for (int32_t t = 0; t < PA.nnodes; ++t) {
    const int64_t u = (int64_t)PA.nodes[t].ku * PB.nodes[t].ku;
    const int64_t v = (int64_t)PA.nodes[t].kv * PB.nodes[t].kv;
    if (u > kMaxRank || v > kMaxRank) return HSS_EUNSUP;
    ku[t] = (int32_t)u;
    kv[t] = (int32_t)v;
  }
  const hss_tree_desc td{PA.n, PA.p, 0, PA.leaf_off.data(), ku.data(), kv.data()};
  Plan P;
  hss_status st = build_plan(&td, P, nullptr);
  if (st) return st > 0 ? st : HSS_EUNSUP;
  hipStream_t s = (hipStream_t)stream;
  hss_handle* h = nullptr;
  if ((st = new_handle(std::move(P), alloc, s, &h))) return st;
  launch_hadamard(A->d_nodes, B->d_nodes, h->d_nodes, A->g64, B->g64, h->g64, h->plan.nD,
                  h->plan.nnodes, h->plan.p, s);
  if ((st = last_launch_status()) || (st = finish_handle(h, s))) {
    hss_destroy(h);
    return st;
  }
  *out = h;
  return HSS_OK;
}

hss_status hss_compress(const hss_handle* A, double tau, const hss_alloc* alloc, void* stream,
                        hss_handle** out) {
  if (!out) return -5;
  *out = nullptr;
  if (!A) return -1;
  if (!(tau >= 0.0) || std::isinf(tau)) return -2;
  if (alloc && (!alloc->alloc || !alloc->free)) return -3;
  const Plan& PA = A->plan;
  const int32_t nn = PA.nnodes, p = PA.p;
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> ku(nn, 0), kv(nn, 0);
  TempDev tmp(alloc);
  const int64_t sizes[6] = {PA.nU, PA.nV, PA.nR, PA.nW, PA.nB12, PA.nB21};
  double* work[6] = {};
  const size_t slot = (size_t)kMaxRank * kMaxRank;
  for (int i = 0; i < 6; ++i) work[i] = (double*)tmp.get(sizeof(double) * (size_t)sizes[i]);
  double* TU = (double*)tmp.get(sizeof(double) * slot * nn);
  double* TV = (double*)tmp.get(sizeof(double) * slot * nn);
  double* su = (double*)tmp.get(sizeof(double) * (size_t)kMaxRank * nn);
  double* sv = (double*)tmp.get(sizeof(double) * (size_t)kMaxRank * nn);
  int32_t* rk = (int32_t*)tmp.get(sizeof(int32_t) * 4 * (size_t)nn + 8);
  for (int i = 0; i < 6; ++i)
    if (!work[i]) return HSS_ENOMEM;
  if (!TU || !TV || !su || !sv || !rk) return HSS_ENOMEM;
  hss_status st = HSS_OK;
  if (p > 0) {
    for (int i = 0; i < 6; ++i)
      if (sizes[i] > 0 && hipMemcpyAsync(work[i], A->g64[i + 1], sizeof(double) * sizes[i],
                                         hipMemcpyDeviceToDevice, s) != hipSuccess)
        st = HSS_EHIP;
    launch_fill(reinterpret_cast<double*>(rk), 0.0, 2 * (int64_t)nn, s);
    const CompressBufs b{A->d_nodes, work[0], work[1], work[2], work[3], work[4], work[5], TU, TV,
                         su,         sv,      rk,      rk + nn, rk + 2 * nn, rk + 3 * nn};
    const int leaf0 = (1 << p) - 1;
    // phase 1: proper form, bottom-up
    launch_compress(CompressStep::LeafQR, b, leaf0, 1 << p, tau, s);
    for (int l = p - 1; l >= 1; --l) launch_compress(CompressStep::UpQR, b, (1 << l) - 1, 1 << l, tau, s);
    launch_compress(CompressStep::Core, b, 0, leaf0, tau, s);
    // phase 2: truncated SVDs, top-down
    for (int l = 1; l <= p; ++l) {
      launch_compress(CompressStep::Svd, b, (1 << l) - 1, 1 << l, tau, s);
      launch_compress(CompressStep::ApplyParent, b, (1 << (l - 1)) - 1, 1 << (l - 1), tau, s);
      launch_compress(CompressStep::ApplyChild, b, (1 << l) - 1, 1 << l, tau, s);
    }
    if (hipMemcpyAsync(ku.data(), rk + 2 * nn, sizeof(int32_t) * nn, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipMemcpyAsync(kv.data(), rk + 3 * nn, sizeof(int32_t) * nn, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
      st = HSS_EHIP;
    if (!st) st = last_launch_status();
  }
  if (hipStreamSynchronize(s) != hipSuccess && !st) st = HSS_EHIP;
  if (st) return st;
  ku[0] = kv[0] = 0;
  const hss_tree_desc td{PA.n, p, 0, PA.leaf_off.data(), ku.data(), kv.data()};
  Plan P;
  st = build_plan(&td, P, nullptr);
  if (st) return st > 0 ? st : HSS_EUNSUP;
  hss_handle* h = nullptr;
  if ((st = new_handle(std::move(P), alloc, s, &h))) return st;
  if (PA.nD > 0 && hipMemcpyAsync(h->g64[0], A->g64[0], sizeof(double) * PA.nD,
                                  hipMemcpyDeviceToDevice, s) != hipSuccess)
    st = HSS_EHIP;
  if (!st && p > 0) {
    const double* wk[6] = {work[0], work[1], work[2], work[3], work[4], work[5]};
    double* dst[6] = {h->g64[1], h->g64[2], h->g64[3], h->g64[4], h->g64[5], h->g64[6]};
    launch_compress_gather(A->d_nodes, h->d_nodes, wk, dst, nn, s);
    st = last_launch_status();
  }
  if (!st) st = finish_handle(h, s);
  if (st) {
    (void)hipStreamSynchronize(s);
    hss_destroy(h);
    return st;
  }
  *out = h;
  return HSS_OK;
}

// Dense-to-HSS construction (Sec. 3.2): the levels from the leaves up, each
// a truncation launch (block rows of X and of X^T), a rank read-back, and
// the reduced matrix of the next level, M <- blkdiag(R_t)^T M blkdiag(W_t)
// (at the leaves blkdiag(U_i)^T A blkdiag(V_i)) as Y = X blkdiag(W),
// M^T = Y^T blkdiag(R), M = (M^T)^T.  Every reduced matrix is kept until the
// end: the core blocks of the nodes one level up are its blocks.
}  // extern "C"

namespace {

struct CnLevel {
  double* M = nullptr;    // Ku x Kv (ld Ku): blkdiag(U^_t)^T A blkdiag(V^_t), t on the level
  double* Mt = nullptr;   // its transpose
  int64_t Ku = 0, Kv = 0;
  std::vector<int64_t> ro, co;   // row / column block offsets of the level's nodes
  // the product task lists, kept until the call has synchronized (their
  // uploads are asynchronous)
  std::vector<CnRmul> ta, tb;
};

template <typename V>
hss_status upload(TempDev& tmp, const std::vector<V>& v, V** d, hipStream_t s) {
  *d = (V*)tmp.get(sizeof(V) * std::max<size_t>(v.size(), 1));
  if (!*d) return HSS_ENOMEM;
  if (!v.empty() &&
      hipMemcpyAsync(*d, v.data(), sizeof(V) * v.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return HSS_EHIP;
  return HSS_OK;
}

}  // namespace

extern "C" {

hss_status hss_construct_dense(const double* A, int64_t lda, int64_t n, int32_t p,
                               const int64_t* leaf_off, double eps, const hss_alloc* alloc,
                               void* stream, hss_handle** out) {
  if (!out) return -9;
  *out = nullptr;
  if (!A) return -1;
  if (n < 1) return -3;
  if (lda < n) return -2;
  if (p < 0 || p > 30) return -4;
  if (!leaf_off) return -5;
  if (!(eps >= 0.0) || std::isinf(eps)) return -6;
  if (alloc && (!alloc->alloc || !alloc->free)) return -7;
  const int32_t nn = (int32_t)((2ll << p) - 1), leaf0 = (int32_t)((1ll << p) - 1);
  // node ranges; the plan below validates the offsets again
  std::vector<int64_t> st(nn), sz(nn);
  if (leaf_off[0] != 0 || leaf_off[1ll << p] != n) return -5;
  for (int32_t i = 0; i < (1 << p); ++i) {
    if (leaf_off[i + 1] <= leaf_off[i]) return -5;
    if (leaf_off[i + 1] - leaf_off[i] > kCnMaxRows) return HSS_EUNSUP;
    st[leaf0 + i] = leaf_off[i];
    sz[leaf0 + i] = leaf_off[i + 1] - leaf_off[i];
  }
  for (int32_t t = leaf0 - 1; t >= 0; --t) {
    st[t] = st[2 * t + 1];
    sz[t] = sz[2 * t + 1] + sz[2 * t + 2];
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<int32_t> ku(nn, 0), kv(nn, 0);
  TempDev tmp(alloc);
  hss_status stt = HSS_OK;
  // left singular vectors of every truncation: two slots per node
  const size_t slot = (size_t)kCnMaxRows * kCnMaxRows;
  double* Ub = p > 0 ? (double*)tmp.get(sizeof(double) * slot * 2 * nn) : nullptr;
  double* sg = p > 0 ? (double*)tmp.get(sizeof(double) * kCnMaxRows * 2 * nn) : nullptr;
  int32_t* rk = p > 0 ? (int32_t*)tmp.get(sizeof(int32_t) * 2 * nn) : nullptr;
  double* At = p > 0 ? (double*)tmp.get(sizeof(double) * (size_t)n * n) : nullptr;
  if (p > 0 && (!Ub || !sg || !rk || !At)) return HSS_ENOMEM;
  auto uslot = [&](int32_t t, int side) { return Ub + slot * (2 * (size_t)t + side); };
  std::vector<CnLevel> lev(p + 1);   // lev[l]: reduced matrix of level l (l = 1 .. p)
  // every exit waits for the stream before the host task lists above go away
  struct SyncOnExit {
    hipStream_t s;
    ~SyncOnExit() { (void)hipStreamSynchronize(s); }
  } sync_on_exit{s};
  std::vector<int32_t> rk_h(2 * nn, 0);
  // truncations of the nodes of one level: row side on X, column side on Xt
  auto truncate_level = [&](int l, const double* X, int64_t ldx, int64_t nx, const double* Xt,
                            int64_t ldxt, int64_t nxt, const std::vector<int64_t>& r0,
                            const std::vector<int64_t>& rsz, const std::vector<int64_t>& c0,
                            const std::vector<int64_t>& csz) -> hss_status {
    const int32_t t0 = (1 << l) - 1, cnt = 1 << l;
    std::vector<CnTask> tasks(2 * (size_t)cnt);
    for (int32_t j = 0; j < cnt; ++j) {
      const int32_t t = t0 + j;
      if (rsz[j] > kCnMaxRows || csz[j] > kCnMaxRows) return HSS_EUNSUP;
      tasks[2 * j] = CnTask{X,          ldx,       r0[j],        (int32_t)rsz[j], 0, nx,
                            c0[j],      c0[j] + csz[j], uslot(t, 0), sg + (size_t)kCnMaxRows * 2 * t,
                            rk + 2 * t};
      tasks[2 * j + 1] = CnTask{Xt,     ldxt,      c0[j],        (int32_t)csz[j], 0, nxt,
                                r0[j],  r0[j] + rsz[j], uslot(t, 1),
                                sg + (size_t)kCnMaxRows * (2 * t + 1), rk + 2 * t + 1};
    }
    CnTask* dt = nullptr;
    hss_status e = upload(tmp, tasks, &dt, s);
    if (e) return e;
    launch_cn_trunc(dt, 2 * cnt, eps, l == p, s);
    if ((e = last_launch_status())) {
      (void)hipStreamSynchronize(s);
      return e;
    }
    if (hipMemcpyAsync(rk_h.data() + 2 * t0, rk + 2 * t0, sizeof(int32_t) * 2 * cnt,
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return HSS_EHIP;
    for (int32_t j = 0; j < cnt; ++j) {
      ku[t0 + j] = rk_h[2 * (t0 + j)];
      kv[t0 + j] = rk_h[2 * (t0 + j) + 1];
      if (ku[t0 + j] > kMaxRank || kv[t0 + j] > kMaxRank) return HSS_EUNSUP;
    }
    return HSS_OK;
  };
  // the reduced matrix of level l from X (rows x cols) and the level's factors
  auto reduce_level = [&](int l, const double* X, int64_t ldx, int64_t rows,
                          const std::vector<int64_t>& r0, const std::vector<int64_t>& rsz,
                          const std::vector<int64_t>& c0,
                          const std::vector<int64_t>& csz) -> hss_status {
    const int32_t t0 = (1 << l) - 1, cnt = 1 << l;
    CnLevel& L = lev[l];
    L.ro.assign(cnt + 1, 0);
    L.co.assign(cnt + 1, 0);
    for (int32_t j = 0; j < cnt; ++j) {
      L.ro[j + 1] = L.ro[j] + ku[t0 + j];
      L.co[j + 1] = L.co[j] + kv[t0 + j];
    }
    L.Ku = L.ro[cnt];
    L.Kv = L.co[cnt];
    double* Y = (double*)tmp.get(sizeof(double) * (size_t)rows * L.Kv);
    double* Yt = (double*)tmp.get(sizeof(double) * (size_t)rows * L.Kv);
    L.M = (double*)tmp.get(sizeof(double) * (size_t)L.Ku * L.Kv);
    L.Mt = (double*)tmp.get(sizeof(double) * (size_t)L.Ku * L.Kv);
    if (!Y || !Yt || !L.M || !L.Mt) return HSS_ENOMEM;
    std::vector<CnRmul>& a = L.ta;
    std::vector<CnRmul>& b = L.tb;
    a.resize(cnt);
    b.resize(cnt);
    for (int32_t j = 0; j < cnt; ++j) {
      const int32_t t = t0 + j;
      a[j] = CnRmul{X, ldx, rows, c0[j], (int32_t)csz[j], kv[t], uslot(t, 1), kCnMaxRows,
                    Y, rows, L.co[j]};
      b[j] = CnRmul{Yt, L.Kv, L.Kv, r0[j], (int32_t)rsz[j], ku[t], uslot(t, 0), kCnMaxRows,
                    L.Mt, L.Kv, L.ro[j]};
    }
    CnRmul *da = nullptr, *db = nullptr;
    hss_status e;
    if ((e = upload(tmp, a, &da, s)) || (e = upload(tmp, b, &db, s))) return e;
    launch_cn_rmul(da, cnt, rows, s);
    launch_cn_trans(Y, rows, rows, L.Kv, Yt, L.Kv, s);
    launch_cn_rmul(db, cnt, L.Kv, s);
    launch_cn_trans(L.Mt, L.Kv, L.Kv, L.Ku, L.M, L.Ku, s);
    return last_launch_status();
  };
  if (p > 0) {
    launch_cn_trans(A, lda, n, n, At, n, s);
    std::vector<int64_t> r0(1 << p), rsz(1 << p);
    for (int32_t j = 0; j < (1 << p); ++j) {
      r0[j] = st[leaf0 + j];
      rsz[j] = sz[leaf0 + j];
    }
    if ((stt = truncate_level(p, A, lda, n, At, n, n, r0, rsz, r0, rsz))) return stt;
    if ((stt = reduce_level(p, A, lda, n, r0, rsz, r0, rsz))) return stt;
    for (int l = p - 1; l >= 1; --l) {
      const CnLevel& B = lev[l + 1];
      const int32_t cnt = 1 << l;
      std::vector<int64_t> q0(cnt), qs(cnt), w0(cnt), ws(cnt);
      for (int32_t j = 0; j < cnt; ++j) {
        q0[j] = B.ro[2 * j];
        qs[j] = B.ro[2 * j + 2] - B.ro[2 * j];
        w0[j] = B.co[2 * j];
        ws[j] = B.co[2 * j + 2] - B.co[2 * j];
      }
      if ((stt = truncate_level(l, B.M, B.Ku, B.Kv, B.Mt, B.Kv, B.Ku, q0, qs, w0, ws))) return stt;
      if ((stt = reduce_level(l, B.M, B.Ku, B.Ku, q0, qs, w0, ws))) return stt;
    }
  }
  ku[0] = kv[0] = 0;
  const hss_tree_desc td{n, p, 0, leaf_off, ku.data(), kv.data()};
  Plan P;
  stt = build_plan(&td, P, nullptr);
  if (stt) return stt > 0 ? stt : -5;
  hss_handle* h = nullptr;
  if ((stt = new_handle(std::move(P), alloc, s, &h))) return stt;
  const Plan& Q = h->plan;
  std::vector<CnCopy> cp;
  cp.reserve(4 * (size_t)nn);
  for (int32_t t = 0; t < nn; ++t) {
    const NodeInfo& ni = Q.nodes[t];
    if (t >= leaf0) {
      const int32_t m = (int32_t)sz[t];
      cp.push_back(CnCopy{A + st[t] + st[t] * lda, lda, h->g64[0] + ni.oD, m, m});
      if (p > 0) {
        cp.push_back(CnCopy{uslot(t, 0), kCnMaxRows, h->g64[1] + ni.oU, m, ku[t]});
        cp.push_back(CnCopy{uslot(t, 1), kCnMaxRows, h->g64[2] + ni.oV, m, kv[t]});
      }
      continue;
    }
    const int32_t c1 = 2 * t + 1, c2 = 2 * t + 2;
    if (t != 0) {
      cp.push_back(CnCopy{uslot(t, 0), kCnMaxRows, h->g64[3] + ni.oR, ku[c1] + ku[c2], ku[t]});
      cp.push_back(CnCopy{uslot(t, 1), kCnMaxRows, h->g64[4] + ni.oW, kv[c1] + kv[c2], kv[t]});
    }
    // core blocks: blocks of the reduced matrix of the children's level
    const int l = Q.nodes[c1].level;
    const CnLevel& L = lev[l];
    const int32_t j1 = c1 - ((1 << l) - 1), j2 = j1 + 1;
    cp.push_back(CnCopy{L.M + L.ro[j1] + L.co[j2] * L.Ku, L.Ku, h->g64[5] + ni.oB12, ku[c1], kv[c2]});
    cp.push_back(CnCopy{L.M + L.ro[j2] + L.co[j1] * L.Ku, L.Ku, h->g64[6] + ni.oB21, ku[c2], kv[c1]});
  }
  CnCopy* dcp = nullptr;
  if (!(stt = upload(tmp, cp, &dcp, s))) {
    launch_cn_copy(dcp, (int)cp.size(), s);
    stt = last_launch_status();
  }
  if (!stt) stt = finish_handle(h, s);
  if (!stt && hipStreamSynchronize(s) != hipSuccess) stt = HSS_EHIP;
  if (stt) {
    (void)hipStreamSynchronize(s);
    hss_destroy(h);
    return stt;
  }
  *out = h;
  return HSS_OK;
}

hss_status hss_ranks(const hss_handle* h, int32_t* ku, int32_t* kv) {
  if (!h) return -1;
  if (!ku) return -2;
  if (!kv) return -3;
  for (int32_t t = 0; t < h->plan.nnodes; ++t) {
    ku[t] = h->plan.nodes[t].ku;
    kv[t] = h->plan.nodes[t].kv;
  }
  return HSS_OK;
}

hss_status hss_get_generators(const hss_handle* h, const hss_gen_out* g, void* stream) {
  if (!h) return -1;
  if (!g) return -2;
  const Plan& P = h->plan;
  const int64_t sizes[7] = {P.nD, P.nU, P.nV, P.nR, P.nW, P.nB12, P.nB21};
  double* dst[7] = {g->D, g->U, g->V, g->R, g->W, g->B12, g->B21};
  for (int i = 0; i < 7; ++i)
    if (sizes[i] > 0 && !dst[i]) return -2;
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < 7; ++i)
    if (sizes[i] > 0 && hipMemcpyAsync(dst[i], h->g64[i], sizeof(double) * sizes[i],
                                       hipMemcpyDeviceToHost, s) != hipSuccess)
      return HSS_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? HSS_OK : HSS_EHIP;
}

hss_status hss_destroy(hss_handle* h) {
  if (!h) return HSS_OK;
  (void)hipDeviceSynchronize();
  while (!h->blocks.empty()) dev_free(h, h->blocks.back().first);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->side) (void)hipStreamDestroy(h->side);
  delete h;
  return HSS_OK;
}

hss_status hss_matmul(hss_handle* h, int32_t op, int32_t prec, int64_t nrhs, const void* X,
                      int64_t ldx, void* Y, int64_t ldy, void* stream) {
  if (!h) return -1;
  if (op != HSS_OP_N && op != HSS_OP_T) return -2;
  if (prec != HSS_F64 && prec != HSS_F32) return -3;
  if (nrhs < 0) return -4;
  if (nrhs == 0) return HSS_OK;
  if (!X) return -5;
  if (ldx < h->plan.n) return -6;
  if (!Y) return -7;
  if (ldy < h->plan.n) return -8;
  const size_t es = prec == HSS_F64 ? 8 : 4;
  const char* x0 = (const char*)X;
  const char* y0 = (const char*)Y;
  const char* x1 = x0 + es * (size_t)(ldx * (nrhs - 1) + h->plan.n);
  const char* y1 = y0 + es * (size_t)(ldy * (nrhs - 1) + h->plan.n);
  if (x0 < y1 && y0 < x1) return -7;   // X and Y overlap
  hipStream_t s = (hipStream_t)stream;
  hss_status st;
  if (prec == HSS_F64) {
    if ((st = ensure_work_mm<double>(h, nrhs))) return st;
    run_matmul<double>(h, op, nrhs, (const double*)X, ldx, (double*)Y, ldy, s);
  } else {
    if ((st = ensure_work_mm<float>(h, nrhs))) return st;
    run_matmul<float>(h, op, nrhs, (const float*)X, ldx, (float*)Y, ldy, s);
  }
  return last_launch_status();
}

hss_status hss_matmul_noalloc(hss_handle* h, int32_t op, int32_t prec, int64_t nrhs,
                              const void* X, int64_t ldx, void* Y, int64_t ldy, void* stream) {
  if (!h) return -1;
  if (op != HSS_OP_N && op != HSS_OP_T) return -2;
  if (prec != HSS_F64 && prec != HSS_F32) return -3;
  if (nrhs < 0) return -4;
  if (nrhs == 0) return HSS_OK;
  if (!X) return -5;
  if (ldx < h->plan.n) return -6;
  if (!Y) return -7;
  if (ldy < h->plan.n) return -8;
  const size_t es = prec == HSS_F64 ? 8 : 4;
  const char* x0 = (const char*)X;
  const char* y0 = (const char*)Y;
  const char* x1 = x0 + es * (size_t)(ldx * (nrhs - 1) + h->plan.n);
  const char* y1 = y0 + es * (size_t)(ldy * (nrhs - 1) + h->plan.n);
  if (x0 < y1 && y0 < x1) return -7;   // X and Y overlap
  if (noalloc_bytes(h->plan, nrhs, es) > (int64_t)kNoAllocScratchBytes) return HSS_ESCRATCH;
  char* sp = nullptr;
  hss_status st = noalloc_scratch(&sp);
  if (st) return st;
  const int64_t half = h->plan.ldm * std::max<int64_t>(nrhs, kNoAllocMinCols) * (int64_t)es;
  hipStream_t s = (hipStream_t)stream;
  if (prec == HSS_F64)
    run_matmul<double>(h, op, nrhs, (const double*)X, ldx, (double*)Y, ldy, s, nullptr,
                       reinterpret_cast<double*>(sp), reinterpret_cast<double*>(sp + half));
  else
    run_matmul<float>(h, op, nrhs, (const float*)X, ldx, (float*)Y, ldy, s, nullptr,
                      reinterpret_cast<float*>(sp), reinterpret_cast<float*>(sp + half));
  return last_launch_status();
}

int64_t hss_matmul_noalloc_max_rhs(hss_handle* h, int32_t prec) {
  if (!h || (prec != HSS_F64 && prec != HSS_F32)) return -1;
  const int64_t es = prec == HSS_F64 ? 8 : 4;
  const int64_t cols = (int64_t)kNoAllocScratchBytes / (2 * h->plan.ldm * es);
  return cols >= kNoAllocMinCols ? cols : 0;
}

hss_status hss_ulv_factor(hss_handle* h, int32_t prec, void* stream) {
  if (!h) return -1;
  if (prec != HSS_F64 && prec != HSS_F32) return -2;
  hipStream_t s = (hipStream_t)stream;
  hss_status st;
  launch_fill(reinterpret_cast<double*>(h->d_status), 0.0, 2, s);
  if (prec == HSS_F64) {
    if ((st = ensure_factors<double>(h))) return st;
    run_factor<double>(h, s);
    h->f64.valid = true;
  } else {
    if ((st = ensure_factors<float>(h))) return st;
    run_factor<float>(h, s);
    h->f32.valid = true;
  }
  return last_launch_status();
}

}  // extern "C"

namespace {

// The refined solve; fused: the factorization with opt.prec first, its
// forward sweep overlapped with the factorization (run_factor_solve).
hss_status ulv_solve_impl(hss_handle* h, int64_t nrhs, double* B, int64_t ldb,
                          const hss_solve_opts& opt, hss_solve_info* info, hipStream_t s,
                          bool fused) {
  const bool is64 = opt.prec == HSS_F64;
  if (!fused && (is64 ? !h->f64.valid : !h->f32.valid)) return HSS_ESTATE;
  const int64_t n = h->plan.n;
  const bool need_eta = nrhs > 0 && (opt.want_eta || opt.tol > 0.0);
  hss_status st;
  if (fused) {
    launch_fill(reinterpret_cast<double*>(h->d_status), 0.0, 2, s);
    if ((st = is64 ? ensure_factors<double>(h) : ensure_factors<float>(h))) return st;
  }
  if (is64) {
    if ((st = ensure_work_sv<double>(h, nrhs))) return st;
  } else {
    if ((st = ensure_work_sv<float>(h, nrhs))) return st;
  }
  if ((st = ensure_ir(h, nrhs))) return st;
  if (need_eta && (st = ensure_work_mm<double>(h, nrhs))) return st;
  double* ss = h->stats;      // bmax at 4 nrhs; [eta_max, 0, eta_0 ..] at 6 nrhs
  double* bmax = ss + 4 * nrhs;
  double* outv = ss + 6 * nrhs;
  int32_t* stb = h->d_status;
  const int32_t* gate = stb + kStGate;
  if (nrhs > 0) {
    if (need_eta) launch_copy2d(B, ldb, h->b0, n, n, nrhs, s);
    // One correction: x (+)= A^-1 rhs with the chosen factors.  FP32: each
    // column scaled by its max |.| before rounding (scaled: rmax of the last
    // check already holds it).  g: the refinement gate (NULL for the first
    // solve, which always runs).
    auto correction = [&](const double* rhs, int64_t ldr, double* x, int64_t ldx, bool accumulate,
                          const int32_t* g, bool scaled) {
      if (is64) {
        double* d = accumulate ? h->d64 : x;
        const int64_t ldd = accumulate ? n : ldx;
        if (rhs != d) launch_copy2d(rhs, ldr, d, ldd, n, nrhs, s, g);
        if (fused && !accumulate) run_factor_solve<double>(h, nrhs, d, ldd, s);
        else run_solve<double>(h, nrhs, d, ldd, s, g);
        if (accumulate) launch_axpy64(d, ldd, x, ldx, n, nrhs, s, g);
      } else {
        if (!scaled) launch_colmax(rhs, ldr, n, nrhs, h->part, h->chk_cnt, bmax, s);
        launch_scale_cast(rhs, ldr, h->r32, n, n, nrhs, bmax, s, g);
        if (fused && !accumulate) run_factor_solve<float>(h, nrhs, h->r32, n, s);
        else run_solve<float>(h, nrhs, h->r32, n, s, g);
        if (accumulate) launch_axpy_cast(h->r32, n, x, ldx, n, nrhs, bmax, s, g);
        else launch_cast_back(h->r32, n, x, ldx, n, nrhs, bmax, s);
      }
    };
    // check of step k: r = b - A x, eta, and the gate of the next correction
    auto check = [&](int k, const int32_t* g) {
      run_matmul<double>(h, HSS_OP_N, nrhs, B, ldb, h->res, n, s, g);
      launch_check(h->b0, n, h->res, n, B, ldb, n, nrhs, h->norm2, h->part, h->chk_cnt, stb,
                   bmax, outv, g, opt.tol, k, opt.max_refine, s);
    };
    correction(B, ldb, B, ldb, false, nullptr, false);
    if (need_eta) {
      check(0, nullptr);
      // refinement steps, each gated on the device by the check before it
      const int steps = opt.tol > 0.0 ? opt.max_refine : 0;
      for (int k = 1; k <= steps; ++k) {
        correction(h->res, n, B, ldb, true, gate, true);
        check(k, gate);
      }
    }
  } else if (fused) {
    if (is64) run_factor<double>(h, s);
    else run_factor<float>(h, s);
  }
  if (fused) (is64 ? h->f64.valid : h->f32.valid) = true;
  if (info) launch_solve_info(info, nrhs, outv, stb, h->norm2, opt.tol, need_eta, s);
  return last_launch_status();
}

}  // namespace

extern "C" {

hss_status hss_ulv_solve(hss_handle* h, int64_t nrhs, double* B, int64_t ldb,
                         const hss_solve_opts* o, hss_solve_info* info, void* stream) {
  if (!h) return -1;
  if (nrhs < 0) return -2;
  if (nrhs > 0 && !B) return -3;
  if (ldb < h->plan.n) return -4;
  hss_solve_opts opt{HSS_F64, 10, 0.0, 0, 0};
  if (o) opt = *o;
  if (opt.prec != HSS_F64 && opt.prec != HSS_F32) return -5;
  if (opt.max_refine < 0 || !(opt.tol >= 0.0)) return -5;
  return ulv_solve_impl(h, nrhs, B, ldb, opt, info, (hipStream_t)stream, false);
}

hss_status hss_ulv_factor_solve(hss_handle* h, int64_t nrhs, double* B, int64_t ldb,
                                const hss_solve_opts* o, hss_solve_info* info, void* stream) {
  if (!h) return -1;
  if (nrhs < 0) return -2;
  if (nrhs > 0 && !B) return -3;
  if (ldb < h->plan.n) return -4;
  hss_solve_opts opt{HSS_F64, 10, 0.0, 0, 0};
  if (o) opt = *o;
  if (opt.prec != HSS_F64 && opt.prec != HSS_F32) return -5;
  if (opt.max_refine < 0 || !(opt.tol >= 0.0)) return -5;
  return ulv_solve_impl(h, nrhs, B, ldb, opt, info, (hipStream_t)stream, true);
}

hss_status hss_query(hss_handle* h, int32_t key, void* out, void* stream) {
  if (!h) return -1;
  if (!out) return -3;
  switch (key) {
    case HSS_Q_N: *(int64_t*)out = h->plan.n; return HSS_OK;
    case HSS_Q_P: *(int32_t*)out = h->plan.p; return HSS_OK;
    case HSS_Q_RESIDENT_BYTES: *(int64_t*)out = h->resident; return HSS_OK;
    case HSS_Q_GEN_ENTRIES: *(int64_t*)out = h->plan.gen_entries(); return HSS_OK;
    case HSS_Q_FACTOR_ENTRIES: *(int64_t*)out = h->plan.factor_entries(); return HSS_OK;
    case HSS_Q_NORM2: *(double*)out = h->norm2; return HSS_OK;
    default: return -2;
  }
}

hss_status hss_batch_matmul(hss_handle* const* hs, int32_t count, int32_t op, int32_t prec,
                            const int64_t* nrhs, const void* const* X, const int64_t* ldx,
                            void* const* Y, const int64_t* ldy, void* stream) {
  if (!hs) return -1;
  if (count < 0) return -2;
  if (op != HSS_OP_N && op != HSS_OP_T) return -3;
  if (prec != HSS_F64 && prec != HSS_F32) return -4;
  if (count > 0 && (!nrhs || !X || !ldx || !Y || !ldy)) return -5;
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i] || nrhs[i] < 0 || (nrhs[i] > 0 && (!X[i] || !Y[i])) || ldx[i] < hs[i]->plan.n ||
        ldy[i] < hs[i]->plan.n)
      return -5;
  }
  if (count == 0) return HSS_OK;
  hipStream_t s = (hipStream_t)stream;
  return prec == HSS_F64
             ? batch_matmul<double>(hs, count, op, nrhs, X, ldx, Y, ldy, s)
             : batch_matmul<float>(hs, count, op, nrhs, X, ldx, Y, ldy, s);
}

hss_status hss_batch_ulv_factor(hss_handle* const* hs, int32_t count, int32_t prec, void* stream) {
  if (!hs) return -1;
  if (count < 0) return -2;
  if (prec != HSS_F64 && prec != HSS_F32) return -3;
  for (int32_t i = 0; i < count; ++i)
    if (!hs[i]) return -1;
  if (count == 0) return HSS_OK;
  hipStream_t s = (hipStream_t)stream;
  return prec == HSS_F64 ? batch_factor<double>(hs, count, s) : batch_factor<float>(hs, count, s);
}

hss_status hss_batch_ulv_solve(hss_handle* const* hs, int32_t count, const int64_t* nrhs,
                               double* const* B, const int64_t* ldb, const hss_solve_opts* o,
                               hss_solve_info* const* info, void* stream) {
  if (!hs) return -1;
  if (count < 0) return -2;
  if (count > 0 && (!nrhs || !B || !ldb)) return -3;
  hss_solve_opts opt{HSS_F64, 10, 0.0, 0, 0};
  if (o) opt = *o;
  if (opt.prec != HSS_F64 && opt.prec != HSS_F32) return -6;
  if (opt.max_refine < 0 || !(opt.tol >= 0.0)) return -6;
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i] || nrhs[i] < 0 || (nrhs[i] > 0 && !B[i]) || ldb[i] < hs[i]->plan.n) return -3;
    if (opt.prec == HSS_F64 ? !hs[i]->f64.valid : !hs[i]->f32.valid) return HSS_ESTATE;
  }
  if (count == 0) return HSS_OK;
  return batch_solve(hs, count, nrhs, B, ldb, opt, info, (hipStream_t)stream);
}

hss_status hss_autotune(hss_handle* h, int64_t nrhs, int32_t prec, void* stream, char* report,
                        int64_t cap) {
  if (!h) return -1;
  if (nrhs < 1) return -2;
  if (prec != HSS_F64 && prec != HSS_F32) return -3;
  hipStream_t s = (hipStream_t)stream;
  const TuneKey key = tune_key(h->plan, prec, nrhs);
  TuneVal tv;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) tv = it->second;
  }
  bool did_mm = false, did_sv = false;
  const hss_status st = prec == HSS_F64 ? autotune<double>(h, nrhs, s, tv, did_mm, did_sv)
                                        : autotune<float>(h, nrhs, s, tv, did_mm, did_sv);
  if (st) return st;
  if (did_mm || did_sv) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = tv;
  }
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "{\"leaf_mp\": %d, \"max_k\": %d, \"depth\": %d, \"prec\": %d, "
                "\"rhs_bucket\": %d, \"product_tuned\": %s, \"product_us\": [%.2f, %.2f], "
                "\"product_wide\": %d, \"solve_tuned\": %s, \"solve_us\": [%.2f, %.2f], "
                "\"solve_cpw\": %d}",
                key.leaf_mp, key.max_k, key.p, key.prec, key.bucket, did_mm ? "true" : "false",
                tv.t_mm[0], tv.t_mm[1], tv.mm, did_sv ? "true" : "false", tv.t_sv[0], tv.t_sv[1],
                tv.cpw);
  return copy_out(buf, report, cap);
}

hss_status hss_tune_table(char* buf, int64_t cap) {
  std::string txt;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto& kv : g_tune) txt += tune_line(kv.first, kv.second);
  }
  if (!buf) return -1;
  if (cap <= 0) return -2;
  return copy_out(txt, buf, cap);
}

hss_status hss_tune_load(const char* text) {
  if (!text) return -1;
  std::vector<std::pair<TuneKey, TuneVal>> rows;
  const char* p = text;
  while (*p) {
    TuneKey k{};
    TuneVal v;
    int used = 0;
    const int got = std::sscanf(p, "%d %d %d %d %d %d %d %lf %lf %lf %lf%n", &k.leaf_mp, &k.max_k,
                                &k.p, &k.prec, &k.bucket, &v.mm, &v.cpw, &v.t_mm[0], &v.t_mm[1],
                                &v.t_sv[0], &v.t_sv[1], &used);
    if (got != 11) return -1;
    if (v.mm < -1 || v.mm > 1 || (v.cpw != 0 && v.cpw != 1 && v.cpw != 4) || k.bucket < 0 ||
        k.bucket > 5 || (k.prec != HSS_F64 && k.prec != HSS_F32))
      return -1;
    rows.emplace_back(k, v);
    p += used;
    while (*p == '\n' || *p == ' ' || *p == '\r' || *p == '\t') ++p;
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto& r : rows) g_tune[r.first] = r.second;
  return HSS_OK;
}

hss_status hss_tune_reset(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
  return HSS_OK;
}

}  // extern "C"
