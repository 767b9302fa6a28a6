// Host plan builder.  Heap numbering (children 2t+1, 2t+2); levels are
// contiguous heap ranges, so a level launch covers nodes 2^l-1 .. 2^(l+1)-2.
#include "plan.hpp"

#include <algorithm>

namespace hss {

int32_t default_depth(int64_t n, int64_t nmin) {
  // Sec. 3.1: ceil-halving until every block has at most nmin indices; the
  // largest block of level l has ceil(n / 2^l) indices.
  if (n <= 0 || nmin <= 0) return -1;
  int32_t p = 0;
  int64_t big = n;
  while (big > nmin) {
    big = (big + 1) / 2;
    ++p;
  }
  return p;
}

hss_status build_plan(const hss_tree_desc* tree, Plan& P, std::string* why) {
  auto fail = [&](hss_status s, const char* msg) {
    if (why) *why = msg;
    return s;
  };
  if (!tree) return fail(-1, "tree is NULL");
  if (tree->n <= 0) return fail(-1, "n must be positive");
  if (tree->p < 0 || tree->p > 24) return fail(-1, "p out of range");
  if (!tree->leaf_off || !tree->ku || !tree->kv) return fail(-1, "tree arrays are NULL");
  const int32_t p = tree->p;
  const int64_t nleaf = int64_t(1) << p;
  const int32_t nn = int32_t((int64_t(2) << p) - 1);
  if (tree->leaf_off[0] != 0 || tree->leaf_off[nleaf] != tree->n)
    return fail(-1, "leaf_off must run from 0 to n");
  for (int64_t i = 0; i < nleaf; ++i)
    if (tree->leaf_off[i + 1] <= tree->leaf_off[i])
      return fail(-1, "leaf_off must be strictly increasing (empty leaves unsupported)");
  for (int32_t t = 1; t < nn; ++t) {
    if (tree->ku[t] < 0 || tree->kv[t] < 0) return fail(-1, "negative rank");
    if (tree->ku[t] > kMaxRank || tree->kv[t] > kMaxRank)
      return fail(HSS_EUNSUP, "rank above the supported maximum");
  }
  P = Plan();
  P.n = tree->n;
  P.p = p;
  P.nnodes = nn;
  P.leaf_off.assign(tree->leaf_off, tree->leaf_off + nleaf + 1);
  P.nodes.assign(nn, NodeInfo{});
  // index sets: leaves from leaf_off, parents as unions
  for (int32_t t = nn - 1; t >= 0; --t) {
    NodeInfo& d = P.nodes[t];
    int32_t l = 0;
    while ((int64_t(2) << l) - 1 <= t) ++l;
    d.level = l;
    d.is_leaf = (l == p);
    d.ku = t == 0 ? 0 : tree->ku[t];
    d.kv = t == 0 ? 0 : tree->kv[t];
    if (d.is_leaf) {
      const int64_t i = t - (nleaf - 1);
      d.row0 = tree->leaf_off[i];
      d.m = int32_t(tree->leaf_off[i + 1] - tree->leaf_off[i]);
      if (tree->leaf_off[i + 1] - tree->leaf_off[i] > kMaxBlock)
        return fail(HSS_EUNSUP, "leaf larger than the supported block size");
    } else {
      const NodeInfo& a = P.nodes[2 * t + 1];
      const NodeInfo& b = P.nodes[2 * t + 2];
      d.row0 = a.row0;
      const int64_t m = int64_t(a.m) + b.m;
      d.m = m > INT32_MAX ? INT32_MAX : int32_t(m);
    }
  }
  // merged block sizes (Sec. 4.3 Step 3): leaf mp = m; internal mp = kept(c1) + kept(c2)
  for (int32_t t = nn - 1; t >= 0; --t) {
    NodeInfo& d = P.nodes[t];
    if (d.is_leaf) d.mp = d.m;
    else d.mp = P.nodes[2 * t + 1].kept + P.nodes[2 * t + 2].kept;
    if (t == 0) {
      d.e = 0;
      d.kept = d.mp;
    } else {
      d.e = std::max(d.mp - d.ku, 0);
      d.kept = d.mp - d.e;
    }
    if (d.mp > kMaxBlock) return fail(HSS_EUNSUP, "merged block larger than supported");
  }
  // offsets
  int64_t oD = 0, oU = 0, oV = 0, oR = 0, oW = 0, o12 = 0, o21 = 0;
  int64_t oFD = 0, oFU = 0, oFV = 0, otq = 0, otz = 0, oFZ = 0, oOP = 0;
  int64_t oxh = 0, oc = 0, oz = 0, oy = 0;
  for (int32_t t = 0; t < nn; ++t) {
    NodeInfo& d = P.nodes[t];
    d.oD = d.oU = d.oV = d.oR = d.oW = d.oB12 = d.oB21 = -1;
    if (d.is_leaf) {
      d.oD = oD; oD += int64_t(d.m) * d.m;
      if (p > 0) {
        d.oU = oU; oU += int64_t(d.m) * d.ku;
        d.oV = oV; oV += int64_t(d.m) * d.kv;
      }
    } else {
      const NodeInfo& a = P.nodes[2 * t + 1];
      const NodeInfo& b = P.nodes[2 * t + 2];
      if (t != 0) {
        d.oR = oR; oR += int64_t(a.ku + b.ku) * d.ku;
        d.oW = oW; oW += int64_t(a.kv + b.kv) * d.kv;
      }
      d.oB12 = o12; o12 += int64_t(a.ku) * b.kv;
      d.oB21 = o21; o21 += int64_t(b.ku) * a.kv;
    }
    const int32_t kmax = std::max(d.ku, d.kv);
    d.oxh = oxh;
    d.oyh = oxh;   // x^ and y^ live in separate buffers with the same row offsets
    oxh += kmax;
    d.oFD = oFD; oFD += int64_t(d.mp) * d.mp;
    d.oFU = oFU; oFU += int64_t(d.mp) * d.ku;
    d.oFV = oFV; oFV += int64_t(d.mp) * d.kv;
    d.otq = otq; otq += d.ku;
    d.otz = otz; otz += d.e;
    d.oFZ = oFZ; oFZ += int64_t(d.mp) * d.e;
    int child_k = 0;
    if (!d.is_leaf) {
      const NodeInfo& a = P.nodes[2 * t + 1];
      const NodeInfo& b = P.nodes[2 * t + 2];
      child_k = std::max(std::max(a.ku, a.kv), std::max(b.ku, b.kv));
    }
    if (fwd_op_ok(d.is_leaf, t, d.mp, d.e, d.ku, d.kv, child_k)) {
      d.oOP = oOP; oOP += kRecSize;
    } else {
      d.oOP = -1;
    }
    d.oc = oc; d.ox = oc; oc += d.kept;
    d.oz = oz; oz += d.kv;
    d.oy = oy; oy += d.e;
    P.max_m = std::max(P.max_m, d.is_leaf ? d.m : 0);
    P.max_mp = std::max(P.max_mp, d.mp);
    P.max_k = std::max(P.max_k, kmax);
    if (d.is_leaf) P.leaf_max_ku = std::max(P.leaf_max_ku, d.ku);
  }
  P.level_fwd_stage.assign(p + 1, 0);
  P.level_bwd_stage.assign(p + 1, 0);
  for (int32_t t = 0; t < nn; ++t) {
    const NodeInfo& d = P.nodes[t];
    if (d.is_leaf) continue;
    const NodeInfo& a = P.nodes[2 * t + 1];
    const NodeInfo& b = P.nodes[2 * t + 2];
    const int64_t kw = a.kv + b.kv;
    const int64_t f = int64_t(d.mp) * (d.e > 0 ? d.ku : 0) + int64_t(d.mp) * d.e +
                      int64_t(d.e) * d.kv + kw * d.kv + int64_t(a.kept) * a.ku +
                      int64_t(b.kept) * b.ku + int64_t(a.ku) * b.kv + int64_t(b.ku) * a.kv;
    P.level_fwd_stage[d.level] = std::max(P.level_fwd_stage[d.level], f);
    P.level_bwd_stage[d.level] =
        std::max(P.level_bwd_stage[d.level], int64_t(d.mp) * d.e);
  }
  P.level_fwd_op.assign(p + 1, 1);
  for (int32_t t = 0; t < nn; ++t)
    if (P.nodes[t].oOP < 0) P.level_fwd_op[P.nodes[t].level] = 0;
  P.level_max_mp.assign(p + 1, 0);
  for (int32_t t = 0; t < nn; ++t)
    P.level_max_mp[P.nodes[t].level] = std::max(P.level_max_mp[P.nodes[t].level], P.nodes[t].mp);
  P.nD = oD; P.nU = oU; P.nV = oV; P.nR = oR; P.nW = oW; P.nB12 = o12; P.nB21 = o21;
  P.nFD = oFD; P.nFU = oFU; P.nFV = oFV; P.ntq = otq; P.ntz = otz; P.nFZ = oFZ;
  P.nOP = oOP;
  P.ldm = std::max<int64_t>(oxh, 1);
  P.lds = std::max<int64_t>(std::max(oc, std::max(oz, oy)), 1);
  return HSS_OK;
}

}  // namespace hss
