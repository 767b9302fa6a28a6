// Host plan: validated tree, per-node sizes and every packed / work / factor
// offset (integer arithmetic only; Def. 2.1 cluster tree, Sec. 2.2 generator
// shapes, Sec. 4.3 merged block sizes).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hss.h"
#include "hss_internal.hpp"

namespace hss {

struct Plan {
  int64_t n = 0;
  int32_t p = 0;
  int32_t nnodes = 0;
  std::vector<int64_t> leaf_off;
  std::vector<NodeInfo> nodes;
  // packed generator sizes (entries)
  int64_t nD = 0, nU = 0, nV = 0, nR = 0, nW = 0, nB12 = 0, nB21 = 0;
  // factor sizes (entries)
  int64_t nFD = 0, nFU = 0, nFV = 0, ntq = 0, ntz = 0, nFZ = 0;
  int64_t nOP = 0;   // forward-operator records of the internal nodes
  int64_t ldm = 0;   // product work rows
  int64_t lds = 0;   // solve work rows
  int32_t max_m = 0, max_mp = 0, max_k = 0;
  int32_t leaf_max_ku = 0;
  std::vector<int32_t> level_max_mp;   // per level l = 0..p
  // LDS copies (elements) the forward / backward sweeps of an internal level
  // need when they stage a node's factors (max over the level); root: the
  // children's blocks only (its FP64 LU is added separately)
  std::vector<int64_t> level_fwd_stage, level_bwd_stage;
  // per level: every node has a forward-operator record
  std::vector<int8_t> level_fwd_op;
  int64_t gen_entries() const { return nD + nU + nV + nR + nW + nB12 + nB21; }
  int64_t factor_entries() const { return nFD + nFU + nFV + ntq + ntz + nFZ + nOP; }
};

// Returns 0 or a status (negative = invalid argument index as in hss.h).
hss_status build_plan(const hss_tree_desc* tree, Plan& plan, std::string* why);

int32_t default_depth(int64_t n, int64_t nmin);

}  // namespace hss
