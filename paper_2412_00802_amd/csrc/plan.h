// Host-side evaluation plans: a batch of postfix hypotheses becomes one
// canonical DAG (shared subexpressions evaluated once) scheduled by role
// nesting level.  The paper generates an evaluation plan per hypothesis on the
// CPU before running its DL operations (Section 4, "evaluation plan").
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "kb_handle.h"

namespace hth {

// A cross-batch cache of role-node rows (plan.cpp): canonical subexpressions
// of every batch compiled with it are interned in one persistent DAG, so that
// equal subexpressions of different batches get the same id; a role node whose
// id holds a row is read from that row, and a role node without one may be
// given the least recently used row to write its result into.
struct SubexprCache;
SubexprCache* cache_new(uint32_t n_rows);
void cache_delete(SubexprCache* c);
struct CacheCounters {
  uint64_t hits = 0, misses = 0, admitted = 0, evictions = 0, batches = 0;
  uint32_t entries = 0, rows = 0;
};
CacheCounters cache_counters(const SubexprCache* c);
// Undo the admissions of the last compiled batch (its launch did not happen).
void cache_rollback(SubexprCache* c);

struct PlanOptions {
  SubexprCache* cache = nullptr; // cross-batch cache of role-node rows (the set table)
  bool instances = false;        // write the (single) root's instance set
  uint32_t group_min = 0xFFFFFFFFu;  // (role, dir, level) buckets with at least this many
                                     // role nodes use a shared CSR pass; others run alone
  uint32_t group_k = 64;             // most role nodes per shared pass
};

struct PlanLevel {
  std::vector<RegionTask> mat;      // children materialised before this level's role passes
  std::vector<RoleTask> roles;      // single role nodes (k = 1)
  std::vector<GroupTask> groups;    // shared passes (k <= 64)
  std::vector<GroupMember> members;
};

struct Plan {
  std::vector<ThrTask> thr;
  std::vector<NumTask> num;         // restrictions on numeric concrete roles
  // the numeric concrete roles the plan was compiled against
  const uint32_t* num_roff = nullptr;
  const float* num_val = nullptr;
  const uint32_t* num_heavy_rows = nullptr;
  const HeavyChunk* num_heavy_chunks = nullptr;
  std::vector<uint32_t> num_chunk_first;
  std::vector<uint64_t> num_bounds;        // [P+1] first value of each numeric role
  std::vector<StrTask> str;                // restrictions on string concrete roles
  const uint32_t* str_roff = nullptr;
  const int32_t* str_ids = nullptr;
  const uint32_t* str_heavy_rows = nullptr;
  const HeavyChunk* str_heavy_chunks = nullptr;
  std::vector<uint32_t> str_chunk_first;
  std::vector<uint64_t> str_bounds;
  const int64_t* dict_off = nullptr;
  const uint8_t* dict_chars = nullptr;
  const int64_t* pat_off = nullptr;
  const uint8_t* pat_chars = nullptr;
  uint32_t n_strings = 0;
  std::vector<uint32_t> code;
  std::vector<PlanLevel> levels;
  std::vector<RegionTask> roots;
  uint32_t n_slots = 0;
  const uint64_t* sets = nullptr;   // the set table the plan's HTH_SET rows refer to
  uint32_t n_sets = 0;
  // statistics
  uint32_t n_input_nodes = 0, n_canonical = 0, n_role_nodes = 0;
};

// Compile hypotheses nodes[hyp_off[h] .. hyp_off[h+1]) (local child indices).
hth_status compile_plan(const hth_kb_s& kb, const hth_node* nodes, const uint32_t* hyp_off,
                        uint32_t n_hyps, const uint32_t* children, uint32_t n_children,
                        const PlanOptions& opt, Plan& out);

}  // namespace hth
