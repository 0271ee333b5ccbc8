// Internal declarations shared by the host code and the kernels of libhthedl.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "hthedl.h"

namespace hth {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kStackDepth = 16;       // region-program value stack (per lane, in LDS)
constexpr int kRegionThreads = 256;   // lanes = words
constexpr int kMaxK = 64;             // role nodes sharing one CSR pass (bits of a T row)

// ---------------------------------------------------------------------------
// region programs: postfix bytecode over bit rows, one lane per 64-bit word
//   bits 0-3 opcode, bit 4 negate (LEAF only), bits 5-31 argument
// ---------------------------------------------------------------------------
enum : uint32_t {
  RP_LEAF = 0,   // push row `arg` (see row_ptr)
  RP_TOP = 1,
  RP_BOT = 2,
  RP_NOT = 3,    // complement the top of the stack
  RP_AND = 4,    // pop b, top &= b
  RP_OR = 5,     // pop b, top |= b
};
__host__ __device__ inline uint32_t rp_ins(uint32_t op, uint32_t neg, uint32_t arg) {
  return op | (neg << 4) | (arg << 5);
}

// One boolean region evaluated over all words.
struct RegionTask {
  uint32_t code_off;   // into the code table
  uint32_t code_len;
  uint32_t out_row;    // row id to write (n_concepts + slot), kNone = none, kInstances
  uint32_t cover;      // hypothesis index for coverage, kNone = none
};
constexpr uint32_t kInstances = 0xFFFFFFFEu;   // out_row: the caller's instance buffer

// One numeric threshold row: bit x = value_p(x) >= t (cmp 0), <= t (cmp 1)
// or == t (cmp 2); NaN -> 0.
struct ThrTask {
  uint32_t prop;
  uint32_t cmp;
  float t;
  uint32_t out_row;
};

// One restriction on a multi-valued numeric concrete role: bit x = some value
// of x in role `role` is >= t (cmp 0), <= t (cmp 1) or == t (cmp 2).  Heavy
// rows of the role (see HeavyChunk; numeric tables) are tested chunk by chunk.
struct NumTask {
  uint32_t role;
  uint32_t cmp;
  float t;
  uint32_t out_row;
  uint32_t h_first;    // first block of this task in its heavy-row launch
  uint32_t hc0;        // first chunk of the role in the numeric chunk table
  uint32_t base_lo, base_hi;   // the role's first value (its offsets are relative to it)
};

// One restriction on a string concrete role: bit x = some value id of x in
// role `role` equals q (kind 0, EQUAL) or lies in the id set at word
// `set_word` of the plan's id-set area (kind 1, CONTAIN: the dictionary ids
// whose string holds pattern q, written first by k_contains).
struct StrTask {
  uint32_t role;
  uint32_t kind;
  uint32_t q;
  uint32_t out_row;
  uint32_t h_first;    // first block of this task in its heavy-row launch
  uint32_t hc0;        // first chunk of the role in the string chunk table
  uint32_t set_word;
  uint32_t pad;
  uint32_t base_lo, base_hi;   // the role's first value (its offsets are relative to it)
};

// The thresholds on one property, tasks[first .. first + n) (n <= 32).
// Thresholds on one property served by one pass over its column (the values
// stay in registers while each threshold's words are written).
constexpr uint32_t kThrPerPass = 32;
struct ThrGroup {
  uint32_t prop;
  uint32_t first;
  uint32_t n;
  uint32_t pad;
};

// One role restriction over one CSR direction, evaluated alone (k = 1).
//   cnt(x) = #{y in succ(x) : bit(child, y) ^ neg};  result = lo <= cnt <= hi
//   counting may stop at `sat` (every predicate is decided once cnt >= sat).
struct RoleTask {
  uint32_t role;
  uint32_t inv;
  uint32_t child_row;  // concept id or n_concepts + slot
  uint32_t neg;        // 0/1: complement the child before counting
  uint32_t lo, hi, sat;
  uint32_t out_row;    // n_concepts + slot
  uint32_t n_words;    // non-empty words of (role, inv), set at launch
  // heavy rows of (role, inv), set at launch (see HeavyChunk)
  uint32_t h_first;    // first block of this task in its level's heavy-row launch
  uint32_t c_first;    // first (task, heavy row) pair of this task in its level
  uint32_t hc0;        // first chunk of the direction in the chunk table
  uint32_t hr0;        // first heavy row of the direction in the heavy-row table
};

// Subjects with more than DevKB::heavy_min assertions in a direction ("heavy
// rows") are left out of the one-wave-per-word pass: their assertions are cut
// into chunks of kHeavyChunk, every chunk is counted by one block into a
// partial count of its own, and a last kernel sums the partials of each
// (task, heavy row) and sets the row's bit.  The chunk table lists, per
// direction, chunk k of heavy row `hrow` (an index into the heavy-row table,
// which holds the subjects); heavy_chunk0[hrow] is the row's first chunk.
constexpr uint32_t kHeavyChunk = 4096;
constexpr uint32_t kHeavyMinFloor = 1024;   // smallest heavy-row threshold
struct HeavyChunk {
  uint32_t hrow;
  uint32_t k;
};

// Output rows of role nodes whose (role, direction) has words without any
// assertion: those words hold the zero-count result, all ones or all zeros.
struct FillTask {
  uint32_t out_row;
  uint32_t ones;
};

// A CSR pass shared by up to 64 role nodes of one (role, direction, level):
// the children are first transposed into T[y] (bit j = child j contains y,
// after its negation flag), then one pass over the CSR counts all of them.
// Members count with saturating 3-bit counters (0..7, and >= 8), so a group
// only holds nodes whose predicate is decided there: lo <= 8 and hi <= 7 or
// unbounded.  acc[v] bit j = member j accepts count v (acc[8]: count >= 8).
struct GroupTask {
  uint32_t role;
  uint32_t inv;
  uint32_t k;          // nodes in the group, 1..64
  uint32_t first;      // index of the group's first member in the member table
  uint64_t acc[9];
  uint32_t n_words;    // non-empty words of (role, inv), set at launch
  uint32_t compact;    // 1: T holds the direction's objects only, indexed by object rank
  uint64_t t_off;      // first T row of the group in the T area (in T rows)
  uint32_t short_rows; // 1: every row of (role, inv) is short: one lane walks each subject
  uint32_t n_obj_words;  // words holding objects of (role, inv): the non-empty words of
                         // the other direction (its word list), set with n_words
};
constexpr uint32_t kGroupMaxCount = 8;
// A member whose node is the root of exactly one hypothesis and read by no
// other node has no output row (out_row = kNone): the pass adds its words'
// coverage of the examples into that hypothesis's counts (cover) instead.
struct GroupMember {
  uint32_t child_row;
  uint32_t neg;
  uint32_t lo, hi, sat;
  uint32_t out_row;    // n_fixed + slot, or kNone with cover set
  uint32_t cover;      // hypothesis index, or kNone
  uint32_t pad;
};

// Device view of the knowledge base and of one call's buffers (by value).
struct DevKB {
  const uint64_t* concepts;   // [C][S]
  const uint64_t* sets;       // [n_sets][S] caller's set table (HTH_SET leaves)
  uint64_t* slots;            // [n_slots][S] (workspace)
  const float* data;          // [D][N]
  const uint32_t* fwd_off;    // [R][N+1], relative to the role's first assertion
  const uint32_t* inv_off;    // [R][N+1]
  const int32_t* fwd_tg;      // [E]
  const int32_t* inv_tg;      // [E]
  const uint64_t* role_base;  // [R] first assertion of each role (both directions)
  const uint32_t* words;      // [R][2][W] non-empty words (role r, direction d at row 2r + d)
  const uint64_t* objmask;    // [R][2][W] objects of each role direction
  const uint32_t* objbase;    // [R][2][W+1] objects before each word
  const int32_t* ctg_fwd;     // [E] object ranks of the forward targets
  const int32_t* ctg_inv;     // [E] object ranks of the inverse targets
  const uint32_t* heavy_rows; // subjects of the heavy rows, by direction 2r + dir, increasing
  const HeavyChunk* heavy_chunks;  // by direction, then heavy row, then k
  const uint32_t* heavy_chunk0;    // [heavy rows + 1] first chunk of each heavy row
  const uint32_t* num_roff;        // [P][N+1] numeric concrete roles, relative to each role's first value
  const float* num_val;            // [V]
  const uint32_t* num_heavy_rows;  // subjects of the numeric roles' heavy rows, by role
  const HeavyChunk* num_heavy_chunks;
  const uint32_t* str_roff;        // [Q][N+1] string concrete roles, relative to each role's first id
  const int32_t* str_ids;          // [V'] dictionary ids
  const uint32_t* str_heavy_rows;
  const HeavyChunk* str_heavy_chunks;
  const int64_t* dict_off;         // [n_strings+1] the dictionary
  const uint8_t* dict_chars;
  const int64_t* pat_off;          // [n_patterns+1] CONTAIN patterns
  const uint8_t* pat_chars;
  uint64_t* idsets;                // the plan's id-set area (workspace)
  uint32_t n_strings;
  const uint64_t* pos;        // [S]
  const uint64_t* neg;        // [S]
  uint32_t* counts;           // [n_hyps][2]
  uint64_t* instances;        // [S] or null
  uint32_t n_concepts;
  uint32_t n_fixed;           // n_concepts + n_sets: first workspace slot row
  uint32_t N, W, S;
  uint32_t heavy_min;         // rows with more assertions are heavy rows
  uint64_t tail;              // valid-bit mask of word W-1
};

// Row ids: [0, C) concepts, [C, C + n_sets) the set table, then workspace slots.
__device__ __forceinline__ const uint64_t* row_ptr(const DevKB& kb, uint32_t id) {
  if (id < kb.n_concepts) return kb.concepts + (size_t)id * kb.S;
  if (id < kb.n_fixed) return kb.sets + (size_t)(id - kb.n_concepts) * kb.S;
  return kb.slots + (size_t)(id - kb.n_fixed) * kb.S;
}
__device__ __forceinline__ uint64_t* out_ptr(const DevKB& kb, uint32_t id) {
  if (id == kInstances) return kb.instances;
  // a row of the set table: written when the table is a subexpression cache
  if (id < kb.n_fixed) return const_cast<uint64_t*>(kb.sets) + (size_t)(id - kb.n_concepts) * kb.S;
  return kb.slots + (size_t)(id - kb.n_fixed) * kb.S;
}

}  // namespace hth

