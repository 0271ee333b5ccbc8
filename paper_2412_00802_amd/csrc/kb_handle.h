// Host state of a knowledge-base handle, the schedule knobs and the error
// helpers (host code only; the device-side structures are in hth_internal.h).
#pragma once

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "hth_internal.h"

// ---------------------------------------------------------------------------
// the knowledge-base handle
// ---------------------------------------------------------------------------
struct hth_kb_s {
  hth_kb_desc d;
  uint32_t N = 0, W = 0, S = 0;
  uint64_t tail = 0;
  uint32_t* fwd_off = nullptr;
  uint32_t* inv_off = nullptr;
  int32_t* inv_tg = nullptr;
  uint64_t* role_base_dev = nullptr;
  uint32_t* words = nullptr;           // [R][2][W] non-empty words per role and direction
  std::vector<uint32_t> n_words;       // [R][2]
  std::vector<uint64_t> role_base;     // [R+1]
  std::vector<uint32_t> max_deg[2];    // [R] forward, inverse
  uint64_t* objmask = nullptr;         // [R][2][W] objects of each role direction
  uint32_t* objbase = nullptr;         // [R][2][W+1] objects before each word
  int32_t* ctg_fwd = nullptr;          // [E] object ranks of the forward targets
  int32_t* ctg_inv = nullptr;          // [E] object ranks of the inverse targets
  std::vector<uint32_t> n_obj;         // [R][2]; ranks exist where 2 n_obj <= N
  uint32_t heavy_min = 2048;           // rows with more assertions are heavy rows
  uint32_t* heavy_rows = nullptr;      // subjects of the heavy rows, by direction
  hth::HeavyChunk* heavy_chunks = nullptr;
  uint32_t* heavy_chunk0 = nullptr;    // first chunk of each heavy row, then the total
  std::vector<uint32_t> heavy_first;   // [2R+1] first heavy row of direction 2r + dir
  std::vector<uint32_t> chunk_first;   // [2R+1] first chunk of direction 2r + dir
  uint32_t heavy_most = 0;             // most heavy rows in one direction
  uint32_t chunk_most = 0;             // most heavy chunks in one direction
  std::vector<uint32_t> concept_pop;   // [C] members of each concept
  // multi-valued numeric concrete roles (hth_kb_set_numeric): caller's arrays
  uint32_t n_num = 0;
  const int64_t* num_off = nullptr;    // [n_num][N+1]
  const float* num_val = nullptr;
  uint32_t* num_heavy_rows = nullptr;  // in the caller's numeric derived buffer
  hth::HeavyChunk* num_heavy_chunks = nullptr;
  std::vector<uint32_t> num_chunk_first;   // [n_num+1] first chunk of each role
  std::vector<uint64_t> num_bounds;        // [n_num+1] first value of each role
  uint32_t* num_roff = nullptr;            // [n_num][N+1] relative offsets (numeric derived buffer)
  // string concrete roles (hth_kb_set_strings) and CONTAIN patterns
  uint32_t n_str = 0, n_strings = 0, n_patterns = 0;
  const int64_t* str_off = nullptr;
  const int32_t* str_ids = nullptr;
  const int64_t* dict_off = nullptr;
  const uint8_t* dict_chars = nullptr;
  const int64_t* pat_off = nullptr;
  const uint8_t* pat_chars = nullptr;
  uint32_t* str_heavy_rows = nullptr;
  hth::HeavyChunk* str_heavy_chunks = nullptr;
  std::vector<uint32_t> str_chunk_first;   // [n_str+1]
  std::vector<uint64_t> str_bounds;        // [n_str+1]
  uint32_t* str_roff = nullptr;            // [n_str][N+1] relative offsets (string derived buffer)
  const uint64_t* pos = nullptr;
  const uint64_t* neg = nullptr;
  const uint64_t* sets = nullptr;      // caller's set table (hth_kb_set_sets)
  uint32_t n_sets = 0;
  int device = 0;
  int n_cu = 256;
  size_t lds_per_block = 65536;
  std::mutex mu;
  // measurement (hth_profile_begin/end)
  struct ProfRec {
    int kind;
    double bytes;
    hipEvent_t a, b;
  };
  bool prof = false;
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> event_pool;
  ~hth_kb_s() {
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
  }
  // schedule choices of the batched executor (defaults, environment overrides
  // HTHEDL_GROUP_MIN / _GROUP_K / _XCD / _TBUDGET_MB)
  struct Tuning {
    uint32_t group_min = 2;      // smallest (role, dir, level) bucket run as shared passes
    uint32_t group_k = 64;       // most role nodes per shared pass (T row width)
    uint32_t xcd_local = 1;      // 1: all blocks of a shared pass on one XCD
    size_t t_budget = 1024ull << 20; // bytes of T rows one launch of shared passes may use
    uint32_t group_unroll = 16;  // assertions in flight per lane in a dense shared pass
    uint32_t region_reg = 2;     // words per lane of the register-stack region kernel (0: LDS kernel)
    uint32_t t_compact = 1;      // 1: T rows of objects only where they are <= N/2
    uint32_t t_segment_kb = 0;   // T bytes per pass of a shared pass (0: one pass over all rows)
    uint32_t push_pct = 2;       // single ∃ρ.A with A under this % of N: pushed from A's members (0: never)
    uint32_t short_rows = 12;    // shared passes over directions whose rows are all at most this long walk
                                 // one subject per lane (0: never)
  } tune;
};

namespace hth {

// error reporting (thread-local message)
void set_error(const std::string& msg);
hth_status fail(hth_status code, const std::string& msg);
hth_status hip_fail(hipError_t e, const char* what);

#define HTH_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return ::hth::hip_fail(_e, #call); \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// The smallest bucket of role nodes over direction rd (2 role + dir) that runs
// as shared passes, given the schedule's group_min (0xFFFFFFFF: never): one
// node where the direction's rows are all short or at most half of its words
// hold assertions (a one-node shared pass is faster there than the single-node
// kernel, which walks every listed word for one node), else group_min.
inline uint32_t bucket_min(const hth_kb_s& kb, uint32_t rd, uint32_t group_min) {
  if (group_min == 0xFFFFFFFFu) return group_min;
  const bool short_dir = kb.tune.short_rows && kb.max_deg[rd & 1][rd >> 1] <= kb.tune.short_rows;
  const bool sparse = rd < kb.n_words.size() && 2ull * kb.n_words[rd] <= kb.W;
  return short_dir || sparse ? std::min<uint32_t>(group_min, 1u) : group_min;
}

}  // namespace hth
