// Kernels and the executor of libhthedl.
//
// Work decomposition (all bit rows are uint64 words, 64 individuals each):
//   k_threshold  numeric restriction (Algorithms 9/10): one lane per individual,
//                one wave ballot per output word.
//   k_region     n-ary and/or/not over bit rows (Algorithms 1/2): one lane per
//                word, the region's postfix bytecode interpreted with a value
//                stack in LDS; coverage (Algorithm 15) fused: popcount against
//                the example rows, wave reduction, one atomic per wave.
//   k_role       role restrictions (Algorithms 3-8) over a CSR direction: one
//                wave per 64 consecutive subjects; the wave walks the subjects'
//                concatenated assertion range in chunks of 64 (coalesced target
//                loads, eight chunks' loads in flight), tests each object against
//                the child row, and each subject lane counts its own assertions
//                in a chunk as popcount(ballot & its lane range).  Skewed degrees
//                are balanced inside the wave by construction; rows stop
//                contributing once their count decides the predicate, and the
//                walk jumps past chunks that hold only decided rows.  Rows above
//                the heavy-row threshold are counted on many blocks instead
//                (k_role_heavy).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "kb_handle.h"
#include "plan.h"

namespace hth {

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ---------------------------------------------------------------------------
// numeric thresholds
// ---------------------------------------------------------------------------
// All thresholds requested on one property in one pass over its column: one
// lane per individual over 8 consecutive words (values loaded once, kept in
// registers), one wave ballot per threshold and word; lanes 0..7 then store
// the 8 words of a threshold's row together (a full 64-byte line).
__global__ void __launch_bounds__(256)
k_threshold(DevKB kb, const ThrGroup* __restrict__ groups, const ThrTask* __restrict__ tasks, uint32_t bpt) {
  const uint32_t gi = blockIdx.x / bpt, b = blockIdx.x % bpt;
  const ThrGroup G = groups[gi];
  const float* col = kb.data + (size_t)G.prop * kb.N;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t n_blk = (kb.W + 7) / 8;
  for (uint32_t blk = b * 4 + wv; blk < n_blk; blk += bpt * 4) {
    const uint32_t w0 = blk * 8;
    float f[8];
    bool in[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t x = (w0 + j) * 64 + lane;
      in[j] = w0 + j < kb.W && x < kb.N;
      f[j] = in[j] ? col[x] : 0.0f;
    }
    for (uint32_t i = 0; i < G.n; ++i) {
      const ThrTask T = tasks[G.first + i];
      uint64_t mine = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        // NaN (no value) compares false
        const bool pass = T.cmp == 0 ? f[j] >= T.t : T.cmp == 1 ? f[j] <= T.t : f[j] == T.t;
        const uint64_t m = __ballot(in[j] && pass);
        if (lane == j) mine = m;
      }
      if (lane < 8 && w0 + lane < kb.W) out_ptr(kb, T.out_row)[w0 + lane] = mine;
    }
  }
}

// ---------------------------------------------------------------------------
// multi-valued numeric concrete roles (Algorithms 9/10)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool num_pass(float v, uint32_t cmp, float t) {
  return cmp == 0 ? v >= t : cmp == 1 ? v <= t : v == t;
}

// Value roles (numeric and string concrete roles): one wave per 64 consecutive
// subjects, as in the role pass.  The wave walks the subjects' concatenated
// values in chunks of 64 (eight chunks' loads in flight), each subject lane
// takes its own values in a chunk from the ballot of passing values, and the
// walk stops once every subject with values left has found one.  Rows above
// the heavy-row threshold are left to value_heavy (their bits here are 0).
constexpr int kNumChunks = 8;
// off: the role's 32-bit offsets relative to vals, its first value.
template <typename V, class Pass>
__device__ __forceinline__ void value_walk(const DevKB& kb, const uint32_t* __restrict__ off,
                                           const V* __restrict__ vals, Pass pass, uint64_t* __restrict__ out,
                                           uint32_t b, uint32_t bpt) {
  const int lane = threadIdx.x & 63;
  for (uint32_t w = b * 4 + (threadIdx.x >> 6); w < kb.W; w += bpt * 4) {
    const uint32_t x = w * 64 + lane;
    const bool in = x < kb.N;
    const uint32_t olo = off[in ? x : kb.N];
    uint32_t ohi = in ? off[x + 1] : olo;
    const bool heavy = ohi - olo > kb.heavy_min;
    if (heavy) ohi = olo;
    const uint32_t ee = (uint32_t)__shfl((int)ohi, 63, 64);
    uint32_t i0 = (uint32_t)__shfl((int)olo, 0, 64);
    bool hit = false;
    while (i0 < ee) {
      V v[kNumChunks];
#pragma unroll
      for (int c = 0; c < kNumChunks; ++c) {
        const uint64_t e = (uint64_t)i0 + 64 * c + lane;
        v[c] = e < ee ? vals[e] : V(0);
      }
#pragma unroll
      for (int c = 0; c < kNumChunks; ++c) {
        const uint64_t base = (uint64_t)i0 + 64 * c;
        const uint64_t m = __ballot(base + lane < ee && pass(v[c]));
        const uint64_t a = olo > base ? min((uint64_t)olo - base, (uint64_t)64) : 0;
        const uint64_t bb = ohi > base ? min((uint64_t)ohi - base, (uint64_t)64) : 0;
        if (bb > a) {
          const uint64_t rm = (bb - a == 64) ? ~0ull : (((1ull << (bb - a)) - 1ull) << a);
          hit |= (m & rm) != 0;
        }
      }
      const uint64_t step = 64 * kNumChunks;
      const uint64_t pend = __ballot(in && !hit && ohi > i0 + step);
      if (!pend) break;
      const int l = __ffsll((unsigned long long)pend) - 1;
      const uint32_t nxt = (uint32_t)__shfl((int)olo, l, 64);
      i0 = (uint32_t)max((uint64_t)i0 + step, (uint64_t)nxt);
    }
    const uint64_t word = __ballot(in && !heavy && hit);
    if (lane == 0) out[w] = word;
  }
}

// One chunk of kHeavyChunk values of one heavy row per block: a passing value
// sets the row's bit (after the walk wrote the word; an existential result
// only ever gains bits, so blocks need no ordering among themselves).  Chunk
// blocks that find the bit already set skip the atomic.
template <typename V, class Pass>
__device__ __forceinline__ void value_heavy(const DevKB& kb, const uint32_t* __restrict__ off,
                                            const V* __restrict__ vals, Pass pass, uint64_t* __restrict__ out,
                                            uint32_t x, uint32_t k) {
  __shared__ uint32_t s_any[4];
  const uint32_t e0 = off[x] + k * kHeavyChunk;
  const uint32_t e1 = min(off[x + 1], e0 + kHeavyChunk);
  bool any = false;
#pragma unroll
  for (uint32_t j = 0; j < kHeavyChunk / 256; ++j) {
    const uint32_t e = e0 + j * 256 + threadIdx.x;
    if (e < e1) any |= pass(vals[e]);
  }
  const uint64_t m = __ballot(any);
  if ((threadIdx.x & 63) == 0) s_any[threadIdx.x >> 6] = m != 0;
  __syncthreads();
  if (threadIdx.x == 0 && (s_any[0] | s_any[1] | s_any[2] | s_any[3])) {
    unsigned long long* word = reinterpret_cast<unsigned long long*>(out) + (x >> 6);
    const unsigned long long bit = 1ull << (x & 63);
    if (!(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit)) atomicOr(word, bit);
  }
}

// the task of heavy block b: the last task whose first block is <= b
template <class Task>
__device__ __forceinline__ uint32_t value_task(const Task* __restrict__ tasks, uint32_t n, uint32_t b) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tasks[mid].h_first <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256)
k_numrole(DevKB kb, const NumTask* __restrict__ tasks, uint32_t bpt) {
  const NumTask T = tasks[blockIdx.x / bpt];
  const float* vals = kb.num_val + ((uint64_t)T.base_hi << 32 | T.base_lo);
  value_walk<float>(kb, kb.num_roff + (size_t)T.role * (kb.N + 1), vals,
                    [&](float v) { return num_pass(v, T.cmp, T.t); }, out_ptr(kb, T.out_row), blockIdx.x % bpt, bpt);
}

__global__ void __launch_bounds__(256)
k_numrole_heavy(DevKB kb, const NumTask* __restrict__ tasks, uint32_t n_tasks, uint32_t b0) {
  const uint32_t b = b0 + blockIdx.x;
  const NumTask T = tasks[value_task(tasks, n_tasks, b)];
  const HeavyChunk c = kb.num_heavy_chunks[T.hc0 + (b - T.h_first)];
  const float* vals = kb.num_val + ((uint64_t)T.base_hi << 32 | T.base_lo);
  value_heavy<float>(kb, kb.num_roff + (size_t)T.role * (kb.N + 1), vals,
                     [&](float v) { return num_pass(v, T.cmp, T.t); }, out_ptr(kb, T.out_row),
                     kb.num_heavy_rows[c.hrow], c.k);
}

// CONTAIN, first step: for every dictionary string, whether it holds the
// task's pattern (one lane per string, a plain scan of the string; the empty
// pattern is in every string).  A wave ballot writes one word of the task's
// id set per 64 strings.  The per-assertion test then reads one bit.
__global__ void __launch_bounds__(256)
k_contains(DevKB kb, const StrTask* __restrict__ tasks, uint32_t tiles) {
  const StrTask T = tasks[blockIdx.x / tiles];
  const uint32_t s = (blockIdx.x % tiles) * 256 + threadIdx.x;
  const int64_t p0 = kb.pat_off[T.q], pl = kb.pat_off[T.q + 1] - p0;
  const uint8_t* pat = kb.pat_chars + p0;
  bool hit = false;
  if (s < kb.n_strings) {
    const int64_t s0 = kb.dict_off[s], sl = kb.dict_off[s + 1] - s0;
    const uint8_t* str = kb.dict_chars + s0;
    for (int64_t i = 0; i + pl <= sl && !hit; ++i) {
      int64_t j = 0;
      while (j < pl && str[i + j] == pat[j]) ++j;
      hit = j == pl;
    }
  }
  const uint64_t m = __ballot(hit);
  const uint32_t w = s >> 6;
  if ((threadIdx.x & 63) == 0 && (uint64_t)w * 64 < kb.n_strings) kb.idsets[T.set_word + w] = m;
}

__global__ void __launch_bounds__(256)
k_strrole(DevKB kb, const StrTask* __restrict__ tasks, uint32_t bpt) {
  const StrTask T = tasks[blockIdx.x / bpt];
  const uint32_t* off = kb.str_roff + (size_t)T.role * (kb.N + 1);
  const int32_t* ids = kb.str_ids + ((uint64_t)T.base_hi << 32 | T.base_lo);
  uint64_t* out = out_ptr(kb, T.out_row);
  if (T.kind == 0) {
    value_walk<int32_t>(kb, off, ids, [&](int32_t id) { return (uint32_t)id == T.q; }, out,
                        blockIdx.x % bpt, bpt);
  } else {
    const uint64_t* set = kb.idsets + T.set_word;
    value_walk<int32_t>(kb, off, ids, [&](int32_t id) { return (set[(uint32_t)id >> 6] >> (id & 63)) & 1; },
                        out, blockIdx.x % bpt, bpt);
  }
}

__global__ void __launch_bounds__(256)
k_strrole_heavy(DevKB kb, const StrTask* __restrict__ tasks, uint32_t n_tasks, uint32_t b0) {
  const uint32_t b = b0 + blockIdx.x;
  const StrTask T = tasks[value_task(tasks, n_tasks, b)];
  const HeavyChunk c = kb.str_heavy_chunks[T.hc0 + (b - T.h_first)];
  const uint32_t* off = kb.str_roff + (size_t)T.role * (kb.N + 1);
  const int32_t* ids = kb.str_ids + ((uint64_t)T.base_hi << 32 | T.base_lo);
  const uint32_t x = kb.str_heavy_rows[c.hrow];
  uint64_t* out = out_ptr(kb, T.out_row);
  if (T.kind == 0) {
    value_heavy<int32_t>(kb, off, ids, [&](int32_t id) { return (uint32_t)id == T.q; }, out, x, c.k);
  } else {
    const uint64_t* set = kb.idsets + T.set_word;
    value_heavy<int32_t>(kb, off, ids, [&](int32_t id) { return (set[(uint32_t)id >> 6] >> (id & 63)) & 1; },
                         out, x, c.k);
  }
}

// ---------------------------------------------------------------------------
// boolean regions (+ coverage)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kRegionThreads)
k_region(DevKB kb, const RegionTask* __restrict__ tasks, const uint32_t* __restrict__ code,
         uint32_t n_tasks) {
  __shared__ uint64_t stk[kStackDepth][kRegionThreads];
  const uint32_t tile = blockIdx.x / n_tasks, task = blockIdx.x % n_tasks;
  const RegionTask T = tasks[task];
  if (T.out_row == kNone && T.cover == kNone) return;   // a root whose coverage a shared pass adds
  const uint32_t tid = threadIdx.x;
  const uint32_t w = tile * kRegionThreads + tid;
  const bool live = w < kb.W;
  uint64_t top = 0;
  int sp = 0;
  for (uint32_t pc = 0; pc < T.code_len; ++pc) {
    const uint32_t ins = code[T.code_off + pc];
    const uint32_t op = ins & 15u, arg = ins >> 5;
    const uint64_t negm = (ins & 16u) ? ~0ull : 0ull;
    switch (op) {
      case RP_LEAF:
      case RP_TOP:
      case RP_BOT: {
        uint64_t v;
        if (op == RP_LEAF) v = live ? (row_ptr(kb, arg)[w] ^ negm) : 0ull;
        else v = op == RP_TOP ? ~0ull : 0ull;
        if (pc) stk[sp++][tid] = top;
        top = v;
        break;
      }
      case RP_NOT: top = ~top; break;
      case RP_AND: top &= stk[--sp][tid]; break;
      default: top |= stk[--sp][tid]; break;
    }
  }
  if (!live) top = 0;
  else if (w == kb.W - 1) top &= kb.tail;
  if (T.out_row != kNone && w < kb.S) {
    // kInstances: the caller's rows, one per covered hypothesis
    uint64_t* o = T.out_row == kInstances ? kb.instances + (size_t)T.cover * kb.S : out_ptr(kb, T.out_row);
    o[w] = top;
  }
  if (T.cover != kNone) {
    uint32_t p = live ? (uint32_t)__popcll(top & kb.pos[w]) : 0u;
    uint32_t q = live ? (uint32_t)__popcll(top & kb.neg[w]) : 0u;
    p = wave_sum(p);
    q = wave_sum(q);
    if ((tid & 63) == 0 && (p | q)) {
      if (p) atomicAdd(kb.counts + 2 * T.cover, p);
      if (q) atomicAdd(kb.counts + 2 * T.cover + 1, q);
    }
  }
}

// The same regions with the value stack in registers (a shift register of
// depth D, enough for most programs) and R words per lane, so that no LDS
// limits occupancy.  A block takes one task and a run of `tpb` consecutive
// tiles (256 R words each) and walks them in order: while it evaluates one
// tile, the words of the program's first kRegLeaves leaves and the example
// words of the next tile are already in flight.  The program runs leaf by
// leaf from registers; leaves beyond the first kRegLeaves are loaded where
// they occur.  An operand directly followed by AND or OR is combined with
// the top at once, so flat conjunctions and disjunctions never move the stack.  Lane t handles words tile*256R + R*t + r (consecutive: 16-byte loads).
// Coverage is summed over the block's tiles and added with one atomic pair.
// A root whose coverage a shared pass adds has an empty task: its blocks
// leave at once.
constexpr int kRegDepth = 6;     // D: most stack entries a program may need
constexpr int kRegLeaves = 2;    // leaves whose words are loaded ahead
template <int D, int R>
__global__ void __launch_bounds__(256)
k_region_reg(DevKB kb, const RegionTask* __restrict__ tasks, const uint32_t* __restrict__ code,
             uint32_t n_tasks, uint32_t tiles, uint32_t tpb) {
  __shared__ uint32_t s_pq[2][4];
  const uint32_t run = blockIdx.x / n_tasks, task = blockIdx.x % n_tasks;
  const RegionTask T = tasks[task];
  if (T.out_row == kNone && T.cover == kNone) return;
  const uint32_t tid = threadIdx.x;
  const uint32_t* prog = code + T.code_off;
  const uint32_t len = T.code_len;
  // the first kRegLeaves leaves' rows (a program with fewer reads the example
  // row in their place and never uses it)
  const uint64_t* lrow[kRegLeaves];
  {
    uint32_t pc = 0;
#pragma unroll
    for (int j = 0; j < kRegLeaves; ++j) {
      while (pc < len && (prog[pc] & 15u) != RP_LEAF) ++pc;
      lrow[j] = pc < len ? row_ptr(kb, prog[pc] >> 5) : kb.pos;
      if (pc < len) ++pc;
    }
  }
  const bool cover = T.cover != kNone;
  uint64_t* out = T.out_row == kNone ? nullptr
                  : T.out_row == kInstances ? kb.instances + (size_t)T.cover * kb.S
                                            : out_ptr(kb, T.out_row);
  // loads of one tile: a lane's R consecutive words, at an index clamped into
  // the row (rows hold S words, S a multiple of 8; words past W are masked
  // later), R-word vector loads with no branch around them
  auto load_words = [&](const uint64_t* row, uint32_t wc, uint64_t (&v)[R]) {
    if constexpr (R == 1) {
      v[0] = row[wc];
    } else {
#pragma unroll
      for (int r = 0; r < R; r += 2) {
        const ulonglong2 q = *reinterpret_cast<const ulonglong2*>(row + wc + r);
        v[r] = q.x;
        v[r + 1] = q.y;
      }
    }
  };
  auto fetch = [&](uint32_t tile, uint64_t (&lv)[kRegLeaves][R], uint64_t (&ep)[R], uint64_t (&en)[R]) {
    const uint32_t wc = min(tile * (256 * R) + tid * R, kb.S - R);
#pragma unroll
    for (int j = 0; j < kRegLeaves; ++j) load_words(lrow[j], wc, lv[j]);
    load_words(kb.pos, wc, ep);
    load_words(kb.neg, wc, en);
  };
  const uint32_t t_end = min((run + 1) * tpb, tiles);
  uint64_t lv[kRegLeaves][R], ep[R], en[R];
  fetch(run * tpb, lv, ep, en);
  uint32_t p = 0, q = 0;
  for (uint32_t tile = run * tpb; tile < t_end; ++tile) {
    uint64_t nlv[kRegLeaves][R], nep[R], nen[R];
    if (tile + 1 < t_end) fetch(tile + 1, nlv, nep, nen);
    const uint32_t w0 = tile * (256 * R) + tid * R;
    uint64_t top[R], st[D > 1 ? D - 1 : 1][R];
#pragma unroll
    for (int r = 0; r < R; ++r) top[r] = 0;
    uint32_t pc = 0;
    // segment j runs the program up to and including its j-th leaf; the last
    // segment runs the rest, loading its leaves itself
#pragma unroll
    for (int j = 0; j <= kRegLeaves; ++j) {
      while (pc < len) {
        const uint32_t ins = prog[pc++];
        const uint32_t op = ins & 15u, arg = ins >> 5;
        if (op <= RP_BOT) {
          uint64_t val[R];                        // the operand's words
          const bool ahead = op == RP_LEAF && j < kRegLeaves;
          if (op == RP_LEAF) {
            const uint64_t negm = (ins & 16u) ? ~0ull : 0ull;
            if (ahead) {
#pragma unroll
              for (int r = 0; r < R; ++r) val[r] = lv[j < kRegLeaves ? j : 0][r] ^ negm;
            } else {
              const uint64_t* row = row_ptr(kb, arg);
#pragma unroll
              for (int r = 0; r < R; ++r) {
                const uint32_t w = w0 + r;
                val[r] = w < kb.W ? (row[w] ^ negm) : 0ull;
              }
            }
          } else {
#pragma unroll
            for (int r = 0; r < R; ++r) val[r] = op == RP_TOP ? ~0ull : 0ull;
          }
          // an operand followed by AND / OR folds into the top: no push, no pop
          // (every operand of a flattened conjunction or disjunction but the first)
          const uint32_t nop = pc < len ? (prog[pc] & 15u) : (uint32_t)RP_LEAF;
          if (pc > 1 && (nop == RP_AND || nop == RP_OR)) {
#pragma unroll
            for (int r = 0; r < R; ++r) top[r] = nop == RP_AND ? (top[r] & val[r]) : (top[r] | val[r]);
            ++pc;
          } else {
            if (pc > 1) {                         // push: shift the stack down
#pragma unroll
              for (int i = D - 2; i > 0; --i)
#pragma unroll
                for (int r = 0; r < R; ++r) st[i][r] = st[i - 1][r];
#pragma unroll
              for (int r = 0; r < R; ++r) st[0][r] = top[r];
            }
#pragma unroll
            for (int r = 0; r < R; ++r) top[r] = val[r];
          }
          if (ahead) break;
        } else if (op == RP_NOT) {
#pragma unroll
          for (int r = 0; r < R; ++r) top[r] = ~top[r];
        } else {                                  // pop b, top = top op b
          const bool conj = op == RP_AND;
#pragma unroll
          for (int r = 0; r < R; ++r) top[r] = conj ? (top[r] & st[0][r]) : (top[r] | st[0][r]);
#pragma unroll
          for (int i = 0; i + 1 < D - 1; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r) st[i][r] = st[i + 1][r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t w = w0 + r;
      uint64_t v = top[r];
      if (w >= kb.W) v = 0;
      else if (w == kb.W - 1) v &= kb.tail;
      if (out && w < kb.S) out[w] = v;
      if (cover) {
        p += (uint32_t)__popcll(v & ep[r]);
        q += (uint32_t)__popcll(v & en[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ep[r] = nep[r];
      en[r] = nen[r];
#pragma unroll
      for (int j = 0; j < kRegLeaves; ++j) lv[j][r] = nlv[j][r];
    }
  }
  if (cover) {
    p = wave_sum(p);
    q = wave_sum(q);
    if ((tid & 63) == 0) {
      s_pq[0][tid >> 6] = p;
      s_pq[1][tid >> 6] = q;
    }
    __syncthreads();
    if (tid == 0) {
      const uint32_t P = s_pq[0][0] + s_pq[0][1] + s_pq[0][2] + s_pq[0][3];
      const uint32_t Q = s_pq[1][0] + s_pq[1][1] + s_pq[1][2] + s_pq[1][3];
      if (P) atomicAdd(kb.counts + 2 * T.cover, P);
      if (Q) atomicAdd(kb.counts + 2 * T.cover + 1, Q);
    }
  }
}

// ---------------------------------------------------------------------------
// single role restriction, one wave per 64 subjects
// ---------------------------------------------------------------------------
constexpr int kRoleChunks = 8;   // 64-assertion chunks whose loads a wave issues together
template <bool STAGE>
__device__ __forceinline__ void role_word(const DevKB& kb, const uint32_t* __restrict__ off,
                                          const int32_t* __restrict__ tg,
                                          const uint64_t* __restrict__ child, uint32_t neg,
                                          uint32_t lo, uint32_t hi, uint32_t sat,
                                          uint64_t* __restrict__ out, uint32_t w, int lane) {
  const uint32_t x = w * 64 + lane;
  const bool in = x < kb.N;
  const uint32_t xe = in ? x : kb.N;
  const uint32_t olo = off[xe];
  uint32_t ohi = in ? off[x + 1] : olo;
  const bool heavy = ohi - olo > kb.heavy_min;   // counted by k_role_heavy instead
  if (heavy) ohi = olo;
  const uint32_t ee = (uint32_t)__shfl((int)ohi, 63, 64);
  uint32_t i0 = (uint32_t)__shfl((int)olo, 0, 64);
  uint32_t cnt = 0;
  while (i0 < ee) {
    // kRoleChunks consecutive chunks of 64 assertions: all target loads first
    int32_t t[kRoleChunks];
#pragma unroll
    for (int c = 0; c < kRoleChunks; ++c) {
      const uint32_t e = i0 + 64 * c + lane;
      t[c] = e < ee ? tg[e] : -1;
    }
#pragma unroll
    for (int c = 0; c < kRoleChunks; ++c) {
      const uint32_t base = i0 + 64 * c;
      bool v = false;
      if (t[c] >= 0) {
        const uint32_t y = (uint32_t)t[c];
        v = ((uint32_t)(child[y >> 6] >> (y & 63)) & 1u) ^ neg;
      }
      const uint64_t m = __ballot(v);
      const uint32_t a = olo > base ? min(olo - base, 64u) : 0u;
      const uint32_t b = ohi > base ? min(ohi - base, 64u) : 0u;
      if (b > a) {
        const uint64_t rm = (b - a == 64) ? ~0ull : (((1ull << (b - a)) - 1ull) << a);
        cnt += (uint32_t)__popcll(m & rm);
      }
    }
    const uint32_t step = 64 * kRoleChunks;
    const uint64_t pend = __ballot(in && cnt < sat && ohi > i0 + step);
    if (!pend) break;
    const int l = __ffsll((unsigned long long)pend) - 1;
    const uint32_t nxt = (uint32_t)__shfl((int)olo, l, 64);
    i0 = max(i0 + step, nxt);
  }
  const bool res = in && !heavy && cnt >= lo && cnt <= hi;
  const uint64_t word = __ballot(res);
  if (lane == 0) out[w] = word;
}

template <bool STAGE>
__global__ void __launch_bounds__(STAGE ? 1024 : 256)
k_role(DevKB kb, const RoleTask* __restrict__ tasks, uint32_t bpt) {
  extern __shared__ uint64_t lds_child[];
  const uint32_t task = blockIdx.x / bpt, b = blockIdx.x % bpt;
  const RoleTask T = tasks[task];
  const uint64_t* child = row_ptr(kb, T.child_row);
  if (STAGE) {
    for (uint32_t i = threadIdx.x; i < kb.W; i += blockDim.x) lds_child[i] = child[i];
    __syncthreads();
    child = lds_child;
  }
  const size_t ro = (size_t)T.role * (kb.N + 1);
  const uint32_t* off = (T.inv ? kb.inv_off : kb.fwd_off) + ro;
  const int32_t* tg = (T.inv ? kb.inv_tg : kb.fwd_tg) + kb.role_base[T.role];
  uint64_t* out = out_ptr(kb, T.out_row);
  const uint32_t* words = kb.words + (size_t)(2 * T.role + T.inv) * kb.W;
  const uint32_t nw = blockDim.x >> 6;
  const int lane = threadIdx.x & 63;
  for (uint32_t i = b * nw + (threadIdx.x >> 6); i < T.n_words; i += bpt * nw)
    role_word<STAGE>(kb, off, tg, child, T.neg, T.lo, T.hi, T.sat, out, words[i], lane);
}

// The task of heavy-row block b or counter i: the last task whose first block
// (counter) is <= b; tasks without heavy rows own empty ranges.
template <bool BLOCKS>
__device__ __forceinline__ uint32_t heavy_task(const RoleTask* __restrict__ tasks, uint32_t n, uint32_t b) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((BLOCKS ? tasks[mid].h_first : tasks[mid].c_first) <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One chunk of kHeavyChunk assertions of one heavy row per block: the count
// of child members among them goes to partial[block] (no early exit: every
// chunk is counted, so that no two blocks touch the same word).
__global__ void __launch_bounds__(256)
k_role_heavy(DevKB kb, const RoleTask* __restrict__ tasks, uint32_t n_tasks, uint32_t b0,
             uint32_t* __restrict__ partial) {
  __shared__ uint32_t s_part[4];
  const uint32_t b = b0 + blockIdx.x;
  const RoleTask T = tasks[heavy_task<true>(tasks, n_tasks, b)];
  const HeavyChunk c = kb.heavy_chunks[T.hc0 + (b - T.h_first)];
  const uint32_t x = kb.heavy_rows[c.hrow];
  const uint32_t* off = (T.inv ? kb.inv_off : kb.fwd_off) + (size_t)T.role * (kb.N + 1);
  const int32_t* tg = (T.inv ? kb.inv_tg : kb.fwd_tg) + kb.role_base[T.role];
  const uint64_t* child = row_ptr(kb, T.child_row);
  const uint32_t e0 = off[x] + c.k * kHeavyChunk;
  const uint32_t e1 = min(off[x + 1], e0 + kHeavyChunk);
  uint32_t cnt = 0;
#pragma unroll
  for (uint32_t j = 0; j < kHeavyChunk / 256; ++j) {
    const uint32_t e = e0 + j * 256 + threadIdx.x;
    if (e < e1) {
      const uint32_t t = (uint32_t)tg[e];
      cnt += ((uint32_t)(child[t >> 6] >> (t & 63)) & 1u) ^ T.neg;
    }
  }
  cnt = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) partial[b] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
}

// One block per (task, heavy row): the sum of the row's chunk partials gives
// the row's bit.  Runs after k_role has written the rows' words (with the
// heavy bits clear).
__global__ void __launch_bounds__(256)
k_role_heavy_fix(DevKB kb, const RoleTask* __restrict__ tasks, uint32_t n_tasks, uint32_t i0,
                 const uint32_t* __restrict__ partial) {
  __shared__ uint32_t s_part[4];
  const uint32_t i = i0 + blockIdx.x;
  const RoleTask T = tasks[heavy_task<false>(tasks, n_tasks, i)];
  const uint32_t hrow = T.hr0 + (i - T.c_first);
  const uint32_t c0 = kb.heavy_chunk0[hrow], n = kb.heavy_chunk0[hrow + 1] - c0;
  const uint32_t* p = partial + T.h_first + (c0 - T.hc0);
  uint32_t cnt = 0;
#pragma unroll 8
  for (uint32_t c = threadIdx.x; c < n; c += 256) cnt += p[c];
  cnt = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    cnt = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    const uint32_t x = kb.heavy_rows[hrow];
    const unsigned long long bit = 1ull << (x & 63);
    unsigned long long* word = reinterpret_cast<unsigned long long*>(out_ptr(kb, T.out_row) + (x >> 6));
    if (cnt >= T.lo && cnt <= T.hi) atomicOr(word, bit);
    else atomicAnd(word, ~bit);
  }
}

// A single ∃ρ.A (lo = 1, hi unbounded) or ¬∃ρ.A (lo = hi = 0) whose atomic
// child A is sparse, pushed from A's members: every y in A takes the subjects
// x that reach it (its row in the opposite direction) and sets (∃) or clears
// (¬∃) their bits in the output row, which a fill task has set to all zeros
// or all ones before.  One wave per word of A, a lane per member walking its
// row alone, so it is only chosen where every row of the opposite direction
// is short (kPushMaxDeg).
__global__ void __launch_bounds__(256)
k_push(DevKB kb, const RoleTask* __restrict__ tasks, uint32_t tiles) {
  const uint32_t t = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const uint32_t w = tile * 4 + (threadIdx.x >> 6);
  if (w >= kb.W) return;
  const RoleTask T = tasks[t];
  const int lane = threadIdx.x & 63;
  const uint64_t cw = row_ptr(kb, T.child_row)[w];
  if (!((cw >> lane) & 1ull)) return;
  const uint32_t y = w * 64 + lane;
  const uint32_t* off = (T.inv ? kb.fwd_off : kb.inv_off) + (size_t)T.role * (kb.N + 1);
  const int32_t* tg = (T.inv ? kb.fwd_tg : kb.inv_tg) + kb.role_base[T.role];
  unsigned long long* out = reinterpret_cast<unsigned long long*>(out_ptr(kb, T.out_row));
  const uint32_t e1 = off[y + 1];
  const bool mark = T.lo == 1;
#pragma unroll 4
  for (uint32_t e = off[y]; e < e1; ++e) {
    const uint32_t x = (uint32_t)tg[e];
    const unsigned long long bit = 1ull << (x & 63);
    if (mark) atomicOr(out + (x >> 6), bit);
    else atomicAnd(out + (x >> 6), ~bit);
  }
}

// Zero-count results for the words of a role direction without assertions:
// the whole row, four words (two 16-byte stores) per thread.  Rows are
// stride_words apart, a multiple of 8, so a thread's words never cross a row.
constexpr uint32_t kFillWords = 4;
inline uint32_t fill_tiles(uint32_t S) { return (S + 256 * kFillWords - 1) / (256 * kFillWords); }
__global__ void __launch_bounds__(256)
k_fill_rows(DevKB kb, const FillTask* __restrict__ tasks, uint32_t tiles) {
  const uint32_t t = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const FillTask F = tasks[t];
  const uint32_t w0 = (tile * 256 + threadIdx.x) * kFillWords;
  if (w0 >= kb.S) return;
  uint64_t v[kFillWords];
#pragma unroll
  for (uint32_t i = 0; i < kFillWords; ++i) {
    const uint32_t w = w0 + i;
    v[i] = F.ones && w < kb.W ? (w == kb.W - 1 ? kb.tail : ~0ull) : 0ull;
  }
  ulonglong2* q = reinterpret_cast<ulonglong2*>(out_ptr(kb, F.out_row) + w0);
  q[0] = make_ulonglong2(v[0], v[1]);
  q[1] = make_ulonglong2(v[2], v[3]);
}

}  // namespace hth

#include "group_kernels.h"

namespace hth {

// ---------------------------------------------------------------------------
// executor
// ---------------------------------------------------------------------------
// The T rows of the groups of one launch stay within kb.tune.t_budget bytes so
// that the random T fetches of a launch stay in the last-level caches.
inline uint32_t t_width_bytes(uint32_t k) { return k <= 8 ? 1 : k <= 16 ? 2 : k <= 32 ? 4 : 8; }
inline size_t t_area_bytes(const hth_kb_s& kb) {
  return std::max<size_t>(kb.tune.t_budget, align_up(kb.N, 64) * 8);
}
// T rows of a group: the objects of its direction (compact) or all individuals
inline uint64_t t_rows(const hth_kb_s& kb, const GroupTask& g) {
  return align_up(g.compact ? kb.n_obj[2 * g.role + g.inv] : kb.N, 64);
}

// Consecutive groups of a level share a launch while their T rows, at the
// widest T width among them, fit the budget; sets each group's T offset.
struct GroupChunk {
  size_t first;
  uint32_t n, wb;
  uint32_t rounds;     // XCD-local: rounds of the slot table (0 = chip-wide launch)
  size_t slot_off;     // its first entry in the plan's slot table
};
// XCD-local placement of a chunk's groups: longest first onto the least loaded
// XCD (cost ~ assertions + 64 per visited word); slot (round, xcd) -> group.
void place_on_xcds(const hth_kb_s& kb, const std::vector<GroupTask>& gs, GroupChunk& c,
                   std::vector<uint32_t>& xslots) {
  std::vector<std::pair<double, uint32_t>> cost;
  for (uint32_t i = 0; i < c.n; ++i) {
    const GroupTask& g = gs[c.first + i];
    const double e = (double)(kb.role_base[g.role + 1] - kb.role_base[g.role]);
    cost.push_back({e + 64.0 * kb.n_words[2 * g.role + g.inv], i});
  }
  std::stable_sort(cost.begin(), cost.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<uint32_t> per[8];
  for (const auto& [w, i] : cost) {
    const int x = (int)(std::min_element(load, load + 8) - load);
    load[x] += w;
    per[x].push_back(i);
  }
  size_t rounds = 0;
  for (int x = 0; x < 8; ++x) rounds = std::max(rounds, per[x].size());
  c.rounds = (uint32_t)rounds;
  c.slot_off = xslots.size();
  xslots.resize(xslots.size() + rounds * 8, kNone);
  for (int x = 0; x < 8; ++x)
    for (size_t r = 0; r < per[x].size(); ++r) xslots[c.slot_off + r * 8 + x] = per[x][r];
}

// groups per launch stay few enough for the pass's grid (at most 8 x 256
// blocks per XCD round) to stay far below 2^31 work-items
constexpr size_t kMaxGroupsPerLaunch = 2048;

// Role direction rd = 2 role + inv holds only short rows: its shared passes
// walk one subject per lane (k_group_short)
inline bool short_rows(const hth_kb_s& kb, uint32_t rd) {
  return kb.tune.short_rows && kb.max_deg[rd & 1][rd >> 1] <= kb.tune.short_rows;
}

std::vector<GroupChunk> chunk_groups(const hth_kb_s& kb, std::vector<GroupTask>& gs) {
  std::vector<GroupChunk> out;
  size_t i = 0;
  while (i < gs.size()) {
    uint32_t wb = t_width_bytes(gs[i].k);
    uint64_t rows = t_rows(kb, gs[i]);
    size_t j = i + 1;
    while (j < gs.size() && j - i < kMaxGroupsPerLaunch && gs[j].short_rows == gs[i].short_rows) {
      const uint32_t nwb = std::max(wb, t_width_bytes(gs[j].k));
      if ((rows + t_rows(kb, gs[j])) * nwb > kb.tune.t_budget) break;
      rows += t_rows(kb, gs[j]);
      wb = nwb;
      ++j;
    }
    uint64_t off = 0;
    for (size_t q = i; q < j; ++q) {
      gs[q].t_off = off;
      off += t_rows(kb, gs[q]);
    }
    out.push_back({i, (uint32_t)(j - i), wb, 0, 0});
    i = j;
  }
  return out;
}

// T bytes the chunks of one level use at most: a chunk's rows run from its
// first group's t_off (0) to the end of its last group's, at the chunk's width.
inline size_t chunks_t_bytes(const hth_kb_s& kb, const std::vector<GroupTask>& gs,
                             const std::vector<GroupChunk>& cs) {
  size_t most = 0;
  for (const GroupChunk& c : cs) {
    const GroupTask& last = gs[c.first + c.n - 1];
    most = std::max<size_t>(most, (size_t)(last.t_off + t_rows(kb, last)) * c.wb);
  }
  return align_up(most, 256);
}

// Target segments of a chunk: its passes cover T rows in ranges of at most
// t_segment bytes (at the chunk's T width), when that takes 2..kMaxSegments
// passes; otherwise one pass over all rows.  seg_rows: T rows per pass.
constexpr uint32_t kMaxSegments = 4;
uint32_t chunk_segments(const hth_kb_s& kb, const std::vector<GroupTask>& gs, const GroupChunk& c,
                        uint64_t* seg_rows) {
  uint64_t rows = 0;
  for (uint32_t i = 0; i < c.n; ++i) rows = std::max(rows, t_rows(kb, gs[c.first + i]));
  *seg_rows = rows;
  const uint64_t seg = (uint64_t)kb.tune.t_segment_kb << 10;
  if (!seg || rows * c.wb <= seg) return 1;
  const uint64_t P = (rows * c.wb + seg - 1) / seg;
  if (P > kMaxSegments) return 1;
  *seg_rows = align_up((rows + P - 1) / P, 64);
  return (uint32_t)P;
}
// partial counts carried between the passes of a segmented chunk
inline size_t chunk_partial_bytes(const hth_kb_s& kb, const std::vector<GroupTask>& gs, const GroupChunk& c) {
  uint64_t sr;
  return chunk_segments(kb, gs, c, &sr) > 1 ? (size_t)c.n * kb.W * 256 * c.wb : 0;
}

namespace {

struct Blob {
  std::vector<char> bytes;
  template <class T>
  size_t add(const std::vector<T>& v) {
    size_t at = align_up(bytes.size(), 256);
    bytes.resize(at + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(bytes.data() + at, v.data(), v.size() * sizeof(T));
    return at;
  }
};

size_t table_bound(uint32_t max_nodes, uint32_t max_hyps) {
  const size_t n = max_nodes + 2;
  size_t b = 0;
  b += align_up(n * sizeof(ThrTask), 256);
  b += align_up(n * sizeof(ThrGroup), 256);
  b += align_up(n * sizeof(NumTask), 256);
  b += align_up(n * sizeof(StrTask), 256);
  b += align_up((n + max_hyps) * sizeof(RegionTask), 256);
  b += align_up(n * sizeof(RoleTask), 256);
  b += align_up(n * sizeof(RoleTask), 256);                // pushed role tasks
  b += align_up(n * sizeof(GroupTask), 256);
  b += align_up(n * sizeof(GroupMember), 256);
  b += align_up(n * sizeof(FillTask), 256);
  b += align_up((4 * n + 16) * sizeof(uint32_t), 256);
  b += align_up((9 * n + 8) * sizeof(uint32_t), 256);     // XCD slot tables
  return b + 4096;
}

DevKB dev_view(const hth_kb_s& kb) {
  DevKB d{};
  d.concepts = kb.d.concept_bits;
  d.data = kb.d.data;
  d.fwd_off = kb.fwd_off;
  d.inv_off = kb.inv_off;
  d.fwd_tg = kb.d.role_targets;
  d.inv_tg = kb.inv_tg;
  d.role_base = kb.role_base_dev;
  d.words = kb.words;
  d.objmask = kb.objmask;
  d.objbase = kb.objbase;
  d.ctg_fwd = kb.ctg_fwd;
  d.ctg_inv = kb.ctg_inv;
  d.heavy_rows = kb.heavy_rows;
  d.heavy_chunks = kb.heavy_chunks;
  d.heavy_chunk0 = kb.heavy_chunk0;
  d.heavy_min = kb.heavy_min;
  d.pos = kb.pos;
  d.neg = kb.neg;
  d.n_concepts = kb.d.n_concepts;
  d.n_fixed = kb.d.n_concepts;
  d.N = kb.N;
  d.W = kb.W;
  d.S = kb.S;
  d.tail = kb.tail;
  return d;
}

// Kernel launches, each optionally bracketed by timing events.
struct Launcher {
  hth_kb_s& kb;
  hipStream_t st;
  // the (role, direction) CSRs already counted in this sweep (one role-nesting
  // level): the byte model reads each once per sweep however many passes use it
  std::vector<uint32_t> csr_seen;

  double csr_once(uint32_t role, uint32_t inv);

  hth_status event(hipEvent_t* e) {
    if (!kb.event_pool.empty()) {
      *e = kb.event_pool.back();
      kb.event_pool.pop_back();
      return HTH_OK;
    }
    HTH_HIP(hipEventCreate(e));
    return HTH_OK;
  }
  template <class F>
  hth_status run(int kind, double bytes, F&& launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (kb.prof) {
      hth_status s = event(&a);
      if (!s) s = event(&b);
      if (s) return s;
      HTH_HIP(hipEventRecord(a, st));
    }
    launch();
    HTH_HIP(hipGetLastError());
    if (kb.prof) {
      HTH_HIP(hipEventRecord(b, st));
      kb.prof_recs.push_back({kind, bytes, a, b});
    }
    return HTH_OK;
  }
};

// Launches of `items` work items, `per` blocks of `threads` lanes each, split
// so that no dispatch holds 2^31 work-items or more (a dispatch counts its
// grid in work-items in 32 bits; a larger grid would wrap, not fail).
// launch(first_item, item_count, blocks) issues one of them.
template <class F>
hth_status split_launch(Launcher& L, int kind, double bytes, uint64_t items, uint64_t per, uint32_t threads,
                        F&& launch) {
  const uint64_t max_blocks = (1ull << 31) / threads - 1;
  const uint64_t chunk = std::max<uint64_t>(1, max_blocks / std::max<uint64_t>(per, 1));
  for (uint64_t i0 = 0; i0 < items; i0 += chunk) {
    const uint64_t m = std::min(chunk, items - i0);
    hth_status s = L.run(kind, i0 ? 0.0 : bytes, [&] { launch((uint32_t)i0, (uint32_t)m, (uint32_t)(per * m)); });
    if (s) return s;
  }
  return HTH_OK;
}

// algorithmic bytes of the region tasks of one sweep (byte model): every
// distinct row they read once, each output row once, the two example rows
// once and 8 bytes of counts per hypothesis whose coverage they take
double region_bytes(const hth_kb_s& kb, const std::vector<RegionTask>& tasks, const std::vector<uint32_t>& code) {
  const double w8 = (double)kb.W * 8;
  std::vector<uint32_t> leaves;
  double b = 0;
  bool cover = false;
  for (const RegionTask& t : tasks) {
    for (uint32_t i = 0; i < t.code_len; ++i) {
      const uint32_t ins = code[t.code_off + i];
      if ((ins & 15u) == RP_LEAF) leaves.push_back(ins >> 5);
    }
    if (t.out_row != kNone) b += w8;
    if (t.cover != kNone) {
      b += 8;
      cover = true;
    }
  }
  std::sort(leaves.begin(), leaves.end());
  leaves.erase(std::unique(leaves.begin(), leaves.end()), leaves.end());
  return b + leaves.size() * w8 + (cover ? 2 * w8 : 0.0);
}

// a CSR direction scanned once: 32-bit row offsets and the role's targets
double csr_bytes(const hth_kb_s& kb, uint32_t role, uint32_t inv) {
  const double words = kb.n_words.empty() ? kb.W : kb.n_words[2 * role + inv];
  return 4.0 * std::min<double>((double)kb.N + 1, 65.0 * words) +
         4.0 * (double)(kb.role_base[role + 1] - kb.role_base[role]);
}

double Launcher::csr_once(uint32_t role, uint32_t inv) {
  const uint32_t key = 2 * role + inv;
  if (std::find(csr_seen.begin(), csr_seen.end(), key) != csr_seen.end()) return 0.0;
  csr_seen.push_back(key);
  return csr_bytes(kb, role, inv);
}

// tiles one block of the register region kernel walks (with the next tile's
// loads in flight while it evaluates one)
constexpr uint32_t kRegionTilesPerBlock = 16;
constexpr uint64_t kRegionMinBlocks = 16384;

// n region tasks whose programs need at most `depth` stack entries
hth_status launch_regions_n(Launcher& L, const DevKB& d, const RegionTask* tasks, const uint32_t* code,
                            uint32_t n, int depth, double bytes) {
  if (!n) return HTH_OK;
  // the register kernel when every program's stack fits its shift register
  if (depth <= kRegDepth && L.kb.tune.region_reg) {
    const uint32_t rw = L.kb.tune.region_reg;     // words per lane: 1, 2 or 4
    const uint32_t tiles = (d.S + 256 * rw - 1) / (256 * rw);
    // a block walks up to kRegionTilesPerBlock tiles of its task, fewer when
    // the launch would otherwise have under kRegionMinBlocks blocks
    const uint64_t per = std::max<uint64_t>(1, (uint64_t)n * tiles / kRegionMinBlocks);
    const uint32_t tpb = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(tiles, kRegionTilesPerBlock), per);
    const uint32_t runs = (tiles + tpb - 1) / tpb;
    return split_launch(L, HTH_K_REGION, bytes, n, runs, 256, [&](uint32_t t0, uint32_t m, uint32_t blocks) {
      const dim3 grid(blocks), block(256);
      if (rw == 1)
        hipLaunchKernelGGL((k_region_reg<kRegDepth, 1>), grid, block, 0, L.st, d, tasks + t0, code, m, tiles, tpb);
      else if (rw == 2)
        hipLaunchKernelGGL((k_region_reg<kRegDepth, 2>), grid, block, 0, L.st, d, tasks + t0, code, m, tiles, tpb);
      else
        hipLaunchKernelGGL((k_region_reg<kRegDepth, 4>), grid, block, 0, L.st, d, tasks + t0, code, m, tiles, tpb);
    });
  }
  const uint32_t tiles = (d.S + kRegionThreads - 1) / kRegionThreads;
  return split_launch(L, HTH_K_REGION, bytes, n, tiles, kRegionThreads, [&](uint32_t t0, uint32_t m, uint32_t blocks) {
    hipLaunchKernelGGL(k_region, dim3(blocks), dim3(kRegionThreads), 0, L.st, d, tasks + t0, code, m);
  });
}

hth_status launch_regions(Launcher& L, const DevKB& d, const RegionTask* tasks, const uint32_t* code,
                          const std::vector<RegionTask>& host, const std::vector<uint32_t>& hcode) {
  const double bytes = L.kb.prof ? region_bytes(L.kb, host, hcode) : 0.0;
  int depth = 0;
  for (const RegionTask& t : host) {
    int sp = 0;
    for (uint32_t i = 0; i < t.code_len; ++i) {
      const uint32_t op = hcode[t.code_off + i] & 15u;
      if (op <= RP_BOT) sp += i ? 1 : 0;
      else if (op != RP_NOT) --sp;
      depth = std::max(depth, sp + 1);
    }
  }
  return launch_regions_n(L, d, tasks, code, (uint32_t)host.size(), depth, bytes);
}

hth_status launch_roles_n(Launcher& L, const DevKB& d, const RoleTask* tasks, uint32_t n, double bytes) {
  const hth_kb_s& kb = L.kb;
  if (!n) return HTH_OK;
  const size_t lds = (size_t)kb.W * 8;
  if (lds <= kb.lds_per_block) {
    // one 1024-lane block per CU holds the child row in LDS: one round of blocks,
    // so that each CU stages the row once
    uint32_t bpt = std::max<uint32_t>(1, (kb.n_cu + n - 1) / n);
    bpt = std::min<uint32_t>(bpt, (kb.W + 15) / 16);
    return split_launch(L, HTH_K_ROLE, bytes, n, bpt, 1024, [&](uint32_t t0, uint32_t, uint32_t blocks) {
      hipLaunchKernelGGL(k_role<true>, dim3(blocks), dim3(1024), lds, L.st, d, tasks + t0, bpt);
    });
  }
  uint32_t bpt = std::max<uint32_t>(1, (8 * kb.n_cu + n - 1) / n);
  bpt = std::min<uint32_t>(bpt, (kb.W + 3) / 4);
  return split_launch(L, HTH_K_ROLE, bytes, n, bpt, 256, [&](uint32_t t0, uint32_t, uint32_t blocks) {
    hipLaunchKernelGGL(k_role<false>, dim3(blocks), dim3(256), 0, L.st, d, tasks + t0, bpt);
  });
}

hth_status launch_roles(Launcher& L, const DevKB& d, const RoleTask* tasks,
                        const std::vector<RoleTask>& host) {
  // per node: its CSR once per sweep, its child row in, its listed words out
  double bytes = 0;
  for (const RoleTask& t : host)
    bytes += L.csr_once(t.role, t.inv) + 8.0 * L.kb.W + 8.0 * L.kb.n_words[2 * t.role + t.inv];
  return launch_roles_n(L, d, tasks, (uint32_t)host.size(), bytes);
}

template <typename TW>
hth_status launch_group_chunk(Launcher& L, const DevKB& d, const GroupTask* groups,
                              const GroupMember* members, const std::vector<GroupTask>& host,
                              const GroupChunk& c, const uint32_t* xslots_all, void* tarea, void* parea) {
  const hth_kb_s& kb = L.kb;
  const size_t g0 = c.first;
  const uint32_t n = c.n;
  // byte model: the transpose reads the members' child rows (T is an
  // intermediate of this design, not counted); the pass reads its CSR once per
  // sweep and writes the members' listed words (the other words are filled)
  double tb = 0, gb = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const GroupTask& G = host[g0 + i];
    tb += (double)G.k * kb.W * 8;
    gb += L.csr_once(G.role, G.inv) + (double)G.k * G.n_words * 8;
  }
  TW* T = static_cast<TW*>(tarea);
  // 256 words per block: every word, or the object words of a compact group
  uint32_t span = 1;
  for (uint32_t i = 0; i < n; ++i) {
    const GroupTask& G = host[g0 + i];
    span = std::max(span, G.compact ? G.n_obj_words : kb.W);
  }
  const uint32_t tiles = (span + 255) / 256;
  hth_status s = split_launch(L, HTH_K_TBUILD, tb, n, tiles, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
    hipLaunchKernelGGL(k_tbuild<TW>, dim3(blocks), dim3(256), 0, L.st, d, groups + g0 + i0, members, T, tiles);
  });
  if (s) return s;
  const uint32_t* xslots = c.rounds ? xslots_all + c.slot_off : nullptr;
  uint32_t bpg, nblocks;
  if (xslots) {
    bpg = std::min<uint32_t>(std::max<uint32_t>(1, kb.n_cu / 8 * 8), (kb.W + 3) / 4);
    nblocks = 8 * bpg * c.rounds;
  } else {
    bpg = std::max<uint32_t>(1, (8 * kb.n_cu + n - 1) / n);
    bpg = std::min<uint32_t>(bpg, (kb.W + 3) / 4);
    nblocks = bpg * n;
  }
  // several list words per wave iteration where words hold few assertions
  double ew = 0, nwd = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const GroupTask& G = host[g0 + i];
    ew += (double)(kb.role_base[G.role + 1] - kb.role_base[G.role]);
    nwd += G.n_words;
  }
  const bool multi = nwd > 0 && ew < 96.0 * nwd;
  if (host[g0].short_rows) {   // every row short: a lane per subject, one pass
    // exact 3-bit counts when no row of the launch's directions holds 8 assertions
    uint32_t most = 0;
    for (uint32_t i = 0; i < n; ++i) {
      const GroupTask& G = host[g0 + i];
      most = std::max(most, kb.max_deg[G.inv][G.role]);
    }
    return L.run(HTH_K_GROUP_SHORT, gb, [&] {
      if (most < kGroupMaxCount)
        hipLaunchKernelGGL((k_group_short<TW, kShortWords, kShortSub, true>), dim3(nblocks), dim3(256), 0, L.st,
                           d, groups + g0, members, T, bpg, xslots);
      else
        hipLaunchKernelGGL((k_group_short<TW, kShortWords, kShortSub, false>), dim3(nblocks), dim3(256), 0, L.st,
                           d, groups + g0, members, T, bpg, xslots);
    });
  }
  uint64_t seg_rows;
  const uint32_t P = chunk_segments(kb, host, c, &seg_rows);
  for (uint32_t sg = 0; sg < P; ++sg) {
    SegPass<TW> sp{0, 0xFFFFFFFFu, 1, 1, nullptr, (size_t)kb.W * 256};
    if (P > 1) {
      sp.lo = (uint32_t)(sg * seg_rows);
      sp.hi = (uint32_t)std::min<uint64_t>((sg + 1) * seg_rows, 0xFFFFFFFFu);
      sp.first = sg == 0;
      sp.last = sg == P - 1;
      sp.part = static_cast<TW*>(parea);
    }
    s = L.run(HTH_K_GROUP, sg ? 0.0 : gb, [&] {
      const dim3 grid(nblocks), block(256);
      const bool u16 = kb.tune.group_unroll >= 16;
      if (multi) {   // few assertions per lane: 8 in flight
        hipLaunchKernelGGL((k_group<TW, 8, 4>), grid, block, 0, L.st, d, groups + g0, members, T, bpg, xslots, sp);
      } else {
        if (u16)
          hipLaunchKernelGGL((k_group<TW, 16, 1>), grid, block, 0, L.st, d, groups + g0, members, T, bpg, xslots, sp);
        else
          hipLaunchKernelGGL((k_group<TW, 8, 1>), grid, block, 0, L.st, d, groups + g0, members, T, bpg, xslots, sp);
      }
    });
    if (s) return s;
  }
  return HTH_OK;
}

hth_status launch_groups(Launcher& L, const DevKB& d, const GroupTask* groups,
                         const GroupMember* members, const std::vector<GroupTask>& host,
                         const std::vector<GroupChunk>& chunks, const uint32_t* xslots, void* tarea,
                         void* parea) {
  for (const GroupChunk& c : chunks) {
    hth_status s;
    switch (c.wb) {
      case 1: s = launch_group_chunk<uint8_t>(L, d, groups, members, host, c, xslots, tarea, parea); break;
      case 2: s = launch_group_chunk<uint16_t>(L, d, groups, members, host, c, xslots, tarea, parea); break;
      case 4: s = launch_group_chunk<uint32_t>(L, d, groups, members, host, c, xslots, tarea, parea); break;
      default: s = launch_group_chunk<uint64_t>(L, d, groups, members, host, c, xslots, tarea, parea); break;
    }
    if (s) return s;
  }
  return HTH_OK;
}

// heavy-row scratch of a plan: a partial count per (role task, chunk of its
// direction), the largest level's worth (levels run one after the other)
size_t heavy_counter_bytes(const hth_kb_s& kb, const Plan& P) {
  size_t most = 0;
  for (const PlanLevel& PL : P.levels) {
    size_t nb = 0;
    for (const RoleTask& t : PL.roles)
      nb += kb.chunk_first[2 * t.role + t.inv + 1] - kb.chunk_first[2 * t.role + t.inv];
    most = std::max(most, nb);
  }
  return align_up(most * 4, 256);
}

// A single role node evaluated by k_push: ∃ρ.A or ¬∃ρ.A over an atomic A with
// fewer than push_pct percent of the individuals, where no row of the
// opposite direction is longer than kPushMaxDeg (a member's row is walked by
// one lane).  Otherwise it is counted per subject (k_role).
constexpr uint32_t kPushMaxDeg = 64;
inline bool pushed(const hth_kb_s& kb, const RoleTask& t) {
  if (!kb.tune.push_pct || t.neg || t.child_row >= kb.d.n_concepts) return false;
  const bool exists = t.lo == 1 && t.hi == 0xFFFFFFFFu, none = t.lo == 0 && t.hi == 0;
  if (!exists && !none) return false;
  if (kb.max_deg[t.inv ? 0 : 1][t.role] > kPushMaxDeg) return false;
  return (uint64_t)kb.concept_pop[t.child_row] * 100 < (uint64_t)kb.tune.push_pct * kb.N;
}

// The shared passes of a level as launched: word counts and T layout set.
// Short-row groups first, so that a launch holds groups of one kind.
std::vector<GroupTask> level_groups(const hth_kb_s& kb, const PlanLevel& PL) {
  std::vector<GroupTask> out;
  for (GroupTask g : PL.groups) {
    g.n_words = kb.n_words[2 * g.role + g.inv];
    g.n_obj_words = kb.n_words[(2 * g.role + g.inv) ^ 1u];
    g.compact = kb.tune.t_compact && 2ull * kb.n_obj[2 * g.role + g.inv] <= kb.N;
    g.short_rows = short_rows(kb, 2 * g.role + g.inv);
    out.push_back(g);
  }
  std::stable_partition(out.begin(), out.end(), [](const GroupTask& g) { return g.short_rows != 0; });
  return out;
}

// partial counts of the segmented chunks of a plan (the largest chunk's worth)
size_t partial_bytes(const hth_kb_s& kb, const Plan& P) {
  size_t most = 0;
  for (const PlanLevel& PL : P.levels) {
    std::vector<GroupTask> gs = level_groups(kb, PL);
    for (const GroupChunk& c : chunk_groups(kb, gs)) most = std::max(most, chunk_partial_bytes(kb, gs, c));
  }
  return align_up(most, 256);
}

// the id sets of a plan's CONTAIN restrictions: one bit per dictionary string each
inline size_t idset_words(uint32_t n_strings) { return align_up(((size_t)n_strings + 63) / 64, 8); }
size_t idset_bytes(const Plan& P) {
  size_t n = 0;
  for (const StrTask& t : P.str) n += t.kind == 1;
  return align_up(n * idset_words(P.n_strings) * 8, 256);
}

// bytes of the packed tables plus slots plus T area for a plan
// The T area a plan needs: the most any launch's chunk uses, over its levels
// (the shared passes as launched; never more than t_area_bytes)
size_t plan_t_bytes(const hth_kb_s& kb, const Plan& P) {
  size_t most = 0;
  for (const PlanLevel& PL : P.levels) {
    if (PL.groups.empty()) continue;
    std::vector<GroupTask> gs = level_groups(kb, PL);
    const std::vector<GroupChunk> cs = chunk_groups(kb, gs);
    most = std::max(most, chunks_t_bytes(kb, gs, cs));
  }
  return most;
}

size_t plan_workspace_bytes(const hth_kb_s& kb, const Plan& P) {
  size_t tables = 0;
  auto add = [&](size_t n, size_t each) { tables = align_up(tables, 256) + n * each; };
  size_t n_reg = P.roots.size(), n_role = 0, n_grp = 0, n_mem = 0, n_fill = 0, max_groups = 0;
  for (const PlanLevel& PL : P.levels) {
    n_reg += PL.mat.size();
    n_role += PL.roles.size();
    n_grp += PL.groups.size();
    n_mem += PL.members.size();
    n_fill += PL.roles.size() + PL.members.size();
    max_groups = std::max(max_groups, PL.groups.size());
  }
  add(P.thr.size(), sizeof(ThrTask));
  add(P.thr.size(), sizeof(ThrGroup));
  add(P.num.size(), sizeof(NumTask));
  add(P.str.size(), sizeof(StrTask));
  add(n_reg, sizeof(RegionTask));
  add(n_role, sizeof(RoleTask));
  add(n_role, sizeof(RoleTask));            // pushed role tasks (a subset of the role nodes)
  add(n_grp, sizeof(GroupTask));
  add(n_mem, sizeof(GroupMember));
  add(n_fill, sizeof(FillTask));
  add(P.code.size(), sizeof(uint32_t));
  add(9 * n_grp + 8, sizeof(uint32_t));     // XCD slot tables: at most 8 more than groups per chunk
  return align_up(tables, 256) + (size_t)P.n_slots * kb.S * 8 + (max_groups ? plan_t_bytes(kb, P) : 0) +
         heavy_counter_bytes(kb, P) + partial_bytes(kb, P) + idset_bytes(P);
}

std::once_flag g_attr_once;

// A compiled plan laid out for the device: the table blob with its offsets and
// the host side of the launch sequence.  Built once; uploaded into a workspace
// with one copy; launched any number of times (kernels only).
struct Prepared {
  Plan P;
  Blob blob;
  struct LevelAt { size_t mat, role, group, fill, nrole, ngroup, nfill, nhb, nhc, push, npush; double fill_bytes; };
  std::vector<LevelAt> at;
  size_t root_at = 0;
  std::vector<std::vector<RoleTask>> lv_roles;
  std::vector<std::vector<RoleTask>> lv_push;
  std::vector<std::vector<GroupTask>> lv_groups;
  std::vector<std::vector<GroupChunk>> lv_chunks;
  size_t n_thr_groups = 0, n_thr_tasks = 0;
  size_t o_thr = 0, o_thg = 0, o_reg = 0, o_role = 0, o_grp = 0, o_mem = 0, o_fill = 0, o_code = 0, o_xslot = 0;
  size_t o_push = 0;
  size_t o_num = 0, n_num_blocks = 0;   // numeric concrete-role tasks, their heavy-row blocks
  size_t o_str = 0, n_str_blocks = 0, n_contains = 0;   // string concrete-role tasks
  size_t o_idset = 0;                   // the CONTAIN id sets (workspace offset)
  size_t o_hcnt = 0;   // heavy-row counters (workspace offset)
  size_t o_part = 0;   // partial counts of segmented shared passes (workspace offset)
  size_t tables = 0, need = 0;
  uint32_t n_hyps = 0;
};

void prepare(const hth_kb_s& kb, Plan&& plan, uint32_t n_hyps, Prepared& X) {
  X.P = std::move(plan);
  const Plan& P = X.P;
  X.n_hyps = n_hyps;
  std::vector<RegionTask> regions;
  std::vector<RoleTask> roles;
  std::vector<GroupTask> groups;
  std::vector<GroupMember> members;
  std::vector<FillTask> fills;
  std::vector<RoleTask> pushes;
  std::vector<uint32_t> xslots;
  const size_t NL = P.levels.size();
  X.at.assign(NL, {});
  X.lv_roles.assign(NL, {});
  X.lv_push.assign(NL, {});
  X.lv_groups.assign(NL, {});
  X.lv_chunks.assign(NL, {});
  for (size_t L = 0; L < NL; ++L) {
    const PlanLevel& PL = P.levels[L];
    X.at[L] = {regions.size(), roles.size(), groups.size(), fills.size(), 0, 0, 0, 0, 0, pushes.size(), 0, 0.0};
    regions.insert(regions.end(), PL.mat.begin(), PL.mat.end());
    for (RoleTask t : PL.roles) {
      const uint32_t rd = 2 * t.role + t.inv;
      t.n_words = kb.n_words[rd];
      if (pushed(kb, t)) {
        fills.push_back(FillTask{t.out_row, t.lo == 0 ? 1u : 0u});
        X.at[L].fill_bytes += 8.0 * kb.W;
        pushes.push_back(t);
        X.lv_push[L].push_back(t);
        continue;
      }
      t.hr0 = kb.heavy_first[rd];
      t.hc0 = kb.chunk_first[rd];
      t.h_first = (uint32_t)X.at[L].nhb;
      t.c_first = (uint32_t)X.at[L].nhc;
      X.at[L].nhb += kb.chunk_first[rd + 1] - kb.chunk_first[rd];
      X.at[L].nhc += kb.heavy_first[rd + 1] - kb.heavy_first[rd];
      if (t.n_words < kb.W) {
        fills.push_back(FillTask{t.out_row, t.lo == 0 ? 1u : 0u});
        X.at[L].fill_bytes += 8.0 * (kb.W - t.n_words);
      }
      roles.push_back(t);
      X.lv_roles[L].push_back(t);
    }
    const uint32_t mbase = (uint32_t)members.size();
    for (GroupTask g : level_groups(kb, PL)) {
      if (g.n_words < kb.W) {
        for (uint32_t j = 0; j < g.k; ++j) {
          const uint32_t r = PL.members[g.first + j].out_row;
          if (r == kNone) continue;              // coverage added by the pass, no row
          fills.push_back(FillTask{r, (uint32_t)((g.acc[0] >> j) & 1)});
          X.at[L].fill_bytes += 8.0 * (kb.W - g.n_words);
        }
      }
      g.first += mbase;
      X.lv_groups[L].push_back(g);
    }
    X.lv_chunks[L] = chunk_groups(kb, X.lv_groups[L]);
    for (GroupChunk& c : X.lv_chunks[L])
      if (kb.tune.xcd_local && c.n >= 8) place_on_xcds(kb, X.lv_groups[L], c, xslots);
    groups.insert(groups.end(), X.lv_groups[L].begin(), X.lv_groups[L].end());
    members.insert(members.end(), PL.members.begin(), PL.members.end());
    X.at[L].nrole = roles.size() - X.at[L].role;
    X.at[L].ngroup = groups.size() - X.at[L].group;
    X.at[L].nfill = fills.size() - X.at[L].fill;
    X.at[L].npush = pushes.size() - X.at[L].push;
  }
  X.root_at = regions.size();
  regions.insert(regions.end(), P.roots.begin(), P.roots.end());
  // thresholds grouped by property (at most kThrPerPass per group): one column pass each
  std::vector<ThrTask> thr_tasks(P.thr);
  std::stable_sort(thr_tasks.begin(), thr_tasks.end(),
                   [](const ThrTask& a, const ThrTask& b) { return a.prop < b.prop; });
  std::vector<ThrGroup> thr_groups;
  for (uint32_t i = 0; i < thr_tasks.size(); ++i) {
    if (thr_groups.empty() || thr_groups.back().prop != thr_tasks[i].prop || thr_groups.back().n == kThrPerPass)
      thr_groups.push_back(ThrGroup{thr_tasks[i].prop, i, 0, 0});
    thr_groups.back().n++;
  }
  std::vector<NumTask> num(P.num);
  for (NumTask& t : num) {
    t.base_lo = (uint32_t)P.num_bounds[t.role];
    t.base_hi = (uint32_t)(P.num_bounds[t.role] >> 32);
    t.h_first = (uint32_t)X.n_num_blocks;
    t.hc0 = P.num_chunk_first[t.role];
    X.n_num_blocks += P.num_chunk_first[t.role + 1] - P.num_chunk_first[t.role];
  }
  X.o_num = X.blob.add(num);
  // string tasks: CONTAIN first (k_contains takes them as one range), each
  // with its id set; heavy-row blocks numbered in table order
  std::vector<StrTask> str(P.str);
  std::stable_partition(str.begin(), str.end(), [](const StrTask& t) { return t.kind == 1; });
  for (StrTask& t : str) {
    t.base_lo = (uint32_t)P.str_bounds[t.role];
    t.base_hi = (uint32_t)(P.str_bounds[t.role] >> 32);
    t.hc0 = P.str_chunk_first[t.role];
    t.h_first = (uint32_t)X.n_str_blocks;
    X.n_str_blocks += P.str_chunk_first[t.role + 1] - P.str_chunk_first[t.role];
    if (t.kind == 1) t.set_word = (uint32_t)(X.n_contains++ * idset_words(P.n_strings));
  }
  X.o_str = X.blob.add(str);
  X.n_thr_groups = thr_groups.size();
  X.n_thr_tasks = thr_tasks.size();
  X.o_thr = X.blob.add(thr_tasks);
  X.o_thg = X.blob.add(thr_groups);
  X.o_reg = X.blob.add(regions);
  X.o_role = X.blob.add(roles);
  X.o_grp = X.blob.add(groups);
  X.o_mem = X.blob.add(members);
  X.o_fill = X.blob.add(fills);
  X.o_code = X.blob.add(P.code);
  X.o_xslot = X.blob.add(xslots);
  X.o_push = X.blob.add(pushes);
  X.tables = align_up(X.blob.bytes.size(), 256);
  size_t t_bytes = 0;   // the T area: the most one chunk of the plan uses
  for (size_t L = 0; L < NL; ++L) t_bytes = std::max(t_bytes, chunks_t_bytes(kb, X.lv_groups[L], X.lv_chunks[L]));
  X.o_hcnt = X.tables + (size_t)P.n_slots * kb.S * 8 + t_bytes;
  X.o_part = X.o_hcnt + heavy_counter_bytes(kb, P);
  size_t part = 0;
  for (size_t L = 0; L < NL; ++L)
    for (const GroupChunk& c : X.lv_chunks[L]) part = std::max(part, chunk_partial_bytes(kb, X.lv_groups[L], c));
  X.o_idset = X.o_part + align_up(part, 256);
  X.need = X.o_idset + idset_bytes(P);
}

hth_status check_ws(const Prepared& X, const char* ws, size_t ws_bytes) {
  if (X.need > ws_bytes)
    return fail(HTH_E_NOMEM, "workspace too small: need " + std::to_string(X.need) + " bytes, have " +
                                 std::to_string(ws_bytes));
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(HTH_E_INVALID, "workspace must be 256-byte aligned");
  return HTH_OK;
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// k_role<true> stages the child row in up to lds_per_block bytes of LDS
void role_attributes(const hth_kb_s& kb) {
  std::call_once(g_attr_once, [&] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_role<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kb.lds_per_block);
  });
}

// The kernels of a prepared plan whose tables are in ws: no copies, no
// allocation and no memset (the counts are cleared by a kernel).
hth_status launch_prepared(hth_kb_s& kb, const Prepared& X, char* ws, uint32_t* counts, uint64_t* instances,
                           hipStream_t st) {
  role_attributes(kb);
  const Plan& P = X.P;
  const size_t slot_bytes = (size_t)kb.S * 8;
  DevKB d = dev_view(kb);
  d.sets = P.sets;
  d.n_fixed = kb.d.n_concepts + P.n_sets;
  d.num_roff = P.num_roff;
  d.num_val = P.num_val;
  d.num_heavy_rows = P.num_heavy_rows;
  d.num_heavy_chunks = P.num_heavy_chunks;
  d.str_roff = P.str_roff;
  d.str_ids = P.str_ids;
  d.str_heavy_rows = P.str_heavy_rows;
  d.str_heavy_chunks = P.str_heavy_chunks;
  d.dict_off = P.dict_off;
  d.dict_chars = P.dict_chars;
  d.pat_off = P.pat_off;
  d.pat_chars = P.pat_chars;
  d.n_strings = P.n_strings;
  d.idsets = reinterpret_cast<uint64_t*>(ws + X.o_idset);
  d.slots = reinterpret_cast<uint64_t*>(ws + X.tables);
  d.counts = counts;
  d.instances = instances;
  void* tarea = ws + X.tables + (size_t)P.n_slots * slot_bytes;
  const uint32_t nc = 2 * X.n_hyps;
  hipLaunchKernelGGL(k_zero_u32, dim3((nc + 255) / 256), dim3(256), 0, st, counts, nc);
  HTH_HIP(hipGetLastError());
  const ThrTask* thr = reinterpret_cast<const ThrTask*>(ws + X.o_thr);
  const ThrGroup* thg = reinterpret_cast<const ThrGroup*>(ws + X.o_thg);
  const RegionTask* reg = reinterpret_cast<const RegionTask*>(ws + X.o_reg);
  const RoleTask* rol = reinterpret_cast<const RoleTask*>(ws + X.o_role);
  const GroupTask* grp = reinterpret_cast<const GroupTask*>(ws + X.o_grp);
  const GroupMember* mem = reinterpret_cast<const GroupMember*>(ws + X.o_mem);
  const FillTask* fil = reinterpret_cast<const FillTask*>(ws + X.o_fill);
  const uint32_t* code = reinterpret_cast<const uint32_t*>(ws + X.o_code);
  Launcher Lc{kb, st};
  if (!P.num.empty()) {
    const uint32_t n = (uint32_t)P.num.size();
    const NumTask* nt = reinterpret_cast<const NumTask*>(ws + X.o_num);
    const uint32_t bpt = std::max<uint32_t>(1, std::min<uint32_t>((kb.W + 7) / 8, (32 * kb.n_cu + n - 1) / n));
    double bytes = 0;   // per task: the role's offsets and values once, its row out
    for (const NumTask& t : P.num)
      bytes += 4.0 * (kb.N + 1) + 4.0 * (double)(P.num_bounds[t.role + 1] - P.num_bounds[t.role]) + 8.0 * kb.W;
    hth_status s = split_launch(Lc, HTH_K_THRESHOLD, bytes, n, bpt, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
      hipLaunchKernelGGL(k_numrole, dim3(blocks), dim3(256), 0, st, d, nt + i0, bpt);
    });
    if (s) return s;
    if (X.n_num_blocks) {
      s = split_launch(Lc, HTH_K_THRESHOLD, 0.0, X.n_num_blocks, 1, 256, [&](uint32_t b0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_numrole_heavy, dim3(blocks), dim3(256), 0, st, d, nt, n, b0);
      });
      if (s) return s;
    }
  }
  if (!P.str.empty()) {
    const uint32_t n = (uint32_t)P.str.size();
    const StrTask* sk = reinterpret_cast<const StrTask*>(ws + X.o_str);
    hth_status s = HTH_OK;
    if (X.n_contains) {   // the id sets: the dictionary strings holding each pattern
      const uint32_t tiles = std::max<uint32_t>(1, (P.n_strings + 255) / 256);
      s = split_launch(Lc, HTH_K_THRESHOLD, 0.0, X.n_contains, tiles, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_contains, dim3(blocks), dim3(256), 0, st, d, sk + i0, tiles);
      });
      if (s) return s;
    }
    const uint32_t bpt = std::max<uint32_t>(1, std::min<uint32_t>((kb.W + 7) / 8, (32 * kb.n_cu + n - 1) / n));
    double bytes = 0;   // per task: the role's offsets and ids once, its row out
    for (const StrTask& t : P.str)
      bytes += 4.0 * (kb.N + 1) + 4.0 * (double)(P.str_bounds[t.role + 1] - P.str_bounds[t.role]) + 8.0 * kb.W;
    s = split_launch(Lc, HTH_K_THRESHOLD, bytes, n, bpt, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
      hipLaunchKernelGGL(k_strrole, dim3(blocks), dim3(256), 0, st, d, sk + i0, bpt);
    });
    if (s) return s;
    if (X.n_str_blocks) {
      s = split_launch(Lc, HTH_K_THRESHOLD, 0.0, X.n_str_blocks, 1, 256, [&](uint32_t b0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_strrole_heavy, dim3(blocks), dim3(256), 0, st, d, sk, n, b0);
      });
      if (s) return s;
    }
  }
  if (X.n_thr_groups) {
    // about 32 words per wave: enough independent column loads in flight
    const uint32_t n = (uint32_t)X.n_thr_groups;
    const uint32_t bpt = std::max<uint32_t>(1, (kb.W + 127) / 128);
    std::vector<uint32_t> props;
    for (const ThrTask& t : P.thr) props.push_back(t.prop);
    std::sort(props.begin(), props.end());
    const double bytes = 4.0 * kb.N * (double)(std::unique(props.begin(), props.end()) - props.begin());
    hth_status s = split_launch(Lc, HTH_K_THRESHOLD, bytes, n, bpt, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
      hipLaunchKernelGGL(k_threshold, dim3(blocks), dim3(256), 0, st, d, thg + i0, thr, bpt);
    });
    if (s) return s;
  }
  for (size_t L = 0; L < P.levels.size(); ++L) {
    const PlanLevel& PL = P.levels[L];
    const Prepared::LevelAt& at = X.at[L];
    Lc.csr_seen.clear();
    hth_status s = launch_regions(Lc, d, reg + at.mat, code, PL.mat, P.code);
    if (s) return s;
    if (at.nfill) {
      const uint32_t n = (uint32_t)at.nfill, tiles = fill_tiles(kb.S);
      s = split_launch(Lc, HTH_K_FILL, at.fill_bytes, n, tiles, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_fill_rows, dim3(blocks), dim3(256), 0, st, d, fil + at.fill + i0, tiles);
      });
      if (s) return s;
    }
    if (at.npush) {   // after the fills that set their rows to all zeros / all ones
      const uint32_t n = (uint32_t)at.npush, tiles = (kb.W + 3) / 4;
      const RoleTask* pt = reinterpret_cast<const RoleTask*>(ws + X.o_push) + at.push;
      double bytes = 0;
      for (const RoleTask& t : X.lv_push[L])
        bytes += (double)kb.W * 8 * 2 + 8.0 * kb.concept_pop[t.child_row] +
                 4.0 * kb.concept_pop[t.child_row] *
                     ((double)(kb.role_base[t.role + 1] - kb.role_base[t.role]) / kb.N);
      s = split_launch(Lc, HTH_K_ROLE, bytes, n, tiles, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_push, dim3(blocks), dim3(256), 0, st, d, pt + i0, tiles);
      });
      if (s) return s;
    }
    s = launch_roles(Lc, d, rol + at.role, X.lv_roles[L]);
    if (s) return s;
    if (at.nhc) {   // heavy rows: chunk partials, then the rows' bits
      uint32_t* partial = reinterpret_cast<uint32_t*>(ws + X.o_hcnt);
      const uint32_t nt = (uint32_t)at.nrole;
      s = split_launch(Lc, HTH_K_ROLE, 0.0, at.nhb, 1, 256, [&](uint32_t b0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_role_heavy, dim3(blocks), dim3(256), 0, st, d, rol + at.role, nt, b0, partial);
      });
      if (s) return s;
      s = split_launch(Lc, HTH_K_ROLE, 0.0, at.nhc, 1, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_role_heavy_fix, dim3(blocks), dim3(256), 0, st, d, rol + at.role, nt, i0, partial);
      });
      if (s) return s;
    }
    s = launch_groups(Lc, d, grp + at.group, mem, X.lv_groups[L], X.lv_chunks[L],
                      reinterpret_cast<const uint32_t*>(ws + X.o_xslot), tarea, ws + X.o_part);
    if (s) return s;
  }
  return launch_regions(Lc, d, reg + X.root_at, code, P.roots, P.code);
}

hth_status run_plan(hth_kb_s& kb, Plan&& P, char* ws, size_t ws_bytes, uint32_t* counts, uint32_t n_hyps,
                    uint64_t* instances, hipStream_t st) {
  Prepared X;
  prepare(kb, std::move(P), n_hyps, X);
  hth_status s = check_ws(X, ws, ws_bytes);
  if (s) return s;
  HTH_HIP(hipMemcpyAsync(ws, X.blob.bytes.data(), X.blob.bytes.size(), hipMemcpyHostToDevice, st));
  return launch_prepared(kb, X, ws, counts, instances, st);
}

}  // namespace
}  // namespace hth

using namespace hth;

extern "C" hth_status hth_workspace_bytes(hth_kb kb, uint32_t max_nodes, uint32_t max_hyps,
                                          size_t* bytes) {
  if (!kb || !bytes) return fail(HTH_E_INVALID, "NULL argument");
  if (max_hyps == 0 || max_nodes < max_hyps) return fail(HTH_E_RANGE, "need max_nodes >= max_hyps >= 1");
  // a chunk's T rows: at most t_area_bytes, and at most one row of the widest
  // T word per individual for each of the plan's nodes
  const size_t t_bound = std::min(t_area_bytes(*kb), (size_t)max_nodes * align_up(kb->N, 64) * 8);
  *bytes = align_up(table_bound(max_nodes, max_hyps), 256) + (size_t)(max_nodes + 2) * kb->S * 8 +
           t_bound + align_up((size_t)(max_nodes + 2) * kb->chunk_most * 4, 256) +
           align_up((size_t)(max_nodes + 2) * idset_words(kb->n_strings) * 8, 256);
  return HTH_OK;
}

extern "C" hth_status hth_eval_one(hth_kb kb, const hth_node* nodes, uint32_t n_nodes,
                                   const uint32_t* children, uint32_t n_children, void* ws,
                                   size_t ws_bytes, uint64_t* d_instances, uint32_t* d_counts,
                                   void* stream) {
  if (!kb || !nodes || !ws || !d_counts) return fail(HTH_E_INVALID, "NULL argument");
  if (n_children && !children) return fail(HTH_E_INVALID, "children is NULL");
  uint32_t offs[2] = {0, n_nodes};
  PlanOptions opt;
  opt.instances = d_instances != nullptr;
  Plan P;
  hth_status s = compile_plan(*kb, nodes, offs, 1, children, n_children, opt, P);
  if (s) return s;
  std::lock_guard<std::mutex> g(kb->mu);
  return run_plan(*kb, std::move(P), static_cast<char*>(ws), ws_bytes, d_counts, 1, d_instances,
                  static_cast<hipStream_t>(stream));
}

// The workspace of hth_eval_one_noalloc: a fixed array in the code object's
// device data, one copy per GPU, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host it is only
// a stand-in); it uses the device address hipGetSymbolAddress gives for the
// GPU the call runs on.
namespace hth {
namespace {
__device__ __align__(256) uint64_t scratch[HTH_NOALLOC_SCRATCH_BYTES / 8];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// The scratch array's address on `device`, looked up once per device with
// that device current (the caller's current device is restored).
hth_status scratch_on(int device, char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(HTH_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[device]) {
    int cur = 0;
    HTH_HIP(hipGetDevice(&cur));
    if (cur != device) HTH_HIP(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) HTH_HIP(hipSetDevice(cur));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || reinterpret_cast<uintptr_t>(p) % 256) return fail(HTH_E_DEVICE, "scratch address not 256-byte aligned");
    g_scratch[device] = static_cast<char*>(p);
  }
  *out = g_scratch[device];
  return HTH_OK;
}
}  // namespace
}  // namespace hth

extern "C" hth_status hth_eval_one_noalloc(hth_kb kb, const hth_node* nodes, uint32_t n_nodes,
                                           const uint32_t* children, uint32_t n_children,
                                           uint64_t* d_instances, uint32_t* d_counts, void* stream) {
  if (!kb || !nodes || !d_counts) return fail(HTH_E_INVALID, "NULL argument");
  if (n_children && !children) return fail(HTH_E_INVALID, "children is NULL");
  uint32_t offs[2] = {0, n_nodes};
  PlanOptions opt;
  opt.instances = d_instances != nullptr;
  Plan P;
  hth_status s = compile_plan(*kb, nodes, offs, 1, children, n_children, opt, P);
  if (s) return s;
  char* ws = nullptr;
  s = scratch_on(kb->device, &ws);
  if (s) return s;
  std::lock_guard<std::mutex> g(kb->mu);
  Prepared X;
  prepare(*kb, std::move(P), 1, X);
  if (X.need > (size_t)HTH_NOALLOC_SCRATCH_BYTES)
    return fail(HTH_E_NOMEM, "hth_eval_one_noalloc: this hypothesis needs " + std::to_string(X.need) +
                                 " bytes of workspace; the fixed scratch holds " +
                                 std::to_string((size_t)HTH_NOALLOC_SCRATCH_BYTES) +
                                 " (use hth_eval_one with a caller workspace)");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  HTH_HIP(hipMemcpyAsync(ws, X.blob.bytes.data(), X.blob.bytes.size(), hipMemcpyHostToDevice, st));
  return launch_prepared(*kb, X, ws, d_counts, d_instances, st);
}

namespace {
hth_status eval_batch_impl(hth_kb kb, const hth_node* nodes, const uint32_t* hyp_node_offsets,
                           uint32_t n_hyps, const uint32_t* children, uint32_t n_children, void* ws,
                           size_t ws_bytes, uint64_t* d_sets, uint32_t* d_counts, void* stream) {
  if (!kb || !nodes || !hyp_node_offsets || !ws || !d_counts)
    return fail(HTH_E_INVALID, "NULL argument");
  if (n_children && !children) return fail(HTH_E_INVALID, "children is NULL");
  if (n_hyps == 0) return HTH_OK;
  if (hyp_node_offsets[0] != 0) return fail(HTH_E_INVALID, "hyp_node_offsets[0] must be 0");
  PlanOptions opt;
  opt.group_min = kb->tune.group_min ? kb->tune.group_min : 0xFFFFFFFFu;
  opt.group_k = kb->tune.group_k;
  opt.instances = d_sets != nullptr;
  Plan P;
  hth_status s = compile_plan(*kb, nodes, hyp_node_offsets, n_hyps, children, n_children, opt, P);
  if (s) return s;
  std::lock_guard<std::mutex> g(kb->mu);
  return run_plan(*kb, std::move(P), static_cast<char*>(ws), ws_bytes, d_counts, n_hyps, d_sets,
                  static_cast<hipStream_t>(stream));
}
}  // namespace

extern "C" hth_status hth_eval_batch(hth_kb kb, const hth_node* nodes, const uint32_t* hyp_node_offsets,
                                     uint32_t n_hyps, const uint32_t* children, uint32_t n_children,
                                     void* ws, size_t ws_bytes, uint32_t* d_counts, void* stream) {
  return eval_batch_impl(kb, nodes, hyp_node_offsets, n_hyps, children, n_children, ws, ws_bytes,
                         nullptr, d_counts, stream);
}

extern "C" hth_status hth_eval_batch_sets(hth_kb kb, const hth_node* nodes,
                                          const uint32_t* hyp_node_offsets, uint32_t n_hyps,
                                          const uint32_t* children, uint32_t n_children, void* ws,
                                          size_t ws_bytes, uint64_t* d_sets, uint32_t* d_counts,
                                          void* stream) {
  if (!d_sets) return fail(HTH_E_INVALID, "d_sets is NULL");
  return eval_batch_impl(kb, nodes, hyp_node_offsets, n_hyps, children, n_children, ws, ws_bytes,
                         d_sets, d_counts, stream);
}

// The cross-batch subexpression cache (hth_cache_*): the library's LRU over
// the caller's rows, registered as the kb's set table.
struct hth_cache_s {
  hth_kb kb = nullptr;
  hth::SubexprCache* c = nullptr;
  uint64_t* rows = nullptr;
  uint32_t n_rows = 0;
  std::mutex mu;   // one cached evaluation at a time: compile, admit, launch
  ~hth_cache_s() { hth::cache_delete(c); }
};

extern "C" hth_status hth_cache_create(hth_kb kb, uint64_t* d_rows, uint32_t n_rows, hth_cache* out) {
  if (!kb || !d_rows || !out) return fail(HTH_E_INVALID, "NULL argument");
  if (n_rows == 0 || n_rows >= (1u << 24)) return fail(HTH_E_RANGE, "a cache holds 1 .. 2^24 - 1 rows");
  if (reinterpret_cast<uintptr_t>(d_rows) % 64) return fail(HTH_E_INVALID, "cache rows must be 64-byte aligned");
  hth_cache_s* c = new (std::nothrow) hth_cache_s();
  if (!c) return fail(HTH_E_NOMEM, "host allocation failed");
  c->c = cache_new(n_rows);
  if (!c->c) {
    delete c;
    return fail(HTH_E_NOMEM, "host allocation failed");
  }
  c->kb = kb;
  c->rows = d_rows;
  c->n_rows = n_rows;
  std::lock_guard<std::mutex> g(kb->mu);
  kb->sets = d_rows;
  kb->n_sets = n_rows;
  *out = c;
  return HTH_OK;
}

extern "C" hth_status hth_cache_destroy(hth_cache cache) {
  if (!cache) return HTH_OK;
  {
    std::lock_guard<std::mutex> g(cache->kb->mu);
    if (cache->kb->sets == cache->rows) {
      cache->kb->sets = nullptr;
      cache->kb->n_sets = 0;
    }
  }
  delete cache;
  return HTH_OK;
}

extern "C" hth_status hth_cache_stats(hth_cache cache, hth_cache_info* out) {
  if (!cache || !out) return fail(HTH_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(cache->mu);
  const CacheCounters k = cache_counters(cache->c);
  *out = hth_cache_info{k.hits, k.misses, k.admitted, k.evictions, k.batches, k.entries, k.rows};
  return HTH_OK;
}

extern "C" hth_status hth_eval_batch_cached(hth_kb kb, hth_cache cache, const hth_node* nodes,
                                            const uint32_t* hyp_node_offsets, uint32_t n_hyps,
                                            const uint32_t* children, uint32_t n_children, void* ws,
                                            size_t ws_bytes, uint32_t* d_counts, void* stream) {
  if (!kb || !cache || !nodes || !hyp_node_offsets || !ws || !d_counts) return fail(HTH_E_INVALID, "NULL argument");
  if (cache->kb != kb) return fail(HTH_E_INVALID, "the cache belongs to another kb");
  if (n_children && !children) return fail(HTH_E_INVALID, "children is NULL");
  if (n_hyps == 0) return HTH_OK;
  if (hyp_node_offsets[0] != 0) return fail(HTH_E_INVALID, "hyp_node_offsets[0] must be 0");
  std::lock_guard<std::mutex> gc(cache->mu);
  {
    std::lock_guard<std::mutex> g(kb->mu);
    if (kb->sets != cache->rows) return fail(HTH_E_STATE, "another set table replaced the cache's rows");
  }
  for (uint32_t h = 0; h < n_hyps; ++h)
    for (uint32_t i = hyp_node_offsets[h]; i < hyp_node_offsets[h + 1]; ++i)
      if (nodes[i].op == HTH_SET)
        return fail(HTH_E_UNSUPPORTED, "set-table leaves are the cache's own rows in a cached evaluation");
  PlanOptions opt;
  opt.group_min = kb->tune.group_min ? kb->tune.group_min : 0xFFFFFFFFu;
  opt.group_k = kb->tune.group_k;
  opt.cache = cache->c;
  Plan P;
  hth_status s = compile_plan(*kb, nodes, hyp_node_offsets, n_hyps, children, n_children, opt, P);
  if (s) {
    cache_rollback(cache->c);
    return s;
  }
  std::lock_guard<std::mutex> g(kb->mu);
  s = run_plan(*kb, std::move(P), static_cast<char*>(ws), ws_bytes, d_counts, n_hyps, nullptr,
               static_cast<hipStream_t>(stream));
  if (s) cache_rollback(cache->c);
  return s;
}

// A compiled batch kept for repeated launches (hth_plan_*).
struct hth_plan_s {
  hth_kb kb = nullptr;
  hth::Prepared X;
  hth_kb_s::Tuning tune;   // the schedule the tables were laid out for
};

namespace hth {
// The kb's schedule replaced by a plan's for the duration of its launch (the
// caller holds kb.mu): the launch sizes and the workspace areas it was laid
// out with stay consistent whatever hth_kb_set_tuning did since.
struct TuneScope {
  hth_kb_s& kb;
  hth_kb_s::Tuning saved;
  TuneScope(hth_kb_s& k, const hth_kb_s::Tuning& t) : kb(k), saved(k.tune) { kb.tune = t; }
  ~TuneScope() { kb.tune = saved; }
};
}  // namespace hth

extern "C" hth_status hth_plan_create(hth_kb kb, const hth_node* nodes, const uint32_t* hyp_node_offsets,
                                      uint32_t n_hyps, const uint32_t* children, uint32_t n_children,
                                      hth_plan* out, size_t* ws_bytes) {
  if (!kb || !nodes || !hyp_node_offsets || !out || !ws_bytes) return fail(HTH_E_INVALID, "NULL argument");
  if (n_children && !children) return fail(HTH_E_INVALID, "children is NULL");
  if (n_hyps == 0) return fail(HTH_E_RANGE, "a plan needs at least one hypothesis");
  if (hyp_node_offsets[0] != 0) return fail(HTH_E_INVALID, "hyp_node_offsets[0] must be 0");
  PlanOptions opt;
  opt.group_min = kb->tune.group_min ? kb->tune.group_min : 0xFFFFFFFFu;
  opt.group_k = kb->tune.group_k;
  Plan P;
  hth_status s = compile_plan(*kb, nodes, hyp_node_offsets, n_hyps, children, n_children, opt, P);
  if (s) return s;
  hth_plan_s* pl = new (std::nothrow) hth_plan_s();
  if (!pl) return fail(HTH_E_NOMEM, "host allocation failed");
  pl->kb = kb;
  pl->tune = kb->tune;
  prepare(*kb, std::move(P), n_hyps, pl->X);
  *out = pl;
  *ws_bytes = pl->X.need;
  return HTH_OK;
}

extern "C" hth_status hth_plan_upload(hth_plan plan, void* ws, size_t ws_bytes, void* stream) {
  if (!plan || !ws) return fail(HTH_E_INVALID, "NULL argument");
  hth_status s = check_ws(plan->X, static_cast<char*>(ws), ws_bytes);
  if (s) return s;
  HTH_HIP(hipMemcpyAsync(ws, plan->X.blob.bytes.data(), plan->X.blob.bytes.size(), hipMemcpyHostToDevice,
                         static_cast<hipStream_t>(stream)));
  return HTH_OK;
}

extern "C" hth_status hth_plan_launch(hth_plan plan, void* ws, size_t ws_bytes, uint32_t* d_counts,
                                      void* stream) {
  if (!plan || !ws || !d_counts) return fail(HTH_E_INVALID, "NULL argument");
  hth_status s = check_ws(plan->X, static_cast<char*>(ws), ws_bytes);
  if (s) return s;
  std::lock_guard<std::mutex> g(plan->kb->mu);
  TuneScope ts(*plan->kb, plan->tune);
  return launch_prepared(*plan->kb, plan->X, static_cast<char*>(ws), d_counts, nullptr,
                         static_cast<hipStream_t>(stream));
}

extern "C" hth_status hth_plan_destroy(hth_plan plan) {
  delete plan;
  return HTH_OK;
}

extern "C" hth_status hth_batch_workspace_bytes(hth_kb kb, const hth_node* nodes,
                                                 const uint32_t* hyp_node_offsets, uint32_t n_hyps,
                                                 const uint32_t* children, uint32_t n_children,
                                                 size_t* bytes) {
  if (!kb || !nodes || !hyp_node_offsets || !bytes) return fail(HTH_E_INVALID, "NULL argument");
  if (n_children && !children) return fail(HTH_E_INVALID, "children is NULL");
  if (n_hyps == 0) {
    *bytes = 0;
    return HTH_OK;
  }
  PlanOptions opt;
  opt.group_min = kb->tune.group_min ? kb->tune.group_min : 0xFFFFFFFFu;
  opt.group_k = kb->tune.group_k;
  Plan P;
  hth_status s = compile_plan(*kb, nodes, hyp_node_offsets, n_hyps, children, n_children, opt, P);
  if (s) return s;
  *bytes = plan_workspace_bytes(*kb, P) + 4096;
  return HTH_OK;
}

extern "C" hth_status hth_profile_begin(hth_kb kb) {
  if (!kb) return fail(HTH_E_INVALID, "kb is NULL");
  std::lock_guard<std::mutex> g(kb->mu);
  if (kb->prof) return fail(HTH_E_STATE, "profiling already active");
  kb->prof = true;
  kb->prof_recs.clear();
  return HTH_OK;
}

extern "C" hth_status hth_profile_end(hth_kb kb, hth_prof_entry* out) {
  if (!kb || !out) return fail(HTH_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(kb->mu);
  if (!kb->prof) return fail(HTH_E_STATE, "profiling not active");
  kb->prof = false;
  for (int k = 0; k < HTH_K_NUM; ++k) out[k] = hth_prof_entry{0, 0.0, 0.0};
  hth_status st = HTH_OK;
  for (auto& r : kb->prof_recs) {
    float ms = 0;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && st == HTH_OK) st = hip_fail(e, "hipEventElapsedTime");
    out[r.kind].launches += 1;
    out[r.kind].ms += ms;
    out[r.kind].bytes += r.bytes;
    kb->event_pool.push_back(r.a);
    kb->event_pool.push_back(r.b);
  }
  kb->prof_recs.clear();
  return st;
}

#include "devplan.h"
