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
//                concatenated assertion range 64 at a time (coalesced target
//                loads), tests each object against the child row, and each
//                subject lane counts its own assertions in the chunk as
//                popcount(ballot & its lane range).  Skewed degrees are balanced
//                inside the wave by construction; rows stop contributing once
//                their count decides the predicate, and the walk jumps past
//                chunks that hold only decided rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hth_internal.h"
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
__global__ void __launch_bounds__(256)
k_threshold(DevKB kb, const ThrTask* __restrict__ tasks, uint32_t bpt) {
  const uint32_t task = blockIdx.x / bpt, b = blockIdx.x % bpt;
  const ThrTask T = tasks[task];
  const float* col = kb.data + (size_t)T.prop * kb.N;
  uint64_t* out = out_ptr(kb, T.out_row);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint32_t w = b * 4 + wv; w < kb.W; w += bpt * 4) {
    const uint32_t x = w * 64 + lane;
    bool v = false;
    if (x < kb.N) {
      const float f = col[x];
      v = T.le ? (f <= T.t) : (f >= T.t);   // NaN (no value) compares false
    }
    const uint64_t m = __ballot(v);
    if (lane == 0) out[w] = m;
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
  if (T.out_row != kNone && w < kb.S) out_ptr(kb, T.out_row)[w] = top;
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

// ---------------------------------------------------------------------------
// single role restriction, one wave per 64 subjects
// ---------------------------------------------------------------------------
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
  const uint32_t ohi = in ? off[x + 1] : olo;
  const uint32_t ee = (uint32_t)__shfl((int)ohi, 63, 64);
  uint32_t i0 = (uint32_t)__shfl((int)olo, 0, 64);
  uint32_t cnt = 0;
  while (i0 < ee) {
    const uint32_t e = i0 + lane;
    bool v = false;
    if (e < ee) {
      const uint32_t t = (uint32_t)tg[e];
      const uint64_t word = child[t >> 6];
      v = ((uint32_t)(word >> (t & 63)) & 1u) ^ neg;
    }
    const uint64_t m = __ballot(v);
    const uint32_t a = olo > i0 ? min(olo - i0, 64u) : 0u;
    const uint32_t b = ohi > i0 ? min(ohi - i0, 64u) : 0u;
    if (b > a) {
      const uint64_t rm = (b - a == 64) ? ~0ull : (((1ull << (b - a)) - 1ull) << a);
      cnt += (uint32_t)__popcll(m & rm);
    }
    const uint64_t pend = __ballot(in && cnt < sat && ohi > i0 + 64);
    if (!pend) break;
    const int l = __ffsll((unsigned long long)pend) - 1;
    const uint32_t nxt = (uint32_t)__shfl((int)olo, l, 64);
    i0 = max(i0 + 64, nxt);
  }
  const bool res = in && cnt >= lo && cnt <= hi;
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


// ---------------------------------------------------------------------------
// shared role passes: up to 64 role nodes of one (role, direction, level)
// ---------------------------------------------------------------------------
// 64 x 64 bit-matrix transpose in registers: on entry a[j] bit b = M[j][b], on
// exit a[b] bit j = M[j][b].  Recursive exchange of off-diagonal blocks.
__device__ __forceinline__ void transpose64(uint64_t (&a)[64]) {
  uint64_t m = 0x00000000FFFFFFFFull;
#pragma unroll
  for (int j = 32; j != 0; j >>= 1, m ^= (m << j)) {
#pragma unroll
    for (int k = 0; k < 64; k = ((k | j) + 1) & ~j) {
      const uint64_t t = ((a[k] >> j) ^ a[k | j]) & m;
      a[k | j] ^= t;
      a[k] ^= t << j;
    }
  }
}

// T_g[y] bit j = bit(child_j, y) ^ neg_j for the groups of one launch; one lane
// per 64-individual word, transposed in registers.  T rows are TW wide
// (8 * sizeof(TW) >= every group's k).
template <typename TW>
__global__ void __launch_bounds__(256)
k_tbuild(DevKB kb, const GroupTask* __restrict__ groups, const GroupMember* __restrict__ members,
         TW* __restrict__ tarea, uint64_t t_stride, uint32_t tiles) {
  constexpr int KB = 8 * sizeof(TW);
  const uint32_t g = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const GroupTask G = groups[g];
  const uint32_t w = tile * 256 + threadIdx.x;
  if (w >= kb.W) return;
  uint64_t a[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    uint64_t v = 0;
    if (j < KB && (uint32_t)j < G.k) {
      const GroupMember M = members[G.first + j];
      v = row_ptr(kb, M.child_row)[w] ^ (M.neg ? ~0ull : 0ull);
    }
    a[j] = v;
  }
  transpose64(a);
  TW* T = tarea + (size_t)g * t_stride + (size_t)w * 64;
#pragma unroll
  for (int b = 0; b < 64; ++b) T[b] = (TW)a[b];
}

// Saturating per-member counters for all members of a group at once, one bit
// per member in each plane: count = c2 c1 c0 (0..7) unless ov (count >= 8).
template <typename TW>
struct Planes {
  TW c0, c1, c2, ov;
};

template <typename TW>
__device__ __forceinline__ void planes_inc(Planes<TW>& p, TW v) {   // +1 where v has a bit
  const TW k0 = p.c0 & v;
  p.c0 ^= v;
  const TW k1 = p.c1 & k0;
  p.c1 ^= k0;
  const TW k2 = p.c2 & k1;
  p.c2 ^= k1;
  p.ov |= k2;
}

template <typename TW>
__device__ __forceinline__ void planes_add(Planes<TW>& a, const Planes<TW>& b) {
  const TW s0 = a.c0 ^ b.c0, k0 = a.c0 & b.c0;
  const TW t1 = a.c1 ^ b.c1, s1 = t1 ^ k0, k1 = (a.c1 & b.c1) | (k0 & t1);
  const TW t2 = a.c2 ^ b.c2, s2 = t2 ^ k1, k2 = (a.c2 & b.c2) | (k1 & t2);
  a.c0 = s0;
  a.c1 = s1;
  a.c2 = s2;
  a.ov = a.ov | b.ov | k2;
}

template <typename TW>
__device__ __forceinline__ TW shfl_up_w(TW v, int d) {
  if constexpr (sizeof(TW) == 8) return (TW)__shfl_up((unsigned long long)v, d, 64);
  else return (TW)__shfl_up((unsigned int)v, d, 64);
}

template <typename TW>
__device__ __forceinline__ Planes<TW> planes_shfl_up(const Planes<TW>& p, int d) {
  return Planes<TW>{shfl_up_w(p.c0, d), shfl_up_w(p.c1, d), shfl_up_w(p.c2, d), shfl_up_w(p.ov, d)};
}

// Zero-count results for the words of a role direction without assertions.
__global__ void __launch_bounds__(256)
k_fill_rows(DevKB kb, const FillTask* __restrict__ tasks, uint32_t tiles) {
  const uint32_t t = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const FillTask F = tasks[t];
  const uint32_t w = tile * 256 + threadIdx.x;
  if (w >= kb.S) return;
  uint64_t v = 0;
  if (F.ones && w < kb.W) v = w == kb.W - 1 ? kb.tail : ~0ull;
  out_ptr(kb, F.out_row)[w] = v;
}

// 64 x 64 bit transpose across the lanes of a wave: on entry lane l holds row
// l (bit j = M[l][j]); on exit lane l holds column l (bit j = M[j][l]).  Six
// butterfly stages, each swapping the off-diagonal blocks with the partner lane.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x, int lane) {
  uint64_t m = 0x00000000FFFFFFFFull;
#pragma unroll
  for (int d = 32; d != 0; d >>= 1, m ^= (m << d)) {
    const uint64_t y = __shfl_xor((unsigned long long)x, d, 64);
    x = (lane & d) ? (((y >> d) & m) | (x & ~m)) : ((x & m) | ((y << d) & ~m));
  }
  return x;
}

// One wave per 64 subjects (one word of every member's output row), all members
// of the group at once.  The word's assertions are cut into 64 contiguous
// slices of ceil(E_w / 64), one per lane (balanced whatever the degrees); a lane
// walks its slice, fetches each object's T row (one load serves every member)
// and adds it into bit-sliced counters, closing a row's counters when the row
// ends.  Rows that straddle slices leave a tail partial in each lane they cross;
// one segmented scan over the lanes adds them up for the lane holding the row's
// last assertion.  Finally lane x evaluates every member's predicate for
// subject x from the acceptance masks and the result is transposed by ballots.
template <typename TW, int U, bool NT>   // U: assertions in flight per lane;
                                          // NT: stream the CSR past the caches
__global__ void __launch_bounds__(256)
k_group(DevKB kb, const GroupTask* __restrict__ groups, const GroupMember* __restrict__ members,
        const TW* __restrict__ tarea, uint64_t t_stride, uint32_t bpg, uint32_t n_groups,
        uint32_t xcd_local) {
  constexpr uint32_t kStage = 1024;   // assertions of a word staged in LDS
  __shared__ uint32_t s_ro[4][65];
  __shared__ TW s_fin[4][4][64];
  __shared__ int32_t s_tg[4][kStage];
  uint32_t g, b;
  if (xcd_local) {
    // workgroups are dealt to the 8 XCDs round robin: keep every block of a
    // group on one XCD so that its L2 serves that group's T rows
    const uint32_t x = blockIdx.x & 7, j = blockIdx.x >> 3;
    g = x + 8 * (j / bpg);
    b = j % bpg;
    if (g >= n_groups) return;
  } else {
    g = blockIdx.x / bpg;
    b = blockIdx.x % bpg;
  }
  const GroupTask* G = groups + g;
  const uint32_t k = G->k;
  const TW* T = tarea + (size_t)g * t_stride;
  const size_t roff = (size_t)G->role * (kb.N + 1);
  const uint32_t* off = (G->inv ? kb.inv_off : kb.fwd_off) + roff;
  const int32_t* tg = (G->inv ? kb.inv_tg : kb.fwd_tg) + kb.role_base[G->role];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t* ro = s_ro[wv];
  TW(*fin)[64] = s_fin[wv];
  TW acc[kGroupMaxCount + 1];
#pragma unroll
  for (int v = 0; v <= (int)kGroupMaxCount; ++v) acc[v] = (TW)G->acc[v];
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wstep = bpg * nw;
  const uint32_t* words = kb.words + (size_t)(2 * G->role + G->inv) * kb.W;
  const uint32_t n_words = G->n_words;
  uint32_t i = b * nw + wv;
  uint32_t olo_n = 0, ohi_n = 0;     // row offsets of the wave's next word, fetched ahead
  if (i < n_words) {
    const uint32_t xn = words[i] * 64 + lane;
    olo_n = off[xn < kb.N ? xn : kb.N];
    ohi_n = xn < kb.N ? off[xn + 1] : olo_n;
  }
  for (; i < n_words; i += wstep) {
    const uint32_t w = words[i];
    const uint32_t x = w * 64 + lane;
    const bool in = x < kb.N;
    const uint32_t olo = olo_n, ohi = ohi_n;
    if (i + wstep < n_words) {
      const uint32_t xn = words[i + wstep] * 64 + lane;
      olo_n = off[xn < kb.N ? xn : kb.N];
      ohi_n = xn < kb.N ? off[xn + 1] : olo_n;
    }
    ro[lane] = olo;
    if (lane == 63) ro[64] = ohi;
    fin[0][lane] = fin[1][lane] = fin[2][lane] = fin[3][lane] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t E0 = (uint32_t)__shfl((int)olo, 0, 64);
    const uint32_t E1 = (uint32_t)__shfl((int)ohi, 63, 64);
    const uint32_t S = (E1 - E0 + 63) >> 6;
    const uint32_t s = E0 + lane * S;
    const uint32_t se = min(s + S, E1);
    // the word's targets, loaded coalesced into LDS when they fit; lanes then
    // read their contiguous slices from there
    int32_t* stg = s_tg[wv];
    const bool staged = E1 - E0 <= kStage;
    if (staged) {
#pragma unroll 4
      for (uint32_t i = lane; i < E1 - E0; i += 64) stg[i] = tg[E0 + i];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    Planes<TW> cur{0, 0, 0, 0}, hp{0, 0, 0, 0}, tp{0, 0, 0, 0};
    int hp_row = -1, key = -2 - lane;
    if (s < se) {
      int r = 0;
#pragma unroll
      for (int step = 32; step; step >>= 1)
        if (r + step <= 63 && ro[r + step] <= s) r += step;
      bool head = ro[r] < s;
      uint32_t rend = ro[r + 1];
      for (uint32_t e0 = s; e0 < se; e0 += U) {
        int32_t t[U];
        TW v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
          t[u] = (e0 + u < se)
                     ? (staged ? stg[e0 + u - E0]
                               : (NT ? __builtin_nontemporal_load(tg + e0 + u) : tg[e0 + u]))
                     : 0;
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = (e0 + u < se) ? T[(uint32_t)t[u]] : (TW)0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t e = e0 + u;
          if (e < se) {
            while (e >= rend) {          // row r is complete in this slice
              if (head) {
                hp = cur;
                hp_row = r;
              } else {
                fin[0][r] = cur.c0;
                fin[1][r] = cur.c1;
                fin[2][r] = cur.c2;
                fin[3][r] = cur.ov;
              }
              cur = Planes<TW>{0, 0, 0, 0};
              head = false;
              ++r;
              rend = ro[r + 1];
            }
            planes_inc(cur, v[u]);
          }
        }
      }
      if (rend > se) {                    // the row continues past this slice
        tp = cur;
        key = r;
      } else if (head) {
        hp = cur;
        hp_row = r;
      } else {
        fin[0][r] = cur.c0;
        fin[1][r] = cur.c1;
        fin[2][r] = cur.c2;
        fin[3][r] = cur.ov;
      }
    }
    // segmented inclusive scan of the tail partials, keyed by row; stops once no
    // segment is longer than the distance covered (most rows cross one boundary)
    for (int d = 1; d < 64; d <<= 1) {
      const int pk = __shfl_up(key, d, 64);
      if (!__ballot(lane >= d && pk == key)) break;
      const Planes<TW> pp = planes_shfl_up(tp, d);
      if (lane >= d && pk == key) planes_add(tp, pp);
    }
    {
      const int pk = __shfl_up(key, 1, 64);
      const Planes<TW> pp = planes_shfl_up(tp, 1);
      if (hp_row >= 0) {
        if (lane > 0 && pk == hp_row) planes_add(hp, pp);
        fin[0][hp_row] = hp.c0;
        fin[1][hp_row] = hp.c1;
        fin[2][hp_row] = hp.c2;
        fin[3][hp_row] = hp.ov;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // predicate of every member for subject x
    const TW c0 = fin[0][lane], c1 = fin[1][lane], c2 = fin[2][lane], ov = fin[3][lane];
    const TW n0 = ~c0, n1 = ~c1, n2 = ~c2;
    TW res = (n2 & n1 & n0 & acc[0]) | (n2 & n1 & c0 & acc[1]) | (n2 & c1 & n0 & acc[2]) |
             (n2 & c1 & c0 & acc[3]) | (c2 & n1 & n0 & acc[4]) | (c2 & n1 & c0 & acc[5]) |
             (c2 & c1 & n0 & acc[6]) | (c2 & c1 & c0 & acc[7]);
    res = (res & ~ov) | (ov & acc[8]);
    if (!in) res = 0;
    const uint64_t mine = wave_transpose64((uint64_t)res, lane);
    if ((uint32_t)lane < k) out_ptr(kb, members[G->first + lane].out_row)[w] = mine;
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------------------
// executor
// ---------------------------------------------------------------------------
// The T rows of the groups of one launch stay within kb.tune.t_budget bytes so
// that the random T fetches of a launch stay in the last-level caches.
inline uint32_t t_width_bytes(uint32_t k) { return k <= 8 ? 1 : k <= 16 ? 2 : k <= 32 ? 4 : 8; }
inline size_t t_area_bytes(const hth_kb_s& kb) {
  return std::max<size_t>(kb.tune.t_budget, align_up(kb.N, 64) * 8);
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
  b += align_up((n + max_hyps) * sizeof(RegionTask), 256);
  b += align_up(n * sizeof(RoleTask), 256);
  b += align_up(n * sizeof(GroupTask), 256);
  b += align_up(n * sizeof(GroupMember), 256);
  b += align_up((4 * n + 16) * sizeof(uint32_t), 256);
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
  d.pos = kb.pos;
  d.neg = kb.neg;
  d.n_concepts = kb.d.n_concepts;
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

// algorithmic bytes of a region task: every distinct row it reads once, its
// output row once, the two example rows when it counts coverage
double region_bytes(const hth_kb_s& kb, const RegionTask& t, const std::vector<uint32_t>& code) {
  const double w8 = (double)kb.W * 8;
  std::vector<uint32_t> leaves;
  for (uint32_t i = 0; i < t.code_len; ++i) {
    const uint32_t ins = code[t.code_off + i];
    if ((ins & 15u) == RP_LEAF) leaves.push_back(ins >> 5);
  }
  std::sort(leaves.begin(), leaves.end());
  leaves.erase(std::unique(leaves.begin(), leaves.end()), leaves.end());
  double b = leaves.size() * w8;
  if (t.out_row != kNone) b += w8;
  if (t.cover != kNone) b += 2 * w8 + 8;
  return b;
}

// a CSR direction scanned once: 32-bit row offsets and the role's targets
double csr_bytes(const hth_kb_s& kb, uint32_t role, uint32_t inv) {
  const double words = kb.n_words.empty() ? kb.W : kb.n_words[2 * role + inv];
  return 4.0 * std::min<double>((double)kb.N + 1, 65.0 * words) +
         4.0 * (double)(kb.role_base[role + 1] - kb.role_base[role]);
}

hth_status launch_regions(Launcher& L, const DevKB& d, const RegionTask* tasks, const uint32_t* code,
                          const std::vector<RegionTask>& host, const std::vector<uint32_t>& hcode) {
  const uint32_t n = (uint32_t)host.size();
  if (!n) return HTH_OK;
  double bytes = 0;
  if (L.kb.prof)
    for (const RegionTask& t : host) bytes += region_bytes(L.kb, t, hcode);
  const uint32_t tiles = (d.S + kRegionThreads - 1) / kRegionThreads;
  return L.run(HTH_K_REGION, bytes, [&] {
    hipLaunchKernelGGL(k_region, dim3(tiles * n), dim3(kRegionThreads), 0, L.st, d, tasks, code, n);
  });
}

hth_status launch_roles(Launcher& L, const DevKB& d, const RoleTask* tasks,
                        const std::vector<RoleTask>& host) {
  const hth_kb_s& kb = L.kb;
  const uint32_t n = (uint32_t)host.size();
  if (!n) return HTH_OK;
  double bytes = 0;
  for (const RoleTask& t : host) bytes += csr_bytes(kb, t.role, t.inv) + 2.0 * kb.W * 8;
  const size_t lds = (size_t)kb.W * 8;
  if (lds <= kb.lds_per_block) {
    uint32_t bpt = std::max<uint32_t>(1, (2 * kb.n_cu + n - 1) / n);
    bpt = std::min<uint32_t>(bpt, (kb.W + 15) / 16);
    return L.run(HTH_K_ROLE, bytes, [&] {
      hipLaunchKernelGGL(k_role<true>, dim3(bpt * n), dim3(1024), lds, L.st, d, tasks, bpt);
    });
  }
  uint32_t bpt = std::max<uint32_t>(1, (8 * kb.n_cu + n - 1) / n);
  bpt = std::min<uint32_t>(bpt, (kb.W + 3) / 4);
  return L.run(HTH_K_ROLE, bytes, [&] {
    hipLaunchKernelGGL(k_role<false>, dim3(bpt * n), dim3(256), 0, L.st, d, tasks, bpt);
  });
}

template <typename TW>
hth_status launch_group_chunk(Launcher& L, const DevKB& d, const GroupTask* groups,
                              const GroupMember* members, const std::vector<GroupTask>& host,
                              size_t g0, uint32_t n, void* tarea) {
  const hth_kb_s& kb = L.kb;
  const uint64_t t_stride = align_up(kb.N, 64);
  double tb = 0, gb = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const GroupTask& G = host[g0 + i];
    tb += (double)G.k * kb.W * 8 + (double)t_stride * sizeof(TW);     // child rows in, T out
    gb += csr_bytes(kb, G.role, G.inv) + (double)t_stride * sizeof(TW) + (double)G.k * kb.W * 8;
  }
  TW* T = static_cast<TW*>(tarea);
  const uint32_t tiles = (kb.W + 255) / 256;
  hth_status s = L.run(HTH_K_TBUILD, tb, [&] {
    hipLaunchKernelGGL(k_tbuild<TW>, dim3(tiles * n), dim3(256), 0, L.st, d, groups + g0, members,
                       T, t_stride, tiles);
  });
  if (s) return s;
  const uint32_t xcd = kb.tune.xcd_local && n >= 8;
  uint32_t bpg, nblocks;
  if (xcd) {
    bpg = std::min<uint32_t>(std::max<uint32_t>(1, kb.n_cu / 8 * 8), (kb.W + 3) / 4);
    nblocks = 8 * bpg * ((n + 7) / 8);
  } else {
    bpg = std::max<uint32_t>(1, (8 * kb.n_cu + n - 1) / n);
    bpg = std::min<uint32_t>(bpg, (kb.W + 3) / 4);
    nblocks = bpg * n;
  }
  return L.run(HTH_K_GROUP, gb, [&] {
    const dim3 grid(nblocks), block(256);
    if (kb.tune.group_unroll >= 16) {
      if (kb.tune.nontemporal)
        hipLaunchKernelGGL((k_group<TW, 16, true>), grid, block, 0, L.st, d, groups + g0, members, T,
                           t_stride, bpg, n, xcd);
      else
        hipLaunchKernelGGL((k_group<TW, 16, false>), grid, block, 0, L.st, d, groups + g0, members, T,
                           t_stride, bpg, n, xcd);
    } else {
      if (kb.tune.nontemporal)
        hipLaunchKernelGGL((k_group<TW, 8, true>), grid, block, 0, L.st, d, groups + g0, members, T,
                           t_stride, bpg, n, xcd);
      else
        hipLaunchKernelGGL((k_group<TW, 8, false>), grid, block, 0, L.st, d, groups + g0, members, T,
                           t_stride, bpg, n, xcd);
    }
  });
}

hth_status launch_groups(Launcher& L, const DevKB& d, const GroupTask* groups,
                         const GroupMember* members, const std::vector<GroupTask>& host,
                         void* tarea) {
  const size_t t_stride = align_up(L.kb.N, 64);
  size_t i = 0;
  while (i < host.size()) {
    uint32_t wb = 1;
    size_t j = i;
    while (j < host.size()) {
      const uint32_t nwb = std::max(wb, t_width_bytes(host[j].k));
      if (j > i && (j - i + 1) * t_stride * nwb > L.kb.tune.t_budget) break;
      wb = nwb;
      ++j;
    }
    const uint32_t n = (uint32_t)(j - i);
    hth_status s;
    switch (wb) {
      case 1: s = launch_group_chunk<uint8_t>(L, d, groups, members, host, i, n, tarea); break;
      case 2: s = launch_group_chunk<uint16_t>(L, d, groups, members, host, i, n, tarea); break;
      case 4: s = launch_group_chunk<uint32_t>(L, d, groups, members, host, i, n, tarea); break;
      default: s = launch_group_chunk<uint64_t>(L, d, groups, members, host, i, n, tarea); break;
    }
    if (s) return s;
    i = j;
  }
  return HTH_OK;
}

// bytes of the packed tables plus slots plus T area for a plan
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
  add(n_reg, sizeof(RegionTask));
  add(n_role, sizeof(RoleTask));
  add(n_grp, sizeof(GroupTask));
  add(n_mem, sizeof(GroupMember));
  add(n_fill, sizeof(FillTask));
  add(P.code.size(), sizeof(uint32_t));
  return align_up(tables, 256) + (size_t)P.n_slots * kb.S * 8 + (max_groups ? t_area_bytes(kb) : 0);
}

std::once_flag g_attr_once;

hth_status run_plan(hth_kb_s& kb, const Plan& P, char* ws, size_t ws_bytes, uint32_t* counts,
                    uint32_t n_hyps, uint64_t* instances, hipStream_t st) {
  std::call_once(g_attr_once, [&] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_role<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kb.lds_per_block);
  });
  std::vector<RegionTask> regions;
  std::vector<RoleTask> roles;
  std::vector<GroupTask> groups;
  std::vector<GroupMember> members;
  std::vector<FillTask> fills;
  struct LevelAt { size_t mat, role, group, fill, nrole, ngroup, nfill; };
  std::vector<LevelAt> at(P.levels.size());
  std::vector<std::vector<RoleTask>> lv_roles(P.levels.size());
  std::vector<std::vector<GroupTask>> lv_groups(P.levels.size());
  for (size_t L = 0; L < P.levels.size(); ++L) {
    const PlanLevel& PL = P.levels[L];
    at[L] = {regions.size(), roles.size(), groups.size(), fills.size(), 0, 0, 0};
    regions.insert(regions.end(), PL.mat.begin(), PL.mat.end());
    for (RoleTask t : PL.roles) {
      t.n_words = kb.n_words[2 * t.role + t.inv];
      if (t.n_words < kb.W) fills.push_back(FillTask{t.out_row, t.lo == 0 ? 1u : 0u});
      roles.push_back(t);
      lv_roles[L].push_back(t);
    }
    const uint32_t mbase = (uint32_t)members.size();
    for (GroupTask g : PL.groups) {
      g.n_words = kb.n_words[2 * g.role + g.inv];
      if (g.n_words < kb.W)
        for (uint32_t j = 0; j < g.k; ++j)
          fills.push_back(FillTask{PL.members[g.first + j].out_row, (uint32_t)((g.acc[0] >> j) & 1)});
      g.first += mbase;
      groups.push_back(g);
      lv_groups[L].push_back(g);
    }
    members.insert(members.end(), PL.members.begin(), PL.members.end());
    at[L].nrole = roles.size() - at[L].role;
    at[L].ngroup = groups.size() - at[L].group;
    at[L].nfill = fills.size() - at[L].fill;
  }
  const size_t root_at = regions.size();
  regions.insert(regions.end(), P.roots.begin(), P.roots.end());
  Blob blob;
  const size_t o_thr = blob.add(P.thr);
  const size_t o_reg = blob.add(regions);
  const size_t o_role = blob.add(roles);
  const size_t o_grp = blob.add(groups);
  const size_t o_mem = blob.add(members);
  const size_t o_fill = blob.add(fills);
  const size_t o_code = blob.add(P.code);
  const size_t tables = align_up(blob.bytes.size(), 256);
  const size_t slot_bytes = (size_t)kb.S * 8;
  size_t max_groups = 0;
  for (const PlanLevel& PL : P.levels) max_groups = std::max(max_groups, PL.groups.size());
  const size_t t_bytes = max_groups ? t_area_bytes(kb) : 0;
  const size_t need = tables + (size_t)P.n_slots * slot_bytes + t_bytes;
  if (need > ws_bytes)
    return fail(HTH_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes, have " +
                                 std::to_string(ws_bytes));
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(HTH_E_INVALID, "workspace must be 256-byte aligned");

  DevKB d = dev_view(kb);
  d.slots = reinterpret_cast<uint64_t*>(ws + tables);
  d.counts = counts;
  d.instances = instances;
  void* tarea = ws + tables + (size_t)P.n_slots * slot_bytes;
  HTH_HIP(hipMemcpyAsync(ws, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice, st));
  HTH_HIP(hipMemsetAsync(counts, 0, (size_t)n_hyps * 8, st));
  const ThrTask* thr = reinterpret_cast<const ThrTask*>(ws + o_thr);
  const RegionTask* reg = reinterpret_cast<const RegionTask*>(ws + o_reg);
  const RoleTask* rol = reinterpret_cast<const RoleTask*>(ws + o_role);
  const GroupTask* grp = reinterpret_cast<const GroupTask*>(ws + o_grp);
  const GroupMember* mem = reinterpret_cast<const GroupMember*>(ws + o_mem);
  const FillTask* fil = reinterpret_cast<const FillTask*>(ws + o_fill);
  const uint32_t* code = reinterpret_cast<const uint32_t*>(ws + o_code);
  Launcher Lc{kb, st};
  if (!P.thr.empty()) {
    const uint32_t n = (uint32_t)P.thr.size();
    uint32_t bpt = std::max<uint32_t>(1, (4 * kb.n_cu + n - 1) / n);
    bpt = std::min<uint32_t>(bpt, (kb.W + 3) / 4);
    const double bytes = n * (4.0 * kb.N + 8.0 * kb.W);
    hth_status s = Lc.run(HTH_K_THRESHOLD, bytes, [&] {
      hipLaunchKernelGGL(k_threshold, dim3(bpt * n), dim3(256), 0, st, d, thr, bpt);
    });
    if (s) return s;
  }
  for (size_t L = 0; L < P.levels.size(); ++L) {
    const PlanLevel& PL = P.levels[L];
    hth_status s = launch_regions(Lc, d, reg + at[L].mat, code, PL.mat, P.code);
    if (s) return s;
    if (at[L].nfill) {
      const uint32_t n = (uint32_t)at[L].nfill, tiles = (kb.S + 255) / 256;
      s = Lc.run(HTH_K_FILL, (double)n * kb.W * 8, [&] {
        hipLaunchKernelGGL(k_fill_rows, dim3(tiles * n), dim3(256), 0, st, d, fil + at[L].fill, tiles);
      });
      if (s) return s;
    }
    s = launch_roles(Lc, d, rol + at[L].role, lv_roles[L]);
    if (s) return s;
    s = launch_groups(Lc, d, grp + at[L].group, mem, lv_groups[L], tarea);
    if (s) return s;
  }
  return launch_regions(Lc, d, reg + root_at, code, P.roots, P.code);
}

}  // namespace
}  // namespace hth

using namespace hth;

extern "C" hth_status hth_workspace_bytes(hth_kb kb, uint32_t max_nodes, uint32_t max_hyps,
                                          size_t* bytes) {
  if (!kb || !bytes) return fail(HTH_E_INVALID, "NULL argument");
  if (max_hyps == 0 || max_nodes < max_hyps) return fail(HTH_E_RANGE, "need max_nodes >= max_hyps >= 1");
  *bytes = align_up(table_bound(max_nodes, max_hyps), 256) + (size_t)(max_nodes + 2) * kb->S * 8 +
           t_area_bytes(*kb);
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
  return run_plan(*kb, P, static_cast<char*>(ws), ws_bytes, d_counts, 1, d_instances,
                  static_cast<hipStream_t>(stream));
}

extern "C" hth_status hth_eval_batch(hth_kb kb, const hth_node* nodes, const uint32_t* hyp_node_offsets,
                                     uint32_t n_hyps, const uint32_t* children, uint32_t n_children,
                                     void* ws, size_t ws_bytes, uint32_t* d_counts, void* stream) {
  if (!kb || !nodes || !hyp_node_offsets || !ws || !d_counts)
    return fail(HTH_E_INVALID, "NULL argument");
  if (n_children && !children) return fail(HTH_E_INVALID, "children is NULL");
  if (n_hyps == 0) return HTH_OK;
  if (hyp_node_offsets[0] != 0) return fail(HTH_E_INVALID, "hyp_node_offsets[0] must be 0");
  PlanOptions opt;
  opt.group_min = kb->tune.group_min ? kb->tune.group_min : 0xFFFFFFFFu;
  opt.group_k = kb->tune.group_k;
  Plan P;
  hth_status s = compile_plan(*kb, nodes, hyp_node_offsets, n_hyps, children, n_children, opt, P);
  if (s) return s;
  std::lock_guard<std::mutex> g(kb->mu);
  return run_plan(*kb, P, static_cast<char*>(ws), ws_bytes, d_counts, n_hyps, nullptr,
                  static_cast<hipStream_t>(stream));
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
