// Shared role passes: the transposed child rows T and the counting pass over
// one CSR direction for up to 64 role nodes at once (Algorithms 3-8 evaluated
// for a whole group per assertion fetch).  Included by exec.hip only.
#pragma once

#include "hth_internal.h"

namespace hth {

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

// Word `byte_off / 8` of a row whose address every lane holds: the address
// goes to scalar registers and the load takes the lane's 32-bit byte offset.
__device__ __forceinline__ uint64_t uniform_row_word(const uint64_t* row, uint32_t byte_off) {
  typedef const char __attribute__((address_space(1)))* GlobalBytes;
  const uint64_t v = reinterpret_cast<uint64_t>(row);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  const GlobalBytes base = (GlobalBytes)(((uint64_t)hi << 32) | lo);
  return *(const uint64_t __attribute__((address_space(1)))*)(base + byte_off);
}

// A 32-bit word that every lane reads at the same address, through the
// scalar cache: its wait does not also wait for the wave's vector stores.
__device__ __forceinline__ uint32_t scalar_u32(const uint32_t* p) {
  return *(const __attribute__((address_space(4))) uint32_t*)p;
}
__device__ __forceinline__ uint64_t scalar_u64(const uint64_t* p) {
  return *(const __attribute__((address_space(4))) uint64_t*)p;
}

// T_g[y] bit j = bit(child_j, y) ^ neg_j for the groups of one launch; one lane
// per 64-individual word, transposed in registers.  T rows are TW wide
// (8 * sizeof(TW) >= every group's k).  A compact group keeps the rows of its
// direction's objects only, at their ranks, and its lanes take the words that
// hold objects (a list), not every word.
// The members' row addresses are resolved once per block into LDS, so that a
// lane issues all of its member loads before it waits for any of them; slots
// beyond k read member 0's row again and drop it.
constexpr int kTStage = 1024;   // T rows a wave stages in LDS
template <typename TW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_tbuild(DevKB kb, const GroupTask* __restrict__ groups, const GroupMember* __restrict__ members,
         TW* __restrict__ tarea, uint32_t tiles) {
  constexpr int KB = 8 * sizeof(TW);
  __shared__ const uint64_t* s_row[KB];
  __shared__ uint64_t s_flip[KB];
  __shared__ TW s_t[4][kTStage];   // each wave's compact T rows before they go out as one run
  const uint32_t g = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const GroupTask G = groups[g];
  if (threadIdx.x < (uint32_t)KB) {
    const uint32_t j = threadIdx.x, m = j < G.k ? j : 0u;   // every group has a member 0
    const GroupMember M = members[G.first + m];
    s_row[j] = row_ptr(kb, M.child_row);
    s_flip[j] = M.neg ? ~0ull : 0ull;
  }
  __syncthreads();
  const uint32_t rd = 2 * G.role + G.inv;
  TW* T = tarea + G.t_off;
  // the words of lane's 64 individuals from every member's child row, flipped
  // where the member counts the complement, transposed into T rows
  auto build = [&](uint32_t w, uint64_t (&a)[64]) {
#pragma unroll
    for (int j = 0; j < KB; ++j) a[j] = uniform_row_word(s_row[j], w * 8u);
#pragma unroll
    for (int j = 0; j < 64; ++j) a[j] = j < KB && (j == 0 || (uint32_t)j < G.k) ? a[j] ^ s_flip[j] : 0ull;
    transpose64(a);
  };
  if (!G.compact) {
    const uint32_t w = tile * 256 + threadIdx.x;
    if (w >= kb.W) return;
    uint64_t a[64];
    build(w, a);
    T += (size_t)w * 64;
#pragma unroll
    for (int b = 0; b < 64; ++b) T[b] = (TW)a[b];
    return;
  }
  // a compact group visits only the words that hold objects of its direction
  // (the other direction's non-empty words, in its word list).  A wave's
  // objects have consecutive ranks, so their rows are gathered in LDS and
  // written as one run (a wave with more rows than the stage stores directly).
  const uint32_t i = tile * 256 + threadIdx.x;
  const bool valid = i < G.n_obj_words;
  const uint32_t w = valid ? kb.words[(size_t)(rd ^ 1u) * kb.W + i] : 0u;
  const uint64_t omask = valid ? kb.objmask[(size_t)rd * kb.W + w] : 0ull;
  const uint64_t act = __ballot(omask != 0ull);
  if (!act) return;
  const uint32_t r0 = omask ? kb.objbase[(size_t)rd * (kb.W + 1) + w] : 0u;
  uint64_t a[64];
  if (omask) build(w, a);
  const int first = __ffsll((unsigned long long)act) - 1, last = 63 - __clzll(act);
  const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)r0, first);
  const uint32_t end = (uint32_t)__builtin_amdgcn_readlane((int)(r0 + (uint32_t)__popcll(omask)), last);
  const uint32_t cnt = end - base;
  if (cnt <= (uint32_t)kTStage) {
    TW* st = s_t[threadIdx.x >> 6];
    if (omask) {
#pragma unroll
      for (int b = 0; b < 64; ++b)
        if ((omask >> b) & 1ull) st[r0 - base + __popcll(omask & ((1ull << b) - 1ull))] = (TW)a[b];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t j = threadIdx.x & 63; j < cnt; j += 64) T[base + j] = st[j];
  } else if (omask) {
    T += r0;
#pragma unroll
    for (int b = 0; b < 64; ++b)
      if ((omask >> b) & 1ull) T[__popcll(omask & ((1ull << b) - 1ull))] = (TW)a[b];
  }
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

// Lane exchange with the partner lane ^ D, for a compile-time D: quad
// permutations through DPP for 1 and 2, swizzles within 32 lanes for 4 to 16,
// a permute across the halves for 32.  Every lane of the wave takes part.
template <int D>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  if constexpr (D == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
  else if constexpr (D == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
  else if constexpr (D < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (D << 10));
  else return (uint32_t)__shfl_xor((int)v, D, 64);
}

// One butterfly stage of the lane transpose below, on both 32-bit halves: the
// lane whose bit D is clear keeps the bits of the D-blocks selected by M and
// takes the partner's such blocks into the other blocks; its partner keeps the
// other blocks and takes this lane's remaining blocks.  Each lane rotates what
// it gives away into the position where the partner needs it (right by D, or
// left by D), so one rotate, one exchange and one bit insert per half suffice.
template <int D, uint32_t M>
__device__ __forceinline__ void transpose_stage(uint32_t& lo, uint32_t& hi, int lane) {
  const bool up = lane & D;
  const uint32_t sh = up ? 32u - D : (uint32_t)D, keep = up ? ~M : M;
  const uint32_t rl = lane_xor<D>(__builtin_amdgcn_alignbit(lo, lo, sh));
  const uint32_t rh = lane_xor<D>(__builtin_amdgcn_alignbit(hi, hi, sh));
  lo = (keep & lo) | (~keep & rl);
  hi = (keep & hi) | (~keep & rh);
}

// 64 x 64 bit transpose across the lanes of a wave: on entry lane l holds row
// l (bit j = M[l][j]); on exit lane l holds column l (bit j = M[j][l]).  Six
// butterfly stages (block sizes 32, 16, ..., 1), each exchanging off-diagonal
// blocks with the partner lane.  Called with every lane of the wave active.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x, int lane) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  // the stages' per-lane shift counts and masks are derived from the lane here
  // rather than kept live across the caller's loop (they would cost registers
  // the caller needs for occupancy)
  asm volatile("" : "+v"(lane));
  {   // 32-bit blocks: the lower half of the wave trades its high words for
      // the upper half's low words
    const bool up = lane & 32;
    const uint32_t r = lane_xor<32>(up ? lo : hi);
    lo = up ? r : lo;
    hi = up ? hi : r;
  }
  transpose_stage<16, 0x0000FFFFu>(lo, hi, lane);
  transpose_stage<8, 0x00FF00FFu>(lo, hi, lane);
  transpose_stage<4, 0x0F0F0F0Fu>(lo, hi, lane);
  transpose_stage<2, 0x33333333u>(lo, hi, lane);
  transpose_stage<1, 0x55555555u>(lo, hi, lane);
  return ((uint64_t)hi << 32) | lo;
}

// Lane l's value, in every lane (l the same in all of them).
template <typename TW>
__device__ __forceinline__ uint64_t read_lane(TW v, int l) {
  if constexpr (sizeof(TW) == 8) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
  } else {
    return (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  }
}

// The members' acceptance of a count held in bit-sliced planes: bit j of the
// result = member j accepts the count of its bit j.
// A select tree over the planes: c0 picks within each pair of counts, c1
// between pairs, c2 between halves, ov the count >= 8.  The first level
// takes acc[2i] ^ (c0 & (acc[2i] ^ acc[2i + 1])), so that no instruction
// needs two of the (uniform) acceptance words at once.
// SAT = false: the count is below 8 (ov is not read).
template <typename TW, bool SAT = true>
__device__ __forceinline__ TW accept(const Planes<TW>& p, const TW (&acc)[kGroupMaxCount + 1]) {
  auto pick = [](TW m, TW a, TW b) { return (m & a) | (~m & b); };   // a where m, else b
  const TW p0 = acc[0] ^ (p.c0 & (acc[0] ^ acc[1])), p1 = acc[2] ^ (p.c0 & (acc[2] ^ acc[3]));
  const TW p2 = acc[4] ^ (p.c0 & (acc[4] ^ acc[5])), p3 = acc[6] ^ (p.c0 & (acc[6] ^ acc[7]));
  const TW q = pick(p.c2, pick(p.c1, p3, p2), pick(p.c1, p1, p0));
  if constexpr (SAT) return pick(p.ov, acc[8], q);
  else return q;
}

// Coverage of a member without an output row (GroupMember::cover): lane j
// keeps member j's counts of covered positives and negatives.  A member that
// accepts the zero count (z) also holds every individual of the words its
// direction lists no assertion for, and those words are never visited: each
// wave therefore adds z * popcount(P) over its share of all words and takes
// z * popcount(P) off again for every word it visits (counts wrap modulo 2^32
// in between; the total is exact).
struct Cover {
  uint32_t h;          // hypothesis, or kNone
  bool z;              // the member accepts the zero count
  uint32_t p, q;
};
__device__ __forceinline__ Cover cover_of(const GroupTask* G, const GroupMember* members, uint32_t k, int lane) {
  Cover c{kNone, false, 0u, 0u};
  if ((uint32_t)lane < k) {
    c.h = members[G->first + lane].cover;
    c.z = (G->acc[0] >> lane) & 1ull;
  }
  return c;
}
__device__ __forceinline__ void cover_word(Cover& c, const DevKB& kb, uint32_t w, uint64_t v) {
  w = __builtin_amdgcn_readfirstlane(w);   // the same word on every lane: scalar loads
  const uint64_t P = scalar_u64(kb.pos + w), N = scalar_u64(kb.neg + w);
  c.p += (uint32_t)__popcll(v & P) - (c.z ? (uint32_t)__popcll(P) : 0u);
  c.q += (uint32_t)__popcll(v & N) - (c.z ? (uint32_t)__popcll(N) : 0u);
}
// wave `wave` of `waves`: its share of all words, then the member's atomics
__device__ __forceinline__ void cover_finish(Cover& c, const DevKB& kb, uint32_t wave, uint32_t waves, int lane) {
  if (__ballot(c.h != kNone && c.z)) {
    for (uint32_t w0 = wave * 64; w0 < kb.W; w0 += waves * 64) {
      const uint32_t w = w0 + lane;
      uint32_t pp = w < kb.W ? (uint32_t)__popcll(kb.pos[w]) : 0u;
      uint32_t qq = w < kb.W ? (uint32_t)__popcll(kb.neg[w]) : 0u;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        pp += __shfl_xor(pp, d, 64);
        qq += __shfl_xor(qq, d, 64);
      }
      if (c.h != kNone && c.z) {
        c.p += pp;
        c.q += qq;
      }
    }
  }
  if (c.h != kNone) {
    if (c.p) atomicAdd(kb.counts + 2 * c.h, c.p);
    if (c.q) atomicAdd(kb.counts + 2 * c.h + 1, c.q);
  }
}

// A shared pass cut by T row ("target segments"), so that the T rows one pass
// fetches fit an XCD's L2: pass s counts only the assertions whose T row is in
// [lo, hi).  Every pass walks the same rows; the counts of a row finished in
// an earlier pass come in through `part` (bit-sliced planes per subject, for
// the group at index g of the launch at part + g * stride: W words x 4 planes
// x 64 subjects) and go out to it for the next pass; the last pass writes the
// members' output words.  One pass: lo = 0, hi = ~0, first = last = 1.
template <typename TW>
struct SegPass {
  uint32_t lo, hi;
  uint32_t first, last;
  TW* part;
  size_t stride;   // TW elements per group
};

// One wave per MW consecutive entries of the direction's non-empty word list
// (64 MW subjects: one word of every member's output row per entry), all
// members of the group at once.  Words between two list entries hold no
// assertions, so the entries' assertions are one contiguous range; it is cut
// into 64 contiguous slices of ceil(E / 64), one per lane (balanced whatever
// the degrees).  A lane walks its slice, fetches each object's T row (one load
// serves every member) and adds it into bit-sliced counters; a row complete in
// the slice has its acceptance written to LDS at once.  Rows that straddle
// slices leave a tail partial in each lane they cross; one segmented scan over
// the lanes adds them up for the lane holding the row's last assertion.  Only
// non-empty rows are walked: they are packed by a ballot, so that a lane steps
// from one row to the next in one LDS read however many empty subjects lie
// between.  A finished row's counters go to LDS (a few stores, so that lanes
// crossing a row boundary at different steps stay cheap); afterwards every lane turns
// its own subject's counters into the members' predicates at once, and each
// word's predicates are transposed by a wave butterfly into one word per
// member (a word with at most kSparseWord non-empty rows instead starts from
// the zero count's predicates and takes the others' bits lane by lane).  MW > 1 serves directions with few assertions per word.
constexpr int kSparseWord = 4;   // words with at most this many non-empty rows skip the transpose
template <typename TW, int U, int MW>   // U: assertions in flight per lane
__global__ void __launch_bounds__(256)
k_group(DevKB kb, const GroupTask* __restrict__ groups, const GroupMember* __restrict__ members,
        const TW* __restrict__ tarea, uint32_t bpg, const uint32_t* __restrict__ xslots, SegPass<TW> sp) {
  constexpr int R = 64 * MW;          // subjects per iteration
  __shared__ uint32_t s_ro[4][R + 1];
  __shared__ TW s_pl[4][4][R];        // counters of the rows finished in this iteration
  uint32_t g, b;
  if (xslots) {
    // workgroups are dealt to the 8 XCDs round robin: keep every block of a
    // group on one XCD so that its L2 serves that group's T rows.  xslots
    // lists each XCD's groups round by round (balanced on the host).
    const uint32_t x = blockIdx.x & 7, j = blockIdx.x >> 3;
    g = xslots[(j / bpg) * 8 + x];
    b = j % bpg;
    if (g == kNone) return;
  } else {
    g = blockIdx.x / bpg;
    b = blockIdx.x % bpg;
  }
  const GroupTask* G = groups + g;
  const uint32_t k = G->k;
  TW* part = sp.first && sp.last ? nullptr : sp.part + (size_t)g * sp.stride;
  const TW* T = tarea + G->t_off;
  const size_t roff = (size_t)G->role * (kb.N + 1);
  const uint32_t* off = (G->inv ? kb.inv_off : kb.fwd_off) + roff;
  const uint32_t off_end = off[kb.N];
  // a compact group reads each assertion's object rank instead of its object
  const int32_t* tg = (G->compact ? (G->inv ? kb.ctg_inv : kb.ctg_fwd) : (G->inv ? kb.inv_tg : kb.fwd_tg)) +
                      kb.role_base[G->role];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* ro = s_ro[wv];
  TW (*pl)[R] = s_pl[wv];
  TW acc[kGroupMaxCount + 1];
#pragma unroll
  for (int v = 0; v <= (int)kGroupMaxCount; ++v) acc[v] = (TW)G->acc[v];
  const uint32_t seg_n = sp.hi - sp.lo;
  const uint32_t my_row = (uint32_t)lane < k ? members[G->first + lane].out_row : kNone;
  uint64_t* const my_out = my_row != kNone ? out_ptr(kb, my_row) : nullptr;
  __shared__ uint64_t* s_dst[64];     // every member's output row
  if (threadIdx.x < 64) s_dst[threadIdx.x] = my_out;
  __syncthreads();
  Cover cv = cover_of(G, members, k, lane);
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t istep = bpg * nw;
  const uint32_t* words = kb.words + (size_t)(2 * G->role + G->inv) * kb.W;
  const uint32_t n_words = G->n_words;
  const uint32_t n_iter = (n_words + MW - 1) / MW;

  // Software pipeline over the wave's iterations: while iteration i is walked,
  // the row offsets of i + 2 and the slice targets of i + 1 are in flight, and
  // the T rows of i + 1 are fetched before i's counters are turned into
  // predicates.  A slice longer than U fetches its further blocks in place.
  struct Rows {
    uint32_t lo[MW], hi[MW], wd[MW];
  };
  // loads without branches around them (clamped indices, results masked
  // after), so that a wave has all of an iteration's loads in flight at once
  auto fetch = [&](uint32_t it, Rows& q) {
    uint32_t w[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) w[m] = scalar_u32(words + min(it * MW + m, n_words - 1));
#pragma unroll
    for (int m = 0; m < MW; ++m) {
      const bool in = it < n_iter && it * MW + m < n_words;
      const uint32_t x = w[m] * 64 + lane, xc = min(x, kb.N - 1);
      const uint32_t lo = off[xc], hi = off[xc + 1];
      q.wd[m] = in ? w[m] : kNone;   // lo and hi of an entry past the list are never read
      q.lo[m] = x < kb.N ? lo : off_end;
      q.hi[m] = x < kb.N ? hi : off_end;
    }
  };
  auto words_in = [&](uint32_t it) { return it < n_iter ? min((uint32_t)MW, n_words - it * MW) : 0u; };
  // the lane's slice [s, se) of the iteration's contiguous assertion range
  auto slice = [&](const Rows& q, uint32_t it, uint32_t& s, uint32_t& se) {
    const uint32_t mc = words_in(it);
    uint32_t hl = q.hi[0];
#pragma unroll
    for (int m = 1; m < MW; ++m)
      if ((uint32_t)m < mc) hl = q.hi[m];
    const uint32_t E0 = (uint32_t)__shfl((int)q.lo[0], 0, 64), E1 = (uint32_t)__shfl((int)hl, 63, 64);
    const uint32_t S = (E1 - E0 + 63) >> 6;
    s = mc ? E0 + lane * S : 0;
    se = mc ? min(s + S, E1) : 0;
    if (se < s) se = s;
  };
  auto load_t = [&](uint32_t e0, uint32_t se, int32_t (&t)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = (e0 + u < se) ? tg[e0 + u] : 0;
  };
  auto gather = [&](uint32_t e0, uint32_t se, const int32_t (&t)[U], TW (&v)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = (e0 + u < se && (uint32_t)t[u] - sp.lo < seg_n) ? T[(uint32_t)t[u]] : (TW)0;
  };

  uint32_t it = b * nw + wv;
  Rows rw, rn;
  fetch(it, rw);
  fetch(it + istep, rn);
  uint32_t s, se;
  slice(rw, it, s, se);
  int32_t t[U];
  TW v[U];
  load_t(s, se, t);
  gather(s, se, t, v);
  for (; it < n_iter; it += istep) {
    const uint32_t mc = words_in(it);
    // the iteration's non-empty rows in subject order, by compact index: row i
    // holds assertions [ro[i], ro[i + 1]).  Empty rows are never walked; their
    // subjects take the zero count.
    uint64_t nzm[MW];
    uint32_t nzb[MW], nnz = 0;
#pragma unroll
    for (int m = 0; m < MW; ++m) {
      nzm[m] = (uint32_t)m < mc ? __ballot(rw.lo[m] < rw.hi[m]) : 0ull;
      nzb[m] = nnz;
      nnz += __popcll(nzm[m]);
    }
    auto compact = [&](int m) {   // the compact index of this lane's subject of word m
      return nzb[m] + __builtin_amdgcn_mbcnt_hi((uint32_t)(nzm[m] >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)nzm[m], 0u));
    };
#pragma unroll
    for (int m = 0; m < MW; ++m)
      if ((nzm[m] >> lane) & 1ull) ro[compact(m)] = rw.lo[m];
    {
      uint32_t hl = rw.hi[0];
#pragma unroll
      for (int m = 1; m < MW; ++m)
        if ((uint32_t)m < mc) hl = rw.hi[m];
      if (lane == 63) ro[nnz] = hl;
    }
    // the pipeline's next stages: offsets of it + 2 istep, targets of it + istep
    Rows rnn;
    fetch(it + 2 * istep, rnn);
    uint32_t ns, nse;
    slice(rn, it + istep, ns, nse);
    int32_t nt[U];
    load_t(ns, nse, nt);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // a row's count is complete in this slice walk
    auto finish = [&](int r, const Planes<TW>& p) {
      pl[0][r] = p.c0;
      pl[1][r] = p.c1;
      pl[2][r] = p.c2;
      pl[3][r] = p.ov;
    };
    Planes<TW> cur{0, 0, 0, 0}, hp{0, 0, 0, 0}, tp{0, 0, 0, 0};
    int hp_row = -1, key = -2 - lane;
    if (s < se) {
      // the row holding assertion s: the last r with ro[r] <= s
      int r = 0;
#pragma unroll
      for (int step = R / 2; step; step >>= 1)
        if (r + step < (int)nnz && ro[r + step] <= s) r += step;
      bool head = ro[r] < s;
      uint32_t rend = ro[r + 1];
      for (uint32_t e0 = s; e0 < se; e0 += U) {
        if (e0 != s) {                   // beyond the prefetched block
          load_t(e0, se, t);
          gather(e0, se, t, v);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t e = e0 + u;
          if (e < se) {
            while (e >= rend) {          // row r is complete in this slice
              if (head) {
                hp = cur;
                hp_row = r;
              } else {
                finish(r, cur);
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
        finish(r, cur);
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
        finish(hp_row, hp);
      }
    }
    // the next iteration's T rows, in flight while this one's words are written
    gather(ns, nse, nt, v);
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = nt[u];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // each word: lane l's subject 64 w + l.  Its counts go on to the next
    // pass of a cut shared pass, or become every member's predicate,
    // transposed into one output word per member.
    uint64_t mine_m[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) {
      mine_m[m] = 0;
      if ((uint32_t)m < mc) {
        Planes<TW> p{0, 0, 0, 0};
        if ((nzm[m] >> lane) & 1ull) {
          const int r = compact(m);
          p = Planes<TW>{pl[0][r], pl[1][r], pl[2][r], pl[3][r]};
        }
        if (part) {
          TW* q = part + (size_t)rw.wd[m] * 256 + lane;
          if (!sp.first) planes_add(p, Planes<TW>{q[0], q[64], q[128], q[192]});
          if (!sp.last) {
            q[0] = p.c0;
            q[64] = p.c1;
            q[128] = p.c2;
            q[192] = p.ov;
          }
        }
        if (sp.last) {
          TW rv = accept(p, acc);
          if (rw.wd[m] * 64 + lane >= kb.N) rv = 0;
          uint64_t mine;
          if (__popcll(nzm[m]) <= kSparseWord) {
            // the subjects without assertions take the zero count, so member
            // j's word is acc[0]'s bit j at each of them; the bits of the few
            // others are read from their lanes
            const uint32_t x0 = rw.wd[m] * 64;
            const uint64_t live = x0 + 64 <= kb.N ? ~0ull : ((1ull << (kb.N - x0)) - 1ull);
            mine = (((uint64_t)acc[0] >> lane) & 1ull) ? live : 0ull;
            for (uint64_t z = nzm[m]; z; z &= z - 1) {
              const int l = __builtin_ctzll(z);
              const uint64_t bit = (read_lane(rv, l) >> lane) & 1ull;
              mine = (mine & ~(1ull << l)) | (bit << l);
            }
          } else {
            mine = wave_transpose64((uint64_t)rv, lane);
          }
          mine_m[m] = mine;
          if (cv.h != kNone) cover_word(cv, kb, rw.wd[m], mine);
        }
      }
    }
    if (sp.last) {
      if constexpr (sizeof(TW) == 8 && MW > 1 && 64 % MW == 0) {
        // the members' words go out with MW consecutive lanes on one member's
        // row (64 / MW rows per store, not 64), through the counter planes'
        // LDS (read above, not needed again before the next walk)
        uint64_t* sw = reinterpret_cast<uint64_t*>(&pl[0][0]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int m = 0; m < MW; ++m) sw[lane * MW + m] = mine_m[m];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int m = lane % MW;
        uint32_t wm = rw.wd[0];
#pragma unroll
        for (int k = 1; k < MW; ++k)
          if (m == k) wm = rw.wd[k];
#pragma unroll
        for (int r = 0; r < MW; ++r) {
          const int j = r * (64 / MW) + lane / MW;   // member
          uint64_t* dst = s_dst[j];
          if (dst && (uint32_t)m < mc) dst[wm] = sw[j * MW + m];
        }
      } else if (my_out) {
#pragma unroll
        for (int m = 0; m < MW; ++m)
          if ((uint32_t)m < mc) my_out[rw.wd[m]] = mine_m[m];
      }
    }
    __builtin_amdgcn_wave_barrier();
    rw = rn;
    rn = rnn;
    s = ns;
    se = nse;
  }
  if (sp.last) cover_finish(cv, kb, b * nw + wv, bpg * nw, lane);
}

// A shared pass over a role direction whose rows are all short (at most the
// schedule's short_rows assertions): lane l of a wave owns subject 64 w + l of
// each of MW consecutive entries of the direction's word list and walks that
// subject's row alone, all MW rows in step.  A lane's counters are its own
// subject's, so the words' assertion ranges are not sliced and nothing is
// scanned across lanes.  The members' predicates are transposed into one word
// per member.  A wave takes SUB * MW consecutive entries as SUB such
// iterations and keeps the members' words in LDS; a member's SUB * MW
// consecutive, aligned words then go out as one segment of a 128-byte line,
// written by SUB * MW / 2 lanes with 16-byte stores (so that a store
// instruction touches 64 / (SUB * MW / 2) lines, not 64).  The staged words of
// a wave's previous entries go out after its next loads: a wait on a load also
// waits for every store issued before it.
constexpr int kShortWords = 4;   // MW
constexpr int kShortSub = 2;     // SUB
// EXACT: every row of the launch's directions holds at most 7 assertions, so
// c2 c1 c0 count exactly and the saturation plane stays empty (not kept).
template <typename TW, int MW, int SUB, bool EXACT>
__global__ void __launch_bounds__(256)
k_group_short(DevKB kb, const GroupTask* __restrict__ groups, const GroupMember* __restrict__ members,
              const TW* __restrict__ tarea, uint32_t bpg, const uint32_t* __restrict__ xslots) {
  constexpr int SW = SUB * MW;            // words per wave iteration
  constexpr int LPM = SW / 2;             // lanes per member line (16 bytes each)
  static_assert(SW * 8 <= 128 && 64 % LPM == 0, "a member's words of one iteration lie in one 128-byte line");
  __shared__ uint64_t s_out[4][64][SW + 1];   // + 1 word: rows fall on different banks
  __shared__ uint64_t* s_dst[64];
  uint32_t g, b;
  if (xslots) {
    const uint32_t x = blockIdx.x & 7, j = blockIdx.x >> 3;
    g = xslots[(j / bpg) * 8 + x];
    b = j % bpg;
    if (g == kNone) return;
  } else {
    g = blockIdx.x / bpg;
    b = blockIdx.x % bpg;
  }
  const GroupTask* G = groups + g;
  const uint32_t k = G->k;
  const TW* T = tarea + G->t_off;
  const uint32_t* off = (G->inv ? kb.inv_off : kb.fwd_off) + (size_t)G->role * (kb.N + 1);
  const int32_t* tg = (G->compact ? (G->inv ? kb.ctg_inv : kb.ctg_fwd) : (G->inv ? kb.inv_tg : kb.fwd_tg)) +
                      kb.role_base[G->role];
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  TW acc[kGroupMaxCount + 1];
#pragma unroll
  for (int v = 0; v <= (int)kGroupMaxCount; ++v) acc[v] = (TW)G->acc[v];
  const uint32_t my_row = (uint32_t)lane < k ? members[G->first + lane].out_row : kNone;
  uint64_t* const my_out = my_row != kNone ? out_ptr(kb, my_row) : nullptr;
  if (threadIdx.x < 64) s_dst[threadIdx.x] = my_out;
  __syncthreads();
  Cover cv = cover_of(G, members, k, lane);
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t* words = kb.words + (size_t)(2 * G->role + G->inv) * kb.W;
  const uint32_t n_words = G->n_words;
  const uint32_t n_super = (n_words + SW - 1) / SW;
  uint64_t (*so)[SW + 1] = s_out[wv];
  uint32_t pw[SW];   // words staged in LDS, not yet written
#pragma unroll
  for (int i = 0; i < SW; ++i) pw[i] = kNone;
  auto flush = [&]() {
    if (pw[0] == kNone) return;
    if (pw[SW - 1] != kNone && pw[SW - 1] - pw[0] == SW - 1 && pw[0] % SW == 0) {
      const int part = lane % LPM;
#pragma unroll
      for (int r = 0; r < LPM; ++r) {
        const int j = r * (64 / LPM) + lane / LPM;
        uint64_t* dst = s_dst[j];
        if (dst) {
          ulonglong2* q = reinterpret_cast<ulonglong2*>(dst + pw[0]) + part;
          *q = make_ulonglong2(so[j][2 * part], so[j][2 * part + 1]);
        }
      }
    } else if (my_out) {
#pragma unroll
      for (int i = 0; i < SW; ++i)
        if (pw[i] != kNone) my_out[pw[i]] = so[lane][i];
    }
  };
  for (uint32_t si = b * nw + wv; si < n_super; si += bpg * nw) {
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub) {
      const uint32_t it = si * SUB + sub;
      uint32_t wd[MW], e[MW], ee[MW];
#pragma unroll
      for (int m = 0; m < MW; ++m) wd[m] = scalar_u32(words + min(it * MW + m, n_words - 1));
#pragma unroll
      for (int m = 0; m < MW; ++m) {
        const uint32_t x = wd[m] * 64 + lane, xc = min(x, kb.N - 1);
        e[m] = off[xc];
        ee[m] = off[xc + 1];
        const bool in = it * MW + m < n_words && x < kb.N;
        if (!in) ee[m] = e[m];
        if (it * MW + m >= n_words) wd[m] = kNone;
      }
      Planes<TW> p[MW];
#pragma unroll
      for (int m = 0; m < MW; ++m) p[m] = Planes<TW>{0, 0, 0, 0};
      for (;;) {
        bool open = false;
#pragma unroll
        for (int m = 0; m < MW; ++m) open |= e[m] < ee[m];
        if (!__ballot(open)) break;
        int32_t t[MW];
#pragma unroll
        for (int m = 0; m < MW; ++m) t[m] = tg[e[m] < ee[m] ? e[m] : 0u];
        TW v[MW];
#pragma unroll
        for (int m = 0; m < MW; ++m) v[m] = T[e[m] < ee[m] ? (uint32_t)t[m] : 0u];
#pragma unroll
        for (int m = 0; m < MW; ++m) {
          const bool o = e[m] < ee[m];
          if constexpr (EXACT) {
            const TW w = o ? v[m] : (TW)0;
            const TW k0 = p[m].c0 & w;
            p[m].c0 ^= w;
            const TW k1 = p[m].c1 & k0;
            p[m].c1 ^= k0;
            p[m].c2 ^= k1;
          } else {
            planes_inc(p[m], o ? v[m] : (TW)0);
          }
          e[m] += o;
        }
      }
      if (sub == 0) {   // the previous entries' words, after this iteration's loads
        flush();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
#pragma unroll
      for (int m = 0; m < MW; ++m) {
        TW rv = accept<TW, !EXACT>(p[m], acc);
        if (wd[m] == kNone || wd[m] * 64 + lane >= kb.N) rv = 0;
        const uint64_t o = wave_transpose64((uint64_t)rv, lane);
        so[lane][sub * MW + m] = o;
        pw[sub * MW + m] = wd[m];
        if (cv.h != kNone && wd[m] != kNone) cover_word(cv, kb, wd[m], o);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  flush();
  cover_finish(cv, kb, b * nw + wv, bpg * nw, lane);
}

}  // namespace hth
