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

// T_g[y] bit j = bit(child_j, y) ^ neg_j for the groups of one launch; one lane
// per 64-individual word, transposed in registers.  T rows are TW wide
// (8 * sizeof(TW) >= every group's k).  A compact group keeps the rows of its
// direction's objects only, at their ranks; words without objects are skipped.
template <typename TW>
__global__ void __launch_bounds__(256)
k_tbuild(DevKB kb, const GroupTask* __restrict__ groups, const GroupMember* __restrict__ members,
         TW* __restrict__ tarea, uint32_t tiles) {
  constexpr int KB = 8 * sizeof(TW);
  const uint32_t g = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const GroupTask G = groups[g];
  const uint32_t w = tile * 256 + threadIdx.x;
  if (w >= kb.W) return;
  const uint32_t rd = 2 * G.role + G.inv;
  const uint64_t omask = G.compact ? kb.objmask[(size_t)rd * kb.W + w] : ~0ull;
  if (!omask) return;
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
  TW* T = tarea + G.t_off;
  if (!G.compact) {
    T += (size_t)w * 64;
#pragma unroll
    for (int b = 0; b < 64; ++b) T[b] = (TW)a[b];
  } else {
    T += kb.objbase[(size_t)rd * (kb.W + 1) + w];
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
        const TW* __restrict__ tarea, uint32_t bpg, uint32_t n_groups,
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
  const TW* T = tarea + G->t_off;
  const size_t roff = (size_t)G->role * (kb.N + 1);
  const uint32_t* off = (G->inv ? kb.inv_off : kb.fwd_off) + roff;
  // a compact group reads each assertion's object rank instead of its object
  const int32_t* tg = (G->compact ? (G->inv ? kb.ctg_inv : kb.ctg_fwd) : (G->inv ? kb.inv_tg : kb.fwd_tg)) +
                      kb.role_base[G->role];
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

}  // namespace hth
