// Knowledge-base loading: validation on the device and the derived layouts
// (32-bit per-role row offsets in both directions and the inverse-role CSR).
//
// The paper keeps role assertions as (subject, object) rows grouped per role
// with an offset table (Section 3.1) and obtains inverse restrictions by
// swapping subjects and objects (end of Section 3.2.2).  Here the forward
// assertions arrive as a CSR per role and the inverse is its exact transpose,
// built once at load time so that both directions are scanned row-parallel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "kb_handle.h"

namespace hth {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
hth_status fail(hth_status code, const std::string& msg) {
  g_err = msg;
  return code;
}
hth_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return HTH_E_DEVICE;
}

enum : uint32_t {
  F_NONMONO = 1,   // offsets decrease or leave the role's range
  F_TARGET = 2,    // target outside [0, N)
  F_ORDER = 4,     // targets not strictly increasing inside a row
  F_PAD = 8,       // a padding bit is set
};

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr uint32_t kScanBlock = kScanThreads * kScanItems;

__global__ void k_gather_bases(const int64_t* __restrict__ off, uint32_t R, uint32_t N,
                               uint64_t* __restrict__ base) {
  uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) base[r] = (uint64_t)off[(size_t)r * (N + 1)];
  if (r == R - 1) base[R] = (uint64_t)off[(size_t)r * (N + 1) + N];
}

// One thread per (role, subject): check the row, write its relative offset,
// count its assertions per object into inv_off[r][y + 1].  Rows with more
// than hmin assertions (heavy rows) only get their offsets checked here; their
// assertions are checked and counted chunk by chunk by k_validate_heavy.
__global__ void k_validate_rows(const int64_t* __restrict__ off, const int32_t* __restrict__ tg,
                                const uint64_t* __restrict__ base, uint32_t N, uint32_t hmin,
                                uint32_t* __restrict__ fwd_off, uint32_t* __restrict__ inv_cnt,
                                uint32_t* __restrict__ maxdeg, uint32_t* __restrict__ flags) {
  uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t r = blockIdx.y;
  if (x >= N) return;
  const int64_t* o = off + (size_t)r * (N + 1);
  int64_t o0 = o[x], o1 = o[x + 1];
  int64_t b0 = (int64_t)base[r], b1 = (int64_t)base[r + 1];
  uint32_t* fo = fwd_off + (size_t)r * (N + 1);
  if (o0 < b0 || o1 < o0 || o1 > b1) {
    atomicOr(flags, F_NONMONO);
    return;
  }
  fo[x] = (uint32_t)(o0 - b0);
  if (x == N - 1) fo[N] = (uint32_t)(o1 - b0);
  atomicMax(maxdeg + r, (uint32_t)(o1 - o0));
  if (o1 - o0 > (int64_t)hmin) return;
  uint32_t* cnt = inv_cnt + (size_t)r * (N + 1);
  int32_t prev = -1;
  uint32_t bad = 0;
  for (int64_t e = o0; e < o1; ++e) {
    int32_t t = tg[e];
    if (t < 0 || (uint32_t)t >= N) {
      bad |= F_TARGET;
      continue;
    }
    if (t <= prev) bad |= F_ORDER;
    prev = t;
    atomicAdd(cnt + t + 1, 1u);
  }
  if (bad) atomicOr(flags, bad);
}

// Members of each row (one block per row): the plan's push/pull choice.
__global__ void __launch_bounds__(256)
k_row_pop(const uint64_t* __restrict__ rows, uint32_t W, uint32_t S, uint32_t* __restrict__ out) {
  __shared__ uint32_t part[4];
  const uint64_t* p = rows + (size_t)blockIdx.x * S;
  uint32_t c = 0;
  for (uint32_t w = threadIdx.x; w < W; w += 256) c += (uint32_t)__popcll(p[w]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Bits past N in word W-1 and words W..S-1 of every bit row must be zero.
__global__ void k_check_padding(const uint64_t* __restrict__ rows, uint32_t n_rows, uint32_t W,
                                uint32_t S, uint64_t tail, uint32_t* __restrict__ flags) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows) return;
  const uint64_t* p = rows + (size_t)i * S;
  uint64_t bad = p[W - 1] & ~tail;
  for (uint32_t w = W; w < S; ++w) bad |= p[w];
  if (bad) atomicOr(flags, F_PAD);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) p[i] = v;
}

__global__ void k_copy_u32(const uint32_t* __restrict__ s, uint32_t* __restrict__ d, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) d[i] = s[i];
}

// Inclusive wave scan of one value per lane.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread (blockDim = 1024); returns
// the exclusive prefix and writes the block total to *total.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t s = lane < kScanThreads / 64 ? wsum[lane] : 0;
    uint32_t si = wave_incl_scan(s);
    if (lane < kScanThreads / 64) wsum[lane] = si - s;
    if (lane == kScanThreads / 64 - 1) *total = si;
  }
  __syncthreads();
  uint32_t r = inc - v + wsum[wid];
  __syncthreads();
  return r;
}

// Phase 1: per-block sums (and maxima) of a[r][1 .. N] (the per-object counts).
__global__ void __launch_bounds__(kScanThreads)
k_scan_sums(const uint32_t* __restrict__ a, uint32_t N, uint32_t nb, uint32_t* __restrict__ bsum,
            uint32_t* __restrict__ maxdeg) {
  uint32_t r = blockIdx.y;
  const uint32_t* p = a + (size_t)r * (N + 1) + 1;
  uint32_t start = blockIdx.x * kScanBlock;
  uint32_t s = 0, m = 0;
  for (int k = 0; k < kScanItems; ++k) {
    uint32_t i = start + k * kScanThreads + threadIdx.x;
    if (i < N) {
      uint32_t v = p[i];
      s += v;
      m = max(m, v);
    }
  }
  __shared__ uint32_t ss[kScanThreads / 64], mm[kScanThreads / 64];
  for (int d = 32; d >= 1; d >>= 1) {
    s += __shfl_xor(s, d, 64);
    m = max(m, __shfl_xor(m, d, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    ss[threadIdx.x >> 6] = s;
    mm[threadIdx.x >> 6] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ts = 0, tm = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
      ts += ss[i];
      tm = max(tm, mm[i]);
    }
    bsum[(size_t)r * nb + blockIdx.x] = ts;
    atomicMax(maxdeg + r, tm);
  }
}

// Phase 2: exclusive scan of the block sums of each role (one block per role).
__global__ void __launch_bounds__(kScanThreads)
k_scan_block_sums(uint32_t* __restrict__ bsum, uint32_t nb) {
  uint32_t* p = bsum + (size_t)blockIdx.x * nb;
  __shared__ uint32_t carry_s;
  __shared__ uint32_t tot;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (uint32_t c = 0; c < nb; c += kScanThreads) {
    uint32_t i = c + threadIdx.x;
    uint32_t v = i < nb ? p[i] : 0;
    uint32_t ex = block_excl_scan(v, &tot);
    uint32_t carry = carry_s;
    if (i < nb) p[i] = ex + carry;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + tot;
    __syncthreads();
  }
}

// Phase 3: inclusive scan inside each block plus its block offset.
__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(uint32_t* __restrict__ a, uint32_t N, uint32_t nb, const uint32_t* __restrict__ bsum) {
  uint32_t r = blockIdx.y;
  uint32_t* p = a + (size_t)r * (N + 1) + 1;
  uint32_t start = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    uint32_t i = start + k;
    v[k] = i < N ? p[i] : 0;
    s += v[k];
  }
  __shared__ uint32_t tot;
  uint32_t ex = block_excl_scan(s, &tot) + bsum[(size_t)r * nb + blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    uint32_t i = start + k;
    ex += v[k];
    if (i < N) p[i] = ex;
  }
}

// Scatter: assertion (x, y) of role r becomes (y, x) of r^-.  Row order inside
// an inverse row follows the atomics and is not fixed; evaluation results do
// not depend on it.
// Heavy rows (more than hmin assertions) are scattered by k_scatter_heavy.
__global__ void k_scatter_inverse(const uint32_t* __restrict__ fwd_off, const int32_t* __restrict__ tg,
                                  const uint64_t* __restrict__ base, uint32_t N, uint32_t hmin,
                                  uint32_t* __restrict__ cursor, int32_t* __restrict__ inv_tg) {
  uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t r = blockIdx.y;
  if (x >= N) return;
  const uint32_t* fo = fwd_off + (size_t)r * (N + 1);
  if (fo[x + 1] - fo[x] > hmin) return;
  const int32_t* t = tg + base[r];
  int32_t* it = inv_tg + base[r];
  uint32_t* cur = cursor + (size_t)r * (N + 1);
  for (uint32_t e = fo[x]; e < fo[x + 1]; ++e) {
    uint32_t y = (uint32_t)t[e];
    uint32_t pos = atomicAdd(cur + y, 1u);
    it[pos] = (int32_t)x;
  }
}

// The assertions of the forward heavy rows of one role, one block per chunk of
// kHeavyChunk (tg and fo: the role's targets and relative offsets, inv_cnt and
// cursor its inverse rows).  Validation: every target in [0, N), strictly
// increasing inside the row; each assertion counted for its object.
__global__ void __launch_bounds__(256)
k_validate_heavy(const int32_t* __restrict__ tg, const uint32_t* __restrict__ fo, const uint32_t* __restrict__ rows,
                 const HeavyChunk* __restrict__ chunks, uint32_t N, uint32_t* __restrict__ inv_cnt,
                 uint32_t* __restrict__ flags) {
  const HeavyChunk c = chunks[blockIdx.x];
  const uint32_t x = rows[c.hrow];
  const uint32_t end = fo[x + 1];
  const uint32_t e0 = fo[x] + c.k * kHeavyChunk, e1 = min(end, e0 + kHeavyChunk);
  uint32_t bad = 0;
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int32_t t = tg[e];
    if (t < 0 || (uint32_t)t >= N) {
      bad |= F_TARGET;
      continue;
    }
    if (e + 1 < end && tg[e + 1] <= t) bad |= F_ORDER;
    atomicAdd(inv_cnt + t + 1, 1u);
  }
  if (bad) atomicOr(flags, bad);
}

// Scatter of the forward heavy rows' assertions (after validation).
__global__ void __launch_bounds__(256)
k_scatter_heavy(const int32_t* __restrict__ tg, const uint32_t* __restrict__ fo, const uint32_t* __restrict__ rows,
                const HeavyChunk* __restrict__ chunks, uint32_t* __restrict__ cursor, int32_t* __restrict__ inv_tg) {
  const HeavyChunk c = chunks[blockIdx.x];
  const uint32_t x = rows[c.hrow];
  const uint32_t e0 = fo[x] + c.k * kHeavyChunk, e1 = min(fo[x + 1], e0 + kHeavyChunk);
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const uint32_t y = (uint32_t)tg[e];
    inv_tg[atomicAdd(cursor + y, 1u)] = (int32_t)x;
  }
}

// Objects of a role direction: the individuals that occur as targets in it
// (for the forward direction the subjects of non-empty inverse rows, and the
// other way round).  mask row 2r + dir holds one bit per individual; base row
// 2r + dir the number of objects in the words before each word (entry W =
// their total); ctg maps each assertion's target to its rank among the
// objects, so that a shared pass can index transposed child rows that hold
// the objects only.
__global__ void __launch_bounds__(256)
k_object_mask(const uint32_t* __restrict__ opp_off, uint32_t N, uint32_t W, uint64_t* __restrict__ mask) {
  const uint32_t r = blockIdx.y;
  const uint32_t y = blockIdx.x * 256 + threadIdx.x;
  const uint32_t* o = opp_off + (size_t)r * (N + 1);
  const bool obj = y < N && o[y + 1] > o[y];
  const uint64_t m = __ballot(obj);
  const uint32_t w = y >> 6;
  if ((threadIdx.x & 63) == 0 && w < W) mask[(size_t)r * 2 * W + w] = m;
}

// One block per mask row: exclusive prefix of the words' popcounts.
__global__ void __launch_bounds__(kScanThreads)
k_object_base(const uint64_t* __restrict__ mask, uint32_t W, uint32_t* __restrict__ base) {
  const uint64_t* m = mask + (size_t)blockIdx.x * W;
  uint32_t* b = base + (size_t)blockIdx.x * (W + 1);
  const uint32_t per = (W + kScanThreads - 1) / kScanThreads;
  const uint32_t w0 = threadIdx.x * per, w1 = min(W, w0 + per);
  uint32_t s = 0;
  for (uint32_t w = w0; w < w1; ++w) s += (uint32_t)__popcll(m[w]);
  __shared__ uint32_t tot;
  uint32_t ex = block_excl_scan(s, &tot);
  for (uint32_t w = w0; w < w1; ++w) {
    b[w] = ex;
    ex += (uint32_t)__popcll(m[w]);
  }
  if (threadIdx.x == 0) b[W] = tot;
}

__global__ void __launch_bounds__(256)
k_object_rank(const int32_t* __restrict__ tg, uint64_t e0, uint64_t n, const uint64_t* __restrict__ mask,
              const uint32_t* __restrict__ base, int32_t* __restrict__ ctg) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint32_t y = (uint32_t)tg[e0 + i];
    const uint64_t m = mask[y >> 6];
    ctg[e0 + i] = (int32_t)(base[y >> 6] + (uint32_t)__popcll(m & ((1ull << (y & 63)) - 1ull)));
  }
}

struct DerivedLayout {
  size_t fwd_off, inv_off, inv_tg, cursor, bsum, base, meta, words, wbase, objmask, objbase, ctg;
  size_t heavy, hchunk, hchunk0, cpop, total;
  uint32_t nb;
  size_t heavy_cap, chunk_cap;   // entries
};

// Heavy rows of one direction (more than hmin assertions), appended in any
// order as (direction 2r + dir, subject, degree); the host sorts them and
// writes the heavy-row and chunk tables.  A direction holds at most
// E_dir / (hmin + 1) of them, so `cap` (from the floor of hmin) is never
// reached; the check keeps the writes in bounds regardless.
__global__ void __launch_bounds__(256)
k_heavy_rows(const uint32_t* __restrict__ o, uint32_t N, uint32_t hmin, uint32_t rd, uint32_t cap,
             uint32_t* __restrict__ count, uint32_t* __restrict__ out) {
  const uint32_t x = blockIdx.x * 256 + threadIdx.x;
  if (x >= N) return;
  const uint32_t deg = o[x + 1] - o[x];
  if (deg <= hmin) return;
  const uint32_t slot = atomicAdd(count, 1u);
  if (slot < cap) {
    out[3 * (size_t)slot] = rd;
    out[3 * (size_t)slot + 1] = x;
    out[3 * (size_t)slot + 2] = deg;
  }
}

// Words (64 consecutive subjects) with at least one assertion, per role and
// direction, in increasing order: the role passes visit only these, and a
// pass may take several consecutive entries at once (their assertions form
// one contiguous range).  Three steps per list: per-block counts (256 words a
// block), an exclusive scan of the block counts, then each block writes its
// words at its scanned base.
__device__ __forceinline__ bool word_nonempty(const uint32_t* __restrict__ o, uint32_t N, uint32_t W,
                                              uint32_t w) {
  if (w >= W) return false;
  const uint32_t a = w * 64, b = min(a + 64, N);
  return o[b] != o[a];
}

__global__ void __launch_bounds__(256)
k_nonempty_count(const uint32_t* __restrict__ o, uint32_t N, uint32_t W, uint32_t* __restrict__ bcnt,
                 uint32_t* __restrict__ count) {
  __shared__ uint32_t wsum[4];
  const uint32_t w = blockIdx.x * 256 + threadIdx.x;
  const uint64_t m = __ballot(word_nonempty(o, N, W, w));
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    bcnt[blockIdx.x] = tot;
    if (tot) atomicAdd(count, tot);
  }
}

__global__ void __launch_bounds__(256)
k_nonempty_words(const uint32_t* __restrict__ o, uint32_t N, uint32_t W, const uint32_t* __restrict__ bbase,
                 uint32_t* __restrict__ list) {
  __shared__ uint32_t wsum[4];
  const uint32_t w = blockIdx.x * 256 + threadIdx.x;
  const bool ne = word_nonempty(o, N, W, w);
  const uint64_t m = __ballot(ne);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) wsum[wv] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t before = bbase[blockIdx.x];
  for (int i = 0; i < wv; ++i) before += wsum[i];
  if (ne) list[before + (uint32_t)__popcll(m & ((1ull << lane) - 1))] = w;
}

static DerivedLayout layout_for(const hth_kb_desc& d) {
  DerivedLayout L{};
  size_t R = d.n_roles, N = d.n_individuals;
  size_t offs = align_up(R * (N + 1) * 4, 256);
  L.nb = (uint32_t)((N + kScanBlock - 1) / kScanBlock);
  size_t at = 0;
  L.fwd_off = at; at += offs;
  L.inv_off = at; at += offs;
  L.inv_tg = at; at += align_up((size_t)d.n_edges * 4, 256);
  L.cursor = at; at += offs;
  L.bsum = at; at += align_up(R * L.nb * 4 + 4, 256);
  L.base = at; at += align_up((R + 1) * 8, 256);
  L.meta = at; at += align_up((4 + 4 * R) * 4, 256);
  L.words = at; at += align_up(2 * R * ((N + 63) / 64) * 4, 256);
  L.wbase = at; at += align_up(2 * R * (((N + 63) / 64 + 255) / 256) * 4, 256);
  L.objmask = at; at += align_up(2 * R * ((N + 63) / 64) * 8, 256);
  L.objbase = at; at += align_up(2 * R * ((N + 63) / 64 + 1) * 4, 256);
  L.ctg = at; at += align_up((size_t)d.n_edges * 8, 256);     // both directions
  L.heavy_cap = 2 * (d.n_edges / (kHeavyMinFloor + 1)) + 2;
  L.chunk_cap = 2 * (d.n_edges / kHeavyChunk) + L.heavy_cap + 2;
  L.heavy = at; at += align_up(L.heavy_cap * 12, 256);
  L.hchunk = at; at += align_up(L.chunk_cap * sizeof(HeavyChunk), 256);
  L.hchunk0 = at; at += align_up((L.heavy_cap + 1) * 4, 256);
  L.cpop = at; at += align_up((size_t)d.n_concepts * 4 + 4, 256);
  L.total = at;
  return L;
}

static hth_status check_desc(const hth_kb_desc* d) {
  if (!d) return fail(HTH_E_INVALID, "desc is NULL");
  if (d->n_individuals == 0 || d->n_individuals >= (1u << 31))
    return fail(HTH_E_RANGE, "n_individuals must be in [1, 2^31)");
  uint32_t W = (d->n_individuals + 63) / 64;
  if (d->stride_words < W || d->stride_words % 8)
    return fail(HTH_E_INVALID, "stride_words must be >= ceil(N/64) and a multiple of 8");
  if (d->n_concepts && !d->concept_bits) return fail(HTH_E_INVALID, "concept_bits is NULL");
  if ((reinterpret_cast<uintptr_t>(d->concept_bits) | reinterpret_cast<uintptr_t>(d->pos_bits) |
       reinterpret_cast<uintptr_t>(d->neg_bits)) % 16)
    return fail(HTH_E_INVALID, "bit rows must be 16-byte aligned");
  if (d->n_roles && (!d->role_offsets || (d->n_edges && !d->role_targets)))
    return fail(HTH_E_INVALID, "role arrays are NULL");
  if (d->n_roles > 65535) return fail(HTH_E_RANGE, "at most 65535 roles");
  if (d->n_edges >= (1ull << 40)) return fail(HTH_E_RANGE, "too many assertions");
  if (d->n_data && !d->data) return fail(HTH_E_INVALID, "data is NULL");
  if (!d->pos_bits || !d->neg_bits) return fail(HTH_E_INVALID, "example rows are NULL");
  if (d->n_concepts >= (1u << 26)) return fail(HTH_E_RANGE, "too many concepts");
  return HTH_OK;
}

}  // namespace hth

using namespace hth;

extern "C" hth_status hth_kb_derived_bytes(const hth_kb_desc* desc, size_t* bytes) {
  hth_status s = check_desc(desc);
  if (s) return s;
  if (!bytes) return fail(HTH_E_INVALID, "bytes is NULL");
  *bytes = layout_for(*desc).total;
  return HTH_OK;
}

// A device error flag word -> HTH_E_INVALID with the reasons.
static hth_status check_flags(const uint32_t* flags, hipStream_t st) {
  uint32_t hflags = 0;
  HTH_HIP(hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, st));
  HTH_HIP(hipStreamSynchronize(st));
  if (!hflags) return HTH_OK;
  std::string m = "invalid knowledge base:";
  if (hflags & F_NONMONO) m += " role offsets not monotone;";
  if (hflags & F_TARGET) m += " role target outside [0, N);";
  if (hflags & F_ORDER) m += " role targets not strictly increasing in a row;";
  if (hflags & F_PAD) m += " padding bits set in a bit row;";
  return fail(HTH_E_INVALID, m);
}

// Appends to `trip` the heavy rows of direction `dir` of every role whose
// largest degree there exceeds heavy_min, as (2r + dir, subject, degree).
static hth_status find_heavy(hth_kb_s* kb, const DerivedLayout& L, int dir, uint32_t* count,
                             std::vector<uint32_t>& trip, hipStream_t st) {
  const uint32_t R = kb->d.n_roles, N = kb->N;
  bool any = false;
  for (uint32_t r = 0; r < R; ++r) any |= kb->max_deg[dir][r] > kb->heavy_min;
  if (!any) return HTH_OK;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, count, (size_t)1, 0u);
  for (uint32_t r = 0; r < R; ++r)
    if (kb->max_deg[dir][r] > kb->heavy_min)
      hipLaunchKernelGGL(k_heavy_rows, dim3((N + 255) / 256), dim3(256), 0, st,
                         (dir ? kb->inv_off : kb->fwd_off) + (size_t)r * (N + 1), N, kb->heavy_min,
                         2 * r + dir, (uint32_t)L.heavy_cap, count, kb->heavy_rows);
  HTH_HIP(hipGetLastError());
  uint32_t nh = 0;
  HTH_HIP(hipMemcpyAsync(&nh, count, 4, hipMemcpyDeviceToHost, st));
  HTH_HIP(hipStreamSynchronize(st));
  if (nh > L.heavy_cap || trip.size() / 3 + nh > L.heavy_cap) return fail(HTH_E_RANGE, "heavy-row table overflow");
  const size_t at = trip.size();
  trip.resize(at + 3 * (size_t)nh);
  HTH_HIP(hipMemcpyAsync(trip.data() + at, kb->heavy_rows, 3 * (size_t)nh * 4, hipMemcpyDeviceToHost, st));
  HTH_HIP(hipStreamSynchronize(st));
  return HTH_OK;
}

struct HeavyTables {
  std::vector<uint32_t> heavy_first, chunk_first;   // [2R+1]
  uint32_t heavy_most = 0, chunk_most = 0;
};

// Sorts the heavy rows by (direction, subject) and writes the heavy-row,
// chunk and first-chunk tables to the device.
static hth_status upload_heavy(hth_kb_s* kb, const DerivedLayout& L, const std::vector<uint32_t>& trip,
                               HeavyTables& T, hipStream_t st) {
  const uint32_t R = kb->d.n_roles;
  const uint32_t nh = (uint32_t)(trip.size() / 3);
  T.heavy_first.assign(2 * R + 1, 0);
  T.chunk_first.assign(2 * R + 1, 0);
  if (!nh) return HTH_OK;
  std::vector<uint32_t> ord(nh);
  for (uint32_t i = 0; i < nh; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) {
    return trip[3 * a] != trip[3 * b] ? trip[3 * a] < trip[3 * b] : trip[3 * a + 1] < trip[3 * b + 1];
  });
  std::vector<uint32_t> rows(nh), chunk0(nh + 1);
  std::vector<HeavyChunk> chunks;
  std::vector<uint32_t> per(2 * R, 0), cper(2 * R, 0);
  for (uint32_t i = 0; i < nh; ++i) {
    const uint32_t* t = &trip[3 * (size_t)ord[i]];
    rows[i] = t[1];
    per[t[0]]++;
    const uint32_t nc = (t[2] + kHeavyChunk - 1) / kHeavyChunk;
    cper[t[0]] += nc;
    chunk0[i] = (uint32_t)chunks.size();
    for (uint32_t k = 0; k < nc; ++k) chunks.push_back(HeavyChunk{i, k});
  }
  chunk0[nh] = (uint32_t)chunks.size();
  if (chunks.size() > L.chunk_cap) return fail(HTH_E_RANGE, "heavy chunk table overflow");
  for (uint32_t rd = 0; rd < 2 * R; ++rd) {
    T.heavy_first[rd + 1] = T.heavy_first[rd] + per[rd];
    T.chunk_first[rd + 1] = T.chunk_first[rd] + cper[rd];
    T.heavy_most = std::max(T.heavy_most, per[rd]);
    T.chunk_most = std::max(T.chunk_most, cper[rd]);
  }
  HTH_HIP(hipMemcpyAsync(kb->heavy_rows, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, st));
  HTH_HIP(hipMemcpyAsync(kb->heavy_chunks, chunks.data(), chunks.size() * sizeof(HeavyChunk),
                         hipMemcpyHostToDevice, st));
  HTH_HIP(hipMemcpyAsync(kb->heavy_chunk0, chunk0.data(), chunk0.size() * 4, hipMemcpyHostToDevice, st));
  HTH_HIP(hipStreamSynchronize(st));
  return HTH_OK;
}

static hth_status kb_build(hth_kb_s* kb, char* derived, hipStream_t st) {
  const hth_kb_desc& d = kb->d;
  const uint32_t R = d.n_roles, N = kb->N;
  DerivedLayout L = layout_for(d);
  kb->fwd_off = reinterpret_cast<uint32_t*>(derived + L.fwd_off);
  kb->inv_off = reinterpret_cast<uint32_t*>(derived + L.inv_off);
  kb->inv_tg = reinterpret_cast<int32_t*>(derived + L.inv_tg);
  uint32_t* cursor = reinterpret_cast<uint32_t*>(derived + L.cursor);
  uint32_t* bsum = reinterpret_cast<uint32_t*>(derived + L.bsum);
  uint64_t* base = reinterpret_cast<uint64_t*>(derived + L.base);
  uint32_t* meta = reinterpret_cast<uint32_t*>(derived + L.meta);
  uint32_t* flags = meta;
  uint32_t* maxdeg = meta + 4;   // [2][R]
  kb->role_base_dev = base;

  const size_t offs = (size_t)R * (N + 1);
  auto fill = [&](uint32_t* p, size_t n, uint32_t v) {
    if (!n) return;
    unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, st, p, n, v);
  };
  fill(meta, 4 + 4 * R, 0);
  const uint32_t tb = 256;
  // padding of concept rows and example rows
  if (d.n_concepts)
    hipLaunchKernelGGL(k_check_padding, dim3((d.n_concepts + tb - 1) / tb), dim3(tb), 0, st,
                       d.concept_bits, d.n_concepts, kb->W, kb->S, kb->tail, flags);
  hipLaunchKernelGGL(k_check_padding, dim3(1), dim3(1), 0, st, d.pos_bits, 1u, kb->W, kb->S,
                     kb->tail, flags);
  hipLaunchKernelGGL(k_check_padding, dim3(1), dim3(1), 0, st, d.neg_bits, 1u, kb->W, kb->S,
                     kb->tail, flags);
  kb->concept_pop.assign(d.n_concepts, 0);
  if (d.n_concepts) {
    uint32_t* cpop = reinterpret_cast<uint32_t*>(derived + L.cpop);
    hipLaunchKernelGGL(k_row_pop, dim3(d.n_concepts), dim3(256), 0, st, d.concept_bits, kb->W, kb->S, cpop);
    HTH_HIP(hipGetLastError());
    HTH_HIP(hipMemcpyAsync(kb->concept_pop.data(), cpop, (size_t)d.n_concepts * 4, hipMemcpyDeviceToHost, st));
  }
  kb->role_base.assign(R + 1, 0);
  kb->max_deg[0].assign(R, 0);
  kb->max_deg[1].assign(R, 0);
  if (R) {
    hipLaunchKernelGGL(k_gather_bases, dim3((R + 255) / 256), dim3(256), 0, st, d.role_offsets,
                       R, N, base);
    HTH_HIP(hipGetLastError());
    HTH_HIP(hipMemcpyAsync(kb->role_base.data(), base, (R + 1) * 8, hipMemcpyDeviceToHost, st));
    HTH_HIP(hipStreamSynchronize(st));
    if (kb->role_base[0] != 0) return fail(HTH_E_INVALID, "role_offsets[0][0] must be 0");
    if (kb->role_base[R] != d.n_edges)
      return fail(HTH_E_INVALID, "role_offsets[R-1][N] must equal n_edges");
    for (uint32_t r = 0; r < R; ++r) {
      if (kb->role_base[r + 1] < kb->role_base[r])
        return fail(HTH_E_INVALID, "role offsets decrease between roles");
      if (kb->role_base[r + 1] - kb->role_base[r] >= (1ull << 32))
        return fail(HTH_E_RANGE, "a role has 2^32 or more assertions");
    }
    fill(kb->inv_off, offs, 0);
    dim3 g((N + tb - 1) / tb, R);
    hipLaunchKernelGGL(k_validate_rows, g, dim3(tb), 0, st, d.role_offsets, d.role_targets, base,
                       N, kb->heavy_min, kb->fwd_off, kb->inv_off, maxdeg, flags);
    HTH_HIP(hipGetLastError());
    HTH_HIP(hipMemcpyAsync(kb->max_deg[0].data(), maxdeg, R * 4, hipMemcpyDeviceToHost, st));
    hth_status fs = check_flags(flags, st);
    if (fs) return fs;
    // forward heavy rows: checked, counted and later scattered chunk by chunk
    // (tables of the forward direction only until the inverse exists)
    kb->heavy_rows = reinterpret_cast<uint32_t*>(derived + L.heavy);
    kb->heavy_chunks = reinterpret_cast<HeavyChunk*>(derived + L.hchunk);
    kb->heavy_chunk0 = reinterpret_cast<uint32_t*>(derived + L.hchunk0);
    std::vector<uint32_t> trip;
    fs = find_heavy(kb, L, 0, meta + 1, trip, st);
    if (fs) return fs;
    HeavyTables fwd;
    fs = upload_heavy(kb, L, trip, fwd, st);
    if (fs) return fs;
    for (uint32_t r = 0; r < R; ++r)
      if (uint32_t nc = fwd.chunk_first[2 * r + 1] - fwd.chunk_first[2 * r])
        hipLaunchKernelGGL(k_validate_heavy, dim3(nc), dim3(256), 0, st, d.role_targets + kb->role_base[r],
                           kb->fwd_off + (size_t)r * (N + 1), kb->heavy_rows,
                           kb->heavy_chunks + fwd.chunk_first[2 * r], N, kb->inv_off + (size_t)r * (N + 1), flags);
    HTH_HIP(hipGetLastError());
    fs = check_flags(flags, st);
    if (fs) return fs;
    dim3 gs(L.nb, R);
    hipLaunchKernelGGL(k_scan_sums, gs, dim3(kScanThreads), 0, st, kb->inv_off, N, L.nb, bsum,
                       maxdeg + R);
    hipLaunchKernelGGL(k_scan_block_sums, dim3(R), dim3(kScanThreads), 0, st, bsum, L.nb);
    hipLaunchKernelGGL(k_scan_apply, gs, dim3(kScanThreads), 0, st, kb->inv_off, N, L.nb, bsum);
    {
      unsigned gg = (unsigned)std::min<size_t>((offs + 255) / 256, 65536);
      hipLaunchKernelGGL(k_copy_u32, dim3(gg), dim3(256), 0, st, kb->inv_off, cursor, offs);
    }
    hipLaunchKernelGGL(k_scatter_inverse, g, dim3(tb), 0, st, kb->fwd_off, d.role_targets, base,
                       N, kb->heavy_min, cursor, kb->inv_tg);
    for (uint32_t r = 0; r < R; ++r)
      if (uint32_t nc = fwd.chunk_first[2 * r + 1] - fwd.chunk_first[2 * r])
        hipLaunchKernelGGL(k_scatter_heavy, dim3(nc), dim3(256), 0, st, d.role_targets + kb->role_base[r],
                           kb->fwd_off + (size_t)r * (N + 1), kb->heavy_rows,
                           kb->heavy_chunks + fwd.chunk_first[2 * r], cursor + (size_t)r * (N + 1),
                           kb->inv_tg + kb->role_base[r]);
    HTH_HIP(hipGetLastError());
    HTH_HIP(hipMemcpyAsync(kb->max_deg[1].data(), maxdeg + R, R * 4, hipMemcpyDeviceToHost, st));
    // non-empty word lists; the two directions' offsets are [R][N+1] each, so
    // run the kernel once per direction with list rows 2r + dir
    uint32_t* words = reinterpret_cast<uint32_t*>(derived + L.words);
    uint32_t* wcount = meta + 4 + 2 * R;                  // [R][2]
    kb->words = words;
    const uint32_t nwb = (kb->W + 255) / 256;
    uint32_t* wbase = reinterpret_cast<uint32_t*>(derived + L.wbase);
    for (int dir = 0; dir < 2; ++dir) {
      const uint32_t* off = dir ? kb->inv_off : kb->fwd_off;
      for (uint32_t r = 0; r < R; ++r) {
        const uint32_t* o = off + (size_t)r * (N + 1);
        uint32_t* bb = wbase + (size_t)(2 * r + dir) * nwb;
        hipLaunchKernelGGL(k_nonempty_count, dim3(nwb), dim3(256), 0, st, o, N, kb->W, bb, wcount + 2 * r + dir);
        hipLaunchKernelGGL(k_scan_block_sums, dim3(1), dim3(kScanThreads), 0, st, bb, nwb);
        hipLaunchKernelGGL(k_nonempty_words, dim3(nwb), dim3(256), 0, st, o, N, kb->W, bb,
                           words + (size_t)(2 * r + dir) * kb->W);
      }
    }
    HTH_HIP(hipGetLastError());
    kb->n_words.assign(2 * R, 0);
    HTH_HIP(hipMemcpyAsync(kb->n_words.data(), wcount, 2 * R * 4, hipMemcpyDeviceToHost, st));
    // objects of each direction and, where they are at most half of the
    // individuals, every assertion's object rank
    const uint32_t W = kb->W;
    kb->objmask = reinterpret_cast<uint64_t*>(derived + L.objmask);
    kb->objbase = reinterpret_cast<uint32_t*>(derived + L.objbase);
    kb->ctg_fwd = reinterpret_cast<int32_t*>(derived + L.ctg);
    kb->ctg_inv = kb->ctg_fwd + d.n_edges;
    for (int dir = 0; dir < 2; ++dir)
      hipLaunchKernelGGL(k_object_mask, dim3((N + 255) / 256, R), dim3(256), 0, st,
                         dir ? kb->fwd_off : kb->inv_off, N, W, kb->objmask + (size_t)dir * W);
    hipLaunchKernelGGL(k_object_base, dim3(2 * R), dim3(kScanThreads), 0, st, kb->objmask, W, kb->objbase);
    HTH_HIP(hipGetLastError());
    std::vector<uint32_t> nobj(2 * R);
    for (uint32_t rd = 0; rd < 2 * R; ++rd)
      HTH_HIP(hipMemcpyAsync(&nobj[rd], kb->objbase + (size_t)rd * (W + 1) + W, 4, hipMemcpyDeviceToHost, st));
    HTH_HIP(hipStreamSynchronize(st));
    kb->n_obj = nobj;
    for (uint32_t r = 0; r < R; ++r) {
      const uint64_t e0 = kb->role_base[r], n = kb->role_base[r + 1] - e0;
      if (!n) continue;
      const unsigned g = (unsigned)std::min<uint64_t>((n + 255) / 256, 65536);
      for (int dir = 0; dir < 2; ++dir) {
        if ((uint64_t)nobj[2 * r + dir] * 2 > N) continue;
        hipLaunchKernelGGL(k_object_rank, dim3(g), dim3(256), 0, st,
                           dir ? (const int32_t*)kb->inv_tg : d.role_targets, e0, n,
                           kb->objmask + (size_t)(2 * r + dir) * W, kb->objbase + (size_t)(2 * r + dir) * (W + 1),
                           dir ? kb->ctg_inv : kb->ctg_fwd);
      }
    }
    HTH_HIP(hipGetLastError());
    // the heavy-row tables of both directions
    fs = find_heavy(kb, L, 1, meta + 1, trip, st);
    if (fs) return fs;
    HeavyTables all;
    fs = upload_heavy(kb, L, trip, all, st);
    if (fs) return fs;
    kb->heavy_first = all.heavy_first;
    kb->chunk_first = all.chunk_first;
    kb->heavy_most = all.heavy_most;
    kb->chunk_most = all.chunk_most;
  }
  uint32_t hflags = 0;
  HTH_HIP(hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, st));
  HTH_HIP(hipStreamSynchronize(st));
  if (hflags & F_PAD) return fail(HTH_E_INVALID, "invalid knowledge base: padding bits set in a bit row");
  return HTH_OK;
}

extern "C" hth_status hth_kb_create(const hth_kb_desc* desc, void* derived, size_t derived_bytes,
                                    void* stream, hth_kb* out) {
  hth_status s = check_desc(desc);
  if (s) return s;
  if (!out) return fail(HTH_E_INVALID, "out is NULL");
  DerivedLayout L = layout_for(*desc);
  if (!derived || derived_bytes < L.total)
    return fail(HTH_E_NOMEM, "derived buffer smaller than hth_kb_derived_bytes");
  if (reinterpret_cast<uintptr_t>(derived) % 256)
    return fail(HTH_E_INVALID, "derived buffer must be 256-byte aligned");
  hth_kb_s* kb = new (std::nothrow) hth_kb_s();
  if (!kb) return fail(HTH_E_NOMEM, "host allocation failed");
  kb->d = *desc;
  kb->N = desc->n_individuals;
  kb->W = (kb->N + 63) / 64;
  kb->S = desc->stride_words;
  kb->tail = (kb->N & 63) ? ((1ull << (kb->N & 63)) - 1) : ~0ull;
  kb->pos = desc->pos_bits;
  kb->neg = desc->neg_bits;
  hipError_t e = hipGetDevice(&kb->device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, kb->device);
  if (e != hipSuccess) {
    delete kb;
    return hip_fail(e, "hipGetDeviceProperties");
  }
  kb->n_cu = prop.multiProcessorCount;
  auto env_u = [](const char* n, uint64_t dflt) {
    const char* e = std::getenv(n);
    return e ? (uint64_t)std::strtoull(e, nullptr, 10) : dflt;
  };
  kb->tune.group_min = (uint32_t)env_u("HTHEDL_GROUP_MIN", kb->tune.group_min);
  kb->tune.group_k = (uint32_t)std::min<uint64_t>(64, std::max<uint64_t>(1, env_u("HTHEDL_GROUP_K", kb->tune.group_k)));
  kb->tune.xcd_local = (uint32_t)env_u("HTHEDL_XCD", kb->tune.xcd_local);
  kb->tune.t_budget = env_u("HTHEDL_TBUDGET_MB", kb->tune.t_budget >> 20) << 20;
  kb->tune.group_unroll = (uint32_t)env_u("HTHEDL_GROUP_UNROLL", kb->tune.group_unroll);
  kb->tune.region_reg = (uint32_t)env_u("HTHEDL_REGION_REG", kb->tune.region_reg);
  kb->tune.t_compact = (uint32_t)env_u("HTHEDL_T_COMPACT", kb->tune.t_compact);
  kb->tune.t_segment_kb = (uint32_t)std::min<uint64_t>(1u << 22, env_u("HTHEDL_TSEG_KB", kb->tune.t_segment_kb));
  kb->tune.push_pct = (uint32_t)std::min<uint64_t>(100, env_u("HTHEDL_PUSH_PCT", kb->tune.push_pct));
  kb->tune.short_rows = (uint32_t)std::min<uint64_t>(64, env_u("HTHEDL_SHORT_ROWS", kb->tune.short_rows));
  kb->heavy_min = (uint32_t)std::min<uint64_t>(
      1u << 30, std::max<uint64_t>(kHeavyMinFloor, env_u("HTHEDL_HEAVY_MIN", kb->heavy_min)));
  kb->lds_per_block = prop.sharedMemPerBlock;
  s = kb_build(kb, static_cast<char*>(derived), static_cast<hipStream_t>(stream));
  if (s) {
    delete kb;
    return s;
  }
  *out = kb;
  return HTH_OK;
}

// ---------------------------------------------------------------------------
// multi-valued numeric concrete roles
// ---------------------------------------------------------------------------
namespace hth {

struct NumLayout {
  size_t heavy, hchunk, hchunk0, meta, roff, total;
  size_t heavy_cap, chunk_cap;
};
static NumLayout num_layout(uint32_t N, uint32_t n_roles, uint64_t n_values) {
  NumLayout L{};
  L.heavy_cap = n_values / (kHeavyMinFloor + 1) + 2;
  L.chunk_cap = n_values / kHeavyChunk + L.heavy_cap + 2;
  size_t at = 0;
  L.heavy = at; at += align_up(L.heavy_cap * 12, 256);
  L.hchunk = at; at += align_up(L.chunk_cap * sizeof(HeavyChunk), 256);
  L.hchunk0 = at; at += align_up((L.heavy_cap + 1) * 4, 256);
  L.meta = at; at += align_up((4 + (size_t)n_roles) * 4, 256);
  L.roff = at; at += align_up((size_t)n_roles * (N + 1) * 4, 256);
  L.total = at;
  return L;
}

// One thread per (role, subject): offsets within [lo, hi] and non-decreasing;
// the role's largest degree.
__global__ void k_validate_num_rows(const int64_t* __restrict__ off, uint32_t N, uint64_t n_values,
                                    uint32_t* __restrict__ maxdeg, uint32_t* __restrict__ flags) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (x >= N) return;
  const int64_t* o = off + (size_t)r * (N + 1);
  const int64_t a = o[x], b = o[x + 1];
  if (a < 0 || b < a || (uint64_t)b > n_values) {
    atomicOr(flags, F_NONMONO);
    return;
  }
  if (b - a >= (1ll << 32)) {
    atomicOr(flags, F_NONMONO);
    return;
  }
  atomicMax(maxdeg + r, (uint32_t)(b - a));
}

__global__ void k_check_values(const float* __restrict__ v, uint64_t n, uint32_t* __restrict__ flags) {
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    bad |= v[i] != v[i];
  if (bad) atomicOr(flags, F_TARGET);
}

// 32-bit offsets relative to each role's first value (one thread per entry).
__global__ void k_rel_offsets(const int64_t* __restrict__ off, uint32_t N, uint32_t* __restrict__ rel) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (x > N) return;
  const int64_t* o = off + (size_t)r * (N + 1);
  rel[(size_t)r * (N + 1) + x] = (uint32_t)(o[x] - o[0]);
}

// Heavy rows of numeric role r (more than hmin values) as (r, subject, degree).
__global__ void __launch_bounds__(256)
k_heavy_rows64(const int64_t* __restrict__ o, uint32_t N, uint32_t hmin, uint32_t r, uint32_t cap,
               uint32_t* __restrict__ count, uint32_t* __restrict__ out) {
  const uint32_t x = blockIdx.x * 256 + threadIdx.x;
  if (x >= N) return;
  const uint64_t deg = (uint64_t)(o[x + 1] - o[x]);
  if (deg <= hmin) return;
  const uint32_t slot = atomicAdd(count, 1u);
  if (slot < cap) {
    out[3 * (size_t)slot] = r;
    out[3 * (size_t)slot + 1] = x;
    out[3 * (size_t)slot + 2] = (uint32_t)deg;
  }
}

}  // namespace hth

extern "C" hth_status hth_numeric_derived_bytes(hth_kb kb, uint32_t n_roles, uint64_t n_values, size_t* bytes) {
  if (!kb || !bytes) return fail(HTH_E_INVALID, "NULL argument");
  if (n_roles >= (1u << 16) || n_values >= (1ull << 40)) return fail(HTH_E_RANGE, "too many numeric roles or values");
  *bytes = num_layout(kb->N, n_roles, n_values).total;
  return HTH_OK;
}

namespace hth {

// Ids in [0, n) and non-decreasing offsets from 0 (string dictionary, patterns).
__global__ void k_check_ids(const int32_t* __restrict__ ids, uint64_t n, uint32_t n_strings,
                            uint32_t* __restrict__ flags) {
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    bad |= ids[i] < 0 || (uint32_t)ids[i] >= n_strings;
  if (bad) atomicOr(flags, F_TARGET);
}
__global__ void k_check_monotone64(const int64_t* __restrict__ o, uint64_t n, uint32_t* __restrict__ flags) {
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    bad |= (i == 0 && o[0] != 0) || (i > 0 && o[i] < o[i - 1]);
  if (bad) atomicOr(flags, F_ORDER);
}

// The tables of a registration of value roles (numeric or string): heavy rows
// and their chunks in the caller's derived buffer, per-role first chunk and
// first value on the host.
struct ValueRoles {
  uint32_t* roff = nullptr;   // [n_roles][N+1] relative offsets
  uint32_t* rows = nullptr;
  HeavyChunk* chunks = nullptr;
  std::vector<uint32_t> chunk_first;
  std::vector<uint64_t> bounds;
};

// Validates the chain and monotonicity of offsets [n_roles][N+1] against
// n_values; `extra` (run on the stream before the check) adds the kind's own
// value checks into flags.  Then builds the heavy-row tables.
template <class Extra>
static hth_status value_roles(hth_kb_s* kb, uint32_t n_roles, const int64_t* offsets, uint64_t n_values,
                              char* dv, const NumLayout& L, hipStream_t st, Extra&& extra, ValueRoles& out) {
  const uint32_t N = kb->N;
  uint32_t* meta = reinterpret_cast<uint32_t*>(dv + L.meta);
  uint32_t* flags = meta;
  uint32_t* count = meta + 1;
  uint32_t* maxdeg = meta + 4;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, meta, (size_t)4 + n_roles, 0u);
  std::vector<int64_t> ends(2 * (size_t)n_roles);
  for (uint32_t r = 0; r < n_roles; ++r) {
    HTH_HIP(hipMemcpyAsync(&ends[2 * r], offsets + (size_t)r * (N + 1), 8, hipMemcpyDeviceToHost, st));
    HTH_HIP(hipMemcpyAsync(&ends[2 * r + 1], offsets + (size_t)r * (N + 1) + N, 8, hipMemcpyDeviceToHost, st));
  }
  HTH_HIP(hipStreamSynchronize(st));
  if (ends[0] != 0) return fail(HTH_E_INVALID, "value role offsets[0][0] must be 0");
  for (uint32_t r = 1; r < n_roles; ++r)
    if (ends[2 * r] != ends[2 * r - 1]) return fail(HTH_E_INVALID, "value role ranges must follow one another");
  if ((uint64_t)ends[2 * (size_t)n_roles - 1] != n_values)
    return fail(HTH_E_INVALID, "value role offsets[n_roles-1][N] must equal n_values");
  hipLaunchKernelGGL(k_validate_num_rows, dim3((N + 255) / 256, n_roles), dim3(256), 0, st, offsets, N, n_values,
                     maxdeg, flags);
  extra(flags);
  HTH_HIP(hipGetLastError());
  uint32_t hflags = 0;
  std::vector<uint32_t> md(n_roles);
  HTH_HIP(hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, st));
  HTH_HIP(hipMemcpyAsync(md.data(), maxdeg, (size_t)n_roles * 4, hipMemcpyDeviceToHost, st));
  HTH_HIP(hipStreamSynchronize(st));
  if (hflags & F_NONMONO) return fail(HTH_E_INVALID, "value role offsets not monotone or out of range");
  if (hflags & F_TARGET) return fail(HTH_E_INVALID, "a value is NaN or a string id is out of range");
  if (hflags & F_ORDER) return fail(HTH_E_INVALID, "string or pattern offsets not non-decreasing from 0");
  // heavy rows, sorted by (role, subject), and their chunk tables
  out.rows = reinterpret_cast<uint32_t*>(dv + L.heavy);
  out.chunks = reinterpret_cast<HeavyChunk*>(dv + L.hchunk);
  out.chunk_first.assign(n_roles + 1, 0);
  bool any = false;
  for (uint32_t r = 0; r < n_roles; ++r)
    if (md[r] > kb->heavy_min) {
      any = true;
      hipLaunchKernelGGL(k_heavy_rows64, dim3((N + 255) / 256), dim3(256), 0, st, offsets + (size_t)r * (N + 1), N,
                         kb->heavy_min, r, (uint32_t)L.heavy_cap, count, out.rows);
    }
  HTH_HIP(hipGetLastError());
  if (any) {
    uint32_t nh = 0;
    HTH_HIP(hipMemcpyAsync(&nh, count, 4, hipMemcpyDeviceToHost, st));
    HTH_HIP(hipStreamSynchronize(st));
    if (nh > L.heavy_cap) return fail(HTH_E_RANGE, "heavy-row table overflow");
    std::vector<uint32_t> trip(3 * (size_t)nh);
    HTH_HIP(hipMemcpyAsync(trip.data(), out.rows, trip.size() * 4, hipMemcpyDeviceToHost, st));
    HTH_HIP(hipStreamSynchronize(st));
    std::vector<uint32_t> ord(nh);
    for (uint32_t i = 0; i < nh; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) {
      return trip[3 * a] != trip[3 * b] ? trip[3 * a] < trip[3 * b] : trip[3 * a + 1] < trip[3 * b + 1];
    });
    std::vector<uint32_t> hrows(nh);
    std::vector<HeavyChunk> chunks;
    std::vector<uint32_t> cper(n_roles, 0);
    for (uint32_t i = 0; i < nh; ++i) {
      const uint32_t* t = &trip[3 * (size_t)ord[i]];
      hrows[i] = t[1];
      const uint32_t nc = (t[2] + kHeavyChunk - 1) / kHeavyChunk;
      cper[t[0]] += nc;
      for (uint32_t k = 0; k < nc; ++k) chunks.push_back(HeavyChunk{i, k});
    }
    if (chunks.size() > L.chunk_cap) return fail(HTH_E_RANGE, "heavy chunk table overflow");
    for (uint32_t r = 0; r < n_roles; ++r) out.chunk_first[r + 1] = out.chunk_first[r] + cper[r];
    HTH_HIP(hipMemcpyAsync(out.rows, hrows.data(), hrows.size() * 4, hipMemcpyHostToDevice, st));
    HTH_HIP(hipMemcpyAsync(out.chunks, chunks.data(), chunks.size() * sizeof(HeavyChunk), hipMemcpyHostToDevice, st));
    HTH_HIP(hipStreamSynchronize(st));
  }
  out.bounds.assign(n_roles + 1, 0);
  for (uint32_t r = 0; r < n_roles; ++r) out.bounds[r + 1] = (uint64_t)ends[2 * r + 1];
  out.roff = reinterpret_cast<uint32_t*>(dv + L.roff);
  hipLaunchKernelGGL(k_rel_offsets, dim3((N + 256) / 256, n_roles), dim3(256), 0, st, offsets, N, out.roff);
  HTH_HIP(hipGetLastError());
  HTH_HIP(hipStreamSynchronize(st));
  return HTH_OK;
}

static unsigned grid_for(uint64_t n) { return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 65536)); }

}  // namespace hth

extern "C" hth_status hth_kb_set_numeric(hth_kb kb, uint32_t n_roles, const int64_t* offsets, const float* values,
                                         uint64_t n_values, void* derived, size_t derived_bytes, void* stream) {
  if (!kb) return fail(HTH_E_INVALID, "kb is NULL");
  std::lock_guard<std::mutex> g(kb->mu);
  if (n_roles == 0) {
    kb->n_num = 0;
    kb->num_off = nullptr;
    kb->num_val = nullptr;
    kb->num_chunk_first.assign(1, 0);
    kb->num_bounds.assign(1, 0);
    return HTH_OK;
  }
  if (!offsets || (n_values && !values) || !derived) return fail(HTH_E_INVALID, "NULL argument");
  if (n_roles >= (1u << 16) || n_values >= (1ull << 40)) return fail(HTH_E_RANGE, "too many numeric roles or values");
  const NumLayout L = num_layout(kb->N, n_roles, n_values);
  if (derived_bytes < L.total) return fail(HTH_E_NOMEM, "numeric derived buffer smaller than hth_numeric_derived_bytes");
  if (reinterpret_cast<uintptr_t>(derived) % 256) return fail(HTH_E_INVALID, "derived buffer must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  ValueRoles V;
  hth_status s = value_roles(kb, n_roles, offsets, n_values, static_cast<char*>(derived), L, st, [&](uint32_t* flags) {
    if (n_values) hipLaunchKernelGGL(k_check_values, dim3(grid_for(n_values)), dim3(256), 0, st, values, n_values, flags);
  }, V);
  if (s) return s;
  kb->n_num = n_roles;
  kb->num_off = offsets;
  kb->num_val = values;
  kb->num_roff = V.roff;
  kb->num_heavy_rows = V.rows;
  kb->num_heavy_chunks = V.chunks;
  kb->num_chunk_first = V.chunk_first;
  kb->num_bounds = V.bounds;
  return HTH_OK;
}

extern "C" hth_status hth_string_derived_bytes(hth_kb kb, uint32_t n_roles, uint64_t n_values, size_t* bytes) {
  return hth_numeric_derived_bytes(kb, n_roles, n_values, bytes);
}

extern "C" hth_status hth_kb_set_strings(hth_kb kb, uint32_t n_roles, const int64_t* offsets, const int32_t* ids,
                                         uint64_t n_values, uint32_t n_strings, const int64_t* str_offsets,
                                         const uint8_t* chars, void* derived, size_t derived_bytes, void* stream) {
  if (!kb) return fail(HTH_E_INVALID, "kb is NULL");
  std::lock_guard<std::mutex> g(kb->mu);
  if (n_roles == 0) {
    kb->n_str = 0;
    kb->str_off = nullptr;
    kb->str_ids = nullptr;
    kb->str_chunk_first.assign(1, 0);
    kb->str_bounds.assign(1, 0);
    return HTH_OK;
  }
  if (!offsets || (n_values && !ids) || !derived || !str_offsets) return fail(HTH_E_INVALID, "NULL argument");
  if (n_roles >= (1u << 16) || n_values >= (1ull << 40)) return fail(HTH_E_RANGE, "too many string roles or values");
  if (n_strings >= (1u << 31)) return fail(HTH_E_RANGE, "n_strings >= 2^31");
  const NumLayout L = num_layout(kb->N, n_roles, n_values);
  if (derived_bytes < L.total) return fail(HTH_E_NOMEM, "string derived buffer smaller than hth_string_derived_bytes");
  if (reinterpret_cast<uintptr_t>(derived) % 256) return fail(HTH_E_INVALID, "derived buffer must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  ValueRoles V;
  hth_status s = value_roles(kb, n_roles, offsets, n_values, static_cast<char*>(derived), L, st, [&](uint32_t* flags) {
    if (n_values) hipLaunchKernelGGL(k_check_ids, dim3(grid_for(n_values)), dim3(256), 0, st, ids, n_values, n_strings, flags);
    hipLaunchKernelGGL(k_check_monotone64, dim3(grid_for((uint64_t)n_strings + 1)), dim3(256), 0, st, str_offsets,
                       (uint64_t)n_strings + 1, flags);
  }, V);
  if (s) return s;
  kb->n_str = n_roles;
  kb->n_strings = n_strings;
  kb->str_off = offsets;
  kb->str_ids = ids;
  kb->dict_off = str_offsets;
  kb->dict_chars = chars;
  kb->str_roff = V.roff;
  kb->str_heavy_rows = V.rows;
  kb->str_heavy_chunks = V.chunks;
  kb->str_chunk_first = V.chunk_first;
  kb->str_bounds = V.bounds;
  return HTH_OK;
}

extern "C" hth_status hth_kb_set_patterns(hth_kb kb, uint32_t n_patterns, const int64_t* offsets, const uint8_t* chars,
                                          void* stream) {
  if (!kb) return fail(HTH_E_INVALID, "kb is NULL");
  if (n_patterns && !offsets) return fail(HTH_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(kb->mu);
  if (n_patterns) {   // a short table: its offsets are checked on the host
    std::vector<int64_t> o((size_t)n_patterns + 1);
    hipStream_t st = static_cast<hipStream_t>(stream);
    HTH_HIP(hipMemcpyAsync(o.data(), offsets, o.size() * 8, hipMemcpyDeviceToHost, st));
    HTH_HIP(hipStreamSynchronize(st));
    if (o[0] != 0) return fail(HTH_E_INVALID, "pattern offsets[0] must be 0");
    for (size_t i = 1; i < o.size(); ++i)
      if (o[i] < o[i - 1]) return fail(HTH_E_INVALID, "pattern offsets must be non-decreasing");
    if (o.back() > 0 && !chars) return fail(HTH_E_INVALID, "pattern chars are NULL");
  }
  kb->n_patterns = n_patterns;
  kb->pat_off = n_patterns ? offsets : nullptr;
  kb->pat_chars = n_patterns ? chars : nullptr;
  return HTH_OK;
}

extern "C" hth_status hth_kb_set_examples(hth_kb kb, const uint64_t* pos, const uint64_t* neg) {
  if (!kb) return fail(HTH_E_INVALID, "kb is NULL");
  if (!pos || !neg) return fail(HTH_E_INVALID, "example rows are NULL");
  if ((reinterpret_cast<uintptr_t>(pos) | reinterpret_cast<uintptr_t>(neg)) % 16)
    return fail(HTH_E_INVALID, "example rows must be 16-byte aligned");
  std::lock_guard<std::mutex> g(kb->mu);
  kb->pos = pos;
  kb->neg = neg;
  return HTH_OK;
}

extern "C" hth_status hth_kb_set_sets(hth_kb kb, const uint64_t* rows, uint32_t n_rows) {
  if (!kb) return fail(HTH_E_INVALID, "kb is NULL");
  if (n_rows && !rows) return fail(HTH_E_INVALID, "set rows are NULL");
  if (n_rows >= (1u << 24)) return fail(HTH_E_RANGE, "set table holds at most 2^24 - 1 rows");
  if (reinterpret_cast<uintptr_t>(rows) % 16) return fail(HTH_E_INVALID, "set rows must be 16-byte aligned");
  std::lock_guard<std::mutex> g(kb->mu);
  kb->sets = n_rows ? rows : nullptr;
  kb->n_sets = n_rows;
  return HTH_OK;
}

extern "C" hth_status hth_kb_max_degree(hth_kb kb, uint32_t role, uint32_t inv, uint32_t* out) {
  if (!kb || !out) return fail(HTH_E_INVALID, "NULL argument");
  if (role >= kb->d.n_roles || inv > 1) return fail(HTH_E_RANGE, "role or direction out of range");
  *out = kb->max_deg[inv][role];
  return HTH_OK;
}

extern "C" hth_status hth_kb_get_tuning(hth_kb kb, hth_tuning* out) {
  if (!kb || !out) return fail(HTH_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> g(kb->mu);
  out->group_min = kb->tune.group_min;
  out->group_k = kb->tune.group_k;
  out->xcd_local = kb->tune.xcd_local;
  out->t_budget_mb = (uint32_t)(kb->tune.t_budget >> 20);
  out->unroll = kb->tune.group_unroll;
  out->region_reg = kb->tune.region_reg;
  out->t_compact = kb->tune.t_compact;
  out->t_segment_kb = kb->tune.t_segment_kb;
  out->push_pct = kb->tune.push_pct;
  out->short_rows = kb->tune.short_rows;
  return HTH_OK;
}

extern "C" hth_status hth_kb_set_tuning(hth_kb kb, const hth_tuning* t) {
  if (!kb || !t) return fail(HTH_E_INVALID, "NULL argument");
  if (t->group_k < 1 || t->group_k > 64 || t->xcd_local > 1 || t->t_budget_mb < 1 ||
      t->t_budget_mb > (1u << 20) || (t->unroll != 8 && t->unroll != 16) ||
      (t->region_reg != 0 && t->region_reg != 1 && t->region_reg != 2 && t->region_reg != 4) ||
      t->t_compact > 1 || t->t_segment_kb > (1u << 22) || t->push_pct > 100 || t->short_rows > 64)
    return fail(HTH_E_RANGE, "tuning value out of range");
  std::lock_guard<std::mutex> g(kb->mu);
  kb->tune.group_min = t->group_min;
  kb->tune.group_k = t->group_k;
  kb->tune.xcd_local = t->xcd_local;
  kb->tune.t_budget = (size_t)t->t_budget_mb << 20;
  kb->tune.group_unroll = t->unroll;
  kb->tune.region_reg = t->region_reg;
  kb->tune.t_compact = t->t_compact;
  kb->tune.t_segment_kb = t->t_segment_kb;
  kb->tune.push_pct = t->push_pct;
  kb->tune.short_rows = t->short_rows;
  return HTH_OK;
}

extern "C" hth_status hth_kb_destroy(hth_kb kb) {
  delete kb;
  return HTH_OK;
}

extern "C" hth_status hth_sync(void* stream) {
  HTH_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" const char* hth_status_str(hth_status s) {
  switch (s) {
    case HTH_OK: return "HTH_OK";
    case HTH_E_INVALID: return "HTH_E_INVALID";
    case HTH_E_RANGE: return "HTH_E_RANGE";
    case HTH_E_NOMEM: return "HTH_E_NOMEM";
    case HTH_E_DEVICE: return "HTH_E_DEVICE";
    case HTH_E_PLAN: return "HTH_E_PLAN";
    case HTH_E_STATE: return "HTH_E_STATE";
    case HTH_E_UNSUPPORTED: return "HTH_E_UNSUPPORTED";
    default: return "HTH_E_UNKNOWN";
  }
}

extern "C" size_t hth_last_error(char* buf, size_t n) {
  const std::string& m = g_err;
  if (buf && n) {
    size_t k = std::min(n - 1, m.size());
    std::memcpy(buf, m.data(), k);
    buf[k] = 0;
  }
  return m.size();
}
