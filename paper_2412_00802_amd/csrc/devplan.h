// Evaluation plans generated on the device (hth_dplan_*).
//
// The paper builds an evaluation plan per hypothesis on CPU threads and names
// plan generation on the GPU, with little or no CPU involvement, as future
// work (Sections 4 and 8).  Here the hypotheses of a batch are already in
// device memory (hth_node arrays, as hth_eval_batch takes them on the host),
// and two passes of one thread per hypothesis build the plan there:
//   k_dp_count  validates every node, computes each node's role-nesting level,
//               region-program stack depth and program length, hash-conses
//               the batch (each node gets a representative: the first equal
//               node, by construct, arguments and children's representatives)
//               and threshold leaves, numbers the rows of representative role
//               nodes and of the compound fillers they materialise, and counts
//               the plan's tables: role nodes per (level, role direction)
//               bucket, distinct thresholds per property, regions, program
//               words.  The counts are the only data the host reads back;
//   (host)      from the counts alone: table bases, the shared CSR passes of
//               each large bucket (ceil(count / group_k) passes), their T rows
//               and XCD placement, threshold groups, the workspace layout;
//   k_dp_emit   writes the threshold, role, fill and region tasks and the
//               shared passes' members (and acceptance masks) of the
//               representatives at per-table cursors, and every region program.
// Unlike the host compiler, children of and / or are not sorted or flattened
// (and(a, b) and and(b, a) are two subexpressions), and single existential
// restrictions are not pushed.  Every node of a hypothesis is evaluated,
// reachable from its root or not.  Concrete-role constructs (HTH_NUM_*,
// HTH_STR_*) are not generated.
// Included by exec.hip only.
#pragma once

namespace hth {
namespace {

constexpr uint32_t kDpLevels = 64;          // most role-nesting levels
constexpr uint32_t kDpNest = 32;            // most operators nested inside one region
constexpr uint32_t kDpMaxLen = 1u << 30;    // longest region program (instructions)

// reasons of a count-pass error (the first in hypothesis, then node order wins)
enum : uint32_t {
  DP_EMPTY = 1, DP_OFFSETS, DP_OP, DP_CONCEPT, DP_SET, DP_CHILD, DP_CHILDREN, DP_ROLE, DP_INV, DP_N,
  DP_PROP, DP_NAN, DP_CONCRETE, DP_LEVELS, DP_DEPTH, DP_NEST, DP_LONG,
};

struct DpSummary {
  unsigned long long err;       // lowest (hypothesis << 32 | node << 8 | reason); ~0 = none
  unsigned long long code;      // region-program instructions of all regions
  uint32_t levels, mat_depth, root_depth, pad;         // maxima
  uint32_t n_thr;               // summed per block (contiguous with the per-level array below)
  uint32_t n_slots;             // row counter: role and filler rows are numbered from it
  uint32_t mat[kDpLevels];
};
constexpr int kDpSums = 2 + kDpLevels;

// Role nodes are counted per bucket (level, direction 2r + dir): bk[0][L][rd]
// those a shared pass can decide (see GroupTask), bk[1][L][rd] the others.
// The host turns the counts into the buckets' shared passes (DpBucket) and the
// per-level tables of the role nodes that run alone.
struct DpBucket {
  uint32_t first_group;          // the bucket's first shared pass; kNone: its nodes run alone
  uint32_t member_base;          // member table index of that pass's first member
  uint32_t k;                    // members per pass (the last may hold fewer)
  uint32_t pad;
};

struct DpCursor {                // allocation cursors of the emit pass
  unsigned long long code;
  uint32_t mat[kDpLevels], role[kDpLevels], fill[kDpLevels];
};

struct DpBases {                 // each level's first entry in the task tables
  uint32_t mat[kDpLevels], role[kDpLevels], fill[kDpLevels];
  uint32_t nrole[kDpLevels];     // role nodes that run alone, per level
};

struct DpKB {                    // what the passes read of the knowledge base
  uint32_t n_concepts, n_sets, n_roles, n_data, W;
  uint32_t n_fixed;              // the first slot row: the all-zero row
  uint32_t n_dir;                // 2 R + 1
  const uint32_t* dir;           // [3][2R+1]: non-empty words, first heavy chunk, first heavy row
  uint32_t* pk;                  // [n_data] distinct thresholds per property (count pass)
  unsigned long long* tkey;      // threshold table: keys (kDpEmpty = free) ...
  uint32_t* tval;                // ... and per entry: index within its property, owning node
  uint32_t tmask;                // entries - 1 (a power of two above twice the nodes)
  uint32_t n_thr;                // distinct thresholds (emit pass): their rows come first
  // hash-consing of the batch (count pass): canon[g] = the representative of
  // node g (the first equal node to claim the key), crep the table of
  // representatives (same size as the threshold table), nbase[g] = the first
  // node of g's hypothesis; per representative: rowidx (role nodes) and, for
  // a compound filler, matclaim (the role node that materialises it) and matrow
  uint32_t* canon;                // leaves: synthetic ids from n_nodes up (see dp_leaf_id)
  uint32_t* nbase;
  uint32_t* crep;
  uint32_t* rowidx;
  uint32_t* matclaim;
  uint32_t* matrow;
  // per representative: kDpRead when some node reads it, plus the number of
  // hypotheses it is the root of (a role node read by nothing else and the
  // root of one hypothesis adds its coverage in its shared pass, without a row)
  uint32_t* ruse;
  uint32_t n_nodes;
};
constexpr uint32_t kDpRead = 1u << 31;

// The representative of a leaf is an id of its own, never a node index:
// n_nodes + 0 (top), + 1 (bottom), + 2 + a (atom a), + 2 + C + s (set row s),
// + 2 + C + n_sets + slot (threshold in the threshold table's slot).  Leaf ids
// are only compared, never used to index per-node arrays.
__device__ __forceinline__ uint32_t dp_leaf_id(const DpKB& K, const hth_node& x, uint32_t thr_slot) {
  switch (x.op) {
    case HTH_TOP: return K.n_nodes;
    case HTH_BOT: return K.n_nodes + 1;
    case HTH_ATOM: return K.n_nodes + 2 + x.arg;
    case HTH_SET: return K.n_nodes + 2 + K.n_concepts + x.arg;
    default: return K.n_nodes + 2 + K.n_concepts + K.n_sets + thr_slot;
  }
}

constexpr unsigned long long kDpEmpty = ~0ull;

// A threshold leaf's key: property, comparison and the threshold's bits.
__device__ __forceinline__ unsigned long long dp_thr_key(const hth_node& x) {
  const uint32_t cmp = x.op == HTH_DATA_GE ? 0u : x.op == HTH_DATA_LE ? 1u : 2u;
  return ((unsigned long long)(x.arg * 4u + cmp) << 32) | x.q.n;
}
__device__ __forceinline__ uint32_t dp_hash(unsigned long long k, uint32_t mask) {
  k ^= k >> 33;
  k *= 0xFF51AFD7ED558CCDull;
  k ^= k >> 33;
  k *= 0xC4CEB9FE1A85EC53ull;
  k ^= k >> 33;
  return (uint32_t)k & mask;
}

struct DpTables {
  ThrTask* thr;
  RegionTask* mat;
  RegionTask* roots;
  RoleTask* roles;
  FillTask* fills;               // fills[0]: the zero row
  uint32_t* code;
  GroupTask* groups;             // the shared passes (copied from the plan's shells each launch)
  GroupMember* members;
  const DpBucket* buckets;       // [kDpLevels][2R]
  uint32_t* bcur;                // [kDpLevels][2R] member cursors
  const uint32_t* pbase;         // [n_data] first threshold task of each property
};

// per-node facts of the count pass: bits 0-7 role-nesting height + 1 (0: no
// role below), 8-15 region stack depth, 16-23 operator nesting, bit 24 a
// row of its own (atom, set row, threshold, role node), bit 25 the complement
// of such a row
constexpr uint32_t kDpRow = 1u << 24, kDpNotRow = 1u << 25;

__device__ __forceinline__ bool dp_role(uint8_t op) { return op >= HTH_EXISTS && op <= HTH_EXACTLY; }
__device__ __forceinline__ bool dp_column(uint8_t op) {
  return op == HTH_DATA_GE || op == HTH_DATA_LE || op == HTH_DATA_EQ;
}

__device__ __forceinline__ uint32_t dp_nwords(const DpKB& K, uint32_t rd) { return K.dir[rd]; }
__device__ __forceinline__ uint32_t dp_chunks(const DpKB& K, uint32_t rd) {
  return K.dir[K.n_dir + rd + 1] - K.dir[K.n_dir + rd];
}
__device__ __forceinline__ uint32_t dp_heavy(const DpKB& K, uint32_t rd) {
  return K.dir[2 * K.n_dir + rd + 1] - K.dir[2 * K.n_dir + rd];
}

// The fields that decide a node's meaning (others are ignored: q of ∃/∀, inv
// outside role constructs, the child field of leaves), packed for hashing and
// comparison; the children's representatives complete the key.
struct DpKey {
  uint32_t head, arg, q;
};
__device__ __forceinline__ DpKey dp_key(const hth_node& x) {
  const bool role = dp_role(x.op), card = x.op >= HTH_ATLEAST && x.op <= HTH_EXACTLY;
  const bool nary = x.op == HTH_AND || x.op == HTH_OR;
  const bool has_arg = role || x.op == HTH_ATOM || x.op == HTH_SET || dp_column(x.op);
  DpKey k;
  k.head = (uint32_t)x.op | ((role ? (uint32_t)x.inv : 0u) << 8) | ((nary ? (uint32_t)x.arity : 0u) << 16);
  k.arg = has_arg ? x.arg : 0u;
  k.q = (card || dp_column(x.op)) ? x.q.n : 0u;
  return k;
}
__device__ __forceinline__ uint64_t dp_mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  return h * 0xFF51AFD7ED558CCDull;
}
// Representatives and bases are read and written by threads on every XCD
// while the count pass runs: device-scope atomic accesses, which bypass the
// caches that are not coherent between XCDs.
__device__ __forceinline__ uint32_t dp_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dp_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// child j of node x (hypothesis at b): its representative
__device__ __forceinline__ uint32_t dp_child_rep(const DpKB& K, const hth_node& x, const uint32_t* kids, uint32_t b,
                                                 uint32_t j) {
  const uint32_t c = (x.op == HTH_AND || x.op == HTH_OR) ? kids[x.child + j] : x.child;
  return dp_load(K.canon + b + c);
}
__device__ __forceinline__ uint32_t dp_n_children(const hth_node& x) {
  if (x.op == HTH_AND || x.op == HTH_OR) return x.arity;
  return (x.op == HTH_NOT || dp_role(x.op)) ? 1u : 0u;
}

// The representative of node g (local index i of the hypothesis at b), whose
// children already have theirs.  Open addressing over crep: a free slot is
// claimed with a release compare-and-swap; an occupied one (read with
// acquire) holds a representative whose key is compared exactly: its fields,
// and its children's representatives, which its own thread stored before the
// claim.  No thread ever waits for another.
__device__ uint32_t dp_canon(const DpKB& K, const hth_node* __restrict__ nodes, const uint32_t* __restrict__ kids,
                             uint32_t b, uint32_t g, const hth_node& x) {
  const DpKey k = dp_key(x);
  const uint32_t nc = dp_n_children(x);
  uint64_t h = dp_mix(dp_mix(dp_mix(0, k.head), k.arg), k.q);
  for (uint32_t j = 0; j < nc; ++j) h = dp_mix(h, dp_child_rep(K, x, kids, b, j));
  dp_store(K.nbase + g, b);
  for (uint32_t hs = (uint32_t)(h ^ (h >> 32)) & K.tmask;; hs = (hs + 1) & K.tmask) {
    uint32_t r = __hip_atomic_load(K.crep + hs, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (r == kNone) {
      uint32_t expected = kNone;
      if (__hip_atomic_compare_exchange_strong(K.crep + hs, &expected, g, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE,
                                               __HIP_MEMORY_SCOPE_AGENT))
        return g;
      r = expected;                     // the representative that claimed the slot first
    }
    const hth_node y = nodes[r];
    const DpKey ky = dp_key(y);
    if (ky.head != k.head || ky.arg != k.arg || ky.q != k.q) continue;
    const uint32_t by = dp_load(K.nbase + r);
    bool same = true;
    for (uint32_t j = 0; j < nc && same; ++j) same = dp_child_rep(K, y, kids, by, j) == dp_child_rep(K, x, kids, b, j);
    if (same) return r;
  }
}

// a shared pass decides the node (saturating counts up to kGroupMaxCount)
__device__ __forceinline__ bool dp_groupable(const hth_node& x) {
  return x.op == HTH_EXISTS || x.op == HTH_FORALL ||
         (x.op == HTH_ATLEAST ? x.q.n <= kGroupMaxCount : x.q.n < kGroupMaxCount);
}

__global__ void __launch_bounds__(256)
k_dp_count(const hth_node* __restrict__ nodes, const uint32_t* __restrict__ offs,
           const uint32_t* __restrict__ kids, uint32_t n_nodes, uint32_t n_kids, uint32_t n_hyps, DpKB K,
           uint32_t* __restrict__ info, uint32_t* __restrict__ len, DpSummary* __restrict__ sum,
           uint32_t* __restrict__ bk) {
  __shared__ uint32_t s_sum[kDpSums];
  __shared__ unsigned long long s_code;
  __shared__ uint32_t s_max[3];
  for (uint32_t i = threadIdx.x; i < kDpSums; i += blockDim.x) s_sum[i] = 0;
  if (threadIdx.x < 3) s_max[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_code = 0;
  __syncthreads();
  uint32_t* const s_thr = s_sum;
  uint32_t* const s_mat = s_sum + 2;
  const uint32_t nbk = kDpLevels * (K.n_dir - 1);
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < n_hyps) {
    auto err = [&](uint32_t node, uint32_t why) {
      atomicMin(&sum->err, ((unsigned long long)h << 32) | ((unsigned long long)node << 8) | why);
    };
    const uint32_t b = offs[h], e = offs[h + 1];
    bool ok = true;
    if (e < b || e > n_nodes) {
      err(0, DP_OFFSETS);
      ok = false;
    } else if (e == b) {
      err(0, DP_EMPTY);
      ok = false;
    }
    const uint32_t n = ok ? e - b : 0;
    for (uint32_t i = 0; i < n && ok; ++i) {
      const hth_node x = nodes[b + i];
      uint32_t hgt = 0, dep = 1, nest = 0, flags = 0;
      uint32_t role_lvl = kNone, mat_c = kNone;   // a role node's level and compound filler
      uint32_t thr_slot = 0;                       // a threshold's slot in the threshold table
      uint64_t L = 1;
      uint32_t why = 0;
      switch (x.op) {
        case HTH_TOP:
        case HTH_BOT:
          break;
        case HTH_ATOM:
          if (x.arg >= K.n_concepts) why = DP_CONCEPT;
          flags = kDpRow;
          break;
        case HTH_SET:
          if (x.arg >= K.n_sets) why = DP_SET;
          flags = kDpRow;
          break;
        case HTH_DATA_GE:
        case HTH_DATA_LE:
        case HTH_DATA_EQ:
          if (x.arg >= K.n_data) why = DP_PROP;
          else if (x.q.t != x.q.t) why = DP_NAN;
          flags = kDpRow;
          if (!why) {
            // one task and row per distinct threshold of the batch: the first
            // node to claim a key owns it
            const unsigned long long key = dp_thr_key(x);
            for (uint32_t hs = dp_hash(key, K.tmask);; hs = (hs + 1) & K.tmask) {
              const unsigned long long prev = atomicCAS(K.tkey + hs, kDpEmpty, key);
              if (prev == kDpEmpty) {
                K.tval[2 * hs] = atomicAdd(K.pk + x.arg, 1u);
                K.tval[2 * hs + 1] = b + i;
                atomicAdd(s_thr, 1u);
                thr_slot = hs;
                break;
              }
              if (prev == key) {
                thr_slot = hs;
                break;
              }
            }
          }
          break;
        case HTH_NOT: {
          if (x.child >= i) {
            why = DP_CHILD;
            break;
          }
          const uint32_t ci = info[b + x.child];
          hgt = ci & 255u;
          if (ci & kDpRow) {
            flags = kDpNotRow;
          } else {
            dep = (ci >> 8) & 255u;
            nest = ((ci >> 16) & 255u) + 1;
            L = (uint64_t)len[b + x.child] + 1;
          }
          break;
        }
        case HTH_AND:
        case HTH_OR: {
          if ((uint64_t)x.child + x.arity > n_kids) {
            why = DP_CHILDREN;
            break;
          }
          if (!x.arity) break;            // the empty conjunction / disjunction
          uint32_t d1 = 0, d2 = 0, nm = 0;
          uint64_t s = x.arity - 1;       // one and / or per child after the first
          for (uint32_t j = 0; j < x.arity; ++j) {
            const uint32_t c = kids[x.child + j];
            if (c >= i) {
              why = DP_CHILD;
              break;
            }
            const uint32_t ci = info[b + c];
            hgt = max(hgt, ci & 255u);
            const uint32_t d = (ci >> 8) & 255u;
            if (d > d1) {
              d2 = d1;
              d1 = d;
            } else if (d > d2) {
              d2 = d;
            }
            nm = max(nm, (ci >> 16) & 255u);
            s += len[b + c];
          }
          // deepest child first: it needs d1 entries, every later one its own + 1
          dep = max(d1, d2 + 1);
          nest = nm + 1;
          L = s;
          break;
        }
        case HTH_EXISTS:
        case HTH_FORALL:
        case HTH_ATLEAST:
        case HTH_ATMOST:
        case HTH_EXACTLY: {
          if (x.arg >= K.n_roles) why = DP_ROLE;
          else if (x.inv > 1) why = DP_INV;
          else if (x.child >= i) why = DP_CHILD;
          else if (x.op >= HTH_ATLEAST && x.q.n > 0x7FFFFFFFu) why = DP_N;
          if (why) break;
          const uint32_t c = b + x.child, ci = info[c];
          const uint32_t lvl = ci & 255u;    // this node's level: the height of its filler
          if (lvl >= kDpLevels) {
            why = DP_LEVELS;
            break;
          }
          hgt = lvl + 1;
          flags = kDpRow;
          const uint8_t cop = nodes[c].op;
          if (cop != HTH_TOP && cop != HTH_BOT && !(ci & (kDpRow | kDpNotRow))) {
            // a compound filler: materialised by a region at this level
            if (((ci >> 8) & 255u) > (uint32_t)kStackDepth) {
              why = DP_DEPTH;
              break;
            }
            if (((ci >> 16) & 255u) > kDpNest) {
              why = DP_NEST;
              break;
            }
            mat_c = c;
          }
          role_lvl = lvl;
          break;
        }
        case HTH_NUM_GE:
        case HTH_NUM_LE:
        case HTH_NUM_EQ:
        case HTH_STR_EQ:
        case HTH_STR_CONTAINS:
          why = DP_CONCRETE;
          break;
        default:
          why = DP_OP;
          break;
      }
      if (!why && L > kDpMaxLen) why = DP_LONG;
      if (why) {
        err(i, why);
        ok = false;
        break;
      }
      info[b + i] = hgt | (min(dep, 255u) << 8) | (min(nest, 255u) << 16) | flags;
      len[b + i] = (uint32_t)L;
      const uint32_t g = b + i;
      const bool leaf = x.op == HTH_TOP || x.op == HTH_BOT || x.op == HTH_ATOM || x.op == HTH_SET || dp_column(x.op);
      const uint32_t rep = leaf ? dp_leaf_id(K, x, thr_slot) : dp_canon(K, nodes, kids, b, g, x);
      dp_store(K.canon + g, rep);
      if (rep == g) {   // its children are read (an equal node's are the same representatives)
        const uint32_t nc = dp_n_children(x);
        for (uint32_t j = 0; j < nc; ++j) {
          const uint32_t cr = dp_child_rep(K, x, kids, b, j);
          if (cr < K.n_nodes) atomicOr(K.ruse + cr, kDpRead);
        }
      }
      if (role_lvl != kNone && rep == g) {
        // a representative role node: its row, its task in its bucket, and the
        // materialisation of its compound filler unless an equal one is claimed
        const uint32_t lvl = role_lvl, rd = 2 * x.arg + x.inv;
        K.rowidx[g] = atomicAdd(&sum->n_slots, 1u);
        atomicAdd(bk + (dp_groupable(x) ? 0u : nbk) + lvl * (K.n_dir - 1) + rd, 1u);
        atomicMax(s_max, lvl + 1);
        if (mat_c != kNone) {
          const uint32_t cc = dp_load(K.canon + mat_c);
          if (atomicCAS(K.matclaim + cc, kNone, g) == kNone) {
            K.matrow[cc] = atomicAdd(&sum->n_slots, 1u);
            atomicAdd(s_mat + lvl, 1u);
            atomicAdd(&s_code, (unsigned long long)len[mat_c]);
            atomicMax(s_max + 1, (info[mat_c] >> 8) & 255u);
          }
        }
      }
    }
    if (ok) {   // the root's region, with coverage
      const uint32_t r = b + n - 1, ri = info[r];
      const uint32_t rr = dp_load(K.canon + r);
      if (rr < K.n_nodes) atomicAdd(K.ruse + rr, 1u);
      if (((ri >> 8) & 255u) > (uint32_t)kStackDepth) err(n - 1, DP_DEPTH);
      else if (((ri >> 16) & 255u) > kDpNest) err(n - 1, DP_NEST);
      atomicAdd(&s_code, (unsigned long long)len[r]);
      atomicMax(s_max + 2, (ri >> 8) & 255u);
    }
  }
  __syncthreads();
  uint32_t* const out = &sum->n_thr;
  for (uint32_t i = threadIdx.x; i < kDpSums; i += blockDim.x)
    if (s_sum[i]) atomicAdd(out + i, s_sum[i]);
  if (threadIdx.x == 0) {
    atomicMax(&sum->levels, s_max[0]);
    atomicMax(&sum->mat_depth, s_max[1]);
    atomicMax(&sum->root_depth, s_max[2]);
    if (s_code) atomicAdd(&sum->code, s_code);
  }
}

// The bit row a leaf-like node reads (atom, set row, or the node's own row).
__device__ __forceinline__ uint32_t dp_leaf_row(const DpKB& K, const hth_node* nodes, const uint32_t* row,
                                                uint32_t g) {
  const hth_node x = nodes[g];
  if (x.op == HTH_ATOM) return x.arg;
  if (x.op == HTH_SET) return K.n_concepts + x.arg;
  return row[g];
}

// The region program of local node r of the hypothesis at b, written to out:
// postfix over bit rows, the deepest operand of each and / or first (the
// stack then holds the fewest values).  An explicit frame stack stands in for
// recursion; the count pass has bounded the nesting by kDpNest.
__device__ void dp_program(const DpKB& K, const hth_node* __restrict__ nodes, const uint32_t* __restrict__ kids,
                           const uint32_t* __restrict__ info, const uint32_t* __restrict__ row, uint32_t b,
                           uint32_t r, uint32_t* __restrict__ out) {
  struct Frame {
    uint32_t node, j, k;
  };
  Frame st[kDpNest + 2];
  int sp = 0;
  uint32_t pc = 0;
  st[sp++] = Frame{r, 0, 0};
  while (sp) {
    Frame& f = st[sp - 1];
    const hth_node x = nodes[b + f.node];
    if (x.op == HTH_NOT) {
      if (f.j == 0) {
        if (info[b + x.child] & kDpRow) {
          out[pc++] = rp_ins(RP_LEAF, 1, dp_leaf_row(K, nodes, row, b + x.child));
          --sp;
        } else {
          f.j = 1;
          st[sp++] = Frame{x.child, 0, 0};
        }
      } else {
        out[pc++] = rp_ins(RP_NOT, 0, 0);
        --sp;
      }
      continue;
    }
    if ((x.op == HTH_AND || x.op == HTH_OR) && x.arity) {
      const uint32_t a = x.arity;
      if (f.j == 0) {
        uint32_t k = 0, dk = 0;
        for (uint32_t j = 0; j < a; ++j) {
          const uint32_t d = (info[b + kids[x.child + j]] >> 8) & 255u;
          if (d > dk) {
            dk = d;
            k = j;
          }
        }
        f.k = k;
        f.j = 1;
        st[sp++] = Frame{kids[x.child + k], 0, 0};
        continue;
      }
      if (f.j >= 2) out[pc++] = rp_ins(x.op == HTH_AND ? RP_AND : RP_OR, 0, 0);
      if (f.j == a) {
        --sp;
        continue;
      }
      uint32_t m = f.j - 1;               // the next operand in order, skipping the first one
      if (m >= f.k) ++m;
      ++f.j;
      st[sp++] = Frame{kids[x.child + m], 0, 0};
      continue;
    }
    if (x.op == HTH_TOP || x.op == HTH_AND) out[pc++] = rp_ins(RP_TOP, 0, 0);
    else if (x.op == HTH_BOT || x.op == HTH_OR) out[pc++] = rp_ins(RP_BOT, 0, 0);
    else out[pc++] = rp_ins(RP_LEAF, 0, dp_leaf_row(K, nodes, row, b + f.node));
    --sp;
  }
}

__global__ void __launch_bounds__(256)
k_dp_emit(const hth_node* __restrict__ nodes, const uint32_t* __restrict__ offs,
          const uint32_t* __restrict__ kids, uint32_t n_hyps, DpKB K, const uint32_t* __restrict__ info,
          const uint32_t* __restrict__ len, uint32_t* __restrict__ row, DpCursor* __restrict__ cur, DpBases B,
          DpTables T) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h == 0) T.fills[0] = FillTask{K.n_fixed, 0u};
  if (h >= n_hyps) return;
  const uint32_t b = offs[h], n = offs[h + 1] - b;
  bool root_fused = false;
  for (uint32_t i = 0; i < n; ++i) {
    const hth_node x = nodes[b + i];
    if (dp_column(x.op)) {
      // the distinct threshold's task (the property's tasks are contiguous:
      // one column pass serves up to 32) and row
      const unsigned long long key = dp_thr_key(x);
      uint32_t hs = dp_hash(key, K.tmask);
      while (K.tkey[hs] != key) hs = (hs + 1) & K.tmask;
      const uint32_t t = T.pbase[x.arg] + K.tval[2 * hs];
      const uint32_t r = K.n_fixed + 1 + t;
      row[b + i] = r;
      if (K.tval[2 * hs + 1] == b + i) {
        ThrTask tt;
        tt.prop = x.arg;
        tt.cmp = x.op == HTH_DATA_GE ? 0u : x.op == HTH_DATA_LE ? 1u : 2u;
        tt.t = x.q.t;
        tt.out_row = r;
        T.thr[t] = tt;
      }
    } else if (dp_role(x.op)) {
      // rows of role nodes and materialised fillers were numbered by the count
      // pass, per representative; a node equal to an earlier one has no task
      const uint32_t rep = K.canon[b + i];
      const uint32_t r = K.n_fixed + 1 + K.n_thr + K.rowidx[rep];
      row[b + i] = r;
      if (rep != b + i) continue;
      const uint32_t c = b + x.child, ci = info[c], lvl = ci & 255u;
      const uint8_t cop = nodes[c].op;
      uint32_t crow, neg = 0;
      if (cop == HTH_TOP || cop == HTH_BOT) {
        crow = K.n_fixed;                   // the zero row, complemented for top
        neg = cop == HTH_TOP;
      } else if (ci & kDpRow) {
        crow = dp_leaf_row(K, nodes, row, c);
      } else if (ci & kDpNotRow) {
        crow = dp_leaf_row(K, nodes, row, b + nodes[c].child);
        neg = 1;
      } else {
        const uint32_t cc = K.canon[c];
        crow = K.n_fixed + 1 + K.n_thr + K.matrow[cc];
        if (K.matclaim[cc] == b + i) {
          const unsigned long long off = atomicAdd(&cur->code, (unsigned long long)len[c]);
          dp_program(K, nodes, kids, info, row, b, x.child, T.code + off);
          T.mat[B.mat[lvl] + atomicAdd(&cur->mat[lvl], 1u)] = RegionTask{(uint32_t)off, len[c], crow, kNone};
        }
      }
      // count predicate (lo <= cnt <= hi over the successors in the child, or
      // outside it for the universal restriction)
      constexpr uint32_t kInf = 0xFFFFFFFFu;
      uint32_t lo, hi;
      switch (x.op) {
        case HTH_EXISTS: lo = 1; hi = kInf; break;
        case HTH_FORALL: lo = 0; hi = 0; neg ^= 1u; break;
        case HTH_ATLEAST: lo = x.q.n; hi = kInf; break;
        case HTH_ATMOST: lo = 0; hi = x.q.n; break;
        default: lo = x.q.n; hi = x.q.n; break;
      }
      const uint32_t rd = 2 * x.arg + x.inv;
      const uint32_t nw = dp_nwords(K, rd);
      const uint32_t q = lvl * (K.n_dir - 1) + rd;
      const DpBucket bu = T.buckets[q];
      const bool member = bu.first_group != kNone && dp_groupable(x);
      // the root of this hypothesis only, read by no node: its shared pass adds
      // its coverage, it gets no row (its fill task writes the zero row, which
      // holds zeros already) and the hypothesis no root region
      const bool fused = member && i + 1 == n && K.ruse[b + i] == 1u;
      root_fused |= fused;
      if (nw < K.W)
        T.fills[B.fill[lvl] + atomicAdd(&cur->fill[lvl], 1u)] =
            fused ? FillTask{K.n_fixed, 0u} : FillTask{r, lo == 0 ? 1u : 0u};
      if (member) {
        // a member of one of its bucket's shared passes
        const uint32_t j = atomicAdd(T.bcur + q, 1u);
        GroupMember m;
        m.child_row = crow;
        m.neg = neg;
        m.lo = lo;
        m.hi = hi;
        m.sat = hi == kInf ? lo : hi + 1;
        m.out_row = fused ? kNone : r;
        m.cover = fused ? h : kNone;
        m.pad = 0;
        T.members[bu.member_base + j] = m;
        unsigned long long* acc =
            reinterpret_cast<unsigned long long*>(T.groups[bu.first_group + j / bu.k].acc);
        const unsigned long long bit = 1ull << (j % bu.k);
        for (uint32_t v = 0; v <= kGroupMaxCount; ++v) {
          const bool ok = v < kGroupMaxCount ? (lo <= v && v <= hi) : (hi == kInf && lo <= kGroupMaxCount);
          if (ok) atomicOr(acc + v, bit);
        }
        continue;
      }
      RoleTask t;
      t.role = x.arg;
      t.inv = x.inv;
      t.child_row = crow;
      t.neg = neg;
      t.lo = lo;
      t.hi = hi;
      t.sat = hi == kInf ? lo : hi + 1;
      t.out_row = r;
      t.n_words = nw;
      t.h_first = 0;                         // set by k_dp_heavy where heavy rows exist
      t.c_first = 0;
      t.hc0 = K.dir[K.n_dir + rd];
      t.hr0 = K.dir[2 * K.n_dir + rd];
      T.roles[B.role[lvl] + atomicAdd(&cur->role[lvl], 1u)] = t;
    }
  }
  if (root_fused) {
    T.roots[h] = RegionTask{0u, 0u, kNone, kNone};
    return;
  }
  const unsigned long long off = atomicAdd(&cur->code, (unsigned long long)len[b + n - 1]);
  dp_program(K, nodes, kids, info, row, b, n - 1, T.code + off);
  T.roots[h] = RegionTask{(uint32_t)off, len[b + n - 1], kNone, h};
}

// Block-wide exclusive scan of one value per lane (1024 lanes); returns the
// lane's prefix and leaves the block total in *total.
__device__ __forceinline__ uint32_t dp_block_scan(uint32_t v, uint32_t* s_w, uint32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < 16; ++w) {
      const uint32_t t = s_w[w];
      s_w[w] = run;
      run += t;
    }
    s_w[16] = run;
  }
  __syncthreads();
  const uint32_t r = s_w[wv] + inc - v;
  *total = s_w[16];
  __syncthreads();
  return r;
}

// The heavy-row block and counter ranges of each level's role tasks, in task
// order (k_role_heavy finds a block's task by binary search over them).
// One 1024-lane block per level.
__global__ void __launch_bounds__(1024)
k_dp_heavy(RoleTask* __restrict__ roles, DpBases B, DpKB K) {
  __shared__ uint32_t s_w[17];
  const uint32_t L = blockIdx.x;
  const uint32_t n = B.nrole[L], base = B.role[L];
  uint32_t carry_b = 0, carry_c = 0;
  for (uint32_t i0 = 0; i0 < n; i0 += blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    uint32_t nb = 0, nc = 0;
    if (i < n) {
      const RoleTask& t = roles[base + i];
      const uint32_t rd = 2 * t.role + t.inv;
      nb = dp_chunks(K, rd);
      nc = dp_heavy(K, rd);
    }
    uint32_t tb, tc;
    const uint32_t eb = dp_block_scan(nb, s_w, &tb);
    const uint32_t ec = dp_block_scan(nc, s_w, &tc);
    if (i < n) {
      roles[base + i].h_first = carry_b + eb;
      roles[base + i].c_first = carry_c + ec;
    }
    carry_b += tb;
    carry_c += tc;
  }
}

// dst[i] = src[i] for i < n (the shared passes' shells, fresh for each launch)
__global__ void __launch_bounds__(256)
k_dp_copy(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace
}  // namespace hth

// A plan generated on the device (hth_dplan_*).
struct hth_dplan_s {
  hth_kb kb = nullptr;
  const hth_node* nodes = nullptr;
  const uint32_t* offs = nullptr;
  const uint32_t* kids = nullptr;
  uint32_t n_nodes = 0, n_hyps = 0, n_kids = 0;
  const uint64_t* sets = nullptr;
  uint32_t n_sets = 0;
  char* buf = nullptr;     // the caller's scratch (see DpScratch)
  uint32_t* info = nullptr;
  uint32_t* len = nullptr;
  uint32_t* row = nullptr;
  hth::DpSummary* d_sum = nullptr;
  hth::DpCursor* d_cur = nullptr;
  uint32_t* d_bk = nullptr;
  hth::GroupTask* d_shells = nullptr;
  hth::DpBucket* d_buckets = nullptr;
  uint32_t* d_xslots = nullptr;
  uint32_t* d_bcur = nullptr;
  uint32_t* d_pbase = nullptr;        // first threshold task of each property
  hth::ThrGroup* d_thg = nullptr;     // threshold groups: up to 32 tasks of one property
  uint32_t n_buckets = 0, n_thg = 0;
  hth::DpKB K{};
  hth::DpSummary sum{};
  hth::DpBases B{};
  uint32_t n_mat = 0, n_role = 0, n_groups = 0, n_members = 0;
  uint32_t fills[hth::kDpLevels] = {};
  uint64_t nhb[hth::kDpLevels] = {}, nhc[hth::kDpLevels] = {};
  uint64_t max_nhb = 0;
  std::vector<std::vector<hth::GroupTask>> lv_groups;
  std::vector<std::vector<hth::GroupChunk>> lv_chunks;
  std::vector<size_t> lv_gbase;
  size_t o_thr = 0, o_mat = 0, o_root = 0, o_role = 0, o_fill = 0, o_code = 0, o_part = 0,
         o_grp = 0, o_mem = 0, o_tarea = 0, o_gpart = 0, o_slot = 0, need = 0;
  hth_kb_s::Tuning tune;              // the schedule the plan was laid out for
  hipEvent_t done = nullptr;          // recorded after each launch: destroy waits for it
  ~hth_dplan_s() {
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
  }
};

namespace hth {
namespace {

// The plan's scratch (caller memory, hth_dplan_scratch_bytes): per-node facts
// and rows, the count pass's summary and counts, cursors, the direction table,
// the threshold hash table, and the host-built tables with bounds from the node
// count (a shared pass holds at least one node, an XCD slot round at most
// eight passes, a threshold group at least one threshold).
struct DpScratch {
  size_t info, len, row, canon, nbase, rowidx, matclaim, matrow, ruse, sum, cur, bk, pk, dir, tkey, tval, crep, shell,
      bucket, xslot, bcur, thg, pbase, total;
  uint32_t tcap;
};
DpScratch dp_scratch(const hth_kb_s& kb, uint32_t n_nodes) {
  DpScratch L{};
  const size_t n = n_nodes, nd = 2 * (size_t)kb.d.n_roles + 1, nb = kDpLevels * (nd - 1);
  L.tcap = 1024;
  while (L.tcap < 2ull * n) L.tcap <<= 1;
  size_t at = 0;
  auto area = [&](size_t bytes) {
    const size_t a = at;
    at = align_up(at + bytes, 256);
    return a;
  };
  L.info = area(n * 4);
  L.len = area(n * 4);
  L.row = area(n * 4);
  L.canon = area(n * 4);
  L.nbase = area(n * 4);
  L.rowidx = area(n * 4);
  L.matclaim = area(n * 4);
  L.matrow = area(n * 4);
  L.ruse = area(n * 4);
  L.sum = area(sizeof(DpSummary));
  L.cur = area(sizeof(DpCursor));
  L.bk = area(2 * nb * 4);
  L.pk = area((size_t)kb.d.n_data * 4);
  L.dir = area(3 * nd * 4);
  L.tkey = area((size_t)L.tcap * 8);
  L.tval = area((size_t)L.tcap * 8);
  L.crep = area((size_t)L.tcap * 4);
  L.shell = area(n * sizeof(GroupTask));
  L.bucket = area(nb * sizeof(DpBucket));
  L.xslot = area(8 * n * 4);
  L.bcur = area(nb * 4);
  L.thg = area(n * sizeof(ThrGroup));
  L.pbase = area((size_t)kb.d.n_data * 4);
  L.total = at;
  return L;
}

const char* dp_reason(uint32_t why, hth_status* code) {
  switch (why) {
    case DP_EMPTY: *code = HTH_E_PLAN; return "hypothesis has no nodes";
    case DP_OFFSETS: *code = HTH_E_INVALID; return "node offsets decrease or pass n_nodes";
    case DP_OP: *code = HTH_E_INVALID; return "unknown op";
    case DP_CONCEPT: *code = HTH_E_RANGE; return "concept id out of range";
    case DP_SET: *code = HTH_E_RANGE; return "set row outside the registered set table";
    case DP_CHILD: *code = HTH_E_PLAN; return "child index not before its parent";
    case DP_CHILDREN: *code = HTH_E_RANGE; return "children range outside the children array";
    case DP_ROLE: *code = HTH_E_RANGE; return "role id out of range";
    case DP_INV: *code = HTH_E_INVALID; return "inv must be 0 or 1";
    case DP_N: *code = HTH_E_RANGE; return "n > 2^31-1";
    case DP_PROP: *code = HTH_E_RANGE; return "property id out of range";
    case DP_NAN: *code = HTH_E_INVALID; return "threshold is NaN";
    case DP_CONCRETE: *code = HTH_E_UNSUPPORTED; return "concrete-role constructs are not generated on the device";
    case DP_LEVELS: *code = HTH_E_UNSUPPORTED; return "role restrictions nested more than 64 deep";
    case DP_DEPTH: *code = HTH_E_UNSUPPORTED; return "boolean region nested deeper than 16 operand levels";
    case DP_NEST: *code = HTH_E_UNSUPPORTED; return "boolean region with more than 32 nested operators";
    default: *code = HTH_E_RANGE; return "region program longer than 2^30 instructions";
  }
}

// The host's part of a device plan: from the count pass's summary and bucket
// counts, the per-level table bases, the shared passes (a bucket with at least
// group_min decidable nodes gets ceil(count / group_k) passes, its nodes taken
// in the order the emit pass reaches them), their T rows and XCD placement,
// and the workspace layout.  A bucket is large enough from bucket_min nodes.
hth_status dp_schedule(hth_dplan_s& p, const std::vector<uint32_t>& bk, std::vector<DpBucket>& buckets,
                       std::vector<uint32_t>& xslots) {
  const hth_kb_s& kb = *p.kb;
  const DpSummary& S = p.sum;
  const uint32_t R2 = p.K.n_dir - 1, nbk = kDpLevels * R2;
  const uint32_t group_min = kb.tune.group_min ? kb.tune.group_min : 0xFFFFFFFFu;
  const uint32_t gk = std::max<uint32_t>(1, std::min<uint32_t>(kb.tune.group_k, kMaxK));
  buckets.assign(nbk, DpBucket{kNone, 0, 0, 0});
  p.lv_groups.assign(S.levels, {});
  p.lv_chunks.assign(S.levels, {});
  p.lv_gbase.assign(S.levels, 0);
  uint32_t fill = 1;                        // fills[0]: the zero row
  for (uint32_t L = 0; L < kDpLevels; ++L) {
    p.B.mat[L] = p.n_mat;
    p.B.role[L] = p.n_role;
    p.B.fill[L] = fill;
    p.n_mat += S.mat[L];
    if (L >= S.levels) continue;
    uint64_t solo = 0, nb = 0, nc = 0, nf = 0;
    for (uint32_t rd = 0; rd < R2; ++rd) {
      const uint64_t g = bk[L * R2 + rd], o = bk[nbk + L * R2 + rd];
      const bool grouped = g && g >= bucket_min(kb, rd, group_min);
      const uint64_t alone = o + (grouped ? 0 : g);
      solo += alone;
      nb += alone * (kb.chunk_first[rd + 1] - kb.chunk_first[rd]);
      nc += alone * (kb.heavy_first[rd + 1] - kb.heavy_first[rd]);
      if (kb.n_words[rd] < kb.W) nf += g + o;
    }
    // the shared passes, those over short-row directions first (a launch
    // holds passes of one kind); a bucket's passes stay consecutive
    for (int want_short = 1; want_short >= 0; --want_short)
      for (uint32_t rd = 0; rd < R2; ++rd) {
        const uint64_t g = bk[L * R2 + rd];
        const bool sr = short_rows(kb, rd);
        if (!(g && g >= bucket_min(kb, rd, group_min)) || (int)sr != want_short) continue;
        DpBucket& bu = buckets[L * R2 + rd];
        bu.first_group = p.n_groups + (uint32_t)p.lv_groups[L].size();
        bu.member_base = p.n_members;
        bu.k = gk;
        for (uint64_t i0 = 0; i0 < g; i0 += gk) {
          GroupTask gt{};
          gt.role = rd / 2;
          gt.inv = rd & 1;
          gt.k = (uint32_t)std::min<uint64_t>(gk, g - i0);
          gt.first = (uint32_t)(p.n_members + i0);
          gt.n_words = kb.n_words[rd];
          gt.n_obj_words = kb.n_words[rd ^ 1u];
          gt.compact = kb.tune.t_compact && 2ull * kb.n_obj[rd] <= kb.N;
          gt.short_rows = sr;
          p.lv_groups[L].push_back(gt);
        }
        p.n_members += (uint32_t)g;
      }
    if (nb >= (1ull << 32) || nc >= (1ull << 32)) return fail(HTH_E_RANGE, "heavy-row blocks of one level exceed 2^32");
    p.B.nrole[L] = (uint32_t)solo;
    p.n_role += (uint32_t)solo;
    p.fills[L] = (uint32_t)nf;
    fill += (uint32_t)nf;
    p.nhb[L] = nb;
    p.nhc[L] = nc;
    p.max_nhb = std::max(p.max_nhb, nb);
    p.lv_gbase[L] = p.n_groups;
    p.lv_chunks[L] = chunk_groups(kb, p.lv_groups[L]);
    for (GroupChunk& c : p.lv_chunks[L])
      if (kb.tune.xcd_local && c.n >= 8) place_on_xcds(kb, p.lv_groups[L], c, xslots);
    p.n_groups += (uint32_t)p.lv_groups[L].size();
  }
  size_t gpart = 0;
  for (uint32_t L = 0; L < S.levels; ++L)
    for (const GroupChunk& c : p.lv_chunks[L]) gpart = std::max(gpart, chunk_partial_bytes(kb, p.lv_groups[L], c));
  size_t at = 0;
  auto area = [&](size_t bytes) {
    const size_t a = at;
    at = align_up(at + bytes, 256);
    return a;
  };
  p.o_thr = area((size_t)S.n_thr * sizeof(ThrTask));
  p.o_mat = area((size_t)p.n_mat * sizeof(RegionTask));
  p.o_root = area((size_t)p.n_hyps * sizeof(RegionTask));
  p.o_role = area((size_t)p.n_role * sizeof(RoleTask));
  p.o_fill = area((size_t)fill * sizeof(FillTask));
  p.o_code = area((size_t)S.code * 4);
  p.o_part = area((size_t)p.max_nhb * 4);
  p.o_grp = area((size_t)p.n_groups * sizeof(GroupTask));
  p.o_mem = area((size_t)p.n_members * sizeof(GroupMember));
  size_t t_bytes = 0;   // the T area: the most one chunk of the plan uses
  for (uint32_t L = 0; L < S.levels; ++L) t_bytes = std::max(t_bytes, chunks_t_bytes(kb, p.lv_groups[L], p.lv_chunks[L]));
  p.o_tarea = area(t_bytes);
  p.o_gpart = area(gpart);
  p.o_slot = area(((size_t)S.n_slots + S.n_thr + 1) * kb.S * 8);
  p.need = at;
  return HTH_OK;
}

}  // namespace
}  // namespace hth

extern "C" hth_status hth_dplan_scratch_bytes(hth_kb kb, uint32_t n_nodes, size_t* bytes) {
  using namespace hth;
  if (!kb || !bytes) return fail(HTH_E_INVALID, "NULL argument");
  *bytes = dp_scratch(*kb, n_nodes).total;
  return HTH_OK;
}

extern "C" hth_status hth_dplan_create(hth_kb kb, const hth_node* d_nodes, uint32_t n_nodes,
                                       const uint32_t* d_hyp_node_offsets, uint32_t n_hyps,
                                       const uint32_t* d_children, uint32_t n_children, void* scratch,
                                       size_t scratch_bytes, void* stream, hth_dplan* out, size_t* ws_bytes) {
  using namespace hth;
  if (!kb || !d_nodes || !d_hyp_node_offsets || !scratch || !out || !ws_bytes)
    return fail(HTH_E_INVALID, "NULL argument");
  if (reinterpret_cast<uintptr_t>(scratch) % 256) return fail(HTH_E_INVALID, "scratch must be 256-byte aligned");
  if (n_children && !d_children) return fail(HTH_E_INVALID, "children is NULL");
  if (n_hyps == 0) return fail(HTH_E_RANGE, "a plan needs at least one hypothesis");
  if (n_nodes > (1u << 24)) return fail(HTH_E_RANGE, "more than 2^24 nodes in one call");
  if (kb->d.n_data >= (1u << 29)) return fail(HTH_E_RANGE, "more than 2^29 properties");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hth_dplan_s* p = new (std::nothrow) hth_dplan_s();
  if (!p) return fail(HTH_E_NOMEM, "host allocation failed");
  std::unique_ptr<hth_dplan_s> guard(p);
  p->kb = kb;
  p->nodes = d_nodes;
  p->offs = d_hyp_node_offsets;
  p->kids = d_children;
  p->n_nodes = n_nodes;
  p->n_hyps = n_hyps;
  p->n_kids = n_children;
  std::vector<uint32_t> dir;
  std::lock_guard<std::mutex> g(kb->mu);
  p->sets = kb->sets;
  p->n_sets = kb->n_sets;
  p->tune = kb->tune;
  const uint32_t nd = 2 * kb->d.n_roles + 1;
  dir.assign(3 * (size_t)nd, 0);
  for (uint32_t rd = 0; rd + 1 < nd; ++rd) dir[rd] = kb->n_words[rd];
  for (uint32_t rd = 0; rd < nd; ++rd) {
    dir[nd + rd] = kb->chunk_first[rd];
    dir[2 * nd + rd] = kb->heavy_first[rd];
  }
  p->K.n_concepts = kb->d.n_concepts;
  p->K.n_sets = kb->n_sets;
  p->K.n_roles = kb->d.n_roles;
  p->K.n_data = kb->d.n_data;
  p->K.W = kb->W;
  p->K.n_fixed = kb->d.n_concepts + kb->n_sets;
  p->K.n_dir = nd;
  p->n_buckets = kDpLevels * (nd - 1);
  const size_t nbk2 = 2 * (size_t)p->n_buckets;
  const size_t nd_data = kb->d.n_data;
  const DpScratch L = dp_scratch(*kb, n_nodes);
  if (scratch_bytes < L.total)
    return fail(HTH_E_NOMEM, "scratch too small: need " + std::to_string(L.total) + " bytes, have " +
                                 std::to_string(scratch_bytes));
  const uint32_t tcap = L.tcap;
  HTH_HIP(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
  p->buf = static_cast<char*>(scratch);
  p->info = reinterpret_cast<uint32_t*>(p->buf + L.info);
  p->len = reinterpret_cast<uint32_t*>(p->buf + L.len);
  p->row = reinterpret_cast<uint32_t*>(p->buf + L.row);
  p->d_sum = reinterpret_cast<DpSummary*>(p->buf + L.sum);
  p->d_cur = reinterpret_cast<DpCursor*>(p->buf + L.cur);
  p->d_bk = reinterpret_cast<uint32_t*>(p->buf + L.bk);
  p->K.dir = reinterpret_cast<const uint32_t*>(p->buf + L.dir);
  p->K.pk = reinterpret_cast<uint32_t*>(p->buf + L.pk);
  p->K.tkey = reinterpret_cast<unsigned long long*>(p->buf + L.tkey);
  p->K.tval = reinterpret_cast<uint32_t*>(p->buf + L.tval);
  p->K.tmask = tcap - 1;
  p->K.canon = reinterpret_cast<uint32_t*>(p->buf + L.canon);
  p->K.nbase = reinterpret_cast<uint32_t*>(p->buf + L.nbase);
  p->K.crep = reinterpret_cast<uint32_t*>(p->buf + L.crep);
  p->K.rowidx = reinterpret_cast<uint32_t*>(p->buf + L.rowidx);
  p->K.matclaim = reinterpret_cast<uint32_t*>(p->buf + L.matclaim);
  p->K.matrow = reinterpret_cast<uint32_t*>(p->buf + L.matrow);
  p->K.ruse = reinterpret_cast<uint32_t*>(p->buf + L.ruse);
  p->K.n_nodes = n_nodes;
  HTH_HIP(hipMemcpyAsync(p->buf + L.dir, dir.data(), dir.size() * 4, hipMemcpyHostToDevice, st));
  DpSummary init{};
  init.err = ~0ull;
  HTH_HIP(hipMemcpyAsync(p->d_sum, &init, sizeof(init), hipMemcpyHostToDevice, st));
  HTH_HIP(hipMemsetAsync(p->d_bk, 0, nbk2 * 4, st));
  if (nd_data) HTH_HIP(hipMemsetAsync(p->K.pk, 0, nd_data * 4, st));
  HTH_HIP(hipMemsetAsync(p->K.tkey, 0xFF, (size_t)tcap * 8, st));
  HTH_HIP(hipMemsetAsync(p->K.crep, 0xFF, (size_t)tcap * 4, st));
  if (n_nodes) HTH_HIP(hipMemsetAsync(p->K.matclaim, 0xFF, (size_t)n_nodes * 4, st));
  if (n_nodes) HTH_HIP(hipMemsetAsync(p->K.ruse, 0, (size_t)n_nodes * 4, st));
  hipLaunchKernelGGL(k_dp_count, dim3((n_hyps + 255) / 256), dim3(256), 0, st, d_nodes, d_hyp_node_offsets,
                     d_children, n_nodes, n_children, n_hyps, p->K, p->info, p->len, p->d_sum, p->d_bk);
  HTH_HIP(hipGetLastError());
  std::vector<uint32_t> bk(nbk2);
  HTH_HIP(hipMemcpyAsync(&p->sum, p->d_sum, sizeof(DpSummary), hipMemcpyDeviceToHost, st));
  HTH_HIP(hipMemcpyAsync(bk.data(), p->d_bk, nbk2 * 4, hipMemcpyDeviceToHost, st));
  std::vector<uint32_t> pk(nd_data);
  if (nd_data) HTH_HIP(hipMemcpyAsync(pk.data(), p->K.pk, nd_data * 4, hipMemcpyDeviceToHost, st));
  HTH_HIP(hipStreamSynchronize(st));
  const DpSummary& S = p->sum;
  if (S.err != ~0ull) {
    hth_status code;
    const char* why = dp_reason((uint32_t)(S.err & 255), &code);
    return fail(code, "hypothesis " + std::to_string(S.err >> 32) + " node " +
                          std::to_string((S.err >> 8) & 0xFFFFFF) + ": " + why);
  }
  if (S.code >= (1ull << 32)) return fail(HTH_E_RANGE, "region programs exceed 2^32 instructions");
  // row ids must fit the 27-bit argument of the region bytecode
  if ((uint64_t)p->K.n_fixed + 1 + S.n_thr + S.n_slots >= (1ull << 27)) return fail(HTH_E_RANGE, "too many bit rows");
  std::vector<DpBucket> buckets;
  std::vector<uint32_t> xslots;
  hth_status s = dp_schedule(*p, bk, buckets, xslots);
  if (s) return s;
  std::vector<GroupTask> shells;
  for (const auto& lg : p->lv_groups) shells.insert(shells.end(), lg.begin(), lg.end());
  // thresholds: each property's tasks together, in groups of at most kThrPerPass
  std::vector<uint32_t> pbase(nd_data);
  std::vector<ThrGroup> thg;
  uint32_t tsum = 0;
  for (uint32_t q = 0; q < nd_data; ++q) {
    pbase[q] = tsum;
    for (uint32_t i = 0; i < pk[q]; i += kThrPerPass)
      thg.push_back(ThrGroup{q, tsum + i, std::min<uint32_t>(kThrPerPass, pk[q] - i), 0});
    tsum += pk[q];
  }
  if (tsum != S.n_thr) return fail(HTH_E_DEVICE, "threshold counts disagree");
  p->K.n_thr = S.n_thr;
  p->n_thg = (uint32_t)thg.size();
  if (shells.size() > n_nodes || xslots.size() > 8ull * n_nodes || thg.size() > n_nodes)
    return fail(HTH_E_DEVICE, "plan tables beyond their bounds");
  p->d_shells = reinterpret_cast<GroupTask*>(p->buf + L.shell);
  p->d_buckets = reinterpret_cast<DpBucket*>(p->buf + L.bucket);
  p->d_xslots = reinterpret_cast<uint32_t*>(p->buf + L.xslot);
  p->d_bcur = reinterpret_cast<uint32_t*>(p->buf + L.bcur);
  p->d_thg = reinterpret_cast<ThrGroup*>(p->buf + L.thg);
  p->d_pbase = reinterpret_cast<uint32_t*>(p->buf + L.pbase);
  if (!thg.empty())
    HTH_HIP(hipMemcpyAsync(p->d_thg, thg.data(), thg.size() * sizeof(ThrGroup), hipMemcpyHostToDevice, st));
  if (nd_data) HTH_HIP(hipMemcpyAsync(p->d_pbase, pbase.data(), nd_data * 4, hipMemcpyHostToDevice, st));
  if (!shells.empty())
    HTH_HIP(hipMemcpyAsync(p->d_shells, shells.data(), shells.size() * sizeof(GroupTask), hipMemcpyHostToDevice, st));
  HTH_HIP(hipMemcpyAsync(p->d_buckets, buckets.data(), buckets.size() * sizeof(DpBucket), hipMemcpyHostToDevice, st));
  if (!xslots.empty())
    HTH_HIP(hipMemcpyAsync(p->d_xslots, xslots.data(), xslots.size() * 4, hipMemcpyHostToDevice, st));
  HTH_HIP(hipStreamSynchronize(st));   // the host vectors above end here
  *ws_bytes = p->need;
  *out = guard.release();
  return HTH_OK;
}

extern "C" hth_status hth_dplan_launch(hth_dplan plan, void* ws, size_t ws_bytes, uint32_t* d_counts,
                                       void* stream) {
  using namespace hth;
  if (!plan || !ws || !d_counts) return fail(HTH_E_INVALID, "NULL argument");
  hth_dplan_s& p = *plan;
  if (p.need > ws_bytes)
    return fail(HTH_E_NOMEM, "workspace too small: need " + std::to_string(p.need) + " bytes, have " +
                                 std::to_string(ws_bytes));
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(HTH_E_INVALID, "workspace must be 256-byte aligned");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hth_kb_s& kb = *p.kb;
  std::lock_guard<std::mutex> g(kb.mu);
  TuneScope ts(kb, p.tune);
  role_attributes(kb);
  char* w = static_cast<char*>(ws);
  DpTables T;
  T.thr = reinterpret_cast<ThrTask*>(w + p.o_thr);
  T.mat = reinterpret_cast<RegionTask*>(w + p.o_mat);
  T.roots = reinterpret_cast<RegionTask*>(w + p.o_root);
  T.roles = reinterpret_cast<RoleTask*>(w + p.o_role);
  T.fills = reinterpret_cast<FillTask*>(w + p.o_fill);
  T.code = reinterpret_cast<uint32_t*>(w + p.o_code);
  T.groups = reinterpret_cast<GroupTask*>(w + p.o_grp);
  T.members = reinterpret_cast<GroupMember*>(w + p.o_mem);
  T.buckets = p.d_buckets;
  T.bcur = p.d_bcur;
  T.pbase = p.d_pbase;
  DevKB d = dev_view(kb);
  d.sets = p.sets;
  d.n_fixed = p.K.n_fixed;
  d.slots = reinterpret_cast<uint64_t*>(w + p.o_slot);
  d.counts = d_counts;
  d.instances = nullptr;
  const uint32_t nc = 2 * p.n_hyps;
  hipLaunchKernelGGL(k_zero_u32, dim3((nc + 255) / 256), dim3(256), 0, st, d_counts, nc);
  HTH_HIP(hipGetLastError());
  const uint32_t ncur = (uint32_t)(sizeof(DpCursor) / 4);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(p.d_cur), ncur);
  HTH_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_zero_u32, dim3((p.n_buckets + 255) / 256), dim3(256), 0, st, p.d_bcur, p.n_buckets);
  HTH_HIP(hipGetLastError());
  if (p.n_groups) {
    const uint32_t nw = (uint32_t)(p.n_groups * sizeof(GroupTask) / 4);
    hipLaunchKernelGGL(k_dp_copy, dim3((nw + 255) / 256), dim3(256), 0, st, reinterpret_cast<uint32_t*>(T.groups),
                       reinterpret_cast<const uint32_t*>(p.d_shells), nw);
    HTH_HIP(hipGetLastError());
  }
  const DpSummary& S = p.sum;
  Launcher Lc{kb, st};
  hth_status s = Lc.run(HTH_K_PLAN, 0.0, [&] {
    hipLaunchKernelGGL(k_dp_emit, dim3((p.n_hyps + 255) / 256), dim3(256), 0, st, p.nodes, p.offs, p.kids,
                       p.n_hyps, p.K, p.info, p.len, p.row, p.d_cur, p.B, T);
  });
  if (s) return s;
  bool heavy = false;
  for (uint32_t L = 0; L < S.levels; ++L) heavy |= p.nhc[L] > 0;
  if (heavy) {
    s = Lc.run(HTH_K_PLAN, 0.0, [&] {
      hipLaunchKernelGGL(k_dp_heavy, dim3(S.levels), dim3(1024), 0, st, T.roles, p.B, p.K);
    });
    if (s) return s;
  }
  const uint32_t ftiles = fill_tiles(kb.S);
  s = Lc.run(HTH_K_FILL, (double)kb.W * 8, [&] {   // the zero row
    hipLaunchKernelGGL(k_fill_rows, dim3(ftiles), dim3(256), 0, st, d, T.fills, ftiles);
  });
  if (s) return s;
  if (p.n_thg) {
    const uint32_t n = p.n_thg, bpt = std::max<uint32_t>(1, (kb.W + 127) / 128);
    const double bytes = n * 4.0 * kb.N;   // the columns (model bytes; rows are an intermediate)
    s = split_launch(Lc, HTH_K_THRESHOLD, bytes, n, bpt, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
      hipLaunchKernelGGL(k_threshold, dim3(blocks), dim3(256), 0, st, d, p.d_thg + i0, T.thr, bpt);
    });
    if (s) return s;
  }
  void* tarea = w + p.o_tarea;
  for (uint32_t L = 0; L < S.levels; ++L) {
    Lc.csr_seen.clear();
    s = launch_regions_n(Lc, d, T.mat + p.B.mat[L], T.code, S.mat[L], (int)S.mat_depth, 0.0);
    if (s) return s;
    if (p.fills[L]) {
      const uint32_t n = p.fills[L];
      s = split_launch(Lc, HTH_K_FILL, (double)n * kb.W * 8, n, ftiles, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_fill_rows, dim3(blocks), dim3(256), 0, st, d, T.fills + p.B.fill[L] + i0, ftiles);
      });
      if (s) return s;
    }
    const RoleTask* rol = T.roles + p.B.role[L];
    const uint32_t nt = p.B.nrole[L];
    s = launch_roles_n(Lc, d, rol, nt, 0.0);
    if (s) return s;
    if (p.nhc[L]) {
      uint32_t* partial = reinterpret_cast<uint32_t*>(w + p.o_part);
      s = split_launch(Lc, HTH_K_ROLE, 0.0, p.nhb[L], 1, 256, [&](uint32_t b0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_role_heavy, dim3(blocks), dim3(256), 0, st, d, rol, nt, b0, partial);
      });
      if (s) return s;
      s = split_launch(Lc, HTH_K_ROLE, 0.0, p.nhc[L], 1, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_role_heavy_fix, dim3(blocks), dim3(256), 0, st, d, rol, nt, i0, partial);
      });
      if (s) return s;
    }
    if (!p.lv_groups[L].empty()) {
      s = launch_groups(Lc, d, T.groups + p.lv_gbase[L], T.members, p.lv_groups[L], p.lv_chunks[L], p.d_xslots,
                        tarea, w + p.o_gpart);
      if (s) return s;
    }
  }
  s = launch_regions_n(Lc, d, T.roots, T.code, p.n_hyps, (int)S.root_depth, 0.0);
  if (s) return s;
  HTH_HIP(hipEventRecord(p.done, st));
  return HTH_OK;
}

extern "C" hth_status hth_dplan_stats(hth_dplan plan, hth_dplan_info* out) {
  using namespace hth;
  if (!plan || !out) return hth::fail(HTH_E_INVALID, "NULL argument");
  const hth_dplan_s& p = *plan;
  out->levels = p.sum.levels;
  out->role_nodes = p.n_role + p.n_members;
  out->shared_passes = p.n_groups;
  out->thresholds = p.sum.n_thr;
  uint32_t mats = 0;
  for (uint32_t L = 0; L < kDpLevels; ++L) mats += p.sum.mat[L];
  out->materialised = mats;
  out->rows = p.sum.n_slots + p.sum.n_thr + 1;
  return HTH_OK;
}

extern "C" hth_status hth_dplan_destroy(hth_dplan plan) {
  delete plan;
  return HTH_OK;
}
