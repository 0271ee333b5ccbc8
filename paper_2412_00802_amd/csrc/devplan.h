// Evaluation plans generated on the device (hth_dplan_*).
//
// The paper builds an evaluation plan per hypothesis on CPU threads and names
// plan generation on the GPU, with little or no CPU involvement, as future
// work (Sections 4 and 7).  Here the hypotheses of a batch are already in
// device memory (hth_node arrays, as hth_eval_batch takes them on the host),
// and two passes of one thread per hypothesis build the plan there:
//   k_dp_count  validates every node, computes each node's role-nesting level,
//               region-program stack depth and program length, and sums the
//               table sizes per level into a small summary -- the only data the
//               host reads back (it sizes the workspace and the launches);
//   k_dp_emit   assigns bit rows, writes the threshold, role, fill and region
//               tasks at per-level cursors and writes every region program.
// The plan is the per-hypothesis plan of the paper: each DL operation of each
// hypothesis is one task (no subexpression sharing across hypotheses, no
// shared CSR passes, no push), scheduled level by level on the executor's own
// kernels.  Every node of a hypothesis is evaluated, reachable from its root
// or not.  Concrete-role constructs (HTH_NUM_*, HTH_STR_*) are not generated.
// Included by exec.hip only.
#pragma once

namespace hth {
namespace {

constexpr uint32_t kDpLevels = 16;          // most role-nesting levels
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
  unsigned long long nhb[kDpLevels], nhc[kDpLevels];   // heavy-row blocks / (task, heavy row) pairs
  uint32_t levels, mat_depth, root_depth, pad;         // maxima
  uint32_t n_thr, n_slots;      // sums (contiguous with the per-level arrays below)
  uint32_t mat[kDpLevels], role[kDpLevels], fill[kDpLevels];
};
constexpr int kDpSums = 2 + 3 * kDpLevels;

struct DpCursor {                // allocation cursors of the emit pass
  unsigned long long code;
  uint32_t thr, slots;
  uint32_t mat[kDpLevels], role[kDpLevels], fill[kDpLevels];
};

struct DpBases {                 // each level's first entry in the task tables
  uint32_t mat[kDpLevels], role[kDpLevels], fill[kDpLevels];
};

struct DpKB {                    // what the passes read of the knowledge base
  uint32_t n_concepts, n_sets, n_roles, n_data, W;
  uint32_t n_fixed;              // the first slot row: the all-zero row
  uint32_t n_dir;                // 2 R + 1
  const uint32_t* dir;           // [3][2R+1]: non-empty words, first heavy chunk, first heavy row
};

struct DpTables {
  ThrTask* thr;
  ThrGroup* thg;
  RegionTask* mat;
  RegionTask* roots;
  RoleTask* roles;
  FillTask* fills;               // fills[0]: the zero row
  uint32_t* code;
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

__global__ void __launch_bounds__(256)
k_dp_count(const hth_node* __restrict__ nodes, const uint32_t* __restrict__ offs,
           const uint32_t* __restrict__ kids, uint32_t n_nodes, uint32_t n_kids, uint32_t n_hyps, DpKB K,
           uint32_t* __restrict__ info, uint32_t* __restrict__ len, DpSummary* __restrict__ sum) {
  __shared__ uint32_t s_sum[kDpSums];
  __shared__ unsigned long long s_nhb[kDpLevels], s_nhc[kDpLevels], s_code;
  __shared__ uint32_t s_max[3];
  for (uint32_t i = threadIdx.x; i < kDpSums; i += blockDim.x) s_sum[i] = 0;
  if (threadIdx.x < kDpLevels) s_nhb[threadIdx.x] = s_nhc[threadIdx.x] = 0;
  if (threadIdx.x < 3) s_max[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_code = 0;
  __syncthreads();
  uint32_t* const s_thr = s_sum;
  uint32_t* const s_slots = s_sum + 1;
  uint32_t* const s_mat = s_sum + 2;
  uint32_t* const s_role = s_mat + kDpLevels;
  uint32_t* const s_fill = s_role + kDpLevels;
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
          atomicAdd(s_thr, 1u);
          atomicAdd(s_slots, 1u);
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
            atomicAdd(s_mat + lvl, 1u);
            atomicAdd(s_slots, 1u);
            atomicAdd(&s_code, (unsigned long long)len[c]);
            atomicMax(s_max + 1, (ci >> 8) & 255u);
          }
          const uint32_t rd = 2 * x.arg + x.inv;
          atomicAdd(s_role + lvl, 1u);
          atomicAdd(s_slots, 1u);
          if (dp_nwords(K, rd) < K.W) atomicAdd(s_fill + lvl, 1u);
          if (const uint32_t nb = dp_chunks(K, rd)) {
            atomicAdd(s_nhb + lvl, (unsigned long long)nb);
            atomicAdd(s_nhc + lvl, (unsigned long long)dp_heavy(K, rd));
          }
          atomicMax(s_max, lvl + 1);
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
    }
    if (ok) {   // the root's region, with coverage
      const uint32_t r = b + n - 1, ri = info[r];
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
  if (threadIdx.x < kDpLevels) {
    if (s_nhb[threadIdx.x]) atomicAdd(&sum->nhb[threadIdx.x], s_nhb[threadIdx.x]);
    if (s_nhc[threadIdx.x]) atomicAdd(&sum->nhc[threadIdx.x], s_nhc[threadIdx.x]);
  }
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
  for (uint32_t i = 0; i < n; ++i) {
    const hth_node x = nodes[b + i];
    if (dp_column(x.op)) {
      const uint32_t r = K.n_fixed + 1 + atomicAdd(&cur->slots, 1u);
      row[b + i] = r;
      const uint32_t t = atomicAdd(&cur->thr, 1u);
      ThrTask tt;
      tt.prop = x.arg;
      tt.cmp = x.op == HTH_DATA_GE ? 0u : x.op == HTH_DATA_LE ? 1u : 2u;
      tt.t = x.q.t;
      tt.out_row = r;
      T.thr[t] = tt;
      T.thg[t] = ThrGroup{x.arg, t, 1u, 0u};
    } else if (dp_role(x.op)) {
      const uint32_t r = K.n_fixed + 1 + atomicAdd(&cur->slots, 1u);
      row[b + i] = r;
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
        crow = K.n_fixed + 1 + atomicAdd(&cur->slots, 1u);
        const unsigned long long off = atomicAdd(&cur->code, (unsigned long long)len[c]);
        dp_program(K, nodes, kids, info, row, b, x.child, T.code + off);
        T.mat[B.mat[lvl] + atomicAdd(&cur->mat[lvl], 1u)] = RegionTask{(uint32_t)off, len[c], crow, kNone};
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
      RoleTask t;
      t.role = x.arg;
      t.inv = x.inv;
      t.child_row = crow;
      t.neg = neg;
      t.lo = lo;
      t.hi = hi;
      t.sat = hi == kInf ? lo : hi + 1;
      t.out_row = r;
      t.n_words = dp_nwords(K, rd);
      t.h_first = 0;                         // set by k_dp_heavy where heavy rows exist
      t.c_first = 0;
      t.hc0 = K.dir[K.n_dir + rd];
      t.hr0 = K.dir[2 * K.n_dir + rd];
      T.roles[B.role[lvl] + atomicAdd(&cur->role[lvl], 1u)] = t;
      if (t.n_words < K.W)
        T.fills[B.fill[lvl] + atomicAdd(&cur->fill[lvl], 1u)] = FillTask{r, lo == 0 ? 1u : 0u};
    }
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
k_dp_heavy(RoleTask* __restrict__ roles, DpBases B, const DpSummary* __restrict__ sum, DpKB K) {
  __shared__ uint32_t s_w[17];
  const uint32_t L = blockIdx.x;
  const uint32_t n = sum->role[L], base = B.role[L];
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
  char* buf = nullptr;                // per-node facts and rows, summary, cursors, direction table
  uint32_t* info = nullptr;
  uint32_t* len = nullptr;
  uint32_t* row = nullptr;
  hth::DpSummary* d_sum = nullptr;
  hth::DpCursor* d_cur = nullptr;
  hth::DpKB K{};
  hth::DpSummary sum{};
  hth::DpBases B{};
  uint32_t n_mat = 0, n_role = 0, n_fill = 0;
  uint64_t max_nhb = 0;
  size_t o_thr = 0, o_thg = 0, o_mat = 0, o_root = 0, o_role = 0, o_fill = 0, o_code = 0, o_part = 0,
         o_slot = 0, need = 0;
  hipEvent_t done = nullptr;          // recorded after each launch: destroy waits for it
  ~hth_dplan_s() {
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    if (buf) (void)hipFree(buf);
  }
};

namespace hth {
namespace {

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
    case DP_LEVELS: *code = HTH_E_UNSUPPORTED; return "role restrictions nested more than 16 deep";
    case DP_DEPTH: *code = HTH_E_UNSUPPORTED; return "boolean region nested deeper than 16 operand levels";
    case DP_NEST: *code = HTH_E_UNSUPPORTED; return "boolean region with more than 32 nested operators";
    default: *code = HTH_E_RANGE; return "region program longer than 2^30 instructions";
  }
}

}  // namespace
}  // namespace hth

extern "C" hth_status hth_dplan_create(hth_kb kb, const hth_node* d_nodes, uint32_t n_nodes,
                                       const uint32_t* d_hyp_node_offsets, uint32_t n_hyps,
                                       const uint32_t* d_children, uint32_t n_children, void* stream,
                                       hth_dplan* out, size_t* ws_bytes) {
  using namespace hth;
  if (!kb || !d_nodes || !d_hyp_node_offsets || !out || !ws_bytes) return fail(HTH_E_INVALID, "NULL argument");
  if (n_children && !d_children) return fail(HTH_E_INVALID, "children is NULL");
  if (n_hyps == 0) return fail(HTH_E_RANGE, "a plan needs at least one hypothesis");
  if (n_nodes > (1u << 24)) return fail(HTH_E_RANGE, "more than 2^24 nodes in one call");
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
  {
    std::lock_guard<std::mutex> g(kb->mu);
    p->sets = kb->sets;
    p->n_sets = kb->n_sets;
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
  }
  const size_t o_info = 0, o_len = align_up((size_t)n_nodes * 4, 256), o_row = o_len + o_len;
  const size_t o_sum = o_row + o_len, o_cur = o_sum + align_up(sizeof(DpSummary), 256);
  const size_t o_dir = o_cur + align_up(sizeof(DpCursor), 256);
  const size_t total = o_dir + dir.size() * 4;
  HTH_HIP(hipMalloc(reinterpret_cast<void**>(&p->buf), total));
  HTH_HIP(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
  p->info = reinterpret_cast<uint32_t*>(p->buf + o_info);
  p->len = reinterpret_cast<uint32_t*>(p->buf + o_len);
  p->row = reinterpret_cast<uint32_t*>(p->buf + o_row);
  p->d_sum = reinterpret_cast<DpSummary*>(p->buf + o_sum);
  p->d_cur = reinterpret_cast<DpCursor*>(p->buf + o_cur);
  p->K.dir = reinterpret_cast<const uint32_t*>(p->buf + o_dir);
  HTH_HIP(hipMemcpyAsync(p->buf + o_dir, dir.data(), dir.size() * 4, hipMemcpyHostToDevice, st));
  DpSummary init{};
  init.err = ~0ull;
  HTH_HIP(hipMemcpyAsync(p->d_sum, &init, sizeof(init), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_dp_count, dim3((n_hyps + 255) / 256), dim3(256), 0, st, d_nodes, d_hyp_node_offsets,
                     d_children, n_nodes, n_children, n_hyps, p->K, p->info, p->len, p->d_sum);
  HTH_HIP(hipGetLastError());
  HTH_HIP(hipMemcpyAsync(&p->sum, p->d_sum, sizeof(DpSummary), hipMemcpyDeviceToHost, st));
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
  if ((uint64_t)p->K.n_fixed + 1 + S.n_slots >= (1ull << 27)) return fail(HTH_E_RANGE, "too many bit rows");
  uint32_t fill = 1;                        // fills[0]: the zero row
  for (uint32_t L = 0; L < kDpLevels; ++L) {
    if (S.nhb[L] >= (1ull << 32) || S.nhc[L] >= (1ull << 32))
      return fail(HTH_E_RANGE, "heavy-row blocks of one level exceed 2^32");
    p->B.mat[L] = p->n_mat;
    p->B.role[L] = p->n_role;
    p->B.fill[L] = fill;
    p->n_mat += S.mat[L];
    p->n_role += S.role[L];
    fill += S.fill[L];
    p->max_nhb = std::max<uint64_t>(p->max_nhb, S.nhb[L]);
  }
  p->n_fill = fill;
  size_t at = 0;
  auto area = [&](size_t bytes) {
    const size_t a = at;
    at = align_up(at + bytes, 256);
    return a;
  };
  p->o_thr = area((size_t)S.n_thr * sizeof(ThrTask));
  p->o_thg = area((size_t)S.n_thr * sizeof(ThrGroup));
  p->o_mat = area((size_t)p->n_mat * sizeof(RegionTask));
  p->o_root = area((size_t)n_hyps * sizeof(RegionTask));
  p->o_role = area((size_t)p->n_role * sizeof(RoleTask));
  p->o_fill = area((size_t)fill * sizeof(FillTask));
  p->o_code = area((size_t)S.code * 4);
  p->o_part = area((size_t)p->max_nhb * 4);
  p->o_slot = area(((size_t)S.n_slots + 1) * kb->S * 8);
  p->need = at;
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
  role_attributes(kb);
  char* w = static_cast<char*>(ws);
  DpTables T;
  T.thr = reinterpret_cast<ThrTask*>(w + p.o_thr);
  T.thg = reinterpret_cast<ThrGroup*>(w + p.o_thg);
  T.mat = reinterpret_cast<RegionTask*>(w + p.o_mat);
  T.roots = reinterpret_cast<RegionTask*>(w + p.o_root);
  T.roles = reinterpret_cast<RoleTask*>(w + p.o_role);
  T.fills = reinterpret_cast<FillTask*>(w + p.o_fill);
  T.code = reinterpret_cast<uint32_t*>(w + p.o_code);
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
  const DpSummary& S = p.sum;
  Launcher Lc{kb, st};
  hth_status s = Lc.run(HTH_K_PLAN, 0.0, [&] {
    hipLaunchKernelGGL(k_dp_emit, dim3((p.n_hyps + 255) / 256), dim3(256), 0, st, p.nodes, p.offs, p.kids,
                       p.n_hyps, p.K, p.info, p.len, p.row, p.d_cur, p.B, T);
  });
  if (s) return s;
  bool heavy = false;
  for (uint32_t L = 0; L < S.levels; ++L) heavy |= S.nhc[L] > 0;
  if (heavy) {
    s = Lc.run(HTH_K_PLAN, 0.0, [&] {
      hipLaunchKernelGGL(k_dp_heavy, dim3(S.levels), dim3(1024), 0, st, T.roles, p.B, p.d_sum, p.K);
    });
    if (s) return s;
  }
  const uint32_t ftiles = (kb.S + 255) / 256;
  s = Lc.run(HTH_K_FILL, (double)kb.W * 8, [&] {   // the zero row
    hipLaunchKernelGGL(k_fill_rows, dim3(ftiles), dim3(256), 0, st, d, T.fills, ftiles);
  });
  if (s) return s;
  if (S.n_thr) {
    const uint32_t n = S.n_thr, bpt = std::max<uint32_t>(1, (kb.W + 127) / 128);
    const double bytes = n * (4.0 * kb.N + 8.0 * kb.W);
    s = split_launch(Lc, HTH_K_THRESHOLD, bytes, n, bpt, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
      hipLaunchKernelGGL(k_threshold, dim3(blocks), dim3(256), 0, st, d, T.thg + i0, T.thr, bpt);
    });
    if (s) return s;
  }
  for (uint32_t L = 0; L < S.levels; ++L) {
    s = launch_regions_n(Lc, d, T.mat + p.B.mat[L], T.code, S.mat[L], (int)S.mat_depth, 0.0);
    if (s) return s;
    if (S.fill[L]) {
      const uint32_t n = S.fill[L];
      s = split_launch(Lc, HTH_K_FILL, (double)n * kb.W * 8, n, ftiles, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_fill_rows, dim3(blocks), dim3(256), 0, st, d, T.fills + p.B.fill[L] + i0, ftiles);
      });
      if (s) return s;
    }
    const RoleTask* rol = T.roles + p.B.role[L];
    s = launch_roles_n(Lc, d, rol, S.role[L], 0.0);
    if (s) return s;
    if (S.nhc[L]) {
      uint32_t* partial = reinterpret_cast<uint32_t*>(w + p.o_part);
      const uint32_t nt = S.role[L];
      s = split_launch(Lc, HTH_K_ROLE, 0.0, S.nhb[L], 1, 256, [&](uint32_t b0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_role_heavy, dim3(blocks), dim3(256), 0, st, d, rol, nt, b0, partial);
      });
      if (s) return s;
      s = split_launch(Lc, HTH_K_ROLE, 0.0, S.nhc[L], 1, 256, [&](uint32_t i0, uint32_t, uint32_t blocks) {
        hipLaunchKernelGGL(k_role_heavy_fix, dim3(blocks), dim3(256), 0, st, d, rol, nt, i0, partial);
      });
      if (s) return s;
    }
  }
  s = launch_regions_n(Lc, d, T.roots, T.code, p.n_hyps, (int)S.root_depth, 0.0);
  if (s) return s;
  HTH_HIP(hipEventRecord(p.done, st));
  return HTH_OK;
}

extern "C" hth_status hth_dplan_destroy(hth_dplan plan) {
  delete plan;
  return HTH_OK;
}
