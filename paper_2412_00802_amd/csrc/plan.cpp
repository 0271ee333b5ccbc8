// Plan compiler: validation, canonicalisation, hash-consing across the batch,
// role-nesting levels, row assignment and region bytecode.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>

namespace hth {
namespace {

constexpr uint32_t kInf = 0xFFFFFFFFu;

struct CNode {
  uint8_t op = 0, inv = 0;
  uint32_t arg = 0, q = 0;
  uint32_t a = kNone;            // NOT / role child
  uint32_t kid_off = 0, kid_n = 0;  // AND / OR children (canonical ids, sorted)
};

inline uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  return h * 0xFF51AFD7ED558CCDull;
}

class Dag {
 public:
  std::vector<CNode> nodes;
  std::vector<uint32_t> kids;

  Dag() { table_.assign(1 << 12, kNone); }

  uint32_t top() { return leaf(HTH_TOP, 0, 0, 0); }
  uint32_t bot() { return leaf(HTH_BOT, 0, 0, 0); }
  uint32_t leaf(uint8_t op, uint8_t inv, uint32_t arg, uint32_t q) {
    CNode n;
    n.op = op;
    n.inv = inv;
    n.arg = arg;
    n.q = q;
    return intern(n, nullptr, 0);
  }
  uint32_t mk_not(uint32_t c) {
    const CNode& x = nodes[c];
    if (x.op == HTH_NOT) return x.a;
    if (x.op == HTH_TOP) return bot();
    if (x.op == HTH_BOT) return top();
    CNode n;
    n.op = HTH_NOT;
    n.a = c;
    return intern(n, nullptr, 0);
  }
  uint32_t mk_role(uint8_t op, uint8_t inv, uint32_t r, uint32_t q, uint32_t c) {
    if (op == HTH_ATLEAST && q == 0) return top();
    CNode n;
    n.op = op;
    n.inv = inv;
    n.arg = r;
    n.q = (op == HTH_EXISTS || op == HTH_FORALL) ? 0 : q;
    n.a = c;
    return intern(n, nullptr, 0);
  }
  uint32_t mk_nary(uint8_t op, std::vector<uint32_t>& in) {
    const uint8_t ident = op == HTH_AND ? HTH_TOP : HTH_BOT;
    const uint8_t absorb = op == HTH_AND ? HTH_BOT : HTH_TOP;
    tmp_.clear();
    for (uint32_t c : in) {
      const CNode& x = nodes[c];
      if (x.op == op) {
        for (uint32_t j = 0; j < x.kid_n; ++j) tmp_.push_back(kids[x.kid_off + j]);
      } else {
        tmp_.push_back(c);
      }
    }
    std::vector<uint32_t> v;
    v.reserve(tmp_.size());
    for (uint32_t c : tmp_) {
      uint8_t o = nodes[c].op;
      if (o == absorb) return c;
      if (o == ident) continue;
      v.push_back(c);
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    if (v.empty()) return op == HTH_AND ? top() : bot();
    if (v.size() == 1) return v[0];
    CNode n;
    n.op = op;
    return intern(n, v.data(), (uint32_t)v.size());
  }

 private:
  std::vector<uint32_t> table_;
  std::vector<uint32_t> tmp_;

  static uint64_t hash_of(const CNode& n, const uint32_t* k, uint32_t kn) {
    uint64_t h = mix(0x1234567ull, n.op | (uint64_t)n.inv << 8);
    h = mix(h, n.arg);
    h = mix(h, n.q);
    h = mix(h, n.a);
    for (uint32_t i = 0; i < kn; ++i) h = mix(h, k[i]);
    return h;
  }
  bool same(const CNode& x, const CNode& n, const uint32_t* k, uint32_t kn) const {
    if (x.op != n.op || x.inv != n.inv || x.arg != n.arg || x.q != n.q || x.a != n.a ||
        x.kid_n != kn)
      return false;
    return kn == 0 || std::memcmp(&kids[x.kid_off], k, kn * 4) == 0;
  }
  uint32_t intern(CNode n, const uint32_t* k, uint32_t kn) {
    if (nodes.size() * 2 >= table_.size()) rehash();
    uint64_t h = hash_of(n, k, kn);
    size_t mask = table_.size() - 1;
    size_t i = h & mask;
    while (table_[i] != kNone) {
      if (same(nodes[table_[i]], n, k, kn)) return table_[i];
      i = (i + 1) & mask;
    }
    n.kid_off = (uint32_t)kids.size();
    n.kid_n = kn;
    kids.insert(kids.end(), k, k + kn);
    uint32_t id = (uint32_t)nodes.size();
    nodes.push_back(n);
    table_[i] = id;
    return id;
  }
  void rehash() {
    std::vector<uint32_t> t(table_.size() * 2, kNone);
    size_t mask = t.size() - 1;
    for (uint32_t id = 0; id < nodes.size(); ++id) {
      const CNode& n = nodes[id];
      size_t i = hash_of(n, kids.data() + n.kid_off, n.kid_n) & mask;
      while (t[i] != kNone) i = (i + 1) & mask;
      t[i] = id;
    }
    table_.swap(t);
  }
};

}  // namespace

// The cache: a persistent DAG of every subexpression seen, and rows kept in
// least-recently-used order (rows[] is a doubly linked list through prev/next,
// most recent at head).  A batch stamps every row it reads or writes, and
// only rows stamped by earlier batches are evicted.
struct SubexprCache {
  static constexpr uint32_t kMaxNodes = 1u << 24;   // the DAG is flushed beyond this
  Dag g;
  struct Row {
    uint32_t gid = kNone;
    uint64_t stamp = 0;
    uint32_t prev = kNone, next = kNone;
  };
  std::vector<Row> rows;
  std::unordered_map<uint32_t, uint32_t> row_of;   // DAG id -> row
  uint32_t head = kNone, tail = kNone;
  uint64_t batch = 0;
  std::vector<uint32_t> admitted_now;   // rows given out by the batch being compiled
  CacheCounters cnt;

  explicit SubexprCache(uint32_t n) : rows(n) {
    for (uint32_t i = 0; i < n; ++i) push_front(i);
    cnt.rows = n;
  }
  void unlink(uint32_t i) {
    Row& r = rows[i];
    if (r.prev != kNone) rows[r.prev].next = r.next; else head = r.next;
    if (r.next != kNone) rows[r.next].prev = r.prev; else tail = r.prev;
    r.prev = r.next = kNone;
  }
  void push_front(uint32_t i) {
    rows[i].prev = kNone;
    rows[i].next = head;
    if (head != kNone) rows[head].prev = i;
    head = i;
    if (tail == kNone) tail = i;
  }
  void touch(uint32_t i) {
    rows[i].stamp = batch;
    unlink(i);
    push_front(i);
  }
  void flush() {
    g = Dag();
    row_of.clear();
    for (Row& r : rows) r.gid = kNone;
    cnt.entries = 0;
  }
  // a new batch: the DAG is flushed when it has grown past its bound
  void begin() {
    ++batch;
    ++cnt.batches;
    admitted_now.clear();
    if (g.nodes.size() > kMaxNodes) flush();
  }
  uint32_t lookup(uint32_t gid) const {
    auto it = row_of.find(gid);
    return it == row_of.end() ? kNone : it->second;
  }
  // the least recently used row not stamped by this batch, for `gid`
  uint32_t admit(uint32_t gid) {
    if (tail == kNone || rows[tail].stamp == batch) return kNone;
    const uint32_t i = tail;
    if (rows[i].gid != kNone) {
      row_of.erase(rows[i].gid);
      ++cnt.evictions;
      --cnt.entries;
    }
    rows[i].gid = gid;
    row_of[gid] = i;
    ++cnt.entries;
    ++cnt.admitted;
    touch(i);
    admitted_now.push_back(i);
    return i;
  }
  void rollback() {
    for (uint32_t i : admitted_now) {
      if (rows[i].gid != kNone) {
        row_of.erase(rows[i].gid);
        --cnt.entries;
      }
      rows[i].gid = kNone;
      rows[i].stamp = 0;
      unlink(i);
      // a freed row goes to the tail: the next one to be given out
      rows[i].prev = tail;
      rows[i].next = kNone;
      if (tail != kNone) rows[tail].next = i; else head = i;
      tail = i;
    }
    cnt.admitted -= admitted_now.size();
    admitted_now.clear();
  }
};

SubexprCache* cache_new(uint32_t n_rows) { return new (std::nothrow) SubexprCache(n_rows); }
void cache_delete(SubexprCache* c) { delete c; }
CacheCounters cache_counters(const SubexprCache* c) { return c->cnt; }
void cache_rollback(SubexprCache* c) { c->rollback(); }

namespace {

inline bool is_role(uint8_t op) { return op >= HTH_EXISTS && op <= HTH_EXACTLY; }
inline bool is_column(uint8_t op) { return op == HTH_DATA_GE || op == HTH_DATA_LE || op == HTH_DATA_EQ; }
inline bool is_numeric(uint8_t op) { return op == HTH_NUM_GE || op == HTH_NUM_LE || op == HTH_NUM_EQ; }
inline bool is_string(uint8_t op) { return op == HTH_STR_EQ || op == HTH_STR_CONTAINS; }
inline bool is_data(uint8_t op) { return is_column(op) || is_numeric(op) || is_string(op); }
inline bool is_leaflike(uint8_t op) {
  return op == HTH_ATOM || op == HTH_SET || is_data(op) || is_role(op);
}

struct Compiler {
  const hth_kb_s& kb;
  Dag dag;
  std::vector<uint32_t> roots;
  // per canonical node
  std::vector<int32_t> height;   // role nesting below (and including) the node, -1 = none
  std::vector<uint8_t> live;
  std::vector<uint32_t> row;     // bit row of data / role / materialised nodes
  std::vector<int32_t> depth;    // stack depth of the node's region program
  uint32_t n_slots = 0;
  uint32_t zero_row = kNone;

  explicit Compiler(const hth_kb_s& k) : kb(k) {}

  hth_status add_hypothesis(const hth_node* nd, uint32_t nn, const uint32_t* children,
                            uint32_t n_children, uint32_t h) {
    if (nn == 0) return fail(HTH_E_PLAN, "hypothesis " + std::to_string(h) + " has no nodes");
    std::vector<uint32_t> map(nn);
    std::vector<uint32_t> ks;
    const hth_kb_desc& d = kb.d;
    for (uint32_t i = 0; i < nn; ++i) {
      const hth_node& x = nd[i];
      auto bad = [&](hth_status c, const char* why) {
        return fail(c, "hypothesis " + std::to_string(h) + " node " + std::to_string(i) + ": " + why);
      };
      switch (x.op) {
        case HTH_TOP: map[i] = dag.top(); break;
        case HTH_BOT: map[i] = dag.bot(); break;
        case HTH_ATOM:
          if (x.arg >= d.n_concepts) return bad(HTH_E_RANGE, "concept id out of range");
          map[i] = dag.leaf(HTH_ATOM, 0, x.arg, 0);
          break;
        case HTH_SET:
          if (x.arg >= kb.n_sets) return bad(HTH_E_RANGE, "set row outside the registered set table");
          map[i] = dag.leaf(HTH_SET, 0, x.arg, 0);
          break;
        case HTH_NOT:
          if (x.child >= i) return bad(HTH_E_PLAN, "child index not before its parent");
          map[i] = dag.mk_not(map[x.child]);
          break;
        case HTH_AND:
        case HTH_OR: {
          if ((uint64_t)x.child + x.arity > n_children)
            return bad(HTH_E_RANGE, "children range outside the children array");
          ks.clear();
          for (uint32_t j = 0; j < x.arity; ++j) {
            uint32_t c = children[x.child + j];
            if (c >= i) return bad(HTH_E_PLAN, "child index not before its parent");
            ks.push_back(map[c]);
          }
          map[i] = dag.mk_nary(x.op, ks);
          break;
        }
        case HTH_EXISTS:
        case HTH_FORALL:
        case HTH_ATLEAST:
        case HTH_ATMOST:
        case HTH_EXACTLY:
          if (x.arg >= d.n_roles) return bad(HTH_E_RANGE, "role id out of range");
          if (x.inv > 1) return bad(HTH_E_INVALID, "inv must be 0 or 1");
          if (x.child >= i) return bad(HTH_E_PLAN, "child index not before its parent");
          if (x.op >= HTH_ATLEAST && x.q.n > 0x7FFFFFFFu) return bad(HTH_E_RANGE, "n > 2^31-1");
          map[i] = dag.mk_role(x.op, x.inv, x.arg, x.q.n, map[x.child]);
          break;
        case HTH_DATA_GE:
        case HTH_DATA_LE:
        case HTH_DATA_EQ:
        case HTH_NUM_GE:
        case HTH_NUM_LE:
        case HTH_NUM_EQ: {
          if (is_column(x.op) && x.arg >= d.n_data) return bad(HTH_E_RANGE, "property id out of range");
          if (is_numeric(x.op) && x.arg >= kb.n_num)
            return bad(HTH_E_RANGE, "numeric concrete role id outside the registered roles");
          if (std::isnan(x.q.t)) return bad(HTH_E_INVALID, "threshold is NaN");
          uint32_t bits;
          std::memcpy(&bits, &x.q.t, 4);
          map[i] = dag.leaf(x.op, 0, x.arg, bits);
          break;
        }
        case HTH_STR_EQ:
        case HTH_STR_CONTAINS:
          if (x.arg >= kb.n_str) return bad(HTH_E_RANGE, "string concrete role id outside the registered roles");
          if (x.op == HTH_STR_EQ && x.q.n == 0xFFFFFFFFu) {   // a string absent from the dictionary
            map[i] = dag.bot();
            break;
          }
          if (x.op == HTH_STR_EQ && x.q.n >= kb.n_strings) return bad(HTH_E_RANGE, "string id out of range");
          if (x.op == HTH_STR_CONTAINS && x.q.n >= kb.n_patterns)
            return bad(HTH_E_RANGE, "pattern id outside the registered patterns");
          map[i] = dag.leaf(x.op, 0, x.arg, x.q.n);
          break;
        default:
          return bad(HTH_E_INVALID, "unknown op");
      }
    }
    roots.push_back(map[nn - 1]);
    return HTH_OK;
  }

  uint32_t new_row() { return kb.d.n_concepts + kb.n_sets + n_slots++; }

  int32_t region_depth(uint32_t v) {
    if (depth[v] >= 0) return depth[v];
    const CNode& n = dag.nodes[v];
    int32_t r = 1;
    if (n.op == HTH_NOT) {
      r = is_leaflike(dag.nodes[n.a].op) ? 1 : region_depth(n.a);
    } else if (n.op == HTH_AND || n.op == HTH_OR) {
      std::vector<int32_t> ds;
      for (uint32_t j = 0; j < n.kid_n; ++j) ds.push_back(region_depth(dag.kids[n.kid_off + j]));
      std::sort(ds.rbegin(), ds.rend());
      r = 0;
      for (size_t j = 0; j < ds.size(); ++j) r = std::max<int32_t>(r, ds[j] + (j ? 1 : 0));
    }
    depth[v] = r;
    return r;
  }

  uint32_t leaf_row(uint32_t v) const {
    const CNode& n = dag.nodes[v];
    if (n.op == HTH_ATOM) return n.arg;
    if (n.op == HTH_SET) return kb.d.n_concepts + n.arg;
    return row[v];
  }

  void emit(uint32_t v, std::vector<uint32_t>& code) {
    const CNode& n = dag.nodes[v];
    switch (n.op) {
      case HTH_TOP: code.push_back(rp_ins(RP_TOP, 0, 0)); return;
      case HTH_BOT: code.push_back(rp_ins(RP_BOT, 0, 0)); return;
      case HTH_NOT:
        if (is_leaflike(dag.nodes[n.a].op)) {
          code.push_back(rp_ins(RP_LEAF, 1, leaf_row(n.a)));
        } else {
          emit(n.a, code);
          code.push_back(rp_ins(RP_NOT, 0, 0));
        }
        return;
      case HTH_AND:
      case HTH_OR: {
        std::vector<uint32_t> ks(dag.kids.begin() + n.kid_off, dag.kids.begin() + n.kid_off + n.kid_n);
        std::stable_sort(ks.begin(), ks.end(),
                         [&](uint32_t a, uint32_t b) { return region_depth(a) > region_depth(b); });
        emit(ks[0], code);
        for (size_t j = 1; j < ks.size(); ++j) {
          emit(ks[j], code);
          code.push_back(rp_ins(n.op == HTH_AND ? RP_AND : RP_OR, 0, 0));
        }
        return;
      }
      default:
        code.push_back(rp_ins(RP_LEAF, 0, leaf_row(v)));
        return;
    }
  }

  hth_status program(uint32_t v, std::vector<uint32_t>& code, uint32_t& off, uint32_t& len) {
    if (region_depth(v) > kStackDepth)
      return fail(HTH_E_UNSUPPORTED, "boolean region nested deeper than 16 operand levels");
    off = (uint32_t)code.size();
    emit(v, code);
    len = (uint32_t)code.size() - off;
    return HTH_OK;
  }

  // The batch's canonical nodes in the cache's persistent DAG (children first,
  // so each node's children already have their ids there).
  void cache_ids(SubexprCache& C, std::vector<uint32_t>& gid) {
    gid.assign(dag.nodes.size(), kNone);
    std::vector<uint32_t> ks;
    for (uint32_t v = 0; v < dag.nodes.size(); ++v) {
      const CNode& n = dag.nodes[v];
      if (n.op == HTH_NOT) gid[v] = C.g.mk_not(gid[n.a]);
      else if (is_role(n.op)) gid[v] = C.g.mk_role(n.op, n.inv, n.arg, n.q, gid[n.a]);
      else if (n.op == HTH_AND || n.op == HTH_OR) {
        ks.clear();
        for (uint32_t j = 0; j < n.kid_n; ++j) ks.push_back(gid[dag.kids[n.kid_off + j]]);
        gid[v] = C.g.mk_nary(n.op, ks);
      } else {
        gid[v] = C.g.leaf(n.op, n.inv, n.arg, n.q);
      }
    }
  }

  hth_status build(const PlanOptions& opt, Plan& P) {
    const size_t nv = dag.nodes.size();
    height.assign(nv, -1);
    live.assign(nv, 0);
    row.assign(nv, kNone);
    depth.assign(nv, -1);
    // cross-batch cache: a role node whose subexpression holds a row is a
    // leaf of this plan (read from that row); its subtree is not evaluated
    SubexprCache* C = opt.cache;
    std::vector<uint32_t> gid, hit_row(nv, kNone);
    if (C) {
      C->begin();
      cache_ids(*C, gid);
      for (uint32_t v = 0; v < nv; ++v)
        if (is_role(dag.nodes[v].op)) hit_row[v] = C->lookup(gid[v]);
    }
    for (uint32_t v = 0; v < nv; ++v) {
      const CNode& n = dag.nodes[v];
      if (hit_row[v] != kNone) continue;           // a cached row: no role below it to run
      if (n.op == HTH_NOT) height[v] = height[n.a];
      else if (n.op == HTH_AND || n.op == HTH_OR) {
        int32_t h = -1;
        for (uint32_t j = 0; j < n.kid_n; ++j) h = std::max(h, height[dag.kids[n.kid_off + j]]);
        height[v] = h;
      } else if (is_role(n.op)) {
        height[v] = height[n.a] + 1;
      }
    }
    for (uint32_t r : roots) live[r] = 1;
    for (size_t i = nv; i-- > 0;) {
      if (!live[i] || hit_row[i] != kNone) continue;
      const CNode& n = dag.nodes[i];
      if (n.a != kNone) live[n.a] = 1;
      for (uint32_t j = 0; j < n.kid_n; ++j) live[dag.kids[n.kid_off + j]] = 1;
    }
    // the rows this batch reads stay until it has run; live role nodes without
    // one are given rows of their own while the cache has rows older than this
    // batch (their results then stay for later batches)
    std::vector<uint8_t> in_cache(nv, 0);
    if (C) {
      // every row read is stamped first, so that no admission below evicts it
      for (uint32_t v = 0; v < nv; ++v) {
        if (!live[v] || hit_row[v] == kNone) continue;
        C->touch(hit_row[v]);
        C->cnt.hits++;
        row[v] = kb.d.n_concepts + hit_row[v];
      }
      for (uint32_t v = 0; v < nv; ++v) {
        if (!live[v] || !is_role(dag.nodes[v].op) || hit_row[v] != kNone) continue;
        C->cnt.misses++;
        const uint32_t r = C->admit(gid[v]);
        if (r != kNone) {
          row[v] = kb.d.n_concepts + r;
          in_cache[v] = 1;
        }
      }
    }
    // a role node that is the root of one hypothesis and read by no other node
    // needs no row when it runs in a shared pass: the pass adds its coverage
    // into that hypothesis's counts, and the hypothesis has no root region
    std::vector<uint8_t> used(nv, 0);
    std::vector<uint32_t> root_uses(nv, 0), root_hyp(nv, kNone);
    for (size_t i = 0; i < nv; ++i) {
      if (!live[i]) continue;
      const CNode& n = dag.nodes[i];
      if (n.a != kNone) used[n.a] = 1;
      for (uint32_t j = 0; j < n.kid_n; ++j) used[dag.kids[n.kid_off + j]] = 1;
    }
    for (uint32_t h = 0; h < roots.size(); ++h) {
      root_uses[roots[h]]++;
      root_hyp[roots[h]] = h;
    }
    std::vector<uint8_t> covered_by_pass(roots.size(), 0);
    int32_t max_level = -1;
    for (uint32_t v = 0; v < nv; ++v) {
      if (!live[v]) continue;
      const CNode& n = dag.nodes[v];
      if (is_column(n.op)) {
        row[v] = new_row();
        ThrTask t;
        t.prop = n.arg;
        t.cmp = n.op == HTH_DATA_GE ? 0 : n.op == HTH_DATA_LE ? 1 : 2;
        std::memcpy(&t.t, &n.q, 4);
        t.out_row = row[v];
        P.thr.push_back(t);
      } else if (is_numeric(n.op)) {
        row[v] = new_row();
        NumTask t{};
        t.role = n.arg;
        t.cmp = n.op == HTH_NUM_GE ? 0 : n.op == HTH_NUM_LE ? 1 : 2;
        std::memcpy(&t.t, &n.q, 4);
        t.out_row = row[v];
        P.num.push_back(t);
      } else if (is_string(n.op)) {
        row[v] = new_row();
        StrTask t{};
        t.role = n.arg;
        t.kind = n.op == HTH_STR_CONTAINS ? 1 : 0;
        std::memcpy(&t.q, &n.q, 4);
        t.out_row = row[v];
        P.str.push_back(t);
      } else if (is_role(n.op) && hit_row[v] == kNone) {
        if (!in_cache[v]) row[v] = new_row();
        max_level = std::max(max_level, height[v]);
        P.n_role_nodes++;
      }
    }
    P.levels.assign(max_level + 1, PlanLevel());
    // role children: resolve to (row, negation), materialising compound children
    std::vector<uint32_t> matrow(nv, kNone);
    struct Pending { uint32_t v, child_row, neg; };
    std::vector<std::vector<Pending>> per_level(max_level + 1);
    for (uint32_t v = 0; v < nv; ++v) {
      if (!live[v] || !is_role(dag.nodes[v].op) || hit_row[v] != kNone) continue;
      const CNode& n = dag.nodes[v];
      const uint32_t c = n.a;
      const CNode& cn = dag.nodes[c];
      uint32_t crow, neg = 0;
      if (cn.op == HTH_TOP || cn.op == HTH_BOT) {
        if (zero_row == kNone) {
          zero_row = new_row();
          RegionTask z;
          z.code_off = (uint32_t)P.code.size();
          P.code.push_back(rp_ins(RP_BOT, 0, 0));
          z.code_len = 1;
          z.out_row = zero_row;
          z.cover = kNone;
          P.levels[0].mat.push_back(z);
        }
        crow = zero_row;
        neg = cn.op == HTH_TOP;
      } else if (is_leaflike(cn.op)) {
        crow = leaf_row(c);
      } else if (cn.op == HTH_NOT && is_leaflike(dag.nodes[cn.a].op)) {
        crow = leaf_row(cn.a);
        neg = 1;
      } else {
        if (matrow[c] == kNone) {
          matrow[c] = new_row();
          RegionTask m;
          hth_status s = program(c, P.code, m.code_off, m.code_len);
          if (s) return s;
          m.out_row = matrow[c];
          m.cover = kNone;
          P.levels[height[v]].mat.push_back(m);
        }
        crow = matrow[c];
      }
      per_level[height[v]].push_back({v, crow, neg});
    }
    // role tasks, grouped per (role, direction) when the bucket is large
    for (int32_t L = 0; L <= max_level; ++L) {
      PlanLevel& PL = P.levels[L];
      auto& items = per_level[L];
      std::stable_sort(items.begin(), items.end(), [&](const Pending& a, const Pending& b) {
        const CNode& x = dag.nodes[a.v];
        const CNode& y = dag.nodes[b.v];
        return x.arg != y.arg ? x.arg < y.arg : x.inv < y.inv;
      });
      size_t i = 0;
      while (i < items.size()) {
        size_t j = i;
        const CNode& first = dag.nodes[items[i].v];
        while (j < items.size() && dag.nodes[items[j].v].arg == first.arg &&
               dag.nodes[items[j].v].inv == first.inv)
          ++j;
        // nodes a shared pass can decide (see GroupTask) form groups when the
        // bucket is large enough; the rest run alone
        std::vector<Pending> solo, grp;
        for (size_t q = i; q < j; ++q) {
          const CNode& n = dag.nodes[items[q].v];
          const bool groupable = n.op == HTH_EXISTS || n.op == HTH_FORALL ||
                                 (n.op == HTH_ATLEAST ? n.q <= kGroupMaxCount : n.q < kGroupMaxCount);
          (groupable ? grp : solo).push_back(items[q]);
        }
        if (grp.size() < bucket_min(kb, 2 * first.arg + first.inv, opt.group_min)) {
          solo.insert(solo.end(), grp.begin(), grp.end());
          grp.clear();
        }
        auto predicate = [&](const Pending& it, uint32_t& lo, uint32_t& hi, uint32_t& neg) {
          const CNode& n = dag.nodes[it.v];
          neg = it.neg;
          switch (n.op) {
            case HTH_EXISTS: lo = 1; hi = kInf; break;
            case HTH_FORALL: lo = 0; hi = 0; neg ^= 1; break;
            case HTH_ATLEAST: lo = n.q; hi = kInf; break;
            case HTH_ATMOST: lo = 0; hi = n.q; break;
            default: lo = n.q; hi = n.q; break;
          }
        };
        for (const Pending& it : solo) {
          const CNode& n = dag.nodes[it.v];
          RoleTask t;
          t.role = n.arg;
          t.inv = n.inv;
          t.child_row = it.child_row;
          predicate(it, t.lo, t.hi, t.neg);
          t.sat = t.hi == kInf ? t.lo : t.hi + 1;
          t.out_row = row[it.v];
          PL.roles.push_back(t);
        }
        const size_t gk = std::max<uint32_t>(1, std::min<uint32_t>(opt.group_k, kMaxK));
        for (size_t g0 = 0; g0 < grp.size(); g0 += gk) {
          const size_t g1 = std::min(grp.size(), g0 + gk);
          GroupTask gt{};
          gt.role = first.arg;
          gt.inv = first.inv;
          gt.k = (uint32_t)(g1 - g0);
          gt.first = (uint32_t)PL.members.size();
          for (size_t q = g0; q < g1; ++q) {
            GroupMember m{};
            predicate(grp[q], m.lo, m.hi, m.neg);
            m.sat = m.hi == kInf ? m.lo : m.hi + 1;
            m.child_row = grp[q].child_row;
            const uint32_t v = grp[q].v;
            m.out_row = row[v];
            m.cover = kNone;
            if (!opt.instances && !used[v] && root_uses[v] == 1 && !in_cache[v]) {
              m.out_row = kNone;
              m.cover = root_hyp[v];
              covered_by_pass[root_hyp[v]] = 1;
            }
            const uint32_t jbit = (uint32_t)(q - g0);
            for (uint32_t v = 0; v <= kGroupMaxCount; ++v) {
              const bool ok = v < kGroupMaxCount ? (m.lo <= v && v <= m.hi)
                                                 : (m.hi == kInf && m.lo <= kGroupMaxCount);
              if (ok) gt.acc[v] |= 1ull << jbit;
            }
            PL.members.push_back(m);
          }
          PL.groups.push_back(gt);
        }
        i = j;
      }
    }
    // roots with coverage
    for (uint32_t h = 0; h < roots.size(); ++h) {
      if (covered_by_pass[h]) continue;
      RegionTask t;
      hth_status s = program(roots[h], P.code, t.code_off, t.code_len);
      if (s) return s;
      t.out_row = opt.instances ? kInstances : kNone;
      t.cover = h;
      P.roots.push_back(t);
    }
    P.n_slots = n_slots;
    P.sets = kb.sets;
    P.n_sets = kb.n_sets;
    if (!P.num.empty()) {
      P.num_roff = kb.num_roff;
      P.num_val = kb.num_val;
      P.num_heavy_rows = kb.num_heavy_rows;
      P.num_heavy_chunks = kb.num_heavy_chunks;
      P.num_chunk_first = kb.num_chunk_first;
      P.num_bounds = kb.num_bounds;
    }
    if (!P.str.empty()) {
      P.str_roff = kb.str_roff;
      P.str_ids = kb.str_ids;
      P.str_heavy_rows = kb.str_heavy_rows;
      P.str_heavy_chunks = kb.str_heavy_chunks;
      P.str_chunk_first = kb.str_chunk_first;
      P.str_bounds = kb.str_bounds;
      P.dict_off = kb.dict_off;
      P.dict_chars = kb.dict_chars;
      P.pat_off = kb.pat_off;
      P.pat_chars = kb.pat_chars;
      P.n_strings = kb.n_strings;
    }
    P.n_canonical = (uint32_t)nv;
    return HTH_OK;
  }
};

}  // namespace

hth_status compile_plan(const hth_kb_s& kb, const hth_node* nodes, const uint32_t* hyp_off,
                        uint32_t n_hyps, const uint32_t* children, uint32_t n_children,
                        const PlanOptions& opt, Plan& out) {
  out = Plan();
  Compiler c(kb);
  for (uint32_t h = 0; h < n_hyps; ++h) {
    uint32_t b = hyp_off[h], e = hyp_off[h + 1];
    if (e < b) return fail(HTH_E_INVALID, "hyp_node_offsets decrease");
    hth_status s = c.add_hypothesis(nodes + b, e - b, children, n_children, h);
    if (s) return s;
    out.n_input_nodes += e - b;
    // row ids (concepts < 2^26, set rows < 2^24, one slot per node) fit the
    // 27-bit argument of the region bytecode
    if (out.n_input_nodes > (1u << 24)) return fail(HTH_E_RANGE, "more than 2^24 nodes in one call");
  }
  return c.build(opt, out);
}

}  // namespace hth
