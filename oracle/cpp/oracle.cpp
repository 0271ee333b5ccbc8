// Plain CPU oracle for exact ALCQI(D) hypothesis evaluation, in C++ with
// OpenMP over hypotheses.  TEST INFRASTRUCTURE ONLY: the test suite and the
// benchmark's CPU-baseline leg load it; the library's compute path never
// does, and this file shares no code, header or table with it.
//
// What it computes is the plain set semantics of the constructs HT-HEDL
// evaluates (Section 3.2; coverage as in Algorithm 15), under the closed-world
// and unique-name assumptions of Section 3.1.  Memberships are one byte per
// individual, as in the paper's concepts matrix (Section 3.1).  Each
// hypothesis is evaluated recursively: every sub-result is a full membership
// vector over all N individuals; there is no plan, no sharing of
// sub-results and no reordering.  Readings of the paper (the same as the
// Python oracle's):
//  - at-most n is the textbook one, {x : cnt(x) <= n}: individuals with no
//    matching successor belong to it;
//  - a role is a set of assertions, so counting assertions (Algorithms 7/8)
//    and counting distinct successors agree;
//  - the inverse role swaps subject and object of every assertion (end of
//    Section 3.2.2): its count is taken over the same assertions with the
//    roles of the two ends exchanged, so no transposed table is built;
//  - empty conjunction = top, empty disjunction = bottom;
//  - a data restriction holds when the individual has a value (not NaN) and
//    the float32 comparison holds (Section 3.2.3, Algorithms 9/10).
//
// Hypotheses arrive as prefix token streams (int64), one per hypothesis:
//   TOP 0 | BOT 1 | ATOM 2 a | NOT 3 C | AND 4 k C1..Ck | OR 5 k C1..Ck
//   EXISTS 6 r inv C | FORALL 7 r inv C
//   ATLEAST 8 n r inv C | ATMOST 9 n r inv C | EXACTLY 10 n r inv C
//   DGE 11 p bits | DLE 12 p bits | DEQ 13 p bits   (bits: the float32 threshold)
#include <omp.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <vector>

namespace {

enum : int64_t {
  TOP = 0, BOT = 1, ATOM = 2, NOT = 3, AND = 4, OR = 5, EXISTS = 6, FORALL = 7,
  ATLEAST = 8, ATMOST = 9, EXACTLY = 10, DGE = 11, DLE = 12, DEQ = 13
};

struct KB {
  int64_t n = 0;
  int32_t n_concepts = 0, n_roles = 0, n_data = 0;
  std::vector<uint8_t> concepts;   // [C][N], one byte per membership
  const int64_t* off = nullptr;    // [R][N+1], absolute into tg (caller's)
  const int32_t* tg = nullptr;     // (caller's)
  const float* data = nullptr;     // [D][N] (caller's)
  std::vector<uint8_t> pos, neg;   // [N]
};

// Per-thread scratch: a stack of membership vectors and one count vector.
struct Scratch {
  int64_t n;
  std::vector<std::unique_ptr<uint8_t[]>> stack;
  std::vector<uint32_t> cnt;
  size_t top = 0;
  explicit Scratch(int64_t n_) : n(n_), cnt(n_) {}
  uint8_t* push() {
    if (top == stack.size()) stack.emplace_back(new uint8_t[n > 0 ? n : 1]);
    return stack[top++].get();
  }
  void pop() { --top; }
};

struct Bad {};   // malformed token stream

struct Eval {
  const KB& kb;
  Scratch& s;
  const int64_t* t;
  int64_t len, pos = 0;

  int64_t next() {
    if (pos >= len) throw Bad{};
    return t[pos++];
  }

  // cnt(x) = #{assertions (x, y) of role r (subject and object swapped when
  // inv) with y in c}
  void count(int64_t r, int64_t inv, const uint8_t* c) {
    if (r < 0 || r >= kb.n_roles) throw Bad{};
    const int64_t n = kb.n;
    uint32_t* cnt = s.cnt.data();
    std::memset(cnt, 0, n * sizeof(uint32_t));
    const int64_t* off = kb.off + r * (n + 1);
    for (int64_t x = 0; x < n; ++x)
      for (int64_t e = off[x]; e < off[x + 1]; ++e) {
        const int64_t y = kb.tg[e];
        if (!inv) cnt[x] += c[y];
        else cnt[y] += c[x];
      }
  }

  // evaluate the sub-expression at the cursor into out[0..N)
  void eval(uint8_t* out) {
    const int64_t n = kb.n;
    const int64_t op = next();
    switch (op) {
      case TOP: std::memset(out, 1, n); return;
      case BOT: std::memset(out, 0, n); return;
      case ATOM: {
        const int64_t a = next();
        if (a < 0 || a >= kb.n_concepts) throw Bad{};
        std::memcpy(out, kb.concepts.data() + a * n, n);
        return;
      }
      case NOT: {
        eval(out);
        for (int64_t x = 0; x < n; ++x) out[x] = !out[x];
        return;
      }
      case AND:
      case OR: {
        const int64_t k = next();
        std::memset(out, op == AND ? 1 : 0, n);
        uint8_t* c = s.push();
        for (int64_t i = 0; i < k; ++i) {
          eval(c);
          if (op == AND) for (int64_t x = 0; x < n; ++x) out[x] &= c[x];
          else for (int64_t x = 0; x < n; ++x) out[x] |= c[x];
        }
        s.pop();
        return;
      }
      case EXISTS:
      case FORALL:
      case ATLEAST:
      case ATMOST:
      case EXACTLY: {
        const int64_t q = (op == EXISTS || op == FORALL) ? 0 : next();
        const int64_t r = next(), inv = next();
        uint8_t* c = s.push();
        eval(c);
        if (op == FORALL)                       // no successor outside C
          for (int64_t x = 0; x < n; ++x) c[x] = !c[x];
        count(r, inv, c);
        s.pop();
        const uint32_t* cnt = s.cnt.data();
        for (int64_t x = 0; x < n; ++x) {
          const int64_t v = cnt[x];
          out[x] = op == EXISTS    ? v >= 1
                 : op == FORALL    ? v == 0
                 : op == ATLEAST   ? v >= q
                 : op == ATMOST    ? v <= q
                                   : v == q;
        }
        return;
      }
      case DGE:
      case DLE:
      case DEQ: {
        const int64_t p = next(), bits = next();
        if (p < 0 || p >= kb.n_data) throw Bad{};
        float t;
        const uint32_t b = (uint32_t)bits;
        std::memcpy(&t, &b, 4);
        const float* col = kb.data + p * n;
        // an ordered comparison: NaN (no value) satisfies none of them
        for (int64_t x = 0; x < n; ++x)
          out[x] = op == DGE ? col[x] >= t : op == DLE ? col[x] <= t : col[x] == t;
        return;
      }
      default: throw Bad{};
    }
  }
};

void unpack(const uint64_t* words, int64_t n, uint8_t* out) {
  for (int64_t x = 0; x < n; ++x) out[x] = (uint8_t)((words[x >> 6] >> (x & 63)) & 1u);
}

}  // namespace

extern "C" {

// concept_bits [n_concepts][words] and pos/neg [words]: bit x of word x/64
// (least significant first).  offsets/targets/data stay owned by the caller
// and must outlive the handle.  Returns NULL on bad sizes.
void* ocpp_create(int64_t n, int32_t n_concepts, int64_t words, const uint64_t* concept_bits,
                  int32_t n_roles, const int64_t* offsets, const int32_t* targets, int32_t n_data,
                  const float* data, const uint64_t* pos, const uint64_t* neg) {
  if (n < 0 || words < (n + 63) / 64 || n_concepts < 0 || n_roles < 0 || n_data < 0) return nullptr;
  KB* kb = new KB;
  kb->n = n;
  kb->n_concepts = n_concepts;
  kb->n_roles = n_roles;
  kb->n_data = n_data;
  kb->off = offsets;
  kb->tg = targets;
  kb->data = data;
  kb->concepts.resize((size_t)n_concepts * n);
#pragma omp parallel for schedule(static)
  for (int32_t a = 0; a < n_concepts; ++a)
    unpack(concept_bits + (size_t)a * words, n, kb->concepts.data() + (size_t)a * n);
  kb->pos.resize(n);
  kb->neg.resize(n);
  unpack(pos, n, kb->pos.data());
  unpack(neg, n, kb->neg.data());
  return kb;
}

void ocpp_destroy(void* h) { delete static_cast<KB*>(h); }

// Membership vector of one hypothesis (tokens[0..n_tokens)) into out[N].
// Returns 0, or -1 for a malformed stream.
int ocpp_ext(void* h, const int64_t* tokens, int64_t n_tokens, uint8_t* out) {
  const KB& kb = *static_cast<KB*>(h);
  Scratch s(kb.n);
  Eval e{kb, s, tokens, n_tokens};
  try {
    e.eval(out);
  } catch (Bad&) {
    return -1;
  }
  return e.pos == n_tokens ? 0 : -1;
}

// counts[i] = (#(ext(H_i) & P), #(ext(H_i) & Ng)) for hypothesis i =
// tokens[hyp_off[i] .. hyp_off[i+1]), on n_threads OpenMP threads (0: the
// runtime's default), dynamic schedule.  Returns 0, or -1 - i for the first
// malformed hypothesis i.
int64_t ocpp_coverage(void* h, const int64_t* tokens, const int64_t* hyp_off, int64_t n_hyps,
                      int32_t n_threads, uint32_t* counts) {
  const KB& kb = *static_cast<KB*>(h);
  int64_t bad = -1;
  const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
  {
    Scratch s(kb.n);
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < n_hyps; ++i) {
      Eval e{kb, s, tokens + hyp_off[i], hyp_off[i + 1] - hyp_off[i]};
      uint8_t* m = s.push();
      bool ok = true;
      try {
        e.eval(m);
        ok = e.pos == e.len;
      } catch (Bad&) {
        ok = false;
      }
      uint32_t p = 0, q = 0;
      if (ok)
        for (int64_t x = 0; x < kb.n; ++x) {
          p += m[x] & kb.pos[x];
          q += m[x] & kb.neg[x];
        }
      s.pop();
      counts[2 * i] = p;
      counts[2 * i + 1] = q;
      if (!ok) {
#pragma omp critical
        if (bad < 0 || i < bad) bad = i;
      }
    }
  }
  return bad < 0 ? 0 : -1 - bad;
}

int ocpp_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
