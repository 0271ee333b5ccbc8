// Refinement candidates written on the device (hth_draw_conjuncts, hth_conjoin).
//
// The paper leaves generating evaluation plans on the GPU as future work
// (Section 8, Conclusion and future work); this file covers the step before the plan, for the one-step
// specialisation that adds a conjunct: candidate = P ⊓ X, where P is a parent
// whose instance set is a row of the caller's set table and X is an atomic
// concept, an existential ∃r.A / ∃r⁻.A over an atomic concept, or a threshold
// on a property.  hth_draw_conjuncts draws the conjuncts from a counter-based
// generator (SplitMix64: Steele, Lea and Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014), so that draw i depends on (seed, i) only;
// hth_conjoin writes each candidate as four hth_node records and two children
// entries, ready for hth_dplan_create.
#include <hip/hip_runtime.h>

#include <cstring>

#include "kb_handle.h"

namespace hth {
namespace {

// value i of the SplitMix64 sequence started at `seed`
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Draw i uses sequence values 4i .. 4i+3: u0 picks the kind (atom 5 in 10,
// existential 3 in 10, threshold 2 in 10; a kind the KB has nothing for falls
// back to an atom), u1 .. u3 its arguments, each as u mod the range.  The
// parent is parent_rows[i / per_parent].
__global__ void __launch_bounds__(256)
k_draw_conjuncts(uint64_t seed, const uint32_t* __restrict__ parent_rows, uint32_t per_parent, uint32_t n,
                 uint32_t n_concepts, uint32_t n_roles, uint32_t n_data, const float* __restrict__ deciles,
                 hth_conjunct* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t u0 = splitmix64(seed, 4ull * i), u1 = splitmix64(seed, 4ull * i + 1);
  const uint64_t u2 = splitmix64(seed, 4ull * i + 2), u3 = splitmix64(seed, 4ull * i + 3);
  uint32_t kind = (uint32_t)(u0 % 10);
  kind = kind < 5 ? HTH_CJ_ATOM : kind < 8 ? HTH_CJ_EXISTS : (u3 & 1) ? HTH_CJ_LE : HTH_CJ_GE;
  if ((kind == HTH_CJ_EXISTS && !n_roles) || ((kind == HTH_CJ_GE || kind == HTH_CJ_LE) && !n_data))
    kind = HTH_CJ_ATOM;
  hth_conjunct c;
  c.parent = parent_rows[i / per_parent];
  c.kind = (uint8_t)kind;
  c.inv = 0;
  c.pad = 0;
  c.a = 0;
  c.b = 0;
  if (kind == HTH_CJ_ATOM) {
    c.a = (uint32_t)(u1 % n_concepts);
  } else if (kind == HTH_CJ_EXISTS) {
    c.b = (uint32_t)(u1 % n_roles);
    c.inv = (uint8_t)((u1 >> 32) & 1);
    c.a = (uint32_t)(u2 % n_concepts);
  } else {
    c.a = (uint32_t)(u1 % n_data);
    const float t = deciles[(size_t)c.a * 9 + (uint32_t)(u2 % 9)];
    std::memcpy(&c.b, &t, 4);
  }
  out[i] = c;
}

__device__ __forceinline__ hth_node mk_node(uint8_t op, uint8_t inv, uint16_t arity, uint32_t arg, uint32_t child,
                                            uint32_t q) {
  hth_node x;
  x.op = op;
  x.inv = inv;
  x.arity = arity;
  x.arg = arg;
  x.child = child;
  x.q.n = q;
  return x;
}

// Candidate i: nodes 4i .. 4i+3 = SET(parent), the conjunct's leaf, the
// existential over it (or an unreferenced ⊤), AND(set, conjunct); children
// 2i, 2i+1; offsets[i] = node_base + 4i, and the AND's children start at
// child_base + 2i (the candidates may follow other hypotheses in one batch).
// A kind outside HTH_CJ_* writes an op that hth_dplan_create rejects.
__global__ void __launch_bounds__(256)
k_conjoin(const hth_conjunct* __restrict__ specs, uint32_t n, hth_node* __restrict__ nodes,
          uint32_t* __restrict__ offs, uint32_t* __restrict__ kids, uint32_t node_base, uint32_t child_base) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  offs[i] = node_base + 4 * i;
  if (i == n) return;
  const hth_conjunct c = specs[i];
  hth_node* o = nodes + 4 * (size_t)i;
  o[0] = mk_node(HTH_SET, 0, 0, c.parent, 0, 0);
  uint32_t x = 1;
  switch (c.kind) {
    case HTH_CJ_ATOM:
      o[1] = mk_node(HTH_ATOM, 0, 0, c.a, 0, 0);
      o[2] = mk_node(HTH_TOP, 0, 0, 0, 0, 0);
      break;
    case HTH_CJ_EXISTS:
      o[1] = mk_node(HTH_ATOM, 0, 0, c.a, 0, 0);
      o[2] = mk_node(HTH_EXISTS, c.inv, 0, c.b, 1, 0);
      x = 2;
      break;
    case HTH_CJ_GE:
    case HTH_CJ_LE:
    case HTH_CJ_EQ:
      o[1] = mk_node(c.kind == HTH_CJ_GE ? HTH_DATA_GE : c.kind == HTH_CJ_LE ? HTH_DATA_LE : HTH_DATA_EQ, 0, 0,
                     c.a, 0, c.b);
      o[2] = mk_node(HTH_TOP, 0, 0, 0, 0, 0);
      break;
    default:
      o[1] = mk_node(0xFF, 0, 0, 0, 0, 0);
      o[2] = mk_node(HTH_TOP, 0, 0, 0, 0, 0);
      break;
  }
  o[3] = mk_node(HTH_AND, 0, 2, 0, child_base + 2 * i, 0);
  kids[2 * (size_t)i] = 0;
  kids[2 * (size_t)i + 1] = x;
}

}  // namespace
}  // namespace hth

using namespace hth;

extern "C" hth_status hth_draw_conjuncts(hth_kb kb, uint64_t seed, const uint32_t* d_parent_rows, uint32_t n_parents,
                                         uint32_t per_parent, const float* d_deciles, hth_conjunct* d_specs,
                                         void* stream) {
  if (!kb || !d_parent_rows || !d_specs) return fail(HTH_E_INVALID, "NULL argument");
  if (!n_parents || !per_parent) return HTH_OK;
  if ((uint64_t)n_parents * per_parent >= (1ull << 31)) return fail(HTH_E_RANGE, "more than 2^31 - 1 draws");
  if (!kb->d.n_concepts) return fail(HTH_E_RANGE, "the KB has no concepts to draw");
  if (kb->d.n_data && !d_deciles) return fail(HTH_E_INVALID, "deciles is NULL");
  const uint32_t n = n_parents * per_parent;
  hipLaunchKernelGGL(k_draw_conjuncts, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), seed,
                     d_parent_rows, per_parent, n, kb->d.n_concepts, kb->d.n_roles, kb->d.n_data, d_deciles,
                     d_specs);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_conjoin(const hth_conjunct* d_specs, uint32_t n, hth_node* d_nodes,
                                  uint32_t* d_hyp_node_offsets, uint32_t* d_children, uint32_t node_base,
                                  uint32_t child_base, void* stream) {
  if (!d_specs || !d_nodes || !d_hyp_node_offsets || !d_children) return fail(HTH_E_INVALID, "NULL argument");
  if (n >= (1u << 22)) return fail(HTH_E_RANGE, "more than 2^22 - 1 candidates (2^24 nodes)");
  if ((uint64_t)node_base + 4ull * n >= (1ull << 32) || (uint64_t)child_base + 2ull * n >= (1ull << 32))
    return fail(HTH_E_RANGE, "node or children index beyond 2^32");
  hipLaunchKernelGGL(k_conjoin, dim3((n + 1 + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), d_specs,
                     n, d_nodes, d_hyp_node_offsets, d_children, node_base, child_base);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}
