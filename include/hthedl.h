/*
 * hthedl.h -- C ABI of libhthedl.so: exact evaluation of ALCQI(D) concept
 * hypotheses over a knowledge base resident in the memory of one MI355X GPU.
 *
 * The problem statement follows HT-HEDL (Algahtani, "HT-HEDL: High-Throughput
 * Hypothesis Evaluation in Description Logic"):
 *   - the knowledge base lives entirely in device memory (Section 3.1): concept
 *     memberships as rows over individuals (the transposed concepts matrix),
 *     role assertions grouped per role, numeric concrete-role values, and the
 *     learning-examples matrix;
 *   - a hypothesis is an array of DL operations in consecutive memory
 *     (Section 4), here in postfix order;
 *   - its result is the instance set and the (covered positives, covered
 *     negatives) pair of the coverage matrix (Section 4, Algorithm 15).
 *
 * Conventions for every call:
 *   - Every call returns hth_status; nothing throws or longjmps across the ABI.
 *   - Validation happens before anything is launched.  On error no output is
 *     written and hth_last_error() returns a message for the calling thread.
 *   - "device" pointers are HIP device memory owned by the caller.  The library
 *     never allocates or frees device memory; the knowledge base, the derived
 *     buffer, the workspace and every output belong to the caller and must
 *     outlive the calls (and the kb handle) that use them.
 *   - "host" pointers are read during the call only.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     asynchronous on it unless stated otherwise.  One kb may be used from
 *     several streams at once only with a distinct workspace per stream.
 *   - Bit rows: individual i is bit (i & 63) of uint64 word (i >> 6), least
 *     significant bit first.  Bits at positions >= N must be zero on input and
 *     are zero on output.
 */
#ifndef HTHEDL_H
#define HTHEDL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hth_status;
enum {
  HTH_OK = 0,
  HTH_E_INVALID = -1,     /* malformed argument or knowledge base */
  HTH_E_RANGE = -2,       /* id, index or size out of range */
  HTH_E_NOMEM = -3,       /* caller-provided buffer too small */
  HTH_E_DEVICE = -4,      /* a HIP call failed (text in hth_last_error) */
  HTH_E_PLAN = -5,        /* hypothesis not in postfix form */
  HTH_E_STATE = -6,       /* handle used in the wrong state */
  HTH_E_UNSUPPORTED = -7  /* valid request outside the library's limits */
};

/* DL constructs (Section 3.2): the boolean constructs, the object-role
 * restrictions, single-valued data thresholds, and the concrete-role
 * restrictions over multi-valued numeric roles (MIN, MAX, EXACT) and string
 * roles (EQUAL, CONTAIN) of Section 3.2.3.  The inverse-role CSR is always
 * derived by the library (hth_kb_create); a caller cannot hand one in. */
enum {
  HTH_TOP = 0,      /* every individual */
  HTH_BOT = 1,      /* no individual */
  HTH_ATOM = 2,     /* arg = concept id: one row of the concepts matrix */
  HTH_NOT = 3,      /* complement in the domain (closed world, Section 3.1) */
  HTH_AND = 4,      /* n-ary conjunction (Algorithms 1/2); arity 0 = TOP */
  HTH_OR = 5,       /* n-ary disjunction; arity 0 = BOT */
  HTH_EXISTS = 6,   /* {x : some successor in C} (Algorithms 3/4) */
  HTH_FORALL = 7,   /* {x : every successor in C}, incl. x without successors (Algorithms 5/6) */
  HTH_ATLEAST = 8,  /* {x : cnt(x) >= n}, cnt = successors in C (Algorithms 7/8) */
  HTH_ATMOST = 9,   /* {x : cnt(x) <= n}; textbook reading: includes cnt = 0 */
  HTH_EXACTLY = 10, /* {x : cnt(x) == n} */
  HTH_DATA_GE = 11, /* {x : value of property arg defined and >= t} (Algorithms 9/10) */
  HTH_DATA_LE = 12, /* {x : value of property arg defined and <= t} */
  HTH_SET = 13,     /* arg = row of the set table registered with hth_kb_set_sets: an
                       instance set the caller computed earlier (for example the
                       unchanged subtrees of a refined parent), used as a leaf */
  HTH_DATA_EQ = 14, /* {x : value of property arg defined and == t} (EXACT, Algorithms 9/10) */
  HTH_NUM_GE = 15,  /* {x : some value of numeric concrete role arg is >= t} (MIN,
                       Section 3.2.3, Algorithms 9/10; roles from hth_kb_set_numeric) */
  HTH_NUM_LE = 16,  /* {x : some value of numeric concrete role arg is <= t} (MAX) */
  HTH_NUM_EQ = 17,  /* {x : some value of numeric concrete role arg is == t} (EXACT) */
  HTH_STR_EQ = 18,  /* {x : some value of string concrete role arg is dictionary string q.n}
                       (EQUAL, Algorithms 11/12; roles from hth_kb_set_strings);
                       q.n = 0xFFFFFFFF: a string absent from the dictionary, no individual */
  HTH_STR_CONTAINS = 19, /* {x : some value of string concrete role arg has pattern q.n as a
                       substring} (CONTAIN, Algorithms 13/14; patterns from hth_kb_set_patterns) */
  HTH_NUM_OPS = 20
};

/* One node of a hypothesis, 16 bytes.  Nodes are in postfix order: every child
 * index is smaller than its parent's index; the root is the last node of the
 * hypothesis.  Nodes may be shared (a DAG). */
typedef struct {
  uint8_t op;       /* HTH_* construct */
  uint8_t inv;      /* role constructs: 1 = inverse role r^- (subject and object swapped) */
  uint16_t arity;   /* AND/OR: number of children; 0 otherwise */
  uint32_t arg;     /* ATOM: concept id; role constructs: role id; DATA_*: property id;
                       NUM_*: numeric concrete role id; STR_*: string concrete role id */
  uint32_t child;   /* NOT and role constructs: child node index (local to the
                       hypothesis); AND/OR: first entry in the children array */
  union {
    uint32_t n;     /* ATLEAST/ATMOST/EXACTLY: n (<= 2^31 - 1); STR_EQ: string id; STR_CONTAINS:
                       pattern id */
    float t;        /* DATA_* and NUM_*: threshold (not NaN; +-inf allowed) */
  } q;
} hth_node;

typedef struct hth_kb_s* hth_kb;   /* opaque host handle */

/* The knowledge base (Section 3.1).  Every pointer is device memory; the bit
 * rows (concept_bits, pos_bits, neg_bits) are 16-byte aligned. */
typedef struct {
  uint32_t n_individuals;        /* N, 1 <= N < 2^31 */
  uint32_t stride_words;         /* words per bit row: >= ceil(N/64), a multiple of 8 */
  uint32_t n_concepts;
  const uint64_t* concept_bits;  /* [n_concepts][stride_words] membership rows */
  uint32_t n_roles;
  uint64_t n_edges;              /* E: total role assertions over all roles */
  const int64_t* role_offsets;   /* [n_roles][N+1]: assertions of role r with subject x are
                                    role_targets[role_offsets[r][x] .. role_offsets[r][x+1]);
                                    role_offsets[0][0] = 0, role_offsets[r][0] =
                                    role_offsets[r-1][N], role_offsets[n_roles-1][N] = E */
  const int32_t* role_targets;   /* [E] objects; strictly increasing inside each row (a role is
                                    a set of assertions); each < N.  E_r < 2^32 per role. */
  uint32_t n_data;
  const float* data;             /* [n_data][N] one value per individual and property; NaN = none */
  const uint64_t* pos_bits;      /* [stride_words] positive examples */
  const uint64_t* neg_bits;      /* [stride_words] negative examples (may overlap pos) */
} hth_kb_desc;

/* Size of the derived buffer that hth_kb_create fills: per-role 32-bit row
 * offsets for both directions, the inverse-role CSR (transpose), the
 * non-empty words of each role direction, and each direction's objects (a
 * bit row, per-word counts, and the object rank of every assertion's target,
 * filled where the objects are at most half of the individuals). */
hth_status hth_kb_derived_bytes(const hth_kb_desc* desc, size_t* bytes);

/* Validate the knowledge base on the device and build the derived layouts into
 * `derived` (device memory of at least hth_kb_derived_bytes).  Synchronous:
 * returns after validation and the build have finished on `stream`.  Errors:
 * HTH_E_INVALID (non-monotone offsets, target out of range, duplicate or
 * unsorted targets, set padding bits, bit rows not 16-byte aligned),
 * HTH_E_NOMEM (derived too small),
 * HTH_E_RANGE (sizes beyond the limits above). */
hth_status hth_kb_create(const hth_kb_desc* desc, void* derived, size_t derived_bytes,
                         void* stream, hth_kb* out);

/* Replace the example rows (device [stride_words] each, zero padding, 16-byte
 * aligned; HTH_E_INVALID otherwise). */
hth_status hth_kb_set_examples(hth_kb kb, const uint64_t* pos_bits, const uint64_t* neg_bits);

/* Register the set table that HTH_SET leaves read: device uint64
 * [n_rows][stride_words], zero padding bits, owned by the caller and read by
 * later evaluations in stream order (rows may be rewritten between calls, for
 * instance by hth_eval_batch_sets).  rows = NULL with n_rows = 0 removes it.
 * Must not run concurrently with an evaluation on the same kb.  Errors:
 * HTH_E_INVALID (NULL rows with n_rows > 0, rows not 16-byte aligned),
 * HTH_E_RANGE (n_rows >= 2^24). */
hth_status hth_kb_set_sets(hth_kb kb, const uint64_t* rows, uint32_t n_rows);

/* Multi-valued numeric concrete roles (Section 3.1: a concrete role is a list
 * of (subject, value) assertions, a subject may hold many; Section 3.2.3).
 * offsets: device int64 [n_roles][N+1], absolute into values: role p's values
 * of subject x are values[offsets[p][x] .. offsets[p][x+1]), with
 * offsets[0][0] = 0, offsets[p][0] = offsets[p-1][N] and
 * offsets[n_roles-1][N] = n_values.  values: device float32 [n_values], none
 * NaN (an absent value is an absent assertion).  Both stay the caller's and
 * must outlive every evaluation that uses them.  derived: device memory of at
 * least hth_numeric_derived_bytes (256-byte aligned, caller-owned) for the
 * library's tables of heavy rows (subjects above the heavy-row threshold).
 * Validates on the device and returns after `stream` has finished.  Replaces
 * the previous registration (n_roles = 0 removes it); plans compiled before
 * keep the registration they were compiled with.  Must not run concurrently
 * with an evaluation on the same kb.  Errors: HTH_E_INVALID (NULL arrays,
 * offsets not monotone or not chained as above, NaN values, misaligned
 * derived), HTH_E_NOMEM (derived too small), HTH_E_RANGE (n_roles >= 2^16,
 * n_values >= 2^40 or a role with 2^32 or more values). */
hth_status hth_numeric_derived_bytes(hth_kb kb, uint32_t n_roles, uint64_t n_values, size_t* bytes);
hth_status hth_kb_set_numeric(hth_kb kb, uint32_t n_roles, const int64_t* offsets, const float* values,
                              uint64_t n_values, void* derived, size_t derived_bytes, void* stream);

/* String concrete roles (Section 3.1: (subject, string) assertions; Section
 * 3.2.3).  The strings are interned: a dictionary of n_strings distinct
 * strings, string s = chars[str_offsets[s] .. str_offsets[s+1]) (device int64
 * [n_strings+1], non-decreasing from 0; device bytes), and every assertion
 * holds a dictionary id.  offsets: device int64 [n_roles][N+1], absolute into
 * ids and chained as for hth_kb_set_numeric; ids: device int32 [n_values] in
 * [0, n_strings).  All arrays stay the caller's.  derived: device memory of at
 * least hth_string_derived_bytes (256-byte aligned) for heavy-row tables.
 * Validates on the device and returns after `stream` has finished; replaces
 * the previous registration (n_roles = 0 removes it; plans compiled before
 * keep theirs).  Errors as for hth_kb_set_numeric, plus HTH_E_INVALID for an
 * id out of range or non-monotone string offsets, and HTH_E_RANGE for
 * n_strings >= 2^31. */
hth_status hth_string_derived_bytes(hth_kb kb, uint32_t n_roles, uint64_t n_values, size_t* bytes);
hth_status hth_kb_set_strings(hth_kb kb, uint32_t n_roles, const int64_t* offsets, const int32_t* ids,
                              uint64_t n_values, uint32_t n_strings, const int64_t* str_offsets,
                              const uint8_t* chars, void* derived, size_t derived_bytes, void* stream);

/* The CONTAIN patterns that HTH_STR_CONTAINS nodes name by index: pattern k =
 * chars[offsets[k] .. offsets[k+1]) (device int64 [n_patterns+1],
 * non-decreasing; device bytes; the empty pattern is a substring of every
 * string).  Owned by the caller and read by later evaluations; plans compiled
 * before keep the table they were compiled with.  n_patterns = 0 removes it.
 * The offsets are checked on `stream` (synchronous).  Errors: HTH_E_INVALID
 * (NULL arrays with n_patterns > 0, offsets not non-decreasing from 0). */
hth_status hth_kb_set_patterns(hth_kb kb, uint32_t n_patterns, const int64_t* offsets, const uint8_t* chars,
                               void* stream);

/* Largest out-degree of role r in direction inv (0 = forward, 1 = inverse). */
hth_status hth_kb_max_degree(hth_kb kb, uint32_t role, uint32_t inv, uint32_t* out);

/* Schedule of the batched executor (no effect on results, only on speed).
 * group_min: smallest (role, direction, level) bucket of role nodes evaluated
 *   by shared CSR passes (0 = never share); on a direction whose rows are all
 *   within short_rows, or whose non-empty words are at most half of all words,
 *   a bucket of one node is shared as well;
 * group_k: most role nodes per shared pass (1..64; sets the transposed child
 *   row width 8/16/32/64 bits);
 * xcd_local: 1 = keep each shared pass on one XCD (its L2 holds the pass's
 *   transposed child rows);
 * t_budget_mb: most transposed child rows one launch of shared passes builds
 *   and reads (MiB; default 1024).  A plan's workspace holds the most any of
 *   its launches uses, not the budget;
 * unroll: assertions in flight per lane in passes over directions with many
 *   assertions per word (8 or 16; sparse directions always use 8);
 * region_reg: 1, 2 or 4 = boolean regions whose value stack fits six entries
 *   run with the stack in registers and that many words per lane (0 = the
 *   LDS-stack kernel for every region);
 * t_compact: 1 = shared passes over a role direction whose objects (targets)
 *   are at most half of the individuals keep transposed child rows for those
 *   objects only, indexed by object rank (0 = rows for every individual);
 * t_segment_kb: KiB of transposed child rows fetched per pass: a shared pass
 *   whose rows are larger runs as 2..4 passes over consecutive row ranges,
 *   carrying each subject's partial counts between them, so that each pass's
 *   rows fit one XCD's L2 (0 = one pass over all rows; at most 2^22);
 * push_pct: an existential restriction over an atomic concept evaluated on
 *   its own (not in a shared pass) whose concept holds under this percentage
 *   of the individuals is evaluated from the concept's members: each marks
 *   the subjects that reach it, where no row of the other direction holds
 *   more than 64 assertions (0 = always count per subject; at most 100;
 *   default 2);
 * short_rows: a shared pass over a role direction whose rows all hold at most
 *   this many assertions walks each subject's row on one lane (no slicing of
 *   the words' assertion ranges, no scan across lanes) and stores eight words
 *   of each member's output at once (0 = never; at most 64; default 12). */
typedef struct {
  uint32_t group_min;
  uint32_t group_k;
  uint32_t xcd_local;
  uint32_t t_budget_mb;
  uint32_t unroll;
  uint32_t region_reg;
  uint32_t t_compact;
  uint32_t t_segment_kb;
  uint32_t push_pct;
  uint32_t short_rows;
} hth_tuning;
hth_status hth_kb_get_tuning(hth_kb kb, hth_tuning* out);
hth_status hth_kb_set_tuning(hth_kb kb, const hth_tuning* t);   /* HTH_E_RANGE if out of range */

/* Free the host handle.  Device memory is the caller's. */
hth_status hth_kb_destroy(hth_kb kb);

/* Workspace needed to evaluate up to max_hyps hypotheses with at most
 * max_nodes nodes in total per call (device memory, caller-owned, no
 * initialisation required). */
hth_status hth_workspace_bytes(hth_kb kb, uint32_t max_nodes, uint32_t max_hyps, size_t* bytes);

/* Evaluate one hypothesis (Section 4): plan on the host, then a short kernel
 * sequence on `stream`.  nodes/children are host arrays.  d_counts: device
 * uint32[2] <- (covered positives, covered negatives) (Algorithm 15).
 * d_instances: NULL or device uint64[stride_words] <- the instance set. */
hth_status hth_eval_one(hth_kb kb, const hth_node* nodes, uint32_t n_nodes,
                        const uint32_t* children, uint32_t n_children,
                        void* ws, size_t ws_bytes, uint64_t* d_instances, uint32_t* d_counts,
                        void* stream);

/* hth_eval_one for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * workspace is a fixed array of HTH_NOALLOC_SCRATCH_BYTES in the library's
 * device data, one per GPU, held until the process ends; its address is looked
 * up once per device on the first call there.  The call allocates nothing:
 * the caller passes only the inputs and outputs, as for hth_eval_one.
 * Results are those of hth_eval_one (the same plan and kernels).
 * - HTH_E_NOMEM, before any launch, when the hypothesis's plan needs more than
 *   HTH_NOALLOC_SCRATCH_BYTES (about (role nodes + materialised fillers + 2)
 *   bit rows of 8 * stride_words bytes, plus a few KB of tables); use
 *   hth_eval_one with a workspace then.
 * - Every call on one GPU shares that GPU's array: calls that overlap on the
 *   device (several streams, or several host threads) race and are not
 *   supported.  Calls in order on one stream are fine.  No scratch content
 *   needs to start at zero; each call writes what it reads.
 * - The node arrays are copied from the host on `stream` during the call. */
#define HTH_NOALLOC_SCRATCH_BYTES (64u << 20)
hth_status hth_eval_one_noalloc(hth_kb kb, const hth_node* nodes, uint32_t n_nodes,
                                const uint32_t* children, uint32_t n_children,
                                uint64_t* d_instances, uint32_t* d_counts, void* stream);

/* Exact workspace hth_eval_batch needs for this batch (the batch is compiled on
 * the host; nothing is launched).  Same arguments as hth_eval_batch. */
hth_status hth_batch_workspace_bytes(hth_kb kb, const hth_node* nodes, const uint32_t* hyp_node_offsets,
                                     uint32_t n_hyps, const uint32_t* children, uint32_t n_children,
                                     size_t* bytes);

/* Evaluate a batch.  Hypothesis h is nodes[hyp_node_offsets[h] .. hyp_node_offsets[h+1]),
 * its child indices local to that range; children[] entries are local too.
 * The batch is compiled once (shared subexpressions across hypotheses are
 * evaluated once), then run level by level.  d_counts: device uint32[n_hyps][2]. */
hth_status hth_eval_batch(hth_kb kb, const hth_node* nodes, const uint32_t* hyp_node_offsets,
                          uint32_t n_hyps, const uint32_t* children, uint32_t n_children,
                          void* ws, size_t ws_bytes, uint32_t* d_counts, void* stream);

/* hth_eval_batch that also writes each hypothesis's instance set: d_sets is
 * device uint64 [n_hyps][stride_words] (padding words and bits written as 0).
 * Used to fill the set table with the subtrees of the hypotheses kept for the
 * next refinement round.  d_sets must not overlap the rows this batch reads
 * through HTH_SET leaves.  Same workspace as hth_eval_batch. */
hth_status hth_eval_batch_sets(hth_kb kb, const hth_node* nodes, const uint32_t* hyp_node_offsets,
                               uint32_t n_hyps, const uint32_t* children, uint32_t n_children,
                               void* ws, size_t ws_bytes, uint64_t* d_sets, uint32_t* d_counts,
                               void* stream);

/* A cross-batch cache of role-restriction results (this library's extension of
 * the per-batch shared subexpressions of Section 4's evaluation plans):
 * d_rows is caller device memory [n_rows][stride_words] (64-byte aligned),
 * registered as the kb's set table for as long as the cache lives.  Every
 * subexpression of a batch evaluated with hth_eval_batch_cached is interned by
 * its canonical form in one persistent table, so equal subexpressions of
 * different batches are recognised exactly (no hash is trusted alone).  A
 * role restriction whose subexpression holds a row is read from that row and
 * its subtree is not evaluated; one without a row is given the least recently
 * used row that no subexpression of the current batch reads, and its result is
 * written there for later batches (when every row is in use by the batch, it
 * runs in the workspace as in hth_eval_batch).  The table of interned forms is
 * cleared, with every row, when it passes 2^24 entries.
 * - hth_cache_create: n_rows 1 .. 2^24 - 1; replaces any registered set table.
 *   The rows' contents need no initialisation.
 * - hth_eval_batch_cached: as hth_eval_batch (same workspace bound from
 *   hth_batch_workspace_bytes); HTH_SET leaves are rejected (HTH_E_UNSUPPORTED),
 *   and HTH_E_STATE when another set table replaced the cache's.  Batches must
 *   run in order on one stream (a batch reads rows earlier batches wrote).  On
 *   an error the batch's admissions are undone.  Calls on one cache are
 *   serialised.
 * - hth_cache_stats: counters since creation (hits and misses count the
 *   batches' distinct live role restrictions).
 * - hth_cache_destroy: unregisters the rows (the caller then frees them). */
typedef struct hth_cache_s* hth_cache;
typedef struct {
  uint64_t hits, misses, admitted, evictions, batches;
  uint32_t entries, rows;
} hth_cache_info;
hth_status hth_cache_create(hth_kb kb, uint64_t* d_rows, uint32_t n_rows, hth_cache* out);
hth_status hth_eval_batch_cached(hth_kb kb, hth_cache cache, const hth_node* nodes,
                                 const uint32_t* hyp_node_offsets, uint32_t n_hyps, const uint32_t* children,
                                 uint32_t n_children, void* ws, size_t ws_bytes, uint32_t* d_counts,
                                 void* stream);
hth_status hth_cache_stats(hth_cache cache, hth_cache_info* out);
hth_status hth_cache_destroy(hth_cache cache);

/* Compiled batches for repeated evaluation.  hth_plan_create compiles a batch
 * as hth_eval_batch does (same arguments, host arrays) and reports the
 * workspace it needs; the plan keeps the kb's schedule and set table as they
 * were at creation.  hth_plan_upload copies the plan's tables into a workspace
 * (once per workspace); hth_plan_launch then runs the plan's kernels on
 * `stream` with no copy, no allocation and no memset (the counts are cleared
 * by a kernel), so a caller may capture it in a HIP graph and replay it.  The
 * KB's rows (concepts, data, examples, set rows) are read at each launch.
 * Profiling must be off while a launch is captured.  Errors: as hth_eval_batch;
 * HTH_E_RANGE for an empty batch.  The plan must not outlive its kb. */
typedef struct hth_plan_s* hth_plan;
hth_status hth_plan_create(hth_kb kb, const hth_node* nodes, const uint32_t* hyp_node_offsets, uint32_t n_hyps,
                           const uint32_t* children, uint32_t n_children, hth_plan* out, size_t* ws_bytes);
hth_status hth_plan_upload(hth_plan plan, void* ws, size_t ws_bytes, void* stream);
hth_status hth_plan_launch(hth_plan plan, void* ws, size_t ws_bytes, uint32_t* d_counts /* [n_hyps][2] */,
                           void* stream);
hth_status hth_plan_destroy(hth_plan plan);

/* Plans generated on the device.  The paper generates each hypothesis's
 * evaluation plan on CPU threads and leaves generation on the GPU, with little
 * or no CPU involvement, as future work (Sections 4 and 8).  Here the batch is
 * already in DEVICE memory, in the layout hth_eval_batch takes on the host:
 * d_nodes [n_nodes], d_hyp_node_offsets [n_hyps + 1] (hypothesis h is
 * d_nodes[offsets[h] .. offsets[h+1]), local child indices; offsets need not
 * start at 0, so a chunk of a larger batch is the same arrays with the offsets
 * pointer advanced), d_children [n_children].  Equal subexpressions of the
 * batch (same construct, arguments and equal children, children in the given
 * order) are evaluated once; every distinct DL operation is one task (every
 * node is evaluated, reachable from its root or not), run level by level on
 * the executor's kernels with the kb's schedule:
 * role nodes of one (level, role, direction) share CSR passes, thresholds on
 * one property a column pass.
 *
 * hth_dplan_create runs the count pass on `stream` (validation, role-nesting
 * levels, region programs' sizes, table sizes) and waits for its counts (a few
 * bytes per role direction and property): the only data the host reads; the
 * host builds the shared passes and the table layout from them.  *ws_bytes
 * receives the workspace that hth_dplan_launch needs.  `scratch` is device
 * memory of at least hth_dplan_scratch_bytes(kb, n_nodes) (about 270 bytes per
 * node: per-node facts, the hash-consing tables, the plan's own tables),
 * 256-byte aligned, owned by the caller and held by the plan until it is
 * destroyed.  The plan keeps the kb's set table and schedule as they were at
 * creation.  The node arrays must stay allocated and unchanged until the
 * plan's last launch.
 * hth_dplan_launch writes the plan's tables into ws on the device and runs
 * every kernel of the evaluation on `stream`, without waiting; d_counts
 * [n_hyps][2] as hth_eval_batch.  Launches of one plan must not overlap;
 * hth_dplan_destroy waits for the plan's last launch (the caller may then
 * free or reuse the scratch).
 * Errors (create): as hth_eval_batch, with the first failing hypothesis and
 * node; HTH_E_UNSUPPORTED for HTH_NUM_* / HTH_STR_* nodes, role restrictions
 * nested more than 64 deep, and regions with more than 32 nested operators;
 * HTH_E_RANGE for n_hyps = 0 or n_nodes > 2^24; HTH_E_NOMEM / HTH_E_INVALID
 * for a short or misaligned scratch.  (launch) HTH_E_NOMEM when
 * ws_bytes is short, HTH_E_INVALID when ws is not 256-byte aligned.  The plan
 * must not outlive its kb. */
typedef struct hth_dplan_s* hth_dplan;
hth_status hth_dplan_scratch_bytes(hth_kb kb, uint32_t n_nodes, size_t* bytes);
hth_status hth_dplan_create(hth_kb kb, const hth_node* d_nodes, uint32_t n_nodes,
                            const uint32_t* d_hyp_node_offsets, uint32_t n_hyps, const uint32_t* d_children,
                            uint32_t n_children, void* scratch, size_t scratch_bytes, void* stream,
                            hth_dplan* out, size_t* ws_bytes);
hth_status hth_dplan_launch(hth_dplan plan, void* ws, size_t ws_bytes, uint32_t* d_counts /* [n_hyps][2] */,
                            void* stream);
hth_status hth_dplan_destroy(hth_dplan plan);
/* The structure of a device plan, as its count pass and the host's schedule
 * left it: role-nesting levels; distinct role nodes (one per class of equal
 * role subexpressions), of which shared_passes groups hold the members of
 * shared CSR passes; distinct thresholds; materialised compound fillers; bit
 * rows of the workspace.  Errors: HTH_E_INVALID (NULL). */
typedef struct {
  uint32_t levels, role_nodes, shared_passes, thresholds, materialised, rows;
} hth_dplan_info;
hth_status hth_dplan_stats(hth_dplan plan, hth_dplan_info* out);

/* Refinement candidates written on the device: the one-step specialisation
 * that adds a conjunct, candidate = P and X, for parents P whose instance sets
 * are rows of the registered set table (hth_kb_set_sets).  With
 * hth_dplan_create this keeps a refinement round's candidates and plans on the
 * device (the paper's Section 8 future work; the paper defines no refinement
 * operator, the conjunct family is this library's).  16 bytes per spec. */
enum {
  HTH_CJ_ATOM = 0,     /* X = atomic concept a */
  HTH_CJ_EXISTS = 1,   /* X = exists role b (inv: inverse) . atomic concept a */
  HTH_CJ_GE = 2,       /* X = property a >= threshold (b: float bits) */
  HTH_CJ_LE = 3,       /* X = property a <= threshold */
  HTH_CJ_EQ = 4        /* X = property a == threshold */
};
typedef struct {
  uint32_t parent;     /* set-table row of P */
  uint8_t kind;        /* HTH_CJ_* */
  uint8_t inv;
  uint16_t pad;
  uint32_t a, b;
} hth_conjunct;

/* n = n_parents * per_parent specs into d_specs (device [n]): spec i refines
 * the parent in set-table row d_parent_rows[i / per_parent] (device [n_parents]).
 * Draw i reads values 4i .. 4i+3 of the SplitMix64 sequence (Steele, Lea and
 * Flood, OOPSLA 2014) started at `seed`, so it depends on (seed, i) only:
 *   u0 mod 10: 0-4 an atom, 5-7 an existential, 8-9 a threshold (u3 bit 0:
 *   1 = LE, 0 = GE); an existential without roles or a threshold without
 *   properties becomes an atom;
 *   atom: a = u1 mod n_concepts;  existential: b = u1 mod n_roles, inv = bit
 *   32 of u1, a = u2 mod n_concepts;  threshold: a = u1 mod n_data, the
 *   threshold d_deciles[a][u2 mod 9] (device float [n_data][9]).
 * Duplicate draws are possible.  Asynchronous on `stream`.  Errors:
 * HTH_E_INVALID (NULL arguments; deciles NULL with n_data > 0), HTH_E_RANGE
 * (n >= 2^31, no concepts). */
hth_status hth_draw_conjuncts(hth_kb kb, uint64_t seed, const uint32_t* d_parent_rows, uint32_t n_parents,
                              uint32_t per_parent, const float* d_deciles, hth_conjunct* d_specs, void* stream);

/* Candidate i of d_specs (device [n]) as hypotheses in the layout
 * hth_eval_batch and hth_dplan_create take: d_nodes [4n], d_hyp_node_offsets
 * [n+1] (= node_base + 4i), d_children [2n], the AND of candidate i starting
 * at children entry child_base + 2i.  With both bases 0 the arrays are a batch
 * of their own; otherwise the three pointers point into a larger batch at
 * node node_base and children entry child_base (its first hypotheses written
 * by someone else), so that one plan covers the whole batch.  Hypothesis i is
 * SET(parent), X's leaf, X's existential (or an unreferenced TOP), AND(SET, X).
 * Nothing is validated here: hth_dplan_create validates the nodes (a kind
 * outside HTH_CJ_* becomes an op it rejects).  Asynchronous on `stream`.
 * Errors: HTH_E_INVALID (NULL), HTH_E_RANGE (n >= 2^22, or an index beyond
 * 2^32). */
hth_status hth_conjoin(const hth_conjunct* d_specs, uint32_t n, hth_node* d_nodes, uint32_t* d_hyp_node_offsets,
                       uint32_t* d_children, uint32_t node_base, uint32_t child_base, void* stream);

/* Measurement.  Between hth_profile_begin and hth_profile_end every kernel the
 * library launches for this kb is bracketed by two HIP events recorded on the
 * launch stream, and the host adds up the algorithmic HBM bytes of the launch
 * (each input array the kernel must read once, each output it writes once).
 * hth_profile_end waits for the recorded events and returns, per kernel kind,
 * the number of launches, their summed event-timed duration (ms) and bytes.
 * Profiling adds two event records per launch; results are unchanged. */
enum {
  HTH_K_THRESHOLD = 0,  /* numeric restriction rows */
  HTH_K_REGION = 1,     /* boolean regions, with or without coverage */
  HTH_K_ROLE = 2,       /* one role restriction per task */
  HTH_K_TBUILD = 3,     /* transposed child rows for shared role passes */
  HTH_K_GROUP = 4,      /* shared role passes (up to 64 role nodes per CSR scan) */
  HTH_K_FILL = 5,       /* zero-count results of words without assertions */
  HTH_K_PLAN = 6,       /* plan generation on the device (hth_dplan_launch) */
  HTH_K_GROUP_SHORT = 7, /* shared role passes over directions of short rows (a lane per subject) */
  HTH_K_NUM = 8
};
typedef struct {
  uint64_t launches;
  double ms;
  double bytes;
} hth_prof_entry;
hth_status hth_profile_begin(hth_kb kb);
hth_status hth_profile_end(hth_kb kb, hth_prof_entry* out /* [HTH_K_NUM] */);

/* ---------------------------------------------------------------------------
 * Learned screener (a project extension, not in the paper): it ranks refinement
 * candidates so that only the best fraction is evaluated exactly.  All buffers
 * are device memory owned by the caller; bf16 values travel as uint16_t bit
 * patterns; every matrix is row-major with the given leading dimension.
 * ------------------------------------------------------------------------- */

/* Hashed subtree features.  For each hypothesis (postfix nodes, local child
 * indices, as in hth_eval_batch but in device memory) every node's subtree gets
 * a 64-bit hash: FNV-1a over 12 header bytes (op, inv, arity as 2 LE bytes, arg
 * and q as 4 LE bytes each; fields a construct does not use are zero), followed
 * for NOT and role constructs by the child's hash (8 LE bytes) and for AND/OR
 * by the wrapping sum of splitmix64(child hash) over the children (8 LE bytes,
 * order independent).  d_feat[i] = hash[i] mod 4096.  d_hash: scratch uint64
 * [n_nodes].  A malformed child index, or an op that is not a DL construct
 * (HTH_SET leaves carry no syntax to hash), sets *d_bad to 1 and hashes the
 * node as 0; nothing traps. */
hth_status hth_features(const hth_node* d_nodes, const uint32_t* d_hyp_node_offsets, uint32_t n_hyps,
                        const uint32_t* d_children, uint32_t n_children, uint64_t* d_hash,
                        uint16_t* d_feat, uint32_t* d_bad, void* stream);

/* Dense bf16 feature rows: d_x[r][f] = number of subtrees of hypothesis row0 + r
 * with feature index f, for r < n_rows (d_x is [n_rows][4096]). */
hth_status hth_densify(const uint16_t* d_feat, const uint32_t* d_hyp_node_offsets, uint32_t row0,
                       uint32_t n_rows, uint16_t* d_x, void* stream);

/* Feature rows of refinements relative to their parents: d_x[r][f] = (subtrees
 * of hypothesis row0 + r with feature f) - (subtrees of parent p with feature
 * f), p = d_parent_index[row0 + r] indexing a second feature set
 * (d_parent_feat, d_parent_offsets) of the parents.  What the refinement
 * added is positive, what it replaced negative; unchanged subtrees cancel.
 * parent_context = 1 also adds the parent's own subtree counts at feature
 * f XOR 2048 (the other half of the index space), so that the screener sees
 * what the refinement changed and what it was applied to; 0 leaves them out.
 * Errors: HTH_E_INVALID (NULL), HTH_E_RANGE (parent_context > 1). */
hth_status hth_densify_delta(const uint16_t* d_feat, const uint32_t* d_hyp_node_offsets, uint32_t row0,
                             uint32_t n_rows, const uint16_t* d_parent_feat, const uint32_t* d_parent_offsets,
                             const uint32_t* d_parent_index, uint32_t parent_context, uint16_t* d_x,
                             void* stream);

/* C[M][N] = op(A) op(B) on the MFMA units (bf16 operands, fp32 accumulation).
 * trans_a = 0: A is [M][lda]; 1: A is given transposed as [K][lda].
 * trans_b = 0: B is [K][ldb]; 1: B is given as [N][ldb].  (Both transposed is
 * HTH_E_UNSUPPORTED.)  Epilogue, in this order: + bias[n] (if bias), max(.,0)
 * (if relu), zero where mask[m][n] <= 0 (if mask, bf16 [M][ldm]); then stored
 * to c32 (fp32 [M][ldc]) and/or cbf (bf16 [M][ldcb]).  The contiguous
 * dimension of each operand and its leading dimension must be multiples of 8
 * and A, B 16-byte aligned. */
hth_status hth_gemm_bf16(int trans_a, int trans_b, int M, int N, int K, const uint16_t* A, int lda,
                         const uint16_t* B, int ldb, const float* bias, int relu, const uint16_t* mask,
                         int ldm, float* c32, int ldc, uint16_t* cbf, int ldcb, void* stream);

/* Output layer of width 2: z[b] = h[b] . w[:, o] + bias[o] (h bf16 [Bn][Kd],
 * w fp32 [Kd][2]).  With targets y (fp32 [Bn][2]) it adds the summed loss into
 * *loss and writes dz = dloss/dz * scale; loss_kind 0: BCE-with-logits (y are
 * fractions in [0, 1]); 1: squared error (z - y)^2 / 2 (y real). */
hth_status hth_head_forward(const uint16_t* h, int Bn, int Kd, const float* w, const float* bias,
                            float* z, const float* y, float* dz, float scale, float* loss, int loss_kind,
                            void* stream);

/* Screening score from the outputs z (fp32 [Bn][2]): the F1 of the predicted
 * coverage (p, q), 2p / (p + q + n_pos), with (P_b, N_b) the row's base
 * coverage (device uint32 [Bn][2], e.g. a refinement's parent) or, when base
 * is NULL, (n_pos, n_neg).  kind 0: p = sigmoid(z0) P_b, q = sigmoid(z1) N_b
 * (kept shares); kind 1 (needs base): p = P_b - expm1(z0), q = N_b - expm1(z1),
 * clamped to [0, base] (z = log(1 + removed count)). */
hth_status hth_head_score(const float* z, int Bn, float n_pos, float n_neg, const uint32_t* base, int kind,
                          float* score, void* stream);

/* Backward of the output layer: dw[k][o] = sum_b h[b][k] dz[b][o];
 * dh[b][k] = (dz[b] . w[k]) where h[b][k] > 0, else 0 (ReLU of the layer below). */
hth_status hth_head_backward(const uint16_t* h, int Bn, int Kd, const float* w, const float* dz,
                             float* dw, uint16_t* dh, void* stream);

/* out[n] = sum over m of d[m][n] (d bf16 if is_bf16, else fp32; [M][N]),
 * accumulated in fp32 in an order fixed by (M, N) alone, so repeated calls give
 * identical bits.  HTH_E_RANGE for negative sizes. */
hth_status hth_colsum(const void* d, int is_bf16, int M, int N, float* out, void* stream);

/* AdamW (decoupled weight decay) on fp32 parameters p with gradient g and
 * moments m, v; step counts from 1; pbf (optional) receives a bf16 copy. */
hth_status hth_adamw(float* p, const float* g, float* m, float* v, uint16_t* pbf, size_t n, float lr,
                     float beta1, float beta2, float eps, float wd, int step, void* stream);

/* d[i] = bf16(s[i]) (round to nearest even). */
hth_status hth_to_bf16(const float* s, uint16_t* d, size_t n, void* stream);

/* dst [cols][rows] = the transpose of the bf16 matrix src [rows][cols] (not in
 * place): the weights in the [N][K] layout that the forward layers' products
 * (trans_b = 1) read.  Errors: HTH_E_INVALID (NULL or src == dst),
 * HTH_E_RANGE (rows or cols not positive). */
hth_status hth_transpose_bf16(const uint16_t* src, int rows, int cols, uint16_t* dst, void* stream);

/* Indices of the k largest scores (d_idx [k], in no particular order; among
 * equal scores at the threshold, which ones are taken is unspecified; NaN
 * ranks last).  d_work: uint32 [65538].  Synchronous on `stream`. */
hth_status hth_topk(const float* d_scores, uint32_t n, uint32_t k, uint32_t* d_idx, uint32_t* d_work,
                    void* stream);

/* Wait for `stream`; turn an asynchronous device error into HTH_E_DEVICE. */
hth_status hth_sync(void* stream);

/* Name of a status code (static string). */
const char* hth_status_str(hth_status s);

/* Copy the calling thread's last error message into buf (NUL-terminated,
 * truncated to n bytes); returns the full message length. */
size_t hth_last_error(char* buf, size_t n);

#ifdef __cplusplus
}
#endif
#endif /* HTHEDL_H */
