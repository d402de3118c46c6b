/*
 * scuba.h - C ABI of the MI355X OOB-query decision library.
 *
 * What is decided.  For every static memory access the bounds analysis
 * builds one constraint set (paper Sec. 4.1 and Sec. 5.2, constraint kinds
 * 1-3): thread/block ids below their dimensions (kind 1), the access
 * offset reaching the allocation or partition size (kind 2), and the
 * equalities that define offset, size, grid dimensions and asserts through
 * expression trees (kind 3, Sec. 5.1, Fig. 8, Fig. 9).  The set is
 * satisfiable iff some legal input makes the access out of bounds; the paper
 * hands each set to a SAT solver and reports the satisfying ones (Sec. 5.2).
 * Here each set is a *query*; SCUBA_SAT means "OOB possible", with a witness
 * input, SCUBA_UNSAT means "in bounds for every input".
 *
 * Path: scuba_bitblast (word-level normalisation + Tseitin CNF, host)
 *       -> scuba_split (unit propagation + cube splitting, host)
 *       -> device unit propagation and bit-sliced leaf evaluation (HIP,
 *          gfx950) -> results (verdict, verified witness, leaf counts).
 * scuba_decide runs the whole loop, splitting lazily until every query is
 * decided or out of budget; scuba_solve evaluates a given cube list.
 *
 * Conventions
 *  - Every call returns scuba_status (0 = OK, < 0 = error).  Out-parameters
 *    are written only on SCUBA_OK.  No C++ exception crosses the ABI; the
 *    text of the last error of a context is returned by scuba_last_error.
 *  - Inputs are copied; the library never keeps a caller pointer after a
 *    call returns.  Handles (scuba_cnf, scuba_cubes, scuba_results) are owned
 *    by the caller and released with their *_free function.  Pointers inside
 *    a view are borrowed and stay valid until the handle is freed.
 *  - One context per host thread.  A context owns pinned host staging
 *    buffers and is bound to one HIP device, which is opened at the first
 *    call that needs it (the host-only calls work without a GPU).
 *  - Device memory is supplied by the caller as one workspace (device
 *    pointer + size); its required size comes from the *_workspace calls.
 *    Streams are hipStream_t passed as void* (0 = the null stream).  Calls
 *    that take a stream return after that stream has been synchronised.
 *  - CNF: variables 1..n_vars, DIMACS literals (+v / -v), clause c of query
 *    q spans lits[clause_off[c] .. clause_off[c+1]).  A clause may not repeat
 *    a variable.  An empty clause makes the query UNSAT.
 */
#ifndef SCUBA_H
#define SCUBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif
#if defined(__GNUC__)
#pragma GCC visibility push(default)
#endif

typedef int32_t scuba_status;
#define SCUBA_OK 0
#define SCUBA_E_INVALID (-1)   /* malformed input or argument            */
#define SCUBA_E_WIDTH (-2)     /* input width outside 1..64              */
#define SCUBA_E_NOMEM (-3)     /* host allocation failed                 */
#define SCUBA_E_DEVICE (-4)    /* a HIP call or a device check failed    */
#define SCUBA_E_CAPACITY (-5)  /* workspace or a fixed limit too small   */
#define SCUBA_E_STATE (-6)     /* call not valid for this handle         */
#define SCUBA_E_INTERNAL (-7)  /* unexpected internal error              */

typedef int32_t scuba_verdict;
#define SCUBA_UNSAT 0    /* no input makes the access out of bounds */
#define SCUBA_SAT 1      /* some input does; a witness is available  */
#define SCUBA_UNKNOWN 2  /* a budget ran out before a decision        */

/* ---------------------------------------------------------------- queries
 * A query is a DAG in topological order (Sec. 5.1: leaves are constants or
 * unknown inputs, inner nodes operators; an input used by several trees is
 * one node).  a/b index earlier nodes of the same query.
 *   VAR   width 1..64, imm = declaration number (0,1,2,... in node order);
 *         value range 0 .. 2^width - 1.
 *   CONST imm = unsigned value.
 *   ADD SUB MUL                 exact integers (no wrap-around)
 *   SHL imm<=64, UDIV/UREM imm>0 (operand must be >= 0 for every input)
 *   LT LE GT GE EQ NE           integer comparison -> boolean
 *   AND OR (a, b)  NOT (a)      boolean connectives
 * roots: boolean nodes that must all hold.                                   */
#define SCUBA_OP_VAR 0
#define SCUBA_OP_CONST 1
#define SCUBA_OP_ADD 2
#define SCUBA_OP_SUB 3
#define SCUBA_OP_MUL 4
#define SCUBA_OP_SHL 5
#define SCUBA_OP_UDIV 6
#define SCUBA_OP_UREM 7
#define SCUBA_OP_LT 8
#define SCUBA_OP_LE 9
#define SCUBA_OP_GT 10
#define SCUBA_OP_GE 11
#define SCUBA_OP_EQ 12
#define SCUBA_OP_NE 13
#define SCUBA_OP_AND 14
#define SCUBA_OP_OR 15
#define SCUBA_OP_NOT 16

typedef struct {
  uint32_t op, a, b, width;
  uint64_t imm;
} scuba_node; /* 24 bytes */

typedef struct scuba_ctx scuba_ctx;
typedef struct scuba_cnf scuba_cnf;
typedef struct scuba_cubes scuba_cubes;
typedef struct scuba_results scuba_results;

/* Context for HIP device `device` (checked at the first device call). */
scuba_status scuba_ctx_create(int32_t device, scuba_ctx** out);
void scuba_ctx_destroy(scuba_ctx* ctx);
const char* scuba_last_error(const scuba_ctx* ctx);
const char* scuba_status_str(scuba_status s);
/* Library version and the number of exported entry points (self check). */
uint32_t scuba_abi_version(void);

/* ---------------------------------------------------------------- bit-blast
 * Word-level normalisation, then Tseitin encoding (host).
 * Normalisation writes every comparison as a bound on a polynomial over the
 * inputs with coprime integer coefficients (this cancels common additive
 * terms and common positive factors), intersects the bounds the roots put on
 * the same polynomial, and marks the query UNSAT at the root when an
 * intersection is empty.  It keeps the set of satisfying inputs unchanged.
 * Encoding: exact two's-complement widths from value ranges; gates are
 * full equivalences, so auxiliary variables are functions of the inputs and
 * the CNF has exactly one model per satisfying input tuple.  Input bits get
 * the first CNF variables: declared variable i, bit j (LSB first) is
 * variable first_var[i] + j.
 * nodes/roots: concatenated per query; node_start/root_start: nq+1 offsets.
 * flags: SCUBA_BB_NO_REWRITE encodes the DAG as given (no normalisation).
 *   SCUBA_BB_WRAP(m), 1 <= m <= 64: machine integers of m bits instead of
 *   exact ones (m = 32: CUDA's 32-bit unsigned arithmetic, where an index
 *   computation can overflow).  Every integer node is an unsigned m-bit
 *   word; ADD, SUB, MUL and SHL are taken modulo 2^m; UDIV / UREM are the
 *   unsigned quotient and remainder; comparisons are unsigned; constants
 *   are reduced modulo 2^m; inputs may be at most m bits wide (else
 *   SCUBA_E_WIDTH).  No normalisation (it assumes exact integers), and the
 *   witness check uses the same arithmetic.
 * Errors: SCUBA_E_INVALID (bad op, order, type, negative division operand),
 * SCUBA_E_WIDTH (width outside 1..64).                                      */
#define SCUBA_BB_NO_REWRITE 1u
#define SCUBA_BB_WRAP(m) ((uint32_t)(m) << 8)
scuba_status scuba_bitblast(scuba_ctx* ctx, uint32_t nq, const scuba_node* nodes,
                            const uint64_t* node_start, const uint32_t* roots,
                            const uint64_t* root_start, uint32_t flags, scuba_cnf** out);

/* A CNF batch from raw arrays (random k-SAT, pigeonhole, ...).
 * n_vars[nq]; q_clause_start[nq+1] indexes clauses; clause_off[C+1] indexes
 * lits (global, non-decreasing).  Rejects repeated variables in a clause and
 * literals outside 1..n_vars (SCUBA_E_INVALID).                              */
scuba_status scuba_cnf_from_arrays(scuba_ctx* ctx, uint32_t nq, const uint32_t* n_vars,
                                   const uint64_t* q_clause_start, const uint64_t* clause_off,
                                   const int32_t* lits, scuba_cnf** out);

typedef struct {
  uint32_t n_vars;
  uint32_t n_inputs;          /* declared input variables (0 for raw CNF)   */
  uint64_t n_clauses;
  uint64_t n_lits;
  const uint64_t* clause_off; /* n_clauses+1, relative to lits below        */
  const int32_t* lits;
  int32_t root_unsat;         /* 1: normalisation proved UNSAT              */
} scuba_cnf_view;

uint32_t scuba_cnf_count(const scuba_cnf* cnf);
scuba_status scuba_cnf_view_get(const scuba_cnf* cnf, uint32_t qi, scuba_cnf_view* out);
/* first_var[i], width[i] for each declared input (cap entries at most). */
scuba_status scuba_cnf_input_map(const scuba_cnf* cnf, uint32_t qi, uint32_t* first_var,
                                 uint32_t* width, uint32_t cap);
void scuba_cnf_free(scuba_cnf* cnf);

/* ---------------------------------------------------------------- split
 * Cube splitting (host).  From the root, unit propagation runs to its
 * fixpoint; a node whose propagation conflicts is a refuted cube; a node
 * with at most k active variables (unassigned and occurring in a clause not
 * yet satisfied) becomes a leaf; otherwise the scorer picks a branching
 * variable and the 0-child is explored before the 1-child; backjumping
 * prunes a 1-child when every failure below its 0-sibling was a host
 * conflict that does not involve the branching variable.  The static
 * scorer takes the active variable with the most literal occurrences in the
 * original CNF, ties to the lowest index.  Cubes hold the branching literals
 * only.  A query whose tree exceeds max_cubes is cut (UNKNOWN).             */
#define SCUBA_SCORER_STATIC 0u
#define SCUBA_SCORER_LEARNED 1u
/* Word ordering (bit-blasted queries): the active input bit of highest
 * significance first, ties to the lowest variable, so that each decision
 * halves one input's value range and small inputs are tried first; the
 * static order for auxiliary variables and raw CNFs. */
#define SCUBA_SCORER_WORD 2u
/* Learned ordering: at a decision node the top `candidates` active variables
 * of the static order, and the most significant active bit of each input
 * word, are scored by the perceptron below (scuba_mlp_*),
 * batched over all queries on the device; the ranking orders the decisions
 * of that node and of `rescore` levels below it.  Non-finite scores fall
 * back to the static order.  master / wbf16: device parameter block and its
 * bf16 copy (see the learned-scorer section). */
typedef struct {
  const float* master;
  const uint16_t* wbf16;
  uint32_t candidates;   /* 2..64 */
  uint32_t rescore;      /* >= 1 */
} scuba_learned_scorer;

typedef struct {
  uint32_t k;            /* max active variables per leaf (<= 38)            */
  uint32_t scorer;       /* SCUBA_SCORER_*                                   */
  uint64_t max_cubes;    /* per query, leaves + refuted (at most 2^26)        */
  uint32_t max_residual; /* a leaf must also have at most this many residual
                            clauses (0 = the device limit)                   */
  uint32_t reserved;
  /* SCUBA_SCORER_LEARNED only: the scorer, device memory of at least
     scuba_scorer_workspace(cnf, candidates) bytes, and the stream         */
  const scuba_learned_scorer* learned;
  void* dev_ws;
  size_t ws_bytes;
  void* hip_stream;
} scuba_split_opts;
/* Device bytes the learned scorer needs for a batch (one row per candidate
 * of every query: `candidates` from the static order plus one per input
 * word). */
size_t scuba_scorer_workspace(const scuba_cnf* cnf, uint32_t candidates);

#define SCUBA_CUBE_LEAF 0
#define SCUBA_CUBE_REFUTED 1   /* unit propagation of the cube conflicts        */
#define SCUBA_CUBE_PRUNED 2    /* a 1-branch whose 0-sibling failed by host
                                  conflicts independent of the branching
                                  variable (backjumping): no model, but not
                                  necessarily refuted by propagation alone   */
scuba_status scuba_split(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_split_opts* opts,
                         scuba_cubes** out);
/* Cubes from arrays: q_cube_start[nq+1] indexes cubes, cube_off[ncubes+1]
 * indexes cube_lits.  Every cube is evaluated as given (no validation of
 * completeness; clashing literals make a refuted cube).                     */
scuba_status scuba_cubes_from_arrays(scuba_ctx* ctx, const scuba_cnf* cnf,
                                     const uint64_t* q_cube_start, const uint64_t* cube_off,
                                     const int32_t* cube_lits, scuba_cubes** out);
typedef struct {
  uint64_t n_cubes;
  const uint64_t* cube_off;  /* n_cubes+1, relative to lits                  */
  const int32_t* lits;
  const int32_t* kind;       /* SCUBA_CUBE_LEAF / SCUBA_CUBE_REFUTED (host)   */
  const int32_t* f;          /* active variables of leaves (host), -1 refuted */
  int32_t complete;          /* 1 if the tree was not cut by max_cubes        */
} scuba_cubes_view;
scuba_status scuba_cubes_view_get(const scuba_cubes* cubes, uint32_t qi, scuba_cubes_view* out);
void scuba_cubes_free(scuba_cubes* cubes);

/* Traces for training the scorer: the static walk of every query, and at
 * every `every`-th decision node above depth `depth` the features of the
 * candidates (the top `candidates` variables of the static order and the
 * most significant active bit of each input word) with a one-step lookahead
 * label: log2(1 + f - f0) + log2(1 + f - f1) + (r - r0) + (r - r1), with f
 * the node's active count and f0 / f1 those after propagating the variable
 * to 0 / 1 (0 for a conflict), and r, r0, r1 the same for the inputs' range
 * width in bits (sum over input words of log2(hi - lo + 1), ranges narrowed
 * by the root facts; 0 for raw CNFs and conflicts).  Rows of a node are
 * contiguous; node = query index << 32 | decision number. */
typedef struct scuba_trace scuba_trace;
typedef struct {
  uint32_t k, candidates, every, depth;
  uint64_t max_cubes;
} scuba_trace_opts;
scuba_status scuba_trace_run(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_trace_opts* opts,
                             scuba_trace** out);
/* Borrowed arrays: features[rows * 16], labels[rows], nodes[rows]. */
scuba_status scuba_trace_view(const scuba_trace* t, uint64_t* rows, const float** features,
                              const float** labels, const uint64_t** nodes);
void scuba_trace_free(scuba_trace* t);

/* ---------------------------------------------------------------- solve */
#define SCUBA_MODE_DECIDE 0u   /* stop a query at its first satisfying leaf  */
#define SCUBA_MODE_COUNT 1u    /* count every leaf's satisfying assignments   */
/* Capture each device round (upload, propagation kernel, leaf kernel,
 * download) as a HIP graph, once per round shape, and replay it on a
 * library-owned stream ordered after the caller's stream; later rounds of
 * the same shape (the same batch solved again) replay without capture.
 * The graphs belong to the context (at most 64, least recently used
 * dropped) and are released by scuba_ctx_destroy. */
#define SCUBA_SOLVE_GRAPH 1u
/* scuba_decide only: split on the device instead of the host.  Each open
 * query's root is the start node of a work stack in device memory; every
 * step pops up to split_batch nodes, propagates each from its parent's
 * fixpoint and one decision literal, and turns it into a refuted cube, a
 * leaf (at most k active variables and max_residual unsatisfied clauses:
 * evaluated by the leaf kernel in the same step) or a branching node whose
 * two children are pushed (the branching variable is the first active one
 * of the static or word order, its 0-branch explored first).  Sec. 4.1 and
 * Sec. 5.2 fix what a query decides; the splitting order is the solver's.
 * Without host word-level bounds or backjumping, the device tree holds the
 * host tree's leaves that have models and possibly more model-free ones;
 * verdicts are the same.  DECIDE or COUNT mode (COUNT: scuba_leaf_get gives
 * each leaf in emission order); static or word scorer; no graphs.
 * Steps shrink to single nodes (depth first) when the stack nears its
 * capacity, which never runs out as long as it holds the start nodes and
 * one path.  scuba_decide_workspace gives the bytes for the default stack
 * (64 x split_batch nodes plus one path); a larger workspace holds a
 * larger stack and needs fewer single-node steps.                         */
#define SCUBA_SOLVE_DEVICE_SPLIT 2u
/* Leaf evaluation with the block-level skip test on the vector unit: 64
 * clauses per test and ballot, each clause that no block-level literal
 * satisfies broadcast to the wave; without this flag the test runs per
 * clause on the scalar unit.  Same counts, witnesses and verdicts.        */
#define SCUBA_SOLVE_LEAF_VECTOR 4u
/* With SCUBA_SOLVE_LEAF_VECTOR: each work item's clause records are staged
 * in LDS by the whole workgroup first (when they fit), instead of every
 * wave reading them through the caches (not with the device split).     */
#define SCUBA_SOLVE_LEAF_LDS 8u
typedef struct {
  uint32_t mode;             /* SCUBA_MODE_*                                  */
  uint32_t k;                /* split bound for scuba_decide (<= 38)          */
  uint64_t max_cubes;        /* per query budget for scuba_decide (<= 2^26;
                                0 = 100000)                                   */
  uint32_t leaves_per_round; /* lazily split leaves per query per round       */
  uint32_t chunk_log2;       /* leaf work item = 2^chunk_log2 blocks of 4096
                                assignments                                   */
  uint32_t grid;             /* persistent workgroups (0 = 8 per CU)          */
  uint32_t max_rounds;       /* scuba_decide rounds (0 = unbounded)           */
  uint32_t scorer;           /* SCUBA_SCORER_*                                */
  uint32_t flags;            /* SCUBA_SOLVE_*                                 */
  const scuba_learned_scorer* learned;   /* SCUBA_SCORER_LEARNED only; its
                                 buffers come from the end of the workspace */
  uint32_t max_residual;     /* scuba_decide: a leaf's residual clauses must
                                fit this tile (16 B each, in LDS; 0 = 2048,
                                at most 8192)                                 */
  uint32_t split_batch;      /* SCUBA_SOLVE_DEVICE_SPLIT: nodes expanded per
                                step (0 = 16384, fewer when the residual
                                records of that many leaves would exceed
                                512 MiB; at most 2^20)                        */
} scuba_solve_opts;

/* Device bytes scuba_solve / scuba_decide need for this batch. */
scuba_status scuba_solve_workspace(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_cubes* cubes,
                                   const scuba_solve_opts* opts, size_t* bytes);
scuba_status scuba_decide_workspace(scuba_ctx* ctx, const scuba_cnf* cnf,
                                    const scuba_solve_opts* opts, size_t* bytes);

/* Evaluate every cube of `cubes` on the device: unit propagation, then
 * the bit-sliced exhaustive leaf evaluation.  COUNT mode fills per-cube
 * (refuted, f, m, count, first satisfying index); DECIDE mode stops a query
 * at its first satisfying leaf (smallest cube index, then smallest
 * assignment index).  Verdict: SAT if a leaf is satisfiable, UNSAT if the
 * cube list is complete and no leaf is, else UNKNOWN.
 * dev_ws: device memory of at least scuba_solve_workspace bytes.           */
scuba_status scuba_solve(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_cubes* cubes,
                         const scuba_solve_opts* opts, void* dev_ws, size_t ws_bytes,
                         void* hip_stream, scuba_results** out);

/* The whole path for a batch: split lazily (leaves_per_round per query per
 * round, DFS order), evaluate each round's leaves on the device, drop the
 * queries that are decided, repeat until every query is decided, its tree
 * is exhausted, or its budget is spent.  With a learned scorer the scoring
 * passes run on a library-owned stream ordered after the caller's stream
 * (so after its earlier work, such as scuba_mlp_sync of the weights), and
 * do not wait for the CNF upload that this call queues on the caller's
 * stream.                                                                  */
scuba_status scuba_decide(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_solve_opts* opts,
                          void* dev_ws, size_t ws_bytes, void* hip_stream, scuba_results** out);

/* Allocation-free scuba_decide, for callers that cannot allocate: code
 * under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same loop, kernels and results as scuba_decide, with the
 * device workspace taken from a scratch array of the library's own
 * (SCUBA_NOALLOC_SCRATCH_BYTES, one per GPU, held until the process ends)
 * and the host staging in pageable memory: the call makes no hipMalloc,
 * hipFree, hipHostMalloc or hipHostFree (host heap memory of the splitter
 * aside).
 * Errors: SCUBA_E_CAPACITY when the batch needs more device bytes than the
 * scratch holds (scuba_decide_workspace gives the need; split the batch);
 * SCUBA_E_INVALID with SCUBA_SOLVE_GRAPH (no graphs are captured here).
 * Every call on one GPU shares that GPU's scratch and leaves its contents
 * there; each call uploads everything its kernels read before they run, so
 * consecutive calls are independent, but calls that overlap in time on one
 * GPU (two contexts on two threads) race and give wrong results.          */
#define SCUBA_NOALLOC_SCRATCH_BYTES (128u << 20)
scuba_status scuba_decide_noalloc(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_solve_opts* opts,
                                  void* hip_stream, scuba_results** out);

/* ---------------------------------------------------------------- autotune
 * Picks k, chunk_log2, leaves_per_round and grid for scuba_decide on this
 * batch.  A size-stratified sample of the queries is decided at every
 * point of a coordinate sweep, one coordinate at a time, each keeping the
 * best point before the next: k in {16, 20, 24, 28, 30}, chunk_log2 in
 * {4, 6, 8, 10, 12}, leaves_per_round in {1, 2, 4, 8, 16}, grid in
 * {2, 4, 8, 16} workgroups per CU, leaf tile (max_residual) in {1024,
 * 2048, 4096, 8192} clauses, leaf variant (scalar skip test, vector skip
 * test, vector with LDS-staged records); a point's time is the best wall time of
 * `reps` runs.  Every point must give the same decided verdicts (UNKNOWN is
 * compatible with SAT and UNSAT); a contradiction is SCUBA_E_INTERNAL.  The
 * choice is cached in the context per bucket (log2 of the mean clause
 * count, log2 of the batch size, scorer, flags): a cached bucket returns
 * at once.  Points whose workspace exceeds ws_bytes are skipped;
 * scuba_autotune_workspace gives the bytes for every point.             */
typedef struct {
  uint32_t sample;       /* queries decided per point (0 = 128)              */
  uint32_t reps;         /* timed runs per point, best taken (0 = 2)         */
  uint64_t max_cubes;    /* per query while tuning (0 = 20000)               */
  uint32_t scorer;       /* SCUBA_SCORER_STATIC or SCUBA_SCORER_WORD          */
  uint32_t flags;        /* SCUBA_SOLVE_* used while tuning and returned     */
  uint32_t refresh;      /* 1: ignore the cache                              */
  uint32_t reserved;
} scuba_tune_opts;
typedef struct {
  uint32_t points;       /* points decided (0 when served from the cache)    */
  uint32_t cached;       /* 1 when served from the cache                     */
  double best_ms;        /* sample wall time at the chosen point             */
  double default_ms;     /* sample wall time at the library defaults         */
} scuba_tune_report;
scuba_status scuba_autotune_workspace(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_tune_opts* opts,
                                      size_t* bytes);
/* The autotuner's cache of a context, persisted: scuba_tune_cache_save
 * writes one JSON object per line (the device's architecture name, the
 * bucket and the chosen options); scuba_tune_cache_load adds the lines of
 * the device this context runs on and reports how many (lines of another
 * architecture are skipped; a malformed line or options the library would
 * reject are SCUBA_E_INVALID).  A context without a device keys its lines
 * "no-device".                                                            */
scuba_status scuba_tune_cache_save(scuba_ctx* ctx, const char* path);
scuba_status scuba_tune_cache_load(scuba_ctx* ctx, const char* path, uint32_t* loaded);
/* best: a complete scuba_solve_opts for scuba_decide on this batch. */
scuba_status scuba_autotune(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_tune_opts* opts, void* dev_ws,
                            size_t ws_bytes, void* hip_stream, scuba_solve_opts* best,
                            scuba_tune_report* report);

/* ---------------------------------------------------------------- learned scorer
 * A perceptron scoring candidate branching variables: 16 features -> 128 ->
 * 128 -> 1, ReLU, bf16 weights and activations, fp32 accumulation on the
 * matrix cores; trained by mean squared error with Adam on fp32 master
 * weights.  Parameter block (fp32, scuba_mlp_param_count() values):
 *   W1[16][128] | b1[128] | W2[128][128] | b2[128] | w3[128] | b3[1]
 * and a bf16 copy with the same offsets.  All pointers below are device
 * pointers (row-major); the calls queue work on the stream and return
 * without synchronising it.  x: batch x 16 bf16; a1, a2, dz1, dz2:
 * batch x 128 bf16; y, target: batch fp32; grad/m/v: parameter-sized fp32. */
#define SCUBA_MLP_FEATURES 16
#define SCUBA_MLP_HIDDEN 128
uint32_t scuba_mlp_param_count(void);
scuba_status scuba_mlp_sync(scuba_ctx* ctx, const float* master, uint16_t* wbf16, void* hip_stream);
scuba_status scuba_mlp_forward(scuba_ctx* ctx, const uint16_t* wbf16, const float* master, const uint16_t* x,
                               uint32_t batch, uint16_t* a1, uint16_t* a2, float* y, void* hip_stream);
scuba_status scuba_mlp_backward(scuba_ctx* ctx, const uint16_t* wbf16, const uint16_t* x, const uint16_t* a1,
                                const uint16_t* a2, const float* y, const float* target, uint32_t batch,
                                uint16_t* dz1, uint16_t* dz2, float* grad, void* hip_stream);
scuba_status scuba_mlp_adam(scuba_ctx* ctx, float* master, const float* grad, float* m, float* v,
                            uint16_t* wbf16, uint32_t step, float lr, float beta1, float beta2, float eps,
                            void* hip_stream);

/* ---------------------------------------------------------------- results */
#define SCUBA_HOW_ROOT 0    /* decided by normalisation / root propagation */
#define SCUBA_HOW_DEVICE 1  /* decided by device leaves                      */
#define SCUBA_HOW_BUDGET 2  /* undecided: budget                             */
typedef struct {
  scuba_verdict verdict;
  int32_t how;               /* SCUBA_HOW_*                                   */
  uint64_t cubes_total;      /* leaves + refuted cubes produced               */
  uint64_t cubes_refuted;    /* refuted by host propagation                   */
  uint64_t leaves_sent;      /* leaves evaluated on the device                */
  uint64_t leaves_refuted;   /* leaves the device propagation refuted         */
  uint64_t blocks_evaluated; /* 4096-assignment blocks evaluated              */
  uint64_t clause_blocks;    /* clause x block evaluations on the VALU        */
  uint32_t rounds;
  int32_t witness_checked;   /* 1: model satisfies every clause and (for
                                bit-blasted queries) the exact integer query */
  uint64_t word_ops;         /* 64-bit word operations of the leaf
                                evaluation: 64 words x (|c| + 1) for every
                                residual clause c evaluated on a block     */
} scuba_query_result;

typedef struct {
  int32_t refuted;           /* 1: device propagation conflicted             */
  int32_t f, m;              /* active / other unassigned variables          */
  int32_t reserved;
  uint64_t count;            /* satisfying assignments of the active vars    */
  int64_t first;             /* smallest satisfying index (-1 none; DECIDE:
                                only the deciding leaf)                      */
} scuba_leaf_result;

scuba_status scuba_result_get(const scuba_results* r, uint32_t qi, scuba_query_result* out);
/* Integer value of each declared input for a SAT query (n <= 64 bits each). */
scuba_status scuba_witness_get(const scuba_results* r, uint32_t qi, uint64_t* values, uint32_t n);
/* Full CNF model (n_vars+1 bytes, index 0 unused) of a SAT query. */
scuba_status scuba_model_get(const scuba_results* r, uint32_t qi, uint8_t* bits, uint32_t n);
/* Per-cube results of scuba_solve (cube order of the input list). */
scuba_status scuba_leaf_get(const scuba_results* r, uint32_t qi, uint64_t cube,
                            scuba_leaf_result* out);
/* Stage times in ms: [0] host split, [1] upload, [2] device kernels (HIP
 * events on the caller's stream), [3] download, [4] verify, [5] total wall,
 * [6] propagation kernel, [7] leaf kernel; then launch counts: [8]
 * propagation kernel, [9] leaf kernel; with SCUBA_SOLVE_GRAPH: [10] graph
 * replays in ms (copies included; [1], [3], [6], [7] stay 0), [11] graph
 * replays, [12] graph captures; with the learned scorer (scuba_decide):
 * [13] ms in the scoring passes' copies, kernel and wait, [14] passes,
 * [15] candidate rows scored; [16] cubes and [17] leaf work items sent to
 * the kernels; [18] propagation launches whose cubes all carried the
 * host's fixpoint (fix_kernel, counted in [8] too).  n <= 19.               */
scuba_status scuba_results_timing(const scuba_results* r, double* ms, uint32_t n);
void scuba_results_free(scuba_results* r);

#if defined(__GNUC__)
#pragma GCC visibility pop
#endif
#ifdef __cplusplus
}
#endif
#endif /* SCUBA_H */
