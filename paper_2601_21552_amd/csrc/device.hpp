// Plain C++ interface between the host library and the HIP code.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace scuba {

// One query's CNF on the device.
struct DevQueryDesc {
  uint64_t coff_base;   // index into the clause-offset array (u32, relative)
  uint64_t lit_base;    // index into the literal array
  uint64_t occ_off_base;  // index into the occurrence offsets (u32, relative;
                          // literal index 2*v + (negative))
  uint64_t occ_base;    // index into the occurrence lists (clause numbers)
  uint32_t n_clauses;
  uint32_t n_vars;
  uint32_t staged;      // 1: the propagation kernel copies the CNF to LDS
  uint32_t pad;
};

// One cube to evaluate.  Either its literals (propagated from the empty
// assignment) or, with kCubeFixpoint set in n_lits, a fixpoint the host has
// already propagated: 2*nw words at lit_off, the bitmaps T then F (variable
// true / false) of nw = n_vars/32 + 1 words each, which the device checks by
// visiting every clause once (and propagates further should any be unit).
constexpr uint32_t kCubeFixpoint = 1u << 31;
struct DevCubeDesc {
  uint32_t qid;
  uint32_t lit_off;     // into the round's cube literal array
  uint32_t n_lits;      // literals, or kCubeFixpoint | 2*nw words
  uint32_t seq;         // position of the cube in its query's cube order
  int32_t f_expect;     // host propagation's active count (-1: unknown)
  uint32_t nres_cap;    // residual records reserved for this cube
  uint64_t res_base;    // first residual record
};

// Per-cube device results.
struct DevCubeOut {
  int32_t status;       // 0 ok, 1 refuted, 2 host/device mismatch, 3 capacity
  int32_t f, m, nres;
  uint64_t count;       // satisfying assignments (COUNT mode)
  uint64_t first;       // smallest satisfying index (~0: none found)
  uint64_t blocks;      // 4096-assignment blocks evaluated
  uint64_t clause_blocks;  // clause x block evaluations on the VALU
  uint64_t word_ops;       // sum over them of 64 words x (|c| + 1)
};

// A slice of one leaf: blocks [it_lo, it_hi) of 4096 assignments.
struct DevItem {
  uint32_t cube, it_lo, it_hi, pad;
};

struct RoundTimes {
  double up_ms = 0, leaf_ms = 0, h2d_ms = 0, d2h_ms = 0;
  uint32_t up_launches = 0, leaf_launches = 0;
  uint32_t fix_launches = 0;      // propagation launches of the host-fixpoint kernel
  double graph_ms = 0;            // replays of captured rounds (copies included)
  uint32_t graph_launches = 0, graph_captures = 0;
  uint64_t cubes = 0, items = 0;  // sent to the kernels
};

// Captured rounds (HIP graphs) of one context, keyed by everything a
// round's graph bakes in (pointers, sizes, launch shapes), with the stream
// they are captured and replayed on.
struct DevGraphs;
DevGraphs* dev_graphs_create(int device);
void dev_graphs_destroy(DevGraphs* g);

// Bytes of the per-device scratch array of the allocation-free decide
// entry point (SCUBA_NOALLOC_SCRATCH_BYTES in the C header).
constexpr size_t kScratchBytes = size_t(SCUBA_NOALLOC_SCRATCH_BYTES);

// Device context: a device id, its CU count and events.
struct DeviceInfo {
  int device = 0;
  int cus = 256;
  void* scratch = nullptr;     // device address of the scratch array
  size_t scratch_bytes = 0;
  size_t max_lds = 65536;      // dynamic LDS a kernel may use by default
  size_t up_lds_max = 65536;   // dynamic LDS the propagation kernel may use
  size_t leaf_lds_max = 65536; // dynamic LDS the leaf kernel may use
  char arch[64] = "";          // gcnArchName of the device
};

// Host staging for one launch pair; the layout inside the workspace is
// computed by the device code.
struct RoundHost {
  std::vector<DevCubeDesc> cubes;
  std::vector<int32_t> cube_lits;
  std::vector<DevItem> items;
  uint64_t res_records = 0;   // residual records to reserve
  uint32_t tile_max = 0;      // largest residual of a cube
  uint32_t nw_max = 0;        // largest bitmap (32-bit words) of a query
  uint32_t leaf_variant = 0;  // kLeafScalar / kLeafVector / kLeafVectorLds
};
// Leaf-evaluation variants: the per-clause block-level skip test on the
// scalar unit (records read with scalar loads), on the vector unit (64
// clauses per test, records read with vector loads), or on the vector unit
// with each work item's records staged in LDS first.
constexpr uint32_t kLeafScalar = 0, kLeafVector = 1, kLeafVectorLds = 2;

// Device image of a CNF batch: descriptors and array sizes.  The arrays
// (query-relative clause offsets, literals, per-literal occurrence offsets
// and lists) are written straight into the staging buffer at upload.
struct CnfHost {
  const scuba_cnf* src = nullptr;
  std::vector<DevQueryDesc> q;
  size_t n_coff = 0, n_lits = 0;
  size_t n_occ_off = 0;       // per query: 2*(n_vars+1)+1 offsets
  size_t n_occ = 0;           // per query: the clauses of each literal
  size_t stage_bytes = 0;     // LDS for the largest staged CNF (16-bit form)
  bool skip_root_unsat = false;   // queries decided at the root are not uploaded
  bool no_occ = false;            // uploaded without occurrence lists (host-fixpoint rounds only)
};

void dev_init(DeviceInfo* info, int device);
void dev_copy_h2d(void* dst, const void* src, size_t bytes, void* stream);
void dev_copy_d2h(void* dst, const void* src, size_t bytes, void* stream);
void dev_sync(void* stream);
void* dev_score_stream(int device, void* after);
void* dev_pinned(size_t bytes);          // pinned host memory (or throws)
void dev_pinned_free(void* p);

// Frontier queue of the propagation kernel (entries per buffer; two buffers
// in LDS).  A round whose new assignments overflow it is followed by a full
// clause scan.
constexpr uint32_t kUpQueue = 512;
// Cubes per workgroup of the propagation kernel (one per wave); they share
// the staged CNF of their query.
constexpr uint32_t kUpWaves = 4;

// Workspace layout.  The CNF region persists across rounds of one call.
size_t dev_cnf_bytes(const CnfHost& cnf);
size_t dev_round_bytes(size_t n_cubes, size_t n_cube_lits, size_t n_items, uint64_t res_records);

// Upload the CNF and reset the per-query witness keys (stream-ordered).
// With wait false the copy may still run on return: the staging buffer must
// stay untouched until the stream has passed it.  Without with_occ the
// occurrence lists are neither written nor copied: only rounds whose cubes
// all carry host fixpoints (fix_kernel) may follow.
void dev_upload_cnf(const DeviceInfo& info, void* ws, size_t ws_bytes, const CnfHost& cnf,
                    void* stream, void* staging, size_t staging_bytes, bool wait, bool with_occ = true);

// Run one round: upload, unit propagation kernel, leaf kernel, download.
// outs (n_cubes) and qkeys (nq) are filled; the stream is synchronised.
// With graphs, the round is captured once per shape and replayed on the
// cache's stream (ordered after the caller's stream).
void dev_round(const DeviceInfo& info, void* ws, size_t ws_bytes, const CnfHost& cnf,
               const RoundHost& round, uint32_t mode, uint32_t grid, void* stream, void* staging,
               size_t staging_bytes, std::vector<DevCubeOut>* outs, std::vector<uint64_t>* qkeys,
               RoundTimes* times, DevGraphs* graphs = nullptr);

// The same round in two halves, so that the host can work while it runs:
// dev_round_begin enqueues it (the staging buffer and the workspace's round
// region belong to it until dev_round_end), dev_round_end waits for it and
// fills outs and qkeys.  A pending round that is never ended is waited for
// and released by the destructor.
struct DevRoundPending {
  bool active = false, graph = false;
  int device = 0;
  void* sync_stream = nullptr;
  void* ev[9] = {};
  uint32_t gu = 0, gl = 0, fix_only = 0;
  size_t nc = 0, nq = 0;
  void* staging = nullptr;
  DevRoundPending() = default;
  DevRoundPending(const DevRoundPending&) = delete;
  DevRoundPending& operator=(const DevRoundPending&) = delete;
  ~DevRoundPending();
};
void dev_round_begin(const DeviceInfo& info, void* ws, size_t ws_bytes, const CnfHost& cnf, const RoundHost& rh,
                     uint32_t mode, uint32_t grid, void* stream, void* staging, size_t staging_bytes,
                     RoundTimes* times, DevGraphs* graphs, DevRoundPending* pend);
void dev_round_end(DevRoundPending* pend, std::vector<DevCubeOut>* outs, std::vector<uint64_t>* qkeys,
                   RoundTimes* times);
void dev_round_release(DevRoundPending* pend);

// ---------------------------------------------------------------- device split
// Splitting on the device (scuba_decide with SCUBA_SOLVE_DEVICE_SPLIT): a
// work stack of nodes in device memory.  A node is a query, the fixpoint of
// its parent (two bitmaps of nw_max words, T then F, stored beside the
// stack) and the decision literal to add; a start node (lit = 0) is
// propagated from the empty assignment with its literals
// [lit_off, lit_off + n_lits) of the start-literal array.
struct DevSplitNode {
  uint32_t qid;
  int32_t lit;
  uint32_t lit_off, n_lits;
};
// What the expansion of one popped node found.
struct DevSplitOut {
  uint32_t kind;        // kSplit* below
  int32_t lit;          // branch: the literal of the branch explored first
  int32_t f, m;         // active / other unassigned variables
  uint32_t nres, qid, pad0, pad1;
};
constexpr uint32_t kSplitDropped = 0;   // its query is decided or out of budget
constexpr uint32_t kSplitLeaf = 1;
constexpr uint32_t kSplitBranch = 2;
constexpr uint32_t kSplitRefuted = 3;
// A leaf's blocks are cut into at most this many work items.
constexpr uint32_t kSplitItemsPerLeaf = 64;
// A query with this many clauses or more is split "wide": a node's slots are
// its unassigned variables (no active-set scan per node), the branch is the
// first unassigned variable of the order, and the batch is one node per
// query (each query's walk goes depth-first).
constexpr uint64_t kSplitWideClauses = 16384;
// Per-query counters of the device split.
struct DevSplitStat {
  unsigned long long cubes;    // leaves + refuted nodes
  unsigned long long refuted;
  unsigned long long leaves;   // leaves evaluated
  unsigned long long blocks, clause_blocks, word_ops;
  uint32_t budget;             // 1: a node was dropped for the cube budget
  uint32_t pad;
};

struct SplitRun {
  uint32_t k = 30, max_res = 2048, mode = 0, chunk_log2 = 8, grid = 0;
  uint32_t batch = 0;          // nodes expanded per step
  uint64_t max_cubes = 0;
  uint32_t nw_max = 1;         // bitmap words of the largest query
  uint32_t nres_max = 1;       // residual records a leaf may need
  size_t stack_cap = 0;        // nodes the stack holds
  uint32_t leaf_variant = 0;   // kLeaf*
};
struct SplitOutput {
  std::vector<uint64_t> qkeys;              // per query: smallest (leaf sequence << 38 | index), ~0 none
  std::vector<DevSplitStat> stats;          // per query
  std::vector<uint32_t> wit;                // per query 2*nw_max words: T, F of the witness leaf
  std::vector<std::vector<DevCubeOut>> leaves;   // COUNT mode: each query's leaves, in emission order
  bool stopped = false;                     // the leaf sequence space ran out: open queries undecided
  uint64_t steps = 0, nodes = 0, max_stack = 0;
  double expand_ms = 0, leaf_ms = 0, other_ms = 0;
};
// Device bytes of the split region (after the CNF) for `cnf`, an order
// array of n_order entries and the run's batch, residual bound and stack.
size_t dev_split_bytes(const CnfHost& cnf, size_t n_order, const SplitRun& r);
// Bytes of one stack node (record and fixpoint).
size_t dev_split_node_bytes(uint32_t nw_max);
// Host staging bytes dev_split needs.
size_t dev_split_staging(const CnfHost& cnf, size_t n_order, size_t n_start, const SplitRun& r);
// The whole split-and-evaluate loop for the start queries `start` (one start
// node each, from the root).  order_off[q] indexes the concatenated branch
// orders (variables, first choice first).  The CNF must already be uploaded
// (dev_upload_cnf); the stream is synchronised on return.
void dev_split(const DeviceInfo& info, void* ws, size_t ws_bytes, const CnfHost& cnf,
               const std::vector<uint64_t>& order_off, const std::vector<uint32_t>& order,
               const std::vector<uint32_t>& start, const SplitRun& r, void* stream, void* staging,
               size_t staging_bytes, SplitOutput* out);

}  // namespace scuba
