// C ABI of the library: handles, the split/solve/decide drivers and results.
#include <algorithm>
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <limits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>

#include "bigint.hpp"
#include "common.hpp"
#include "device.hpp"
#include "mlp.hpp"
#include "parallel.hpp"
#include "split.hpp"

using namespace scuba;

struct scuba_ctx {
  int32_t device = 0;
  bool dev_ready = false;
  DeviceInfo dev;
  std::string err;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  // pinned staging of the CNF upload, apart from the rounds' staging so that
  // the upload can run while the host splits
  void* cnf_pinned = nullptr;
  size_t cnf_pinned_bytes = 0;
  DevGraphs* graphs = nullptr;
  // staging in pageable host memory instead of pinned (the allocation-free
  // entry point sets it for the duration of its call)
  bool pageable = false;
  std::vector<char> pageable_stg, pageable_cnf_stg, pageable_score_stg;
  // the learned scorer's own staging: its passes run while a round, which
  // owns the round staging until it ends, is on the device
  void* score_pinned = nullptr;
  size_t score_pinned_bytes = 0;
  // autotuner choices per size bucket (see scuba_autotune)
  std::map<std::vector<uint64_t>, scuba_solve_opts> tuned;

  void ensure_device() {
    if (!dev_ready) {
      dev_init(&dev, device);
      dev_ready = true;
    }
  }
  void* staging(size_t bytes) {
    if (pageable) {
      if (bytes > pageable_stg.size()) pageable_stg.resize(bytes);
      return pageable_stg.data();
    }
    if (bytes > pinned_bytes) {
      dev_pinned_free(pinned);
      pinned = nullptr;
      pinned_bytes = 0;
      size_t want = std::max<size_t>(bytes, size_t(1) << 20);
      pinned = dev_pinned(want);
      pinned_bytes = want;
    }
    return pinned;
  }
  void* cnf_staging(size_t bytes) {
    if (pageable) {
      if (bytes > pageable_cnf_stg.size()) pageable_cnf_stg.resize(bytes);
      return pageable_cnf_stg.data();
    }
    if (bytes > cnf_pinned_bytes) {
      dev_pinned_free(cnf_pinned);
      cnf_pinned = nullptr;
      cnf_pinned_bytes = 0;
      size_t want = std::max<size_t>(bytes, size_t(1) << 20);
      cnf_pinned = dev_pinned(want);
      cnf_pinned_bytes = want;
    }
    return cnf_pinned;
  }
  void* score_staging(size_t bytes) {
    if (pageable) {
      if (bytes > pageable_score_stg.size()) pageable_score_stg.resize(bytes);
      return pageable_score_stg.data();
    }
    if (bytes > score_pinned_bytes) {
      dev_pinned_free(score_pinned);
      score_pinned = nullptr;
      score_pinned_bytes = 0;
      score_pinned = dev_pinned(bytes);
      score_pinned_bytes = bytes;
    }
    return score_pinned;
  }
  size_t staging_size() const { return pageable ? pageable_stg.size() : pinned_bytes; }
  size_t cnf_staging_size() const { return pageable ? pageable_cnf_stg.size() : cnf_pinned_bytes; }
  DevGraphs* graph_cache() {
    if (!graphs) graphs = dev_graphs_create(device);
    return graphs;
  }
  ~scuba_ctx() {
    dev_graphs_destroy(graphs);
    dev_pinned_free(pinned);
    dev_pinned_free(cnf_pinned);
    dev_pinned_free(score_pinned);
  }
};

struct scuba_cubes {
  struct Q {
    std::vector<uint64_t> off{0};
    std::vector<int32_t> lits;
    std::vector<int32_t> kind, f;
    std::vector<uint32_t> nres;
    bool complete = true;
  };
  std::vector<Q> q;
};

struct scuba_results {
  struct Q {
    scuba_query_result r{};
    std::vector<uint8_t> model;
    std::vector<uint64_t> witness;
    std::vector<scuba_leaf_result> leaves;
  };
  std::vector<Q> q;
  double ms[19] = {};
};

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

template <typename F>
scuba_status guard(scuba_ctx* ctx, F&& f) {
  try {
    f();
    return SCUBA_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "out of host memory";
    return SCUBA_E_NOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return SCUBA_E_INTERNAL;
  } catch (...) {
    if (ctx) ctx->err = "unknown error";
    return SCUBA_E_INTERNAL;
  }
}

constexpr uint32_t kDefaultK = 30;
constexpr uint32_t kDefaultLeavesPerRound = 4;
constexpr uint32_t kDefaultChunkLog2 = 8;
constexpr uint64_t kDefaultMaxCubes = 100000;
constexpr uint32_t kMaxCubeLen = 4096;
constexpr uint64_t kMaxCubesPerQuery = uint64_t(1) << 26;

struct Opts {
  uint32_t mode, k, lpr, chunk_log2, grid, max_rounds, scorer;
  uint64_t max_cubes;
  const scuba_learned_scorer* learned;
  uint32_t flags;
  uint32_t max_res;
  uint32_t split_batch;
};
Opts resolve(const scuba_solve_opts* o) {
  Opts r{SCUBA_MODE_DECIDE, kDefaultK, kDefaultLeavesPerRound, kDefaultChunkLog2, 0, 0, 0, kDefaultMaxCubes,
         nullptr, 0, kDefaultMaxResidual, 0};
  if (o) {
    r.mode = o->mode;
    if (o->k) r.k = o->k;
    if (o->leaves_per_round) r.lpr = o->leaves_per_round;
    if (o->chunk_log2) r.chunk_log2 = o->chunk_log2;
    r.grid = o->grid;
    r.max_rounds = o->max_rounds;
    r.scorer = o->scorer;
    if (o->max_cubes) r.max_cubes = o->max_cubes;
    r.learned = o->learned;
    r.flags = o->flags;
    if (o->max_residual) r.max_res = o->max_residual;
    r.split_batch = o->split_batch;
  }
  if (r.max_res > 8192) fail(SCUBA_E_INVALID, "max_residual above 8192");
  // the device's witness key is (cube sequence << 38) | assignment index:
  // a query's cube sequence numbers must stay below 2^26
  if (r.max_cubes > kMaxCubesPerQuery) fail(SCUBA_E_INVALID, "max_cubes above 2^26 per query");
  if (r.flags & ~(SCUBA_SOLVE_GRAPH | SCUBA_SOLVE_DEVICE_SPLIT | SCUBA_SOLVE_LEAF_VECTOR | SCUBA_SOLVE_LEAF_LDS))
    fail(SCUBA_E_INVALID, "unknown solve flags");
  if ((r.flags & SCUBA_SOLVE_LEAF_LDS) && !(r.flags & SCUBA_SOLVE_LEAF_VECTOR))
    fail(SCUBA_E_INVALID, "SCUBA_SOLVE_LEAF_LDS needs SCUBA_SOLVE_LEAF_VECTOR");
  if (r.flags & SCUBA_SOLVE_DEVICE_SPLIT) {
    if (r.flags & SCUBA_SOLVE_GRAPH) fail(SCUBA_E_INVALID, "the device split captures no graphs");
    if (r.scorer == SCUBA_SCORER_LEARNED) fail(SCUBA_E_INVALID, "the device split takes the static or word order");
    if (r.split_batch > (1u << 20)) fail(SCUBA_E_INVALID, "split_batch above 2^20");
    if (r.flags & SCUBA_SOLVE_LEAF_LDS) fail(SCUBA_E_INVALID, "the device split reads leaf records from memory");
  }
  if (r.mode > SCUBA_MODE_COUNT) fail(SCUBA_E_INVALID, "unknown mode");
  if (r.k > kMaxLeafVars) fail(SCUBA_E_INVALID, "k above the leaf limit of 38 variables");
  if (r.chunk_log2 > 26) fail(SCUBA_E_INVALID, "chunk_log2 above 26");
  if (r.scorer > SCUBA_SCORER_WORD) fail(SCUBA_E_INVALID, "unknown scorer");
  if (r.scorer == SCUBA_SCORER_LEARNED) {
    const scuba_learned_scorer* l = r.learned;
    if (!l || !l->master || !l->wbf16) fail(SCUBA_E_INVALID, "learned scorer without parameters");
    if (l->candidates < 2 || l->candidates > 64) fail(SCUBA_E_INVALID, "scorer candidates outside 2..64");
    if (l->rescore < 1) fail(SCUBA_E_INVALID, "scorer rescore must be >= 1");
  } else {
    r.learned = nullptr;
  }
  return r;
}

// Device image of the CNF batch.  A query whose CNF fits the LDS left over
// by the propagation kernel's bitmaps (16-bit literals and offsets) is
// marked for staging; lds_limit = 0 disables staging.
uint32_t leaf_variant(const Opts& o) {
  if (!(o.flags & SCUBA_SOLVE_LEAF_VECTOR)) return kLeafScalar;
  return (o.flags & SCUBA_SOLVE_LEAF_LDS) ? kLeafVectorLds : kLeafVector;
}

// Device descriptors of a CNF batch.  With skip_root_unsat, the queries
// decided at the root get empty descriptors and are not uploaded (DECIDE
// sends them no cube).
CnfHost cnf_host(const scuba_cnf* cnf, size_t lds_limit = 0, bool skip_root_unsat = false) {
  CnfHost h;
  h.src = cnf;
  h.skip_root_unsat = skip_root_unsat;
  uint32_t nw_all = 0;
  for (const CnfQuery& q : cnf->q) nw_all = std::max(nw_all, (q.n_vars >> 5) + 1);
  // per wave: four bitmaps, two frontier queues and 128 words of scan space
  const size_t bitmaps = kUpWaves * (size_t(nw_all) * 16 + 2 * kUpQueue * 4 + 128 * 4);
  const size_t budget = lds_limit > bitmaps ? lds_limit - bitmaps : 0;
  for (const CnfQuery& q : cnf->q) {
    DevQueryDesc d{};
    d.coff_base = h.n_coff;
    d.lit_base = h.n_lits;
    d.occ_off_base = h.n_occ_off;
    d.occ_base = h.n_occ;
    if (skip_root_unsat && q.root_unsat) {
      h.q.push_back(d);
      continue;
    }
    if (q.n_clauses() >= (uint64_t(1) << 32) || q.lits.size() >= (uint64_t(1) << 32))
      fail(SCUBA_E_CAPACITY, "query with 2^32 or more clauses or literals");
    d.n_clauses = uint32_t(q.n_clauses());
    d.n_vars = q.n_vars;
    // staged in 16-bit form: clause offsets, literals, occurrence offsets
    // and occurrence lists
    const size_t bytes =
        ((q.n_clauses() + 1 + q.lits.size() + 2 * (size_t(q.n_vars) + 1) + 1 + q.lits.size()) * 2 + 3) &
        ~size_t(3);
    if (q.n_vars < 32768 && q.lits.size() < 65536 && bytes <= budget) {
      d.staged = 1;
      h.stage_bytes = std::max(h.stage_bytes, bytes);
    }
    h.n_coff += q.off.size();
    h.n_lits += q.lits.size();
    h.n_occ_off += 2 * (size_t(q.n_vars) + 1) + 1;
    h.n_occ += q.lits.size();
    h.q.push_back(d);
  }
  return h;
}
// LDS the propagation kernel may use (the device's opt-in size when the
// kernel attribute could be set)
size_t up_lds_limit(const scuba_ctx* ctx) { return ctx->dev.up_lds_max; }

uint64_t blocks_of(int32_t f) { return f >= 12 ? (uint64_t(1) << (f - 12)) : 1; }

// Append one cube to a round; returns its index within the round.  A cube
// the host refuted is sent too (its device refutation is checked) but gets
// no leaf work.  Work items are made afterwards by make_items.
uint32_t add_cube(RoundHost& rh, uint32_t qid, uint32_t seq, const Cube& c, uint32_t n_vars) {
  if (c.lits.size() > kMaxCubeLen) fail(SCUBA_E_CAPACITY, "cube longer than 4096 literals");
  if (!c.refuted() && (c.f < 0 || uint32_t(c.f) > kMaxLeafVars))
    fail(SCUBA_E_CAPACITY, "leaf with more than 38 active variables");
  DevCubeDesc d;
  d.qid = qid;
  d.lit_off = uint32_t(rh.cube_lits.size());
  d.n_lits = uint32_t(c.lits.size());
  // a leaf whose fixpoint the splitter kept goes as that fixpoint (two
  // bitmaps), so the device confirms it instead of propagating the cube
  // again; 2 * (n_vars/32 + 1) words fit the literal bound of a round
  const bool fix = !c.refuted() && c.assign.size() == size_t(n_vars) + 1 && n_vars >= 2 &&
                   2 * ((n_vars >> 5) + 1) <= kMaxCubeLen;
  if (fix) d.n_lits = kCubeFixpoint | (2 * ((n_vars >> 5) + 1));
  d.seq = seq;
  d.f_expect = c.refuted() ? -1 : c.f;
  d.nres_cap = c.refuted() ? 0 : c.nres;
  d.res_base = rh.res_records;
  rh.res_records += d.nres_cap;
  rh.tile_max = std::max(rh.tile_max, d.nres_cap);
  rh.nw_max = std::max(rh.nw_max, (n_vars >> 5) + 1);
  if (fix) {
    const uint32_t nw = (n_vars >> 5) + 1;
    const size_t base = rh.cube_lits.size();
    rh.cube_lits.resize(base + 2 * size_t(nw), 0);
    uint32_t* words = reinterpret_cast<uint32_t*>(rh.cube_lits.data() + base);
    for (uint32_t v = 1; v <= n_vars; v++)
      if (c.assign[v] >= 0) words[(c.assign[v] ? 0 : nw) + (v >> 5)] |= 1u << (v & 31);
  } else {
    rh.cube_lits.insert(rh.cube_lits.end(), c.lits.begin(), c.lits.end());
  }
  uint32_t ci = uint32_t(rh.cubes.size());
  rh.cubes.push_back(d);
  return ci;
}

// Item sizes in 4096-assignment blocks.  DECIDE: sizes grow geometrically
// from 4 blocks (one per wave) to the cap, so that the first blocks of every
// leaf are reached early (witnesses tend to sit at small indices), and the
// items of all leaves are ordered by their first block.  COUNT: every item
// has the cap size, the cap chosen so that the round has a few items per
// workgroup.
template <typename F>
void for_each_item(uint64_t nb, uint64_t cap, bool geometric, F&& emit) {
  uint64_t lo = 0, size = geometric ? std::min<uint64_t>(4, cap) : cap;
  while (lo < nb) {
    uint64_t hi = std::min(nb, lo + size);
    emit(lo, hi);
    lo = hi;
    if (geometric) size = std::min(size * 2, cap);
  }
}
uint64_t count_items(uint64_t nb, uint64_t cap, bool geometric) {
  uint64_t n = 0;
  for_each_item(nb, cap, geometric, [&](uint64_t, uint64_t) { n++; });
  return n;
}
uint64_t item_cap(const RoundHost& rh, uint32_t mode, uint32_t chunk_log2, uint32_t grid) {
  const uint64_t cap = uint64_t(1) << chunk_log2;
  uint64_t total = 0;
  for (const DevCubeDesc& d : rh.cubes)
    if (d.f_expect >= 0) total += blocks_of(d.f_expect);
  if (mode == SCUBA_MODE_DECIDE) {
    // items past the geometric ramp: at least the configured size, larger
    // when the round holds far more blocks than a few per workgroup (so that
    // skipping the items of decided queries stays cheap)
    const uint64_t want = total / (uint64_t(16) * std::max<uint32_t>(grid, 1));
    uint64_t c = cap;
    while (c * 2 <= want && c < (uint64_t(1) << 16)) c *= 2;
    return c;
  }
  const uint64_t want = total / (uint64_t(4) * std::max<uint32_t>(grid, 1));
  uint64_t c = 4;
  while (c * 2 <= want && c * 2 <= cap) c *= 2;
  return std::min(c, cap);
}
void make_items(RoundHost& rh, uint32_t mode, uint32_t chunk_log2, uint32_t grid) {
  const bool geometric = mode == SCUBA_MODE_DECIDE;
  const uint64_t cap = item_cap(rh, mode, chunk_log2, grid);
  rh.items.clear();
  for (uint32_t ci = 0; ci < rh.cubes.size(); ci++) {
    if (rh.cubes[ci].f_expect < 0) continue;
    for_each_item(blocks_of(rh.cubes[ci].f_expect), cap, geometric, [&](uint64_t lo, uint64_t hi) {
      rh.items.push_back({ci, uint32_t(lo), uint32_t(hi), 0});
    });
  }
  if (geometric)
    std::stable_sort(rh.items.begin(), rh.items.end(),
                     [](const DevItem& a, const DevItem& b) { return a.it_lo < b.it_lo; });
}

size_t round_bound(const scuba_cnf* cnf, size_t n_cubes, const Opts& o, uint32_t max_res) {
  uint32_t max_vars = 0;
  for (const CnfQuery& q : cnf->q) max_vars = std::max(max_vars, q.n_vars);
  size_t lits = n_cubes * std::min<uint32_t>(max_vars + 1, kMaxCubeLen);
  uint64_t per = count_items(blocks_of(int32_t(o.k)), uint64_t(1) << o.chunk_log2, true);
  return dev_round_bytes(n_cubes, lits, n_cubes * per, uint64_t(n_cubes) * max_res);
}

// Model of a SAT leaf: the leaf's fixpoint (kept by the splitter, else the
// propagation of the cube again), slot j = bit j of `a`, remaining
// unassigned variables 0.  Then the checks of the result stage: every clause
// and the exact integer query.
void assemble_witness(const CnfQuery& q, Splitter* sp, const Cube& cube, uint64_t a, scuba_results::Q& out) {
  std::vector<int8_t> assign;
  std::vector<int32_t> active;
  if (!cube.assign.empty()) {   // the leaf's fixpoint, kept by the splitter
    assign = cube.assign;
    active = cube.active;
  } else {
    uint32_t nres = 0;
    if (!sp || !sp->leaf_of(cube.lits, &assign, &active, &nres))
      fail(SCUBA_E_INTERNAL, "witness cube conflicts on the host");
  }
  if (active.size() > 64 || assign.size() != size_t(q.n_vars) + 1)
    fail(SCUBA_E_INTERNAL, "leaf state does not match the query");
  for (size_t j = 0; j < active.size(); j++) assign[active[j]] = int8_t((a >> j) & 1);
  out.model.assign(size_t(q.n_vars) + 1, 0);
  for (uint32_t v = 1; v <= q.n_vars; v++) out.model[v] = assign[v] > 0 ? 1 : 0;
  // every clause must hold
  for (uint64_t c = 0; c < q.n_clauses(); c++) {
    bool sat = false;
    for (uint64_t i = q.off[c]; i < q.off[c + 1] && !sat; i++) {
      int32_t l = q.lits[i];
      sat = (out.model[std::abs(l)] == 1) == (l > 0);
    }
    if (!sat) fail(SCUBA_E_INTERNAL, "device witness violates a clause");
  }
  out.witness.clear();
  for (size_t i = 0; i < q.in_first.size(); i++) {
    uint64_t v = 0;
    for (uint32_t b = 0; b < q.in_width[i]; b++)
      if (out.model[q.in_first[i] + b]) v |= uint64_t(1) << b;
    out.witness.push_back(v);
  }
  if (!int_check_query(q, out.witness)) fail(SCUBA_E_INTERNAL, "witness fails the exact integer query");
  out.r.witness_checked = 1;
}

// The device's propagation must reach the host's fixpoint: the same
// refutation, active count and number of unsatisfied clauses.
void check_out(const DevCubeOut& o, const Cube& host) {
  if (host.refuted()) {
    if (o.status != 1) fail(SCUBA_E_DEVICE, "device kept a cube the host propagation refuted");
    return;
  }
  if (o.status == 2) fail(SCUBA_E_DEVICE, "device propagation disagrees with the host (active count)");
  if (o.status == 3) fail(SCUBA_E_DEVICE, "device residual exceeds the host's count");
  if (o.status == 1) fail(SCUBA_E_DEVICE, "device refuted a leaf the host propagation kept");
  if (o.f != host.f || uint32_t(o.nres) != host.nres)
    fail(SCUBA_E_DEVICE, "device leaf disagrees with the host (active count or residual)");
}

// Batched device scoring for learned orderings: the candidates of every
// waiting walk go through the perceptron in one pass.  Workspace layout:
// x bf16 [cap x 16] | a1 bf16 [cap x 128] | a2 bf16 [cap x 128] | y f32 [cap].
// Candidate rows of one scoring pass over every query: the static
// candidates plus one per input word.
size_t scorer_rows(const scuba_cnf* cnf, uint32_t candidates) {
  size_t rows = 0;
  for (const CnfQuery& q : cnf->q) rows += std::max<uint32_t>(candidates, 1) + q.in_first.size();
  return std::max<size_t>(rows, 1);
}
size_t scorer_bytes(size_t rows) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al(rows * kMlpF * 2) + 2 * al(rows * kMlpH * 2) + al(rows * 4);
}
uint16_t to_bf16(float f) {   // round to nearest, ties to even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return uint16_t((u >> 16) | 0x40);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

struct ScorerRunner {
  scuba_ctx* ctx;
  const scuba_learned_scorer* s;
  char* ws;
  size_t rows_cap;
  void* stream;
  uint64_t rows_scored = 0, passes = 0;
  double device_ms = 0;   // staging, copies, kernel and wait of the passes

  void score(const std::vector<Splitter*>& waiting) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t i = 0;
    while (i < waiting.size()) {
      // as many whole requests as fit
      size_t j = i, rows = 0;
      while (j < waiting.size() && rows + waiting[j]->request_vars().size() <= rows_cap) {
        rows += waiting[j]->request_vars().size();
        j++;
      }
      if (j == i) fail(SCUBA_E_CAPACITY, "scorer workspace smaller than one request");
      void* stg = ctx->score_staging(std::max(rows * kMlpF * 2, rows * 4) + 256);
      uint16_t* xh = static_cast<uint16_t*>(stg);
      // each request's rows at their offset, converted on the host pool
      std::vector<size_t> at(j - i + 1, 0);
      for (size_t q = i; q < j; q++) at[q - i + 1] = at[q - i] + waiting[q]->request_features().size();
      parallel_for(j - i, [&](size_t t) {
        const std::vector<float>& fe = waiting[i + t]->request_features();
        uint16_t* dst = xh + at[t];
        for (size_t e = 0; e < fe.size(); e++) dst[e] = to_bf16(fe[e]);
      });
      uint16_t* x = reinterpret_cast<uint16_t*>(ws);
      uint16_t* a1 = reinterpret_cast<uint16_t*>(ws + al(rows_cap * kMlpF * 2));
      uint16_t* a2 = reinterpret_cast<uint16_t*>(ws + al(rows_cap * kMlpF * 2) + al(rows_cap * kMlpH * 2));
      float* y = reinterpret_cast<float*>(ws + al(rows_cap * kMlpF * 2) + 2 * al(rows_cap * kMlpH * 2));
      auto td = Clock::now();
      dev_copy_h2d(x, xh, rows * kMlpF * 2, stream);
      mlp_forward(s->wbf16, s->master, x, uint32_t(rows), a1, a2, y, stream);
      dev_copy_d2h(stg, y, rows * 4, stream);
      dev_sync(stream);
      device_ms += ms_since(td);
      const float* yh = static_cast<const float*>(stg);
      size_t off = 0;
      for (size_t q = i; q < j; q++) {
        waiting[q]->provide_scores(yh + off);
        off += waiting[q]->request_vars().size();
      }
      rows_scored += rows;
      passes++;
      i = j;
    }
  }
};

// Advance every walk until it has produced max_leaves leaves (or ended),
// scoring on the device whenever walks wait for a learned decision.
void run_walks(std::vector<Splitter*>& walks, uint32_t max_leaves, std::vector<std::vector<Cube>>& out,
               bool keep, std::vector<Splitter::State>& state, ScorerRunner* runner) {
  std::vector<size_t> todo(walks.size());
  for (size_t i = 0; i < todo.size(); i++) todo[i] = i;
  while (!todo.empty()) {
    parallel_for(todo.size(), [&](size_t t) {
      const size_t i = todo[t];
      state[i] = walks[i]->next(max_leaves, out[i], keep);
    });
    std::vector<Splitter*> waiting;
    std::vector<size_t> next;
    for (size_t i : todo)
      if (state[i] == Splitter::kNeedScore) {
        waiting.push_back(walks[i]);
        next.push_back(i);
      }
    if (waiting.empty()) break;
    if (!runner) fail(SCUBA_E_INTERNAL, "learned walk without a scorer");
    runner->score(waiting);
    todo.swap(next);
  }
}

void check_learned(const scuba_learned_scorer* l) {
  scuba_solve_opts so{};
  so.scorer = SCUBA_SCORER_LEARNED;
  so.learned = l;
  resolve(&so);
}

}  // namespace

// ---------------------------------------------------------------- context

extern "C" {

uint32_t scuba_abi_version(void) { return 1; }

scuba_status scuba_ctx_create(int32_t device, scuba_ctx** out) {
  if (!out) return SCUBA_E_INVALID;
  try {
    auto* c = new scuba_ctx();
    c->device = device;
    *out = c;
    return SCUBA_OK;
  } catch (...) {
    return SCUBA_E_NOMEM;
  }
}

void scuba_ctx_destroy(scuba_ctx* ctx) { delete ctx; }

const char* scuba_last_error(const scuba_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

const char* scuba_status_str(scuba_status s) {
  switch (s) {
    case SCUBA_OK: return "ok";
    case SCUBA_E_INVALID: return "invalid input";
    case SCUBA_E_WIDTH: return "input width outside 1..64";
    case SCUBA_E_NOMEM: return "out of host memory";
    case SCUBA_E_DEVICE: return "device error";
    case SCUBA_E_CAPACITY: return "capacity exceeded";
    case SCUBA_E_STATE: return "invalid state";
    case SCUBA_E_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

// ---------------------------------------------------------------- CNF

scuba_status scuba_bitblast(scuba_ctx* ctx, uint32_t nq, const scuba_node* nodes, const uint64_t* node_start,
                            const uint32_t* roots, const uint64_t* root_start, uint32_t flags,
                            scuba_cnf** out) {
  if (!ctx || !out || (nq && (!node_start || !root_start))) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    auto cnf = std::make_unique<scuba_cnf>();
    cnf->q.resize(nq);
    for (uint32_t i = 0; i < nq; i++)
      if (node_start[i + 1] < node_start[i] || root_start[i + 1] < root_start[i])
        fail(SCUBA_E_INVALID, "offsets must not decrease");
    // queries are independent: encode them on the host thread pool
    parallel_for(nq, [&](size_t i) {
      uint64_t n0 = node_start[i], n1 = node_start[i + 1], r0 = root_start[i], r1 = root_start[i + 1];
      try {
        cnf->q[i] = bitblast_query(nodes + n0, n1 - n0, roots + r0, r1 - r0, flags);
      } catch (const Error& e) {
        throw Error(e.code, "query " + std::to_string(i) + ": " + e.what());
      }
    });
    *out = cnf.release();
  });
}

scuba_status scuba_cnf_from_arrays(scuba_ctx* ctx, uint32_t nq, const uint32_t* n_vars,
                                   const uint64_t* q_clause_start, const uint64_t* clause_off,
                                   const int32_t* lits, scuba_cnf** out) {
  if (!ctx || !out || (nq && (!n_vars || !q_clause_start || !clause_off))) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    auto cnf = std::make_unique<scuba_cnf>();
    for (uint32_t i = 0; i < nq; i++) {
      CnfQuery q;
      q.n_vars = n_vars[i];
      uint64_t c0 = q_clause_start[i], c1 = q_clause_start[i + 1];
      if (c1 < c0) fail(SCUBA_E_INVALID, "clause ranges must not decrease");
      std::vector<uint32_t> seen(size_t(q.n_vars) + 1, 0);
      uint32_t stamp = 0;
      for (uint64_t c = c0; c < c1; c++) {
        if (clause_off[c + 1] < clause_off[c]) fail(SCUBA_E_INVALID, "clause offsets must not decrease");
        stamp++;
        for (uint64_t j = clause_off[c]; j < clause_off[c + 1]; j++) {
          int32_t l = lits[j];
          uint32_t v = uint32_t(l > 0 ? l : -int64_t(l));
          if (l == 0 || v > q.n_vars) fail(SCUBA_E_INVALID, "query " + std::to_string(i) + ": literal out of range");
          if (seen[v] == stamp) fail(SCUBA_E_INVALID, "query " + std::to_string(i) + ": clause repeats a variable");
          seen[v] = stamp;
          q.lits.push_back(l);
        }
        q.off.push_back(q.lits.size());
      }
      q.build_occurrences();
      cnf->q.push_back(std::move(q));
    }
    *out = cnf.release();
  });
}

uint32_t scuba_cnf_count(const scuba_cnf* cnf) { return cnf ? uint32_t(cnf->q.size()) : 0; }

scuba_status scuba_cnf_view_get(const scuba_cnf* cnf, uint32_t qi, scuba_cnf_view* out) {
  if (!cnf || !out || qi >= cnf->q.size()) return SCUBA_E_INVALID;
  const CnfQuery& q = cnf->q[qi];
  out->n_vars = q.n_vars;
  out->n_inputs = uint32_t(q.in_first.size());
  out->n_clauses = q.n_clauses();
  out->n_lits = q.lits.size();
  out->clause_off = q.off.data();
  out->lits = q.lits.data();
  out->root_unsat = q.root_unsat ? 1 : 0;
  return SCUBA_OK;
}

scuba_status scuba_cnf_input_map(const scuba_cnf* cnf, uint32_t qi, uint32_t* first_var, uint32_t* width,
                                 uint32_t cap) {
  if (!cnf || qi >= cnf->q.size()) return SCUBA_E_INVALID;
  const CnfQuery& q = cnf->q[qi];
  if (cap < q.in_first.size() || (!q.in_first.empty() && (!first_var || !width))) return SCUBA_E_CAPACITY;
  for (size_t i = 0; i < q.in_first.size(); i++) {
    first_var[i] = q.in_first[i];
    width[i] = q.in_width[i];
  }
  return SCUBA_OK;
}

// The queries' memory is released on the host pool: each query was built on
// a pool thread, so its blocks go back to the allocator arena that the next
// bit-blast reuses.
void scuba_cnf_free(scuba_cnf* cnf) {
  if (!cnf) return;
  try {
    parallel_for(cnf->q.size(), [&](size_t i) { cnf->q[i] = CnfQuery(); });
  } catch (...) {
  }
  delete cnf;
}

// ---------------------------------------------------------------- cubes

size_t scuba_scorer_workspace(const scuba_cnf* cnf, uint32_t candidates) {
  return cnf ? scorer_bytes(scorer_rows(cnf, candidates)) : 0;
}

scuba_status scuba_split(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_split_opts* opts, scuba_cubes** out) {
  if (!ctx || !cnf || !opts || !out) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    if (opts->k > kMaxLeafVars) fail(SCUBA_E_INVALID, "k above the leaf limit of 38 variables");
    if (opts->scorer > SCUBA_SCORER_WORD) fail(SCUBA_E_INVALID, "unknown scorer");
    const bool learned = opts->scorer == SCUBA_SCORER_LEARNED;
    uint32_t max_res = opts->max_residual ? opts->max_residual : kDefaultMaxResidual;
    uint64_t max_cubes = opts->max_cubes ? opts->max_cubes : kDefaultMaxCubes;
    if (max_cubes > kMaxCubesPerQuery) fail(SCUBA_E_INVALID, "max_cubes above 2^26 per query");
    const size_t nq = cnf->q.size();
    std::unique_ptr<ScorerRunner> runner;
    if (learned) {
      check_learned(opts->learned);
      const size_t rows = scorer_rows(cnf, opts->learned->candidates);
      if (!opts->dev_ws || opts->ws_bytes < scorer_bytes(rows))
        fail(SCUBA_E_CAPACITY, "scorer workspace smaller than scuba_scorer_workspace");
      ctx->ensure_device();
      runner.reset(new ScorerRunner{ctx, opts->learned, static_cast<char*>(opts->dev_ws),
                                    rows, opts->hip_stream});
    }
    std::vector<std::unique_ptr<Splitter>> sp(nq);
    std::vector<Splitter*> walks(nq);
    parallel_for(nq, [&](size_t qi) {
      sp[qi] = std::make_unique<Splitter>(cnf->q[qi], opts->k, max_res, max_cubes);
      if (learned) sp[qi]->set_learned(opts->learned->candidates, opts->learned->rescore);
      if (opts->scorer == SCUBA_SCORER_WORD) sp[qi]->set_word_order();
      walks[qi] = sp[qi].get();
    });
    std::vector<std::vector<Cube>> all(nq);
    std::vector<Splitter::State> state(nq, Splitter::kRunning);
    run_walks(walks, UINT32_MAX, all, true, state, runner.get());
    auto cubes = std::make_unique<scuba_cubes>();
    cubes->q.resize(nq);
    parallel_for(nq, [&](size_t qi) {
      scuba_cubes::Q& cq = cubes->q[qi];
      cq.complete = state[qi] == Splitter::kExhausted;
      for (const Cube& c : all[qi]) {
        cq.lits.insert(cq.lits.end(), c.lits.begin(), c.lits.end());
        cq.off.push_back(cq.lits.size());
        cq.kind.push_back(c.kind == CubeKind::kLeaf ? SCUBA_CUBE_LEAF
                          : c.kind == CubeKind::kRefuted ? SCUBA_CUBE_REFUTED : SCUBA_CUBE_PRUNED);
        cq.f.push_back(c.refuted() ? -1 : c.f);
        cq.nres.push_back(c.nres);
      }
    });
    *out = cubes.release();
  });
}

struct scuba_trace {
  std::vector<float> feats, labels;
  std::vector<uint64_t> nodes;
};

scuba_status scuba_trace_run(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_trace_opts* opts,
                             scuba_trace** out) {
  if (!ctx || !cnf || !opts || !out) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    if (opts->k > kMaxLeafVars) fail(SCUBA_E_INVALID, "k above the leaf limit of 38 variables");
    if (opts->candidates < 1 || opts->candidates > 64) fail(SCUBA_E_INVALID, "trace candidates outside 1..64");
    const size_t nq = cnf->q.size();
    const uint64_t max_cubes = opts->max_cubes ? opts->max_cubes : kDefaultMaxCubes;
    std::vector<std::unique_ptr<Splitter>> sp(nq);
    parallel_for(nq, [&](size_t qi) {
      if (cnf->q[qi].root_unsat) return;
      sp[qi] = std::make_unique<Splitter>(cnf->q[qi], opts->k, kDefaultMaxResidual, max_cubes);
      sp[qi]->set_trace(opts->candidates, opts->every, opts->depth);
      std::vector<Cube> sink;
      while (sp[qi]->next(4096, sink, false) == Splitter::kRunning) sink.clear();
    });
    auto t = std::make_unique<scuba_trace>();
    for (size_t qi = 0; qi < nq; qi++) {
      if (!sp[qi]) continue;
      const auto& f = sp[qi]->trace_features();
      const auto& l = sp[qi]->trace_labels();
      const auto& n = sp[qi]->trace_nodes();
      t->feats.insert(t->feats.end(), f.begin(), f.end());
      t->labels.insert(t->labels.end(), l.begin(), l.end());
      for (uint32_t d : n) t->nodes.push_back(uint64_t(qi) << 32 | d);
      sp[qi].reset();
    }
    *out = t.release();
  });
}

scuba_status scuba_trace_view(const scuba_trace* t, uint64_t* rows, const float** features,
                              const float** labels, const uint64_t** nodes) {
  if (!t || !rows || !features || !labels || !nodes) return SCUBA_E_INVALID;
  *rows = t->labels.size();
  *features = t->feats.data();
  *labels = t->labels.data();
  *nodes = t->nodes.data();
  return SCUBA_OK;
}

void scuba_trace_free(scuba_trace* t) { delete t; }


scuba_status scuba_cubes_from_arrays(scuba_ctx* ctx, const scuba_cnf* cnf, const uint64_t* q_cube_start,
                                     const uint64_t* cube_off, const int32_t* cube_lits, scuba_cubes** out) {
  if (!ctx || !cnf || !q_cube_start || !cube_off || !out) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    for (size_t i = 0; i < cnf->q.size(); i++) {
      if (q_cube_start[i + 1] < q_cube_start[i]) fail(SCUBA_E_INVALID, "cube ranges must not decrease");
      for (uint64_t c = q_cube_start[i]; c < q_cube_start[i + 1]; c++) {
        if (cube_off[c + 1] < cube_off[c]) fail(SCUBA_E_INVALID, "cube offsets must not decrease");
        for (uint64_t j = cube_off[c]; j < cube_off[c + 1]; j++) {
          int32_t l = cube_lits[j];
          if (l == 0 || uint32_t(l > 0 ? l : -int64_t(l)) > cnf->q[i].n_vars)
            fail(SCUBA_E_INVALID, "cube literal out of range");
        }
      }
    }
    auto cubes = std::make_unique<scuba_cubes>();
    cubes->q.resize(cnf->q.size());
    parallel_for(cnf->q.size(), [&](size_t i) {
      const CnfQuery& q = cnf->q[i];
      scuba_cubes::Q& cq = cubes->q[i];
      Splitter sp(q, 0, 0, 1);
      for (uint64_t c = q_cube_start[i]; c < q_cube_start[i + 1]; c++) {
        std::vector<int32_t> lits(cube_lits + cube_off[c], cube_lits + cube_off[c + 1]);
        std::vector<int8_t> assign;
        std::vector<int32_t> active;
        uint32_t nres = 0;
        bool ok = sp.leaf_of(lits, &assign, &active, &nres);
        cq.lits.insert(cq.lits.end(), lits.begin(), lits.end());
        cq.off.push_back(cq.lits.size());
        // every given cube goes to the device; host-conflicting ones are
        // marked so that the device's refutation can be checked
        cq.kind.push_back(ok ? SCUBA_CUBE_LEAF : SCUBA_CUBE_REFUTED);
        cq.f.push_back(ok ? int32_t(active.size()) : -1);
        cq.nres.push_back(ok ? nres : 0);
      }
      cq.complete = false;
    });
    *out = cubes.release();
  });
}

scuba_status scuba_cubes_view_get(const scuba_cubes* cubes, uint32_t qi, scuba_cubes_view* out) {
  if (!cubes || !out || qi >= cubes->q.size()) return SCUBA_E_INVALID;
  const auto& q = cubes->q[qi];
  out->n_cubes = q.kind.size();
  out->cube_off = q.off.data();
  out->lits = q.lits.data();
  out->kind = q.kind.data();
  out->f = q.f.data();
  out->complete = q.complete ? 1 : 0;
  return SCUBA_OK;
}

void scuba_cubes_free(scuba_cubes* cubes) { delete cubes; }

// ---------------------------------------------------------------- solve

// Round of a given cube list (every cube of every query, in order).
struct SolveRound {
  RoundHost rh;
  std::vector<std::pair<uint32_t, uint64_t>> where;   // round cube -> (query, cube)
  std::vector<Cube> host;
};
SolveRound solve_round(const scuba_cnf* cnf, const scuba_cubes* cubes, const Opts& o, uint32_t grid) {
  SolveRound sr;
  for (size_t qi = 0; qi < cnf->q.size(); qi++) {
    const auto& cq = cubes->q[qi];
    for (size_t c = 0; c < cq.kind.size(); c++) {
      Cube cube;
      cube.lits.assign(cq.lits.begin() + cq.off[c], cq.lits.begin() + cq.off[c + 1]);
      // pruned cubes are refuted through their sibling's subtree, not by
      // propagation alone: they are not sent
      if (cq.kind[c] == SCUBA_CUBE_PRUNED) continue;
      cube.kind = cq.kind[c] == SCUBA_CUBE_LEAF ? CubeKind::kLeaf : CubeKind::kRefuted;
      cube.f = cq.f[c];
      cube.nres = cq.nres[c];
      add_cube(sr.rh, uint32_t(qi), uint32_t(c), cube, cnf->q[qi].n_vars);
      sr.where.push_back({uint32_t(qi), c});
      sr.host.push_back(std::move(cube));
    }
  }
  make_items(sr.rh, o.mode, o.chunk_log2, grid);
  sr.rh.leaf_variant = leaf_variant(o);
  return sr;
}

uint32_t grid_of(const scuba_ctx* ctx, const Opts& o) { return o.grid ? o.grid : uint32_t(ctx->dev.cus) * 8; }

scuba_status scuba_solve_workspace(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_cubes* cubes,
                                   const scuba_solve_opts* opts, size_t* bytes) {
  if (!ctx || !cnf || !cubes || !bytes || cubes->q.size() != cnf->q.size()) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    Opts o = resolve(opts);
    ctx->ensure_device();
    CnfHost h = cnf_host(cnf);
    SolveRound sr = solve_round(cnf, cubes, o, grid_of(ctx, o));
    *bytes = dev_cnf_bytes(h) +
             dev_round_bytes(sr.rh.cubes.size(), sr.rh.cube_lits.size(), sr.rh.items.size(), sr.rh.res_records);
  });
}

// ---------------------------------------------------------------- device split

namespace {

// Run parameters of the device split for a batch: bitmap width and residual
// bound from the open queries, nodes per step, and the default stack.
SplitRun split_run(const scuba_cnf* cnf, const Opts& o, size_t* n_order) {
  SplitRun r;
  r.k = o.k;
  r.max_res = o.max_res;
  r.mode = o.mode;
  r.chunk_log2 = o.chunk_log2;
  r.grid = o.grid;
  r.max_cubes = o.max_cubes;
  r.leaf_variant = leaf_variant(o);
  uint32_t nw = 1;
  uint64_t nc = 1;
  *n_order = 0;
  for (const CnfQuery& q : cnf->q) {
    if (q.root_unsat) continue;
    nw = std::max(nw, (q.n_vars >> 5) + 1);
    nc = std::max<uint64_t>(nc, q.n_clauses());
    *n_order += q.n_vars;
  }
  r.nw_max = nw;
  r.nres_max = uint32_t(std::min<uint64_t>(o.max_res, nc));
  // a batch with a wide query (kSplitWideClauses clauses or more) expands
  // one node per open query per step, so that every query's walk goes
  // depth-first; else up to 16384 nodes, fewer when leaves are large
  size_t n_open = 0;
  bool wide = false;
  for (const CnfQuery& q : cnf->q)
    if (!q.root_unsat) {
      n_open++;
      wide |= q.n_clauses() >= kSplitWideClauses;
    }
  uint64_t b = o.split_batch ? o.split_batch : 16384;
  if (!o.split_batch) {
    b = std::min<uint64_t>(b, std::max<uint64_t>(256, (uint64_t(512) << 20) / (32 * r.nres_max)));
    if (wide) b = std::min<uint64_t>(std::max<uint64_t>(64, n_open), uint64_t(1) << 20);
  }
  r.batch = uint32_t(b);
  // room for 64 breadth-limited steps (256 depth-first levels of every
  // query when wide), then depth-first steps within the reserve
  uint32_t nv_max = 0;
  for (const CnfQuery& q : cnf->q)
    if (!q.root_unsat) nv_max = std::max(nv_max, q.n_vars);
  r.stack_cap = (wide ? 256 : 64) * size_t(b) + size_t(nv_max) + 2 + cnf->q.size();
  return r;
}

size_t split_need(const scuba_cnf* cnf, const Opts& o) {
  CnfHost h = cnf_host(cnf, 0, true);
  size_t n_order;
  SplitRun r = split_run(cnf, o, &n_order);
  return dev_split_bytes(h, n_order, r);
}

// scuba_decide with the split on the device: branch orders on the host pool,
// then the device loop, then the witnesses of the SAT queries built from
// their leaves' fixpoints and checked like every witness.
std::unique_ptr<scuba_results> decide_split_impl(scuba_ctx* ctx, const scuba_cnf* cnf, const Opts& o, void* dev_ws,
                                                 size_t ws_bytes, void* hip_stream) {
  auto t0 = Clock::now();
  ctx->ensure_device();
  const size_t nq = cnf->q.size();
  CnfHost h = cnf_host(cnf, 0, true);
  auto res = std::make_unique<scuba_results>();
  res->q.resize(nq);
  std::vector<uint32_t> start;
  for (size_t qi = 0; qi < nq; qi++) {
    if (cnf->q[qi].root_unsat) {
      res->q[qi].r.verdict = SCUBA_UNSAT;
      res->q[qi].r.how = SCUBA_HOW_ROOT;
    } else {
      start.push_back(uint32_t(qi));
    }
  }
  auto ts = Clock::now();
  std::vector<std::vector<int32_t>> ords(nq);
  parallel_for(start.size(), [&](size_t j) {
    const uint32_t qi = start[j];
    Splitter sp(cnf->q[qi], o.k, o.max_res, o.max_cubes);
    if (o.scorer == SCUBA_SCORER_WORD) sp.set_word_order();
    ords[qi] = sp.branch_order();
  });
  std::vector<uint64_t> order_off(nq, 0);
  size_t n_order = 0;
  for (uint32_t qi : start) {
    order_off[qi] = n_order;
    n_order += cnf->q[qi].n_vars;
    if (ords[qi].size() != cnf->q[qi].n_vars) fail(SCUBA_E_INTERNAL, "branch order misses variables");
  }
  std::vector<uint32_t> order(n_order);
  for (uint32_t qi : start)
    for (size_t i = 0; i < ords[qi].size(); i++) order[order_off[qi] + i] = uint32_t(ords[qi][i]);
  ords.clear();
  const double order_ms = ms_since(ts);
  size_t n_ord;
  SplitRun r = split_run(cnf, o, &n_ord);
  // the stack takes what the workspace holds beyond the fixed regions
  {
    SplitRun r0 = r;
    r0.stack_cap = 0;
    const size_t fixed = dev_split_bytes(h, n_order, r0) + 1024;
    const size_t per = dev_split_node_bytes(r.nw_max);
    if (ws_bytes < fixed + per * 2 * size_t(r.batch))
      fail(SCUBA_E_CAPACITY, "workspace smaller than scuba_decide_workspace");
    // (dev_split checks the stack against the start nodes and the reserve)
    r.stack_cap = std::min<size_t>((ws_bytes - fixed) / per, size_t(1) << 31);
    while (r.stack_cap && dev_split_bytes(h, n_order, r) > ws_bytes) r.stack_cap -= 256;
    if (r.stack_cap < 2 * size_t(r.batch)) fail(SCUBA_E_CAPACITY, "workspace smaller than scuba_decide_workspace");
  }
  SplitOutput so;
  double verify_ms = 0;
  if (!start.empty()) {
    const size_t cnf_b = dev_cnf_bytes(h);
    void* cstg = ctx->cnf_staging(cnf_b);
    dev_upload_cnf(ctx->dev, dev_ws, ws_bytes, h, hip_stream, cstg, ctx->cnf_staging_size(), false);
    void* stg = ctx->staging(dev_split_staging(h, n_order, start.size(), r));
    dev_split(ctx->dev, dev_ws, ws_bytes, h, order_off, order, start, r, hip_stream, stg, ctx->staging_size(), &so);
    auto tv = Clock::now();
    const size_t fw = 2 * size_t(r.nw_max);
    parallel_for(start.size(), [&](size_t j) {
      const uint32_t qi = start[j];
      const CnfQuery& q = cnf->q[qi];
      auto& rq = res->q[qi];
      const DevSplitStat& st = so.stats[qi];
      rq.r.cubes_total = st.cubes;
      rq.r.cubes_refuted = st.refuted;
      rq.r.leaves_sent = st.leaves;
      rq.r.blocks_evaluated = st.blocks;
      rq.r.clause_blocks = st.clause_blocks;
      rq.r.word_ops = st.word_ops;
      rq.r.rounds = uint32_t(std::min<uint64_t>(so.steps, UINT32_MAX));
      rq.r.how = SCUBA_HOW_DEVICE;
      const bool undecided = st.budget || so.stopped;
      if (o.mode == SCUBA_MODE_COUNT) {
        bool any = false;
        for (const DevCubeOut& lo : so.leaves[qi]) {
          scuba_leaf_result lr{};
          lr.refuted = lo.status != 0;
          lr.f = lo.f;
          lr.m = lo.m;
          lr.count = lo.count;
          lr.first = lo.first == ~0ull ? -1 : int64_t(lo.first);
          any |= lo.count != 0;
          rq.leaves.push_back(lr);
        }
        rq.r.verdict = any ? SCUBA_SAT : (undecided ? SCUBA_UNKNOWN : SCUBA_UNSAT);
        if (!any && undecided) rq.r.how = SCUBA_HOW_BUDGET;
        return;
      }
      if (so.qkeys[qi] == ~0ull) {
        rq.r.verdict = undecided ? SCUBA_UNKNOWN : SCUBA_UNSAT;
        if (undecided) rq.r.how = SCUBA_HOW_BUDGET;
        return;
      }
      // the witness leaf's fixpoint: assigned variables, then its active
      // variables (unassigned, in an unsatisfied clause) in increasing
      // order as slots 0.., as the device numbered them
      const uint32_t* T = so.wit.data() + qi * fw;
      const uint32_t* F = T + r.nw_max;
      Cube cube;
      cube.assign.assign(size_t(q.n_vars) + 1, -1);
      for (uint32_t v = 1; v <= q.n_vars; v++) {
        const bool t = (T[v >> 5] >> (v & 31)) & 1u, f = (F[v >> 5] >> (v & 31)) & 1u;
        if (t && f) fail(SCUBA_E_DEVICE, "device split witness leaf assigns a variable both ways");
        if (t || f) cube.assign[v] = t ? 1 : 0;
      }
      std::vector<uint8_t> act(size_t(q.n_vars) + 1, 0);
      for (uint64_t c = 0; c < q.n_clauses(); c++) {
        bool sat = false;
        for (uint64_t i = q.off[c]; i < q.off[c + 1] && !sat; i++) {
          const int32_t l = q.lits[i];
          sat = cube.assign[std::abs(l)] == (l > 0 ? 1 : 0);
        }
        if (sat) continue;
        for (uint64_t i = q.off[c]; i < q.off[c + 1]; i++)
          if (cube.assign[std::abs(q.lits[i])] < 0) act[std::abs(q.lits[i])] = 1;
      }
      for (uint32_t v = 1; v <= q.n_vars; v++)
        if (act[v]) cube.active.push_back(int32_t(v));
      const uint64_t a = so.qkeys[qi] & ((uint64_t(1) << 38) - 1);
      if (cube.active.size() > kMaxLeafVars || (cube.active.size() < 38 && (a >> cube.active.size())))
        fail(SCUBA_E_DEVICE, "device split witness index outside its leaf");
      rq.r.verdict = SCUBA_SAT;
      assemble_witness(q, nullptr, cube, a, rq);
    });
    verify_ms = ms_since(tv);
  }
  res->ms[0] = order_ms;
  res->ms[2] = so.expand_ms + so.leaf_ms;
  res->ms[4] = verify_ms;
  res->ms[5] = ms_since(t0);
  res->ms[6] = so.expand_ms;
  res->ms[7] = so.leaf_ms;
  res->ms[8] = double(so.steps);
  res->ms[9] = double(so.steps);
  res->ms[16] = double(so.nodes);
  res->ms[17] = double(so.max_stack);
  return res;
}

}  // namespace

scuba_status scuba_decide_workspace(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_solve_opts* opts,
                                    size_t* bytes) {
  if (!ctx || !cnf || !bytes) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    Opts o = resolve(opts);
    if (o.flags & SCUBA_SOLVE_DEVICE_SPLIT) {
      *bytes = split_need(cnf, o);
      return;
    }
    CnfHost h = cnf_host(cnf, 0, true);
    *bytes = dev_cnf_bytes(h) + round_bound(cnf, size_t(cnf->q.size()) * o.lpr, o, o.max_res);
    if (o.scorer == SCUBA_SCORER_LEARNED)
      *bytes += scorer_bytes(scorer_rows(cnf, o.learned->candidates)) + 256;
  });
}

scuba_status scuba_solve(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_cubes* cubes,
                         const scuba_solve_opts* opts, void* dev_ws, size_t ws_bytes, void* hip_stream,
                         scuba_results** out) {
  if (!ctx || !cnf || !cubes || !out || !dev_ws || cubes->q.size() != cnf->q.size()) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    auto t0 = Clock::now();
    Opts o = resolve(opts);
    if (o.flags & SCUBA_SOLVE_DEVICE_SPLIT) fail(SCUBA_E_INVALID, "scuba_solve takes given cubes: no device split");
    ctx->ensure_device();
    CnfHost h = cnf_host(cnf, up_lds_limit(ctx));
    auto res = std::make_unique<scuba_results>();
    res->q.resize(cnf->q.size());
    for (size_t qi = 0; qi < cnf->q.size(); qi++) {
      auto& rq = res->q[qi];
      const auto& cq = cubes->q[qi];
      rq.leaves.assign(cq.kind.size(), scuba_leaf_result{});
      for (size_t c = 0; c < cq.kind.size(); c++) {
        rq.leaves[c].first = -1;
        rq.leaves[c].refuted = cq.kind[c] == SCUBA_CUBE_PRUNED;
        if (rq.leaves[c].refuted) rq.leaves[c].f = rq.leaves[c].m = -1;
      }
      rq.r.cubes_total = cq.kind.size();
      for (int32_t k : cq.kind) rq.r.cubes_refuted += k != SCUBA_CUBE_LEAF;
    }
    SolveRound sr = solve_round(cnf, cubes, o, grid_of(ctx, o));
    const RoundHost& rh = sr.rh;
    size_t cnf_b = dev_cnf_bytes(h);
    size_t round_b = dev_round_bytes(rh.cubes.size(), rh.cube_lits.size(), rh.items.size(), rh.res_records);
    if (cnf_b + round_b > ws_bytes) fail(SCUBA_E_CAPACITY, "workspace smaller than scuba_solve_workspace");
    void* stg = ctx->staging(std::max(cnf_b, round_b) + 4096 + rh.cubes.size() * sizeof(DevCubeOut) + h.q.size() * 8);
    RoundTimes rt;
    dev_upload_cnf(ctx->dev, dev_ws, ws_bytes, h, hip_stream, stg, ctx->staging_size(), true);
    std::vector<DevCubeOut> outs;
    std::vector<uint64_t> qkeys;
    dev_round(ctx->dev, dev_ws, ws_bytes, h, rh, o.mode, o.grid, hip_stream, stg, ctx->staging_size(), &outs,
              &qkeys, &rt, (o.flags & SCUBA_SOLVE_GRAPH) ? ctx->graph_cache() : nullptr);
    auto tv = Clock::now();
    for (size_t i = 0; i < outs.size(); i++) {
      check_out(outs[i], sr.host[i]);
      auto [qi, c] = sr.where[i];
      auto& rq = res->q[qi];
      scuba_leaf_result& lr = rq.leaves[c];
      lr.refuted = outs[i].status == 1;
      lr.f = lr.refuted ? -1 : outs[i].f;
      lr.m = lr.refuted ? -1 : outs[i].m;
      lr.count = outs[i].count;
      lr.first = outs[i].first == ~0ull ? -1 : int64_t(outs[i].first);
      if (sr.host[i].refuted()) continue;
      rq.r.leaves_sent++;
      rq.r.leaves_refuted += lr.refuted;
      rq.r.blocks_evaluated += outs[i].blocks;
      rq.r.clause_blocks += outs[i].clause_blocks;
      rq.r.word_ops += outs[i].word_ops;
    }
    parallel_for(cnf->q.size(), [&](size_t qi) {
      auto& rq = res->q[qi];
      rq.r.rounds = 1;
      rq.r.how = SCUBA_HOW_DEVICE;
      // first satisfying leaf in cube order
      int64_t sat_cube = -1;
      for (size_t c = 0; c < rq.leaves.size(); c++)
        if (rq.leaves[c].first >= 0) { sat_cube = int64_t(c); break; }
      if (sat_cube >= 0) {
        rq.r.verdict = SCUBA_SAT;
        const auto& cq = cubes->q[qi];
        std::vector<int32_t> lits(cq.lits.begin() + cq.off[sat_cube], cq.lits.begin() + cq.off[sat_cube + 1]);
        Splitter sp(cnf->q[qi], 0, 0, 1);
        Cube cb;
        cb.lits = std::move(lits);
        assemble_witness(cnf->q[qi], &sp, cb, uint64_t(rq.leaves[sat_cube].first), rq);
      } else {
        rq.r.verdict = cubes->q[qi].complete ? SCUBA_UNSAT : SCUBA_UNKNOWN;
        if (cnf->q[qi].root_unsat) { rq.r.verdict = SCUBA_UNSAT; rq.r.how = SCUBA_HOW_ROOT; }
      }
    });
    res->ms[1] = rt.h2d_ms;
    res->ms[2] = rt.up_ms + rt.leaf_ms + rt.graph_ms;
    res->ms[3] = rt.d2h_ms;
    res->ms[4] = ms_since(tv);
    res->ms[5] = ms_since(t0);
    res->ms[6] = rt.up_ms;
    res->ms[7] = rt.leaf_ms;
    res->ms[8] = rt.up_launches;
    res->ms[9] = rt.leaf_launches;
    res->ms[10] = rt.graph_ms;
    res->ms[11] = rt.graph_launches;
    res->ms[12] = rt.graph_captures;
    res->ms[16] = double(rt.cubes);
    res->ms[17] = double(rt.items);
    res->ms[18] = rt.fix_launches;
    *out = res.release();
  });
}

// The lazy split / device round loop of scuba_decide (options resolved).
std::unique_ptr<scuba_results> decide_impl(scuba_ctx* ctx, const scuba_cnf* cnf, const Opts& o, void* dev_ws,
                                           size_t ws_bytes, void* hip_stream) {
  {
    auto t0 = Clock::now();
    if (o.mode != SCUBA_MODE_DECIDE) fail(SCUBA_E_INVALID, "scuba_decide runs in DECIDE mode");
    ctx->ensure_device();
    const size_t nq = cnf->q.size();
    CnfHost h = cnf_host(cnf, up_lds_limit(ctx), true);
    auto res = std::make_unique<scuba_results>();
    res->q.resize(nq);
    std::vector<std::unique_ptr<Splitter>> sp(nq);
    std::vector<char> open(nq, 0);
    std::vector<uint32_t> seq(nq, 0);
    double split_ms = 0, verify_ms = 0;
    auto ts = Clock::now();
    for (size_t qi = 0; qi < nq; qi++) {
      auto& r = res->q[qi].r;
      if (cnf->q[qi].root_unsat) {
        r.verdict = SCUBA_UNSAT;
        r.how = SCUBA_HOW_ROOT;
        continue;
      }
      open[qi] = 1;
    }
    const bool learned = o.scorer == SCUBA_SCORER_LEARNED;
    parallel_for(nq, [&](size_t qi) {
      if (!open[qi]) return;
      sp[qi] = std::make_unique<Splitter>(cnf->q[qi], o.k, o.max_res, o.max_cubes);
      sp[qi]->set_keep_leaf_state();   // witnesses are built from the leaf's fixpoint
      if (learned) sp[qi]->set_learned(o.learned->candidates, o.learned->rescore);
      if (o.scorer == SCUBA_SCORER_WORD) sp[qi]->set_word_order();
    });
    split_ms += ms_since(ts);
    size_t cnf_b = dev_cnf_bytes(h);
    // the scorer's buffers sit at the end of the workspace
    std::unique_ptr<ScorerRunner> runner;
    if (learned) {
      const size_t rows = scorer_rows(cnf, o.learned->candidates);
      const size_t sb = scorer_bytes(rows);
      if (sb + 256 + cnf_b > ws_bytes) fail(SCUBA_E_CAPACITY, "workspace too small for the scorer");
      uintptr_t base = (reinterpret_cast<uintptr_t>(dev_ws) + ws_bytes - sb) & ~uintptr_t(255);
      ws_bytes = base - reinterpret_cast<uintptr_t>(dev_ws);
      // the passes run on the library's scoring stream, ordered after the
      // caller's stream as it stands now: they do not queue behind the CNF
      // upload enqueued next, which the walks overlap
      runner.reset(new ScorerRunner{ctx, o.learned, reinterpret_cast<char*>(base), rows,
                                    dev_score_stream(ctx->dev.device, hip_stream)});
    }
    if (cnf_b > ws_bytes) fail(SCUBA_E_CAPACITY, "workspace too small for the CNF batch");
    // the CNF upload does not depend on the split: it runs while the walks do.
    // Every leaf goes to the device as its host fixpoint when the fixpoint
    // fits a cube and the query fits the host-fixpoint kernel; then only
    // that kernel runs and the occurrence lists stay on the host.
    bool uploaded = false;
    h.no_occ = true;
    for (size_t qi = 0; qi < nq; qi++)
      if (open[qi]) {
        const CnfQuery& q = cnf->q[qi];
        if (q.n_vars < 2 || 2 * ((q.n_vars >> 5) + 1) > kMaxCubeLen || q.lits.size() >= (size_t(1) << 30) ||
            q.n_clauses() >= (uint64_t(1) << 30))
          h.no_occ = false;
      }
    if (std::find(open.begin(), open.end(), 1) != open.end()) {
      void* cstg = ctx->cnf_staging(cnf_b);
      dev_upload_cnf(ctx->dev, dev_ws, ws_bytes, h, hip_stream, cstg, ctx->cnf_staging_size(), false, !h.no_occ);
      uploaded = true;
    }
    RoundTimes rt;
    const uint32_t grid = grid_of(ctx, o);
    // One round's leaves as the walks produced them, with each walk's
    // counters at that point.
    struct Batch {
      std::vector<std::vector<Cube>> leaves;
      std::vector<Splitter::State> state;
      std::vector<uint64_t> cubes_total, cubes_refuted;
    };
    // every open query's walk advances on the host pool
    auto split_round = [&](Batch& b) {
      ts = Clock::now();
      b.leaves.assign(nq, {});
      b.state.assign(nq, Splitter::kRunning);
      b.cubes_total.assign(nq, 0);
      b.cubes_refuted.assign(nq, 0);
      std::vector<Splitter*> walks;
      std::vector<size_t> wq;
      for (size_t qi = 0; qi < nq; qi++)
        if (open[qi]) {
          walks.push_back(sp[qi].get());
          wq.push_back(qi);
        }
      std::vector<std::vector<Cube>> wl(walks.size());
      std::vector<Splitter::State> ws(walks.size(), Splitter::kRunning);
      run_walks(walks, o.lpr, wl, false, ws, runner.get());
      for (size_t i = 0; i < wq.size(); i++) {
        b.leaves[wq[i]].swap(wl[i]);
        b.state[wq[i]] = ws[i];
        b.cubes_total[wq[i]] = sp[wq[i]]->cubes_total();
        b.cubes_refuted[wq[i]] = sp[wq[i]]->cubes_refuted();
      }
      split_ms += ms_since(ts);
    };
    // Rounds overlap with the host when the device bounds them: while the
    // device evaluates round r, the walks of the queries still open produce
    // round r + 1's leaves, and a query that round r decides drops them.
    // Speculation costs the walks of queries the round decides (a walk whose
    // leaf decides its query never finishes the branch otherwise), so it
    // runs only after a round whose kernels took longer than its split.
    DevRoundPending pend;
    Batch next;
    split_round(next);
    double last_split_ms = split_ms, last_dev_ms = 0;
    for (uint32_t round = 0; o.max_rounds == 0 || round < o.max_rounds; round++) {
      ts = Clock::now();
      RoundHost rh;
      std::vector<std::pair<uint32_t, Cube>> sent;
      for (size_t qi = 0; qi < nq; qi++) {
        if (!open[qi]) continue;
        auto& r = res->q[qi].r;
        r.rounds++;
        for (Cube& c : next.leaves[qi]) {
          add_cube(rh, uint32_t(qi), seq[qi]++, c, cnf->q[qi].n_vars);
          sent.push_back({uint32_t(qi), std::move(c)});
        }
        r.cubes_total = next.cubes_total[qi];
        r.cubes_refuted = next.cubes_refuted[qi];
        if (next.leaves[qi].empty()) {
          // nothing left for the device: the tree is done or cut
          open[qi] = 0;
          const Splitter::State st = next.state[qi];
          r.verdict = st == Splitter::kExhausted ? SCUBA_UNSAT : SCUBA_UNKNOWN;
          r.how = st == Splitter::kExhausted ? (r.leaves_sent ? SCUBA_HOW_DEVICE : SCUBA_HOW_ROOT)
                                             : SCUBA_HOW_BUDGET;
        }
      }
      make_items(rh, SCUBA_MODE_DECIDE, o.chunk_log2, grid);
      rh.leaf_variant = leaf_variant(o);
      split_ms += ms_since(ts);
      if (rh.cubes.empty()) break;
      size_t round_b = dev_round_bytes(rh.cubes.size(), rh.cube_lits.size(), rh.items.size(), rh.res_records);
      if (cnf_b + round_b > ws_bytes) fail(SCUBA_E_CAPACITY, "workspace smaller than this round needs");
      void* stg = ctx->staging(std::max(cnf_b, round_b) + 4096 + rh.cubes.size() * sizeof(DevCubeOut) + nq * 8);
      dev_round_begin(ctx->dev, dev_ws, ws_bytes, h, rh, SCUBA_MODE_DECIDE, o.grid, hip_stream, stg,
                      ctx->staging_size(), &rt, (o.flags & SCUBA_SOLVE_GRAPH) ? ctx->graph_cache() : nullptr,
                      &pend);
      // the next round's leaves while this one runs, when rounds are
      // bound by the device
      Batch after;
      const bool more = o.max_rounds == 0 || round + 1 < o.max_rounds;
      const bool speculate = more && last_dev_ms > last_split_ms;
      const double split_before = split_ms;
      if (speculate) split_round(after);
      std::vector<DevCubeOut> outs;
      std::vector<uint64_t> qkeys;
      const double dev_before = rt.up_ms + rt.leaf_ms + rt.graph_ms;
      dev_round_end(&pend, &outs, &qkeys, &rt);
      last_dev_ms = rt.up_ms + rt.leaf_ms + rt.graph_ms - dev_before;
      auto tv = Clock::now();
      for (size_t i = 0; i < outs.size(); i++) {
        check_out(outs[i], sent[i].second);
        auto& r = res->q[sent[i].first].r;
        r.leaves_sent++;
        r.leaves_refuted += outs[i].status == 1;
        r.blocks_evaluated += outs[i].blocks;
        r.clause_blocks += outs[i].clause_blocks;
        r.word_ops += outs[i].word_ops;
      }
      // queries with a witness are SAT; the witness is from this round
      std::vector<size_t> first_of(nq, SIZE_MAX);
      for (size_t i = 0; i < sent.size(); i++)
        if (first_of[sent[i].first] == SIZE_MAX) first_of[sent[i].first] = i;
      std::vector<uint32_t> sat_q;
      for (size_t qi = 0; qi < nq; qi++)
        if (qkeys[qi] != ~0ull && res->q[qi].r.verdict != SCUBA_SAT && first_of[qi] != SIZE_MAX)
          sat_q.push_back(uint32_t(qi));
      parallel_for(sat_q.size(), [&](size_t j) {
        const uint32_t qi = sat_q[j];
        uint32_t s = uint32_t(qkeys[qi] >> 38);
        uint64_t a = qkeys[qi] & ((uint64_t(1) << 38) - 1);
        // locate the cube with that sequence number among this round's leaves
        const Cube* cube = nullptr;
        for (size_t i = first_of[qi]; i < sent.size() && sent[i].first == qi; i++)
          if (rh.cubes[i].seq == s) { cube = &sent[i].second; break; }
        if (!cube) fail(SCUBA_E_INTERNAL, "witness from an unknown cube");
        auto& rq = res->q[qi];
        rq.r.verdict = SCUBA_SAT;
        rq.r.how = SCUBA_HOW_DEVICE;
        assemble_witness(cnf->q[qi], sp[qi].get(), *cube, a, rq);
      });
      for (uint32_t qi : sat_q) open[qi] = 0;
      verify_ms += ms_since(tv);
      if (!speculate && more) split_round(after);   // only the queries still open
      last_split_ms = split_ms - split_before;
      next = std::move(after);
    }
    for (size_t qi = 0; qi < nq; qi++)
      if (open[qi]) {  // round limit reached
        res->q[qi].r.verdict = SCUBA_UNKNOWN;
        res->q[qi].r.how = SCUBA_HOW_BUDGET;
      }
    // the upload's pinned staging is free again only once the copy is done
    if (uploaded) dev_sync(hip_stream);
    // the walks' state (per-query counters, trails, orders) is released on
    // the pool rather than one query after another at scope exit
    parallel_for(nq, [&](size_t qi) { sp[qi].reset(); });
    res->ms[0] = split_ms;
    res->ms[1] = rt.h2d_ms;
    res->ms[2] = rt.up_ms + rt.leaf_ms + rt.graph_ms;
    res->ms[3] = rt.d2h_ms;
    res->ms[4] = verify_ms;
    res->ms[5] = ms_since(t0);
    res->ms[6] = rt.up_ms;
    res->ms[7] = rt.leaf_ms;
    res->ms[8] = rt.up_launches;
    res->ms[9] = rt.leaf_launches;
    res->ms[10] = rt.graph_ms;
    res->ms[11] = rt.graph_launches;
    if (runner) {
      res->ms[13] = runner->device_ms;
      res->ms[14] = double(runner->passes);
      res->ms[15] = double(runner->rows_scored);
    }
    res->ms[12] = rt.graph_captures;
    res->ms[16] = double(rt.cubes);
    res->ms[17] = double(rt.items);
    res->ms[18] = rt.fix_launches;
    return res;
  }
}

scuba_status scuba_decide(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_solve_opts* opts, void* dev_ws,
                          size_t ws_bytes, void* hip_stream, scuba_results** out) {
  if (!ctx || !cnf || !out || !dev_ws) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    Opts o = resolve(opts);
    if (o.flags & SCUBA_SOLVE_DEVICE_SPLIT)
      *out = decide_split_impl(ctx, cnf, o, dev_ws, ws_bytes, hip_stream).release();
    else
      *out = decide_impl(ctx, cnf, o, dev_ws, ws_bytes, hip_stream).release();
  });
}

scuba_status scuba_decide_noalloc(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_solve_opts* opts,
                                  void* hip_stream, scuba_results** out) {
  if (!ctx || !cnf || !out) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    Opts o = resolve(opts);
    if (o.flags & SCUBA_SOLVE_GRAPH)
      fail(SCUBA_E_INVALID, "scuba_decide_noalloc captures no graphs: clear SCUBA_SOLVE_GRAPH");
    if (o.flags & SCUBA_SOLVE_DEVICE_SPLIT)
      fail(SCUBA_E_INVALID, "scuba_decide_noalloc splits on the host: clear SCUBA_SOLVE_DEVICE_SPLIT");
    // the same bound as scuba_decide_workspace, checked before any device work
    CnfHost h = cnf_host(cnf, 0, true);
    size_t need = dev_cnf_bytes(h) + round_bound(cnf, size_t(cnf->q.size()) * o.lpr, o, o.max_res);
    if (o.scorer == SCUBA_SCORER_LEARNED) need += scorer_bytes(scorer_rows(cnf, o.learned->candidates)) + 256;
    if (need > kScratchBytes)
      fail(SCUBA_E_CAPACITY, "batch needs " + std::to_string(need) + " device bytes; the allocation-free "
           "entry point has " + std::to_string(kScratchBytes) + " (split the batch or use scuba_decide)");
    ctx->ensure_device();
    if (!ctx->dev.scratch || ctx->dev.scratch_bytes < need) fail(SCUBA_E_INTERNAL, "device scratch missing");
    struct Pageable {   // restores pinned staging on every exit
      scuba_ctx* c;
      explicit Pageable(scuba_ctx* c_) : c(c_) { c->pageable = true; }
      ~Pageable() { c->pageable = false; }
    } pg(ctx);
    *out = decide_impl(ctx, cnf, o, ctx->dev.scratch, ctx->dev.scratch_bytes, hip_stream).release();
  });
}

// ---------------------------------------------------------------- autotune

namespace {

constexpr uint32_t kTuneK[] = {16, 20, 24, 28, 30};
constexpr uint32_t kTuneChunk[] = {4, 6, 8, 10, 12};
constexpr uint32_t kTuneLpr[] = {1, 2, 4, 8, 16};
constexpr uint32_t kTuneGridPerCu[] = {2, 4, 8, 16};
constexpr uint32_t kTuneTile[] = {1024, 2048, 4096, 8192};
// leaf-evaluation variants: scalar skip test, vector skip test, vector
// skip test with the records staged in LDS
constexpr uint32_t kTuneLeaf[] = {0, SCUBA_SOLVE_LEAF_VECTOR, SCUBA_SOLVE_LEAF_VECTOR | SCUBA_SOLVE_LEAF_LDS};

struct TuneSetup {
  uint32_t sample, reps, scorer, flags;
  uint64_t max_cubes;
};

TuneSetup tune_setup(const scuba_tune_opts* t) {
  TuneSetup r{128, 2, SCUBA_SCORER_STATIC, 0, 20000};
  if (t) {
    if (t->sample) r.sample = t->sample;
    if (t->reps) r.reps = t->reps;
    if (t->max_cubes) r.max_cubes = t->max_cubes;
    r.scorer = t->scorer;
    r.flags = t->flags;
  }
  if (r.scorer != SCUBA_SCORER_STATIC && r.scorer != SCUBA_SCORER_WORD)
    fail(SCUBA_E_INVALID, "the autotuner tunes the static or the word ordering");
  if (r.flags & ~SCUBA_SOLVE_GRAPH) fail(SCUBA_E_INVALID, "unknown solve flags");
  return r;
}

// Queries spread over the size range: sorted by clause count, evenly spaced.
scuba_cnf tune_sample(const scuba_cnf* cnf, uint32_t n) {
  std::vector<size_t> idx(cnf->q.size());
  for (size_t i = 0; i < idx.size(); i++) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(),
                   [&](size_t a, size_t b) { return cnf->q[a].n_clauses() < cnf->q[b].n_clauses(); });
  scuba_cnf out;
  const size_t m = std::min<size_t>(n, idx.size());
  for (size_t j = 0; j < m; j++) out.q.push_back(cnf->q[idx[j * idx.size() / m]]);
  return out;
}

std::vector<uint64_t> tune_bucket(const scuba_cnf* cnf, const TuneSetup& ts) {
  double mean = 0;
  for (const CnfQuery& q : cnf->q) mean += double(q.n_clauses());
  mean /= double(std::max<size_t>(cnf->q.size(), 1));
  auto lg = [](double x) { return uint64_t(x < 1 ? 0 : std::log2(x)); };
  return {lg(mean), lg(double(cnf->q.size())), ts.scorer, ts.flags};
}

Opts tune_point(const TuneSetup& ts, uint32_t k, uint32_t chunk, uint32_t lpr, uint32_t grid,
                uint32_t tile = kDefaultMaxResidual, uint32_t leaf = 0) {
  Opts o{SCUBA_MODE_DECIDE, k, lpr, chunk, grid, 0, ts.scorer, ts.max_cubes, nullptr, ts.flags | leaf, tile, 0};
  return o;
}

size_t tune_bytes(const scuba_cnf* sample, const Opts& o) {
  CnfHost h = cnf_host(sample);
  return dev_cnf_bytes(h) + round_bound(sample, sample->q.size() * o.lpr, o, o.max_res);
}

}  // namespace

scuba_status scuba_autotune_workspace(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_tune_opts* opts,
                                      size_t* bytes) {
  if (!ctx || !cnf || !bytes) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    TuneSetup ts = tune_setup(opts);
    scuba_cnf sample = tune_sample(cnf, ts.sample);
    size_t most = 0;
    for (uint32_t k : kTuneK)
      for (uint32_t c : kTuneChunk)
        for (uint32_t l : kTuneLpr)
          for (uint32_t t : kTuneTile) most = std::max(most, tune_bytes(&sample, tune_point(ts, k, c, l, 0, t)));
    *bytes = most;
  });
}

scuba_status scuba_autotune(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_tune_opts* opts, void* dev_ws,
                            size_t ws_bytes, void* hip_stream, scuba_solve_opts* best,
                            scuba_tune_report* report) {
  if (!ctx || !cnf || !dev_ws || !best) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    TuneSetup ts = tune_setup(opts);
    ctx->ensure_device();
    scuba_tune_report rep{};
    const std::vector<uint64_t> bucket = tune_bucket(cnf, ts);
    auto hit = ctx->tuned.find(bucket);
    if (hit != ctx->tuned.end() && !(opts && opts->refresh)) {
      *best = hit->second;
      rep.cached = 1;
      if (report) *report = rep;
      return;
    }
    scuba_cnf sample = tune_sample(cnf, ts.sample);
    const uint32_t cus = uint32_t(ctx->dev.cus);
    std::vector<int32_t> verdicts(sample.q.size(), SCUBA_UNKNOWN);
    // wall time of the sample at a point (best of reps); +inf when skipped
    auto measure = [&](const Opts& o) {
      if (tune_bytes(&sample, o) > ws_bytes) return std::numeric_limits<double>::infinity();
      double bestt = std::numeric_limits<double>::infinity();
      for (uint32_t r = 0; r < ts.reps; r++) {
        auto t0 = Clock::now();
        std::unique_ptr<scuba_results> res = decide_impl(ctx, &sample, o, dev_ws, ws_bytes, hip_stream);
        bestt = std::min(bestt, ms_since(t0));
        for (size_t i = 0; i < verdicts.size(); i++) {
          const int32_t v = res->q[i].r.verdict;
          if (v == SCUBA_UNKNOWN) continue;
          if (verdicts[i] != SCUBA_UNKNOWN && verdicts[i] != v)
            fail(SCUBA_E_INTERNAL, "tuning points disagree on a verdict");
          verdicts[i] = v;
        }
      }
      rep.points++;
      return bestt;
    };
    uint32_t k = kDefaultK, chunk = kDefaultChunkLog2, lpr = kDefaultLeavesPerRound, gpc = 8;
    uint32_t tile = kDefaultMaxResidual, leaf = 0;
    double cur = measure(tune_point(ts, k, chunk, lpr, gpc * cus, tile, leaf));
    rep.default_ms = cur;
    auto sweep = [&](uint32_t* var, const uint32_t* vals, size_t n) {
      for (size_t i = 0; i < n; i++) {
        if (vals[i] == *var) continue;
        const uint32_t keep = *var;
        *var = vals[i];
        double t = measure(tune_point(ts, k, chunk, lpr, gpc * cus, tile, leaf));
        if (t < cur) cur = t;
        else *var = keep;
      }
    };
    sweep(&k, kTuneK, std::size(kTuneK));
    sweep(&chunk, kTuneChunk, std::size(kTuneChunk));
    sweep(&lpr, kTuneLpr, std::size(kTuneLpr));
    sweep(&gpc, kTuneGridPerCu, std::size(kTuneGridPerCu));
    sweep(&tile, kTuneTile, std::size(kTuneTile));
    sweep(&leaf, kTuneLeaf, std::size(kTuneLeaf));
    if (!std::isfinite(cur)) fail(SCUBA_E_CAPACITY, "no tuning point fits the workspace");
    scuba_solve_opts b{};
    b.mode = SCUBA_MODE_DECIDE;
    b.k = k;
    b.max_cubes = 0;
    b.leaves_per_round = lpr;
    b.chunk_log2 = chunk;
    b.grid = gpc * cus;
    b.scorer = ts.scorer;
    b.flags = ts.flags | leaf;
    b.max_residual = tile;
    ctx->tuned[bucket] = b;
    *best = b;
    rep.best_ms = cur;
    if (report) *report = rep;
  });
}

// One cache line: {"gpu":"<arch>","bucket":[b0,b1,b2,b3],"k":..,"chunk_log2":..,
// "leaves_per_round":..,"grid":..,"scorer":..,"flags":..,"max_residual":..}
namespace {
std::string device_key(scuba_ctx* ctx) {
  try {
    ctx->ensure_device();
    return ctx->dev.arch;
  } catch (const Error&) {
    return "no-device";   // a context without a device (the cache still round-trips)
  }
}
bool json_u64(const std::string& line, const char* key, uint64_t* out) {
  const std::string k = std::string("\"") + key + "\":";
  const size_t p = line.find(k);
  if (p == std::string::npos) return false;
  const char* s = line.c_str() + p + k.size();
  char* e = nullptr;
  const unsigned long long v = std::strtoull(s, &e, 10);
  if (e == s) return false;
  *out = v;
  return true;
}
}  // namespace

scuba_status scuba_tune_cache_save(scuba_ctx* ctx, const char* path) {
  if (!ctx || !path) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    const std::string gpu = device_key(ctx);
    FILE* f = std::fopen(path, "w");
    if (!f) fail(SCUBA_E_INVALID, std::string("cannot write ") + path);
    for (const auto& [b, o] : ctx->tuned) {
      if (b.size() != 4) continue;
      std::fprintf(f,
                   "{\"gpu\":\"%s\",\"bucket\":[%llu,%llu,%llu,%llu],\"k\":%u,\"chunk_log2\":%u,"
                   "\"leaves_per_round\":%u,\"grid\":%u,\"scorer\":%u,\"flags\":%u,\"max_residual\":%u}\n",
                   gpu.c_str(), (unsigned long long)b[0], (unsigned long long)b[1], (unsigned long long)b[2],
                   (unsigned long long)b[3], o.k, o.chunk_log2, o.leaves_per_round, o.grid, o.scorer, o.flags,
                   o.max_residual);
    }
    if (std::fclose(f) != 0) fail(SCUBA_E_INVALID, std::string("cannot write ") + path);
  });
}

scuba_status scuba_tune_cache_load(scuba_ctx* ctx, const char* path, uint32_t* loaded) {
  if (!ctx || !path) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    const std::string gpu = device_key(ctx);
    FILE* f = std::fopen(path, "r");
    if (!f) fail(SCUBA_E_INVALID, std::string("cannot read ") + path);
    uint32_t n = 0;
    char buf[1024];
    while (std::fgets(buf, sizeof buf, f)) {
      std::string line;   // without whitespace (JSON writers differ in spacing)
      for (const char* c = buf; *c; c++)
        if (!std::isspace(static_cast<unsigned char>(*c))) line.push_back(*c);
      if (line.find("\"gpu\":\"" + gpu + "\"") == std::string::npos) continue;   // another GPU's choice
      const size_t bp = line.find("\"bucket\":[");
      if (bp == std::string::npos) continue;
      std::vector<uint64_t> b(4);
      const char* s = line.c_str() + bp + 10;
      bool ok = true;
      for (int i = 0; i < 4 && ok; i++) {
        char* e = nullptr;
        b[i] = std::strtoull(s, &e, 10);
        ok = e != s && (*e == ',' || *e == ']');
        s = e + 1;
      }
      uint64_t k, c, l, g, sc, fl, mr;
      ok = ok && json_u64(line, "k", &k) && json_u64(line, "chunk_log2", &c) &&
           json_u64(line, "leaves_per_round", &l) && json_u64(line, "grid", &g) && json_u64(line, "scorer", &sc) &&
           json_u64(line, "flags", &fl) && json_u64(line, "max_residual", &mr);
      if (!ok) {
        std::fclose(f);
        fail(SCUBA_E_INVALID, std::string("malformed tune cache line in ") + path);
      }
      scuba_solve_opts o{};
      o.mode = SCUBA_MODE_DECIDE;
      o.k = uint32_t(k);
      o.chunk_log2 = uint32_t(c);
      o.leaves_per_round = uint32_t(l);
      o.grid = uint32_t(g);
      o.scorer = uint32_t(sc);
      o.flags = uint32_t(fl);
      o.max_residual = uint32_t(mr);
      resolve(&o);   // a line whose options the library would reject is an error
      ctx->tuned[b] = o;
      n++;
    }
    std::fclose(f);
    if (loaded) *loaded = n;
  });
}

// ---------------------------------------------------------------- learned scorer

uint32_t scuba_mlp_param_count(void) { return uint32_t(kMlpParams); }

scuba_status scuba_mlp_sync(scuba_ctx* ctx, const float* master, uint16_t* wbf16, void* hip_stream) {
  if (!ctx || !master || !wbf16) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    ctx->ensure_device();
    mlp_sync(master, wbf16, hip_stream);
  });
}

scuba_status scuba_mlp_forward(scuba_ctx* ctx, const uint16_t* wbf16, const float* master, const uint16_t* x,
                               uint32_t batch, uint16_t* a1, uint16_t* a2, float* y, void* hip_stream) {
  if (!ctx || !wbf16 || !master || (batch && (!x || !a1 || !a2 || !y))) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    ctx->ensure_device();
    mlp_forward(wbf16, master, x, batch, a1, a2, y, hip_stream);
  });
}

scuba_status scuba_mlp_backward(scuba_ctx* ctx, const uint16_t* wbf16, const uint16_t* x, const uint16_t* a1,
                                const uint16_t* a2, const float* y, const float* target, uint32_t batch,
                                uint16_t* dz1, uint16_t* dz2, float* grad, void* hip_stream) {
  if (!ctx || !wbf16 || !grad || (batch && (!x || !a1 || !a2 || !y || !target || !dz1 || !dz2)))
    return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    ctx->ensure_device();
    mlp_backward(wbf16, x, a1, a2, y, target, batch, dz1, dz2, grad, hip_stream);
  });
}

scuba_status scuba_mlp_adam(scuba_ctx* ctx, float* master, const float* grad, float* m, float* v,
                            uint16_t* wbf16, uint32_t step, float lr, float beta1, float beta2, float eps,
                            void* hip_stream) {
  if (!ctx || !master || !grad || !m || !v || !wbf16 || step == 0) return SCUBA_E_INVALID;
  return guard(ctx, [&] {
    ctx->ensure_device();
    mlp_adam(master, grad, m, v, wbf16, step, lr, beta1, beta2, eps, hip_stream);
  });
}

// ---------------------------------------------------------------- results

scuba_status scuba_result_get(const scuba_results* r, uint32_t qi, scuba_query_result* out) {
  if (!r || !out || qi >= r->q.size()) return SCUBA_E_INVALID;
  *out = r->q[qi].r;
  return SCUBA_OK;
}

scuba_status scuba_witness_get(const scuba_results* r, uint32_t qi, uint64_t* values, uint32_t n) {
  if (!r || qi >= r->q.size()) return SCUBA_E_INVALID;
  const auto& q = r->q[qi];
  if (q.r.verdict != SCUBA_SAT) return SCUBA_E_STATE;
  if (n < q.witness.size() || (!q.witness.empty() && !values)) return SCUBA_E_CAPACITY;
  std::copy(q.witness.begin(), q.witness.end(), values);
  return SCUBA_OK;
}

scuba_status scuba_model_get(const scuba_results* r, uint32_t qi, uint8_t* bits, uint32_t n) {
  if (!r || qi >= r->q.size()) return SCUBA_E_INVALID;
  const auto& q = r->q[qi];
  if (q.r.verdict != SCUBA_SAT) return SCUBA_E_STATE;
  if (n < q.model.size() || !bits) return SCUBA_E_CAPACITY;
  std::copy(q.model.begin(), q.model.end(), bits);
  return SCUBA_OK;
}

scuba_status scuba_leaf_get(const scuba_results* r, uint32_t qi, uint64_t cube, scuba_leaf_result* out) {
  if (!r || !out || qi >= r->q.size()) return SCUBA_E_INVALID;
  if (cube >= r->q[qi].leaves.size()) return SCUBA_E_STATE;
  *out = r->q[qi].leaves[cube];
  return SCUBA_OK;
}

scuba_status scuba_results_timing(const scuba_results* r, double* ms, uint32_t n) {
  if (!r || !ms || n > 19) return SCUBA_E_INVALID;
  std::copy(r->ms, r->ms + n, ms);
  return SCUBA_OK;
}

void scuba_results_free(scuba_results* r) { delete r; }

}  // extern "C"
