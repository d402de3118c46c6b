// Host-side exercise of the library's C ABI for the AddressSanitizer /
// UndefinedBehaviorSanitizer build: bit-blast, split (static and word
// orderings), traces, raw CNFs, given cubes, views and every error path that
// needs no GPU.  Inputs are files written by the test: query batches in the
// boundary's layout and raw CNF batches.  Exits non-zero on an unexpected
// status; the sanitizers abort on the first memory or UB error.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "scuba.h"

namespace {

template <typename T>
std::vector<T> read_array(FILE* f) {
  uint64_t n = 0;
  if (fread(&n, 8, 1, f) != 1) { fprintf(stderr, "short file\n"); exit(2); }
  std::vector<T> v(n);
  if (n && fread(v.data(), sizeof(T), n, f) != n) { fprintf(stderr, "short file\n"); exit(2); }
  return v;
}

#define CHECK(x)                                                                         \
  do {                                                                                   \
    scuba_status st_ = (x);                                                              \
    if (st_ != SCUBA_OK) {                                                               \
      fprintf(stderr, "%s failed: %s (%s)\n", #x, scuba_status_str(st_), scuba_last_error(ctx)); \
      exit(1);                                                                           \
    }                                                                                    \
  } while (0)
#define EXPECT_FAIL(x)                                                                   \
  do {                                                                                   \
    if ((x) == SCUBA_OK) { fprintf(stderr, "%s succeeded unexpectedly\n", #x); exit(1); } \
  } while (0)

void walk_cubes(scuba_ctx* ctx, const scuba_cnf* cnf, const scuba_cubes* cubes) {
  for (uint32_t q = 0; q < scuba_cnf_count(cnf); q++) {
    scuba_cubes_view v;
    CHECK(scuba_cubes_view_get(cubes, q, &v));
    uint64_t lits = 0;
    for (uint64_t c = 0; c < v.n_cubes; c++) lits += v.cube_off[c + 1] - v.cube_off[c];
    (void)lits;
  }
}

void queries(scuba_ctx* ctx, const char* path, uint32_t flags) {
  FILE* f = fopen(path, "rb");
  if (!f) { perror(path); exit(2); }
  std::vector<scuba_node> nodes = read_array<scuba_node>(f);
  std::vector<uint64_t> nstart = read_array<uint64_t>(f);
  std::vector<uint32_t> roots = read_array<uint32_t>(f);
  std::vector<uint64_t> rstart = read_array<uint64_t>(f);
  fclose(f);
  const uint32_t nq = uint32_t(nstart.size() - 1);
  scuba_cnf* cnf = nullptr;
  CHECK(scuba_bitblast(ctx, nq, nodes.data(), nstart.data(), roots.data(), rstart.data(), flags, &cnf));
  for (uint32_t q = 0; q < nq; q++) {
    scuba_cnf_view v;
    CHECK(scuba_cnf_view_get(cnf, q, &v));
    std::vector<uint32_t> first(v.n_inputs + 1), width(v.n_inputs + 1);
    CHECK(scuba_cnf_input_map(cnf, q, first.data(), width.data(), v.n_inputs));
  }
  for (uint32_t scorer : {SCUBA_SCORER_STATIC, SCUBA_SCORER_WORD}) {
    scuba_split_opts so{};
    so.k = 20;
    so.scorer = scorer;
    so.max_cubes = 200;
    scuba_cubes* cubes = nullptr;
    CHECK(scuba_split(ctx, cnf, &so, &cubes));
    walk_cubes(ctx, cnf, cubes);
    scuba_cubes_free(cubes);
  }
  scuba_trace_opts to{16, 8, 1, 12, 64};
  scuba_trace* tr = nullptr;
  CHECK(scuba_trace_run(ctx, cnf, &to, &tr));
  uint64_t rows = 0;
  const float *fe = nullptr, *la = nullptr;
  const uint64_t* no = nullptr;
  CHECK(scuba_trace_view(tr, &rows, &fe, &la, &no));
  scuba_trace_free(tr);
  // malformed input: a node that refers forward, a bad op, a zero width
  if (nq && nstart[1] > 1) {
    std::vector<scuba_node> bad(nodes.begin(), nodes.begin() + nstart[1]);
    bad.back().a = uint32_t(bad.size());
    uint64_t ns[2] = {0, bad.size()}, rs[2] = {0, 0};
    scuba_cnf* out = nullptr;
    EXPECT_FAIL(scuba_bitblast(ctx, 1, bad.data(), ns, roots.data(), rs, 0, &out));
    bad.back() = nodes[0];
    bad.back().op = 99;
    EXPECT_FAIL(scuba_bitblast(ctx, 1, bad.data(), ns, roots.data(), rs, 0, &out));
    bad[0].width = 0;
    EXPECT_FAIL(scuba_bitblast(ctx, 1, bad.data(), ns, roots.data(), rs, 0, &out));
  }
  scuba_cnf_free(cnf);
}

void raw(scuba_ctx* ctx, const char* path) {
  FILE* f = fopen(path, "rb");
  if (!f) { perror(path); exit(2); }
  std::vector<uint32_t> nv = read_array<uint32_t>(f);
  std::vector<uint64_t> qs = read_array<uint64_t>(f);
  std::vector<uint64_t> off = read_array<uint64_t>(f);
  std::vector<int32_t> lits = read_array<int32_t>(f);
  fclose(f);
  const uint32_t nq = uint32_t(nv.size());
  scuba_cnf* cnf = nullptr;
  CHECK(scuba_cnf_from_arrays(ctx, nq, nv.data(), qs.data(), off.data(), lits.data(), &cnf));
  scuba_split_opts so{};
  so.k = 10;
  so.max_cubes = 5000;
  scuba_cubes* cubes = nullptr;
  CHECK(scuba_split(ctx, cnf, &so, &cubes));
  walk_cubes(ctx, cnf, cubes);
  scuba_cubes_free(cubes);
  // given cubes: one per query, the first literal of its first clause
  std::vector<uint64_t> cq(nq + 1), co(nq + 1);
  std::vector<int32_t> cl;
  for (uint32_t q = 0; q < nq; q++) {
    cq[q] = q;
    co[q] = cl.size();
    if (qs[q + 1] > qs[q]) cl.push_back(lits[off[qs[q]]]);
  }
  cq[nq] = nq;
  co[nq] = cl.size();
  if (cl.empty()) cl.push_back(1);
  CHECK(scuba_cubes_from_arrays(ctx, cnf, cq.data(), co.data(), cl.data(), &cubes));
  walk_cubes(ctx, cnf, cubes);
  scuba_cubes_free(cubes);
  // a literal outside the formula is refused
  std::vector<int32_t> bad(lits);
  if (!bad.empty()) {
    bad[0] = int32_t(nv[0] + 1);
    scuba_cnf* out = nullptr;
    EXPECT_FAIL(scuba_cnf_from_arrays(ctx, nq, nv.data(), qs.data(), off.data(), bad.data(), &out));
  }
  scuba_cnf_free(cnf);
}

}  // namespace

int main(int argc, char** argv) {
  scuba_ctx* ctx = nullptr;
  if (scuba_ctx_create(0, &ctx) != SCUBA_OK) return 1;
  for (int i = 1; i + 1 < argc; i += 2) {
    const std::string kind = argv[i];
    if (kind == "queries") queries(ctx, argv[i + 1], 0);
    else if (kind == "norewrite") queries(ctx, argv[i + 1], SCUBA_BB_NO_REWRITE);
    else if (kind == "wrap32") queries(ctx, argv[i + 1], SCUBA_BB_WRAP(32));
    else if (kind == "raw") raw(ctx, argv[i + 1]);
    else { fprintf(stderr, "unknown input kind %s\n", kind.c_str()); return 2; }
  }
  scuba_ctx_destroy(ctx);
  printf("host check ok\n");
  return 0;
}
