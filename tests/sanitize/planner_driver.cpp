// Host-only driver of the library's validator and planner, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitized_planner.py. It needs no GPU: every call below
// either plans on the host (cbc_query, cbc_plan_info, cbc_plan_bonds) or fails argument checks
// before any device work. It prints one line per call; the test compares them with the expected
// status codes and fails on any sanitizer report.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "cbc.h"

namespace {

struct TreeDef {
  std::string name;
  std::vector<int32_t> parent, phys, chi, dop;
  int32_t max_bond;
  int expect;   // status of cbc_query
};

// bond of every edge: min(cap, product of the physical dims on the smaller side of the cut)
std::vector<int32_t> cut(const std::vector<int32_t>& parent, const std::vector<int32_t>& phys,
                         int cap, int power) {
  const int n = (int)parent.size();
  std::vector<double> below(n, 1.0);
  double total = 1.0;
  for (int i = 0; i < n; ++i) total *= phys[i];
  // children have larger indices than their parents in every tree built here
  for (int i = n - 1; i >= 0; --i) {
    below[i] *= phys[i];
    if (parent[i] >= 0) below[parent[i]] *= below[i];
  }
  std::vector<int32_t> b(n, 1);
  for (int i = 0; i < n; ++i) {
    if (parent[i] < 0) continue;
    double side = below[i] < total / below[i] ? below[i] : total / below[i];
    double v = 1.0;
    for (int p = 0; p < power; ++p) v *= side;
    b[i] = v < cap ? (int32_t)v : cap;
  }
  return b;
}

TreeDef kary(const std::string& name, int n, int k, int d, int chi, int D, int mb, int expect) {
  TreeDef t;
  t.name = name;
  for (int i = 0; i < n; ++i) t.parent.push_back(i == 0 ? -1 : (k == 1 ? i - 1 : (i - 1) / k));
  t.phys.assign(n, d);
  t.chi = cut(t.parent, t.phys, chi, 1);
  t.dop = cut(t.parent, t.phys, D, 2);
  t.max_bond = mb;
  t.expect = expect;
  return t;
}

cbc_tree view(TreeDef& t) {
  cbc_tree c;
  c.n_nodes = (int32_t)t.parent.size();
  c.parent = t.parent.data();
  c.phys = t.phys.data();
  c.chi = t.chi.data();
  c.dop = t.dop.data();
  return c;
}

int failures = 0;
void expect(const char* what, const std::string& name, int got, int want) {
  std::printf("%s %s %d\n", what, name.c_str(), got);
  if (got != want) {
    std::printf("MISMATCH %s %s: %d, expected %d\n", what, name.c_str(), got, want);
    ++failures;
  }
}

}  // namespace

int main(int argc, char** argv) {
  std::vector<TreeDef> trees;
  trees.push_back(kary("chain8", 8, 1, 2, 8, 4, 32, 0));
  trees.push_back(kary("chain64", 64, 1, 2, 64, 8, 64, 0));
  trees.push_back(kary("chain10_large_bond", 10, 1, 4, 256, 16, 256, 0));
  trees.push_back(kary("binary31", 31, 2, 2, 32, 6, 32, 0));
  trees.push_back(kary("ternary13", 13, 3, 2, 6, 3, 5, 0));
  trees.push_back(kary("ternary13_d4", 13, 3, 4, 32, 12, 32, 0));
  trees.push_back(kary("single", 1, 1, 3, 1, 1, 2, 0));
  {
    TreeDef t = kary("leafphys", 7, 2, 2, 4, 4, 3, 0);
    t.phys = {1, 1, 1, 2, 2, 2, 2};
    t.chi = cut(t.parent, t.phys, 4, 1);
    t.dop = cut(t.parent, t.phys, 4, 2);
    trees.push_back(t);
  }
  {
    TreeDef t = kary("two_roots", 3, 1, 2, 2, 2, 4, CBC_ESHAPE);
    t.parent = {-1, -1, 0};
    trees.push_back(t);
  }
  {
    TreeDef t = kary("cycle", 3, 1, 2, 2, 2, 4, CBC_ESHAPE);
    t.parent = {1, 2, 0};
    trees.push_back(t);
  }
  {
    TreeDef t = kary("parent_out_of_range", 3, 1, 2, 2, 2, 4, CBC_ESHAPE);
    t.parent = {-1, 5, 0};
    trees.push_back(t);
  }
  {
    TreeDef t = kary("zero_bond", 2, 1, 2, 2, 2, 4, CBC_ESHAPE);
    t.chi = {1, 0};
    trees.push_back(t);
  }
  {
    TreeDef t = kary("oversized_gram", 2, 1, 2, 2, 2, 64, CBC_EUNSUP);
    t.phys = {2065, 2};
    t.chi = {1, 2065};
    t.dop = {1, 1};
    trees.push_back(t);
  }
  {
    TreeDef t = kary("beyond_32bit_offsets", 2, 1, 2, 2, 2, 4, CBC_EUNSUP);
    t.phys = {46341, 2};
    t.chi = {1, 2};
    t.dop = {1, 4};
    trees.push_back(t);
  }

  cbc_ctx* ctx = nullptr;
  expect("create", "ctx", cbc_create(&ctx), CBC_OK);
  for (TreeDef& t : trees) {
    cbc_tree c = view(t);
    const int n = c.n_nodes;
    std::vector<int64_t> off(n + 1, 0);
    for (int prec = 0; prec < 2; ++prec) {
      for (int method = 0; method < 5; ++method) {
        size_t ws = 0;
        const int rc = cbc_query(ctx, &c, t.max_bond, (cbc_precision)prec, method, &ws, off.data());
        // the naive method forms the exact product, whose Grams exceed the limit sooner
        if (method == 0) expect("query", t.name, rc, t.expect);
        if (rc != CBC_OK) continue;
        for (int tol_on = 0; tol_on < 2; ++tol_on) {
          cbc_plan_summary info;
          std::memset(&info, 0, sizeof(info));
          expect("plan_info", t.name,
                 cbc_plan_info(ctx, &c, t.max_bond, (cbc_precision)prec, method, tol_on, &info),
                 CBC_OK);
          if (info.persistent_bytes + info.scratch_bytes > ws) {
            std::printf("MISMATCH plan_info %s: parts exceed the queried workspace\n",
                        t.name.c_str());
            ++failures;
          }
        }
      }
    }
    std::vector<int32_t> bond(n, 0);
    const int rb = cbc_plan_bonds(ctx, &c, t.max_bond, 0, bond.data());
    expect("plan_bonds", t.name, rb, t.expect == CBC_EUNSUP ? CBC_EUNSUP : t.expect);
    if (t.expect != CBC_OK) continue;
    // cbc_apply argument errors, all found before any device work
    std::vector<int64_t> soff(n, 0), ooff(n, 0);
    int64_t se = 0, oe = 0;
    for (int i = 0; i < n; ++i) {
      int64_t a = t.phys[i], b = (int64_t)t.phys[i] * t.phys[i];
      a *= t.chi[i];
      b *= t.dop[i];
      for (int j = 0; j < n; ++j)
        if (t.parent[j] == i) {
          a *= t.chi[j];
          b *= t.dop[j];
        }
      soff[i] = se;
      ooff[i] = oe;
      se += a;
      oe += b;
    }
    size_t ws = 0;
    cbc_query(ctx, &c, t.max_bond, CBC_PREC_FP64, 0, &ws, off.data());
    cbc_tensors ttns{(const void*)0x1000, soff.data()};
    cbc_tensors ttno{(const void*)0x1000, ooff.data()};
    cbc_out out{(void*)0x1000, off.data(), bond.data()};
    void* wsp = (void*)0x1000;
    expect("apply_small_ws", t.name,
           cbc_apply(ctx, &ttno, &ttns, &c, t.max_bond, 0.0, CBC_PREC_FP64, wsp, ws - 1, &out,
                     nullptr, nullptr),
           CBC_ENOMEM);
    expect("apply_neg_tol", t.name,
           cbc_apply(ctx, &ttno, &ttns, &c, t.max_bond, -1.0, CBC_PREC_FP64, wsp, ws, &out,
                     nullptr, nullptr),
           CBC_EINVAL);
    expect("apply_bad_prec", t.name,
           cbc_apply(ctx, &ttno, &ttns, &c, t.max_bond, 0.0, (cbc_precision)7, wsp, ws, &out,
                     nullptr, nullptr),
           CBC_EINVAL);
    std::vector<int64_t> bad = soff;
    bad[n - 1] += 1000000;
    cbc_tensors ttns_bad{(const void*)0x1000, bad.data()};
    expect("apply_unpacked", t.name,
           cbc_apply(ctx, &ttno, &ttns_bad, &c, t.max_bond, 0.0, CBC_PREC_FP64, wsp, ws, &out,
                     nullptr, nullptr),
           CBC_EINVAL);
    expect("apply_split_null", t.name,
           cbc_apply_split(ctx, &ttno, &ttns, &c, t.max_bond, 0.0, CBC_PREC_FP64, wsp, ws,
                           nullptr, 0, &out, nullptr, nullptr),
           CBC_EINVAL);
    expect("apply_batched_zero", t.name,
           cbc_apply_batched(ctx, 0, &ttno, &ttns, &c, t.max_bond, 0.0, CBC_PREC_FP64, wsp, ws,
                             &out, nullptr, nullptr),
           CBC_EINVAL);
  }
  // autotune cache parsing: foreign, malformed and valid lines
  if (argc > 1) {
    FILE* f = std::fopen(argv[1], "w");
    std::fprintf(f, "cbc-gemm 1 1 0 0 64 64 128 1 0 1 0 4 0.010\ncbc-gemm 1 1 0 0 64 64 128 1 0 1 7 "
                    "4 0.010\nsome other text\ncbc-gemm 1 2\ncbc-gemm");
    std::fclose(f);
    expect("autotune", "cache", cbc_autotune(ctx, argv[1]), CBC_OK);
  }
  expect("report_null", "rep", cbc_read_report(nullptr, 0, 0, nullptr, nullptr), CBC_EINVAL);
  expect("many_empty", "many", cbc_apply_many(ctx, 0, nullptr, CBC_PREC_FP64, 4, nullptr, nullptr,
                                               nullptr), CBC_OK);
  {
    cbc_problem probs[2];
    std::memset(probs, 0, sizeof(probs));
    expect("many_null_problem", "many", cbc_apply_many(ctx, 2, probs, CBC_PREC_FP64, 2, nullptr,
                                                       nullptr, nullptr), CBC_EINVAL);
  }
  cbc_destroy(ctx);
  std::printf("failures %d\n", failures);
  return failures == 0 ? 0 : 1;
}
