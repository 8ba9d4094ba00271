// C ABI, host-side validation, planner and executor for Cholesky-based compression on gfx950.
//
// The planner turns a tree, its dimensions, a target bond dimension and a precision into a static
// sequence of kernel launches: every tensor shape is fixed by max_bond before any device work, so a
// call is a fixed launch sequence (and is replayed from a captured hipGraph after the first call).
// Data-dependent truncation by a tolerance only zeroes slices on device.
//
// Sweeps (Sec. III B; Sec. III A is the chain rooted at its first site, which needs only sweeps 2-3):
//   1. leaves -> root : L^{[i]}     from T, W and the children's L^{[c]} (Eq. cbc_tree_first_contraction)
//   2. root -> leaves : L^{[(i,k)]} from T, W, L^{[(p,i)]} and siblings' L^{[c]} (Eq. cbc_tree_second_contraction)
//   3. leaves -> root : Z = T W prod_c R^{[c]}; S = L^{[(p,i)]} Z (Eq. cbc_tree_third_contraction);
//      QR on the parent leg (Eq. cbc_tree_qr); R^{[i]} = Q^* Z (Eq. cbc_final_contraction, with the
//      conjugate as in the tensor-train update); the root keeps S.
// Each truncation joins (sigma', chi...) and keeps the top-k eigenspace of the FP64 Gram matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cbc.h"
#include "cbc_internal.h"

using namespace cbc;

namespace {

// ------------------------------------------------------------------------------------------------
// plan representation

enum Src : int { S_NONE = -1, S_WS = 0, S_SCR = 1, S_STATE = 2, S_OP = 3, S_OUT = 4, S_SKETCH = 5 };

struct TRef {
  int src = S_NONE;
  int64_t off = 0;   // bytes for S_WS/S_SCR; node index for S_STATE/S_OP/S_OUT
  DType dt = DT_C128;
};

struct Ten {
  TRef ref;
  std::vector<int> legs;
  bool cj = false;   // enters contractions complex-conjugated (the bra copies of a network)
};

enum OpKind : int { K_GEMM, K_EIG, K_FORM_N, K_CHOL, K_CONVERT, K_IDENT, K_WRITE, K_ZERO, K_HEADER,
                     K_NORM };

// Start of every instance's workspace: the call's report (read by cbc_read_report). The kernels
// store a failure code into `status` (first one wins) and add dropped pivots to `ndrop`; the
// truncation records (cbc_trunc_record) start `rec_off` bytes into the workspace.
struct WsHeader {
  uint32_t magic;
  int32_t status;
  int32_t ndrop;
  int32_t n_rec;
  int64_t rec_off;
  int64_t reserved[5];
};
static_assert(sizeof(WsHeader) == 64, "report header layout");
constexpr uint32_t REPORT_MAGIC = 0x31434243u;   // "CBC1"
constexpr int64_t HDR_STATUS = 4, HDR_NDROP = 8;

struct Op {
  OpKind kind;
  int cls = CBC_K_OTHER;     // kernel class for statistics
  double flops = 0.0, bytes = 0.0;
  // GEMM
  TRef A, B, C;
  int M = 0, N = 0, K = 0;
  int64_t tAm = 0, tAk = 0, tBk = 0, tBn = 0, tCm = 0, tCn = 0;
  int conjA = 0, conjB = 0, akf = 0, bkf = 0, tile = 0, ksplit = 1;
  int herm = 0;   // a Gram of one tensor with its own conjugate: the lower half, mirrored
  // a leg shared by A, B and C (element-wise, not summed): zb instances, one per index value, the
  // operands advanced by zsA / zsB / zsC elements per instance (0 where an operand lacks the leg)
  int zb = 1;
  int64_t zsA = 0, zsB = 0, zsC = 0;
  int kcap = 1;   // largest split the scratch `part` has room for
  bool tuned = false;   // tile and split set by the autotuner for the current batch
  TRef part;   // split-K chunk sums (scratch)
  DType ta = DT_C128, tb = DT_C128, tc = DT_C128, acc = DT_C128;
  double alpha = 1.0;
  TRef adev, adev2;
  // EIG / FORM_N / CHOL
  TRef G, U, lam, kkeep, invs, work, Cinv, logs, scale, ndrop, L, rec, status;
  int s = 0, kmax = 0, n = 0;
  int rec_node = -1, rec_sweep = 0, rec_index = -1;
  double shift_rel = 0.0, drop_rel = 0.0;
  // CONVERT / IDENT / WRITE / ZERO
  TRef src, dst;
  DType ts = DT_C128, td = DT_C128;
  int64_t count = 0;
  int a = 0, b = 0;
  int64_t rest = 0;
  int nlogs = 0;
};

struct Plan {
  std::vector<Op> ops;
  // offset tables of the contractions: table_entries int32 values, filled on the host only for plans
  // that will run (sizes-only plans for queries skip them), freed there once copied to d_tables
  std::vector<int32_t> tables;
  int32_t* d_tables = nullptr;
  int64_t table_entries = 0;
  bool has_tables = false;
  size_t persist_bytes = 0, scratch_bytes = 0;
  std::vector<int64_t> out_off;
  std::vector<int32_t> out_bond;
  double cflops = 0.0, gflops = 0.0;
  int n_eig = 0, max_eig = 0;
  bool unsupported = false;   // a step exceeds this build's kernel limits
  bool has_gate = false;      // some eigensolve's workgroups wait for each other (see mw_gate_*)
  int n_rec = 0;              // truncation records
  int64_t rec_off = 0;        // their byte offset in the workspace
  bool tune = false;          // built for autotuning: scratch for split candidates reserved
  int tuned_batch = 0;        // batch the contractions were last tuned for (0: not tuned)
  int launches[CBC_K_NCLASS] = {0};
  double flops[CBC_K_NCLASS] = {0.0};
  double bytes[CBC_K_NCLASS] = {0.0};
  std::vector<hipEvent_t> events;
  // misc device slots (persistent workspace offsets)
  int64_t logs_off = 0;
  int64_t state_conv_off = -1, op_conv_off = -1, sketch_conv_off = -1;
  int64_t state_elems = 0, op_elems = 0, sketch_elems = 0;
  // captured graphs, one per buffer set (key: buffers, offsets, batch, tol), each with an event
  // recorded after its last launch so that it is destroyed only once it has finished
  struct Exec {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    uint64_t used = 0;
  };
  std::map<std::vector<uintptr_t>, Exec> graphs;
  uint64_t graph_clock = 0;
  static constexpr size_t MAX_GRAPHS = 32;
  void drop_graph(std::map<std::vector<uintptr_t>, Exec>::iterator it) {
    if (it->second.done) {
      (void)hipEventSynchronize(it->second.done);
      (void)hipEventDestroy(it->second.done);
    }
    if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
    graphs.erase(it);
  }
  void drop_graphs() {
    while (!graphs.empty()) drop_graph(graphs.begin());
  }
  ~Plan() {
    drop_graphs();
    if (d_tables) (void)hipFree(d_tables);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
  }
};

struct Problem {
  int n;
  std::vector<int> parent, phys, chi, dop;
  std::vector<std::vector<int>> ch;
  int root;
  std::vector<int> post;  // children before parents
};

// ------------------------------------------------------------------------------------------------
// validation

cbc_status validate_tree(const cbc_tree* t, Problem& P) {
  if (!t || !t->parent || !t->phys || !t->chi || !t->dop) return CBC_EINVAL;
  const int n = t->n_nodes;
  if (n < 1 || n > (1 << 20)) return CBC_ESHAPE;
  P.n = n;
  P.parent.assign(t->parent, t->parent + n);
  P.phys.assign(t->phys, t->phys + n);
  P.chi.assign(t->chi, t->chi + n);
  P.dop.assign(t->dop, t->dop + n);
  P.root = -1;
  for (int i = 0; i < n; ++i) {
    const int p = P.parent[i];
    if (p == -1) {
      if (P.root >= 0) return CBC_ESHAPE;
      P.root = i;
    } else if (p < 0 || p >= n || p == i) {
      return CBC_ESHAPE;
    }
    if (P.phys[i] < 1 || P.chi[i] < 1 || P.dop[i] < 1) return CBC_ESHAPE;
    if (P.phys[i] > 65536 || P.chi[i] > 65536 || P.dop[i] > 65536) return CBC_ESHAPE;
  }
  if (P.root < 0) return CBC_ESHAPE;
  if (P.chi[P.root] != 1 || P.dop[P.root] != 1) return CBC_ESHAPE;
  // every node must reach the root (no cycles)
  for (int i = 0; i < n; ++i) {
    int j = i, steps = 0;
    while (j != P.root) {
      j = P.parent[j];
      if (++steps > n) return CBC_ESHAPE;
    }
  }
  P.ch.assign(n, {});
  for (int i = 0; i < n; ++i)
    if (P.parent[i] >= 0) P.ch[P.parent[i]].push_back(i);
  // post-order (iterative)
  P.post.clear();
  std::vector<std::pair<int, int>> st{{P.root, 0}};
  while (!st.empty()) {
    auto& [node, idx] = st.back();
    if (idx < (int)P.ch[node].size()) {
      const int c = P.ch[node][idx++];
      st.push_back({c, 0});
    } else {
      P.post.push_back(node);
      st.pop_back();
    }
  }
  return CBC_OK;
}

// ------------------------------------------------------------------------------------------------
// planner

static constexpr int TUNE_KS = 8;   // largest split-K the autotuner tries

struct Builder {
  Plan& P;
  const Problem& pr;
  int max_bond;
  bool tol_on;
  DType ct, cacc;           // contraction storage type and accumulator
  std::vector<int64_t> legdim;
  size_t persist = 0, scratch = 0, scratch_max = 0;

  bool bad = false;         // an internal planning invariant failed (reported as CBC_ESHAPE)
  bool fill_tables = true;  // false: sizes only (offsets into the tables are still assigned)
  static constexpr int64_t ELEM_LIMIT = (int64_t)1 << 31;   // 32-bit element offsets

  Builder(Plan& p, const Problem& q, int mb, bool tol, cbc_precision prec)
      : P(p), pr(q), max_bond(mb), tol_on(tol) {
    ct = prec == CBC_PREC_MIXED ? DT_C64 : DT_C128;
    cacc = ct;
  }

  int leg(int64_t d) {
    legdim.push_back(d);
    return (int)legdim.size() - 1;
  }
  static size_t esz(DType t) { return t == DT_C128 ? 16 : 8; }
  static size_t al(size_t x) { return (x + 255) & ~size_t(255); }
  TRef wsp(size_t bytes, DType dt) {
    TRef r;
    r.src = S_WS;
    r.off = (int64_t)persist;
    r.dt = dt;
    persist += al(bytes);
    return r;
  }
  TRef scr(size_t bytes, DType dt) {
    TRef r;
    r.src = S_SCR;
    r.off = (int64_t)scratch;
    r.dt = dt;
    scratch += al(bytes);
    scratch_max = std::max(scratch_max, scratch);
    return r;
  }
  void reset_scratch() { scratch = 0; }
  int64_t elems(const std::vector<int>& legs) const {
    int64_t e = 1;
    for (int l : legs) e *= legdim[l];
    return e;
  }
  Ten alloc(const std::vector<int>& legs, DType dt, bool persistent) {
    Ten t;
    t.legs = legs;
    const size_t bytes = (size_t)elems(legs) * esz(dt);
    t.ref = persistent ? wsp(bytes, dt) : scr(bytes, dt);
    return t;
  }
  std::vector<int64_t> strides(const std::vector<int>& legs) const {
    std::vector<int64_t> s(legs.size());
    int64_t acc = 1;
    for (int i = (int)legs.size() - 1; i >= 0; --i) {
      s[i] = acc;
      acc *= legdim[legs[i]];
    }
    return s;
  }
  static int pos(const std::vector<int>& v, int x) {
    for (int i = 0; i < (int)v.size(); ++i)
      if (v[i] == x) return i;
    return -1;
  }
  // enumerate a multi-index over `legs` (last fastest) -> offsets in two tensors
  int64_t table(const std::vector<int>& legs, const std::vector<int64_t>& s1,
                const std::vector<int64_t>& s2, int64_t& t2) {
    int64_t cnt = 1;
    for (int l : legs) cnt *= legdim[l];
    const int64_t t1 = P.table_entries;
    P.table_entries += 2 * cnt;
    t2 = t1 + cnt;
    if (!fill_tables) return t1;
    P.tables.resize((size_t)P.table_entries);
    std::vector<int64_t> idx(legs.size(), 0);
    for (int64_t e = 0; e < cnt; ++e) {
      int64_t o1 = 0, o2 = 0;
      for (size_t j = 0; j < legs.size(); ++j) {
        o1 += idx[j] * s1[j];
        o2 += idx[j] * s2[j];
      }
      P.tables[t1 + e] = (int32_t)o1;
      P.tables[t2 + e] = (int32_t)o2;
      for (int j = (int)legs.size() - 1; j >= 0; --j) {
        if (++idx[j] < legdim[legs[j]]) break;
        idx[j] = 0;
      }
    }
    return t1;
  }

  // C[out] = alpha * sum opA(A) opB(B); legs shared by A and B and absent from `out` are summed.
  Ten contract(const Ten& A, bool conjA, const Ten& B, bool conjB, const std::vector<int>& out,
               const TRef& Cref, DType tc, DType acc, int bucket, double alpha = 1.0,
               TRef adev = TRef(), TRef adev2 = TRef()) {
    std::vector<int> ml, nl, kl, zl;
    for (int l : A.legs) {
      if (pos(out, l) >= 0) (pos(B.legs, l) >= 0 ? zl : ml).push_back(l);
      else if (pos(B.legs, l) >= 0) kl.push_back(l);
      else bad = true;   // a leg of A that is neither summed nor kept
    }
    for (int l : B.legs) {
      if (pos(out, l) >= 0) {
        if (pos(A.legs, l) < 0) nl.push_back(l);
      } else if (pos(A.legs, l) < 0) {
        bad = true;
      }
    }
    if (zl.size() > 1) bad = true;   // at most one element-wise leg per contraction
    // the kernels address operands with 32-bit element offsets from tables
    if (elems(A.legs) >= ELEM_LIMIT || elems(B.legs) >= ELEM_LIMIT || elems(out) >= ELEM_LIMIT)
      P.unsupported = true;
    if (bad || P.unsupported) {
      Ten r;
      r.ref = Cref;
      r.ref.dt = tc;
      r.legs = out;
      return r;
    }
    const auto sA = strides(A.legs), sB = strides(B.legs), sC = strides(out);
    auto pick = [&](const std::vector<int>& legs, const std::vector<int>& of,
                    const std::vector<int64_t>& st) {
      std::vector<int64_t> r;
      for (int l : legs) r.push_back(st[pos(of, l)]);
      return r;
    };
    Op op;
    op.kind = K_GEMM;
    op.A = A.ref;
    op.B = B.ref;
    op.C = Cref;
    op.M = (int)elems(ml);
    op.N = (int)elems(nl);
    op.K = (int)elems(kl);
    op.tAm = table(ml, pick(ml, A.legs, sA), pick(ml, out, sC), op.tCm);
    op.tBn = table(nl, pick(nl, B.legs, sB), pick(nl, out, sC), op.tCn);
    op.tAk = table(kl, pick(kl, A.legs, sA), pick(kl, B.legs, sB), op.tBk);
    if (!zl.empty()) {
      const int z = zl[0];
      op.zb = (int)legdim[z];
      op.zsA = sA[pos(A.legs, z)];
      op.zsB = sB[pos(B.legs, z)];
      op.zsC = sC[pos(out, z)];
    }
    op.conjA = conjA;
    op.conjB = conjB;
    // Hermitian by construction: B is A itself (same data, type and strides) over relabelled legs,
    // conjugated on exactly one side, so element (n, m) is the conjugate of (m, n)
    if (bucket == 1 && zl.empty() && conjA != conjB && A.ref.src == B.ref.src &&
        A.ref.off == B.ref.off && A.ref.dt == B.ref.dt && ml.size() == nl.size() &&
        pick(ml, A.legs, sA) == pick(nl, B.legs, sB) && pick(kl, A.legs, sA) == pick(kl, B.legs, sB)) {
      bool same = true;
      for (size_t i = 0; i < ml.size(); ++i) same = same && legdim[ml[i]] == legdim[nl[i]];
      op.herm = same ? 1 : 0;
    }
    op.akf = !A.legs.empty() && pos(kl, A.legs.back()) >= 0;
    op.bkf = !B.legs.empty() && pos(kl, B.legs.back()) >= 0;
    op.ta = A.ref.dt;
    op.tb = B.ref.dt;
    op.tc = tc;
    op.acc = acc;
    op.alpha = alpha;
    op.adev = adev;
    op.adev2 = adev2;
    // tile chosen at launch (it depends on the batch); a split reduction needs scratch, so it is
    // decided here, for one instance
    op.tile = GEMM_AUTO;
    if (op.zb > 1) {
      op.kcap = 1;   // the element-wise leg fills the grid's third dimension: no split
    } else {
      const bool f64 = acc == DT_C128;
      const int t1 = gemm_pick_tile(op.M, op.N, op.K, 1, f64);
      int ks = gemm_pick_ksplit(op.M, op.N, op.K, 1, t1);
      // FP64-accumulated Grams with a long reduction are bound by the latency of each workgroup's
      // k-steps even when their tiles fill the GPU: four chunks (measured on MI355X, 1024 x 1024 x
      // 4096 from FP32 operands: 854 -> 696 us)
      if (bucket == 1 && f64 && ks == 1 && op.K >= 2048) ks = 4;
      int kcap = ks;
      // the autotuner also tries splits of up to TUNE_KS chunks where the output is small
      const int64_t tiles32 = (int64_t)((op.M + 31) / 32) * ((op.N + 31) / 32);
      if (P.tune && tiles32 < 512 && op.K >= 32) kcap = std::max(kcap, TUNE_KS);
      if (ks > 1) {
        op.tile = t1;
        op.ksplit = ks;
      }
      op.kcap = kcap;
      if (kcap > 1) op.part = scr((size_t)kcap * op.M * op.N * (f64 ? 16 : 8), acc);
    }
    const double f = 8.0 * (double)op.M * op.N * op.K * op.zb;
    op.cls = bucket == 0 ? CBC_K_CONTRACT : bucket == 1 ? CBC_K_GRAM : bucket == 2 ? CBC_K_QRMUL
                                                                              : CBC_K_OTHER;
    // a Hermitian Gram counts half its complex MACs as algorithmic work; layout copies count none
    op.flops = bucket == 1 ? 0.5 * f : bucket == 3 ? 0.0 : f;
    op.bytes = ((double)esz(op.ta) * op.M * op.K + (double)esz(op.tb) * op.K * op.N +
                (double)esz(tc) * op.M * op.N) * op.zb;
    if (bucket == 0) P.cflops += f;
    else if (bucket == 1) P.gflops += 0.5 * f;
    else if (bucket == 2) P.gflops += f;
    P.ops.push_back(op);
    Ten r;
    r.ref = Cref;
    r.ref.dt = tc;
    r.legs = out;
    return r;
  }

  // ---- problem-level legs ----
  std::vector<int> sig, sigp, ealpha, ebeta;  // per node; edge legs indexed by child node
  int rootA = -1, rootB = -1;
  std::vector<int> slot_alpha(int i) const {
    std::vector<int> v{pr.parent[i] >= 0 ? ealpha[i] : rootA};
    for (int c : pr.ch[i]) v.push_back(ealpha[c]);
    return v;
  }
  std::vector<int> slot_beta(int i) const {
    std::vector<int> v{pr.parent[i] >= 0 ? ebeta[i] : rootB};
    for (int c : pr.ch[i]) v.push_back(ebeta[c]);
    return v;
  }
  TRef node_ref(int src, int i) const {
    TRef r;
    r.src = src;
    r.off = i;
    r.dt = ct;
    return r;
  }

  // Contract X with every tensor of `rem`, one at a time: each step takes the tensor whose product
  // with the running result has the fewest elements (ties: the order of `rem`). A leg of both
  // operands is summed unless `out` or a tensor still to come has it, in which case it stays as the
  // step's element-wise leg. `front`, where an intermediate has it, is moved to its first position
  // (an element-wise leg then advances every operand by whole blocks).
  Ten chain(Ten X, std::vector<Ten> rem, const std::vector<int>& out, const TRef& dst,
            int front = -1) {
    while (rem.size() > 1) {
      size_t best = 0;
      int64_t best_e = -1;
      std::vector<int> best_legs;
      for (size_t c = 0; c < rem.size(); ++c) {
        auto needed = [&](int l) {
          if (pos(out, l) >= 0) return true;
          for (size_t o = 0; o < rem.size(); ++o)
            if (o != c && pos(rem[o].legs, l) >= 0) return true;
          return false;
        };
        std::vector<int> o;
        for (int l : X.legs)
          if (pos(rem[c].legs, l) < 0 || needed(l)) o.push_back(l);
        for (int l : rem[c].legs)
          if (pos(X.legs, l) < 0) o.push_back(l);
        const int fp = front >= 0 ? pos(o, front) : -1;
        if (fp > 0) {
          o.erase(o.begin() + fp);
          o.insert(o.begin(), front);
        }
        const int64_t e = elems(o);
        if (best_e < 0 || e < best_e) {
          best = c;
          best_e = e;
          best_legs = o;
        }
      }
      Ten Xn = alloc(best_legs, ct, false);
      X = contract(X, X.cj, rem[best], rem[best].cj, best_legs, Xn.ref, ct, cacc, 0);
      rem.erase(rem.begin() + (ptrdiff_t)best);
    }
    return contract(X, X.cj, rem[0], rem[0].cj, out, dst, ct, cacc, 0);
  }

  Ten state_node(int i) const {
    Ten T;
    T.ref = node_ref(S_STATE, i);
    T.legs.push_back(sig[i]);
    for (int l : slot_alpha(i)) T.legs.push_back(l);
    return T;
  }
  Ten op_node(int i) const {
    Ten W;
    W.ref = node_ref(S_OP, i);
    W.legs = {sigp[i], sig[i]};
    for (int l : slot_beta(i)) W.legs.push_back(l);
    return W;
  }

  // T_i contracted with the environments (slot -> env tensor [chi, alpha, beta]) and with W_i,
  // through chain(): absorbing every environment before W_i leaves all of a node's operator legs
  // open at once (chi * alpha * D per leg); at nodes with three or more environments W_i is taken
  // earlier, which bounds the largest intermediate.
  Ten node_contract(int i, const std::vector<std::pair<int, Ten>>& envs, const std::vector<int>& out,
                    const TRef& dst) {
    std::vector<Ten> rem;
    for (const auto& se : envs) rem.push_back(se.second);
    rem.push_back(op_node(i));
    return chain(state_node(i), rem, out, dst);
  }

  // X /= ||X||_F in place; the log of the factor to `logslot` if given.
  void normalize(const Ten& X, TRef logslot = TRef()) {
    Op o;
    o.kind = K_NORM;
    o.dst = X.ref;
    o.td = X.ref.dt;
    o.count = elems(X.legs);
    o.logs = logslot;
    o.status.src = S_WS;
    o.status.off = HDR_STATUS;
    o.work = scr(sizeof(double) * NORM_MAX_BLOCKS, DT_C128);
    o.bytes = 3.0 * (double)esz(X.ref.dt) * (double)o.count;
    P.ops.push_back(o);
  }

  // A truncation eigensolve op: its record (node, sweep) and the status word.
  void add_eig(Op& e, int node, int sweep) {
    e.rec_node = node;
    e.rec_sweep = sweep;
    e.rec_index = P.n_rec++;
    e.status.src = S_WS;
    e.status.off = HDR_STATUS;
    if (eig_needs_gate(e.s)) P.has_gate = true;
    P.ops.push_back(e);
  }

  // Truncate the joined leg of Lp (legs: row legs..., a_o, b_o) -> L [chi_new, a_o, b_o] (persistent);
  // the edge from `node` to its parent, in sweep `sweep`.
  Ten truncate(const Ten& Lp, int a_o, int b_o, bool& alias_ok, int node, int sweep) {
    std::vector<int> rows(Lp.legs.begin(), Lp.legs.end() - 2);
    const int64_t m = elems(rows), n = legdim[a_o] * legdim[b_o];
    const int64_t kmax = std::min<int64_t>({(int64_t)max_bond, m, n});
    alias_ok = false;
    if (!tol_on && m <= max_bond && m <= n) {
      // nothing to truncate: L = L' (the joined leg becomes the new leg)
      alias_ok = true;
      const int nl = leg(m);
      Ten L;
      L.ref = Lp.ref;
      L.legs = {nl, a_o, b_o};
      return L;
    }
    const int r = leg(m), c = leg(n), r2 = leg(m), c2 = leg(n);
    Ten M1{Lp.ref, {r, c}}, M2{Lp.ref, {r2, c}}, M3{Lp.ref, {r, c2}};
    const int nl = leg(kmax);
    Ten L = alloc({nl, a_o, b_o}, ct, true);
    const bool mside = m <= n;
    const int s = (int)(mside ? m : n);
    Ten G = alloc(mside ? std::vector<int>{r, r2} : std::vector<int>{c, c2}, DT_C128, false);
    if (mside) contract(M1, false, M2, true, {r, r2}, G.ref, DT_C128, DT_C128, 1);  // M M^H
    else contract(M1, true, M3, false, {c, c2}, G.ref, DT_C128, DT_C128, 1);       // M^H M
    Ten U = alloc({mside ? r : c, nl}, DT_C128, false);
    TRef lam = scr(sizeof(double) * kmax, DT_C128);
    TRef kk = scr(256, DT_C128);
    TRef invs = scr(256, DT_C128);
    TRef work = scr(sizeof(double) * eig_work_doubles(s, (int)kmax), DT_C128);
    Op e;
    e.kind = K_EIG;
    e.G = G.ref;
    e.s = s;
    e.kmax = (int)kmax;
    e.U = U.ref;
    e.lam = lam;
    e.kkeep = kk;
    e.invs = invs;
    e.work = work;
    e.cls = CBC_K_EIG;
    // Householder reduction (16/3 s^3) plus back-transformation of kmax vectors (8 s^2 kmax)
    e.flops = 16.0 / 3.0 * (double)s * s * s + 8.0 * (double)s * s * kmax;
    e.bytes = 16.0 * (double)s * s + 16.0 * (double)s * kmax;
    add_eig(e, node, sweep);
    P.n_eig++;
    P.max_eig = std::max(P.max_eig, s);
    if (!eig_size_supported(s)) P.unsupported = true;
    if (mside) {
      // L = U^H M / sqrt(lambda_0)
      Ten Uv{U.ref, {r, nl}};
      Ten Mv{Lp.ref, {r, a_o, b_o}};
      contract(Uv, true, Mv, false, {nl, a_o, b_o}, L.ref, ct, cacc, 0, 1.0, invs);
    } else {
      Op f;
      f.kind = K_FORM_N;
      f.U = U.ref;
      f.lam = lam;
      f.kkeep = kk;
      f.n = (int)n;
      f.kmax = (int)kmax;
      f.L = L.ref;
      f.td = ct;
      f.cls = CBC_K_OTHER;
      P.ops.push_back(f);
    }
    return L;
  }

  // Top-kmax eigenvectors of a Hermitian FP64 Gram G (s x s, row-major): U (s x kmax) with legs
  // [row legs..., nl] (persistent if asked).
  Ten eig_op(const TRef& G, int s, int kmax, const std::vector<int>& rowlegs, int nl, bool persistent,
             int node, TRef* lam_out = nullptr, TRef* kk_out = nullptr, int sweep = 0) {
    std::vector<int> ul = rowlegs;
    ul.push_back(nl);
    Ten U = alloc(ul, DT_C128, persistent);
    TRef lam = scr(sizeof(double) * kmax, DT_C128);
    TRef kk = scr(256, DT_C128);
    TRef invs = scr(256, DT_C128);
    TRef work = scr(sizeof(double) * eig_work_doubles(s, kmax), DT_C128);
    Op e;
    e.kind = K_EIG;
    e.G = G;
    e.s = s;
    e.kmax = kmax;
    e.U = U.ref;
    e.lam = lam;
    e.kkeep = kk;
    e.invs = invs;
    e.work = work;
    e.cls = CBC_K_EIG;
    e.flops = 16.0 / 3.0 * (double)s * s * s + 8.0 * (double)s * s * kmax;
    e.bytes = 16.0 * (double)s * s + 16.0 * (double)s * kmax;
    add_eig(e, node, sweep);
    P.n_eig++;
    P.max_eig = std::max(P.max_eig, s);
    if (!eig_size_supported(s)) P.unsupported = true;
    if (lam_out) *lam_out = lam;
    if (kk_out) *kk_out = kk;
    return U;
  }

  static std::vector<int> without(const std::vector<int>& v, int x) {
    std::vector<int> r;
    for (int l : v)
      if (l != x) r.push_back(l);
    return r;
  }
  static std::vector<int> replaced(const std::vector<int>& v, int x, int y) {
    std::vector<int> r = v;
    for (int& l : r)
      if (l == x) l = y;
    return r;
  }

  // Orthonormal columns: X with legs (rows..., col somewhere) -> Q with legs (rows..., qcol) spanning
  // the column space of X over `col` (three Cholesky-QR passes, the first shifted; complex128).
  Ten cholqr_cols(const Ten& X, int col, int qcol, bool persistent, bool qcol_first = false) {
    const std::vector<int> rows = without(X.legs, col);
    const int64_t k = legdim[col];
    const int64_t mrows = elems(rows);
    const double u = 1.1102230246251565e-16;
    Ten cur = X;
    int cur_col = col;
    for (int pass = 0; pass < 3; ++pass) {
      const int c2 = leg(k);
      Ten curb{cur.ref, replaced(cur.legs, cur_col, c2)};
      Ten G = alloc({cur_col, c2}, DT_C128, false);
      contract(cur, true, curb, false, {cur_col, c2}, G.ref, DT_C128, DT_C128, 1);
      Ten Ci = alloc({qcol, cur_col}, DT_C128, false);
      Op c;
      c.kind = K_CHOL;
      c.G = G.ref;
      c.s = (int)k;
      c.shift_rel = pass == 0 ? 11.0 * ((double)mrows * k + (double)k * (k + 1)) * u : 0.0;
      c.drop_rel = pass == 0 ? 0.0 : 1e-13;
      c.Cinv = Ci.ref;
      c.ndrop.src = S_WS;
      c.ndrop.off = HDR_NDROP;
      c.status.src = S_WS;
      c.status.off = HDR_STATUS;
      c.cls = CBC_K_CHOL;
      if (k > CHOL_LDS_MAX) c.work = scr(sizeof(double) * chol_work_doubles((int)k), DT_C128);
      c.flops = 8.0 / 3.0 * (double)k * k * k;
      c.bytes = 32.0 * (double)k * k;
      P.ops.push_back(c);
      std::vector<int> qo = rows;
      if (pass == 2 && qcol_first) qo.insert(qo.begin(), qcol);
      else qo.push_back(qcol);
      Ten Q = alloc(qo, DT_C128, persistent && pass == 2);
      contract(cur, false, Ci, true, qo, Q.ref, DT_C128, DT_C128, 2);
      if (pass == 2) return Q;
      const int nc = leg(k);
      std::vector<int> nl = rows;
      nl.push_back(nc);
      cur = Ten{Q.ref, nl};
      cur_col = nc;
    }
    return cur;
  }

  // Q-factor of S [k, rest...] on its first leg: returns Q [k_new, rest...] (scratch, complex128)
  // and the per-node scale slot. k < prod(rest) is required.
  Ten cholqr(const Ten& S, int knew_leg, TRef logslot, TRef scaleslot) {
    const int k = (int)legdim[S.legs[0]];
    std::vector<int> rest(S.legs.begin() + 1, S.legs.end());
    const int64_t ns = elems(rest);
    const int kr = S.legs[0];
    const int kc = leg(k);
    Ten cur = S;
    int cur_row = kr;
    const double u = 1.1102230246251565e-16;
    for (int pass = 0; pass < 3; ++pass) {
      // Gram of the current factor: G[r, r'] = sum cur[r, rest] conj(cur[r', rest])
      std::vector<int> l2{kc};
      for (int l : rest) l2.push_back(l);
      Ten curb{cur.ref, l2};
      Ten G = alloc({cur_row, kc}, DT_C128, false);
      contract(cur, false, curb, true, {cur_row, kc}, G.ref, DT_C128, DT_C128, 1);
      Ten Ci = alloc({knew_leg, cur_row}, DT_C128, false);
      Op c;
      c.kind = K_CHOL;
      c.G = G.ref;
      c.s = k;
      c.shift_rel = pass == 0 ? 11.0 * ((double)ns * k + (double)k * (k + 1)) * u : 0.0;
      c.drop_rel = pass == 0 ? 0.0 : 1e-13;
      c.Cinv = Ci.ref;
      if (pass == 0) {
        c.logs = logslot;
        c.scale = scaleslot;
      }
      c.ndrop.src = S_WS;
      c.ndrop.off = HDR_NDROP;
      c.status.src = S_WS;
      c.status.off = HDR_STATUS;
      c.cls = CBC_K_CHOL;
      if (k > CHOL_LDS_MAX) c.work = scr(sizeof(double) * chol_work_doubles((int)k), DT_C128);
      // Cholesky (4/3 k^3) plus triangular inverse (4/3 k^3), complex
      c.flops = 8.0 / 3.0 * (double)k * k * k;
      c.bytes = 32.0 * (double)k * k;
      P.ops.push_back(c);
      // Q = C^{-1} cur
      std::vector<int> qo{knew_leg};
      for (int l : rest) qo.push_back(l);
      Ten Q = alloc(qo, DT_C128, false);
      contract(Ci, false, cur, false, qo, Q.ref, DT_C128, DT_C128, 2);
      // next pass works on Q with a fresh row leg id
      const int nr = leg(k);
      std::vector<int> ql{nr};
      for (int l : rest) ql.push_back(l);
      cur = Ten{Q.ref, ql};
      cur_row = nr;
      if (pass == 2) return Ten{Q.ref, qo};
    }
    return cur;
  }
};

// Persistent slots every plan starts with: the report header at offset 0 (initialised by the first
// op of every call), the per-node log-scales (zeroed), and in mixed precision the converted inputs.
void plan_prologue(Builder& B, Plan& P, cbc_precision prec, int n) {
  B.persist = Builder::al(sizeof(WsHeader));
  P.logs_off = (int64_t)B.persist;
  B.persist += Builder::al(sizeof(double) * n);
  {
    Op h;
    h.kind = K_HEADER;   // n_rec and rec_off are filled in by plan_epilogue
    h.dst.src = S_WS;
    h.dst.off = 0;
    P.ops.push_back(h);
    Op z;
    z.kind = K_ZERO;
    z.dst.src = S_WS;
    z.dst.off = P.logs_off;
    z.count = (int64_t)(B.persist - P.logs_off);
    P.ops.push_back(z);
  }
  if (prec == CBC_PREC_MIXED) {
    P.state_conv_off = (int64_t)B.persist;
    B.persist += Builder::al(8 * (size_t)P.state_elems);
    P.op_conv_off = (int64_t)B.persist;
    B.persist += Builder::al(8 * (size_t)P.op_elems);
    Op c1;
    c1.kind = K_CONVERT;
    c1.src.src = S_STATE;
    c1.src.off = -1;
    c1.ts = DT_C128;
    c1.dst.src = S_WS;
    c1.dst.off = P.state_conv_off;
    c1.td = DT_C64;
    c1.count = P.state_elems;
    P.ops.push_back(c1);
    Op c2 = c1;
    c2.src.src = S_OP;
    c2.dst.off = P.op_conv_off;
    c2.count = P.op_elems;
    P.ops.push_back(c2);
  }
}

// Truncation records at the end of the persistent region; sizes and per-class totals.
cbc_status plan_epilogue(Builder& B, Plan& P) {
  if (B.bad) return CBC_ESHAPE;
  P.rec_off = (int64_t)B.persist;
  B.persist += Builder::al(sizeof(cbc_trunc_record) * (size_t)P.n_rec);
  for (Op& op : P.ops) {
    if (op.kind == K_HEADER) {
      op.count = P.n_rec;
      op.rest = P.rec_off;
    } else if (op.kind == K_EIG) {
      op.rec.src = S_WS;
      op.rec.off = P.rec_off + (int64_t)sizeof(cbc_trunc_record) * op.rec_index;
    }
  }
  P.persist_bytes = B.persist;
  P.scratch_bytes = B.scratch_max;
  for (const Op& op : P.ops) {
    P.launches[op.cls] += 1;
    P.flops[op.cls] += op.flops;
    P.bytes[op.cls] += op.bytes;
  }
  return CBC_OK;
}

cbc_status build_plan(Plan& P, const Problem& pr, int max_bond, bool tol_on, cbc_precision prec,
                      bool fill_tables) {
  Builder B(P, pr, max_bond, tol_on, prec);
  B.fill_tables = fill_tables;
  const int n = pr.n;
  B.sig.resize(n);
  B.sigp.resize(n);
  B.ealpha.assign(n, -1);
  B.ebeta.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    B.sig[i] = B.leg(pr.phys[i]);
    B.sigp[i] = B.leg(pr.phys[i]);
    if (pr.parent[i] >= 0) {
      B.ealpha[i] = B.leg(pr.chi[i]);
      B.ebeta[i] = B.leg(pr.dop[i]);
    }
  }
  B.rootA = B.leg(1);
  B.rootB = B.leg(1);

  plan_prologue(B, P, prec, n);

  // which sweep-1 environments are consumed
  std::vector<char> need(n, 0);
  {
    std::vector<int> pre(pr.post.rbegin(), pr.post.rend());
    for (int i : pre) {
      const int p = pr.parent[i];
      if (p < 0) continue;
      need[i] = (pr.ch[p].size() >= 2) || (p != pr.root && need[p]);
    }
  }
  std::vector<Ten> Lsub(n), Lpar(n), R(n);
  // sweep 1: leaves -> root
  for (int i : pr.post) {
    if (i == pr.root || !need[i]) continue;
    B.reset_scratch();
    std::vector<std::pair<int, Ten>> envs;
    std::vector<int> out{B.sigp[i]};
    for (size_t j = 0; j < pr.ch[i].size(); ++j) {
      const int c = pr.ch[i][j];
      envs.push_back({1 + (int)j, Lsub[c]});
      out.push_back(Lsub[c].legs[0]);
    }
    out.push_back(B.ealpha[i]);
    out.push_back(B.ebeta[i]);
    const int64_t m = B.elems(std::vector<int>(out.begin(), out.end() - 2));
    const bool alias = !tol_on && m <= max_bond && m <= (int64_t)pr.chi[i] * pr.dop[i];
    Ten Lp = B.alloc(out, B.ct, alias);
    Lp = B.node_contract(i, envs, out, Lp.ref);
    bool al;
    Lsub[i] = B.truncate(Lp, B.ealpha[i], B.ebeta[i], al, i, 1);
  }
  // sweep 2: root -> leaves
  {
    std::vector<int> pre(pr.post.rbegin(), pr.post.rend());
    for (int i : pre) {
      for (size_t kp = 0; kp < pr.ch[i].size(); ++kp) {
        const int k = pr.ch[i][kp];
        B.reset_scratch();
        std::vector<std::pair<int, Ten>> envs;
        std::vector<int> out{B.sigp[i]};
        if (i != pr.root) {
          envs.push_back({0, Lpar[i]});
          out.push_back(Lpar[i].legs[0]);
        }
        for (size_t j = 0; j < pr.ch[i].size(); ++j) {
          if (j == kp) continue;
          const int c = pr.ch[i][j];
          envs.push_back({1 + (int)j, Lsub[c]});
          out.push_back(Lsub[c].legs[0]);
        }
        if (i == pr.root) {
          out.push_back(B.rootA);
          out.push_back(B.rootB);
        }
        out.push_back(B.ealpha[k]);
        out.push_back(B.ebeta[k]);
        const int64_t m = B.elems(std::vector<int>(out.begin(), out.end() - 2));
        const bool alias = !tol_on && m <= max_bond && m <= (int64_t)pr.chi[k] * pr.dop[k];
        Ten Lp = B.alloc(out, B.ct, alias);
        Lp = B.node_contract(i, envs, out, Lp.ref);
        bool al;
        Lpar[k] = B.truncate(Lp, B.ealpha[k], B.ebeta[k], al, k, 2);
      }
    }
  }
  // sweep 3: leaves -> root
  P.out_off.assign(n + 1, 0);
  P.out_bond.assign(n, 1);
  std::vector<int64_t> out_elems(n, 0);
  std::vector<Op> writes;  // output writes are queued in node order at the end of each node
  // output sizes are known only after the children are processed; first compute bonds
  std::vector<int> kout(n, 1);
  for (int i : pr.post) {
    if (i == pr.root) continue;
    int64_t ns = pr.phys[i];
    for (int c : pr.ch[i]) ns *= kout[c];
    const int64_t k = B.legdim[Lpar[i].legs[0]];
    // Without a tolerance the economy QR gives min(k, ns) rows. With one, Q keeps all k rows (those
    // beyond the row space of S are zero), because the kept count is only known on device.
    kout[i] = tol_on ? (int)k : (int)std::min<int64_t>(k, ns);
  }
  // Output slots are sized for the planned environment bond on every edge (the tolerance-mode
  // shape), so the packing is the same with and without a tolerance; a node is written as a prefix
  // of its slot with its actual bonds.
  for (int i = 0; i < n; ++i) {
    const int64_t kcap_i = i == pr.root ? 1 : B.legdim[Lpar[i].legs[0]];
    int64_t e = pr.phys[i] * kcap_i;
    for (int c : pr.ch[i]) e *= B.legdim[Lpar[c].legs[0]];
    P.out_off[i + 1] = P.out_off[i] + e;
    P.out_bond[i] = kout[i];
  }
  std::vector<int> rleg(n, -1);
  for (int i : pr.post) {
    B.reset_scratch();
    std::vector<std::pair<int, Ten>> envs;
    std::vector<int> zl{B.sigp[i]};
    for (size_t j = 0; j < pr.ch[i].size(); ++j) {
      const int c = pr.ch[i][j];
      envs.push_back({1 + (int)j, R[c]});
      zl.push_back(R[c].legs[0]);
    }
    if (i == pr.root) {
      std::vector<int> zr{B.rootA};
      zr.insert(zr.end(), zl.begin(), zl.end());
      zr.push_back(B.rootB);
      Ten Z = B.alloc(zr, B.ct, false);
      Z = B.node_contract(i, envs, zr, Z.ref);
      Op w;
      w.kind = K_WRITE;
      w.src = Z.ref;
      w.ts = B.ct;
      w.a = 1;
      w.b = pr.phys[i];
      w.rest = B.elems(zr) / pr.phys[i];
      w.dst.src = S_OUT;
      w.dst.off = i;
      w.logs.src = S_WS;
      w.logs.off = P.logs_off;
      w.nlogs = n;
      P.ops.push_back(w);
      continue;
    }
    zl.push_back(B.ealpha[i]);
    zl.push_back(B.ebeta[i]);
    int64_t ns = pr.phys[i];
    for (int c : pr.ch[i]) ns *= kout[c];
    const int64_t k = B.legdim[Lpar[i].legs[0]];
    // With a tolerance the kept bond can be smaller than planned, so S may be rank-deficient and Q
    // must span only its row space: the identity shortcut is taken only without one.
    const bool ident = !tol_on && k >= ns;
    Ten Z = B.alloc(zl, B.ct, ident);
    Z = B.node_contract(i, envs, zl, Z.ref);
    std::vector<int> rest(zl.begin(), zl.end() - 2);
    if (ident) {
      // Q is the identity on the joined leg: R^{[i]} = Z with (sigma', chi_c...) as its new leg
      const int nl = B.leg(ns);
      R[i] = Ten{Z.ref, {nl, B.ealpha[i], B.ebeta[i]}};
      TRef q = B.scr(16 * (size_t)ns * ns, DT_C128);
      Op f;
      f.kind = K_IDENT;
      f.dst = q;
      f.td = DT_C128;
      f.a = (int)ns;
      f.b = (int)ns;
      P.ops.push_back(f);
      Op w;
      w.kind = K_WRITE;
      w.src = q;
      w.ts = DT_C128;
      w.a = (int)ns;
      w.b = pr.phys[i];
      w.rest = ns / pr.phys[i];
      w.dst.src = S_OUT;
      w.dst.off = i;
      P.ops.push_back(w);
      continue;
    }
    // S = L^{[(p,i)]} Z  -> [chi_p, sigma', chi_c...]
    std::vector<int> sl{Lpar[i].legs[0]};
    sl.insert(sl.end(), rest.begin(), rest.end());
    Ten S = B.alloc(sl, B.ct, false);
    S = B.contract(Lpar[i], false, Z, false, sl, S.ref, B.ct, B.cacc, 0);
    TRef logslot;
    logslot.src = S_WS;
    logslot.off = P.logs_off + 8 * (int64_t)i;
    TRef scl = B.scr(256, DT_C128);
    const int knew = B.leg(k);
    Ten Q = B.cholqr(S, knew, logslot, scl);
    // R^{[i]} = scale * sum conj(Q) Z
    Ten Rt = B.alloc({knew, B.ealpha[i], B.ebeta[i]}, B.ct, true);
    R[i] = B.contract(Q, true, Z, false, {knew, B.ealpha[i], B.ebeta[i]}, Rt.ref, B.ct, B.cacc, 0,
                      1.0, scl);
    Op w;
    w.kind = K_WRITE;
    w.src = Q.ref;
    w.ts = DT_C128;
    w.a = (int)k;
    w.b = pr.phys[i];
    w.rest = ns / pr.phys[i];
    w.dst.src = S_OUT;
    w.dst.off = i;
    P.ops.push_back(w);
  }
  return plan_epilogue(B, P);
}

// ------------------------------------------------------------------------------------------------
// successive randomised compression (Sec. III C, the randomised counterpart of CBC): the truncated
// environments of sweeps 1 and 2 become exact Khatri-Rao sketches of the subtree below a node (K) and
// of the rest of the tree (E), and sweep 3 takes each node's basis from a Cholesky-QR of the sketched
// columns Y = Z E instead of a QR on the parent leg. Sketches and environments are normalised after
// every node step (only column spaces matter for the sketches; the environments' logs rescale the
// root output).

cbc_status build_plan_src(Plan& P, const Problem& pr, int max_bond, cbc_precision prec,
                          bool fill_tables) {
  Builder B(P, pr, max_bond, false, prec);
  B.fill_tables = fill_tables;
  const int n = pr.n;
  B.sig.resize(n);
  B.sigp.resize(n);
  B.ealpha.assign(n, -1);
  B.ebeta.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    B.sig[i] = B.leg(pr.phys[i]);
    B.sigp[i] = B.leg(pr.phys[i]);
    if (pr.parent[i] >= 0) {
      B.ealpha[i] = B.leg(pr.chi[i]);
      B.ebeta[i] = B.leg(pr.dop[i]);
    }
  }
  B.rootA = B.leg(1);
  B.rootB = B.leg(1);
  const int rl = B.leg(max_bond);   // the sketch index, shared by every node (Khatri-Rao product)
  plan_prologue(B, P, prec, n);
  P.sketch_elems = 0;
  for (int i = 0; i < n; ++i) P.sketch_elems += (int64_t)pr.phys[i] * max_bond;
  if (prec == CBC_PREC_MIXED) {
    P.sketch_conv_off = (int64_t)B.persist;
    B.persist += Builder::al(8 * (size_t)P.sketch_elems);
    Op c;
    c.kind = K_CONVERT;
    c.src.src = S_SKETCH;
    c.src.off = -1;
    c.ts = DT_C128;
    c.dst.src = S_WS;
    c.dst.off = P.sketch_conv_off;
    c.td = DT_C64;
    c.count = P.sketch_elems;
    P.ops.push_back(c);
  }
  auto sketch_of = [&](int i) {
    Ten O;
    O.ref = B.node_ref(S_SKETCH, i);
    O.legs = {B.sigp[i], rl};
    return O;
  };
  // output bonds: node i keeps min(rows, max_bond) with rows = sigma'_i x its children's bonds
  std::vector<int> kout(n, 1);
  std::vector<int64_t> rows(n, 1);
  for (int i : pr.post) {
    rows[i] = pr.phys[i];
    for (int c : pr.ch[i]) rows[i] *= kout[c];
    if (i != pr.root) kout[i] = (int)std::min<int64_t>(rows[i], max_bond);
  }
  // sketches needed: E at every compressed node and at the non-root ancestors its E is built from;
  // K of the siblings along the way, and of everything below them
  std::vector<char> needE(n, 0), needK(n, 0);
  for (int i = 0; i < n; ++i) {
    if (i == pr.root || rows[i] <= max_bond) continue;
    for (int q = i; q != pr.root && !needE[q]; q = pr.parent[q]) needE[q] = 1;
  }
  std::function<void(int)> mark = [&](int c) {
    if (needK[c]) return;
    needK[c] = 1;
    for (int cc : pr.ch[c]) mark(cc);
  };
  for (int k = 0; k < n; ++k) {
    if (!needE[k]) continue;
    for (int c : pr.ch[pr.parent[k]])
      if (c != k) mark(c);
  }
  std::vector<Ten> K(n), E(n), R(n);
  // sweep 1, leaves to root: subtree sketches K^{[i]} [r, alpha_i, beta_i]
  for (int i : pr.post) {
    if (!needK[i]) continue;
    B.reset_scratch();
    std::vector<Ten> rem;
    for (int c : pr.ch[i]) rem.push_back(K[c]);
    rem.push_back(B.op_node(i));
    rem.push_back(sketch_of(i));
    const std::vector<int> out{rl, B.ealpha[i], B.ebeta[i]};
    Ten Kt = B.alloc(out, B.ct, true);
    K[i] = B.chain(B.state_node(i), rem, out, Kt.ref, rl);
    B.normalize(K[i]);
  }
  // sweep 2, root to leaves: sketches of the rest of the tree E^{[k]} [r, alpha_k, beta_k]
  {
    std::vector<int> pre(pr.post.rbegin(), pr.post.rend());
    for (int i : pre) {
      for (int k : pr.ch[i]) {
        if (!needE[k]) continue;
        B.reset_scratch();
        std::vector<Ten> rem;
        if (i != pr.root) rem.push_back(E[i]);
        for (int c : pr.ch[i])
          if (c != k) rem.push_back(K[c]);
        rem.push_back(B.op_node(i));
        rem.push_back(sketch_of(i));
        std::vector<int> out{rl};
        if (i == pr.root) {   // the root's trivial parent legs stay on the result (dimension 1)
          out.push_back(B.rootA);
          out.push_back(B.rootB);
        }
        out.push_back(B.ealpha[k]);
        out.push_back(B.ebeta[k]);
        Ten Et = B.alloc(out, B.ct, true);
        Et = B.chain(B.state_node(i), rem, out, Et.ref, rl);
        E[k] = Ten{Et.ref, {rl, B.ealpha[k], B.ebeta[k]}};
        B.normalize(E[k]);
      }
    }
  }
  // sweep 3, leaves to root: Z^{[i]}, bases from Y = Z E, environments R = Q^H Z
  P.out_off.assign(n + 1, 0);
  P.out_bond.assign(n, 1);
  for (int i = 0; i < n; ++i) {
    int64_t e = (int64_t)pr.phys[i] * kout[i];
    for (int c : pr.ch[i]) e *= kout[c];
    P.out_off[i + 1] = P.out_off[i] + e;
    P.out_bond[i] = kout[i];
  }
  for (int i : pr.post) {
    B.reset_scratch();
    std::vector<std::pair<int, Ten>> envs;
    std::vector<int> zl{B.sigp[i]};
    for (size_t j = 0; j < pr.ch[i].size(); ++j) {
      const int c = pr.ch[i][j];
      envs.push_back({1 + (int)j, R[c]});
      zl.push_back(R[c].legs[0]);
    }
    if (i == pr.root) {
      std::vector<int> zr{B.rootA};
      zr.insert(zr.end(), zl.begin(), zl.end());
      zr.push_back(B.rootB);
      Ten Z = B.alloc(zr, B.ct, false);
      Z = B.node_contract(i, envs, zr, Z.ref);
      Op w;
      w.kind = K_WRITE;
      w.src = Z.ref;
      w.ts = B.ct;
      w.a = 1;
      w.b = pr.phys[i];
      w.rest = B.elems(zr) / pr.phys[i];
      w.dst.src = S_OUT;
      w.dst.off = i;
      w.logs.src = S_WS;
      w.logs.off = P.logs_off;
      w.nlogs = n;
      P.ops.push_back(w);
      continue;
    }
    zl.push_back(B.ealpha[i]);
    zl.push_back(B.ebeta[i]);
    const int64_t ns = rows[i];
    std::vector<int> rest(zl.begin(), zl.end() - 2);
    const bool ident = ns <= max_bond;
    Ten Z = B.alloc(zl, B.ct, ident);
    Z = B.node_contract(i, envs, zl, Z.ref);
    if (ident) {
      // nothing to compress: the basis is the identity and R^{[i]} = Z with (sigma', chi_c...) as
      // its new leg
      const int nl = B.leg(ns);
      R[i] = Ten{Z.ref, {nl, B.ealpha[i], B.ebeta[i]}};
      TRef q = B.scr(16 * (size_t)ns * ns, DT_C128);
      Op f;
      f.kind = K_IDENT;
      f.dst = q;
      f.td = DT_C128;
      f.a = (int)ns;
      f.b = (int)ns;
      P.ops.push_back(f);
      Op w;
      w.kind = K_WRITE;
      w.src = q;
      w.ts = DT_C128;
      w.a = (int)ns;
      w.b = pr.phys[i];
      w.rest = ns / pr.phys[i];
      w.dst.src = S_OUT;
      w.dst.off = i;
      P.ops.push_back(w);
      continue;
    }
    // Y = Z E^{[i]} [sigma', chi_c..., r]
    std::vector<int> yl = rest;
    yl.push_back(rl);
    Ten Y = B.alloc(yl, B.ct, false);
    Y = B.contract(Z, false, E[i], false, yl, Y.ref, B.ct, B.cacc, 0);
    const int knew = B.leg(max_bond);
    Ten Q = B.cholqr_cols(Y, rl, knew, false, true);        // [k, sigma', chi_c...], complex128
    Ten Rt = B.alloc({knew, B.ealpha[i], B.ebeta[i]}, B.ct, true);
    R[i] = B.contract(Q, true, Z, false, {knew, B.ealpha[i], B.ebeta[i]}, Rt.ref, B.ct, B.cacc, 0);
    TRef logslot;
    logslot.src = S_WS;
    logslot.off = P.logs_off + 8 * (int64_t)i;
    B.normalize(R[i], logslot);
    Op w;
    w.kind = K_WRITE;
    w.src = Q.ref;
    w.ts = DT_C128;
    w.a = max_bond;
    w.b = pr.phys[i];
    w.rest = ns / pr.phys[i];
    w.dst.src = S_OUT;
    w.dst.off = i;
    P.ops.push_back(w);
  }
  return plan_epilogue(B, P);
}

// Sweep 3 of the density-matrix and Zip-Up methods (as in CBC, Eqs. cbc_tree_third_contraction,
// cbc_final_contraction): Z^{[i]} = T W prod_c R^{[c]}, leaves to root; a node whose rows exceed its
// new bond takes its basis from the top eigenvectors of rho = Z B Z^H (density-matrix method, B the
// exact environment of the rest of the tree) or rho = Z Z^H (Zip-Up, no environment: the node's own
// product with its compressed children), FP64 through the truncation eigensolver; R^{[i]} = Q^H Z
// carries its normalisation in the node's log slot; the root writes Z.
static void sweep3_density(Builder& B, Plan& P, const Problem& pr, const std::vector<int>& kout,
                           const std::vector<int64_t>& rows, const std::vector<Ten>* env,
                           const std::vector<int>& ealphap, const std::vector<int>& ebetap,
                           int rec_sweep) {
  const int n = pr.n;
  std::vector<Ten> R(n);
  P.out_off.assign(n + 1, 0);
  P.out_bond.assign(n, 1);
  for (int i = 0; i < n; ++i) {
    int64_t e = (int64_t)pr.phys[i] * kout[i];
    for (int c : pr.ch[i]) e *= kout[c];
    P.out_off[i + 1] = P.out_off[i] + e;
    P.out_bond[i] = kout[i];
  }
  TRef one = B.wsp(256, DT_C128);
  {
    Op f;
    f.kind = K_IDENT;
    f.dst = one;
    f.td = DT_C128;
    f.a = 1;
    f.b = 1;
    P.ops.push_back(f);
  }
  for (int i : pr.post) {
    B.reset_scratch();
    std::vector<std::pair<int, Ten>> envs;
    std::vector<int> zl{B.sigp[i]};
    for (size_t j = 0; j < pr.ch[i].size(); ++j) {
      const int c = pr.ch[i][j];
      envs.push_back({1 + (int)j, R[c]});
      zl.push_back(R[c].legs[0]);
    }
    if (i == pr.root) {
      std::vector<int> zr{B.rootA};
      zr.insert(zr.end(), zl.begin(), zl.end());
      zr.push_back(B.rootB);
      Ten Z = B.alloc(zr, B.ct, false);
      Z = B.node_contract(i, envs, zr, Z.ref);
      Op w;
      w.kind = K_WRITE;
      w.src = Z.ref;
      w.ts = B.ct;
      w.a = 1;
      w.b = pr.phys[i];
      w.rest = B.elems(zr) / pr.phys[i];
      w.dst.src = S_OUT;
      w.dst.off = i;
      w.logs.src = S_WS;
      w.logs.off = P.logs_off;
      w.nlogs = n;
      P.ops.push_back(w);
      continue;
    }
    zl.push_back(B.ealpha[i]);
    zl.push_back(B.ebeta[i]);
    const int64_t ns = rows[i];
    std::vector<int> rest(zl.begin(), zl.end() - 2);
    const bool ident = ns <= kout[i];
    Ten Z = B.alloc(zl, B.ct, ident);
    Z = B.node_contract(i, envs, zl, Z.ref);
    if (ident) {
      const int nl = B.leg(ns);
      R[i] = Ten{Z.ref, {nl, B.ealpha[i], B.ebeta[i]}};
      TRef q = B.scr(16 * (size_t)ns * ns, DT_C128);
      Op f;
      f.kind = K_IDENT;
      f.dst = q;
      f.td = DT_C128;
      f.a = (int)ns;
      f.b = (int)ns;
      P.ops.push_back(f);
      Op w;
      w.kind = K_WRITE;
      w.src = q;
      w.ts = DT_C128;
      w.a = (int)ns;
      w.b = pr.phys[i];
      w.rest = ns / pr.phys[i];
      w.dst.src = S_OUT;
      w.dst.off = i;
      P.ops.push_back(w);
      continue;
    }
    std::vector<int> rowsp;
    for (int l : rest) rowsp.push_back(B.leg(B.legdim[l]));
    std::vector<int> rl = rest;
    rl.insert(rl.end(), rowsp.begin(), rowsp.end());
    Ten rho = B.alloc(rl, DT_C128, false);
    if (env) {
      // X = Z B over the parent bond's ket legs: [rows..., beta'_i, alpha'_i]
      std::vector<int> xl = rest;
      xl.push_back(ebetap[i]);
      xl.push_back(ealphap[i]);
      Ten X = B.alloc(xl, B.ct, false);
      X = B.contract(Z, false, (*env)[i], false, xl, X.ref, B.ct, B.cacc, 0);
      // rho = X conj(Z') over the bra legs, in FP64: [rows..., rows'...]
      std::vector<int> zbl = rowsp;
      zbl.push_back(ealphap[i]);
      zbl.push_back(ebetap[i]);
      B.contract(X, false, Ten{Z.ref, zbl, true}, true, rl, rho.ref, DT_C128, DT_C128, 1);
    } else {
      // rho = Z conj(Z') over the parent bond (alpha_i, beta_i), in FP64: [rows..., rows'...]
      std::vector<int> zbl = rowsp;
      zbl.push_back(B.ealpha[i]);
      zbl.push_back(B.ebeta[i]);
      B.contract(Z, false, Ten{Z.ref, zbl, true}, true, rl, rho.ref, DT_C128, DT_C128, 1);
    }
    const int kev = B.leg(kout[i]);
    Ten Ue = B.eig_op(rho.ref, (int)ns, kout[i], rest, kev, false, i, nullptr, nullptr, rec_sweep);
    // The kept eigenvectors of a rank-deficient rho (a bond whose rank is below the target) include
    // vectors of its zero eigenvalue, which the eigensolver need not return orthonormal; a
    // Cholesky-QR of the columns makes the basis a (partial) isometry with the same span, so the
    // weight-carrying directions and the state are unchanged.
    const int knew = B.leg(kout[i]);
    Ten U = B.cholqr_cols(Ue, kev, knew, false);
    Ten Rt = B.alloc({knew, B.ealpha[i], B.ebeta[i]}, B.ct, true);
    R[i] = B.contract(U, true, Z, false, {knew, B.ealpha[i], B.ebeta[i]}, Rt.ref, B.ct, B.cacc, 0);
    TRef logslot;
    logslot.src = S_WS;
    logslot.off = P.logs_off + 8 * (int64_t)i;
    B.normalize(R[i], logslot);
    // output node [sigma', k, chi_c...] from U [sigma', chi_c..., k] (a layout copy)
    std::vector<int> ol{B.sigp[i], knew};
    ol.insert(ol.end(), rest.begin() + 1, rest.end());
    TRef dst;
    dst.src = S_OUT;
    dst.off = i;
    dst.dt = DT_C128;
    B.contract(U, false, Ten{one, {}}, false, ol, dst, DT_C128, DT_C128, 3);
  }
}

// ------------------------------------------------------------------------------------------------
// density-matrix compression (the method CBC is built from, Sec. III): sweeps 1 and 2 contract the
// exact environments of <Phi|Phi>, Phi = O|psi> (legs: ket state, ket operator, bra operator, bra
// state), and sweep 3 takes each node's basis from the top eigenvectors of its reduced density
// matrix rho = Z B Z^H. The environments are normalised after every node step (a positive factor
// does not change an eigenvector); R carries its factor in the node's log slot as in CBC.

cbc_status build_plan_dm(Plan& P, const Problem& pr, int max_bond, cbc_precision prec,
                         bool fill_tables) {
  Builder B(P, pr, max_bond, false, prec);
  B.fill_tables = fill_tables;
  const int n = pr.n;
  B.sig.resize(n);
  B.sigp.resize(n);
  B.ealpha.assign(n, -1);
  B.ebeta.assign(n, -1);
  std::vector<int> sigpp(n), ealphap(n, -1), ebetap(n, -1);
  for (int i = 0; i < n; ++i) {
    B.sig[i] = B.leg(pr.phys[i]);
    B.sigp[i] = B.leg(pr.phys[i]);
    sigpp[i] = B.leg(pr.phys[i]);
    if (pr.parent[i] >= 0) {
      B.ealpha[i] = B.leg(pr.chi[i]);
      B.ebeta[i] = B.leg(pr.dop[i]);
      ealphap[i] = B.leg(pr.chi[i]);
      ebetap[i] = B.leg(pr.dop[i]);
    }
  }
  B.rootA = B.leg(1);
  B.rootB = B.leg(1);
  const int rootAp = B.leg(1), rootBp = B.leg(1);
  plan_prologue(B, P, prec, n);
  // the bra copies: conj(W_i) [sigma', sigma'', beta'...] and conj(T_i) [sigma'', alpha'...]
  auto op_bra = [&](int i) {
    Ten W = B.op_node(i);
    W.legs = {B.sigp[i], sigpp[i], pr.parent[i] >= 0 ? ebetap[i] : rootBp};
    for (int c : pr.ch[i]) W.legs.push_back(ebetap[c]);
    W.cj = true;
    return W;
  };
  auto state_bra = [&](int i) {
    Ten T = B.state_node(i);
    T.legs = {sigpp[i], pr.parent[i] >= 0 ? ealphap[i] : rootAp};
    for (int c : pr.ch[i]) T.legs.push_back(ealphap[c]);
    T.cj = true;
    return T;
  };
  std::vector<int> kout(n, 1);
  std::vector<int64_t> rows(n, 1);
  for (int i : pr.post) {
    rows[i] = pr.phys[i];
    for (int c : pr.ch[i]) rows[i] *= kout[c];
    if (i != pr.root) kout[i] = (int)std::min<int64_t>(rows[i], max_bond);
  }
  // environments needed: B at every truncated node and the non-root ancestors it is built from; A
  // of the siblings along the way and of everything below them
  std::vector<char> needB(n, 0), needA(n, 0);
  for (int i = 0; i < n; ++i) {
    if (i == pr.root || rows[i] <= max_bond) continue;
    for (int q = i; q != pr.root && !needB[q]; q = pr.parent[q]) needB[q] = 1;
  }
  std::function<void(int)> mark = [&](int c) {
    if (needA[c]) return;
    needA[c] = 1;
    for (int cc : pr.ch[c]) mark(cc);
  };
  for (int k = 0; k < n; ++k) {
    if (!needB[k]) continue;
    for (int c : pr.ch[pr.parent[k]])
      if (c != k) mark(c);
  }
  std::vector<Ten> A(n), Bv(n);
  // sweep 1, leaves to root: A^{[i]} [alpha_i, beta_i, beta'_i, alpha'_i]
  for (int i : pr.post) {
    if (!needA[i]) continue;
    B.reset_scratch();
    std::vector<Ten> rem;
    for (int c : pr.ch[i]) rem.push_back(A[c]);
    rem.push_back(B.op_node(i));
    rem.push_back(op_bra(i));
    rem.push_back(state_bra(i));
    const std::vector<int> out{B.ealpha[i], B.ebeta[i], ebetap[i], ealphap[i]};
    Ten At = B.alloc(out, B.ct, true);
    A[i] = B.chain(B.state_node(i), rem, out, At.ref);
    B.normalize(A[i]);
  }
  // sweep 2, root to leaves: B^{[k]} [alpha_k, beta_k, beta'_k, alpha'_k]
  {
    std::vector<int> pre(pr.post.rbegin(), pr.post.rend());
    for (int i : pre) {
      for (int k : pr.ch[i]) {
        if (!needB[k]) continue;
        B.reset_scratch();
        std::vector<Ten> rem;
        if (i != pr.root) rem.push_back(Bv[i]);
        for (int c : pr.ch[i])
          if (c != k) rem.push_back(A[c]);
        rem.push_back(B.op_node(i));
        rem.push_back(op_bra(i));
        rem.push_back(state_bra(i));
        std::vector<int> out;
        if (i == pr.root) {   // the root's trivial parent legs stay on the result (dimension 1)
          out = {B.rootA, B.rootB, rootBp, rootAp};
        }
        out.push_back(B.ealpha[k]);
        out.push_back(B.ebeta[k]);
        out.push_back(ebetap[k]);
        out.push_back(ealphap[k]);
        Ten Bt = B.alloc(out, B.ct, true);
        Bt = B.chain(B.state_node(i), rem, out, Bt.ref);
        Bv[k] = Ten{Bt.ref, {B.ealpha[k], B.ebeta[k], ebetap[k], ealphap[k]}};
        B.normalize(Bv[k]);
      }
    }
  }
  sweep3_density(B, P, pr, kout, rows, &Bv, ealphap, ebetap, 3);
  return plan_epilogue(B, P);
}

// ------------------------------------------------------------------------------------------------
// Zip-Up (Sec. III C): one sweep, leaves to root, each node compressed on the spot from its own
// product with the already compressed children: sweep 3 of the density-matrix method with no
// environment, the basis from the top eigenvectors of Z Z^H (the left singular vectors of Z's
// unfolding (sigma', children's bonds) x (alpha_p, beta_p)).

cbc_status build_plan_zipup(Plan& P, const Problem& pr, int max_bond, cbc_precision prec,
                            bool fill_tables) {
  Builder B(P, pr, max_bond, false, prec);
  B.fill_tables = fill_tables;
  const int n = pr.n;
  B.sig.resize(n);
  B.sigp.resize(n);
  B.ealpha.assign(n, -1);
  B.ebeta.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    B.sig[i] = B.leg(pr.phys[i]);
    B.sigp[i] = B.leg(pr.phys[i]);
    if (pr.parent[i] >= 0) {
      B.ealpha[i] = B.leg(pr.chi[i]);
      B.ebeta[i] = B.leg(pr.dop[i]);
    }
  }
  B.rootA = B.leg(1);
  B.rootB = B.leg(1);
  plan_prologue(B, P, prec, n);
  std::vector<int> kout(n, 1);
  std::vector<int64_t> rows(n, 1);
  for (int i : pr.post) {
    rows[i] = pr.phys[i];
    for (int c : pr.ch[i]) rows[i] *= kout[c];
    if (i != pr.root) kout[i] = (int)std::min<int64_t>(rows[i], max_bond);
  }
  sweep3_density(B, P, pr, kout, rows, nullptr, {}, {}, 4);
  return plan_epilogue(B, P);
}

// ------------------------------------------------------------------------------------------------
// the naive (direct) method of Sec. III C: exact product, canonical form, truncated-SVD sweep

cbc_status build_plan_naive(Plan& P, const Problem& pr, int max_bond, bool tol_on,
                            cbc_precision prec, bool fill_tables) {
  Builder B(P, pr, max_bond, tol_on, prec);
  B.fill_tables = fill_tables;
  const int n = pr.n;
  B.sig.resize(n);
  B.sigp.resize(n);
  B.ealpha.assign(n, -1);
  B.ebeta.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    B.sig[i] = B.leg(pr.phys[i]);
    B.sigp[i] = B.leg(pr.phys[i]);
    if (pr.parent[i] >= 0) {
      B.ealpha[i] = B.leg(pr.chi[i]);
      B.ebeta[i] = B.leg(pr.dop[i]);
    }
  }
  B.rootA = B.leg(1);
  B.rootB = B.leg(1);
  plan_prologue(B, P, prec, n);
  const DType ct = B.ct;

  // fused product bonds, one leg per edge (the root's trivial leg included)
  std::vector<int> edge(n);
  for (int i = 0; i < n; ++i)
    edge[i] = B.leg(pr.parent[i] >= 0 ? (int64_t)pr.chi[i] * pr.dop[i] : 1);
  // 1. product node tensors P_i[sigma', (a_p b_p), (a_c b_c)...] = sum_sigma W T
  std::vector<Ten> node(n);
  for (int i = 0; i < n; ++i) {
    B.reset_scratch();
    const auto sa = B.slot_alpha(i), sb = B.slot_beta(i);
    Ten T{B.node_ref(S_STATE, i), {B.sig[i]}};
    for (int l : sa) T.legs.push_back(l);
    Ten W{B.node_ref(S_OP, i), {B.sigp[i], B.sig[i]}};
    for (int l : sb) W.legs.push_back(l);
    std::vector<int> out{B.sigp[i]};
    for (size_t j = 0; j < sa.size(); ++j) {
      out.push_back(sa[j]);
      out.push_back(sb[j]);
    }
    Ten X = B.alloc(out, ct, true);
    B.contract(T, false, W, false, out, X.ref, ct, B.cacc, 0);
    std::vector<int> fused{B.sigp[i], edge[i]};
    for (int c : pr.ch[i]) fused.push_back(edge[c]);
    node[i] = Ten{X.ref, fused};
  }
  // Economy QR of node `ch` on its bond `col` to node `par`, R absorbed by `par`; returns the new bond
  // leg (dimension min(rest, dim col) as in an economy QR).
  TRef one = B.wsp(256, DT_C128);
  {
    Op f;
    f.kind = K_IDENT;
    f.dst = one;
    f.td = DT_C128;
    f.a = 1;
    f.b = 1;
    P.ops.push_back(f);
  }
  auto qr_toward = [&](int ch, int par, int col) -> int {
    const std::vector<int> rows = Builder::without(node[ch].legs, col);
    const int64_t rest = B.elems(rows), pd = B.legdim[col];
    if (rest <= pd) {
      // Q = identity on the joined leg, R = the node itself: the parent absorbs the node and the
      // node's remaining legs become the (fused) bond
      const int nl = B.leg(rest);
      std::vector<int> il = rows;
      il.push_back(nl);
      Ten I = B.alloc(il, DT_C128, true);
      Op f;
      f.kind = K_IDENT;
      f.dst = I.ref;
      f.td = DT_C128;
      f.a = (int)rest;
      f.b = (int)rest;
      P.ops.push_back(f);
      std::vector<int> pl, pv;
      for (int l : node[par].legs) {
        if (l == col) {
          pl.insert(pl.end(), rows.begin(), rows.end());
          pv.push_back(nl);
        } else {
          pl.push_back(l);
          pv.push_back(l);
        }
      }
      Ten Pn = B.alloc(pl, ct, true);
      B.contract(node[par], false, node[ch], false, pl, Pn.ref, ct, B.cacc, 0);
      node[par] = Ten{Pn.ref, pv};
      node[ch] = Ten{I.ref, il};
      return nl;
    }
    const int nl = B.leg(pd);
    Ten Q = B.cholqr_cols(node[ch], col, nl, true);
    Ten R = B.alloc({nl, col}, DT_C128, false);
    B.contract(Q, true, node[ch], false, {nl, col}, R.ref, DT_C128, DT_C128, 0);
    const auto pl = Builder::replaced(node[par].legs, col, nl);
    Ten Pn = B.alloc(pl, ct, true);
    B.contract(node[par], false, R, false, pl, Pn.ref, ct, B.cacc, 0);
    node[par] = Pn;
    node[ch] = Q;
    return nl;
  };
  // 2. canonical form toward the root
  for (int i : pr.post) {
    if (i == pr.root) continue;
    B.reset_scratch();
    edge[i] = qr_toward(i, pr.parent[i], edge[i]);
  }
  // 3. truncated-SVD sweep, depth first from the root, moving the orthogonality centre
  std::function<void(int)> visit = [&](int i) {
    for (int c : pr.ch[i]) {
      B.reset_scratch();
      const Ten M = node[i];
      const int col = edge[c];
      const std::vector<int> rows = Builder::without(M.legs, col);
      const int64_t m = B.elems(rows), nn = B.legdim[col];
      const int kmax = (int)std::min<int64_t>({(int64_t)max_bond, m, nn});
      int K = B.leg(kmax);
      Ten U;
      if (m <= nn) {
        std::vector<int> rows2;
        for (int l : rows) rows2.push_back(B.leg(B.legdim[l]));
        Ten M2{M.ref, M.legs};
        for (size_t j = 0; j < rows.size(); ++j) M2.legs = Builder::replaced(M2.legs, rows[j], rows2[j]);
        std::vector<int> gl = rows;
        gl.insert(gl.end(), rows2.begin(), rows2.end());
        Ten G = B.alloc(gl, DT_C128, false);
        B.contract(M, false, M2, true, gl, G.ref, DT_C128, DT_C128, 1);
        U = B.eig_op(G.ref, (int)m, kmax, rows, K, true, c);
      } else {
        const int col2 = B.leg(nn);
        Ten M2{M.ref, Builder::replaced(M.legs, col, col2)};
        Ten G = B.alloc({col, col2}, DT_C128, false);
        B.contract(M, true, M2, false, {col, col2}, G.ref, DT_C128, DT_C128, 1);
        Ten V = B.eig_op(G.ref, (int)nn, kmax, {col}, K, false, c);
        std::vector<int> wl = rows;
        wl.push_back(K);
        Ten Wt = B.alloc(wl, DT_C128, false);
        B.contract(M, false, V, false, wl, Wt.ref, DT_C128, DT_C128, 0);
        const int K2 = B.leg(kmax);
        U = B.cholqr_cols(Wt, K, K2, true);
        K = K2;
      }
      // the child absorbs U^H M on the truncated bond
      Ten Y = B.alloc({K, col}, DT_C128, false);
      B.contract(U, true, M, false, {K, col}, Y.ref, DT_C128, DT_C128, 0);
      const auto cl = Builder::replaced(node[c].legs, col, K);
      Ten Cn = B.alloc(cl, ct, true);
      B.contract(Y, false, node[c], false, cl, Cn.ref, ct, B.cacc, 0);
      node[i] = U;
      node[c] = Cn;
      edge[c] = K;
      visit(c);
      // move the centre back: child = Q R on its parent bond, R absorbed by node i
      B.reset_scratch();
      edge[c] = qr_toward(c, i, edge[c]);
    }
  };
  visit(pr.root);
  // 4. outputs in the (sigma', parent, children...) layout, complex128
  P.out_off.assign(n + 1, 0);
  P.out_bond.assign(n, 1);
  for (int i = 0; i < n; ++i) {
    int64_t e = pr.phys[i] * B.legdim[edge[i]];
    for (int c : pr.ch[i]) e *= B.legdim[edge[c]];
    P.out_off[i + 1] = P.out_off[i] + e;
    P.out_bond[i] = (int)B.legdim[edge[i]];
  }
  for (int i = 0; i < n; ++i) {
    B.reset_scratch();
    std::vector<int> ol{B.sigp[i], edge[i]};
    for (int c : pr.ch[i]) ol.push_back(edge[c]);
    TRef dst;
    dst.src = S_OUT;
    dst.off = i;
    dst.dt = DT_C128;
    B.contract(node[i], false, Ten{one, {}}, false, ol, dst, DT_C128, DT_C128, 3);
  }
  return plan_epilogue(B, P);
}

// ------------------------------------------------------------------------------------------------
// context and execution

struct Call {
  char* ws;
  const char* state;
  const char* op;
  char* out;
  const int64_t* st_off;
  const int64_t* op_off;
  const int64_t* out_off;
  size_t persist;
  // batch: instance b uses every buffer advanced by b times its per-instance byte stride
  int batch = 1;
  int64_t ws_inst = 0, st_inst = 0, op_inst = 0, out_inst = 0;
  bool caller_capture = false;   // recorded into a stream capture of the caller's (or a call of
                                 // cbc_apply_noalloc): eigensolves take the two-stage reduction
  const int32_t* tables = nullptr;   // device copy of the plan's offset tables
  char* scr = nullptr;   // scratch given apart from the workspace (cbc_apply_split), else null
  const char* sketch = nullptr;        // the randomised method's sketch matrices (cbc_apply_src)
  const int64_t* sk_off = nullptr;
};

}  // namespace

struct cbc_ctx {
  std::map<std::vector<int64_t>, std::unique_ptr<Plan>> plans;
  int device = -1;
  // autotuning: contraction configuration (tile, split) per GEMM key, and the cache file
  bool tune = false;
  std::string tune_path;
  std::map<std::vector<int64_t>, std::pair<int, int>> tuned;
  // streams of cbc_apply_many (default priority) with the events that fork and join them
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> join_ev;
  hipEvent_t fork_ev = nullptr;
  ~cbc_ctx() {
    plans.clear();   // a plan waits for its graphs' last launches before it goes
    for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
  }
};

namespace {

void* resolve(const Plan& P, const Call& c, const TRef& r) {
  switch (r.src) {
    case S_WS: return c.ws + r.off;
    case S_SCR: return (c.scr ? c.scr : c.ws + c.persist) + r.off;
    case S_STATE:
      if (r.off < 0) return (void*)c.state;
      if (P.state_conv_off >= 0) return c.ws + P.state_conv_off + 8 * c.st_off[r.off];
      return (void*)(c.state + 16 * c.st_off[r.off]);
    case S_OP:
      if (r.off < 0) return (void*)c.op;
      if (P.op_conv_off >= 0) return c.ws + P.op_conv_off + 8 * c.op_off[r.off];
      return (void*)(c.op + 16 * c.op_off[r.off]);
    case S_OUT: return c.out + 16 * c.out_off[r.off];
    case S_SKETCH:
      if (r.off < 0) return (void*)c.sketch;
      if (P.sketch_conv_off >= 0) return c.ws + P.sketch_conv_off + 8 * c.sk_off[r.off];
      return (void*)(c.sketch + 16 * c.sk_off[r.off]);
    default: return nullptr;
  }
}

int64_t stride_of(const Plan& P, const Call& c, const TRef& r) {
  switch (r.src) {
    case S_WS:
    case S_SCR: return c.ws_inst;
    case S_STATE: return (r.off >= 0 && P.state_conv_off >= 0) ? c.ws_inst : c.st_inst;
    case S_OP: return (r.off >= 0 && P.op_conv_off >= 0) ? c.ws_inst : c.op_inst;
    case S_OUT: return c.out_inst;
    case S_SKETCH: return (r.off >= 0 && P.sketch_conv_off >= 0) ? c.ws_inst : 0;
    default: return 0;
  }
}

// Tile and split of a contraction for the call's batch: the autotuner's choice, or the fixed policy
// (the split planned for one instance is reduced when the batch already fills the GPU; without a
// split the tile is chosen at launch for the batch).
std::pair<int, int> gemm_config(const Op& op, int batch) {
  if (op.zb > 1) batch = op.zb;
  if (op.tuned || batch == 1 || op.ksplit == 1) return {op.tile, op.ksplit};
  const int ks = std::min(op.ksplit, gemm_pick_ksplit(op.M, op.N, op.K, batch, op.tile));
  return {ks > 1 ? op.tile : GEMM_AUTO, ks};
}

GemmArgs gemm_args(const Plan& P, const Call& c, const Op& op, int ksplit) {
  GemmArgs g;
  g.A = resolve(P, c, op.A);
  g.B = resolve(P, c, op.B);
  g.C = resolve(P, c, op.C);
  g.M = op.M;
  g.N = op.N;
  g.K = op.K;
  g.offAm = c.tables + op.tAm;
  g.offAk = c.tables + op.tAk;
  g.offBk = c.tables + op.tBk;
  g.offBn = c.tables + op.tBn;
  g.offCm = c.tables + op.tCm;
  g.offCn = c.tables + op.tCn;
  g.conjA = op.conjA;
  g.conjB = op.conjB;
  g.herm = op.herm;
  g.a_kfast = op.akf;
  g.b_kfast = op.bkf;
  g.alpha_dev = op.adev.src == S_NONE ? nullptr : (const double*)resolve(P, c, op.adev);
  g.alpha_dev2 = op.adev2.src == S_NONE ? nullptr : (const double*)resolve(P, c, op.adev2);
  g.alpha = op.alpha;
  g.batch = c.batch;
  g.bsA = stride_of(P, c, op.A);
  g.bsB = stride_of(P, c, op.B);
  g.bsC = stride_of(P, c, op.C);
  g.bsAlpha = stride_of(P, c, op.adev);
  g.bsAlpha2 = stride_of(P, c, op.adev2);
  if (op.zb > 1) {
    // the element-wise leg takes the grid's batch dimension (plans holding one run single calls)
    auto es = [](DType t) { return (int64_t)(t == DT_C128 ? 16 : 8); };
    g.batch = op.zb;
    g.bsA = op.zsA * es(op.ta);
    g.bsB = op.zsB * es(op.tb);
    g.bsC = op.zsC * es(op.tc);
    g.bsAlpha = 0;
    g.bsAlpha2 = 0;
  }
  g.mbase = 0;
  g.ksplit = ksplit;
  g.kchunk = ((op.K + ksplit - 1) / ksplit + 15) / 16 * 16;
  g.part = ksplit > 1 ? resolve(P, c, op.part) : nullptr;
  g.bsPart = ksplit > 1 ? stride_of(P, c, op.part) : 0;
  return g;
}

hipError_t run_ops(const Plan& P, const Call& c, hipStream_t st, hipEvent_t* ev = nullptr) {
  size_t idx = 0;
  for (const Op& op : P.ops) {
    hipError_t e = hipSuccess;
    if (ev) {
      e = hipEventRecord(ev[2 * idx], st);
      if (e != hipSuccess) return e;
    }
    switch (op.kind) {
      case K_GEMM: {
        const auto cf = gemm_config(op, c.batch);
        e = launch_gemm(gemm_args(P, c, op, cf.second), op.ta, op.tb, op.tc, op.acc, cf.first, st);
        break;
      }
      case K_EIG: {
        EigArgs a;
        a.G = (double2*)resolve(P, c, op.G);
        a.s = op.s;
        a.kmax = op.kmax;
        a.tol = 0.0;
        a.U = (double2*)resolve(P, c, op.U);
        a.lam = (double*)resolve(P, c, op.lam);
        a.kkeep = (int*)resolve(P, c, op.kkeep);
        a.inv_sqrt_l0 = (double*)resolve(P, c, op.invs);
        a.work = (double*)resolve(P, c, op.work);
        a.tol = op.shift_rel;  // tolerance stored per call below
        a.tstamp = nullptr;
        a.batch = c.batch;
        a.bs = c.ws_inst;
        a.status = (int*)resolve(P, c, op.status);
        a.rec = (cbc_trunc_record*)resolve(P, c, op.rec);
        a.rec_node = op.rec_node;
        a.rec_sweep = op.rec_sweep;
        a.reduction = eig_pick_reduction(op.s, c.batch, c.caller_capture);
        e = launch_eig(a, st);
        break;
      }
      case K_FORM_N:
        e = launch_form_l_nside((const double2*)resolve(P, c, op.U), (const double*)resolve(P, c, op.lam),
                                (const int*)resolve(P, c, op.kkeep), op.n, op.kmax,
                                resolve(P, c, op.L), op.td, c.batch, c.ws_inst, st);
        break;
      case K_CHOL: {
        CholArgs a;
        a.G = (double2*)resolve(P, c, op.G);
        a.k = op.s;
        a.shift_rel = op.shift_rel;
        a.drop_rel = op.drop_rel;
        a.Cinv = (double2*)resolve(P, c, op.Cinv);
        a.log_scale = op.logs.src == S_NONE ? nullptr : (double*)resolve(P, c, op.logs);
        a.scale = op.scale.src == S_NONE ? nullptr : (double*)resolve(P, c, op.scale);
        a.ndrop = (int*)resolve(P, c, op.ndrop);
        a.tstamp = nullptr;
        a.batch = c.batch;
        a.bs = c.ws_inst;
        a.work = op.work.src == S_NONE ? nullptr : (double2*)resolve(P, c, op.work);
        a.status = (int*)resolve(P, c, op.status);
        e = launch_chol_inv(a, st);
        break;
      }
      case K_CONVERT:
        e = launch_convert(resolve(P, c, op.src), op.ts, resolve(P, c, op.dst), op.td, op.count,
                           c.batch, stride_of(P, c, op.src), stride_of(P, c, op.dst), st);
        break;
      case K_IDENT:
        e = launch_fill_identity(resolve(P, c, op.dst), op.td, op.a, op.b, c.batch,
                                 stride_of(P, c, op.dst), st);
        break;
      case K_WRITE:
        e = launch_write_out(resolve(P, c, op.src), op.ts, op.a, op.b, op.rest,
                             (double2*)resolve(P, c, op.dst),
                             op.logs.src == S_NONE ? nullptr : (const double*)resolve(P, c, op.logs),
                             op.nlogs, c.batch, stride_of(P, c, op.src), stride_of(P, c, op.dst),
                             stride_of(P, c, op.logs), st);
        break;
      case K_ZERO:
        e = launch_zero(resolve(P, c, op.dst), op.count, c.batch, stride_of(P, c, op.dst), st);
        break;
      case K_NORM:   // single calls only (plans of the randomised method)
        e = launch_normalize(resolve(P, c, op.dst), op.td, op.count, (double*)resolve(P, c, op.work),
                             op.scale.src == S_NONE ? nullptr : (double*)resolve(P, c, op.scale),
                             op.logs.src == S_NONE ? nullptr : (double*)resolve(P, c, op.logs),
                             (int*)resolve(P, c, op.status), st);
        break;
      case K_HEADER:
        e = launch_report_header(resolve(P, c, op.dst), REPORT_MAGIC, (int)op.count, op.rest,
                                 (int64_t)sizeof(cbc_trunc_record), c.batch,
                                 stride_of(P, c, op.dst), st);
        break;
    }
    if (e != hipSuccess) return e;
    if (ev) {
      e = hipEventRecord(ev[2 * idx + 1], st);
      if (e != hipSuccess) return e;
    }
    ++idx;
  }
  return hipSuccess;
}

std::vector<int64_t> plan_key(const Problem& pr, int max_bond, bool tol_on, cbc_precision prec,
                              int method, int64_t se, int64_t oe) {
  std::vector<int64_t> k{pr.n, max_bond, tol_on, (int64_t)prec, method, se, oe};
  for (int i = 0; i < pr.n; ++i) {
    k.push_back(pr.parent[i]);
    k.push_back(pr.phys[i]);
    k.push_back(pr.chi[i]);
    k.push_back(pr.dop[i]);
  }
  return k;
}

int64_t tensor_elems_state(const Problem& pr, int i) {
  int64_t e = (int64_t)pr.phys[i] * pr.chi[i];
  for (int c : pr.ch[i]) e *= pr.chi[c];
  return e;
}
int64_t tensor_elems_op(const Problem& pr, int i) {
  int64_t e = (int64_t)pr.phys[i] * pr.phys[i] * pr.dop[i];
  for (int c : pr.ch[i]) e *= pr.dop[c];
  return e;
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

// ---- autotuner -------------------------------------------------------------------------------
std::vector<int64_t> tune_key(const Op& op, int batch) {
  return {(int64_t)op.ta, (int64_t)op.tb, (int64_t)op.tc, (int64_t)op.acc, op.M, op.N, op.K,
          batch, op.akf, op.bkf};
}

// Feasible (tile, split) configurations of a contraction: the three tile kernels (the pipelined one
// accumulates in FP32 only), and splits of the reduction into 2, 4 or 8 chunks of at least 16 for
// the kernels that take them, within the scratch the plan reserved.
std::vector<std::pair<int, int>> tune_candidates(const Op& op, int batch) {
  std::vector<std::pair<int, int>> cand;
  const bool f64 = op.acc == DT_C128;
  for (int tile : {GEMM_TILE32, GEMM_TILE64, GEMM_PIPE64, GEMM_PIPE128}) {
    if ((tile == GEMM_PIPE64 || tile == GEMM_PIPE128) && f64) continue;
    if (tile == GEMM_PIPE128 && (op.M < 128 || op.N < 128)) continue;
    for (int ks = 1; ks <= TUNE_KS; ks *= 2) {
      if (ks > 1 && (tile == GEMM_TILE64 || ks > op.kcap)) continue;
      const int kchunk = ((op.K + ks - 1) / ks + 15) / 16 * 16;
      if (ks > 1 && (int64_t)kchunk * (ks - 1) >= op.K) continue;   // an empty chunk
      if ((int64_t)batch * ks > 65535) continue;
      cand.emplace_back(tile, ks);
    }
  }
  return cand;
}

hipError_t tune_plan(cbc_ctx* ctx, Plan& P, const Call& c, hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::FILE* f = nullptr;
  if (e == hipSuccess && !ctx->tune_path.empty()) f = std::fopen(ctx->tune_path.c_str(), "a");
  constexpr int reps = 3;
  for (Op& op : P.ops) {
    if (e != hipSuccess) break;
    if (op.kind != K_GEMM) continue;
    const int eb = op.zb > 1 ? op.zb : c.batch;
    const auto key = tune_key(op, eb);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end() && it->second.second <= op.kcap) {
      op.tile = it->second.first;
      op.ksplit = it->second.second;
      op.tuned = true;
      continue;
    }
    std::pair<int, int> best{op.tile, op.ksplit};
    float best_ms = 0.0f;
    bool have = false;
    for (const auto& cf : tune_candidates(op, eb)) {
      op.tile = cf.first;
      op.ksplit = cf.second;
      // one launch to warm up, then the timed ones; results are recomputed by the call afterwards
      const GemmArgs g = gemm_args(P, c, op, op.ksplit);
      hipError_t r = launch_gemm(g, op.ta, op.tb, op.tc, op.acc, op.tile, st);
      if (r == hipSuccess) r = hipEventRecord(e0, st);
      for (int i = 0; i < reps && r == hipSuccess; ++i) r = launch_gemm(g, op.ta, op.tb, op.tc, op.acc, op.tile, st);
      if (r == hipSuccess) r = hipEventRecord(e1, st);
      if (r == hipSuccess) r = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
      if (r != hipSuccess) {
        e = r;
        break;
      }
      if (!have || ms < best_ms) {
        best = cf;
        best_ms = ms;
        have = true;
      }
    }
    op.tile = best.first;
    op.ksplit = best.second;
    if (e != hipSuccess) break;
    op.tuned = true;
    ctx->tuned[key] = best;
    if (f) {
      std::fprintf(f, "cbc-gemm");
      for (int64_t v : key) std::fprintf(f, " %lld", (long long)v);
      std::fprintf(f, " %d %d %.6f\n", best.first, best.second, best_ms / reps);
    }
  }
  if (f) std::fclose(f);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

// The context's plan for a problem. need_tables: the plan will run, so its offset tables are built
// (a plan cached by a query has sizes only and is rebuilt here). Host allocation failures while
// planning are reported as CBC_ENOMEM.
cbc_status get_plan(cbc_ctx* ctx, const Problem& pr, int max_bond, bool tol_on, cbc_precision prec,
                    int method, int64_t state_span, int64_t op_span, Plan** out,
                    bool need_tables) {
  auto key = plan_key(pr, max_bond, tol_on, prec, method, state_span, op_span);
  key.push_back(ctx->tune ? 1 : 0);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end() && (!need_tables || it->second->has_tables)) {
    *out = it->second.get();
    return CBC_OK;
  }
  try {
    auto P = std::make_unique<Plan>();
    P->state_elems = state_span;
    P->op_elems = op_span;
    P->tune = ctx->tune;
    cbc_status s = method == 0   ? build_plan(*P, pr, max_bond, tol_on, prec, need_tables)
                   : method == 1 ? build_plan_naive(*P, pr, max_bond, tol_on, prec, need_tables)
                   : method == 2 ? build_plan_src(*P, pr, max_bond, prec, need_tables)
                   : method == 3 ? build_plan_dm(*P, pr, max_bond, prec, need_tables)
                                 : build_plan_zipup(*P, pr, max_bond, prec, need_tables);
    if (s != CBC_OK) return s;
    if (P->unsupported) return CBC_EUNSUP;
    P->has_tables = need_tables;
    *out = P.get();
    ctx->plans[key] = std::move(P);
  } catch (const std::bad_alloc&) {
    return CBC_ENOMEM;
  } catch (const std::length_error&) {
    return CBC_ENOMEM;
  }
  return CBC_OK;
}

// Device copy of the plan's offset tables; the host copy is released once it is made.
cbc_status upload_tables(Plan* P) {
  if (P->d_tables || P->tables.empty()) return CBC_OK;
  if (hipMalloc(&P->d_tables, P->tables.size() * sizeof(int32_t)) != hipSuccess) return CBC_ENOMEM;
  if (hipMemcpy(P->d_tables, P->tables.data(), P->tables.size() * sizeof(int32_t),
                hipMemcpyHostToDevice) != hipSuccess)
    return CBC_EHIP;
  std::vector<int32_t>().swap(P->tables);
  return CBC_OK;
}

}  // namespace

extern "C" {

cbc_status cbc_create(cbc_ctx** ctx) {
  if (!ctx) return CBC_EINVAL;
  try {
    *ctx = new cbc_ctx();
  } catch (...) {
    return CBC_ENOMEM;
  }
  return CBC_OK;
}

void cbc_destroy(cbc_ctx* ctx) { delete ctx; }

cbc_status cbc_autotune(cbc_ctx* ctx, const char* cache_path) {
  if (!ctx) return CBC_EINVAL;
  ctx->tune = true;
  if (!cache_path || !cache_path[0]) return CBC_OK;
  ctx->tune_path = cache_path;
  std::FILE* f = std::fopen(cache_path, "r");
  if (!f) {
    // a new cache: create it now, so that an unwritable path is reported here
    f = std::fopen(cache_path, "a");
    if (!f) return CBC_EINVAL;
    std::fclose(f);
    return CBC_OK;
  }
  // lines "cbc-gemm ta tb tc acc M N K batch akf bkf tile ksplit ms"; anything else is skipped
  char tag[16];
  while (std::fscanf(f, "%15s", tag) == 1) {
    long long v[10];
    int tile = 0, ks = 0;
    double ms = 0.0;
    bool ok = std::strcmp(tag, "cbc-gemm") == 0;
    for (int i = 0; ok && i < 10; ++i) ok = std::fscanf(f, "%lld", &v[i]) == 1;
    ok = ok && std::fscanf(f, "%d %d %lf", &tile, &ks, &ms) == 3;
    ok = ok && (tile == GEMM_TILE32 || tile == GEMM_TILE64 || tile == GEMM_PIPE64 ||
                tile == GEMM_PIPE128) &&
         (ks == 1 || ks == 2 || ks == 4 || ks == 8);
    if (ok) ctx->tuned[std::vector<int64_t>(v, v + 10)] = {tile, ks};
    int ch;
    while ((ch = std::fgetc(f)) != EOF && ch != '\n') {
    }
  }
  std::fclose(f);
  return CBC_OK;
}

const char* cbc_status_str(cbc_status s) {
  switch (s) {
    case CBC_OK: return "ok";
    case CBC_EINVAL: return "invalid argument (null pointer, max_bond < 1, bad tol or precision)";
    case CBC_ESHAPE: return "invalid tree or dimensions";
    case CBC_ENOMEM: return "workspace too small or allocation failed";
    case CBC_EHIP: return "HIP runtime error";
    case CBC_ENOTPD: return "factorisation failed after fallbacks";
    case CBC_EUNSUP:
      return "unsupported configuration (an eigensolve beyond the solver's size limit, or a tensor "
             "of 2^31 or more elements)";
    case CBC_ENOTBUILT: return "no usable gfx950 device";
    case CBC_ETIMEOUT: return "a bounded wait between cooperating workgroups expired on the device";
  }
  return "unknown status";
}

static cbc_status common_checks(const cbc_tree* tree, int32_t max_bond, cbc_precision prec,
                                Problem& pr) {
  if (max_bond < 1) return CBC_EINVAL;
  if (prec != CBC_PREC_FP64 && prec != CBC_PREC_MIXED) return CBC_EINVAL;
  return validate_tree(tree, pr);
}

cbc_status cbc_query(cbc_ctx* ctx, const cbc_tree* tree, int32_t max_bond, cbc_precision prec,
                     int32_t method, size_t* workspace_bytes, int64_t* out_offset) {
  if (!ctx || !workspace_bytes || !out_offset) return CBC_EINVAL;
  if (method < 0 || method > 4) return CBC_EINVAL;
  if (method == 2 && max_bond > 65535) return CBC_EUNSUP;
  Problem pr;
  cbc_status s = common_checks(tree, max_bond, prec, pr);
  if (s != CBC_OK) return s;
  int64_t se = 0, oe = 0;
  for (int i = 0; i < pr.n; ++i) {
    se += tensor_elems_state(pr, i);
    oe += tensor_elems_op(pr, i);
  }
  Plan* P = nullptr;
  // the workspace does not depend on tol; plan with tolerance off and on, report the larger
  size_t ws = 0;
  for (int t = 0; t < 2; ++t) {
    s = get_plan(ctx, pr, max_bond, t == 1, prec, method, se, oe, &P, false);
    if (s != CBC_OK) return s;
    ws = std::max(ws, P->persist_bytes + P->scratch_bytes);
  }
  *workspace_bytes = ws;
  for (int i = 0; i <= pr.n; ++i) out_offset[i] = P->out_off[i];
  return CBC_OK;
}

cbc_status cbc_plan_info(cbc_ctx* ctx, const cbc_tree* tree, int32_t max_bond, cbc_precision prec,
                         int32_t method, int32_t tol_on, cbc_plan_summary* info) {
  if (!ctx || !info) return CBC_EINVAL;
  if (method < 0 || method > 4) return CBC_EINVAL;
  if (method == 2 && max_bond > 65535) return CBC_EUNSUP;
  Problem pr;
  cbc_status s = common_checks(tree, max_bond, prec, pr);
  if (s != CBC_OK) return s;
  int64_t se = 0, oe = 0;
  for (int i = 0; i < pr.n; ++i) {
    se += tensor_elems_state(pr, i);
    oe += tensor_elems_op(pr, i);
  }
  Plan* P = nullptr;
  s = get_plan(ctx, pr, max_bond, tol_on != 0, prec, method, se, oe, &P, false);
  if (s != CBC_OK) return s;
  info->persistent_bytes = P->persist_bytes;
  info->scratch_bytes = P->scratch_bytes;
  info->table_bytes = (size_t)P->table_entries * sizeof(int32_t);
  for (int k = 0; k < CBC_K_NCLASS; ++k) {
    info->launches[k] = P->launches[k];
    info->flops[k] = P->flops[k];
  }
  return CBC_OK;
}

cbc_status cbc_plan_bonds(cbc_ctx* ctx, const cbc_tree* tree, int32_t max_bond, int32_t tol_on,
                          int32_t* bond) {
  if (!ctx || !bond) return CBC_EINVAL;
  Problem pr;
  cbc_status s = common_checks(tree, max_bond, CBC_PREC_FP64, pr);
  if (s != CBC_OK) return s;
  int64_t se = 0, oe = 0;
  for (int i = 0; i < pr.n; ++i) {
    se += tensor_elems_state(pr, i);
    oe += tensor_elems_op(pr, i);
  }
  Plan* P = nullptr;
  s = get_plan(ctx, pr, max_bond, tol_on != 0, CBC_PREC_FP64, 0, se, oe, &P, false);
  if (s != CBC_OK) return s;
  for (int i = 0; i < pr.n; ++i) bond[i] = P->out_bond[i];
  return CBC_OK;
}

static cbc_status apply_impl(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                             const cbc_tree* tree, int32_t max_bond, double tol,
                             cbc_precision prec, void* workspace, size_t workspace_bytes,
                             cbc_out* out, void* stream, cbc_stats* stats, int method,
                             int32_t batch = 1, bool noalloc = false, void* scratch = nullptr,
                             size_t scratch_bytes = 0, const cbc_tensors* sketch = nullptr) {
  if (batch < 1 || batch > 65535) return CBC_EINVAL;
  if (method == 2 && (!sketch || !sketch->data || !sketch->offset || batch != 1 || noalloc ||
                      scratch || tol != 0.0))
    return CBC_EINVAL;
  if (method >= 3 && (batch != 1 || noalloc || scratch || tol != 0.0)) return CBC_EINVAL;
  if (noalloc && (batch != 1 || (stats && stats->profile))) return CBC_EINVAL;
  const bool split = scratch != nullptr;
  if (split && (batch != 1 || noalloc)) return CBC_EINVAL;
  if (!ctx || !ttno || !ttns || !out || !ttno->data || !ttns->data || !ttno->offset ||
      !ttns->offset || !out->data || !out->offset || !out->bond)
    return CBC_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return CBC_EINVAL;
  Problem pr;
  cbc_status s = common_checks(tree, max_bond, prec, pr);
  if (s != CBC_OK) return s;
  // inputs must be packed: every node inside [0, total) where total is the sum of node sizes
  int64_t se = 0, oe = 0;
  for (int i = 0; i < pr.n; ++i) {
    se += tensor_elems_state(pr, i);
    oe += tensor_elems_op(pr, i);
  }
  for (int i = 0; i < pr.n; ++i) {
    if (ttns->offset[i] < 0 || ttno->offset[i] < 0) return CBC_EINVAL;
    if (ttns->offset[i] + tensor_elems_state(pr, i) > se) return CBC_EINVAL;
    if (ttno->offset[i] + tensor_elems_op(pr, i) > oe) return CBC_EINVAL;
  }
  if (method == 2) {
    if (max_bond > 65535) return CBC_EUNSUP;
    int64_t ke = 0;
    for (int i = 0; i < pr.n; ++i) ke += (int64_t)pr.phys[i] * max_bond;
    for (int i = 0; i < pr.n; ++i)
      if (sketch->offset[i] < 0 || sketch->offset[i] + (int64_t)pr.phys[i] * max_bond > ke)
        return CBC_EINVAL;
  }
  Plan* P = nullptr;
  s = get_plan(ctx, pr, max_bond, tol > 0.0, prec, method, se, oe, &P, true);
  if (s != CBC_OK) return s;
  const size_t ws_inst = P->persist_bytes + P->scratch_bytes;
  const int32_t* tables = nullptr;
  hipStream_t st = (hipStream_t)stream;
  if (noalloc) {
    // the plan's offset tables, then the workspace, in the static scratch array of this device
    const size_t tbytes = ((size_t)P->table_entries * sizeof(int32_t) + 255) & ~(size_t)255;
    if (tbytes + ws_inst > NOALLOC_SCRATCH_BYTES) return CBC_EUNSUP;
    void* base = nullptr;
    if (noalloc_scratch(&base) != hipSuccess) return CBC_EHIP;
    workspace = (char*)base + tbytes;
    workspace_bytes = ws_inst;
    tables = (const int32_t*)base;
  }
  if (split) {
    if (!workspace || workspace_bytes < P->persist_bytes || scratch_bytes < P->scratch_bytes)
      return CBC_ENOMEM;
  } else if (!workspace || workspace_bytes / (size_t)batch < ws_inst) {
    return CBC_ENOMEM;
  }
  for (int i = 0; i <= pr.n; ++i)
    if (out->offset[i] != P->out_off[i]) return CBC_EINVAL;
  if (noalloc) {
    // from the host copy, or device to device once a cbc_apply call has moved them there
    const size_t tb = (size_t)P->table_entries * sizeof(int32_t);
    if (tb > 0) {
      const hipError_t e =
          P->tables.empty()
              ? hipMemcpyAsync((void*)tables, P->d_tables, tb, hipMemcpyDeviceToDevice, st)
              : hipMemcpyAsync((void*)tables, P->tables.data(), tb, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return CBC_EHIP;
    }
  } else {
    s = upload_tables(P);
    if (s != CBC_OK) return s;
    tables = P->d_tables;
  }
  // tolerance is a per-call value carried by the eigensolve ops
  for (auto& op : P->ops)
    if (op.kind == K_EIG) op.shift_rel = tol;
  Call c;
  c.ws = (char*)workspace;
  c.state = (const char*)ttns->data;
  c.op = (const char*)ttno->data;
  c.out = (char*)out->data;
  c.st_off = ttns->offset;
  c.op_off = ttno->offset;
  c.out_off = P->out_off.data();
  c.persist = P->persist_bytes;
  c.batch = batch;
  c.ws_inst = (int64_t)ws_inst;
  c.st_inst = 16 * se;
  c.op_inst = 16 * oe;
  c.out_inst = 16 * P->out_off[pr.n];
  c.tables = tables;
  c.scr = (char*)scratch;
  if (method == 2) {
    c.sketch = (const char*)sketch->data;
    c.sk_off = sketch->offset;
  }
  const bool profile = stats && stats->profile;
  int replayed = 0;
  if (!noalloc && P->tune && ctx->tune && P->tuned_batch != batch &&
      !(st != nullptr && capturing(st))) {
    // the contractions' configurations change: a captured graph of the old ones is dropped
    if (tune_plan(ctx, *P, c, st) != hipSuccess) return CBC_EHIP;
    P->tuned_batch = batch;
    P->drop_graphs();
  }
  if (noalloc) {
    // no graph, no tuning, no events and no device-wide gate: the kernels go straight onto the
    // stream, eigensolves through the two-stage reduction
    c.caller_capture = true;
    if (run_ops(*P, c, st) != hipSuccess) return CBC_EHIP;
  } else if (profile) {
    const size_t ne = 2 * P->ops.size();
    while (P->events.size() < ne) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) return CBC_EHIP;
      P->events.push_back(ev);
    }
    if (run_ops(*P, c, st, P->events.data()) != hipSuccess) return CBC_EHIP;
  } else if (st != nullptr && capturing(st)) {
    // the caller is capturing this stream into a graph of its own: record the kernels into it
    c.caller_capture = true;
    if (run_ops(*P, c, st) != hipSuccess) return CBC_EHIP;
  } else if (st != nullptr) {
    // replay a captured graph of the whole launch sequence when the buffers are unchanged
    std::vector<uintptr_t> key{(uintptr_t)c.ws, (uintptr_t)c.state, (uintptr_t)c.op,
                               (uintptr_t)c.out, (uintptr_t)batch, (uintptr_t)c.scr};
    uint64_t tb;
    memcpy(&tb, &tol, sizeof(tb));
    key.push_back((uintptr_t)tb);
    for (int i = 0; i < pr.n; ++i) {
      key.push_back((uintptr_t)c.st_off[i]);
      key.push_back((uintptr_t)c.op_off[i]);
    }
    if (c.sketch) {
      key.push_back((uintptr_t)c.sketch);
      for (int i = 0; i < pr.n; ++i) key.push_back((uintptr_t)c.sk_off[i]);
    }
    auto it = P->graphs.find(key);
    if (it == P->graphs.end()) {
      if (P->graphs.size() >= Plan::MAX_GRAPHS) {
        auto lru = P->graphs.begin();
        for (auto g2 = P->graphs.begin(); g2 != P->graphs.end(); ++g2)
          if (g2->second.used < lru->second.used) lru = g2;
        P->drop_graph(lru);
      }
      Plan::Exec ex;
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return CBC_EHIP;
      const hipError_t e1 = run_ops(*P, c, st);
      const hipError_t e2 = hipStreamEndCapture(st, &g);
      if (e1 != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return CBC_EHIP;
      }
      const hipError_t e3 = hipGraphInstantiate(&ex.exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e3 != hipSuccess) return CBC_EHIP;
      if (hipEventCreateWithFlags(&ex.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGraphExecDestroy(ex.exec);
        return CBC_EHIP;
      }
      it = P->graphs.emplace(key, ex).first;
    } else {
      replayed = 1;
    }
    it->second.used = ++P->graph_clock;
    // a graph holding a multi-workgroup eigensolve runs after the previous one on the device
    if (P->has_gate && mw_gate_enter(st) != hipSuccess) return CBC_EHIP;
    if (hipGraphLaunch(it->second.exec, st) != hipSuccess) return CBC_EHIP;
    if (P->has_gate && mw_gate_leave(st) != hipSuccess) return CBC_EHIP;
    if (hipEventRecord(it->second.done, st) != hipSuccess) return CBC_EHIP;
  } else {
    if (run_ops(*P, c, st) != hipSuccess) return CBC_EHIP;
  }
  // Shapes are static, so the bonds are known here; only the profiling mode waits for the device.
  if (profile && hipStreamSynchronize(st) != hipSuccess) return CBC_EHIP;
  for (int i = 0; i < pr.n; ++i) out->bond[i] = P->out_bond[i];
  if (stats) {
    stats->n_kernels = (int32_t)P->ops.size();
    stats->n_eig = P->n_eig;
    stats->max_eig_dim = P->max_eig;
    stats->graph_replayed = replayed;
    for (int k = 0; k < CBC_K_NCLASS; ++k) {
      stats->launches[k] = P->launches[k];
      stats->flops[k] = P->flops[k];
      stats->bytes[k] = P->bytes[k];
      stats->ms[k] = 0.0;
    }
    if (profile) {
      for (size_t i = 0; i < P->ops.size(); ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, P->events[2 * i], P->events[2 * i + 1]) != hipSuccess)
          return CBC_EHIP;
        stats->ms[P->ops[i].cls] += ms;
      }
    }
  }
  return CBC_OK;
}

cbc_status cbc_read_report(const void* workspace, size_t instance_bytes, int32_t instance,
                           void* stream, cbc_report* rep) {
  if (!workspace || !rep || instance < 0) return CBC_EINVAL;
  if (rep->capacity < 0 || (rep->capacity > 0 && !rep->trunc)) return CBC_EINVAL;
  if (instance > 0 && instance_bytes == 0) return CBC_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return CBC_EHIP;
  const char* base = (const char*)workspace + instance_bytes * (size_t)instance;
  WsHeader h;
  if (hipMemcpy(&h, base, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return CBC_EHIP;
  if (h.magic != REPORT_MAGIC || h.n_rec < 0 || h.rec_off < (int64_t)sizeof(WsHeader))
    return CBC_EINVAL;
  rep->status = h.status;
  rep->dropped_pivots = h.ndrop;
  rep->n_trunc = h.n_rec;
  const int nc = std::min(rep->capacity, h.n_rec);
  if (nc > 0 && hipMemcpy(rep->trunc, base + h.rec_off, sizeof(cbc_trunc_record) * (size_t)nc,
                          hipMemcpyDeviceToHost) != hipSuccess)
    return CBC_EHIP;
  return (cbc_status)h.status;
}

cbc_status cbc_apply(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                     const cbc_tree* tree, int32_t max_bond, double tol, cbc_precision prec,
                     void* workspace, size_t workspace_bytes, cbc_out* out, void* stream,
                     cbc_stats* stats) {
  return apply_impl(ctx, ttno, ttns, tree, max_bond, tol, prec, workspace, workspace_bytes, out,
                    stream, stats, 0);
}

cbc_status cbc_apply_noalloc(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                             const cbc_tree* tree, int32_t max_bond, double tol, cbc_precision prec,
                             cbc_out* out, void* stream, cbc_stats* stats) {
  return apply_impl(ctx, ttno, ttns, tree, max_bond, tol, prec, nullptr, 0, out, stream, stats, 0,
                    1, true);
}

cbc_status cbc_apply_split(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                           const cbc_tree* tree, int32_t max_bond, double tol, cbc_precision prec,
                           void* workspace, size_t workspace_bytes, void* scratch,
                           size_t scratch_bytes, cbc_out* out, void* stream, cbc_stats* stats) {
  if (!scratch) return CBC_EINVAL;
  return apply_impl(ctx, ttno, ttns, tree, max_bond, tol, prec, workspace, workspace_bytes, out,
                    stream, stats, 0, 1, false, scratch, scratch_bytes);
}

cbc_status cbc_apply_src(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                         const cbc_tensors* sketch, const cbc_tree* tree, int32_t max_bond,
                         cbc_precision prec, void* workspace, size_t workspace_bytes, cbc_out* out,
                         void* stream, cbc_stats* stats) {
  if (!sketch) return CBC_EINVAL;
  return apply_impl(ctx, ttno, ttns, tree, max_bond, 0.0, prec, workspace, workspace_bytes, out,
                    stream, stats, 2, 1, false, nullptr, 0, sketch);
}

cbc_status cbc_apply_many(cbc_ctx* ctx, int32_t count, const cbc_problem* problems,
                          cbc_precision prec, int32_t nstreams, void* const* scratch,
                          const size_t* scratch_bytes, void* stream) {
  if (!ctx || count < 0 || (count > 0 && !problems) || nstreams < 1 || nstreams > CBC_MAX_STREAMS)
    return CBC_EINVAL;
  if (scratch && !scratch_bytes) return CBC_EINVAL;
  for (int32_t j = 0; j < count; ++j) {
    const cbc_problem& p = problems[j];
    if (!p.tree || !p.ttno || !p.ttns || !p.out || !p.workspace) return CBC_EINVAL;
    if (scratch && !scratch[j % nstreams]) return CBC_EINVAL;
  }
  if (count == 0) return CBC_OK;
  while ((int)ctx->streams.size() < nstreams) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return CBC_EHIP;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(s);
      return CBC_EHIP;
    }
    ctx->streams.push_back(s);
    ctx->join_ev.push_back(e);
  }
  if (!ctx->fork_ev && hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) != hipSuccess)
    return CBC_EHIP;
  hipStream_t st = (hipStream_t)stream;
  const int used = std::min<int32_t>(nstreams, count);
  // fork: every stream used starts after the work queued on `stream` (inside a capture of `stream`
  // this makes them part of the same graph)
  if (hipEventRecord(ctx->fork_ev, st) != hipSuccess) return CBC_EHIP;
  for (int s = 0; s < used; ++s)
    if (hipStreamWaitEvent(ctx->streams[s], ctx->fork_ev, 0) != hipSuccess) return CBC_EHIP;
  cbc_status rc = CBC_OK;
  for (int32_t j = 0; j < count && rc == CBC_OK; ++j) {
    const cbc_problem& p = problems[j];
    const int s = j % nstreams;
    rc = apply_impl(ctx, p.ttno, p.ttns, p.tree, p.max_bond, p.tol, prec, p.workspace,
                    p.workspace_bytes, p.out, ctx->streams[s], p.stats, 0, 1, false,
                    scratch ? scratch[s] : nullptr, scratch ? scratch_bytes[s] : 0);
  }
  // join: `stream` continues after every problem (also after a failed call, so that a capture
  // of `stream` can be ended)
  for (int s = 0; s < used; ++s) {
    if (hipEventRecord(ctx->join_ev[s], ctx->streams[s]) != hipSuccess) return CBC_EHIP;
    if (hipStreamWaitEvent(st, ctx->join_ev[s], 0) != hipSuccess) return CBC_EHIP;
  }
  return rc;
}

cbc_status cbc_apply_dm(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                        const cbc_tree* tree, int32_t max_bond, cbc_precision prec, void* workspace,
                        size_t workspace_bytes, cbc_out* out, void* stream, cbc_stats* stats) {
  return apply_impl(ctx, ttno, ttns, tree, max_bond, 0.0, prec, workspace, workspace_bytes, out,
                    stream, stats, 3);
}

cbc_status cbc_apply_zipup(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                           const cbc_tree* tree, int32_t max_bond, cbc_precision prec,
                           void* workspace, size_t workspace_bytes, cbc_out* out, void* stream,
                           cbc_stats* stats) {
  return apply_impl(ctx, ttno, ttns, tree, max_bond, 0.0, prec, workspace, workspace_bytes, out,
                    stream, stats, 4);
}

cbc_status cbc_apply_batched(cbc_ctx* ctx, int32_t batch, const cbc_tensors* ttno,
                             const cbc_tensors* ttns, const cbc_tree* tree, int32_t max_bond,
                             double tol, cbc_precision prec, void* workspace,
                             size_t workspace_bytes, cbc_out* out, void* stream,
                             cbc_stats* stats) {
  return apply_impl(ctx, ttno, ttns, tree, max_bond, tol, prec, workspace, workspace_bytes, out,
                    stream, stats, 0, batch);
}

cbc_status cbc_apply_naive(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                           const cbc_tree* tree, int32_t max_bond, double tol, cbc_precision prec,
                           void* workspace, size_t workspace_bytes, cbc_out* out, void* stream,
                           cbc_stats* stats) {
  return apply_impl(ctx, ttno, ttns, tree, max_bond, tol, prec, workspace, workspace_bytes, out,
                    stream, stats, 1);
}

}  // extern "C"
