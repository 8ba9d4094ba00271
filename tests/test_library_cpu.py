"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every declared
symbol, validates arguments before any device work, and plans the same output bond dimensions as
the oracle produces."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2601_19650_amd import cbc
from paper_2601_19650_amd.inputs import chain_parent, config_problem, kary_parent, random_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in ("cbc.h", "cbc_testing.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(cbc_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_declared_symbols():
    L = cbc.lib()
    names = declared_functions()
    assert "cbc_apply" in names and "cbc_apply_naive" in names and "cbc_query" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(cbc.EXPORTED) | set(cbc.TESTING_EXPORTED) == set(names)


def _query(tree, max_bond=8, prec=0, method=0):
    ctx = cbc.Context()
    ws = ctypes.c_size_t()
    off = np.zeros(tree.n + 1, dtype=np.int64)
    rc = cbc.lib().cbc_query(ctx.h, ctypes.byref(tree.c), max_bond, prec, method, ctypes.byref(ws),
                             off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return rc, int(ws.value), off


def T(parent, phys=2, chi=None, dop=None):
    n = len(parent)
    chi = chi if chi is not None else [1 if p < 0 else 2 for p in parent]
    dop = dop if dop is not None else [1 if p < 0 else 2 for p in parent]
    return cbc.Tree(parent, [phys] * n if np.isscalar(phys) else phys, chi, dop)


@pytest.mark.parametrize("parent", [[-1, -1, 0], [1, 2, 0], [-1, 5, 0], [-1, 1], [0, 0]])
def test_bad_topology_rejected(parent):
    rc, _, _ = _query(T(parent))
    assert rc == -2


def test_bad_dims_rejected():
    assert _query(T([-1, 0], chi=[2, 2]))[0] == -2          # root bond must be 1
    assert _query(T([-1, 0], chi=[1, 0]))[0] == -2
    assert _query(T([-1, 0], phys=[2, 0]))[0] == -2
    assert _query(T([-1, 0]), max_bond=0)[0] == -1
    assert _query(T([-1, 0]), prec=7)[0] == -1
    assert _query(T([-1, 0]), method=5)[0] == -1


def test_oversized_truncation_is_unsupported():
    """A truncation Gram above the eigensolver's limit (2064, the two-stage reduction's panel of
    2048 rows plus the band) is reported at query time, on the host, as CBC_EUNSUP; Grams at the
    limit and the largest-bond workload (Grams of 1024) are accepted."""
    # two-site chain: the first site's joined leg is d * 1 = s wide against chi * D = s
    big = T([-1, 0], phys=2065, chi=[1, 2065], dop=[1, 1])
    assert _query(big, max_bond=64)[0] == -6
    edge = T([-1, 0], phys=2064, chi=[1, 2064], dop=[1, 1])
    assert _query(edge, max_bond=64)[0] == 0
    assert _query(cbc.Tree.of(config_problem("C4", n=10)), max_bond=256)[0] == 0


def test_apply_argument_errors_need_no_device():
    p = config_problem("C1")
    tree = cbc.Tree.of(p)
    ctx = cbc.Context()
    I64 = ctypes.POINTER(ctypes.c_int64)
    off = np.zeros(p.n, dtype=np.int64)
    sizes = [t.size for t in p.state]
    off[1:] = np.cumsum(sizes)[:-1]
    ooff = np.zeros(p.n, dtype=np.int64)
    osz = [w.size for w in p.op]
    ooff[1:] = np.cumsum(osz)[:-1]
    rc, ws, outoff = _query(tree, p.max_bond)
    assert rc == 0 and ws > 0
    bond = np.zeros(p.n, dtype=np.int32)
    ttns = cbc._Tensors(0x1000, off.ctypes.data_as(I64))
    ttno = cbc._Tensors(0x1000, ooff.ctypes.data_as(I64))
    out = cbc._Out(0x1000, outoff.ctypes.data_as(I64), bond.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    stats = cbc.Stats()
    f = cbc.lib().cbc_apply
    args = lambda tol, wsb, mb=p.max_bond: (ctx.h, ctypes.byref(ttno), ctypes.byref(ttns),
                                            ctypes.byref(tree.c), mb, tol, 0, 0x1000, wsb,
                                            ctypes.byref(out), None, ctypes.byref(stats))
    assert f(*args(-1.0, ws)) == -1
    assert f(*args(float("nan"), ws)) == -1
    assert f(*args(float("inf"), ws)) == -1
    assert f(*args(0.0, ws - 1)) == -3                       # workspace too small
    assert f(*args(0.0, ws, 0)) == -1
    assert f(ctx.h, None, ctypes.byref(ttns), ctypes.byref(tree.c), 4, 0.0, 0, 0x1000, ws,
             ctypes.byref(out), None, None) == -1
    # offsets that are not a packed layout are rejected
    bad = off.copy()
    bad[-1] += 10 ** 6
    ttns_bad = cbc._Tensors(0x1000, bad.ctypes.data_as(I64))
    assert f(ctx.h, ctypes.byref(ttno), ctypes.byref(ttns_bad), ctypes.byref(tree.c), 4, 0.0, 0,
             0x1000, ws, ctypes.byref(out), None, None) == -1


def planned_bonds(tree, max_bond):
    """The static output bonds fixed before device work (tol = 0)."""
    ctx = cbc.Context()
    bond = np.zeros(tree.n, dtype=np.int32)
    rc = cbc.lib().cbc_plan_bonds(ctx.h, ctypes.byref(tree.c), max_bond, 0,
                                  bond.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert rc == 0
    return [int(b) for b in bond]


@pytest.mark.parametrize("maker", [
    lambda: config_problem("C1"), lambda: config_problem("C2", n=16), lambda: config_problem("C3", n=15),
    lambda: random_problem(kary_parent(13, 3), 2, 6, 3, 5, seed=4),
    lambda: random_problem(chain_parent(7), [3, 1, 2, 2, 1, 3, 2], 5, 4, 6, seed=5)])
def test_planned_bonds_match_oracle(maker):
    """The static output bond dimensions the planner fixes before any device work equal the bond
    dimensions of the oracle's output (tol = 0)."""
    from oracle import cbc_tree
    p = maker()
    tree = cbc.Tree.of(p)
    rc, ws, off = _query(tree, p.max_bond)
    assert rc == 0
    ref = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    sizes = np.diff(off)
    assert all(int(s) >= t.size for s, t in zip(sizes, ref))
    # the bonds the library will report equal the oracle's output bonds
    bonds = planned_bonds(tree, p.max_bond)
    assert bonds == [t.shape[1] for t in ref]
    for prec in (0, 1):
        assert _query(tree, p.max_bond, prec)[0] == 0


@pytest.mark.parametrize("maker", [
    lambda: config_problem("C1"), lambda: config_problem("C2", n=12),
    lambda: random_problem(kary_parent(7, 2), 2, 8, 4, 4, seed=3),
    lambda: random_problem(kary_parent(13, 3), 2, 6, 3, 5, seed=4)])
def test_naive_plan_sizes_match_oracle(maker):
    """The naive baseline's planned output node sizes equal those of the oracle's naive method."""
    from oracle import tn
    p = maker()
    rc, ws, off = _query(cbc.Tree.of(p), p.max_bond, 0, 1)
    assert rc == 0 and ws > 0
    ref = tn.naive_compress(p.parent, p.op, p.state, p.max_bond)
    assert [int(s) for s in np.diff(off)] == [t.size for t in ref]


def test_autotune_arguments_and_cache_file(tmp_path):
    """cbc_autotune needs no device: it rejects a null context and an unwritable cache, creates a
    new cache file, and reads a cache whose foreign, malformed or invalid lines it skips."""
    L = cbc.lib()
    assert L.cbc_autotune(None, None) == -1
    path = tmp_path / "tune.txt"
    cbc.Context().autotune(path)
    assert path.exists()
    path.write_text("cbc-gemm 1 1 0 0 64 64 128 1 0 1 0 4 0.010\n"
                    "cbc-gemm 1 1 0 0 64 64 128 1 0 1 7 4 0.010\n"
                    "some other text\n"
                    "cbc-gemm 1 2\n")
    ctx = cbc.Context().autotune(path)
    assert ctx.autotune(None) is ctx
    assert L.cbc_autotune(ctx.h, str(tmp_path / "no_such_dir" / "t.txt").encode()) == -1


def test_autotune_reserves_split_scratch():
    """Plans built for autotuning reserve scratch for the split candidates, so cbc_query reports a
    larger workspace than for the fixed policy."""
    p = config_problem("C2", n=12)
    tree = cbc.Tree.of(p)
    sizes = []
    for tune in (False, True):
        ctx = cbc.Context()
        if tune:
            ctx.autotune()
        ws = ctypes.c_size_t()
        off = np.zeros(tree.n + 1, dtype=np.int64)
        rc = cbc.lib().cbc_query(ctx.h, ctypes.byref(tree.c), p.max_bond, 1, 0, ctypes.byref(ws),
                                 off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        assert rc == 0
        sizes.append(int(ws.value))
    assert sizes[1] > sizes[0]


def test_tensors_beyond_32bit_offsets_are_unsupported():
    """The kernels address operands with 32-bit element offsets: a plan whose contraction touches a
    tensor of 2^31 or more elements is rejected on the host with CBC_EUNSUP (here the root's
    operator tensor, 46341^2 x 4 elements), not truncated silently."""
    big = cbc.Tree([-1, 0], [46341, 2], [1, 2], [1, 4])
    assert _query(big, max_bond=4)[0] == -6
    ok = cbc.Tree([-1, 0], [512, 2], [1, 2], [1, 4])
    assert _query(ok, max_bond=4)[0] == 0


def test_read_report_argument_errors_need_no_device():
    """cbc_read_report validates its arguments before touching the device."""
    L = cbc.lib()
    rep = cbc.Report(0, 0, 0, 0, None)
    assert L.cbc_read_report(None, 0, 0, None, ctypes.byref(rep)) == -1
    assert L.cbc_read_report(ctypes.c_void_p(0x1000), 0, 0, None, None) == -1
    assert L.cbc_read_report(ctypes.c_void_p(0x1000), 0, -1, None, ctypes.byref(rep)) == -1
    bad = cbc.Report(0, 0, 0, 4, None)                    # capacity without an array
    assert L.cbc_read_report(ctypes.c_void_p(0x1000), 0, 0, None, ctypes.byref(bad)) == -1
    assert L.cbc_read_report(ctypes.c_void_p(0x1000), 0, 1, None, ctypes.byref(rep)) == -1


def test_status_strings():
    L = cbc.lib()
    for code in range(-8, 1):
        assert L.cbc_status_str(code)
    assert b"wait" in L.cbc_status_str(-8)


def test_plan_info_splits_the_queried_workspace():
    """cbc_plan_info needs no device: its persistent and scratch parts add up to cbc_query's
    workspace (the larger of the plans with and without a tolerance), and its per-class flops are
    the planner's algorithmic counts (a 31-node binary tree: Cholesky-QRs of three passes at the
    non-root nodes whose joined leg exceeds the environment bond, none where Q is the identity)."""
    p = config_problem("C3")
    tree = cbc.Tree.of(p)
    for prec in ("fp64", "mixed"):
        ctx = cbc.Context()
        infos = [cbc.plan_info(tree, p.max_bond, prec, tol_on=t, ctx=ctx) for t in (False, True)]
        rc, ws, _ = _query(tree, p.max_bond, cbc.PRECISIONS[prec])
        assert rc == 0
        assert ws == max(i["persistent_bytes"] + i["scratch_bytes"] for i in infos)
        for i in infos:
            assert i["persistent_bytes"] > 0 and i["scratch_bytes"] > 0 and i["table_bytes"] > 0
            nq = i["launches"]["chol"]
            assert nq % 3 == 0 and 0 < nq <= 3 * (p.n - 1)
            assert all(v >= 0 for v in i["flops"].values()) and i["flops"]["contract"] > 0
    # naive plans are described as well
    assert cbc.plan_info(tree, p.max_bond, "fp64", method="naive")["flops"]["eig"] > 0


def test_apply_split_argument_errors_need_no_device():
    """cbc_apply_split rejects a null scratch and buffers below the planned parts before any
    device work."""
    p = config_problem("C1")
    tree = cbc.Tree.of(p)
    ctx = cbc.Context()
    info = cbc.plan_info(tree, p.max_bond, "fp64", ctx=ctx)
    I64 = ctypes.POINTER(ctypes.c_int64)
    off = np.zeros(p.n, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in p.state])[:-1]
    ooff = np.zeros(p.n, dtype=np.int64)
    ooff[1:] = np.cumsum([w.size for w in p.op])[:-1]
    rc, ws, outoff = _query(tree, p.max_bond)
    bond = np.zeros(p.n, dtype=np.int32)
    ttns = cbc._Tensors(0x1000, off.ctypes.data_as(I64))
    ttno = cbc._Tensors(0x1000, ooff.ctypes.data_as(I64))
    out = cbc._Out(0x1000, outoff.ctypes.data_as(I64), bond.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    f = cbc.lib().cbc_apply_split
    pb, sb = info["persistent_bytes"], info["scratch_bytes"]
    call = lambda wsb, scr, scrb: f(ctx.h, ctypes.byref(ttno), ctypes.byref(ttns), ctypes.byref(tree.c),
                                    p.max_bond, 0.0, 0, 0x1000, wsb, scr, scrb, ctypes.byref(out),
                                    None, None)
    assert call(pb, None, sb) == -1
    assert call(pb - 1, 0x2000, sb) == -3
    assert call(pb, 0x2000, sb - 1) == -3


def test_ternary_node_contraction_order_fits_offsets():
    """At a node with a parent and three children the operator tensor is contracted after two of
    the three environments: taking every environment first would leave sigma * alpha_p * (chi *
    alpha * D)^3 elements open at once (here 4 * 32 * (32 * 12)^3 = 7.2e9, beyond the kernels'
    32-bit offsets), while the chosen order peaks at 6.0e8 elements. Ternary trees of the uneven
    batch workload with d = 4, chi = 32, D = 12 are therefore supported."""
    parent = kary_parent(13, 3)
    from paper_2601_19650_amd.inputs import cut_bonds
    phys = [4] * 13
    tree = cbc.Tree(parent, phys, cut_bonds(parent, phys, 32, 1), cut_bonds(parent, phys, 12, 2))
    assert _query(tree, max_bond=32)[0] == 0
    info = cbc.plan_info(tree, 32, "mixed")
    # the largest scratch intermediate holds 6.0e8 complex64 elements (two live at once)
    assert info["scratch_bytes"] < 3 * 8 * 4 * 32 ** 4 * 12 * 12


def test_query_plans_without_tables_stay_small():
    """Plans built for queries hold no offset tables on the host, so sizing the whole 256-instance
    uneven batch draw in one context takes seconds and little memory."""
    import resource
    import time
    from paper_2601_19650_amd.inputs import _parent_of, batch_shapes, cut_bonds
    ctx = cbc.Context()
    t0 = time.perf_counter()
    rss0 = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss
    unsupported = 0
    for j, kind, n, d, chi, D, _ in batch_shapes():
        parent = _parent_of(kind, n)
        tree = cbc.Tree(parent, [d] * n, cut_bonds(parent, [d] * n, chi, 1),
                        cut_bonds(parent, [d] * n, D, 2))
        ws = ctypes.c_size_t()
        off = np.zeros(n + 1, dtype=np.int64)
        rc = cbc.lib().cbc_query(ctx.h, ctypes.byref(tree.c), chi, 1, 0, ctypes.byref(ws),
                                 off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        unsupported += rc == -6
        assert rc in (0, -6)
    assert unsupported == 0
    assert time.perf_counter() - t0 < 60
    assert resource.getrusage(resource.RUSAGE_SELF).ru_maxrss - rss0 < 2_000_000   # KiB


def test_uneven_batch_graph_groups():
    """Batches are recorded as consecutive groups of at most `cap` launches; an instance larger
    than the cap forms a group of its own, and every instance is in exactly one group."""
    assert cbc.graph_groups([5, 5, 5], 10) == [[0, 1], [2]]
    assert cbc.graph_groups([5, 20, 5, 5], 10) == [[0], [1], [2, 3]]
    assert cbc.graph_groups([], 10) == []
    counts = [int(x) for x in np.random.default_rng(0).integers(50, 1200, 256)]
    groups = cbc.graph_groups(counts, cbc.UnevenBatch.MAX_GRAPH_LAUNCHES)
    assert [k for g in groups for k in g] == list(range(256))
    assert all(sum(counts[k] for k in g) <= cbc.UnevenBatch.MAX_GRAPH_LAUNCHES for g in groups)


@pytest.mark.parametrize("maker", [
    lambda: config_problem("C1"), lambda: config_problem("C2", n=12), lambda: config_problem("C3"),
    lambda: random_problem(kary_parent(13, 3), 2, 6, 3, 5, seed=4),
    lambda: random_problem(kary_parent(7, 2), [1, 1, 1, 2, 2, 2, 2], 4, 4, 3, seed=6)])
def test_src_plan_sizes_match_oracle(maker):
    """The randomised method's planned output node sizes equal those of the SRC oracle, and its plan
    holds no eigensolve (only contractions, Cholesky-QRs and normalisations)."""
    from oracle.src import src_tree
    from paper_2601_19650_amd.inputs import sketch_matrices
    p = maker()
    tree = cbc.Tree.of(p)
    for prec in (0, 1):
        rc, ws, off = _query(tree, p.max_bond, prec, 2)
        assert rc == 0 and ws > 0
    ref = src_tree(p.parent, p.state, p.op, p.max_bond, sketch_matrices(p.phys, p.max_bond, 3))
    assert [int(s) for s in np.diff(off)] == [t.size for t in ref]
    info = cbc.plan_info(tree, p.max_bond, "mixed", method="src")
    assert info["launches"]["eig"] == 0 and info["flops"]["eig"] == 0.0
    assert _query(tree, p.max_bond, 0, 5)[0] == -1


def test_apply_many_argument_errors_need_no_device():
    """cbc_apply_many checks its arguments (counts, stream count, problems, scratch) before any
    device work; an empty batch is a no-op."""
    L = cbc.lib()
    ctx = cbc.Context()
    P = ctypes.POINTER(cbc.CProblem)
    assert L.cbc_apply_many(None, 1, None, 0, 1, None, None, None) == -1
    assert L.cbc_apply_many(ctx.h, -1, None, 0, 1, None, None, None) == -1
    assert L.cbc_apply_many(ctx.h, 1, None, 0, 1, None, None, None) == -1
    assert L.cbc_apply_many(ctx.h, 0, None, 0, 1, None, None, None) == 0
    probs = (cbc.CProblem * 2)()
    assert L.cbc_apply_many(ctx.h, 2, ctypes.cast(probs, P), 0, 1, None, None, None) == -1
    assert L.cbc_apply_many(ctx.h, 0, None, 0, 0, None, None, None) == -1
    assert L.cbc_apply_many(ctx.h, 0, None, 0, 65, None, None, None) == -1
    scr = (ctypes.c_void_p * 1)(0x1000)
    assert L.cbc_apply_many(ctx.h, 0, None, 0, 1, scr, None, None) == -1


@pytest.mark.parametrize("maker", [
    lambda: config_problem("C1"), lambda: config_problem("C2", n=12),
    lambda: random_problem(kary_parent(13, 3), 2, 6, 3, 5, seed=4),
    lambda: random_problem(kary_parent(7, 2), [1, 1, 1, 2, 2, 2, 2], 4, 4, 3, seed=6)])
def test_dm_plan_sizes_match_oracle(maker):
    """The density-matrix method's planned output node sizes equal those of the DM oracle, and it
    plans one eigensolve per truncated node."""
    from oracle.dm import dm_tree
    p = maker()
    tree = cbc.Tree.of(p)
    for prec in (0, 1):
        rc, ws, off = _query(tree, p.max_bond, prec, 3)
        assert rc == 0 and ws > 0
    ref = dm_tree(p.parent, p.state, p.op, p.max_bond)
    assert [int(s) for s in np.diff(off)] == [t.size for t in ref]
    info = cbc.plan_info(tree, p.max_bond, "fp64", method="dm")
    truncated = sum(1 for i, t in enumerate(ref) if p.parent[i] >= 0 and
                    t.shape[1] < t.size // t.shape[1])
    assert info["launches"]["eig"] == truncated


@pytest.mark.parametrize("maker", [
    lambda: config_problem("C1"), lambda: config_problem("C2", n=12),
    lambda: random_problem(kary_parent(13, 3), 2, 6, 3, 5, seed=4),
    lambda: random_problem(kary_parent(7, 2), [1, 1, 1, 2, 2, 2, 2], 4, 4, 3, seed=6)])
def test_zipup_plan_sizes_match_oracle(maker):
    """Zip-Up's planned output node sizes equal those of the Zip-Up oracle; it plans one eigensolve
    per truncated node and no environment sweeps (fewer contraction flops than the density-matrix
    method on the same problem)."""
    from oracle.zipup import zipup_tree
    p = maker()
    tree = cbc.Tree.of(p)
    for prec in (0, 1):
        rc, ws, off = _query(tree, p.max_bond, prec, 4)
        assert rc == 0 and ws > 0
    ref = zipup_tree(p.parent, p.state, p.op, p.max_bond)
    assert [int(s) for s in np.diff(off)] == [t.size for t in ref]
    info = cbc.plan_info(tree, p.max_bond, "fp64", method="zipup")
    truncated = sum(1 for i, t in enumerate(ref) if p.parent[i] >= 0 and
                    t.shape[1] < t.size // t.shape[1])
    assert info["launches"]["eig"] == truncated
    dm = cbc.plan_info(tree, p.max_bond, "fp64", method="dm")
    assert info["flops"]["contract"] < dm["flops"]["contract"]
