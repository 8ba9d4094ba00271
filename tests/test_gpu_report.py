"""The call's report read through cbc_read_report (GPU): truncation records against the oracle's
singular values, device status words for non-finite input and for an expired cross-workgroup wait,
and the device-wide ordering of the multi-workgroup eigensolves inside a captured graph."""
import os
import re

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import cbc_tt, tn  # noqa: E402
from paper_2601_19650_amd.inputs import chain_parent, config_problem, kary_parent, random_problem  # noqa: E402


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_report_records_match_oracle(lib, prec):
    """Every truncation of the 20-site chain (d=2, chi=64, D=8, max_bond=64) is recorded with its
    node, Gram dimension, kept count, discarded weight sum_{j>=k} s_j^2 / sum_j s_j^2 and the
    relative gap of the Gram's eigenvalues at the cut, equal to what the oracle's SVDs give."""
    p = config_problem("C2", n=20)
    rec = []
    cbc_tt(tn.tree_to_mps(p.state), tn.tree_to_mpo(p.op), p.max_bond, record=rec)
    print(f"report {prec}", flush=True)
    out, comp = lib.compress(p, precision=prec)
    r = comp.report()
    assert r["status"] == "ok" and r["dropped_pivots"] == 0
    # the oracle truncates at every site of the forward sweep; the library only where the joined
    # leg exceeds max_bond (elsewhere L' is kept as it is, which discards nothing)
    cut = {i + 1: s for i, s in enumerate(rec) if len(s) > p.max_bond}
    # the library also factorises the smaller-side Gram where it is already no larger than max_bond
    # (a change of basis of the new leg that discards nothing); such records keep every direction
    nodes = sorted(t["node"] for t in r["trunc"])
    assert set(cut) <= set(nodes) and len(set(nodes)) == len(nodes)
    tol = 1e-12 if prec == "fp64" else 1e-5
    for t in r["trunc"]:
        s = rec[t["node"] - 1]
        lam = s ** 2
        assert t["sweep"] == 2 and t["dim"] == len(s)
        if t["node"] not in cut:
            assert t["kmax"] == t["kept"] == t["dim"] <= p.max_bond
            assert abs(t["discarded"]) <= tol and t["gap"] == 1.0
            continue
        k = p.max_bond
        assert t["kmax"] == k and t["kept"] == k
        assert abs(t["discarded"] - lam[k:].sum() / lam.sum()) <= tol
        assert abs(t["gap"] - (lam[k - 1] - lam[k]) / lam[k - 1]) <= 1e3 * tol + 1e-9
        assert t["flags"] == 0


def test_report_tolerance_kept_counts(lib):
    """With a tolerance the kept counts fall below kmax and the records say so."""
    p = config_problem("C2", n=16)
    out, comp = lib.compress(p, precision="fp64", tol=0.45)
    r = comp.report()
    assert r["status"] == "ok"
    assert any(t["kept"] < t["kmax"] for t in r["trunc"])
    for t in r["trunc"]:
        assert 1 <= t["kept"] <= t["kmax"] and 0.0 <= t["discarded"] < 1.0


def test_report_tree_sweeps(lib):
    """A binary tree records sweep-1 (subtree) and sweep-2 truncations."""
    p = config_problem("C3")
    out, comp = lib.compress(p, precision="mixed")
    r = comp.report()
    assert r["status"] == "ok"
    sweeps = {t["sweep"] for t in r["trunc"]}
    assert sweeps == {1, 2}
    assert all(0 <= t["node"] < p.n and p.parent[t["node"]] >= 0 for t in r["trunc"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_nonfinite_input_reports_enotpd(lib, prec):
    """A NaN in the input reaches a Gram matrix; the factorisations record CBC_ENOTPD (the kernels
    run to their normal end on NaN data) and check() raises."""
    p = random_problem(chain_parent(8), 2, 8, 4, 4, seed=3)
    p.state[3] = p.state[3].copy()
    p.state[3].reshape(-1)[0] = np.nan
    ctx = lib.Context()
    tree = lib.Tree.of(p)
    st, so = lib.pack(p.state, "cuda")
    op, oo = lib.pack(p.op, "cuda")
    c = lib.Compressor(ctx, tree, p.max_bond, prec)
    c.run(op, oo, st, so)
    r = c.report()
    assert r["status"] == "enotpd"
    with pytest.raises(lib.CbcError):
        c.check()
    # a later call with finite input on the same workspace reports ok again
    p2 = random_problem(chain_parent(8), 2, 8, 4, 4, seed=3)
    st2, so2 = lib.pack(p2.state, "cuda")
    c.run(op, oo, st2, so2)
    assert c.report()["status"] == "ok"


def _herm(rng, s):
    a = rng.standard_normal((s, s + 7)) + 1j * rng.standard_normal((s, s + 7))
    return a @ a.conj().T


def test_eig_record_and_forced_timeout(lib):
    """The multi-workgroup reduction (s = 200): its record matches numpy.linalg.eigvalsh, and with
    its wait limit forced below zero (every workgroup leaves at its first barrier) the status word
    receives CBC_ETIMEOUT instead of the call hanging or reporting success."""
    rng = np.random.default_rng(5)
    g = _herm(rng, 200)
    G = torch.from_numpy(g).cuda()
    status, rec, U, lam, kept = lib.test_eig_report(G, 50)
    assert status == 0
    w = np.sort(np.linalg.eigvalsh(g))[::-1]
    assert rec["node"] == 7 and rec["sweep"] == 2 and rec["dim"] == 200 and rec["kept"] == 50
    assert abs(rec["discarded"] - w[50:].sum() / w.sum()) <= 1e-12
    assert abs(rec["gap"] - (w[49] - w[50]) / w[49]) <= 1e-9
    status, rec, U, lam, kept = lib.test_eig_report(G, 50, force_timeout=True)
    assert status == -8
    # the device is usable afterwards
    status, rec, U, lam, kept = lib.test_eig_report(G, 50)
    assert status == 0


def test_uneven_capture_with_large_grams_replays(lib):
    """Instances whose truncation Grams exceed 128, forked over several streams and recorded into one
    caller-captured graph: the captured eigensolves take the two-stage reduction (no workgroups that
    wait for each other, so no device-wide ordering is recorded inside the capture), and every replay,
    with eager work in between, matches the eager result of the same instances (which took the
    multi-workgroup reduction) to the parity bar of its precision."""
    probs = [random_problem(kary_parent(7, 2), 4, 150, 12, 140, seed=7 + k, name=f"big{k}")
             for k in range(4)]
    ub = lib.UnevenBatch(probs, precision="fp64", nstreams=3)
    ub.run()
    torch.cuda.synchronize()
    assert all(comp.stats.max_eig_dim > 128 for comp, _ in ub.items)
    eager = [comp.unpack() for comp, _ in ub.items]
    for comp, _ in ub.items:
        assert comp.report()["status"] == "ok"
    ub.capture()
    for rep in range(3):
        for comp, _ in ub.items:
            comp.out.zero_()
        torch.cuda.synchronize()
        ub.run()
        torch.cuda.synchronize()
        x = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")   # eager work
        torch.cuda.synchronize()
        del x
        for (comp, _), p, ref in zip(ub.items, probs, eager):
            assert comp.report()["status"] == "ok"
            out = comp.unpack()
            assert tn.rel_error(p.parent, out, ref) <= 1e-10, (rep, p.name)
