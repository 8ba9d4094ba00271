"""Host checks of the seeded workload generators: the tree shapes of the random-network experiment
(Sec. IV A) and the entry distribution it draws from."""
import numpy as np
import pytest

from paper_2601_19650_amd.inputs import PAPER_WORKLOADS, paper_problem


def legs(p):
    """Per node: non-trivial virtual legs and physical dimension."""
    nv = [0] * p.n
    for j, q in enumerate(p.parent):
        if q >= 0 and p.chi[j] > 1:
            nv[j] += 1
            nv[q] += 1
    return nv, p.phys


def test_paper_tree_sizes():
    """Tensor train of 50 sites; T-tree of one centre and three chains of 20; perfect binary tree of
    depth 6 (127 nodes, 64 leaves carrying the physical legs); fork structure of 8 virtual nodes each
    holding a chain of 8 physical nodes. All physical legs have d = 3."""
    expect = {"mps": (50, 50), "ttree": (61, 60), "binary": (127, 64), "fork": (72, 64)}
    for kind, (n, nphys) in expect.items():
        p = paper_problem(kind, 2)
        assert p.n == n and p.parent.count(-1) == 1
        assert sum(1 for d in p.phys if d > 1) == nphys
        assert set(p.phys) <= {1, 3}


@pytest.mark.parametrize("kind", ["ttree", "binary", "fork"])
def test_paper_trees_are_t3ns(kind):
    """The three non-chain shapes are T3NS (Sec. II B): no node has more than three non-trivial
    legs, so a node with three virtual legs carries no physical leg."""
    p = paper_problem(kind, 2)
    nv, phys = legs(p)
    assert max(nv) == 3
    for v, d in zip(nv, phys):
        assert v + (d > 1) <= 3
    if kind == "binary":
        ch = [0] * p.n
        for q in p.parent:
            if q >= 0:
                ch[q] += 1
        assert all((c == 0) == (d > 1) for c, d in zip(ch, phys))    # leaves only
        assert set(ch) == {0, 2}


def test_paper_bonds_and_sweep():
    """State and operator bonds are the experiment's (40 for the tensor train, 10 otherwise; smaller
    only where a cut cannot carry them), and the target bonds run 2, 4, ... up to that bond."""
    for kind, (_, _, d, D, sweep) in PAPER_WORKLOADS.items():
        p = paper_problem(kind, sweep[-1])
        assert max(p.chi) == D and max(p.dop) == D
        assert sweep == list(range(2, D + 1, 2))
        assert p.max_bond == D


def test_paper_entry_distribution():
    """Real and imaginary parts are drawn from U[-0.5, 1] (then each network is scaled by one
    positive factor per tensor): the parts of every large tensor fill [-a/2, a] for its own a, with
    mean a/4."""
    p = paper_problem("mps", 8)
    big = [t for t in p.state + p.op if t.size >= 4000]
    assert len(big) > 40
    for t in big:
        for part in (t.real, t.imag):
            hi, lo = part.max(), part.min()
            assert -0.52 * hi <= lo <= -0.48 * hi
            assert abs(part.mean() / hi - 0.25) < 0.03
