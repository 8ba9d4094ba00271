"""Parity of the GPU randomised compression (cbc_apply_src, through the C ABI) with the SRC oracle on
the same seeded inputs and sketch matrices. Bars as for CBC: FP64 within 1e-10 relative state error,
mixed within 1e-5 infidelity and 1e-3 relative state error."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import tn  # noqa: E402
from oracle.src import src_tree  # noqa: E402
from paper_2601_19650_amd.inputs import (chain_parent, config_problem, kary_parent,  # noqa: E402
                                         paper_problem, random_problem, sketch_matrices)

FP64_BAR = 1e-10
MIXED_BAR = 1e-5
MIXED_REL_BAR = 1e-3

MAKERS = [
    lambda: config_problem("C1"),
    lambda: config_problem("C2", n=16),
    lambda: config_problem("C3"),
    lambda: random_problem(chain_parent(10), 3, 9, 4, 7, seed=2, name="mps10d3"),
    lambda: random_problem(kary_parent(13, 3), 2, 6, 3, 5, seed=4, name="ter13"),
    lambda: random_problem(kary_parent(7, 2), [1, 1, 1, 2, 2, 2, 2], 4, 4, 3, seed=6, name="leafphys"),
    lambda: random_problem([-1], 3, 1, 1, 2, seed=7, name="single"),
    lambda: paper_problem("ttree", 4, size=4, bond=4),
    lambda: paper_problem("fork", 3, size=3, bond=4),
]


def check_src(lib, p, prec, seed=11, ref=None):
    sk = sketch_matrices(p.phys, p.max_bond, seed)
    print(f"src {p.name} n={p.n} prec={prec}", flush=True)
    if ref is None:
        ref = src_tree(p.parent, p.state, p.op, p.max_bond, sk)
    out, comp = lib.compress(p, precision=prec, method="src", sketch=sk)
    assert [t.shape for t in out] == [t.shape for t in ref]
    err = tn.rel_error(p.parent, out, ref)
    if prec == "fp64":
        assert err <= FP64_BAR, err
    else:
        infid = 1.0 - tn.fidelity(p.parent, out, ref)
        assert infid <= MIXED_BAR and err <= MIXED_REL_BAR, (infid, err)
    # non-root nodes are partial isometries toward their parent: where the sketched columns have
    # lower rank than the target bond (the sketch already holds the exact rank) the Cholesky-QR
    # drops the surplus pivots and those directions are zero, so m m^H is a projector
    root = p.parent.index(-1)
    for i, t in enumerate(out):
        if i != root and t.size:
            m = np.moveaxis(t, 1, 0).reshape(t.shape[1], -1)
            g = m @ m.conj().T
            assert np.linalg.norm(g @ g - g) <= 1e-12 * max(1.0, np.linalg.norm(g))
            assert np.allclose(np.diag(g).real, np.round(np.diag(g).real), atol=1e-12)
    assert comp.stats.n_eig == 0
    return out, comp


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("maker", MAKERS)
def test_src_parity(lib, maker, prec):
    check_src(lib, maker(), prec)


def test_src_exact_case_matches_dense(lib):
    """The 8-site chain with target bond 32 (every rank is at most 32): the sketch captures every
    range, so the result equals O|psi>."""
    p = config_problem("C1")
    out, _ = check_src(lib, p, "fp64")
    phi = tn.apply_dense(p.parent, p.op, tn.to_dense(p.parent, p.state))
    psi = tn.to_dense(p.parent, out)
    assert np.linalg.norm(phi - psi) <= 1e-12 * np.linalg.norm(phi)


@pytest.fixture(scope="module")
def c4_cut():
    p = config_problem("C4", n=10)
    sk = sketch_matrices(p.phys, p.max_bond, 11)
    print("oracle SRC, large-bond shape cut to 10 sites", flush=True)
    return p, src_tree(p.parent, p.state, p.op, p.max_bond, sk)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_src_large_bond_shape(lib, c4_cut, prec):
    """The large-bond shape (d=4, chi=256, D=16, target bond 256) cut to 10 sites: Y is 1024 x 256 at
    the bulk sites, sketches of width 256."""
    p, ref = c4_cut
    check_src(lib, p, prec, ref=ref)


def test_src_graph_replay_is_bitwise(lib):
    """Later calls replay the captured graph; every replay equals the first call bit for bit."""
    p = config_problem("C3")
    sk = sketch_matrices(p.phys, p.max_bond, 11)
    ctx = lib.Context()
    tree = lib.Tree.of(p)
    st, so = lib.pack(p.state, "cuda")
    op, oo = lib.pack(p.op, "cuda")
    skb = lib.pack(sk, "cuda")
    c = lib.Compressor(ctx, tree, p.max_bond, "mixed", method="src")
    s = torch.cuda.Stream()
    outs = []
    for r in range(3):
        c.out.zero_()
        torch.cuda.synchronize()
        c.run(op, oo, st, so, stream=s.cuda_stream, sketch=skb)
        assert c.stats.graph_replayed == (1 if r > 0 else 0)
        outs.append(c.unpack())
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
