"""Parity of the GPU Zip-Up compression (cbc_apply_zipup, through the C ABI) with the Zip-Up oracle
on the same seeded inputs. Bars as for CBC: FP64 within 1e-10 relative state error, mixed within
1e-5 infidelity and 1e-3 relative state error."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import tn  # noqa: E402
from oracle.zipup import zipup_tree  # noqa: E402
from paper_2601_19650_amd.inputs import (chain_parent, config_problem, kary_parent,  # noqa: E402
                                         paper_problem, random_problem)

FP64_BAR = 1e-10
MIXED_BAR = 1e-5
MIXED_REL_BAR = 1e-3

MAKERS = [
    lambda: config_problem("C1"),
    lambda: config_problem("C2", n=16),
    lambda: config_problem("C3", n=15),
    lambda: random_problem(chain_parent(10), 3, 9, 4, 7, seed=2, name="mps10d3"),
    lambda: random_problem(kary_parent(13, 3), 2, 6, 3, 5, seed=4, name="ter13"),
    lambda: random_problem(kary_parent(7, 2), [1, 1, 1, 2, 2, 2, 2], 4, 4, 3, seed=6, name="leafphys"),
    lambda: random_problem([-1], 3, 1, 1, 2, seed=7, name="single"),
    lambda: random_problem(chain_parent(5), 8, 2, 2, 5, seed=9, name="thin-unfoldings"),
    lambda: paper_problem("mps", 6, size=12, bond=6),
    lambda: paper_problem("ttree", 4, size=4, bond=4),
    lambda: paper_problem("binary", 4, size=3, bond=4),
    lambda: paper_problem("fork", 3, size=3, bond=4),
]


def check_zipup(lib, p, prec, ref=None):
    print(f"zipup {p.name} n={p.n} prec={prec}", flush=True)
    if ref is None:
        ref = zipup_tree(p.parent, p.state, p.op, p.max_bond)
    out, comp = lib.compress(p, precision=prec, method="zipup")
    assert [t.shape for t in out] == [t.shape for t in ref]
    err = tn.rel_error(p.parent, out, ref)
    if prec == "fp64":
        assert err <= FP64_BAR, err
    else:
        infid = 1.0 - tn.fidelity(p.parent, out, ref)
        assert infid <= MIXED_BAR and err <= MIXED_REL_BAR, (infid, err)
    # non-root nodes are (partial) isometries toward their parent: where an unfolding has fewer
    # columns than the new bond, the completion of the rank-deficient Z Z^H may have zero columns
    root = p.parent.index(-1)
    for i, t in enumerate(out):
        if i != root and t.size:
            m = np.moveaxis(t, 1, 0).reshape(t.shape[1], -1)
            g = m @ m.conj().T
            assert np.linalg.norm(g @ g - g) <= 1e-12 * max(1.0, np.linalg.norm(g))
            assert np.allclose(np.diag(g).real, np.round(np.diag(g).real), atol=1e-12)
    assert all(r["sweep"] == 4 for r in comp.report()["trunc"])
    return out, comp


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("maker", MAKERS)
def test_zipup_parity(lib, maker, prec):
    check_zipup(lib, maker(), prec)


def test_zipup_exact_case_matches_dense(lib):
    """The 8-site chain with target bond 32 covers every rank: the result equals O|psi>."""
    p = config_problem("C1")
    out, _ = check_zipup(lib, p, "fp64")
    phi = tn.apply_dense(p.parent, p.op, tn.to_dense(p.parent, p.state))
    psi = tn.to_dense(p.parent, out)
    assert np.linalg.norm(phi - psi) <= 1e-12 * np.linalg.norm(phi)


def test_zipup_is_an_orthogonal_projection(lib):
    """<Phi|psi'> = <psi'|psi'> for the result psi' of a truncating call (the root's children's
    subtree bases are isometries), checked with the oracle's sandwich contractions."""
    p = paper_problem("binary", 3, size=4, bond=4)
    out, _ = check_zipup(lib, p, "fp64")
    prod = tn.product_ttn(p.parent, p.op, p.state)
    v, ls = tn.overlap(p.parent, prod, out)
    w, lw = tn.overlap(p.parent, out, out)
    assert abs(v * np.exp(ls - lw) - w) <= 1e-10 * abs(w)


@pytest.fixture(scope="module")
def c4_cut():
    p = config_problem("C4", n=10)
    print("oracle Zip-Up, large-bond shape cut to 10 sites", flush=True)
    return p, zipup_tree(p.parent, p.state, p.op, p.max_bond)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_zipup_large_bond_shape(lib, c4_cut, prec):
    """The large-bond shape (d=4, chi=256, D=16, target bond 256) cut to 10 sites: local Grams of
    1024 x 1024 at the bulk sites, through the multi-workgroup reduction."""
    p, ref = c4_cut
    check_zipup(lib, p, prec, ref=ref)
