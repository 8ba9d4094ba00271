"""Pins for the SRC oracle (oracle/src.py): checks against what the method and the mathematics fix,
never against the oracle itself. CPU only, small dense systems."""
import numpy as np
import pytest

from oracle import tn
from oracle.src import src_tree
from paper_2601_19650_amd.inputs import chain_parent, kary_parent, random_problem, sketch_matrices


def dense_phi(p):
    return tn.apply_dense(p.parent, p.op, tn.to_dense(p.parent, p.state))


def subtree(parent, i):
    out, stack = [], [i]
    while stack:
        j = stack.pop()
        out.append(j)
        stack.extend(c for c, q in enumerate(parent) if q == j)
    return sorted(out)


def khatri_rao(mats):
    """Column-wise Kronecker product, first factor slowest."""
    out = np.ones((1, mats[0].shape[1]), dtype=np.complex128)
    for m in mats:
        out = (out[:, None, :] * m[None, :, :]).reshape(-1, m.shape[1])
    return out


def dense_src(p, max_bond, sketch):
    """SRC written with dense unfoldings: at every non-root node (leaves first) the unfolding of
    O|psi> between the node's subtree and the rest, times the Khatri-Rao sketch of the rest, with
    each child's subtree indices projected onto that child's basis; the node's basis spans its
    columns (identity where the rows do not exceed max_bond). The result is O|psi> with the basis
    projectors of the root's children applied."""
    n, parent = p.n, p.parent
    phi = dense_phi(p).reshape(p.phys)
    ch = [[c for c, q in enumerate(parent) if q == i] for i in range(n)]
    root = parent.index(-1)
    U = {}
    for i in tn.postorder(parent):
        if i == root:
            continue
        sub = subtree(parent, i)
        rest = [j for j in range(n) if j not in sub]
        # rows ordered (sigma_i, then each child's subtree nodes), columns the rest
        order = [i] + [j for c in ch[i] for j in subtree(parent, c)]
        m = np.transpose(phi, order + rest).reshape(int(np.prod([p.phys[j] for j in order])), -1)
        y = m @ khatri_rao([sketch[j] for j in rest])
        # project the children's subtrees onto their bases: rows become (sigma_i, k_c...)
        y = y.reshape([p.phys[i]] + [int(np.prod([p.phys[j] for j in subtree(parent, c)]))
                                     for c in ch[i]] + [max_bond])
        for pos, c in enumerate(ch[i]):
            y = np.moveaxis(np.tensordot(U[c][0].conj(), y, axes=([0], [1 + pos])), 0, 1 + pos)
        rows = int(np.prod(y.shape[:-1]))
        if rows <= max_bond:
            q = np.eye(rows, dtype=np.complex128)
        else:
            q, _ = np.linalg.qr(y.reshape(rows, max_bond), mode="reduced")
        q = q.reshape(y.shape[:-1] + (q.shape[1],))
        # the basis on the subtree's physical indices, rows in the order (sigma_i, children's
        # subtree nodes...)
        for pos, c in enumerate(ch[i]):
            q = np.moveaxis(np.tensordot(U[c][0], q, axes=([1], [1 + pos])), 0, 1 + pos)
        U[i] = (q.reshape(-1, q.shape[-1]), order)
    res = phi
    for c in ch[root]:
        basis, order = U[c]
        others = [j for j in range(n) if j not in order]
        x = np.transpose(res, order + others).reshape(basis.shape[0], -1)
        x = basis @ (basis.conj().T @ x)
        res = np.transpose(x.reshape([p.phys[j] for j in order + others]),
                           np.argsort(order + others))
    return res.reshape(-1), phi.reshape(-1)


CASES = [
    ("chain7", chain_parent(7), 2, 4, 3, 3, 1),
    ("chain6d3", chain_parent(6), 3, 6, 3, 4, 2),
    ("bin7", kary_parent(7, 2), 2, 4, 3, 3, 3),
    ("ter10", kary_parent(10, 3), 2, 4, 2, 3, 4),
    ("bin7-internal-d1", kary_parent(7, 2), [1, 1, 1, 2, 2, 2, 2], 4, 3, 3, 5),
    ("uneven9", [-1, 0, 0, 1, 1, 1, 2, 2, 6], 2, 4, 3, 3, 6),
]


@pytest.mark.parametrize("name,parent,phys,chi,D,mb,seed", CASES, ids=[c[0] for c in CASES])
def test_src_dense_formulation(name, parent, phys, chi, D, mb, seed):
    """The network sweeps equal the dense formulation (unfoldings times Khatri-Rao sketches)."""
    p = random_problem(parent, phys, chi, D, mb, seed=seed)
    sk = sketch_matrices(p.phys, mb, seed + 100)
    got = tn.to_dense(p.parent, src_tree(p.parent, p.state, p.op, mb, sk)).reshape(-1)
    ref, phi = dense_src(p, mb, sk)
    assert np.linalg.norm(got - phi) > 1e-3 * np.linalg.norm(phi)        # really truncating
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(phi)


@pytest.mark.parametrize("name,parent,phys,chi,D,mb,seed", CASES, ids=[c[0] for c in CASES])
def test_src_projection_isometries_and_eckart_young(name, parent, phys, chi, D, mb, seed):
    """The result is an orthogonal projection of O|psi> (<phi|psi'> = ||psi'||^2), every non-root
    node is an isometry toward its parent, and the error is at least the optimal truncation error
    of every cut to the bond the result has there."""
    p = random_problem(parent, phys, chi, D, mb, seed=seed)
    sk = sketch_matrices(p.phys, mb, seed + 100)
    out = src_tree(p.parent, p.state, p.op, mb, sk)
    phi = dense_phi(p)
    psi = tn.to_dense(p.parent, out)
    assert abs(np.vdot(phi, psi) - np.vdot(psi, psi)) <= 1e-12 * np.vdot(phi, phi).real
    root = p.parent.index(-1)
    for i, t in enumerate(out):
        if i != root:
            assert tn.isometry_error(t) <= 1e-12
    err = np.linalg.norm(phi - psi)
    for i in range(p.n):
        if i == root:
            continue
        sub = subtree(p.parent, i)
        rest = [j for j in range(p.n) if j not in sub]
        m = np.transpose(phi, sub + rest).reshape(int(np.prod([p.phys[j] for j in sub])), -1)
        s = np.linalg.svd(m, compute_uv=False)
        k = out[i].shape[1]
        assert err >= np.sqrt(np.sum(s[k:] ** 2)) * (1 - 1e-10)


def test_src_exact_when_the_sketch_covers_every_rank():
    """With bonds chi * D = 4 and physical dimensions 8 (a chain) or 6 (a root with three leaves)
    the compressed nodes have more rows than the target bond 5, which is above every rank: the
    sketch captures every range exactly and the result is O|psi>."""
    p = random_problem(chain_parent(4), 8, 2, 2, 5, seed=9)
    sk = sketch_matrices(p.phys, 5, 19)
    out = src_tree(p.parent, p.state, p.op, 5, sk)
    phi = dense_phi(p)
    psi = tn.to_dense(p.parent, out)
    assert np.linalg.norm(phi - psi) <= 1e-12 * np.linalg.norm(phi)
    assert any(t.shape[1] == 5 for t in out)       # the QR path was taken
    tree = random_problem(kary_parent(4, 3), 6, 2, 2, 5, seed=10)
    sk = sketch_matrices(tree.phys, 5, 20)
    out = src_tree(tree.parent, tree.state, tree.op, 5, sk)
    assert all(t.shape[1] == 5 for t in out[1:])
    psi = tn.to_dense(tree.parent, out)
    phi = dense_phi(tree)
    assert np.linalg.norm(phi - psi) <= 1e-12 * np.linalg.norm(phi)


@pytest.mark.parametrize("name,parent,phys,chi,D,mb,seed", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_src_sketch_symmetries(name, parent, phys, chi, D, mb, seed):
    """Scaling column r of every node's sketch by its own nonzero factor scales column r of every Y
    by their product, and permuting the columns of all sketches alike permutes those of Y: neither
    changes a column space, so the result is the same state."""
    p = random_problem(parent, phys, chi, D, mb, seed=seed)
    sk = sketch_matrices(p.phys, mb, seed + 100)
    base = tn.to_dense(p.parent, src_tree(p.parent, p.state, p.op, mb, sk))
    rng = np.random.default_rng(seed)
    scaled = [m * (rng.uniform(0.5, 2.0, mb) * np.exp(1j * rng.uniform(0, 6.28, mb)))[None, :]
              for m in sk]
    perm = rng.permutation(mb)
    permuted = [m[:, perm] for m in sk]
    for variant in (scaled, permuted):
        psi = tn.to_dense(p.parent, src_tree(p.parent, p.state, p.op, mb, variant))
        assert np.linalg.norm(psi - base) <= 1e-10 * np.linalg.norm(base)
    # a sketch drawn afresh gives a different (but still projected) result
    other = tn.to_dense(p.parent, src_tree(p.parent, p.state, p.op, mb,
                                           sketch_matrices(p.phys, mb, seed + 999)))
    assert np.linalg.norm(other - base) > 1e-6 * np.linalg.norm(base)


def test_src_error_close_to_optimal_on_average():
    """A Gaussian sketch of width D-bar finds a near-optimal subspace on average: over 20 sketches
    the mean error of a truncating 6-site chain stays within 3x of the direct method's (truncated
    SVDs of the exact product, an upper bound on the optimal error at these bonds)."""
    p = random_problem(chain_parent(6), 2, 4, 3, 3, seed=31)
    phi = dense_phi(p)
    direct = np.linalg.norm(tn.to_dense(p.parent, tn.naive_compress(p.parent, p.op, p.state, 3)) - phi)
    errs = []
    for s in range(20):
        sk = sketch_matrices(p.phys, 3, 1000 + s)
        errs.append(np.linalg.norm(tn.to_dense(p.parent, src_tree(p.parent, p.state, p.op, 3, sk)) - phi))
    assert direct > 1e-3 * np.linalg.norm(phi)
    assert min(errs) >= direct * 0.5 and np.mean(errs) <= 3.0 * direct
