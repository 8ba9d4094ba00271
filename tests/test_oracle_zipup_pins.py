"""Pins for the Zip-Up oracle (oracle/zipup.py): checks against what the method and the mathematics
fix, never against the oracle itself. CPU only, small dense systems."""
import numpy as np
import pytest

from oracle import tn
from oracle.zipup import zipup_tree
from paper_2601_19650_amd.inputs import chain_parent, kary_parent, random_problem


def dense_phi(p):
    return tn.apply_dense(p.parent, p.op, tn.to_dense(p.parent, p.state))


def subtree(parent, i):
    out, stack = [], [i]
    while stack:
        j = stack.pop()
        out.append(j)
        stack.extend(c for c, q in enumerate(parent) if q == j)
    return sorted(out)


def dense_subtree_product(p, i):
    """The exact product O|psi> restricted to the subtree of i, as an array over the subtree's
    physical legs (node order) and the fused bond (alpha_i, beta_i) to i's parent."""
    prod = tn.product_ttn(p.parent, p.op, p.state)
    nodes = subtree(p.parent, i)
    ch = [[c for c, q in enumerate(p.parent) if q == j] for j in range(p.n)]
    n = p.n
    args = []
    for j in nodes:
        args += [prod[j], [j, n + j] + [n + c for c in ch[j]]]
    return np.einsum(*args, nodes + [n + i], optimize="greedy")


def dense_zipup(p, max_bond):
    """Zip-Up written with dense unfoldings: at every non-root node (leaves first) the unfolding of
    the node's exact subtree product between (sigma_i, the children's subtrees) and the bond to the
    parent, each child's subtree indices projected onto that child's basis; the node's basis is the
    top max_bond left singular vectors (identity where the rows do not exceed max_bond). The result
    is O|psi> with the basis projectors of the root's children applied."""
    n, parent = p.n, p.parent
    phi = dense_phi(p).reshape(p.phys)
    ch = [[c for c, q in enumerate(parent) if q == i] for i in range(n)]
    root = parent.index(-1)
    U = {}
    for i in tn.postorder(parent):
        if i == root:
            continue
        nodes = subtree(parent, i)
        order = [i] + [j for c in ch[i] for j in subtree(parent, c)]
        m = dense_subtree_product(p, i)
        m = np.transpose(m, [nodes.index(j) for j in order] + [len(nodes)])
        m = m.reshape([p.phys[i]] + [int(np.prod([p.phys[j] for j in subtree(parent, c)]))
                                     for c in ch[i]] + [-1])
        for pos, c in enumerate(ch[i]):
            m = np.moveaxis(np.tensordot(U[c][0].conj(), m, axes=([0], [1 + pos])), 0, 1 + pos)
        rows = int(np.prod(m.shape[:-1]))
        if rows <= max_bond:
            q = np.eye(rows, dtype=np.complex128)
        else:
            u, s, _ = np.linalg.svd(m.reshape(rows, -1), full_matrices=True)
            q = u[:, :max_bond]
        q = q.reshape(m.shape[:-1] + (q.shape[1],))
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
def test_zipup_dense_formulation(name, parent, phys, chi, D, mb, seed):
    """The single sweep equals the dense formulation (top singular vectors of projected subtree
    unfoldings)."""
    p = random_problem(parent, phys, chi, D, mb, seed=seed)
    got = tn.to_dense(p.parent, zipup_tree(p.parent, p.state, p.op, mb)).reshape(-1)
    ref, phi = dense_zipup(p, mb)
    assert np.linalg.norm(got - phi) > 1e-3 * np.linalg.norm(phi)        # really truncating
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(phi)


@pytest.mark.parametrize("name,parent,phys,chi,D,mb,seed", CASES, ids=[c[0] for c in CASES])
def test_zipup_projection_isometries_and_lower_bound(name, parent, phys, chi, D, mb, seed):
    """The result is an orthogonal projection of O|psi> (the root's children's subtree bases are
    isometries), every non-root node is an isometry, and the error is at least the optimal tail of
    every cut (the result has at most the kept bond across it)."""
    p = random_problem(parent, phys, chi, D, mb, seed=seed)
    out = zipup_tree(p.parent, p.state, p.op, mb)
    phi = dense_phi(p)
    psi = tn.to_dense(p.parent, out)
    assert abs(np.vdot(phi, psi) - np.vdot(psi, psi)) <= 1e-12 * np.vdot(phi, phi).real
    root = p.parent.index(-1)
    err = np.linalg.norm(phi - psi)
    for i in range(p.n):
        if i == root:
            continue
        assert tn.isometry_error(out[i]) <= 1e-12
        sub = subtree(p.parent, i)
        rest = [j for j in range(p.n) if j not in sub]
        m = np.transpose(phi.reshape(p.phys), sub + rest).reshape(
            int(np.prod([p.phys[j] for j in sub])), -1)
        s = np.linalg.svd(m, compute_uv=False)
        assert err >= np.sqrt(np.sum(s[out[i].shape[1]:] ** 2)) * (1 - 1e-10)


def test_zipup_exact_when_the_bond_covers_every_rank():
    """With the target bond at least every rank the result is O|psi>: a chain with d = 8 and
    chi * D = 4 (rows above the target 5, unfoldings with fewer columns than the target, so the
    completed singular vectors are used) and a ternary tree."""
    p = random_problem(chain_parent(4), 8, 2, 2, 5, seed=9)
    out = zipup_tree(p.parent, p.state, p.op, 5)
    assert any(t.shape[1] == 5 for t in out)
    phi = dense_phi(p)
    assert np.linalg.norm(tn.to_dense(p.parent, out) - phi) <= 1e-12 * np.linalg.norm(phi)
    p = random_problem(kary_parent(4, 3), 6, 2, 2, 5, seed=10)
    out = zipup_tree(p.parent, p.state, p.op, 5)
    phi = dense_phi(p)
    assert np.linalg.norm(tn.to_dense(p.parent, out) - phi) <= 1e-12 * np.linalg.norm(phi)


def _identity_chain_op(n, d):
    eye = np.eye(d, dtype=np.complex128)
    return [eye.reshape(d, d, 1, 1) if i < n - 1 else eye.reshape(d, d, 1) for i in range(n)]


def _canonical_toward_leaf(state):
    """QR sweep from the root (node 0) along the chain: every node but the leaf becomes an isometry
    from (sigma, parent bond) onto its child bond; the leaf holds the norm."""
    st = [t.copy() for t in state]
    for j in range(len(st) - 1):
        d, a, b = st[j].shape
        q, r = np.linalg.qr(st[j].reshape(d * a, b))
        st[j] = q.reshape(d, a, q.shape[1])
        st[j + 1] = np.einsum("xb,sbc->sxc" if st[j + 1].ndim == 3 else "xb,sb->sx", r, st[j + 1])
    return st


def _tt_svd_from_leaf(psi, phys, mb):
    """Sequential truncated SVD of a dense vector from the last site to the first: at site j the
    tail (sites j..n-1), already projected onto the kept basis of sites j+1..n-1, keeps its top mb
    left singular vectors against the prefix."""
    n = len(phys)
    b = np.ones((1, 1), dtype=np.complex128)        # basis of the empty tail
    for j in range(n - 1, 0, -1):
        c = np.kron(np.eye(phys[j]), b)              # candidate basis of sites j..n-1
        m = psi.reshape(int(np.prod(phys[:j])), -1)  # prefix x tail
        a = c.conj().T @ m.T
        if a.shape[0] <= mb:
            u = np.eye(a.shape[0], dtype=np.complex128)
        else:
            u = np.linalg.svd(a, full_matrices=False)[0][:, :mb]
        b = c @ u
    m = psi.reshape(phys[0], -1)
    return (m @ b.conj() @ b.T).reshape(-1)


@pytest.mark.parametrize("n,d,chi,mb,seed", [(6, 2, 6, 3, 11), (5, 3, 8, 4, 12)])
def test_zipup_identity_operator_on_canonical_chain_is_tt_svd(n, d, chi, mb, seed):
    """For the identity operator and a chain whose not-yet-visited part is an isometry (canonical
    form with the centre at the first visited site), each local truncation sees the exact singular
    vectors of its cut: Zip-Up is then the sequential truncated SVD of the dense state."""
    p = random_problem(chain_parent(n), d, chi, 1, mb, seed=seed)
    state = _canonical_toward_leaf(p.state)
    op = _identity_chain_op(n, d)
    psi = tn.to_dense(p.parent, state).reshape(-1)
    got = tn.to_dense(p.parent, zipup_tree(p.parent, state, op, mb)).reshape(-1)
    ref = _tt_svd_from_leaf(psi, [d] * n, mb)
    assert np.linalg.norm(got - psi) > 1e-3 * np.linalg.norm(psi)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(psi)


def test_zipup_two_site_brute_force():
    """Root and one leaf with d above the target bond: the leaf keeps the top left singular vectors
    of its own product tensor (sigma') x (alpha, beta) and the result is O|psi> with that projector
    on the leaf's physical leg."""
    p = random_problem(chain_parent(2), 6, 3, 2, 2, seed=13)
    t1, w1 = p.state[1], p.op[1]                              # (s, a), (s', s, b)
    loc = np.einsum("usb,sa->uab", w1, t1).reshape(t1.shape[0], -1)
    u = np.linalg.svd(loc, full_matrices=False)[0][:, :2]
    phi = dense_phi(p).reshape(p.phys)
    ref = np.einsum("xk,yk,sy->sx", u, u.conj(), phi)
    got = tn.to_dense(p.parent, zipup_tree(p.parent, p.state, p.op, 2))
    assert np.linalg.norm(got.reshape(-1) - ref.reshape(-1)) <= 1e-12 * np.linalg.norm(phi)
