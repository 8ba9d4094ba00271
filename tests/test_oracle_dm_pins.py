"""Pins for the DM oracle (oracle/dm.py): checks against what the method and the mathematics fix,
never against the oracle itself. CPU only, small dense systems."""
import numpy as np
import pytest

from oracle import tn
from oracle.dm import dm_tree
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


def dense_dm(p, max_bond):
    """DM written with dense unfoldings: at every non-root node (leaves first) the unfolding of
    O|psi> between (sigma_i, the children's subtrees) and the rest, each child's subtree indices
    projected onto that child's basis; the node's basis is the top max_bond left singular vectors
    (identity where the rows do not exceed max_bond). The result is O|psi> with the basis projectors
    of the root's children applied."""
    n, parent = p.n, p.parent
    phi = dense_phi(p).reshape(p.phys)
    ch = [[c for c, q in enumerate(parent) if q == i] for i in range(n)]
    root = parent.index(-1)
    U = {}
    for i in tn.postorder(parent):
        if i == root:
            continue
        order = [i] + [j for c in ch[i] for j in subtree(parent, c)]
        rest = [j for j in range(n) if j not in order]
        m = np.transpose(phi, order + rest)
        m = m.reshape([p.phys[i]] + [int(np.prod([p.phys[j] for j in subtree(parent, c)]))
                                     for c in ch[i]] + [-1])
        for pos, c in enumerate(ch[i]):
            m = np.moveaxis(np.tensordot(U[c][0].conj(), m, axes=([0], [1 + pos])), 0, 1 + pos)
        rows = int(np.prod(m.shape[:-1]))
        if rows <= max_bond:
            q = np.eye(rows, dtype=np.complex128)
        else:
            u, s, _ = np.linalg.svd(m.reshape(rows, -1), full_matrices=False)
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
def test_dm_dense_formulation(name, parent, phys, chi, D, mb, seed):
    """The environment sweeps equal the dense formulation (top singular vectors of unfoldings)."""
    p = random_problem(parent, phys, chi, D, mb, seed=seed)
    got = tn.to_dense(p.parent, dm_tree(p.parent, p.state, p.op, mb)).reshape(-1)
    ref, phi = dense_dm(p, mb)
    assert np.linalg.norm(got - phi) > 1e-3 * np.linalg.norm(phi)        # really truncating
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(phi)


@pytest.mark.parametrize("name,parent,phys,chi,D,mb,seed", CASES, ids=[c[0] for c in CASES])
def test_dm_projection_isometries_and_truncation_bounds(name, parent, phys, chi, D, mb, seed):
    """The result is an orthogonal projection of O|psi>, every non-root node is an isometry, and
    the error lies between the largest optimal tail of a single cut and the root of the sum of the
    cuts' squared tails (each cut is truncated optimally for the state it sees, whose singular
    values the earlier projections can only lower)."""
    p = random_problem(parent, phys, chi, D, mb, seed=seed)
    out = dm_tree(p.parent, p.state, p.op, mb)
    phi = dense_phi(p)
    psi = tn.to_dense(p.parent, out)
    assert abs(np.vdot(phi, psi) - np.vdot(psi, psi)) <= 1e-12 * np.vdot(phi, phi).real
    root = p.parent.index(-1)
    err = np.linalg.norm(phi - psi)
    tails = []
    for i in range(p.n):
        if i == root:
            continue
        assert tn.isometry_error(out[i]) <= 1e-12
        sub = subtree(p.parent, i)
        rest = [j for j in range(p.n) if j not in sub]
        m = np.transpose(phi, sub + rest).reshape(int(np.prod([p.phys[j] for j in sub])), -1)
        s = np.linalg.svd(m, compute_uv=False)
        tails.append(np.sqrt(np.sum(s[out[i].shape[1]:] ** 2)))
    assert err >= max(tails) * (1 - 1e-10)
    assert err <= np.sqrt(np.sum(np.square(tails))) * (1 + 1e-10)


def test_dm_exact_when_the_bond_covers_every_rank():
    """With target bond at least every rank (chi * D = 4 per bond, target 5) the result is O|psi>,
    for a chain with d = 8 (rows above the target, so the eigenvector path is taken) and a tree."""
    p = random_problem(chain_parent(4), 8, 2, 2, 5, seed=9)
    out = dm_tree(p.parent, p.state, p.op, 5)
    assert any(t.shape[1] == 5 for t in out)
    phi = dense_phi(p)
    assert np.linalg.norm(tn.to_dense(p.parent, out) - phi) <= 1e-12 * np.linalg.norm(phi)
    tree = random_problem(kary_parent(4, 3), 6, 2, 2, 5, seed=10)
    out = dm_tree(tree.parent, tree.state, tree.op, 5)
    phi = dense_phi(tree)
    assert np.linalg.norm(tn.to_dense(tree.parent, out) - phi) <= 1e-12 * np.linalg.norm(phi)


def test_dm_two_site_is_the_optimal_truncation():
    """On two sites there is one cut: DM keeps the top singular vectors of O|psi>'s unfolding, the
    optimal truncation (Eckart-Young), so the error equals the tail exactly."""
    p = random_problem(chain_parent(2), 6, 6, 6, 3, seed=12)
    out = dm_tree(p.parent, p.state, p.op, 3)
    phi = dense_phi(p).reshape(6, 6)
    s = np.linalg.svd(phi, compute_uv=False)
    err = np.linalg.norm(tn.to_dense(p.parent, out).reshape(6, 6) - phi)
    assert abs(err - np.sqrt(np.sum(s[3:] ** 2))) <= 1e-12 * np.linalg.norm(phi)
