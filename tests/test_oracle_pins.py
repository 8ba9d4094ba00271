"""Pins for the oracle: checks against what the paper and the mathematics fix, never against the
oracle's own formulas retyped.

Each test names the property it pins and the part of the oracle a plausible mistake would break.
"""
import math

import numpy as np
import pytest

from oracle import cbc_tree, cbc_tt, truncate_joined, lq, tn
from paper_2601_19650_amd.inputs import (chain_parent, config_problem, kary_parent,
                                         random_problem)


def dense_phi(p):
    return tn.apply_dense(p.parent, p.op, tn.to_dense(p.parent, p.state))


def dense_err(p, out):
    phi = dense_phi(p)
    psi = tn.to_dense(p.parent, out)
    rel = np.linalg.norm(phi - psi) / np.linalg.norm(phi)
    fid = abs(np.vdot(phi, psi)) ** 2 / (np.vdot(phi, phi).real * np.vdot(psi, psi).real)
    return rel, 1.0 - fid, phi, psi


# ---------------------------------------------------------------------------------------------
# P1: exact reproduction when max_bond covers every rank (brute force dense contraction)

def test_c1_exact_dense():
    """The C1 workload (8-site MPS, chi=8, D=4, max_bond=32) reproduces O|psi> exactly."""
    p = config_problem("C1")
    out = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    rel, infid, _, _ = dense_err(p, out)
    assert rel <= 1e-12 and infid <= 1e-12


@pytest.mark.parametrize("kind,n,d,chi,D", [
    ("binary", 7, 2, 4, 3), ("ternary", 7, 2, 4, 2), ("binary", 10, 2, 3, 3),
    ("mps", 9, 3, 5, 2), ("ternary", 4, 3, 3, 2)])
def test_exact_trees_dense(kind, n, d, chi, D):
    parent = {"mps": chain_parent(n), "binary": kary_parent(n, 2), "ternary": kary_parent(n, 3)}[kind]
    p = random_problem(parent, d, chi, D, 10 ** 6, seed=11 + n)
    out = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    rel, infid, _, _ = dense_err(p, out)
    assert rel <= 1e-12 and infid <= 1e-12


def test_exact_with_d1_internal_nodes():
    """Tree nodes without a physical leg (d_i = 1, Sec. II A) are handled."""
    parent = kary_parent(7, 2)
    phys = [1, 1, 1, 2, 2, 2, 2]
    p = random_problem(parent, phys, 4, 4, 10 ** 6, seed=3)
    out = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    rel, infid, _, _ = dense_err(p, out)
    assert rel <= 1e-12


def test_tt_formulation_equals_tree_formulation():
    """Sec. III A (tensor train) and Sec. III B (tree, rooted at the first site) agree on chains."""
    p = config_problem("C2", n=12, max_bond=12)
    a = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    b = tn.mps_to_tree(cbc_tt(tn.tree_to_mps(p.state), tn.tree_to_mpo(p.op), p.max_bond))
    assert tn.rel_error(p.parent, b, a) <= 1e-11


# ---------------------------------------------------------------------------------------------
# P2/P3: projection and isometry invariants (hold for any truncation)

@pytest.mark.parametrize("kind,n,d,chi,D,mb", [
    ("mps", 8, 2, 8, 4, 5), ("binary", 7, 2, 8, 4, 4), ("ternary", 7, 2, 6, 3, 3),
    ("binary", 9, 2, 6, 4, 3)])
def test_projection_property_dense(kind, n, d, chi, D, mb):
    """psi' is an orthogonal projection of Phi: <psi'|Phi> = ||psi'||^2 and
    ||Phi - psi'||^2 = ||Phi||^2 - ||psi'||^2."""
    parent = {"mps": chain_parent(n), "binary": kary_parent(n, 2), "ternary": kary_parent(n, 3)}[kind]
    p = random_problem(parent, d, chi, D, mb, seed=100 + n)
    out = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    rel, _, phi, psi = dense_err(p, out)
    assert rel > 1e-3                           # really truncating
    ov = np.vdot(psi, phi)
    nn = np.vdot(psi, psi).real
    assert abs(ov - nn) <= 1e-12 * np.vdot(phi, phi).real
    lhs = np.linalg.norm(phi - psi) ** 2
    rhs = np.vdot(phi, phi).real - nn
    assert abs(lhs - rhs) <= 1e-12 * np.vdot(phi, phi).real


def test_projection_and_isometry_mid_size():
    """Same invariants on a 24-site chain and a 15-node binary tree via network contractions."""
    for p in [config_problem("C2", n=24), config_problem("C3", n=15)]:
        out = cbc_tree(p.parent, p.state, p.op, p.max_bond)
        root = p.parent.index(-1)
        for i, t in enumerate(out):
            if i != root:
                assert tn.isometry_error(t) <= 1e-13
        phi2 = tn.applied_norm_sq(p.parent, p.op, p.state)
        psi2 = tn.norm_sq(p.parent, out)
        # ||psi'|| equals the root tensor's Frobenius norm when all other nodes are isometries
        assert abs(psi2 - np.linalg.norm(out[root]) ** 2) <= 1e-12 * psi2
        # <psi'|Phi> through the exact product network
        prod = tn.product_ttn(p.parent, p.op, p.state)
        v, l = tn.overlap(p.parent, out, prod)
        ov = v * math.exp(l)
        assert abs(ov.imag) <= 1e-11 * phi2
        assert abs(ov.real - psi2) <= 1e-11 * phi2
        assert psi2 < phi2


# ---------------------------------------------------------------------------------------------
# P4: the truncation step against textbook identities

def test_truncation_step_identities():
    rng = np.random.default_rng(0)
    lp = rng.standard_normal((6, 4, 5, 7)) + 1j * rng.standard_normal((6, 4, 5, 7))
    m = lp.reshape(24, 35)
    k = 9
    lt = truncate_joined(lp, 2, k, 0.0)
    assert lt.shape == (k, 5, 7)
    lmat = lt.reshape(k, 35)
    # rows are orthogonal with norms equal to the top-k singular values of the joined matrix
    s = np.linalg.svd(m, compute_uv=False)
    g = lmat @ lmat.conj().T
    assert np.allclose(np.diag(g).real, s[:k] ** 2, rtol=1e-12)
    assert np.abs(g - np.diag(np.diag(g))).max() <= 1e-12 * s[0] ** 2
    # L^dagger L is M^dagger P_k M with P_k the projector on the top-k left singular subspace
    w, u = np.linalg.eigh(m @ m.conj().T)
    uk = u[:, ::-1][:, :k]
    assert np.allclose(lmat.conj().T @ lmat, m.conj().T @ uk @ uk.conj().T @ m, atol=1e-12 * s[0] ** 2)
    # tolerance: keep only s_j > tol * s_0
    tol = s[4] / s[0] * 1.0000001
    assert truncate_joined(lp, 2, k, tol).shape[0] == 4


def test_lq_step():
    rng = np.random.default_rng(1)
    for shape in [(5, 12), (12, 5), (7, 7)]:
        s = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        q = lq(s)
        assert q.shape == (min(shape), shape[1])
        assert np.allclose(q @ q.conj().T, np.eye(min(shape)), atol=1e-14)
        # rows of Q span the row space of S: S = (S Q^dagger) Q
        assert np.allclose(s @ q.conj().T @ q, s, atol=1e-13)


# ---------------------------------------------------------------------------------------------
# P5: Eckart-Young lower bound at every cut (dense)

def _cut_tails(phi, parent, max_bond):
    """For every edge, the Frobenius norm of the singular values beyond max_bond of Phi across it."""
    n = len(parent)
    tails = []
    for i in range(n):
        if parent[i] < 0:
            continue
        sub = set()
        stack = [i]
        while stack:
            j = stack.pop()
            sub.add(j)
            stack += [c for c, pp in enumerate(parent) if pp == j]
        inside = sorted(sub)
        outside = [j for j in range(n) if j not in sub]
        mat = np.transpose(phi, inside + outside).reshape(
            int(np.prod([phi.shape[j] for j in inside])), -1)
        s = np.linalg.svd(mat, compute_uv=False)
        tails.append(math.sqrt(float(np.sum(s[max_bond:] ** 2))))
    return tails


@pytest.mark.parametrize("kind,n,mb", [("mps", 8, 4), ("binary", 7, 3), ("ternary", 7, 3)])
def test_eckart_young_bounds(kind, n, mb):
    parent = {"mps": chain_parent(n), "binary": kary_parent(n, 2), "ternary": kary_parent(n, 3)}[kind]
    p = random_problem(parent, 2, 8, 4, mb, seed=21)
    out = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    phi = dense_phi(p)
    tails = _cut_tails(phi, p.parent, mb)
    err_cbc = np.linalg.norm(phi - tn.to_dense(p.parent, out))
    err_svd = np.linalg.norm(phi - tn.to_dense(p.parent, tn.naive_compress(p.parent, p.op, p.state, mb)))
    assert err_cbc >= max(tails) * (1 - 1e-12)
    # the naive sweep obeys the hierarchical-SVD bounds: max tail <= err <= sqrt(sum of tails^2)
    assert max(tails) * (1 - 1e-12) <= err_svd <= math.sqrt(sum(t * t for t in tails)) * (1 + 1e-12)
    # paper: CBC is slightly less accurate than direct compression at a given bond dimension
    assert 0.5 <= err_cbc / err_svd <= 5.0


# ---------------------------------------------------------------------------------------------
# P6: N = 2 closed form.  psi' = Phi Pi_{rowspace(U_k^dagger Phi)} with U_k the top-k left singular
# vectors of the first site's product block A_1 (d x chi D).

def test_two_site_closed_form():
    p = random_problem(chain_parent(2), 5, 5, 5, 3, seed=5)
    t1, t2 = p.state
    w1, w2 = p.op
    # build the blocks independently of the oracle's contraction code
    d = 5
    A1 = np.zeros((d, t1.shape[2] * w1.shape[3]), dtype=complex)
    for sp in range(d):
        for s in range(d):
            A1[sp] += np.kron(t1[s, 0, :], w1[sp, s, 0, :])
    B2 = np.zeros((t2.shape[1] * w2.shape[2], d), dtype=complex)
    for sp in range(d):
        for s in range(d):
            B2[:, sp] += np.kron(t2[s, :], w2[sp, s, :])
    phi = A1 @ B2
    assert np.allclose(phi, dense_phi(p))
    u, _, _ = np.linalg.svd(A1)
    uk = u[:, :3]
    x = uk.conj().T @ phi
    _, sx, vxh = np.linalg.svd(x)
    r = int(np.count_nonzero(sx > 1e-12 * sx[0]))
    proj = vxh[:r].conj().T @ vxh[:r]
    expect = phi @ proj
    out = cbc_tree(p.parent, p.state, p.op, 3)
    got = tn.to_dense(p.parent, out)
    assert np.linalg.norm(got - expect) <= 1e-12 * np.linalg.norm(phi)
    assert np.linalg.norm(got - phi) > 1e-3 * np.linalg.norm(phi)


# ---------------------------------------------------------------------------------------------
# P7: covariances

def _gauge(p, rng, unitary=True):
    """Insert X X^{-1} on every state bond and Y Y^{-1} on every operator bond."""
    ch = [[j for j, q in enumerate(p.parent) if q == i] for i in range(p.n)]
    st = [t.copy() for t in p.state]
    op = [w.copy() for w in p.op]
    for i in range(p.n):
        par = p.parent[i]
        if par < 0:
            continue
        slot = 2 + ch[par].index(i)
        for tens, ax_child, ax_par, dim in [(st, 1, slot, p.chi[i]), (op, 2, slot + 1, p.dop[i])]:
            z = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
            if unitary:
                x, _ = np.linalg.qr(z)
                xi = x.conj().T
            else:
                x = z + 3 * np.eye(dim)
                xi = np.linalg.inv(x)
            # parent side gets X (on its child leg), child side gets X^{-1} (on its parent leg)
            tens[par] = np.moveaxis(np.tensordot(tens[par], x, axes=([ax_par], [0])), -1, ax_par)
            tens[i] = np.moveaxis(np.tensordot(xi, tens[i], axes=([1], [ax_child])), 0, ax_child)
    return st, op


@pytest.mark.parametrize("kind,n", [("mps", 8), ("binary", 7)])
def test_unitary_gauge_invariance(kind, n):
    parent = chain_parent(n) if kind == "mps" else kary_parent(n, 2)
    p = random_problem(parent, 2, 6, 3, 4, seed=31)
    rng = np.random.default_rng(9)
    st, op = _gauge(p, rng, unitary=True)
    assert np.allclose(tn.to_dense(p.parent, st), tn.to_dense(p.parent, p.state))
    a = tn.to_dense(p.parent, cbc_tree(p.parent, p.state, p.op, p.max_bond))
    b = tn.to_dense(p.parent, cbc_tree(p.parent, st, op, p.max_bond))
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
    # a non-unitary gauge represents the same product but generally changes a truncating CBC
    st2, op2 = _gauge(p, rng, unitary=False)
    c = tn.to_dense(p.parent, cbc_tree(p.parent, st2, op2, p.max_bond))
    assert np.linalg.norm(a - c) > 1e-8 * np.linalg.norm(a)


def test_scalar_covariance():
    p = config_problem("C3", n=15)
    out = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    c, c2 = 2.5 - 1.0j, 0.3j
    st = [t.copy() for t in p.state]
    op = [w.copy() for w in p.op]
    st[4] *= c
    op[9] *= c2
    out2 = cbc_tree(p.parent, st, op, p.max_bond)
    root = p.parent.index(-1)
    ref = [t.copy() for t in out]
    ref[root] = ref[root] * (c * c2)
    assert tn.rel_error(p.parent, out2, ref) <= 1e-12


# ---------------------------------------------------------------------------------------------
# P8: special cases

def test_identity_operator_returns_state():
    p = config_problem("C3", n=15)
    ident = []
    for i in range(p.n):
        k = len(p.children(i))
        d = p.phys[i]
        ident.append(np.eye(d, dtype=complex).reshape((d, d) + (1,) * (1 + k)))
    out = cbc_tree(p.parent, p.state, ident, max(p.chi))
    assert tn.rel_error(p.parent, out, p.state) <= 1e-12


def test_product_state_product_operator():
    p = random_problem(kary_parent(10, 3), 3, 1, 1, 4, seed=2)
    out = cbc_tree(p.parent, p.state, p.op, p.max_bond)
    assert all(max(t.shape[1:], default=1) == 1 for t in out)
    rel, _, _, _ = dense_err(p, out)
    assert rel <= 1e-13


def test_tolerance_reduces_bonds():
    p = config_problem("C2", n=16)
    full = cbc_tree(p.parent, p.state, p.op, 64)
    tl = cbc_tree(p.parent, p.state, p.op, 64, tol=0.5)
    assert sum(t.size for t in tl) < sum(t.size for t in full)
    # still a projection of the same product, hence no larger than it
    assert tn.norm_sq(p.parent, tl) <= tn.norm_sq(p.parent, full) * (1 + 1e-12)


# ---------------------------------------------------------------------------------------------
# P9: independent dense formulation of the tensor-train sweep on truncating tiny chains.
# Forward:  P_i = (P_{i-1} (x) 1_d) U_i, U_i = top-k_i left singular vectors of (P_{i-1}^+ (x) 1_d) A_i,
#           A_i the d^i x (chi_i D_i) left block of the product network.
# Backward: W_N = rowspace(P_{N-1}^+ Phi[N-1|N]); W_i = rowspace(P_{i-1}^+ Phi[i-1|..] (1_d (x) Pi_{W_{i+1}}));
#           psi' = Phi (1_d (x) Pi_{W_2}).

def _dense_cbc_chain(p, max_bond):
    n = p.n
    d = p.phys[0]
    # left blocks A_i by brute force from the dense product of the first i sites
    mps = tn.tree_to_mps(p.state)
    mpo = tn.tree_to_mpo(p.op)
    blk = np.ones((1, 1), dtype=complex)                 # (phys..., (alpha,beta))
    blocks = []
    for i in range(n):
        t, w = mps[i], mpo[i]
        prod = np.zeros((d, t.shape[1] * w.shape[2], t.shape[2] * w.shape[3]), dtype=complex)
        for sp in range(d):
            for s in range(d):
                prod[sp] += np.kron(t[s], w[sp, s])
        # blk: (D_prev_phys, left bond) ; new: (prev_phys * d, right bond)
        blk = np.einsum("xl,slr->xsr", blk, prod).reshape(blk.shape[0] * d, -1)
        blocks.append(blk)
    phi = blocks[-1].reshape(-1)
    ps = [np.ones((1, 1), dtype=complex)]
    for i in range(n - 1):
        a = blocks[i]
        m = np.kron(ps[-1].conj().T, np.eye(d)) @ a
        u, s, _ = np.linalg.svd(m, full_matrices=False)
        k = min(max_bond, len(s))
        ps.append(np.kron(ps[-1], np.eye(d)) @ u[:, :k])
    proj = None
    for i in range(n, 1, -1):          # 1-based site i
        pm = phi.reshape(d ** (i - 1), d ** (n - i + 1))
        x = ps[i - 1].conj().T @ pm
        if proj is not None:
            x = x @ np.kron(np.eye(d), proj)
        _, s, vh = np.linalg.svd(x, full_matrices=False)
        r = min(x.shape)
        proj = vh[:r].conj().T @ vh[:r]
    return phi.reshape(d, -1) @ proj


@pytest.mark.parametrize("n,d,chi,D,mb", [(6, 2, 4, 3, 3), (7, 2, 6, 2, 4), (5, 3, 4, 2, 3)])
def test_dense_reformulation_chain(n, d, chi, D, mb):
    p = random_problem(chain_parent(n), d, chi, D, mb, seed=40 + n)
    got = tn.to_dense(p.parent, cbc_tree(p.parent, p.state, p.op, mb)).reshape(-1)
    ref = _dense_cbc_chain(p, mb).reshape(-1)
    phi = dense_phi(p).reshape(-1)
    assert np.linalg.norm(got - phi) > 1e-3 * np.linalg.norm(phi)
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(phi)


# ---------------------------------------------------------------------------------------------
# P9b: independent dense formulation of tree CBC (Sec. III B) on truncating trees of up to 12
# nodes, written with subspaces of the physical space instead of environment tensors.
#   Cutting the edge of node i from its parent splits O|psi> = sum_{alpha beta} A_i B_i, with A_i
#   the product network contracted over the subtree sub(i) and B_i over the rest out(i), both
#   contracted here by brute force from the input tensors.
#   Sweep 1 (Eq. cbc_tree_first_contraction): P_i = (1_{d_i} (x) P_c ...) U_i, an isometry into the
#     physical space of sub(i), with U_i the top-k left singular vectors of (1 (x) P_c^H ...) A_i.
#   Sweep 2 (Eq. cbc_tree_second_contraction): Q_k = (1_{d_i} (x) Q_i (x) P_c ..., c != k) U, an
#     isometry into the physical space of out(k), U from (1 (x) Q_i^H (x) P_c^H ...) B_k.
#   Sweep 3 (Eqs. cbc_tree_third_contraction, cbc_tree_qr, cbc_final_contraction): the output
#     isometry of node i spans the column space of (1_{d_i} (x) Pi_c ...) Phi_i^T conj(Q_i), with
#     Phi_i = O|psi> read as out(i) x sub(i) and Pi_c the children's output projectors; the root
#     keeps (1 (x) Pi_c ...) O|psi>.
# A leg order, conjugate or environment mistake at a node with several children changes which
# subspace is kept, which the projection invariants alone do not see.

def _ein(*args):
    """einsum over arbitrary hashable labels: _ein(t1, labels1, t2, labels2, ..., out_labels)."""
    *pairs, out = args
    ids = {}

    def m(ls):
        return [ids.setdefault(l, len(ids)) for l in ls]

    ops = []
    for k in range(0, len(pairs), 2):
        ops += [pairs[k], m(pairs[k + 1])]
    return np.einsum(*ops, m(out), optimize="greedy")


def _subtree(parent, i):
    s, st = set(), [i]
    while st:
        j = st.pop()
        s.add(j)
        st += [c for c, q in enumerate(parent) if q == j]
    return sorted(s)


def _block(p, nodes, edge):
    """The product network contracted over `nodes`; open legs sigma'_j (j in nodes) and, unless
    edge is None, the state and operator legs of the edge from node `edge` to its parent."""
    ch = [[c for c, q in enumerate(p.parent) if q == i] for i in range(p.n)]
    args = []
    for j in nodes:
        up_a = ("a", j) if p.parent[j] >= 0 else ("ra",)
        up_b = ("b", j) if p.parent[j] >= 0 else ("rb",)
        args += [p.state[j], [("s", j), up_a] + [("a", c) for c in ch[j]]]
        args += [p.op[j], [("sp", j), ("s", j), up_b] + [("b", c) for c in ch[j]]]
    if p.parent.index(-1) in nodes:
        args += [np.ones(1), [("ra",)], np.ones(1), [("rb",)]]
    out = [("sp", j) for j in nodes] + ([] if edge is None else [("a", edge), ("b", edge)])
    return _ein(*args, out)


def _top_left(t, nrow, k):
    """Top-k left singular vectors of t read as (first nrow legs) x (rest), as a tensor."""
    u, s, _ = np.linalg.svd(t.reshape(int(np.prod(t.shape[:nrow])), -1), full_matrices=False)
    kk = min(k, len(s))
    return u[:, :kk].reshape(t.shape[:nrow] + (kk,))


def _project(x, lab, w, legs, tag):
    """Apply W W^H (W an isometry with legs `legs` + [tag]) to the legs `legs` of x."""
    rest = [l for l in lab if l not in legs]
    t = _ein(x, lab, w.conj(), legs + [tag], rest + [tag])
    return _ein(t, rest + [tag], w, legs + [tag], lab)


def _dense_cbc_tree(p, max_bond):
    n, parent = p.n, p.parent
    ch = [[c for c, q in enumerate(parent) if q == i] for i in range(n)]
    root = parent.index(-1)
    sub = {i: _subtree(parent, i) for i in range(n)}
    out = {i: [j for j in range(n) if j not in sub[i]] for i in range(n)}
    sp = lambda nodes: [("sp", j) for j in nodes]
    post = tn.postorder(parent)
    P = {}
    for i in post:                                  # sweep 1
        if i == root:
            continue
        args, rows = [_block(p, sub[i], i), sp(sub[i]) + ["a", "b"]], [("sp", i)]
        for c in ch[i]:
            args += [P[c].conj(), sp(sub[c]) + [("x", c)]]
            rows.append(("x", c))
        U = _top_left(_ein(*args, rows + ["a", "b"]), len(rows), max_bond)
        args = [U, rows + [("x", i)]]
        for c in ch[i]:
            args += [P[c], sp(sub[c]) + [("x", c)]]
        P[i] = _ein(*args, sp(sub[i]) + [("x", i)])
    Q = {}
    for i in reversed(post):                        # sweep 2
        for k in ch[i]:
            args, rows = [_block(p, out[k], k), sp(out[k]) + ["a", "b"]], [("sp", i)]
            basis = []
            if i != root:
                basis.append((Q[i], sp(out[i]) + [("y", i)]))
            basis += [(P[c], sp(sub[c]) + [("x", c)]) for c in ch[i] if c != k]
            for t, lab in basis:
                args += [t.conj(), lab]
                rows.append(lab[-1])
            U = _top_left(_ein(*args, rows + ["a", "b"]), len(rows), max_bond)
            args = [U, rows + [("y", k)]]
            for t, lab in basis:
                args += [t, lab]
            Q[k] = _ein(*args, sp(out[k]) + [("y", k)])
    phi = _block(p, list(range(n)), None)
    W = {}
    for i in post:                                  # sweep 3
        if i == root:
            continue
        lab = sp(sub[i]) + [("y", i)]
        x = _ein(phi, sp(range(n)), Q[i].conj(), sp(out[i]) + [("y", i)], lab)
        for c in ch[i]:
            x = _project(x, lab, W[c], sp(sub[c]), ("z", c))
        u, s, _ = np.linalg.svd(x.reshape(-1, x.shape[-1]), full_matrices=False)
        r = int(np.count_nonzero(s > 1e-10 * s[0]))
        rest = p.phys[i] * int(np.prod([W[c].shape[-1] for c in ch[i]]))
        assert r == min(x.shape[-1], rest)          # generic: S has full rank
        W[i] = u[:, :r].reshape(x.shape[:-1] + (r,))
    res = phi
    for c in ch[root]:
        res = _project(res, sp(range(n)), W[c], sp(sub[c]), ("z", c))
    return res.reshape(-1), phi.reshape(-1)


@pytest.mark.parametrize("parent,phys,chi,D,mb,seed", [
    (kary_parent(7, 2), 2, 4, 3, 3, 1),
    (kary_parent(10, 3), 2, 4, 2, 3, 2),
    (kary_parent(7, 2), [1, 1, 1, 2, 2, 2, 2], 4, 3, 3, 3),
    ([-1, 0, 0, 1, 1, 1, 2, 2, 6], 2, 4, 3, 3, 4),
    (kary_parent(12, 2), 2, 4, 2, 3, 5),
    (chain_parent(7), 2, 4, 3, 3, 6)],
    ids=["bin7", "ter10", "bin7-d1-internal", "uneven9", "bin12", "chain7"])
def test_dense_reformulation_tree(parent, phys, chi, D, mb, seed):
    p = random_problem(parent, phys, chi, D, mb, seed=seed)
    got = tn.to_dense(p.parent, cbc_tree(p.parent, p.state, p.op, mb)).reshape(-1)
    ref, phi = _dense_cbc_tree(p, mb)
    assert np.linalg.norm(got - phi) > 1e-3 * np.linalg.norm(phi)      # really truncating
    assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(phi)


# ---------------------------------------------------------------------------------------------
# metric utilities against dense forms

def test_metrics_against_dense():
    p = random_problem(kary_parent(8, 2), 2, 4, 3, 3, seed=77)
    out = cbc_tree(p.parent, p.state, p.op, 3)
    a = tn.to_dense(p.parent, out)
    b = tn.to_dense(p.parent, p.state)
    v, l = tn.overlap(p.parent, out, p.state)
    assert abs(v * math.exp(l) - np.vdot(a, b)) <= 1e-13
    assert abs(tn.diff_norm(p.parent, out, p.state) - np.linalg.norm(a - b)) <= 1e-13
    assert abs(tn.canonical_norm(p.parent, out) - np.linalg.norm(a)) <= 1e-13
    phi = dense_phi(p)
    assert abs(tn.applied_norm_sq(p.parent, p.op, p.state) - np.vdot(phi, phi).real) <= 1e-12
    prod = tn.product_ttn(p.parent, p.op, p.state)
    assert np.allclose(tn.to_dense(p.parent, prod), phi, atol=1e-14)
    f = tn.fidelity(p.parent, out, p.state)
    assert abs(f - abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)) <= 1e-12


def test_naive_exact_case():
    p = config_problem("C1")
    out = tn.naive_compress(p.parent, p.op, p.state, 64)
    rel, _, _, _ = dense_err(p, out)
    assert rel <= 1e-12
