"""Oracle for successive randomised compression (SRC) on trees: plain, slow, complex128 NumPy.

TEST INFRASTRUCTURE ONLY, like oracle/cbc.py: the reference the GPU library's SRC path is checked
against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the library never calls it. It shares no code with the GPU path.

What it computes (arXiv 2601.19650, Sec. III C): SRC is the randomised counterpart of CBC. One
random matrix of size d x D-bar per site, combined over sites by the Khatri-Rao product, sketches
the part of O|psi> outside the node being compressed; the compression then needs only contractions
and a QR, no SVD. The paper describes the method in words (it cites the tensor-train algorithm and
compares with it); the steps below restate it on the tree sweeps of Sec. III B:
  * sweep 1, leaves to root: the sketch K^{[i]} of the subtree below node i, the exact contraction of
    that subtree of O|psi> with the sketch matrices on its output physical legs (legs: alpha_i and
    beta_i toward the parent, and the sketch index r);
  * sweep 2, root to leaves: the sketch E^{[k]} of everything outside the subtree of k, from the
    parent's node tensors, the parent's own E and the K of k's siblings (legs alpha_k, beta_k, r);
  * sweep 3, leaves to root, as in CBC (Eqs. cbc_tree_third_contraction, cbc_final_contraction):
    Z^{[i]} = T W prod_c R^{[c]}; the new basis of node i spans the columns of Y = Z^{[i]} E^{[i]}
    (rows: sigma' and the children's new bonds; columns: r), from a thin QR; R^{[i]} = Q^H Z^{[i]};
    the root keeps Z.

Readings taken where the paper is silent:
  * the sketch matrix of node i, Omega_i (d_i x D-bar, d_i the physical dimension), acts on the
    output physical leg sigma'_i without conjugation; the sketch of a set of nodes is the Khatri-Rao
    product of theirs: column r is the product state with factors Omega_k[:, r];
  * the sketch width is the target bond D-bar (no oversampling), and the random numbers are inputs;
  * the new bond of node i is k = min(D-bar, rows); where rows <= D-bar there is nothing to compress
    and the basis is the identity (the columns of Y span everything for a generic sketch);
  * legs and storage order as in oracle/cbc.py: (sigma, parent, children...) for states,
    (sigma', sigma, parent, children...) for operators.

Parity pins (tests/test_oracle_src_pins.py): an independent dense formulation (unfoldings of the
dense O|psi> times the Khatri-Rao sketch of the complement, children projected onto their bases),
exactness when the sketch covers every rank, the orthogonal-projection property, isometries,
invariance under per-column rescaling and permutation of the sketch, and the Eckart-Young lower
bound at every cut; tests/test_oracle_mutations.py plants mistakes here and checks they fail.
"""
from __future__ import annotations

import numpy as np

from oracle.cbc import _children, _node_contraction, _pairwise, _postorder

__all__ = ["src_tree"]


def _sketch_node(t, w, om, envs, open_slot):
    """Node i with its output physical leg sketched: T_i, the sketch environments ``envs`` (slot ->
    tensor (alpha, beta, r)), W_i and Omega_i contracted, the slot ``open_slot`` left open. The
    sketch index r is shared by Omega_i and every environment (Khatri-Rao product). Result legs
    (alpha_open, beta_open, r). Slots that are neither open nor given an environment have dimension
    1 (the root's parent leg)."""
    nslot = t.ndim - 1
    sig, sigp, r = 0, 1, 2
    alpha = [3 + j for j in range(nslot)]
    beta = [3 + nslot + j for j in range(nslot)]
    terms = [(t, [sig] + alpha)]
    for slot in sorted(envs):
        terms.append((envs[slot], [alpha[slot], beta[slot], r]))
    terms.append((w, [sigp, sig] + beta))
    terms.append((om, [sigp, r]))
    return _pairwise(terms, [alpha[open_slot], beta[open_slot], r])


def src_tree(parent, state, op, max_bond, sketch):
    """SRC on the tree ``parent`` with sketch matrices ``sketch[i]`` (d_i x max_bond); returns the
    new node tensors (sigma', parent, children...)."""
    n = len(parent)
    ch = _children(parent)
    root = parent.index(-1)
    post = _postorder(parent)
    pre = list(reversed(post))
    for i in range(n):
        assert sketch[i].shape == (state[i].shape[0], max_bond), "sketch is d_i x max_bond"

    # sweep 1, leaves to root: sketches of the subtrees
    ksub = {}
    for i in post:
        if i == root:
            continue
        envs = {1 + j: ksub[c] for j, c in enumerate(ch[i])}
        ksub[i] = _sketch_node(state[i], op[i], sketch[i], envs, 0)

    # sweep 2, root to leaves: sketches of the rest of the tree
    epar = {}
    for i in pre:
        for kpos, k in enumerate(ch[i]):
            envs = {}
            if i != root:
                envs[0] = epar[i]
            for j, c in enumerate(ch[i]):
                if c != k:
                    envs[1 + j] = ksub[c]
            epar[k] = _sketch_node(state[i], op[i], sketch[i], envs, 1 + kpos)

    # sweep 3, leaves to root: bases from the sketched columns, environments R = Q^H Z
    renv = {}
    out = [None] * n
    for i in post:
        envs = {1 + j: renv[c] for j, c in enumerate(ch[i])}
        z = _node_contraction(state[i], op[i], envs, 0, None)   # (sigma', chi_c..., alpha_p, beta_p)
        shp = z.shape
        rows = int(np.prod(shp[:-2]))
        if i == root:
            out[i] = z.reshape(shp[:-2])[:, None]                 # (sigma', 1, chi_c...)
            continue
        zm = z.reshape(rows, shp[-2] * shp[-1])
        if rows <= max_bond:
            q = np.eye(rows, dtype=np.complex128)
        else:
            y = zm @ epar[i].reshape(shp[-2] * shp[-1], max_bond)
            q, _ = np.linalg.qr(y, mode="reduced")
        k = q.shape[1]
        out[i] = np.moveaxis(q.reshape(shp[:-2] + (k,)), -1, 1)    # (sigma', k, chi_c...)
        renv[i] = (q.conj().T @ zm).reshape(k, shp[-2], shp[-1])
    return out
