"""Oracle for density-matrix (DM) compression on trees: plain, slow, complex128 NumPy.

TEST INFRASTRUCTURE ONLY, like oracle/cbc.py: the reference the GPU library's DM path is checked
against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the library never calls it. It shares no code with the GPU path.

What it computes (arXiv 2601.19650, Sec. III): the density-matrix method that CBC is built from.
Each bond is truncated with the top eigenvectors of the reduced density matrix of the product
state O|psi> on one side of it; CBC obtains the same kind of matrix as a Gram M M^H of a factor M,
whereas DM contracts the exact environments of <Phi|Phi>, Phi = O|psi> (Tab. time_scal and
mem_scal give its cost: environments of (D_S D_O)^2 per bond). On the tree sweeps of Sec. III B:
  * sweep 1, leaves to root: the exact subtree environments of <Phi|Phi>,
    A^{[i]}[alpha_i, beta_i, beta'_i, alpha'_i] (ket state, ket operator, bra operator, bra state
    legs of the bond from node i to its parent);
  * sweep 2, root to leaves: the exact environments of the rest of the tree B^{[k]} (same legs),
    from the parent's tensors, the parent's B and the siblings' A;
  * sweep 3, leaves to root, as in CBC (Eqs. cbc_tree_third_contraction, cbc_final_contraction):
    Z^{[i]} = T W prod_c R^{[c]}; rho_i = Z^{[i]} B^{[i]} Z^{[i]H} (contracted over the parent bond)
    is the reduced density matrix of the partly compressed state on the subtree of i; its top
    k = min(D-bar, rows) eigenvectors form Q; R^{[i]} = Q^H Z^{[i]}; the root keeps Z.

Readings taken where the paper is silent:
  * the sweep order and output gauge are CBC's (bases toward the root, the root holds the norm), so
    the three methods of this repository return the same kind of network;
  * a node whose rows do not exceed D-bar keeps the identity basis (nothing to truncate);
  * legs and storage order as in oracle/cbc.py.

Parity pins (tests/test_oracle_dm_pins.py): an independent dense formulation (top left singular
vectors of each node's unfolding of O|psi>, children projected onto their bases), exactness when
D-bar covers every rank, the projection property, isometries, and the sequential-truncation bounds
max_cut tail <= ||O psi - psi'|| <= sqrt(sum of the cuts' tails^2); tests/test_oracle_mutations.py
plants mistakes here and checks they fail.
"""
from __future__ import annotations

import numpy as np

from oracle.cbc import _children, _node_contraction, _pairwise, _postorder

__all__ = ["dm_tree"]


def _density_node(t, w, envs, open_slot):
    """Node i of <Phi|Phi>: T_i, W_i, conj(W_i), conj(T_i) and the environments ``envs`` (slot ->
    tensor (alpha, beta, beta', alpha')), the slot ``open_slot`` left open. Result legs
    (alpha_open, beta_open, beta'_open, alpha'_open). Slots that are neither open nor given an
    environment have dimension 1 (the root's parent leg)."""
    nslot = t.ndim - 1
    sig, sigp, sigpp = 0, 1, 2       # ket input, output (shared by W and conj W), bra input
    alpha = [3 + j for j in range(nslot)]
    beta = [3 + nslot + j for j in range(nslot)]
    betap = [3 + 2 * nslot + j for j in range(nslot)]
    alphap = [3 + 3 * nslot + j for j in range(nslot)]
    terms = [(t, [sig] + alpha)]
    for slot in sorted(envs):
        terms.append((envs[slot], [alpha[slot], beta[slot], betap[slot], alphap[slot]]))
    terms.append((w, [sigp, sig] + beta))
    terms.append((w.conj(), [sigp, sigpp] + betap))
    terms.append((t.conj(), [sigpp] + alphap))
    o = open_slot
    return _pairwise(terms, [alpha[o], beta[o], betap[o], alphap[o]])


def dm_tree(parent, state, op, max_bond):
    """DM compression on the tree ``parent``; returns the new node tensors (sigma', parent,
    children...)."""
    n = len(parent)
    ch = _children(parent)
    root = parent.index(-1)
    post = _postorder(parent)
    pre = list(reversed(post))

    # sweep 1, leaves to root: exact subtree environments of <Phi|Phi>
    asub = {}
    for i in post:
        if i == root:
            continue
        envs = {1 + j: asub[c] for j, c in enumerate(ch[i])}
        asub[i] = _density_node(state[i], op[i], envs, 0)

    # sweep 2, root to leaves: exact environments of the rest of the tree
    bpar = {}
    for i in pre:
        for kpos, k in enumerate(ch[i]):
            envs = {}
            if i != root:
                envs[0] = bpar[i]
            for j, c in enumerate(ch[i]):
                if c != k:
                    envs[1 + j] = asub[c]
            bpar[k] = _density_node(state[i], op[i], envs, 1 + kpos)

    # sweep 3, leaves to root: bases from the reduced density matrices, R = Q^H Z
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
        ab = shp[-2] * shp[-1]
        zm = z.reshape(rows, ab)
        if rows <= max_bond:
            q = np.eye(rows, dtype=np.complex128)
        else:
            # B (alpha, beta, beta', alpha') as a matrix over (alpha, beta) x (alpha', beta')
            bm = np.transpose(bpar[i], (0, 1, 3, 2)).reshape(ab, ab)
            rho = zm @ bm @ zm.conj().T
            rho = 0.5 * (rho + rho.conj().T)
            lam, vec = np.linalg.eigh(rho)
            q = vec[:, ::-1][:, :max_bond]
        k = q.shape[1]
        out[i] = np.moveaxis(q.reshape(shp[:-2] + (k,)), -1, 1)    # (sigma', k, chi_c...)
        renv[i] = (q.conj().T @ zm).reshape(k, shp[-2], shp[-1])
    return out
