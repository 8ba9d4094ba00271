"""Oracle for the Zip-Up method on trees: plain, slow, complex128 NumPy.

TEST INFRASTRUCTURE ONLY, like oracle/cbc.py: the reference the GPU library's Zip-Up path is checked
against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the library never calls it. It shares no code with the GPU path.

What it computes (arXiv 2601.19650, Sec. III C; Tab. time_scal and mem_scal, Zip-Up rows): the
Zip-Up method passes over the network once and compresses each node on the spot, from the node's
own tensors and the already compressed part below it; nothing of the rest of the network enters a
truncation, which is why it is fast and less accurate. The paper describes it in words and
compares with it; on the tree sweeps of Sec. III B it reads:
  * one sweep, leaves to root (CBC's third sweep, Eqs. cbc_tree_third_contraction and
    cbc_final_contraction, without the environments of sweeps 1 and 2):
    Z^{[i]} = T W prod_c R^{[c]}, legs (sigma', the children's new bonds) x (alpha_p, beta_p);
  * the node's basis Q is the top k left singular vectors of that unfolding of Z^{[i]} (a truncated
    SVD of the local tensor); R^{[i]} = Q^H Z^{[i]} carries the rest upward; the root keeps Z.

Readings taken where the paper is silent:
  * the new bond of node i is k = min(D-bar, rows), as for the other methods here; where rows <=
    D-bar nothing is compressed and the basis is the identity; where the unfolding has fewer
    columns than k, the singular vectors are completed to k orthonormal ones (their directions
    carry no weight and do not change the state);
  * the input state is used in the gauge it is given: the paper mentions bringing it into a
    canonical form first as an optional refinement, and on a tree swept from many leaves at once
    there is no single orthogonality centre that serves every truncation;
  * sweep order and output gauge as CBC's (bases toward the root, the root holds the norm); legs
    and storage order as in oracle/cbc.py.

Parity pins (tests/test_oracle_zipup_pins.py): an independent dense formulation (unfoldings of each
subtree's exact product, children projected onto their bases), exactness when D-bar covers every
rank, isometries, the sequential truncated SVD of a canonical tensor train for the identity
operator, a brute-force two-site case and the optimal-truncation lower bound at every cut;
tests/test_oracle_mutations.py plants mistakes here and checks they fail.
"""
from __future__ import annotations

import numpy as np

from oracle.cbc import _children, _node_contraction, _postorder

__all__ = ["zipup_tree"]


def zipup_tree(parent, state, op, max_bond):
    """Zip-Up on the tree ``parent``; returns the new node tensors (sigma', parent, children...)."""
    n = len(parent)
    ch = _children(parent)
    root = parent.index(-1)
    renv = {}
    out = [None] * n
    for i in _postorder(parent):
        envs = {1 + j: renv[c] for j, c in enumerate(ch[i])}
        z = _node_contraction(state[i], op[i], envs, 0, None)   # (sigma', chi_c..., alpha_p, beta_p)
        shp = z.shape
        rows = int(np.prod(shp[:-2]))
        if i == root:
            out[i] = z.reshape(shp[:-2])[:, None]                 # (sigma', 1, chi_c...)
            continue
        cols = shp[-2] * shp[-1]
        zm = z.reshape(rows, cols)
        if rows <= max_bond:
            q = np.eye(rows, dtype=np.complex128)
        else:
            # the local compression: a truncated SVD of the node's unfolding (complete U when the
            # unfolding has fewer columns than the new bond)
            u, _, _ = np.linalg.svd(zm, full_matrices=cols < max_bond)
            q = u[:, :max_bond]
        k = q.shape[1]
        out[i] = np.moveaxis(q.reshape(shp[:-2] + (k,)), -1, 1)    # (sigma', k, chi_c...)
        renv[i] = (q.conj().T @ zm).reshape(k, shp[-2], shp[-1])
    return out
