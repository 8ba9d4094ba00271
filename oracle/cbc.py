"""Oracle for Cholesky-based compression (CBC): plain, slow, complex128 NumPy.

TEST INFRASTRUCTURE ONLY. This module is the reference the GPU library is checked against. Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it; the library itself
never calls it. It shares no code with the GPU path (only the seeded input generators are common).

What it computes (arXiv 2601.19650, "Efficient Application of Tensor Network Operators to Tensor
Network States"):
  * ``cbc_tt``   -- Sec. III A, tensor trains: the forward contraction and truncation of
    Eq. (tt_cbc_first_contraction), the backward contraction of Eq. (right_sweep_init_contr), the QR
    of Eq. (tt_cbc_qr_decomp), the update of Eq. (tt_cbc_final_contraction) and the output rule that
    closes Sec. III A (S at the root site, Q elsewhere).
  * ``cbc_tree`` -- Sec. III B, general trees: the leaves-to-root sweep of
    Eq. (cbc_tree_first_contraction), the root-to-leaves sweep of Eq. (cbc_tree_second_contraction),
    and the final leaves-to-root sweep of Eqs. (cbc_tree_third_contraction), (cbc_tree_qr) and
    (cbc_final_contraction), with the output rule that closes Sec. III B.

Readings taken where the paper is silent or garbled:
  * the truncation (Sec. III A leaves the method open and names the SVD) is the optimal truncated
    SVD of the joined-leg matrix: keep ``k = min(max_bond, len(s))`` singular triplets, and with a
    tolerance ``tol > 0`` (Sec. V: a tolerance for the SVD) additionally only ``s_j > tol * s_0``,
    never fewer than one; the isometry on the joined leg is dropped, so ``L = diag(s_k) Vh_k``;
  * the QR on the leg chi_{i-1} is an economy LQ: ``S = R Q`` with Q's rows orthonormal, new bond
    ``min(dim chi_{i-1}, rest)``;
  * in Eq. (cbc_final_contraction) Q enters complex-conjugated, as in the tensor-train update;
  * the output case for i = 0 in Sec. III A is the root site (the first site);
  * legs are identified by name; storage order is (sigma, parent, children...) for states and
    (sigma', sigma, parent, children...) for operators.

Parity pins: tests/test_oracle_pins.py checks this module against dense contraction, the projection
and isometry invariants, the Eckart-Young bound, an N=2 closed form, gauge and scalar covariances,
special cases and independent dense reformulations of the tensor-train sweep and of the three tree
sweeps (subspaces of the physical space, truncating trees with several children per node);
tests/test_oracle_mutations.py shows that plausible mistakes planted in this module fail them.
"""
from __future__ import annotations

import numpy as np

__all__ = ["cbc_tt", "cbc_tree", "truncate_joined", "lq"]


# ----------------------------------------------------------------------------------------------
# local linear algebra steps

def truncate_joined(lp, n_row_legs, max_bond, tol, record=None):
    """Join the first ``n_row_legs`` legs of ``lp`` into one and compress it (Sec. III A).

    Returns ``L`` with legs ``(chi_new, *remaining legs)``, equal to ``diag(s_k) Vh_k`` of the SVD of
    the joined-leg matrix; the left isometry U is dropped.
    """
    shp = lp.shape
    rows = int(np.prod(shp[:n_row_legs]))
    m = lp.reshape(rows, -1)
    _, s, vh = np.linalg.svd(m, full_matrices=False)
    k = min(int(max_bond), len(s))
    if tol > 0.0 and len(s) > 0:
        k = min(k, int(np.count_nonzero(s > tol * s[0])))
    k = max(k, 1)
    if record is not None:
        record.append(s.copy())
    lmat = s[:k, None] * vh[:k]
    return lmat.reshape((k,) + shp[n_row_legs:])


def lq(smat):
    """Economy LQ: ``smat = R @ Q`` with the rows of Q orthonormal; returns Q."""
    qh, _ = np.linalg.qr(smat.conj().T, mode="reduced")
    return qh.conj().T


# ----------------------------------------------------------------------------------------------
# Sec. III A: tensor trains.  MPS tensors T[i] legs (sigma, alpha_{i-1}, alpha_i) with outer legs of
# dimension 1; MPO tensors W[i] legs (sigma', sigma, beta_{i-1}, beta_i).

def cbc_tt(mps, mpo, max_bond, tol=0.0, record=None):
    """CBC of Sec. III A for a tensor train; returns the new MPS tensors (same leg order)."""
    n = len(mps)
    one = np.ones((1, 1, 1), dtype=np.complex128)
    # forward sweep: left environments L^{[i]}, i = 1..L-1 (Eq. tt_cbc_first_contraction)
    lenv = [one]
    for i in range(n - 1):
        t, w, lprev = mps[i], mpo[i], lenv[-1]
        # L'[chi_{i-1}, sigma', alpha_i, beta_i] = sum_{sigma, alpha_{i-1}, beta_{i-1}} L W T
        lp = np.einsum("xap,tupq,uab->xtbq", lprev, w, t, optimize=["einsum_path", (0, 2), (0, 1)])
        # join (chi_{i-1}, sigma') and compress
        lenv.append(truncate_joined(lp, 2, max_bond, tol, record))
    # backward sweep (Eqs. right_sweep_init_contr, tt_cbc_qr_decomp, tt_cbc_final_contraction)
    out = [None] * n
    r = one
    for i in range(n - 1, -1, -1):
        t, w, lprev = mps[i], mpo[i], lenv[i]
        # S[sigma', chi_{i-1}, chi_i] = sum L W T R
        s = np.einsum("xap,tupq,uab,ybq->txy", lprev, w, t, r,
                      optimize=["einsum_path", (2, 3), (1, 2), (0, 1)])
        if i == 0:
            out[0] = s
            break
        d, kl, kr = s.shape
        q = lq(s.transpose(1, 0, 2).reshape(kl, d * kr))
        q3 = q.reshape(q.shape[0], d, kr)                  # Q[chi'_{i-1}, sigma', chi_i]
        out[i] = q3.transpose(1, 0, 2)
        # R^{[i-1]}[chi'_{i-1}, alpha_{i-1}, beta_{i-1}] = sum Q* T W R
        r = np.einsum("ztx,uab,tupq,xbq->zap", q3.conj(), t, w, r,
                      optimize=["einsum_path", (1, 3), (1, 2), (0, 1)])
    return out


# ----------------------------------------------------------------------------------------------
# Sec. III B: general trees.

def _children(parent):
    ch = [[] for _ in parent]
    for j, p in enumerate(parent):
        if p >= 0:
            ch[p].append(j)
    return ch


def _postorder(parent):
    ch = _children(parent)
    root = parent.index(-1)
    out = []

    def visit(i):
        for c in ch[i]:
            visit(c)
        out.append(i)

    visit(root)
    return out


def _pairwise(terms, out):
    """Contract a list of (tensor, labels) pairs one pair at a time, left to right, keeping every label
    that is still needed by a later term or by ``out``."""
    x, lx = terms[0]
    for k in range(1, len(terms)):
        y, ly = terms[k]
        later = set(out)
        for _, lz in terms[k + 1:]:
            later |= set(lz)
        keep = [l for l in lx if l in later] + [l for l in ly if l in later and l not in lx]
        x = np.einsum(x, lx, y, ly, keep, optimize=True)
        lx = keep
    return np.einsum(x, lx, out)


def _node_contraction(t, w, envs, open_leg, leg_ids):
    """Contract T^{[i]}, the operator tensor and the environments ``envs``.

    ``envs`` maps a neighbour slot (0 = parent leg, 1.. = child legs in order) to an environment
    tensor with legs (chi, alpha, beta). ``open_leg`` is the slot left open (its alpha and beta legs
    stay on the result). Result legs: (sigma', chi of each env in slot order, alpha_open, beta_open),
    or (sigma', chi...) if ``open_leg`` is None. The sum is taken one tensor at a time: the state
    tensor, then each environment, then the operator tensor.
    """
    nslot = t.ndim - 1
    sig, sigp = 0, 1
    alpha = [2 + j for j in range(nslot)]
    beta = [2 + nslot + j for j in range(nslot)]
    chi = [2 + 2 * nslot + j for j in range(nslot)]
    terms = [(t, [sig] + alpha)]
    out = [sigp]
    for slot in sorted(envs):
        terms.append((envs[slot], [chi[slot], alpha[slot], beta[slot]]))
        out.append(chi[slot])
    terms.append((w, [sigp, sig] + beta))
    if open_leg is not None:
        out += [alpha[open_leg], beta[open_leg]]
    return _pairwise(terms, out)


def cbc_tree(parent, state, op, max_bond, tol=0.0, record=None):
    """CBC of Sec. III B on the tree ``parent``; returns new node tensors (sigma', parent, children...)."""
    n = len(parent)
    ch = _children(parent)
    root = parent.index(-1)
    post = _postorder(parent)
    pre = list(reversed(post))  # a valid root-first order (parents before children)
    one = np.ones((1, 1, 1), dtype=np.complex128)

    # sweep 1, leaves to root (Eq. cbc_tree_first_contraction): subtree tensors L^{[i]}
    lsub = {}
    for i in post:
        if i == root:
            continue
        envs = {1 + j: lsub[c] for j, c in enumerate(ch[i])}
        lp = _node_contraction(state[i], op[i], envs, 0, None)
        # join (sigma', chi_children...) and compress
        lsub[i] = truncate_joined(lp, 1 + len(ch[i]), max_bond, tol, record)

    # sweep 2, root to leaves (Eq. cbc_tree_second_contraction): L^{[(i,k)]}
    lpar = {root: one}
    for i in pre:
        for kpos, k in enumerate(ch[i]):
            envs = {0: lpar[i]}
            for j, c in enumerate(ch[i]):
                if c != k:
                    envs[1 + j] = lsub[c]
            lp = _node_contraction(state[i], op[i], envs, 1 + kpos, None)
            lpar[k] = truncate_joined(lp, 1 + len(envs), max_bond, tol, record)

    # sweep 3, leaves to root (Eqs. cbc_tree_third_contraction, cbc_tree_qr, cbc_final_contraction)
    renv = {}
    out = [None] * n
    for i in post:
        envs = {0: lpar[i]}
        for j, c in enumerate(ch[i]):
            envs[1 + j] = renv[c]
        s = _node_contraction(state[i], op[i], envs, None, None)   # (sigma', chi_p, chi_c...)
        if i == root:
            out[i] = s
            continue
        shp = s.shape
        sm = np.moveaxis(s, 1, 0)                                    # (chi_p, sigma', chi_c...)
        q = lq(sm.reshape(shp[1], -1))
        qt = q.reshape((q.shape[0], shp[0]) + shp[2:])               # Q[chi'_i, sigma', chi_c...]
        out[i] = np.moveaxis(qt, 0, 1)                               # (sigma', chi'_i, chi_c...)
        # R^{[i]}[chi'_i, alpha_p, beta_p] = sum T W Q* prod_c R^{[c]}
        renv[i] = _r_update(state[i], op[i], qt.conj(), [renv[c] for c in ch[i]])
    return out


def _r_update(t, w, qc, rch):
    nslot = t.ndim - 1
    sig, sigp, znew = 0, 1, 2
    alpha = [3 + j for j in range(nslot)]
    beta = [3 + nslot + j for j in range(nslot)]
    chi = [3 + 2 * nslot + j for j in range(nslot)]
    terms = [(t, [sig] + alpha)]
    for j, r in enumerate(rch):
        terms.append((r, [chi[1 + j], alpha[1 + j], beta[1 + j]]))
    terms.append((w, [sigp, sig] + beta))
    terms.append((qc, [znew, sigp] + chi[1:]))
    return _pairwise(terms, [znew, alpha[0], beta[0]])
