"""Oracle-side tensor-network utilities: dense contraction, overlaps, norms, state differences, and the
naive contract-then-SVD compression (the "direct" method of Sec. III C).

TEST INFRASTRUCTURE ONLY (see oracle/cbc.py). Plain complex128 NumPy; shares no code with the GPU path.

Tree conventions are those of Sec. II A: ``parent[i]`` (-1 at the root), children in increasing id;
state node legs (sigma, parent, children...), operator node legs (sigma', sigma, parent, children...).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "children", "postorder", "to_dense", "apply_dense", "overlap", "norm_sq", "applied_norm_sq",
    "direct_sum", "canonical_norm", "diff_norm", "rel_error", "fidelity", "product_ttn",
    "naive_compress", "mps_to_tree", "tree_to_mps", "isometry_error",
]


def children(parent):
    ch = [[] for _ in parent]
    for j, p in enumerate(parent):
        if p >= 0:
            ch[p].append(j)
    return ch


def postorder(parent):
    ch = children(parent)
    root = parent.index(-1)
    out, stack = [], [(root, False)]
    while stack:
        i, done = stack.pop()
        if done:
            out.append(i)
            continue
        stack.append((i, True))
        for c in reversed(ch[i]):
            stack.append((c, False))
    return out


# ----------------------------------------------------------------------------------------------
# dense forms (tiny systems only)

def to_dense(parent, state):
    """Contract a TTNS (Eq. ttns) to its state vector, axes in node order."""
    n = len(parent)
    ch = children(parent)
    sig = list(range(n))
    bond = [n + i for i in range(n)]
    args = []
    for i in range(n):
        args += [state[i], [sig[i], bond[i]] + [bond[c] for c in ch[i]]]
    return np.einsum(*args, sig, optimize="greedy")


def apply_dense(parent, op, vec):
    """Apply a TTNO (Eq. ttno) to a dense state vector (axes in node order)."""
    n = len(parent)
    ch = children(parent)
    sig = list(range(n))
    sigp = [n + i for i in range(n)]
    beta = [2 * n + i for i in range(n)]
    args = [vec, sig]
    for i in range(n):
        args += [op[i], [sigp[i], sig[i], beta[i]] + [beta[c] for c in ch[i]]]
    return np.einsum(*args, sigp, optimize="greedy")


# ----------------------------------------------------------------------------------------------
# overlaps and norms by leaves-to-root contraction (with per-node rescaling)

def overlap(parent, a, b):
    """<a|b> for two TTNS on the same tree; returns (value, log-scale): <a|b> = value * exp(logscale)."""
    ch = children(parent)
    env = {}
    logs = 0.0
    for i in postorder(parent):
        x = b[i]
        for j, c in enumerate(ch[i]):
            e = env.pop(c)                       # e[alpha_a, alpha_b]
            x = np.tensordot(x, e, axes=([2 + j], [1]))
            x = np.moveaxis(x, -1, 2 + j)
        axes = [0] + list(range(2, x.ndim))
        e = np.tensordot(a[i].conj(), x, axes=(axes, axes))    # (alpha_a_parent, alpha_b_parent)
        s = np.abs(e).max()
        if s == 0.0:
            return 0.0 + 0.0j, 0.0
        env[i] = e / s
        logs += math.log(s)
    root = parent.index(-1)
    return complex(env[root].reshape(-1)[0]), logs


def norm_sq(parent, a):
    v, l = overlap(parent, a, a)
    return v.real * math.exp(l)


def _pairwise(terms, out):
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


def applied_norm_sq(parent, op, state):
    """||O psi||^2 = <psi|O^dagger O|psi> by a leaves-to-root sandwich contraction."""
    ch = children(parent)
    env = {}
    logs = 0.0
    for i in postorder(parent):
        t, w = state[i], op[i]
        k = len(ch[i])
        # labels: ket sigma 0, sigma' 1, bra sigma 2; legs per slot
        a = [3 + j for j in range(k + 1)]
        b = [3 + (k + 1) + j for j in range(k + 1)]
        bb = [3 + 2 * (k + 1) + j for j in range(k + 1)]
        aa = [3 + 3 * (k + 1) + j for j in range(k + 1)]
        terms = [(t, [0] + a)]
        for j, c in enumerate(ch[i]):
            terms.append((env.pop(c), [a[1 + j], b[1 + j], bb[1 + j], aa[1 + j]]))
        terms += [(w, [1, 0] + b), (w.conj(), [1, 2] + bb), (t.conj(), [2] + aa)]
        e = _pairwise(terms, [a[0], b[0], bb[0], aa[0]])
        s = np.abs(e).max()
        env[i] = e / s
        logs += math.log(s)
    root = parent.index(-1)
    return env[root].reshape(-1)[0].real * math.exp(logs)


# ----------------------------------------------------------------------------------------------
# state differences via the direct-sum network (resolution ~1e-16 relative, unlike the overlap form)

def direct_sum(parent, a, b, sign_b=-1.0):
    """TTNS of |a> + sign_b |b>: block-diagonal in every virtual leg, blocks summed at the root."""
    ch = children(parent)
    out = []
    for i in range(len(parent)):
        ta, tb = a[i], b[i]
        root = parent[i] < 0
        shape = [ta.shape[0]]
        sl_a, sl_b = [slice(None)], [slice(None)]
        for ax in range(1, ta.ndim):
            if ax == 1 and root:
                shape.append(1)
                sl_a.append(slice(0, 1))
                sl_b.append(slice(0, 1))
            else:
                na, nb = ta.shape[ax], tb.shape[ax]
                shape.append(na + nb)
                sl_a.append(slice(0, na))
                sl_b.append(slice(na, na + nb))
        x = np.zeros(shape, dtype=np.complex128)
        x[tuple(sl_a)] += ta
        x[tuple(sl_b)] += (sign_b if root else 1.0) * tb
        out.append(x)
    return out


def canonical_norm(parent, tensors):
    """||X|| by QR-orthogonalising every non-root node toward the root (accurate to ~u ||X||)."""
    ch = children(parent)
    t = [x.copy() for x in tensors]
    for i in postorder(parent):
        p = parent[i]
        if p < 0:
            return float(np.linalg.norm(t[i]))
        x = np.moveaxis(t[i], 1, -1)
        shp = x.shape
        q, r = np.linalg.qr(x.reshape(-1, shp[-1]), mode="reduced")
        t[i] = np.moveaxis(q.reshape(shp[:-1] + (q.shape[1],)), -1, 1)
        slot = 2 + ch[p].index(i)
        y = np.tensordot(t[p], r, axes=([slot], [1]))
        t[p] = np.moveaxis(y, -1, slot)
    raise ValueError("no root")


def diff_norm(parent, a, b):
    """||a - b|| computed on the direct-sum network."""
    return canonical_norm(parent, direct_sum(parent, a, b, -1.0))


def rel_error(parent, approx, ref):
    """||approx - ref|| / ||ref||."""
    return diff_norm(parent, approx, ref) / canonical_norm(parent, ref)


def fidelity(parent, a, b):
    """|<a|b>|^2 / (<a|a><b|b>)."""
    v, l = overlap(parent, a, b)
    va, la = overlap(parent, a, a)
    vb, lb = overlap(parent, b, b)
    return (abs(v) ** 2) * math.exp(2 * l - la - lb) / (va.real * vb.real)


def isometry_error(t):
    """max |Q Q^dagger - I| for a node tensor read as (parent leg) x (all other legs)."""
    q = np.moveaxis(t, 1, 0).reshape(t.shape[1], -1)
    g = q @ q.conj().T
    return float(np.abs(g - np.eye(g.shape[0])).max())


# ----------------------------------------------------------------------------------------------
# the "direct" method of Sec. III C: exact product, then a truncated-SVD sweep

def product_ttn(parent, op, state):
    """Exact product O|psi> as a TTNS with fused bonds (alpha, beta) -> chi * D."""
    out = []
    for t, w in zip(state, op):
        k = t.ndim - 1
        a = [2 + j for j in range(k)]
        b = [2 + k + j for j in range(k)]
        inter = []
        for j in range(k):
            inter += [a[j], b[j]]
        p = np.einsum(w, [1, 0] + b, t, [0] + a, [1] + inter, optimize="greedy")
        shp = [p.shape[0]] + [t.shape[1 + j] * w.shape[2 + j] for j in range(k)]
        out.append(p.reshape(shp))
    return out


def naive_compress(parent, op, state, max_bond, tol=0.0):
    """Contract-then-compress: product TTNS, QR canonical form toward the root, then truncated SVDs
    of every bond in a depth-first sweep from the root (orthogonality centre moved along)."""
    ch = children(parent)
    t = product_ttn(parent, op, state)
    # canonicalise toward the root
    for i in postorder(parent):
        p = parent[i]
        if p < 0:
            break
        x = np.moveaxis(t[i], 1, -1)
        shp = x.shape
        q, r = np.linalg.qr(x.reshape(-1, shp[-1]), mode="reduced")
        t[i] = np.moveaxis(q.reshape(shp[:-1] + (q.shape[1],)), -1, 1)
        slot = 2 + ch[p].index(i)
        t[p] = np.moveaxis(np.tensordot(t[p], r, axes=([slot], [1])), -1, slot)

    def visit(i):
        for j, c in enumerate(ch[i]):
            slot = 2 + j
            x = np.moveaxis(t[i], slot, -1)
            shp = x.shape
            u, s, vh = np.linalg.svd(x.reshape(-1, shp[-1]), full_matrices=False)
            k = min(int(max_bond), len(s))
            if tol > 0.0:
                k = min(k, int(np.count_nonzero(s > tol * s[0])))
            k = max(k, 1)
            t[i] = np.moveaxis(u[:, :k].reshape(shp[:-1] + (k,)), -1, slot)
            sv = s[:k, None] * vh[:k]
            t[c] = np.moveaxis(np.tensordot(t[c], sv, axes=([1], [1])), -1, 1)
            visit(c)
            y = np.moveaxis(t[c], 1, -1)
            shp = y.shape
            q, r = np.linalg.qr(y.reshape(-1, shp[-1]), mode="reduced")
            t[c] = np.moveaxis(q.reshape(shp[:-1] + (q.shape[1],)), -1, 1)
            t[i] = np.moveaxis(np.tensordot(t[i], r, axes=([slot], [1])), -1, slot)

    visit(parent.index(-1))
    return t


# ----------------------------------------------------------------------------------------------
# format conversions between the tree layout and the tensor-train layout of Sec. II B

def tree_to_mps(state):
    """Chain rooted at node 0 (tree layout) -> MPS tensors (sigma, alpha_{i-1}, alpha_i)."""
    n = len(state)
    out = []
    for i, t in enumerate(state):
        out.append(t if i < n - 1 else t[:, :, None])
    return out


def tree_to_mpo(op):
    n = len(op)
    return [w if i < n - 1 else w[:, :, :, None] for i, w in enumerate(op)]


def mps_to_tree(mps):
    n = len(mps)
    return [t if i < n - 1 else t[:, :, 0] for i, t in enumerate(mps)]
