"""Seeded synthetic inputs: tree topologies, bond dimensions and random TTNS/TTNO node tensors.

This module is shared by the oracle, the tests and the benchmark. It holds none of the compression
method's arithmetic: it only draws tensors and rescales them.

Tensor conventions (the rooted-tree data model of Sec. II A-C, Eqs. ttns and ttno):
  * ``parent[i]`` is the parent node of ``i``; exactly one node has ``parent == -1`` (the root).
    The children of ``i`` are the nodes ``j`` with ``parent[j] == i``, in increasing ``j``.
  * state node ``i`` has legs ``(sigma_i, alpha_parent, alpha_child_1, ..., alpha_child_K)``;
  * operator node ``i`` has legs ``(sigma'_i, sigma_i, beta_parent, beta_child_1, ..., beta_child_K)``;
  * the root's parent leg is a trivial leg of dimension 1 (Sec. II B: the MPS's outer legs have
    dimension 1; the chain is rooted at its first site).

Input recipe (stands in for the random-TN workload of Sec. IV A):
  * entries are ``(N(0,1) + i N(0,1)) / sqrt(2)`` drawn with ``numpy.random.default_rng(seed)``,
    state nodes first (node order), then operator nodes (node order);
  * ``dist="paper"`` instead draws real and imaginary parts from U[-0.5, 1] as in Sec. IV A;
  * bond dimensions are capped by the dimension of the smaller side of each cut, so no bond is
    redundant: ``chi_i = min(chi, prod_{j in sub(i)} d_j, prod_{j not in sub(i)} d_j)`` for the state
    and the same with ``d_j**2`` for the operator;
  * every node is scaled to unit Frobenius norm, then every state node is divided by
    ``||psi||**(1/N)`` so that ``||psi|| = 1``, and every operator node by
    ``(||O||_HS / sqrt(prod d))**(1/N)`` so that a random state keeps norm ~1 under ``O``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "chain_parent", "kary_parent", "cut_bonds", "random_problem",
    "config_problem", "batch_problems", "batch_shapes", "CONFIGS",
    "t_tree", "balanced_binary", "fork_tree", "paper_problem", "PAPER_WORKLOADS", "sketch_matrices",
]


def chain_parent(n: int) -> list[int]:
    """Tensor train rooted at its first site: ``parent[i] = i - 1``."""
    return [i - 1 for i in range(n)]


def kary_parent(n: int, k: int) -> list[int]:
    """Complete k-ary tree in heap order: ``parent[i] = (i - 1) // k``."""
    return [-1] + [(i - 1) // k for i in range(1, n)]


def _children(parent):
    ch = [[] for _ in parent]
    for j, p in enumerate(parent):
        if p >= 0:
            ch[p].append(j)
    return ch


def _subtree_nodes(parent):
    ch = _children(parent)
    root = parent.index(-1)
    order, stack = [], [root]
    while stack:
        i = stack.pop()
        order.append(i)
        stack.extend(ch[i])
    sub = [None] * len(parent)
    for i in reversed(order):
        s = {i}
        for c in ch[i]:
            s |= sub[c]
        sub[i] = s
    return sub


def cut_bonds(parent, phys, cap, power=1):
    """Bond to the parent for every node: min(cap, dim of the smaller side of the cut)."""
    sub = _subtree_nodes(parent)
    n = len(parent)
    out = []
    for i in range(n):
        if parent[i] < 0:
            out.append(1)
            continue
        inside = 1
        outside = 1
        for j in range(n):
            if j in sub[i]:
                inside = min(inside * phys[j] ** power, 1 << 62)
            else:
                outside = min(outside * phys[j] ** power, 1 << 62)
        out.append(int(min(cap, inside, outside)))
    return out


@dataclass
class Problem:
    """One compression instance: tree, random TTNS, random TTNO, target bond dimension."""
    parent: list
    phys: list
    chi: list          # state bond to parent (1 at the root)
    dop: list          # operator bond to parent (1 at the root)
    state: list        # complex128 node tensors
    op: list           # complex128 node tensors
    max_bond: int
    tol: float = 0.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return len(self.parent)

    def children(self, i):
        return [j for j, p in enumerate(self.parent) if p == i]


def _draw(rng, shape, dist):
    if dist == "gauss":
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        return (re + 1j * im) / math.sqrt(2.0)
    if dist == "paper":
        re = rng.uniform(-0.5, 1.0, shape)
        im = rng.uniform(-0.5, 1.0, shape)
        return re + 1j * im
    raise ValueError(dist)


def _log_norm(parent, tensors, nphys):
    """log ||X|| of a tree network whose nodes carry ``nphys`` leading physical legs.

    Leaves-to-root transfer contraction with per-node rescaling (input preparation only).
    """
    ch = _children(parent)
    root = parent.index(-1)
    order, stack = [], [root]
    while stack:
        i = stack.pop()
        order.append(i)
        stack.extend(ch[i])
    env = {}
    logs = 0.0
    for i in reversed(order):
        t = tensors[i]
        shp = t.shape
        dphys = int(np.prod(shp[:nphys]))
        t = t.reshape((dphys,) + shp[nphys:])
        # absorb children environments E_c[a_c, a_c'] into ket copy
        x = t
        for c_pos, c in enumerate(ch[i]):
            e = env.pop(c)
            ax = 2 + c_pos
            x = np.tensordot(x, e, axes=([ax], [0]))     # new leg at the end
            x = np.moveaxis(x, -1, ax)
        # contract with bra over phys and children legs -> (a_p, a_p')
        axes = [0] + list(range(2, t.ndim))
        e = np.tensordot(x, t.conj(), axes=(axes, axes))
        s = np.abs(e).max()
        if s == 0.0:
            return -np.inf
        env[i] = e / s
        logs += math.log(s)
    val = env[root].reshape(-1)[0].real
    return 0.5 * (logs + math.log(val))


def random_problem(parent, phys, chi, dop_cap, max_bond, seed, tol=0.0, dist="gauss", name=""):
    """Draw one instance on the tree ``parent`` with physical dims ``phys``.

    ``chi`` / ``dop_cap`` cap the state / operator bonds (then cut-capped as described above).
    """
    n = len(parent)
    phys = list(phys) if hasattr(phys, "__len__") else [int(phys)] * n
    chib = cut_bonds(parent, phys, chi, 1)
    dopb = cut_bonds(parent, phys, dop_cap, 2)
    ch = _children(parent)
    rng = np.random.default_rng(seed)
    state, op = [], []
    for i in range(n):
        shape = (phys[i], chib[i]) + tuple(chib[c] for c in ch[i])
        t = _draw(rng, shape, dist)
        state.append(t / np.linalg.norm(t))
    for i in range(n):
        shape = (phys[i], phys[i], dopb[i]) + tuple(dopb[c] for c in ch[i])
        w = _draw(rng, shape, dist)
        op.append(w / np.linalg.norm(w))
    lp = _log_norm(parent, state, 1)
    f = math.exp(-lp / n)
    state = [t * f for t in state]
    lo = _log_norm(parent, op, 2) - 0.5 * sum(math.log(d) for d in phys)
    g = math.exp(-lo / n)
    op = [w * g for w in op]
    return Problem(parent=list(parent), phys=phys, chi=chib, dop=dopb, state=state, op=op,
                   max_bond=int(max_bond), tol=float(tol), name=name,
                   meta=dict(seed=seed, chi_cap=chi, dop_cap=dop_cap, dist=dist))


# The five workloads the library is measured and checked on.
CONFIGS = {
    "C1": dict(kind="mps", n=8, d=2, chi=8, D=4, max_bond=32, seed=1),
    "C2": dict(kind="mps", n=64, d=2, chi=64, D=8, max_bond=64, seed=2),
    "C3": dict(kind="binary", n=31, d=2, chi=32, D=6, max_bond=32, seed=3),
    "C4": dict(kind="mps", n=128, d=4, chi=256, D=16, max_bond=256, seed=4),
}


def _parent_of(kind, n):
    if kind == "mps":
        return chain_parent(n)
    if kind == "binary":
        return kary_parent(n, 2)
    if kind == "ternary":
        return kary_parent(n, 3)
    raise ValueError(kind)


def config_problem(name, **over):
    """Problem for a named workload (C1..C4); keyword overrides allowed (e.g. n=16)."""
    c = dict(CONFIGS[name])
    c.update(over)
    parent = _parent_of(c["kind"], c["n"])
    return random_problem(parent, c["d"], c["chi"], c["D"], c["max_bond"], c["seed"],
                          tol=c.get("tol", 0.0), dist=c.get("dist", "gauss"), name=name)


def batch_shapes(count=256, seed=5, ternary_chi_cap=32, n_range=(16, 64), chi_range=(16, 128)):
    """The shapes of the uneven batch workload without its tensors: per instance
    (index, kind, N, d, chi, D, tensor seed), drawn exactly as batch_problems draws them."""
    seeds = np.random.SeedSequence(seed).spawn(count)
    out = []
    for j, ss in enumerate(seeds):
        rng = np.random.default_rng(ss)
        kind = ["mps", "binary", "ternary"][int(rng.integers(0, 3))]
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int([2, 4][int(rng.integers(0, 2))])
        chi = int(chi_range[0] + rng.integers(0, 113) * (chi_range[1] - chi_range[0]) // 112)
        D = int(rng.integers(4, 13))
        if kind == "ternary":
            chi = min(chi, ternary_chi_cap)
        out.append((j, kind, n, d, chi, D, int(rng.integers(0, 2**31 - 1))))
    return out


def batch_problems(count=256, seed=5, ternary_chi_cap=32, n_range=(16, 64), chi_range=(16, 128),
                   indices=None):
    """The uneven batch workload: per instance a tensor train, binary or ternary tree with
    N in n_range, d in {2,4}, chi in chi_range, D in [4,12], max_bond = chi.

    Ternary trees have their chi clamped to ``ternary_chi_cap`` (their nodes carry four virtual
    legs, so an unclamped draw is dominated by a handful of ternary instances). The same sequence of
    random draws is used whatever the ranges, so instance j keeps its kind, N, d and D. ``indices``
    selects instances of the sequence (each is drawn from its own seed, so a selection holds the
    same tensors as the full draw); None gives all of them.
    """
    out = []
    for j, kind, n, d, chi, D, sub_seed in batch_shapes(count, seed, ternary_chi_cap, n_range,
                                                         chi_range):
        if indices is not None and j not in indices:
            continue
        out.append(random_problem(_parent_of(kind, n), d, chi, D, chi, sub_seed,
                                  name=f"B{j}:{kind}:n{n}:d{d}:chi{chi}:D{D}"))
    return out


# ---- the random-network workload of Sec. IV A --------------------------------------------------
# Four tree shapes, entries with real and imaginary parts uniform on [-0.5, 1] (dist="paper"), the
# TTNO on the same tree as the TTNS. Readings where the text leaves a detail open (the figure that
# shows the shapes is not part of the text):
#   * T-tree: the central node (the root) carries no physical leg; each of its three chains has L
#     nodes with one physical leg each;
#   * balanced binary tree of depth L: L edges from the root to every leaf (2^(L+1) - 1 nodes),
#     physical legs on the 2^L leaves only;
#   * fork tensor product structure: a chain of L virtual nodes (no physical leg; the first is the
#     root), each with an attached chain of L physical nodes.

def t_tree(L, d):
    """T-shaped tree: node 0 (root, d = 1) with three chains of L physical nodes."""
    parent, phys = [-1], [1]
    for k in range(3):
        for j in range(L):
            parent.append(0 if j == 0 else len(parent) - 1)
            phys.append(d)
    return parent, phys


def balanced_binary(depth, d):
    """Perfect binary tree of the given depth in heap order; physical legs on the leaves only."""
    n = 2 ** (depth + 1) - 1
    parent = kary_parent(n, 2)
    first_leaf = 2 ** depth - 1
    phys = [d if i >= first_leaf else 1 for i in range(n)]
    return parent, phys


def fork_tree(L, d):
    """Fork tensor product structure: virtual chain 0..L-1 (root 0), physical chain of L nodes on
    every virtual node."""
    parent = [i - 1 for i in range(L)]
    phys = [1] * L
    for k in range(L):
        for j in range(L):
            parent.append(k if j == 0 else len(parent) - 1)
            phys.append(d)
    return parent, phys


# name: (tree builder, system size, d, state and operator bond, target bonds swept in Sec. IV A)
PAPER_WORKLOADS = {
    "mps": (lambda L, d: (chain_parent(L), [d] * L), 50, 3, 40, list(range(2, 41, 2))),
    "ttree": (t_tree, 20, 3, 10, list(range(2, 11, 2))),
    "binary": (balanced_binary, 6, 3, 10, list(range(2, 11, 2))),
    "fork": (fork_tree, 8, 3, 10, list(range(2, 11, 2))),
}


def paper_problem(kind, max_bond, size=None, bond=None, seed=7):
    """An instance of the random-network workload: tree `kind` of PAPER_WORKLOADS (its system size and
    bonds unless overridden), U[-0.5, 1] entries, target bond `max_bond`."""
    build, L, d, D, _ = PAPER_WORKLOADS[kind]
    parent, phys = build(size if size is not None else L, d)
    D = bond if bond is not None else D
    return random_problem(parent, phys, D, D, max_bond, seed, dist="paper",
                          name=f"paper-{kind}-L{size if size is not None else L}-D{D}-Dbar{max_bond}")


def sketch_matrices(phys, width, seed):
    """Random sketch matrices of the randomised compression (one per node, d_i x width): complex
    Gaussian entries (N(0,1) + i N(0,1))/sqrt(2), drawn node by node from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for d in phys:
        re = rng.standard_normal((int(d), int(width)))
        im = rng.standard_normal((int(d), int(width)))
        out.append((re + 1j * im) / math.sqrt(2.0))
    return out
