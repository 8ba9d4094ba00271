"""Conditioning of the large-bond workload's shape (tensor train, d=4, chi=256, D=16, max_bond=256;
Sec. III A), measured on the oracle alone.

Every truncation of this shape keeps 256 of 1024 directions whose singular values are close together
(relative gaps at the cut of 1e-4 to 1e-2), so the compressed state is an ill-conditioned function of
the input: a rounding-level relative perturbation of every input entry moves the oracle's own output
by an amount that grows geometrically with the number of truncating sites. This bounds the chain
length at which any two implementations (the GPU paths included) can agree with the oracle, and
is why full-size parity at 128 sites is checked by properties rather than element by element.
CPU only.
"""
import math

import numpy as np

from oracle import cbc_tt, tn
from paper_2601_19650_amd.inputs import config_problem


def _self_perturbation(n, eps=1e-15, seed=123):
    p = config_problem("C4", n=n)
    rec = []
    ref = tn.mps_to_tree(cbc_tt(tn.tree_to_mps(p.state), tn.tree_to_mpo(p.op), p.max_bond,
                                record=rec))
    rng = np.random.default_rng(seed)
    st = [t * (1 + eps * rng.standard_normal(t.shape)) for t in p.state]
    op = [w * (1 + eps * rng.standard_normal(w.shape)) for w in p.op]
    pert = tn.mps_to_tree(cbc_tt(tn.tree_to_mps(st), tn.tree_to_mpo(op), p.max_bond))
    k = p.max_bond
    # relative gap (s_k - s_{k+1}) / s_k at every truncation that cuts
    gaps = [(s[k - 1] - s[k]) / s[k - 1] for s in rec if len(s) > k]
    return tn.rel_error(p.parent, pert, ref), gaps


def test_large_bond_shape_is_ill_conditioned():
    delta = {}
    for n in (8, 12, 16):
        d, gaps = _self_perturbation(n)
        delta[n] = d
        print(f"n={n}: output moved by {d:.2e} under 1e-15 input noise; {len(gaps)} truncations, "
              f"smallest relative gap at the cut {min(gaps):.1e}")
        assert all(0.0 < g < 1e-1 for g in gaps)
    # geometric growth, about 1.6x per added site (measured 5e-15, 4e-14, 3e-13 at 8, 12, 16 sites
    # and 5e-12, 6e-12 at 20, 24 sites)
    rate = math.exp(math.log(delta[16] / delta[8]) / 8)
    print(f"growth per site {rate:.2f}")
    assert 1.3 <= rate <= 2.2, rate
    # up to 16 sites the oracle is still reproducible far below the FP64 parity bar (1e-10)
    assert delta[16] <= 1e-11
