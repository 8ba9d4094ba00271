"""The oracle's pins catch plausible mistakes in the oracle.

Each case edits the oracle's source the way a plausible mistake would (a dropped term, a wrong sign
or conjugate, transposed legs, an off-by-one bond), executes the edited module, and runs a set of
the pins of test_oracle_pins against it: at least one must fail. The unedited oracle must pass them
all. CPU only.
"""
import importlib.util
import os
import types

import pytest

import oracle.cbc as ocbc

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_SRC = open(ocbc.__file__).read()


def _load_pins():
    spec = importlib.util.spec_from_file_location("pins_for_mutation", os.path.join(HERE, "test_oracle_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


PINS = _load_pins()

CHECKS = [
    ("exact 8-site chain vs dense", lambda: PINS.test_c1_exact_dense()),
    ("exact binary tree vs dense", lambda: PINS.test_exact_trees_dense("binary", 7, 2, 4, 3)),
    ("chain = tree formulation", lambda: PINS.test_tt_formulation_equals_tree_formulation()),
    ("projection invariants", lambda: PINS.test_projection_property_dense("binary", 7, 2, 8, 4, 4)),
    ("two-site closed form", lambda: PINS.test_two_site_closed_form()),
    ("dense reformulation", lambda: PINS.test_dense_reformulation_chain(6, 2, 4, 3, 3)),
    ("dense tree reformulation, binary", lambda: PINS.test_dense_reformulation_tree(
        PINS.kary_parent(7, 2), 2, 4, 3, 3, 1)),
    ("dense tree reformulation, ternary", lambda: PINS.test_dense_reformulation_tree(
        PINS.kary_parent(10, 3), 2, 4, 2, 3, 2)),
    ("truncation identities", lambda: PINS.test_truncation_step_identities()),
    ("LQ step", lambda: PINS.test_lq_step()),
]

MUTATIONS = [
    ("LQ without the final conjugate", "return qh.conj().T", "return qh.T"),
    ("truncation drops diag(s)", "lmat = s[:k, None] * vh[:k]", "lmat = vh[:k]"),
    ("truncation keeps one direction too few", "k = max(k, 1)", "k = max(k - 1, 1)"),
    ("tree R update without conj(Q)", "_r_update(state[i], op[i], qt.conj(),", "_r_update(state[i], op[i], qt,"),
    ("chain R update without conj(Q)", 'r = np.einsum("ztx,uab,tupq,xbq->zap", q3.conj(),', 'r = np.einsum("ztx,uab,tupq,xbq->zap", q3,'),
    ("operator legs transposed in the node contraction", "    terms.append((w, [sigp, sig] + beta))\n    if open_leg", "    terms.append((w, [sig, sigp] + beta))\n    if open_leg"),
    ("operator legs transposed in the chain forward sweep", '"xap,tupq,uab->xtbq"', '"xap,utpq,uab->xtbq"'),
    ("operator legs transposed in the tree R update", "    terms.append((w, [sigp, sig] + beta))\n    terms.append((qc", "    terms.append((w, [sig, sigp] + beta))\n    terms.append((qc"),
    ("sweep 2 keeps the target child's own environment", "                if c != k:", "                if True:"),
    ("sweep 2 omits the siblings' environments", "envs[1 + j] = lsub[c]", "pass"),
    ("sweep 1 attaches the children's environments in reverse order",
     "envs = {1 + j: lsub[c] for j, c in enumerate(ch[i])}",
     "envs = {len(ch[i]) - j: lsub[c] for j, c in enumerate(ch[i])}"),
    ("sweep 3 attaches the children's R in reverse order", "envs[1 + j] = renv[c]",
     "envs[len(ch[i]) - j] = renv[c]"),
]


def _with_oracle(src):
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src, "oracle_mutant", "exec"), mod.__dict__)
    saved = {k: getattr(PINS, k) for k in ("cbc_tree", "cbc_tt", "truncate_joined", "lq")}
    for k in saved:
        setattr(PINS, k, getattr(mod, k))
    return saved


def _restore(saved):
    for k, v in saved.items():
        setattr(PINS, k, v)


def _failing_checks(src):
    saved = _with_oracle(src)
    failed = []
    try:
        for name, fn in CHECKS:
            try:
                fn()
            except Exception:   # an assertion or a shape error: the pin rejects the mutant
                failed.append(name)
    finally:
        _restore(saved)
    return failed


def test_unmutated_oracle_passes_every_check():
    assert _failing_checks(ORACLE_SRC) == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(name, old, new):
    assert ORACLE_SRC.count(old) == 1, f"mutation site not unique: {old!r}"
    failed = _failing_checks(ORACLE_SRC.replace(old, new))
    assert failed, f"no pin catches: {name}"


# ---------------------------------------------------------------------------------------------
# the SRC oracle (oracle/src.py) and its pins (tests/test_oracle_src_pins.py)

import oracle.src as osrc  # noqa: E402

SRC_SRC = open(osrc.__file__).read()


def _load_src_pins():
    spec = importlib.util.spec_from_file_location("src_pins_for_mutation",
                                                  os.path.join(HERE, "test_oracle_src_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


SRC_PINS = _load_src_pins()
_C = {c[0]: c[1:] for c in SRC_PINS.CASES}

SRC_CHECKS = [
    ("dense formulation, chain", lambda: SRC_PINS.test_src_dense_formulation("chain7", *_C["chain7"])),
    ("dense formulation, binary", lambda: SRC_PINS.test_src_dense_formulation("bin7", *_C["bin7"])),
    ("dense formulation, ternary", lambda: SRC_PINS.test_src_dense_formulation("ter10", *_C["ter10"])),
    ("projection, isometries, Eckart-Young", lambda: SRC_PINS.test_src_projection_isometries_and_eckart_young(
        "uneven9", *_C["uneven9"])),
    ("exact when the sketch covers the ranks", lambda: SRC_PINS.test_src_exact_when_the_sketch_covers_every_rank()),
]

SRC_MUTATIONS = [
    ("sketch conjugated", "    terms.append((om, [sigp, r]))", "    terms.append((om.conj(), [sigp, r]))"),
    ("sketch on the input physical leg", "    terms.append((om, [sigp, r]))", "    terms.append((om, [sig, r]))"),
    ("sweep 2 omits the siblings' sketches", "envs[1 + j] = ksub[c]", "pass"),
    ("sweep 2 omits the parent's sketch", "                envs[0] = epar[i]", "                pass"),
    ("sweep 3 bases from Z instead of Z E", "            y = zm @ epar[i].reshape(shp[-2] * shp[-1], max_bond)",
     "            y = zm[:, :max_bond]"),
    ("R update without conj(Q)", "renv[i] = (q.conj().T @ zm)", "renv[i] = (q.T @ zm)"),
    ("sweep 3 attaches the children's R in reverse order", "envs = {1 + j: renv[c] for j, c in enumerate(ch[i])}",
     "envs = {len(ch[i]) - j: renv[c] for j, c in enumerate(ch[i])}"),
    ("operator legs transposed in the sketch", "    terms.append((w, [sigp, sig] + beta))\n    terms.append((om",
     "    terms.append((w, [sig, sigp] + beta))\n    terms.append((om"),
]


def _failing_src_checks(src):
    mod = types.ModuleType("src_oracle_mutant")
    exec(compile(src, "src_oracle_mutant", "exec"), mod.__dict__)
    saved = SRC_PINS.src_tree
    SRC_PINS.src_tree = mod.src_tree
    failed = []
    try:
        for name, fn in SRC_CHECKS:
            try:
                fn()
            except Exception:
                failed.append(name)
    finally:
        SRC_PINS.src_tree = saved
    return failed


def test_unmutated_src_oracle_passes_every_check():
    assert _failing_src_checks(SRC_SRC) == []


@pytest.mark.parametrize("name,old,new", SRC_MUTATIONS, ids=[m[0] for m in SRC_MUTATIONS])
def test_src_mutation_is_caught(name, old, new):
    assert SRC_SRC.count(old) == 1, f"mutation site not unique: {old!r}"
    failed = _failing_src_checks(SRC_SRC.replace(old, new))
    assert failed, f"no pin catches: {name}"


# ---------------------------------------------------------------------------------------------
# the DM oracle (oracle/dm.py) and its pins (tests/test_oracle_dm_pins.py)

import oracle.dm as odm  # noqa: E402

DM_SRC = open(odm.__file__).read()


def _load_dm_pins():
    spec = importlib.util.spec_from_file_location("dm_pins_for_mutation",
                                                  os.path.join(HERE, "test_oracle_dm_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


DM_PINS = _load_dm_pins()
_D = {c[0]: c[1:] for c in DM_PINS.CASES}

DM_CHECKS = [
    ("dense formulation, chain", lambda: DM_PINS.test_dm_dense_formulation("chain7", *_D["chain7"])),
    ("dense formulation, binary", lambda: DM_PINS.test_dm_dense_formulation("bin7", *_D["bin7"])),
    ("dense formulation, ternary", lambda: DM_PINS.test_dm_dense_formulation("ter10", *_D["ter10"])),
    ("projection, isometries, bounds", lambda: DM_PINS.test_dm_projection_isometries_and_truncation_bounds(
        "uneven9", *_D["uneven9"])),
    ("two-site optimum", lambda: DM_PINS.test_dm_two_site_is_the_optimal_truncation()),
]

DM_MUTATIONS = [
    ("bra operator not conjugated", "terms.append((w.conj(), [sigp, sigpp] + betap))",
     "terms.append((w, [sigp, sigpp] + betap))"),
    ("bra state not conjugated", "terms.append((t.conj(), [sigpp] + alphap))",
     "terms.append((t, [sigpp] + alphap))"),
    ("sweep 2 omits the siblings' environments", "envs[1 + j] = asub[c]", "pass"),
    ("sweep 2 omits the parent's environment", "                envs[0] = bpar[i]", "                pass"),
    ("environment legs paired wrongly", "bm = np.transpose(bpar[i], (0, 1, 3, 2)).reshape(ab, ab)",
     "bm = bpar[i].reshape(ab, ab)"),
    ("smallest eigenvectors kept", "q = vec[:, ::-1][:, :max_bond]", "q = vec[:, :max_bond]"),
    ("R update without conj(Q)", "renv[i] = (q.conj().T @ zm)", "renv[i] = (q.T @ zm)"),
    ("density matrix without the environment", "rho = zm @ bm @ zm.conj().T", "rho = zm @ zm.conj().T"),
]


def _failing_dm_checks(src):
    mod = types.ModuleType("dm_oracle_mutant")
    exec(compile(src, "dm_oracle_mutant", "exec"), mod.__dict__)
    saved = DM_PINS.dm_tree
    DM_PINS.dm_tree = mod.dm_tree
    failed = []
    try:
        for name, fn in DM_CHECKS:
            try:
                fn()
            except Exception:
                failed.append(name)
    finally:
        DM_PINS.dm_tree = saved
    return failed


def test_unmutated_dm_oracle_passes_every_check():
    assert _failing_dm_checks(DM_SRC) == []


@pytest.mark.parametrize("name,old,new", DM_MUTATIONS, ids=[m[0] for m in DM_MUTATIONS])
def test_dm_mutation_is_caught(name, old, new):
    assert DM_SRC.count(old) == 1, f"mutation site not unique: {old!r}"
    failed = _failing_dm_checks(DM_SRC.replace(old, new))
    assert failed, f"no pin catches: {name}"


# ---------------------------------------------------------------------------------------------
# the Zip-Up oracle (oracle/zipup.py) and its pins (tests/test_oracle_zipup_pins.py)

import oracle.zipup as ozu  # noqa: E402

ZIPUP_SRC = open(ozu.__file__).read()


def _load_zipup_pins():
    spec = importlib.util.spec_from_file_location("zipup_pins_for_mutation",
                                                  os.path.join(HERE, "test_oracle_zipup_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


ZIPUP_PINS = _load_zipup_pins()
_Z = {c[0]: c[1:] for c in ZIPUP_PINS.CASES}

ZIPUP_CHECKS = [
    ("dense formulation, chain", lambda: ZIPUP_PINS.test_zipup_dense_formulation("chain7", *_Z["chain7"])),
    ("dense formulation, binary", lambda: ZIPUP_PINS.test_zipup_dense_formulation("bin7", *_Z["bin7"])),
    ("dense formulation, ternary", lambda: ZIPUP_PINS.test_zipup_dense_formulation("ter10", *_Z["ter10"])),
    ("projection, isometries, lower bound", lambda: ZIPUP_PINS.test_zipup_projection_isometries_and_lower_bound(
        "uneven9", *_Z["uneven9"])),
    ("exact case", lambda: ZIPUP_PINS.test_zipup_exact_when_the_bond_covers_every_rank()),
    ("identity operator = TT-SVD", lambda: ZIPUP_PINS.test_zipup_identity_operator_on_canonical_chain_is_tt_svd(
        6, 2, 6, 3, 11)),
    ("two-site brute force", lambda: ZIPUP_PINS.test_zipup_two_site_brute_force()),
]

ZIPUP_MUTATIONS = [
    ("R update without conj(Q)", "renv[i] = (q.conj().T @ zm)", "renv[i] = (q.T @ zm)"),
    ("smallest singular vectors kept", "q = u[:, :max_bond]", "q = u[:, ::-1][:, :max_bond]"),
    ("basis from the conjugated unfolding", "np.linalg.svd(zm,", "np.linalg.svd(zm.conj(),"),
    ("unfolding with the bond legs first", "zm = z.reshape(rows, cols)",
     "zm = np.moveaxis(z.reshape(rows, cols).reshape(cols, rows), 0, 1).copy()"),
    ("children's R attached in reverse order", "envs = {1 + j: renv[c] for j, c in enumerate(ch[i])}",
     "envs = {len(ch[i]) - j: renv[c] for j, c in enumerate(ch[i])}"),
    ("no truncation", "if rows <= max_bond:", "if True:"),
    ("root conjugated", "out[i] = z.reshape(shp[:-2])[:, None]", "out[i] = z.conj().reshape(shp[:-2])[:, None]"),
    ("no completion of the singular vectors", "full_matrices=cols < max_bond", "full_matrices=False"),
]


def _failing_zipup_checks(src):
    mod = types.ModuleType("zipup_oracle_mutant")
    exec(compile(src, "zipup_oracle_mutant", "exec"), mod.__dict__)
    saved = ZIPUP_PINS.zipup_tree
    ZIPUP_PINS.zipup_tree = mod.zipup_tree
    failed = []
    try:
        for name, fn in ZIPUP_CHECKS:
            try:
                fn()
            except Exception:
                failed.append(name)
    finally:
        ZIPUP_PINS.zipup_tree = saved
    return failed


def test_unmutated_zipup_oracle_passes_every_check():
    assert _failing_zipup_checks(ZIPUP_SRC) == []


@pytest.mark.parametrize("name,old,new", ZIPUP_MUTATIONS, ids=[m[0] for m in ZIPUP_MUTATIONS])
def test_zipup_mutation_is_caught(name, old, new):
    assert ZIPUP_SRC.count(old) == 1, f"mutation site not unique: {old!r}"
    failed = _failing_zipup_checks(ZIPUP_SRC.replace(old, new))
    assert failed, f"no pin catches: {name}"
