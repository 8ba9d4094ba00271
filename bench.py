#!/usr/bin/env python
"""Benchmark of the CBC hot path on one MI355X.

Workload (default): the large-bond MPS, N=128 sites, d=4, state bond chi=256, MPO bond D=16,
complex Gaussian entries, target bond 256 (truncating 4096 -> 256 at every bulk site). One step is
one complete compression (forward and backward sweeps, every truncation and QR) of that input,
already resident in HBM. The headline value is compressions/s of the mixed form (FP32 MFMA
contractions, FP64 Gram/eigen/Cholesky); the plain FP64 form is timed beside it on the same input.
The smaller workloads (8-site exact chain, 64-site chain, 31-node binary tree), the naive baseline,
batched and uneven batches are reported beside the headline.

Prints one JSON line. `--gpus N` with N > 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "fp32_mfma": 157.3e12, "fp64_mfma": 78.6e12, "fp64_alu": 78.6e12, "hbm": 8.0e12,
}
WORKLOADS = {
    "C4": "MPS N=128 d=4 chi=256 D=16 max_bond=256 (large bond, truncating 4096 -> 256), complex Gaussian",
    "C2": "MPS N=64 d=2 chi=64 D=8 max_bond=64 (truncating 512 -> 64), complex Gaussian",
    "C1": "MPS N=8 d=2 chi=8 D=4 max_bond=32 (exact), complex Gaussian",
    "C3": "binary tree 31 nodes d=2 chi=32 D=6 max_bond=32, complex Gaussian",
}


AUTOTUNE = False   # contexts tune their contractions (cbc_autotune) when set


def new_context(cbc):
    ctx = cbc.Context()
    if AUTOTUNE:
        ctx.autotune()
    return ctx


def measure(cbc, p, precs, steps, warmup, stream):
    """Time `steps` compressions of problem p per precision (after `warmup`), then the same number
    with per-op HIP events for the kernel-class times. Returns per-precision results and outputs."""
    import torch  # noqa: F401
    tree = cbc.Tree.of(p)
    st, so = cbc.pack(p.state, "cuda:0")
    op, oo = cbc.pack(p.op, "cuda:0")
    ctx = new_context(cbc)
    res, outputs = {}, {}
    run_args = (op, oo, st, so, 0.0)
    comps = {prec: cbc.Compressor(ctx, tree, p.max_bond, prec, device="cuda:0") for prec in precs}
    for prec in precs:
        timed_runs(comps[prec], run_args, stream, 0, warmup)
    # the forms' timed calls alternate, each between device synchronisations, so that a drift of
    # the device's speed during the run (the eigensolve's grid barrier varies by several per cent)
    # falls on every form alike
    total = {prec: 0.0 for prec in precs}
    for _ in range(steps):
        for prec in precs:
            total[prec] += timed_runs(comps[prec], run_args, stream, 1, 0)
    for prec in precs:
        comp = comps[prec]
        sec = total[prec] / steps
        replayed = int(comp.stats.graph_replayed)
        outputs[prec] = comp.unpack()
        kms = profiled_runs(comp, run_args, stream, max(2, min(steps, 10)))
        st_d = comp.stats.as_dict()
        res[prec] = dict(sec=sec, kms=kms, stats=st_d, replayed=replayed,
                         n_kernels=int(comp.stats.n_kernels))
        print(f"[bench] {p.name} {prec}: {sec * 1e3:.3f} ms/compression, kernels/call "
              f"{comp.stats.n_kernels}, graph replay {replayed}", file=sys.stderr, flush=True)
    del comps
    return res, outputs


def contraction_roofline(r, prec, cls):
    """Contraction kernels (the MFMA GEMMs of the sweeps) against the MFMA peak of their type:
    algorithmic flops per compression over their event-timed kernel time per compression."""
    k = cls.index("contract")
    flops = r["stats"]["contract"]["flops"]
    ms = r["kms"][k]
    peak = PEAK["fp32_mfma"] if prec == "mixed" else PEAK["fp64_mfma"]
    achieved = flops / (ms * 1e-3) if ms > 0 else 0.0
    return {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "kernel_ms_per_step": ms,
            "launches_per_step": r["stats"]["contract"]["launches"],
            "flops_per_step": flops}


def precision_line(r, prec, cls, ncls):
    """Compressions/s, contraction throughput and kernel-class times of one measured precision."""
    return {"value": 1.0 / r["sec"], "unit": "compressions/s", "ms_per_step": r["sec"] * 1e3,
            "contraction_tflops_wall": r["stats"]["contract"]["flops"] / r["sec"] / 1e12,
            "contraction_roofline": contraction_roofline(r, prec, cls),
            "kernel_ms_per_step": {cls[k]: r["kms"][k] for k in range(ncls)},
            "kernels_per_step": r["n_kernels"]}


def gpu_vs_oracle(cbc, p, ref, precs=("fp64", "mixed")):
    """Error of each GPU precision against an oracle result `ref` of the same problem."""
    from oracle import tn
    errs = {}
    for prec in precs:
        out, _ = cbc.compress(p, precision=prec, device="cuda:0")
        errs[prec] = dict(rel_state_error=tn.rel_error(p.parent, out, ref),
                          infidelity=1.0 - tn.fidelity(p.parent, out, ref))
    return errs


def oracle_result(p):
    from oracle import cbc_tree, cbc_tt, tn
    if all(q == i - 1 for i, q in enumerate(p.parent)):
        return tn.mps_to_tree(cbc_tt(tn.tree_to_mps(p.state), tn.tree_to_mpo(p.op), p.max_bond))
    return cbc_tree(p.parent, p.state, p.op, p.max_bond)


def _chain_fidelity(a, b):
    """|<a|b>|^2 / (<a|a><b|b>) of two tensor trains (nodes (sigma, left, right), site 0 the root),
    by transfer matrices on the device (plain torch; a measurement helper of this script)."""
    import torch

    def overlap(x, y):
        e = torch.ones((1, 1), dtype=torch.complex128, device="cuda:0")
        for i in range(len(x) - 1, -1, -1):
            xi = torch.from_numpy(x[i]).to("cuda:0")
            yi = torch.from_numpy(y[i]).to("cuda:0")
            if xi.dim() == 2:
                xi, yi = xi.unsqueeze(-1), yi.unsqueeze(-1)
            t = torch.tensordot(yi, e, dims=([2], [1]))          # sigma, pb, ca
            xa = xi.permute(1, 0, 2).reshape(xi.shape[1], -1).conj().contiguous()
            tb = t.permute(1, 0, 2).reshape(t.shape[1], -1).transpose(0, 1).contiguous()
            e = xa @ tb
        return complex(e.reshape(-1)[0].item())

    ab = overlap(a, b)
    return abs(ab) ** 2 / (overlap(a, a).real * overlap(b, b).real)


def uneven_full_run(stream_count=8):
    """The whole 256-instance uneven draw (tensor trains, binary and ternary trees, N in [16, 64],
    d in {2, 4}, chi in [16, 128] with ternary trees at chi <= 32, D in [4, 12], max_bond = chi),
    mixed precision, forked over `stream_count` streams whose instances share one scratch buffer
    per stream, captured into graphs of at most UnevenBatch.MAX_GRAPH_LAUNCHES launches each and
    replayed in order (one launch per graph)."""
    import torch
    from paper_2601_19650_amd import cbc
    from paper_2601_19650_amd.inputs import batch_problems
    t0 = time.perf_counter()
    probs = batch_problems()
    ub = cbc.UnevenBatch(probs, precision="mixed", nstreams=stream_count, autotune=AUTOTUNE,
                         share_scratch=True)
    t1 = time.perf_counter()
    print(f"[bench] uneven full draw: {len(probs)} instances set up in {t1 - t0:.1f} s",
          file=sys.stderr, flush=True)
    # first (eager) pass, 16 instances per call: builds every plan's offset tables and its graph
    for lo in range(0, len(ub.items), 16):
        hi = min(lo + 16, len(ub.items))
        ub.run_range(lo, hi)
        torch.cuda.synchronize()
        print(f"[bench] uneven full draw: first pass {hi} instances, "
              f"{time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    bad = [comp.report()["status"] for comp, _ in ub.items]
    bad = [b for b in bad if b != "ok"]
    t2 = time.perf_counter()
    ub.capture()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    print(f"[bench] uneven full draw: captured into {len(ub.graphs)} graphs in {t3 - t2:.1f} s",
          file=sys.stderr, flush=True)
    ub.run()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t3
    flops = ub.flops()
    mem = (sum(c.workspace.numel() for c, _ in ub.items) + sum(x.numel() for x in ub.scratch))
    print(f"[bench] uneven full draw: one replay {sec:.2f} s", file=sys.stderr, flush=True)
    return {"instances": len(probs), "value": len(probs) / sec, "unit": "compressions/s",
            "seconds": sec, "contraction_tflops": flops / sec / 1e12,
            "planned_contraction_tflop": flops / 1e12, "streams": stream_count,
            "workspace_gb": mem / 1e9, "failed_instances": len(bad),
            "launch": f"{len(ub.graphs)} captured graphs replayed in order, scratch shared per stream",
            "graphs": len(ub.graphs),
            "first_pass_seconds": t2 - t1,
            "recipe": "uneven draw (seed 5): MPS/binary/ternary, N 16-64, d 2|4, D 4-12, "
                      "chi 16-128 (ternary <= 32), all 256 instances"}


def _dev(t):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(t)).to("cuda:0")


def _gpu_sandwich(parent, bra, state, op, twice=False):
    """<bra| O |psi> (twice=False) or <psi| O^H O |psi> (twice=True, bra ignored) of tree networks
    given as numpy node tensors, contracted leaves to root on the device in complex128 (plain torch;
    a measurement helper of this script). Legs: states (sigma, parent, children...), operators
    (sigma', sigma, parent, children...)."""
    import torch
    ch = _gpu_children(parent)
    root = parent.index(-1)
    order, stack = [], [root]
    while stack:
        i = stack.pop()
        order.append(i)
        stack.extend(ch[i])
    env = {}
    for i in reversed(order):
        k = len(ch[i])
        letters = iter("cdefghijklmnopqrvzCDEFGHIJKLMNOPQRVWZ")
        A = [next(letters) for _ in range(k)]     # ket state legs of the children
        Bk = [next(letters) for _ in range(k)]    # operator legs
        X = [next(letters) for _ in range(k)]     # bra legs (or the second operator's)
        Y = [next(letters) for _ in range(k)]     # bra state legs (twice=True)
        x, lx = _dev(state[i]), "sa" + "".join(A)
        for j, c in enumerate(ch[i]):
            if twice:
                e, le = env.pop(c), Y[j] + X[j] + Bk[j] + A[j]
            else:
                e, le = env.pop(c), X[j] + Bk[j] + A[j]
            out = lx.replace(A[j], "") + le.replace(A[j], "")
            x, lx = torch.einsum(f"{lx},{le}->{out}", x, e), out
        w = _dev(op[i])
        lw = "ts" + "b" + "".join(Bk)
        out = "".join(ch_ for ch_ in lx if ch_ not in "s" + "".join(Bk)) + "tb"
        x, lx = torch.einsum(f"{lx},{lw}->{out}", x, w), out
        if twice:
            lw2 = "tu" + "x" + "".join(X)
            out = "".join(ch_ for ch_ in lx if ch_ not in "t" + "".join(X)) + "ux"
            x, lx = torch.einsum(f"{lx},{lw2}->{out}", x, w.conj()), out
            lt = "u" + "y" + "".join(Y)
            out = "".join(ch_ for ch_ in lx if ch_ not in "u" + "".join(Y)) + "y"
            x, lx = torch.einsum(f"{lx},{lt}->{out}", x, _dev(state[i]).conj()), out
            env[i] = torch.einsum(f"{lx}->yxba", x)
        else:
            lb = "t" + "x" + "".join(X)
            out = "".join(ch_ for ch_ in lx if ch_ not in "t" + "".join(X)) + "x"
            x, lx = torch.einsum(f"{lx},{lb}->{out}", x, _dev(bra[i]).conj()), out
            env[i] = torch.einsum(f"{lx}->xba", x)
    return complex(env[root].reshape(-1)[0].item())


def _rel_error_vs_exact(parent, out, state, op, norm_phi_sq, weight=False):
    """||O psi - psi'|| / ||O psi|| from <psi'|O|psi>, <psi'|psi'> and ||O psi||^2; with `weight`
    also the captured weight ||psi'||^2 / ||O psi||^2 (for a projection of O psi the squared error is
    one minus it, which stays informative where the error itself rounds to 1)."""
    ov = _gpu_sandwich(parent, out, state, op)
    outs = [_dev(t) for t in out]
    nq = _gpu_overlap(parent, outs, outs).real
    err = math.sqrt(max(norm_phi_sq - 2.0 * ov.real + nq, 0.0) / norm_phi_sq)
    return (err, nq / norm_phi_sq) if weight else err


def method_run(cbc, p, stream, steps, warmup, method, seed=11, nphi=None):
    """Another method of the library (method "src": cbc_apply_src with sketch matrices drawn from
    `seed`; "zipup": cbc_apply_zipup; "dm": cbc_apply_dm) on workload p in both precisions: time per compression (graph
    replay), kernel-class times, and the relative error and captured weight against the exact
    product O|psi> (||O psi||^2 = nphi)."""
    import torch
    from paper_2601_19650_amd.inputs import sketch_matrices
    tree = cbc.Tree.of(p)
    st, so = cbc.pack(p.state, "cuda:0")
    op, oo = cbc.pack(p.op, "cuda:0")
    kw = {}
    res = {}
    if method == "src":
        kw = {"sketch": cbc.pack(sketch_matrices(p.phys, p.max_bond, seed), "cuda:0")}
        res["sketch_seed"] = seed
    ctx = new_context(cbc)
    outs = {}
    for prec in ("mixed", "fp64"):
        comp = cbc.Compressor(ctx, tree, p.max_bond, prec, method=method, device="cuda:0")
        sec = timed_runs(comp, (op, oo, st, so, 0.0), stream, steps, warmup, **kw)
        print(f"[bench] {method} {p.name} {prec}: timed", file=sys.stderr, flush=True)
        outs[prec] = comp.unpack()
        kms = profiled_runs(comp, (op, oo, st, so, 0.0), stream, 2, **kw)
        res[prec] = {"value": 1.0 / sec, "unit": "compressions/s", "ms_per_step": sec * 1e3,
                     "kernel_ms_per_step": {c: kms[k] for k, c in enumerate(cbc.CLASSES)},
                     "kernels_per_step": int(comp.stats.n_kernels),
                     "contraction_tflops": comp.stats.flops[0] / sec / 1e12,
                     "workspace_gb": comp.ws_bytes / 1e9}
        print(f"[bench] {method} {p.name} {prec}: {sec * 1e3:.3f} ms/compression", file=sys.stderr,
              flush=True)
        del comp
    torch.cuda.synchronize()
    if nphi is None:
        nphi = _gpu_sandwich(p.parent, None, p.state, p.op, twice=True).real
    for prec, o in outs.items():
        e, w = _rel_error_vs_exact(p.parent, o, p.state, p.op, nphi, weight=True)
        res[prec]["rel_error_vs_exact"] = e
        res[prec]["captured_weight_fraction"] = w
    print(f"[bench] {method} {p.name}: captured weight " + ", ".join(
        f"{k} {res[k]['captured_weight_fraction']:.4e}" for k in outs), file=sys.stderr, flush=True)
    return res


def other_methods(cbc, p, stream, steps, warmup, cbc_outputs, methods):
    """SRC, Zip-Up and DM beside CBC on the headline workload, with every method's captured
    weight."""
    import torch
    torch.cuda.synchronize()
    nphi = _gpu_sandwich(p.parent, None, p.state, p.op, twice=True).real
    res = {"workload": WORKLOADS[p.name] if p.name in WORKLOADS else p.name, "cbc": {}}
    for k, o in cbc_outputs.items():
        e, w = _rel_error_vs_exact(p.parent, o, p.state, p.op, nphi, weight=True)
        res["cbc"][k] = {"rel_error_vs_exact": e, "captured_weight_fraction": w}
    for m in methods:
        res[m] = method_run(cbc, p, stream, steps, warmup, m, nphi=nphi)
    return res


def _gpu_children(parent):
    ch = [[] for _ in parent]
    for j, q in enumerate(parent):
        if q >= 0:
            ch[q].append(j)
    return ch


def _gpu_overlap(parent, A, B):
    """<A|B> of two tree networks with node legs (sigma, parent, children...) as torch tensors on
    the device, by a leaves-to-root contraction (plain torch; a measurement helper of this script)."""
    import torch
    ch = _gpu_children(parent)
    root = parent.index(-1)
    order, stack = [], [root]
    while stack:
        i = stack.pop()
        order.append(i)
        stack.extend(ch[i])
    env = {}
    for i in reversed(order):
        x = B[i]
        for pos, c in enumerate(ch[i]):
            e = env.pop(c)                               # (a_c of A, b_c of B)
            x = torch.tensordot(x, e, dims=([2 + pos], [1]))   # b_c -> a_c, moved to the end
            x = torch.movedim(x, -1, 2 + pos)
        a = A[i].conj()
        axes = [0] + list(range(2, a.dim()))
        env[i] = torch.tensordot(a, x, dims=(axes, axes))    # (a_p, b_p)
    return complex(env[root].reshape(-1)[0].item())


def _gpu_product(parent, state, op):
    """Node tensors of the exact product O|psi> (bonds fused, alpha-major), on the device."""
    import torch
    ch = _gpu_children(parent)
    out = []
    for i in range(len(parent)):
        t = torch.from_numpy(state[i]).to("cuda:0")
        w = torch.from_numpy(op[i]).to("cuda:0")
        k = t.dim() - 1                                   # virtual legs
        x = torch.tensordot(w, t, dims=([1], [0]))       # (s', b_1..b_k, a_1..a_k)
        perm = [0] + [q for j in range(k) for q in (1 + k + j, 1 + j)]
        x = x.permute(*perm).contiguous()
        shape = [x.shape[0]] + [x.shape[1 + 2 * j] * x.shape[2 + 2 * j] for j in range(k)]
        out.append(x.reshape(shape))
    return out


def paper_workloads(cbc, stream, full=False, steps=2):
    """The random-network workload of Sec. IV A on the GPU: tensor train (L=50, d=3, D=40), T-tree
    (L=20), balanced binary tree (depth 6, physical legs on the leaves) and fork tensor product
    structure (L=8), all d=3, D=10, entries U[-0.5, 1]; CBC, the randomised compression (sketch
    seed 11) and Zip-Up (mixed and FP64), the density-matrix method and the naive
    contract-then-compress baseline (FP64) over a sweep of target bonds: time per compression and relative error
    ||O psi - psi'|| / ||O psi||, with O psi contracted exactly on the device."""
    import dataclasses
    import torch
    from paper_2601_19650_amd.inputs import PAPER_WORKLOADS, paper_problem, sketch_matrices
    res = {}
    for kind, (_, L, d, D, sweep) in PAPER_WORKLOADS.items():
        dbars = sweep if full or len(sweep) <= 5 else [
            sweep[0], sweep[len(sweep) // 3], sweep[2 * len(sweep) // 3], sweep[-1]]
        base = paper_problem(kind, dbars[-1])
        P = _gpu_product(base.parent, base.state, base.op)
        nP = _gpu_overlap(base.parent, P, P).real
        tree = cbc.Tree.of(base)
        st, so = cbc.pack(base.state, "cuda:0")
        op, oo = cbc.pack(base.op, "cuda:0")
        ctx = new_context(cbc)
        pts = []
        for dbar in dbars:
            pt = {"target_bond": dbar}
            sk = cbc.pack(sketch_matrices(base.phys, dbar, 11), "cuda:0")
            for method, prec in (("cbc", "mixed"), ("cbc", "fp64"), ("src", "mixed"),
                                 ("src", "fp64"), ("zipup", "mixed"), ("zipup", "fp64"),
                                 ("dm", "fp64"), ("naive", "fp64")):
                comp = cbc.Compressor(ctx, tree, dbar, prec, method=method, device="cuda:0")
                kw = {"sketch": sk} if method == "src" else {}
                sec = timed_runs(comp, (op, oo, st, so, 0.0), stream, steps, 1, **kw)
                out = [torch.from_numpy(t).to("cuda:0") for t in comp.unpack()]
                nq = _gpu_overlap(base.parent, out, out).real
                ov = _gpu_overlap(base.parent, P, out).real
                err = math.sqrt(max(nP - 2.0 * ov + nq, 0.0) / nP)
                pt[f"{method}_{prec}"] = {"ms": sec * 1e3, "rel_error": err}
                del comp
            pts.append(pt)
            print(f"[bench] paper {kind} target bond {dbar}: " + ", ".join(
                f"{k} {v['ms']:.2f} ms err {v['rel_error']:.2e}" for k, v in pt.items()
                if isinstance(v, dict)), file=sys.stderr, flush=True)
        res[kind] = {"nodes": base.n, "phys": d, "state_bond": D, "operator_bond": D,
                     "size": L, "points": pts}
        del P, st, op
    return res


def recorded_traffic(workload, precision, op):
    """HBM bytes per launch of `op` from a committed counter summary (profiles/*_hbm_counters.md),
    or None when there is none for this workload, or a kernel source changed since it was taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_counters.md"))):
        text = open(path).read()
        if "```json" not in text:
            continue
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if (rec.get("workload"), rec.get("precision"), rec.get("op")) != (workload, precision, op):
            continue
        for src, sha in rec.get("sources_sha256", {}).items():
            with open(os.path.join(ROOT, src), "rb") as fh:
                if hashlib.sha256(fh.read()).hexdigest() != sha:
                    return None
        return float(rec["hbm_bytes_per_launch"])
    return None


def timed_runs(comp, args_run, stream, steps, warmup, **kw):
    import torch
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            comp.run(*args_run, stream=stream.cuda_stream, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            comp.run(*args_run, stream=stream.cuda_stream, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps if steps > 0 else 0.0


def profiled_runs(comp, args_run, stream, steps, **kw):
    """Per-kernel-class time from HIP events the library records on its own stream."""
    import torch
    from paper_2601_19650_amd import cbc
    tot = [0.0] * cbc.NCLASS
    with torch.cuda.stream(stream):
        for _ in range(steps):
            comp.run(*args_run, stream=stream.cuda_stream, profile=True, **kw)
            for k in range(cbc.NCLASS):
                tot[k] += comp.stats.ms[k]
    torch.cuda.synchronize()
    return [t / steps for t in tot]


def cpu_baseline_large(cbc):
    """The oracle on the large-bond workload, timed on a bounded sample: the same chain shape cut to
    10 and 11 sites (the 11th adds one bulk site with bonds 256 on both sides), on all host cores and
    on one thread. The full 128-site compression is extrapolated as t(11) + 117 (t(11) - t(10)),
    i.e. every further site at the measured bulk-site cost. The GPU results of the 10-site problem
    are compared with the oracle's (error_vs_oracle)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from paper_2601_19650_amd.inputs import config_problem
    ncores = len(os.sched_getaffinity(0))
    legs = {}
    refs = {}
    for label, lim in (("all_cores", ncores), ("one_thread", 1)):
        with threadpool_limits(limits=lim):
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
            t = {}
            for n in (10, 11):
                p = config_problem("C4", n=n)
                t0 = time.perf_counter()
                refs[n] = oracle_result(p)
                t[n] = time.perf_counter() - t0
        site = max(t[11] - t[10], 0.0)
        full = t[11] + (128 - 11) * site
        legs[label] = {"value": 1.0 / full, "unit": "compressions/s", "cores": int(threads),
                       "seconds_per_compression": full, "seconds_10_sites": t[10],
                       "seconds_11_sites": t[11], "seconds_per_bulk_site": site}
        print(f"[bench] oracle {label} ({threads} threads): 10 sites {t[10]:.2f} s, 11 sites "
              f"{t[11]:.2f} s, 128 sites extrapolated {full:.0f} s", file=sys.stderr, flush=True)
    errs = gpu_vs_oracle(cbc, config_problem("C4", n=10), refs[10])
    a = legs["all_cores"]
    return {"value": a["value"], "unit": "compressions/s", "cores": a["cores"], "kind": "oracle",
            "sample": "NumPy complex128 oracle (tensor-train sweep) on the large-bond chain cut to 10 "
                      "and 11 sites; the 128-site time extrapolated as t(11) + 117 x (t(11) - t(10)) "
                      "(one bulk site per step)",
            "one_thread": legs["one_thread"], "all_cores": a}, errs


def small_workload(cbc, name, stream, steps, precs=("mixed", "fp64")):
    """A latency-bound workload (C1, C2 or C3): compressions/s per precision and the error of each
    GPU result against the oracle (the 8-site exact chain also against the dense product O|psi>)."""
    from oracle import tn
    from paper_2601_19650_amd.inputs import config_problem
    p = config_problem(name)
    res, outputs = measure(cbc, p, list(precs), steps, 2, stream)
    t0 = time.perf_counter()
    ref = oracle_result(p)
    t_oracle = time.perf_counter() - t0
    line = {"workload": WORKLOADS[name]}
    for prec in precs:
        r = res[prec]
        line[prec] = {"value": 1.0 / r["sec"], "unit": "compressions/s",
                      "ms_per_step": r["sec"] * 1e3,
                      "kernel_ms_per_step": {cbc.CLASSES[k]: r["kms"][k] for k in range(cbc.NCLASS)},
                      "kernels_per_step": r["n_kernels"],
                      "error_vs_oracle": dict(
                          rel_state_error=tn.rel_error(p.parent, outputs[prec], ref),
                          infidelity=1.0 - tn.fidelity(p.parent, outputs[prec], ref))}
    if "mixed" in res and "fp64" in res:
        line["speedup_mixed_vs_fp64"] = res["fp64"]["sec"] / res["mixed"]["sec"]
    line["oracle_seconds_per_compression"] = t_oracle
    if name == "C1":
        phi = tn.apply_dense(p.parent, p.op, tn.to_dense(p.parent, p.state))
        for prec in precs:
            v = tn.to_dense(p.parent, outputs[prec])
            line[prec]["rel_error_vs_dense_product"] = float(
                __import__("numpy").linalg.norm(v - phi) / __import__("numpy").linalg.norm(phi))
    return line


def naive_run(cbc, name, stream, steps):
    """The naive contract-then-SVD baseline (Sec. III C) timed on the GPU beside CBC."""
    from paper_2601_19650_amd.inputs import config_problem
    p = config_problem(name)
    tree = cbc.Tree.of(p)
    st, so = cbc.pack(p.state, "cuda:0")
    op, oo = cbc.pack(p.op, "cuda:0")
    ctx = new_context(cbc)
    out = {"workload": WORKLOADS[name]}
    for prec in ("mixed", "fp64"):
        comp = cbc.Compressor(ctx, tree, p.max_bond, prec, method="naive", device="cuda:0")
        sec = timed_runs(comp, (op, oo, st, so, 0.0), stream, steps, 2)
        out[prec] = {"value": 1.0 / sec, "unit": "compressions/s", "ms_per_step": sec * 1e3,
                     "workspace_gb": comp.ws_bytes / 1e9}
        print(f"[bench] naive {name} {prec}: {sec * 1e3:.3f} ms/compression", file=sys.stderr,
              flush=True)
        del comp
    return out


def batched_run(args, cbc, p, stream):
    """Throughput of `batch` independent instances of the workload's shape in one launch sequence
    (mixed precision), inputs resident in HBM."""
    import torch
    from paper_2601_19650_amd.inputs import config_problem
    probs = [p] + [config_problem(p.name, seed=1000 + b) for b in range(1, args.batch)]
    tree = cbc.Tree.of(p)
    st, so = cbc.pack_batch([q.state for q in probs], "cuda:0")
    op, oo = cbc.pack_batch([q.op for q in probs], "cuda:0")
    ctx = new_context(cbc)
    comp = cbc.Compressor(ctx, tree, p.max_bond, "mixed", device="cuda:0", batch=args.batch)
    steps = max(2, args.small_steps // 4)
    sec = timed_runs(comp, (op, oo, st, so, 0.0), stream, steps, 1)
    print(f"[bench] batched x{args.batch}: {sec * 1e3:.3f} ms per launch sequence", file=sys.stderr,
          flush=True)
    return {"batch": args.batch, "value": args.batch / sec, "unit": "compressions/s",
            "ms_per_step": sec * 1e3, "steps": steps, "precision": "mixed",
            "contraction_tflops": args.batch * comp.stats.flops[0] / sec / 1e12,
            "workspace_gb": comp.ws_bytes / 1e9}


def uneven_run(count, stream_count=8):
    """Throughput of an uneven batch: `count` instances drawn as tensor trains, binary and ternary
    trees with N in [16, 64], d in {2, 4}, D in [4, 12], max_bond = chi, mixed precision, forked over
    several streams inside one captured graph that is replayed with a single launch. The bond range
    is reduced to chi in [16, 48] (ternary chi <= 16): with the full [16, 128] draw single node steps
    of binary and ternary instances need intermediates of 1e9 elements."""
    import torch
    from paper_2601_19650_amd import cbc
    from paper_2601_19650_amd.inputs import batch_problems
    probs = batch_problems(count=count, seed=5, chi_range=(16, 48), ternary_chi_cap=16)
    ub = cbc.UnevenBatch(probs, precision="mixed", nstreams=stream_count, device="cuda:0",
                         autotune=AUTOTUNE)
    ub.capture()                  # every instance, forked over the streams, in one graph
    ub.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ub.run()                      # one graph launch for the whole batch
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    print(f"[bench] uneven batch of {count}: {sec * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {"instances": count, "value": count / sec, "unit": "compressions/s", "seconds": sec,
            "contraction_tflops": ub.flops() / sec / 1e12, "streams": stream_count,
            "launch": "one captured graph for the whole batch",
            "recipe": "uneven draw (seed 5): MPS/binary/ternary, N 16-64, d 2|4, D 4-12, chi 16-48 "
                      "(ternary <= 16), first instances of the sequence"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3,
                    help="timed compressions of the headline workload per precision")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C4", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None)
    ap.add_argument("--small-steps", type=int, default=20,
                    help="timed compressions of the 8-site, 64-site and tree workloads (0: skip)")
    ap.add_argument("--batch", type=int, default=64,
                    help="instances of the 64-site shape per launch sequence (0: skip)")
    ap.add_argument("--uneven", type=int, default=16,
                    help="instances of the uneven batch workload to time (0: skip)")
    ap.add_argument("--src", choices=["on", "off"], default="on",
                    help="also time the randomised compression (cbc_apply_src) on the headline "
                         "workload, with the errors of it and of CBC against the exact product")
    ap.add_argument("--zipup", choices=["on", "off"], default="on",
                    help="also time Zip-Up (cbc_apply_zipup) on the headline workload")
    ap.add_argument("--dm", choices=["on", "off"], default="off",
                    help="also time the density-matrix method (cbc_apply_dm) on the headline "
                         "workload (seconds per compression there; the random-network section "
                         "times it by default)")
    ap.add_argument("--uneven-full", action="store_true",
                    help="also time the whole 256-instance uneven draw (several minutes)")
    ap.add_argument("--paper", choices=["off", "short", "full"], default="short",
                    help="random-network workload of the paper's Sec. IV A: CBC and naive over target "
                         "bonds (short: four of the tensor train's twenty)")
    ap.add_argument("--autotune", choices=["on", "off"], default="on",
                    help="tune the contractions' tile and split per shape before timing (cbc_autotune)")
    ap.add_argument("--sites", type=int, default=0,
                    help="cut the headline workload to its first N nodes (profiler runs of its bulk "
                         "node shapes; 0: the full workload)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times) and exit; used to "
                         "scale the HBM byte counters of a profiler run")
    args = ap.parse_args()
    global AUTOTUNE
    AUTOTUNE = args.autotune == "on"
    args.src = args.src == "on"
    args.dm = args.dm == "on"
    args.zipup = args.zipup == "on"
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2601_19650_amd import cbc
    from paper_2601_19650_amd.inputs import config_problem

    torch.cuda.set_device(0)
    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": n * 4, "bytes_written": n * 4,
                                               "launches": 5}}))
        return
    p = config_problem(args.workload, n=args.sites) if args.sites > 0 else config_problem(args.workload)
    stream = torch.cuda.Stream()
    precs = [args.only] if args.only else ["mixed", "fp64"]
    res, outputs = measure(cbc, p, precs, args.steps, args.warmup, stream)

    head = precs[0]
    r = res[head]
    sec = r["sec"]
    cls = cbc.CLASSES
    # dominant kernel class by profiled time
    kd = max(range(cbc.NCLASS), key=lambda k: r["kms"][k])
    launches = r["stats"][cls[kd]]["launches"]
    avg_ms = r["kms"][kd] / max(launches, 1)
    flops_per_launch = r["stats"][cls[kd]]["flops"] / max(launches, 1)
    if cls[kd] in ("contract",):
        bound, peak = "mfma", PEAK["fp32_mfma"] if head == "mixed" else PEAK["fp64_mfma"]
    elif cls[kd] in ("gram", "qrmul"):
        bound, peak = "mfma", PEAK["fp64_mfma"]
    else:
        bound, peak = "alu", PEAK["fp64_alu"]
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    contraction_flops = r["stats"]["contract"]["flops"]
    line = {
        "metric": "CBC compressions/s (mixed FP32-MFMA contractions + FP64 Gram/eigen/Cholesky)",
        "value": 1.0 / sec,
        "unit": "compressions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if head == "mixed" else "c128",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + (
                       f", cut to {p.n} sites" if args.sites > 0 else ""), "name": args.workload,
                   "precision": head, "max_bond": p.max_bond, "n_nodes": p.n,
                   "contraction_config": "autotuned" if AUTOTUNE else "fixed policy"},
        "contraction_tflops": contraction_flops / sec / 1e12,
        "roofline": {"bound": bound, "kernel": cls[kd], "achieved": achieved,
                     "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved * 1e12 / peak,
                     "traffic": recorded_traffic(args.workload, head, cls[kd]), "avg_launch_ms": avg_ms,
                     "flops_per_launch": flops_per_launch},
        "contraction_roofline": contraction_roofline(r, head, cls),
        "kernel_ms_per_step": {cls[k]: r["kms"][k] for k in range(cbc.NCLASS)},
        "kernels_per_step": r["n_kernels"],
        "graph_replayed": r["replayed"],
    }
    if "fp64" in res and "mixed" in res:
        line["fp64"] = precision_line(res["fp64"], "fp64", cls, cbc.NCLASS)
        line["speedup_mixed_vs_fp64"] = res["fp64"]["sec"] / res["mixed"]["sec"]
        if args.workload == "C4" and args.sites == 0:
            # At 128 sites the compressed state is ill-conditioned (a rounding-level input change
            # grows ~1.6x per site), so mixed and FP64 results are compared by the weight they
            # capture; the non-root nodes are isometries, so ||psi'||^2 is the root's squared norm.
            w = {k: float(sum(abs(x) ** 2 for x in v[0].reshape(-1))) for k, v in outputs.items()}
            line["full_size_mixed_vs_fp64"] = {
                "captured_weight": w, "captured_weight_ratio": w["mixed"] / w["fp64"],
                "fidelity": _chain_fidelity(outputs["mixed"], outputs["fp64"])}
    methods = [m for m, on in (("src", args.src), ("zipup", args.zipup), ("dm", args.dm)) if on]
    if methods:
        line["other_methods"] = other_methods(cbc, p, stream, args.steps, args.warmup, outputs,
                                              methods)
    del outputs
    if args.small_steps > 0:
        line["small_workloads"] = {}
        for name in ("C1", "C2", "C3"):
            if name == args.workload:
                continue
            line["small_workloads"][name] = small_workload(cbc, name, stream, args.small_steps)
            print(f"[bench] {name}: mixed {line['small_workloads'][name]['mixed']['value']:.1f} "
                  f"compressions/s", file=sys.stderr, flush=True)
        line["naive_baseline"] = naive_run(cbc, "C2", stream, max(2, args.small_steps // 4))
    if args.batch > 1:
        line["batched"] = batched_run(args, cbc, config_problem("C2"), stream)
    if args.uneven > 0:
        line["uneven_batch"] = uneven_run(args.uneven)
    if args.uneven_full:
        line["uneven_full_draw"] = uneven_full_run()
    if args.paper != "off":
        line["paper_random_networks"] = paper_workloads(cbc, stream, full=args.paper == "full")
    if not args.no_cpu_baseline and args.workload == "C4" and args.sites == 0:
        cb, errs = cpu_baseline_large(cbc)
        line["cpu_baseline"] = cb
        line["error_vs_oracle"] = {"C4 shape, 10 sites": errs}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
