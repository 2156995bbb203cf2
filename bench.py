"""Benchmark: chemistry cell-steps/s (FP64) on the RDE-shaped 1,048,576-cell
field, persistent vs plain form at the same tolerance, with the FP64 ALU
roofline of the integration kernel and the CPU oracle as a baseline.

One step = every cell of the field advanced over one flow step dt = 5e-9 s
(rtol 1e-8, atol 1e-12), starting each step from the same initial field (a
device-to-device restore is part of the step).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12          # MI355X FP64 vector peak, FLOP/s
RODAS4_STAGES = 6
TRAFFIC_PROFILE = "profiles/chem_persistent_rde1m_counters.md"
_T_START = time.perf_counter()


def progress(msg: str) -> None:
    """One line on stderr as each part of the run ends (the JSON line alone
    goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(mech_file: str) -> str:
    """Identity of a mechanism's device code: the complete source the library
    generates and compiles for it (dumped through CHEM_DUMP_SOURCE while a
    handle is loaded) plus the file that holds the compile options.  HBM
    traffic and counters recorded under profiles/ apply only while it is
    unchanged."""
    import hashlib
    import tempfile

    from paper_2508_16105_amd import _lib
    with tempfile.TemporaryDirectory() as d:
        dump = os.path.join(d, "source.hip")
        old = os.environ.get("CHEM_DUMP_SOURCE")
        os.environ["CHEM_DUMP_SOURCE"] = dump
        try:
            h = _lib.load_mechanism_handle(os.path.join(ROOT, mech_file))
            _lib.lib().chem_free_mechanism(h)
        finally:
            if old is None:
                del os.environ["CHEM_DUMP_SOURCE"]
            else:
                os.environ["CHEM_DUMP_SOURCE"] = old
        with open(dump, "rb") as fh:
            src = fh.read()
    hh = hashlib.sha256(src)
    with open(os.path.join(ROOT, "paper_2508_16105_amd/csrc/module.cpp"), "rb") as fh:
        hh.update(fh.read())
    return hh.hexdigest()[:16]


def recorded_traffic(mech_file: str):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE for the
    current kernel sources, or None if the kernel changed since."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    want = kernel_source_hash(mech_file)
    if f"kernel source hash: {want}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith("| HBM bytes per launch |"):
            return float(line.strip("| \n").split("|")[-1])
    return None


def recorded_counters(mech_file: str):
    """SQ counters per launch of the headline kernel from the committed
    rocprofv3 summary, or None if the kernel changed since it was taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if f"kernel source hash: {kernel_source_hash(mech_file)}" not in text:
        return None
    out = {}
    for line in text.splitlines():
        parts = [x.strip() for x in line.strip().strip("|").split("|")]
        if len(parts) == 2 and parts[0].startswith("SQ_"):
            try:
                out[parts[0]] = float(parts[1])
            except ValueError:
                pass
    return out or None


def flops_per_substep(ns: int, nr: int, s: int = RODAS4_STAGES) -> float:
    """Algorithmic FP64 flops of one RODAS4 substep attempt (FMA = 2 flops):
    Jacobian 50 nr + 4 n^2, LU (2/3) n^3, and per stage a source-term
    evaluation 40 ns + 30 nr, two triangular solves 2 n^2 and the stage
    combinations 2 s n.  Transcendentals (2 nr + 1 per source evaluation)
    are not counted."""
    n = ns + 1
    f_rhs = 40 * ns + 30 * nr
    f_jac = 50 * nr + 4 * n * n
    return f_jac + (2.0 / 3.0) * n**3 + s * (f_rhs + 2 * n * n + 2 * s * n)


def host_cores() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    return len(os.sched_getaffinity(0))


def cpu_baseline(T, p, Y, w, frac, seed=7):
    """The oracle on a uniform random sample of the field (the same mix of
    fresh, front and burnt cells), all host cores."""
    import oracle
    from workloads import mech_path
    om = oracle.Mechanism(mech_path(w["mech"]))
    rng = np.random.default_rng(seed)
    n = max(1, int(frac * len(T)))
    idx = np.sort(rng.choice(len(T), n, replace=False))
    cores = host_cores()
    t0 = time.perf_counter()
    om.integrate(T[idx], p[idx], Y[idx], w["dt"], w["rtol"], w["atol"], nthreads=cores)
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} cells ({frac:.0%} uniform random sample of the field, seed {seed}), "
                      f"{el:.2f} s wall"}


def amr_leg(chem, torch, dev, steps, plain_mechs=("m9", "m13"), mechs=None):
    """64 independent fields of log-uniform 10k-2M cells (28.0 M cells in all),
    RDE-shaped states, for the 9- and the 13-species (third-body + Troe)
    mechanism: one persistent work-stealing launch over all fields against one
    plain launch per field, same tolerances.  Each timed step restores the
    initial fields first (device-to-device copies, inside the timing)."""
    from workloads import WORKLOADS, mech_path, mech_text
    from workloads.states import amr_field_sizes, rde_field_n
    w = WORKLOADS["amr64"]
    sizes = amr_field_sizes(w["seed"], w["n_fields"])
    out = {"workload": "amr64", "fields": len(sizes), "cells": int(sum(sizes)), "dt": w["dt"],
           "rtol": w["rtol"], "atol": w["atol"]}
    for name in (mechs or w["mechs"]):
        mech = chem.Mechanism(mech_path(name))
        text = mech_text(name)
        init, work = [], []
        for i, n in enumerate(sizes):
            T, p, Y, _ = rde_field_n(text, n, w["seed"] * 100 + i)
            t = [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev) for a in (T, p, Y)]
            init.append(t)
            work.append([x.clone() for x in t])

        def restore():
            for (T0, _, Y0), (Tw, _, Yw) in zip(init, work):
                Tw.copy_(T0)
                Yw.copy_(Y0)

        def persistent(stats=False):
            return chem.integrate_batched(mech, [f[0] for f in work], [f[1] for f in work],
                                          [f[2] for f in work], w["dt"], w["rtol"], w["atol"],
                                          form=chem.FORM_PERSISTENT, stats=stats)

        def plain():
            for Tw, pw, Yw in work:
                chem.integrate(mech, Tw, pw, Yw, w["dt"], w["rtol"], w["atol"], form=chem.FORM_PLAIN,
                               inplace=True, stats=False)

        restore()
        st = persistent(stats=True)                      # autotunes on first use
        res = {}
        legs = [("persistent", persistent)] + ([("plain_per_field", plain)] if name in plain_mechs else [])
        for form, fn in legs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                restore()
                fn()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / steps
            res[form] = {"ms_per_step": ms, "cell_steps_per_s": out["cells"] / (ms * 1e-3)}
        if "plain_per_field" in res:
            res["persistent_over_plain"] = res["plain_per_field"]["ms_per_step"] / res["persistent"]["ms_per_step"]
        res["substeps"] = st["accepted"] + st["rejected"]
        res["failed"] = st["failed"]
        res["mechanism"] = f"{name} ({mech.ns} species, {mech.nr} reactions)"
        out[name] = res
        del init, work, mech
        torch.cuda.empty_cache()
    return out


def big_leg(chem, torch, dev, steps):
    """The 2048 x 2048 RDE-shaped field (4,194,304 cells) with the 32-species /
    150-reaction mechanism (third-body + Troe on 15 reactions), which runs in
    the wave-cooperative form (one 64-lane wave per cell): plain and
    persistent launches, same tolerances."""
    from workloads import WORKLOADS, mech_path, mech_text
    from workloads.states import rde_field
    w = WORKLOADS["big4m"]
    mech = chem.Mechanism(mech_path(w["mech"]))
    T, p, Y, _ = rde_field(mech_text(w["mech"]), w["width"], w["height"], w["seed"])
    n = len(T)
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    T0, p0, Y0 = t(T), t(p), t(Y)
    Tw, Yw = T0.clone(), Y0.clone()
    fper = flops_per_substep(mech.ns, mech.nr)
    out = {"workload": "big4m", "cells": n, "mechanism": f"{w['mech']} ({mech.ns} species, {mech.nr} reactions)",
           "dt": w["dt"], "rtol": w["rtol"], "atol": w["atol"], "flops_per_substep": fper}
    for name, form in (("persistent", chem.FORM_PERSISTENT), ("plain", chem.FORM_PLAIN)):
        def step(stats=False):
            Tw.copy_(T0)
            Yw.copy_(Y0)
            return chem.integrate(mech, Tw, p0, Yw, w["dt"], w["rtol"], w["atol"], form=form, inplace=True,
                                  stats=stats)[2]
        st = step(stats=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        subs = st["accepted"] + st["rejected"]
        out[name] = {"ms_per_step": ms, "cell_steps_per_s": n / (ms * 1e-3), "substeps": subs,
                     "max_substeps_cell": st["max_substeps"], "kernel_ms": st["kernel_ms"],
                     "achieved_tflops": subs * fper / (ms * 1e-3) / 1e12,
                     "frac_fp64_peak": subs * fper / (ms * 1e-3) / PEAK_FP64_VALU}
    return out


def adjoint_leg(chem, torch, dev, steps, cpu_cells, workload="adj256k"):
    """The discrete adjoint on the 512 x 512 adjoint field (262,144 cells, dt
    1e-8 s, 9 species), or on the 2048 x 2048 32-species field (wave-
    cooperative form): L = sum over cells of T_end / 1000 K + Y_H2O,end;
    gradients with respect to T0, Y0 and every reaction's ln A, b, Ea.  Times
    whole calls (sizing pass, arena set-up, adjoint kernel, parameter
    reduction) against the forward integration of the same field in both
    forms."""
    from workloads import WORKLOADS, mech_path, mech_text
    from workloads.states import parse_species, rde_field
    w = WORKLOADS[workload]
    mech = chem.Mechanism(mech_path(w["mech"]))
    T, p, Y, _ = rde_field(mech_text(w["mech"]), w["width"], w["height"], w["seed"])
    n = len(T)
    species = parse_species(mech_text(w["mech"]))[0]
    gT = np.full(n, 1.0 / w.get("t_ref", 1000.0))
    gY = np.zeros((n, len(species)))
    gY[:, species.index("H2O")] = 1.0
    t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    T0, p0, Y0, gTd, gYd = t(T), t(p), t(Y), t(gT), t(gY)
    args = (mech, T0, p0, Y0, w["dt"], w["rtol"], w["atol"])
    fwd = {}
    for name, form in (("plain", chem.FORM_PLAIN), ("persistent", chem.FORM_PERSISTENT)):
        chem.integrate(*args, form=form)                                # warm (and tune)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            chem.integrate(*args, form=form)
        fwd[name] = 1e3 * (time.perf_counter() - t0) / steps
    # the workload's checkpoint interval: every 4th accepted substep
    chem.integrate_adjoint(*args, gTd, gYd, checkpoint_every=4)       # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kms = []
    for _ in range(steps):
        out = chem.integrate_adjoint(*args, gTd, gYd, checkpoint_every=4)
        kms.append(out[7]["kernel_ms"])
    adj_ms = 1e3 * (time.perf_counter() - t0) / steps
    st = out[7]
    # the library's default interval (every step when the arena fits), one call;
    # and the workload's interval given the step counts of a forward
    # integration of the same field (as in autograd, where the forward ran
    # first), which spares the sizing pass
    auto = hinted = None
    if workload == "adj256k":
        nacc = chem.integrate(*args, form=chem.FORM_PERSISTENT, return_counts=True)[4]
        chem.integrate_adjoint(*args, gTd, gYd, checkpoint_every=4, forward_nacc=nacc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            oh = chem.integrate_adjoint(*args, gTd, gYd, checkpoint_every=4, forward_nacc=nacc)
        hinted = {"ms_per_call": 1e3 * (time.perf_counter() - t0) / steps,
                  "adjoint_kernel_ms": oh[7]["kernel_ms"], "checkpoint_every": 4}
        # what ChemIntegrate's backward runs: the forward's counts, the default interval
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ob = chem.integrate_adjoint(*args, gTd, gYd, forward_nacc=nacc)
        hinted["default_checkpoints_ms_per_call"] = 1e3 * (time.perf_counter() - t0)
        hinted["default_checkpoints_kernel_ms"] = ob[7]["kernel_ms"]
        chem.integrate_adjoint(*args, gTd, gYd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        oa = chem.integrate_adjoint(*args, gTd, gYd)
        auto = {"ms_per_call": 1e3 * (time.perf_counter() - t0), "adjoint_kernel_ms": oa[7]["kernel_ms"],
                "checkpoint_every": "densest interval whose arena fits a quarter of free memory (1 here)"}
    res = {"workload": workload, "cells": n,
           "mechanism": f"{w['mech']} ({mech.ns} species, {mech.nr} reactions)",
           "dt": w["dt"], "params": 3 * mech.nr,
           "ms_per_call": adj_ms, "adjoint_kernel_ms": float(np.mean(kms)),
           "forward_ms": fwd, "adjoint_over_forward": {k: adj_ms / v for k, v in fwd.items()},
           "cell_steps_per_s": n / (adj_ms * 1e-3),
           "accepted": st["accepted"], "max_substeps_cell": st["max_substeps"],
           "checkpoint_every": 4,
           "lane_groups": "cells >= 0.6 x the largest step count on 8-lane groups (one cell per lane form)"}
    if auto:
        res["default_checkpoints"] = auto
    if hinted:
        res["with_forward_step_counts"] = hinted
    if cpu_cells:
        import oracle
        om = oracle.Mechanism(mech_path(w["mech"]))
        idx = np.sort(np.random.default_rng(8).choice(n, cpu_cells, replace=False))
        cores = host_cores()
        t0 = time.perf_counter()
        om.adjoint(T[idx], p[idx], Y[idx], w["dt"], w["rtol"], w["atol"], gT[idx], gY[idx],
                   nthreads=cores)
        el = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": cpu_cells / el, "unit": "cell-steps/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{cpu_cells} cells (uniform random sample of the field, "
                                         f"seed 8), {el:.2f} s wall"}
    return res


def euler_leg(chem, torch, dev, n=65536, steps=20, warmup=3):
    """The 1D reactive-Euler driver (chem_euler1d_step): a detonation tube of
    n cells of 25 um with the one-step global H2-air reaction (3000 K / 40 atm
    driver over the first 5 %, stoichiometric H2-air at 300 K / 1 atm), dt =
    2 ns; time per driver step (primitive recovery, coupled chemistry step,
    flux update, and the host synchronisation the step does for its checks)."""
    import tempfile
    from workloads import tiny
    from workloads.states import parse_species, stoich_air
    text = tiny.global_h2_air()
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "global.mech")
        with open(path, "w") as f:
            f.write(text)
        gm = chem.Mechanism(path)
    names, W = parse_species(text)
    Y0 = stoich_air(names, W)
    dx, dt = 2.5e-5, 2e-9
    hot = np.arange(n) < n // 20
    g = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    T = g(np.where(hot, 3000.0, 300.0))
    U = chem.euler1d_init(gm, T, g(np.where(hot, 40 * 101325.0, 101325.0)), g(np.tile(Y0, (n, 1))))
    for _ in range(warmup):
        U, T, _, cfl = chem.euler1d_step(gm, U, dx, dt, T=T, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        U, T, _, cfl = chem.euler1d_step(gm, U, dx, dt, T=T, stats=False)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    return {"cells": n, "steps": steps, "ms_per_step": ms, "cell_steps_per_s": n / (ms * 1e-3),
            "mechanism": "one-step global H2-air (4 species)", "dt": dt, "dx": dx, "max_cfl": cfl}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rde1m")
    ap.add_argument("--cpu-sample", type=float, default=0.05)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="persistent,persistent_adjacent,persistent_history,"
                                        "persistent_natural,plain")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-euler", action="store_true")
    ap.add_argument("--no-amr", action="store_true")
    ap.add_argument("--no-big", action="store_true")
    ap.add_argument("--big-only", action="store_true")
    ap.add_argument("--amr-only", action="store_true")
    ap.add_argument("--amr-mechs", default="m9,m13", help="mechanisms of the batched leg (--amr-only)")
    ap.add_argument("--amr-plain", default="m9,m13", help="mechanisms whose per-field plain launches are timed")
    ap.add_argument("--adjoint-only", action="store_true")
    ap.add_argument("--adjoint-cpu-cells", type=int, default=192)
    ap.add_argument("--adjoint-workload", default="adj256k")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 512 MiB device to device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (cells are "
              f"independent, so a multi-GPU run would shard the field by predicted cost).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        a = torch.empty(64 << 20, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8}))
        return
    import paper_2508_16105_amd as chem
    from workloads import WORKLOADS, mech_path, mech_text
    from workloads.states import rde_field

    if args.big_only:
        print(json.dumps({"big4m": big_leg(chem, torch, torch.device("cuda:0"), max(1, args.steps))}))
        return
    if args.amr_only:
        print(json.dumps({"amr64": amr_leg(chem, torch, torch.device("cuda:0"), max(1, args.steps),
                                           plain_mechs=tuple(x for x in args.amr_plain.split(",") if x),
                                           mechs=[x for x in args.amr_mechs.split(",") if x])}))
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(chem, torch, torch.device("cuda:0"), max(1, args.steps),
                                                 0 if args.no_cpu else args.adjoint_cpu_cells,
                                                 args.adjoint_workload)}))
        return

    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    mech = chem.Mechanism(mech_path(w["mech"]))
    T, p, Y, reg = rde_field(mech_text(w["mech"]), w["width"], w["height"], w["seed"])
    ncell = len(T)
    T0 = torch.tensor(T, device=dev)
    Y0 = torch.tensor(Y, device=dev)
    pg = torch.tensor(p, device=dev)
    Tw, Yw = T0.clone(), Y0.clone()
    stream = torch.cuda.current_stream()
    fper = flops_per_substep(mech.ns, mech.nr)
    # persistent: cells started most-expensive-first, cost predicted from the state;
    # persistent_adjacent: cost = each cell's substep count in the adjacent flow
    # step of the same field (the field one dt later), as a time-stepping solver
    # has it from its previous step;
    # persistent_history: cost = substep counts of this very step (upper bound);
    # persistent_natural: index order; plain: one launch, one cell per lane.
    forms = {"persistent": (chem.FORM_PERSISTENT, {}),
             "persistent_adjacent": (chem.FORM_PERSISTENT, {"adjacent": True}),
             "persistent_history": (chem.FORM_PERSISTENT, {"history": True}),
             "persistent_natural": (chem.FORM_PERSISTENT, {"order": chem.ORDER_NATURAL}),
             "plain": (chem.FORM_PLAIN, {})}
    _, _, _, _, na0, nr0 = chem.integrate(mech, T0, pg, Y0, w["dt"], w["rtol"], w["atol"],
                                          form=chem.FORM_PLAIN, return_counts=True)
    prev_cost = (na0 + nr0).contiguous()
    T1, Y1, _ = chem.integrate(mech, T0, pg, Y0, w["dt"], w["rtol"], w["atol"], form=chem.FORM_PLAIN)
    _, _, _, _, na1, nr1 = chem.integrate(mech, T1, pg, Y1, w["dt"], w["rtol"], w["atol"],
                                          form=chem.FORM_PLAIN, return_counts=True)
    adjacent_cost = (na1 + nr1).contiguous()
    del T1, Y1

    results = {}
    for name in args.forms.split(","):
        form, extra = forms[name]
        kw = {}
        if extra.get("history"):
            kw["cost"] = prev_cost
        if extra.get("adjacent"):
            kw["cost"] = adjacent_cost
        if "order" in extra:
            kw["order"] = extra["order"]

        def step(stats=False):
            Tw.copy_(T0)
            Yw.copy_(Y0)
            return chem.integrate(mech, Tw, pg, Yw, w["dt"], w["rtol"], w["atol"], form=form,
                                  inplace=True, stats=stats, **kw)[2]

        st = step(stats=True)                      # includes the autotune on first use
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for i in range(args.steps):
            Tw.copy_(T0)
            Yw.copy_(Y0)
            ev[i][0].record(stream)
            chem.integrate(mech, Tw, pg, Yw, w["dt"], w["rtol"], w["atol"], form=form,
                           inplace=True, stats=False, **kw)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        subs = st["accepted"] + st["rejected"]
        progress(f"{args.workload} {name}: {1e3 * wall / args.steps:.2f} ms per step")
        results[name] = dict(ms_per_step=1e3 * wall / args.steps, kernel_ms=kms,
                             cell_steps_per_s=ncell * args.steps / wall,
                             substeps=subs, accepted=st["accepted"], rejected=st["rejected"],
                             max_substeps_cell=st["max_substeps"],
                             achieved_tflops=subs * fper / (kms * 1e-3) / 1e12)

    head = "persistent" if "persistent" in results else next(iter(results))
    r = results[head]
    line = {
        "metric": "chemistry cell-steps/s (FP64) + % FP64 peak; persistent vs plain, same tol",
        "value": r["cell_steps_per_s"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": ncell,
                   "mechanism": f"{w['mech']} ({mech.ns} species, {mech.nr} reactions)",
                   "dt": w["dt"], "rtol": w["rtol"], "atol": w["atol"], "form": head,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": r["achieved_tflops"], "peak": PEAK_FP64_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": r["achieved_tflops"] / (PEAK_FP64_VALU / 1e12),
                     "traffic": recorded_traffic(os.path.relpath(mech_path(w["mech"]), ROOT))
                     if head in ("persistent", "persistent_adjacent", "persistent_history") else None,
                     "kernel": "chem_persistent" if head == "persistent" else "chem_plain",
                     "kernel_ms": r["kernel_ms"],
                     "flops_per_substep": fper, "substeps_per_launch": r["substeps"]},
        "forms": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in results.items()},
    }
    # the field's critical path: its most expensive cell integrated alone (one
    # lane of one wave), which no schedule of the whole field can beat
    tot = (na0 + nr0).cpu().numpy()
    ci = int(np.argmax(tot))
    Tc, pc, Yc = T0[ci:ci + 1].clone(), pg[ci:ci + 1].clone(), Y0[ci:ci + 1].clone()
    chem.integrate(mech, Tc, pc, Yc, w["dt"], w["rtol"], w["atol"], form=chem.FORM_PLAIN)
    solo = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        chem.integrate(mech, Tc, pc, Yc, w["dt"], w["rtol"], w["atol"], form=chem.FORM_PLAIN, stats=False)
        b.record(stream)
        torch.cuda.synchronize()
        solo.append(a.elapsed_time(b))
    solo_ms = float(np.median(solo))
    line["critical_path"] = {"cell": ci, "substeps": int(tot[ci]), "solo_ms": solo_ms,
                             "us_per_substep": 1e3 * solo_ms / max(1, int(tot[ci])),
                             "of_kernel_ms": solo_ms / r["kernel_ms"]}
    ctr = recorded_counters(os.path.relpath(mech_path(w["mech"]), ROOT)) if head == "persistent" else None
    if ctr and "SQ_INSTS_VALU" in ctr:
        wave_substeps = r["substeps"] / 64.0
        c = {"profile": TRAFFIC_PROFILE, "SQ_INSTS_VALU": ctr["SQ_INSTS_VALU"],
             "valu_per_wave_substep": ctr["SQ_INSTS_VALU"] / wave_substeps}
        if "SQ_INSTS_VALU_FLOPS_FP64" in ctr:
            # counted per wave instruction: x 64 lanes, inactive lanes and the
            # exp/log sequences included
            tf = ctr["SQ_INSTS_VALU_FLOPS_FP64"] * 64 / (r["kernel_ms"] * 1e-3) / 1e12
            c["fp64_counter_tflops"] = tf
            c["fp64_counter_frac"] = tf / (PEAK_FP64_VALU / 1e12)
        if "SQ_THREAD_CYCLES_VALU" in ctr and "SQ_ACTIVE_INST_VALU" in ctr:
            c["valu_utilization"] = ctr["SQ_THREAD_CYCLES_VALU"] / (64.0 * ctr["SQ_ACTIVE_INST_VALU"])
        line["counters"] = c
    if "plain" in results and "persistent" in results:
        line["persistent_over_plain"] = results["plain"]["ms_per_step"] / results["persistent"]["ms_per_step"]
    if "persistent" in results:
        # the operator-split coupling: the same persistent step returning the
        # mean reaction rates wdot and heat release qdot (chem_integrate_source)
        def source_step():
            Tw.copy_(T0)
            Yw.copy_(Y0)
            return chem.integrate_source(mech, Tw, pg, Yw, w["dt"], w["rtol"], w["atol"],
                                         form=chem.FORM_PERSISTENT, inplace=True, stats=False)
        source_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            source_step()
        torch.cuda.synchronize()
        sms = 1e3 * (time.perf_counter() - t0) / args.steps
        line["source_mode"] = {"form": "persistent", "ms_per_step": sms,
                               "over_integrate": sms / results["persistent"]["ms_per_step"]}
    if not args.no_euler:
        line["euler1d"] = euler_leg(chem, torch, dev)
        progress("1D driver leg done")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(T, p, Y, w, args.cpu_sample)
        progress("CPU baseline done")
    if not args.no_amr:   # the 13-species per-field plain launches (~80 s) only with --amr-only
        line["amr64"] = amr_leg(chem, torch, dev, 1, plain_mechs=("m9",))
        progress("64-field leg done")
    if not args.no_big:
        line["big4m"] = big_leg(chem, torch, dev, 2)
        progress("32-species field done")
    if not args.no_adjoint:
        line["adjoint"] = adjoint_leg(chem, torch, dev, 1, 0 if args.no_cpu else args.adjoint_cpu_cells)
        progress("adjoint done")
        if not args.no_big:
            line["adjoint_big4m"] = adjoint_leg(chem, torch, dev, 1, 0 if args.no_cpu else 16, "big4m")
            progress("32-species adjoint done")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
