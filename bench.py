#!/usr/bin/env python3
"""Throughput of the DG Euler hot path (fused RHS + LSERK45 stage update) on
one MI355X, in GDOF-RK-stages per second (solution nodes x RK stages / s, the
paper's DOF count: Section V), with the roofline of the dominant kernel and
the CPU oracle timed on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--precision fp64|fp32]

One bench step is one LSERK45 time step (five fused stages) over the whole
mesh.  The timed region is one call that advances K steps, bracketed by
device synchronisation; Q and res are resident in HBM before it starts.
Prints ONE JSON line.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0         # MI355X HBM3E, published
FP64_PEAK_TFS = 78.6          # MI355X FP64 vector, published
ALG_BYTES_PER_DOF_STAGE = 160  # read Q, res; write Q, res (FP64, 5 fields)
ALG_BYTES_PER_DOF_FIRST_STAGE = 120  # first stage (a = 0): read Q; write Q, res

WORKLOADS = {
    # name: (n, p, steps of the configuration, description)
    "tgv32_p3": (32, 3, 100, "Taylor-Green vortex, [0,2pi]^3, Mach 0.1, 32^3 elements, p=3, "
                             "dt from CFL 0.3, 100 LSERK45 steps"),
    "tgv48_p4": (48, 4, 50, "Taylor-Green vortex, [0,2pi]^3, Mach 0.1, 48^3 elements, p=4 "
                            "(one GPU's share at the paper's per-GPU size), 50 LSERK45 steps"),
    "tgv48_p4_re1600": (48, 4, 50, "viscous Taylor-Green vortex (Navier-Stokes, BR1 viscous terms), [0,2pi]^3, "
                                   "Mach 0.1, Re 1600 (mu = 1/1600, Pr 0.71), 48^3 elements, p=4, 50 LSERK45 steps"),
    "tgv48_p4_kep": (48, 4, 50, "Taylor-Green vortex with the kinetic-energy-preserving split form (Kennedy-Gruber "
                                "two-point flux), [0,2pi]^3, Mach 0.1, 48^3 elements, p=4, 50 LSERK45 steps"),
    "tgv40_p6": (40, 6, 100, "Taylor-Green vortex, [0,2pi]^3, Mach 0.1, 40^3 elements, p=6 "
                             "(the paper's degree), 100 LSERK45 steps"),
    "adjoint16_p3": (16, 3, 40, "gradient of the integrated kinetic energy after 40 LSERK45 steps with respect to "
                                "the initial state: perturbed Taylor-Green vortex (seed 1, amplitude 1e-2), 16^3 "
                                "elements, p=3, dt from CFL 0.3, Q checkpointed every 8 steps; one bench step is "
                                "one whole gradient (forward pass, recomputation and reverse pass)"),
    "tgv48_varp": (48, None, 50, "Taylor-Green vortex, [0,2pi]^3, Mach 0.1, 48^3 elements with a degree per "
                                 "element, 3..5 from the initial enstrophy density (p = 3 + round(|curl u|), "
                                 "22/72/5% of the elements, 6% of the faces between two degrees), mortar faces "
                                 "between degrees, dt from CFL 0.3 at the highest degree, 50 LSERK45 steps"),
    "tgv40_hp": (40, None, 50, "Taylor-Green vortex, [0,2pi]^3, Mach 0.1, 40^3 cells, the cells of initial "
                               "enstrophy indicator |curl u|/2 >= 0.7 refined once into 2x2x2 children (7.8% of "
                               "the cells, 98944 elements), degrees 3..5 from the indicator (children take their "
                               "cell's), 14.0 M nodes, mortar faces between degrees and hanging faces between "
                               "sizes, dt from CFL 0.3 at the highest degree and smallest element, 50 LSERK45 "
                               "steps"),
    "batch512": (None, None, 20, "512 independent periodic meshes from seed 15698: density waves on "
                                 "[0,1]^3 and TGVs on [0,2pi]^3, n^3 elements with n uniform in 6..24, "
                                 "p uniform in 1..5, amplitudes uniform in [0.05,0.3], each mesh with "
                                 "its own CFL-0.3 dt; per RK stage one launch per degree present, "
                                 "graph-replayed"),
}


# Viscous workloads: (dynamic viscosity, Prandtl number).
VISCOUS = {"tgv48_p4_re1600": (1.0 / 1600.0, 0.71)}
# Bytes per node and stage of the viscous decomposition (FP64, 5 fields, 12
# viscous-flux values).  Fused (default): k_visc_flux forms the inviscid rate
# too (read Q, write the flux and R) 176; k_visc_apply (read the flux, R, Q,
# res; write Q, res) 296.  Separate: the inviscid rate (read Q, write R) 80,
# k_visc_flux (read Q, write the flux) 136, k_visc_apply 296.
VISC_BYTES = {"rhs": 80, "visc": 136 + 296}
VISC_BYTES_FUSED = {"visc": 176 + 296}
# Workloads on the split-form volume term (DG_VOLUME_KEP).
SPLIT_FORM = {"tgv48_p4_kep"}


def flops_per_dof_stage(N):
    """Algorithmic flops per node and stage: volume 38 + 30 N (the flop
    model of the paper's volume kernel), surface 3 (40 N + 76) / N (trace
    interpolation, local Lax-Friedrichs flux and lift per face point), inverse
    mass and RK update 30."""
    return 38 + 30 * N + 3 * (40 * N + 76) / N + 30


# The device sources each measured kernel is built from (the C ABI header
# only declares host entry points), per kernel family: the
# single-mesh stage kernel in either precision (neighbour-read form, its
# tables and launch parameters), the batched kernels and the
# neighbour-read adjoint kernel.
_COMMON_SOURCES = ["paper_2006_15698_amd/csrc/dg_internal.h",
                   "paper_2006_15698_amd/csrc/stage_fp64.h", "paper_2006_15698_amd/csrc/stage_nb.h"]
_FP32_SOURCES = ["paper_2006_15698_amd/csrc/stage_fp32.h", "paper_2006_15698_amd/csrc/stage_nb32.h"]
STAGE_SOURCES = {
    "fp64": _COMMON_SOURCES + ["paper_2006_15698_amd/csrc/kern_fp64.hip"],
    "fp32": _COMMON_SOURCES + _FP32_SOURCES + ["paper_2006_15698_amd/csrc/kern_fp32.hip"],
    "batch": _COMMON_SOURCES + _FP32_SOURCES + ["paper_2006_15698_amd/csrc/dg_batch.h",
                                                "paper_2006_15698_amd/csrc/kern_batch.hip",
                                                "paper_2006_15698_amd/csrc/batch_api.cpp"],
    "vjp": _COMMON_SOURCES + ["paper_2006_15698_amd/csrc/kern_vjp.hip"],
    "visc": _COMMON_SOURCES + ["paper_2006_15698_amd/csrc/kern_visc.hip"],
    "split": _COMMON_SOURCES + ["paper_2006_15698_amd/csrc/kern_split.hip"],
    "varp": _COMMON_SOURCES + ["paper_2006_15698_amd/csrc/dg_varp.h", "paper_2006_15698_amd/csrc/kern_varp.hip",
                               "paper_2006_15698_amd/csrc/kern_varp_hang.hip",
                               "paper_2006_15698_amd/csrc/varp_api.cpp"],
}


def _code_only(text):
    """Source text without comments and blank space, so that editing a
    comment does not mark counters stale."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(family="fp64"):
    """Hash of a kernel family's code: counters taken on other code are
    stale."""
    h = hashlib.sha256()
    for f in STAGE_SOURCES[family]:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, family, options):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source
    (family as in STAGE_SOURCES) with the same options."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(f"{workload}:{family}")
    if not ent or ent.get("kernel_src") != kernel_source_hash(family) or ent.get("options") != options:
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(n, p, L, budget_s, viscous=None, split=False):
    """The oracle (plain dense FP64 numpy) advancing RK stages of the same
    workload on the host for about ``budget_s`` seconds.  With viscosity
    (mu, Pr) the Navier-Stokes oracle, and for the split form the split-form
    oracle, runs on a 16^3-element periodic block of the same element size
    and degree (its cost per node is that of the whole mesh; one stage of
    the full 48^3 mesh takes minutes)."""
    import numpy as np
    import workloads as W
    from oracle import lserk
    from oracle.dg import DG
    from oracle.splitform import SplitFormDG
    from oracle.viscous import NavierStokesDG
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count()
    sample = ""
    if viscous is None and not split:
        ora = DG((n, n, n), p, L=L)
        Q = W.tgv(n, p)
    else:
        m = min(n, 16)
        Lm = tuple(Ld * m / n for Ld in L)
        if split:
            ora = SplitFormDG((m, m, m), p, L=Lm)
        else:
            ora = NavierStokesDG((m, m, m), p, L=Lm, mu=viscous[0], prandtl=viscous[1])
        Q = W.tgv(m, p, L=Lm)
        sample = f"a {m}^3-element block of the same element size and degree: "
    res = np.zeros_like(Q)
    dt = ora.dt_cfl(Q, 0.3)
    t0 = time.perf_counter()
    stages = 0
    while True:
        lserk.stage(stages % 5, Q, res, dt, ora.rhs)
        stages += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    dof = ora.num_dof()
    return {"value": dof * stages / el / 1e9, "unit": "GDOF-RK-stages/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample}{stages} RK stages of the same workload ({dof} nodes) in {el:.1f} s; "
                      f"BLAS threads {threads}, host cpu_count {os.cpu_count()}"}


GOLDEN_48 = os.path.join(ROOT, "tests", "golden", "tgv48_p4_50steps.npz")


def _errors_vs_stored_oracle(Qf, Q0, golden):
    """L2 error of a GPU state after the stored run's steps against the
    oracle's state, on the stored sampled elements (all nodes and fields):
    relative to the oracle state and to the oracle's change over the run,
    overall and per field."""
    import numpy as np
    import torch
    ex, ey, ez = (torch.from_numpy(c).to(Qf.device) for c in golden["elems"].T)
    got = Qf[:, ez, ey, ex].cpu().numpy()
    start = Q0[:, ez, ey, ex].cpu().numpy()
    ref = golden["samples"]
    d = (got - ref).reshape(5, -1)
    ch = (ref - start).reshape(5, -1)
    rf = ref.reshape(5, -1)
    return {"l2_rel_state": float(np.linalg.norm(d) / np.linalg.norm(rf)),
            "l2_rel_change": float(np.linalg.norm(d) / np.linalg.norm(ch)),
            "l2_rel_change_per_field": [float(v) for v in np.linalg.norm(d, axis=1) / np.linalg.norm(ch, axis=1)]}


def precision_clause(args, n, p, L, Q0, dt, K, Wm, graph, value):
    """The FP32 matrix-core form against the plain FP64 form on the same GPU:
    the other form's rate over the same Wm + K steps and its stage kernel's
    average launch, the speedup of FP32 over FP64, and the L2 error of both
    forms against the FP64 oracle after the stored oracle run's 50 steps
    from the initial state (48^3 p=4 only; other workloads report the L2
    difference between the two forms after the timed steps)."""
    import numpy as np
    import torch
    from paper_2006_15698_amd import dg

    primary = args.precision
    other = "fp32" if primary == "fp64" else "fp64"
    mode = {"fp64": dg.DG_FP64, "fp32": dg.DG_FP32_MFMA}
    so = dg.Solver((n, n, n), p, L=L, precision=mode[other])
    Qo = Q0.clone()
    ro = torch.zeros_like(Qo)
    if Wm > 0:
        so.step(Qo, ro, dt, nsteps=Wm, graph=graph)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    so.step(Qo, ro, dt, nsteps=K, graph=graph)
    ev1.record()
    torch.cuda.synchronize()
    v_other = n ** 3 * (p + 1) ** 3 * 5 * K / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    dg.dg_set_timing(so.ctx, True)
    so.step(Qo, ro, dt, nsteps=K)
    t = dg.dg_timing_read(so.ctx)
    dg.dg_set_timing(so.ctx, False)
    rates = {primary: value, other: v_other}
    out = {"fp32_value": rates["fp32"], "fp64_value": rates["fp64"], "unit": "GDOF-RK-stages/sec",
           "speedup_fp32_over_fp64": rates["fp32"] / rates["fp64"],
           "steps_timed": K,
           f"{other}_stage_kernel_avg_us": t["stage"][0] / t["stage"][1] * 1e3}
    if args.workload == "tgv48_p4" and os.path.exists(GOLDEN_48):
        golden = dict(np.load(GOLDEN_48, allow_pickle=False))
        gdt, steps = float(golden["dt"]), int(golden["steps"])
        errs = {}
        for form in ("fp64", "fp32"):
            sf = so if form == other else dg.Solver((n, n, n), p, L=L, precision=mode[form])
            Qf = Q0.clone()
            rf = torch.zeros_like(Qf)
            sf.step(Qf, rf, gdt, nsteps=steps)
            torch.cuda.synchronize()
            errs[form] = _errors_vs_stored_oracle(Qf, Q0, golden)
            del Qf, rf
        out["l2_err_vs_oracle"] = errs
        out["error_run"] = (f"{steps} LSERK45 steps from the initial state at the oracle run's dt {gdt:.6e}, "
                            f"untimed; L2 over {golden['elems'].shape[0]} seeded sampled elements "
                            f"(all nodes, all fields) against the stored FP64 oracle state "
                            f"(tests/golden/tgv48_p4_50steps.npz)")
    else:
        fin = {}
        for form in ("fp64", "fp32"):
            sf = so if form == other else dg.Solver((n, n, n), p, L=L, precision=mode[form])
            Qf = Q0.clone()
            rf = torch.zeros_like(Qf)
            sf.step(Qf, rf, dt, nsteps=K)
            fin[form] = Qf
        diff = float(torch.linalg.vector_norm(fin["fp32"] - fin["fp64"]))
        out["l2_diff_between_forms"] = {
            "rel_state": diff / float(torch.linalg.vector_norm(fin["fp64"])),
            "rel_change": diff / float(torch.linalg.vector_norm(fin["fp64"] - Q0)), "steps": K,
            "note": "no stored oracle run for this workload: FP32 form against the GPU's FP64 form"}
    return out


def run_adjoint(args):
    """The adjoint configuration: K whole gradients (forward 40 steps storing
    Q every 8, then per segment recompute the stage inputs and run the stages
    backwards through dg_rk_stage_vjp).  Rate: forward RK stages of the
    gradient's trajectory per second.  Roofline of dg_rhs_vjp (one
    neighbour-read adjoint launch, 120 algorithmic bytes per node: read Q and
    gR, write gQ) from HIP events around each call, at this size and at TGV
    32^3 p=3."""
    import torch
    import workloads as W
    from paper_2006_15698_amd import dg

    n, p, nsteps, desc = WORKLOADS["adjoint16_p3"]
    K = 3 if args.steps is None else args.steps
    L = (2 * math.pi,) * 3
    s = dg.Solver((n, n, n), p, L=L)
    Q0 = torch.from_numpy(W.perturbed_tgv(n, p, seed=1)).cuda()
    dt = s.dt_cfl(Q0, 0.3)
    grad = dg.kinetic_energy_grad(s)
    for _ in range(max(args.warmup, 1)):
        dg.rk_gradient(s, Q0, dt, nsteps, grad, every=8)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        g, _ = dg.rk_gradient(s, Q0, dt, nsteps, grad, every=8)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    dof = s.num_dof
    value = dof * 5 * nsteps / (ms * 1e-3) / 1e9

    def vjp_rate(solver, Q, reps=20):
        """Average duration of dg_rhs_vjp: HIP events on the stream the
        kernel runs on (torch's current stream) around ``reps`` back-to-back
        calls, after three warm-up calls."""
        gR = torch.randn_like(Q)
        out = torch.empty_like(Q)
        for _ in range(3):
            solver.rhs_vjp(Q, gR, out)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            solver.rhs_vjp(Q, gR, out)
        b.record()
        torch.cuda.synchronize()
        avg_s = a.elapsed_time(b) / reps * 1e-3
        nd = solver.num_dof
        return avg_s, 120 * nd / avg_s / 1e9

    avg16, gbs16 = vjp_rate(s, Q0)
    s32 = dg.Solver((32,) * 3, 3, L=L)
    avg32, gbs32 = vjp_rate(s32, torch.from_numpy(W.tgv(32, 3)).cuda())
    return {
        "metric": "GDOF-RK-stages/sec", "value": value, "unit": "GDOF-RK-stages/sec", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"adjoint16_p3: {desc}", "elements": n ** 3, "p": p, "dof": dof, "rk_steps": nsteps,
                   "checkpoint_every": 8, "dt": dt},
        "roofline": {"bound": "hbm", "achieved": gbs32, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs32 / HBM_PEAK_GBS,
                     "traffic": measured_traffic("tgv32_p3", "vjp", s32.options()),
                     "kernel": "k_vjp_nb (dg_rhs_vjp) on TGV 32^3 p=3",
                     "avg_launch_us": avg32 * 1e6, "alg_bytes_per_launch": 120 * s32.num_dof,
                     "at_16p3": {"avg_launch_us": avg16 * 1e6, "achieved": gbs16}},
    }


def run_batch(args):
    """The batched configuration: every mesh advanced together, one
    graph-replayed launch per stage."""
    import torch
    import workloads as W
    from paper_2006_15698_amd import dg

    _, _, cfg_steps, desc = WORKLOADS["batch512"]
    K = cfg_steps if args.steps is None else args.steps
    specs = W.batch_specs(count=512, seed=15698)
    prec = dg.DG_FP64 if args.precision == "fp64" else dg.DG_FP32_MFMA
    b = dg.Batch([(sp["n"],) * 3 for sp in specs], [sp["p"] for sp in specs], [sp["L"] for sp in specs],
                 precision=prec)
    Q0 = b.empty()
    dts = []
    for i, sp in enumerate(specs):
        st = torch.from_numpy(W.batch_state(sp))
        b.view(Q0, i).copy_(st)
    torch.cuda.synchronize()
    for i, sp in enumerate(specs):
        s1 = dg.Solver((sp["n"],) * 3, sp["p"], L=sp["L"])
        dts.append(s1.dt_cfl(b.view(Q0, i), 0.3))
        del s1
    b.set_dt(dts)
    dof = sum(sp["n"] ** 3 * (sp["p"] + 1) ** 3 for sp in specs)
    Q = Q0.clone()
    res = torch.zeros_like(Q)
    b.step(Q, res, nsteps=max(args.warmup, 1), graph=True)
    torch.cuda.synchronize()

    def timed(k):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(Q, res, nsteps=k, graph=True)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)
    ms = timed(K)
    value = dof * 5 * K / (ms * 1e-3) / 1e9
    # stage-launch average without the once-per-call trace launch:
    # (T(2K) - T(K)) / (5 K)
    t2 = timed(2 * K)
    avg_s = (t2 - ms) / (5 * K) * 1e-3
    achieved = ALG_BYTES_PER_DOF_STAGE * dof / avg_s / 1e9
    degs = {}
    for sp in specs:
        degs[sp["p"]] = degs.get(sp["p"], 0) + 1
    # the other launch form (one persistent launch per stage, or one launch
    # per degree) on the same state and steps; its results are bitwise the same
    opts = b.options()
    other = dg.DG_BATCH_PERSISTENT if opts["batch_launch"] == dg.DG_BATCH_PER_DEGREE else dg.DG_BATCH_PER_DEGREE
    b.set_option(dg.DG_OPT_BATCH_LAUNCH, other)
    b.step(Q, res, nsteps=1, graph=True)
    torch.cuda.synchronize()
    ms_other = timed(K)
    b.set_option(dg.DG_OPT_BATCH_LAUNCH, opts["batch_launch"])
    form_name = {dg.DG_BATCH_PERSISTENT: "one persistent launch per RK stage (k_batch_stage)",
                 dg.DG_BATCH_PER_DEGREE: "one launch per degree and RK stage (k_batch_degree)"}
    return {
        "metric": "GDOF-RK-stages/sec", "value": value, "unit": "GDOF-RK-stages/sec", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 contractions, f64 state",
        "data": "synthetic",
        "config": {"workload": f"batch512: {desc}", "meshes": len(specs), "dof": dof,
                   "meshes_per_degree": degs, "tiles": b.tiles, "precision": args.precision,
                   "options": b.options()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("batch512", "batch", {"precision": args.precision,
                                                                       "tiles": {str(k): v for k, v in
                                                                                 sorted(b.tiles.items())},
                                                                       "options": b.options()}),
                     "kernel": ("k_batch_degree<N, EPB> (one launch per degree present; the five launches of "
                                "one RK stage timed together)"
                                if b.options()["batch_launch"] == dg.DG_BATCH_PER_DEGREE
                                else "k_batch_stage (persistent, all meshes)"), "avg_launch_us": avg_s * 1e6,
                     "alg_bytes_per_launch": ALG_BYTES_PER_DOF_STAGE * dof},
        "other_launch_form": {"form": form_name[other], "ms_per_step": ms_other / K,
                              "value": dof * 5 * K / (ms_other * 1e-3) / 1e9},
    }


def varp_cpu_baseline(deg, h, budget_s, m=8):
    """The variable-degree oracle advancing RK stages on the host for about
    ``budget_s`` seconds on an m^3-element periodic block of the same
    element size carrying the degrees of the m^3 block of the mesh (corners
    on a 4-element lattice) whose share of nodes per degree is closest to
    the whole mesh's (its cost per node is then about that of the whole
    mesh)."""
    import numpy as np
    import workloads as W
    from oracle import lserk
    from oracle.varp import VariableDegreeDG
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count()
    def node_share(d):
        c = np.bincount(d.ravel(), minlength=8) * (np.arange(8) + 1) ** 3
        return c / c.sum()
    want = node_share(deg)
    best = None
    for oz in range(0, deg.shape[0] - m + 1, 4):
        for oy in range(0, deg.shape[1] - m + 1, 4):
            for ox in range(0, deg.shape[2] - m + 1, 4):
                blk = deg[oz:oz + m, oy:oy + m, ox:ox + m]
                gap = float(np.abs(node_share(blk) - want).sum())
                if best is None or gap < best[0]:
                    best = (gap, blk)
    dm = np.ascontiguousarray(best[1])
    Lm = tuple(float(hd) * m for hd in h)
    ora = VariableDegreeDG((m, m, m), dm, L=Lm)
    Q = W.varp_state((m, m, m), dm, W.tgv_primitives, L=Lm)
    res = np.zeros_like(Q)
    dt = ora.dt_cfl(Q, 0.3)
    t0 = time.perf_counter()
    stages = 0
    while True:
        lserk.stage(stages % 5, Q, res, dt, ora.rhs)
        stages += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    dof = ora.num_dof()
    return {"value": dof * stages / el / 1e9, "unit": "GDOF-RK-stages/s", "cores": threads, "kind": "oracle",
            "sample": f"a {m}^3-element block of the same element size with the degrees of the mesh block closest "
                      f"to its node share per degree ({np.bincount(dm.ravel()).tolist()} elements per degree): "
                      f"{stages} RK stages "
                      f"({dof} nodes) in {el:.1f} s; BLAS threads {threads}, host cpu_count {os.cpu_count()}"}


def varp_roofline(v, Q, res, dt, K, nodes, faces, workload):
    """Per-launch HIP events on the library's stream over a second pass of
    the same K steps: every kernel's average launch and, for the stage
    kernels, the algorithmic rate (160 B per node and stage, 120 in the
    first stage).  The dominant kernel is the stage kernel of the degree
    with the most nodes, stages 2..5 (its launches over both element sizes
    where the mesh has refined cells).  nodes: {degree: nodes}; faces:
    {"mortar": count, "hanging": count}."""
    v.set_timing(1)
    v.step(Q, res, dt, nsteps=K)
    t = v.timing_read()
    v.set_timing(0)
    kernels = {}

    def label(p, mode):
        return f"k_varp p={p} {'stages 2..5' if mode == 1 else 'first stage'}"
    for key, (k_ms, k_n) in t.items():
        a_s = k_ms / k_n * 1e-3
        if key in ("mortar", "hanging"):
            kernels[f"k_varp_{key}"] = {"avg_launch_us": a_s * 1e6, "launches": k_n, "faces": faces.get(key)}
            continue
        p, mode = key
        per = ALG_BYTES_PER_DOF_STAGE if mode == 1 else ALG_BYTES_PER_DOF_FIRST_STAGE
        stages = 4 * K if mode == 1 else K
        total = per * nodes[p] * stages
        kernels[label(p, mode)] = {"avg_launch_us": a_s * 1e6, "launches": k_n,
                                   "alg_bytes_per_launch": total / k_n, "achieved": total / (k_ms * 1e-3) / 1e9}
    pdom = max(nodes, key=nodes.get)
    dom = kernels[label(pdom, 1)]
    return {"bound": "hbm", "achieved": dom["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dom["achieved"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(workload, "varp", {}),
            "kernel": f"k_varp<{pdom + 1}> (degree {pdom}: fused RHS + LSERK45 stage, stages 2..5)",
            "avg_launch_us": dom["avg_launch_us"], "launches": dom["launches"],
            "alg_bytes_per_launch": dom["alg_bytes_per_launch"], "kernels": kernels,
            "stage_bytes_per_node": ALG_BYTES_PER_DOF_STAGE}


def hp_cpu_baseline(ref, deg, h, budget_s, m=6):
    """The refined-mesh oracle advancing RK stages on the host for about
    ``budget_s`` seconds on an m^3-cell periodic block of the same cell size
    carrying the refinement and degrees of the m^3 block of the mesh
    (corners on a 2-cell lattice) whose share of nodes per (degree, size)
    is closest to the whole mesh's."""
    import numpy as np
    import workloads as W
    from oracle import lserk
    from oracle.hp import RefinedMeshDG
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count()
    n = ref.shape
    cfirst = np.concatenate([[0], np.cumsum(np.where(ref.reshape(-1) == 1, 8, 1))])

    def elements(cz, cy, cx):
        c = (cz * n[1] + cy) * n[2] + cx
        return deg[cfirst[c]:cfirst[c + 1]]

    def node_share(r, d):
        # nodes per (degree, level) over cells with refinement r and element degrees d
        c = np.zeros(16)
        lev = np.repeat(r.reshape(-1), np.where(r.reshape(-1) == 1, 8, 1))
        np.add.at(c, d * 2 + lev, (d + 1) ** 3)
        return c / c.sum()
    want = node_share(ref, deg)
    best = None
    for oz in range(0, n[0] - m + 1, 2):
        for oy in range(0, n[1] - m + 1, 2):
            for ox in range(0, n[2] - m + 1, 2):
                r = ref[oz:oz + m, oy:oy + m, ox:ox + m]
                d = np.concatenate([elements(oz + k, oy + j, ox + i) for k in range(m) for j in range(m)
                                    for i in range(m)])
                gap = float(np.abs(node_share(r, d) - want).sum())
                if best is None or gap < best[0]:
                    best = (gap, np.ascontiguousarray(r), d)
    _, rm, dm = best
    Lm = tuple(float(hd) * m for hd in h)
    ora = RefinedMeshDG((m, m, m), rm, dm, L=Lm)
    Q = W.hp_state((m, m, m), rm, dm, W.tgv_primitives, L=Lm)
    res = np.zeros_like(Q)
    dt = ora.dt_cfl(Q, 0.3)
    t0 = time.perf_counter()
    stages = 0
    while True:
        lserk.stage(stages % 5, Q, res, dt, ora.rhs)
        stages += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    dof = ora.num_dof()
    return {"value": dof * stages / el / 1e9, "unit": "GDOF-RK-stages/s", "cores": threads, "kind": "oracle",
            "sample": f"a {m}^3-cell block of the same cell size with the refinement and degrees of the mesh block "
                      f"closest to its node share per (degree, element size) ({int(rm.sum())} cells refined, "
                      f"{ora.E} elements, degrees {np.bincount(dm).tolist()}): {stages} RK stages ({dof} nodes) "
                      f"in {el:.1f} s; BLAS threads {threads}, host cpu_count {os.cpu_count()}"}


def run_hp(args):
    """The refined-mesh configuration: per stage the launches of the faces
    between degrees and of the hanging faces, then one fused stage launch
    per (degree, element size)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2006_15698_amd import dg

    n, _, cfg_steps, desc = WORKLOADS["tgv40_hp"]
    K = cfg_steps if args.steps is None else args.steps
    L = (2 * math.pi,) * 3
    ref, deg = W.tgv_refined_mesh((n, n, n))
    v = dg.VariableDegree((n, n, n), deg, L=L, refine=ref)
    Qh = W.hp_state((n, n, n), ref, deg, W.tgv_primitives, L=L)
    # dt = CFL / ((2 p_max + 1) max over nodes of sum_d (|u_d| + c) / h_d),
    # h the node's element size
    _, size, _ = W.hp_geometry((n, n, n), ref, L)
    hn = np.repeat(size, (deg + 1) ** 3, axis=0)
    rho = Qh[0]
    vel = Qh[1:4] / rho
    c = np.sqrt(W.GAMMA * (W.GAMMA - 1) * (Qh[4] - 0.5 * rho * (vel ** 2).sum(axis=0)) / rho)
    rate = float(np.max(sum((np.abs(vel[d]) + c) / hn[:, d] for d in range(3))))
    dt = 0.3 / ((2 * int(deg.max()) + 1) * rate)
    Q0 = torch.from_numpy(Qh.reshape(-1)).cuda()
    dof = v.num_dof()
    Q = Q0.clone()
    res = torch.zeros_like(Q)
    if args.warmup > 0:
        v.step(Q, res, dt, nsteps=args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    v.step(Q, res, dt, nsteps=K)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    value = dof * 5 * K / (ms * 1e-3) / 1e9
    counts = np.bincount(deg, minlength=8)
    nodes = {int(p): int(counts[p]) * (p + 1) ** 3 for p in range(8) if counts[p]}
    # faces: hanging sub-faces (4 per refined-unrefined cell pair), and
    # same-size faces between degrees (whole cells, or 4 fine faces between
    # two refined cells; siblings share their cell's degree)
    cdeg = deg[np.concatenate([[0], np.cumsum(np.where(ref.reshape(-1) == 1, 8, 1))])[:-1]].reshape(ref.shape)
    nhang = nmortar = 0
    for ax in range(3):
        rn, dn = np.roll(ref, -1, axis=ax), np.roll(cdeg, -1, axis=ax)
        nhang += 4 * int(np.sum(ref != rn))
        nmortar += int(np.sum((ref == 0) & (rn == 0) & (cdeg != dn))) + 4 * int(np.sum((ref == 1) & (rn == 1) &
                                                                                    (cdeg != dn)))
    out = {
        "metric": "GDOF-RK-stages/sec", "value": value, "unit": "GDOF-RK-stages/sec", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"tgv40_hp: {desc}", "cells": n ** 3, "refined_cells": int(ref.sum()),
                   "elements": int(deg.size), "dof": dof, "dt": dt,
                   "elements_per_degree": {int(p): int(counts[p]) for p in range(8) if counts[p]},
                   "mortar_faces": nmortar, "hanging_subfaces": nhang, "precision": "fp64"},
    }
    if not args.no_roofline:
        out["roofline"] = varp_roofline(v, Q, res, dt, K, nodes, {"mortar": nmortar, "hanging": nhang}, "tgv40_hp")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = hp_cpu_baseline(ref, deg, np.array(L) / n, args.cpu_seconds)
    return out


def run_varp(args):
    """The variable-degree configuration: per stage the mortar-face launch
    and one fused stage launch per degree."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2006_15698_amd import dg

    n, _, cfg_steps, desc = WORKLOADS["tgv48_varp"]
    K = cfg_steps if args.steps is None else args.steps
    L = (2 * math.pi,) * 3
    deg = W.tgv_degrees((n, n, n))
    v = dg.VariableDegree((n, n, n), deg, L=L)
    Qh = W.varp_state((n, n, n), deg, W.tgv_primitives, L=L)
    # dt = CFL / ((2 p_max + 1) max over nodes of sum_d (|u_d| + c) / h_d)
    h = np.array(L) / n
    rho = Qh[0]
    vel = Qh[1:4] / rho
    c = np.sqrt(W.GAMMA * (W.GAMMA - 1) * (Qh[4] - 0.5 * rho * (vel ** 2).sum(axis=0)) / rho)
    rate = float(np.max(sum((np.abs(vel[d]) + c) / h[d] for d in range(3))))
    dt = 0.3 / ((2 * int(deg.max()) + 1) * rate)
    Q0 = torch.from_numpy(Qh.reshape(-1)).cuda()
    dof = v.num_dof()
    Q = Q0.clone()
    res = torch.zeros_like(Q)
    if args.warmup > 0:
        v.step(Q, res, dt, nsteps=args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    v.step(Q, res, dt, nsteps=K)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    value = dof * 5 * K / (ms * 1e-3) / 1e9
    counts = np.bincount(deg.ravel(), minlength=8)
    nodes = {int(p): int(counts[p]) * (p + 1) ** 3 for p in range(8) if counts[p]}
    nmortar = sum(int(np.sum(deg != np.roll(deg, 1, axis=a))) for a in range(3))
    out = {
        "metric": "GDOF-RK-stages/sec", "value": value, "unit": "GDOF-RK-stages/sec", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"tgv48_varp: {desc}", "elements": n ** 3, "dof": dof, "dt": dt,
                   "elements_per_degree": {int(p): int(counts[p]) for p in range(8) if counts[p]},
                   "mortar_faces": nmortar, "precision": "fp64"},
    }
    if not args.no_roofline:
        out["roofline"] = varp_roofline(v, Q, res, dt, K, nodes, {"mortar": nmortar}, "tgv48_varp")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = varp_cpu_baseline(deg, h, args.cpu_seconds)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tgv48_p4", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-precision-clause", action="store_true",
                    help="skip the FP32-form rate and both forms' errors against the oracle")
    ap.add_argument("--exchange", default="neighbour", choices=["neighbour", "traces"],
                    help="how a stage obtains its neighbours' face traces (FP64 path)")
    ap.add_argument("--xcd-remap", type=int, default=None, choices=[0, 1],
                    help="1: each XCD takes a contiguous part of the visiting order (default: library's)")
    ap.add_argument("--order", default=None, choices=["linear", "pencil"],
                    help="element-block visiting order of the stage kernel (default: library's)")
    ap.add_argument("--pencil-x", type=int, default=None, help="pencil extent along x in elements (0: row)")
    ap.add_argument("--pencil-z", type=int, default=None, help="pencil extent along z in element planes")
    ap.add_argument("--graph", type=int, default=0, choices=[0, 1],
                    help="1: advance the timed steps by replaying captured HIP graphs (dg_rk_graph_steps); "
                         "measured no faster than direct launches at these sizes, so off by default")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="instead of the solver, time a plain device-to-device copy of MIB MiB "
                         "(calibrates HBM byte counters; reports the copy bandwidth)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}): it measures "
              "one GPU's share of the mesh; the face exchange between GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2006_15698_amd import dg

    if args.copy_probe:
        nbytes = args.copy_probe << 20
        x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes,
                          "ms_per_copy": ms, "GBps_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}))
        return

    if args.workload == "batch512":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.workload == "adjoint16_p3":
        print(json.dumps(run_adjoint(args)), flush=True)
        return
    if args.workload == "tgv48_varp":
        print(json.dumps(run_varp(args)), flush=True)
        return
    if args.workload == "tgv40_hp":
        print(json.dumps(run_hp(args)), flush=True)
        return

    n, p, cfg_steps, desc = WORKLOADS[args.workload]
    K = cfg_steps if args.steps is None else args.steps
    Wm = args.warmup
    L = (2 * math.pi,) * 3
    prec = dg.DG_FP64 if args.precision == "fp64" else dg.DG_FP32_MFMA
    viscous = VISCOUS.get(args.workload)
    mu, prandtl = viscous if viscous else (0.0, 0.72)
    split = args.workload in SPLIT_FORM
    s = dg.Solver((n, n, n), p, L=L, precision=prec, mu=mu, prandtl=prandtl,
                  volume_form=dg.DG_VOLUME_KEP if split else dg.DG_VOLUME_STANDARD)
    s.set_option(dg.DG_OPT_EXCHANGE, dg.DG_EXCHANGE_NEIGHBOUR if args.exchange == "neighbour"
                 else dg.DG_EXCHANGE_TRACES)
    for key, val in ((dg.DG_OPT_XCD_REMAP, args.xcd_remap),
                     (dg.DG_OPT_ORDER, None if args.order is None
                      else dg.DG_ORDER_PENCIL if args.order == "pencil" else dg.DG_ORDER_LINEAR),
                     (dg.DG_OPT_PENCIL_X, args.pencil_x), (dg.DG_OPT_PENCIL_Z, args.pencil_z)):
        if val is not None:
            s.set_option(key, val)
    dof = s.num_dof
    Q0 = torch.from_numpy(W.tgv(n, p)).cuda()
    dt = s.dt_cfl(Q0, 0.3)
    Q = Q0.clone()
    res = torch.zeros_like(Q)
    graph = bool(args.graph)
    if Wm > 0:
        s.step(Q, res, dt, nsteps=Wm, graph=graph)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    s.step(Q, res, dt, nsteps=K, graph=graph)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    value = dof * 5 * K / (ms * 1e-3) / 1e9

    out = {
        "metric": "GDOF-RK-stages/sec",
        "value": value,
        "unit": "GDOF-RK-stages/sec",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 contractions, f64 state",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "elements": n ** 3, "p": p,
                   "dof": dof, "precision": args.precision, "dt": dt,
                   "options": s.options(), "graph_replay": graph},
    }
    if viscous:
        out["config"].update({"mu": mu, "prandtl": prandtl})

    if viscous and not args.no_roofline:
        # Per stage the viscous flux (with the inviscid rate, when fused) and
        # the viscous rate with the RK update, timed together; unfused, the
        # inviscid rate's launch before them.  Average durations from the
        # library's HIP events on its stream.
        dg.dg_set_timing(s.ctx, True)
        s.step(Q, res, dt, nsteps=K)
        t = dg.dg_timing_read(s.ctx)
        dg.dg_set_timing(s.ctx, False)
        fused = t["rhs"][1] == 0
        vb = VISC_BYTES_FUSED if fused else VISC_BYTES
        labels = {"rhs": "inviscid rate (k_stage_nb, RHS mode)",
                  "visc": ("k_visc_flux (with the inviscid rate) + k_visc_apply" if fused
                           else "k_visc_flux + k_visc_apply")}
        parts = {}
        for kind in vb:
            k_ms, k_n = t[kind]
            a_s = k_ms / k_n * 1e-3
            parts[kind] = {"kernel": labels[kind], "avg_launch_us": a_s * 1e6, "launches": k_n,
                           "alg_bytes_per_launch": vb[kind] * dof,
                           "achieved": vb[kind] * dof / a_s / 1e9}
        v = parts["visc"]
        out["roofline"] = {"bound": "hbm", "achieved": v["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": v["achieved"] / HBM_PEAK_GBS,
                           "traffic": measured_traffic(args.workload, "visc", s.options()),
                           "kernel": (("k_visc_flux (viscous flux and inviscid rate) + k_visc_apply (viscous "
                                       "rate and LSERK45 update), one stage") if fused else
                                      "k_visc_flux + k_visc_apply (viscous terms and LSERK45 update, one stage)"),
                           "avg_launch_us": v["avg_launch_us"], "launches": v["launches"],
                           "alg_bytes_per_launch": v["alg_bytes_per_launch"],
                           "stage_bytes_per_node": sum(vb.values())}
        if not fused:
            out["roofline"]["inviscid_rate"] = parts["rhs"]
    elif not args.no_roofline:
        # Dominant kernel: the fused stage kernel of stages 2..5 (four of the
        # five launches of a step; the first stage's kernel, which does not
        # read the residual, is reported beside it).  Average launch duration
        # from HIP events that the library records around every launch on the
        # stream it launches on (a second pass over the same K steps).
        dg.dg_set_timing(s.ctx, True)
        s.step(Q, res, dt, nsteps=K)
        t = dg.dg_timing_read(s.ctx)
        dg.dg_set_timing(s.ctx, False)
        st_ms, st_n = t["stage"]
        avg_s = st_ms / st_n * 1e-3
        alg_bytes = ALG_BYTES_PER_DOF_STAGE * dof
        achieved = alg_bytes / avg_s / 1e9
        f_ms, f_n = t["stage_first"]
        f_s = f_ms / f_n * 1e-3
        traffic = measured_traffic(args.workload, args.precision, s.options())
        kname = {("neighbour", "fp64"): "k_stage_nb", ("neighbour", "fp32"): "k_stage_nb32",
                 ("traces", "fp64"): "k_stage", ("traces", "fp32"): "k_stage32"}[(args.exchange, args.precision)]
        if split:
            kname = "k_split (split-form volume term, Kennedy-Gruber two-point flux)"
            traffic = measured_traffic(args.workload, "split", s.options())
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel": kname + " (fused RHS + LSERK45 stage, stages 2..5)",
                           "avg_launch_us": avg_s * 1e6, "launches": st_n,
                           "alg_bytes_per_launch": alg_bytes,
                           "first_stage": {"avg_launch_us": f_s * 1e6, "launches": f_n,
                                           "alg_bytes_per_launch": ALG_BYTES_PER_DOF_FIRST_STAGE * dof,
                                           "achieved": ALG_BYTES_PER_DOF_FIRST_STAGE * dof / f_s / 1e9}}
        fl = flops_per_dof_stage(p + 1) * dof
        out["fp64_rate"] = {"achieved_tflops": fl / avg_s / 1e12, "peak_tflops": FP64_PEAK_TFS,
                            "frac": fl / avg_s / 1e12 / FP64_PEAK_TFS,
                            "flops_per_dof_stage": flops_per_dof_stage(p + 1)}

    if not args.no_precision_clause and not viscous and not split:
        out["fp32_mfma_vs_fp64"] = precision_clause(args, n, p, L, Q0, dt, K, Wm, graph, value)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, p, L, args.cpu_seconds, viscous, split)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
