#!/usr/bin/env python3
"""Benchmark of the fused reaction-diffusion program on one MI355X.

    python bench.py [--steps K] [--warmup W] [--seed S] [--forms main|all]
                    [--no-cpu-baseline] [--calibrate-copy]

Workload (the headline configuration): a 512^3 float64 grid, periodic
boundary, u0 ~ U[-1,1], f = 8 seeded low-frequency sinusoids, alpha=1,
beta=0.1, gamma=0.5, h=1, dt=0.1.  One timed step is one dcp_run of T=100
fused time steps with the FP64 energy and residual norms of every step
(inputs resident in HBM; each step continues from the state the previous
one left).  W untimed steps, then exactly K timed steps between two device
synchronisations.  `value` is lattice-point updates per second (GLUP/s =
N*T*K / seconds / 1e9).

In the same run (--forms all, the default) every other form of the metric
is timed on the same inputs, each in its own event-timed region: the
unfused single-operator chain, the float32 forms, the 1024x1024x512 grid
(rows longer than a whole-row tile), one GPU's 512x512x64 share of an
8-way z-slab split, the adjoint kernel and
the end-to-end gradient (forward with checkpoints + checkpointed adjoint);
one step (and one adjoint step) run by kernels the fusing compiler
generates (fused, and one kernel per statement) beside the hand-written
one-step kernels; then the two
Jacobi listings (jacobi_1d, jacobi_2d) at the paper's problem sizes and
weak-scaled to 1296 processes, with and without temporal blocking.

Prints ONE JSON line.  With --gpus N, N > 1, it exits with a message: this
benchmark runs on one GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# MI355X FP64 vector: 78.6 TFLOP/s counting an FMA as two flops; adds and
# multiplies issue at the same instruction rate and count one flop each.
FP64_NONFMA_PEAK_TFLOPS = 78.6 / 2
KERNEL_SRCS = {1: os.path.join(ROOT, "paper_2107_00555_amd", "csrc", "dcp_kernels.hip"),
               2: os.path.join(ROOT, "paper_2107_00555_amd", "csrc", "dcp_tblock.hip"),
               3: os.path.join(ROOT, "paper_2107_00555_amd", "csrc", "dcp_tbk.hip")}
COUNTERS = {1: os.path.join(ROOT, "profiles", "stencil_fused_f64_512_counters.md"),
            2: os.path.join(ROOT, "profiles", "tb2_fused_f64_512_counters.md"),
            3: os.path.join(ROOT, "profiles", "tbr3_fused_f64_512_counters.md")}
KERNEL_NAMES = {1: "stencil_kernel<double,2,1,4,4,PERIODIC,FWD,norms> (one step per launch)",
                2: "tb2_kernel<double,2,4,1024,2,PERIODIC,FWD,norms> (two steps per launch)",
                3: "tbr_kernel<double,2,3,768,2,PERIODIC,segments,norms> (three steps per launch, register rings)"}


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--forms", choices=["main", "all", "jacobi", "generated", "ceiling", "adjoint"], default="all",
                   help="main: the headline only; all: every form; jacobi / generated / ceiling / adjoint: "
                        "the Jacobi forms, the fusing compiler's forms, the streaming ceiling or the adjoint "
                        "kernel forms only (no headline line; for profiling)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-errors", action="store_true",
                   help="skip the per-form error check against the oracle (run after the CPU baseline)")
    p.add_argument("--jacobi-workloads", default="all",
                   help="comma-separated Jacobi workloads to time (names in inputs.JACOBI_WORKLOADS)")
    p.add_argument("--jacobi-no-compare", action="store_true",
                   help="skip the one-half-step-per-pass comparison runs of the Jacobi forms")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a plain 1 GiB device copy (counter calibration)")
    p.add_argument("--tblock", type=int, default=3,
                   help="time steps fused per pass over memory in the headline run (1, 2 or 3)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bootstrap_ci(xs, reps=2000, seed=0):
    """Median and 95% nonparametric bootstrap interval of the median."""
    import numpy as np
    xs = np.asarray(xs, dtype=np.float64)
    if xs.size == 0:
        return None, None, None
    r = np.random.default_rng(seed)
    meds = np.median(r.choice(xs, size=(reps, xs.size), replace=True), axis=1)
    return float(np.median(xs)), float(np.percentile(meds, 2.5)), float(np.percentile(meds, 97.5))


def timed(fn, k, w, stream):
    """W untimed calls, then K calls with an event between each; returns
    (total_ms by events, per-call ms list, wall seconds).  Python's garbage
    collector is switched off for the timed calls only: a collection pass
    there would show up as idle GPU time."""
    import gc
    import torch
    for _ in range(w):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
    was_enabled = gc.isenabled()
    gc.disable()
    try:
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(k):
            fn()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        if was_enabled:
            gc.enable()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(k)]
    return ev[0].elapsed_time(ev[k]), per, wall


def counter_traffic(tblock):
    """HBM bytes per launch of the headline kernel from the committed
    rocprofv3 counter summary, or None if the kernel source changed since."""
    path = COUNTERS.get(tblock)
    if path is None or not os.path.exists(path):
        return None
    src = hashlib.sha256(open(KERNEL_SRCS[tblock], "rb").read()).hexdigest()
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != src:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str | None:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


ORACLE_STEPS = 15


def cpu_baseline(u0, f, coeffs, bc):
    """The oracle as it stands, serial, on 15 of the 100 steps of the same
    512^3 workload (full grid; about 20 s on one host core), with the calling
    thread pinned to one core for the run (the mask is restored afterwards).
    Returns the baseline entry and the oracle's (u_15, E_t, R_t)."""
    import oracle
    T = ORACLE_STEPS
    mask = os.sched_getaffinity(0)
    core = min(mask)
    os.sched_setaffinity(0, {core})
    try:
        t0 = time.perf_counter()
        uT, e, r = oracle.run(u0, f, coeffs, T, bc, norms=True)
        dt = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, mask)
    n = u0.size
    base = {"value": n * T / dt / 1e9, "unit": "GLUP/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle_run (serial FP64, every temporary materialised) for {T} of the 100 "
                      f"steps on the full 512^3 periodic grid, {dt:.1f} s, pinned to core {core}",
            "cpu": {"model": cpu_model(), "nproc": os.cpu_count(), "usable_cores": len(mask)}}
    return base, (uT, e, r)


def form_errors(dev, u0, f64, u0_h, f_h, coeffs, bc, ref64) -> dict:
    """Error of each GPU form against the oracle after the same 15 steps from
    u0 on the headline workload: the normwise field error max|a-b|/max|b|
    and the largest relative error of E_t and R_t over the steps.  float64
    forms against the oracle run of the CPU baseline; float32 forms against
    the oracle run on the float32-rounded inputs (run here, untimed)."""
    import numpy as np
    import oracle
    import torch

    from paper_2107_00555_amd import api
    T = ORACLE_STEPS

    def measure(u, out, ref):
        uT, e_or, r_or = ref
        o = torch.from_numpy(uT).to(dev)
        field = float((u.double() - o).abs().max() / o.abs().max())
        e = out["energy"].cpu().numpy()
        r = out["resid"].cpu().numpy()
        del o
        return {"field_normwise": field,
                "energy_max_rel": float(np.max(np.abs(e - e_or) / e_or)),
                "resid_max_rel": float(np.max(np.abs(r - r_or) / r_or))}

    errs = {"steps": T, "reference": "oracle (FP64, serial) after the same steps from u0"}
    for name, impl, tb in (("fused_f64_tblock3", "fused", 3), ("fused_f64_tblock2", "fused", 2),
                           ("fused_f64_tblock1", "fused", 1), ("unfused_f64", "unfused", 1)):
        u = u0.clone()
        out = api.run(u, f64, coeffs, T, bc, impl=impl, tblock=tb, norms=True)
        torch.cuda.synchronize()
        errs[name] = measure(u, out, ref64)
        if impl == "unfused":
            errs[name]["bitwise_equal"] = bool(torch.equal(u, torch.from_numpy(ref64[0]).to(dev)))
        del u
    log("oracle on the float32-rounded inputs (for the float32 errors) ...")
    u32h = u0_h.astype(np.float32).astype(np.float64)
    f32h = f_h.astype(np.float32).astype(np.float64)
    ref32 = oracle.run(u32h, f32h, coeffs, T, bc, norms=True)
    f32 = f64.to(torch.float32)
    for tb in (3, 2, 1):
        u = u0.to(torch.float32)
        out = api.run(u, f32, coeffs, T, bc, impl="fused", tblock=tb, norms=True)
        torch.cuda.synchronize()
        errs[f"fused_f32_tblock{tb}"] = measure(u, out, ref32)
        del u
    errs["bounds"] = {"f64": 1e-12, "f32": 1e-5}
    return errs


def stream_ceiling(dev, stream, reps: int = 20) -> dict:
    """HBM bandwidth a plain streaming kernel reaches on this GPU (the
    library's dcp_stream_probe over 1 GiB buffers): copy, two reads + one
    write (the stencil's traffic shape), read and fill, each with ordinary
    and with streaming (non-temporal) loads and stores; GB/s of bytes moved."""
    import ctypes
    import torch

    from paper_2107_00555_amd import _lib
    nbytes = 1 << 30
    a = torch.rand(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.rand(nbytes // 8, dtype=torch.float64, device=dev)
    o = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    L = _lib.lib()
    sp = ctypes.c_void_p(stream.cuda_stream)
    out = {}
    for kind, name, moved in ((0, "copy", 2), (1, "two_reads_one_write", 3), (2, "read", 1), (3, "fill", 1)):
        for nt in (0, 1):
            def call():
                _lib.check("dcp_stream_probe", L.dcp_stream_probe(kind, nt, ctypes.c_void_p(a.data_ptr()),
                                                                  ctypes.c_void_p(b.data_ptr()),
                                                                  ctypes.c_void_p(o.data_ptr()), nbytes, sp))
            ms, _, _ = timed(call, reps, 3, stream)
            gbs = moved * nbytes / (ms / reps * 1e-3) / 1e9
            out[f"{name}{'_nt' if nt else ''}"] = round(gbs, 1)
    del a, b, o
    torch.cuda.empty_cache()
    out["unit"] = "GB/s"
    return out


def adjoint_forms(dev, stream, u0, f64, coeffs, bc, kk) -> dict:
    """The adjoint kernel on the headline grid, both dtypes: 10 adjoint steps
    from checkpoints of every step (no recomputation), alone and with the
    running sum for dL/df and dL/dgamma."""
    import torch

    from paper_2107_00555_amd import _lib, api
    nz, ny, nx = u0.shape
    N = u0.numel()
    forms = {}
    for name, dtype in (("f64", torch.float64), ("f32", torch.float32)):
        S = 8 if dtype == torch.float64 else 4
        Ta = 10
        fld = u0.to(dtype)
        ff = f64.to(dtype)
        ua = fld.clone()
        ck = api.run(ua, ff, coeffs, Ta, bc, norms=False, ckpt_every=1)["ckpt"]
        lam = (ua - fld).contiguous()
        wsa = api.workspace(_lib.workspace_bytes(_lib.OP_ADJOINT, 0 if S == 8 else 1, nx, ny, nz,
                                                 T=Ta, ckpt_every=1, tblock=3), dev)
        g = torch.empty_like(lam)
        log(f"timing adjoint kernel {name}")
        ms_a, _, _ = timed(lambda: api.adjoint_run(ck, 1, ff, lam, coeffs, Ta, bc, ws=wsa, grad_u0=g),
                           kk, 1, stream)
        ms_a /= kk
        # two adjoint steps per pass (the default): a pass reads lambda_{t+1},
        # u_t and u_{t-1} and writes lambda_{t-1}, 2*S bytes per point update;
        # "effective" prices every update at the one-step 3*S
        glups = N * Ta / (ms_a / 1e3) / 1e9
        forms[f"adjoint_{name}"] = {"glups": round(glups, 3), "ms_per_step": round(ms_a / Ta, 4),
                                    "effective_hbm_frac": round(glups * 3 * S / HBM_PEAK_GBS, 4),
                                    "hbm_frac_per_launch": round(glups * 2 * S / HBM_PEAK_GBS, 4)}
        # the same steps also accumulating the sum of the adjoint inputs
        # (dL/df, dL/dgamma): one more read and write of a field per pass
        log(f"timing adjoint kernel {name} with dL/df and dL/dgamma")
        ms_al, _, _ = timed(lambda: api.adjoint_run(ck, 1, ff, lam, coeffs, Ta, bc, ws=wsa, grad_u0=g,
                                                    want_f=True, want_gamma=True), kk, 1, stream)
        ms_al /= kk
        forms[f"adjoint_{name}_with_f_gamma"] = {"glups": round(N * Ta / (ms_al / 1e3) / 1e9, 3),
                                                 "ms_per_step": round(ms_al / Ta, 4)}
        del ck, wsa, g, lam, ua, fld, ff
        torch.cuda.empty_cache()
    return forms


def jacobi_forms(args, dev, stream) -> dict:
    """The two Jacobi listings at the paper's sizes and weak-scaled to 1296
    processes: event-timed runs of the library's default schedule, the pass
    schedule, per-pass HBM traffic and useful FP64 rate, and (small sizes)
    the speedup over one half-step per pass."""
    import torch

    from paper_2107_00555_amd import _lib, api, inputs
    jac = {}
    pick = None if args.jacobi_workloads == "all" else set(args.jacobi_workloads.split(","))
    if pick is not None and not pick <= set(inputs.JACOBI_WORKLOADS):
        raise SystemExit(f"unknown Jacobi workload in {sorted(pick)}")
    if args.calibrate_copy:
        # the library's own copy kernel, 1 GiB read + 1 GiB write (counter
        # calibration): a one-step dcp_run with a checkpoint every step
        # copies u into slot 0 first
        uc = torch.rand(512, 512, 512, dtype=torch.float64, device=dev)
        api.run(uc, torch.zeros_like(uc), dict(inputs.BASE_COEFFS), 1, inputs.PERIODIC, norms=False,
                ckpt_every=1)
        torch.cuda.synchronize()
        del uc
    for name, w in inputs.JACOBI_WORKLOADS.items():
        if pick is not None and name not in pick:
            continue
        dims, n, Tj = w["dims"], w["n"], w["tsteps"]
        n1 = n if dims == 2 else 1
        a, b = inputs.jacobi_fields_device(dims, n, seed=args.seed, device=dev)
        wsj = api.workspace(_lib.jacobi_workspace_bytes(dims, n, n1, Tj, 0), dev)
        run_j = api.jacobi_1d if dims == 1 else api.jacobi_2d
        N = a.numel()
        lups = (n - 2) ** dims * 2 * (Tj - 1)   # interior points x half-steps
        flops = 3 if dims == 1 else 5           # adds and one multiply per update
        big = N > (1 << 26)
        kj = max(1, min(args.steps, 3 if big else 10))
        log(f"timing {name} (n={n}, T={Tj})")
        # each call continues from the arrays the previous one left
        ms_j, per_j, _ = timed(lambda: run_j(a, b, Tj, 0, ws=wsj), kj, max(0, min(args.warmup, 1)), stream)
        ms_j /= kj
        passes, halo = _lib.jacobi_plan(dims, n, n1, Tj, 0)
        pass_ms = ms_j / passes
        gbs = 16 * N / (pass_ms * 1e-3) / 1e9
        tfl = lups * flops / (ms_j * 1e-3) / 1e12
        ent = {"dims": dims, "n": n, "tsteps": Tj, "passes": passes, "halfsteps_per_pass": halo,
               "ms": round(ms_j, 4), "ms_median_ci95": [round(x, 4) for x in bootstrap_ci(per_j)],
               "glups": round(lups / (ms_j * 1e-3) / 1e9, 2),
               # a pass reads A and writes A (16 B per element); the last also writes B
               "hbm_per_pass": {"bytes": 16 * N, "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)},
               "alu_useful": {"tflops": round(tfl, 3), "peak": FP64_NONFMA_PEAK_TFLOPS,
                              "frac": round(tfl / FP64_NONFMA_PEAK_TFLOPS, 4)}}
        if not big and not args.jacobi_no_compare:
            ms_1, _, _ = timed(lambda: run_j(a, b, Tj, 1, ws=wsj), 3, 1, stream)
            ms_1 /= 3
            ent["ms_one_halfstep_per_pass"] = round(ms_1, 3)
            ent["speedup_over_one_halfstep_per_pass"] = round(ms_1 / ms_j, 2)
        jac[name] = ent
        del a, b, wsj
        torch.cuda.empty_cache()
    return jac


def step_program(dtype: str, h: float):
    """The reaction-diffusion step as a single-operator array program for the
    fusing compiler (each operator one statement, Python's evaluation order)."""
    from paper_2107_00555_amd import fuse
    P = fuse.Program(dtype)
    u, f = P.input("u", "f")
    alpha, beta, gamma, dt = P.param("alpha", "beta", "gamma", "dt")
    lap = fuse.lap7(u, h)
    P.output("unew", u + dt * ((alpha * lap - beta * ((u * u) * u)) + gamma * f))
    return P


def adjoint_step_program(dtype: str, h: float):
    """The adjoint step lambda + dt*(alpha*Lap7(lambda) - 3*beta*u^2*lambda)
    as a single-operator program (the Laplacian is symmetric)."""
    from paper_2107_00555_amd import fuse
    P = fuse.Program(dtype)
    lam, u = P.input("lam", "u")
    alpha, beta, dt = P.param("alpha", "beta", "dt")
    P.output("lam_prev", lam + dt * (alpha * fuse.lap7(lam, h) - (3.0 * beta) * ((u * u) * lam)))
    return P


def program_bytes_unfused(text: str, S: int) -> int:
    """Per-point algorithmic bytes of the unfused program: every field
    statement reads its field operands and writes its result."""
    fields = set()
    total = 0
    for ln in text.splitlines():
        t = ln.split()
        if not t:
            continue
        if t[0] == "input":
            fields.update(t[1:])
        elif len(t) > 2 and t[1] == "=":
            ops = t[3:4] if t[2] == "shift" else t[3:]
            nf = sum(1 for a in ops if a in fields)
            if nf:
                fields.add(t[0])
                total += (nf + 1) * S
    return total


def generated_forms(args, dev, stream, u0, f64, coeffs, bc) -> dict:
    """One reaction-diffusion step at 512^3 run by kernels the fusing compiler
    generates (one fused kernel, or one kernel per statement) against the
    library's hand-written one-step kernels, FP64 and FP32."""
    import torch

    from paper_2107_00555_amd import api
    gen = {}
    N = u0.numel()
    params = {k: coeffs[k] for k in ("alpha", "beta", "gamma", "dt")}
    k = max(3, min(args.steps, 10))
    for dname, tdt, S in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        u = u0.to(tdt)
        f = f64.to(tdt)
        out = torch.empty_like(u)
        P = step_program(dname, coeffs["h"])
        ent = {}
        for label, fuse in (("generated_fused", True), ("generated_unfused", False)):
            prog = P.compile(fuse=fuse)
            wsb = prog.workspace_bytes(tuple(u.shape))
            ws = api.workspace(wsb, dev)
            log(f"timing {label} {dname} ({prog.n_kernels} kernels)")
            ms, per, _ = timed(lambda: prog.run([u, f], params, bc=bc, outputs=[out], ws=ws), k, 2, stream)
            ms /= k
            bpp = 3 * S if fuse else program_bytes_unfused(P.text(), S)
            ent[label] = {"kernels": prog.n_kernels, "ms": round(ms, 4),
                          "glups": round(N / (ms * 1e-3) / 1e9, 3),
                          "bytes_per_point": bpp,
                          "hbm_frac": round(bpp * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del prog, ws
        for label, impl in (("handwritten_fused", "fused"), ("handwritten_unfused", "unfused")):
            log(f"timing {label} {dname}")
            ms, _, _ = timed(lambda: api.step(u, f, coeffs, bc, impl=impl, out=out), k, 2, stream)
            ms /= k
            ent[label] = {"ms": round(ms, 4), "glups": round(N / (ms * 1e-3) / 1e9, 3)}
        ent["generated_fused_over_unfused"] = round(ent["generated_unfused"]["ms"] / ent["generated_fused"]["ms"], 2)
        ent["generated_fused_vs_handwritten_fused"] = round(ent["handwritten_fused"]["ms"] /
                                                             ent["generated_fused"]["ms"], 3)
        gen[f"step_{dname}"] = ent
        # the adjoint step, the method's second expression (no hand-written
        # counterpart: the library's adjoint kernel also forms the parameter sums)
        A = adjoint_step_program(dname, coeffs["h"])
        aprm = {k: coeffs[k] for k in ("alpha", "beta", "dt")}
        ent_a = {}
        for label, fuse in (("generated_fused", True), ("generated_unfused", False)):
            prog = A.compile(fuse=fuse)
            ws = api.workspace(prog.workspace_bytes(tuple(u.shape)), dev)
            log(f"timing adjoint step {label} {dname} ({prog.n_kernels} kernels)")
            ms, _, _ = timed(lambda: prog.run([f, u], aprm, bc=bc, outputs=[out], ws=ws), k, 2, stream)
            ms /= k
            bpp = 3 * S if fuse else program_bytes_unfused(A.text(), S)
            ent_a[label] = {"kernels": prog.n_kernels, "ms": round(ms, 4), "glups": round(N / (ms * 1e-3) / 1e9, 3),
                            "bytes_per_point": bpp,
                            "hbm_frac": round(bpp * N / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del prog, ws
        ent_a["generated_fused_over_unfused"] = round(ent_a["generated_unfused"]["ms"] /
                                                      ent_a["generated_fused"]["ms"], 2)
        gen[f"adjoint_step_{dname}"] = ent_a
        del u, f, out
        torch.cuda.empty_cache()
    return gen


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only (the single-GPU kernels are the measured path); "
              "multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2107_00555_amd import _lib, api, inputs

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.forms == "jacobi":
        print(json.dumps({"forms": {"jacobi": jacobi_forms(args, dev, stream)}, "data": "synthetic"}), flush=True)
        return
    if args.forms == "ceiling":
        print(json.dumps({"streaming_ceiling": stream_ceiling(dev, stream)}), flush=True)
        return
    nx = ny = nz = 512
    N = nx * ny * nz
    T = 100
    bc = inputs.PERIODIC
    coeffs = dict(inputs.BASE_COEFFS)

    log("generating inputs 512^3 ...")
    t0 = time.perf_counter()
    u0_h, f_h = inputs.make_fields("fwd_512_f64", seed=args.seed)
    log(f"  inputs ready in {time.perf_counter() - t0:.1f} s")
    u0 = torch.from_numpy(u0_h).to(dev)
    f64 = torch.from_numpy(f_h).to(dev)
    u = u0.clone()
    if args.forms == "generated":
        print(json.dumps({"forms": {"generated": generated_forms(args, dev, stream, u0, f64, coeffs, bc)},
                          "data": "synthetic"}), flush=True)
        return
    if args.calibrate_copy:
        # the library's own copy kernel, 1 GiB read + 1 GiB write: a dcp_run of
        # one step with a checkpoint every step copies u into slot 0 first
        uc = u0.clone()
        api.run(uc, f64, coeffs, 1, bc, norms=False, ckpt_every=1)
        torch.cuda.synchronize()
        del uc
    if args.forms == "adjoint":
        print(json.dumps({"forms": adjoint_forms(dev, stream, u0, f64, coeffs, bc, max(1, min(args.steps, 3))),
                          "data": "synthetic"}), flush=True)
        return

    # ---------------------------------------------------------- headline
    ws = api.workspace(_lib.workspace_bytes(_lib.OP_RUN, _lib.F64, nx, ny, nz, T=T, norms=True,
                                            tblock=3), dev)
    res = {}

    def fused_step():
        res["out"] = api.run(u, f64, coeffs, T, bc, impl="fused", tblock=args.tblock, norms=True, ws=ws)

    if args.tblock not in (1, 2, 3):
        raise SystemExit("--tblock must be 1, 2 or 3")
    plan = _lib.run_plan(_lib.F64, nx, ny, nz, T, args.tblock)
    log(f"timing fused f64: T={T}, tblock={args.tblock}, K={args.steps}, W={args.warmup}, passes {plan['passes']}")
    total_ms, per, wall = timed(fused_step, args.steps, args.warmup, stream)
    ms_step = total_ms / args.steps
    value = N * T * args.steps / (total_ms / 1e3) / 1e9
    # launches of the dominant kernel per benchmark step (passes of tblock
    # steps); the remainder passes of fewer steps (T mod tblock) are taken
    # out, so the average is that kernel's alone.  A remainder pass of L
    # steps is timed inside one run of 10 such passes (T = 10 L, tblock L,
    # the same kernel as in the benchmark's run), so that the host's time
    # between calls stays out of it
    B = plan["steps_per_pass"]
    launches = plan["passes"][B - 1]
    rest = [(n_, L_ + 1) for L_, n_ in enumerate(plan["passes"]) if L_ + 1 != B and n_]
    rest_ms = 0.0
    for n_, L_ in rest:
        ur = u0.clone()
        ms_r, _, _ = timed(lambda: api.run(ur, f64, coeffs, 10 * L_, bc, impl="fused", tblock=L_,
                                           norms=True, ws=ws), args.steps, 1, stream)
        rest_ms += n_ * ms_r / args.steps / 10
        del ur
    launch_ms = (ms_step - rest_ms) / launches     # includes the tiny finalize of the norms
    bytes_per_launch = 3 * 8 * N                    # read u, read f, write the result (algorithmic)
    achieved = bytes_per_launch / (launch_ms / 1e3) / 1e9
    med, lo, hi = bootstrap_ci(per)
    e = res["out"]["energy"]
    if not torch.isfinite(e).all():
        raise RuntimeError("non-finite norms in the timed run")
    traffic = counter_traffic(args.tblock)

    out = {
        "metric": "GLUP/s and % HBM roofline, fused vs unfused, fwd+adjoint, FP64/FP32 at 512^3",
        "value": round(value, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded: u0 ~ U[-1,1], f = 8 low-frequency sinusoids)",
        "config": {"workload": "fwd_512_f64: 512^3 float64, periodic, fused forward, T=100 steps "
                               "per step of the benchmark, FP64 energy+residual norms every step, "
                               f"up to {args.tblock} time step(s) per pass over memory",
                   "grid": [nx, ny, nz], "T": T, "bc": "periodic", "impl": "fused",
                   "tblock": args.tblock, "passes": plan["passes"], "coeffs": coeffs,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": KERNEL_NAMES[B],
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": round(launch_ms, 5),
                     "launches_per_step": launches,
                     "other_passes_ms_per_step": round(rest_ms, 4),
                     # lattice updates x the one-step algorithmic 24 B, over the peak:
                     # above 1 once a launch fuses more than one time step
                     "effective_frac": round(value * 24 / HBM_PEAK_GBS, 4)},
        "stats": {"median_ms": med, "ci95_ms": [lo, hi], "wall_s": round(wall, 4)},
    }

    # ------------------------------------------------------- other forms
    if args.forms == "all":
        log("streaming ceiling of this GPU (dcp_stream_probe)")
        ceil = stream_ceiling(dev, stream)
        out["roofline"]["streaming_ceiling_gbs"] = ceil
        out["roofline"]["frac_of_streaming_ceiling"] = round(achieved / ceil["two_reads_one_write_nt"], 4)
        forms = {}
        out["forms"] = forms
        kk = max(1, min(args.steps, 3))

        def glups(ms, steps=T, n=N):
            return n * steps / (ms / 1e3) / 1e9

        def frac(ms, bpl, steps=T, n=N):
            return (bpl * n * steps / (ms / 1e3) / 1e9) / HBM_PEAK_GBS

        def fused_entry(ms, S, tb, shape=(nx, ny, nz), steps=T):
            # effective: every update priced at the one-step 3*S bytes;
            # per pass: the algorithmic 3*S bytes of each pass over memory
            code = _lib.F64 if S == 8 else _lib.F32
            pl = _lib.run_plan(code, *shape, steps, tb)
            n = shape[0] * shape[1] * shape[2]
            return {"glups": round(glups(ms, steps, n), 3), "ms": round(ms, 3), "passes": pl["passes"],
                    "segmented": pl["segmented"], "effective_hbm_frac": round(frac(ms, 3 * S, steps, n), 4),
                    "hbm_frac_per_pass": round(frac(ms, 3 * S * sum(pl["passes"]) / steps, steps, n), 4)}

        ms_f = {args.tblock: ms_step}
        for tb in (1, 2, 3):
            if tb == args.tblock:
                continue
            uo = u0.clone()
            log(f"timing fused f64 tblock={tb}")
            ms_o, _, _ = timed(lambda: api.run(uo, f64, coeffs, T, bc, impl="fused", tblock=tb, norms=True,
                                               ws=ws), args.steps, 1, stream)
            ms_f[tb] = ms_o / args.steps
            del uo
        for tb in (1, 2, 3):
            forms[f"fused_f64_tblock{tb}"] = fused_entry(ms_f[tb], 8, tb)

        # unfused chain, float64
        wsu = api.workspace(_lib.workspace_bytes(_lib.OP_RUN, _lib.F64, nx, ny, nz, T=T, norms=True,
                                                 impl=_lib.UNFUSED), dev)
        uu = u0.clone()
        log("timing unfused f64")
        ms_u, per_u, _ = timed(lambda: api.run(uu, f64, coeffs, T, bc, impl="unfused", norms=True, ws=wsu),
                               kk, 1, stream)
        ms_u /= kk
        forms["unfused_f64"] = {"glups": round(glups(ms_u), 3), "ms": round(ms_u, 3),
                                "bytes_per_lup": 21 * 8 + 16,
                                "hbm_frac": round(frac(ms_u, 21 * 8 + 16), 4)}
        forms["fused_speedup_over_unfused_f64"] = {f"tblock{tb}": round(ms_u / ms_f[tb], 3) for tb in (1, 2, 3)}
        del wsu, uu

        # float32 forms
        u32 = u0.to(torch.float32)
        f32 = f64.to(torch.float32)
        ws32 = api.workspace(max(_lib.workspace_bytes(_lib.OP_RUN, _lib.F32, nx, ny, nz, T=T, norms=True,
                                                      impl=_lib.UNFUSED),
                                 _lib.workspace_bytes(_lib.OP_RUN, _lib.F32, nx, ny, nz, T=T, norms=True,
                                                      tblock=3)), dev)
        ms32 = {}
        for tb in (1, 2, 3):
            log(f"timing fused f32 tblock={tb}")
            ms_f32, _, _ = timed(lambda: api.run(u32, f32, coeffs, T, bc, impl="fused", tblock=tb, norms=True,
                                                 ws=ws32), args.steps, 1, stream)
            ms32[tb] = ms_f32 / args.steps
            forms[f"fused_f32_tblock{tb}"] = fused_entry(ms32[tb], 4, tb)
        u32b = u0.to(torch.float32)
        log("timing unfused f32")
        ms_u32, _, _ = timed(lambda: api.run(u32b, f32, coeffs, T, bc, impl="unfused", norms=True, ws=ws32),
                             kk, 1, stream)
        ms_u32 /= kk
        forms["unfused_f32"] = {"glups": round(glups(ms_u32), 3), "ms": round(ms_u32, 3),
                                "hbm_frac": round(frac(ms_u32, 21 * 4 + 8), 4)}
        forms["fused_speedup_over_unfused_f32"] = {f"tblock{tb}": round(ms_u32 / ms32[tb], 3) for tb in (1, 2, 3)}
        del ws32, u32b

        # rows longer than a whole-row tile holds in LDS: 1024 x 1024 x 512
        # (multi-step passes over x-segments), both dtypes, 24 steps
        wshape = (1024, 1024, 512)
        Tw = 24
        for dname, tdt, S, code in (("f64", torch.float64, 8, _lib.F64), ("f32", torch.float32, 4, _lib.F32)):
            gw = torch.Generator(device=dev)
            gw.manual_seed(args.seed + 11)
            uw0 = torch.empty((wshape[2], wshape[1], wshape[0]), dtype=tdt, device=dev).uniform_(-1, 1, generator=gw)
            fw = torch.empty_like(uw0).uniform_(-1, 1, generator=gw)
            uw = uw0.clone()
            wsw = api.workspace(_lib.workspace_bytes(_lib.OP_RUN, code, *wshape, T=Tw, norms=True, tblock=3), dev)
            ref = None
            for tb in (1, 2, 3):
                log(f"timing wide rows {wshape} {dname} tblock={tb}")
                uw.copy_(uw0)
                api.run(uw, fw, coeffs, Tw, bc, impl="fused", tblock=tb, norms=True, ws=wsw)
                torch.cuda.synchronize()
                if ref is None:
                    ref = uw.clone()
                elif not torch.equal(ref, uw):
                    raise RuntimeError(f"wide-row passes of {tb} steps differ from one-step passes")
                ms_w, _, _ = timed(lambda: api.run(uw, fw, coeffs, Tw, bc, impl="fused", tblock=tb, norms=True,
                                                   ws=wsw), kk, 1, stream)
                ent = fused_entry(ms_w / kk, S, tb, shape=wshape, steps=Tw)
                ent["T"] = Tw
                forms[f"wide_1024x1024x512_{dname}_tblock{tb}"] = ent
            del uw0, fw, uw, wsw, ref
            torch.cuda.empty_cache()

        # one GPU's share of the 512^3 grid split into 8 z-slabs: 512 x 512 x 64
        # planes, T = 100, FP64, periodic along z in place of the halo planes
        # a neighbour would send (the kernels' work per GPU at its real shape;
        # nothing crosses GPUs here)
        sshape = (nx, ny, nz // 8)
        us0 = u0[: nz // 8].clone()
        fs = f64[: nz // 8].clone()
        us = us0.clone()
        wss = api.workspace(_lib.workspace_bytes(_lib.OP_RUN, _lib.F64, *sshape, T=T, norms=True, tblock=3), dev)
        ref = None
        for tb in (1, 2, 3):
            log(f"timing one 8-way z-slab {sshape} f64 tblock={tb}")
            us.copy_(us0)
            api.run(us, fs, coeffs, T, bc, impl="fused", tblock=tb, norms=True, ws=wss)
            torch.cuda.synchronize()
            if ref is None:
                ref = us.clone()
            elif not torch.equal(ref, us):
                raise RuntimeError(f"z-slab passes of {tb} steps differ from one-step passes")
            ms_s, _, _ = timed(lambda: api.run(us, fs, coeffs, T, bc, impl="fused", tblock=tb, norms=True,
                                               ws=wss), kk, 1, stream)
            forms[f"zslab_512x512x64_f64_tblock{tb}"] = fused_entry(ms_s / kk, 8, tb, shape=sshape)
        del us0, fs, us, wss, ref
        torch.cuda.empty_cache()

        # adjoint kernel alone: k = 1 (no recomputation), 10 steps
        forms.update(adjoint_forms(dev, stream, u0, f64, coeffs, bc, kk))

        # end-to-end gradient, float64: forward T=100 with checkpoints every 10, then adjoint
        kck = 10
        ug = u0.clone()
        ck = torch.empty((T // kck, nz, ny, nx), dtype=torch.float64, device=dev)
        wsf = api.workspace(_lib.workspace_bytes(_lib.OP_RUN, _lib.F64, nx, ny, nz, T=T, tblock=2), dev)
        wsa = api.workspace(_lib.workspace_bytes(_lib.OP_ADJOINT, _lib.F64, nx, ny, nz, T=T, ckpt_every=kck,
                                                 tblock=3), dev)
        g = torch.empty_like(u0)

        def grad_step():
            ug.copy_(u0)
            api.run(ug, f64, coeffs, T, bc, tblock=args.tblock, norms=False, ckpt_every=kck, ws=wsf, ckpt=ck)
            api.adjoint_run(ck, kck, f64, ug, coeffs, T, bc, ws=wsa, grad_u0=g)

        log("timing end-to-end gradient f64")
        ms_g, _, _ = timed(grad_step, kk, 1, stream)
        ms_g /= kk
        forms["gradient_f64_T100_k10"] = {"ms": round(ms_g, 3),
                                          "ms_over_forward": round(ms_g / ms_step, 3)}

        def grad_step_all():
            ug.copy_(u0)
            api.run(ug, f64, coeffs, T, bc, tblock=args.tblock, norms=False, ckpt_every=kck, ws=wsf, ckpt=ck)
            api.adjoint_run(ck, kck, f64, ug, coeffs, T, bc, ws=wsa, grad_u0=g, want_f=True, want_gamma=True)

        log("timing end-to-end gradient f64 with dL/df and dL/dgamma")
        ms_ga, _, _ = timed(grad_step_all, kk, 1, stream)
        ms_ga /= kk
        forms["gradient_f64_T100_k10_all_inputs"] = {"ms": round(ms_ga, 3),
                                                     "ms_over_forward": round(ms_ga / ms_step, 3)}
        del ck, wsf, wsa

        # the two gradient workloads as stated: 256^3 float64 ghost-zero,
        # T=50, a checkpoint every 10 steps; 1024x1024x512 float32 periodic,
        # T=200, every 20 steps.  Loss 0.5*||u_T - u_tgt||^2, so the adjoint
        # starts from u_T - u_tgt.  One benchmark step: the forward run with
        # checkpoints, then the checkpointed adjoint (recomputation included).
        GiB = float(1 << 30)
        for wname in ("grad_256_f64", "grad_large_f32"):
            w = inputs.WORKLOADS[wname]
            gx, gy, gz = w["shape"]
            Tg, kg, bcg = w["T"], w["ckpt_every"], w["bc"]
            tdt = torch.float64 if w["dtype"] == "f64" else torch.float32
            code = _lib.F64 if w["dtype"] == "f64" else _lib.F32
            log(f"timing gradient workload {wname}: inputs ...")
            gu0_h, gf_h = inputs.make_fields(wname, seed=args.seed)
            gu0 = torch.from_numpy(gu0_h).to(dev, tdt)
            gf = torch.from_numpy(gf_h).to(dev, tdt)
            del gu0_h, gf_h
            gtgt = torch.from_numpy(inputs.target(gx, gy, gz, seed=args.seed)).to(dev, tdt)
            gN = gx * gy * gz
            gu = gu0.clone()
            gck = torch.empty((api.num_slots(Tg, kg), gz, gy, gx), dtype=tdt, device=dev)
            gwsf = api.workspace(_lib.workspace_bytes(_lib.OP_RUN, code, gx, gy, gz, T=Tg, tblock=3), dev)
            gwsa = api.workspace(_lib.workspace_bytes(_lib.OP_ADJOINT, code, gx, gy, gz, T=Tg, ckpt_every=kg,
                                                      tblock=3), dev)
            gg = torch.empty_like(gu0)
            glam = torch.empty_like(gu0)

            def fwd_only():
                gu.copy_(gu0)
                api.run(gu, gf, coeffs, Tg, bcg, tblock=3, norms=False, ckpt_every=kg, ws=gwsf, ckpt=gck)

            def adj_only():
                api.adjoint_run(gck, kg, gf, glam, coeffs, Tg, bcg, ws=gwsa, grad_u0=gg)

            def full():
                fwd_only()
                torch.sub(gu, gtgt, out=glam)
                adj_only()

            log(f"timing gradient workload {wname}")
            ms_full, _, _ = timed(full, kk, 1, stream)
            ms_fwd, _, _ = timed(fwd_only, kk, 1, stream)
            full()
            ms_adj, _, _ = timed(adj_only, kk, 1, stream)
            ms_full, ms_fwd, ms_adj = ms_full / kk, ms_fwd / kk, ms_adj / kk
            S = 8 if tdt == torch.float64 else 4
            mem = (gck.numel() * S + (gwsf.numel() if gwsf is not None else 0) + gwsa.numel()
                   + 5 * gN * S)  # u0, u, f, u_tgt (lam), dL/du0
            forms[f"gradient_{wname}"] = {
                "grid": [gx, gy, gz], "dtype": w["dtype"], "bc": "periodic" if bcg == inputs.PERIODIC else "dirichlet0",
                "T": Tg, "ckpt_every": kg, "ms": round(ms_full, 3),
                "forward_with_checkpoints_ms": round(ms_fwd, 3),
                "adjoint_ms": round(ms_adj, 3),
                "adjoint_glups_incl_recompute": round(glups(ms_adj, Tg, gN), 3),
                "device_memory_gib": round(mem / GiB, 2)}
            del gu0, gf, gtgt, gu, gck, gwsf, gwsa, gg, glam
            torch.cuda.empty_cache()

        # memory-bounded gradient over T=1000 steps: binomial checkpointing
        # with 8 snapshots against a checkpoint every 32 steps
        Tr, slots, kr = 1000, 8, 32
        log(f"timing gradient f64 T={Tr}: binomial checkpointing with {slots} snapshots")

        def rev_grad():
            ug.copy_(u0)
            wsr = api.revolve_forward(ug, f64, coeffs, Tr, bc, slots, tblock=args.tblock)
            api.revolve_adjoint(wsr, f64, ug, coeffs, Tr, bc, slots, tblock=args.tblock)

        ms_r, _, _ = timed(rev_grad, 2, 1, stream)
        ms_r /= 2
        _, fwd_steps = _lib.revolve_schedule(Tr, slots)
        mem_r = _lib.revolve_workspace_bytes(_lib.F64, nx, ny, nz, Tr, slots)
        log(f"timing gradient f64 T={Tr}: checkpoint every {kr} steps")
        ck = torch.empty(((Tr + kr - 1) // kr, nz, ny, nx), dtype=torch.float64, device=dev)
        wsf = api.workspace(_lib.workspace_bytes(_lib.OP_RUN, _lib.F64, nx, ny, nz, T=Tr, tblock=2), dev)
        wsa = api.workspace(_lib.workspace_bytes(_lib.OP_ADJOINT, _lib.F64, nx, ny, nz, T=Tr, ckpt_every=kr,
                                                 tblock=3), dev)

        def uni_grad():
            ug.copy_(u0)
            api.run(ug, f64, coeffs, Tr, bc, tblock=args.tblock, norms=False, ckpt_every=kr, ws=wsf, ckpt=ck)
            api.adjoint_run(ck, kr, f64, ug, coeffs, Tr, bc, ws=wsa, grad_u0=g)

        ms_u1, _, _ = timed(uni_grad, 2, 1, stream)
        ms_u1 /= 2
        mem_u = ck.numel() * 8 + wsa.numel() + (wsf.numel() if wsf is not None else 0)
        forms[f"gradient_f64_T{Tr}_revolve{slots}"] = {
            "ms": round(ms_r, 1), "forward_steps": int(fwd_steps) + 1, "adjoint_steps": Tr,
            "device_memory_gib": round(mem_r / GiB, 2),
            "vs_checkpoint_every_32": {"ms": round(ms_u1, 1), "forward_steps": 2 * Tr - (Tr + kr - 1) // kr,
                                       "device_memory_gib": round(mem_u / GiB, 2)}}
        del ck, wsf, wsa, g, ug, u32, f32

    # --------------------------------- kernels of the fusing compiler
    if args.forms == "all":
        torch.cuda.empty_cache()
        out["forms"]["generated"] = generated_forms(args, dev, stream, u0, f64, coeffs, bc)

    # ------------------------------------------------ the Jacobi listings
    if args.forms == "all":
        torch.cuda.empty_cache()
        out["forms"]["jacobi"] = jacobi_forms(args, dev, stream)

    # --------------------------------------------------------- CPU oracle
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (bounded sample) ...")
        out["cpu_baseline"], ref64 = cpu_baseline(u0_h, f_h, coeffs, bc)
        if not args.no_errors:
            log("errors of the GPU forms against the oracle ...")
            out["errors"] = form_errors(dev, u0, f64, u0_h, f_h, coeffs, bc, ref64)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
